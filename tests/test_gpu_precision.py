"""Reduced-precision weight storage against the FP32 path (teacher-forced).

The 64x64 / 256-agent world runs three times on the GPU (FP32, BF16 and FP8
E4M3 storage, every one with the same FP32 master), all driven by the same
actions (the oracle's own samples of its FP32 world), so the integer states
stay identical and each policy is evaluated on the same observation and the
same uniform.  Reported per step: the sampled actions of each storage format,
the logit error against the FP64 oracle on the FP32 master (quantisation +
accumulation), and against the FP64 oracle on the same quantised weights
(accumulation only).
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2510_18221_amd import workloads as wl

from gpu_util import LOGIT_TOL, logit_err, need_gpu, say
from worldstate import assert_same_state

pytestmark = pytest.mark.gpu


def test_bf16_fp8_agreement_1000_steps():
    need_gpu()
    from paper_2510_18221_amd import eco
    steps = 1000
    cfgs = {k: wl.world_small(seed=0, wdtype=v) for k, v in (("fp32", 0), ("bf16", 1), ("fp8", 2))}
    g = {k: eco.World(c) for k, c in cfgs.items()}
    o = {k: orc.OracleWorld(c) for k, c in cfgs.items()}
    for w in g.values():
        w.set_flags(eco.RT_KEEP_LOGITS)
    agree = {"bf16": [0, 0], "fp8": [0, 0]}
    err_master = {"fp32": [], "bf16": [], "fp8": []}
    err_same = {"fp32": [], "bf16": [], "fp8": []}
    pops = []
    for t in range(steps):
        alive = o["fp32"].state()["alive"].astype(bool)
        pops.append(int(alive.sum()))
        if not alive.any():
            break
        ref = {}
        ref["fp32"], sampled = o["fp32"].step(want_logits=True, want_sampled=True)
        acts = np.where(alive, sampled, 0).astype(np.uint8)
        for k in ("bf16", "fp8"):
            ref[k], _ = o[k].step(actions=acts, want_logits=True)
        for k, w in g.items():
            w.step_with_actions(acts)
        s32 = g["fp32"].read_sampled()[alive]
        for k in g:
            lg = g[k].read_logits()[alive]
            err_master[k].append(float(logit_err(lg, ref["fp32"][alive]).max()))
            err_same[k].append(float(logit_err(lg, ref[k][alive]).max()))
            if k != "fp32":
                sk = g[k].read_sampled()[alive]
                agree[k][0] += int((sk == s32).sum())
                agree[k][1] += int(alive.sum())
        if t % 100 == 0:
            st = g["fp32"].read_state()
            for k in ("bf16", "fp8"):
                assert_same_state(g[k].read_state(), st, f"{k} step {t}")
    rates = {k: v[0] / max(v[1], 1) for k, v in agree.items()}
    for k in g:
        say(f"[precision] {k}: max logit error vs FP64 on the FP32 master {max(err_master[k]):.3e} "
            f"(median of per-step max {np.median(err_master[k]):.3e}); vs FP64 on the stored weights "
            f"{max(err_same[k]):.3e}")
    say(f"[precision] action agreement with the FP32 path over {len(pops)} steps, {sum(pops)} agent-steps: "
        f"BF16 {100 * rates['bf16']:.3f}%, FP8 {100 * rates['fp8']:.3f}%; population {pops[0]} -> {pops[-1]}")
    assert max(err_same["fp32"]) <= LOGIT_TOL
    assert max(err_same["bf16"]) <= LOGIT_TOL
    assert max(err_same["fp8"]) <= LOGIT_TOL
    assert rates["bf16"] >= 0.999
    for w in g.values():
        w.close()

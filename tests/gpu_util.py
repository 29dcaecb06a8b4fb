"""Shared helpers of the GPU tests: world pairs (HIP library + oracle) and comparisons."""
import sys

import numpy as np
import pytest

from worldstate import assert_same_state

LOGIT_TOL = 1e-5    # normwise relative, FP32 GPU vs FP64 oracle on the same stored weights
TRAIT_RTOL = 1e-9   # FP64 trait moments, relative (derivation in assert_stats_match)


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def logit_err(gpu, ref):
    """Per-agent normwise relative error max|l_gpu - l_ref| / max(max|l_ref|, 1e-30)."""
    num = np.abs(gpu.astype(np.float64) - ref).max(axis=-1)
    den = np.maximum(np.abs(ref).max(axis=-1), 1e-30)
    return num / den


def assert_weights_close(gpu, ref, what, ulps=4):
    """FP32 master / storage values: identical up to a few FP32 ulps (the Box-Muller
    transform runs on libm on the CPU and on ocml on the GPU; both within an ulp
    in FP64, which moves the FP32 result by at most one rounding step)."""
    tol = ulps * np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
    bad = np.abs(gpu - ref) > tol
    assert not bad.any(), (what, int(bad.sum()), np.nonzero(bad)[0][:5])


def assert_stats_match(g, o, what, check_trait=True):
    for k in ("step", "population", "births", "deaths", "killed", "eaten", "regrown", "moves_ok", "moves_blocked",
              "births_blocked_cell", "births_blocked_capacity", "resource_total", "action_hist", "water_total",
              "biomass_total", "hp_total"):
        assert g[k] == o[k], (what, k, g[k], o[k])
    assert g["energy_total"] == o["energy_total"], (what, "energy_total")
    if check_trait:
        # Relative bound.  Each agent's |theta|^2 is a sum of P exact FP64 squares of
        # FP32 values, added in different orders on the two sides (relative
        # difference ~ sqrt(P) u <= 4e-14 for P <= 133,767, u = 2^-53, under the
        # random-rounding model); the variance amplifies it by at most
        # 2 mean / sd (~200 for these policies); both population reductions are
        # two-pass (the oracle's sequential one, the GPU's tile-wise one merged by
        # the Chan-Golub-LeVeque update), each ~1e-14 relative.  1e-9 leaves a
        # margin of 50x over the sum.
        for k in ("trait_mean", "trait_var"):
            assert abs(g[k] - o[k]) <= TRAIT_RTOL * abs(o[k]), (what, k, g[k], o[k])


def compare_world(gw, ow, what, world=0, weights_slots=8):
    gs, os_ = gw.read_state(world), ow.state()
    assert_same_state(gs, os_, what)
    live = np.nonzero(os_["alive"])[0]
    for s in live[:: max(1, len(live) // weights_slots)][:weights_slots]:
        assert_weights_close(gw.read_weights(int(s), world, master=True), ow.weights(int(s), master=True),
                             f"{what} master slot {s}")
        assert_weights_close(gw.read_weights(int(s), world), ow.weights(int(s)), f"{what} storage slot {s}")
    if gw.cfgs[world].get("flags", 0) & 4:   # colour traits of every live slot
        gc = gw.read_colours(world)
        assert np.all(np.isnan(gc[~os_["alive"].astype(bool)]))
        oc = np.array([ow.colour(int(s)) for s in live], np.float64).reshape(-1, 3)
        assert_weights_close(gc[live].astype(np.float64).reshape(-1), oc.reshape(-1), f"{what} colours")
    return gs


def run_pair(eco, cfg, steps, actions_fn=None, check_logits=True, what="", every=1, launch=None, flags=0):
    """Step GPU and oracle together.  actions_fn(step) -> actions, or None for the
    oracle's own sampled actions, which are injected into the GPU world.
    launch: optional policy-kernel shape (waves per block, blocks per CU, unroll).
    flags: runtime flags added to RT_KEEP_LOGITS (RT_SPLIT_STEP: a small world's
    step as separate kernels instead of the fused launch)."""
    from oracle import oracle as orc
    ow = orc.OracleWorld(cfg)
    gw = eco.World(cfg)
    if launch:
        gw.set_launch(*launch)
    gw.set_flags(eco.RT_KEEP_LOGITS | flags)
    compare_world(gw, ow, f"{what} init")
    assert_stats_match(gw.stats()[0], ow.stats(), f"{what} init")
    worst = 0.0
    mismatched = 0
    for t in range(steps):
        pre_alive = ow.state()["alive"].astype(bool)
        if actions_fn is None:
            logits, sampled = ow.step(want_logits=True, want_sampled=True)
            acts = sampled.copy()
            acts[~pre_alive] = 0
        else:
            acts = actions_fn(t)
            logits, sampled = ow.step(actions=acts, want_logits=True, want_sampled=True)
        gw.step_with_actions(acts)
        if check_logits:
            gl = gw.read_logits()
            err = logit_err(gl[pre_alive], logits[pre_alive])
            worst = max(worst, float(err.max(initial=0.0)))
            assert np.all(np.isnan(gl[~pre_alive]))
            gs = gw.read_sampled()
            mismatched += int((gs[pre_alive] != sampled[pre_alive]).sum())
        if t % every == 0 or t == steps - 1:
            compare_world(gw, ow, f"{what} step {t}")
            assert_stats_match(gw.stats()[0], ow.stats(), f"{what} step {t}")
    gw.close()
    say(f"{what}: worst normwise logit error {worst:.3e}, sampled-action mismatches {mismatched}")
    assert worst <= LOGIT_TOL
    return worst, mismatched

"""Parity at the benchmark sizes, on outputs the oracle can compute one by one.

The oracle runs in lineage mode (integer world exact, weights rebuilt on demand
for sampled agents), driven by seeded actions from the input generators; the
GPU world runs in the default launch configuration of the library.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2510_18221_amd import workloads as wl

from gpu_util import LOGIT_TOL, assert_weights_close, logit_err, need_gpu, say
from worldstate import assert_same_state, check_invariants

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eco():
    need_gpu()
    from paper_2510_18221_amd import eco as m
    m.lib()
    return m


def perturb_energies(st, seed):
    """Seeded energies so that the first steps contain both deaths and births."""
    rng = np.random.default_rng(seed)
    live = np.nonzero(st["alive"])[0]
    e = rng.choice(np.array([1, 2, 100, 250, 400], np.int32), size=len(live), p=[0.05, 0.05, 0.5, 0.3, 0.1])
    st["energy"][live] = e
    return st


def sample_slots(st, n, seed):
    live = np.nonzero(st["alive"])[0]
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(live, size=min(n, len(live)), replace=False))


def fullsize_parity(eco, cfgs, worlds_checked, steps, n_sample, seed):
    gw = eco.World(cfgs)
    gw.set_flags(eco.RT_KEEP_LOGITS)
    ows = {i: orc.OracleWorld(cfgs[i], materialize=False) for i in worlds_checked}
    for i, ow in ows.items():
        say(f"[fullsize] world {i}: init state")
        assert_same_state(gw.read_state(i), ow.state(), f"world {i} init")
        st = perturb_energies(ow.state(), seed + i)
        ow.write_state(st)
        gw.write_state(st, i)
        assert_same_state(gw.read_state(i), ow.state(), f"world {i} written")
    for t in range(steps):
        acts = [wl.biased_actions(c["capacity"], c["n_actions"], seed + i, t) for i, c in enumerate(cfgs)]
        checks = {}
        for i, ow in ows.items():
            st = ow.state()
            slots = sample_slots(st, n_sample, seed + 100 * t + i)
            checks[i] = (st, slots, np.stack([ow.agent_logits(int(s)) for s in slots]))
        gw.step_with_actions(np.concatenate(acts))
        for i, ow in ows.items():
            ow.step(actions=acts[i])
            st_pre, slots, ref = checks[i]
            gl = gw.read_logits(i)[slots]
            err = logit_err(gl, ref)
            say(f"[fullsize] world {i} step {t}: max normwise logit error {err.max():.2e} over {len(slots)} agents")
            assert err.max() <= LOGIT_TOL
            gs, os_ = gw.read_state(i), ow.state()
            assert_same_state(gs, os_, f"world {i} step {t}")
            births = np.nonzero(os_["alive"] & (os_["age"] == 0) & (os_["parent_uid"] != 0xFFFFFFFFFFFFFFFF))[0]
            for c in births[:: max(1, len(births) // 3)][:3]:
                assert_weights_close(gw.read_weights(int(c), i, master=True), ow.weights(int(c), master=True),
                                     f"world {i} child {c}")
                assert_weights_close(gw.read_weights(int(c), i), ow.weights(int(c)), f"world {i} child {c} storage")
            st_g = gw.stats()[i]
            ost = ow.stats()
            for k in ("population", "births", "deaths", "eaten", "regrown", "moves_ok", "moves_blocked",
                      "births_blocked_cell", "births_blocked_capacity", "resource_total", "action_hist"):
                assert st_g[k] == ost[k], (i, t, k)
            assert st_g["energy_total"] == ost["energy_total"]
            if t == 0:
                assert ost["births"] > 0 and ost["deaths"] > 0
    return gw


def free_running_invariants(gw, cfgs, steps):
    prev = gw.stats()
    for t in range(steps):
        gw.step(1)
        cur = gw.stats()
        for i, c in enumerate(cfgs):
            p, s = prev[i], cur[i]
            assert s["population"] == p["population"] + s["births"] - s["deaths"]
            assert s["resource_total"] == p["resource_total"] - s["eaten"] + s["regrown"]
            assert s["energy_total"] == (p["energy_total"] + c["e_eat"] * s["eaten"] - c["e_cost"] * p["population"])
            assert sum(s["action_hist"]) == p["population"]
        prev = cur
    for i, c in enumerate(cfgs[:4]):
        check_invariants(gw.read_state(i), c["width"], c["height"])


def test_65k_world_bench_configuration(eco):
    """1024x1024, 65,536 agents, capacity 131,072, FP32 492->64->64->7."""
    cfg = wl.world_65k(seed=0)
    gw = fullsize_parity(eco, [cfg], [0], steps=3, n_sample=96, seed=1)
    gw.set_flags(eco.RT_USE_GRAPH)
    free_running_invariants(gw, [cfg], 20)
    gw.close()


@pytest.mark.parametrize("wdtype", [1, 2])
def test_65k_world_quantised_storage(eco, wdtype):
    cfg = wl.world_65k(seed=2, wdtype=wdtype)
    gw = fullsize_parity(eco, [cfg], [0], steps=2, n_sample=48, seed=2)
    gw.close()


def test_batch_of_64_worlds(eco):
    """64 worlds, sides log-uniform in [128, 1024], 6.25% occupancy, BF16 + FP32 master."""
    cfgs = wl.world_batch(64)
    say(f"[fullsize] batch: {sum(c['n_agents_init'] for c in cfgs)} agents, "
        f"{sum(c['capacity'] for c in cfgs)} slots")
    order = np.argsort([c["width"] for c in cfgs])
    checked = [int(order[0]), int(order[31]), int(order[-1])]
    gw = fullsize_parity(eco, cfgs, checked, steps=2, n_sample=24, seed=3)
    gw.set_flags(eco.RT_USE_GRAPH)
    free_running_invariants(gw, cfgs, 498)   # the configuration's 500 steps in all
    gw.close()


def test_large_world(eco):
    """2048x2048, capacity 262,144 half full, 908->128->128->7 BF16 + FP32 master."""
    cfg = wl.world_large(seed=0)
    gw = fullsize_parity(eco, [cfg], [0], steps=2, n_sample=32, seed=4)
    gw.set_flags(eco.RT_USE_GRAPH)
    free_running_invariants(gw, [cfg], 9998)   # the configuration's 10,000 steps in all
    say(f"[fullsize] large world after 10,000 steps: population {gw.stats()[0]['population']}")
    gw.close()


def test_65k_world_1000_steps(eco):
    """The 65,536-agent FP32 world over the configuration's 1,000 steps under seeded
    actions (energies perturbed so births and deaths start at once): statistics
    equal every step, the whole integer state every 250 steps, and the logits of
    sampled agents (weights rebuilt from their lineages) at the end."""
    cfg = wl.world_65k(seed=5)
    gw = eco.World(cfg)
    ow = orc.OracleWorld(cfg, materialize=False)
    st = perturb_energies(ow.state(), 5)
    ow.write_state(st)
    gw.write_state(st)
    births = deaths = 0
    for t in range(1000):
        acts = wl.biased_actions(cfg["capacity"], 7, 5, t)
        if t == 999:
            gw.set_flags(eco.RT_KEEP_LOGITS)
            st_pre = ow.state()
            slots = sample_slots(st_pre, 48, 55)
            ref = np.stack([ow.agent_logits(int(s)) for s in slots])
        ow.step(actions=acts)
        gw.step_with_actions(acts)
        g, o = gw.stats()[0], ow.stats()
        for k in ("population", "births", "deaths", "eaten", "regrown", "moves_ok", "moves_blocked",
                  "births_blocked_cell", "births_blocked_capacity", "resource_total", "action_hist", "energy_total"):
            assert g[k] == o[k], (t, k, g[k], o[k])
        births += o["births"]
        deaths += o["deaths"]
        if t % 250 == 249:
            assert_same_state(gw.read_state(), ow.state(), f"step {t}")
            say(f"[fullsize] 1000-step run: step {t + 1} population {o['population']}, births {births}, "
                f"deaths {deaths}")
    err = logit_err(gw.read_logits()[slots], ref)
    say(f"[fullsize] 1000-step run: max normwise logit error {err.max():.2e} over {len(slots)} agents at step 1000")
    assert err.max() <= LOGIT_TOL and births > 0 and deaths > 0
    gw.close()

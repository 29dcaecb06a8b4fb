"""The fused small-world step (k_step_small: one launch after the policy kernel for
an object of one world of at most 8,192 slots and 16,384 cells)
against the separate kernels (ECO_RT_SPLIT_STEP) and against the oracle.

The fused launch applies the same per-agent and per-cell rules and does the
world's scans inside one block, so the integer state, the weights, the logits and
every integer statistic are identical to the separate kernels' step for step;
only the trait moments, merged in another order, may differ in the last bits.
"""
import numpy as np
import pytest

from paper_2510_18221_amd import eco as eco_mod
from paper_2510_18221_amd import workloads as wl

from gpu_util import need_gpu, run_pair, say
from worldstate import assert_same_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eco():
    need_gpu()
    from paper_2510_18221_amd import eco as m
    m.lib()
    return m


def busy(**kw):
    """A small world with births every step: agents start at the reproduction
    threshold and the step costs nothing, so parents reproduce whenever the cell
    behind is free and newborns (born with no energy) die at their first step."""
    base = dict(width=24, height=20, n_agents_init=120, capacity=300, resource_density=0.3, regrow_prob=0.05,
                mutation_sigma=0.05, window=5, n_scalars=8, hidden1=32, hidden2=32, n_actions=7, e_init=200,
                e_cost=0, e_child=0, seed=11)
    base.update(kw)
    return wl.desc(**base)


CASES = {
    "config1": wl.world_small(seed=3),
    "busy_fp32": busy(),
    "busy_bf16": busy(wdtype=wl.BF16, seed=12),
    "busy_fp8_h64": busy(wdtype=wl.FP8, hidden1=64, hidden2=64, seed=13),
    "busy_h128_a5": busy(hidden1=128, hidden2=128, n_actions=5, window=3, n_scalars=4, seed=14),
    "attack": busy(attack_enabled=1, e_init=150, e_cost=1, e_child=40, seed=15),
    "colour_temp": busy(flags=eco_mod.DESC_COLOUR_VISION | eco_mod.DESC_EVOLVE_TEMPERATURE, seed=16),
    "full_capacity": busy(n_agents_init=200, capacity=200, seed=17),
    # every (storage type, hidden width) instantiation of the fused kernel
    "busy_fp32_h64": busy(hidden1=64, hidden2=64, seed=19),
    "busy_bf16_h64": busy(wdtype=wl.BF16, hidden1=64, hidden2=64, seed=20),
    "busy_bf16_h128": busy(wdtype=wl.BF16, hidden1=128, hidden2=128, window=3, seed=21),
    "busy_fp8_h32": busy(wdtype=wl.FP8, seed=22),
    "busy_fp8_h128": busy(wdtype=wl.FP8, hidden1=128, hidden2=128, window=3, n_actions=5, n_scalars=4, seed=23),
    # the largest object the fused launch takes: 8,192 slots (both passes of four
    # slots per thread full) and 16,384 cells (four passes of the cell loops)
    "limits": busy(width=128, height=128, n_agents_init=5000, capacity=8192, seed=24),
}


def eco_world(**kw):
    """A small world of the three-resource ecology with births: agents start with
    the biomass and energy to reproduce, and meals are cheap."""
    base = dict(width=24, height=20, n_agents_init=120, capacity=300, window=5, hidden1=32, hidden2=32,
                mutation_sigma=0.05, e_init=250, seed=31)
    e = kw.pop("eco", {})
    base.update(kw)
    return wl.ecology_desc(eco=dict(w_cost=1, age_shift=6, b_init=4, **e), **base)


ECO = eco_mod.DESC_ECOLOGY
CASES.update({
    # the ecology: photosynthesis and the three totals in the record
    "eco": eco_world(),
    "eco_bf16_h64": eco_world(wdtype=wl.BF16, hidden1=64, hidden2=64, seed=32),
    # strikes as the ninth action (health damage, marks cleared by the cell pass)
    "eco_attack": eco_world(attack_enabled=1, eco=dict(attack_damage=50), seed=33),
    # terrain (the flow gather and its copy-back) with the rendered colour window
    "eco_terrain_colour": eco_world(window=7, flags=ECO | eco_mod.DESC_TERRAIN | eco_mod.DESC_COLOUR_VISION,
                                    eco=dict(terrain_scale=12, sea_level=12, water_per_depth=3), seed=34),
    # the paper's Ocean agent in a small world: the same with full-strength strikes
    # and the evolving temperature, FP8 weights
    "eco_ocean_fp8": eco_world(window=7, n_actions=9, attack_enabled=1, wdtype=wl.FP8,
                               flags=ECO | eco_mod.DESC_TERRAIN | eco_mod.DESC_COLOUR_VISION
                               | eco_mod.DESC_EVOLVE_TEMPERATURE,
                               eco=dict(terrain_scale=12, sea_level=12, water_per_depth=3), seed=35),
    # the largest ecology object the fused launch takes (four passes of the cell loops),
    # with terrain, colour and strikes
    "eco_limits": eco_world(width=128, height=128, n_agents_init=3000, capacity=8192, window=7, n_actions=9,
                            attack_enabled=1, flags=ECO | eco_mod.DESC_TERRAIN | eco_mod.DESC_COLOUR_VISION,
                            eco=dict(terrain_scale=12, sea_level=12, water_per_depth=3, attack_damage=50), seed=36),
    # a width that is not a multiple of 4 (the flow's per-cell neighbour path) and a
    # ragged last group of cells (127 x 129 = 16,383 cells)
    "eco_odd": eco_world(width=127, height=129, n_agents_init=1500, capacity=4000, window=7,
                         flags=ECO | eco_mod.DESC_TERRAIN, eco=dict(terrain_scale=12, sea_level=12, water_per_depth=3),
                         seed=37),
})


def trait_close(a, b):
    return abs(a - b) <= 1e-12 * max(abs(a), abs(b), 1e-300)


@pytest.mark.parametrize("name", sorted(CASES))
def test_fused_equals_split(eco, name):
    cfg = CASES[name]
    steps = 25
    fused, split = eco.World(cfg), eco.World(cfg)
    fused.set_flags(eco.RT_KEEP_LOGITS | eco.RT_USE_GRAPH)
    split.set_flags(eco.RT_KEEP_LOGITS | eco.RT_USE_GRAPH | eco.RT_SPLIT_STEP)
    births = 0
    for t in range(steps):
        fused.step(1)
        split.step(1)
        a, b = fused.read_state(), split.read_state()
        assert_same_state(a, b, f"{name} step {t}")
        np.testing.assert_array_equal(fused.read_logits(), split.read_logits())
        sa, sb = fused.stats()[0], split.stats()[0]
        for k, v in sa.items():
            if k in ("trait_mean", "trait_var"):
                assert trait_close(v, sb[k]), (name, t, k, v, sb[k])
            else:
                assert v == sb[k], (name, t, k, v, sb[k])
        births += sa["births"]
    live = np.nonzero(a["alive"])[0]
    for s in live[:: max(1, len(live) // 6)]:
        for master in (True, False):
            np.testing.assert_array_equal(fused.read_weights(int(s), master=master),
                                          split.read_weights(int(s), master=master))
    fused.close()
    split.close()
    say(f"{name}: {steps} steps, {births} births, fused == split")
    if name.startswith(("busy", "eco")) or name == "limits":
        assert births > 0


def test_fused_path_is_the_one_that_runs(eco):
    """Kernel-group timers: the fused launch is timed as MOVE, with no separate
    birth-claim, ranking, commit or compaction launches; RT_SPLIT_STEP runs them."""
    cfg = CASES["busy_fp32"]
    for flags, fused in ((eco.RT_TIME_KERNELS, True), (eco.RT_TIME_KERNELS | eco.RT_SPLIT_STEP, False)):
        w = eco.World(cfg)
        w.set_flags(flags)
        w.step(3)
        kt = w.kernel_times(reset=True)
        w.close()
        assert kt["forward"][1] == 3 and kt["move"][1] == 3
        for k in ("birth_claim", "birth_scan", "birth_commit", "compact"):
            assert (kt[k][1] == 0) == fused, (flags, k, kt[k])


def test_large_object_takes_the_split_kernels(eco):
    cfg = busy(width=160, height=128, n_agents_init=2000, capacity=4000, seed=18)   # 20,480 cells: above the limit
    w = eco.World(cfg)
    w.set_flags(eco.RT_TIME_KERNELS)
    w.step(2)
    kt = w.kernel_times(reset=True)
    w.close()
    assert kt["compact"][1] == 2


@pytest.mark.parametrize("name", ["config1", "busy_bf16", "eco_terrain_colour", "eco_odd"])
def test_split_kernels_match_oracle_on_small_worlds(eco, name):
    """The separate kernels keep their oracle parity on small worlds too (the
    ecology's cell passes in cell tiles, with a ragged last tile and group)."""
    cfg = CASES[name]
    acts = lambda t: wl.biased_actions(cfg["capacity"], cfg["n_actions"], 7, t, p_forward=0.35, p_eat=0.3)
    run_pair(eco, cfg, 8, actions_fn=acts, what=f"split {name}", flags=eco.RT_SPLIT_STEP)


@pytest.mark.parametrize("name", ["busy_fp32", "attack", "busy_fp8_h64", "busy_bf16_h128", "limits", "eco",
                                  "eco_attack", "eco_terrain_colour", "eco_ocean_fp8", "eco_limits", "eco_odd"])
def test_fused_matches_oracle(eco, name):
    cfg = CASES[name]
    acts = lambda t: wl.biased_actions(cfg["capacity"], cfg["n_actions"], 5, t, p_forward=0.3, p_eat=0.3,
                                       **({"p_attack": 0.1} if cfg.get("attack_enabled") else {}))
    run_pair(eco, cfg, 10, actions_fn=acts, what=f"fused {name}")

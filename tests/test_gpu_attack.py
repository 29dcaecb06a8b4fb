"""Attacks and the death deposit on the GPU against the oracle (the "+A" worlds:
Sec. 3.2 actions and health points; App. "Varying Attack Strength", full
strength).  An attacker kills every other agent in the 3x3 square directly in
front of it after the moves of the step; each victim leaves one resource unit
on its cell.  Integer state bit-exact, statistics (killed included) equal,
logits within the FP32 tolerance.  The hand-built cases are the oracle's
hand-traced attack pins, replayed through the C ABI.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2510_18221_amd import workloads as wl

from gpu_util import assert_stats_match, compare_world, need_gpu, run_pair, say
from worldstate import N, E, S, W, assert_same_state, check_invariants, empty_state, place

pytestmark = pytest.mark.gpu

ATK = 6


@pytest.fixture(scope="module")
def eco():
    need_gpu()
    from paper_2510_18221_amd import eco as m
    m.lib()
    return m


def _cfg(**kw):
    c = wl.desc(width=8, height=8, n_agents_init=0, capacity=8, window=3, n_scalars=4, hidden1=32, hidden2=32,
                n_actions=7, attack_enabled=1, resource_density=0.0, regrow_prob=0.0, seed=1)
    c.update(kw)
    return c


def _case(name):
    cfg, st = _cfg(), empty_state(8, 8, 8)
    acts = [0] * 8
    if name == "square":
        for k, (x, y, f) in enumerate([(3, 5, N), (2, 4, E), (4, 2, S), (3, 1, N), (5, 3, N), (3, 6, N)]):
            place(st, 8, k, x, y, f, 100)
        acts[0] = ATK
    elif name == "wrap":
        for k, (x, y, f) in enumerate([(7, 3, E), (0, 4, N), (2, 2, N), (3, 3, N), (6, 0, N), (7, 6, W), (5, 4, W)]):
            place(st, 8, k, x, y, f, 100)
        acts[0] = acts[4] = ATK
    elif name == "mutual":
        place(st, 8, 0, 3, 2, S, 100); place(st, 8, 1, 3, 4, N, 100)
        acts[0] = acts[1] = ATK
    elif name == "moves_first":
        for k, (x, y, f) in enumerate([(3, 5, N), (3, 1, S), (2, 4, W), (4, 4, E), (5, 4, N)]):
            place(st, 8, k, x, y, f, 100)
        acts[:4] = [ATK, 3, 3, 3]
    elif name == "no_meal":
        place(st, 8, 0, 3, 5, N, 100); place(st, 8, 1, 3, 4, N, 100); st["res"][4 * 8 + 3] = 1
        acts[:2] = [ATK, 4]
    elif name == "disabled":
        cfg = _cfg(attack_enabled=0)
        place(st, 8, 0, 3, 5, N, 100); place(st, 8, 1, 3, 4, N, 100)
        acts[0] = ATK
    elif name == "tiny_torus":
        cfg, st = _cfg(width=3, height=3, window=1, capacity=4), empty_state(3, 3, 4)
        place(st, 3, 0, 1, 1, N, 100); place(st, 3, 1, 0, 0, E, 100); place(st, 3, 2, 2, 2, W, 100)
        acts = [ATK, 0, 0, 0]
    elif name == "reuse":
        cfg, st = _cfg(capacity=3), empty_state(8, 8, 3, uid_next=100)
        place(st, 8, 0, 3, 5, N, 100); place(st, 8, 1, 4, 2, N, 100); place(st, 8, 2, 5, 2, E, 250, uid=42)
        acts = [ATK, 0, 5]
    elif name == "walls":
        place(st, 8, 0, 3, 5, N, 100); place(st, 8, 1, 3, 3, N, 100)
        st["wall"][4 * 8 + 3] = 1                   # a wall between attacker and victim does not shield it
        acts[0] = ATK
    return cfg, st, acts


@pytest.mark.parametrize("case", ["square", "wrap", "mutual", "moves_first", "no_meal", "disabled", "tiny_torus",
                                  "reuse", "walls"])
def test_hand_built_attacks(eco, case):
    cfg, st, acts = _case(case)
    ow = orc.OracleWorld(cfg)
    ow.write_state(st)
    gw = eco.World(cfg)
    gw.write_state(st)
    a = np.array(acts, np.uint8)
    ow.step(actions=a)
    gw.step_with_actions(a)
    assert_same_state(gw.read_state(), ow.state(), case)
    assert_stats_match(gw.stats()[0], ow.stats(), case)
    check_invariants(gw.read_state(), cfg["width"], cfg["height"])
    if case not in ("disabled",):
        assert ow.stats()["killed"] > 0, case
    gw.close()


def _attack_world(seed=0, wdtype=0, **kw):
    """96x80 torus, 450 agents, 11x11 window, 492->64->64->7 (several policy tiles and a ragged tail)."""
    d = wl.desc(width=96, height=80, n_agents_init=450, capacity=700, resource_density=0.3, regrow_prob=0.02,
                mutation_sigma=0.01, window=11, n_scalars=8, hidden1=64, hidden2=64, n_actions=7, wdtype=wdtype,
                seed=seed, e_init=170, attack_enabled=1)
    d.update(kw)
    return d


@pytest.mark.parametrize("wdtype", [0, 1, 2])
def test_attack_world_seeded_actions(eco, wdtype):
    cfg = _attack_world(seed=21 + wdtype, wdtype=wdtype)
    acts = lambda t: wl.biased_actions(cfg["capacity"], 7, 21, t, p_attack=0.1)
    killed = []
    ow = orc.OracleWorld(cfg)
    run_pair(eco, cfg, 15, actions_fn=acts, what=f"attack wdtype {wdtype}", every=3)
    for t in range(15):
        ow.step(actions=acts(t))
        killed.append(ow.stats()["killed"])
    say(f"attack wdtype {wdtype}: killed per step {killed}")
    assert sum(killed) > 50


def test_attack_world_policy_actions(eco):
    """Actions the policies sample (the oracle's draws injected into the GPU world)."""
    cfg = _attack_world(seed=30, e_init=120)
    run_pair(eco, cfg, 10, what="attack free-running")


def test_attack_graph_and_eager_agree(eco):
    """Free-running GPU worlds with attacks (the policy kernel's own samples decide
    who attacks): step graphs, eager launches and the timed graph give the same
    state and statistics."""
    cfg = _attack_world(seed=31, e_init=150)
    a, b, c = eco.World(cfg), eco.World(cfg), eco.World(cfg)
    b.set_flags(0)
    c.set_flags(eco.RT_USE_GRAPH | eco.RT_TIME_KERNELS)
    a.step(20)
    b.step(20)
    for n in (8, 12):
        c.step(n)
    assert_same_state(a.read_state(), b.read_state(), "graph vs eager")
    assert_same_state(a.read_state(), c.read_state(), "graph vs timed graph")
    assert a.stats() == b.stats() == c.stats()
    hist = a.stats_history(0, 21)
    assert sum(h["killed"] for h in hist) > 0
    for w in (a, b, c):
        w.close()


def test_mixed_attack_flags_in_one_object(eco):
    """Per-world switch: worlds with and without attacks stepped together."""
    cfgs = [_attack_world(seed=40 + i, width=40 + 8 * i, height=30, n_agents_init=120, capacity=256,
                          attack_enabled=i % 2) for i in range(4)]
    gw = eco.World(cfgs)
    ows = [orc.OracleWorld(c) for c in cfgs]
    for t in range(8):
        acts = [wl.biased_actions(c["capacity"], 7, 40 + i, t, p_attack=0.15) for i, c in enumerate(cfgs)]
        for ow, x in zip(ows, acts):
            ow.step(actions=x)
        gw.step_with_actions(np.concatenate(acts))
        stats = gw.stats()
        for i, ow in enumerate(ows):
            compare_world(gw, ow, f"world {i} step {t}", world=i, weights_slots=2)
            assert_stats_match(stats[i], ow.stats(), f"world {i} step {t}")
            if not cfgs[i]["attack_enabled"]:
                assert stats[i]["killed"] == 0
    gw.close()


def test_stamps_cleared_by_state_writes(eco):
    """A state written back to an earlier step carries no attack of the later run:
    the stamps of the first run's steps 0..2 would otherwise strike again."""
    cfg = _attack_world(seed=50, e_init=150)
    acts = lambda t: wl.biased_actions(cfg["capacity"], 7, 50, t, p_attack=0.2)
    gw = eco.World(cfg)
    st0 = gw.read_state()
    for t in range(3):
        gw.step_with_actions(acts(t))
    gw.write_state(st0)           # back to step 0: the stamps of steps 0..2 must not strike again
    ow = orc.OracleWorld(cfg)
    for t in range(3):
        a = wl.biased_actions(cfg["capacity"], 7, 51, t, p_attack=0.0)
        ow.step(actions=a)
        gw.step_with_actions(a)
        assert_same_state(gw.read_state(), ow.state(), f"after rewind step {t}")
        assert_stats_match(gw.stats()[0], ow.stats(), f"after rewind step {t}", check_trait=False)
    gw.close()

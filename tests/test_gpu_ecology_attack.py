"""Attack in the three-resource ecology on the GPU against the oracle (Sec. 3.2
actions and health points; App. "Varying Attack Strength"): the ninth action
strikes the 3x3 square ahead after the moves, each strike costs the struck agent
attack_damage health (full 100, half 50, quarter 25) in its health update, and a
struck agent that dies leaves everything it carries on its cell; an attacker
strikes each distinct cell of its square once, also where a narrow torus folds
the square onto itself.  Integer state
bit-exact, statistics (killed included) equal, logits (nine of them) within the
FP32 tolerance.  The hand-built cases are the oracle's hand-traced pins, replayed
through the C ABI.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2510_18221_amd import workloads as wl

from gpu_util import assert_stats_match, compare_world, need_gpu, run_pair, say
from worldstate import N, S, W, assert_same_state, check_invariants, empty_state, place

pytestmark = pytest.mark.gpu

ATK = 8
HAND = dict(water_density=0.0, energy_density=0.0, biomass_density=0.0, water_site=0, energy_site=0, biomass_site=0,
            eat_water=10, eat_biomass=1, cap_water=60, cap_energy=400, cap_biomass=8, e_cost_move=2, w_cost=3,
            photo_rate=0.0, cell_energy_max=40, hp_max=100, hp_child=50, hp_overspend=20, hp_heal=10, heal_energy=1,
            age_shift=31, w_init=30, b_init=2, w_child=10, b_child=1, b_repro=2)
STRENGTHS = {"full": wl.ATTACK_FULL, "half": wl.ATTACK_HALF, "quarter": wl.ATTACK_QUARTER}


@pytest.fixture(scope="module")
def eco():
    need_gpu()
    from paper_2510_18221_amd import eco as m
    m.lib()
    return m


def _hand_cfg(damage):
    return wl.ecology_desc(eco=dict(HAND, attack_damage=damage), width=6, height=6, n_agents_init=0, capacity=4,
                           window=3, hidden1=32, hidden2=32, resource_density=0.0, regrow_prob=0.0, seed=1, e_eat=10,
                           e_cost=1, e_repro=200, e_child=50, attack_enabled=1)


def _put(st, slot, x, y, f, E_, W_, B_, hp):
    place(st, 6, slot, x, y, f, E_)
    st["water"][slot], st["biomass"][slot], st["hp"][slot] = W_, B_, hp


def _case(name):
    st = empty_state(6, 6, 4, ecology=True, uid_next=100)
    if name == "full":          # the victim eats, then dies; its body feeds the cell
        _put(st, 0, 2, 4, N, 100, 30, 2, 100); _put(st, 1, 2, 3, N, 100, 30, 2, 100)
        _put(st, 2, 5, 5, N, 100, 30, 2, 100)
        st["cell_biomass"][3 * 6 + 2] = 3
        return _hand_cfg(100), st, [ATK, 6, 0, 0]
    if name == "half":          # one strike wounds (then heals), two kill
        _put(st, 0, 1, 4, N, 100, 30, 2, 100); _put(st, 1, 3, 4, N, 100, 30, 2, 100)
        _put(st, 2, 2, 2, N, 100, 30, 2, 100); _put(st, 3, 4, 1, N, 100, 30, 2, 100)
        return _hand_cfg(50), st, [ATK, ATK, 0, 0]
    if name == "quarter":       # attackers strike each other; an overspend death is not a kill
        _put(st, 0, 2, 4, N, 100, 30, 2, 100); _put(st, 1, 2, 1, S, 100, 30, 2, 100)
        _put(st, 2, 3, 2, N, 100, 30, 2, 40); _put(st, 3, 0, 0, N, 100, 0, 2, 15)
        return _hand_cfg(25), st, [ATK, ATK, 0, 0]
    if name == "moves":         # moves resolve before the strikes
        _put(st, 0, 2, 4, N, 100, 30, 2, 100); _put(st, 1, 2, 0, S, 100, 30, 2, 100)
        _put(st, 2, 1, 3, W, 100, 30, 2, 100); _put(st, 3, 3, 2, N, 100, 30, 2, 100)
        return _hand_cfg(100), st, [ATK, 3, 3, 3]
    if name == "narrow":        # a 2-wide torus: the square's two side columns are one; each cell struck once
        cfg = wl.ecology_desc(eco=dict(HAND, attack_damage=50), width=2, height=5, n_agents_init=0, capacity=4,
                              window=1, hidden1=32, hidden2=32, resource_density=0.0, regrow_prob=0.0, seed=1,
                              e_eat=10, e_cost=1, e_repro=200, e_child=50, attack_enabled=1)
        st = empty_state(2, 5, 4, ecology=True, uid_next=100)
        for slot, (x, y) in enumerate([(0, 4), (1, 2), (0, 0)]):
            place(st, 2, slot, x, y, N, 100)
            st["water"][slot], st["biomass"][slot], st["hp"][slot] = 30, 2, 100
        return cfg, st, [ATK, 0, 0, 0]
    if name == "wall":          # a wall does not shield (no line of sight)
        _put(st, 0, 2, 4, N, 100, 30, 2, 100); _put(st, 1, 2, 1, N, 100, 30, 2, 100)
        st["wall"][3 * 6 + 2] = 1
        return _hand_cfg(100), st, [ATK, 0, 0, 0]
    raise ValueError(name)


@pytest.mark.parametrize("case", ["full", "half", "quarter", "moves", "wall", "narrow"])
def test_hand_built(eco, case):
    cfg, st, acts = _case(case)
    ow, gw = orc.OracleWorld(cfg), eco.World(cfg)
    ow.write_state(st)
    gw.write_state(st)
    gw.set_flags(eco.RT_KEEP_LOGITS)
    assert_same_state(gw.read_state(), ow.state(), f"{case} written")
    a = np.array(acts, np.uint8)
    lo, _ = ow.step(actions=a, want_logits=True)
    gw.step_with_actions(a)
    assert_same_state(gw.read_state(), ow.state(), case)
    assert_stats_match(gw.stats()[0], ow.stats(), case)
    assert gw.stats()[0]["killed"] >= (case != "narrow") and gw.stats()[0]["action_hist"][ATK] >= 1
    if case == "narrow":
        assert gw.read_state()["hp"][1] == 60   # one half-strength strike, then healing
    gl = gw.read_logits()
    assert gl.shape == (4, 9)
    live = ~np.isnan(lo[:, 0])
    np.testing.assert_allclose(gl[live], lo[live], rtol=0, atol=1e-5 * max(1.0, float(np.abs(lo[live]).max())))
    assert np.all(np.isnan(gl[~live]))
    gw.close()


def _world(seed=0, wdtype=0, damage=100, **kw):
    """96x80 torus, 450 agents, 11x11 window, 492->64->64->9: several policy tiles and a ragged tail."""
    d = wl.ecology_desc(eco=dict(w_cost=2, age_shift=5, w_init=20, w_child=8, attack_damage=damage), width=96,
                        height=80, n_agents_init=450, capacity=700, mutation_sigma=0.01, window=11, n_scalars=12,
                        hidden1=64, hidden2=64, wdtype=wdtype, seed=seed, e_init=230, attack_enabled=1)
    d.update(kw)
    return d


@pytest.mark.parametrize("wdtype,strength", [(0, "full"), (0, "half"), (0, "quarter"), (1, "half"), (2, "full")])
def test_seeded_actions(eco, wdtype, strength):
    seed = 300 + 10 * wdtype + len(strength)
    cfg = _world(seed=seed, wdtype=wdtype, damage=STRENGTHS[strength])
    acts = lambda t: wl.biased_actions(cfg["capacity"], 9, seed, t, p_forward=0.3, p_eat=0.3, p_attack=0.12)
    run_pair(eco, cfg, 20, actions_fn=acts, what=f"ecology attack {strength} wdtype {wdtype}", every=4)
    ow = orc.OracleWorld(cfg, materialize=False)
    tot = dict(births=0, deaths=0, killed=0, eaten=0)
    for t in range(20):
        ow.step(actions=acts(t))
        for k in tot:
            tot[k] += ow.stats()[k]
    say(f"ecology attack {strength} wdtype {wdtype}: {tot}")
    assert all(v > 0 for v in tot.values()), tot


def test_policy_actions(eco):
    cfg = _world(seed=395, e_init=260, damage=50)
    _, mism = run_pair(eco, cfg, 10, what="ecology attack free-running")
    assert mism <= 3


@pytest.mark.parametrize("window,hidden,wdtype,launch", [(1, 32, 0, (4, 2, 4)), (3, 64, 1, (2, 4, 8)),
                                                         (15, 32, 2, (8, 2, 16)), (7, 128, 0, (4, 2, 8)),
                                                         (7, 128, 1, (8, 2, 16)), (5, 128, 2, (2, 4, 4))])
def test_shapes(eco, window, hidden, wdtype, launch):
    """Windows 1..15, hidden widths 32..128 (the ninth row's lane split differs per
    width), every storage type, several launch shapes."""
    cfg = wl.ecology_desc(eco=dict(w_cost=2, age_shift=4, attack_damage=50), width=23, height=19,
                          n_agents_init=70, capacity=130, window=window, n_scalars=12, hidden1=hidden, hidden2=hidden,
                          wdtype=wdtype, seed=window + hidden, e_init=230, mutation_sigma=0.05, attack_enabled=1)
    acts = lambda t: wl.biased_actions(cfg["capacity"], 9, window + hidden, t, p_forward=0.3, p_eat=0.3,
                                       p_attack=0.15)
    run_pair(eco, cfg, 8, actions_fn=acts, launch=launch,
             what=f"ecology attack S={window} H={hidden} wdtype {wdtype} launch {launch}")


def test_graph_eager_and_timed_graph_agree(eco):
    cfg = _world(seed=397, damage=25)
    a, b, c = eco.World(cfg), eco.World(cfg), eco.World(cfg)
    b.set_flags(0)
    c.set_flags(eco.RT_USE_GRAPH | eco.RT_TIME_KERNELS)
    a.step(25)
    b.step(25)
    for n in (10, 15):
        c.step(n)
    assert_same_state(a.read_state(), b.read_state(), "graph vs eager")
    assert_same_state(a.read_state(), c.read_state(), "graph vs timed graph")
    assert a.stats() == b.stats() == c.stats()
    hist = a.stats_history(0, 26)
    assert sum(h["action_hist"][ATK] for h in hist[1:]) > 0
    for w in (a, b, c):
        w.close()


def test_multi_world_strengths(eco):
    """Three attack worlds of uneven size in one object, at full, half and quarter
    strength, stepped together under seeded actions; each against its own oracle."""
    cfgs = [_world(seed=400 + i, damage=dmg, width=w, height=h, n_agents_init=n, capacity=cap)
            for i, (dmg, w, h, n, cap) in enumerate([(100, 40, 30, 90, 160), (50, 96, 80, 450, 700),
                                                     (25, 17, 23, 40, 64)])]
    gw = eco.World(cfgs)
    ows = [orc.OracleWorld(c) for c in cfgs]
    killed = [0, 0, 0]
    for t in range(10):
        acts = [wl.biased_actions(c["capacity"], 9, 400 + i, t, p_forward=0.3, p_eat=0.3, p_attack=0.15)
                for i, c in enumerate(cfgs)]
        for ow, a in zip(ows, acts):
            ow.step(actions=a)
        gw.step_with_actions(np.concatenate(acts))
        stats = gw.stats()
        for i, ow in enumerate(ows):
            assert_stats_match(stats[i], ow.stats(), f"world {i} step {t}")
            killed[i] += stats[i]["killed"]
            if t % 3 == 2:
                compare_world(gw, ow, f"world {i} step {t}", world=i, weights_slots=2)
    say(f"kills at full / half / quarter strength: {killed}")
    assert all(k > 0 for k in killed)
    gw.close()


def test_conservation_free_running_full_size(eco):
    """The 1024x1024 ecology with 65,536 agents and full-strength attacks,
    free-running for 40 steps: water and biomass totals never change,
    N' = N + births - deaths, killed <= deaths, one agent per cell."""
    cfg = wl.ecology_desc(width=1024, height=1024, n_agents_init=65536, capacity=131072, window=11, n_scalars=12,
                          hidden1=64, hidden2=64, mutation_sigma=0.01, e_init=230, seed=5, attack_enabled=1)
    gw = eco.World(cfg)
    s0 = gw.stats()[0]
    gw.step(40)
    hist = gw.stats_history(0, 41)
    for prev, h in zip(hist, hist[1:]):
        assert h["water_total"] == s0["water_total"] and h["biomass_total"] == s0["biomass_total"]
        assert h["population"] == prev["population"] + h["births"] - h["deaths"]
        assert h["killed"] <= h["deaths"]
    st = gw.read_state()
    check_invariants(st, 1024, 1024)
    live = st["alive"].astype(bool)
    assert np.all((st["hp"][live] > 0) & (st["hp"][live] <= cfg["eco"]["hp_max"]))
    attacks = sum(h["action_hist"][ATK] for h in hist[1:])
    kills = sum(h["killed"] for h in hist[1:])
    say(f"ecology attack 65k: {attacks} attacks, {kills} kills, population {hist[0]['population']} -> "
        f"{hist[-1]['population']}")
    assert attacks > 0 and kills > 0
    gw.close()


def test_long_run_half_strength(eco):
    """The 65,536-agent ecology with half-strength attacks free-running for 300
    steps (the policies' own actions, births mutating the nine-logit heads), with
    no energy or water costs and no overspend or age damage, so that strikes are
    the only harm and the population lives on (≈84k at its peak, ≈32k at the end,
    ≈95k kills): every death is a kill; conservation and bookkeeping every step
    from the statistics ring; the integer state's invariants at the end."""
    e = dict(attack_damage=wl.ATTACK_HALF, e_cost_move=0, w_cost=0, hp_overspend=0, age_shift=31)
    cfg = wl.ecology_desc(eco=e, width=1024, height=1024, n_agents_init=65536, capacity=131072, window=11,
                          n_scalars=12, hidden1=64, hidden2=64, mutation_sigma=0.01, e_init=230, e_cost=0, seed=11,
                          attack_enabled=1)
    gw = eco.World(cfg)
    s0 = gw.stats()[0]
    gw.step(300)
    hist = gw.stats_history(0, 301)
    assert len(hist) == 301 and hist[-1]["step"] == 300
    for prev, h in zip(hist, hist[1:]):
        assert h["water_total"] == s0["water_total"] and h["biomass_total"] == s0["biomass_total"]
        assert h["population"] == prev["population"] + h["births"] - h["deaths"]
        assert h["killed"] == h["deaths"] and sum(h["action_hist"]) == prev["population"]
    st = gw.read_state()
    check_invariants(st, 1024, 1024)
    live = st["alive"].astype(bool)
    assert np.all((st["hp"][live] > 0) & (st["hp"][live] <= cfg["eco"]["hp_max"]))
    assert int(st["cell_biomass"].sum()) + int(st["biomass"][live].sum()) == s0["biomass_total"]
    kills = sum(h["killed"] for h in hist[1:])
    births = sum(h["births"] for h in hist[1:])
    say(f"ecology half-strength attack, 300 steps: population {hist[0]['population']} -> {hist[-1]['population']}, "
        f"{births} births, {kills} kills")
    assert kills > 10000 and births > 10000 and hist[-1]["population"] > 1000
    gw.close()


@pytest.mark.parametrize("attack,wdtype", [(0, 0), (0, 1), (1, 0), (1, 2)])
def test_evolving_temperature(eco, attack, wdtype):
    """The paper's evolving softmax temperature in the ecology: its parameter follows
    the eight output biases (read as the ninth logit of a zero weight row) or the
    nine (bias slot 9); births mutate it with the weights.  Seeded actions, then the
    policies' own tempered samples."""
    seed = 500 + 10 * attack + wdtype
    cfg = _world(seed=seed, wdtype=wdtype, damage=50, flags=8 | 2)
    if not attack:
        cfg.update(attack_enabled=0, n_actions=8)
    A = cfg["n_actions"]
    acts = lambda t: wl.biased_actions(cfg["capacity"], A, seed, t, p_forward=0.3, p_eat=0.3, p_attack=0.1)
    run_pair(eco, cfg, 12, actions_fn=acts, what=f"ecology temperature A={A} wdtype {wdtype}", every=3)
    _, mism = run_pair(eco, dict(cfg, seed=seed + 1, e_init=260), 6, what=f"ecology temperature A={A} sampled")
    assert mism <= 3


def test_errors(eco):
    e = dict(wl.ECOLOGY)
    for bad in [dict(n_actions=9, n_scalars=8, flags=8, eco=e),                          # nine without attack
                dict(n_actions=9, n_scalars=8, attack_enabled=1),                         # nine without the ecology
                dict(n_actions=8, n_scalars=8, flags=8, attack_enabled=1, eco=e),         # attack needs nine
                dict(n_actions=9, n_scalars=8, flags=8, attack_enabled=1, eco=dict(e, attack_damage=-1))]:
        with pytest.raises(eco.EcoError) as err:
            eco.World(wl.desc(**bad))
        assert err.value.status == eco.ECO_EINVAL, bad

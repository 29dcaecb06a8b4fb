"""The three-resource ecology with health on the GPU against the oracle (Sec. 3.2
"Resources" and health points; App. "Varying Resource Rules", "Varying Agent
HP"): water, energy and biomass on the grid and in capped stomachs, the three eat
actions, energy and water costs, overspend and age damage, healing, death that
returns what is carried, reproduction with spare biomass, photosynthesis.
Integer state (stomachs, health, the three grid layers) bit-exact; statistics
(water and biomass totals, health total) equal; logits within the FP32
tolerance.  The hand-built cases are the oracle's hand-traced ecology pins,
replayed through the C ABI.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2510_18221_amd import workloads as wl

from gpu_util import assert_stats_match, compare_world, need_gpu, run_pair, say
from worldstate import N, E, S, W, assert_same_state, check_invariants, empty_state, place

pytestmark = pytest.mark.gpu

HAND = dict(water_density=0.0, energy_density=0.0, biomass_density=0.0, water_site=0, energy_site=0, biomass_site=0,
            eat_water=10, eat_biomass=1, cap_water=60, cap_energy=400, cap_biomass=8, e_cost_move=2, w_cost=3,
            photo_rate=0.0, cell_energy_max=40, hp_max=100, hp_child=50, hp_overspend=20, hp_heal=10, heal_energy=1,
            age_shift=31, w_init=30, b_init=2, w_child=10, b_child=1, b_repro=2)


@pytest.fixture(scope="module")
def eco():
    need_gpu()
    from paper_2510_18221_amd import eco as m
    m.lib()
    return m


def _hand_cfg(**e):
    return wl.ecology_desc(eco=dict(HAND, **e), width=6, height=6, n_agents_init=0, capacity=4, window=3,
                           hidden1=32, hidden2=32, resource_density=0.0, regrow_prob=0.0, seed=1, e_eat=10, e_cost=1,
                           e_repro=200, e_child=50)


def _put(st, slot, x, y, f, E_, W_, B_, hp, age=0):
    place(st, 6, slot, x, y, f, E_, age=age)
    st["water"][slot], st["biomass"][slot], st["hp"][slot] = W_, B_, hp


def _c(x, y):
    return y * 6 + x


def _case(name):
    st = empty_state(6, 6, 4, ecology=True, uid_next=100)
    cfg = _hand_cfg()
    if name == "eat":
        _put(st, 0, 1, 1, N, 395, 30, 2, 100); _put(st, 1, 3, 1, N, 100, 55, 2, 100)
        _put(st, 2, 1, 3, N, 100, 30, 7, 100); _put(st, 3, 3, 3, N, 100, 30, 2, 100)
        st["cell_energy"][_c(1, 1)] = 20; st["cell_water"][_c(3, 1)] = 20; st["cell_biomass"][_c(1, 3)] = 3
        acts = [4, 5, 6, 0]
    elif name == "damage":
        cfg = _hand_cfg(age_shift=2)
        _put(st, 0, 1, 1, N, 1, 1, 3, 30); _put(st, 1, 3, 1, N, 1, 0, 3, 30)
        _put(st, 2, 1, 3, N, 50, 30, 2, 75, age=8); _put(st, 3, 3, 3, N, 300, 30, 2, 100, age=3)
        acts = [0, 4, 0, 0]
    elif name == "birth":
        _put(st, 0, 2, 2, N, 250, 30, 2, 100); _put(st, 2, 4, 4, N, 250, 30, 1, 100)
        _put(st, 3, 0, 0, N, 250, 5, 2, 100)
        acts = [7, 0, 7, 7]
    elif name == "photosynthesis":
        cfg = _hand_cfg(photo_rate=0.5)
        _put(st, 0, 0, 0, N, 100, 30, 2, 100)
        st["cell_biomass"][_c(2, 2)] = 2; st["cell_biomass"][_c(4, 4)] = 3; st["cell_energy"][_c(4, 4)] = 40
        st["cell_energy"][_c(1, 4)] = 7
        acts = [0, 0, 0, 0]
    elif name == "walls":   # a wall ahead blocks the move and stays out of the window's channels
        _put(st, 0, 1, 1, E, 100, 30, 2, 100)
        st["wall"][_c(2, 1)] = 1
        acts = [3, 0, 0, 0]
    return cfg, st, acts


@pytest.mark.parametrize("case", ["eat", "damage", "birth", "photosynthesis", "walls"])
def test_hand_built(eco, case):
    cfg, st, acts = _case(case)
    ow, gw = orc.OracleWorld(cfg), eco.World(cfg)
    ow.write_state(st)
    gw.write_state(st)
    gw.set_flags(eco.RT_KEEP_LOGITS)
    assert_same_state(gw.read_state(), ow.state(), f"{case} written")
    assert_stats_match(gw.stats()[0], ow.stats(), f"{case} written")
    a = np.array(acts, np.uint8)
    lo, _ = ow.step(actions=a, want_logits=True)
    gw.step_with_actions(a)
    assert_same_state(gw.read_state(), ow.state(), case)
    assert_stats_match(gw.stats()[0], ow.stats(), case)
    gl = gw.read_logits()
    live = ~np.isnan(lo[:, 0])
    np.testing.assert_allclose(gl[live], lo[live], rtol=0, atol=1e-5 * max(1.0, float(np.abs(lo[live]).max())))
    gw.close()


def _world(seed=0, wdtype=0, **kw):
    """96x80 torus, 450 agents, 11x11 window, 492->64->64->8: several policy tiles and a ragged tail."""
    d = wl.ecology_desc(eco=dict(w_cost=2, age_shift=5, w_init=20, w_child=8), width=96, height=80,
                        n_agents_init=450, capacity=700,
                        mutation_sigma=0.01, window=11, n_scalars=12, hidden1=64, hidden2=64, wdtype=wdtype, seed=seed,
                        e_init=230)
    d.update(kw)
    return d


@pytest.mark.parametrize("wdtype", [0, 1, 2])
def test_seeded_actions(eco, wdtype):
    cfg = _world(seed=90 + wdtype, wdtype=wdtype)
    acts = lambda t: wl.biased_actions(cfg["capacity"], 8, 90 + wdtype, t, p_forward=0.3, p_eat=0.35)
    ow = orc.OracleWorld(cfg)
    tot = dict(births=0, deaths=0, eaten=0, regrown=0)
    run_pair(eco, cfg, 20, actions_fn=acts, what=f"ecology wdtype {wdtype}", every=4)
    for t in range(20):
        ow.step(actions=acts(t))
        for k in tot:
            tot[k] += ow.stats()[k]
    say(f"ecology wdtype {wdtype}: {tot}")
    assert all(v > 0 for v in tot.values()), tot


def test_policy_actions(eco):
    cfg = _world(seed=95, e_init=260)
    _, mism = run_pair(eco, cfg, 10, what="ecology free-running")
    assert mism <= 3


@pytest.mark.parametrize("window,n_scalars,launch", [(1, 8, (4, 2, 4)), (3, 12, (2, 4, 8)), (15, 8, (8, 2, 16)),
                                                     (15, 12, (4, 4, 4))])
def test_window_sizes(eco, window, n_scalars, launch):
    cfg = wl.ecology_desc(eco=dict(w_cost=2, age_shift=4), width=23, height=19, n_agents_init=70, capacity=130,
                          window=window, n_scalars=n_scalars, hidden1=32, hidden2=32, seed=window + n_scalars,
                          e_init=230, mutation_sigma=0.05)
    acts = lambda t: wl.biased_actions(cfg["capacity"], 8, window + n_scalars, t, p_forward=0.35, p_eat=0.35)
    run_pair(eco, cfg, 8, actions_fn=acts, launch=launch, what=f"ecology S={window} ns={n_scalars} launch {launch}")


def test_graph_eager_and_timed_graph_agree(eco):
    cfg = _world(seed=97)
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
    for w in (a, b, c):
        w.close()


def test_conservation_free_running_full_size(eco):
    """The 1024x1024 world with 65,536 agents free-running for 60 steps: water and
    biomass totals never change, N' = N + births - deaths, one agent per cell."""
    cfg = wl.ecology_desc(width=1024, height=1024, n_agents_init=65536, capacity=131072, window=11, n_scalars=12,
                          hidden1=64, hidden2=64, mutation_sigma=0.01, e_init=230, seed=3)
    gw = eco.World(cfg)
    s0 = gw.stats()[0]
    gw.step(60)
    hist = gw.stats_history(0, 61)
    assert len(hist) == 61
    for prev, h in zip(hist, hist[1:]):
        assert h["water_total"] == s0["water_total"] and h["biomass_total"] == s0["biomass_total"]
        assert h["population"] == prev["population"] + h["births"] - h["deaths"]
    st = gw.read_state()
    check_invariants(st, 1024, 1024)
    live = st["alive"].astype(bool)
    e = cfg["eco"]
    assert np.all((st["hp"][live] > 0) & (st["hp"][live] <= e["hp_max"]))
    assert int(st["cell_water"].sum()) + int(st["water"][live].sum()) == s0["water_total"]
    assert hist[-1]["hp_total"] == int(st["hp"][live].sum())
    say(f"ecology 65k: population {hist[0]['population']} -> {hist[-1]['population']}, "
        f"births {sum(h['births'] for h in hist[1:])}, deaths {sum(h['deaths'] for h in hist[1:])}")
    gw.close()


def test_ecology_errors(eco):
    for bad in [dict(n_actions=8),
                dict(n_actions=8, n_scalars=8, flags=8, attack_enabled=1, eco=wl.ECOLOGY),
                dict(n_actions=7, n_scalars=8, flags=8, eco=wl.ECOLOGY),
                dict(n_actions=8, n_scalars=4, flags=8, eco=wl.ECOLOGY),
                dict(n_actions=8, n_scalars=8, flags=8, eco=dict(wl.ECOLOGY, hp_child=0))]:
        with pytest.raises(eco.EcoError) as e:
            eco.World(wl.desc(**bad))
        assert e.value.status == eco.ECO_EINVAL, bad
    gw = eco.World(wl.ecology_desc(seed=4))
    st = gw.read_state()
    st["cell_water"][5] = -1
    with pytest.raises(eco.EcoError):
        gw.write_state(st)
    gw.close()


# ---------------------------------------------------------------------------
# Terrain: rock layer, sea, downhill water flow; colour windows in the ecology
# with the elevation channel
# ---------------------------------------------------------------------------
TERRAIN, COLOUR = 16, 4


def _terrain_world(seed, flags, wdtype=0, **kw):
    d = _world(seed=seed, wdtype=wdtype, flags=8 | flags)
    d["eco"] = dict(d["eco"], terrain_scale=12, sea_level=12, water_per_depth=3)
    d.update(kw)
    return d


@pytest.mark.parametrize("size,scale", [((96, 80), 12), ((33, 17), 5), ((64, 64), 200)])
def test_terrain_generator_parity(eco, size, scale):
    cfg = _terrain_world(7, TERRAIN, width=size[0], height=size[1], n_agents_init=40, capacity=64)
    cfg["eco"]["terrain_scale"] = scale
    ow, gw = orc.OracleWorld(cfg, materialize=False), eco.World(cfg)
    np.testing.assert_array_equal(gw.read_terrain(), ow.terrain())
    assert_same_state(gw.read_state(), ow.state(), "init")   # the sea's water included
    gw.close()


def test_flow_hand_traced(eco):
    cfg = wl.ecology_desc(eco=dict(HAND, terrain_scale=6, sea_level=0, water_per_depth=3), flags=8 | TERRAIN,
                          width=6, height=6, n_agents_init=0, capacity=4, window=3, hidden1=32, hidden2=32, seed=1,
                          e_eat=10, e_cost=1, e_repro=200, e_child=50)
    rock = np.full((6, 6), 10, np.int32)
    rock[2, 2] = 5; rock[2, 3] = 7; rock[3, 2] = 5; rock[0, 4] = 9; rock[1, 5] = 9
    st = empty_state(6, 6, 4, ecology=True)
    _put(st, 0, 0, 5, N, 100, 30, 2, 100)
    cw = np.zeros((6, 6), np.int32)
    cw[2, 3] = 12; cw[2, 2] = 4; cw[1, 2] = 5; cw[1, 4] = 7; cw[4, 4] = 2
    st["cell_water"] = cw.reshape(-1)
    ow, gw = orc.OracleWorld(cfg), eco.World(cfg)
    for w in (ow, gw):
        w.write_terrain(rock.reshape(-1))
        w.write_state(st)
    for t in range(3):
        a = np.zeros(4, np.uint8)
        ow.step(actions=a)
        gw.step_with_actions(a)
        assert_same_state(gw.read_state(), ow.state(), f"flow step {t}")
        assert_stats_match(gw.stats()[0], ow.stats(), f"flow step {t}")
    assert gw.read_state()["cell_water"].reshape(6, 6)[2, 2] == 21
    with pytest.raises(eco.EcoError):
        gw.write_terrain(np.full(36, 40, np.int32))
    gw.close()


@pytest.mark.parametrize("flags,wdtype", [(TERRAIN, 0), (TERRAIN | COLOUR, 0), (TERRAIN | COLOUR, 2), (COLOUR, 1),
                                          (TERRAIN | COLOUR | 1, 0)])
def test_terrain_seeded_actions(eco, flags, wdtype):
    """Seeded actions on the 96x80 world with terrain (water flowing) and/or colour
    windows (with the elevation channel), several policy tiles and a ragged tail."""
    cfg = _terrain_world(100 + flags, flags, wdtype=wdtype)
    acts = lambda t: wl.biased_actions(cfg["capacity"], 8, 100 + flags, t, p_forward=0.3, p_eat=0.35)
    run_pair(eco, cfg, 15, actions_fn=acts, what=f"terrain flags {flags} wdtype {wdtype}", every=3)


def test_terrain_policy_actions(eco):
    cfg = _terrain_world(120, TERRAIN | COLOUR, e_init=260)
    _, mism = run_pair(eco, cfg, 10, what="terrain + colour free-running")
    assert mism <= 3


def test_terrain_graph_eager_agree_and_conserve(eco):
    cfg = _terrain_world(121, TERRAIN | COLOUR)
    a, b = eco.World(cfg), eco.World(cfg)
    b.set_flags(0)
    s0 = a.stats()[0]
    a.step(30)
    b.step(30)
    assert_same_state(a.read_state(), b.read_state(), "graph vs eager")
    assert a.stats() == b.stats()
    for h in a.stats_history(0, 31):
        assert h["water_total"] == s0["water_total"] and h["biomass_total"] == s0["biomass_total"]
    a.close()
    b.close()


def test_terrain_errors(eco):
    with pytest.raises(eco.EcoError) as e:
        eco.World(wl.desc(flags=TERRAIN))
    assert e.value.status == eco.ECO_EINVAL
    with pytest.raises(eco.EcoError) as e:
        eco.World(wl.ecology_desc(flags=8 | TERRAIN, eco=dict(wl.ECOLOGY, terrain_scale=0)))
    assert e.value.status == eco.ECO_EINVAL
    gw = eco.World(wl.ecology_desc(seed=5))
    with pytest.raises(eco.EcoError):
        gw.read_terrain()
    gw.close()


def test_multi_world_ecology_object(eco):
    """Four ecology worlds of uneven size in one object, each with its own
    parameters (costs, caps, photosynthesis rate, sea level, terrain scale), stepped
    together; each against its own oracle, statistics every step, full state and
    sampled weights every other step."""
    base = _terrain_world(0, TERRAIN | COLOUR)
    cfgs = []
    for i, (w, h, n, cap) in enumerate([(40, 30, 70, 128), (96, 80, 450, 700), (17, 23, 20, 64), (60, 60, 200, 320)]):
        d = dict(base, width=w, height=h, n_agents_init=n, capacity=cap, seed=200 + i)
        d["eco"] = dict(base["eco"], w_cost=1 + i % 2, photo_rate=0.01 * (i + 1), cap_water=60 + 20 * i,
                        sea_level=8 + 2 * i, terrain_scale=5 + 3 * i, age_shift=4 + i)
        cfgs.append(d)
    gw = eco.World(cfgs)
    ows = [orc.OracleWorld(c) for c in cfgs]
    for i, ow in enumerate(ows):
        np.testing.assert_array_equal(gw.read_terrain(i), ow.terrain())
        compare_world(gw, ow, f"world {i} init", world=i, weights_slots=2)
    for t in range(10):
        acts = [wl.biased_actions(c["capacity"], 8, 200 + i, t, p_forward=0.3, p_eat=0.35) for i, c in enumerate(cfgs)]
        for ow, a in zip(ows, acts):
            ow.step(actions=a)
        gw.step_with_actions(np.concatenate(acts))
        stats = gw.stats()
        for i, ow in enumerate(ows):
            assert_stats_match(stats[i], ow.stats(), f"world {i} step {t}")
            if t % 2:
                compare_world(gw, ow, f"world {i} step {t}", world=i, weights_slots=2)
    gw.close()

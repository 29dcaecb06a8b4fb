"""Parity of the HIP world step (libeco.so through its C ABI) with the CPU oracle.

Integer world state must match bit for bit given identical actions; FP32
logits within 1e-5 normwise relative of the oracle's FP64 logits on the same
stored weights; weights within a few FP32 ulps.  Actions always come from the
oracle or from the seeded input generators, never from the GPU.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2510_18221_amd import workloads as wl

from gpu_util import LOGIT_TOL, assert_stats_match, assert_weights_close, compare_world, logit_err, need_gpu, run_pair, say
from worldstate import N, E, S, W, assert_same_state, check_invariants, empty_state, place

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eco():
    need_gpu()
    from paper_2510_18221_amd import eco as m
    m.lib()
    return m


def mid_world(seed=0, wdtype=0, **kw):
    """Several forward tiles and a ragged tail: 96x80 torus, 11x11 window, 64-wide MLP."""
    d = wl.desc(width=96, height=80, n_agents_init=450, capacity=700, resource_density=0.3, regrow_prob=0.02,
                mutation_sigma=0.01, window=11, n_scalars=8, hidden1=64, hidden2=64, n_actions=7, wdtype=wdtype,
                seed=seed, e_init=170)
    d.update(kw)
    return d


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_small_world_100_steps_oracle_actions(eco, seed):
    """64x64, 256 agents, D=104, 104->32->32->5 FP32, sigma 0.02: 100 steps."""
    cfg = wl.world_small(seed=seed)
    _, mism = run_pair(eco, cfg, 100, what=f"small seed {seed}", every=5)
    assert mism <= 3


@pytest.mark.parametrize("wdtype", [0, 1, 2])
def test_mid_world_births_and_deaths(eco, wdtype):
    cfg = mid_world(seed=5, wdtype=wdtype)
    acts = lambda t: wl.biased_actions(cfg["capacity"], 7, 5, t)
    run_pair(eco, cfg, 25, actions_fn=acts, what=f"mid wdtype {wdtype}", every=4)


def test_mid_world_free_running_logits(eco):
    cfg = mid_world(seed=9, e_init=100)
    run_pair(eco, cfg, 8, what="mid free-running")


def test_capacity_pressure_and_extinction(eco):
    cfg = mid_world(seed=3, capacity=456, e_init=199, resource_density=1.0)
    acts = lambda t: wl.biased_actions(cfg["capacity"], 7, 3, t, p_forward=0.1, p_eat=0.6)
    run_pair(eco, cfg, 6, actions_fn=acts, what="capacity", check_logits=False)
    cfg = mid_world(seed=3, e_init=2, e_eat=0)
    run_pair(eco, cfg, 4, actions_fn=lambda t: np.zeros(cfg["capacity"], np.uint8), what="extinction",
             check_logits=False)


def test_multi_world_object(eco):
    """Worlds of uneven size in one object, each against its own oracle."""
    cfgs = [mid_world(seed=s, width=w, height=h, n_agents_init=n, capacity=c)
            for s, (w, h, n, c) in enumerate([(40, 30, 70, 128), (96, 80, 450, 700), (17, 23, 20, 64),
                                               (60, 60, 200, 320)])]
    gw = eco.World(cfgs)
    gw.set_flags(eco.RT_KEEP_LOGITS)
    ows = [orc.OracleWorld(c) for c in cfgs]
    for i, ow in enumerate(ows):
        compare_world(gw, ow, f"world {i} init", world=i)
    for t in range(12):
        acts = [wl.biased_actions(c["capacity"], 7, i, t) for i, c in enumerate(cfgs)]
        outs = [ow.step(actions=a, want_logits=True) for ow, a in zip(ows, acts)]
        pre = [ow for ow in ows]
        gw.step_with_actions(np.concatenate(acts))
        for i, ow in enumerate(ows):
            compare_world(gw, ow, f"world {i} step {t}", world=i, weights_slots=2)
            assert_stats_match(gw.stats()[i], ow.stats(), f"world {i} step {t}")
            gl = gw.read_logits(i)
            ok = ~np.isnan(gl[:, 0])
            assert logit_err(gl[ok], outs[i][0][ok]).max(initial=0) <= LOGIT_TOL
    gw.close()


def test_determinism_and_launch_shapes(eco):
    """Free-running GPU worlds: same seed, any launch shape -> identical state."""
    cfg = mid_world(seed=4, e_init=150)
    ref = None
    for lc in [(4, 4, 8), (1, 16, 4), (8, 2, 16), (2, 8, 8)]:
        gw = eco.World(cfg)
        gw.set_launch(*lc)
        gw.step(30)
        st = gw.read_state()
        hist = gw.stats_history(0, 31)
        gw.close()
        if ref is None:
            ref = (st, hist)
        else:
            assert_same_state(st, ref[0], f"launch {lc}")
            assert hist == ref[1]


def test_graph_and_eager_paths_agree(eco):
    cfg = mid_world(seed=6, e_init=150)
    a = eco.World(cfg)
    b = eco.World(cfg)
    c = eco.World(cfg)
    b.set_flags(0)  # eager
    c.set_flags(eco.RT_USE_GRAPH | eco.RT_TIME_KERNELS)  # graphs of whole runs, events around the policy kernel
    c.prepare(7)
    a.step(20)
    b.step(20)
    for n in (7, 7, 6):
        c.step(n)
    assert_same_state(a.read_state(), b.read_state(), "graph vs eager")
    assert_same_state(a.read_state(), c.read_state(), "graph vs timed graph")
    assert a.stats() == b.stats() == c.stats()
    kt = c.kernel_times()
    assert kt["forward"][1] == 20 and kt["forward"][0] > 0.0 and kt["compact"][1] == 0
    for w in (a, b, c):
        w.close()


@pytest.mark.parametrize("split", [False, True], ids=["fused", "split"])
def test_step_graph_chunks_agree_with_eager(eco, split):
    """eco_world_step under ECO_RT_USE_GRAPH runs n steps as 32-step graphs and one
    of the remainder: step counts across the chunk boundary, more distinct counts
    than the graphs kept (the oldest is dropped and rebuilt), and a flag change
    between calls all give the eager path's state and statistics (the small
    world's fused step, and its separate kernels)."""
    cfg = mid_world(seed=8, e_init=150)
    extra = eco.RT_SPLIT_STEP if split else 0
    a = eco.World(cfg)
    b = eco.World(cfg)
    a.set_flags(eco.RT_USE_GRAPH | extra)
    b.set_flags(extra)
    counts = (70, 1, 33, 5, 2, 3, 32, 4)
    for i, n in enumerate(counts):
        if i == 4:   # a flag change drops the built graphs
            a.set_flags(eco.RT_USE_GRAPH | eco.RT_KEEP_LOGITS | extra)
            b.set_flags(eco.RT_KEEP_LOGITS | extra)
        a.step(n)
        b.step(n)
    assert_same_state(a.read_state(), b.read_state(), "step graphs vs eager")
    assert a.stats() == b.stats()
    h = a.stats_history(0, 150)
    assert h == b.stats_history(0, 150) and h[-1]["step"] == sum(counts)
    assert np.array_equal(a.read_logits(), b.read_logits(), equal_nan=True)
    for w in (a, b):
        w.close()


def test_resume_from_state_and_weights(eco):
    cfg = mid_world(seed=7, e_init=150)
    a = eco.World(cfg)
    a.step(15)
    st = a.read_state()
    live = np.nonzero(st["alive"])[0]
    masters = {int(s): a.read_weights(int(s), master=True).astype(np.float32) for s in live}
    b = eco.World(cfg)
    b.write_state(st)
    for s, m in masters.items():
        b.write_weights(s, m)
    a.step(15)
    b.step(15)
    assert_same_state(a.read_state(), b.read_state(), "resume")
    a.close()
    b.close()


# ---------------------------------------------------------------------------
# Hand-built states on the GPU, against the oracle
# ---------------------------------------------------------------------------
def _tiny(**kw):
    c = wl.desc(width=5, height=5, n_agents_init=0, capacity=4, window=3, n_scalars=4, hidden1=32, hidden2=32,
                n_actions=5, resource_density=0.0, regrow_prob=0.0, seed=1)
    c.update(kw)
    return c


@pytest.mark.parametrize("case", ["contest", "chain", "wrap", "swap", "eat", "death_birth", "births", "conflict",
                                  "capacity", "regrow", "walls"])
def test_hand_built_cases(eco, case):
    cfg = _tiny()
    st = empty_state(5, 5, 4)
    acts = [0, 0, 0, 0]
    if case == "contest":
        place(st, 5, 0, 1, 1, E, 100); place(st, 5, 1, 3, 1, W, 100); acts = [3, 3, 0, 0]
    elif case == "chain":
        place(st, 5, 0, 0, 0, E, 100); place(st, 5, 1, 1, 0, E, 100); acts = [3, 3, 0, 0]
    elif case == "wrap":
        place(st, 5, 0, 4, 2, E, 100); acts = [3, 0, 0, 0]
    elif case == "swap":
        place(st, 5, 0, 1, 1, E, 100); place(st, 5, 1, 2, 1, W, 100); acts = [3, 3, 0, 0]
    elif case == "eat":
        place(st, 5, 0, 1, 1, N, 100); place(st, 5, 1, 3, 3, N, 100); st["res"][6] = 1; acts = [4, 4, 0, 0]
    elif case == "death_birth":
        cfg = _tiny(capacity=2)
        st = empty_state(5, 5, 2)
        place(st, 5, 0, 0, 0, N, 1); place(st, 5, 1, 2, 2, N, 300, uid=7); acts = [0, 0]
    elif case == "births":
        place(st, 5, 0, 1, 1, N, 201); place(st, 5, 2, 3, 3, E, 210)
    elif case == "conflict":
        place(st, 5, 0, 1, 0, N, 250); place(st, 5, 1, 1, 2, S, 250)
    elif case == "capacity":
        cfg = _tiny(capacity=2)
        st = empty_state(5, 5, 2)
        place(st, 5, 0, 1, 1, N, 250); place(st, 5, 1, 3, 3, N, 50); acts = [0, 0]
    elif case == "regrow":
        cfg = _tiny(regrow_prob=1.0)
        place(st, 5, 0, 0, 0, N, 100); st["res"][3] = 1
    elif case == "walls":
        place(st, 5, 0, 1, 1, E, 100); place(st, 5, 1, 3, 3, N, 250); acts = [3, 0, 0, 0]
        st["wall"][1 * 5 + 2] = 1; st["wall"][4 * 5 + 3] = 1
    ow = orc.OracleWorld(cfg)
    ow.write_state(st)
    gw = eco.World(cfg)
    gw.write_state(st)
    assert_same_state(gw.read_state(), ow.state(), f"{case} written")
    a = np.array(acts, np.uint8)
    ow.step(actions=a)
    gw.step_with_actions(a)
    assert_same_state(gw.read_state(), ow.state(), case)
    assert_stats_match(gw.stats()[0], ow.stats(), case)
    check_invariants(gw.read_state(), 5, 5)
    gw.close()


def test_errors(eco):
    with pytest.raises(eco.EcoError) as e:
        eco.World(wl.desc(window=4))
    assert e.value.status == eco.ECO_EINVAL
    with pytest.raises(eco.EcoError) as e:
        eco.World(wl.desc(hidden1=48, hidden2=48))
    assert e.value.status == eco.ECO_ENOTSUP
    with pytest.raises(eco.EcoError) as e:
        eco.World(wl.desc(attack_enabled=1))   # attacks need the seven-action head
    assert e.value.status == eco.ECO_EINVAL
    with pytest.raises(eco.EcoError):
        eco.World([wl.desc(), wl.desc(hidden1=64, hidden2=64)])
    gw = eco.World(wl.world_small())
    bad = np.full(4096, 9, np.uint8)
    with pytest.raises(eco.EcoError) as e:
        gw.step_with_actions(bad)
    assert e.value.status == eco.ECO_EINVAL
    st = gw.read_state()
    st["occ"][:] = -1
    with pytest.raises(eco.EcoError):
        gw.write_state(st)
    for field in ("res", "wall"):  # cells hold 0 or 1 of each (the sense byte has one bit per channel)
        st = gw.read_state()
        st[field][7] = 2
        with pytest.raises(eco.EcoError) as e:
            gw.write_state(st)
        assert e.value.status == eco.ECO_EINVAL
    gw.step(2)
    assert gw.stats()[0]["step"] == 2
    gw.close()


def test_stream_read_probe(eco):
    """The measurement helper: a plausible HBM read rate, and its argument checks."""
    g = eco.stream_read_gbps(1 << 30)
    assert 1000.0 < g < 8000.0, g
    with pytest.raises(eco.EcoError) as e:
        eco.stream_read_gbps(1 << 20)
    assert e.value.status == eco.ECO_EINVAL

"""The paper's own policy options on the GPU against the oracle (Sec. 3.3, Sec. 3.2
"Sensors", App. "Varying Vision Range"): the "Front" window, an evolving softmax
temperature (one more mutable parameter per agent, stored after the output
biases) and the colour trait rendered into others' windows.  Integer state
bit-exact, logits within the FP32 tolerance, the sampled actions of the
tempered softmax compared with the oracle's, weights (the log temperature
included) and colours within a few FP32 ulps.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2510_18221_amd import workloads as wl

from gpu_util import assert_stats_match, compare_world, need_gpu, run_pair, say
from worldstate import N, E, S, W, assert_same_state, empty_state, place

pytestmark = pytest.mark.gpu

FRONT, TEMP, COLOUR = 1, 2, 4


@pytest.fixture(scope="module")
def eco():
    need_gpu()
    from paper_2510_18221_amd import eco as m
    m.lib()
    return m


def _world(flags, seed=0, wdtype=0, **kw):
    """96x80 torus, 450 agents, 11x11 window, 492->64->64->7: several policy tiles and a ragged tail."""
    d = wl.desc(width=96, height=80, n_agents_init=450, capacity=700, resource_density=0.3, regrow_prob=0.02,
                mutation_sigma=0.2, window=11, n_scalars=8, hidden1=64, hidden2=64, n_actions=7, wdtype=wdtype,
                seed=seed, e_init=185, flags=flags)
    d.update(kw)
    return d


@pytest.mark.parametrize("flags,wdtype", [(FRONT, 0), (TEMP, 0), (TEMP, 1), (TEMP, 2), (COLOUR, 0), (COLOUR, 1),
                                          (COLOUR, 2), (FRONT | TEMP | COLOUR, 0), (FRONT | TEMP | COLOUR, 2)])
def test_seeded_actions(eco, flags, wdtype):
    """Seeded actions force moves, meals and births (so temperatures and colours mutate)."""
    cfg = _world(flags, seed=60 + flags, wdtype=wdtype)
    acts = lambda t: wl.biased_actions(cfg["capacity"], 7, 60 + flags, t)
    run_pair(eco, cfg, 12, actions_fn=acts, what=f"flags {flags} wdtype {wdtype}", every=3)


@pytest.mark.parametrize("flags", [FRONT, TEMP, COLOUR, FRONT | TEMP | COLOUR])
def test_policy_actions(eco, flags):
    """The policies' own samples (the oracle's draws injected); counts sampled-action mismatches."""
    cfg = _world(flags, seed=70 + flags, e_init=300, n_actions=5)
    _, mism = run_pair(eco, cfg, 10, what=f"flags {flags} free-running")
    assert mism <= 3


@pytest.mark.parametrize("window,flags,launch", [(1, FRONT, (4, 2, 4)), (1, FRONT | COLOUR, (8, 1, 16)),
                                                 (3, FRONT | COLOUR, (2, 4, 8)), (5, COLOUR | TEMP, (8, 4, 4)),
                                                 (15, FRONT | TEMP, (4, 4, 16)), (15, COLOUR, (8, 2, 8))])
def test_window_sizes(eco, window, flags, launch):
    cfg = wl.desc(width=23, height=19, n_agents_init=70, capacity=130, resource_density=0.35, regrow_prob=0.05,
                  mutation_sigma=0.2, window=window, n_scalars=8, hidden1=32, hidden2=32, n_actions=5,
                  seed=window * 10 + flags, e_init=205, flags=flags)
    acts = lambda t: wl.biased_actions(cfg["capacity"], 5, window + flags, t, p_forward=0.35, p_eat=0.35)
    run_pair(eco, cfg, 6, actions_fn=acts, launch=launch, what=f"S={window} flags {flags} launch {launch}")


def test_colour_write_is_seen(eco):
    """A colour written between steps shows in the next step's windows (logits of the
    neighbours change), on both sides alike."""
    cfg = wl.desc(width=9, height=9, n_agents_init=0, capacity=8, window=5, n_scalars=4, hidden1=32, hidden2=32,
                  n_actions=5, resource_density=0.0, regrow_prob=0.0, seed=3, flags=COLOUR)
    st = empty_state(9, 9, 8)
    place(st, 9, 0, 4, 4, N, 100)
    place(st, 9, 1, 4, 3, S, 100)
    place(st, 9, 2, 6, 4, W, 100)
    st["res"][2 * 9 + 3] = 1
    st["wall"][6 * 9 + 2] = 1
    ow, gw = orc.OracleWorld(cfg), eco.World(cfg)
    ow.write_state(st)
    gw.write_state(st)
    gw.set_flags(eco.RT_KEEP_LOGITS)
    for t, (slot, rgb) in enumerate([(1, [0.9, 0.1, 0.4]), (2, [-1.0, 2.0, 0.5]), (0, [0.25, 0.75, 0.125])]):
        ow.write_colour(slot, rgb)
        gw.write_colour(slot, rgb)
        compare_world(gw, ow, f"colour write {t}")
        a = np.zeros(8, np.uint8)
        lo, _ = ow.step(actions=a, want_logits=True)
        gw.step_with_actions(a)
        gl = gw.read_logits()
        for s in range(3):
            np.testing.assert_allclose(gl[s], lo[s], rtol=0, atol=1e-5 * max(1.0, np.abs(lo[s]).max()))
        assert_same_state(gw.read_state(), ow.state(), f"step {t}")
    gw.close()


def test_graph_eager_and_timed_graph_agree(eco):
    cfg = _world(FRONT | TEMP | COLOUR, seed=80, e_init=300, n_actions=5)
    a, b, c = eco.World(cfg), eco.World(cfg), eco.World(cfg)
    b.set_flags(0)
    c.set_flags(eco.RT_USE_GRAPH | eco.RT_TIME_KERNELS)
    a.step(15)
    b.step(15)
    for n in (5, 10):
        c.step(n)
    assert_same_state(a.read_state(), b.read_state(), "graph vs eager")
    assert_same_state(a.read_state(), c.read_state(), "graph vs timed graph")
    assert a.stats() == b.stats() == c.stats()
    np.testing.assert_array_equal(a.read_colours(), b.read_colours())
    live = np.nonzero(a.read_state()["alive"])[0]
    for s in live[:5]:
        np.testing.assert_array_equal(a.read_weights(int(s), master=True), c.read_weights(int(s), master=True))
    for w in (a, b, c):
        w.close()


def test_option_errors(eco):
    with pytest.raises(eco.EcoError) as e:
        eco.World(wl.desc(flags=8))
    assert e.value.status == eco.ECO_EINVAL
    with pytest.raises(eco.EcoError) as e:
        eco.World([wl.desc(), wl.desc(flags=COLOUR)])          # options differ between worlds
    assert e.value.status == eco.ECO_EINVAL
    gw = eco.World(wl.desc(seed=2))
    with pytest.raises(eco.EcoError):
        gw.read_colours()                                      # no colour trait
    gw.close()
    gw = eco.World(wl.desc(seed=2, flags=COLOUR, n_agents_init=10, capacity=16))
    with pytest.raises(eco.EcoError):
        gw.write_colour(12, [0.5, 0.5, 0.5])                   # slot not alive
    with pytest.raises(eco.EcoError):
        gw.write_colour(0, [np.nan, 0.5, 0.5])
    gw.close()
    gw = eco.World(wl.desc(seed=2, flags=TEMP))
    assert gw.P == orc.param_count(wl.desc(flags=TEMP)) == orc.param_count(wl.desc()) + 1
    gw.close()

"""eco_world_step_static (the allocation-free step) against eco_world_step.

Two objects with the same descriptor are stepped, one through eco_world_step (its
own scratch buffers, the replayed graph) and one through eco_world_step_static
(the library's static scratch array, eager launches): the same kernels on the
same inputs, so every integer state array, every statistic (the FP64 energy and
trait moments included), the logits' source weights and the live list must be
identical.  Two calls in a row on different objects, the second smaller, show
that what the first call left in the shared array does not leak into the second;
an object whose scratch exceeds the array is refused before anything runs.
"""
import numpy as np
import pytest

from gpu_util import need_gpu, say
from paper_2510_18221_amd import workloads as wl
from worldstate import assert_same_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eco():
    need_gpu()
    from paper_2510_18221_amd import eco as e
    e.lib()
    return e


def _pair_stepped(eco, cfg, steps, calls):
    """Objects a (eco_world_step) and b (eco_world_step_static) stepped `steps` times in `calls` calls."""
    a, b = eco.World(cfg), eco.World(cfg)
    per = steps // calls
    for _ in range(calls):
        a.step(per)
        b.step_static(per)
    return a, b


def _assert_identical(a, b, what, n_weights=6):
    for w in range(a.n_worlds):
        sa, sb = a.read_state(w), b.read_state(w)
        assert_same_state(sa, sb, f"{what} world {w}")   # per-slot fields compared on live slots
        live_mask = sa["alive"].astype(bool)
        assert np.array_equal(sa["action"][live_mask], sb["action"][live_mask]), (what, w, "action")
        ha, hb = a.stats_history(w, 1024), b.stats_history(w, 1024)
        assert ha == hb, (what, w)
        live = np.nonzero(sa["alive"])[0]
        for s in live[:: max(1, len(live) // n_weights)][:n_weights]:
            assert np.array_equal(a.read_weights(int(s), w, master=True), b.read_weights(int(s), w, master=True)), \
                (what, w, int(s))
            assert np.array_equal(a.read_weights(int(s), w), b.read_weights(int(s), w)), (what, w, int(s))
    return ha


def test_static_step_matches_step_on_two_calls_second_smaller(eco):
    # first call: a 96x80 world with attacks and a steady birth stream (every agent at the
    # threshold, zero-energy children dying at their first step: births and deaths every step),
    # BF16 storage, several slot and cell tiles and a ragged tail
    big = wl.desc(width=96, height=80, n_agents_init=450, capacity=1000, resource_density=0.3, regrow_prob=0.02,
                  mutation_sigma=0.01, window=11, n_scalars=8, hidden1=64, hidden2=64, n_actions=7,
                  wdtype=wl.BF16, seed=5, e_init=200, e_cost=0, e_child=0, attack_enabled=1)
    a, b = _pair_stepped(eco, big, 12, 3)
    hist = _assert_identical(a, b, "first call")
    births = sum(h["births"] for h in hist[1:])
    deaths = sum(h["deaths"] for h in hist[1:])
    say(f"static step, 96x80 world: {births} births, {deaths} deaths over 12 steps, identical")
    assert births > 100 and deaths > 100
    a.close()
    b.close()
    # second call: a smaller object of two worlds (the ecology, fewer tiles than the first)
    small = [wl.ecology_desc(width=24, height=20, n_agents_init=60, capacity=128, window=5, n_scalars=8, hidden1=32,
                             hidden2=32, mutation_sigma=0.05, e_init=260, seed=s) for s in (1, 2)]
    a, b = _pair_stepped(eco, small, 8, 2)
    hist = _assert_identical(a, b, "second call")
    say(f"static step, two 24x20 ecology worlds: {sum(h['births'] for h in hist[1:])} births in world 1")
    a.close()
    b.close()


def test_static_step_refuses_objects_above_the_array(eco):
    # 2.2M slots need ~17.7 MB of birth lists, above the 16 MiB array
    cfg = wl.desc(width=2, height=2, n_agents_init=1, capacity=2_200_000, window=1, n_scalars=4, hidden1=32,
                  hidden2=32, n_actions=5, seed=0)
    w = eco.World(cfg)
    before = w.read_state()
    with pytest.raises(eco.EcoError) as exc:
        w.step_static(1)
    assert exc.value.status == eco.ECO_EINVAL and "static" in str(exc.value)
    after = w.read_state()
    assert after["step"] == before["step"] and np.array_equal(after["alive"], before["alive"])
    w.step(1)   # the object itself is unaffected
    assert w.stats()[0]["step"] == 1
    w.close()

"""Edge cases of the HIP world step against the oracle: a world with no agents,
a world with one agent, and the largest object the library accepts (1024
worlds, each with its own seed and its own slot and cell ranges)."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2510_18221_amd import workloads as wl

from gpu_util import assert_stats_match, compare_world, need_gpu, run_pair
from worldstate import check_invariants

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eco():
    need_gpu()
    from paper_2510_18221_amd import eco as m
    m.lib()
    return m


def test_empty_world(eco):
    """No agents at all: only regrowth runs; the policy kernel has nothing to do."""
    cfg = wl.desc(width=32, height=24, n_agents_init=0, capacity=64, resource_density=0.2, regrow_prob=0.1, seed=11)
    run_pair(eco, cfg, 6, actions_fn=lambda t: np.zeros(cfg["capacity"], np.uint8), what="empty world")


def test_single_agent(eco):
    cfg = wl.desc(width=16, height=16, n_agents_init=1, capacity=8, resource_density=0.5, regrow_prob=0.05,
                  window=7, n_scalars=8, hidden1=64, hidden2=64, n_actions=7, seed=12, e_init=195)
    run_pair(eco, cfg, 10, actions_fn=lambda t: wl.biased_actions(cfg["capacity"], 7, 12, t), what="one agent")


def test_max_worlds(eco):
    """1024 tiny worlds in one object: every world's statistics against its own oracle on
    a sample of worlds, full state on a few, invariants on all."""
    n = 1024
    cfgs = [wl.desc(width=9 + i % 5, height=8 + i % 3, n_agents_init=4 + i % 4, capacity=16 + 8 * (i % 3),
                    resource_density=0.3, regrow_prob=0.05, window=3, seed=1000 + i, e_init=185)
            for i in range(n)]
    gw = eco.World(cfgs)
    sample = list(range(0, n, 97)) + [n - 1]
    ows = {i: orc.OracleWorld(cfgs[i]) for i in sample}
    for t in range(5):
        acts = [wl.biased_actions(c["capacity"], c["n_actions"], i, t) for i, c in enumerate(cfgs)]
        gw.step_with_actions(np.concatenate(acts))
        for i, ow in ows.items():
            ow.step(actions=acts[i])
        stats = gw.stats()
        for i, ow in ows.items():
            assert_stats_match(stats[i], ow.stats(), f"world {i} step {t}")
        for i in sample[:4]:
            compare_world(gw, ows[i], f"world {i} step {t}", world=i, weights_slots=2)
    for i in range(0, n, 31):
        check_invariants(gw.read_state(i), cfgs[i]["width"], cfgs[i]["height"])
    gw.close()

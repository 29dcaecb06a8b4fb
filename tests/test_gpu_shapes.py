"""Parity of the HIP world step with the oracle across the network and sensor
shapes the library accepts: window sides 1..15 (including the window without a
cell ahead, S = 1), hidden widths 32 / 64 / 128, FP32 / BF16 / FP8 storage,
4 or 8 scalar sensors, 5 or 7 actions, and every unroll depth of the policy
kernel.  Small worlds with seeded actions that force moves, meals, births and
deaths; integer state bit-exact, logits within the FP32 tolerance.
"""
import pytest

from paper_2510_18221_amd import workloads as wl

from gpu_util import need_gpu, run_pair

pytestmark = pytest.mark.gpu

# (window, hidden, wdtype, n_scalars, n_actions, launch (waves/block, blocks/CU, unroll))
SHAPES = [
    (1, 32, 0, 4, 5, (4, 2, 4)),
    (1, 128, 2, 8, 7, (8, 1, 16)),
    (3, 64, 1, 8, 7, (2, 4, 8)),
    (3, 128, 0, 4, 5, (1, 8, 16)),
    (5, 64, 0, 4, 7, (8, 4, 4)),
    (7, 32, 2, 8, 7, (4, 4, 8)),
    (7, 128, 1, 4, 7, (8, 2, 8)),
    (9, 128, 2, 4, 5, (4, 1, 4)),
    (13, 32, 0, 8, 5, (2, 2, 16)),
    (15, 32, 1, 4, 5, (8, 4, 16)),
    (15, 64, 2, 8, 7, (4, 8, 4)),
    (15, 128, 0, 8, 7, (8, 4, 8)),
]


@pytest.fixture(scope="module")
def eco():
    need_gpu()
    from paper_2510_18221_amd import eco as m
    m.lib()
    return m


@pytest.mark.parametrize("window,hidden,wdtype,n_scalars,n_actions,launch", SHAPES)
def test_shape(eco, window, hidden, wdtype, n_scalars, n_actions, launch):
    cfg = wl.desc(width=23, height=19, n_agents_init=70, capacity=130, resource_density=0.35, regrow_prob=0.05,
                  mutation_sigma=0.02, window=window, n_scalars=n_scalars, hidden1=hidden, hidden2=hidden,
                  n_actions=n_actions, wdtype=wdtype, seed=window * 1000 + hidden, e_init=185)
    acts = lambda t: wl.biased_actions(cfg["capacity"], n_actions, window + hidden, t, p_forward=0.35, p_eat=0.35)
    run_pair(eco, cfg, 6, actions_fn=acts, launch=launch,
             what=f"S={window} H={hidden} wdtype={wdtype} ns={n_scalars} A={n_actions} launch={launch}")

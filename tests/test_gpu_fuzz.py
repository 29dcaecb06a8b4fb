"""Property-based parity of the HIP world step with the oracle on random tiny
worlds (the same strategy as the oracle cross-check: random sizes, windows,
option combinations, written states, random or sampled actions), each at a random
launch shape of the policy kernel.  Derandomized: the same 100 cases every run.
Integer state bit-exact, statistics equal, weights and colour traits within a
few FP32 ulps, logits within the FP32 tolerance."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from oracle import oracle as orc

from gpu_util import LOGIT_TOL, assert_stats_match, compare_world, logit_err, need_gpu
from test_oracle_fuzz import worlds

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eco():
    need_gpu()
    from paper_2510_18221_amd import eco as m
    m.lib()
    return m


LAUNCHES = [(1, 4, 4), (2, 2, 8), (4, 2, 16), (8, 1, 4), (8, 4, 8), (4, 8, 4)]


def check_world(eco, w, launch):
    """One random world through both sides: written state, then its steps."""
    cfg, s, acts, sampled = w
    ow = orc.OracleWorld(cfg)
    ow.write_state(s)
    gw = eco.World(cfg)
    try:
        gw.set_launch(*launch)
        gw.set_flags(eco.RT_KEEP_LOGITS)
        if cfg["flags"] & orc.TERRAIN:
            np.testing.assert_array_equal(gw.read_terrain(), ow.terrain())
        gw.write_state(ow.state())
        compare_world(gw, ow, "written")
        for t, a in enumerate(acts):
            alive = ow.state()["alive"].astype(bool)
            logits, smp = ow.step(actions=None if sampled else a, want_logits=True, want_sampled=True)
            gw.step_with_actions(np.where(alive, smp, 0).astype(np.uint8) if sampled else a)
            compare_world(gw, ow, f"step {t}")
            assert_stats_match(gw.stats()[0], ow.stats(), f"step {t}", check_trait=False)
            gl = gw.read_logits()
            if alive.any():
                assert logit_err(gl[alive], logits[alive]).max() <= LOGIT_TOL
    finally:
        gw.close()


def test_random_worlds(eco):
    @settings(max_examples=100, deadline=None, derandomize=True, database=None,
              suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large,
                                     HealthCheck.function_scoped_fixture])
    @given(worlds(), st.sampled_from(LAUNCHES))
    def case(w, launch):
        check_world(eco, w, launch)

    case()

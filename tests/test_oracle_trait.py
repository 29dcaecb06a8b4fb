"""Pin of the oracle's trait statistics (CPU).

The measurement interface of App. E reports, per step, the population mean and
the population variance of each live agent's squared parameter norm
||theta_master||^2 (Sec. 3.3: every mutable parameter, the evolving log
temperature included; the colour trait is a separate trait and not in theta).
Here both moments are recomputed with numpy from the FP32 master weights the
oracle reports for every live slot (np.mean, np.var with ddof=0), independently
of the oracle's own reduction, through steps with births at sigma > 0 and at
sigma = 0.  BF16 storage makes the stored copy differ from the master, so a
statistic taken over the stored weights fails; sample variance (ddof=1) differs
by a factor n/(n-1); dropping the log temperature or adding the colour changes
every agent's norm.
"""
import numpy as np
import pytest

from oracle import oracle as orc

RTOL = 1e-10   # FP64 sums of a few thousand exact squares in two orders, then two moments


def _cfg(sigma, flags, wdtype):
    return dict(width=12, height=12, n_agents_init=40, capacity=120, resource_density=0.3, regrow_prob=0.05,
                mutation_sigma=sigma, window=3, n_scalars=4, hidden1=32, hidden2=32, n_actions=5, wdtype=wdtype,
                e_init=260, e_cost=1, e_eat=10, e_repro=200, e_child=100, seed=7, flags=flags)


def _numpy_moments(w):
    st = w.state()
    live = np.nonzero(st["alive"])[0]
    t = np.array([np.sum(w.weights(int(s), master=True) ** 2) for s in live], dtype=np.float64)
    return t, (float(np.mean(t)) if len(t) else 0.0), (float(np.var(t, ddof=0)) if len(t) else 0.0)


def _check(w, what):
    t, mean, var = _numpy_moments(w)
    s = w.stats()
    assert s["population"] == len(t), what
    assert abs(s["trait_mean"] - mean) <= RTOL * abs(mean), (what, s["trait_mean"], mean)
    assert abs(s["trait_var"] - var) <= RTOL * abs(var), (what, s["trait_var"], var)
    return t, var


@pytest.mark.parametrize("sigma", [0.3, 0.0])
@pytest.mark.parametrize("flags,wdtype", [(0, orc.BF16), (orc.EVOLVE_TEMPERATURE | orc.COLOUR_VISION, orc.BF16),
                                          (orc.EVOLVE_TEMPERATURE, orc.FP32)])
def test_trait_moments_match_numpy_on_master_weights(sigma, flags, wdtype):
    cfg = _cfg(sigma, flags, wdtype)
    w = orc.OracleWorld(cfg)
    _check(w, "init")
    births = 0
    for step in range(6):
        w.step(actions=orc_actions(cfg, step))
        births += w.stats()["births"]
        t, var = _check(w, f"step {step}")
    assert births > 10
    n = len(t)
    assert n > 20
    # the alternatives a plausible mistake would produce are all far outside RTOL
    assert abs(var * n / (n - 1) - var) > 1e3 * RTOL * var                     # sample variance
    live = np.nonzero(w.state()["alive"])[0]
    stored = np.array([np.sum(w.weights(int(s)) ** 2) for s in live])
    if wdtype == orc.BF16:
        assert abs(np.mean(stored) - np.mean(t)) > 1e3 * RTOL * np.mean(t)   # storage instead of master
    if flags & orc.EVOLVE_TEMPERATURE and sigma > 0:
        P = w.P
        no_temp = np.array([np.sum(w.weights(int(s), master=True)[:P - 1] ** 2) for s in live])
        assert abs(np.var(no_temp) - var) > 1e3 * RTOL * var                  # log temperature left out
    if flags & orc.COLOUR_VISION:
        with_colour = t + np.array([np.sum(w.colour(int(s)).astype(np.float64) ** 2) for s in live])
        assert abs(np.mean(with_colour) - np.mean(t)) > 1e3 * RTOL * np.mean(t)  # colour counted in theta
    w.close()


def test_sigma_zero_children_carry_the_parents_norm():
    cfg = _cfg(0.0, orc.EVOLVE_TEMPERATURE, orc.BF16)
    w = orc.OracleWorld(cfg)
    before = {int(s): float(np.sum(w.weights(int(s), master=True) ** 2))
              for s in np.nonzero(w.state()["alive"])[0]}
    w.step(actions=orc_actions(cfg, 0))
    st = w.state()
    assert w.stats()["births"] > 0
    uid_to_slot = {int(st["uid"][s]): int(s) for s in np.nonzero(st["alive"])[0]}
    for s in np.nonzero(st["alive"])[0]:
        if st["parent_uid"][s] != np.iinfo(np.uint64).max:
            parent_uid = int(st["parent_uid"][s])
            # the parent's initial slot is its uid (uid = slot at init)
            assert np.sum(w.weights(int(s), master=True) ** 2) == before[parent_uid]
            assert parent_uid in uid_to_slot
    _check(w, "sigma 0")
    w.close()


def test_single_agent_and_empty_world_have_zero_variance():
    cfg = dict(_cfg(0.1, 0, orc.FP32), n_agents_init=1, e_init=50)
    w = orc.OracleWorld(cfg)
    s = w.stats()
    assert s["population"] == 1 and s["trait_var"] == 0.0
    t, mean, var = _numpy_moments(w)
    assert mean == t[0] and abs(s["trait_mean"] - mean) <= RTOL * mean
    w.close()
    w = orc.OracleWorld(dict(cfg, n_agents_init=0))
    s = w.stats()
    assert s["population"] == 0 and s["trait_mean"] == 0.0 and s["trait_var"] == 0.0
    w.close()


def orc_actions(cfg, step):
    """Seeded actions that keep agents moving and eating (five actions: births are automatic)."""
    rng = np.random.default_rng([11, step])
    return rng.integers(0, cfg["n_actions"], size=cfg["capacity"], dtype=np.uint8)

"""Property-based cross-check of the two independently written statements of the
rules (the C oracle and the pure-Python one) on random tiny worlds: random grid
sizes (1 to 9 cells a side), windows, option combinations (attack, "Front" window, evolving
temperature, colour vision, the three-resource ecology with or without attack
at four strike strengths, terrain), random states
written into both (agents, resources, walls, stomachs, health), random actions
or the policies' own samples.  Every step both must give the same state,
statistics and logits.  (CPU only; a fixed, derandomized set of 100 worlds per
run, so the suite's result does not depend on the run.)"""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from oracle import oracle as orc
from oracle import spec
from paper_2510_18221_amd import workloads as wl

from worldstate import assert_same_state, empty_state

STATS = ("births", "deaths", "killed", "eaten", "regrown", "moves_ok", "moves_blocked", "births_blocked_cell",
         "births_blocked_capacity", "population", "resource_total")


@st.composite
def worlds(draw):
    ecology = draw(st.booleans())
    W, H = draw(st.integers(1, 9)), draw(st.integers(1, 9))   # sides below 3 fold the attack square
    window = draw(st.sampled_from([s for s in (1, 3, 5) if s <= min(W, H)]))
    flags = 0
    if draw(st.booleans()):
        flags |= orc.FRONT_VISION
    if draw(st.booleans()):
        flags |= orc.COLOUR_VISION
    attack = 0
    if draw(st.booleans()):
        flags |= orc.EVOLVE_TEMPERATURE
    if ecology:
        flags |= orc.ECOLOGY
        if draw(st.booleans()):
            flags |= orc.TERRAIN
        attack = int(draw(st.booleans()))
        n_actions, n_scalars = 8 + attack, draw(st.sampled_from([8, 12]))
    else:
        n_actions = draw(st.sampled_from([5, 7]))
        attack = int(n_actions == 7 and draw(st.booleans()))
        n_scalars = draw(st.sampled_from([4, 8]))
    cap = draw(st.integers(2, 12))
    eco = dict(wl.ECOLOGY, w_cost=draw(st.integers(0, 3)), age_shift=draw(st.integers(0, 6)),
               cap_water=draw(st.integers(5, 60)), photo_rate=draw(st.sampled_from([0.0, 0.05, 0.5])),
               w_child=draw(st.integers(0, 20)), terrain_scale=draw(st.integers(1, 6)),
               sea_level=draw(st.integers(0, 20)), water_per_depth=draw(st.integers(0, 3)),
               attack_damage=draw(st.sampled_from([0, 25, 50, 100])))
    cfg = wl.desc(width=W, height=H, n_agents_init=0, capacity=cap, window=window, n_scalars=n_scalars,
                  hidden1=32, hidden2=32, n_actions=n_actions, attack_enabled=attack, flags=flags, eco=eco,
                  resource_density=0.0, regrow_prob=draw(st.sampled_from([0.0, 0.2, 1.0])),
                  mutation_sigma=0.1, seed=draw(st.integers(0, 2**32 - 1)), e_init=100)
    # a random state: distinct cells for up to cap agents
    cells = W * H
    n = draw(st.integers(0, min(cap, cells)))
    rng = np.random.default_rng(draw(st.integers(0, 2**32 - 1)))
    s = empty_state(W, H, cap, uid_next=cap, ecology=ecology)
    slots = rng.choice(cap, size=n, replace=False)
    where = rng.choice(cells, size=n, replace=False)
    for slot, c in zip(slots, where):
        s["alive"][slot], s["pos"][slot], s["occ"][c] = 1, c, slot
        s["facing"][slot] = rng.integers(0, 4)
        s["energy"][slot] = rng.choice([1, 2, 3, 50, 150, 210, 260])
        s["age"][slot] = rng.integers(0, 200)
        s["uid"][slot] = slot
    s["res"] = (rng.random(cells) < 0.3).astype(np.uint8)
    s["wall"] = ((rng.random(cells) < 0.1) & (s["occ"] < 0)).astype(np.uint8)
    if ecology:
        s["res"][:] = 0
        for k, hi in (("cell_water", 30), ("cell_energy", 30), ("cell_biomass", 4)):
            s[k] = rng.integers(0, hi, cells).astype(np.int32) * (rng.random(cells) < 0.5)
        live = s["alive"].astype(bool)
        s["water"][live] = rng.integers(0, 40, live.sum())
        s["biomass"][live] = rng.integers(1, 5, live.sum())
        s["hp"][live] = rng.integers(1, 101, live.sum())
    acts = [rng.integers(0, n_actions, cap).astype(np.uint8) for _ in range(4)]
    sampled = draw(st.booleans())
    return cfg, s, acts, sampled


@settings(max_examples=100, deadline=None, derandomize=True, database=None,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large])
@given(worlds())
def test_oracle_and_python_statement_agree(w):
    cfg, s, acts, sampled = w
    o = orc.OracleWorld(cfg)
    o.write_state(s)
    sp = spec.from_state(cfg, o.state())
    if cfg["flags"] & orc.TERRAIN:   # both regenerate the same rock layer from the seed
        np.testing.assert_array_equal(o.terrain(), np.array(sp.rock))
    assert_same_state(o.state(), sp.state(), "written")
    for t, a in enumerate(acts):
        live = sorted(sp.agents)
        spl = {k: sp.logits(k) for k in live}
        logits, _ = o.step(actions=None if sampled else a, want_logits=True, want_sampled=True)
        sst = sp.step(actions=None if sampled else [int(v) for v in a])
        for k in live:
            np.testing.assert_allclose(logits[k], spl[k], rtol=1e-12, atol=1e-12)
        assert_same_state(o.state(), sp.state(), f"step {t}")
        os_ = o.stats()
        for k in STATS:
            assert os_[k] == sst.get(k, 0), (t, k, os_[k], sst.get(k))
        for k in sp.agents:
            np.testing.assert_array_equal(o.weights(k, master=True), np.array(sp.agents[k]["theta"]))
            if cfg["flags"] & orc.COLOUR_VISION:
                np.testing.assert_array_equal(o.colour(k), np.array(sp.agents[k]["colour"], np.float32))

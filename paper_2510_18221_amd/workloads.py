"""Synthetic workload descriptions and seeded input generators.

This module holds parameters and random inputs only (no step arithmetic); both
the GPU path and the oracle consume what it returns.  The worlds stand in for
the paper's runs (Sec. 3.2 grid worlds of 64^2 .. 1024^2 cells with tens of
thousands of agents, Table of runtimes in App. E), on a uniform torus with one
resource.

Energies are integers in units of 0.1 energy: start 10 (100), step cost 0.1 (1),
+1 per resource eaten (10), reproduce at >= 20 (200), child receives 10 (100).
"""
import math

import numpy as np

ENERGY = dict(e_init=100, e_cost=1, e_eat=10, e_repro=200, e_child=100)

FP32, BF16, FP8 = 0, 1, 2


def desc(**kw):
    d = dict(width=64, height=64, n_agents_init=256, capacity=4096, resource_density=0.1, regrow_prob=0.01,
             mutation_sigma=0.02, window=5, n_scalars=4, hidden1=32, hidden2=32, n_actions=5, wdtype=FP32,
             seed=0, **ENERGY)
    d.update(kw)
    return d


# Three-resource ecology parameters (integer units: energy in 0.1 energy, health
# in 0.1 HP).  The paper fixes the photosynthesis rate 0.01, the biomass site
# density 1/4, health 10 HP at most and 5 HP at birth, and healing of 1 HP per
# 0.1 energy; the other amounts are chosen here.
ECOLOGY = dict(water_density=0.1, energy_density=0.05, biomass_density=0.25, water_site=20, energy_site=20,
               biomass_site=2, eat_water=10, eat_biomass=1, cap_water=200, cap_energy=400, cap_biomass=8,
               e_cost_move=2, w_cost=1, photo_rate=0.01, cell_energy_max=40, hp_max=100, hp_child=50,
               hp_overspend=20, hp_heal=10, heal_energy=1, age_shift=9, w_init=100, b_init=2, w_child=50, b_child=1,
               b_repro=2, terrain_scale=32, sea_level=8, water_per_depth=4, attack_damage=100)
ECOLOGY_FLAG = 8
# Attack strengths of the ecology (health per strike): the paper's full (10 HP,
# kills any agent), half (5 HP) and quarter (2.5 HP) settings.
ATTACK_FULL, ATTACK_HALF, ATTACK_QUARTER = 100, 50, 25


def ecology_desc(eco=None, **kw):
    """A world of the three-resource ecology: eight actions, 8 scalars (nine
    actions when attack_enabled=1 is passed)."""
    d = desc(n_actions=8, n_scalars=8, flags=ECOLOGY_FLAG, eco=dict(ECOLOGY, **(eco or {})))
    d.update(kw)
    if d.get("attack_enabled") and "n_actions" not in kw:
        d["n_actions"] = 9
    return d


def world_small(seed=0, wdtype=FP32):
    """64x64 torus, 256 agents, 5x5 window + 4 scalars (D = 104), 104->32->32->5, sigma 0.02."""
    return desc(seed=seed, wdtype=wdtype)


def world_65k(seed=0, wdtype=FP32, frozen=False):
    """1024x1024, 65,536 agents, capacity 131,072, density 0.05, regrowth 0.01,
    11x11 window + 8 scalars (D = 492), 492->64->64->7, sigma 0.01.
    frozen: no step cost and no births, so the population stays at 65,536."""
    d = desc(width=1024, height=1024, n_agents_init=65536, capacity=131072, resource_density=0.05,
             regrow_prob=0.01, mutation_sigma=0.01, window=11, n_scalars=8, hidden1=64, hidden2=64,
             n_actions=7, wdtype=wdtype, seed=seed)
    if frozen:
        d.update(e_cost=0, e_repro=2**30)
    return d


def world_large(seed=0, wdtype=BF16):
    """2048x2048, capacity 262,144 starting half full, density 0.03, regrowth 0.005,
    15x15 window + 8 scalars (D = 908), 908->128->128->7, sigma 0.01."""
    return desc(width=2048, height=2048, n_agents_init=131072, capacity=262144, resource_density=0.03,
                regrow_prob=0.005, mutation_sigma=0.01, window=15, n_scalars=8, hidden1=128, hidden2=128,
                n_actions=7, wdtype=wdtype, seed=seed)


def batch_sides(n_worlds=64, seed=12345, lo=128, hi=1024):
    """Square sides log-uniform in [lo, hi]: one draw per equal-probability
    stratum (stratified sampling, so the batch total is close to its expected
    value), in an order shuffled by a seeded numpy generator."""
    rng = np.random.default_rng(seed)
    u = (np.arange(n_worlds) + rng.random(n_worlds)) / n_worlds
    rng.shuffle(u)
    return [int(round(math.exp(math.log(lo) + x * math.log(hi / lo)))) for x in u]


def world_batch(n_worlds=64, wdtype=BF16, side_seed=12345, scale=1.0):
    """Many independent worlds of uneven size: sides log-uniform in [128, 1024],
    agents on 6.25% of the cells, capacity 1.125x rounded up to 64, the 65k-agent
    world's 492->64->64->7 policy, world seeds 0..n-1.  scale < 1 shrinks the
    sides (for tests)."""
    out = []
    for i, side in enumerate(batch_sides(n_worlds, side_seed)):
        s = max(16, int(round(side * scale)))
        n = int(round(0.0625 * s * s))
        cap = int(math.ceil(1.125 * n / 64.0)) * 64
        out.append(desc(width=s, height=s, n_agents_init=n, capacity=max(cap, 64), resource_density=0.05,
                        regrow_prob=0.01, mutation_sigma=0.01, window=11, n_scalars=8, hidden1=64, hidden2=64,
                        n_actions=7, wdtype=wdtype, seed=i))
    return out


def random_actions(cap, n_actions, seed, step):
    """Seeded uniform actions for driving both implementations with the same input."""
    rng = np.random.default_rng([seed, step, 0xAC7])
    return rng.integers(0, n_actions, size=cap, dtype=np.uint8)


def biased_actions(cap, n_actions, seed, step, p_forward=0.3, p_eat=0.3, p_attack=0.0):
    """Seeded actions with more moves and meals (exercises births and conflicts);
    with seven (nine) actions, p_attack more of them attack."""
    rng = np.random.default_rng([seed, step, 0xB1A5])
    u = rng.random(cap)
    a = rng.integers(0, n_actions, size=cap, dtype=np.uint8)
    a[u < p_forward] = 3
    a[(u >= p_forward) & (u < p_forward + p_eat)] = 4
    if n_actions >= 8:   # the ecology: meals spread over energy, water, biomass; 15% reproduce
        eat = (u >= p_forward) & (u < p_forward + p_eat)
        a[eat] = 4 + (rng.integers(0, 3, size=cap)[eat]).astype(np.uint8)
        p0 = p_forward + p_eat
        a[(u >= p0) & (u < p0 + 0.15)] = 7
        if n_actions == 9:
            a[(u >= p0 + 0.15) & (u < p0 + 0.15 + p_attack)] = 8
    if n_actions == 7:
        p0 = p_forward + p_eat
        a[(u >= p0) & (u < p0 + 0.2)] = 5
        a[(u >= p0 + 0.2) & (u < p0 + 0.2 + p_attack)] = 6
    return a

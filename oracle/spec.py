"""Pure-Python statement of the world step for tiny worlds (TEST INFRASTRUCTURE).

A second, independently written version of the same rules as eco_oracle.c, in
plain Python integers and floats, used to cross-check the C oracle on tiny
worlds and to run the hand-traced cases.  Rules (paper sections):

* Sec. 3.1: an Ecological Game step = observation of each live agent, one
  action each, a synchronous transition, and the population function (who is
  alive, who is whose parent).
* Sec. 3.2: one agent per cell; rotate / forward / eat / reproduce actions;
  moving into an occupied cell or a contested cell does not happen (here the
  lowest slot wins a contested empty cell); every step costs energy; eating
  moves a resource unit into the agent; a child appears directly behind its
  single parent and receives a fixed amount of energy; death at energy <= 0.
  With attacks enabled, an attacker kills every other agent in the 3x3 square
  directly in front of it (rows 1..3 ahead, one column to either side), after
  the moves; each victim leaves one resource unit on its cell (a dead agent's
  carried resources return to the cell it stood on).
* Options (cfg["flags"]): 1 = "Front" vision (the window lies ahead, the agent
  in the middle of its last row; App. "Varying Vision Range"); 2 = an evolving
  softmax temperature, one more mutable parameter (log tau) after the output
  biases (Sec. 3.3); 4 = a 3-channel colour trait that mutates like the
  weights, seen by others through a rendered window (three colour channels and
  an elevation-difference channel, zero on the flat torus; Sec. 3.2, 3.3);
  8 = the three-resource ecology with health (Sec. 3.2 "Resources" and health
  points): water, energy and biomass on cells and in capped stomachs, three eat
  actions, energy and water spent every step (the water back onto the cell),
  damage from overspending and age, healing bought with energy, death at zero
  health returning everything carried, reproduction needing spare biomass,
  energy appearing on biomass (photosynthesis); with attacks enabled the
  ecology has a ninth action, attack, over the same 3x3 square, and every
  strike costs the struck agent eco["attack_damage"] health, in the same health
  update as its other damage (App. "Varying Attack Strength");
  16 = terrain (with 8; Sec. 3.2 "Terrain"): rock heights 0..31 from a seeded
  value-noise field, the sea filling the cells below sea level, all water of a
  cell moving each step to its lowest strictly lower neighbour, and the
  elevation difference in the colour window's fourth channel.
* Sec. 3.3: per-agent MLP with two ReLU hidden layers and a linear head;
  softmax sampling; zero-mean Gaussian initial weights with zero biases;
  children copy the parent's weights plus Gaussian noise.

Random numbers: Philox4x32-10 (Salmon et al., SC'11) computed with Python
integers; Box-Muller (1958) with the math module.
"""
import math
from fractions import Fraction

M32 = 0xFFFFFFFF
REST, TURN_L, TURN_R, FORWARD, EAT, REPRODUCE, ATTACK = range(7)
FRONT, TEMPERATURE, COLOUR, ECOLOGY, TERRAIN = 1, 2, 4, 8, 16
EAT_E, EAT_W, EAT_B, REPRO8, ATTACK9 = 4, 5, 6, 7, 8
HEADINGS = [(0, -1), (1, 0), (0, 1), (-1, 0)]  # N, E, S, W with y pointing down


def philox4x32_10(ctr, key):
    """Ten Philox rounds on a 4-word counter with a 2-word key (SC'11)."""
    x = list(ctr)
    k = list(key)
    for rnd in range(10):
        if rnd:
            k = [(k[0] + 0x9E3779B9) & M32, (k[1] + 0xBB67AE85) & M32]
        a = 0xD2511F53 * x[0]
        b = 0xCD9E8D57 * x[2]
        x = [((b >> 32) ^ x[1] ^ k[0]) & M32, b & M32, ((a >> 32) ^ x[3] ^ k[1]) & M32, a & M32]
    return x


def cos_sin_2pi_u24(j):
    """cos and sin of 2 pi j / 2^24: whole quarter turns removed exactly, the rest
    measured from the nearer end of its quarter, so math.cos / math.sin only see
    angles in [0, pi/4] and the quarter turns give exact zeros."""
    q, r = (j >> 22) & 3, j & 0x3FFFFF
    if r <= 0x200000:
        th = 6.283185307179586 * r / 16777216.0
        c, s = math.cos(th), math.sin(th)
    else:
        th = 6.283185307179586 * (0x400000 - r) / 16777216.0
        c, s = math.sin(th), math.cos(th)
    for _ in range(q):   # a quarter turn: (cos, sin) -> (-sin, cos)
        c, s = -s, c
    return c, s


def gauss4(ctr, key):
    """Box-Muller: z = sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2) for two pairs of draws."""
    x = philox4x32_10(ctr, key)
    out = []
    for i in (0, 2):
        u1 = ((x[i] >> 8) + 1) / 16777216.0
        r = math.sqrt(-2.0 * math.log(u1))
        c, s = cos_sin_2pi_u24(x[i + 1] >> 8)
        out += [r * c, r * s]
    return out


def fma(a, b, c):
    """a*b + c with a single rounding to double (exact rational arithmetic)."""
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def f32(v):
    """Round a Python float to the nearest IEEE single."""
    import struct
    return struct.unpack("<f", struct.pack("<f", v))[0]


class SpecWorld:
    """Tiny-world version of the rules; FP32 weights only (storage == master)."""

    def __init__(self, cfg):
        self.c = dict(cfg)
        c = self.c
        self.W, self.H, self.cap = c["width"], c["height"], c["capacity"]
        self.S = c["window"]
        self.A = c["n_actions"]
        self.key = [c["seed"] & M32, (c["seed"] >> 32) & M32]
        self.D = 4 * self.S * self.S + c["n_scalars"]
        self.shapes = [(c["hidden1"], self.D), (c["hidden2"], c["hidden1"]), (self.A, c["hidden2"])]
        self.flags = c.get("flags", 0)
        self.P = sum(r * k + r for r, k in self.shapes) + (1 if self.flags & TEMPERATURE else 0)
        self.step_no = 0
        self.uid_next = c["n_agents_init"]
        cells = self.W * self.H
        self.occ = [-1] * cells
        self.wall = [0] * cells
        rho = math.floor(f32(c["resource_density"]) * 4294967296.0)  # descriptor fields are float32
        self.eco = c.get("eco", {}) if self.flags & ECOLOGY else None
        if self.eco is None:
            self.res = [1 if philox4x32_10([i, 0, 2, 0], self.key)[0] < rho else 0 for i in range(cells)]
        else:
            e = self.eco
            self.res = [0] * cells
            self.cw, self.ce, self.cb = [0] * cells, [0] * cells, [0] * cells
            tw, te, tb = (math.floor(f32(e[k]) * 4294967296.0)
                          for k in ("water_density", "energy_density", "biomass_density"))
            for i in range(cells):
                x = philox4x32_10([i, 0, 2, 0], self.key)
                self.cw[i] = e["water_site"] if x[1] < tw else 0
                self.ce[i] = e["energy_site"] if x[2] < te else 0
                self.cb[i] = e["biomass_site"] if x[3] < tb else 0
            if self.flags & TERRAIN:
                self.rock = [self._height(i % self.W, i // self.W) for i in range(cells)]
                self.cw = [(e["sea_level"] - r) * e["water_per_depth"] if r < e["sea_level"] else 0 for r in self.rock]
        order = sorted(range(cells), key=lambda i: (philox4x32_10([i, 0, 0, 0], self.key)[0], i))
        self.agents = {}  # slot -> dict
        for j in range(c["n_agents_init"]):
            self._spawn(j, order[j], philox4x32_10([j, 0, 1, 0], self.key)[0] >> 30, c["e_init"], j, None)
            self.agents[j]["theta"] = self._init_theta(j)
            if self.eco is not None:
                self.agents[j].update(water=self.eco["w_init"], biomass=self.eco["b_init"], hp=self.eco["hp_max"])
            if self.flags & COLOUR:
                self.agents[j]["colour"] = self._init_colour(j)

    def _spawn(self, slot, cell, facing, energy, uid, puid):
        self.agents[slot] = {"cell": cell, "facing": facing, "energy": energy, "age": 0,
                             "uid": uid, "puid": puid, "action": 0}
        self.occ[cell] = slot

    def _init_theta(self, j):
        theta = []
        p = 0
        for rows, cols in self.shapes:
            sd = math.sqrt(1.0 / cols)
            for _ in range(rows * cols):
                theta.append(f32(gauss4([j, 0, 3, p // 4], self.key)[p % 4] * sd))
                p += 1
            theta += [0.0] * rows
            p += rows
        if self.flags & TEMPERATURE:
            theta.append(0.0)     # log temperature 0: temperature 1
        return theta

    def _height(self, x, y):
        """Bilinear blend of the four surrounding lattice values (0..31) of a
        seeded torus lattice, spacing terrain_scale, in exact integers."""
        L = self.eco["terrain_scale"]
        nx, ny = max(1, self.W // L), max(1, self.H // L)
        i, fx = divmod(x * nx, self.W)
        j, fy = divmod(y * ny, self.H)
        v = lambda a, b: philox4x32_10([a % nx + (b % ny) * nx, 0, 9, 0], self.key)[0] >> 27
        num = (v(i, j) * (self.W - fx) * (self.H - fy) + v(i + 1, j) * fx * (self.H - fy)
               + v(i, j + 1) * (self.W - fx) * fy + v(i + 1, j + 1) * fx * fy)
        return num // (self.W * self.H)

    def _flow_target(self, i):
        x, y = self._xy(i)
        best, bh = None, self.rock[i]
        for fx, fy in HEADINGS:
            n = self._cell(x + fx, y + fy)
            if self.rock[n] < bh:
                best, bh = n, self.rock[n]
        return best

    def _init_colour(self, j):
        x = philox4x32_10([j, 0, 7, 0], self.key)
        return [(x[k] >> 8) / 16777216.0 for k in range(3)]

    @staticmethod
    def colour_byte(c):
        c = min(max(c, 0.0), 1.0)
        q = Fraction(c) * 255 + Fraction(1, 2)
        return q.numerator // q.denominator

    def _render(self, cell, own=None):
        o = self.occ[cell]
        elev = 0.0
        if self.flags & TERRAIN:
            elev = (self.rock[cell] - self.rock[own]) / 8.0
        if o >= 0:
            q = [self.colour_byte(v) for v in self.agents[o]["colour"]]
        elif self.eco is not None:
            if self.wall[cell]:
                q = [128, 128, 128]
            else:
                q = [min(self.ce[cell] * 16, 255), min(self.cb[cell] * 64, 255), min(self.cw[cell] * 16, 255)]
            return [v / 256.0 for v in q] + [elev]
        elif self.res[cell]:
            q = [0, 255, 0]
        elif self.wall[cell]:
            q = [128, 128, 128]
        else:
            q = [0, 0, 0]
        return [v / 256.0 for v in q] + [elev]

    def _xy(self, cell):
        return cell % self.W, cell // self.W

    def _cell(self, x, y):
        return (y % self.H) * self.W + (x % self.W)

    def observe(self, slot):
        ag = self.agents[slot]
        ax, ay = self._xy(ag["cell"])
        fx, fy = HEADINGS[ag["facing"]]
        rx, ry = -fy, fx
        R = self.S // 2
        top = self.S - 1 if self.flags & FRONT else R   # distance ahead of window row 0
        obs = []
        for r in range(self.S):
            for col in range(self.S):
                ahead, right = top - r, col - R
                cell = self._cell(ax + ahead * fx + right * rx, ay + ahead * fy + right * ry)
                if self.flags & COLOUR:
                    obs += self._render(cell, ag["cell"])
                    continue
                o = self.occ[cell]
                if self.eco is not None:
                    obs += [1.0 if o >= 0 else 0.0] + [min(v[cell], 255) / 16.0 for v in (self.cw, self.ce, self.cb)]
                    continue
                eb = 0
                if o >= 0:  # energy bin of the occupant, 8 bins up to the reproduction threshold
                    eb = min(max(self.agents[o]["energy"] * 8 // self.c["e_repro"], 0), 7)
                obs += [1.0 if o >= 0 else 0.0, float(self.res[cell]), float(self.wall[cell]), float(eb)]
        e = ag["energy"]
        if self.eco is not None:
            here = ag["cell"]
            obs += [e / 256.0, min(ag["age"], 1024) / 1024.0, ag["water"] / 256.0, ag["biomass"] / 8.0,
                    ag["hp"] / 128.0] + [min(v[here], 255) / 16.0 for v in (self.cw, self.ce, self.cb)]
            if self.c["n_scalars"] == 12:
                obs += [1.0 if k == ag["facing"] else 0.0 for k in range(4)]
            return obs
        obs += [e / 256.0, min(ag["age"], 1024) / 1024.0, float(self.res[ag["cell"]]),
                1.0 if e >= self.c["e_repro"] else 0.0]
        if self.c["n_scalars"] == 8:
            obs += [1.0 if k == ag["facing"] else 0.0 for k in range(4)]
        return obs

    def logits(self, slot):
        theta = self.agents[slot]["theta"]
        h = self.observe(slot)
        p = 0
        for li, (rows, cols) in enumerate(self.shapes):
            W = theta[p:p + rows * cols]
            b = theta[p + rows * cols:p + rows * cols + rows]
            p += rows * cols + rows
            out = [b[i] + sum(W[i * cols + k] * h[k] for k in range(cols)) for i in range(rows)]
            h = out if li == 2 else [max(v, 0.0) for v in out]
        return h

    @staticmethod
    def sample(logits, u, log_tau=0.0):
        m = max(logits)
        inv = math.exp(-log_tau)
        w = [1.0 if v == m else math.exp((v - m) * inv) for v in logits]
        cum, acc = [], 0.0
        for v in w:
            acc += v
            cum.append(acc)
        t = u * cum[-1]
        for k, ck in enumerate(cum):
            if t < ck:
                return k
        return max(k for k in range(len(w)) if w[k] > 0)

    def step(self, actions=None):
        c = self.c
        n = self.step_no
        st = {k: 0 for k in ("births", "deaths", "killed", "eaten", "regrown", "moves_ok", "moves_blocked",
                             "births_blocked_cell", "births_blocked_capacity")}
        st["action_hist"] = [0] * 9
        live = sorted(self.agents)
        for s in live:
            if actions is None:
                u = (philox4x32_10([s, n, 4, 0], self.key)[0] >> 8) / 16777216.0
                lt = self.agents[s]["theta"][-1] if self.flags & TEMPERATURE else 0.0
                a = self.sample(self.logits(s), u, lt)
            else:
                a = int(actions[s])
            self.agents[s]["action"] = a
            st["action_hist"][a] += 1
        # turns, then claims on the pre-step occupancy
        for s in live:
            a = self.agents[s]["action"]
            if a == TURN_L:
                self.agents[s]["facing"] = (self.agents[s]["facing"] - 1) % 4
            elif a == TURN_R:
                self.agents[s]["facing"] = (self.agents[s]["facing"] + 1) % 4
        claims = {}
        for s in live:
            ag = self.agents[s]
            if ag["action"] != FORWARD:
                continue
            x, y = self._xy(ag["cell"])
            fx, fy = HEADINGS[ag["facing"]]
            t = self._cell(x + fx, y + fy)
            if self.occ[t] == -1 and not self.wall[t]:
                claims.setdefault(t, []).append(s)
        winners = {min(v): t for t, v in claims.items()}
        for s in live:
            ag = self.agents[s]
            if ag["action"] != FORWARD:
                continue
            if s in winners:
                self.occ[ag["cell"]] = -1
                ag["cell"] = winners[s]
                self.occ[ag["cell"]] = s
                st["moves_ok"] += 1
            else:
                st["moves_blocked"] += 1
        # attacks land on the post-move positions, all at once
        hit = {}   # cell -> number of strikes
        if c.get("attack_enabled", 0):
            for s in live:
                ag = self.agents[s]
                if ag["action"] != (ATTACK9 if self.eco is not None else ATTACK):
                    continue
                x, y = self._xy(ag["cell"])
                fx, fy = HEADINGS[ag["facing"]]
                rx, ry = -fy, fx
                square = {self._cell(x + ahead * fx + side * rx, y + ahead * fy + side * ry)
                          for ahead in (1, 2, 3) for side in (-1, 0, 1)}   # each distinct cell once
                for cell in square - {ag["cell"]}:
                    hit[cell] = hit.get(cell, 0) + 1
        # eat, cost, death, age
        for s in live:
            ag = self.agents[s]
            if self.eco is not None:
                self._ecology_agent(s, st, hit.get(ag["cell"], 0))
                continue
            if ag["cell"] in hit:
                self.occ[ag["cell"]] = -1
                self.res[ag["cell"]] = 1
                del self.agents[s]
                st["deaths"] += 1
                st["killed"] += 1
                continue
            if ag["action"] == EAT and self.res[ag["cell"]] > 0:
                self.res[ag["cell"]] -= 1
                ag["energy"] += c["e_eat"]
                st["eaten"] += 1
            ag["energy"] -= c["e_cost"]
            if ag["energy"] <= 0:
                self.occ[ag["cell"]] = -1
                del self.agents[s]
                st["deaths"] += 1
            else:
                ag["age"] += 1
        # births
        claims = {}
        for s in sorted(self.agents):
            ag = self.agents[s]
            if self.eco is not None:
                e = self.eco
                if (ag["action"] != REPRO8 or ag["energy"] < c["e_repro"] or ag["water"] < e["w_child"]
                        or ag["biomass"] < e["b_repro"]):
                    continue
            elif ag["energy"] < c["e_repro"] or (self.A == 7 and ag["action"] != REPRODUCE):
                continue
            x, y = self._xy(ag["cell"])
            fx, fy = HEADINGS[ag["facing"]]
            t = self._cell(x - fx, y - fy)
            if self.occ[t] == -1 and not self.wall[t]:
                claims.setdefault(t, []).append(s)
            else:
                st["births_blocked_cell"] += 1
        won = sorted(min(v) for v in claims.values())
        st["births_blocked_cell"] += sum(len(v) - 1 for v in claims.values())
        target_of = {min(v): t for t, v in claims.items()}
        free = [s for s in range(self.cap) if s not in self.agents]
        sigma = f32(c["mutation_sigma"])
        nb = 0
        for k, p in enumerate(won):
            if k >= len(free):
                st["births_blocked_capacity"] += 1
                continue
            child = free[k]
            par = self.agents[p]
            par["energy"] -= c["e_child"]
            self._spawn(child, target_of[p], par["facing"], c["e_child"], self.uid_next + k, par["uid"])
            if self.eco is not None:
                e = self.eco
                par["water"] -= e["w_child"]
                par["biomass"] -= e["b_child"]
                self.agents[child].update(water=e["w_child"], biomass=e["b_child"], hp=e["hp_child"])
            theta = []
            for q, v in enumerate(par["theta"]):
                z = gauss4([p, n, 5, q // 4], self.key)[q % 4]
                theta.append(f32(fma(sigma, z, v)))
            self.agents[child]["theta"] = theta
            if self.flags & COLOUR:
                z = gauss4([p, n, 8, 0], self.key)
                self.agents[child]["colour"] = [f32(fma(sigma, z[k], v)) for k, v in enumerate(par["colour"])]
            nb += 1
        st["births"] = nb
        self.uid_next += nb
        # regrowth (ecology: photosynthesis on biomass); cell i draws output i mod 4 of
        # the block (i // 4, step, 6, 0)
        thr = math.floor(f32(c["regrow_prob"]) * 4294967296.0)
        for i in range(self.W * self.H):
            if self.eco is not None:
                b = self.cb[i]
                if b <= 0 or self.ce[i] >= self.eco["cell_energy_max"]:
                    continue
                p = Fraction(f32(self.eco["photo_rate"])) * b
                t = 2 ** 32 if p >= 1 else math.floor(p * 2 ** 32)
                if philox4x32_10([i >> 2, n, 6, 0], self.key)[i & 3] < t:
                    self.ce[i] += 1
                    st["regrown"] += 1
            elif self.res[i] == 0 and philox4x32_10([i >> 2, n, 6, 0], self.key)[i & 3] < thr:
                self.res[i] = 1
                st["regrown"] += 1
        if self.flags & TERRAIN:   # all water one cell downhill, every cell at once
            nw = [0] * (self.W * self.H)
            for i, wv in enumerate(self.cw):
                t = self._flow_target(i)
                nw[i if t is None else t] += wv
            self.cw = nw
        self.step_no += 1
        st["population"] = len(self.agents)
        st["resource_total"] = sum(self.res)
        if self.eco is not None:
            st["resource_total"] = sum(self.ce)
            st["water_total"] = sum(self.cw) + sum(a["water"] for a in self.agents.values())
            st["biomass_total"] = sum(self.cb) + sum(a["biomass"] for a in self.agents.values())
            st["hp_total"] = sum(a["hp"] for a in self.agents.values())
        st["energy_total"] = float(sum(a["energy"] for a in self.agents.values()))
        return st

    def _ecology_agent(self, s, st, strikes=0):
        """Eat, pay energy (destroyed) and water (back to the cell), take damage for
        each overspent resource, for age and for each strike, die at zero health
        leaving everything carried on the cell (killed, when struck), else heal
        with energy and age."""
        e, c = self.eco, self.c
        ag = self.agents[s]
        cell, a = ag["cell"], ag["action"]
        moved = 0
        for act, key, grid, amount, cap in ((EAT_E, "energy", self.ce, c["e_eat"], e["cap_energy"]),
                                            (EAT_W, "water", self.cw, e["eat_water"], e["cap_water"]),
                                            (EAT_B, "biomass", self.cb, e["eat_biomass"], e["cap_biomass"])):
            if a == act:
                moved = min(amount, grid[cell], cap - ag[key])
                if moved > 0:
                    grid[cell] -= moved
                    ag[key] += moved
        if moved > 0:
            st["eaten"] += 1
        over = 0
        ag["energy"] -= c["e_cost"] if a == REST else e["e_cost_move"]
        if ag["energy"] < 0:
            ag["energy"] = 0
            over += 1
        spend = min(ag["water"], e["w_cost"])
        ag["water"] -= spend
        self.cw[cell] += spend
        if spend < e["w_cost"]:
            over += 1
        ag["hp"] -= over * e["hp_overspend"] + (ag["age"] >> e["age_shift"]) + strikes * e.get("attack_damage", 0)
        if ag["hp"] <= 0:
            self.cw[cell] += ag["water"]
            self.ce[cell] += ag["energy"]
            self.cb[cell] += ag["biomass"]
            self.occ[cell] = -1
            del self.agents[s]
            st["deaths"] += 1
            st["killed"] += strikes > 0
            return
        if ag["hp"] < e["hp_max"] and ag["energy"] >= e["heal_energy"]:
            ag["hp"] = min(ag["hp"] + e["hp_heal"], e["hp_max"])
            ag["energy"] -= e["heal_energy"]
        ag["age"] += 1

    def state(self):
        """Same dictionary shape as oracle.unpack_state (dead slots zeroed)."""
        import numpy as np
        cap = self.cap
        out = {"step": self.step_no, "uid_next": self.uid_next,
               "uid": np.zeros(cap, np.uint64), "parent_uid": np.zeros(cap, np.uint64),
               "pos": np.zeros(cap, np.int32), "energy": np.zeros(cap, np.int32),
               "age": np.zeros(cap, np.int32), "facing": np.zeros(cap, np.uint8),
               "alive": np.zeros(cap, np.uint8), "action": np.zeros(cap, np.uint8),
               "occ": np.array(self.occ, np.int32), "res": np.array(self.res, np.uint8),
               "wall": np.array(self.wall, np.uint8)}
        for s, ag in self.agents.items():
            out["uid"][s] = ag["uid"]
            out["parent_uid"][s] = 0xFFFFFFFFFFFFFFFF if ag["puid"] is None else ag["puid"]
            out["pos"][s] = ag["cell"]
            out["energy"][s] = ag["energy"]
            out["age"][s] = ag["age"]
            out["facing"][s] = ag["facing"]
            out["alive"][s] = 1
            out["action"][s] = ag["action"]
        if self.eco is not None:
            out["water"] = np.zeros(cap, np.int32)
            out["biomass"] = np.zeros(cap, np.int32)
            out["hp"] = np.zeros(cap, np.int32)
            for s, ag in self.agents.items():
                out["water"][s], out["biomass"][s], out["hp"][s] = ag["water"], ag["biomass"], ag["hp"]
            out["cell_water"] = np.array(self.cw, np.int32)
            out["cell_energy"] = np.array(self.ce, np.int32)
            out["cell_biomass"] = np.array(self.cb, np.int32)
        return out


def from_state(cfg, st):
    """A SpecWorld holding the integer state `st` (same dict layout as
    oracle.unpack_state); live slots get the initial weights of their index."""
    w = SpecWorld(dict(cfg, n_agents_init=0))
    w.step_no = int(st["step"])
    w.uid_next = int(st["uid_next"])
    w.occ = [int(v) for v in st["occ"]]
    w.res = [int(v) for v in st["res"]]
    w.wall = [int(v) for v in st["wall"]]
    w.agents = {}
    for s in range(w.cap):
        if not st["alive"][s]:
            continue
        puid = int(st["parent_uid"][s])
        w.agents[s] = {"cell": int(st["pos"][s]), "facing": int(st["facing"][s]), "energy": int(st["energy"][s]),
                       "age": int(st["age"][s]), "uid": int(st["uid"][s]),
                       "puid": None if puid == 0xFFFFFFFFFFFFFFFF else puid, "action": int(st["action"][s]),
                       "theta": w._init_theta(s)}
        if w.flags & COLOUR:
            w.agents[s]["colour"] = w._init_colour(s)
        if w.eco is not None:
            w.agents[s].update(water=int(st["water"][s]), biomass=int(st["biomass"][s]), hp=int(st["hp"][s]))
    if w.eco is not None:
        w.cw, w.ce, w.cb = ([int(v) for v in st[k]] for k in ("cell_water", "cell_energy", "cell_biomass"))
    return w

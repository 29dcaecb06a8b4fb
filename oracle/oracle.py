"""ctypes wrapper of the CPU oracle (TEST INFRASTRUCTURE).

Loaded only by tests/, the smoke check and the benchmark's CPU-baseline leg.
The oracle is the plain sequential world step of eco_oracle.c (FP64 policy,
exact integer world); this module only marshals arguments.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# ECO_ORACLE_LIB: another build of the same source (the sanitizer test uses one)
_LIB_PATH = os.environ.get("ECO_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

FP32, BF16, FP8 = 0, 1, 2
REST, TURN_L, TURN_R, FORWARD, EAT, REPRODUCE, ATTACK = range(7)
FRONT_VISION, EVOLVE_TEMPERATURE, COLOUR_VISION, ECOLOGY, TERRAIN = 1, 2, 4, 8, 16   # orc_desc.flags
EAT_ENERGY, EAT_WATER, EAT_BIOMASS, REPRODUCE_ECO, ATTACK_ECO = 4, 5, 6, 7, 8   # the ecology's action set


class OrcEcology(ctypes.Structure):
    _fields_ = [("water_density", ctypes.c_float), ("energy_density", ctypes.c_float),
                ("biomass_density", ctypes.c_float)] + [(n, ctypes.c_int32) for n in (
                    "water_site", "energy_site", "biomass_site", "eat_water", "eat_biomass", "cap_water",
                    "cap_energy", "cap_biomass", "e_cost_move", "w_cost")] + [("photo_rate", ctypes.c_float)] + [
                (n, ctypes.c_int32) for n in ("cell_energy_max", "hp_max", "hp_child", "hp_overspend", "hp_heal",
                                              "heal_energy", "age_shift", "w_init", "b_init", "w_child", "b_child",
                                              "b_repro", "terrain_scale", "sea_level", "water_per_depth",
                                              "attack_damage")]


class OrcDesc(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_uint32), ("height", ctypes.c_uint32),
        ("n_agents_init", ctypes.c_uint32), ("capacity", ctypes.c_uint32),
        ("resource_density", ctypes.c_float), ("regrow_prob", ctypes.c_float),
        ("mutation_sigma", ctypes.c_float),
        ("window", ctypes.c_uint32), ("n_scalars", ctypes.c_uint32),
        ("hidden1", ctypes.c_uint32), ("hidden2", ctypes.c_uint32), ("n_actions", ctypes.c_uint32),
        ("e_init", ctypes.c_int32), ("e_cost", ctypes.c_int32), ("e_eat", ctypes.c_int32),
        ("e_repro", ctypes.c_int32), ("e_child", ctypes.c_int32),
        ("wdtype", ctypes.c_uint32), ("attack_enabled", ctypes.c_uint32),
        ("flags", ctypes.c_uint32), ("eco", OrcEcology), ("seed", ctypes.c_uint64),
    ]


class OrcStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "step", "population", "births", "deaths", "killed", "eaten", "regrown", "moves_ok", "moves_blocked",
        "births_blocked_cell", "births_blocked_capacity", "resource_total")] + [
        ("action_hist", ctypes.c_uint64 * 9),
        ("energy_total", ctypes.c_double), ("trait_mean", ctypes.c_double), ("trait_var", ctypes.c_double),
        ("water_total", ctypes.c_uint64), ("biomass_total", ctypes.c_uint64), ("hp_total", ctypes.c_uint64)]

    def as_dict(self):
        d = {n: getattr(self, n) for n, _ in self._fields_ if n != "action_hist"}
        d["action_hist"] = list(self.action_hist)
        return d


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from oracle import build as _build
            _build.build()
        _lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        _lib.orc_create.restype = P
        _lib.orc_create.argtypes = [ctypes.POINTER(OrcDesc), ctypes.c_int]
        _lib.orc_destroy.argtypes = [P]
        _lib.orc_last_error.restype = ctypes.c_char_p
        _lib.orc_step.argtypes = [P, P, P, P]
        _lib.orc_agent_logits.argtypes = [P, ctypes.c_uint32, P]
        _lib.orc_observe.argtypes = [P, ctypes.c_uint32, P]
        _lib.orc_read_weights.argtypes = [P, ctypes.c_uint32, ctypes.c_int, P]
        _lib.orc_state_bytes.restype = ctypes.c_size_t
        _lib.orc_state_bytes.argtypes = [P]
        _lib.orc_read_state.argtypes = [P, P, ctypes.c_size_t]
        _lib.orc_write_state.argtypes = [P, P, ctypes.c_size_t]
        _lib.orc_stats_get.argtypes = [P, ctypes.POINTER(OrcStats)]
        _lib.orc_input_dim.restype = ctypes.c_uint32
        _lib.orc_input_dim.argtypes = [ctypes.POINTER(OrcDesc)]
        _lib.orc_param_count.restype = ctypes.c_uint64
        _lib.orc_param_count.argtypes = [ctypes.POINTER(OrcDesc)]
        _lib.orc_philox4x32_10.argtypes = [P, P, P]
        _lib.orc_gauss4.argtypes = [P, P, P]
        _lib.orc_cos_sin_2pi_u24.argtypes = [ctypes.c_uint32, P]
        _lib.orc_bf16_rne.restype = ctypes.c_uint16
        _lib.orc_bf16_rne.argtypes = [ctypes.c_float]
        _lib.orc_fp8e4m3_rne_sat.restype = ctypes.c_uint8
        _lib.orc_fp8e4m3_rne_sat.argtypes = [ctypes.c_float]
        _lib.orc_fp8e4m3_decode.restype = ctypes.c_double
        _lib.orc_fp8e4m3_decode.argtypes = [ctypes.c_uint8]
        _lib.orc_sample.restype = ctypes.c_int
        _lib.orc_sample.argtypes = [P, ctypes.c_int, ctypes.c_double]
        _lib.orc_sample_tempered.restype = ctypes.c_int
        _lib.orc_sample_tempered.argtypes = [P, ctypes.c_int, ctypes.c_double, ctypes.c_double]
        _lib.orc_colour_byte.restype = ctypes.c_uint32
        _lib.orc_colour_byte.argtypes = [ctypes.c_float]
        _lib.orc_read_colour.argtypes = [P, ctypes.c_uint32, P]
        _lib.orc_read_terrain.argtypes = [P, P]
        _lib.orc_write_terrain.argtypes = [P, P]
        _lib.orc_write_colour.argtypes = [P, ctypes.c_uint32, P]
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def make_desc(cfg: dict) -> OrcDesc:
    d = OrcDesc()
    for name, _ in OrcDesc._fields_:
        if name == "eco":
            for en, _ in OrcEcology._fields_:
                if en in cfg.get("eco", {}):
                    setattr(d.eco, en, cfg["eco"][en])
        elif name in cfg:
            setattr(d, name, cfg[name])
    return d


def input_dim(cfg):
    d = make_desc(cfg)
    return lib().orc_input_dim(ctypes.byref(d))


def param_count(cfg):
    d = make_desc(cfg)
    return lib().orc_param_count(ctypes.byref(d))


def philox(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def gauss4(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.float64)
    lib().orc_gauss4(_ptr(c), _ptr(k), _ptr(out))
    return out


def cos_sin_2pi_u24(j):
    out = np.zeros(2, dtype=np.float64)
    lib().orc_cos_sin_2pi_u24(int(j), _ptr(out))
    return out


def bf16_rne(x: float) -> int:
    return lib().orc_bf16_rne(ctypes.c_float(x))


def fp8_rne_sat(x: float) -> int:
    return lib().orc_fp8e4m3_rne_sat(ctypes.c_float(x))


def fp8_decode(q: int) -> float:
    return lib().orc_fp8e4m3_decode(q)


def sample(logits, u):
    l = np.ascontiguousarray(logits, dtype=np.float64)
    return lib().orc_sample(_ptr(l), len(l), float(u))


def sample_tempered(logits, log_tau, u):
    l = np.ascontiguousarray(logits, dtype=np.float64)
    return lib().orc_sample_tempered(_ptr(l), len(l), float(log_tau), float(u))


def colour_byte(c: float) -> int:
    return lib().orc_colour_byte(ctypes.c_float(c))


class OracleWorld:
    """One oracle world.  materialize=True keeps all weights (can sample)."""

    def __init__(self, cfg: dict, materialize: bool = True):
        self.cfg = dict(cfg)
        self._desc = make_desc(cfg)
        h = lib().orc_create(ctypes.byref(self._desc), 1 if materialize else 0)
        if not h:
            raise ValueError("oracle create failed: " + lib().orc_last_error().decode())
        self._h = ctypes.c_void_p(h)
        self.W, self.H = cfg["width"], cfg["height"]
        self.cap = cfg["capacity"]
        self.A = cfg["n_actions"]
        self.D = lib().orc_input_dim(ctypes.byref(self._desc))
        self.P = lib().orc_param_count(ctypes.byref(self._desc))

    def close(self):
        if self._h:
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != 0:
            raise RuntimeError("oracle: " + lib().orc_last_error().decode())

    def step(self, actions=None, want_logits=False, want_sampled=False):
        act = None if actions is None else np.ascontiguousarray(actions, dtype=np.uint8)
        logits = np.empty((self.cap, self.A), dtype=np.float64) if want_logits else None
        sampled = np.empty(self.cap, dtype=np.uint8) if want_sampled else None
        self._check(lib().orc_step(self._h, _ptr(act), _ptr(logits), _ptr(sampled)))
        return logits, sampled

    def agent_logits(self, slot):
        out = np.empty(self.A, dtype=np.float64)
        self._check(lib().orc_agent_logits(self._h, slot, _ptr(out)))
        return out

    def colour(self, slot):
        out = np.empty(3, dtype=np.float32)
        self._check(lib().orc_read_colour(self._h, slot, _ptr(out)))
        return out

    def write_colour(self, slot, rgb):
        v = np.ascontiguousarray(rgb, dtype=np.float32)
        self._check(lib().orc_write_colour(self._h, slot, _ptr(v)))

    def terrain(self):
        out = np.empty(self.W * self.H, dtype=np.int32)
        self._check(lib().orc_read_terrain(self._h, _ptr(out)))
        return out

    def write_terrain(self, rock):
        v = np.ascontiguousarray(rock, dtype=np.int32)
        assert v.size == self.W * self.H
        self._check(lib().orc_write_terrain(self._h, _ptr(v)))

    def observe(self, slot):
        out = np.empty(self.D, dtype=np.float64)
        self._check(lib().orc_observe(self._h, slot, _ptr(out)))
        return out

    def weights(self, slot, master=False):
        out = np.empty(self.P, dtype=np.float64)
        self._check(lib().orc_read_weights(self._h, slot, 1 if master else 0, _ptr(out)))
        return out

    def state_bytes(self):
        return lib().orc_state_bytes(self._h)

    def read_state_raw(self):
        buf = np.empty(self.state_bytes(), dtype=np.uint8)
        self._check(lib().orc_read_state(self._h, _ptr(buf), buf.nbytes))
        return buf

    def write_state_raw(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        self._check(lib().orc_write_state(self._h, _ptr(buf), buf.nbytes))

    def state(self):
        return unpack_state(self.read_state_raw(), self.cap, self.W * self.H, self.cfg.get("flags", 0) & ECOLOGY)

    def write_state(self, st: dict):
        self.write_state_raw(pack_state(st, self.W, self.H, self.cap))

    def stats(self):
        s = OrcStats()
        self._check(lib().orc_stats_get(self._h, ctypes.byref(s)))
        return s.as_dict()


# State layout: header (u64 step, u64 uid_next, u32 width, u32 height, u32 cap, u32 0),
# then uid, parent_uid (u64), pos, energy, age (i32) per slot, occ (i32) per cell,
# facing, alive, action (u8) per slot, res, wall (u8) per cell.
_FIELDS = [("uid", np.uint64, "cap"), ("parent_uid", np.uint64, "cap"), ("pos", np.int32, "cap"),
           ("energy", np.int32, "cap"), ("age", np.int32, "cap"), ("occ", np.int32, "cells"),
           ("facing", np.uint8, "cap"), ("alive", np.uint8, "cap"), ("action", np.uint8, "cap"),
           ("res", np.uint8, "cells"), ("wall", np.uint8, "cells")]
# then, in the ecology, water, biomass, hp (i32) per slot and water, energy, biomass (i32) per cell
ECO_FIELDS = [("water", np.int32, "cap"), ("biomass", np.int32, "cap"), ("hp", np.int32, "cap"),
              ("cell_water", np.int32, "cells"), ("cell_energy", np.int32, "cells"),
              ("cell_biomass", np.int32, "cells")]


def unpack_state(buf, cap, cells, ecology=False):
    buf = np.asarray(buf, dtype=np.uint8)
    hdr = buf[:32]
    st = {"step": int(hdr[0:8].view(np.uint64)[0]), "uid_next": int(hdr[8:16].view(np.uint64)[0])}
    off = 32
    for name, dt, kind in _FIELDS + (ECO_FIELDS if ecology else []):
        n = cap if kind == "cap" else cells
        nb = n * np.dtype(dt).itemsize
        st[name] = buf[off:off + nb].view(dt).copy()
        off += nb
    return st


def pack_state(st, width, height, cap):
    cells = width * height
    parts = [np.array([st["step"], st["uid_next"]], dtype=np.uint64).view(np.uint8),
             np.array([width, height, cap, 0], dtype=np.uint32).view(np.uint8)]
    for name, dt, kind in _FIELDS + (ECO_FIELDS if "hp" in st else []):
        n = cap if kind == "cap" else cells
        a = np.ascontiguousarray(st[name], dtype=dt)
        assert a.size == n, name
        parts.append(a.view(np.uint8).ravel())
    return np.concatenate(parts)

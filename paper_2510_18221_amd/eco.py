"""Python binding of libeco.so (argument marshalling only).

Every step of the world runs in the library's HIP kernels; this module only
converts between Python/numpy values and the C ABI of include/eco.h.  PyTorch
supplies the device allocator and the HIP stream.  There is no CPU fallback:
if the library is missing the import fails.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libeco.so")

ECO_OK, ECO_EINVAL, ECO_ENOMEM, ECO_EDEVICE, ECO_ESTATE, ECO_ENOTSUP = 0, -1, -2, -3, -4, -5
RT_KEEP_LOGITS, RT_USE_GRAPH, RT_TIME_KERNELS, RT_SPLIT_STEP = 1, 2, 4, 8
DESC_FRONT_VISION, DESC_EVOLVE_TEMPERATURE, DESC_COLOUR_VISION, DESC_ECOLOGY, DESC_TERRAIN = 1, 2, 4, 8, 16
KERNELS = ["forward", "move", "birth_claim", "birth_scan", "birth_commit", "regrow", "compact", "sense"]

EXPORTS = ["eco_world_create", "eco_world_destroy", "eco_last_error", "eco_world_step", "eco_world_reset",
           "eco_world_stats", "eco_world_stats_history", "eco_world_info", "eco_world_set_flags",
           "eco_world_set_launch", "eco_world_get_launch", "eco_world_autotune", "eco_world_kernel_times",
           "eco_world_step_with_actions", "eco_world_state_bytes", "eco_world_read_state",
           "eco_world_write_state", "eco_world_read_logits", "eco_world_read_sampled", "eco_world_read_weights",
           "eco_world_write_weights", "eco_world_prepare", "eco_stream_read_gbps", "eco_world_read_colours",
           "eco_world_write_colour", "eco_world_read_terrain", "eco_world_write_terrain", "eco_world_step_static",
           "eco_world_autotune_cached"]


class EcoError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"eco status {status}: {msg}")
        self.status = status


class Ecology(ctypes.Structure):
    """eco_ecology of include/eco.h."""
    _fields_ = [("water_density", ctypes.c_float), ("energy_density", ctypes.c_float),
                ("biomass_density", ctypes.c_float)] + [(n, ctypes.c_int32) for n in (
                    "water_site", "energy_site", "biomass_site", "eat_water", "eat_biomass", "cap_water",
                    "cap_energy", "cap_biomass", "e_cost_move", "w_cost")] + [("photo_rate", ctypes.c_float)] + [
                (n, ctypes.c_int32) for n in ("cell_energy_max", "hp_max", "hp_child", "hp_overspend", "hp_heal",
                                              "heal_energy", "age_shift", "w_init", "b_init", "w_child", "b_child",
                                              "b_repro", "terrain_scale", "sea_level", "water_per_depth",
                                              "attack_damage")]


class Desc(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("width", ctypes.c_uint32), ("height", ctypes.c_uint32),
        ("n_agents_init", ctypes.c_uint32), ("capacity", ctypes.c_uint32),
        ("resource_density", ctypes.c_float), ("regrow_prob", ctypes.c_float), ("mutation_sigma", ctypes.c_float),
        ("window", ctypes.c_uint32), ("n_scalars", ctypes.c_uint32), ("hidden1", ctypes.c_uint32),
        ("hidden2", ctypes.c_uint32), ("n_actions", ctypes.c_uint32),
        ("e_init", ctypes.c_int32), ("e_cost", ctypes.c_int32), ("e_eat", ctypes.c_int32),
        ("e_repro", ctypes.c_int32), ("e_child", ctypes.c_int32),
        ("wdtype", ctypes.c_uint32), ("keep_master", ctypes.c_uint32), ("attack_enabled", ctypes.c_uint32),
        ("flags", ctypes.c_uint32), ("eco", Ecology), ("seed", ctypes.c_uint64),
    ]


class Stats(ctypes.Structure):
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


class Launch(ctypes.Structure):
    _fields_ = [("waves_per_block", ctypes.c_uint32), ("blocks_per_cu", ctypes.c_uint32),
                ("unroll", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class Info(ctypes.Structure):
    _fields_ = [("n_worlds", ctypes.c_uint32), ("total_slots", ctypes.c_uint32), ("total_cells", ctypes.c_uint64),
                ("input_dim", ctypes.c_uint32), ("hidden1", ctypes.c_uint32), ("hidden2", ctypes.c_uint32),
                ("n_actions", ctypes.c_uint32), ("param_count", ctypes.c_uint64),
                ("weight_bytes_per_agent", ctypes.c_uint64), ("storage_stride", ctypes.c_uint64),
                ("master_stride", ctypes.c_uint64), ("device_bytes", ctypes.c_uint64), ("n_cus", ctypes.c_uint32),
                ("wdtype", ctypes.c_uint32)]


class KernelTimes(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 8), ("launches", ctypes.c_uint64 * 8)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", ctypes.c_void_p)]


_lib = None


def lib():
    """Load libeco.so; raises if it has not been built (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2510_18221_amd.build`")
        try:   # torch's HIP runtime first, so that the library binds to the same one torch's memory comes from
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        P, U32, I32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int
        L.eco_last_error.restype = ctypes.c_char_p
        L.eco_world_create.argtypes = [ctypes.POINTER(Desc), U32, P, ctypes.POINTER(Allocator),
                                       ctypes.POINTER(ctypes.c_void_p)]
        L.eco_world_destroy.argtypes = [P]
        L.eco_world_destroy.restype = None
        L.eco_world_step.argtypes = [P, U32]
        L.eco_world_step_static.argtypes = [P, U32]
        L.eco_world_autotune_cached.argtypes = [P, ctypes.c_char_p, ctypes.POINTER(Launch), ctypes.POINTER(ctypes.c_int)]
        L.eco_world_prepare.argtypes = [P, U32]
        L.eco_stream_read_gbps.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)]
        L.eco_world_reset.argtypes = [P, P]
        L.eco_world_stats.argtypes = [P, ctypes.POINTER(Stats), U32]
        L.eco_world_stats_history.argtypes = [P, U32, ctypes.POINTER(Stats), U32, ctypes.POINTER(ctypes.c_uint32)]
        L.eco_world_info.argtypes = [P, ctypes.POINTER(Info)]
        L.eco_world_set_flags.argtypes = [P, U32]
        L.eco_world_set_launch.argtypes = [P, ctypes.POINTER(Launch)]
        L.eco_world_get_launch.argtypes = [P, ctypes.POINTER(Launch)]
        L.eco_world_autotune.argtypes = [P, ctypes.POINTER(Launch)]
        L.eco_world_kernel_times.argtypes = [P, ctypes.POINTER(KernelTimes), I32]
        L.eco_world_step_with_actions.argtypes = [P, P]
        L.eco_world_state_bytes.argtypes = [P, U32]
        L.eco_world_state_bytes.restype = ctypes.c_size_t
        L.eco_world_read_state.argtypes = [P, U32, P, ctypes.c_size_t]
        L.eco_world_write_state.argtypes = [P, U32, P, ctypes.c_size_t]
        L.eco_world_read_logits.argtypes = [P, U32, P, ctypes.c_size_t]
        L.eco_world_read_sampled.argtypes = [P, U32, P, ctypes.c_size_t]
        L.eco_world_read_weights.argtypes = [P, U32, U32, I32, P, ctypes.c_size_t]
        L.eco_world_write_weights.argtypes = [P, U32, U32, P, ctypes.c_size_t]
        L.eco_world_read_colours.argtypes = [P, U32, P, ctypes.c_size_t]
        L.eco_world_write_colour.argtypes = [P, U32, U32, P]
        L.eco_world_read_terrain.argtypes = [P, U32, P, ctypes.c_size_t]
        L.eco_world_write_terrain.argtypes = [P, U32, P, ctypes.c_size_t]
        for name in EXPORTS:
            getattr(L, name)
        _lib = L
    return _lib


def _err(status):
    if status != ECO_OK:
        raise EcoError(status, lib().eco_last_error().decode())


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def make_desc(cfg: dict) -> Desc:
    d = Desc()
    for name, _ in Desc._fields_:
        if name == "eco":
            for en, _ in Ecology._fields_:
                if en in cfg.get("eco", {}):
                    setattr(d.eco, en, cfg["eco"][en])
        elif name in cfg:
            setattr(d, name, cfg[name])
    d.struct_size = ctypes.sizeof(Desc)
    return d


class _TorchAllocator:
    """Routes the library's device allocations through torch's caching allocator."""

    def __init__(self, torch, device, stream_ptr):
        self.torch, self.device, self.stream = torch, device, stream_ptr
        self._alloc = ALLOC_FN(self.alloc)
        self._free = FREE_FN(self.free)
        self.struct = Allocator(self._alloc, self._free, None)

    def alloc(self, nbytes, ctx):
        try:
            return self.torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
        except Exception:  # noqa: BLE001 - the library reports ENOMEM
            return None

    def free(self, ptr, ctx):
        cuda = getattr(self.torch, "cuda", None)
        if cuda is None:   # interpreter shutdown: torch's modules are already torn down
            return
        cuda.caching_allocator_delete(ptr)


class World:
    """One libeco object holding one or more worlds (same policy shape)."""

    def __init__(self, descs, stream=None, torch_memory=True):
        if isinstance(descs, dict):
            descs = [descs]
        self.cfgs = [dict(c) for c in descs]
        arr = (Desc * len(descs))(*[make_desc(c) for c in descs])
        self._allocator = None
        stream_ptr = None
        if torch_memory:
            import torch
            dev = torch.cuda.current_device()
            st = stream if stream is not None else torch.cuda.current_stream(dev)
            stream_ptr = st.cuda_stream if hasattr(st, "cuda_stream") else int(st)
            self._allocator = _TorchAllocator(torch, dev, stream_ptr)
        elif stream is not None:
            stream_ptr = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        h = ctypes.c_void_p()
        alloc = ctypes.byref(self._allocator.struct) if self._allocator else None
        _err(lib().eco_world_create(arr, len(descs), stream_ptr, alloc, ctypes.byref(h)))
        self._h = h
        self.n_worlds = len(descs)
        self.A = self.cfgs[0]["n_actions"]
        self.info = self.get_info()
        self.P = self.info["param_count"]

    # -- lifecycle --------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            lib().eco_world_destroy(self._h)
            self._h = None
            if self._allocator is not None:
                self._allocator.torch.cuda.empty_cache()  # hand large blocks back for the next world

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- stepping ---------------------------------------------------------
    def step(self, n=1):
        _err(lib().eco_world_step(self._h, n))

    def step_static(self, n=1):
        """eco_world_step_static: the same steps with the static scratch array (no allocation)."""
        _err(lib().eco_world_step_static(self._h, n))

    def prepare(self, n=1):
        _err(lib().eco_world_prepare(self._h, n))

    def step_with_actions(self, actions):
        a = np.ascontiguousarray(actions, dtype=np.uint8)
        assert a.size == sum(c["capacity"] for c in self.cfgs)
        _err(lib().eco_world_step_with_actions(self._h, _ptr(a)))

    def reset(self, seeds=None):
        if seeds is None:
            _err(lib().eco_world_reset(self._h, None))
        else:
            s = np.ascontiguousarray(seeds, dtype=np.uint64)
            _err(lib().eco_world_reset(self._h, _ptr(s)))

    # -- observation ------------------------------------------------------
    def stats(self):
        arr = (Stats * self.n_worlds)()
        _err(lib().eco_world_stats(self._h, arr, self.n_worlds))
        return [s.as_dict() for s in arr]

    def stats_history(self, world=0, n=1024):
        arr = (Stats * n)()
        got = ctypes.c_uint32()
        _err(lib().eco_world_stats_history(self._h, world, arr, n, ctypes.byref(got)))
        return [arr[i].as_dict() for i in range(got.value)]

    def get_info(self):
        i = Info()
        _err(lib().eco_world_info(self._h, ctypes.byref(i)))
        return {n: getattr(i, n) for n, _ in Info._fields_}

    def set_flags(self, flags):
        _err(lib().eco_world_set_flags(self._h, flags))

    def set_launch(self, waves_per_block, blocks_per_cu, unroll):
        lc = Launch(waves_per_block, blocks_per_cu, unroll, 0)
        _err(lib().eco_world_set_launch(self._h, ctypes.byref(lc)))

    def get_launch(self):
        lc = Launch()
        _err(lib().eco_world_get_launch(self._h, ctypes.byref(lc)))
        return dict(waves_per_block=lc.waves_per_block, blocks_per_cu=lc.blocks_per_cu, unroll=lc.unroll)

    def autotune(self, cache=None):
        """Tune the policy-kernel launch; cache: path of the result cache (JSON lines),
        whose entry for this object's key is used instead of timing when present."""
        lc = Launch()
        if cache is None:
            _err(lib().eco_world_autotune(self._h, ctypes.byref(lc)))
            hit = 0
        else:
            h = ctypes.c_int(0)
            _err(lib().eco_world_autotune_cached(self._h, os.fsencode(cache), ctypes.byref(lc), ctypes.byref(h)))
            hit = h.value
        return dict(waves_per_block=lc.waves_per_block, blocks_per_cu=lc.blocks_per_cu, unroll=lc.unroll,
                    **({"from_cache": bool(hit)} if cache is not None else {}))

    def kernel_times(self, reset=False):
        kt = KernelTimes()
        _err(lib().eco_world_kernel_times(self._h, ctypes.byref(kt), 1 if reset else 0))
        return {k: (kt.ms[i], kt.launches[i]) for i, k in enumerate(KERNELS)}

    def read_state_raw(self, world=0):
        n = lib().eco_world_state_bytes(self._h, world)
        buf = np.empty(n, dtype=np.uint8)
        _err(lib().eco_world_read_state(self._h, world, _ptr(buf), n))
        return buf

    def read_state(self, world=0):
        c = self.cfgs[world]
        return unpack_state(self.read_state_raw(world), c["capacity"], c["width"] * c["height"],
                            c.get("flags", 0) & DESC_ECOLOGY)

    def write_state(self, st, world=0):
        c = self.cfgs[world]
        buf = pack_state(st, c["width"], c["height"], c["capacity"])
        _err(lib().eco_world_write_state(self._h, world, _ptr(buf), buf.nbytes))

    def read_logits(self, world=0):
        cap = self.cfgs[world]["capacity"]
        out = np.empty((cap, self.A), dtype=np.float32)
        _err(lib().eco_world_read_logits(self._h, world, _ptr(out), out.size))
        return out

    def read_sampled(self, world=0):
        cap = self.cfgs[world]["capacity"]
        out = np.empty(cap, dtype=np.uint8)
        _err(lib().eco_world_read_sampled(self._h, world, _ptr(out), cap))
        return out

    def read_weights(self, slot, world=0, master=False):
        out = np.empty(self.P, dtype=np.float64)
        _err(lib().eco_world_read_weights(self._h, world, slot, 1 if master else 0, _ptr(out), self.P))
        return out

    def write_weights(self, slot, master, world=0):
        m = np.ascontiguousarray(master, dtype=np.float32)
        _err(lib().eco_world_write_weights(self._h, world, slot, _ptr(m), m.size))

    def read_terrain(self, world=0):
        c = self.cfgs[world]
        out = np.empty(c["width"] * c["height"], dtype=np.int32)
        _err(lib().eco_world_read_terrain(self._h, world, _ptr(out), out.size))
        return out

    def write_terrain(self, rock, world=0):
        v = np.ascontiguousarray(rock, dtype=np.int32)
        _err(lib().eco_world_write_terrain(self._h, world, _ptr(v), v.size))

    def read_colours(self, world=0):
        cap = self.cfgs[world]["capacity"]
        out = np.empty((cap, 3), dtype=np.float32)
        _err(lib().eco_world_read_colours(self._h, world, _ptr(out), out.size))
        return out

    def write_colour(self, slot, rgb, world=0):
        v = np.ascontiguousarray(rgb, dtype=np.float32)
        assert v.size == 3
        _err(lib().eco_world_write_colour(self._h, world, slot, _ptr(v)))


# State byte layout of include/eco.h (read_state / write_state).
_FIELDS = [("uid", np.uint64, "cap"), ("parent_uid", np.uint64, "cap"), ("pos", np.int32, "cap"),
           ("energy", np.int32, "cap"), ("age", np.int32, "cap"), ("occ", np.int32, "cells"),
           ("facing", np.uint8, "cap"), ("alive", np.uint8, "cap"), ("action", np.uint8, "cap"),
           ("res", np.uint8, "cells"), ("wall", np.uint8, "cells")]
# appended with ECO_DESC_ECOLOGY
_ECO_FIELDS = [("water", np.int32, "cap"), ("biomass", np.int32, "cap"), ("hp", np.int32, "cap"),
               ("cell_water", np.int32, "cells"), ("cell_energy", np.int32, "cells"),
               ("cell_biomass", np.int32, "cells")]


def unpack_state(buf, cap, cells, ecology=False):
    buf = np.asarray(buf, dtype=np.uint8)
    st = {"step": int(buf[0:8].view(np.uint64)[0]), "uid_next": int(buf[8:16].view(np.uint64)[0])}
    off = 32
    for name, dt, kind in _FIELDS + (_ECO_FIELDS if ecology else []):
        n = cap if kind == "cap" else cells
        nb = n * np.dtype(dt).itemsize
        st[name] = buf[off:off + nb].view(dt).copy()
        off += nb
    return st


def pack_state(st, width, height, cap):
    cells = width * height
    parts = [np.array([st["step"], st["uid_next"]], dtype=np.uint64).view(np.uint8),
             np.array([width, height, cap, 0], dtype=np.uint32).view(np.uint8)]
    for name, dt, kind in _FIELDS + (_ECO_FIELDS if "hp" in st else []):
        n = cap if kind == "cap" else cells
        a = np.ascontiguousarray(st[name], dtype=dt)
        assert a.size == n, name
        parts.append(a.view(np.uint8).ravel())
    return np.concatenate(parts)


def stream_read_gbps(nbytes=8 << 30, stream=None):
    """The device's streaming-read rate (GB/s) from the library's probe kernel."""
    import torch
    g = ctypes.c_double(0.0)
    s = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    _err(lib().eco_stream_read_gbps(ctypes.c_void_p(s), nbytes, ctypes.byref(g)))
    return g.value

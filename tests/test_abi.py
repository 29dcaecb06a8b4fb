"""The C-ABI library loads and exports every symbol include/eco.h declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "eco.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(eco_[a-z_]+)\s*\(", text)))


def test_header_declares_boundary():
    names = declared_functions()
    for required in ("eco_world_create", "eco_world_step", "eco_world_reset", "eco_world_stats"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2510_18221_amd import eco
    lib = eco.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(eco.EXPORTS) == sorted(declared_functions())


def test_validation_errors_without_device():
    """Descriptor checks run before any HIP call, so they are testable on the CPU."""
    from paper_2510_18221_amd import eco
    from paper_2510_18221_amd import workloads as wl
    lib = eco.lib()
    out = ctypes.c_void_p()
    assert lib.eco_world_create(None, 0, None, None, ctypes.byref(out)) == eco.ECO_EINVAL
    for bad, status in [(dict(window=4), eco.ECO_EINVAL), (dict(n_scalars=3), eco.ECO_EINVAL),
                        (dict(hidden1=48, hidden2=48), eco.ECO_ENOTSUP), (dict(attack_enabled=1), eco.ECO_EINVAL),
                        (dict(n_actions=7, attack_enabled=2), eco.ECO_EINVAL),
                        (dict(capacity=10), eco.ECO_EINVAL), (dict(e_repro=0), eco.ECO_EINVAL),
                        (dict(window=17), eco.ECO_ENOTSUP), (dict(flags=32), eco.ECO_EINVAL),
                        (dict(n_actions=8), eco.ECO_EINVAL), (dict(flags=16), eco.ECO_EINVAL),
                        (dict(flags=8, n_actions=8, n_scalars=4, eco=wl.ECOLOGY), eco.ECO_EINVAL),
                        (dict(flags=8, n_actions=9, n_scalars=8, eco=wl.ECOLOGY), eco.ECO_EINVAL),
                        (dict(flags=8, n_actions=9, n_scalars=8, attack_enabled=1,
                              eco=dict(wl.ECOLOGY, attack_damage=-1)), eco.ECO_EINVAL),
                        (dict(flags=8 | 16, n_actions=8, n_scalars=8, eco=dict(wl.ECOLOGY, sea_level=40)),
                         eco.ECO_EINVAL),
                        (dict(flags=8, n_actions=8, n_scalars=8, eco=dict(wl.ECOLOGY, b_repro=0)), eco.ECO_EINVAL)]:
        d = (eco.Desc * 1)(eco.make_desc(wl.desc(**bad)))
        assert lib.eco_world_create(d, 1, None, None, ctypes.byref(out)) == status, bad
        assert lib.eco_last_error()
    d = eco.make_desc(wl.desc())
    d.struct_size = 4
    assert lib.eco_world_create((eco.Desc * 1)(d), 1, None, None, ctypes.byref(out)) == eco.ECO_EINVAL
    assert b"struct_size" in lib.eco_last_error()


def test_struct_sizes_match_header(tmp_path):
    """The ctypes mirrors of eco_world_desc, eco_stats and eco_launch have the header's size and
    field offsets (the header compiled by the host C compiler)."""
    import subprocess
    from paper_2510_18221_amd import eco
    fields = {"Desc": [n for n, _ in eco.Desc._fields_], "Stats": [n for n, _ in eco.Stats._fields_],
              "Launch": [n for n, _ in eco.Launch._fields_]}
    cname = {"Desc": "eco_world_desc", "Stats": "eco_stats", "Launch": "eco_launch"}
    src = ["#include <stdio.h>", "#include <stddef.h>", '#include "eco.h"', "int main(void) {"]
    for k, names in fields.items():
        src.append(f'printf("{k} %zu\\n", sizeof({cname[k]}));')
        for n in names:
            src.append(f'printf("{k}.{n} %zu\\n", offsetof({cname[k]}, {n}));')
    src.append("return 0; }")
    (tmp_path / "t.c").write_text("\n".join(src))
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run(["gcc", "-I", inc, "-o", str(tmp_path / "t"), str(tmp_path / "t.c")], check=True)
    out = dict(l.rsplit(" ", 1) for l in subprocess.run([str(tmp_path / "t")], capture_output=True, text=True,
                                                       check=True).stdout.split("\n") if l)
    for k in fields:
        cls = getattr(eco, k)
        assert int(out[k]) == ctypes.sizeof(cls), k
        for n in fields[k]:
            assert int(out[f"{k}.{n}"]) == getattr(cls, n).offset, (k, n)


def _counting_allocator(eco, fail_at):
    """An allocator that hands out distinct fake addresses (never dereferenced on
    these paths) and returns NULL at call number fail_at; it records frees."""
    state = {"calls": 0, "live": set(), "freed": []}

    def alloc(nbytes, ctx):
        i = state["calls"]
        state["calls"] += 1
        if i == fail_at:
            return None
        addr = 0x10000000 + 0x100000 * i
        state["live"].add(addr)
        return addr

    def free(ptr, ctx):
        state["freed"].append(ptr)
        state["live"].discard(ptr)

    fa, ff = eco.ALLOC_FN(alloc), eco.FREE_FN(free)
    return eco.Allocator(fa, ff, None), state, (fa, ff)


def test_allocator_null_gives_enomem_and_no_leak():
    """An allocator that returns NULL on its k-th call: eco_world_create reports
    ECO_ENOMEM, gives every earlier allocation back through the allocator's free,
    and leaves *out NULL.  The allocations come before any device call when the
    caller brings the allocator, so this runs without a GPU."""
    import torch
    from paper_2510_18221_amd import eco
    from paper_2510_18221_amd import workloads as wl
    lib = eco.lib()
    d = (eco.Desc * 1)(eco.make_desc(wl.desc()))
    sentinel = 0xDEAD0000
    n_total = None
    if not torch.cuda.is_available():
        # every allocation succeeds: the device query then fails, and all is given back
        al, st, keep = _counting_allocator(eco, fail_at=-1)
        out = ctypes.c_void_p(sentinel)
        assert lib.eco_world_create(d, 1, None, ctypes.byref(al), ctypes.byref(out)) == eco.ECO_EDEVICE
        assert out.value is None and not st["live"] and len(st["freed"]) == st["calls"] > 10
        n_total = st["calls"]
    for k in [0, 1, 7] + ([n_total // 2, n_total - 1] if n_total else []):
        al, st, keep = _counting_allocator(eco, fail_at=k)
        out = ctypes.c_void_p(sentinel)
        assert lib.eco_world_create(d, 1, None, ctypes.byref(al), ctypes.byref(out)) == eco.ECO_ENOMEM, k
        assert b"allocation" in lib.eco_last_error()
        assert out.value is None, k
        assert st["calls"] == k + 1, (k, st["calls"])      # nothing allocated after the failure
        assert not st["live"] and len(st["freed"]) == k, k  # everything before it given back


def test_create_sets_out_to_null_on_error():
    from paper_2510_18221_amd import eco
    from paper_2510_18221_amd import workloads as wl
    lib = eco.lib()
    out = ctypes.c_void_p(0xDEAD0000)
    d = (eco.Desc * 1)(eco.make_desc(wl.desc(window=4)))
    assert lib.eco_world_create(d, 1, None, None, ctypes.byref(out)) == eco.ECO_EINVAL
    assert out.value is None

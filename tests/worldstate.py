"""Test helpers: hand-built world states and state comparison (no step arithmetic)."""
import numpy as np

N, E, S, W = 0, 1, 2, 3


def empty_state(width, height, cap, step=0, uid_next=100, ecology=False):
    cells = width * height
    st = {"step": step, "uid_next": uid_next,
          "uid": np.zeros(cap, np.uint64), "parent_uid": np.full(cap, 0xFFFFFFFFFFFFFFFF, np.uint64),
          "pos": np.full(cap, -1, np.int32), "energy": np.zeros(cap, np.int32), "age": np.zeros(cap, np.int32),
          "occ": np.full(cells, -1, np.int32), "facing": np.zeros(cap, np.uint8), "alive": np.zeros(cap, np.uint8),
          "action": np.zeros(cap, np.uint8), "res": np.zeros(cells, np.uint8), "wall": np.zeros(cells, np.uint8)}
    if ecology:
        for f in ("water", "biomass", "hp"):
            st[f] = np.zeros(cap, np.int32)
        for f in ("cell_water", "cell_energy", "cell_biomass"):
            st[f] = np.zeros(cells, np.int32)
    return st


def place(st, width, slot, x, y, facing, energy, age=0, uid=None):
    cell = y * width + x
    assert st["occ"][cell] == -1
    st["alive"][slot] = 1
    st["pos"][slot] = cell
    st["occ"][cell] = slot
    st["facing"][slot] = facing
    st["energy"][slot] = energy
    st["age"][slot] = age
    st["uid"][slot] = slot if uid is None else uid
    return st


LIVE_FIELDS = ("uid", "parent_uid", "pos", "energy", "age", "facing")


def assert_same_state(a, b, what=""):
    """Bit-exact comparison of the integer world state; dead slots compare only alive."""
    assert a["step"] == b["step"], (what, "step", a["step"], b["step"])
    assert a["uid_next"] == b["uid_next"], (what, "uid_next")
    np.testing.assert_array_equal(a["alive"], b["alive"], err_msg=f"{what} alive")
    live = a["alive"].astype(bool)
    for f in LIVE_FIELDS:
        np.testing.assert_array_equal(a[f][live], b[f][live], err_msg=f"{what} {f}")
    for f in ("occ", "res", "wall"):
        np.testing.assert_array_equal(a[f], b[f], err_msg=f"{what} {f}")
    assert ("hp" in a) == ("hp" in b), (what, "ecology fields on one side only")
    if "hp" in a:   # the three-resource ecology
        for f in ("water", "biomass", "hp"):
            np.testing.assert_array_equal(a[f][live], b[f][live], err_msg=f"{what} {f}")
        for f in ("cell_water", "cell_energy", "cell_biomass"):
            np.testing.assert_array_equal(a[f], b[f], err_msg=f"{what} {f}")


def check_invariants(st, width, height):
    """Occupancy is a bijection with live positions; no two agents share a cell."""
    live = np.nonzero(st["alive"])[0]
    pos = st["pos"][live]
    assert len(np.unique(pos)) == len(pos), "two agents in one cell"
    assert np.all((pos >= 0) & (pos < width * height))
    np.testing.assert_array_equal(st["occ"][pos], live)
    assert int((st["occ"] >= 0).sum()) == len(live)

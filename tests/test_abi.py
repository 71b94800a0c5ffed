"""Host-side checks of the C-ABI library (no GPU needed): it loads, and it
exports every entry point the public header declares."""
import ctypes
import os
import re

import numpy as np

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vt.h")
LIB = os.path.join(ROOT, "paper_1601_06429_amd", "libvt.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vt_[a-z_]+)\s*\(", src)))


def test_header_declares_the_six_hot_path_calls():
    names = declared_functions()
    for f in ("vt_build", "vt_cells", "vt_density", "vt_gradient", "vt_grid_deposit", "vt_backward"):
        assert f in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libvt.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libvt.so not built")
def test_status_strings():
    lib = ctypes.CDLL(LIB)
    lib.vt_status_string.restype = ctypes.c_char_p
    lib.vt_status_string.argtypes = [ctypes.c_int]
    assert lib.vt_status_string(0) == b"ok"
    assert b"duplicate" in lib.vt_status_string(4)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libvt.so not built")
def test_argument_errors_are_synchronous():
    """Invalid arguments are rejected on the host before anything is enqueued."""
    import paper_1601_06429_amd as vt

    L = vt.lib()
    ctx = ctypes.c_void_p(None)
    items = vt._items([dict(offset=0, n_owned=10, n_ghost=0, periodic=True, lo=[0, 0, 0], hi=[1, 1, 2])])
    # non-cubic periodic box
    assert L.vt_build(ctypes.byref(ctx), ctypes.c_void_p(16), vt.VT_F32, None, items, 1, None, None) == 1
    # items not packed back to back
    items = vt._items([dict(offset=5, n_owned=10, periodic=False, lo=[0, 0, 0], hi=[1, 1, 1])])
    assert L.vt_build(ctypes.byref(ctx), ctypes.c_void_p(16), vt.VT_F32, None, items, 1, None, None) == 1
    # no items / null positions
    assert L.vt_build(ctypes.byref(ctx), None, vt.VT_F32, None, items, 1, None, None) == 1
    assert L.vt_build(ctypes.byref(ctx), ctypes.c_void_p(16), vt.VT_F32, None, items, 0, None, None) == 1
    # an empty world: a build needs at least one owned particle per item
    items = vt._items([dict(offset=0, n_owned=0, n_ghost=0, periodic=False, lo=[0, 0, 0], hi=[1, 1, 1])])
    assert L.vt_build(ctypes.byref(ctx), ctypes.c_void_p(16), vt.VT_F32, None, items, 1, None, None) == 1
    # calls on a context that was never built
    assert L.vt_cells(None, None, None, None, 0, None, None) == 7
    sizes = (ctypes.c_int64 * 3)()
    assert L.vt_structure(None, None, None, 0, None, None, 0, None, None, 0, sizes, None) == 7
    assert L.vt_grid_tensor(None, None, 16, 16, 16, 0, None, None) == 7
    assert L.vt_grid_sample(None, None, 8, 8, 8, 1, None, None, None) == 7


def test_autotune_selection_logic():
    from paper_1601_06429_amd import autotune

    c = autotune.candidates()
    assert len(c) == (len(autotune.K_INITS) * len(autotune.PTS_PER_GRID_CELL) * len(autotune.WAVES_PER_CU) *
                      len(autotune.CELL_MAPPINGS))
    assert all(set(o) == {"k_init", "pts_per_grid_cell", "waves_per_cu", "cell_mapping"} for o in c)
    t = [(c[0], 3.0), (c[1], 1.5), (c[2], 1.5), (c[3], 9.0)]
    assert autotune.pick(t) == c[1]  # fastest, earlier one on ties
    a = autotune.signature("MI355X", "torch.float32", 2_097_152, 1, 0)
    b = autotune.signature("MI355X", "torch.float32", 3_000_000, 1, 0)
    d = autotune.signature("MI355X", "torch.float32", 4_500_000, 1, 0)
    assert a == b and a != d


def test_task_grid_schemes():
    from paper_1601_06429_amd import task_grid

    # the paper's example of scheme (a) (section 2): 32 tasks are 4 x 4 x 2
    assert task_grid(32) == (4, 4, 2)
    for k in range(11):
        nt = task_grid(2 ** k)
        assert nt[0] * nt[1] * nt[2] == 2 ** k
        assert nt[0] >= nt[1] >= nt[2] and nt[0] <= 2 * nt[2]   # cuts balanced over the axes
    assert task_grid(1) == (1, 1, 1) and task_grid(64) == (4, 4, 4)
    # scheme (b): slabs along one axis
    assert task_grid(12, "b") == (12, 1, 1) and task_grid(5, "b", axis=2) == (1, 1, 5)
    with pytest.raises(ValueError):
        task_grid(12)              # scheme (a) needs a power of two
    with pytest.raises(ValueError):
        task_grid(4, "c")


@pytest.mark.skipif(not os.path.exists(LIB), reason="libvt.so not built")
def test_border_thresholds_reproduce_the_papers_worked_example():
    """Section 2: BORDERFACTOR 1.5 with an inter-particle distance of 1.58 computed from the whole
    input gives a 2.37 buffer.  The library's own thickness schedule (the one vt_decompose uses)
    for 1000 particles in a cube of side 15.8, whose mean spacing is 1.58."""
    import json

    import paper_1601_06429_amd as vt

    with open(os.path.join(ROOT, "tests", "golden", "ghost_width.json")) as f:
        ex = json.load(f)
    t = vt.border_thresholds(1000, 0.0, 15.8, border_factor=ex["border_factor"])
    assert round(t[0], ex["printed_decimals"]) == ex["buffer_thickness"]
    # and the growth: 48 thicknesses by default, each 1.1 times the one before
    assert len(t) == 48
    np.testing.assert_allclose(t[1:] / t[:-1], 1.1, rtol=1e-14)
    # the spacing comes from the world's volume: a 4 x 1 x 1 slab of 4000 particles has spacing 0.1
    t = vt.border_thresholds(4000, 0.0, [4.0, 1.0, 1.0], border_factor=1.5, n_steps=3, growth=1.5)
    np.testing.assert_allclose(t, [0.15, 0.225, 0.3375], rtol=1e-14)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libvt.so not built")
def test_decomposition_argument_errors():
    import paper_1601_06429_amd as vt

    L = vt.lib()
    ctx = ctypes.c_void_p(None)
    lo, hi = vt._box3(0.0), vt._box3(1.0)
    nt = (ctypes.c_int32 * 3)(2, 2, 2)
    thick = np.zeros(48)
    bad = vt._border(border_factor=-1.0)
    ok = vt._border()
    fake = ctypes.c_void_p(16)
    assert L.vt_decompose(ctypes.byref(ctx), fake, vt.VT_F32, 100, lo, hi, 1, nt, ctypes.byref(bad),
                          vt._dptr(thick), None, None, None) == 1
    assert L.vt_decomposed_build(ctypes.byref(ctx), fake, vt.VT_F32, 100, lo, hi, 1, nt, ctypes.byref(bad),
                                 None, None, None, None, None) == 1
    zero_nt = (ctypes.c_int32 * 3)(0, 1, 1)
    assert L.vt_decompose(ctypes.byref(ctx), fake, vt.VT_F32, 100, lo, hi, 1, zero_nt, ctypes.byref(ok),
                          vt._dptr(thick), None, None, None) == 1
    # a bounded world's exterior face takes no buffer: a positive thickness there is rejected
    th = np.zeros(48)
    th[0] = 0.1                      # face -x of task 0 lies on the world's -x face
    items = (vt.vt_item * 8)()
    n_out = ctypes.c_int64()
    assert L.vt_decompose_pack(ctypes.byref(ctx), fake, vt.VT_F32, 100, lo, hi, 0, nt, vt._dptr(th), None, None,
                               8, None, None, 0, items, ctypes.byref(n_out), None) == 1
    assert ctx.value is None         # nothing was created or enqueued

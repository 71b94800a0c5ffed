"""MI355X-native Voronoi tessellation hot path (ctypes binding of libvt.so).

The functions below mirror the C ABI in ``include/vt.h`` one to one and only
marshal arguments: every step runs in the HIP kernels of ``libvt.so``.  PyTorch
supplies device memory and the current stream.  There is no CPU fallback: if
the library is missing or no GPU is present, the calls raise.

Per particle the engine returns what the paper's code returns (abstract and
section 2): the neighbours sharing a facet, the cell volume, the density
mass/volume, the density gradient, and the average density on a regular grid;
``VoronoiVolume`` adds the volume adjoint for gradient-based use.
"""
from __future__ import annotations

import ctypes
import os
import threading
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
from . import autotune  # noqa: E402,F401  (launch-option tuner; imports torch lazily)

LIB_PATH = os.path.join(_HERE, "libvt.so")
_lib = None
_lock = threading.Lock()

VT_OK = 0
VT_ERR_CAPACITY = 6
STATUS_NAMES = {0: "ok", 1: "invalid argument", 2: "HIP runtime error", 3: "out of device memory",
                4: "duplicate particles", 5: "periodic box too small", 6: "capacity exceeded",
                7: "invalid call order", 8: "inconsistent clipping topology"}
VT_F32, VT_F64 = 0, 1
PREC_FP64, PREC_MIXED = 0, 1
TENSOR_TIDAL, TENSOR_HESSIAN = 0, 1
TENSOR_COMPONENTS = ("xx", "yy", "zz", "xy", "xz", "yz")
CELL_INCOMPLETE, CELL_RETRIED, CELL_FAILED = 1, 2, 4
MAP_XCD, MAP_GLOBAL = 0, 1


class VTError(RuntimeError):
    def __init__(self, code, what=""):
        super().__init__("%s: %s (code %d)" % (what, STATUS_NAMES.get(code, "unknown"), code))
        self.code = code


class vt_item(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_int64), ("n_owned", ctypes.c_int64), ("n_ghost", ctypes.c_int64),
                ("periodic", ctypes.c_int32), ("walls", ctypes.c_int32),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3)]


class vt_border(ctypes.Structure):
    _fields_ = [("border_factor", ctypes.c_double), ("growth", ctypes.c_double), ("n_steps", ctypes.c_int32),
                ("max_reruns", ctypes.c_int32), ("widen", ctypes.c_double)]


class vt_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("want_faces", ctypes.c_int32), ("radius_factor", ctypes.c_float),
                ("area_eps", ctypes.c_float), ("waves_per_cu", ctypes.c_int32), ("timing", ctypes.c_int32),
                ("pts_per_grid_cell", ctypes.c_float), ("k_init", ctypes.c_int32), ("cell_mapping", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


def _load_cdll():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libvt.so not built; run `python -c 'import __graft_entry__ as g; g.build()'`")
    return ctypes.CDLL(LIB_PATH)


def lib():
    """Load libvt.so (raises if it has not been built).

    PyTorch-ROCm ships its own HIP runtime.  libvt must share the runtime that
    owns the tensors, so torch (and, on a GPU machine, its HIP runtime) is
    loaded before libvt: libvt's HIP symbols then bind to that runtime instead
    of a second copy that would not see the device.
    """
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError("libvt.so not built; run `python -c 'import __graft_entry__ as g; g.build()'`")
            import torch

            if torch.cuda.is_available():
                torch.cuda.init()
            L = _load_cdll()
            P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
            L.vt_build.argtypes = [ctypes.POINTER(P), P, I32, P, ctypes.POINTER(vt_item), I32,
                                   ctypes.POINTER(vt_opts), P]
            L.vt_cells.argtypes = [P, P, P, P, I64, P, P]
            L.vt_density.argtypes = [P, P, I32, P, P]
            L.vt_gradient.argtypes = [P, P, P, P]
            L.vt_grid_deposit.argtypes = [P, P, I32, I32, I32, P, P]
            L.vt_grid_sample.argtypes = [P, P, I32, I32, I32, I32, P, P, P]
            L.vt_backward.argtypes = [P, P, P, P]
            L.vt_query.argtypes = [P, ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(I64)]
            L.vt_stats.argtypes = [P, P, P, P, P]
            L.vt_sizes.argtypes = [P, ctypes.POINTER(I64), ctypes.POINTER(I64)]
            L.vt_timings.argtypes = [P, ctypes.POINTER(ctypes.c_float)]
            D3 = ctypes.POINTER(ctypes.c_double)
            BP = ctypes.POINTER(vt_border)
            L.vt_task_grid.argtypes = [I32, I32, I32, ctypes.POINTER(I32)]
            L.vt_border_thresholds.argtypes = [I64, D3, D3, BP, D3]
            L.vt_decompose.argtypes = [ctypes.POINTER(P), P, I32, I64, D3, D3, I32, ctypes.POINTER(I32), BP, D3,
                                       ctypes.POINTER(I64), ctypes.POINTER(I64), P]
            L.vt_decompose_pack.argtypes = [ctypes.POINTER(P), P, I32, I64, D3, D3, I32, ctypes.POINTER(I32), D3,
                                            P, ctypes.POINTER(I32), I32, P, P, I64, ctypes.POINTER(vt_item),
                                            ctypes.POINTER(I64), P]
            L.vt_decomposed_build.argtypes = [ctypes.POINTER(P), P, I32, I64, D3, D3, I32, ctypes.POINTER(I32), BP,
                                              ctypes.POINTER(vt_opts), D3, ctypes.POINTER(I64),
                                              ctypes.POINTER(I32), P]
            L.vt_structure.argtypes = [P, P, P, I64, P, P, I64, P, P, I64, ctypes.POINTER(I64), P]
            L.vt_grid_tensor.argtypes = [P, P, I32, I32, I32, I32, P, P]
            L.vt_grid_tensor_noalloc.argtypes = [P, P, I32, I32, I32, I32, P, P]
            L.vt_destroy.argtypes = [P]
            L.vt_destroy.restype = None
            L.vt_status_string.argtypes = [I32]
            L.vt_status_string.restype = ctypes.c_char_p
            for f in ("vt_build", "vt_cells", "vt_density", "vt_gradient", "vt_grid_deposit", "vt_backward",
                      "vt_query", "vt_stats", "vt_sizes", "vt_timings", "vt_decompose", "vt_decompose_pack",
                      "vt_grid_sample", "vt_structure", "vt_grid_tensor", "vt_grid_tensor_noalloc", "vt_task_grid", "vt_border_thresholds",
                      "vt_decomposed_build"):
                getattr(L, f).restype = ctypes.c_int32
            _lib = L
    return _lib


def _check(code, what):
    if code != VT_OK:
        raise VTError(code, what)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _require_cuda(t, name):
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


def whole_box(n, box_lo, box_hi, periodic=True, walls=0):
    """Item list for a single world of n owned particles (``walls``: true-boundary faces of a
    bounded world, vt_item.walls; 63 = a whole bounded world)."""
    lo = np.broadcast_to(np.asarray(box_lo, np.float64), 3)
    hi = np.broadcast_to(np.asarray(box_hi, np.float64), 3)
    return [dict(offset=0, n_owned=int(n), n_ghost=0, periodic=bool(periodic), lo=lo, hi=hi,
                 walls=0 if periodic else int(walls))]


def pack_worlds(worlds):
    """Pack bounded worlds into one batch for ``vt_build``.

    ``worlds`` is a sequence of (owned, ghosts, lo, hi): owned and ghost
    positions (n x 3 arrays of one dtype) and the world's box [lo, hi] (the
    owned region plus its buffer).  Returns (positions, items, global_ids):
    positions concatenated world by world, owned first, the item list, and
    int32 global ids equal to the position row.
    """
    parts, items, off = [], [], 0
    for owned, ghosts, lo, hi in worlds:
        parts += [owned, ghosts]
        items.append(dict(offset=off, n_owned=len(owned), n_ghost=len(ghosts), periodic=False,
                          lo=np.broadcast_to(np.asarray(lo, np.float64), 3),
                          hi=np.broadcast_to(np.asarray(hi, np.float64), 3)))
        off += len(owned) + len(ghosts)
    pos = np.ascontiguousarray(np.concatenate(parts))
    return pos, items, np.arange(off, dtype=np.int32)


def _pos_dtype(pos):
    import torch

    _require_cuda(pos, "pos")
    if pos.dim() != 2 or pos.shape[1] != 3:
        raise ValueError("pos must be n x 3")
    if pos.dtype == torch.float32:
        return VT_F32
    if pos.dtype == torch.float64:
        return VT_F64
    raise ValueError("pos must be float32 or float64")


def _box3(v):
    return (ctypes.c_double * 3)(*[float(x) for x in np.broadcast_to(np.asarray(v, np.float64), 3)])


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _items(items):
    arr = (vt_item * len(items))()
    for k, it in enumerate(items):
        arr[k].offset = int(it["offset"])
        arr[k].n_owned = int(it["n_owned"])
        arr[k].n_ghost = int(it.get("n_ghost", 0))
        arr[k].periodic = 1 if it.get("periodic", False) else 0
        arr[k].walls = int(it.get("walls", 0))
        for a in range(3):
            arr[k].lo[a] = float(np.broadcast_to(it["lo"], 3)[a])
            arr[k].hi[a] = float(np.broadcast_to(it["hi"], 3)[a])
    return arr


@dataclass
class Cells:
    volume: object     # torch float64 [n_owned]
    nbr_off: object    # torch int64 [n_owned + 1]
    nbr_ids: object    # torch int32 [nnz]
    status: object     # torch uint8 [n_owned]


@dataclass
class Structure:
    """Cell structure (``Context.vt_structure``): CSR arrays on the device."""
    vert_off: "object"    # n + 1 int64
    verts: "object"       # V x 3 float64, absolute coordinates
    face_off: "object"    # n + 1 int64
    face_nbr: "object"    # F int32: global id across the face, -1 .. -6 for walls
    loop_off: "object"    # F + 1 int64
    loop_vert: "object"   # int32 vertex indices local to the cell

    def cell(self, i):
        """Vertices (numpy, k x 3) and faces [(id, loop indices)] of row i, read back to the host."""
        v0, v1 = int(self.vert_off[i]), int(self.vert_off[i + 1])
        f0, f1 = int(self.face_off[i]), int(self.face_off[i + 1])
        lo = self.loop_off[f0:f1 + 1].cpu().numpy()
        lv = self.loop_vert[int(lo[0]):int(lo[-1])].cpu().numpy() if f1 > f0 else np.zeros(0, np.int32)
        ids = self.face_nbr[f0:f1].cpu().numpy()
        faces = [(int(ids[k]), lv[lo[k] - lo[0]:lo[k + 1] - lo[0]]) for k in range(f1 - f0)]
        return self.verts[v0:v1].cpu().numpy(), faces


class Context:
    """Owns a vt_ctx; methods map one to one onto the C ABI."""

    def __init__(self):
        self._ctx = ctypes.c_void_p(None)
        self._keep = []
        self.n_owned = 0
        self.n_total = 0
        self._pack_cap = 0     # largest batch vt_decompose_pack has written for this context

    def __del__(self):
        try:
            if self._ctx and self._ctx.value and _lib is not None:
                _lib.vt_destroy(self._ctx)
        except Exception:
            pass

    def vt_build(self, pos, items, global_id=None, precision=PREC_FP64, want_faces=False, radius_factor=0.0,
                 area_eps=0.0, waves_per_cu=0, timing=False, pts_per_grid_cell=0.0, k_init=0, cell_mapping=0,
                 stream=None):
        import torch

        _require_cuda(pos, "pos")
        if pos.dim() != 2 or pos.shape[1] != 3:
            raise ValueError("pos must be n x 3")
        if pos.dtype == torch.float32:
            dt = VT_F32
        elif pos.dtype == torch.float64:
            dt = VT_F64
        else:
            raise ValueError("pos must be float32 or float64")
        if global_id is not None:
            _require_cuda(global_id, "global_id")
            if global_id.dtype != torch.int32:
                raise ValueError("global_id must be int32")
        o = vt_opts()
        o.precision = int(precision)
        o.want_faces = 1 if want_faces else 0
        o.radius_factor = float(radius_factor)
        o.area_eps = float(area_eps)
        o.waves_per_cu = int(waves_per_cu)
        o.timing = 1 if timing else 0
        o.pts_per_grid_cell = float(pts_per_grid_cell)
        o.k_init = int(k_init)
        o.cell_mapping = int(cell_mapping)
        arr = _items(items)
        self._keep = [pos, global_id]
        _check(lib().vt_build(ctypes.byref(self._ctx), _ptr(pos), dt, _ptr(global_id), arr, len(items),
                              ctypes.byref(o), _stream(stream)), "vt_build")
        no, nt = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().vt_sizes(self._ctx, ctypes.byref(no), ctypes.byref(nt)), "vt_sizes")
        self.n_owned, self.n_total = no.value, nt.value
        self.device = pos.device
        return self

    def vt_timings(self):
        ms = (ctypes.c_float * 3)()
        _check(lib().vt_timings(self._ctx, ms), "vt_timings")
        return [float(x) for x in ms]

    def vt_query(self):
        nnz, rt, inc = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        code = lib().vt_query(self._ctx, ctypes.byref(nnz), ctypes.byref(rt), ctypes.byref(inc))
        return code, nnz.value, rt.value, inc.value

    def vt_cells(self, nbr_cap=None, stream=None, check=True):
        import torch

        if nbr_cap is None:
            code, nnz, _, _ = self.vt_query()
            if check:
                _check(code, "vt_build (device status)")
            nbr_cap = nnz
        dev = self.device
        vol = torch.empty(self.n_owned, dtype=torch.float64, device=dev)
        off = torch.empty(self.n_owned + 1, dtype=torch.int64, device=dev)
        ids = torch.empty(max(int(nbr_cap), 1), dtype=torch.int32, device=dev)
        st = torch.empty(self.n_owned, dtype=torch.uint8, device=dev)
        _check(lib().vt_cells(self._ctx, _ptr(vol), _ptr(off), _ptr(ids), int(nbr_cap), _ptr(st), _stream(stream)),
               "vt_cells")
        return Cells(vol, off, ids[: int(nbr_cap)], st)

    def vt_structure(self, stream=None):
        """The full structure of the owned cells (needs a build with want_faces): a
        ``Structure`` of device tensors -- vertices (absolute, V x 3) with per-cell offsets,
        faces (the id across each face: a neighbour's global id, or -1 .. -6 for the walls of a
        bounded item) with per-cell offsets, and each face's vertex loop (indices local to the
        cell, counter-clockwise seen from outside) with per-face offsets."""
        import torch

        dev = self.device
        n = self.n_owned
        voff = torch.empty(n + 1, dtype=torch.int64, device=dev)
        foff = torch.empty(n + 1, dtype=torch.int64, device=dev)
        sizes = (ctypes.c_int64 * 3)()
        code = lib().vt_structure(self._ctx, _ptr(voff), None, 0, _ptr(foff), None, 0, None, None, 0, sizes,
                                  _stream(stream))
        if code != VT_ERR_CAPACITY:
            _check(code, "vt_structure")
        nv, nf, nl = int(sizes[0]), int(sizes[1]), int(sizes[2])
        verts = torch.empty((max(nv, 1), 3), dtype=torch.float64, device=dev)
        fnbr = torch.empty(max(nf, 1), dtype=torch.int32, device=dev)
        loff = torch.empty(nf + 1, dtype=torch.int64, device=dev)
        lv = torch.empty(max(nl, 1), dtype=torch.int32, device=dev)
        _check(lib().vt_structure(self._ctx, _ptr(voff), _ptr(verts), nv, _ptr(foff), _ptr(fnbr), nf, _ptr(loff),
                                  _ptr(lv), nl, sizes, _stream(stream)), "vt_structure")
        if nf == 0:
            loff.zero_()
        return Structure(voff, verts[:nv], foff, fnbr[:nf], loff, lv[:nl])

    def vt_cells_into(self, vol, off, ids, status=None, stream=None):
        _check(lib().vt_cells(self._ctx, _ptr(vol), _ptr(off), _ptr(ids), int(ids.numel()), _ptr(status),
                              _stream(stream)), "vt_cells")

    def vt_density(self, mass=None, out=None, stream=None):
        import torch

        rho = out if out is not None else torch.empty(self.n_owned, dtype=torch.float64, device=self.device)
        dt = VT_F64
        if mass is not None:
            _require_cuda(mass, "mass")
            dt = VT_F32 if mass.dtype == torch.float32 else VT_F64
        _check(lib().vt_density(self._ctx, _ptr(mass), dt, _ptr(rho), _stream(stream)), "vt_density")
        return rho

    def vt_gradient(self, rho_all, out=None, stream=None):
        import torch

        _require_cuda(rho_all, "rho")
        g = out if out is not None else torch.empty((self.n_owned, 3), dtype=torch.float64, device=self.device)
        _check(lib().vt_gradient(self._ctx, _ptr(rho_all), _ptr(g), _stream(stream)), "vt_gradient")
        return g

    def vt_grid_deposit(self, value, dims, out=None, stream=None):
        import torch

        _require_cuda(value, "value")
        nx, ny, nz = (int(d) for d in dims)
        g = out if out is not None else torch.empty((nx, ny, nz), dtype=torch.float64, device=self.device)
        _check(lib().vt_grid_deposit(self._ctx, _ptr(value), nx, ny, nz, _ptr(g), _stream(stream)),
               "vt_grid_deposit")
        return g

    def vt_grid_sample(self, value, dims, sub=1, out=None, nearest=False, stream=None):
        """Voxel values from the nearest particle of sub^3 points per voxel; with nearest=True
        also the global id of the particle nearest to each voxel's last point."""
        import torch

        _require_cuda(value, "value")
        nx, ny, nz = (int(d) for d in dims)
        g = out if out is not None else torch.empty((nx, ny, nz), dtype=torch.float64, device=self.device)
        nid = torch.empty((nx, ny, nz), dtype=torch.int32, device=self.device) if nearest else None
        _check(lib().vt_grid_sample(self._ctx, _ptr(value), nx, ny, nz, int(sub), _ptr(g), _ptr(nid),
                                    _stream(stream)), "vt_grid_sample")
        return (g, nid) if nearest else g

    def vt_grid_tensor(self, grid, kind=TENSOR_TIDAL, out=None, stream=None):
        """Tidal tensor (kind TENSOR_TIDAL) or Hessian (TENSOR_HESSIAN) of a grid field on the
        context's periodic box: a 6 x nx x ny x nz tensor, components TENSOR_COMPONENTS."""
        import torch

        _require_cuda(grid, "grid")
        if grid.dim() != 3 or grid.dtype != torch.float64:
            raise ValueError("grid must be an nx x ny x nz float64 tensor")
        nx, ny, nz = grid.shape
        o = out if out is not None else torch.empty((6, nx, ny, nz), dtype=torch.float64, device=self.device)
        _check(lib().vt_grid_tensor(self._ctx, _ptr(grid), nx, ny, nz, int(kind), _ptr(o), _stream(stream)),
               "vt_grid_tensor")
        return o

    def vt_grid_tensor_noalloc(self, grid, kind, out, stream=None):
        """vt_grid_tensor with the library's static scratch instead of the context's: the caller
        passes the output (6 x nx x ny x nz float64); nothing is allocated."""
        _require_cuda(grid, "grid")
        _require_cuda(out, "out")
        nx, ny, nz = grid.shape
        _check(lib().vt_grid_tensor_noalloc(self._ctx, _ptr(grid), nx, ny, nz, int(kind), _ptr(out),
                                            _stream(stream)), "vt_grid_tensor_noalloc")
        return out

    def vt_backward(self, dL_dV, out=None, stream=None):
        import torch

        _require_cuda(dL_dV, "dL_dV")
        g = out if out is not None else torch.empty((self.n_owned, 3), dtype=torch.float64, device=self.device)
        _check(lib().vt_backward(self._ctx, _ptr(dL_dV), _ptr(g), _stream(stream)), "vt_backward")
        return g

    def vt_decompose(self, pos, box_lo, box_hi, nt, border_factor=1.5, periodic=True, growth=0.0, n_steps=0,
                     stream=None):
        """AUTOBORDER thicknesses (n_tasks x 6: faces -x, +x, -y, +y, -z, +z) and the tasks'
        owned and buffer counts, as numpy arrays."""
        dt = _pos_dtype(pos)
        lo, hi, ntc = _box3(box_lo), _box3(box_hi), (ctypes.c_int32 * 3)(*[int(x) for x in nt])
        bp = _border(border_factor, growth, n_steps)
        n_tasks = int(np.prod(nt))
        thick = np.zeros(6 * n_tasks)
        n_own = np.zeros(n_tasks, np.int64)
        n_gh = np.zeros(n_tasks, np.int64)
        _check(lib().vt_decompose(ctypes.byref(self._ctx), _ptr(pos), dt, pos.shape[0], lo, hi, int(bool(periodic)),
                                  ntc, ctypes.byref(bp), _dptr(thick),
                                  n_own.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                  n_gh.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _stream(stream)),
               "vt_decompose")
        return thick.reshape(n_tasks, 6), n_own, n_gh

    def vt_decompose_pack(self, pos, box_lo, box_hi, nt, thick, own_mask=None, tasks=None, periodic=True,
                          stream=None):
        """The batch of the listed tasks for vt_build: (positions float64 n x 3, int32 global ids,
        item list)."""
        import torch

        dt = _pos_dtype(pos)
        if own_mask is not None:
            _require_cuda(own_mask, "own_mask")
            if own_mask.dtype != torch.uint8 or own_mask.shape[0] != pos.shape[0]:
                raise ValueError("own_mask must be uint8 with one byte per particle")
        lo, hi, ntc = _box3(box_lo), _box3(box_hi), (ctypes.c_int32 * 3)(*[int(x) for x in nt])
        th = np.ascontiguousarray(np.asarray(thick, np.float64).reshape(-1))
        n_tasks = int(np.prod(nt))
        tl = None if tasks is None else np.ascontiguousarray(tasks, np.int32)
        n_list = n_tasks if tl is None else len(tl)
        arr = (vt_item * n_list)()
        n_out = ctypes.c_int64()
        tptr = None if tl is None else tl.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        args = (ctypes.byref(self._ctx), _ptr(pos), dt, pos.shape[0], lo, hi, int(bool(periodic)), ntc, _dptr(th),
                _ptr(own_mask), tptr, n_list)
        # outputs sized by the largest batch this context has packed; a larger one is sized by
        # the call that finds it too small, then packed again
        cap = self._pack_cap
        out = gid = None
        code = VT_ERR_CAPACITY
        if cap > 0:
            out = torch.empty((cap, 3), dtype=torch.float64, device=pos.device)
            gid = torch.empty(cap, dtype=torch.int32, device=pos.device)
            code = lib().vt_decompose_pack(*args, _ptr(out), _ptr(gid), cap, arr, ctypes.byref(n_out),
                                           _stream(stream))
        else:
            code = lib().vt_decompose_pack(*args, None, None, 0, arr, ctypes.byref(n_out), _stream(stream))
        if code == VT_ERR_CAPACITY:
            self._pack_cap = max(cap, n_out.value, 1)
            out = torch.empty((self._pack_cap, 3), dtype=torch.float64, device=pos.device)
            gid = torch.empty(self._pack_cap, dtype=torch.int32, device=pos.device)
            code = lib().vt_decompose_pack(*args, _ptr(out), _ptr(gid), self._pack_cap, arr, ctypes.byref(n_out),
                                           _stream(stream))
        _check(code, "vt_decompose_pack")
        items = [dict(offset=arr[k].offset, n_owned=arr[k].n_owned, n_ghost=arr[k].n_ghost, periodic=False,
                      walls=arr[k].walls, lo=np.array(arr[k].lo[:]), hi=np.array(arr[k].hi[:]))
                 for k in range(n_list)]
        return out[:n_out.value], gid[:n_out.value], items

    def vt_decomposed_build(self, pos, box_lo, box_hi, nt, border_factor=1.5, periodic=True, max_reruns=0,
                            widen=0.0, growth=0.0, n_steps=0, precision=PREC_FP64, radius_factor=0.0,
                            waves_per_cu=0, k_init=0, pts_per_grid_cell=0.0, cell_mapping=0, stream=None):
        """The whole AUTOBORDER procedure in the library; afterwards vt_cells / vt_density /
        vt_query answer in particle order.  Returns (first-pass thicknesses n_tasks x 6,
        per-pass [tasks, particles packed, cells built, cells left incomplete])."""
        dt = _pos_dtype(pos)
        lo, hi, ntc = _box3(box_lo), _box3(box_hi), (ctypes.c_int32 * 3)(*[int(x) for x in nt])
        bp = _border(border_factor, growth, n_steps, max_reruns, widen)
        o = vt_opts()
        o.precision = int(precision)
        o.radius_factor = float(radius_factor)
        o.waves_per_cu = int(waves_per_cu)
        o.k_init = int(k_init)
        o.pts_per_grid_cell = float(pts_per_grid_cell)
        o.cell_mapping = int(cell_mapping)
        n_tasks = int(np.prod(nt))
        thick = np.zeros(6 * n_tasks)
        stats = np.zeros((16, 4), np.int64)
        npass = ctypes.c_int32()
        _check(lib().vt_decomposed_build(ctypes.byref(self._ctx), _ptr(pos), dt, pos.shape[0], lo, hi,
                                         int(bool(periodic)), ntc, ctypes.byref(bp), ctypes.byref(o), _dptr(thick),
                                         stats.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ctypes.byref(npass),
                                         _stream(stream)), "vt_decomposed_build")
        no, nt_ = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().vt_sizes(self._ctx, ctypes.byref(no), ctypes.byref(nt_)), "vt_sizes")
        self.n_owned, self.n_total = no.value, nt_.value
        self.device = pos.device
        return thick.reshape(n_tasks, 6), stats[:npass.value]

    def vt_stats(self, stream=None):
        import torch

        nv = torch.empty(self.n_owned, dtype=torch.int32, device=self.device)
        np_ = torch.empty_like(nv)
        nt = torch.empty_like(nv)
        _check(lib().vt_stats(self._ctx, _ptr(nv), _ptr(np_), _ptr(nt), _stream(stream)), "vt_stats")
        return nv, np_, nt


def _border(border_factor=1.5, growth=0.0, n_steps=0, max_reruns=0, widen=0.0):
    bp = vt_border()
    bp.border_factor = float(border_factor)
    bp.growth = float(growth)
    bp.n_steps = int(n_steps)
    bp.max_reruns = int(max_reruns)
    bp.widen = float(widen)
    return bp


def task_grid(n_task, scheme="a", axis=0):
    """Tasks per axis for the paper's two decomposition schemes (section 2; vt_task_grid):
    scheme "a" halves the box along x, y, z in turn until there are n_task regions, scheme "b"
    makes n_task slabs along one axis."""
    if scheme not in ("a", "b"):
        raise ValueError("scheme must be 'a' or 'b'")
    nt = (ctypes.c_int32 * 3)()
    code = _host_lib().vt_task_grid(int(n_task), 0 if scheme == "a" else 1, int(axis), nt)
    if code != VT_OK:
        raise ValueError("no %s layout for %d tasks (axis %d)" % (scheme, n_task, axis))
    return tuple(int(x) for x in nt)


def border_thresholds(n, box_lo, box_hi, border_factor=1.5, growth=0.0, n_steps=0):
    """The AUTOBORDER thicknesses the library tries (vt_border_thresholds; host only)."""
    bp = _border(border_factor, growth, n_steps)
    k = bp.n_steps or 48
    out = np.zeros(k)
    _check(_host_lib().vt_border_thresholds(int(n), _box3(box_lo), _box3(box_hi), ctypes.byref(bp), _dptr(out)),
           "vt_border_thresholds")
    return out


_hlib = None


def _host_lib():
    """libvt for its host-only calls (vt_task_grid, vt_border_thresholds): no device is needed."""
    global _hlib
    with _lock:
        if _hlib is None:
            L = _load_cdll()
            I32, I64 = ctypes.c_int32, ctypes.c_int64
            D3 = ctypes.POINTER(ctypes.c_double)
            L.vt_task_grid.argtypes = [I32, I32, I32, ctypes.POINTER(I32)]
            L.vt_task_grid.restype = I32
            L.vt_border_thresholds.argtypes = [I64, D3, D3, ctypes.POINTER(vt_border), D3]
            L.vt_border_thresholds.restype = I32
            _hlib = L
    return _hlib


def decomposed_build(pos, box_lo, box_hi, nt, border_factor=1.5, periodic=True, ctx=None, **build_opts):
    """Tessellate a periodic box or a bounded world as nt[0] x nt[1] x nt[2] tasks with AUTOBORDER
    buffers, in the library (vt_decomposed_build): all tasks in one batched build, cells left
    incomplete built again with widened buffers.  An integer nt is a task count split by scheme (a).

    Returns a dict with per-particle ``volume``, ``status`` and the neighbour CSR
    ``nbr_off``/``nbr_ids`` in particle order (numpy), the first pass's thicknesses ``thick``
    (n_tasks x 6) and per-pass records ``passes``.
    """
    if np.ndim(nt) == 0:
        nt = task_grid(nt, "a")
    nt = tuple(int(x) for x in nt)
    ctx = ctx or Context()
    thick, stats = ctx.vt_decomposed_build(pos, box_lo, box_hi, nt, border_factor=border_factor,
                                           periodic=periodic, **build_opts)
    cells = ctx.vt_cells()
    passes = [dict(tasks=int(r[0]), particles=int(r[1]), owned=int(r[2]), incomplete=int(r[3])) for r in stats]
    return dict(volume=cells.volume.cpu().numpy(), status=cells.status.cpu().numpy(),
                nbr_off=cells.nbr_off.cpu().numpy(), nbr_ids=cells.nbr_ids.cpu().numpy(), thick=thick,
                passes=passes, ctx=ctx)


def tessellate(pos, box_lo, box_hi, periodic=True, precision=PREC_FP64, want_faces=False, **kw):
    """Convenience: build a single-world context and return (context, cells)."""
    ctx = Context().vt_build(pos, whole_box(pos.shape[0], box_lo, box_hi, periodic), precision=precision,
                             want_faces=want_faces, **kw)
    return ctx, ctx.vt_cells()


def _autograd():
    import torch

    class VoronoiVolume(torch.autograd.Function):
        """V(x) for a periodic box; backward through the hand-written adjoint kernel.

        forward(pos, box_lo, box_hi, precision) -> cell volumes (float64, input order).
        """

        @staticmethod
        def forward(ctx_, pos, box_lo, box_hi, precision=PREC_FP64):
            c = Context().vt_build(pos.detach().contiguous(), whole_box(pos.shape[0], box_lo, box_hi, True),
                                   precision=precision, want_faces=True)
            cells = c.vt_cells()
            ctx_.vt = c
            ctx_.pos_dtype = pos.dtype
            return cells.volume

        @staticmethod
        def backward(ctx_, g):
            dx = ctx_.vt.vt_backward(g.contiguous().to(torch.float64))
            return dx.to(ctx_.pos_dtype), None, None, None

    return VoronoiVolume


def voronoi_volume(pos, box_lo, box_hi, precision=PREC_FP64):
    """Differentiable cell volumes of a periodic box (autograd through vt_backward)."""
    return _autograd().apply(pos, box_lo, box_hi, precision)

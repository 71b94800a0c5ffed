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


class VTError(RuntimeError):
    def __init__(self, code, what=""):
        super().__init__("%s: %s (code %d)" % (what, STATUS_NAMES.get(code, "unknown"), code))
        self.code = code


class vt_item(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_int64), ("n_owned", ctypes.c_int64), ("n_ghost", ctypes.c_int64),
                ("periodic", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3)]


class vt_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("want_faces", ctypes.c_int32), ("radius_factor", ctypes.c_float),
                ("area_eps", ctypes.c_float), ("waves_per_cu", ctypes.c_int32), ("timing", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]


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
            L = ctypes.CDLL(LIB_PATH)
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
            L.vt_decompose.argtypes = [ctypes.POINTER(P), P, I32, I64, D3, D3, ctypes.POINTER(I32), D3, I32, D3,
                                       ctypes.POINTER(I64), ctypes.POINTER(I64), P]
            L.vt_decompose_pack.argtypes = [ctypes.POINTER(P), P, I32, I64, D3, D3, ctypes.POINTER(I32), D3, P,
                                            ctypes.POINTER(I32), I32, P, P, I64, ctypes.POINTER(vt_item),
                                            ctypes.POINTER(I64), P]
            L.vt_structure.argtypes = [P, P, P, I64, P, P, I64, P, P, I64, ctypes.POINTER(I64), P]
            L.vt_grid_tensor.argtypes = [P, P, I32, I32, I32, I32, P, P]
            L.vt_destroy.argtypes = [P]
            L.vt_destroy.restype = None
            L.vt_status_string.argtypes = [I32]
            L.vt_status_string.restype = ctypes.c_char_p
            for f in ("vt_build", "vt_cells", "vt_density", "vt_gradient", "vt_grid_deposit", "vt_backward",
                      "vt_query", "vt_stats", "vt_sizes", "vt_timings", "vt_decompose", "vt_decompose_pack",
                      "vt_grid_sample", "vt_structure", "vt_grid_tensor"):
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


def whole_box(n, box_lo, box_hi, periodic=True):
    """Item list for a single world of n owned particles."""
    lo = np.broadcast_to(np.asarray(box_lo, np.float64), 3)
    hi = np.broadcast_to(np.asarray(box_hi, np.float64), 3)
    return [dict(offset=0, n_owned=int(n), n_ghost=0, periodic=bool(periodic), lo=lo, hi=hi)]


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
                 area_eps=0.0, waves_per_cu=0, timing=False, stream=None):
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

    def vt_backward(self, dL_dV, out=None, stream=None):
        import torch

        _require_cuda(dL_dV, "dL_dV")
        g = out if out is not None else torch.empty((self.n_owned, 3), dtype=torch.float64, device=self.device)
        _check(lib().vt_backward(self._ctx, _ptr(dL_dV), _ptr(g), _stream(stream)), "vt_backward")
        return g

    def vt_decompose(self, pos, box_lo, box_hi, nt, thresholds, stream=None):
        """AUTOBORDER thicknesses (n_tasks x 6: faces -x, +x, -y, +y, -z, +z) and the tasks'
        owned and buffer counts, as numpy arrays."""
        dt = _pos_dtype(pos)
        lo, hi, ntc = _box3(box_lo), _box3(box_hi), (ctypes.c_int32 * 3)(*[int(x) for x in nt])
        thr = np.ascontiguousarray(thresholds, np.float64)
        n_tasks = int(np.prod(nt))
        thick = np.zeros(6 * n_tasks)
        n_own = np.zeros(n_tasks, np.int64)
        n_gh = np.zeros(n_tasks, np.int64)
        _check(lib().vt_decompose(ctypes.byref(self._ctx), _ptr(pos), dt, pos.shape[0], lo, hi, ntc, _dptr(thr),
                                  len(thr), _dptr(thick), n_own.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                  n_gh.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _stream(stream)),
               "vt_decompose")
        return thick.reshape(n_tasks, 6), n_own, n_gh

    def vt_decompose_pack(self, pos, box_lo, box_hi, nt, thick, own_mask=None, tasks=None, stream=None):
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
        args = (ctypes.byref(self._ctx), _ptr(pos), dt, pos.shape[0], lo, hi, ntc, _dptr(th), _ptr(own_mask), tptr,
                n_list)
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
                      lo=np.array(arr[k].lo[:]), hi=np.array(arr[k].hi[:])) for k in range(n_list)]
        return out[:n_out.value], gid[:n_out.value], items

    def vt_stats(self, stream=None):
        import torch

        nv = torch.empty(self.n_owned, dtype=torch.int32, device=self.device)
        np_ = torch.empty_like(nv)
        nt = torch.empty_like(nv)
        _check(lib().vt_stats(self._ctx, _ptr(nv), _ptr(np_), _ptr(nt), _stream(stream)), "vt_stats")
        return nv, np_, nt


def task_grid(n_task, scheme="a", axis=0):
    """Tasks per axis for the paper's two decomposition schemes (section 2).

    Scheme "a" cuts the box in halves, along x, then y, then z, and round again, until there are
    n_task equal regions (n_task a power of two; 32 gives 4 x 4 x 2).  Scheme "b" cuts it
    n_task times along one axis (elongated volumes).
    """
    n_task = int(n_task)
    if n_task < 1:
        raise ValueError("n_task must be positive")
    nt = [1, 1, 1]
    if scheme == "a":
        if n_task & (n_task - 1):
            raise ValueError("scheme a needs a power-of-two task count, got %d" % n_task)
        a = 0
        while nt[0] * nt[1] * nt[2] < n_task:
            nt[a] *= 2
            a = (a + 1) % 3
    elif scheme == "b":
        if axis not in (0, 1, 2):
            raise ValueError("axis must be 0, 1 or 2")
        nt[axis] = n_task
    else:
        raise ValueError("scheme must be 'a' or 'b'")
    return tuple(nt)


def autoborder_thresholds(n, box_lo, box_hi, border_factor=1.5, growth=1.1, steps=48):
    """Buffer thicknesses tried by AUTOBORDER: border_factor times the mean inter-particle
    distance (V / n)^(1/3), grown by the factor ``growth`` per step."""
    L = np.broadcast_to(np.asarray(box_hi, np.float64), 3) - np.broadcast_to(np.asarray(box_lo, np.float64), 3)
    s = (float(np.prod(L)) / n) ** (1.0 / 3.0)
    return border_factor * s * growth ** np.arange(steps, dtype=np.float64)


def task_limits(box_lo, box_hi, nt):
    """Largest buffer thickness per axis (a buffered task spans less than one period)."""
    L = np.broadcast_to(np.asarray(box_hi, np.float64), 3) - np.broadcast_to(np.asarray(box_lo, np.float64), 3)
    nt = np.asarray(nt)
    w = L / nt
    return np.where(nt >= 2, 0.5 * (L - w), 0.5 * L) * (1.0 - 1e-12)


def owner_tasks(pos_np, box_lo, box_hi, nt):
    """Owner task of every particle (the library's rule: cell index floor((x - lo) / w))."""
    lo = np.broadcast_to(np.asarray(box_lo, np.float64), 3)
    L = np.broadcast_to(np.asarray(box_hi, np.float64), 3) - lo
    nt = np.asarray(nt)
    w = L / nt
    i = np.clip(np.floor((np.asarray(pos_np, np.float64) - lo) / w).astype(np.int64), 0, nt - 1)
    return (i[:, 0] * nt[1] + i[:, 1]) * nt[2] + i[:, 2]


def decomposed_build(pos, box_lo, box_hi, nt, border_factor=1.5, growth=1.1, steps=48, reruns=3, widen=2.0,
                     ctx=None, **build_opts):
    """Tessellate a periodic box as nt[0] x nt[1] x nt[2] tasks with AUTOBORDER buffers, all
    tasks in one batched build; cells still incomplete are built again, owned alone, with their
    tasks' buffers widened ``widen`` times (up to ``reruns`` passes).  An integer nt is a task
    count split by scheme (a) (``task_grid``).

    Returns a dict with per-particle ``volume`` (numpy), ``status`` (numpy uint8: the last pass
    that computed the cell), the neighbour CSR ``nbr_off``/``nbr_ids`` in particle order (numpy),
    the thicknesses ``thick`` (n_tasks x 6) of the first pass, per-pass ``passes`` records and the
    ``plan`` of each pass (thicknesses, owner mask, task list) to replay it.
    """
    import torch

    n = pos.shape[0]
    if np.ndim(nt) == 0:
        nt = task_grid(nt, "a")
    nt = tuple(int(x) for x in nt)
    ctx = ctx or Context()
    thr = autoborder_thresholds(n, box_lo, box_hi, border_factor, growth, steps)
    thick, n_own, n_gh = ctx.vt_decompose(pos, box_lo, box_hi, nt, thr)
    tmax = task_limits(box_lo, box_hi, nt)
    vol = np.full(n, np.nan)
    status = np.full(n, 255, np.uint8)
    last = np.full(n, -1, np.int64)     # pass that computed the cell
    row = np.full(n, -1, np.int64)      # its row there
    csr = []                            # per pass: (nbr_off, nbr_ids)
    passes, plan = [], []
    cur = thick.copy()
    mask, tasks = None, None
    for rnd in range(reruns + 1):
        plan.append((cur.copy(), mask, tasks))
        bpos, gid, items = ctx.vt_decompose_pack(pos, box_lo, box_hi, nt, cur, own_mask=mask, tasks=tasks)
        bctx = Context().vt_build(bpos, items, global_id=gid, **build_opts)
        cells = bctx.vt_cells()
        g = gid.cpu().numpy()
        own_gid = np.concatenate([g[it["offset"]:it["offset"] + it["n_owned"]] for it in items])
        v = cells.volume.cpu().numpy()
        st = cells.status.cpu().numpy()
        off = cells.nbr_off.cpu().numpy()
        ids = cells.nbr_ids.cpu().numpy()
        vol[own_gid] = v
        status[own_gid] = st
        last[own_gid] = rnd
        row[own_gid] = np.arange(len(own_gid))
        csr.append((off, ids))
        inc = own_gid[(st & CELL_INCOMPLETE) != 0]
        passes.append(dict(tasks=len(items), particles=int(bpos.shape[0]), owned=int(len(own_gid)),
                           incomplete=int(len(inc))))
        del bctx, cells
        if len(inc) == 0 or rnd == reruns:
            break
        # the incomplete cells again, owned alone, with their tasks' buffers widened
        own = owner_tasks(pos.cpu().numpy(), box_lo, box_hi, nt)
        tl = np.unique(own[inc]).astype(np.int32)
        m = np.zeros(n, np.uint8)
        m[inc] = 1
        mask = torch.from_numpy(m).to(pos.device)
        tasks = tl
        cur = cur.copy()
        cur[tl] = np.minimum(cur[tl] * widen, np.repeat(tmax, 2)[None, :])
    # neighbour rows in particle order, each from the last pass that computed the cell
    cnt = np.zeros(n, np.int64)
    for k, (off, _) in enumerate(csr):
        sel = last == k
        cnt[sel] = off[row[sel] + 1] - off[row[sel]]
    nbr_off = np.zeros(n + 1, np.int64)
    nbr_off[1:] = np.cumsum(cnt)
    nbr_ids = np.zeros(int(nbr_off[-1]), np.int32)
    for k, (off, ids) in enumerate(csr):
        p = np.nonzero(last == k)[0]
        if len(p) == 0:
            continue
        ln = cnt[p]
        src = np.repeat(off[row[p]] - np.cumsum(ln) + ln, ln) + np.arange(ln.sum())
        dst = np.repeat(nbr_off[p] - np.cumsum(ln) + ln, ln) + np.arange(ln.sum())
        nbr_ids[dst] = ids[src]
    return dict(volume=vol, status=status, nbr_off=nbr_off, nbr_ids=nbr_ids, thick=thick, n_owned=n_own,
                n_ghost=n_gh, passes=passes, plan=plan)


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

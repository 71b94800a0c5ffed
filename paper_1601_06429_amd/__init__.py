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
STATUS_NAMES = {0: "ok", 1: "invalid argument", 2: "HIP runtime error", 3: "out of device memory",
                4: "duplicate particles", 5: "periodic box too small", 6: "capacity exceeded",
                7: "invalid call order", 8: "inconsistent clipping topology"}
VT_F32, VT_F64 = 0, 1
PREC_FP64, PREC_MIXED = 0, 1
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
            L.vt_backward.argtypes = [P, P, P, P]
            L.vt_query.argtypes = [P, ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(I64)]
            L.vt_stats.argtypes = [P, P, P, P, P]
            L.vt_sizes.argtypes = [P, ctypes.POINTER(I64), ctypes.POINTER(I64)]
            L.vt_timings.argtypes = [P, ctypes.POINTER(ctypes.c_float)]
            L.vt_destroy.argtypes = [P]
            L.vt_destroy.restype = None
            L.vt_status_string.argtypes = [I32]
            L.vt_status_string.restype = ctypes.c_char_p
            for f in ("vt_build", "vt_cells", "vt_density", "vt_gradient", "vt_grid_deposit", "vt_backward",
                      "vt_query", "vt_stats", "vt_sizes", "vt_timings"):
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


class Context:
    """Owns a vt_ctx; methods map one to one onto the C ABI."""

    def __init__(self):
        self._ctx = ctypes.c_void_p(None)
        self._keep = []
        self.n_owned = 0
        self.n_total = 0

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

    def vt_backward(self, dL_dV, out=None, stream=None):
        import torch

        _require_cuda(dL_dV, "dL_dV")
        g = out if out is not None else torch.empty((self.n_owned, 3), dtype=torch.float64, device=self.device)
        _check(lib().vt_backward(self._ctx, _ptr(dL_dV), _ptr(g), _stream(stream)), "vt_backward")
        return g

    def vt_stats(self, stream=None):
        import torch

        nv = torch.empty(self.n_owned, dtype=torch.int32, device=self.device)
        np_ = torch.empty_like(nv)
        nt = torch.empty_like(nv)
        _check(lib().vt_stats(self._ctx, _ptr(nv), _ptr(np_), _ptr(nt), _stream(stream)), "vt_stats")
        return nv, np_, nt


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

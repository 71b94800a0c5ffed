"""Brute-force FP64 oracle for the per-particle Voronoi tessellation.

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may use this package; the library path never
imports it.  It shares no code with the HIP implementation.

Paper passages followed (Gonzalez, "PARAVT: Parallel Voronoi Tessellation
code", Astronomy & Computing):
  * section 1 -- a particle's cell is the region closer to it than to any other
    particle (with periodic conditions, any periodic image of any particle);
  * section 2, post-processing paragraph -- cell volume from the facets,
    density = mass / volume, a density gradient per particle from densities and
    neighbour information, neighbours = particles sharing a facet, and an
    optional average density on a regular grid;
  * section 2, gather paragraph -- outputs in input order with real ids.

Readings where the paper is silent (documented with the design notes):
  * gradient: unweighted least squares over the Voronoi neighbours,
    grad = G^-1 b, G = sum D D^T, b = sum (rho_j - rho_i) D (the paper's own
    formula is not given; pinned by exact recovery of linear fields and a
    zero gradient on lattices);
  * grid: exact volume average of the piecewise-constant Voronoi density over
    each voxel (pinned by mass conservation and exact lattice cases);
  * adjoint: dV_i/dx_j = A_ij (x_j - c_ij) / d_ij and
    dV_i/dx_i = sum_j A_ij (c_ij - x_i) / d_ij (derived from the motion of the
    bisector plane; pinned by central finite differences of the oracle's own
    volumes).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

FLAG_WALL = 1
FLAG_INCOMPLETE = 2
FLAG_CAPACITY = 4


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            p = ctypes.c_void_p
            i64 = ctypes.c_int64
            lib.ora_cells.argtypes = [i64, p, p, p, p, ctypes.c_int, i64, p, ctypes.c_double, ctypes.c_double,
                                      i64, p, p, p, p, p, p, p, p, p, ctypes.c_int]
            lib.ora_cells.restype = ctypes.c_int
            lib.ora_grid.argtypes = [i64, p, p, p, ctypes.c_int, i64, p, p, ctypes.c_double, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_int, p, ctypes.c_int]
            lib.ora_grid.restype = ctypes.c_int
            _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class Cells:
    """Per-query-cell oracle output (rows follow the query order)."""

    def __init__(self, query, vol, rmax, flags, nnb, topo, nbr, farea, fcen, fdist):
        self.query = query
        self.volume = vol
        self.rmax = rmax
        self.flags = flags
        self.nnb = nnb
        self.topo = topo  # vertices, edges, faces, max vertex degree, planes examined
        self._nbr, self._farea, self._fcen, self._fdist = nbr, farea, fcen, fdist

    def neighbours(self, q):
        return self._nbr[q, : self.nnb[q]]

    def faces(self, q):
        k = self.nnb[q]
        return self._farea[q, :k], self._fcen[q, :k], self._fdist[q, :k]

    def csr(self):
        off = np.zeros(len(self.query) + 1, dtype=np.int64)
        np.cumsum(self.nnb, out=off[1:])
        ids = np.concatenate([self.neighbours(q) for q in range(len(self.query))]) if len(self.query) else \
            np.zeros(0, np.int64)
        return off, ids


def cells(pos, box_lo, box_hi, periodic=True, query=None, gid=None, tol=1e-12, area_eps=1e-12,
          stride=128, nthreads=0) -> Cells:
    """Voronoi cells of the particles in ``query`` (default: all), brute force in FP64."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    n = pos.shape[0]
    lo = np.ascontiguousarray(np.broadcast_to(np.asarray(box_lo, np.float64), 3))
    hi = np.ascontiguousarray(np.broadcast_to(np.asarray(box_hi, np.float64), 3))
    q = np.arange(n, dtype=np.int64) if query is None else np.ascontiguousarray(query, dtype=np.int64)
    g = None if gid is None else np.ascontiguousarray(gid, dtype=np.int64)
    nq = q.shape[0]
    vol = np.zeros(nq)
    rmax = np.zeros(nq)
    flags = np.zeros(nq, np.int32)
    nnb = np.zeros(nq, np.int32)
    topo = np.zeros((nq, 5), np.int64)
    nbr = np.zeros((nq, stride), np.int64)
    farea = np.zeros((nq, stride))
    fcen = np.zeros((nq, stride, 3))
    fdist = np.zeros((nq, stride))
    rc = lib.ora_cells(n, _ptr(pos), _ptr(g), _ptr(lo), _ptr(hi), int(bool(periodic)), nq, _ptr(q), tol, area_eps,
                       stride, _ptr(vol), _ptr(rmax), _ptr(flags), _ptr(nnb), _ptr(topo), _ptr(nbr), _ptr(farea),
                       _ptr(fcen), _ptr(fdist), int(nthreads))
    if rc != 0:
        raise RuntimeError("ora_cells failed with code %d" % rc)
    if np.any(flags & FLAG_CAPACITY):
        raise RuntimeError("ora_cells: a cell has more than %d facets; raise stride" % stride)
    return Cells(q, vol, rmax, flags, nnb, topo, nbr, farea, fcen, fdist)


def density(mass, volume):
    """rho_i = m_i / V_i (section 2)."""
    return np.asarray(mass, np.float64) / np.asarray(volume, np.float64)


def min_image(d, box_len):
    d = np.asarray(d, np.float64)
    L = np.asarray(box_len, np.float64)
    return d - L * np.rint(d / L)


def gradient(pos, box_lo, box_hi, periodic, off, ids, rho, rows=None):
    """Least-squares density gradient over Voronoi neighbours.

    For row i: G = sum_j D_ij D_ij^T, b = sum_j (rho_j - rho_i) D_ij, grad = G^-1 b,
    with D_ij the (minimum image) separation.  ``off``/``ids`` is the CSR of the
    rows listed in ``rows`` (default: all particles, in order); ``rho`` is indexed
    by particle.
    """
    pos = np.asarray(pos, np.float64)
    rows = np.arange(len(off) - 1) if rows is None else np.asarray(rows)
    L = np.asarray(box_hi, np.float64) - np.asarray(box_lo, np.float64)
    cnt = np.diff(off)
    src = np.repeat(rows, cnt)
    D = pos[ids] - pos[src]
    if periodic:
        D = min_image(D, L)
    seg = np.repeat(np.arange(len(rows)), cnt)
    G = np.zeros((len(rows), 3, 3))
    b = np.zeros((len(rows), 3))
    np.add.at(G, seg, D[:, :, None] * D[:, None, :])
    np.add.at(b, seg, (rho[ids] - rho[src])[:, None] * D)
    return np.linalg.solve(G, b[:, :, None])[:, :, 0]


def grid(pos, box_lo, box_hi, periodic, value, dims, query=None, tol=1e-12, nthreads=0):
    """Exact voxel averages of the piecewise-constant field ``value`` (per particle)."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    n = pos.shape[0]
    lo = np.ascontiguousarray(np.broadcast_to(np.asarray(box_lo, np.float64), 3))
    hi = np.ascontiguousarray(np.broadcast_to(np.asarray(box_hi, np.float64), 3))
    q = np.arange(n, dtype=np.int64) if query is None else np.ascontiguousarray(query, dtype=np.int64)
    v = np.ascontiguousarray(value, dtype=np.float64)
    nx, ny, nz = (int(d) for d in dims)
    out = np.zeros((nx, ny, nz))
    rc = lib.ora_grid(n, _ptr(pos), _ptr(lo), _ptr(hi), int(bool(periodic)), q.shape[0], _ptr(q), _ptr(v), tol,
                      nx, ny, nz, _ptr(out), int(nthreads))
    if rc != 0:
        raise RuntimeError("ora_grid failed with code %d" % rc)
    return out


def adjoint(c: Cells, dL_dV, rows_pos=None):
    """dL/dx_k = sum_{j in N(k)} (g_k - g_j) A_kj (c_kj - x_k) / d_kj, g = dL/dV.

    ``c`` must hold every particle (query = all) so that both sides of each
    facet are present; face centroids are seed-relative, so (c_kj - x_k) is the
    stored centroid itself.  ``dL_dV`` is indexed by particle.
    """
    g = np.asarray(dL_dV, np.float64)
    nq = len(c.query)
    out = np.zeros((nq, 3))
    for q in range(nq):
        k = c.query[q]
        ids = c.neighbours(q)
        A, C, d = c.faces(q)
        w = (g[k] - g[ids]) * A / d
        out[q] = (w[:, None] * C).sum(axis=0)
    return out

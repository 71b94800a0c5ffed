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
  * AUTOBORDER (section 2, buffer zones between tasks): per face of each task of
    an equal split of the box, the buffer is the slab beyond the face over the
    face's extent; its thickness is the first of a growing list of thicknesses
    at which the slab holds the mean density times the face area times the
    first thickness (pinned by uniform lattices, where the first thickness
    already suffices, by empty regions, which reach the cap, and by hand-counted
    small sets);
  * nearest-particle grid sampling (a grid variant the paper leaves to future
    work): a sample point takes the value of its nearest particle, ties to the
    smaller index (pinned by lattice points at voxel centres, a two-particle
    bisector, an exact tie, and convergence to the exact overlaps under finer
    sub-sampling);
  * full structure (section 3, memory consumption; section 4): a cell's vertices
    and its faces of area above the facet threshold as loops, counter-clockwise
    seen from outside, ascending by the id across them (pinned by the cube and
    truncated octahedron of lattices, the empty-sphere property of every vertex,
    faces on their bisectors, Euler's formula, the divergence volume and walls);
  * grid tensors (section 4, future grid outputs): tidal tensor d_i d_j phi with
    laplacian(phi) = f / mean(f) - 1, and Hessian d_i d_j f, by numpy.fft on the
    periodic grid, mixed components zero on Nyquist planes (pinned by single-mode
    closed forms, a constant field, trace = density contrast and the Nyquist
    convention);
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
            lib.ora_structure.argtypes = [i64, p, p, p, p, ctypes.c_int, i64, ctypes.c_double, ctypes.c_double,
                                          i64, i64, i64, p, p, p, p, p, p]
            lib.ora_structure.restype = ctypes.c_int
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


def local_cells(pos, box_lo, box_hi, query, periodic=True, moved=None, k0=24, tree=None, workers=16,
                tol=1e-12, area_eps=1e-12, stride=256) -> Cells:
    """The same cells as ``cells`` for the particles in ``query``, each computed in a small
    bounded world around it, so that large inputs take seconds.

    The world of particle i holds every particle (periodic: its minimum image) within a ball of
    radius r around x_i, and its box is the cube of half-side r.  The cell computed there equals
    the cell in the whole input once no box wall remains a face and 2 R < r, R the largest vertex
    distance: every particle that could cut the cell lies within 2 R of x_i (section 2 of the
    paper's security-radius argument for buffer particles), and all of those are in the world.
    Otherwise r is doubled and the cell computed again.  r starts at 3 times the distance to
    the k0-th nearest particle.  ``moved`` ({index: position}) replaces particle positions, for
    finite differences; the moved particles must stay within r of where they were by a margin,
    which the 2 R < 0.999 r test leaves.  Particle selection uses scipy's k-d tree (a library
    search structure, not part of the cell's arithmetic)."""
    from concurrent.futures import ThreadPoolExecutor

    from scipy.spatial import cKDTree

    x = np.ascontiguousarray(pos, np.float64)
    lo = np.broadcast_to(np.asarray(box_lo, np.float64), 3)
    hi = np.broadcast_to(np.asarray(box_hi, np.float64), 3)
    L = hi - lo
    q = np.asarray(query, np.int64)
    if tree is None:
        tree = cKDTree(x - lo, boxsize=L if periodic else None)
    moved = moved or {}
    mv_idx = np.array(sorted(moved), np.int64)
    d0, _ = tree.query(x[q] - lo, k=min(k0 + 1, len(x)))
    r0 = 3.0 * d0[:, -1]

    def one(t):
        i = int(q[t])
        xi = moved.get(i, x[i])
        r = float(r0[t])
        for _ in range(40):
            r_q = min(r, 0.499 * float(L.min())) if periodic else r
            idx = np.asarray(tree.query_ball_point(xi - lo, r_q), np.int64)
            idx = np.union1d(idx, mv_idx[np.linalg.norm(_shift(np.array([moved[k] for k in mv_idx]), xi, L,
                                                                  periodic), axis=1) < r_q]
                             if len(mv_idx) else np.zeros(0, np.int64))
            if i not in idx:
                idx = np.union1d(idx, [i])
            p = x[idx].copy()
            for k, v in moved.items():
                hit = np.nonzero(idx == k)[0]
                if len(hit):
                    p[hit[0]] = v
            p = xi + _shift(p, xi, L, periodic)
            if not periodic:
                keep = np.all((p >= lo) & (p <= hi), axis=1)
                p, idx = p[keep], idx[keep]
            wlo = xi - r_q
            whi = xi + r_q
            if not periodic:
                # the cube, cut by the world's own walls (those are faces of the true cell too)
                wlo = np.maximum(wlo, lo)
                whi = np.minimum(whi, hi)
            me = int(np.nonzero(idx == i)[0][0])
            c = cells(p, wlo, whi, periodic=False, query=[me], gid=idx, tol=tol, area_eps=area_eps, stride=stride,
                      nthreads=1)
            # every particle within 2 R is in the world (the ball of radius r_q), and a cell within
            # R < r_q / 2 of its seed touches no wall of the cube (the world's own walls of a bounded
            # input are faces of the true cell as well)
            if 2.0 * c.rmax[0] < 0.999 * r_q:
                return c
            if periodic and r_q >= 0.499 * float(L.min()):
                raise RuntimeError("local_cells: cell %d reaches half the box" % i)
            r *= 2.0
        raise RuntimeError("local_cells: no world proves cell %d" % i)

    with ThreadPoolExecutor(max_workers=workers) as ex:
        res = list(ex.map(one, range(len(q))))
    nq = len(q)
    vol = np.array([c.volume[0] for c in res])
    rmax = np.array([c.rmax[0] for c in res])
    flags = np.array([c.flags[0] for c in res], np.int32)
    nnb = np.array([c.nnb[0] for c in res], np.int32)
    topo = np.stack([c.topo[0] for c in res]) if nq else np.zeros((0, 5), np.int64)
    nbr = np.stack([c._nbr[0] for c in res]) if nq else np.zeros((0, stride), np.int64)
    farea = np.stack([c._farea[0] for c in res]) if nq else np.zeros((0, stride))
    fcen = np.stack([c._fcen[0] for c in res]) if nq else np.zeros((0, stride, 3))
    fdist = np.stack([c._fdist[0] for c in res]) if nq else np.zeros((0, stride))
    return Cells(q, vol, rmax, flags, nnb, topo, nbr, farea, fcen, fdist)


def _shift(p, xi, L, periodic):
    """Separations p - xi, minimum image in a periodic box."""
    d = np.asarray(p, np.float64) - xi
    return d - L * np.rint(d / L) if periodic else d


def structure(pos, box_lo, box_hi, i, periodic=True, gid=None, tol=1e-12, area_eps=1e-12, cap=4096):
    """Full structure of cell i (section 3, memory consumption; section 4): its vertices
    (absolute, k x 3, every vertex on a face) and its faces of positive area as a list of
    (id across the face, loop of vertex numbers counter-clockwise seen from outside), ascending
    by id; the id is the neighbour's global id, or -1 .. -6 for the walls -x, +x, -y, +y, -z, +z."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    lo = np.ascontiguousarray(np.broadcast_to(np.asarray(box_lo, np.float64), 3))
    hi = np.ascontiguousarray(np.broadcast_to(np.asarray(box_hi, np.float64), 3))
    g = None if gid is None else np.ascontiguousarray(gid, dtype=np.int64)
    verts = np.zeros((cap, 3))
    fid = np.zeros(cap, np.int64)
    floff = np.zeros(cap + 1, np.int64)
    lverts = np.zeros(4 * cap, np.int32)
    nv = np.zeros(1, np.int64)
    nf = np.zeros(1, np.int64)
    rc = lib.ora_structure(pos.shape[0], _ptr(pos), _ptr(g), _ptr(lo), _ptr(hi), int(bool(periodic)), int(i), tol,
                           area_eps, cap, cap, 4 * cap, _ptr(verts), _ptr(nv), _ptr(fid), _ptr(floff), _ptr(nf),
                           _ptr(lverts))
    if rc != 0:
        raise RuntimeError("ora_structure failed with code %d" % rc)
    k, m = int(nv[0]), int(nf[0])
    faces = [(int(fid[a]), lverts[floff[a]:floff[a + 1]].copy()) for a in range(m)]
    return verts[:k].copy(), faces


def grid_tensor(field, box_len, kind="tidal"):
    """Second-derivative tensors of a periodic grid field (section 4 lists tidal-tensor and
    Hessian grid outputs among future work), by the discrete Fourier transform (numpy.fft):
    tidal T_ij = d_i d_j phi with laplacian(phi) = f / mean(f) - 1, Hessian H_ij = d_i d_j f,
    with k_a = 2 pi m / L_a for the signed frequency index m.  A mixed component is zero on the
    Nyquist plane of either of its axes.  Returns 6 x field.shape: xx, yy, zz, xy, xz, yz."""
    f = np.asarray(field, np.float64)
    L = np.broadcast_to(np.asarray(box_len, np.float64), 3)
    F = np.fft.fftn(f)
    ks, nyq = [], []
    for a, n in enumerate(f.shape):
        shape = [1, 1, 1]
        shape[a] = n
        m = np.rint(np.fft.fftfreq(n) * n)
        ks.append((2.0 * np.pi * m / L[a]).reshape(shape))
        nyq.append((np.arange(n) * 2 == n).reshape(shape))
    k2 = ks[0] ** 2 + ks[1] ** 2 + ks[2] ** 2
    out = []
    for i, j in ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)):
        kk = ks[i] * ks[j]
        if kind == "tidal":
            M = np.where(k2 > 0, kk / np.where(k2 > 0, k2, 1.0), 0.0) / f.mean()
        else:
            M = -kk * np.ones_like(k2)
        if i != j:
            M = np.where(nyq[i] | nyq[j], 0.0, M)
        out.append(np.fft.ifftn(M * F).real)
    return np.stack(out)


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


def task_index(pos, box_lo, box_hi, nt):
    """Owner cell index of every particle: floor((x - lo) / w), w = L / nt, clamped to the grid."""
    x = np.asarray(pos, np.float64)
    lo = np.broadcast_to(np.asarray(box_lo, np.float64), 3)
    L = np.broadcast_to(np.asarray(box_hi, np.float64), 3) - lo
    nt = np.asarray(nt, np.int64)
    return np.clip(np.floor((x - lo) / (L / nt)).astype(np.int64), 0, nt - 1)


def mean_spacing(n, box_lo, box_hi):
    """Mean inter-particle distance computed from the whole input (section 2, buffer zones):
    the side of the cube that holds one particle on average, (V / n)^(1/3)."""
    L = np.broadcast_to(np.asarray(box_hi, np.float64), 3) - np.broadcast_to(np.asarray(box_lo, np.float64), 3)
    return float(np.cbrt(np.prod(L) / n))


def _task_bounds(lo, hi, nt, a, j):
    """Lower and upper coordinate of task cell j along axis a (the last cell ends at hi)."""
    w = (hi[a] - lo[a]) / nt[a]
    return lo[a] + j * w, (hi[a] if j + 1 >= nt[a] else lo[a] + (j + 1) * w)


def face_cap(box_lo, box_hi, nt, ii, f, periodic=True):
    """Largest buffer thickness of face f (-x, +x, -y, +y, -z, +z) of the task with cell index ii:
    periodic, a buffered task spans less than one period ((L - w) / 2, L / 2 for a single task along
    the axis); bounded, the buffer stops at the world's face beyond it."""
    lo = np.broadcast_to(np.asarray(box_lo, np.float64), 3)
    hi = np.broadcast_to(np.asarray(box_hi, np.float64), 3)
    a = f // 2
    L = hi[a] - lo[a]
    if periodic:
        w = L / nt[a]
        return (0.5 * (L - w) if nt[a] >= 2 else 0.5 * L) * (1.0 - 1e-12)
    c0, c1 = _task_bounds(lo, hi, nt, a, ii[a])
    return hi[a] - c1 if f % 2 else c0 - lo[a]


def autoborder(pos, box_lo, box_hi, nt, border_factor=1.5, growth=1.1, steps=48, periodic=True):
    """AUTOBORDER thicknesses, n_tasks x 6 (faces -x, +x, -y, +y, -z, +z), section 2.

    The initial zone is border_factor times the mean inter-particle distance s of the whole
    input.  It grows, through border_factor * s * growth^k, until the slab beyond the face holds
    as many particles as the mean density puts in the initial zone.  For the face of task
    (i0, i1, i2) normal to axis a on side +/-, the particles counted are those in the face's column
    (same cell index on the two other axes) at distance d beyond the face:
    d = (x_a - F) or (F - x_a), taken mod L_a in a periodic box; in a bounded world only d >= 0
    counts.  F is the face's coordinate.  A slab of thickness t holds those with d < min(t, cap).
    The thickness is the first t_k whose slab holds at least n / V * A_face * t_0 particles, the
    last one if none does, and at most the face's cap (``face_cap``).
    """
    x = np.asarray(pos, np.float64)
    n = len(x)
    lo = np.broadcast_to(np.asarray(box_lo, np.float64), 3)
    hi = np.broadcast_to(np.asarray(box_hi, np.float64), 3)
    L = hi - lo
    nt = np.asarray(nt, np.int64)
    w = L / nt
    s = mean_spacing(n, lo, hi)
    thr = border_factor * s * growth ** np.arange(steps, dtype=np.float64)
    idx = task_index(x, lo, hi, nt)
    nbar = n / float(np.prod(L))
    out = np.zeros((int(np.prod(nt)), 6))
    for i0 in range(nt[0]):
        for i1 in range(nt[1]):
            for i2 in range(nt[2]):
                b = (i0 * nt[1] + i1) * nt[2] + i2
                ii = (i0, i1, i2)
                for a in range(3):
                    c1, c2 = (a + 1) % 3, (a + 2) % 3
                    col = (idx[:, c1] == ii[c1]) & (idx[:, c2] == ii[c2])
                    expect = nbar * w[c1] * w[c2] * thr[0]
                    f0, f1 = _task_bounds(lo, hi, nt, a, ii[a])
                    for side in (0, 1):
                        cap = face_cap(lo, hi, nt, ii, 2 * a + side, periodic)
                        if side:
                            d = x[col, a] - f1
                        else:
                            d = f0 - x[col, a]
                        if periodic:
                            d = np.mod(d, L[a])
                        else:
                            d = d[d >= 0]
                        t = thr[-1]
                        for tk in thr:
                            if np.count_nonzero(d < min(tk, cap)) >= expect:
                                t = tk
                                break
                        out[b, 2 * a + side] = min(t, cap)
    return out


def task_members(pos, box_lo, box_hi, nt, thick, task, periodic=True):
    """Owned particles of a task and the particle images x + s L (s in {-1, 0, 1}^3 in a periodic
    box, s = 0 in a bounded world) inside its buffered box that it does not own:
    (owned indices, buffer indices, buffer shifts).  A bounded world is closed: its own upper
    faces belong to it."""
    x = np.asarray(pos, np.float64)
    lo = np.broadcast_to(np.asarray(box_lo, np.float64), 3)
    hi = np.broadcast_to(np.asarray(box_hi, np.float64), 3)
    L = hi - lo
    nt = np.asarray(nt, np.int64)
    idx = task_index(x, lo, hi, nt)
    ii = np.array([task // (nt[1] * nt[2]), (task // nt[2]) % nt[1], task % nt[2]])
    t = np.asarray(thick, np.float64).reshape(-1, 6)[task]
    cb = [_task_bounds(lo, hi, nt, a, ii[a]) for a in range(3)]
    blo = np.array([cb[a][0] for a in range(3)]) - t[0::2]
    bhi = np.array([cb[a][1] for a in range(3)]) + t[1::2]
    if not periodic:
        blo = np.maximum(blo, lo)
        bhi = np.minimum(bhi, hi)
    owner = np.all(idx == ii, axis=1)
    shifts = (-1, 0, 1) if periodic else (0,)
    buf_i, buf_s = [], []
    for s0 in shifts:
        for s1 in shifts:
            for s2 in shifts:
                sv = np.array([s0, s1, s2])
                y = x + sv * L
                upper = (y < bhi) | ((bhi >= hi) & (y <= bhi)) if not periodic else (y < bhi)
                inside = np.all((y >= blo) & upper, axis=1)
                if s0 == 0 and s1 == 0 and s2 == 0:
                    inside &= ~owner
                k = np.nonzero(inside)[0]
                buf_i.append(k)
                buf_s.append(np.repeat(sv[None, :], len(k), axis=0))
    return np.nonzero(owner)[0], np.concatenate(buf_i), np.concatenate(buf_s)


def grid_sample(pos, box_lo, box_hi, value, dims, sub=1, chunk=4096):
    """Nearest-particle sampling of a periodic box (a cheaper grid; section 4 lists grid variants
    as future work): every sample point takes the value of the particle nearest to it, by the
    minimum-image squared distance ex*ex + ey*ey + ez*ez (FP64), ties to the smaller index.  A
    voxel averages the sub^3 points at its sub-cell centres.  Brute force over all particles.
    Returns (grid, index of the particle nearest to each voxel's last sample point)."""
    x = np.asarray(pos, np.float64)
    v = np.asarray(value, np.float64)
    lo = np.broadcast_to(np.asarray(box_lo, np.float64), 3)
    L = np.broadcast_to(np.asarray(box_hi, np.float64), 3) - lo
    dims = np.asarray(dims, np.int64)
    h = L / dims
    ii = np.stack(np.meshgrid(*[np.arange(d) for d in dims], indexing="ij"), -1).reshape(-1, 3)
    acc = np.zeros(len(ii))
    last = np.zeros(len(ii), np.int64)
    for s0 in range(sub):
        for s1 in range(sub):
            for s2 in range(sub):
                ss = np.array([s0, s1, s2], np.float64)
                q = lo + (ii + (ss + 0.5) / sub) * h
                for c0 in range(0, len(q), chunk):
                    qc = q[c0:c0 + chunk]
                    e = x[None, :, :] - qc[:, None, :]
                    e = e - L * np.rint(e / L)
                    d2 = e[:, :, 0] * e[:, :, 0] + e[:, :, 1] * e[:, :, 1] + e[:, :, 2] * e[:, :, 2]
                    j = np.argmin(d2, axis=1)        # the first (smallest index) of equal minima
                    acc[c0:c0 + chunk] += v[j]
                    last[c0:c0 + chunk] = j
    return (acc / sub ** 3).reshape(tuple(dims)), last.reshape(tuple(dims))

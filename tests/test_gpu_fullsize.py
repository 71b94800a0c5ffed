"""GPU checks at the full sizes of the benchmark's workloads.

* lattice+halos 16M (FP32, mixed and FP64 paths): sampled cells against the oracle, plus
  volume conservation over the whole box;
* clustered 2M at 256^3 (the benchmark's deposit): a field that is zero except on 96 sampled
  cells (random ones and cells the large kernels handle), every voxel against the oracle's
  exact overlaps of those cells;
* clustered 2M as 4 x 4 x 4 tasks with AUTOBORDER buffers (one batched build, incomplete cells
  re-run with wider buffers): neighbour lists identical to the whole-box build, volumes within
  1e-12;
* clustered 2M sampled at 256^3 (nearest-particle grid variant): the nearest ids of 200k
  random voxel centres against scipy's periodic k-d tree;
* clustered 2M deposit at 256^3: its tidal tensor against the oracle's discrete-Fourier
  reference, its trace against the density contrast;
* clustered 2M full structure: every cell's face ids against its neighbour list, its volume
  by the divergence theorem over its face loops, Euler's formula; 32 sampled cells (the eight
  largest among them) against the oracle's structure;
* diff262k: the adjoint gradient of a density-matching loss at full size against central
  finite differences (h = 1e-6, FP64) on the workload's 512 sampled particles.  Each
  perturbed loss is evaluated exactly on a small bounded world around the moved particle
  (its own cell and its neighbours' cells as owned cells, the surrounding particles as
  buffer); all 3072 worlds go through one batched build, and every owned cell of every
  world must be complete.
"""
import math

import numpy as np
import pytest
from scipy.spatial import cKDTree

from paper_1601_06429_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lattice16m():
    return wl.lattice_halos16m()


@pytest.mark.parametrize("precision", [1, 0])
def test_lattice_halos_16m_sampled(vt, torch_cuda, oracle, lattice16m, precision):
    w = lattice16m
    t = torch_cuda.from_numpy(w.pos).cuda()
    ctx = vt.Context().vt_build(t, vt.whole_box(w.n, w.box_lo, w.box_hi), precision=precision)
    code, nnz, retried, inc = ctx.vt_query()
    assert code == 0
    cells = ctx.vt_cells()
    vol = cells.volume.cpu().numpy()
    assert abs(vol.sum() - 1.0) <= 1e-12
    off = cells.nbr_off.cpu().numpy()
    ids = cells.nbr_ids.cpu().numpy()
    rng = np.random.default_rng(3003)
    sample = np.sort(rng.choice(w.n, 256, replace=False))
    ref = oracle.cells(w.pos.astype(np.float64), w.box_lo, w.box_hi, query=sample)
    tol = 1e-12 if precision == 0 else 2e-5
    for q, i in enumerate(sample):
        assert np.array_equal(ids[off[i]:off[i + 1]], ref.neighbours(q)), i
        assert abs(vol[i] - ref.volume[q]) <= tol * ref.volume[q], i
    del ctx, cells, t
    torch_cuda.cuda.empty_cache()


def test_clustered2m_grid_sampled_cells(vt, torch_cuda, oracle):
    w = wl.clustered2m()
    n = w.n
    t = torch_cuda.from_numpy(w.pos).cuda()
    ctx = vt.Context().vt_build(t, vt.whole_box(n, w.box_lo, w.box_hi), want_faces=True)
    assert ctx.vt_query()[0] == 0
    st = ctx.vt_cells().status.cpu().numpy()
    rng = np.random.default_rng(4004)
    retried = np.nonzero(st & 2)[0]
    sample = np.unique(np.concatenate([rng.choice(n, 80, replace=False),
                                       rng.choice(retried, min(16, retried.size), replace=False)]))
    val = np.zeros(n)
    val[sample] = rng.uniform(0.5, 2.0, sample.size)
    dims = (256, 256, 256)
    g = ctx.vt_grid_deposit(torch_cuda.from_numpy(val).cuda(), dims).cpu().numpy()
    assert ctx.vt_query()[0] == 0
    gref = oracle.grid(w.pos.astype(np.float64), w.box_lo, w.box_hi, True, val, dims, query=sample)
    assert np.abs(g - gref).max() <= 1e-11 * np.abs(gref).max()
    del ctx, t
    torch_cuda.cuda.empty_cache()


def test_clustered2m_autoborder_decomposition_equals_whole_box(vt, torch_cuda):
    w = wl.clustered2m()
    t = torch_cuda.from_numpy(w.pos).cuda()
    res = vt.decomposed_build(t, w.box_lo, w.box_hi, (4, 4, 4), border_factor=1.5)
    print("passes", res["passes"])
    assert np.all((res["status"] & (vt.CELL_INCOMPLETE | vt.CELL_FAILED)) == 0)
    c = vt.Context().vt_build(t, vt.whole_box(w.n, w.box_lo, w.box_hi)).vt_cells()
    assert np.array_equal(res["nbr_off"], c.nbr_off.cpu().numpy())
    assert np.array_equal(res["nbr_ids"], c.nbr_ids.cpu().numpy())
    v = c.volume.cpu().numpy()
    assert np.max(np.abs(res["volume"] - v) / v) <= 1e-12
    del c, t
    torch_cuda.cuda.empty_cache()


def test_clustered2m_grid_sample_against_kdtree(vt, torch_cuda):
    from scipy.spatial import cKDTree

    w = wl.clustered2m()
    t = torch_cuda.from_numpy(w.pos).cuda()
    ctx = vt.Context().vt_build(t, vt.whole_box(w.n, w.box_lo, w.box_hi))
    dims = (256, 256, 256)
    val = torch_cuda.arange(w.n, dtype=torch_cuda.float64).cuda()
    g, near = ctx.vt_grid_sample(val, dims, nearest=True)
    assert ctx.vt_query()[0] == 0
    near = near.cpu().numpy().reshape(-1)
    rng = np.random.default_rng(6006)
    v = rng.choice(near.size, 200_000, replace=False)
    ii = np.stack(np.unravel_index(v, dims), -1)
    q = (ii + 0.5) * (w.box_len / np.asarray(dims))
    p = w.pos.astype(np.float64)
    d, j = cKDTree(p, boxsize=w.box_len).query(q)
    miss = np.nonzero(j != near[v])[0]
    if len(miss):
        e = p[near[v][miss]] - q[miss]
        e -= w.box_len * np.rint(e / w.box_len)
        assert np.allclose(np.sqrt((e * e).sum(1)), d[miss], rtol=1e-14, atol=0)
    assert np.array_equal(g.cpu().numpy().reshape(-1)[v], near[v].astype(np.float64))
    del ctx, t, g
    torch_cuda.cuda.empty_cache()


def test_clustered2m_structure(vt, torch_cuda, oracle):
    """Full structure of every cell: face ids against the neighbour lists, divergence volumes
    against the cell volumes and Euler's formula (on the device), and sampled cells, the
    largest ones included, against the oracle's structure."""
    T = torch_cuda
    w = wl.clustered2m()
    ctx = vt.Context().vt_build(T.from_numpy(w.pos).cuda(), vt.whole_box(w.n, w.box_lo, w.box_hi), want_faces=True)
    cells = ctx.vt_cells()
    st = ctx.vt_structure()
    assert ctx.vt_query()[0] == 0
    n = w.n
    voff, foff, loff = st.vert_off, st.face_off, st.loop_off
    nf = st.face_nbr.numel()
    keep = st.face_nbr >= 0
    assert T.equal(st.face_nbr[keep], cells.nbr_ids)
    cell_of_face = T.repeat_interleave(T.arange(n, device="cuda"), foff.diff())
    assert T.equal(T.bincount(cell_of_face[keep], minlength=n), cells.nbr_off.diff())
    face_of_loop = T.repeat_interleave(T.arange(nf, device="cuda"), loff.diff())
    c = cell_of_face[face_of_loop]
    seeds = T.from_numpy(w.pos.astype(np.float64)).cuda()
    v = st.verts[voff[c] + st.loop_vert.long()] - seeds[c]
    nxt = T.arange(v.shape[0], device="cuda") + 1
    nxt[loff[1:] - 1] = loff[:-1]
    N = T.zeros((nf, 3), dtype=T.float64, device="cuda").index_add_(0, face_of_loop, T.cross(v, v[nxt], dim=1))
    del nxt
    vol = T.zeros(n, dtype=T.float64, device="cuda").index_add_(0, cell_of_face, (N * v[loff[:-1]]).sum(1) / 6.0)
    assert ((vol - cells.volume).abs() / cells.volume).max().item() <= 1e-11
    V, F = voff.diff(), foff.diff()
    Lc = T.bincount(c, minlength=n)
    closed = Lc == 3 * V
    assert T.all((V - Lc // 2 + F)[closed] == 2)
    assert closed.double().mean().item() >= 0.999
    del v, N, c, face_of_loop, cell_of_face
    # sampled cells against the oracle, the largest (cells of the large kernels) among them
    nv = V.cpu().numpy()
    rows = np.concatenate([np.argsort(nv)[-8:], np.random.default_rng(7007).choice(n, 24, replace=False)])
    assert nv[rows].max() > 64
    p64 = w.pos.astype(np.float64)
    for r in rows:
        vg, fg = st.cell(int(r))
        vo, fo = oracle.structure(p64, w.box_lo, w.box_hi, int(r))
        assert len(vg) == len(vo) and [j for j, _ in fg] == [j for j, _ in fo], r
        for (_, lg), (_, lo_) in zip(fg, fo):
            A, B = vg[lg], vo[lo_]
            k = int(np.argmin(((A - B[0]) ** 2).sum(1)))
            assert len(lg) == len(lo_) and np.max(np.abs(np.roll(A, -k, axis=0) - B)) <= 1e-10, r
    del ctx, st, cells
    T.cuda.empty_cache()


def test_clustered2m_tidal_tensor_of_the_deposit(vt, torch_cuda, oracle):
    """The benchmark's 256^3 deposit of the clustered set: its tidal tensor against the oracle's
    discrete-Fourier reference, and its trace against the density contrast."""
    T = torch_cuda
    w = wl.clustered2m()
    ctx = vt.Context().vt_build(T.from_numpy(w.pos).cuda(), vt.whole_box(w.n, w.box_lo, w.box_hi), want_faces=True)
    rho = ctx.vt_density(T.from_numpy(w.mass).cuda())
    g = ctx.vt_grid_deposit(rho, (256, 256, 256))
    tt = ctx.vt_grid_tensor(g, vt.TENSOR_TIDAL)
    assert ctx.vt_query()[0] == 0
    gn = g.cpu().numpy()
    d = gn / gn.mean() - 1
    tr = (tt[0] + tt[1] + tt[2]).cpu().numpy()
    assert np.max(np.abs(tr - d)) <= 1e-12 * np.abs(d).max()
    ref = oracle.grid_tensor(gn, w.box_len, "tidal")
    assert np.max(np.abs(tt.cpu().numpy() - ref)) <= 1e-12 * np.abs(ref).max()
    del ctx, tt, g, ref
    T.cuda.empty_cache()


def _target(torch, x, lam, phi, amp, mean):
    s = torch.ones(x.shape[0], dtype=x.dtype, device=x.device)
    for a in range(3):
        s = s * torch.sin(2.0 * math.pi * x[:, a] / float(lam[a]) + float(phi[a]))
    return mean * (1.0 + amp * s)


def test_diff262k_adjoint_vs_finite_differences(vt, torch_cuda):
    torch = torch_cuda
    w = wl.diff262k()
    n = w.n
    lam, phi, amp = w.extra["target_lambda"], w.extra["target_phase"], w.extra["target_amplitude"]
    mean = float(w.mass.sum())
    p64 = w.pos.astype(np.float64)
    x = torch.from_numpy(p64).cuda().requires_grad_(True)
    V = vt.voronoi_volume(x, 0.0, 1.0)
    loss = ((torch.log(1.0 / V) - torch.log(_target(torch, x, lam, phi, amp, mean))) ** 2).sum()
    loss.backward()
    grad = x.grad.cpu().numpy()

    # neighbour lists of the unperturbed set
    ctx = vt.Context().vt_build(torch.from_numpy(p64).cuda(), vt.whole_box(n, 0.0, 1.0))
    cells = ctx.vt_cells()
    off = cells.nbr_off.cpu().numpy()
    ids = cells.nbr_ids.cpu().numpy()
    tree = cKDTree(p64, boxsize=1.0)
    rows = w.extra["fd_rows"]
    h = 1e-6

    def mind(a, b):
        d = a - b
        return d - np.rint(d)

    def worlds_for(ks, factor):
        # radius: every affected cell's offset from x_k plus `factor` times its largest
        # neighbour distance (a generous scale for twice its security radius)
        worlds, meta = [], []
        for k in ks:
            aff = np.concatenate([[k], ids[off[k]:off[k + 1]]]).astype(np.int64)
            r = 0.0
            for i in aff:
                nb = ids[off[i]:off[i + 1]]
                far = np.sqrt((mind(p64[nb], p64[i]) ** 2).sum(1)).max()
                r = max(r, np.sqrt((mind(p64[i], p64[k]) ** 2).sum()) + factor * far)
            near = np.asarray(tree.query_ball_point(p64[k], min(r, 0.45)), dtype=np.int64)
            loc = np.concatenate([aff, np.setdiff1d(near, aff)])
            d = mind(p64[loc], p64[k])
            rb = np.abs(d).max() * 1.0000001
            base = p64[k] + d
            for a in range(3):
                for s in (1.0, -1.0):
                    q = base.copy()
                    q[0, a] += s * h
                    worlds.append((q[:len(aff)], q[len(aff):], p64[k] - rb, p64[k] + rb))
                    meta.append((k, a, s, len(aff)))
        return worlds, meta

    fd = {}
    todo, factor = list(rows), 2.0
    while todo:
        assert factor <= 16.0, "local worlds keep missing particles"
        worlds, meta = worlds_for(todo, factor)
        pos, desc, gid = vt.pack_worlds(worlds)
        bctx = vt.Context().vt_build(torch.from_numpy(pos).cuda(), desc, global_id=torch.from_numpy(gid).cuda())
        assert bctx.vt_query()[0] == 0
        bc = bctx.vt_cells()
        bvol = bc.volume.cpu().numpy()
        bst = bc.status.cpu().numpy()
        row, redo, part = 0, set(), {}
        for (k, a, s, na), (owned, _, _, _) in zip(meta, worlds):
            v = bvol[row:row + na]
            if (bst[row:row + na] & 1).any():
                redo.add(k)
            rt = wl.target_density(np.mod(owned, 1.0), lam, phi, amp, mean)
            part.setdefault(k, np.zeros(3))[a] += s * float(np.sum((np.log(1.0 / v) - np.log(rt)) ** 2)) / (2 * h)
            row += na
        for k in part:
            if k not in redo:
                fd[k] = part[k]
        print("local worlds: factor %.0f, %d particles, %d to redo" % (factor, len(pos), len(redo)))
        todo, factor = sorted(redo), factor * 2.0
        del bctx, bc
    fd = np.array([fd[k] for k in rows])
    g = grad[rows]
    scale = np.abs(g).max(axis=1, keepdims=True)
    err = np.abs(fd - g) / np.maximum(scale, 1e-3 * np.abs(g).max())
    print("finite differences: max scaled error %.3e, median %.3e" % (err.max(), np.median(err)))
    assert np.median(err) < 1e-6
    assert np.quantile(err, 0.99) < 1e-4

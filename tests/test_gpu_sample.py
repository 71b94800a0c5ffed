"""Nearest-particle grid sampling (vt_grid_sample) on the GPU: grid values and nearest ids
against the brute-force reference (bit-exact, ties to the smaller id) on small inputs, and the
nearest ids of the 262k clustered set at 64^3 against scipy's periodic k-d tree."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

from paper_1601_06429_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("sub", [1, 2])
def test_grid_sample_matches_oracle(vt, torch_cuda, oracle, sub):
    w = wl.uniform4096()
    t = torch_cuda.from_numpy(w.pos).cuda()
    ctx = vt.Context().vt_build(t, vt.whole_box(w.n, w.box_lo, w.box_hi))
    rng = np.random.default_rng(21)
    val = rng.uniform(0.5, 2.0, w.n)
    dims = (32, 24, 20)
    g, near = ctx.vt_grid_sample(torch_cuda.from_numpy(val).cuda(), dims, sub=sub, nearest=True)
    assert ctx.vt_query()[0] == 0
    gref, nref = oracle.grid_sample(w.pos, w.box_lo, w.box_hi, val, dims, sub=sub)
    assert np.array_equal(near.cpu().numpy(), nref)
    assert np.array_equal(g.cpu().numpy(), gref)


def _blob(n, frac, sigma, seed):
    """n particles, frac of them in a Gaussian blob of width sigma at the box centre (wrapped),
    the rest uniform: tiles over the blob hold thousands of candidates."""
    rng = np.random.default_rng(seed)
    nb = int(frac * n)
    p = np.concatenate([np.mod(0.5 + sigma * rng.standard_normal((nb, 3)), 1.0), rng.random((n - nb, 3))])
    return np.ascontiguousarray(p[rng.permutation(n)])


@pytest.mark.parametrize("sub,dims", [(1, (20, 18, 16)), (2, (10, 9, 8))])
def test_grid_sample_dense_blob_matches_oracle(vt, torch_cuda, oracle, sub, dims):
    # the blob's tiles take the per-point search, the rest the shared candidate list
    p = _blob(8192, 0.85, 0.02, 77)
    ctx = vt.Context().vt_build(torch_cuda.from_numpy(p).cuda(), vt.whole_box(len(p), 0.0, 1.0))
    val = np.random.default_rng(78).uniform(0.5, 2.0, len(p))
    g, near = ctx.vt_grid_sample(torch_cuda.from_numpy(val).cuda(), dims, sub=sub, nearest=True)
    assert ctx.vt_query()[0] == 0
    gref, nref = oracle.grid_sample(p, 0.0, 1.0, val, dims, sub=sub, chunk=1024)
    assert np.array_equal(near.cpu().numpy(), nref)
    assert np.array_equal(g.cpu().numpy(), gref)


def test_grid_sample_rejects_bounded_context(vt, torch_cuda):
    p = np.random.default_rng(3).random((4096, 3))
    ctx = vt.Context().vt_build(torch_cuda.from_numpy(p).cuda(), vt.whole_box(len(p), 0.0, 1.0, periodic=False))
    val = torch_cuda.ones(len(p), dtype=torch_cuda.float64, device="cuda")
    with pytest.raises(vt.VTError):
        ctx.vt_grid_sample(val, (8, 8, 8))


def test_grid_sample_lattice_ties(vt, torch_cuda, oracle):
    # a simple-cubic lattice with two lattice spacings per voxel: voxel centres are lattice
    # corners, equidistant from eight particles; the smallest id must win
    n = 16
    gcoord = (np.arange(n) + 0.5) / n
    p = np.stack(np.meshgrid(gcoord, gcoord, gcoord, indexing="ij"), -1).reshape(-1, 3)
    ctx = vt.Context().vt_build(torch_cuda.from_numpy(p).cuda(), vt.whole_box(len(p), 0.0, 1.0))
    val = np.arange(len(p), dtype=np.float64)
    g, near = ctx.vt_grid_sample(torch_cuda.from_numpy(val).cuda(), (8, 8, 8), nearest=True)
    gref, nref = oracle.grid_sample(p, 0.0, 1.0, val, (8, 8, 8))
    assert np.array_equal(near.cpu().numpy(), nref)
    assert np.array_equal(g.cpu().numpy(), gref)


def test_grid_sample_clustered_against_kdtree(vt, torch_cuda):
    w = wl.diff262k()
    t = torch_cuda.from_numpy(w.pos).cuda()
    ctx = vt.Context().vt_build(t, vt.whole_box(w.n, 0.0, 1.0))
    val = np.arange(w.n, dtype=np.float64)
    dims = (64, 64, 64)
    g, near = ctx.vt_grid_sample(torch_cuda.from_numpy(val).cuda(), dims, nearest=True)
    near = near.cpu().numpy().reshape(-1)
    assert np.array_equal(g.cpu().numpy().reshape(-1), near.astype(np.float64))
    p = w.pos.astype(np.float64)
    ii = np.stack(np.meshgrid(*[np.arange(d) for d in dims], indexing="ij"), -1).reshape(-1, 3)
    q = (ii + 0.5) / 64.0
    d, j = cKDTree(p, boxsize=1.0).query(q)
    miss = np.nonzero(j != near)[0]
    if len(miss):
        e = p[near[miss]] - q[miss]
        e -= np.rint(e)
        dn = np.sqrt((e * e).sum(1))
        assert np.allclose(dn, d[miss], rtol=1e-14, atol=0), "a different nearest particle that is farther"
    assert len(miss) <= 1e-5 * len(q)

"""Domain decomposition with AUTOBORDER buffers (section 2), on the GPU.

* vt_decompose's thicknesses equal the reference rule (oracle.autoborder), which derives the mean
  spacing and the thickness schedule itself from the positions, the box and BORDERFACTOR: the two
  share nothing but the positions; its task sizes equal the reference ownership and buffer
  membership;
* vt_decompose_pack writes every task's owned particles and buffer particle images exactly
  (global ids, positions shifted by whole periods);
* the decomposed build (vt_decomposed_build: all tasks in one batched build, incomplete cells
  re-run with wider buffers, in the library) reproduces the whole-box periodic tessellation:
  identical neighbour lists and volumes within 1e-12, every cell complete; sampled cells also
  against the oracle;
* the same for the paper's scheme (b) on its real shape: a bounded, elongated (10 : 1 : 1) survey
  volume cut into slabs, against the whole bounded world's tessellation and the oracle.
"""
import numpy as np
import pytest

from paper_1601_06429_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def clustered262k():
    return wl.diff262k()


@pytest.fixture(scope="module")
def slab262k():
    return wl.survey_slab()


def _whole_world(vt, torch, p, lo, hi, periodic=True):
    ctx = vt.Context().vt_build(torch.from_numpy(p).cuda(), vt.whole_box(len(p), lo, hi, periodic, walls=63))
    code, _, _, inc = ctx.vt_query()
    assert code == 0 and inc == 0
    c = ctx.vt_cells()
    return c.volume.cpu().numpy(), c.nbr_off.cpu().numpy(), c.nbr_ids.cpu().numpy()


def test_decompose_thickness_and_sizes_match_reference(vt, torch_cuda, oracle, clustered262k):
    p = clustered262k.pos
    nt = (4, 4, 4)
    thick, n_own, n_gh = vt.Context().vt_decompose(torch_cuda.from_numpy(p).cuda(), 0.0, 1.0, nt,
                                                   border_factor=1.5)
    ref = oracle.autoborder(p, 0.0, 1.0, nt, border_factor=1.5)
    np.testing.assert_allclose(thick, ref, rtol=1e-14, atol=0)
    s = oracle.mean_spacing(len(p), 0.0, 1.0)
    assert np.any(thick > 1.5 * s * 1.05)     # the clustered set needs wider buffers somewhere
    idx = oracle.task_index(p, 0.0, 1.0, nt)
    owner = (idx[:, 0] * 4 + idx[:, 1]) * 4 + idx[:, 2]
    assert np.array_equal(n_own, np.bincount(owner, minlength=64))
    for b in (0, 21, 42, 63):
        _, buf, _ = oracle.task_members(p, 0.0, 1.0, nt, ref, b)
        assert n_gh[b] == len(buf)


def test_decompose_pack_writes_owned_and_buffer_images(vt, torch_cuda, oracle, clustered262k):
    p = clustered262k.pos
    nt = (4, 4, 4)
    ctx = vt.Context()
    t = torch_cuda.from_numpy(p).cuda()
    thick, _, _ = ctx.vt_decompose(t, 0.0, 1.0, nt, border_factor=1.5)
    bpos, gid, items = ctx.vt_decompose_pack(t, 0.0, 1.0, nt, thick)
    bpos, gid = bpos.cpu().numpy(), gid.cpu().numpy()
    assert items[0]["offset"] == 0 and sum(it["n_owned"] for it in items) == len(p)
    p64 = p.astype(np.float64)
    for b in (0, 5, 42, 63):
        it = items[b]
        o0, o1 = it["offset"], it["offset"] + it["n_owned"]
        own, buf, sh = oracle.task_members(p, 0.0, 1.0, nt, thick, b)
        assert np.array_equal(np.sort(gid[o0:o1]), own)
        assert np.array_equal(bpos[o0:o1], p64[gid[o0:o1]])
        g1 = gid[o1:o1 + it["n_ghost"]]
        got = sorted(zip(g1.tolist(), map(tuple, bpos[o1:o1 + it["n_ghost"]].tolist())))
        want = sorted(zip(buf.tolist(), map(tuple, (p64[buf] + sh).tolist())))
        assert got == want


@pytest.mark.parametrize("nt", [(4, 4, 4), (2, 1, 1), 8])   # 8: scheme (a), 2 x 2 x 2
def test_decomposed_build_equals_whole_box(vt, torch_cuda, oracle, clustered262k, nt):
    p = clustered262k.pos
    print("decomposed build, periodic clustered 262k, tasks", nt, flush=True)
    res = vt.decomposed_build(torch_cuda.from_numpy(p).cuda(), 0.0, 1.0, nt, border_factor=1.5)
    assert np.all((res["status"] & (vt.CELL_INCOMPLETE | vt.CELL_FAILED)) == 0), res["passes"]
    assert res["passes"][-1]["incomplete"] == 0
    vol, off, ids = _whole_world(vt, torch_cuda, p, 0.0, 1.0)
    assert np.array_equal(res["nbr_off"], off)
    assert np.array_equal(res["nbr_ids"], ids)
    assert np.max(np.abs(res["volume"] - vol) / vol) <= 1e-12
    # and sampled cells against the oracle
    rng = np.random.default_rng(5005)
    q = np.sort(rng.choice(len(p), 64, replace=False))
    ref = oracle.cells(p.astype(np.float64), 0.0, 1.0, query=q)
    for k, i in enumerate(q):
        assert np.array_equal(res["nbr_ids"][res["nbr_off"][i]:res["nbr_off"][i + 1]], ref.neighbours(k))
        assert abs(res["volume"][i] - ref.volume[k]) <= 1e-12 * ref.volume[k]


def test_bounded_slab_decompose_matches_reference(vt, torch_cuda, oracle, slab262k):
    w = slab262k
    p = w.pos
    nt = vt.task_grid(8, "b")
    t = torch_cuda.from_numpy(p).cuda()
    ctx = vt.Context()
    thick, n_own, n_gh = ctx.vt_decompose(t, w.box_lo, w.box_hi, nt, border_factor=1.5, periodic=False)
    ref = oracle.autoborder(p, w.box_lo, w.box_hi, nt, border_factor=1.5, periodic=False)
    np.testing.assert_allclose(thick, ref, rtol=1e-14, atol=0)
    assert np.all(thick[:, 2:] == 0.0) and thick[0, 0] == 0.0 and thick[-1, 1] == 0.0
    bpos, gid, items = ctx.vt_decompose_pack(t, w.box_lo, w.box_hi, nt, thick, periodic=False)
    bpos, gid = bpos.cpu().numpy(), gid.cpu().numpy()
    for b in (0, 3, 7):
        it = items[b]
        own, buf, _ = oracle.task_members(p, w.box_lo, w.box_hi, nt, thick, b, periodic=False)
        o0, o1 = it["offset"], it["offset"] + it["n_owned"]
        assert n_own[b] == len(own) and n_gh[b] == len(buf)
        assert np.array_equal(np.sort(gid[o0:o1]), own)
        assert np.array_equal(np.sort(gid[o1:o1 + it["n_ghost"]]), np.sort(buf))
        # the world's own faces are true walls of the item; the cut faces are not
        walls = it["walls"]
        assert walls & 0b111100 == 0b111100
        assert bool(walls & 1) == (b == 0) and bool(walls & 2) == (b == 7 or it["hi"][0] >= w.box_hi[0])


def test_bounded_slab_decomposed_build_equals_whole_world(vt, torch_cuda, oracle, slab262k):
    """Scheme (b) on the shape it is meant for: a bounded 10 x 1 x 1 clustered volume cut into 8
    slabs with AUTOBORDER buffers equals the whole bounded world's tessellation and the oracle."""
    w = slab262k
    p = w.pos
    nt = vt.task_grid(8, "b")
    print("decomposed build, bounded slab 262k, tasks", nt, flush=True)
    res = vt.decomposed_build(torch_cuda.from_numpy(p).cuda(), w.box_lo, w.box_hi, nt, border_factor=1.5,
                              periodic=False)
    assert np.all((res["status"] & (vt.CELL_INCOMPLETE | vt.CELL_FAILED)) == 0), res["passes"]
    vol, off, ids = _whole_world(vt, torch_cuda, p, w.box_lo, w.box_hi, periodic=False)
    assert np.array_equal(res["nbr_off"], off)
    assert np.array_equal(res["nbr_ids"], ids)
    assert np.max(np.abs(res["volume"] - vol) / vol) <= 1e-12
    assert abs(vol.sum() - np.prod(w.box_len)) <= 1e-12 * np.prod(w.box_len)
    # sampled cells (and cells next to the cuts between slabs) against the oracle's bounded world
    rng = np.random.default_rng(6006)
    cut = np.nonzero(np.abs(p[:, 0] - np.round(p[:, 0] / 1.25) * 1.25) < 0.02)[0]
    q = np.unique(np.concatenate([rng.choice(len(p), 48, replace=False), rng.choice(cut, 48, replace=False)]))
    ref = oracle.cells(p.astype(np.float64), w.box_lo, w.box_hi, periodic=False, query=q)
    for k, i in enumerate(q):
        assert np.array_equal(res["nbr_ids"][res["nbr_off"][i]:res["nbr_off"][i + 1]], ref.neighbours(k))
        assert abs(res["volume"][i] - ref.volume[k]) <= 1e-12 * ref.volume[k]

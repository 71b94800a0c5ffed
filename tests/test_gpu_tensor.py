"""Grid tensors (vt_grid_tensor) on the GPU against the oracle's discrete-Fourier reference:
random fields on grids of unequal power-of-two sides (the longest lines, 4096, along a strided
and along the contiguous axis), a deposited density grid, both kinds, within 1e-12 of the
largest component; bad sizes are refused."""
import numpy as np
import pytest

from paper_1601_06429_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _ctx(vt, torch_cuda):
    w = wl.uniform4096()
    return w, vt.Context().vt_build(torch_cuda.from_numpy(w.pos).cuda(), vt.whole_box(w.n, w.box_lo, w.box_hi))


@pytest.mark.parametrize("kind", ["tidal", "hessian"])
@pytest.mark.parametrize("shape", [(32, 16, 64), (8, 128, 4), (2, 2, 2), (4096, 2, 4), (2, 4, 4096)])
def test_grid_tensor_random_field(vt, torch_cuda, oracle, kind, shape):
    w, ctx = _ctx(vt, torch_cuda)
    f = 2.0 + np.random.default_rng(51).random(shape)
    k = vt.TENSOR_TIDAL if kind == "tidal" else vt.TENSOR_HESSIAN
    out = ctx.vt_grid_tensor(torch_cuda.from_numpy(f).cuda(), k).cpu().numpy()
    ref = oracle.grid_tensor(f, w.box_hi - w.box_lo, kind)
    assert np.max(np.abs(out - ref)) <= 1e-12 * max(np.abs(ref).max(), 1e-300)


def test_grid_tensor_of_the_deposited_density(vt, torch_cuda, oracle):
    w = wl.uniform4096()
    ctx = vt.Context().vt_build(torch_cuda.from_numpy(w.pos).cuda(), vt.whole_box(w.n, w.box_lo, w.box_hi),
                                want_faces=True)
    rho = ctx.vt_density()
    g = ctx.vt_grid_deposit(rho, (32, 32, 32))
    T = ctx.vt_grid_tensor(g).cpu().numpy()
    ref = oracle.grid_tensor(g.cpu().numpy(), 1.0, "tidal")
    assert np.max(np.abs(T - ref)) <= 1e-12 * np.abs(ref).max()
    gn = g.cpu().numpy()
    # the trace is the density contrast (the diagonal components keep every mode)
    d = gn / gn.mean() - 1
    assert np.max(np.abs(T[0] + T[1] + T[2] - d)) <= 1e-12 * np.abs(d).max()


def test_grid_tensor_rejects_bad_sizes(vt, torch_cuda):
    _, ctx = _ctx(vt, torch_cuda)
    with pytest.raises(vt.VTError):
        ctx.vt_grid_tensor(torch_cuda.ones((24, 16, 16), dtype=torch_cuda.float64, device="cuda"))
    with pytest.raises(vt.VTError):
        ctx.vt_grid_tensor(torch_cuda.ones((1, 16, 16), dtype=torch_cuda.float64, device="cuda"))

"""The allocation-free entry point vt_grid_tensor_noalloc, through the C ABI: the same output,
bit for bit, as vt_grid_tensor (which keeps its scratch in the context) on two calls in a row, the
second on a smaller grid (the static scratch keeps the first call's contents), and oversized grids
rejected before anything is enqueued."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_noalloc_grid_tensor_equals_the_allocating_one(vt, torch_cuda):
    T = torch_cuda
    rng = np.random.default_rng(77)
    p = rng.random((3000, 3))
    ctx = vt.Context().vt_build(T.from_numpy(p).cuda(), vt.whole_box(len(p), 0.0, 1.0))
    assert ctx.vt_query()[0] == 0
    L = vt.lib()
    for shape, kind in (((64, 32, 128), vt.TENSOR_TIDAL), ((16, 8, 32), vt.TENSOR_HESSIAN)):
        print("grid tensor, no-alloc variant:", shape, kind, flush=True)
        rho = ctx.vt_density(None)
        g = ctx.vt_grid_deposit(rho, shape)
        ref = ctx.vt_grid_tensor(g, kind)
        out = T.full((6,) + shape, np.nan, dtype=T.float64, device="cuda")
        code = L.vt_grid_tensor_noalloc(ctx._ctx, vt._ptr(g), *shape, kind, vt._ptr(out), vt._stream())
        assert code == 0
        T.cuda.synchronize()
        assert ctx.vt_query()[0] == 0
        assert T.equal(out, ref)
    # above the static array's size: rejected synchronously, nothing written
    big = (256, 128, 128)
    assert np.prod(big) > 1 << 21
    out = T.zeros(1, dtype=T.float64, device="cuda")
    g = T.zeros(1, dtype=T.float64, device="cuda")
    assert L.vt_grid_tensor_noalloc(ctx._ctx, vt._ptr(g), *big, vt.TENSOR_TIDAL, vt._ptr(out), vt._stream()) == 1
    assert out.item() == 0.0

// grid.hip -- average Voronoi density on a regular grid (paper section 2,
// optional grid output; also its discussion section).  The paper does not give
// the averaging rule; this is the exact volume average of the
// piecewise-constant field over each voxel:
//   grid[v] = sum_i value_i * vol(cell_i ∩ voxel_v) / vol(voxel_v).
// One wavefront per cell: the cell is rebuilt from its facets (the bisectors
// of its neighbours, from the staging rows of the clip kernel), then clipped
// by the six walls of every voxel its bounding box touches; each overlap volume
// is added to the voxel with an FP64 atomic.  Cells inside one voxel add their
// whole volume directly.
#include "poly.h"

template <int VPL>
struct GridMem {
    double vp[64 * VPL][3];
    uint64_t fm_save[64 * VPL][VPL];
    PolyMem<double, VPL> P;
};

struct GridArgs {
    const void *spos;
    const DevItem *items;
    const int32_t *cells;
    int64_t ncells;
    const int32_t *queue;
    int64_t queue_cap;
    const int64_t *crow;
    const int32_t *ccnt;
    const uint8_t *cstat;
    const double *cvol;
    const int32_t *stage_ids;
    const int32_t *srow;
    const double *value;
    uint32_t *counters;
    double *grid;
    int nx, ny, nz;
};

template <typename PT4>
__device__ __forceinline__ void gpos(const void *spos, int32_t j, double &x, double &y, double &z) {
    PT4 p = ((const PT4 *)spos)[j];
    x = (double)p.x;
    y = (double)p.y;
    z = (double)p.z;
}

__device__ __forceinline__ int64_t wrapi(int64_t i, int n) {
    int64_t r = i % n;
    return r < 0 ? r + n : r;
}

template <typename PT4, int VPL, bool RETRY>
__global__ void __launch_bounds__(256) k_grid(GridArgs A) {
    using M = GridMem<VPL>;
    extern __shared__ char smem[];
    const int wid = threadIdx.x >> 6;
    M &S = *reinterpret_cast<M *>(smem + (size_t)wid * sizeof(M));
    const int lane = lane_id();
    const uint64_t mybit = 1ull << lane;
    const DevItem &it = A.items[0];
    const double h[3] = {it.L[0] / A.nx, it.L[1] / A.ny, it.L[2] / A.nz};
    const double hv = h[0] * h[1] * h[2];
    const int dims[3] = {A.nx, A.ny, A.nz};
    const int64_t ntodo = RETRY ? (int64_t)min((uint64_t)A.counters[CTR_QUEUE], (uint64_t)A.queue_cap) : A.ncells;

    for (;;) {
        int64_t w = 0;
        if (lane == 0) w = (int64_t)atomicAdd(&A.counters[RETRY ? CTR_GRID_RETRY : CTR_GRID], 1u);
        w = (int64_t)__shfl((long long)w, 0);
        if (w >= ntodo) break;
        const int32_t c = RETRY ? A.queue[w] : (int32_t)w;
        const uint8_t st = A.cstat[c];
        if (!RETRY && (st & VT_CELL_RETRIED)) continue;
        if (st & VT_CELL_FAILED) continue;
        const int32_t j0 = A.cells[c];
        const double val = A.value[A.srow[j0]];
        if (val == 0.0) continue;
        double sx, sy, sz;
        gpos<PT4>(A.spos, j0, sx, sy, sz);
        const double xs[3] = {sx, sy, sz};
        double blo[3], bhi[3];
        for (int a = 0; a < 3; ++a) {
            if (it.periodic) {
                blo[a] = -0.5 * it.L[a];
                bhi[a] = 0.5 * it.L[a];
            } else {
                blo[a] = it.lo[a] - xs[a];
                bhi[a] = it.lo[a] + it.L[a] - xs[a];
            }
        }
        Poly<double, VPL> P;
        P.init_box(S.P, blo, bhi);
        bool bad = false;
        const int64_t row = A.crow[c];
        const int32_t cnt = A.ccnt[c];
        for (int32_t t = 0; t < cnt; ++t) {
            const int32_t j = A.stage_ids[row + t];
            double px, py, pz;
            gpos<PT4>(A.spos, j, px, py, pz);
            P4<double> p;
            p.x = px - sx;
            p.y = py - sy;
            p.z = pz - sz;
            if (it.periodic) {
                p.x -= it.L[0] * rint(p.x / it.L[0]);
                p.y -= it.L[1] * rint(p.y / it.L[1]);
                p.z -= it.L[2] * rint(p.z / it.L[2]);
            }
            p.d = 0.5 * (p.x * p.x + p.y * p.y + p.z * p.z);
            int rc = P.clip(S.P, p, j);
            if (rc < 0) {
                bad = true;
                break;
            }
        }
        if (bad) {
            if (lane == 0) atomicOr(&A.counters[CTR_STATUS], VT_DEV_CAPACITY);
            continue;
        }
        // bounding box of the cell -> voxel index ranges
        double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
#pragma unroll
        for (int s = 0; s < VPL; ++s) {
            if (P.alive[s] & mybit) {
                const double v[3] = {P.vx[s], P.vy[s], P.vz[s]};
                for (int a = 0; a < 3; ++a) {
                    mn[a] = fmin(mn[a], v[a]);
                    mx[a] = fmax(mx[a], v[a]);
                }
            }
        }
        int64_t i0[3], i1[3];
        for (int a = 0; a < 3; ++a) {
            mn[a] = wave_min(mn[a]);
            mx[a] = wave_max(mx[a]);
            i0[a] = (int64_t)floor((xs[a] + mn[a] - it.lo[a]) / h[a]);
            i1[a] = (int64_t)floor((xs[a] + mx[a] - it.lo[a]) / h[a]);
            if (!it.periodic) {
                if (i0[a] < 0) i0[a] = 0;
                if (i1[a] > dims[a] - 1) i1[a] = dims[a] - 1;
            }
        }
        if (i0[0] == i1[0] && i0[1] == i1[1] && i0[2] == i1[2]) {
            if (lane == 0) {
                int64_t g = (wrapi(i0[0], dims[0]) * dims[1] + wrapi(i0[1], dims[1])) * dims[2] + wrapi(i0[2], dims[2]);
                unsafeAtomicAdd(&A.grid[g], val * A.cvol[c] / hv);
            }
            continue;
        }
        // save the cell; every voxel starts from it
        const Poly<double, VPL> P0 = P;
#pragma unroll
        for (int r = 0; r < VPL; ++r)
#pragma unroll
            for (int ww = 0; ww < VPL; ++ww) S.fm_save[r * 64 + lane][ww] = S.P.fm[r * 64 + lane][ww];
        wave_sync();
        for (int64_t ix = i0[0]; ix <= i1[0]; ++ix)
            for (int64_t iy = i0[1]; iy <= i1[1]; ++iy)
                for (int64_t iz = i0[2]; iz <= i1[2]; ++iz) {
                    P = P0;
#pragma unroll
                    for (int r = 0; r < VPL; ++r)
#pragma unroll
                        for (int ww = 0; ww < VPL; ++ww) S.P.fm[r * 64 + lane][ww] = S.fm_save[r * 64 + lane][ww];
                    wave_sync();
                    const int64_t idx[3] = {ix, iy, iz};
                    bool empty = false;
                    for (int a = 0; a < 3 && !empty; ++a) {
                        const double vlo = it.lo[a] + idx[a] * h[a] - xs[a];
                        const double vhi = vlo + h[a];
                        for (int sg = 0; sg < 2 && !empty; ++sg) {
                            P4<double> p;
                            p.x = p.y = p.z = 0.0;
                            double nrm = sg ? 1.0 : -1.0;
                            if (a == 0) p.x = nrm;
                            if (a == 1) p.y = nrm;
                            if (a == 2) p.z = nrm;
                            p.d = sg ? vhi : -vlo;
                            int rc = P.clip(S.P, p, -100);
                            if (rc == CLIP_EMPTY) empty = true;
                            else if (rc < 0) {
                                empty = true;
                                if (lane == 0) atomicOr(&A.counters[CTR_STATUS], VT_DEV_CAPACITY);
                            }
                        }
                    }
                    if (empty) continue;
                    const double vol = P.volume(S.P, S.vp);
                    if (lane == 0 && vol > 0.0) {
                        int64_t g = (wrapi(ix, dims[0]) * dims[1] + wrapi(iy, dims[1])) * dims[2] + wrapi(iz, dims[2]);
                        unsafeAtomicAdd(&A.grid[g], val * vol / hv);
                    }
                    wave_sync();
                }
    }
}

__global__ void k_zero_f64(double *p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

template <typename PT4, int VPL, bool RETRY>
static hipError_t launch_grid_one(vt_ctx *c, GridArgs &a, int wpb) {
    const size_t lds = sizeof(GridMem<VPL>) * (size_t)wpb;
    auto kern = k_grid<PT4, VPL, RETRY>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    int ncu = 0;
    hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device);
    if (ncu <= 0) ncu = 256;
    int64_t blocks = RETRY ? (int64_t)ncu : (int64_t)ncu * 8 / wpb;
    kern<<<dim3((unsigned)blocks), dim3(64 * wpb), lds, c->stream>>>(a);
    return hipGetLastError();
}

hipError_t vt_launch_grid(vt_ctx *c, const double *value, int nx, int ny, int nz, double *grid) {
    const int64_t ng = (int64_t)nx * ny * nz;
    k_zero_f64<<<(ng + 255) / 256, 256, 0, c->stream>>>(grid, ng);
    // work counters of the two deposit kernels
    hipError_t ez = vt_launch_zero_u32(c->counters + CTR_GRID, 2, c->stream);
    if (ez != hipSuccess) return ez;
    GridArgs a;
    a.spos = c->spos;
    a.items = c->items;
    a.cells = c->cells;
    a.ncells = c->n_owned;
    a.queue = c->queue;
    a.queue_cap = c->cap_retry;
    a.crow = c->crow;
    a.ccnt = c->ccnt;
    a.cstat = c->cstat;
    a.cvol = c->cvol;
    a.stage_ids = c->stage_ids;
    a.srow = c->srow;
    a.value = value;
    a.counters = c->counters;
    a.grid = grid;
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    hipError_t e;
    if (c->dtype == VT_F32) {
        e = launch_grid_one<float4, 2, false>(c, a, 4);
        if (e == hipSuccess) e = launch_grid_one<float4, 4, true>(c, a, 1);
    } else {
        e = launch_grid_one<double4, 2, false>(c, a, 4);
        if (e == hipSuccess) e = launch_grid_one<double4, 4, true>(c, a, 1);
    }
    return e;
}

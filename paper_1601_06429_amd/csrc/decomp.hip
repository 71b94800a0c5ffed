// decomp.hip -- domain decomposition with AUTOBORDER buffer zones (paper
// section 2: sub-volumes with buffer particles; the buffer grows where the
// particle density in it is below the mean).  The tasks of a periodic box
// become the items of one batched build.
//
// Ownership is by integer cell index, so the tasks partition the particles.
// For the thicknesses, every particle adds itself to a histogram per face over
// the caller's thresholds: beyond the +a face of the task j steps below it
// along axis a at distance u_a + (j - 1) w_a, and beyond the -a face of the task
// j steps above at distance (w_a - u_a) + (j - 1) w_a, u the particle's offset
// in its own task.  The buffer particles of a task are the particle images
// x + s L (s in {-1, 0, 1}^3) inside its buffered box that it does not own; the
// buffered box spans less than one period per axis, so each particle has at
// most one image there.
#include <math.h>

#include <algorithm>
#include <vector>

#include "vt_internal.h"

namespace {

struct DecGeo {
    double lo[3], L[3], w[3], tmax[3];
    int nt[3];
};

template <typename T>
__device__ __forceinline__ void dec_pos(const T *pos, int64_t p, double x[3]) {
    x[0] = (double)pos[3 * p + 0];
    x[1] = (double)pos[3 * p + 1];
    x[2] = (double)pos[3 * p + 2];
}

// owner cell index and the offset inside it, per axis
__device__ __forceinline__ void dec_owner(const DecGeo &g, const double x[3], int i[3], double u[3]) {
    for (int a = 0; a < 3; ++a) {
        int k = (int)floor((x[a] - g.lo[a]) / g.w[a]);
        k = k < 0 ? 0 : (k >= g.nt[a] ? g.nt[a] - 1 : k);
        i[a] = k;
        u[a] = x[a] - (g.lo[a] + (double)k * g.w[a]);
    }
}

__device__ __forceinline__ int dec_task(const DecGeo &g, int i0, int i1, int i2) {
    return (i0 * g.nt[1] + i1) * g.nt[2] + i2;
}

// number of thresholds <= d (the histogram bin of a particle at distance d)
__device__ __forceinline__ int dec_bin(const double *thr, int n_thr, double d) {
    int lo = 0, hi = n_thr;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (thr[mid] <= d) lo = mid + 1; else hi = mid;
    }
    return lo;
}

template <typename T>
__global__ void k_dec_slab(const T *pos, int64_t n, DecGeo g, const double *thr, int n_thr, uint32_t *hist) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    double x[3], u[3];
    int i[3];
    dec_pos(pos, p, x);
    dec_owner(g, x, i, u);
    for (int a = 0; a < 3; ++a) {
        for (int side = 0; side < 2; ++side) {
            // side 1: beyond the +a face of the tasks below; side 0: beyond the -a face of those above
            double d0 = side ? u[a] : g.w[a] - u[a];
            d0 = d0 < 0.0 ? 0.0 : d0;
            for (int j = 1;; ++j) {
                const double d = d0 + (double)(j - 1) * g.w[a];
                if (d >= g.tmax[a]) break;
                const int k = dec_bin(thr, n_thr, d);
                if (k >= n_thr) break;
                int ii[3] = {i[0], i[1], i[2]};
                const int s = side ? -j : j;
                ii[a] = ((i[a] + s) % g.nt[a] + g.nt[a]) % g.nt[a];
                const int b = dec_task(g, ii[0], ii[1], ii[2]);
                atomicAdd(&hist[((int64_t)b * 6 + 2 * a + side) * n_thr + k], 1u);
            }
        }
    }
}

// every (task, image) membership of particle p: f(task, s[3], ghost)
template <typename T, typename F>
__device__ __forceinline__ void dec_members(const T *pos, int64_t p, const DecGeo &g, const double *thick,
                                            const double Tmax[3], const uint8_t *own_mask, const int32_t *tpos,
                                            F f) {
    double x[3], u[3];
    int i[3];
    dec_pos(pos, p, x);
    dec_owner(g, x, i, u);
    const int owner = dec_task(g, i[0], i[1], i[2]);
    const bool owns = own_mask ? own_mask[p] != 0 : true;
    // per axis: image shifts and the task indices whose widest buffered interval holds the image
    int ns[3], sh[3][3], ia[3][3], ib_[3][3];
    for (int a = 0; a < 3; ++a) {
        ns[a] = 0;
        for (int s = -1; s <= 1; ++s) {
            const double y = x[a] + (double)s * g.L[a];
            int k0 = (int)floor((y - g.lo[a] - Tmax[a]) / g.w[a]);
            int k1 = (int)floor((y - g.lo[a] + Tmax[a]) / g.w[a]);
            k0 = k0 < 0 ? 0 : k0;
            k1 = k1 >= g.nt[a] ? g.nt[a] - 1 : k1;
            if (k0 > k1) continue;
            sh[a][ns[a]] = s;
            ia[a][ns[a]] = k0;
            ib_[a][ns[a]] = k1;
            ++ns[a];
        }
    }
    for (int q0 = 0; q0 < ns[0]; ++q0)
        for (int j0 = ia[0][q0]; j0 <= ib_[0][q0]; ++j0)
            for (int q1 = 0; q1 < ns[1]; ++q1)
                for (int j1 = ia[1][q1]; j1 <= ib_[1][q1]; ++j1)
                    for (int q2 = 0; q2 < ns[2]; ++q2)
                        for (int j2 = ia[2][q2]; j2 <= ib_[2][q2]; ++j2) {
                            const int b = dec_task(g, j0, j1, j2);
                            if (tpos && tpos[b] < 0) continue;
                            const int s[3] = {sh[0][q0], sh[1][q1], sh[2][q2]};
                            const int jj[3] = {j0, j1, j2};
                            bool in = true;
                            for (int a = 0; a < 3 && in; ++a) {
                                const double y = x[a] + (double)s[a] * g.L[a];
                                const double blo = g.lo[a] + (double)jj[a] * g.w[a] - thick[6 * b + 2 * a];
                                const double bhi = g.lo[a] + (double)(jj[a] + 1) * g.w[a] + thick[6 * b + 2 * a + 1];
                                in = y >= blo && y < bhi;
                            }
                            if (!in) continue;
                            const bool self = b == owner && s[0] == 0 && s[1] == 0 && s[2] == 0;
                            f(b, s, !(self && owns));
                        }
}

// The per-task counters are few and every particle adds to one or more of them, so a global atomic
// per membership serializes on a few addresses across the whole chip.  Each block therefore counts
// in LDS (nc = 2 per listed task: owned, buffer) and adds its totals once; the scatter reserves one
// range per block and counter, then places its particles within it with LDS atomics.
#define DEC_TPB 256
#define DEC_LDS_COUNTERS 4096   // above this, the kernels count with global atomics directly

template <typename T>
__global__ void __launch_bounds__(DEC_TPB) k_dec_count(const T *pos, int64_t n, DecGeo g, const double *thick,
                                                       double T0, double T1, double T2, const uint8_t *own_mask,
                                                       const int32_t *tpos, int nc, unsigned long long *cnt) {
    extern __shared__ uint32_t lc[];
    const bool lds = nc <= DEC_LDS_COUNTERS;
    if (lds) {
        for (int i = threadIdx.x; i < nc; i += DEC_TPB) lc[i] = 0;
        __syncthreads();
    }
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double Tm[3] = {T0, T1, T2};
    if (p < n)
        dec_members(pos, p, g, thick, Tm, own_mask, tpos, [&](int b, const int *, bool ghost) {
            const int k = 2 * (tpos ? tpos[b] : b) + (ghost ? 1 : 0);
            if (lds) atomicAdd(&lc[k], 1u);
            else atomicAdd(&cnt[k], 1ull);
        });
    if (lds) {
        __syncthreads();
        for (int i = threadIdx.x; i < nc; i += DEC_TPB)
            if (lc[i]) atomicAdd(&cnt[i], (unsigned long long)lc[i]);
    }
}

template <typename T>
__global__ void __launch_bounds__(DEC_TPB) k_dec_scatter(const T *pos, int64_t n, DecGeo g, const double *thick,
                                                         double T0, double T1, double T2, const uint8_t *own_mask,
                                                         const int32_t *tpos, int nc, const int64_t *base,
                                                         unsigned long long *cur, int64_t cap, double *out_pos,
                                                         int32_t *out_gid) {
    extern __shared__ uint32_t lc[];
    unsigned long long *lb = (unsigned long long *)(lc + ((nc + 1) & ~1));  // block's reserved range starts
    const bool lds = nc <= DEC_LDS_COUNTERS;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double Tm[3] = {T0, T1, T2};
    double x[3] = {0.0, 0.0, 0.0};
    if (p < n) dec_pos(pos, p, x);
    if (lds) {
        for (int i = threadIdx.x; i < nc; i += DEC_TPB) lc[i] = 0;
        __syncthreads();
        if (p < n)
            dec_members(pos, p, g, thick, Tm, own_mask, tpos, [&](int b, const int *, bool ghost) {
                atomicAdd(&lc[2 * (tpos ? tpos[b] : b) + (ghost ? 1 : 0)], 1u);
            });
        __syncthreads();
        for (int i = threadIdx.x; i < nc; i += DEC_TPB) {
            lb[i] = lc[i] ? atomicAdd(&cur[i], (unsigned long long)lc[i]) : 0ull;
            lc[i] = 0;
        }
        __syncthreads();
    }
    if (p < n)
        dec_members(pos, p, g, thick, Tm, own_mask, tpos, [&](int b, const int *s, bool ghost) {
            const int k = 2 * (tpos ? tpos[b] : b) + (ghost ? 1 : 0);
            const int64_t slot = lds ? (int64_t)lb[k] + (int64_t)atomicAdd(&lc[k], 1u) : (int64_t)atomicAdd(&cur[k], 1ull);
            const int64_t o = base[k] + slot;
            if (o >= cap) return;  // the count pass sized the output; never write past it
            for (int a = 0; a < 3; ++a) out_pos[3 * o + a] = x[a] + (double)s[a] * g.L[a];
            out_gid[o] = (int32_t)p;
        });
}

static size_t dec_lds_bytes(int nc, bool scatter) {
    if (nc > DEC_LDS_COUNTERS) return 0;
    const size_t c32 = sizeof(uint32_t) * (size_t)((nc + 1) & ~1);
    return scatter ? c32 + sizeof(unsigned long long) * (size_t)nc : c32;
}

template <typename T>
hipError_t dalloc_n(T **p, int64_t n) {
    *p = nullptr;
    return hipMalloc((void **)p, sizeof(T) * (size_t)(n > 0 ? n : 1));
}

// scratch in the context, grown on demand
hipError_t dec_reserve(vt_ctx *c, int64_t n_tasks, int64_t n_hist) {
    if (n_tasks > c->cap_dec_tasks) {
        if (c->dec_cnt) hipFree(c->dec_cnt);
        if (c->dec_base) hipFree(c->dec_base);
        if (c->dec_thick) hipFree(c->dec_thick);
        if (c->dec_tpos) hipFree(c->dec_tpos);
        c->dec_cnt = nullptr;
        c->dec_base = nullptr;
        c->dec_thick = nullptr;
        c->dec_tpos = nullptr;
        c->cap_dec_tasks = 0;
        hipError_t e = dalloc_n(&c->dec_cnt, 2 * n_tasks);
        if (e == hipSuccess) e = dalloc_n(&c->dec_base, 2 * n_tasks);
        if (e == hipSuccess) e = dalloc_n(&c->dec_thick, 6 * n_tasks);
        if (e == hipSuccess) e = dalloc_n(&c->dec_tpos, n_tasks);
        if (e != hipSuccess) return e;
        c->cap_dec_tasks = n_tasks;
    }
    if (n_hist > c->cap_dec_hist) {
        if (c->dec_hist) hipFree(c->dec_hist);
        c->dec_hist = nullptr;
        c->cap_dec_hist = 0;
        hipError_t e = dalloc_n(&c->dec_hist, n_hist);
        if (e != hipSuccess) return e;
        c->cap_dec_hist = n_hist;
    }
    if (!c->dec_thr) {
        hipError_t e = dalloc_n(&c->dec_thr, 64);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

vt_status dec_err(hipError_t e) { return e == hipErrorOutOfMemory ? VT_ERR_OOM : VT_ERR_HIP; }

bool dec_geometry(const double lo[3], const double hi[3], const int32_t nt[3], DecGeo &g) {
    for (int a = 0; a < 3; ++a) {
        if (!(hi[a] > lo[a]) || nt[a] < 1 || nt[a] > 1024) return false;
        g.lo[a] = lo[a];
        g.L[a] = hi[a] - lo[a];
        g.nt[a] = nt[a];
        g.w[a] = g.L[a] / nt[a];
        // the buffered task must span less than one period
        g.tmax[a] = (nt[a] >= 2 ? 0.5 * (g.L[a] - g.w[a]) : 0.5 * g.L[a]) * (1.0 - 1e-12);
    }
    return true;
}

vt_ctx *dec_context(vt_ctx **pctx, void *stream) {
    vt_ctx *c = *pctx;
    if (!c) {
        c = new vt_ctx();
        hipGetDevice(&c->device);
        *pctx = c;
    }
    (void)stream;
    return c;
}

template <typename T>
vt_status dec_count(vt_ctx *c, const T *pos, int64_t n, const DecGeo &g, const double *h_thick, int64_t n_tasks,
                    const uint8_t *own_mask, const int32_t *d_tpos, int64_t n_list, std::vector<int64_t> &cnt,
                    hipStream_t s) {
    double Tm[3] = {0.0, 0.0, 0.0};
    for (int64_t b = 0; b < n_tasks; ++b)
        for (int a = 0; a < 3; ++a) Tm[a] = std::max(Tm[a], std::max(h_thick[6 * b + 2 * a], h_thick[6 * b + 2 * a + 1]));
    hipError_t e = hipMemcpyAsync(c->dec_thick, h_thick, sizeof(double) * 6 * n_tasks, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return dec_err(e);
    e = vt_launch_zero_u32((uint32_t *)c->dec_cnt, 4 * n_list, s);
    if (e != hipSuccess) return dec_err(e);
    const int nc = (int)(2 * n_list);
    k_dec_count<T><<<(n + DEC_TPB - 1) / DEC_TPB, DEC_TPB, dec_lds_bytes(nc, false), s>>>(
        pos, n, g, c->dec_thick, Tm[0], Tm[1], Tm[2], own_mask, d_tpos, nc, (unsigned long long *)c->dec_cnt);
    e = hipGetLastError();
    if (e != hipSuccess) return dec_err(e);
    cnt.assign(2 * n_list, 0);
    e = hipMemcpyAsync(cnt.data(), c->dec_cnt, sizeof(int64_t) * 2 * n_list, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? VT_OK : dec_err(e);
}

template <typename T>
vt_status decompose(vt_ctx *c, const T *pos, int64_t n, const DecGeo &g, const double *thr, int n_thr, double *thick,
                    int64_t *n_owned, int64_t *n_ghost, hipStream_t s) {
    const int64_t n_tasks = (int64_t)g.nt[0] * g.nt[1] * g.nt[2];
    const int64_t n_hist = n_tasks * 6 * n_thr;
    hipError_t e = dec_reserve(c, n_tasks, n_hist);
    if (e != hipSuccess) return dec_err(e);
    e = hipMemcpyAsync(c->dec_thr, thr, sizeof(double) * n_thr, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = vt_launch_zero_u32(c->dec_hist, n_hist, s);
    if (e != hipSuccess) return dec_err(e);
    const int tpb = 256;
    k_dec_slab<T><<<(n + tpb - 1) / tpb, tpb, 0, s>>>(pos, n, g, c->dec_thr, n_thr, c->dec_hist);
    e = hipGetLastError();
    if (e != hipSuccess) return dec_err(e);
    std::vector<uint32_t> hist(n_hist);
    e = hipMemcpyAsync(hist.data(), c->dec_hist, sizeof(uint32_t) * n_hist, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return dec_err(e);
    // thickness: the first threshold whose slab holds the expected count
    const double vol = g.L[0] * g.L[1] * g.L[2];
    const double nbar = (double)n / vol;
    for (int64_t b = 0; b < n_tasks; ++b)
        for (int f = 0; f < 6; ++f) {
            const int a = f >> 1;
            const double area = g.w[(a + 1) % 3] * g.w[(a + 2) % 3];
            const double expect = nbar * area * thr[0];
            double t = thr[n_thr - 1];
            uint64_t cum = 0;
            for (int k = 0; k < n_thr; ++k) {
                cum += hist[(b * 6 + f) * n_thr + k];
                if ((double)cum >= expect) {
                    t = thr[k];
                    break;
                }
            }
            thick[6 * b + f] = std::min(t, g.tmax[a]);
        }
    std::vector<int64_t> cnt;
    vt_status st = dec_count(c, pos, n, g, thick, n_tasks, nullptr, nullptr, n_tasks, cnt, s);
    if (st != VT_OK) return st;
    for (int64_t b = 0; b < n_tasks; ++b) {
        if (n_owned) n_owned[b] = cnt[2 * b];
        if (n_ghost) n_ghost[b] = cnt[2 * b + 1];
    }
    return VT_OK;
}

template <typename T>
vt_status decompose_pack(vt_ctx *c, const T *pos, int64_t n, const DecGeo &g, const double *thick,
                         const uint8_t *own_mask, const int32_t *tasks, int32_t n_list, double *out_pos,
                         int32_t *out_gid, int64_t cap, vt_item *items, int64_t *n_out, hipStream_t s) {
    const int64_t n_tasks = (int64_t)g.nt[0] * g.nt[1] * g.nt[2];
    hipError_t e = dec_reserve(c, n_tasks, 1);
    if (e != hipSuccess) return dec_err(e);
    // task -> position in the list
    std::vector<int32_t> tpos(n_tasks, -1);
    for (int32_t l = 0; l < n_list; ++l) {
        const int32_t b = tasks ? tasks[l] : l;
        if (b < 0 || b >= n_tasks || tpos[b] >= 0) return VT_ERR_ARG;
        tpos[b] = l;
    }
    e = hipMemcpyAsync(c->dec_tpos, tpos.data(), sizeof(int32_t) * n_tasks, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return dec_err(e);
    std::vector<int64_t> cnt;
    vt_status st = dec_count(c, pos, n, g, thick, n_tasks, own_mask, c->dec_tpos, n_list, cnt, s);
    if (st != VT_OK) return st;
    // offsets: per listed task its owned particles, then its buffer particles
    std::vector<int64_t> base(2 * n_list);
    int64_t off = 0;
    for (int32_t l = 0; l < n_list; ++l) {
        const int32_t b = tasks ? tasks[l] : l;
        if (cnt[2 * l] < 1) return VT_ERR_ARG;
        base[2 * l] = off;
        base[2 * l + 1] = off + cnt[2 * l];
        vt_item &it = items[l];
        it.offset = off;
        it.n_owned = cnt[2 * l];
        it.n_ghost = cnt[2 * l + 1];
        it.periodic = 0;
        it.reserved = 0;
        const int ii[3] = {(int)(b / ((int64_t)g.nt[1] * g.nt[2])), (int)((b / g.nt[2]) % g.nt[1]), (int)(b % g.nt[2])};
        for (int a = 0; a < 3; ++a) {
            it.lo[a] = g.lo[a] + (double)ii[a] * g.w[a] - thick[6 * b + 2 * a];
            it.hi[a] = g.lo[a] + (double)(ii[a] + 1) * g.w[a] + thick[6 * b + 2 * a + 1];
        }
        off += cnt[2 * l] + cnt[2 * l + 1];
    }
    *n_out = off;
    if (off > cap) return VT_ERR_CAPACITY;
    e = hipMemcpyAsync(c->dec_base, base.data(), sizeof(int64_t) * 2 * n_list, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = vt_launch_zero_u32((uint32_t *)c->dec_cnt, 4 * n_list, s);
    if (e != hipSuccess) return dec_err(e);
    double Tm[3] = {0.0, 0.0, 0.0};
    for (int64_t b = 0; b < n_tasks; ++b)
        for (int a = 0; a < 3; ++a) Tm[a] = std::max(Tm[a], std::max(thick[6 * b + 2 * a], thick[6 * b + 2 * a + 1]));
    const int nc = 2 * n_list;
    k_dec_scatter<T><<<(n + DEC_TPB - 1) / DEC_TPB, DEC_TPB, dec_lds_bytes(nc, true), s>>>(
        pos, n, g, c->dec_thick, Tm[0], Tm[1], Tm[2], own_mask, c->dec_tpos, nc, c->dec_base,
        (unsigned long long *)c->dec_cnt, off, out_pos, out_gid);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? VT_OK : dec_err(e);
}

}  // namespace

void vt_dec_free(vt_ctx *c) {
    if (c->dec_hist) hipFree(c->dec_hist);
    if (c->dec_cnt) hipFree(c->dec_cnt);
    if (c->dec_base) hipFree(c->dec_base);
    if (c->dec_thick) hipFree(c->dec_thick);
    if (c->dec_tpos) hipFree(c->dec_tpos);
    if (c->dec_thr) hipFree(c->dec_thr);
    c->dec_hist = nullptr;
    c->dec_cnt = nullptr;
    c->dec_base = nullptr;
    c->dec_thick = nullptr;
    c->dec_tpos = nullptr;
    c->dec_thr = nullptr;
    c->cap_dec_tasks = c->cap_dec_hist = 0;
}

extern "C" {

vt_status vt_decompose(vt_ctx **pctx, const void *pos, vt_dtype dtype, int64_t n, const double lo[3],
                       const double hi[3], const int32_t nt[3], const double *thresholds, int32_t n_thr,
                       double *thick, int64_t *n_owned, int64_t *n_ghost, void *stream) {
    if (!pctx || !pos || n < 1 || n >= (int64_t)INT32_MAX || !lo || !hi || !nt || !thresholds || !thick)
        return VT_ERR_ARG;
    if (dtype != VT_F32 && dtype != VT_F64) return VT_ERR_ARG;
    if (n_thr < 1 || n_thr > 64) return VT_ERR_ARG;
    for (int k = 0; k < n_thr; ++k)
        if (!(thresholds[k] > 0.0) || (k > 0 && !(thresholds[k] > thresholds[k - 1]))) return VT_ERR_ARG;
    DecGeo g;
    if (!dec_geometry(lo, hi, nt, g)) return VT_ERR_ARG;
    (void)hipGetLastError();
    vt_ctx *c = dec_context(pctx, stream);
    hipStream_t s = (hipStream_t)stream;
    return dtype == VT_F32 ? decompose<float>(c, (const float *)pos, n, g, thresholds, n_thr, thick, n_owned, n_ghost, s)
                           : decompose<double>(c, (const double *)pos, n, g, thresholds, n_thr, thick, n_owned,
                                               n_ghost, s);
}

vt_status vt_decompose_pack(vt_ctx **pctx, const void *pos, vt_dtype dtype, int64_t n, const double lo[3],
                            const double hi[3], const int32_t nt[3], const double *thick, const uint8_t *own_mask,
                            const int32_t *tasks, int32_t n_list, double *out_pos, int32_t *out_gid, int64_t cap,
                            vt_item *items, int64_t *n_out, void *stream) {
    if (!pctx || !pos || n < 1 || n >= (int64_t)INT32_MAX || !lo || !hi || !nt || !thick || !items || !n_out)
        return VT_ERR_ARG;
    if (dtype != VT_F32 && dtype != VT_F64) return VT_ERR_ARG;
    if (cap < 0 || (cap > 0 && (!out_pos || !out_gid))) return VT_ERR_ARG;
    DecGeo g;
    if (!dec_geometry(lo, hi, nt, g)) return VT_ERR_ARG;
    const int64_t n_tasks = (int64_t)g.nt[0] * g.nt[1] * g.nt[2];
    if (n_list < 1 || (!tasks && n_list != n_tasks) || n_list > n_tasks) return VT_ERR_ARG;
    for (int64_t b = 0; b < n_tasks; ++b)
        for (int f = 0; f < 6; ++f)
            if (!(thick[6 * b + f] >= 0.0) || thick[6 * b + f] > g.tmax[f >> 1]) return VT_ERR_ARG;
    (void)hipGetLastError();
    vt_ctx *c = dec_context(pctx, stream);
    hipStream_t s = (hipStream_t)stream;
    return dtype == VT_F32 ? decompose_pack<float>(c, (const float *)pos, n, g, thick, own_mask, tasks, n_list, out_pos,
                                                   out_gid, cap, items, n_out, s)
                           : decompose_pack<double>(c, (const double *)pos, n, g, thick, own_mask, tasks, n_list,
                                                    out_pos, out_gid, cap, items, n_out, s);
}

}  // extern "C"

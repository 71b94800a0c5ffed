// decomp.hip -- domain decomposition with AUTOBORDER buffer zones (paper
// section 2: sub-volumes with buffer particles; the buffer starts at
// BORDERFACTOR times the mean inter-particle distance and grows where the
// particle density in it is below the mean; section 2 also gives the two task
// layouts, power-of-two near-cubes and slabs for elongated survey volumes).  The
// tasks of a periodic box or of a bounded world become the items of one
// batched build; vt_decomposed_build runs the whole procedure, re-running
// the cells that a pass leaves incomplete with wider buffers.
//
// Ownership is by integer cell index, so the tasks partition the particles.
// For the thicknesses, every particle adds itself to a histogram per face over
// the thresholds: beyond the +a face of the task j steps below it along axis a
// at distance u_a + (j - 1) w_a, and beyond the -a face of the task j steps
// above at distance (w_a - u_a) + (j - 1) w_a, u the particle's offset in its
// own task (periodic worlds wrap j around, bounded ones stop at the world's
// faces).  The buffer particles of a task are the particle images x + s L
// (s in {-1, 0, 1}^3; s = 0 only in a bounded world) inside its buffered box
// that it does not own; the buffered box spans less than one period per axis,
// so each particle has at most one image there.
#include <math.h>

#include <algorithm>
#include <vector>

#include "vt_internal.h"

namespace {

struct DecGeo {
    double lo[3], hi[3], L[3], w[3], tmax[3];
    int nt[3];
    int periodic;
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

// lower and upper coordinate of the task cell j along axis a (the last cell ends at the world's face)
__host__ __device__ __forceinline__ double dec_cell_lo(const DecGeo &g, int a, int j) {
    return g.lo[a] + (double)j * g.w[a];
}
__host__ __device__ __forceinline__ double dec_cell_hi(const DecGeo &g, int a, int j) {
    return j + 1 >= g.nt[a] ? g.hi[a] : g.lo[a] + (double)(j + 1) * g.w[a];
}

// largest thickness of face f of the task with cell index j along f's axis
double dec_face_cap(const DecGeo &g, int j, int f) {
    const int a = f >> 1;
    if (g.periodic) return g.tmax[a];
    // bounded: the distance from the face to the world's face beyond it
    return (f & 1) ? g.hi[a] - dec_cell_hi(g, a, j) : dec_cell_lo(g, a, j) - g.lo[a];
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
            for (int j = 1; j < (g.periodic ? 1 << 30 : g.nt[a]); ++j) {
                const double d = d0 + (double)(j - 1) * g.w[a];
                if (d >= g.tmax[a]) break;
                const int k = dec_bin(thr, n_thr, d);
                if (k >= n_thr) break;
                int ii[3] = {i[0], i[1], i[2]};
                const int s = side ? -j : j;
                if (g.periodic) {
                    ii[a] = ((i[a] + s) % g.nt[a] + g.nt[a]) % g.nt[a];
                } else {
                    ii[a] = i[a] + s;
                    if (ii[a] < 0 || ii[a] >= g.nt[a]) break;
                }
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
            if (s != 0 && !g.periodic) continue;
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
                                double blo = dec_cell_lo(g, a, jj[a]) - thick[6 * b + 2 * a];
                                double bhi = dec_cell_hi(g, a, jj[a]) + thick[6 * b + 2 * a + 1];
                                if (g.periodic) {
                                    in = y >= blo && y < bhi;
                                } else {
                                    // a bounded world is closed: its own upper face belongs to it
                                    blo = fmax(blo, g.lo[a]);
                                    bhi = fmin(bhi, g.hi[a]);
                                    in = y >= blo && (y < bhi || (bhi >= g.hi[a] && y <= bhi));
                                }
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

bool dec_geometry(const double lo[3], const double hi[3], int32_t periodic, const int32_t nt[3], DecGeo &g) {
    g.periodic = periodic ? 1 : 0;
    for (int a = 0; a < 3; ++a) {
        if (!(hi[a] > lo[a]) || nt[a] < 1 || nt[a] > 1024) return false;
        g.lo[a] = lo[a];
        g.hi[a] = hi[a];
        g.L[a] = hi[a] - lo[a];
        g.nt[a] = nt[a];
        g.w[a] = g.L[a] / nt[a];
        // periodic: the buffered task must span less than one period; bounded: the per-face caps
        // (dec_face_cap) are below L, which bounds the histogram's distances
        g.tmax[a] = periodic ? (nt[a] >= 2 ? 0.5 * (g.L[a] - g.w[a]) : 0.5 * g.L[a]) * (1.0 - 1e-12) : g.L[a];
    }
    return true;
}

// defaults of the zero fields; false if a field is out of range
bool border_params(const vt_border *in, vt_border &b) {
    b = vt_border{};
    if (in) b = *in;
    if (b.border_factor == 0.0) b.border_factor = 1.5;
    if (b.growth == 0.0) b.growth = 1.1;
    if (b.n_steps == 0) b.n_steps = 48;
    if (b.max_reruns == 0) b.max_reruns = 3;
    if (b.widen == 0.0) b.widen = 2.0;
    return b.border_factor > 0.0 && b.growth > 1.0 && b.n_steps >= 1 && b.n_steps <= 64 && b.max_reruns >= 0 &&
           b.max_reruns < VT_DEC_MAX_PASSES && b.widen >= 1.0 && std::isfinite(b.border_factor) &&
           std::isfinite(b.growth) && std::isfinite(b.widen);
}

// t_k = border_factor * s * growth^k with s = (V / n)^(1/3), the mean inter-particle distance computed from
// the whole input (section 2)
void border_thresholds(int64_t n, const double L[3], const vt_border &b, double *out) {
    const double s = cbrt(L[0] * L[1] * L[2] / (double)n);
    for (int k = 0; k < b.n_steps; ++k) out[k] = b.border_factor * s * pow(b.growth, (double)k);
}

vt_ctx *dec_context(vt_ctx **pctx) {
    vt_ctx *c = *pctx;
    if (!c) {
        c = new vt_ctx();
        hipGetDevice(&c->device);
        *pctx = c;
    }
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
vt_status decompose(vt_ctx *c, const T *pos, int64_t n, const DecGeo &g, const vt_border &bp, double *thick,
                    int64_t *n_owned, int64_t *n_ghost, hipStream_t s) {
    const int64_t n_tasks = (int64_t)g.nt[0] * g.nt[1] * g.nt[2];
    const int n_thr = bp.n_steps;
    std::vector<double> thr(n_thr);
    border_thresholds(n, g.L, bp, thr.data());
    const int64_t n_hist = n_tasks * 6 * n_thr;
    hipError_t e = dec_reserve(c, n_tasks, n_hist);
    if (e != hipSuccess) return dec_err(e);
    e = hipMemcpyAsync(c->dec_thr, thr.data(), sizeof(double) * n_thr, hipMemcpyHostToDevice, s);
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
    // thickness: the first threshold whose slab holds the expected count, then the face's cap
    const double nbar = (double)n / (g.L[0] * g.L[1] * g.L[2]);
    for (int64_t b = 0; b < n_tasks; ++b) {
        const int ii[3] = {(int)(b / ((int64_t)g.nt[1] * g.nt[2])), (int)((b / g.nt[2]) % g.nt[1]), (int)(b % g.nt[2])};
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
            thick[6 * b + f] = std::min(t, dec_face_cap(g, ii[a], f));
        }
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
        it.walls = 0;
        const int ii[3] = {(int)(b / ((int64_t)g.nt[1] * g.nt[2])), (int)((b / g.nt[2]) % g.nt[1]), (int)(b % g.nt[2])};
        for (int a = 0; a < 3; ++a) {
            it.lo[a] = dec_cell_lo(g, a, ii[a]) - thick[6 * b + 2 * a];
            it.hi[a] = dec_cell_hi(g, a, ii[a]) + thick[6 * b + 2 * a + 1];
            if (!g.periodic) {
                // a buffered box that reaches the world's face stops there: that wall is a true boundary
                if (it.lo[a] <= g.lo[a]) {
                    it.lo[a] = g.lo[a];
                    it.walls |= 1 << (2 * a);
                }
                if (it.hi[a] >= g.hi[a]) {
                    it.hi[a] = g.hi[a];
                    it.walls |= 1 << (2 * a + 1);
                }
            }
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

// ---------------------------------------------------------------- whole decomposed build

// one pass's cell outputs (rows in item order) into particle order: particle p = gid of the row's
// batch entry; cells left incomplete mark their particle (owned alone next pass) and its task
__global__ void k_dres_rows(const int64_t *pitems, int n_list, const int32_t *gid, const double *vol,
                            const uint8_t *stat, int64_t n_rows, int pass, DecGeo g, const double *pos64,
                            double *dvol, uint8_t *dstat, int32_t *dlast, int32_t *drow, uint8_t *mask,
                            int32_t *tflag) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rows) return;
    int lo = 0, hi = n_list - 1;  // the item whose rows start at or before r
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pitems[3 * mid] <= r) lo = mid; else hi = mid - 1;
    }
    const int64_t k = r - pitems[3 * lo];
    const int64_t q = pitems[3 * lo + 1] + k;  // batch entry (an owned particle of item lo)
    const int32_t p = gid[q];
    const uint8_t st = stat[r];
    dvol[p] = vol[r];
    dstat[p] = st;
    dlast[p] = pass;
    drow[p] = (int32_t)r;
    if (st & VT_CELL_INCOMPLETE) {
        mask[p] = 1;
        double x[3], u[3];
        int i[3];
        dec_pos(pos64, q, x);  // the owned entry of the batch is the particle itself
        dec_owner(g, x, i, u);
        tflag[dec_task(g, i[0], i[1], i[2])] = 1;
    }
}

struct PassCsr {
    const int64_t *off[VT_DEC_MAX_PASSES];
    const int32_t *ids[VT_DEC_MAX_PASSES];
};

__global__ void k_dres_count(const int32_t *dlast, const int32_t *drow, int64_t n, PassCsr pc, int64_t *cnt) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int k = dlast[p];
    const int64_t r = drow[p];
    cnt[p] = (k >= 0) ? pc.off[k][r + 1] - pc.off[k][r] : 0;
}

// 16 lanes per particle copy its neighbour row from the pass that computed it
__global__ void k_dres_fill(const int32_t *dlast, const int32_t *drow, int64_t n, PassCsr pc, const int64_t *off,
                            int32_t *ids) {
    const int64_t p = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 16;
    if (p >= n) return;
    const int sub = threadIdx.x & 15;
    const int k = dlast[p];
    if (k < 0) return;
    const int64_t r = drow[p];
    const int64_t src = pc.off[k][r], len = pc.off[k][r + 1] - src, dst = off[p];
    for (int64_t i = sub; i < len; i += 16) ids[dst + i] = pc.ids[k][src + i];
}

template <typename MT>
__global__ void k_dres_density(const MT *mass, const double *vol, int64_t n, double *rho) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) rho[p] = (mass ? (double)mass[p] : 1.0) / vol[p];
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_u8(uint8_t *p, int64_t n, uint8_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

template <typename T>
hipError_t grow(T **p, int64_t &cap, int64_t need) {
    if (need <= cap && *p) return hipSuccess;
    if (*p) hipFree(*p);
    *p = nullptr;
    cap = 0;
    hipError_t e = dalloc_n(p, need);
    if (e == hipSuccess) cap = need;
    return e;
}

#define DTRY(x)                                   \
    do {                                          \
        hipError_t e_ = (x);                      \
        if (e_ != hipSuccess) return dec_err(e_); \
    } while (0)

template <typename T>
vt_status decomposed_build(vt_ctx *c, const T *pos, int64_t n, const DecGeo &g, const vt_border &bp,
                           const vt_opts *opts, double *thick_out, int64_t *pass_stats, int32_t *n_passes,
                           hipStream_t s) {
    const int64_t n_tasks = (int64_t)g.nt[0] * g.nt[1] * g.nt[2];
    c->built = false;
    c->decomposed = false;
    c->stream = s;
    std::vector<double> thick(6 * n_tasks);
    vt_status st = decompose<T>(c, pos, n, g, bp, thick.data(), nullptr, nullptr, s);
    if (st != VT_OK) return st;
    if (thick_out) std::copy(thick.begin(), thick.end(), thick_out);
    // per-particle results
    int64_t cap_n = c->cap_dres, cap_t = c->cap_dres_tasks;
    if (n > cap_n || !c->dres_vol) {
        if (c->dres_vol) hipFree(c->dres_vol);
        if (c->dres_stat) hipFree(c->dres_stat);
        if (c->dres_off) hipFree(c->dres_off);
        if (c->dres_last) hipFree(c->dres_last);
        if (c->dres_row) hipFree(c->dres_row);
        if (c->dres_mask) hipFree(c->dres_mask);
        if (c->dres_cnt) hipFree(c->dres_cnt);
        if (c->dres_scan) hipFree(c->dres_scan);
        c->dres_vol = nullptr, c->dres_stat = nullptr, c->dres_off = nullptr, c->dres_last = nullptr;
        c->dres_row = nullptr, c->dres_mask = nullptr, c->dres_cnt = nullptr, c->dres_scan = nullptr;
        c->cap_dres = 0;
        DTRY(dalloc_n(&c->dres_vol, n));
        DTRY(dalloc_n(&c->dres_stat, n));
        DTRY(dalloc_n(&c->dres_off, n + 1));
        DTRY(dalloc_n(&c->dres_last, n));
        DTRY(dalloc_n(&c->dres_row, n));
        DTRY(dalloc_n(&c->dres_mask, n));
        DTRY(dalloc_n(&c->dres_cnt, n));
        DTRY(dalloc_n(&c->dres_scan, vt_scan_tmp_elems(n + 1) + 1));
        c->cap_dres = n;
    }
    (void)cap_n;
    DTRY(grow(&c->dres_tflag, cap_t, n_tasks));
    c->cap_dres_tasks = cap_t;
    const int tpb = 256;
    const int64_t gb = (n + tpb - 1) / tpb;
    k_fill_i32<<<gb, tpb, 0, s>>>(c->dres_last, n, -1);
    k_fill_u8<<<gb, tpb, 0, s>>>(c->dres_stat, n, (uint8_t)VT_CELL_FAILED);
    DTRY(hipGetLastError());

    vt_opts o{};
    if (opts) o = *opts;
    o.want_faces = 0;
    o.timing = 0;
    std::vector<double> cur = thick;
    std::vector<int32_t> tasks;  // empty: every task
    const uint8_t *mask = nullptr;
    std::vector<vt_item> items;
    int pass = 0;
    int64_t left = 0;
    for (;; ++pass) {
        const int32_t n_list = tasks.empty() ? (int32_t)n_tasks : (int32_t)tasks.size();
        items.assign(n_list, vt_item{});
        int64_t n_out = 0;
        st = decompose_pack<T>(c, pos, n, g, cur.data(), mask, tasks.empty() ? nullptr : tasks.data(), n_list,
                               c->dpack_pos, c->dpack_gid, c->cap_dpack, items.data(), &n_out, s);
        if (st == VT_ERR_CAPACITY) {
            int64_t cp = c->cap_dpack, cg = c->cap_dpack;
            DTRY(grow(&c->dpack_pos, cp, 3 * n_out));
            DTRY(grow(&c->dpack_gid, cg, n_out));
            c->cap_dpack = n_out;
            st = decompose_pack<T>(c, pos, n, g, cur.data(), mask, tasks.empty() ? nullptr : tasks.data(), n_list,
                                   c->dpack_pos, c->dpack_gid, c->cap_dpack, items.data(), &n_out, s);
        }
        if (st != VT_OK) return st;
        st = vt_build(&c->dchild, c->dpack_pos, VT_F64, c->dpack_gid, items.data(), n_list, &o, (void *)s);
        if (st != VT_OK) return st;
        int64_t nnz = 0, retried = 0, inc = 0;
        st = vt_query(c->dchild, &nnz, &retried, &inc);
        if (st != VT_OK) return st;
        int64_t rows = 0;
        std::vector<int64_t> pit(3 * n_list);
        for (int32_t l = 0; l < n_list; ++l) {
            pit[3 * l] = rows;
            pit[3 * l + 1] = items[l].offset;
            pit[3 * l + 2] = items[l].n_owned;
            rows += items[l].n_owned;
        }
        DTRY(grow(&c->dpack_items, c->cap_dpack_items, 3 * (int64_t)n_list));
        int64_t cr = c->cap_dpass_rows;
        DTRY(grow(&c->dpass_vol, cr, rows));
        int64_t cr2 = c->cap_dpass_rows;
        DTRY(grow(&c->dpass_stat, cr2, rows));
        c->cap_dpass_rows = std::min(cr, cr2);
        DTRY(grow(&c->dpass_off[pass], c->dpass_cap_rows[pass], rows + 1));
        DTRY(grow(&c->dpass_ids[pass], c->dpass_cap_ids[pass], nnz));
        DTRY(hipMemcpyAsync(c->dpack_items, pit.data(), sizeof(int64_t) * 3 * n_list, hipMemcpyHostToDevice, s));
        st = vt_cells(c->dchild, c->dpass_vol, c->dpass_off[pass], c->dpass_ids[pass], nnz, c->dpass_stat, (void *)s);
        if (st != VT_OK) return st;
        k_fill_i32<<<(n_tasks + tpb - 1) / tpb, tpb, 0, s>>>(c->dres_tflag, n_tasks, 0);
        k_fill_u8<<<gb, tpb, 0, s>>>(c->dres_mask, n, 0);
        k_dres_rows<<<(rows + tpb - 1) / tpb, tpb, 0, s>>>(c->dpack_items, n_list, c->dpack_gid, c->dpass_vol,
                                                           c->dpass_stat, rows, pass, g, c->dpack_pos, c->dres_vol,
                                                           c->dres_stat, c->dres_last, c->dres_row, c->dres_mask,
                                                           c->dres_tflag);
        DTRY(hipGetLastError());
        if (pass_stats) {
            pass_stats[4 * pass + 0] = n_list;
            pass_stats[4 * pass + 1] = n_out;
            pass_stats[4 * pass + 2] = rows;
            pass_stats[4 * pass + 3] = inc;
        }
        c->dres_retried = retried;
        left = inc;
        if (inc == 0 || pass >= bp.max_reruns) break;
        // the tasks that own an incomplete cell, with their buffers widened (up to the caps)
        std::vector<int32_t> tf(n_tasks);
        DTRY(hipMemcpyAsync(tf.data(), c->dres_tflag, sizeof(int32_t) * n_tasks, hipMemcpyDeviceToHost, s));
        DTRY(hipStreamSynchronize(s));
        tasks.clear();
        for (int64_t b = 0; b < n_tasks; ++b)
            if (tf[b]) {
                tasks.push_back((int32_t)b);
                const int ii[3] = {(int)(b / ((int64_t)g.nt[1] * g.nt[2])), (int)((b / g.nt[2]) % g.nt[1]),
                                   (int)(b % g.nt[2])};
                for (int f = 0; f < 6; ++f)
                    cur[6 * b + f] = std::min(cur[6 * b + f] * bp.widen, dec_face_cap(g, ii[f >> 1], f));
            }
        mask = c->dres_mask;
    }
    // neighbour rows in particle order, each from the last pass that computed the cell
    PassCsr pc{};
    for (int k = 0; k <= pass; ++k) {
        pc.off[k] = c->dpass_off[k];
        pc.ids[k] = c->dpass_ids[k];
    }
    k_dres_count<<<gb, tpb, 0, s>>>(c->dres_last, c->dres_row, n, pc, c->dres_cnt);
    DTRY(hipGetLastError());
    DTRY(vt_launch_scan_i64(c->dres_cnt, c->dres_off, n, c->dres_scan, s));
    int64_t nnz = 0;
    DTRY(hipMemcpyAsync(&nnz, c->dres_off + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    DTRY(hipStreamSynchronize(s));
    int64_t ci = c->cap_dres_ids;
    DTRY(grow(&c->dres_ids, ci, nnz));
    c->cap_dres_ids = ci;
    k_dres_fill<<<(n * 16 + tpb - 1) / tpb, tpb, 0, s>>>(c->dres_last, c->dres_row, n, pc, c->dres_off, c->dres_ids);
    DTRY(hipGetLastError());
    DTRY(hipStreamSynchronize(s));
    c->dres_n = n;
    c->dres_nnz = nnz;
    c->dres_incomplete = left;
    c->dres_status = VT_OK;
    c->dres_capfail = false;
    c->decomposed = true;
    if (n_passes) *n_passes = pass + 1;
    return VT_OK;
}

}  // namespace

void vt_dec_free(vt_ctx *c) {
    auto f = [](auto *&p) {
        if (p) hipFree((void *)p);
        p = nullptr;
    };
    f(c->dec_hist);
    f(c->dec_cnt);
    f(c->dec_base);
    f(c->dec_thick);
    f(c->dec_tpos);
    f(c->dec_thr);
    c->cap_dec_tasks = c->cap_dec_hist = 0;
    f(c->dres_vol);
    f(c->dres_stat);
    f(c->dres_off);
    f(c->dres_ids);
    f(c->dres_last);
    f(c->dres_row);
    f(c->dres_mask);
    f(c->dres_tflag);
    f(c->dres_cnt);
    f(c->dres_scan);
    f(c->dpack_pos);
    f(c->dpack_gid);
    f(c->dpack_items);
    f(c->dpass_vol);
    f(c->dpass_stat);
    for (int k = 0; k < VT_DEC_MAX_PASSES; ++k) {
        f(c->dpass_off[k]);
        f(c->dpass_ids[k]);
        c->dpass_cap_rows[k] = c->dpass_cap_ids[k] = 0;
    }
    c->cap_dres = c->cap_dres_ids = c->cap_dres_tasks = c->cap_dpack = c->cap_dpack_items = c->cap_dpass_rows = 0;
    if (c->dchild) vt_destroy(c->dchild);
    c->dchild = nullptr;
    c->decomposed = false;
}

vt_status vt_dres_cells(vt_ctx *c, double *volume, int64_t *nbr_off, int32_t *nbr_ids, int64_t nbr_cap,
                        uint8_t *cell_status) {
    const int64_t n = c->dres_n;
    hipStream_t s = c->stream;
    DTRY(hipMemcpyAsync(volume, c->dres_vol, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    DTRY(hipMemcpyAsync(nbr_off, c->dres_off, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToDevice, s));
    const int64_t k = std::min(nbr_cap, c->dres_nnz);
    if (k > 0) DTRY(hipMemcpyAsync(nbr_ids, c->dres_ids, sizeof(int32_t) * k, hipMemcpyDeviceToDevice, s));
    if (cell_status) DTRY(hipMemcpyAsync(cell_status, c->dres_stat, (size_t)n, hipMemcpyDeviceToDevice, s));
    c->dres_capfail = c->dres_nnz > nbr_cap;
    return VT_OK;
}

vt_status vt_dres_density(vt_ctx *c, const void *mass, vt_dtype dt, double *rho) {
    const int64_t n = c->dres_n;
    const int tpb = 256;
    if (dt == VT_F32)
        k_dres_density<float><<<(n + tpb - 1) / tpb, tpb, 0, c->stream>>>((const float *)mass, c->dres_vol, n, rho);
    else
        k_dres_density<double><<<(n + tpb - 1) / tpb, tpb, 0, c->stream>>>((const double *)mass, c->dres_vol, n, rho);
    DTRY(hipGetLastError());
    return VT_OK;
}

extern "C" {

vt_status vt_task_grid(int32_t n_task, int32_t scheme, int32_t axis, int32_t nt[3]) {
    if (!nt || n_task < 1 || n_task > 1 << 20) return VT_ERR_ARG;
    nt[0] = nt[1] = nt[2] = 1;
    if (scheme == 0) {
        if (n_task & (n_task - 1)) return VT_ERR_ARG;
        for (int a = 0; nt[0] * nt[1] * nt[2] < n_task; a = (a + 1) % 3) nt[a] *= 2;
        return VT_OK;
    }
    if (scheme == 1 && axis >= 0 && axis < 3 && n_task <= 1024) {
        nt[axis] = n_task;
        return VT_OK;
    }
    return VT_ERR_ARG;
}

vt_status vt_border_thresholds(int64_t n, const double lo[3], const double hi[3], const vt_border *border,
                               double *out) {
    vt_border bp;
    if (n < 1 || !lo || !hi || !out || !border_params(border, bp)) return VT_ERR_ARG;
    double L[3];
    for (int a = 0; a < 3; ++a) {
        if (!(hi[a] > lo[a])) return VT_ERR_ARG;
        L[a] = hi[a] - lo[a];
    }
    border_thresholds(n, L, bp, out);
    return VT_OK;
}

vt_status vt_decompose(vt_ctx **pctx, const void *pos, vt_dtype dtype, int64_t n, const double lo[3],
                       const double hi[3], int32_t periodic, const int32_t nt[3], const vt_border *border,
                       double *thick, int64_t *n_owned, int64_t *n_ghost, void *stream) {
    if (!pctx || !pos || n < 1 || n >= (int64_t)INT32_MAX || !lo || !hi || !nt || !thick) return VT_ERR_ARG;
    if (dtype != VT_F32 && dtype != VT_F64) return VT_ERR_ARG;
    vt_border bp;
    if (!border_params(border, bp)) return VT_ERR_ARG;
    DecGeo g;
    if (!dec_geometry(lo, hi, periodic, nt, g)) return VT_ERR_ARG;
    (void)hipGetLastError();
    vt_ctx *c = dec_context(pctx);
    hipStream_t s = (hipStream_t)stream;
    return dtype == VT_F32 ? decompose<float>(c, (const float *)pos, n, g, bp, thick, n_owned, n_ghost, s)
                           : decompose<double>(c, (const double *)pos, n, g, bp, thick, n_owned, n_ghost, s);
}

vt_status vt_decompose_pack(vt_ctx **pctx, const void *pos, vt_dtype dtype, int64_t n, const double lo[3],
                            const double hi[3], int32_t periodic, const int32_t nt[3], const double *thick,
                            const uint8_t *own_mask, const int32_t *tasks, int32_t n_list, double *out_pos,
                            int32_t *out_gid, int64_t cap, vt_item *items, int64_t *n_out, void *stream) {
    if (!pctx || !pos || n < 1 || n >= (int64_t)INT32_MAX || !lo || !hi || !nt || !thick || !items || !n_out)
        return VT_ERR_ARG;
    if (dtype != VT_F32 && dtype != VT_F64) return VT_ERR_ARG;
    if (cap < 0 || (cap > 0 && (!out_pos || !out_gid))) return VT_ERR_ARG;
    DecGeo g;
    if (!dec_geometry(lo, hi, periodic, nt, g)) return VT_ERR_ARG;
    const int64_t n_tasks = (int64_t)g.nt[0] * g.nt[1] * g.nt[2];
    if (n_list < 1 || (!tasks && n_list != n_tasks) || n_list > n_tasks) return VT_ERR_ARG;
    for (int64_t b = 0; b < n_tasks; ++b) {
        const int ii[3] = {(int)(b / ((int64_t)g.nt[1] * g.nt[2])), (int)((b / g.nt[2]) % g.nt[1]), (int)(b % g.nt[2])};
        for (int f = 0; f < 6; ++f)
            if (!(thick[6 * b + f] >= 0.0) || thick[6 * b + f] > dec_face_cap(g, ii[f >> 1], f)) return VT_ERR_ARG;
    }
    (void)hipGetLastError();
    vt_ctx *c = dec_context(pctx);
    hipStream_t s = (hipStream_t)stream;
    return dtype == VT_F32 ? decompose_pack<float>(c, (const float *)pos, n, g, thick, own_mask, tasks, n_list, out_pos,
                                                   out_gid, cap, items, n_out, s)
                           : decompose_pack<double>(c, (const double *)pos, n, g, thick, own_mask, tasks, n_list,
                                                    out_pos, out_gid, cap, items, n_out, s);
}

vt_status vt_decomposed_build(vt_ctx **pctx, const void *pos, vt_dtype dtype, int64_t n, const double lo[3],
                              const double hi[3], int32_t periodic, const int32_t nt[3], const vt_border *border,
                              const vt_opts *opts, double *thick, int64_t *pass_stats, int32_t *n_passes,
                              void *stream) {
    if (!pctx || !pos || n < 1 || n >= (int64_t)INT32_MAX || !lo || !hi || !nt) return VT_ERR_ARG;
    if (dtype != VT_F32 && dtype != VT_F64) return VT_ERR_ARG;
    if (opts && opts->precision != VT_PREC_FP64 && opts->precision != VT_PREC_MIXED) return VT_ERR_ARG;
    vt_border bp;
    if (!border_params(border, bp)) return VT_ERR_ARG;
    DecGeo g;
    if (!dec_geometry(lo, hi, periodic, nt, g)) return VT_ERR_ARG;
    (void)hipGetLastError();
    vt_ctx *c = dec_context(pctx);
    hipStream_t s = (hipStream_t)stream;
    return dtype == VT_F32 ? decomposed_build<float>(c, (const float *)pos, n, g, bp, opts, thick, pass_stats,
                                                     n_passes, s)
                           : decomposed_build<double>(c, (const double *)pos, n, g, bp, opts, thick, pass_stats,
                                                      n_passes, s);
}

}  // extern "C"

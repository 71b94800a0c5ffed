// post.hip -- per-particle outputs from the clipped cells.
//
// Cells are computed in Morton order into fixed-stride staging rows; these
// kernels produce the caller's input-order arrays (section 2, gather
// paragraph: outputs follow the input order, neighbour ids are real ids):
// the neighbour CSR, volumes, densities m/V, least-squares density gradients
// and the volume adjoint.
#include "vt_internal.h"

__global__ void k_row_counts(const int32_t *row2cell, const int32_t *ccnt, int64_t n, int64_t *cnt) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) cnt[r] = ccnt[row2cell[r]];
}

// a group of 16 lanes per output row: the row's staging slots are read, and its CSR entries
// written, contiguously
__global__ void k_fill(const int32_t *row2cell, const int64_t *crow, const int32_t *ccnt, const double *cvol,
                       const uint8_t *cstat, const int32_t *stage_ids, const int32_t *sgid, const int64_t *off,
                       int64_t n, double *volume, int32_t *nbr_ids, int64_t cap, uint8_t *status, uint32_t *counters) {
    const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 16;
    if (r >= n) return;
    const int sub = threadIdx.x & 15;
    const int32_t c = row2cell[r];
    const int64_t o = off[r], src = crow[c];
    int32_t k = ccnt[c];
    if (sub == 0) {
        volume[r] = cvol[c];
        if (status) status[r] = cstat[c];
    }
    if (o + k > cap) {
        if (sub == 0) atomicOr(&counters[CTR_STATUS], VT_DEV_NBR_CAP);
        k = o >= cap ? 0 : (int32_t)(cap - o);
    }
    for (int32_t i = sub; i < k; i += 16) nbr_ids[o + i] = sgid[stage_ids[src + i]];
}

hipError_t vt_launch_cells(vt_ctx *c, double *volume, int64_t *nbr_off, int32_t *nbr_ids, int64_t nbr_cap,
                           uint8_t *cell_status) {
    const int64_t n = c->n_owned;
    const int tpb = 256;
    const int64_t g = (n + tpb - 1) / tpb;
    k_row_counts<<<g, tpb, 0, c->stream>>>(c->row2cell, c->ccnt, n, c->rowoff);
    hipError_t e = vt_launch_scan_i64(c->rowoff, nbr_off, n, c->scan_tmp, c->stream);
    if (e != hipSuccess) return e;
    k_fill<<<(n * 16 + tpb - 1) / tpb, tpb, 0, c->stream>>>(c->row2cell, c->crow, c->ccnt, c->cvol, c->cstat, c->stage_ids, c->sgid, nbr_off,
                                     n, volume, nbr_ids, nbr_cap, cell_status, c->counters);
    return hipGetLastError();
}

template <typename MT>
__global__ void k_density(const int32_t *row2cell, const int32_t *cells, const int32_t *sorig, const double *cvol,
                          const MT *mass, int64_t n, double *rho) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    int32_t c = row2cell[r];
    double m = mass ? (double)mass[sorig[cells[c]]] : 1.0;
    rho[r] = m / cvol[c];
}

hipError_t vt_launch_density(vt_ctx *c, const void *mass, vt_dtype dt, double *rho) {
    const int64_t n = c->n_owned;
    const int tpb = 256;
    const int64_t g = (n + tpb - 1) / tpb;
    if (dt == VT_F32)
        k_density<float><<<g, tpb, 0, c->stream>>>(c->row2cell, c->cells, c->sorig, c->cvol, (const float *)mass, n,
                                                   rho);
    else
        k_density<double><<<g, tpb, 0, c->stream>>>(c->row2cell, c->cells, c->sorig, c->cvol, (const double *)mass, n,
                                                    rho);
    return hipGetLastError();
}

__device__ __forceinline__ int find_item_p(const DevItem *items, int n_items, int64_t p) {
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (items[mid].start <= p) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <typename PT4>
__device__ __forceinline__ void sep(const PT4 *spos, int32_t i, int32_t j, const DevItem &it, double &dx, double &dy,
                                    double &dz) {
    PT4 a = spos[i], b = spos[j];
    dx = (double)b.x - (double)a.x;
    dy = (double)b.y - (double)a.y;
    dz = (double)b.z - (double)a.z;
    if (it.periodic) {
        dx -= it.L[0] * rint(dx / it.L[0]);
        dy -= it.L[1] * rint(dy / it.L[1]);
        dz -= it.L[2] * rint(dz / it.L[2]);
    }
}

// grad_i = G^-1 b, G = sum D D^T, b = sum (rho_j - rho_i) D  (least squares over Voronoi neighbours)
// The gradient and the adjoint take a group of 16 lanes per cell, in Morton order: the lanes
// read the cell's facet slots together (one contiguous row; a cell has about 15 facets), and the
// neighbours of consecutive cells lie close together, so their positions and values stay in cache.
constexpr int CG = 16;

__device__ __forceinline__ double group_sum(double v) {
    for (int o = CG / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <typename PT4>
__global__ void __launch_bounds__(256) k_gradient(const int32_t *cells, const int32_t *srow, const int32_t *sorig,
                                                  const int64_t *crow, const int32_t *ccnt, const int32_t *stage_ids,
                                                  const PT4 *spos, const DevItem *items, int n_items,
                                                  const double *rho, int64_t n, double *grad) {
    const int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / CG;
    if (c >= n) return;
    const int lane = threadIdx.x & (CG - 1);
    const int32_t i = cells[c];
    const int32_t r = srow[i];
    const DevItem it = items[find_item_p(items, n_items, i)];  // a copy: read once, not at every use
    const double ri = rho[sorig[i]];
    double g00 = 0, g01 = 0, g02 = 0, g11 = 0, g12 = 0, g22 = 0, b0 = 0, b1 = 0, b2 = 0;
    const int64_t src = crow[c];
    const int32_t k = ccnt[c];
    for (int32_t t = lane; t < k; t += CG) {
        const int32_t j = stage_ids[src + t];
        double dx, dy, dz;
        sep<PT4>(spos, i, j, it, dx, dy, dz);
        const double dr = rho[sorig[j]] - ri;
        g00 += dx * dx;
        g01 += dx * dy;
        g02 += dx * dz;
        g11 += dy * dy;
        g12 += dy * dz;
        g22 += dz * dz;
        b0 += dr * dx;
        b1 += dr * dy;
        b2 += dr * dz;
    }
    g00 = group_sum(g00);
    g01 = group_sum(g01);
    g02 = group_sum(g02);
    g11 = group_sum(g11);
    g12 = group_sum(g12);
    g22 = group_sum(g22);
    b0 = group_sum(b0);
    b1 = group_sum(b1);
    b2 = group_sum(b2);
    if (lane == 0) {
        // symmetric 3x3 solve by the adjugate
        const double a00 = g11 * g22 - g12 * g12, a01 = g02 * g12 - g01 * g22, a02 = g01 * g12 - g02 * g11;
        const double a11 = g00 * g22 - g02 * g02, a12 = g01 * g02 - g00 * g12, a22 = g00 * g11 - g01 * g01;
        const double det = g00 * a00 + g01 * a01 + g02 * a02;
        const double inv = det != 0.0 ? 1.0 / det : 0.0;
        grad[3 * (int64_t)r + 0] = (a00 * b0 + a01 * b1 + a02 * b2) * inv;
        grad[3 * (int64_t)r + 1] = (a01 * b0 + a11 * b1 + a12 * b2) * inv;
        grad[3 * (int64_t)r + 2] = (a02 * b0 + a12 * b1 + a22 * b2) * inv;
    }
}

hipError_t vt_launch_gradient(vt_ctx *c, const double *rho, double *grad) {
    const int64_t n = c->n_owned;
    const int64_t g = (n * CG + 255) / 256;
    if (c->dtype == VT_F32)
        k_gradient<float4><<<g, 256, 0, c->stream>>>(c->cells, c->srow, c->sorig, c->crow, c->ccnt, c->stage_ids,
                                                     (const float4 *)c->spos, c->items, c->n_items, rho, n, grad);
    else
        k_gradient<double4><<<g, 256, 0, c->stream>>>(c->cells, c->srow, c->sorig, c->crow, c->ccnt, c->stage_ids,
                                                      (const double4 *)c->spos, c->items, c->n_items, rho, n, grad);
    return hipGetLastError();
}

// dL/dx_k = sum_j (g_k - g_j) A_kj (c_kj - x_k) / d_kj, c seed-relative
template <typename PT4>
__global__ void __launch_bounds__(256) k_backward(const int32_t *cells, const int32_t *srow, const int64_t *crow,
                                                  const int32_t *ccnt, const int32_t *stage_ids,
                                                  const double *stage_area, const double *stage_cen, const PT4 *spos,
                                                  const DevItem *items, int n_items, const double *g, int64_t n,
                                                  double *out) {
    const int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / CG;
    if (c >= n) return;
    const int lane = threadIdx.x & (CG - 1);
    const int32_t i = cells[c];
    const int32_t r = srow[i];
    const DevItem it = items[find_item_p(items, n_items, i)];  // a copy: read once, not at every use
    const double gk = g[r];
    double ox = 0, oy = 0, oz = 0;
    const int64_t src = crow[c];
    const int32_t k = ccnt[c];
    for (int32_t t = lane; t < k; t += CG) {
        const int64_t f = src + t;
        const int32_t j = stage_ids[f];
        const int32_t rj = srow[j];
        const double gj = rj >= 0 ? g[rj] : 0.0;
        double dx, dy, dz;
        sep<PT4>(spos, i, j, it, dx, dy, dz);
        const double d = sqrt(dx * dx + dy * dy + dz * dz);
        const double w = (gk - gj) * stage_area[f] / d;
        ox += w * stage_cen[3 * f + 0];
        oy += w * stage_cen[3 * f + 1];
        oz += w * stage_cen[3 * f + 2];
    }
    ox = group_sum(ox);
    oy = group_sum(oy);
    oz = group_sum(oz);
    if (lane == 0) {
        out[3 * (int64_t)r + 0] = ox;
        out[3 * (int64_t)r + 1] = oy;
        out[3 * (int64_t)r + 2] = oz;
    }
}

hipError_t vt_launch_backward(vt_ctx *c, const double *g, double *out) {
    const int64_t n = c->n_owned;
    const int64_t gr = (n * CG + 255) / 256;
    if (c->dtype == VT_F32)
        k_backward<float4><<<gr, 256, 0, c->stream>>>(c->cells, c->srow, c->crow, c->ccnt, c->stage_ids,
                                                      c->stage_area, c->stage_cen, (const float4 *)c->spos, c->items,
                                                      c->n_items, g, n, out);
    else
        k_backward<double4><<<gr, 256, 0, c->stream>>>(c->cells, c->srow, c->crow, c->ccnt, c->stage_ids,
                                                       c->stage_area, c->stage_cen, (const double4 *)c->spos,
                                                       c->items, c->n_items, g, n, out);
    return hipGetLastError();
}

__global__ void k_stats(const int32_t *row2cell, const int32_t *cnv, const int32_t *cnp, const int32_t *cnt, int64_t n,
                        int32_t *nv, int32_t *np, int32_t *nt) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    int32_t c = row2cell[r];
    if (nv) nv[r] = cnv[c];
    if (np) np[r] = cnp[c];
    if (nt) nt[r] = cnt[c];
}

hipError_t vt_launch_stats(vt_ctx *c, int32_t *nv, int32_t *np, int32_t *nt) {
    const int64_t n = c->n_owned;
    const int tpb = 256;
    k_stats<<<(n + tpb - 1) / tpb, tpb, 0, c->stream>>>(c->row2cell, c->cnv, c->cnp, c->cnt, n, nv, np, nt);
    return hipGetLastError();
}

// vt_api.cpp -- host side of the C ABI declared in include/vt.h.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "vt_internal.h"

namespace {

template <typename T>
hipError_t dalloc(T **p, int64_t n) {
    *p = nullptr;
    if (n <= 0) n = 1;
    return hipMalloc((void **)p, sizeof(T) * (size_t)n);
}

template <typename T>
void dfree(T *&p) {
    if (p) hipFree((void *)p);
    p = nullptr;
}

void free_all(vt_ctx *c) {
    dfree(c->items);
    if (c->h_items) hipHostFree(c->h_items);
    c->h_items = nullptr;
    if (c->h_counters) hipHostFree(c->h_counters);
    c->h_counters = nullptr;
    for (int k = 0; k < 2; ++k) {
        dfree(c->keys[k]);
        dfree(c->vals[k]);
    }
    dfree(c->hist);
    dfree(c->scan_tmp);
    dfree(c->spos);
    dfree(c->sgid);
    dfree(c->srow);
    dfree(c->sorig);
    dfree(c->tab);
    dfree(c->cells);
    dfree(c->cvol);
    dfree(c->crad);
    dfree(c->ccnt);
    dfree(c->crow);
    dfree(c->cstat);
    dfree(c->cnv);
    dfree(c->cnp);
    dfree(c->cnt);
    dfree(c->ctopo);
    dfree(c->cnf);
    dfree(c->stage_ids);
    dfree(c->stage_area);
    dfree(c->stage_cen);
    dfree(c->queue);
    dfree(c->gqueue);
    dfree(c->counters);
    dfree(c->rowoff);
    dfree(c->row2cell);
    c->cap_total = c->cap_owned = c->cap_tab = c->cap_retry = c->cap_items = c->cap_hist = c->cap_scan = 0;
    c->cap_faces = false;
}

vt_status hip_fail(hipError_t e, const char *what, int line) {
    if (getenv("VT_DEBUG")) fprintf(stderr, "libvt: %s failed at vt_api.cpp:%d: %s\n", what, line, hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? VT_ERR_OOM : VT_ERR_HIP;
}

#define TRY(x)                                          \
    do {                                                \
        hipError_t e_ = (x);                            \
        if (e_ != hipSuccess) return hip_fail(e_, #x, __LINE__); \
    } while (0)

// Launch errors are read with hipGetLastError(); clear whatever an earlier,
// unrelated runtime call may have left there before enqueueing anything.
void clear_stale_error() { (void)hipGetLastError(); }

// level of the dense Morton table: about pts particles per finest cell
int table_level(int64_t count, double pts) {
    int T = (int)lround(log((double)std::max<int64_t>(count, 1) / pts) / log(8.0));
    return std::min(std::max(T, 1), 9);
}

}  // namespace

extern "C" {

const char *vt_status_string(vt_status s) {
    switch (s) {
        case VT_OK: return "ok";
        case VT_ERR_ARG: return "invalid argument";
        case VT_ERR_HIP: return "HIP runtime error";
        case VT_ERR_OOM: return "out of device memory";
        case VT_ERR_DUPLICATE: return "duplicate particles";
        case VT_ERR_BOX_TOO_SMALL: return "periodic box too small for a cell (2R >= L/2)";
        case VT_ERR_CAPACITY: return "capacity exceeded";
        case VT_ERR_STATE: return "invalid call order";
        case VT_ERR_TOPOLOGY: return "inconsistent clipping topology";
    }
    return "unknown status";
}

vt_status vt_build(vt_ctx **pctx, const void *pos, vt_dtype dtype, const int32_t *global_id, const vt_item *items,
                   int32_t n_items, const vt_opts *opts, void *stream) {
    if (!pctx || !pos || !items || n_items < 1) return VT_ERR_ARG;
    if (dtype != VT_F32 && dtype != VT_F64) return VT_ERR_ARG;
    // validate the item layout
    int64_t n_total = 0, n_owned = 0;
    for (int b = 0; b < n_items; ++b) {
        const vt_item &it = items[b];
        if (it.offset != n_total || it.n_owned < 1 || it.n_ghost < 0) return VT_ERR_ARG;
        if (it.walls < 0 || it.walls > 63 || (it.periodic && it.walls != 0)) return VT_ERR_ARG;
        for (int a = 0; a < 3; ++a)
            if (!(it.hi[a] > it.lo[a])) return VT_ERR_ARG;
        if (it.periodic) {
            if (it.n_ghost != 0) return VT_ERR_ARG;
            double L0 = it.hi[0] - it.lo[0];
            for (int a = 1; a < 3; ++a)
                if (fabs((it.hi[a] - it.lo[a]) - L0) > 1e-12 * L0) return VT_ERR_ARG;
        }
        n_total += it.n_owned + it.n_ghost;
        n_owned += it.n_owned;
    }
    if (n_total >= (int64_t)INT32_MAX) return VT_ERR_ARG;
    vt_opts o{};
    if (opts) o = *opts;
    if (o.precision != VT_PREC_FP64 && o.precision != VT_PREC_MIXED) return VT_ERR_ARG;
    if (!(o.pts_per_grid_cell >= 0.0f) || o.pts_per_grid_cell > 4096.0f || o.k_init < 0 || o.k_init > 100000 ||
        !(o.radius_factor >= 0.0f) || o.radius_factor > 64.0f || o.waves_per_cu < 0 ||
        (o.cell_mapping != VT_MAP_XCD && o.cell_mapping != VT_MAP_GLOBAL))
        return VT_ERR_ARG;
    if (o.pts_per_grid_cell == 0.0f) o.pts_per_grid_cell = 1.0f;
    if (o.k_init > 0) o.radius_factor = (float)cbrt(3.0 * o.k_init / (4.0 * M_PI));

    vt_ctx *c = *pctx;
    if (!c) {
        c = new vt_ctx();
        hipGetDevice(&c->device);
        *pctx = c;
    }
    c->stream = (hipStream_t)stream;
    c->dtype = dtype;
    c->opts = o;
    c->n_total = n_total;
    c->n_owned = n_owned;
    c->n_items = n_items;
    c->built = false;
    c->decomposed = false;
    c->faces_valid = false;
    int ib = 0;
    while ((1 << ib) < n_items) ++ib;
    c->key_bits = VT_LOCAL_KEY_BITS + ib;

    // per-item device descriptors and table sizes
    std::vector<DevItem> di(n_items);
    int64_t tab_total = 0, owned_base = 0;
    for (int b = 0; b < n_items; ++b) {
        const vt_item &it = items[b];
        DevItem &d = di[b];
        double S = 0;
        for (int a = 0; a < 3; ++a) {
            d.lo[a] = it.lo[a];
            d.L[a] = it.hi[a] - it.lo[a];
            S = std::max(S, d.L[a]);
        }
        d.S = S;
        d.inv_res = (double)(1 << VT_MORTON_BITS) / S;
        d.start = it.offset;
        d.count = it.n_owned + it.n_ghost;
        d.n_owned = it.n_owned;
        d.owned_base = owned_base;
        d.T = table_level(d.count, o.pts_per_grid_cell);
        d.tab_off = tab_total;
        d.periodic = it.periodic ? 1 : 0;
        d.walls = it.periodic ? 0 : it.walls;
        d.pad = 0;
        tab_total += (1ll << (3 * d.T)) + 1;
        owned_base += it.n_owned;
    }

    const int64_t nb = (n_total + 4095) / 4096;
    const int64_t hist_need = 2 * 256 * nb + 1;
    const int64_t scan_need = vt_scan_tmp_elems(std::max<int64_t>(n_total, 256 * nb) + 1) + 1;
    const int64_t retry_need = std::max<int64_t>(4096, n_owned / 16);
    const bool need_faces = o.want_faces != 0;
    // spos is sized for double4, so the position dtype may change between builds
    bool realloc_all = n_total > c->cap_total || n_owned > c->cap_owned || tab_total > c->cap_tab ||
                       n_items > c->cap_items || hist_need > c->cap_hist || scan_need > c->cap_scan ||
                       (need_faces && !c->cap_faces);
    if (realloc_all) {
        hipDeviceSynchronize();
        free_all(c);
        const int64_t NT = n_total, NO = n_owned;
        TRY(dalloc(&c->items, n_items));
        TRY(hipHostMalloc((void **)&c->h_items, sizeof(DevItem) * (size_t)n_items, hipHostMallocDefault));
        TRY(hipHostMalloc((void **)&c->h_counters, sizeof(uint32_t) * CTR_COUNT, hipHostMallocDefault));
        for (int k = 0; k < 2; ++k) {
            TRY(dalloc(&c->keys[k], NT + 1));
            TRY(dalloc(&c->vals[k], NT + 1));
        }
        TRY(dalloc(&c->hist, hist_need));
        TRY(dalloc(&c->scan_tmp, scan_need));
        TRY(hipMalloc(&c->spos, sizeof(double4) * (size_t)NT));
        TRY(dalloc(&c->sgid, NT));
        TRY(dalloc(&c->srow, NT));
        TRY(dalloc(&c->sorig, NT));
        TRY(dalloc(&c->tab, tab_total));
        TRY(dalloc(&c->cells, NO));
        TRY(dalloc(&c->row2cell, NO));
        TRY(dalloc(&c->cvol, NO));
        TRY(dalloc(&c->crad, NO));
        TRY(dalloc(&c->ccnt, NO));
        TRY(dalloc(&c->crow, NO));
        TRY(dalloc(&c->cstat, NO));
        TRY(dalloc(&c->cnv, NO));
        TRY(dalloc(&c->cnp, NO));
        TRY(dalloc(&c->cnt, NO));
        TRY(dalloc(&c->ctopo, NO * VT_TOPO_STRIDE));
        TRY(dalloc(&c->cnf, NO));
        const int64_t slots = NO * VT_FSTRIDE_FAST + retry_need * VT_FSTRIDE_BIG;
        TRY(dalloc(&c->stage_ids, slots));
        if (need_faces) {
            TRY(dalloc(&c->stage_area, slots));
            TRY(dalloc(&c->stage_cen, 3 * slots));
        }
        TRY(dalloc(&c->queue, retry_need));
        TRY(dalloc(&c->gqueue, retry_need));
        TRY(dalloc(&c->counters, CTR_COUNT));
        TRY(dalloc(&c->rowoff, NO + 1));
        c->cap_total = NT;
        c->cap_owned = NO;
        c->cap_tab = tab_total;
        c->cap_items = n_items;
        c->cap_hist = hist_need;
        c->cap_scan = scan_need;
        c->cap_retry = retry_need;
        c->cap_faces = need_faces;
    }
    memcpy(c->h_items, di.data(), sizeof(DevItem) * (size_t)n_items);
    clear_stale_error();
    TRY(hipMemcpyAsync(c->items, c->h_items, sizeof(DevItem) * (size_t)n_items, hipMemcpyHostToDevice, c->stream));
    c->timed = o.timing != 0;
    if (c->timed && !c->ev[0])
        for (int k = 0; k < 4; ++k) TRY(hipEventCreate(&c->ev[k]));
    if (c->timed) TRY(hipEventRecord(c->ev[0], c->stream));
    TRY(vt_launch_zero_u32(c->counters, CTR_COUNT, c->stream));
    TRY(vt_launch_sort(c, pos, global_id));
    if (c->timed) TRY(hipEventRecord(c->ev[1], c->stream));
    TRY(vt_launch_clip(c));
    if (c->timed) TRY(hipEventRecord(c->ev[3], c->stream));
    c->built = true;
    c->faces_valid = need_faces;
    return VT_OK;
}

vt_status vt_cells(vt_ctx *c, double *volume, int64_t *nbr_off, int32_t *nbr_ids, int64_t nbr_cap,
                   uint8_t *cell_status, void *stream) {
    if (!c || !(c->built || c->decomposed)) return VT_ERR_STATE;
    if (!volume || !nbr_off || (!nbr_ids && nbr_cap > 0) || nbr_cap < 0) return VT_ERR_ARG;
    c->stream = (hipStream_t)stream;
    if (c->decomposed) return vt_dres_cells(c, volume, nbr_off, nbr_ids, nbr_cap, cell_status);
    clear_stale_error();
    TRY(vt_launch_cells(c, volume, nbr_off, nbr_ids, nbr_cap, cell_status));
    return VT_OK;
}

vt_status vt_density(vt_ctx *c, const void *mass, vt_dtype dtype, double *rho, void *stream) {
    if (!c || !(c->built || c->decomposed)) return VT_ERR_STATE;
    if (!rho || (dtype != VT_F32 && dtype != VT_F64)) return VT_ERR_ARG;
    c->stream = (hipStream_t)stream;
    if (c->decomposed) {
        clear_stale_error();
        return vt_dres_density(c, mass, dtype, rho);
    }
    clear_stale_error();
    TRY(vt_launch_density(c, mass, dtype, rho));
    return VT_OK;
}

vt_status vt_gradient(vt_ctx *c, const double *rho, double *grad, void *stream) {
    if (!c || !c->built) return VT_ERR_STATE;
    if (!rho || !grad) return VT_ERR_ARG;
    c->stream = (hipStream_t)stream;
    clear_stale_error();
    TRY(vt_launch_gradient(c, rho, grad));
    return VT_OK;
}

vt_status vt_grid_deposit(vt_ctx *c, const double *value, int32_t nx, int32_t ny, int32_t nz, double *grid,
                          void *stream) {
    if (!c || !c->built) return VT_ERR_STATE;
    if (!value || !grid || nx < 1 || ny < 1 || nz < 1 || c->n_items != 1) return VT_ERR_ARG;
    c->stream = (hipStream_t)stream;
    clear_stale_error();
    TRY(vt_launch_grid(c, value, nx, ny, nz, grid));
    return VT_OK;
}

vt_status vt_grid_sample(vt_ctx *c, const double *value, int32_t nx, int32_t ny, int32_t nz, int32_t sub,
                         double *grid, int32_t *nearest_id, void *stream) {
    if (!c || !c->built) return VT_ERR_STATE;
    if (!value || !grid || nx < 1 || ny < 1 || nz < 1 || sub < 1 || sub > 16 || c->n_items != 1) return VT_ERR_ARG;
    if (!c->h_items || !c->h_items[0].periodic) return VT_ERR_ARG;
    c->stream = (hipStream_t)stream;
    clear_stale_error();
    TRY(vt_launch_grid_sample(c, value, nx, ny, nz, sub, grid, nearest_id));
    return VT_OK;
}

vt_status vt_grid_tensor(vt_ctx *c, const double *grid, int32_t nx, int32_t ny, int32_t nz, int32_t kind, double *out,
                         void *stream) {
    if (!c || !c->built) return VT_ERR_STATE;
    if (!grid || !out || c->n_items != 1 || !c->h_items || !c->h_items[0].periodic) return VT_ERR_ARG;
    if (kind != VT_TENSOR_TIDAL && kind != VT_TENSOR_HESSIAN) return VT_ERR_ARG;
    for (int32_t d : {nx, ny, nz})
        if (d < 2 || d > 4096 || (d & (d - 1))) return VT_ERR_ARG;
    c->stream = (hipStream_t)stream;
    clear_stale_error();
    TRY(vt_launch_grid_tensor(c, grid, nx, ny, nz, kind, out));
    return VT_OK;
}

vt_status vt_grid_tensor_noalloc(vt_ctx *c, const double *grid, int32_t nx, int32_t ny, int32_t nz, int32_t kind,
                                 double *out, void *stream) {
    if (!c || !c->built) return VT_ERR_STATE;
    if (!grid || !out || c->n_items != 1 || !c->h_items || !c->h_items[0].periodic) return VT_ERR_ARG;
    if (kind != VT_TENSOR_TIDAL && kind != VT_TENSOR_HESSIAN) return VT_ERR_ARG;
    for (int32_t d : {nx, ny, nz})
        if (d < 2 || d > 4096 || (d & (d - 1))) return VT_ERR_ARG;
    if ((int64_t)nx * ny * nz > VT_NOALLOC_TENSOR_POINTS) return VT_ERR_ARG;
    c->stream = (hipStream_t)stream;
    clear_stale_error();
    TRY(vt_launch_grid_tensor_noalloc(c, grid, nx, ny, nz, kind, out));
    return VT_OK;
}

vt_status vt_structure(vt_ctx *c, int64_t *vert_off, double *verts, int64_t vert_cap, int64_t *face_off,
                       int32_t *face_nbr, int64_t face_cap, int64_t *loop_off, int32_t *loop_vert, int64_t loop_cap,
                       int64_t sizes[3], void *stream) {
    if (!c || !c->built) return VT_ERR_STATE;
    if (!c->faces_valid) return VT_ERR_STATE;
    if (!vert_off || !face_off || !sizes || vert_cap < 0 || face_cap < 0 || loop_cap < 0) return VT_ERR_ARG;
    c->stream = (hipStream_t)stream;
    clear_stale_error();
    bool fits = false;
    TRY(vt_launch_structure(c, vert_off, verts, vert_cap, face_off, face_nbr, face_cap, loop_off, loop_vert, loop_cap,
                            sizes, &fits));
    return fits ? VT_OK : VT_ERR_CAPACITY;
}

vt_status vt_backward(vt_ctx *c, const double *dL_dV, double *dL_dx, void *stream) {
    if (!c || !c->built) return VT_ERR_STATE;
    if (!c->faces_valid) return VT_ERR_STATE;
    if (!dL_dV || !dL_dx) return VT_ERR_ARG;
    c->stream = (hipStream_t)stream;
    clear_stale_error();
    TRY(vt_launch_backward(c, dL_dV, dL_dx));
    return VT_OK;
}

vt_status vt_stats(vt_ctx *c, int32_t *n_vertices, int32_t *n_planes, int32_t *n_tested, void *stream) {
    if (!c || !c->built) return VT_ERR_STATE;
    c->stream = (hipStream_t)stream;
    clear_stale_error();
    if (n_planes) TRY(vt_launch_planes(c));
    TRY(vt_launch_stats(c, n_vertices, n_planes, n_tested));
    return VT_OK;
}

vt_status vt_timings(vt_ctx *c, float ms[3]) {
    if (!c || !c->built || !c->timed || !ms) return VT_ERR_STATE;
    TRY(hipEventSynchronize(c->ev[3]));
    for (int k = 0; k < 3; ++k) TRY(hipEventElapsedTime(&ms[k], c->ev[k], c->ev[k + 1]));
    return VT_OK;
}

vt_status vt_sizes(vt_ctx *c, int64_t *n_owned_total, int64_t *n_total) {
    if (!c) return VT_ERR_ARG;
    if (n_owned_total) *n_owned_total = c->decomposed ? c->dres_n : c->n_owned;
    if (n_total) *n_total = c->decomposed ? c->dres_n : c->n_total;
    return VT_OK;
}

vt_status vt_query(vt_ctx *c, int64_t *nnz, int64_t *n_retried, int64_t *n_incomplete) {
    if (c && c->decomposed) {
        TRY(hipStreamSynchronize(c->stream));
        if (nnz) *nnz = c->dres_nnz;
        if (n_retried) *n_retried = c->dres_retried;
        if (n_incomplete) *n_incomplete = c->dres_incomplete;
        return c->dres_capfail ? VT_ERR_CAPACITY : c->dres_status;
    }
    if (!c || !c->built) return VT_ERR_STATE;
    TRY(hipStreamSynchronize(c->stream));
    TRY(hipMemcpy(c->h_counters, c->counters, sizeof(uint32_t) * CTR_COUNT, hipMemcpyDeviceToHost));
    const uint32_t *h = c->h_counters;
    if (nnz) *nnz = (int64_t)(((uint64_t)h[CTR_NNZ_HI] << 32) | h[CTR_NNZ_LO]);
    if (n_retried) *n_retried = h[CTR_QUEUE];
    if (n_incomplete) *n_incomplete = h[CTR_INCOMPLETE];
    uint32_t st = h[CTR_STATUS];
    if (getenv("VT_DEBUG") && (st || h[CTR_DEBUG]))
        fprintf(stderr, "libvt: device status 0x%x, debug 0x%x, queue %u, rejected records %u\n", st, h[CTR_DEBUG],
                h[CTR_QUEUE], h[CTR_REC_REJECT]);
    if (st & VT_DEV_DUPLICATE) return VT_ERR_DUPLICATE;  // the root cause of any later failure
    if (st & VT_DEV_TOPOLOGY) return VT_ERR_TOPOLOGY;
    if (st & VT_DEV_BOX_TOO_SMALL) return VT_ERR_BOX_TOO_SMALL;
    if (st & (VT_DEV_CAPACITY | VT_DEV_NBR_CAP)) return VT_ERR_CAPACITY;
    return VT_OK;
}

void vt_destroy(vt_ctx *c) {
    if (!c) return;
    hipDeviceSynchronize();
    free_all(c);
    vt_dec_free(c);
    vt_struct_free(c);
    vt_spec_free(c);
    if (c->samp_fine) hipFree(c->samp_fine);
    for (int k = 0; k < 4; ++k)
        if (c->ev[k]) hipEventDestroy(c->ev[k]);
    delete c;
}

}  // extern "C"

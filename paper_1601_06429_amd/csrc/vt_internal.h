// vt_internal.h -- shared declarations of the HIP implementation (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vt.h"

// ---------------------------------------------------------------- constants
#define VT_MORTON_BITS 16          // quantisation bits per axis of the Morton key
#define VT_LOCAL_KEY_BITS 48       // 3 * VT_MORTON_BITS
#define VT_CAND_MAX 128            // candidates per clipping pass held in LDS
#define VT_FSTRIDE_FAST 40         // facet slots per cell, fast kernel (F <= 34 when V <= 64)
#define VT_FSTRIDE_BIG 136         // facet slots per cell, large kernel (F <= 130 when V <= 256)
#define VT_TOPO_FACES 40           // face-table words of a topology record (F <= 34 when V <= 64)
#define VT_TOPO_STRIDE 104         // topology record: VT_TOPO_FACES face tags + 64 vertex triples
#define VT_DEC_MAX_PASSES 16       // vt_decomposed_build: at most 15 re-runs

// device status word bits
#define VT_DEV_DUPLICATE 1u
#define VT_DEV_BOX_TOO_SMALL 2u
#define VT_DEV_CAPACITY 4u
#define VT_DEV_TOPOLOGY 8u
#define VT_DEV_NBR_CAP 16u

// counters[] slots
#define CTR_CELL 0        // persistent work counter, fast kernel
#define CTR_RETRY 1       // persistent work counter, large kernel
#define CTR_QUEUE 2       // retry queue length
#define CTR_STATUS 3      // device status bits
#define CTR_NNZ_LO 4      // total facets (64-bit, two words)
#define CTR_NNZ_HI 5
#define CTR_INCOMPLETE 6
#define CTR_GRID 7        // grid deposit work counters (two words)
#define CTR_GRID_RETRY 8
#define CTR_DEBUG 9        // bit k set: a clip in the grid kernel returned -k (diagnostics)
#define CTR_GRID_Q 10      // grid deposit: cells handed from the normal to the large kernel
#define CTR_STRUCT_Q 11    // structure output: cells handed from the normal to the large kernel
#define CTR_REC_REJECT 12  // topology records that failed their checks (a clip-kernel fault; 0 expected)
#define CTR_SEG0 13        // fast clip kernel: work counters of the XCD segments (VT_XCD_SEGMENTS words)
#define VT_XCD_SEGMENTS 8  // XCDs of an MI355X; workgroups are dealt to them round-robin
#define CTR_TAB_PIECES (CTR_SEG0 + VT_XCD_SEGMENTS)  // level table: pieces of long runs listed for k_level_fill
#define CTR_COUNT (CTR_TAB_PIECES + 1)

// per-item description on the device
struct DevItem {
    double lo[3];
    double L[3];        // box lengths
    double S;           // Morton cube side (max of L)
    double inv_res;     // 2^16 / S
    int64_t start;      // first particle (input order == sorted order range)
    int64_t count;      // n_owned + n_ghost
    int64_t n_owned;
    int64_t owned_base; // first output row
    int64_t tab_off;    // offset of the level table in tab[]
    int32_t T;          // table level
    int32_t periodic;
    int32_t walls;      // bounded: faces that are true boundaries (vt_item.walls)
    int32_t pad;
};

// ---------------------------------------------------------------- context
struct vt_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    vt_dtype dtype = VT_F64;
    vt_opts opts{};
    int64_t n_total = 0, n_owned = 0;
    int32_t n_items = 0;
    int key_bits = 48;
    bool faces_valid = false;
    bool built = false;

    // capacities of the allocations below
    int64_t cap_total = 0, cap_owned = 0, cap_tab = 0, cap_retry = 0, cap_items = 0, cap_hist = 0;
    int64_t cap_scan = 0;
    bool cap_faces = false;

    DevItem *items = nullptr;      // device copy
    DevItem *h_items = nullptr;    // host copy (pinned not needed)
    // sort
    uint64_t *keys[2] = {nullptr, nullptr};
    uint32_t *vals[2] = {nullptr, nullptr};
    int32_t *hist = nullptr;
    int64_t *scan_tmp = nullptr;
    // sorted particle arrays (Morton order)
    void *spos = nullptr;          // float4 or double4
    uint64_t *skey = nullptr;      // alias of keys[final]
    int32_t *sgid = nullptr;       // global id per sorted particle
    int32_t *srow = nullptr;       // output row, -1 for ghosts
    int32_t *sorig = nullptr;      // index in the caller's pos[]
    int32_t *tab = nullptr;        // level tables
    int32_t *cells = nullptr;      // owned sorted indices, in Morton order
    // clip results per cell slot
    double *cvol = nullptr;
    double *crad = nullptr;        // largest vertex distance per cell
    int32_t *ccnt = nullptr;
    int64_t *crow = nullptr;       // staging row start
    uint8_t *cstat = nullptr;
    int32_t *cnv = nullptr, *cnp = nullptr, *cnt = nullptr;
    // topology of each cell the fast clip kernel finished (VT_TOPO_STRIDE words per cell):
    // face tags in face order, then vertex triples as face ranks; cnf = number of faces, 0 = none
    int32_t *ctopo = nullptr;
    int32_t *cnf = nullptr;
    int32_t *stage_ids = nullptr;
    double *stage_area = nullptr;
    double *stage_cen = nullptr;   // 3 per facet
    int32_t *queue = nullptr;
    int32_t *gqueue = nullptr;     // grid deposit overflow queue
    uint32_t *counters = nullptr;  // CTR_*
    // post-processing
    int64_t *rowoff = nullptr;     // facet offsets in output-row order (n_owned + 1)
    int32_t *row2cell = nullptr;   // cell slot of each output row
    uint32_t *h_counters = nullptr;
    // domain decomposition (decomp.hip)
    uint32_t *dec_hist = nullptr;  // per task face and threshold: particles in that distance bin
    int64_t *dec_cnt = nullptr;    // per listed task: owned, buffer counts (then write cursors)
    int64_t *dec_base = nullptr;   // per listed task: output offsets of its owned and buffer particles
    double *dec_thick = nullptr;   // 6 per task
    int32_t *dec_tpos = nullptr;   // task -> position in the list, -1 if not listed
    double *dec_thr = nullptr;     // thresholds (64)
    int64_t cap_dec_tasks = 0, cap_dec_hist = 0;
    // whole decomposed build (decomp.hip): results in particle order, kept for vt_cells,
    // vt_density and vt_query; per pass, the neighbour CSR of the cells it computed
    bool decomposed = false;
    int64_t dres_n = 0, dres_nnz = 0, dres_retried = 0, dres_incomplete = 0;
    vt_status dres_status = VT_OK;
    bool dres_capfail = false;
    double *dres_vol = nullptr;
    uint8_t *dres_stat = nullptr;
    int64_t *dres_off = nullptr;
    int32_t *dres_ids = nullptr;
    int32_t *dres_last = nullptr;   // pass that computed the particle's cell
    int32_t *dres_row = nullptr;    // its row in that pass
    uint8_t *dres_mask = nullptr;   // owner mask of the next pass
    int32_t *dres_tflag = nullptr;  // per task: owns a cell left incomplete
    int64_t *dres_cnt = nullptr;
    int64_t *dres_scan = nullptr;
    int64_t cap_dres = 0, cap_dres_ids = 0, cap_dres_tasks = 0;
    double *dpack_pos = nullptr;    // the batch of a pass
    int32_t *dpack_gid = nullptr;
    int64_t cap_dpack = 0;
    int64_t *dpack_items = nullptr; // per listed task: first output row, batch offset, owned count
    int64_t cap_dpack_items = 0;
    double *dpass_vol = nullptr;    // one pass's cell outputs in its row order
    uint8_t *dpass_stat = nullptr;
    int64_t cap_dpass_rows = 0;
    int64_t *dpass_off[VT_DEC_MAX_PASSES] = {};
    int32_t *dpass_ids[VT_DEC_MAX_PASSES] = {};
    int64_t dpass_cap_rows[VT_DEC_MAX_PASSES] = {}, dpass_cap_ids[VT_DEC_MAX_PASSES] = {};
    vt_ctx *dchild = nullptr;       // context of the passes' builds
    // nearest-particle sampling: per sample point, the nearest particle (sorted index)
    int32_t *samp_fine = nullptr;
    int64_t cap_samp = 0;
    // structure output (structure.hip): per-row counts (vertices, faces, loop entries), loop
    // offsets per row, per-cell large-kernel marks, overflow queue
    int64_t *st_cnt = nullptr;
    int64_t *st_lbase = nullptr;
    uint8_t *smark = nullptr;
    int32_t *squeue = nullptr;
    int64_t cap_struct = 0;
    // grid tensors (spectral.hip): two complex work arrays of the grid's size
    void *spec_buf = nullptr;
    int64_t cap_spec = 0;
    // optional stage timing
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    bool timed = false;
};

// ---------------------------------------------------------------- launchers
hipError_t vt_launch_sort(vt_ctx *c, const void *pos, const int32_t *gid);
hipError_t vt_launch_clip(vt_ctx *c);  // records ev[2] between the two kernels when timing
hipError_t vt_launch_scan_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *tmp, hipStream_t s);
hipError_t vt_launch_scan_i32(const int32_t *in, int32_t *out, int64_t n, int64_t *tmp, hipStream_t s);
hipError_t vt_launch_cells(vt_ctx *c, double *volume, int64_t *nbr_off, int32_t *nbr_ids, int64_t nbr_cap,
                           uint8_t *cell_status);
hipError_t vt_launch_density(vt_ctx *c, const void *mass, vt_dtype dt, double *rho);
hipError_t vt_launch_gradient(vt_ctx *c, const double *rho, double *grad);
hipError_t vt_launch_grid(vt_ctx *c, const double *value, int nx, int ny, int nz, double *grid);
hipError_t vt_launch_grid_sample(vt_ctx *c, const double *value, int nx, int ny, int nz, int sub, double *grid,
                                 int32_t *nearest);
hipError_t vt_launch_backward(vt_ctx *c, const double *g, double *out);
hipError_t vt_launch_stats(vt_ctx *c, int32_t *nv, int32_t *np, int32_t *nt);
hipError_t vt_launch_planes(vt_ctx *c);  // exact planes-examined count of every cell into cnp
hipError_t vt_launch_zero_u32(uint32_t *p, int64_t n, hipStream_t s);

int64_t vt_scan_tmp_elems(int64_t n);
void vt_dec_free(vt_ctx *c);
vt_status vt_dres_cells(vt_ctx *c, double *volume, int64_t *nbr_off, int32_t *nbr_ids, int64_t nbr_cap,
                        uint8_t *cell_status);
vt_status vt_dres_density(vt_ctx *c, const void *mass, vt_dtype dt, double *rho);
hipError_t vt_launch_structure(vt_ctx *c, int64_t *vert_off, double *verts, int64_t vert_cap, int64_t *face_off,
                               int32_t *face_nbr, int64_t face_cap, int64_t *loop_off, int32_t *loop_vert,
                               int64_t loop_cap, int64_t sizes[3], bool *fits);
void vt_struct_free(vt_ctx *c);
hipError_t vt_launch_grid_tensor(vt_ctx *c, const double *grid, int nx, int ny, int nz, int kind, double *out);
hipError_t vt_launch_grid_tensor_noalloc(vt_ctx *c, const double *grid, int nx, int ny, int nz, int kind,
                                         double *out);
void vt_spec_free(vt_ctx *c);

// ---------------------------------------------------------------- device helpers
#ifdef __HIP_DEVICE_COMPILE__
#define VT_DEV __device__ __forceinline__
#else
#define VT_DEV __host__ __device__ inline
#endif

// spread the low 16 bits of v to every third bit
VT_DEV uint64_t vt_spread3(uint64_t x) {
    x &= 0x1fffffull;
    x = (x | x << 32) & 0x1f00000000ffffull;
    x = (x | x << 16) & 0x1f0000ff0000ffull;
    x = (x | x << 8) & 0x100f00f00f00f00full;
    x = (x | x << 4) & 0x10c30c30c30c30c3ull;
    x = (x | x << 2) & 0x1249249249249249ull;
    return x;
}

VT_DEV uint64_t vt_morton(uint64_t ix, uint64_t iy, uint64_t iz) {
    return (vt_spread3(ix) << 2) | (vt_spread3(iy) << 1) | vt_spread3(iz);
}

// quantised coordinate of x (item-relative Morton grid); monotone in x, not clamped
VT_DEV int64_t vt_qraw(double x, double lo, double inv_res) { return (int64_t)floor((x - lo) * inv_res); }

VT_DEV int64_t vt_qclamp(int64_t q) {
    const int64_t m = (1ll << VT_MORTON_BITS) - 1;
    return q < 0 ? 0 : (q > m ? m : q);
}

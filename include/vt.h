/*
 * vt.h -- C ABI of the MI355X Voronoi tessellation engine (libvt.so).
 *
 * The engine computes, for every owned particle of a periodic box or of a
 * bounded sub-volume with its buffer ("ghost") particles, the quantities the
 * paper lists per particle: the immediate-neighbour list, the Voronoi cell
 * volume, the Voronoi density (mass / volume), the density gradient, and the
 * average density on a regular grid (abstract; section 2, post-processing
 * paragraph).  Neighbours are the particles that share a facet with the cell
 * (section 2); outputs come back in input order with neighbour ids replaced by
 * the callers' global ids (section 2, gather paragraph).  Periodic boundary
 * conditions are supported (abstract; section 4).  The volume adjoint
 * (vt_backward) is an extension for gradient-based use; it is not in the paper.
 *
 * Conventions for every entry point:
 *   - Pointers marked "device" are HIP device pointers owned by the caller;
 *     the library never frees them.  Pointers marked "host" are read before
 *     the call returns.
 *   - Every call except vt_query, vt_destroy and vt_status_string only
 *     enqueues work on `stream` (a hipStream_t passed as void*; NULL is the
 *     default stream) and returns; results are ready when the stream is.
 *   - Argument errors are returned synchronously and nothing is enqueued.
 *     Errors found on the device (duplicate particles, a cell that reaches its
 *     own periodic image, a capacity overflow) are recorded in a device status
 *     word that vt_query returns; outputs are undefined after such an error.
 *   - Per-cell soft conditions are reported in cell_status (VT_CELL_* bits).
 *   - The context owns all scratch memory.  vt_build allocates it on first use
 *     and reuses it when called again on the same context with sizes that fit,
 *     so repeated builds of the same shape allocate nothing.
 *   - Calls on one context must be serialised by the caller (same stream).
 */
#ifndef VT_H
#define VT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vt_ctx vt_ctx;

typedef enum {
    VT_OK = 0,
    VT_ERR_ARG = 1,           /* invalid argument (returned synchronously) */
    VT_ERR_HIP = 2,           /* a HIP runtime call failed */
    VT_ERR_OOM = 3,           /* device allocation failed */
    VT_ERR_DUPLICATE = 4,     /* two particles of one world coincide exactly */
    VT_ERR_BOX_TOO_SMALL = 5, /* a periodic cell reaches a second image (2R >= L/2) */
    VT_ERR_CAPACITY = 6,      /* a cell exceeds the largest kernel capacity, or nbr_cap is too small */
    VT_ERR_STATE = 7,         /* call order violated (e.g. vt_backward without faces) */
    VT_ERR_TOPOLOGY = 8       /* inconsistent clipping decision (should not happen) */
} vt_status;

typedef enum { VT_F32 = 0, VT_F64 = 1 } vt_dtype;

typedef enum {
    VT_PREC_FP64 = 0,  /* every step in FP64 */
    VT_PREC_MIXED = 1  /* FP32 clipping with FP64 fallback predicates; FP64 geometry */
} vt_precision;

/* per-cell status bits (cell_status output) */
#define VT_CELL_OK 0
#define VT_CELL_INCOMPLETE 1   /* bounded world: ball(x, 2R) leaves the box, or a wall face survived */
#define VT_CELL_RETRIED 2      /* computed by the large-capacity kernel */
#define VT_CELL_FAILED 4       /* could not be computed (see vt_query status) */

/*
 * One world ("item").  Its particles are pos[offset .. offset + n_owned) (cells
 * are computed for these) followed by pos[offset + n_owned .. + n_ghost) (buffer
 * particles that only clip).  Items must be packed back to back in item order:
 * items[0].offset == 0 and items[b+1].offset == items[b].offset + n_owned + n_ghost.
 *   periodic = 1: the box [lo, hi) is periodic; it must be a cube, every
 *                 particle must lie in it, and n_ghost must be 0.
 *   periodic = 0: the box [lo, hi] bounds the world; its walls are the initial
 *                 cell.  A wall is either a cut through a larger volume (the
 *                 outer side of the buffer zone of section 2) or a true boundary
 *                 of the tessellated world (a survey volume's edge), as `walls`
 *                 says.  A cell that a cut wall still touches, or whose security
 *                 ball crosses a cut wall, is flagged VT_CELL_INCOMPLETE; true
 *                 walls clip cells but never make them incomplete.
 *   walls    (bounded items only) bit f set: box face f (-x, +x, -y, +y, -z, +z
 *            for f = 0 .. 5) is a true boundary.  0 = every wall is a cut.
 * Owned outputs are dense over items: the owned particle k of item b is output
 * row sum_{b' < b} n_owned(b') + k.
 */
typedef struct {
    int64_t offset;
    int64_t n_owned;
    int64_t n_ghost;
    int32_t periodic;
    int32_t walls;
    double lo[3];
    double hi[3];
} vt_item;

/*
 * Options; a zero field selects the default.  None of them changes a result, only speed (the
 * cell is certified by the security radius whatever the search does).
 *   radius_factor, k_init  the first search shell: its radius in local mean spacings, or the
 *                          number of particles it should hold on average (k_init, which sets
 *                          radius_factor = (3 k_init / (4 pi))^(1/3) when given).  Later
 *                          shells grow until the security radius is reached, with no cap on k
 *                          other than the box (a periodic cell must stay within a quarter
 *                          period, else VT_ERR_BOX_TOO_SMALL).
 *   pts_per_grid_cell      resolution of the uniform-grid (Morton level) table of the kNN
 *                          search: level T = round(log8(n / pts_per_grid_cell)), clamped to
 *                          [1, 9], per item (default 1).
 *   waves_per_cu           resident wavefronts of the persistent clip kernel (one cell per
 *                          wavefront; cells that outgrow 64 vertices move to a kernel with one
 *                          wavefront per block and 256 vertex slots).
 *   cell_mapping           which cells each wavefront takes (VT_MAP_*).
 */
typedef struct {
    int32_t precision;       /* vt_precision, default VT_PREC_FP64 */
    int32_t want_faces;      /* keep facet areas and centroids (needed by vt_backward) */
    float radius_factor;     /* first search radius in local mean spacings (default 2.0) */
    float area_eps;          /* facets with area <= area_eps * V^(2/3) are not facets (default 1e-12) */
    int32_t waves_per_cu;    /* persistent clip kernel occupancy (default 16) */
    int32_t timing;          /* record HIP events around the sort and clip kernels (see vt_timings) */
    float pts_per_grid_cell; /* kNN grid resolution, particles per finest table cell (default 1) */
    int32_t k_init;          /* first shell in particles (overrides radius_factor when > 0) */
    int32_t cell_mapping;    /* VT_MAP_*: which cells the clip kernel's wavefronts take (default XCD segments) */
    int32_t reserved;
} vt_opts;

/* vt_opts.cell_mapping: how the persistent clip kernel deals cells (in Morton order) to wavefronts */
#define VT_MAP_XCD 0     /* each XCD (its own L2) takes a contiguous eighth, then helps the others */
#define VT_MAP_GLOBAL 1  /* one queue: consecutive cells go to wavefronts on all XCDs in turn */

/*
 * vt_build -- tessellate.  The cell of a particle is the region closer to it
 * than to any other particle (section 1; with periodic conditions, closer than
 * to any periodic image).  A sub-volume is tessellated together with its
 * buffer particles, which clip the owned cells but get none of their own
 * (section 2, the buffer zone between tasks).  Sorts the particles of each item
 * along a Morton curve, builds the per-item cell tables, then computes every
 * owned cell by clipping with bisector planes in increasing distance order
 * until the security radius certifies it (all particles closer than twice the
 * largest vertex distance have been used).
 *   ctx        in/out: *ctx == NULL creates a context; a context from an
 *              earlier build is reused (its scratch grows only if needed).
 *   pos        device, n_total x 3 positions (AoS), dtype VT_F32 or VT_F64,
 *              n_total = sum of n_owned + n_ghost.
 *   global_id  device, n_total int32 ids reported as neighbour ids; NULL means
 *              the particle's index in pos.
 *   items      host, n_items >= 1 worlds (see vt_item).
 *   opts       host, nullable.
 * Errors: VT_ERR_ARG (bad sizes, an item without owned particles, unpacked
 * items, non-cubic periodic box), VT_ERR_OOM, VT_ERR_HIP.
 */
vt_status vt_build(vt_ctx **ctx, const void *pos, vt_dtype dtype, const int32_t *global_id, const vt_item *items,
                   int32_t n_items, const vt_opts *opts, void *stream);

/*
 * vt_cells -- cell volumes and neighbour lists of the owned particles, in
 * output-row order (section 2: volume; neighbours sharing a facet; real ids).
 *   volume       device, n_owned_total doubles.
 *   nbr_off      device, n_owned_total + 1 int64 CSR offsets.
 *   nbr_ids      device, nbr_cap int32 global ids; row i holds the ascending
 *                ids of the particles that share a facet of positive area
 *                with cell i (self excluded).
 *   cell_status  device, n_owned_total bytes (VT_CELL_* bits), nullable.
 * If the total neighbour count exceeds nbr_cap nothing past nbr_cap is
 * written and vt_query reports VT_ERR_CAPACITY; vt_query also returns the
 * total (nnz) so the caller can size nbr_ids.
 */
vt_status vt_cells(vt_ctx *ctx, double *volume, int64_t *nbr_off, int32_t *nbr_ids, int64_t nbr_cap,
                   uint8_t *cell_status, void *stream);

/*
 * vt_density -- rho_i = m_i / V_i for the owned particles (section 2).
 *   mass  device, n_total masses (dtype), indexed like pos; NULL = unit masses.
 *   rho   device, n_owned_total doubles (output rows).
 */
vt_status vt_density(vt_ctx *ctx, const void *mass, vt_dtype dtype, double *rho, void *stream);

/*
 * vt_gradient -- density gradient per owned particle, built from the densities
 * and the neighbour lists (section 2).  The paper gives no formula; this is the
 * unweighted least-squares fit over the Voronoi neighbours:
 *   grad_i = G^-1 b,  G = sum_j D_ij D_ij^T,  b = sum_j (rho_j - rho_i) D_ij,
 * D_ij the separation (minimum image in periodic boxes).
 *   rho   device, n_total doubles indexed like pos (ghost entries are used
 *         for ghost neighbours).
 *   grad  device, n_owned_total x 3 doubles (output rows).
 */
vt_status vt_gradient(vt_ctx *ctx, const double *rho, double *grad, void *stream);

/*
 * vt_grid_deposit -- average Voronoi density on a regular grid (section 2,
 * optional grid output): grid[(a*ny + b)*nz + c] = sum_i value_i *
 * vol(cell_i ∩ voxel_abc) / vol(voxel), exact polyhedron-voxel overlaps.
 * Voxels tile the box of item 0 (periodic boxes wrap voxel indices); only
 * single-item contexts are supported.
 *   value  device, n_owned_total doubles (output rows), e.g. rho from vt_density.
 *   grid   device, nx*ny*nz doubles; overwritten.
 */
vt_status vt_grid_deposit(vt_ctx *ctx, const double *value, int32_t nx, int32_t ny, int32_t nz, double *grid,
                          void *stream);

/*
 * vt_grid_sample -- a cheaper grid than vt_grid_deposit (the paper lists grid
 * variants as future work, section 4): every sample point takes the value of
 * the particle nearest to it, i.e. of the Voronoi cell that contains it
 * (periodic minimum image, FP64 squared distances; ties go to the smaller
 * global id).  Voxel (a, b, c) averages the sub^3 points at the centres of its
 * sub^3 equal sub-cells; sub = 1 samples the voxel centre.  Periodic
 * single-item contexts only (vt_build takes periodic boxes cubic); anything
 * else returns VT_ERR_ARG and writes nothing.
 *   value       device, n_owned_total doubles (output rows).
 *   sub         1 .. 16.
 *   grid        device, nx*ny*nz doubles; overwritten.
 *   nearest_id  device, nx*ny*nz int32 or NULL: the global id of the particle
 *               nearest to the voxel's last sample point (its centre when
 *               sub = 1).
 */
vt_status vt_grid_sample(vt_ctx *ctx, const double *value, int32_t nx, int32_t ny, int32_t nz, int32_t sub,
                         double *grid, int32_t *nearest_id, void *stream);

/* kinds of grid tensor (vt_grid_tensor) */
#define VT_TENSOR_TIDAL 0     /* d_i d_j phi, laplacian(phi) = f / mean(f) - 1 */
#define VT_TENSOR_HESSIAN 1   /* d_i d_j f */

/*
 * vt_grid_tensor -- second-derivative tensor of a grid field, for the tidal-
 * tensor and Hessian analysis the paper lists among future grid outputs
 * (section 4).  Spectral on the periodic grid of item 0's box, k_a = 2 pi m / L_a
 * with m the signed frequency index:
 *   VT_TENSOR_TIDAL    T_ij = d_i d_j phi with laplacian(phi) = delta,
 *                      delta = f / mean(f) - 1, i.e. T_ij(k) = k_i k_j / |k|^2
 *                      f(k) / mean(f) (0 at k = 0); trace T = delta.
 *   VT_TENSOR_HESSIAN  H_ij = d_i d_j f, H_ij(k) = -k_i k_j f(k).
 * A mixed component is zero on the Nyquist plane of either of its axes.
 *   grid   device, nx*ny*nz doubles laid out like vt_grid_deposit's (e.g. its
 *          output); for VT_TENSOR_TIDAL its mean must not be zero.
 *   out    device, 6 x nx*ny*nz doubles: components xx, yy, zz, xy, xz, yz,
 *          each laid out like grid; overwritten.
 * nx, ny, nz are powers of two from 2 to 4096.  Periodic single-item contexts
 * only.  Scratch: 32 bytes per grid point, kept by the context.
 * Errors: VT_ERR_STATE, VT_ERR_ARG (sizes, kind, context), VT_ERR_OOM,
 * VT_ERR_HIP.
 */
vt_status vt_grid_tensor(vt_ctx *ctx, const double *grid, int32_t nx, int32_t ny, int32_t nz, int32_t kind,
                         double *out, void *stream);

/* Largest grid (points) vt_grid_tensor_noalloc takes: 2^21, e.g. 128^3 (64 MiB of scratch). */
#define VT_NOALLOC_TENSOR_POINTS (1 << 21)

/*
 * vt_grid_tensor_noalloc -- vt_grid_tensor for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same result, bit for bit, with the 32 bytes per
 * grid point of FFT scratch taken from a static device array of the library
 * instead of the context.  The array holds VT_NOALLOC_TENSOR_POINTS points; each
 * device the library runs this on keeps its own copy (64 MiB) until the process
 * ends.  The call allocates nothing (no hipMalloc, hipFree or allocating
 * library routine).  Every call on one device shares that device's array, so
 * calls that overlap on one device (different streams, or different host
 * threads) race and must be serialised by the caller; the array needs no
 * clearing between calls (each call writes its scratch before reading it).
 * Arguments as vt_grid_tensor; nx * ny * nz above VT_NOALLOC_TENSOR_POINTS is
 * rejected with VT_ERR_ARG (synchronously, nothing enqueued).
 */
vt_status vt_grid_tensor_noalloc(vt_ctx *ctx, const double *grid, int32_t nx, int32_t ny, int32_t nz, int32_t kind,
                                 double *out, void *stream);

/*
 * vt_structure -- the full tessellation structure of the owned cells (the
 * paper's optional full structure output: section 3, memory consumption;
 * section 4): every cell's vertices and its faces as vertex loops, CSR in
 * output-row order.
 *   vert_off   device, n_owned_total + 1 int64: cell i's vertices are rows
 *              vert_off[i] .. vert_off[i+1]-1 of verts.
 *   verts      device, vert_cap x 3 doubles: absolute coordinates, the seed
 *              plus the vertex's offset (a cell of a periodic box is kept
 *              whole, so its vertices may lie outside the box).
 *   face_off   device, n_owned_total + 1 int64: cell i's faces.
 *   face_nbr   device, face_cap int32: the global id across each face, or
 *              -1 .. -6 for the walls -x, +x, -y, +y, -z, +z of a bounded
 *              item.  A cell's faces ascend by it.  A particle's face is
 *              listed if the particle is in the cell's neighbour list (faces
 *              of area > area_eps V^(2/3); vt_cells), so the nonnegative
 *              entries of a row are exactly that list; a wall if its area
 *              exceeds the same bound.  A cell that loses a face this way
 *              keeps a hole of at most that area (its loops then hold fewer
 *              than three entries per vertex).
 *   loop_off   device, face_cap + 1 int64: face f's loop is
 *              loop_vert[loop_off[f] .. loop_off[f+1]-1].
 *   loop_vert  device, loop_cap int32: vertex indices local to the cell
 *              (0 .. vertices - 1), counter-clockwise seen from outside the
 *              cell, starting at the face's smallest index.
 *   sizes      host, 3 int64 (out): total vertices, faces and loop entries.
 * The offsets are always written.  If a total exceeds its capacity, or an
 * output pointer is NULL, nothing else is written and VT_ERR_CAPACITY is
 * returned with sizes filled: call again with arrays of those sizes.  Needs a
 * build with want_faces (else VT_ERR_STATE).  Synchronizes the stream (it
 * reads the totals).  A cell whose face loops do not close is left empty and
 * vt_query reports VT_ERR_TOPOLOGY.
 */
vt_status vt_structure(vt_ctx *ctx, int64_t *vert_off, double *verts, int64_t vert_cap, int64_t *face_off,
                       int32_t *face_nbr, int64_t face_cap, int64_t *loop_off, int32_t *loop_vert, int64_t loop_cap,
                       int64_t sizes[3], void *stream);

/*
 * vt_backward -- volume adjoint: given g = dL/dV (device, n_owned_total
 * doubles, output rows; ghost cells carry no volume), writes
 *   dL/dx_k = sum_{j in N(k)} (g_k - g_j) A_kj (c_kj - x_k) / |x_j - x_k|
 * for every owned particle k (device, n_owned_total x 3 doubles, overwritten),
 * A_kj and c_kj the area and centroid of the shared facet.  Requires a build
 * with want_faces (else VT_ERR_STATE).  Ghost neighbours contribute with
 * g_j = 0.
 */
vt_status vt_backward(vt_ctx *ctx, const double *dL_dV, double *dL_dx, void *stream);

/*
 * vt_query -- synchronises the context's last stream and reports: the device
 * status (return value), the total neighbour count, the number of cells that
 * needed the large-capacity kernel, and the number of cells flagged
 * incomplete.  Any pointer may be NULL.
 */
vt_status vt_query(vt_ctx *ctx, int64_t *nnz, int64_t *n_retried, int64_t *n_incomplete);

/*
 * vt_stats -- per-owned-cell diagnostics (device, n_owned_total int32 each,
 * output rows, any may be NULL): final vertex count, planes the security
 * criterion had to examine (particles closer than 2R, R the cell's largest
 * vertex distance, plus one; counted exactly by a pass of its own), and
 * candidates the clip kernel actually tested.  Used by the benchmark's cost
 * model.
 */
vt_status vt_stats(vt_ctx *ctx, int32_t *n_vertices, int32_t *n_planes, int32_t *n_tested, void *stream);

/*
 * vt_timings -- durations (ms) of the last build's stages, measured with HIP
 * events recorded on the build's stream when opts.timing was set:
 * ms[0] = Morton sort and tables, ms[1] = fast clip kernel, ms[2] = large
 * clip kernel.  Synchronises on the events; VT_ERR_STATE if timing was off.
 */
vt_status vt_timings(vt_ctx *ctx, float ms[3]);

/*
 * Domain decomposition with AUTOBORDER (section 2: the volume is split into
 * sub-volumes, each with a buffer zone of boundary particles; the buffer
 * starts at BORDERFACTOR times the mean inter-particle distance, computed from
 * the whole input, and, where the particle density in it is below the mean,
 * grows until it holds the number of particles the mean density puts in the
 * initial zone; cells whose buffer still did not suffice are reported).  On one
 * GPU the tasks become the items of one batched vt_build.
 *
 * The world [lo, hi] is split into nt[0] x nt[1] x nt[2] equal tasks: the
 * paper's scheme (a) is a power-of-two split into near-cubes, scheme (b) a
 * split along one axis into slabs for elongated volumes (survey slices and
 * cones).  Task b = (ix * nt[1] + iy) * nt[2] + iz owns the particles whose
 * cell index floor((x - lo) / w) (clamped to the grid) is (ix, iy, iz),
 * w = (hi - lo) / nt.  The world is either a periodic box [lo, hi) or a bounded
 * volume [lo, hi] (every particle inside; its faces are true walls, see
 * vt_item.walls).  The buffer zone of a task face is the slab beyond it over
 * the face's extent.
 *
 * Reading of the growth rule: with s = (V / n)^(1/3) the mean inter-particle
 * distance (V the world's volume), the thicknesses tried are
 * t_k = border_factor * s * growth^k, k = 0 .. n_steps - 1, and a face takes
 * the smallest t_k whose slab holds at least n / V * A_face * t_0 particles (a
 * particle counts if its distance beyond the face is below t_k), t_{n_steps-1}
 * if none does; then it is capped.  Periodic worlds: a buffered task spans
 * less than one period, so the cap is (L - w) / 2 per axis (L / 2 with one task
 * there).  Bounded worlds: the cap is the face's distance to the world's wall
 * (0 on the world's own faces), so a buffered task never leaves the world.
 */
typedef struct {
    double border_factor;  /* BORDERFACTOR, default 1.5 (the paper's example value) */
    double growth;         /* ratio of consecutive thicknesses, default 1.1 */
    int32_t n_steps;       /* thicknesses tried, 1 .. 64, default 48 */
    int32_t max_reruns;    /* vt_decomposed_build: passes after the first, default 3 */
    double widen;          /* vt_decomposed_build: buffer factor per re-run, default 2 */
} vt_border;

/*
 * vt_task_grid -- tasks per axis for the paper's two layouts (section 2), host
 * only.  scheme 0 (a): the box is halved along x, then y, then z, and round
 * again, until there are n_task equal regions (n_task a power of two; 32 gives
 * 4 x 4 x 2).  scheme 1 (b): n_task slabs along `axis` (elongated volumes).
 * nt: host out, 3 int32.  Errors: VT_ERR_ARG.
 */
vt_status vt_task_grid(int32_t n_task, int32_t scheme, int32_t axis, int32_t nt[3]);

/*
 * vt_border_thresholds -- the thicknesses t_k above for n particles in the
 * world [lo, hi] (host only; no device is touched).  Zero fields of `border`
 * (nullable) take their defaults.  out: host, n_steps doubles.
 * Errors: VT_ERR_ARG.
 */
vt_status vt_border_thresholds(int64_t n, const double lo[3], const double hi[3], const vt_border *border,
                               double *out);

/*
 * vt_decompose -- the AUTOBORDER thicknesses and the task sizes.
 *   ctx          in/out as for vt_build (the decomposition keeps its own
 *                scratch in the context).
 *   pos          device, n x 3 positions (dtype), every particle in the world.
 *   periodic     1: periodic box [lo, hi); 0: bounded world [lo, hi].
 *   nt           host, tasks per axis, each >= 1.
 *   border       host, nullable (defaults).
 *   thick        host out, 6 per task: faces -x, +x, -y, +y, -z, +z.
 *   n_owned      host out (nullable), per task: owned particles.
 *   n_ghost      host out (nullable), per task: buffer particles (particle
 *                images inside the buffered box that the task does not own).
 * Synchronises the stream.  Errors: VT_ERR_ARG, VT_ERR_OOM, VT_ERR_HIP.
 */
vt_status vt_decompose(vt_ctx **ctx, const void *pos, vt_dtype dtype, int64_t n, const double lo[3],
                       const double hi[3], int32_t periodic, const int32_t nt[3], const vt_border *border,
                       double *thick, int64_t *n_owned, int64_t *n_ghost, void *stream);

/*
 * vt_decompose_pack -- the batch for vt_build: for each listed task (in list
 * order), its owned particles and then its buffer particles (periodic worlds:
 * shifted by whole periods next to the task), as FP64 (exact: the shifts are
 * multiples of L).
 *   thick        host, 6 per task (as from vt_decompose, or widened; at most
 *                the caps above).
 *   own_mask     device, n bytes or NULL: if given, a task owns only its
 *                particles with a nonzero byte, and its other particles are
 *                buffer particles (to re-run the incomplete cells of a first
 *                pass with wider buffers).
 *   tasks        host, n_list task indices, or NULL for every task in order.
 *   out_pos      device, cap x 3 doubles; out_gid device, cap int32 (the
 *                particle's index in pos).
 *   items        host out, n_list bounded items (box = the buffered box; in a
 *                bounded world the faces that lie on the world's faces are
 *                marked true walls).
 *   n_out        host out, particles written (or needed, if above cap).
 * A listed task must own at least one particle.  Synchronises the stream.
 * Errors: VT_ERR_ARG, VT_ERR_CAPACITY (cap too small; *n_out is the size
 * needed and nothing was written), VT_ERR_OOM, VT_ERR_HIP.
 */
vt_status vt_decompose_pack(vt_ctx **ctx, const void *pos, vt_dtype dtype, int64_t n, const double lo[3],
                            const double hi[3], int32_t periodic, const int32_t nt[3], const double *thick,
                            const uint8_t *own_mask, const int32_t *tasks, int32_t n_list, double *out_pos,
                            int32_t *out_gid, int64_t cap, vt_item *items, int64_t *n_out, void *stream);

/*
 * vt_decomposed_build -- the whole AUTOBORDER procedure on one device:
 * thicknesses (vt_decompose), all tasks packed and built as one batch, then up
 * to border->max_reruns more passes in which the cells still INCOMPLETE are
 * built again, owned alone by their tasks, whose buffers are widened by
 * border->widen (up to the caps).  Each particle's result is taken from the
 * last pass that computed its cell.  Afterwards the context answers vt_cells,
 * vt_density and vt_query in PARTICLE order (row i = particle i of pos, ids =
 * indices in pos), with VT_CELL_INCOMPLETE left on cells that the last pass
 * still could not complete; vt_query's n_retried and n_incomplete are those of
 * the last pass.  Other calls on the context return VT_ERR_STATE until it is
 * built again.
 *   opts         host, nullable: options of the builds (want_faces ignored).
 *   thick        host out (nullable), 6 per task: the first pass's thicknesses.
 *   pass_stats   host out (nullable), 4 int64 per pass, (max_reruns + 1) rows:
 *                tasks built, particles packed, cells built, cells left
 *                incomplete.
 *   n_passes     host out (nullable): passes run.
 * Synchronises the stream.  Errors: as vt_decompose and vt_build; a device
 * error of a pass's build (vt_query) is returned as is.
 */
vt_status vt_decomposed_build(vt_ctx **ctx, const void *pos, vt_dtype dtype, int64_t n, const double lo[3],
                              const double hi[3], int32_t periodic, const int32_t nt[3], const vt_border *border,
                              const vt_opts *opts, double *thick, int64_t *pass_stats, int32_t *n_passes,
                              void *stream);

/* n_owned_total and n_total of the last build (host, no sync). */
vt_status vt_sizes(vt_ctx *ctx, int64_t *n_owned_total, int64_t *n_total);

void vt_destroy(vt_ctx *ctx);

const char *vt_status_string(vt_status s);

#ifdef __cplusplus
}
#endif

#endif /* VT_H */

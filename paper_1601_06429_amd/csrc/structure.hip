// structure.hip -- the full tessellation structure of the owned cells: every cell's vertices and
// its faces as vertex loops (the full structure output the paper mentions in section 3's
// memory figures and section 4's summary).  Output is CSR in output-row order:
//   vertices  vert_off[row] .. vert_off[row + 1], absolute coordinates (seed + offset);
//   faces     face_off[row] .. face_off[row + 1], ascending by the id across the face: the
//             neighbour's global id, or -1 .. -6 for the walls -x, +x, -y, +y, -z, +z of a
//             bounded item; a particle's face is kept if the particle is in the cell's facet
//             list (the faces of area > area_eps V^(2/3), the neighbour list), a wall if its
//             area is above that threshold;
//   loops     loop_off[f] .. loop_off[f + 1], vertex indices local to the cell, counter-clockwise
//             seen from outside, starting at the face's smallest index.
// Two passes over the cells: the first counts (vertices, faces, loop entries) per row, the host
// scans the counts, and the second writes, after checking that it finds the counted sizes.  A
// cell of a periodic box with a topology record whose faces are all facets is counted from the
// record alone (its vertices, its faces, three loop entries per vertex).  Each pass is one wavefront per cell: the cell is
// rebuilt from its topology record (or its facets), its face loops are walked lane-parallel, one
// face per lane, and sorted by neighbour id with a wave bitonic sort.  Cells with more than 64
// vertices go to a large kernel with four vertex slots per lane.
#include "rebuild.h"

template <int VPL>
struct StructMem {
    double vp[64 * VPL][3];  // vertices, seed-relative
    uint32_t vt[64 * VPL];   // vertex triples (face slots)
    int32_t vidx[64 * VPL];  // local vertex index: rank among the cell's vertices
    int32_t flen[64 * VPL];  // loop length of each kept face slot, 0 otherwise
    int32_t frev[64 * VPL];  // 1: the walk runs clockwise seen from outside and is written reversed
    int32_t fl[64 * VPL];    // the cell's facet list (sorted indices of its neighbours)
    PolyMem<double, VPL> P;
};

struct StructArgs {
    CellSrc src;
    const DevItem *items;
    int n_items;
    const int32_t *cells;     // cell slot -> sorted index of its seed
    int64_t ncells;
    const int32_t *srow;      // sorted index -> output row
    const int32_t *sgid;      // sorted index -> global id
    const uint8_t *cstat;
    const double *cvol;
    const int32_t *queue;     // the clip's retry queue (cells with more than 64 vertices)
    int64_t queue_cap;
    int32_t *squeue;          // cells the normal kernel could not hold, for the large kernel
    int64_t squeue_cap;
    uint8_t *smark;           // per cell slot: 1 if the large kernel takes it
    uint32_t *counters;
    float area_eps;
    int write;                // 0: count, 1: write
    int64_t *nvert, *nface, *nloop;                  // counts per row (count pass)
    const int64_t *vert_off, *face_off, *loop_base;  // row offsets (write pass)
    double *verts;
    int32_t *face_nbr;
    int64_t *loop_off;
    int32_t *loop_vert;
};

__device__ __forceinline__ int item_of(const DevItem *items, int n_items, int64_t p) {
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].start <= p) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// the vertex after u on face f walking the face's loop: u's triple names the face that shares
// the edge leaving u along f; the next vertex is the other vertex on both faces
template <int VPL>
__device__ __forceinline__ int loop_next(const PolyMem<double, VPL> &SP, const uint32_t *vt, int f, const uint64_t *mf,
                                         int u) {
    const uint32_t t = vt[u];
    const int t0 = t & 0xFF, t1 = (t >> 8) & 0xFF, t2 = (t >> 16) & 0xFF;
    const int cf = (t0 == f) ? t2 : (t1 == f) ? t0 : t1;
    int nx = -1;
#pragma unroll
    for (int ww = 0; ww < VPL; ++ww) {
        uint64_t x = mf[ww] & SP.fm[cf][ww];
        if (ww == (u >> 6)) x &= ~(1ull << (u & 63));
        if (nx < 0 && x) nx = ww * 64 + __builtin_ctzll(x);
    }
    return nx;
}

template <typename PT4, int VPL, bool RETRY>
__global__ void __launch_bounds__(256) k_structure(StructArgs A) {
    using M = StructMem<VPL>;
    extern __shared__ char smem[];
    M &S = *reinterpret_cast<M *>(smem + (size_t)(threadIdx.x >> 6) * sizeof(M));
    const int lane = lane_id();
    const uint64_t lt = lanemask_lt();
    const int64_t nq = RETRY ? (int64_t)min((uint64_t)A.counters[CTR_QUEUE], (uint64_t)A.queue_cap) : 0;
    const int64_t ntodo =
        RETRY ? nq + (int64_t)min((uint64_t)A.counters[CTR_STRUCT_Q], (uint64_t)A.squeue_cap) : A.ncells;
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t w = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); w < ntodo; w += nwaves) {
        const int32_t c = RETRY ? (w < nq ? A.queue[w] : A.squeue[w - nq]) : (int32_t)w;
        const uint8_t st = A.cstat[c];
        const int32_t j0 = A.cells[c];
        const int64_t row = A.srow[j0];
        if (!RETRY) {
            // cells the clip kernel retried belong to the large kernel, as do (in the write pass)
            // the ones this kernel handed over in the count pass
            if (st & VT_CELL_RETRIED) continue;
            if (A.write && A.smark[c]) continue;
            if (!A.write && lane == 0) A.smark[c] = 0;
        }
        if (st & VT_CELL_FAILED) {
            if (!A.write && lane == 0) A.nvert[row] = A.nface[row] = A.nloop[row] = 0;
            continue;
        }
        const DevItem it = uniform_item(A.items[item_of(A.items, A.n_items, j0)]);
        if (!RETRY && !A.write && it.periodic) {
            const int nf = A.src.cnf[c], nv = A.src.cnv[c];
            if (nf >= 4 && nf <= VT_TOPO_FACES && nv >= 4 && nv <= 64 && A.src.ccnt[c] == nf) {
                if (lane == 0) {
                    A.nvert[row] = nv;
                    A.nface[row] = nf;
                    A.nloop[row] = 3 * nv;
                }
                continue;
            }
        }
        double xs[3];
        gpos<PT4>(A.src.spos, j0, xs[0], xs[1], xs[2]);
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
        const int rb = rebuild_cell<PT4, VPL, RETRY>(A.src, it, S.P, P, c, xs[0], xs[1], xs[2], blo, bhi);
        if (rb == REBUILD_OVERFLOW) {
            if (lane == 0) {
                if (!A.write) {
                    A.smark[c] = 1;
                    const uint32_t qi = atomicAdd(&A.counters[CTR_STRUCT_Q], 1u);
                    if ((int64_t)qi < A.squeue_cap) A.squeue[qi] = c;
                    else atomicOr(&A.counters[CTR_STATUS], VT_DEV_CAPACITY);
                } else {
                    // counted from its record, but rebuilt from its facets here: no room was
                    // counted for what this pass would write
                    atomicOr(&A.counters[CTR_STATUS], VT_DEV_TOPOLOGY);
                }
            }
            continue;
        }
        bool failed = rb == REBUILD_FAILED;
        // ---- vertices: positions, triples and local indices in LDS
        int nv = 0;
#pragma unroll
        for (int s = 0; s < VPL; ++s) {
            const uint64_t am = P.alive[s];
            const int u = s * 64 + lane;
            if (am & (1ull << lane)) {
                S.vp[u][0] = P.vx[s];
                S.vp[u][1] = P.vy[s];
                S.vp[u][2] = P.vz[s];
                S.vt[u] = P.vt[s];
                S.vidx[u] = nv + __popcll(am & lt);
            }
            nv += __popcll(am);
        }
        wave_sync();
        // ---- the cell's facet list in LDS
        const int32_t fcnt = min(A.src.ccnt[c], 64 * VPL);
        const int64_t frow = A.src.crow[c];
        for (int t = lane; t < fcnt; t += 64) S.fl[t] = A.src.stage_ids[frow + t];
        wave_sync();
        // ---- faces: walk each loop once (one face slot per lane) for its length, area and
        // orientation; a particle's face is kept if the particle is in the facet list, a wall
        // if its area is above the facet threshold (as the clip kernel takes it)
        const double amin = (double)(A.area_eps * exp2f(log2f((float)fabs(A.cvol[c])) * (2.0f / 3.0f)));
        uint64_t key[VPL];
        bool open_loop = false;
#pragma unroll
        for (int r = 0; r < VPL; ++r) {
            const int f = r * 64 + lane;
            key[r] = ~0ull;
            int keep_len = 0, rev = 0;
            if (P.fa[r] & (1ull << lane)) {
                uint64_t mf[VPL];
                int u0 = -1, m = 0;
#pragma unroll
                for (int ww = 0; ww < VPL; ++ww) {
                    mf[ww] = S.P.fm[f][ww];
                    m += __popcll(mf[ww]);
                    if (u0 < 0 && mf[ww]) u0 = ww * 64 + __builtin_ctzll(mf[ww]);
                }
                // Newell's normal: N = sum of v_k x v_k+1 over the loop (twice the vector area)
                double nx = 0.0, ny = 0.0, nz = 0.0;
                int u = u0, k = 0;
                for (; k < m && u >= 0; ++k) {
                    const int un = loop_next<VPL>(S.P, S.vt, f, mf, u);
                    if (un < 0) {
                        u = -1;
                        break;
                    }
                    const double *p = S.vp[u], *q = S.vp[un];
                    nx += p[1] * q[2] - p[2] * q[1];
                    ny += p[2] * q[0] - p[0] * q[2];
                    nz += p[0] * q[1] - p[1] * q[0];
                    u = un;
                }
                if (m > 0 && (k != m || u != u0)) open_loop = true;
                // the area along the face's outward unit normal: negative if the walk runs
                // clockwise seen from outside
                const P4<double> &pl = S.P.pl64[f];
                const double sa = 0.5 * (nx * pl.x + ny * pl.y + nz * pl.z) / sqrt(pl.x * pl.x + pl.y * pl.y + pl.z * pl.z);
                const int32_t tag = S.P.ptag[f];
                bool keep = false;
                if (tag >= 0) {
                    for (int t = 0; t < fcnt; ++t) keep = keep || S.fl[t] == tag;
                } else {
                    keep = fabs(sa) > amin;
                }
                if (m >= 3 && keep) {
                    rev = sa < 0.0 ? 1 : 0;
                    keep_len = m;
                    const int64_t g = tag >= 0 ? (int64_t)A.sgid[tag] : (int64_t)tag;
                    key[r] = ((uint64_t)(g + 16) << 32) | (uint64_t)f;
                }
            }
            S.flen[f] = keep_len;
            S.frev[f] = rev;
        }
        wave_sync();
        if (__ballot(open_loop) != 0ull) failed = true;
        if (failed) {
            if (lane == 0) {
                atomicOr(&A.counters[CTR_STATUS], VT_DEV_TOPOLOGY);
                if (!A.write) A.nvert[row] = A.nface[row] = A.nloop[row] = 0;
            }
            continue;
        }
        // kept faces in ascending order of the id across them
        bitonic_u64<VPL>(key);
        int nkept = 0, nloop = 0;
#pragma unroll
        for (int r = 0; r < VPL; ++r) {
            const bool k = key[r] != ~0ull;
            nkept += __popcll(__ballot(k));
            nloop += uni_i(wave_sum_i(k ? S.flen[(int)(key[r] & 0xFFFFull)] : 0));
        }
        if (!A.write) {
            if (lane == 0) {
                A.nvert[row] = nv;
                A.nface[row] = nkept;
                A.nloop[row] = nloop;
            }
            continue;
        }
        // ---- write pass: only into the room the count pass made for this row
        const int64_t vb = A.vert_off[row], fb = A.face_off[row], lb = A.loop_base[row];
        if (A.vert_off[row + 1] - vb != nv || A.face_off[row + 1] - fb != nkept || A.loop_base[row + 1] - lb != nloop) {
            if (lane == 0) atomicOr(&A.counters[CTR_STATUS], VT_DEV_TOPOLOGY);
            continue;
        }
#pragma unroll
        for (int s = 0; s < VPL; ++s) {
            const int u = s * 64 + lane;
            if (P.alive[s] & (1ull << lane)) {
                const int64_t o = 3 * (vb + S.vidx[u]);
                A.verts[o + 0] = xs[0] + S.vp[u][0];
                A.verts[o + 1] = xs[1] + S.vp[u][1];
                A.verts[o + 2] = xs[2] + S.vp[u][2];
            }
        }
        int64_t carry = 0;
#pragma unroll
        for (int r = 0; r < VPL; ++r) {
            const int e = r * 64 + lane;
            const bool k = e < nkept;
            const int f = k ? (int)(key[r] & 0xFFFFull) : 0;
            const int m = k ? S.flen[f] : 0;
            int tot;
            const int pre = wave_excl_scan(m, &tot);
            if (k) {
                const int64_t lo = lb + carry + pre;
                A.face_nbr[fb + e] = (int32_t)((int64_t)(key[r] >> 32) - 16);
                A.loop_off[fb + e] = lo;
                uint64_t mf[VPL];
                int u0 = -1;
#pragma unroll
                for (int ww = 0; ww < VPL; ++ww) {
                    mf[ww] = S.P.fm[f][ww];
                    if (u0 < 0 && mf[ww]) u0 = ww * 64 + __builtin_ctzll(mf[ww]);
                }
                const bool rv = S.frev[f] != 0;
                int u = u0;
                for (int t = 0; t < m; ++t) {
                    // reversed: the start vertex stays first, the rest run backwards
                    const int pos = (rv && t > 0) ? m - t : t;
                    A.loop_vert[lo + pos] = S.vidx[u];
                    u = loop_next<VPL>(S.P, S.vt, f, mf, u);
                }
            }
            carry += tot;
        }
    }
}

__global__ void k_store_last(int64_t *dst, const int64_t *src) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *src;
}

template <typename PT4, int VPL, bool RETRY>
static hipError_t launch_structure_one(vt_ctx *c, StructArgs &a, int wpb) {
    const size_t lds = sizeof(StructMem<VPL>) * (size_t)wpb;
    auto kern = k_structure<PT4, VPL, RETRY>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    int ncu = 0;
    hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device);
    if (ncu <= 0) ncu = 256;
    const int64_t blocks = RETRY ? (int64_t)ncu : (int64_t)ncu * 16 / wpb;
    kern<<<dim3((unsigned)blocks), dim3(64 * wpb), lds, c->stream>>>(a);
    return hipGetLastError();
}

static hipError_t structure_pass(vt_ctx *c, StructArgs &a) {
    hipError_t e;
    if (c->dtype == VT_F32) {
        e = launch_structure_one<float4, 1, false>(c, a, 4);
        if (e == hipSuccess) e = launch_structure_one<float4, 4, true>(c, a, 1);
    } else {
        e = launch_structure_one<double4, 1, false>(c, a, 4);
        if (e == hipSuccess) e = launch_structure_one<double4, 4, true>(c, a, 1);
    }
    return e;
}

static hipError_t reserve_structure(vt_ctx *c) {
    const int64_t n = c->n_owned;
    if (c->cap_struct >= n && c->st_cnt) return hipSuccess;
    (void)hipFree(c->st_cnt);
    (void)hipFree(c->st_lbase);
    (void)hipFree(c->smark);
    (void)hipFree(c->squeue);
    c->st_cnt = nullptr;
    c->st_lbase = nullptr;
    c->smark = nullptr;
    c->squeue = nullptr;
    c->cap_struct = 0;
    hipError_t e = hipMalloc(&c->st_cnt, sizeof(int64_t) * 3 * (size_t)n);
    if (e == hipSuccess) e = hipMalloc(&c->st_lbase, sizeof(int64_t) * (size_t)(n + 1));
    if (e == hipSuccess) e = hipMalloc(&c->smark, (size_t)n);
    if (e == hipSuccess) e = hipMalloc(&c->squeue, sizeof(int32_t) * (size_t)c->cap_retry);
    if (e == hipSuccess) c->cap_struct = n;
    return e;
}

void vt_struct_free(vt_ctx *c) {
    (void)hipFree(c->st_cnt);
    (void)hipFree(c->st_lbase);
    (void)hipFree(c->smark);
    (void)hipFree(c->squeue);
    c->st_cnt = nullptr;
    c->st_lbase = nullptr;
    c->smark = nullptr;
    c->squeue = nullptr;
    c->cap_struct = 0;
}

// Count, scan, and (if the capacities suffice) write.  sizes[] gets the totals of vertices,
// faces and loop entries; *fits is false when one of them exceeds its capacity (then only the
// offsets are written).  Synchronizes the stream to read the totals.
hipError_t vt_launch_structure(vt_ctx *c, int64_t *vert_off, double *verts, int64_t vert_cap, int64_t *face_off,
                               int32_t *face_nbr, int64_t face_cap, int64_t *loop_off, int32_t *loop_vert,
                               int64_t loop_cap, int64_t sizes[3], bool *fits) {
    const int64_t n = c->n_owned;
    hipError_t e = reserve_structure(c);
    if (e != hipSuccess) return e;
    StructArgs a;
    a.src = CellSrc{c->spos, c->ctopo, c->cnf, c->cnv, c->n_total, c->crow, c->ccnt, c->stage_ids, c->counters};
    a.items = c->items;
    a.n_items = c->n_items;
    a.cells = c->cells;
    a.ncells = n;
    a.srow = c->srow;
    a.sgid = c->sgid;
    a.cstat = c->cstat;
    a.cvol = c->cvol;
    a.queue = c->queue;
    a.queue_cap = c->cap_retry;
    a.squeue = c->squeue;
    a.squeue_cap = c->cap_retry;
    a.smark = c->smark;
    a.counters = c->counters;
    a.area_eps = c->opts.area_eps > 0 ? c->opts.area_eps : 1e-12f;
    a.write = 0;
    a.nvert = c->st_cnt;
    a.nface = c->st_cnt + n;
    a.nloop = c->st_cnt + 2 * n;
    a.vert_off = vert_off;
    a.face_off = face_off;
    a.loop_base = c->st_lbase;
    a.verts = verts;
    a.face_nbr = face_nbr;
    a.loop_off = loop_off;
    a.loop_vert = loop_vert;
    // counts start at zero (a row no kernel reaches keeps an empty structure)
    e = vt_launch_zero_u32((uint32_t *)c->st_cnt, 6 * n, c->stream);
    if (e == hipSuccess) e = vt_launch_zero_u32(c->counters + CTR_STRUCT_Q, 1, c->stream);
    if (e == hipSuccess) e = structure_pass(c, a);
    if (e == hipSuccess) e = vt_launch_scan_i64(a.nvert, vert_off, n, c->scan_tmp, c->stream);
    if (e == hipSuccess) e = vt_launch_scan_i64(a.nface, face_off, n, c->scan_tmp, c->stream);
    if (e == hipSuccess) e = vt_launch_scan_i64(a.nloop, c->st_lbase, n, c->scan_tmp, c->stream);
    if (e != hipSuccess) return e;
    int64_t tot[3];
    e = hipMemcpyAsync(&tot[0], vert_off + n, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&tot[1], face_off + n, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&tot[2], c->st_lbase + n, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return e;
    for (int k = 0; k < 3; ++k) sizes[k] = tot[k];
    *fits = tot[0] <= vert_cap && tot[1] <= face_cap && tot[2] <= loop_cap && verts && face_nbr && loop_off && loop_vert;
    if (!*fits) return hipSuccess;
    a.write = 1;
    e = structure_pass(c, a);
    if (e == hipSuccess) {
        k_store_last<<<1, 64, 0, c->stream>>>(loop_off + tot[1], c->st_lbase + n);
        e = hipGetLastError();
    }
    return e;
}

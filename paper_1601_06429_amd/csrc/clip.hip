// clip.hip -- one Voronoi cell per wavefront: neighbour search and clipping.
//
// The paper's cell (section 1: the region closer to the particle than to any
// other; section 2: volume from the facets, neighbours = particles sharing a
// facet, periodic conditions) is built by clipping the box around the seed
// (the bisectors with the seed's own periodic images, or the walls of a
// bounded world) with the bisector half-spaces {y : y.D <= |D|^2/2} of the
// other particles in increasing distance.  A particle farther than 2R (R the
// largest vertex distance) cannot cut the cell, so the search proceeds in
// shells [r_done, r_next) over Morton-cell ranges of the sorted particles and
// stops once 2R <= r_done (the security radius).
//
// Per shell the candidates (at most VT_CAND_MAX) are gathered into LDS with
// lanes = particles, sorted by quantised distance with a wave bitonic sort,
// and applied one by one; the loop stops at the first candidate beyond 2R.
// Cells that outgrow 64 vertices are handed to a second, persistent kernel
// with room for 256.
#include <algorithm>

#include "poly.h"

#define WAVE 64

// Face slots of the polytope: the fast kernel's cells have at most 64 vertices, so at most 34 faces,
// and its topology record holds VT_TOPO_FACES; fewer slots than 64 leave LDS for a fourth wave per SIMD.
__host__ __device__ constexpr int clip_faces(int vpl) { return vpl == 1 ? VT_TOPO_FACES : 64 * vpl; }

// The large kernel's sweeps cover their shell with boxes refined where they hold many particles
// (cover_fine): two lists of boxes, the input and the output of a refinement round.
#define VT_FINE_CAP 512
struct FineLists {
    uint64_t pk[2][VT_FINE_CAP];  // unwrapped box coordinates and level, packed (pack_box)
    int32_t b[2][VT_FINE_CAP];    // particle range start
    int32_t n[2][VT_FINE_CAP];    // range length; the prefix of the lengths once the list is final
    float d[2][VT_FINE_CAP];      // squared distance of the box from the seed, rounded down
};

template <typename T, int VPL>
struct ClipMemBase {
    union {
        struct {
            double cd[VT_CAND_MAX][3];   // candidate separations (FP64)
            int32_t cid[VT_CAND_MAX];    // candidate sorted index
            uint32_t ckey[VT_CAND_MAX];  // quantised d^2 << 8 | slot
        } c;
        struct {
            double vp[64 * VPL][3];      // final vertex positions (FP64)
            uint32_t vt[64 * VPL];       // final vertex triples
            double fa[64 * VPL];         // facet area
            double fc[64 * VPL][3];      // facet centroid (seed-relative)
        } f;
        struct {
            double vp[64 * VPL][3];      // search: vertex positions (FP64)
            double ve[64 * VPL];         // their error bounds (mixed path; 0 in FP64)
            double vr[64 * VPL];         // radius of each vertex's empty sphere, widened for rounding
        } s;
    } u;
    int32_t rb[216];                     // gather: cell range starts
    int32_t rp[216];                     // gather: prefix of range lengths
    int32_t hist[64];                    // gather: d^2 histogram of the shell
    PolyMem<T, VPL, clip_faces(VPL)> P;
};
template <typename T, int VPL>
struct ClipMem : ClipMemBase<T, VPL> {};
template <typename T>
struct ClipMem<T, 4> : ClipMemBase<T, 4> {
    FineLists fine;
};

// a box of the Morton grid at `level` by its unwrapped integer coordinates (each within 2^17 of
// the grid, 18 bits) and its level, in one word
__device__ __forceinline__ uint64_t pack_box(const int u[3], int level) {
    return ((uint64_t)(uint32_t)(u[0] + (1 << 17)) << 46) | ((uint64_t)(uint32_t)(u[1] + (1 << 17)) << 28) |
           ((uint64_t)(uint32_t)(u[2] + (1 << 17)) << 10) | (uint64_t)(uint32_t)level;
}
__device__ __forceinline__ int unpack_box(uint64_t pk, int u[3]) {
    u[0] = (int)((pk >> 46) & 0x3FFFFu) - (1 << 17);
    u[1] = (int)((pk >> 28) & 0x3FFFFu) - (1 << 17);
    u[2] = (int)((pk >> 10) & 0x3FFFFu) - (1 << 17);
    return (int)(pk & 0x1Fu);
}

struct ClipArgs {
    const void *spos;
    const uint64_t *skey;
    const int32_t *sgid;
    const int32_t *tab;
    const DevItem *items;
    int n_items;
    const int32_t *cells;
    int64_t ncells;
    const int32_t *queue;     // large kernel: cells to do (count in counters[CTR_QUEUE])
    int32_t *queue_out;       // fast kernel: cells that outgrow it
    int64_t queue_cap;
    uint32_t *counters;
    double *cvol;
    double *crad;             // largest vertex distance of each cell
    int32_t *ccnt;
    int64_t *crow;
    uint8_t *cstat;
    int32_t *cnv, *cnt;
    int32_t *ctopo;           // fast kernel: topology record per cell (VT_TOPO_STRIDE words)
    int32_t *cnf;             // faces in the record, 0 = no record
    int32_t *stage_ids;
    double *stage_area;
    double *stage_cen;
    int64_t row_base;
    int64_t fstride;
    int want_faces;
    float radius_factor;
    float area_eps;
    int xcd_segments;         // fast kernel: 1 = one queue; VT_XCD_SEGMENTS = per-XCD Morton segments
};

__device__ __forceinline__ int find_item_d(const DevItem *items, int n_items, int64_t p) {
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (items[mid].start <= p) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int32_t lower_bound_key(const uint64_t *skey, int32_t a, int32_t c, uint64_t k) {
    while (a < c) {
        int32_t mid = (a + c) >> 1;
        if (skey[mid] < k) a = mid + 1; else c = mid;
    }
    return a;
}

// the low 10 bits of x to every third bit (Morton codes of levels up to 10 fit 32 bits)
__device__ __forceinline__ uint32_t spread3_10(uint32_t x) {
    x &= 0x3ffu;
    x = (x | (x << 16)) & 0x030000ffu;
    x = (x | (x << 8)) & 0x0300f00fu;
    x = (x | (x << 4)) & 0x030c30c3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

// sorted-index range of the Morton cell with code m at level l of item `ib`
__device__ __forceinline__ void cell_range_m(const ClipArgs &A, const DevItem &it, int ib, int l, uint64_t m,
                                             int32_t &b, int32_t &e) {
    const int T = it.T;
    if (l <= T) {
        const int sh = 3 * (T - l);
        b = A.tab[it.tab_off + (int64_t)(m << sh)];
        e = A.tab[it.tab_off + (int64_t)((m + 1) << sh)];
    } else {
        const uint64_t mT = m >> (3 * (l - T));
        const int32_t lo = A.tab[it.tab_off + (int64_t)mT], hi = A.tab[it.tab_off + (int64_t)mT + 1];
        const int sh = 3 * (VT_MORTON_BITS - l);
        const uint64_t base = (uint64_t)ib << VT_LOCAL_KEY_BITS;
        b = lower_bound_key(A.skey, lo, hi, base | (m << sh));
        e = lower_bound_key(A.skey, b, hi, base | ((m + 1) << sh));
    }
}

// sorted-index range of the Morton cell (cx, cy, cz) at level l of item `ib`
__device__ __forceinline__ void cell_range(const ClipArgs &A, const DevItem &it, int ib, int l, uint64_t cx,
                                           uint64_t cy, uint64_t cz, int32_t &b, int32_t &e) {
    uint64_t m = vt_morton(cx, cy, cz);
    const int T = it.T;
    if (l <= T) {
        int sh = 3 * (T - l);
        b = A.tab[it.tab_off + (int64_t)(m << sh)];
        e = A.tab[it.tab_off + (int64_t)((m + 1) << sh)];
    } else {
        uint64_t mT = m >> (3 * (l - T));
        int32_t lo = A.tab[it.tab_off + (int64_t)mT], hi = A.tab[it.tab_off + (int64_t)mT + 1];
        int sh = 3 * (VT_MORTON_BITS - l);
        uint64_t base = (uint64_t)ib << VT_LOCAL_KEY_BITS;
        b = lower_bound_key(A.skey, lo, hi, base | (m << sh));
        e = lower_bound_key(A.skey, b, hi, base | ((m + 1) << sh));
    }
}

// local mean spacing around particle j0, from the particle count of the
// smallest Morton cell containing it that holds between 8 and 64 particles.
// The counts of its cells at levels T .. T-3 are prefix differences in the
// dense level-T table, read with independent loads; coarser levels and the
// finer ones a crowded level-T cell needs (binary searches) follow as before.
__device__ double local_spacing(const ClipArgs &A, const DevItem &it, int ib, int32_t j0) {
    const uint64_t lmask = (1ull << VT_LOCAL_KEY_BITS) - 1;
    const uint64_t key = A.skey[j0] & lmask;
    const int T = it.T;
    int cnt4[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const int l = T - d < 0 ? 0 : T - d;
        const int sh = 3 * (T - l);
        const uint64_t ml = key >> (3 * (VT_MORTON_BITS - l));
        cnt4[d] = A.tab[it.tab_off + (int64_t)((ml + 1) << sh)] - A.tab[it.tab_off + (int64_t)(ml << sh)];
    }
    int l = T, cnt = cnt4[0];
#pragma unroll
    for (int d = 1; d < 4; ++d)
        if (cnt < 8 && l > 0) {
            --l;
            cnt = cnt4[d];
        }
    int32_t b = 0, e = 0;
    while (cnt < 8 && l > 0) {
        --l;
        const int sh = 3 * (T - l);
        const uint64_t ml = key >> (3 * (VT_MORTON_BITS - l));
        cnt = A.tab[it.tab_off + (int64_t)((ml + 1) << sh)] - A.tab[it.tab_off + (int64_t)(ml << sh)];
    }
    if (cnt > 64 && l == T) {
        const uint64_t m = key >> (3 * (VT_MORTON_BITS - T));
        b = A.tab[it.tab_off + (int64_t)m];
        e = A.tab[it.tab_off + (int64_t)m + 1];
    }
    const uint64_t base = (uint64_t)ib << VT_LOCAL_KEY_BITS;
    while (cnt > 64 && l >= T && l < VT_MORTON_BITS) {
        ++l;
        const int sh = 3 * (VT_MORTON_BITS - l);
        const uint64_t ml = key >> sh;
        const int32_t nb = lower_bound_key(A.skey, b, e, base | (ml << sh));
        const int32_t ne = lower_bound_key(A.skey, nb, e, base | ((ml + 1) << sh));
        b = nb;
        e = ne;
        cnt = e - b;
    }
    const double cs = it.S / (double)(1ll << l);
    return cs / cbrt((double)(cnt > 0 ? cnt : 1));
}

template <typename PT4>
__device__ __forceinline__ void load_pos(const void *spos, int32_t j, double &x, double &y, double &z) {
    PT4 p = ((const PT4 *)spos)[j];
    x = (double)p.x;
    y = (double)p.y;
    z = (double)p.z;
}

template <typename T, typename PT4, int VPL, bool RETRY>
__device__ __forceinline__ void clip_cells(const ClipArgs &A) {
    using M = ClipMem<T, VPL>;
    constexpr int VMAX = 64 * VPL;
    extern __shared__ char smem[];
    const int wid = threadIdx.x >> 6;
    M &S = *reinterpret_cast<M *>(smem + (size_t)wid * sizeof(M));
    const int lane = lane_id();
    const uint64_t lt = lanemask_lt();
    const uint64_t mybit = 1ull << lane;

    const int64_t ntodo = RETRY ? (int64_t)min((uint64_t)A.counters[CTR_QUEUE], (uint64_t)A.queue_cap) : A.ncells;
    // Work distribution.  The large kernel (and the one-queue mapping) hands out cells from one
    // counter.  With XCD segments, the cells (in Morton order) are cut into nseg contiguous
    // segments; a wavefront of workgroup b starts on segment b % nseg, the XCD its workgroup runs
    // on, so each XCD's L2 serves one compact region, and when that segment is exhausted the
    // wavefront moves to the next one, until it has found all nseg exhausted.  Every counter only
    // grows and a segment is left only once exhausted, so every cell is taken exactly once and
    // every wavefront exits after at most nseg exhausted segments.
    const int nseg = RETRY ? 1 : A.xcd_segments;
    int seg = RETRY ? 0 : (int)(blockIdx.x % (unsigned)nseg);
    int left = nseg;

    for (;;) {
        const int64_t s_lo = RETRY ? 0 : ntodo * seg / nseg, s_hi = RETRY ? ntodo : ntodo * (seg + 1) / nseg;
        int64_t w = 0;
        if (lane == 0) {
            uint32_t *ctr = RETRY ? &A.counters[CTR_RETRY] : nseg == 1 ? &A.counters[CTR_CELL] : &A.counters[CTR_SEG0 + seg];
            w = (int64_t)atomicAdd(ctr, 1u);
        }
        w = (int64_t)uni_i((int)__shfl((long long)w, 0)) + s_lo;
        if (w >= s_hi) {
            if (--left == 0) break;
            seg = seg + 1 == nseg ? 0 : seg + 1;
            continue;
        }
        const int32_t cslot = uni_i(RETRY ? A.queue[w] : (int32_t)w);
        const int32_t j0 = uni_i(A.cells[cslot]);
        const int bi = uni_i(find_item_d(A.items, A.n_items, j0));
        const DevItem it = uniform_item(A.items[bi]);
        double sx, sy, sz;
        load_pos<PT4>(A.spos, j0, sx, sy, sz);
        sx = uni_d(sx);
        sy = uni_d(sy);
        sz = uni_d(sz);
        const double xs[3] = {sx, sy, sz};

        // ---------------- initial polytope: the box around the seed
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
        Poly<T, VPL, clip_faces(VPL)> P;
        P.init_box(S.P, blo, bhi);

        uint32_t dup = 0;
        bool overflow = false, corrupt = false;
        int ntested = 0;
        int ncut = 0;  // planes that have cut the cell so far

        // ---------------- search and clip
        // The first shell [0, r0) is fitted to LDS (a d^2 histogram picks a radius
        // holding at most VT_CAND_MAX particles) and applied nearest first.  Each
        // later shell reaches for the security radius 2R but grows the searched
        // radius by at most 2x; a shell that fits in LDS is applied nearest first,
        // a larger one is swept once with lanes = particles: a plane that cuts no
        // vertex of the current cell is dropped (the cell only shrinks, so it never
        // would cut it), the survivors are applied nearest first.
        double r_done = 0.0;
        double r_next = uni_d((double)A.radius_factor * local_spacing(A, it, bi, j0));
        const double Lmin = fmin(it.L[0], fmin(it.L[1], it.L[2]));
        const double r_cap = it.periodic ? 0.5 * Lmin
                                         : sqrt(it.L[0] * it.L[0] + it.L[1] * it.L[1] + it.L[2] * it.L[2]) * 1.0001;
        if (r_next > r_cap) r_next = r_cap;
        bool complete = false;

        // Morton cells that may hold particles with rmin <= d < r: cells of side in
        // [r/2, r), pruned by their distance to the seed (boxes widened by one
        // quantum, the rounding of the keys), empty ranges dropped; ranges go to
        // S.rb / S.rp compacted.  Returns the number of ranges; *total the particles.
        // With `prune` (sweeps and later passes), a box is also dropped when no vertex's empty sphere
        // (centre v, radius |v| widened, staged by stage_search in S.u.s)
        // reaches it: a particle cuts the current cell only if it lies in such a
        // sphere, and the cell only shrinks, so no particle of the box ever will.
        const double invL[3] = {1.0 / it.L[0], 1.0 / it.L[1], 1.0 / it.L[2]};
        // the cell's vertices for the search-side tests: positions, error bounds and the radius of
        // each vertex's empty sphere (|v|, widened for rounding and, mixed, the vertex error bound)
        auto stage_search = [&]() {
#pragma unroll
            for (int s = 0; s < VPL; ++s)
                if (P.alive[s] & mybit) {
                    const double x = (double)P.vx[s], y = (double)P.vy[s], z = (double)P.vz[s];
                    S.u.s.vp[s * 64 + lane][0] = x;
                    S.u.s.vp[s * 64 + lane][1] = y;
                    S.u.s.vp[s * 64 + lane][2] = z;
                    S.u.s.ve[s * 64 + lane] = (double)P.ve[s];
                    S.u.s.vr[s * 64 + lane] = sqrt(x * x + y * y + z * z) * (1.0 + 1e-7) + 2.0 * (double)P.ve[s];
                }
            wave_sync();
        };
        auto cover = [&](double r, double rmin, int &total, bool prune) -> int {
            int lvl = 0;
            double c = it.S;
            while (lvl < VT_MORTON_BITS && c >= r) {
                c *= 0.5;
                ++lvl;
            }
            const int sh = VT_MORTON_BITS - lvl;
            const int ncl = 1 << lvl;
            const double quantum = it.S / (double)(1 << VT_MORTON_BITS);
            int a0[3], na[3];
            bool all_img = false;  // a periodic window that spans the whole period along some axis
            for (int a = 0; a < 3; ++a) {
                int64_t q0 = vt_qraw(xs[a] - r, it.lo[a], it.inv_res) - 1;
                int64_t q1 = vt_qraw(xs[a] + r, it.lo[a], it.inv_res) + 1;
                int64_t i0 = q0 >> sh, i1 = q1 >> sh;
                if (it.periodic) {
                    if (i1 - i0 + 1 >= ncl) {
                        i0 = 0;
                        i1 = ncl - 1;
                        all_img = true;
                    }
                } else {
                    if (i0 < 0) i0 = 0;
                    if (i1 > ncl - 1) i1 = ncl - 1;
                }
                a0[a] = (int)i0;
                na[a] = i1 >= i0 ? (int)(i1 - i0 + 1) : 0;  // at most 6
            }
            const int nbox = na[0] * na[1] * na[2];
            const double r2 = r * r, rmin2 = rmin * rmin;
            // box u along axis a, widened by one quantum (the rounding of the keys), relative to the
            // seed: [u c + off_lo[a], u c + off_lo[a] + cw]
            const double cw = c + 2.0 * quantum;
            double off_lo[3];
            for (int a = 0; a < 3; ++a) off_lo[a] = it.lo[a] - quantum - xs[a];
            // lane -> (ix, iy, iz): k = ix + na0 (iy + na1 iz) with k < 216, so (k + 1/2) / n in FP32 is
            // at least 1/72 away from an integer and truncates to the exact quotient
            const int na01 = na[0] * na[1];
            const float inv0 = 1.0f / (float)(na[0] > 0 ? na[0] : 1), inv01 = 1.0f / (float)(na01 > 0 ? na01 : 1);
            int count = 0;
            // only vertices whose (widened) sphere reaches past rmin matter: every point of the
            // sphere of v lies within |v| + vr <= 2 vr of the seed, and the shell starts at rmin
            uint64_t farv[VPL];
#pragma unroll
            for (int s_ = 0; s_ < VPL; ++s_) {
                farv[s_] = P.alive[s_];
                if (prune)
                    farv[s_] = __ballot((P.alive[s_] & mybit) && 2.0 * S.u.s.vr[s_ * 64 + lane] * (1.0 + 1e-7) >= rmin);
            }
            for (int base = 0; base < nbox; base += WAVE) {
                const int k = base + lane;
                bool keep = false;
                int32_t b = 0, e = 0;
                if (k < nbox) {
                    const int iz = (int)(((float)k + 0.5f) * inv01);
                    const int rem = k - iz * na01;
                    const int iy = (int)(((float)rem + 0.5f) * inv0);
                    const int u[3] = {a0[0] + rem - iy * na[0], a0[1] + iy, a0[2] + iz};
                    // per axis: nearest and farthest distance from the seed to the box (a lower / upper
                    // bound for the minimum-image distance of every particle in it)
                    double dmin2 = 0.0, dmax2 = 0.0;
                    if (!all_img) {
                        // the window [a0, a0 + na) is centred on the seed: its unwrapped boxes are the
                        // nearest images
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            const double bl = fma((double)u[a], c, off_lo[a]), bh = bl + cw;
                            const double dn = fmax(0.0, fmax(bl, -bh));
                            const double df = fmax(fabs(bl), fabs(bh));
                            dmin2 = fma(dn, dn, dmin2);
                            dmax2 = fma(df, df, dmax2);
                        }
                    } else {
                        // a window that spans the whole period (wrapped to [0, ncl)) needs the three images
                        for (int a = 0; a < 3; ++a) {
                            double dn = 1e300, df = 1e300;
                            const bool img = na[a] == ncl;
                            for (int sh_ = -1; sh_ <= 1; ++sh_) {
                                if (sh_ != 0 && !img) continue;
                                const double lo_ = fma((double)u[a], c, off_lo[a]) + sh_ * it.L[a];
                                const double hi_ = lo_ + cw;
                                dn = fmin(dn, fmax(0.0, fmax(lo_, -hi_)));
                                df = fmin(df, fmax(fabs(lo_), fabs(hi_)));
                            }
                            dmin2 += dn * dn;
                            dmax2 += df * df;
                        }
                    }
                    keep = dmin2 < r2 && dmax2 >= rmin2;
                    if (keep && prune && !all_img) {
                        double bl[3], bh[3];
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            bl[a] = fma((double)u[a], c, off_lo[a]);
                            bh[a] = bl[a] + cw;
                        }
                        // does the empty sphere of vertex k reach the box?
                        auto reaches = [&](int k) -> bool {
                            const double *v = S.u.s.vp[k];
                            const double ex = fmax(0.0, fmax(bl[0] - v[0], v[0] - bh[0]));
                            const double ey = fmax(0.0, fmax(bl[1] - v[1], v[1] - bh[1]));
                            const double ez = fmax(0.0, fmax(bl[2] - v[2], v[2] - bh[2]));
                            const double rv = S.u.s.vr[k];
                            return ex * ex + ey * ey + ez * ez < rv * rv;
                        };
                        bool reached = false;
#pragma unroll
                        for (int s_ = 0; s_ < VPL; ++s_) {
                            // two vertices per step, their loads issued together
                            uint64_t m = farv[s_];
                            while (m && !reached) {
                                const int k0 = __builtin_ctzll(m);
                                m &= m - 1;
                                const int k1 = m ? __builtin_ctzll(m) : k0;
                                m &= m - 1;
                                const bool r0 = reaches(s_ * 64 + k0), r1 = reaches(s_ * 64 + k1);
                                reached = r0 || r1;
                            }
                        }
                        keep = reached;
                    }
                    if (keep) {
                        uint32_t cc[3];
                        for (int a = 0; a < 3; ++a) cc[a] = (uint32_t)(it.periodic ? (u[a] & (ncl - 1)) : u[a]);
                        uint64_t mc;
                        if (lvl <= 10)
                            mc = (uint64_t)((spread3_10(cc[0]) << 2) | (spread3_10(cc[1]) << 1) | spread3_10(cc[2]));
                        else
                            mc = vt_morton(cc[0], cc[1], cc[2]);
                        cell_range_m(A, it, bi, lvl, mc, b, e);
                        keep = e > b;
                    }
                }
                const uint64_t km = __ballot(keep);
                if (keep) {
                    const int slot = count + __popcll(km & lt);
                    S.rb[slot] = b;
                    S.rp[slot] = e - b;  // length for now
                }
                count += __popcll(km);
            }
            wave_sync();
            // lengths -> exclusive prefix
            int carry = 0;
            for (int base = 0; base < count; base += WAVE) {
                const int k = base + lane;
                const int len = k < count ? S.rp[k] : 0;
                int tot;
                const int pre = wave_excl_scan(len, &tot);
                if (k < count) S.rp[k] = carry + pre;
                carry += tot;
            }
            wave_sync();
            total = uni_i(carry);
            return uni_i(count);
        };
        // Particles f = nb + lane of a cover, chunk by chunk in order (nb = 0, 64, ...): its ranges
        // start at pre[0..ncq) (strictly increasing from pre[0] = 0, no range empty) at sorted
        // indices rbase[], and rcur holds the range of the previous chunk's last particle (0 before
        // the first chunk).  The starts of the next 64 ranges, as bits of the chunk, give each lane
        // its range by a population count: one LDS round trip and a wave OR per chunk, instead of a
        // binary search per particle.
        auto chunk_loc = [&](const int32_t *pre, const int32_t *rbase, int ncq, int &rcur, int nb) -> int32_t {
            const int k = rcur + 1 + lane;
            const int32_t s_ = k < ncq ? pre[k] - nb : 64;
            const uint64_t starts = wave_or_u64(s_ >= 0 && s_ < 64 ? 1ull << s_ : 0ull);
            const int r = rcur + __popcll(starts & ((2ull << lane) - 1ull));
            rcur = uni_i(__builtin_amdgcn_readlane(r, 63));
            return rbase[r] + (nb + lane - pre[r]);
        };
        // The large kernel's sweeps: its cells lie next to dense halos, whose thousands of particles
        // sit in a few covering boxes that some vertex's empty sphere reaches at their edge.  The
        // boxes of the plain cover that hold more than 128 particles are split into their eight
        // children, one Morton level finer, for up to three rounds while the list has room; a child
        // is kept when it meets the shell [rmin, r), some vertex's empty sphere reaches it (the test
        // of the plain cover: a particle cuts the cell only from inside such a sphere, and the cell
        // only shrinks) and it holds particles.  The kept boxes are sorted by their distance from the
        // seed, so the sweep takes the shell nearest first and stops at the first box beyond 2R.
        // Returns the number of boxes (their ranges in S.fine.b / .n of list `fin`, .n the prefix of
        // the lengths, .d the squared distances), or -1 for a shell that wraps around the period
        // (the plain cover serves it).
        int fin = 0;
        auto cover_fine = [&](double r, double rmin, int &total) -> int {
            if constexpr (RETRY && VPL > 1) {
                int lvl = 0;
                double c = it.S;
                while (lvl < VT_MORTON_BITS && c >= r) {
                    c *= 0.5;
                    ++lvl;
                }
                const int sh = VT_MORTON_BITS - lvl;
                const int ncl = 1 << lvl;
                const double quantum = it.S / (double)(1 << VT_MORTON_BITS);
                int a0[3], na[3];
                for (int a = 0; a < 3; ++a) {
                    int64_t i0 = (vt_qraw(xs[a] - r, it.lo[a], it.inv_res) - 1) >> sh;
                    int64_t i1 = (vt_qraw(xs[a] + r, it.lo[a], it.inv_res) + 1) >> sh;
                    if (it.periodic) {
                        if (i1 - i0 + 1 >= ncl) return -1;
                    } else {
                        if (i0 < 0) i0 = 0;
                        if (i1 > ncl - 1) i1 = ncl - 1;
                    }
                    a0[a] = (int)i0;
                    na[a] = i1 >= i0 ? (int)(i1 - i0 + 1) : 0;
                }
                const double r2 = r * r, rmin2 = rmin * rmin;
                double off_lo[3];
                for (int a = 0; a < 3; ++a) off_lo[a] = it.lo[a] - quantum - xs[a];
                uint64_t farv[VPL];
#pragma unroll
                for (int s_ = 0; s_ < VPL; ++s_)
                    farv[s_] = __ballot((P.alive[s_] & mybit) && 2.0 * S.u.s.vr[s_ * 64 + lane] * (1.0 + 1e-7) >= rmin);
                // box u at level l (unwrapped coordinates): does it meet the shell and is it reached
                // by a vertex's empty sphere?  dmin2: its squared distance from the seed
                auto box_test = [&](int l, const int u[3], double &dmin2) -> bool {
                    const double cl = it.S / (double)(1 << l), cw = cl + 2.0 * quantum;
                    double bl[3], bh[3], dmax2 = 0.0;
                    dmin2 = 0.0;
                    for (int a = 0; a < 3; ++a) {
                        bl[a] = fma((double)u[a], cl, off_lo[a]);
                        bh[a] = bl[a] + cw;
                        const double dn = fmax(0.0, fmax(bl[a], -bh[a]));
                        const double df = fmax(fabs(bl[a]), fabs(bh[a]));
                        dmin2 = fma(dn, dn, dmin2);
                        dmax2 = fma(df, df, dmax2);
                    }
                    if (!(dmin2 < r2 && dmax2 >= rmin2)) return false;
                    bool reached = false;
#pragma unroll
                    for (int s_ = 0; s_ < VPL; ++s_) {
                        uint64_t m = farv[s_];
                        while (m && !reached) {
                            const int kv = __builtin_ctzll(m);
                            m &= m - 1;
                            const double *v = S.u.s.vp[s_ * 64 + kv];
                            const double ex = fmax(0.0, fmax(bl[0] - v[0], v[0] - bh[0]));
                            const double ey = fmax(0.0, fmax(bl[1] - v[1], v[1] - bh[1]));
                            const double ez = fmax(0.0, fmax(bl[2] - v[2], v[2] - bh[2]));
                            const double rv = S.u.s.vr[s_ * 64 + kv];
                            reached = ex * ex + ey * ey + ez * ez < rv * rv;
                        }
                    }
                    return reached;
                };
                auto box_range = [&](int l, const int u[3], int32_t &b, int32_t &e) {
                    const int n_l = 1 << l;
                    uint32_t cc[3];
                    for (int a = 0; a < 3; ++a) cc[a] = (uint32_t)(it.periodic ? (u[a] & (n_l - 1)) : u[a]);
                    const uint64_t mc = l <= 10 ? (uint64_t)((spread3_10(cc[0]) << 2) | (spread3_10(cc[1]) << 1) |
                                                             spread3_10(cc[2]))
                                                : vt_morton(cc[0], cc[1], cc[2]);
                    cell_range_m(A, it, bi, l, mc, b, e);
                };
                // the coarse window (at most 216 boxes)
                int cur = 0, ncur = 0;
                const int nbox = na[0] * na[1] * na[2], na01 = na[0] * na[1];
                const float inv0 = 1.0f / (float)(na[0] > 0 ? na[0] : 1), inv01 = 1.0f / (float)(na01 > 0 ? na01 : 1);
                for (int base = 0; base < nbox; base += WAVE) {
                    const int k = base + lane;
                    bool keep = false;
                    int32_t b = 0, e = 0;
                    int u[3] = {0, 0, 0};
                    double dm = 0.0;
                    if (k < nbox) {
                        const int iz = (int)(((float)k + 0.5f) * inv01);
                        const int rem = k - iz * na01;
                        const int iy = (int)(((float)rem + 0.5f) * inv0);
                        u[0] = a0[0] + rem - iy * na[0];
                        u[1] = a0[1] + iy;
                        u[2] = a0[2] + iz;
                        keep = box_test(lvl, u, dm);
                        if (keep) {
                            box_range(lvl, u, b, e);
                            keep = e > b;
                        }
                    }
                    const uint64_t km = __ballot(keep);
                    if (keep) {
                        const int slot = ncur + __popcll(km & lt);
                        S.fine.pk[0][slot] = pack_box(u, lvl);
                        S.fine.b[0][slot] = b;
                        S.fine.n[0][slot] = e - b;
                        S.fine.d[0][slot] = __double2float_rd(dm);
                    }
                    ncur += __popcll(km);
                }
                wave_sync();
                // refinement: eight lanes per box, one child each
                for (int round = 0; round < 3; ++round) {
                    int nnext = 0;
                    bool split_any = false;
                    for (int base = 0; base < ncur; base += 8) {
                        const int i = base + (lane >> 3), ch = lane & 7;
                        // room for this step's children and every later box unsplit
                        const bool room = nnext + WAVE + (ncur - base - 8 > 0 ? ncur - base - 8 : 0) <= VT_FINE_CAP;
                        bool keep = false, split = false;
                        uint64_t pk = 0;
                        int32_t b = 0, len = 0;
                        float dd = 0.0f;
                        if (i < ncur) {
                            pk = S.fine.pk[cur][i];
                            b = S.fine.b[cur][i];
                            len = S.fine.n[cur][i];
                            dd = S.fine.d[cur][i];
                            int u[3];
                            const int l = unpack_box(pk, u);
                            split = room && len > 128 && l < VT_MORTON_BITS;
                            if (!split) {
                                keep = ch == 0;
                            } else {
                                const int uc[3] = {2 * u[0] + ((ch >> 2) & 1), 2 * u[1] + ((ch >> 1) & 1), 2 * u[2] + (ch & 1)};
                                double dm = 0.0;
                                keep = box_test(l + 1, uc, dm);
                                if (keep) {
                                    int32_t e;
                                    box_range(l + 1, uc, b, e);
                                    len = e - b;
                                    keep = len > 0;
                                    pk = pack_box(uc, l + 1);
                                    dd = __double2float_rd(dm);
                                }
                            }
                        }
                        split_any |= __ballot(split) != 0;
                        const uint64_t km = __ballot(keep);
                        if (keep) {
                            const int slot = nnext + __popcll(km & lt);
                            S.fine.pk[cur ^ 1][slot] = pk;
                            S.fine.b[cur ^ 1][slot] = b;
                            S.fine.n[cur ^ 1][slot] = len;
                            S.fine.d[cur ^ 1][slot] = dd;
                        }
                        nnext += __popcll(km);
                    }
                    wave_sync();
                    cur ^= 1;
                    ncur = nnext;
                    if (!split_any) break;
                }
                // nearest boxes first (ties by position in the list), lengths -> prefix
                uint64_t kk[VT_FINE_CAP / 64];
#pragma unroll
                for (int q = 0; q < VT_FINE_CAP / 64; ++q) {
                    const int i = q * 64 + lane;
                    kk[q] = i < ncur ? ((uint64_t)__float_as_uint(S.fine.d[cur][i]) << 32) | (uint64_t)i : ~0ull;
                }
                bitonic_u64<VT_FINE_CAP / 64>(kk);
                int carry = 0;
#pragma unroll
                for (int q = 0; q < VT_FINE_CAP / 64; ++q) {
                    const int i = q * 64 + lane, sl = (int)(kk[q] & 0xFFFFu);
                    const bool ok = i < ncur;
                    const int len = ok ? S.fine.n[cur][sl] : 0;
                    int tot;
                    const int pre = wave_excl_scan(len, &tot);
                    if (ok) {
                        S.fine.b[cur ^ 1][i] = S.fine.b[cur][sl];
                        S.fine.n[cur ^ 1][i] = carry + pre;
                        S.fine.d[cur ^ 1][i] = S.fine.d[cur][sl];
                    }
                    carry += tot;
                }
                wave_sync();
                fin = cur ^ 1;
                total = uni_i(carry);
                return uni_i(ncur);
            } else {
                total = 0;
                return -1;
            }
        };
        // a loaded position -> separation from the seed (minimum image), d^2
        auto separation = [&](const PT4 &p, double &dx, double &dy, double &dz) -> double {
            dx = (double)p.x - sx;
            dy = (double)p.y - sy;
            dz = (double)p.z - sz;
            if (it.periodic) {
                dx -= it.L[0] * rint(dx * invL[0]);
                dy -= it.L[1] * rint(dy * invL[1]);
                dz -= it.L[2] * rint(dz * invL[2]);
            }
            return dx * dx + dy * dy + dz * dz;
        };

        // ---- one sweep over the shell [r_lo, r_hi): lanes = particles, planes that cut
        // no vertex of the current cell are dropped, survivors are applied nearest first
        auto sweep = [&](double r_lo, double r_hi) {
            const double rl2 = r_lo * r_lo, rh2 = r_hi * r_hi;
            int total;
            // stage the cell's vertices for the box pruning of the cover (and the first chunk)
            P.update_r2();
            stage_search();
            int ncq = -1;
            if constexpr (RETRY) ncq = cover_fine(r_hi, r_lo, total);
            const bool fine_ = RETRY && ncq >= 0;
            if (!fine_) ncq = cover(r_hi, r_lo, total, true);
            const int32_t *lpre = S.rp, *lrb = S.rb;
            if constexpr (RETRY && VPL > 1) {
                if (fine_) {
                    lpre = S.fine.n[fin];
                    lrb = S.fine.b[fin];
                }
            }
            int rcur = 0;
            bool dirty = false, r2stale = false;
            int rr = 0;  // refined cover: box of the chunk's first particle
            // positions of the next 64 particles are loaded while the current 64 are tested
            int32_t jn = -1;
            PT4 pn{};
            if (total > 0) {
                const int32_t j_ = chunk_loc(lpre, lrb, ncq, rcur, 0);
                if (lane < total) {
                    jn = j_;
                    pn = ((const PT4 *)A.spos)[jn];
                }
            }
            for (int base = 0; base < total && !overflow && !corrupt; base += WAVE) {
                if constexpr (RETRY && VPL > 1) {
                    if (fine_) {
                        // boxes nearest first: once the chunk's first box lies beyond 2R, so do all later ones
                        while (rr + 1 < ncq && S.fine.n[fin][rr + 1] <= base) ++rr;
                        if (r2stale) {
                            P.update_r2();
                            r2stale = false;
                        }
                        if ((double)S.fine.d[fin][rr] >= 4.0 * P.R2) break;
                    }
                }
                const int f = base + lane;
                bool keep = false;
                double dx = 0, dy = 0, dz = 0, d2 = 0;
                const int32_t j = jn;
                const PT4 pc = pn;
                if (base + WAVE < total) {
                    const int32_t j_ = chunk_loc(lpre, lrb, ncq, rcur, base + WAVE);
                    if (f + WAVE < total) {
                        jn = j_;
                        pn = ((const PT4 *)A.spos)[jn];
                    }
                }
                if (f < total) {
                    d2 = separation(pc, dx, dy, dz);
                    if (j != j0) {
                        if (d2 == 0.0) dup = 1;
                        keep = (d2 > 0.0) && (d2 >= rl2) && (d2 < rh2) && (d2 < 4.0 * P.R2);
                    }
                }
                const uint64_t km = __ballot(keep);
                if (km == 0) continue;
                ntested += __popcll(km);
                if (dirty) {
                    P.update_r2();
                    // vertex positions (and, mixed, their error bounds) for the lane-parallel test
                    stage_search();
                    dirty = false;
                }
                const double pd = 0.5 * d2;
                const double nn = sqrt(d2);
                // Only a vertex whose empty sphere (centre v, radius |v|) reaches the chunk's
                // bounding box can be cut by one of its particles.  A vertex with
                // dist(v, box)^2 - |v|^2 above the margin gives sv < -marg for every particle of
                // the chunk, so skipping it leaves each lane's answer unchanged; the particles of
                // a chunk are close together (consecutive Morton ranges), so few vertices remain.
                const double bx0 = uni_d(wave_min_x(keep ? dx : 1e300)), bx1 = uni_d(wave_max_x(keep ? dx : -1e300));
                const double by0 = uni_d(wave_min_x(keep ? dy : 1e300)), by1 = uni_d(wave_max_x(keep ? dy : -1e300));
                const double bz0 = uni_d(wave_min_x(keep ? dz : 1e300)), bz1 = uni_d(wave_max_x(keep ? dz : -1e300));
                const double pmax = uni_d(sqrt(wave_max_x(keep ? d2 : 0.0)));
                uint64_t vm[VPL];
#pragma unroll
                for (int s = 0; s < VPL; ++s) {
                    bool rel = false;
                    if (P.alive[s] & mybit) {
                        const double x = (double)P.vx[s], y = (double)P.vy[s], z = (double)P.vz[s];
                        const double ex = fmax(0.0, fmax(bx0 - x, x - bx1));
                        const double ey = fmax(0.0, fmax(by0 - y, y - by1));
                        const double ez = fmax(0.0, fmax(bz0 - z, z - bz1));
                        const double r2v = x * x + y * y + z * z;
                        const double mg = 2.0 * pmax * ((double)P.ve[s] + 1e-6 * (sqrt(r2v) + pmax));
                        rel = ex * ex + ey * ey + ez * ez - r2v <= mg;
                    }
                    vm[s] = __ballot(rel);
                }
                bool act = false;
                auto cuts_v = [&](int k) -> bool {
                    const double *v = S.u.s.vp[k];
                    const double sv = fma(v[0], dx, fma(v[1], dy, v[2] * dz)) - pd;  // the clip's rounding
                    // FP64 path: the exact predicate; mixed path: widened by the vertex error bound
                    double marg = 0.0;
                    if (std::is_same<T, float>::value)
                        marg = nn * (S.u.s.ve[k] + 1e-6 * (sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) + 0.5 * nn));
                    return sv > -marg;
                };
#pragma unroll
                for (int s = 0; s < VPL; ++s) {
                    uint64_t m = vm[s];
                    while (m) {
                        const int k = __builtin_ctzll(m);
                        m &= m - 1;
                        act |= cuts_v(s * 64 + k);
                    }
                }
                uint64_t am = __ballot(keep && act);
                while (am) {
                    const double key = (am & mybit) ? d2 : 1e300;
                    const double mn = wave_min_x(key);
                    const uint64_t who = __ballot((am & mybit) && d2 == mn);
                    const int k = uni_i(__builtin_ctzll(who));
                    am &= ~(1ull << k);
                    P4<double> p64;
                    p64.x = readlane_dbl(dx, k);
                    p64.y = readlane_dbl(dy, k);
                    p64.z = readlane_dbl(dz, k);
                    p64.d = 0.5 * (p64.x * p64.x + p64.y * p64.y + p64.z * p64.z);
                    const int32_t tag = (int32_t)readlane_u32((uint32_t)j, k);
                    const int rc = P.clip(S.P, p64, tag);
                    if (rc == CLIP_CUT) {
                        dirty = true;
                        r2stale = true;
                        ++ncut;
                    } else if (rc == CLIP_OVERFLOW) {
                        overflow = true;
                        break;
                    } else if (rc < 0) {
                        corrupt = true;
                        break;
                    }
                }
            }
            P.update_r2();
            wave_sync();
        };

        int refine = 0;
        for (int pass = 0; pass < 160; ++pass) {
            const double rh2 = r_next * r_next, rl2 = r_done * r_done;
            const double inv_rh2 = 1.0 / rh2, inv_bin = 64.0 / (rh2 - rl2);
            int total;
            // once the cell has been cut a few times, covering boxes that no vertex's empty sphere
            // reaches hold no particle that can still cut it, as in the sweeps
            const bool prune = r_done > 0.0 && ncut >= 4;
            if (prune) stage_search();
            const int ncq = cover(r_next, r_done, total, prune);
            S.hist[lane] = 0;
            wave_sync();
            // ---- gather particles with r_done <= d < r_next (and a d^2 histogram); the positions
            // of the next 64 are loaded while the current 64 are processed
            int n = 0;
            int32_t jn = -1;
            PT4 pn{};
            int rcur = 0;
            if (total > 0) {
                const int32_t j_ = chunk_loc(S.rp, S.rb, ncq, rcur, 0);
                if (lane < total) {
                    jn = j_;
                    pn = ((const PT4 *)A.spos)[jn];
                }
            }
            for (int base = 0; base < total; base += WAVE) {
                const int f = base + lane;
                bool keep = false;
                double dx = 0, dy = 0, dz = 0, d2 = 0;
                const int32_t j = jn;
                const PT4 pc = pn;
                if (base + WAVE < total) {
                    const int32_t j_ = chunk_loc(S.rp, S.rb, ncq, rcur, base + WAVE);
                    if (f + WAVE < total) {
                        jn = j_;
                        pn = ((const PT4 *)A.spos)[jn];
                    }
                }
                if (f < total) {
                    d2 = separation(pc, dx, dy, dz);
                    if (j != j0) {
                        // a coincident particle has no bisector: report it, do not clip with it
                        if (d2 == 0.0) dup = 1;
                        keep = (d2 > 0.0) && (d2 >= rl2) && (d2 < rh2);
                    }
                }
                const uint64_t km = __ballot(keep);
                if (keep) {
                    const int slot = n + __popcll(km & lt);
                    if (slot < VT_CAND_MAX) {
                        S.u.c.cd[slot][0] = dx;
                        S.u.c.cd[slot][1] = dy;
                        S.u.c.cd[slot][2] = dz;
                        S.u.c.cid[slot] = j;
                        double qf = d2 * inv_rh2 * 16777216.0;
                        uint32_t q = qf >= 16777215.0 ? 16777215u : (uint32_t)qf;
                        S.u.c.ckey[slot] = (q << 8) | (uint32_t)slot;
                    }
                    int bin = (int)((d2 - rl2) * inv_bin);
                    atomicAdd(&S.hist[bin < 0 ? 0 : (bin > 63 ? 63 : bin)], 1);
                }
                n += __popcll(km);
            }
            wave_sync();
            if (n > VT_CAND_MAX && (r_done == 0.0 || ncut < 4) && refine < 16) {
                // Shell too full while the cell is still (nearly) the initial box: the first shell,
                // or a later one when the earlier shells were empty (a sweep applies planes in
                // chunk order, which on an unclipped box can grow the polytope past its slots).
                // The largest b with at most VT_CAND_MAX particles in bins [r_done, b) bounds it.
                const int h = S.hist[lane];
                int tot;
                const int pre = wave_excl_scan(h, &tot);
                const uint64_t fit = __ballot(pre + h <= VT_CAND_MAX);
                int b = (fit == ~0ull) ? 64 : __builtin_ctzll(~fit);
                if (b < 1) b = 1;
                r_next = sqrt(rl2 + (rh2 - rl2) * (double)b / 64.0);
                ++refine;
                continue;
            }
            if (n > VT_CAND_MAX) {
                sweep(r_done, r_next);
            } else {
                // ---- sort by distance
                uint32_t k0 = (lane < n) ? S.u.c.ckey[lane] : 0xFFFFFFFFu;
                uint32_t k1 = (lane + 64 < n) ? S.u.c.ckey[lane + 64] : 0xFFFFFFFFu;
                if (n > 64)
                    bitonic128_x(k0, k1);
                else if (n > 1)
                    k0 = bitonic64_x(k0);
                // ---- clip in increasing distance; stop at the first particle beyond 2R
                // the key of distance 2R: the keys' own scaling (d^2 * inv_rh2 * 2^24, rounded down),
                // so every candidate within 2R has a key below it; one more for safety
                auto q4r = [&](double r2) -> uint32_t {
                    double x = 4.0 * r2 * inv_rh2 * 16777216.0;
                    return x >= 16777215.0 ? 0xFFFFFFu : (uint32_t)x + 1u;
                };
                // Candidates go in chunks of 64 in increasing distance.  Each lane tests its
                // plane against every vertex of the current cell (staged in LDS); a plane that
                // cuts no vertex now never will (the cell only shrinks) and is dropped.  The
                // rest are applied one by one, nearest first, until one lies beyond 2R.
                uint32_t Q4R = q4r(P.R2);
                bool stale = false;  // P.R2 is an upper bound until refreshed
                bool done = false;
                for (int c0 = 0; c0 < n && !done; c0 += 64) {
                    if (stale) {
                        P.update_r2();
                        Q4R = q4r(P.R2);
                        stale = false;
                    }
                    const int i = c0 + lane;
                    const uint32_t key = (i < n) ? (c0 == 0 ? k0 : k1) : 0xFFFFFFFFu;
                    const bool near = i < n && (key >> 8) <= Q4R;
                    if (__ballot(near) == 0) break;
                    // Candidates of this chunk still to apply or drop.  After a few cuts the cell
                    // has shrunk, and testing the rest against it again, in parallel, drops more
                    // of them than applying them one by one would find cutting.
                    uint64_t pend = __ballot(near);
                    while (pend && !done) {
                        // A candidate at distance |D| cuts vertex v only if it lies in the sphere with
                        // centre v through the seed, so only if |D| <= 2 |v|; the smallest pending key
                        // bounds |D| from below, and vertices short of it (with a margin far above the
                        // rounding of the side test and, mixed, the vertex error bound) are not tested.
                        const uint32_t kmin = readlane_u32(key, uni_i(__builtin_ctzll(pend))) >> 8;
                        const double dlo2 = (double)kmin * rh2 * (1.0 / 16777216.0) * (1.0 - 1e-12);
                        uint64_t farv[VPL];
#pragma unroll
                        for (int s = 0; s < VPL; ++s) {
                            bool f = false;
                            if (P.alive[s] & mybit) {
                                S.P.st[s * 64 + lane][0] = P.vx[s];
                                S.P.st[s * 64 + lane][1] = P.vy[s];
                                S.P.st[s * 64 + lane][2] = P.vz[s];
                                if constexpr (std::is_same<T, float>::value) S.P.ste[s * 64 + lane] = P.ve[s];
                                const double x = (double)P.vx[s], y = (double)P.vy[s], z = (double)P.vz[s];
                                const double r2v = x * x + y * y + z * z;
                                if constexpr (std::is_same<T, float>::value) {
                                    const double fv = 2.0 * (sqrt(r2v) + (double)P.ve[s]) * (1.0 + 1e-5);
                                    f = fv * fv >= dlo2;
                                } else {
                                    f = 4.0 * r2v * (1.0 + 2.1e-5) >= dlo2;  // (2 |v| (1 + 1e-5))^2
                                }
                            }
                            farv[s] = __ballot(f);
                        }
                        wave_sync();
                        bool act = false;
                        if (pend & mybit) {
                            const int slot = (int)(key & 0xFFu);
                            const double dx = S.u.c.cd[slot][0], dy = S.u.c.cd[slot][1], dz = S.u.c.cd[slot][2];
                            const double d2 = dx * dx + dy * dy + dz * dz;
                            const double pd = 0.5 * d2;
                            const double nn = sqrt(d2);
                            // does the candidate's plane cut staged vertex k?
                            auto cuts_v = [&](int k) -> bool {
                                const double vx = (double)S.P.st[k][0], vy = (double)S.P.st[k][1], vz = (double)S.P.st[k][2];
                                // same rounding as the clip's own side test
                                const double sv = fma(vx, dx, fma(vy, dy, vz * dz)) - pd;
                                // FP64 path: the exact predicate; mixed path: widened by the vertex error bound
                                double marg = 0.0;
                                if (std::is_same<T, float>::value)
                                    marg = nn * ((double)S.P.ste[k] + 1e-6 * (sqrt(vx * vx + vy * vy + vz * vz) + 0.5 * nn));
                                return sv > -marg;
                            };
#pragma unroll
                            for (int s = 0; s < VPL; ++s) {
                                // two vertices per step, their loads issued together
                                uint64_t m = farv[s];
                                while (m && !act) {
                                    const int k0 = __builtin_ctzll(m);
                                    m &= m - 1;
                                    const int k1 = m ? __builtin_ctzll(m) : k0;
                                    m &= m - 1;
                                    const bool c0 = cuts_v(s * 64 + k0), c1 = cuts_v(s * 64 + k1);
                                    act = c0 || c1;
                                }
                            }
                        }
                        uint64_t am = __ballot((pend & mybit) && act);
                        pend = 0;
                        int cuts = 0;
                        while (am) {
                            const int k = __builtin_ctzll(am);
                            am &= am - 1;
                            const uint32_t kk = readlane_u32(key, k);
                            if ((kk >> 8) > Q4R) {
                                if (!stale) {
                                    done = true;
                                    break;
                                }
                                P.update_r2();
                                Q4R = q4r(P.R2);
                                stale = false;
                                if ((kk >> 8) > Q4R) {
                                    done = true;
                                    break;
                                }
                            }
                            const int slot = (int)(kk & 0xFFu);
                            ++ntested;
                            P4<double> p64;
                            p64.x = S.u.c.cd[slot][0];
                            p64.y = S.u.c.cd[slot][1];
                            p64.z = S.u.c.cd[slot][2];
                            p64.d = 0.5 * (p64.x * p64.x + p64.y * p64.y + p64.z * p64.z);
                            const int rc = P.clip(S.P, p64, S.u.c.cid[slot]);
                            if (rc == CLIP_CUT) {
                                stale = true;
                                ++ncut;
                                if (!RETRY && ++cuts == 8 && __popcll(am) >= 16) {
                                    pend = am;
                                    break;
                                }
                            } else if (rc == CLIP_OVERFLOW) {
                                overflow = true;
                                done = true;
                                break;
                            } else if (rc < 0) {
                                corrupt = true;
                                done = true;
                                break;
                            }
                        }
                        wave_sync();
                    }
                }
                if (stale) P.update_r2();
            }
            if (overflow || corrupt) break;
            r_done = r_next;
            const double need = 2.0 * sqrt(P.R2);
            if (need <= r_done) {
                complete = true;
                break;
            }
            if (r_done >= r_cap) break;
            // next shell: up to the security radius, growing the searched radius by 1.25x to 2x
            r_next = fmin(fmax(need * (1.0 + 1e-9), 1.25 * r_done), 2.0 * r_done);
            if (r_next > r_cap) r_next = r_cap;
        }
        const bool exhausted = !complete && r_done < r_cap;
        dup = __ballot(dup != 0) ? 1u : 0u;

        if (overflow && !RETRY) {
            // hand the cell to the large-capacity kernel
            if (lane == 0) {
                A.cnf[cslot] = 0;
                uint32_t qi = atomicAdd(&A.counters[CTR_QUEUE], 1u);
                if ((int64_t)qi < A.queue_cap) A.queue_out[qi] = cslot;
                else atomicOr(&A.counters[CTR_STATUS], VT_DEV_CAPACITY);
                if (dup) atomicOr(&A.counters[CTR_STATUS], VT_DEV_DUPLICATE);
            }
            continue;
        }
        const int64_t row = A.row_base + (RETRY ? w : (int64_t)cslot) * A.fstride;
        if (overflow || corrupt) {
            if (lane == 0) {
                atomicOr(&A.counters[CTR_STATUS], corrupt ? VT_DEV_TOPOLOGY : VT_DEV_CAPACITY);
                if (dup) atomicOr(&A.counters[CTR_STATUS], VT_DEV_DUPLICATE);
                A.cvol[cslot] = 0.0;
                A.crad[cslot] = 0.0;
                A.ccnt[cslot] = 0;
                A.crow[cslot] = row;
                A.cstat[cslot] = VT_CELL_FAILED | (RETRY ? VT_CELL_RETRIED : 0);
                A.cnv[cslot] = 0;
                A.cnf[cslot] = 0;
                A.cnt[cslot] = ntested;
            }
            continue;
        }

        // ---------------- final geometry in FP64: facet areas, centroids, volume
        wave_sync();
        const int nvert = P.nvertices();
        double r2max = 0.0;
#pragma unroll
        for (int s = 0; s < VPL; ++s) {
            if (P.alive[s] & mybit) {
                double x, y, z;
                P.pos64(S.P, s, x, y, z);
                S.u.f.vp[s * 64 + lane][0] = x;
                S.u.f.vp[s * 64 + lane][1] = y;
                S.u.f.vp[s * 64 + lane][2] = z;
                S.u.f.vt[s * 64 + lane] = P.vt[s];
                r2max = fmax(r2max, x * x + y * y + z * z);
            }
        }
        // the global ids of the faces' particles (the neighbour keys), loaded while the areas are computed
        int32_t tag_l = -1;
        uint32_t gid_l = 0;
        if constexpr (VPL == 1) {
            if (P.fa[0] & mybit) {
                tag_l = S.P.ptag[lane];
                if (tag_l >= 0) gid_l = (uint32_t)A.sgid[tag_l];
            }
        }
        wave_sync();
        double vol_l = 0.0;
        double area_l[VPL];
        double cen_l[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int r = 0; r < VPL; ++r) {
            area_l[r] = 0.0;
            const int f = r * 64 + lane;
            if (!(P.fa[r] & mybit)) continue;
            uint64_t mf[VPL];
            int i0 = -1;
#pragma unroll
            for (int ww = 0; ww < VPL; ++ww) {
                mf[ww] = S.P.fm[f][ww];
                if (i0 < 0 && mf[ww]) i0 = ww * 64 + __builtin_ctzll(mf[ww]);
            }
            // the vertex after u counter-clockwise on face f: it lies on f and on
            // the face that precedes f in u's triple
            auto next_of = [&](int u) -> int {
                uint32_t t = S.u.f.vt[u];
                int t0 = t & 0xFF, t1 = (t >> 8) & 0xFF, t2 = (t >> 16) & 0xFF;
                int c = (t0 == f) ? t2 : (t1 == f) ? t0 : t1;
                int nx = -1;
#pragma unroll
                for (int ww = 0; ww < VPL; ++ww) {
                    uint64_t x = mf[ww] & S.P.fm[c][ww];
                    if (ww == (u >> 6)) x &= ~(1ull << (u & 63));
                    if (nx < 0 && x) nx = ww * 64 + __builtin_ctzll(x);
                }
                return nx;
            };
            const double v0x = S.u.f.vp[i0][0], v0y = S.u.f.vp[i0][1], v0z = S.u.f.vp[i0][2];
            // Fan triangles (v0, v1, v2) are counter-clockwise seen from outside: their areas are half
            // the component of (v1 - v0) x (v2 - v0) along the face's unit normal.  With a = v1 - v0
            // and b = v2 - v0 (the next step's a), the face's area is the sum of the triangles' and its
            // centroid v0 + sum(ta (a + b)) / (3 A); the cell's volume is the sum over faces of
            // A h / 3, h = d / |n| the distance of the face's plane from the seed.
            const P4<double> &pf = S.P.pl64[f];
            const double inn = 1.0 / sqrt(pf.x * pf.x + pf.y * pf.y + pf.z * pf.z);
            const double hx = 0.5 * pf.x * inn, hy = 0.5 * pf.y * inn, hz = 0.5 * pf.z * inn;
            double Mx = 0, My = 0, Mz = 0, at = 0;
            int prev = next_of(i0);
            double ax = 0, ay = 0, az = 0;
            if (prev >= 0) {
                ax = S.u.f.vp[prev][0] - v0x;
                ay = S.u.f.vp[prev][1] - v0y;
                az = S.u.f.vp[prev][2] - v0z;
            }
            int guard = 0;
            while (prev >= 0 && guard < VMAX) {
                const int cur = next_of(prev);
                if (cur < 0 || cur == i0) break;
                const double bx = S.u.f.vp[cur][0] - v0x, by = S.u.f.vp[cur][1] - v0y, bz = S.u.f.vp[cur][2] - v0z;
                const double cx = fma(ay, bz, -(az * by)), cy = fma(az, bx, -(ax * bz)), cz = fma(ax, by, -(ay * bx));
                const double ta = fma(cx, hx, fma(cy, hy, cz * hz));
                Mx = fma(ta, ax + bx, Mx);
                My = fma(ta, ay + by, My);
                Mz = fma(ta, az + bz, Mz);
                at += ta;
                ax = bx;
                ay = by;
                az = bz;
                prev = cur;
                ++guard;
            }
            const double i3a = at > 0 ? 1.0 / (3.0 * at) : 0.0;
            const double cfx = fma(Mx, i3a, v0x), cfy = fma(My, i3a, v0y), cfz = fma(Mz, i3a, v0z);
            area_l[r] = at;
            vol_l = fma(at, pf.d * inn * (1.0 / 3.0), vol_l);
            if constexpr (VPL == 1) {
                cen_l[0] = cfx;
                cen_l[1] = cfy;
                cen_l[2] = cfz;
            } else {
                S.u.f.fa[f] = at;
                S.u.f.fc[f][0] = cfx;
                S.u.f.fc[f][1] = cfy;
                S.u.f.fc[f][2] = cfz;
            }
        }
        const double V = wave_sum_d(vol_l);
        const double Rfin = sqrt(wave_max_x(r2max));
        const double amin = (double)(A.area_eps * exp2f(log2f((float)fabs(V)) * (2.0f / 3.0f)));
        // facets of positive area generated by particles -> neighbour rows, ascending global id
        uint64_t keys[VPL];
        uint32_t wall = 0;  // walls (bit f for tag -1 - f) among this lane's facets
        int cnt = 0;
        if constexpr (VPL == 1) {
            // each face lane holds its facet; its row is the rank of its key (global id, then slot)
            // among the kept facets, counted over their keys read lane by lane
            keys[0] = ~0ull;
            if ((P.fa[0] & mybit) && area_l[0] > amin) {
                if (tag_l < 0) wall |= 1u << ((-1 - tag_l) & 7);
                else keys[0] = ((uint64_t)gid_l << 9) | (uint64_t)lane;
            }
            const uint64_t kept = __ballot(keys[0] != ~0ull);
            cnt = __popcll(kept);
            int rank = 0;
            for (uint64_t m = kept; m; m &= m - 1) {
                const int g = uni_i(__builtin_ctzll(m));
                const uint64_t kg = ((uint64_t)readlane_u32((uint32_t)(keys[0] >> 32), g) << 32) |
                                    (uint64_t)readlane_u32((uint32_t)keys[0], g);
                rank += kg < keys[0] ? 1 : 0;
            }
            if (keys[0] != ~0ull && rank < A.fstride) {
                A.stage_ids[row + rank] = tag_l;  // sorted index; mapped to global ids on output
                if (A.want_faces) {
                    A.stage_area[row + rank] = area_l[0];
                    A.stage_cen[3 * (row + rank) + 0] = cen_l[0];
                    A.stage_cen[3 * (row + rank) + 1] = cen_l[1];
                    A.stage_cen[3 * (row + rank) + 2] = cen_l[2];
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < VPL; ++r) {
                const int f = r * 64 + lane;
                keys[r] = ~0ull;
                if ((P.fa[r] & mybit) && area_l[r] > amin) {
                    int32_t tag = S.P.ptag[f];
                    if (tag < 0) wall |= 1u << ((-1 - tag) & 7);
                    else keys[r] = ((uint64_t)(uint32_t)A.sgid[tag] << 9) | (uint64_t)f;
                }
            }
#pragma unroll
            for (int r = 0; r < VPL; ++r) cnt += __popcll(__ballot(keys[r] != ~0ull));
            bitonic_u64<VPL>(keys);
            wave_sync();
#pragma unroll
            for (int r = 0; r < VPL; ++r) {
                int k = r * 64 + lane;
                if (k < cnt && k < A.fstride) {
                    int f = (int)(keys[r] & 511ull);
                    A.stage_ids[row + k] = S.P.ptag[f];  // sorted index; mapped to global ids on output
                    if (A.want_faces) {
                        A.stage_area[row + k] = S.u.f.fa[f];
                        A.stage_cen[3 * (row + k) + 0] = S.u.f.fc[f][0];
                        A.stage_cen[3 * (row + k) + 1] = S.u.f.fc[f][1];
                        A.stage_cen[3 * (row + k) + 2] = S.u.f.fc[f][2];
                    }
                }
            }
        }
        uint32_t wall_mask = 0;
        for (int f = 0; f < 6; ++f)
            if (__ballot((wall >> f) & 1u) != 0) wall_mask |= 1u << f;
        const bool any_wall = wall_mask != 0;
        // topology record for the grid deposit, which then rebuilds the cell without clipping:
        // the tags of the faces in slot order, then each vertex's face triple as ranks in that
        // order (the triple's order, which fixes the orientation, is kept)
        int32_t nf_rec = 0;
        if constexpr (!RETRY && VPL == 1) {
            const uint64_t fam = P.fa[0];
            const int nf = __popcll(fam);
            if (nf <= VT_TOPO_FACES) {
                const int64_t tb = (int64_t)cslot * VT_TOPO_STRIDE;
                if (fam & mybit) A.ctopo[tb + __popcll(fam & lt)] = S.P.ptag[lane];
                if (P.alive[0] & mybit) {
                    const uint32_t t = P.vt[0];
                    auto rk = [&](uint32_t f) -> uint32_t { return (uint32_t)__popcll(fam & ((1ull << (f & 63u)) - 1ull)); };
                    const uint32_t tr = rk(t & 0xFFu) | (rk((t >> 8) & 0xFFu) << 8) | (rk((t >> 16) & 0xFFu) << 16);
                    A.ctopo[tb + VT_TOPO_FACES + __popcll(P.alive[0] & lt)] = (int32_t)tr;
                }
                nf_rec = nf;
            }
        }
        if (lane == 0) {
            uint8_t st = RETRY ? VT_CELL_RETRIED : 0;
            bool incomplete = false;
            if (exhausted) {
                atomicOr(&A.counters[CTR_STATUS], VT_DEV_CAPACITY);
                st |= VT_CELL_FAILED;
            } else if (it.periodic) {
                if (!complete || any_wall || 4.0 * Rfin >= Lmin) {
                    atomicOr(&A.counters[CTR_STATUS], VT_DEV_BOX_TOO_SMALL);
                    st |= VT_CELL_FAILED;
                }
            } else {
                // only cut walls (not the world's true boundaries) make a cell incomplete
                const uint32_t cut = ~(uint32_t)it.walls;
                for (int a = 0; a < 3; ++a) {
                    if (((cut >> (2 * a)) & 1u) && xs[a] - 2.0 * Rfin < it.lo[a]) incomplete = true;
                    if (((cut >> (2 * a + 1)) & 1u) && xs[a] + 2.0 * Rfin > it.lo[a] + it.L[a]) incomplete = true;
                }
                if (wall_mask & cut) incomplete = true;
            }
            if (incomplete) {
                st |= VT_CELL_INCOMPLETE;
                atomicAdd(&A.counters[CTR_INCOMPLETE], 1u);
            }
            if (dup) atomicOr(&A.counters[CTR_STATUS], VT_DEV_DUPLICATE);
            const int32_t kept = cnt < A.fstride ? cnt : (int32_t)A.fstride;
            if (cnt > A.fstride) atomicOr(&A.counters[CTR_STATUS], VT_DEV_CAPACITY);
            A.cvol[cslot] = V;
            A.crad[cslot] = Rfin;
            A.ccnt[cslot] = kept;
            A.crow[cslot] = row;
            A.cstat[cslot] = st;
            A.cnv[cslot] = nvert;
            A.cnf[cslot] = nf_rec;
            A.cnt[cslot] = ntested;
            atomicAdd((unsigned long long *)&A.counters[CTR_NNZ_LO], (unsigned long long)kept);
        }
    }
}

// ---------------------------------------------------------------- cost-model statistic
// P_i = |{j != i : d_ij < 2 R_i}| + 1 for every computed cell, R_i its largest vertex distance:
// the particles the security criterion has to examine, counted exactly after the build (the clip
// kernel itself may skip particles it can prove irrelevant).  One wavefront per cell: the Morton
// boxes of side in [r/2, r) around the seed, r = 2 R; a box entirely inside the ball counts its
// whole range, a box the sphere crosses has its particles tested one by one.
struct PlanesMem {
    int32_t rb[216];
    int32_t rp[216];
};

template <typename PT4>
__global__ void __launch_bounds__(256) k_planes(ClipArgs A, int32_t *out) {
    __shared__ PlanesMem SM[4];
    PlanesMem &S = SM[threadIdx.x >> 6];
    const int lane = lane_id();
    const uint64_t lt = lanemask_lt();
    const int64_t nw = (int64_t)gridDim.x * 4;
    for (int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); c < A.ncells; c += nw) {
        const uint8_t st = A.cstat[c];
        if (st & VT_CELL_FAILED) {
            if (lane == 0) out[c] = 0;
            continue;
        }
        const int32_t j0 = A.cells[c];
        const int bi = find_item_d(A.items, A.n_items, j0);
        const DevItem it = uniform_item(A.items[bi]);
        double xs[3];
        load_pos<PT4>(A.spos, j0, xs[0], xs[1], xs[2]);
        const double r = 2.0 * A.crad[c], r2 = r * r;
        int lvl = 0;
        double cside = it.S;
        while (lvl < VT_MORTON_BITS && cside >= r) {
            cside *= 0.5;
            ++lvl;
        }
        const int sh = VT_MORTON_BITS - lvl;
        const int64_t ncl = 1ll << lvl;
        const double quantum = it.S / (double)(1 << VT_MORTON_BITS);
        int64_t a0[3];
        int na[3];
        for (int a = 0; a < 3; ++a) {
            int64_t i0 = (vt_qraw(xs[a] - r, it.lo[a], it.inv_res) - 1) >> sh;
            int64_t i1 = (vt_qraw(xs[a] + r, it.lo[a], it.inv_res) + 1) >> sh;
            if (it.periodic) {
                if (i1 - i0 + 1 >= ncl) {
                    i0 = 0;
                    i1 = ncl - 1;
                }
            } else {
                if (i0 < 0) i0 = 0;
                if (i1 > ncl - 1) i1 = ncl - 1;
            }
            a0[a] = i0;
            na[a] = i1 >= i0 ? (int)(i1 - i0 + 1) : 0;
        }
        const int nbox = na[0] * na[1] * na[2];
        int whole = 0, npart = 0;
        for (int base = 0; base < nbox; base += WAVE) {
            const int k = base + lane;
            bool part = false;
            int32_t b = 0, e = 0;
            if (k < nbox) {
                const int64_t u[3] = {a0[0] + k % na[0], a0[1] + (k / na[0]) % na[1], a0[2] + k / (na[0] * na[1])};
                double dmin2 = 0.0, dmax2 = 0.0;
                for (int a = 0; a < 3; ++a) {
                    const bool all_img = it.periodic && na[a] == ncl;
                    double dn = 1e300, df = 1e300;
                    for (int s_ = -1; s_ <= 1; ++s_) {
                        if (s_ != 0 && !all_img) continue;
                        const double lo_ = it.lo[a] + (double)u[a] * cside - quantum + s_ * it.L[a];
                        const double hi_ = it.lo[a] + (double)(u[a] + 1) * cside + quantum + s_ * it.L[a];
                        const double dl = lo_ - xs[a], dh = xs[a] - hi_;
                        dn = fmin(dn, fmax(0.0, fmax(dl, dh)));
                        df = fmin(df, fmax(fabs(dl), fabs(dh)));
                    }
                    dmin2 += dn * dn;
                    dmax2 += df * df;
                }
                if (dmin2 < r2) {
                    uint64_t cc[3];
                    for (int a = 0; a < 3; ++a) cc[a] = (uint64_t)(it.periodic ? (u[a] & (ncl - 1)) : u[a]);
                    cell_range(A, it, bi, lvl, cc[0], cc[1], cc[2], b, e);
                    if (e > b) {
                        // a box whose farthest point (over its images) is within r lies inside the ball
                        // for the minimum-image distances too, which are no larger
                        if (dmax2 < r2 && !(it.periodic && (na[0] == ncl || na[1] == ncl || na[2] == ncl)))
                            whole += (e - b) - ((j0 >= b && j0 < e) ? 1 : 0);
                        else
                            part = true;
                    }
                }
            }
            const uint64_t pm = __ballot(part);
            if (part) {
                const int slot = npart + __popcll(pm & lt);
                S.rb[slot] = b;
                S.rp[slot] = e - b;
            }
            npart += __popcll(pm);
        }
        wave_sync();
        int carry = 0;
        for (int base = 0; base < npart; base += WAVE) {
            const int k = base + lane;
            const int len = k < npart ? S.rp[k] : 0;
            int tot;
            const int pre = wave_excl_scan(len, &tot);
            if (k < npart) S.rp[k] = carry + pre;
            carry += tot;
        }
        wave_sync();
        int inside = 0;
        for (int f = lane; f < carry; f += WAVE) {
            int lo = 0, hi = npart - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (S.rp[mid] <= f) lo = mid; else hi = mid - 1;
            }
            const int32_t j = S.rb[lo] + (f - S.rp[lo]);
            if (j == j0) continue;
            double px, py, pz;
            load_pos<PT4>(A.spos, j, px, py, pz);
            double dx = px - xs[0], dy = py - xs[1], dz = pz - xs[2];
            if (it.periodic) {
                dx -= it.L[0] * rint(dx / it.L[0]);
                dy -= it.L[1] * rint(dy / it.L[1]);
                dz -= it.L[2] * rint(dz / it.L[2]);
            }
            const double d2 = dx * dx + dy * dy + dz * dz;
            if (d2 > 0.0 && d2 < r2) ++inside;
        }
        const int total = wave_sum_i(inside) + whole;
        if (lane == 0) out[c] = total + 1;
        wave_sync();
    }
}

hipError_t vt_launch_planes(vt_ctx *c) {
    ClipArgs a{};
    a.spos = c->spos;
    a.skey = c->skey;
    a.tab = c->tab;
    a.items = c->items;
    a.n_items = c->n_items;
    a.cells = c->cells;
    a.ncells = c->n_owned;
    a.crad = c->crad;
    a.cstat = c->cstat;
    const int64_t blocks = std::min<int64_t>((c->n_owned + 3) / 4, 256 * 16);
    if (c->dtype == VT_F32) k_planes<float4><<<(unsigned)blocks, 256, 0, c->stream>>>(a, c->cnp);
    else k_planes<double4><<<(unsigned)blocks, 256, 0, c->stream>>>(a, c->cnp);
    return hipGetLastError();
}

// The fast kernel is register-capped at four resident waves per SIMD (128 VGPRs; with 40 face
// slots its LDS also fits four): the extra occupancy hides LDS latency better than the spills
// cost.  The large kernel (rare cells, four vertices per lane) keeps its registers.
template <typename T, typename PT4>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) k_clip(ClipArgs A) {
    clip_cells<T, PT4, 1, false>(A);
}

template <typename T, typename PT4>
__global__ void __launch_bounds__(256) k_clip_large(ClipArgs A) {
    clip_cells<T, PT4, 4, true>(A);
}

template <typename T, typename PT4, int VPL, bool RETRY>
static hipError_t launch_one(vt_ctx *c, ClipArgs &a, int wpb) {
    const size_t lds = sizeof(ClipMem<T, VPL>) * (size_t)wpb;
    auto kern = RETRY ? k_clip_large<T, PT4> : k_clip<T, PT4>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    int ncu = 0;
    hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device);
    if (ncu <= 0) ncu = 256;
    const int wpc = c->opts.waves_per_cu > 0 ? c->opts.waves_per_cu : 16;
    int64_t blocks = RETRY ? (int64_t)ncu * 2 : (int64_t)ncu * wpc / wpb;
    if (blocks < 1) blocks = 1;
    kern<<<dim3((unsigned)blocks), dim3(64 * wpb), lds, c->stream>>>(a);
    return hipGetLastError();
}

template <typename T, typename PT4>
static hipError_t launch_prec(vt_ctx *c, ClipArgs &a) {
    a.row_base = 0;
    a.fstride = VT_FSTRIDE_FAST;
    a.queue = nullptr;
    hipError_t e = launch_one<T, PT4, 1, false>(c, a, 4);
    if (e != hipSuccess) return e;
    if (c->timed) {
        e = hipEventRecord(c->ev[2], c->stream);
        if (e != hipSuccess) return e;
    }
    a.row_base = (int64_t)c->cap_owned * VT_FSTRIDE_FAST;
    a.fstride = VT_FSTRIDE_BIG;
    a.queue = c->queue;
    return launch_one<T, PT4, 4, true>(c, a, 1);
}

hipError_t vt_launch_clip(vt_ctx *c) {
    ClipArgs a;
    a.spos = c->spos;
    a.skey = c->skey;
    a.sgid = c->sgid;
    a.tab = c->tab;
    a.items = c->items;
    a.n_items = c->n_items;
    a.cells = c->cells;
    a.ncells = c->n_owned;
    a.queue = nullptr;
    a.queue_out = c->queue;
    a.queue_cap = c->cap_retry;
    a.counters = c->counters;
    a.cvol = c->cvol;
    a.crad = c->crad;
    a.ccnt = c->ccnt;
    a.crow = c->crow;
    a.cstat = c->cstat;
    a.cnv = c->cnv;
    a.cnt = c->cnt;
    a.ctopo = c->ctopo;
    a.cnf = c->cnf;
    a.stage_ids = c->stage_ids;
    a.stage_area = c->stage_area;
    a.stage_cen = c->stage_cen;
    a.want_faces = c->opts.want_faces ? 1 : 0;
    a.radius_factor = c->opts.radius_factor > 0 ? c->opts.radius_factor : 2.0f;
    a.area_eps = c->opts.area_eps > 0 ? c->opts.area_eps : 1e-12f;
    a.xcd_segments = c->opts.cell_mapping == VT_MAP_GLOBAL ? 1 : VT_XCD_SEGMENTS;
    const bool mixed = c->opts.precision == VT_PREC_MIXED;
    if (c->dtype == VT_F32) return mixed ? launch_prec<float, float4>(c, a) : launch_prec<double, float4>(c, a);
    return mixed ? launch_prec<float, double4>(c, a) : launch_prec<double, double4>(c, a);
}

// grid.hip -- average Voronoi density on a regular grid (paper section 2,
// optional grid output).  The paper does not state the averaging rule; this is
// the exact volume average of the piecewise-constant Voronoi field:
//   grid[v] = sum_i value_i * vol(cell_i ∩ voxel_v) / vol(voxel_v).
//
// Overlap volumes without 3D clipping.  For a voxel B = [X_i, X_i+1) x R_jk
// (R_jk a rectangle of the (y, z) grid) the field F = (psi(x), 0, 0) with
// psi(x) = clamp(x - X_i, 0, h_x) inside the column over R_jk has divergence 1_B,
// so by the divergence theorem
//   vol(P ∩ B) = sum over faces f of P of  n_x(f)/|n(f)| * ∫_{f over R_jk} psi dA.
// Projected on the (y, z) plane a face f becomes a convex polygon Omega_f on
// which x is affine, and n_x dA/|n| = sign(n_x) dy dz.  Writing
// G(X) = ∫∫_{Omega ∩ R ∩ {x > X}} (x - X) dy dz, the face contributes
// sign(n_x) (G(X_i) - G(X_i+1)) to voxel i of the column.  Each G is an
// integral of an affine function over a convex polygon, taken over its boundary
// from three families of segments -- edges of Omega, edges of R, and the chord
// x = X -- each clipped against the other two regions (Cyrus-Beck), so every
// lane keeps O(1) state.  Work items (face, rectangle, plane) are spread over
// the lanes of the wavefront that rebuilt the cell from its facets.
//
// The grid lines are evaluated at X_i + 1e-12 h (likewise in y and z): a
// vertex or face exactly on a grid line (lattice inputs) then has no tie; the
// overlap volumes move by at most 1e-12 of a voxel.
#include "rebuild.h"

template <int VPL>
struct GridMem {
    static constexpr int FMAX = 64 * VPL;      // face slots
    static constexpr int LOOP = 3 * 64 * VPL;  // vertex-face incidences (3 per vertex)
    static constexpr int ACC = 256 * VPL;      // voxels of a cell's box summed in LDS
    double vp[64 * VPL][3];  // vertex positions, grid frame (box origin at 0)
    uint32_t vt[64 * VPL];   // vertex triples
    double lp[LOOP][3];      // face vertex loops (seed-relative x, y, z), counter-clockwise in (y, z)
    int32_t loff[FMAX + 1];
    double fn[FMAX][4];      // face plane in the grid frame: n.g = d
    int32_t frect[FMAX][4];  // y range (j0, nj), z range (k0, nk)
    int32_t fpl[FMAX][2];    // planes strictly inside the face's x range: m0, count
    int32_t ipre[FMAX + 1];  // prefix of work items per face
    int32_t fid[FMAX];       // compacted face slots
    uint64_t iq[2][128];     // work items queued for integration (face, plane, rectangle offsets):
                             // [0] the faces' lowest planes (pi == 0), [1] planes that cut a face
    double acc[ACC];         // the cell's contributions per voxel of its box
    PolyMem<double, VPL> P;
};

struct GridArgs {
    const void *spos;
    const DevItem *items;
    const int32_t *cells;
    int64_t ncells;
    const int32_t *queue;
    int64_t queue_cap;
    int32_t *gqueue;          // cells the normal kernel could not hold, for the large kernel
    int64_t gqueue_cap;
    const int64_t *crow;
    const int32_t *ccnt;
    const uint8_t *cstat;
    const double *cvol;
    const double *crad;
    const int32_t *ctopo;     // topology records of the fast clip kernel
    const int32_t *cnf;
    const int32_t *cnv;
    int64_t npos;             // sorted particles (bound of a record's face tags)
    const int32_t *stage_ids;
    const int32_t *srow;
    const double *value;
    uint32_t *counters;
    double *grid;
    int nx, ny, nz;
    int seg;                  // large kernel: which queue (see grid_body)
    int n_large;              // fused launch: leading blocks that run the large kernel
};

__device__ __forceinline__ int64_t wrapi(int64_t i, int n) {
    int64_t r = i % n;
    return r < 0 ? r + n : r;
}

// A cell is smaller than a quarter of the box, so its voxel indices lie within one period of
// [0, n); the exact reduction runs only for an index that does not.
__device__ __forceinline__ int64_t wrap1(int64_t i, int n) {
    int64_t r = i < 0 ? i + n : (i >= n ? i - n : i);
    if (r < 0 || r >= n) r = wrapi(i, n);
    return r;
}

// q = a / b and a % b for 0 <= a, 1 <= b: a float quotient, then one correction step (exact for
// a < 2^22, where the float quotient is within one of the true one); integer division above
__device__ __forceinline__ int divmod_small(int a, int b, int &rem) {
    int q, r;
    if (a < (1 << 22)) {
        q = (int)((float)a * __builtin_amdgcn_rcpf((float)b));
        r = a - q * b;
        if (r < 0) {
            --q;
            r += b;
        }
        if (r >= b) {
            ++q;
            r -= b;
        }
    } else {
        q = a / b;
        r = a - q * b;
    }
    rem = r;
    return q;
}

// Area A of a region D in the (y, z) plane and G = ∫∫_D (x - X) dy dz, x the
// affine height of the face over D.  Both come from the boundary of D by
// Green's theorem, as a fan of triangles (O, p, q) over its directed boundary
// segments (p, q) with O the face's first vertex: each triangle adds its signed
// area times the mean of x - X at its corners.  Heights are taken from the
// face's own 3D vertices where a point lies on a face edge (interpolated), are 0
// on the chord x = X, and come from the plane equation only at points of R's
// edges inside the projection.  A face nearly parallel to x projects to a thin
// sliver on which the plane equation has a large slope; every point used lies
// in the sliver and every triangle has at most its area, so the rounding error
// stays at eps * (cell size)^3 instead of growing like 1/n_x.
struct Reg {
    double A, G;
};

// 1 / d from the hardware reciprocal and two Newton steps (each squares the relative error):
// within a few ulps of the correctly rounded quotient, without the division's branches
__device__ __forceinline__ double rcp_nr(double d) {
    double x = __builtin_amdgcn_rcp(d);
    x = fma(x, fma(-d, x, 1.0), x);
    x = fma(x, fma(-d, x, 1.0), x);
    return x;
}

// restrict the parameter interval [t0, t1] of a segment to g >= 0, g affine along it.  Free of
// branches: the lanes of a wave clip different segments, and a branch around the quotient
// would be taken by the whole wave whenever one lane needs it.  The quotient is used only when
// g0 and g1 differ in sign, so g0 - g1 is then not zero.
__device__ __forceinline__ void cyrus_beck(double g0, double g1, double &t0, double &t1) {
    const bool in0 = g0 >= 0.0, in1 = g1 >= 0.0;
    const double t = g0 * rcp_nr(g0 - g1);
    const double n0 = (!in0 && in1) ? fmax(t0, t) : t0;
    const double n1 = (in0 && !in1) ? fmin(t1, t) : t1;
    const bool none = !in0 && !in1;
    t0 = none ? 1.0 : n0;
    t1 = none ? 0.0 : n1;
}

// restrict [t0, t1] to lo <= a + t b <= hi (one coordinate of a segment against a slab), with
// ib = 1 / b for both sides; a segment parallel to the slab is kept or emptied whole
__device__ __forceinline__ void slab(double a, double b, double ib, double lo, double hi, double &t0, double &t1) {
    const double ta = (lo - a) * ib, tb = (hi - a) * ib;
    const bool flat = b == 0.0, inside = a >= lo && a <= hi;
    const double n0 = fmax(t0, fmin(ta, tb)), n1 = fmin(t1, fmax(ta, tb));
    t0 = flat ? (inside ? t0 : 1.0) : n0;
    t1 = flat ? (inside ? t1 : 0.0) : n1;
}

// D = Omega ∩ R ∩ H in coordinates relative to R's corner (Y0, Z0): Omega the
// counter-clockwise loop lp[o .. o+m) of seed-relative vertices,
// R = [Y0, Y0 + hy] x [Z0, Z0 + hz], H = {hs (e - ny y - nz z) > 0} if useH (the
// part of the face above x = X), with e given for the shifted coordinates and
// rnx = 1 / n_x.  One pass over Omega's edges clips each edge to R ∩ H and, for
// every edge, restricts R's four edges and the chord to its inner side; those
// segments are integrated after the pass.
template <int VPL, bool useH>
__device__ __forceinline__ Reg region_integrals(const GridMem<VPL> &S, int o, int m, double Y0, double Z0, double hy, double hz,
                                double hs, double e, double ny, double nz, double X, double rnx) {
    Reg D = {0.0, 0.0};
    auto gH = [&](double y, double z) { return hs * (e - ny * y - nz * z); };
    const double Oy = S.lp[o][1] - Y0, Oz = S.lp[o][2] - Z0, gO = S.lp[o][0] - X;
    auto tri = [&](double y0, double z0, double g0, double y1, double z1, double g1) {
        const double cr = (y0 - Oy) * (z1 - Oz) - (y1 - Oy) * (z0 - Oz);
        D.A += 0.5 * cr;
        D.G += cr * (gO + g0 + g1) * (1.0 / 6.0);
    };
    auto gplane = [&](double y, double z) { return gO - (ny * (y - Oy) + nz * (z - Oz)) * rnx; };
    // R's edges run counter-clockwise from corner r to corner r + 1
    const double ry[5] = {0.0, hy, hy, 0.0, 0.0}, rz[5] = {0.0, 0.0, hz, hz, 0.0};
    double rt0[4] = {0.0, 0.0, 0.0, 0.0}, rt1[4] = {1.0, 1.0, 1.0, 1.0};
    // the chord x = X: a segment through the point of the line nearest R's centre, long
    // enough to cross R, directed with H on its left (x - X = 0 on it), clipped to R
    double cy0 = 0.0, cz0 = 0.0, cy1 = 0.0, cz1 = 0.0, ct0 = 0.0, ct1 = 0.0;
    if constexpr (useH) {
        const double nn = ny * ny + nz * nz;
        const double cy = 0.5 * hy, cz = 0.5 * hz;
        const double sft = (ny * cy + nz * cz - e) / nn;
        const double py = cy - sft * ny, pz = cz - sft * nz;
        const double L = 4.0 * (hy + hz) / sqrt(nn);
        const double dy = -hs * nz * L, dz = hs * ny * L;
        cy0 = py - dy;
        cz0 = pz - dz;
        cy1 = py + dy;
        cz1 = pz + dz;
        ct1 = 1.0;
        slab(cy0, cy1 - cy0, rcp_nr(cy1 - cy0), 0.0, hy, ct0, ct1);
        slab(cz0, cz1 - cz0, rcp_nr(cz1 - cz0), 0.0, hz, ct0, ct1);
    }
    // (b) R's edges inside Omega come from where Omega's boundary crosses R's four lines.  Omega
    // is convex and counter-clockwise, so crossing a line z = c upwards bounds its chord on the
    // right and downwards on the left; crossing y = c rightwards bounds it from below and
    // leftwards from above.  A line that no edge crosses misses Omega.  Edge r of R runs from
    // corner r to corner r + 1 (counter-clockwise), t along it.
    const double ihy = 1.0 / hy, ihz = 1.0 / hz;
    int crossed[4] = {0, 0, 0, 0};
    double y0 = Oy, z0 = Oz, xa = gO;
    for (int k = 0; k < m; ++k) {
        const int k1 = (k + 1 == m) ? 0 : k + 1;
        const double y1 = S.lp[o + k1][1] - Y0, z1 = S.lp[o + k1][2] - Z0, xb = S.lp[o + k1][0] - X;
        const double dy = y1 - y0, dz = z1 - z0, dx = xb - xa;
        const double iby = rcp_nr(dy), ibz = rcp_nr(dz);
        // (a) the edge of Omega inside R ∩ H
        {
            double t0 = 0.0, t1 = 1.0;
            slab(y0, dy, iby, 0.0, hy, t0, t1);
            slab(z0, dz, ibz, 0.0, hz, t0, t1);
            if constexpr (useH) cyrus_beck(gH(y0, z0), gH(y1, z1), t0, t1);
            if (t0 < t1) tri(y0 + t0 * dy, z0 + t0 * dz, xa + t0 * dx, y0 + t1 * dy, z0 + t1 * dz, xa + t1 * dx);
        }
        // (b) crossings with z = 0 (edge 0, t = y / hy), y = hy (edge 1, t = z / hz),
        // z = hz (edge 2, t = (hy - y) / hy) and y = 0 (edge 3, t = (hz - z) / hz)
        {
            const bool up0 = z0 < 0.0 && !(z1 < 0.0), dn0 = !(z0 < 0.0) && z1 < 0.0;
            const bool up2 = z0 < hz && !(z1 < hz), dn2 = !(z0 < hz) && z1 < hz;
            const bool rt1_ = y0 < hy && !(y1 < hy), lf1 = !(y0 < hy) && y1 < hy;
            const bool rt3 = y0 < 0.0 && !(y1 < 0.0), lf3 = !(y0 < 0.0) && y1 < 0.0;
            const double yc0 = (y0 + (0.0 - z0) * ibz * dy) * ihy;
            const double yc2 = (hy - (y0 + (hz - z0) * ibz * dy)) * ihy;
            const double zc1 = (z0 + (hy - y0) * iby * dz) * ihz;
            const double zc3 = (hz - (z0 + (0.0 - y0) * iby * dz)) * ihz;
            rt1[0] = up0 ? fmin(rt1[0], yc0) : rt1[0];
            rt0[0] = dn0 ? fmax(rt0[0], yc0) : rt0[0];
            rt0[2] = up2 ? fmax(rt0[2], yc2) : rt0[2];
            rt1[2] = dn2 ? fmin(rt1[2], yc2) : rt1[2];
            rt0[1] = rt1_ ? fmax(rt0[1], zc1) : rt0[1];
            rt1[1] = lf1 ? fmin(rt1[1], zc1) : rt1[1];
            rt1[3] = rt3 ? fmin(rt1[3], zc3) : rt1[3];
            rt0[3] = lf3 ? fmax(rt0[3], zc3) : rt0[3];
            crossed[0] |= (up0 || dn0) ? 1 : 0;
            crossed[1] |= (rt1_ || lf1) ? 1 : 0;
            crossed[2] |= (up2 || dn2) ? 1 : 0;
            crossed[3] |= (rt3 || lf3) ? 1 : 0;
        }
        // (c) the chord restricted to the inner side of this edge
        if constexpr (useH) cyrus_beck(dy * (cz0 - z0) - dz * (cy0 - y0), dy * (cz1 - z0) - dz * (cy1 - y0), ct0, ct1);
        y0 = y1;
        z0 = z1;
        xa = xb;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        rt0[r] = crossed[r] ? rt0[r] : 1.0;
        rt1[r] = crossed[r] ? rt1[r] : 0.0;
    }
    // (b) edges of R inside Omega ∩ H
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const double qy0 = ry[r], qz0 = rz[r], qy1 = ry[r + 1], qz1 = rz[r + 1];
        double t0 = rt0[r], t1 = rt1[r];
        if constexpr (useH) cyrus_beck(gH(qy0, qz0), gH(qy1, qz1), t0, t1);
        if (t0 < t1) {
            const double dy = qy1 - qy0, dz = qz1 - qz0;
            const double ya = qy0 + t0 * dy, za = qz0 + t0 * dz, yb = qy0 + t1 * dy, zb = qz0 + t1 * dz;
            tri(ya, za, gplane(ya, za), yb, zb, gplane(yb, zb));
        }
    }
    // (c) the chord inside Omega ∩ R
    if (useH && ct0 < ct1) {
        const double ey = cy1 - cy0, ez = cz1 - cz0;
        tri(cy0 + ct0 * ey, cz0 + ct0 * ez, 0.0, cy0 + ct1 * ey, cz0 + ct1 * ez, 0.0);
    }
    return D;
}

// The deposit of one wavefront (wid its index in the block's LDS).  The large kernel
// (RETRY) takes queued cells: seg 0 both queues, seg 1 the clip's retry queue only (counter
// CTR_GRID_RETRY), seg 2 only the cells the normal kernel handed over (counter CTR_GRID, zeroed
// after the normal kernel has run).
template <typename PT4, int VPL, bool RETRY>
__device__ __forceinline__ void grid_body(const GridArgs &A, char *smem, int wid) {
    using M = GridMem<VPL>;
    M &S = *reinterpret_cast<M *>(smem + (size_t)wid * sizeof(M));
    const int lane = lane_id();
    const uint64_t mybit = 1ull << lane;
    const uint64_t lt = lanemask_lt();
    const DevItem &it = A.items[0];
    const double h[3] = {it.L[0] / A.nx, it.L[1] / A.ny, it.L[2] / A.nz};
    const double ih[3] = {1.0 / h[0], 1.0 / h[1], 1.0 / h[2]};
    const double del[3] = {1e-12 * h[0], 1e-12 * h[1], 1e-12 * h[2]};  // grid-line offset
    const double hv = h[0] * h[1] * h[2];
    const int dims[3] = {A.nx, A.ny, A.nz};
    const int64_t nq = RETRY ? (int64_t)min((uint64_t)A.counters[CTR_QUEUE], (uint64_t)A.queue_cap) : 0;
    int64_t w_lo = 0, ntodo = RETRY ? nq + (int64_t)min((uint64_t)A.counters[CTR_GRID_Q], (uint64_t)A.gqueue_cap)
                                    : A.ncells;
    int ctr = RETRY ? CTR_GRID_RETRY : CTR_GRID;
    if (RETRY && A.seg == 1) ntodo = nq;
    if (RETRY && A.seg == 2) {
        w_lo = nq;
        ctr = CTR_GRID;
    }

    // Cells are taken GB at a time: lane l loads the scalars of the batch's cell l (the latency
    // of those dependent loads is paid once per batch), a cell inside one voxel (its ball of
    // radius R, the largest vertex distance, is) deposits its whole volume from its lane, and
    // the wave then rebuilds the other cells one after another.
    constexpr int GB = 16;
    for (;;) {
        int64_t wb = 0;
        if (lane == 0) wb = (int64_t)atomicAdd(&A.counters[ctr], (uint32_t)GB);
        wb = (int64_t)uni_i((int)__shfl((long long)wb, 0)) + w_lo;
        if (wb >= ntodo) break;
        const int64_t wl = wb + lane;
        int32_t cl = 0;
        double vl = 0.0, xl = 0.0, yl = 0.0, zl = 0.0;
        bool todo = false;
        if (lane < GB && wl < ntodo) {
            cl = RETRY ? (wl < nq ? A.queue[wl] : A.gqueue[wl - nq]) : (int32_t)wl;
            const uint8_t st = A.cstat[cl];
            if ((RETRY || !(st & VT_CELL_RETRIED)) && !(st & VT_CELL_FAILED)) {
                const int32_t j0 = A.cells[cl];
                vl = A.value[A.srow[j0]];
                if (vl != 0.0) {
                    gpos<PT4>(A.spos, j0, xl, yl, zl);
                    const double xq[3] = {xl, yl, zl};
                    const double rc = A.crad[cl];
                    int64_t va[3];
                    bool one = true;
                    for (int a = 0; a < 3; ++a) {
                        const double g = xq[a] - it.lo[a];
                        va[a] = (int64_t)floor((g - rc - del[a]) * ih[a]);
                        one = one && va[a] == (int64_t)floor((g + rc - del[a]) * ih[a]);
                    }
                    if (one) {
                        int64_t g = (wrapi(va[0], dims[0]) * dims[1] + wrapi(va[1], dims[1])) * dims[2] + wrapi(va[2], dims[2]);
                        unsafeAtomicAdd(&A.grid[g], vl * A.cvol[cl] / hv);
                    } else {
                        todo = true;
                    }
                }
            }
        }
        uint64_t tm = __ballot(todo);
        while (tm) {
            const int l = __builtin_ctzll(tm);
            tm &= tm - 1ull;
            const int32_t c = (int32_t)readlane_u32((uint32_t)cl, l);
            const double val = readlane_d(vl, l);
            const double sx = readlane_d(xl, l), sy = readlane_d(yl, l), sz = readlane_d(zl, l);
            const double xs[3] = {sx, sy, sz};
            const double vscale = val / hv;
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
            const CellSrc src{A.spos, A.ctopo, A.cnf, A.cnv, A.npos, A.crow, A.ccnt, A.stage_ids, A.counters};
            const int rb = rebuild_cell<PT4, VPL, RETRY>(src, it, S.P, P, c, sx, sy, sz, blo, bhi);
            if (rb == REBUILD_OVERFLOW) {
                // the cell outgrows the normal kernel: the large one takes it
                if (lane == 0) {
                    const uint32_t qi = atomicAdd(&A.counters[CTR_GRID_Q], 1u);
                    if ((int64_t)qi < A.gqueue_cap) A.gqueue[qi] = c;
                    else atomicOr(&A.counters[CTR_STATUS], VT_DEV_CAPACITY);
                }
                continue;
            }
            if (rb == REBUILD_FAILED) {
                if (lane == 0) atomicOr(&A.counters[CTR_STATUS], VT_DEV_CAPACITY);
                continue;
            }
            // ---- vertices in the grid frame, bounding box, voxel ranges
            double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
#pragma unroll
            for (int s = 0; s < VPL; ++s) {
                if (P.alive[s] & mybit) {
                    const double v[3] = {P.vx[s], P.vy[s], P.vz[s]};
                    for (int a = 0; a < 3; ++a) {
                        S.vp[s * 64 + lane][a] = v[a];
                        mn[a] = fmin(mn[a], v[a]);
                        mx[a] = fmax(mx[a], v[a]);
                    }
                    S.vt[s * 64 + lane] = P.vt[s];
                }
            }
            // seed position in the grid frame; grid line m of axis a lies at m h + del - g0 from the seed
            const double g0[3] = {xs[0] - it.lo[0], xs[1] - it.lo[1], xs[2] - it.lo[2]};
            int64_t i0[3], i1[3];
            bool sane = true;
            for (int a = 0; a < 3; ++a) {
                mn[a] = uni_d(wave_min(mn[a]));
                mx[a] = uni_d(wave_max(mx[a]));
                // a cell spans less than the box (2R < L/2 when periodic): its voxel range is at most
                // the grid's; anything else (a vertex not finite, or far away) is a broken cell, and
                // it must not drive the loops below
                const double lo_ = (g0[a] + mn[a] - del[a]) * ih[a], hi_ = (g0[a] + mx[a] - del[a]) * ih[a];
                sane = sane && isfinite(lo_) && isfinite(hi_) && hi_ >= lo_ && hi_ - lo_ <= (double)dims[a] + 1.0 &&
                       fabs(lo_) < 1e15 && fabs(hi_) < 1e15;
                i0[a] = sane ? (int64_t)floor(lo_) : 0;
                i1[a] = sane ? (int64_t)floor(hi_) : 0;
            }
            if (!sane) {
                if (lane == 0) atomicOr(&A.counters[CTR_STATUS], VT_DEV_TOPOLOGY);
                continue;
            }
            if (i0[0] == i1[0] && i0[1] == i1[1] && i0[2] == i1[2]) {
                if (lane == 0) {
                    int64_t g = (wrapi(i0[0], dims[0]) * dims[1] + wrapi(i0[1], dims[1])) * dims[2] + wrapi(i0[2], dims[2]);
                    unsafeAtomicAdd(&A.grid[g], val * A.cvol[c] / hv);
                }
                continue;
            }
            // the cell's voxel box: contributions are summed in LDS when it fits, and each voxel
            // then takes one global atomic
            const int64_t bx = i1[0] - i0[0] + 1, by = i1[1] - i0[1] + 1, bz = i1[2] - i0[2] + 1;
            const int nacc = bx * by * bz <= M::ACC ? (int)(bx * by * bz) : 0;
            for (int t = lane; t < nacc; t += 64) S.acc[t] = 0.0;
            // ---- faces: compact the alive ones
            int nf = 0;
#pragma unroll
            for (int r = 0; r < VPL; ++r) {
                const uint64_t m = P.fa[r];
                if (m & mybit) S.fid[nf + __popcll(m & lt)] = r * 64 + lane;
                nf += __popcll(m);
            }
            wave_sync();
            // the vertex after u on face f, counter-clockwise seen from outside
            auto next_on = [&](int f, const uint64_t *mf, int u) -> int {
                const uint32_t t = S.vt[u];
                const int t0 = t & 0xFF, t1 = (t >> 8) & 0xFF, t2 = (t >> 16) & 0xFF;
                const int cf = (t0 == f) ? t2 : (t1 == f) ? t0 : t1;
                int nx_ = -1;
#pragma unroll
                for (int ww = 0; ww < VPL; ++ww) {
                    uint64_t x = mf[ww] & S.P.fm[cf][ww];
                    if (ww == (u >> 6)) x &= ~(1ull << (u & 63));
                    if (nx_ < 0 && x) nx_ = ww * 64 + __builtin_ctzll(x);
                }
                return nx_;
            };
            // loop lengths (every vertex on a face is in its mask, so a face's loop has as many
            // vertices as its mask has bits; the loop walk below checks that it closes after as
            // many steps) and planes in the grid frame
            int carry = 0;
            for (int base = 0; base < nf; base += 64) {
                const int q = base + lane;
                int len = 0, f = 0;
                if (q < nf) {
                    f = S.fid[q];
#pragma unroll
                    for (int ww = 0; ww < VPL; ++ww) len += __popcll(S.P.fm[f][ww]);
                }
                if constexpr (VPL == 1) {
                    // faces in order of loop length: the work items a wave takes at once then
                    // mostly share a loop length, and fewer lanes idle in the loop over edges
                    uint64_t kk[1] = {q < nf ? (((uint64_t)len << 8) | (uint64_t)lane) : ~0ull};
                    bitonic_u64<1>(kk);
                    const int src = (int)(kk[0] & 63ull);
                    const int len_s = __shfl(len, src), f_s = __shfl(f, src);
                    len = q < nf ? len_s : 0;
                    f = f_s;
                    if (q < nf) S.fid[q] = f;
                }
                if (q < nf) {
                    const P4<double> &pf = S.P.pl64[f];
                    S.fn[q][0] = pf.x;
                    S.fn[q][1] = pf.y;
                    S.fn[q][2] = pf.z;
                    S.fn[q][3] = pf.d;  // seed-relative plane n.v = d
                }
                int tot;
                const int pre = wave_excl_scan(len, &tot);
                if (q < nf) S.loff[q] = carry + pre;
                carry += tot;
            }
            if (lane == 0) S.loff[nf] = carry;
            wave_sync();
            if (carry > M::LOOP) {
                if (lane == 0) {
                    atomicOr(&A.counters[CTR_STATUS], VT_DEV_CAPACITY);
                    atomicOr(&A.counters[CTR_DEBUG], 1u << 16);
                }
                continue;
            }
            // loops, counter-clockwise in the (y, z) projection (faces seen from -x are reversed);
            // extents and work items: rectangles x (1 + planes strictly inside the face's x range)
            int nitem = 0;
            bool big = false, open_loop = false;
            for (int base = 0; base < nf; base += 64) {
                const int q = base + lane;
                int items = 0;
                if (q < nf) {
                    const int f = S.fid[q];
                    uint64_t mf[VPL];
                    int u0 = -1;
#pragma unroll
                    for (int ww = 0; ww < VPL; ++ww) {
                        mf[ww] = S.P.fm[f][ww];
                        if (u0 < 0 && mf[ww]) u0 = ww * 64 + __builtin_ctzll(mf[ww]);
                    }
                    const int o = S.loff[q], m = S.loff[q + 1] - o;
                    const bool rev = S.fn[q][0] < 0.0;
                    double b[6] = {1e300, -1e300, 1e300, -1e300, 1e300, -1e300};
                    int u = u0, k = 0;
                    for (; k < m && u >= 0; ++k) {
                        const double *p = S.vp[u];
                        double *lq = S.lp[o + (rev ? m - 1 - k : k)];
                        for (int a = 0; a < 3; ++a) {
                            lq[a] = p[a];
                            b[2 * a] = fmin(b[2 * a], p[a]);
                            b[2 * a + 1] = fmax(b[2 * a + 1], p[a]);
                        }
                        u = next_on(f, mf, u);
                    }
                    if (k != m || u != u0) open_loop = true;
                    const double nlen = sqrt(S.fn[q][0] * S.fn[q][0] + S.fn[q][1] * S.fn[q][1] + S.fn[q][2] * S.fn[q][2]);
                    // faces parallel to x add nothing (n_x = 0); nearly parallel ones are bounded by 1e-12 of a voxel
                    if (fabs(S.fn[q][0]) > 1e-12 * nlen) {
                        const int64_t ja = (int64_t)floor((g0[1] + b[2] - del[1]) * ih[1]);
                        const int64_t jb = (int64_t)floor((g0[1] + b[3] - del[1]) * ih[1]);
                        const int64_t ka = (int64_t)floor((g0[2] + b[4] - del[2]) * ih[2]);
                        const int64_t kb = (int64_t)floor((g0[2] + b[5] - del[2]) * ih[2]);
                        // planes X_m = m h + del with xmin < X_m < xmax (grid frame)
                        const int64_t m0 = (int64_t)floor((g0[0] + b[0] - del[0]) * ih[0]) + 1;
                        const int64_t m1 = (int64_t)ceil((g0[0] + b[1] - del[0]) * ih[0]);
                        S.frect[q][0] = (int)ja;
                        S.frect[q][1] = (int)(jb - ja + 1);
                        S.frect[q][2] = (int)ka;
                        S.frect[q][3] = (int)(kb - ka + 1);
                        S.fpl[q][0] = (int)m0;
                        S.fpl[q][1] = (int)(m1 > m0 ? m1 - m0 : 0);
                        // queued items hold the rectangle offsets in 20 bits and the plane index in 16
                        if (jb - ja + 1 >= (1 << 20) || kb - ka + 1 >= (1 << 20) || m1 - m0 + 1 >= (1 << 16)) big = true;
                        else items = S.frect[q][1] * S.frect[q][3] * (1 + S.fpl[q][1]);
                    }
                }
                int tot;
                const int pre = wave_excl_scan(items, &tot);
                if (q < nf) S.ipre[q] = nitem + pre;
                nitem += tot;
            }
            if (lane == 0) S.ipre[nf] = nitem;
            wave_sync();
            nitem = uni_i(nitem);
            if (__ballot(big)) {
                if (lane == 0) atomicOr(&A.counters[CTR_STATUS], VT_DEV_CAPACITY);
                continue;
            }
            if (__ballot(open_loop)) {
                if (lane == 0) atomicOr(&A.counters[CTR_STATUS], VT_DEV_TOPOLOGY);
                continue;
            }
            // ---- work items
            auto emit = [&](int64_t i, int64_t j, int64_t k, double v) {
                if (v == 0.0) return;
                const int64_t li = i - i0[0], lj = j - i0[1], lk = k - i0[2];
                if (nacc > 0 && li >= 0 && li < bx && lj >= 0 && lj < by && lk >= 0 && lk < bz) {
                    unsafeAtomicAdd(&S.acc[(li * by + lj) * bz + lk], v);
                    return;
                }
                int64_t g = (wrap1(i, dims[0]) * dims[1] + wrap1(j, dims[1])) * dims[2] + wrap1(k, dims[2]);
                unsafeAtomicAdd(&A.grid[g], v * vscale);
            };
            // The item's geometry: rectangle corner (seed-relative; integrals are taken relative
            // to it), the face plane n.v = d, and the plane X.  With y, z relative to the corner the
            // plane's value at (X, Y0, Z0) is e = d - nx X - ny Y0 - nz Z0.  pi == 0: the face over
            // this rectangle against the plane below its x minimum (full voxels below it, and the
            // voxel holding its x minimum); pi > 0: G at the plane X_m inside the face's x range,
            // -G to voxel m-1 and +G to voxel m.
            struct ItemGeo {
                double Y0, Z0, X, e, hs;
                int64_t jj, kk, mm;
            };
            auto geometry = [&](int q, int pi, int rj, int rk) -> ItemGeo {
                ItemGeo G_;
                G_.jj = S.frect[q][0] + rj;
                G_.kk = S.frect[q][2] + rk;
                G_.Y0 = G_.jj * h[1] + del[1] - g0[1];
                G_.Z0 = G_.kk * h[2] + del[2] - g0[2];
                G_.mm = (int64_t)S.fpl[q][0] + pi - 1;
                G_.X = G_.mm * h[0] + del[0] - g0[0];
                G_.e = S.fn[q][3] - S.fn[q][0] * G_.X - S.fn[q][1] * G_.Y0 - S.fn[q][2] * G_.Z0;
                G_.hs = S.fn[q][0] > 0.0 ? 1.0 : -1.0;
                return G_;
            };
            // Items are classified 64 at a time: hs (e - ny y - nz z), positive where the face lies
            // above X, is affine over R, so its extremes are at R's corners; a face entirely below X
            // over R adds nothing.  A plane with the face entirely above it over R needs no item of
            // its own: G there is an affine function of X over the same region, G(X) = G(X0) +
            // (X0 - X) A, with X0 the plane below the face's x minimum, whose item (pi == 0)
            // integrates A and G(X0) and also emits these planes' contributions (they are the planes
            // from the lowest up to the first that cuts the face over R, as the bound above falls
            // with X).  The others are queued and integrated 64 at a time, so the lanes of an
            // integration pass all have an item.
            // The two kinds of item go to rings of their own and are integrated 64 at a time, each
            // kind by its own specialisation: a face's lowest plane (pi == 0) never clips the face
            // with H, and a queued plane above it (pi > 0) always does, since it is queued only
            // when the face lies on both sides of it over R (above_min < 0).
            int head[2] = {0, 0}, qn[2] = {0, 0};
            auto integrate = [&](auto kind, bool last) {
                constexpr bool useH = decltype(kind)::value;
                constexpr int w = useH ? 1 : 0;
                while (qn[w] >= 64 || (last && qn[w] > 0)) {
                    wave_sync();
                    const int take = qn[w] < 64 ? qn[w] : 64;
                    if (lane < take) {
                        const uint64_t d = S.iq[w][(head[w] + lane) & 127];
                        const int q = (int)(d & 0xFFull), pi = (int)((d >> 8) & 0xFFFFull);
                        const int rj = (int)((d >> 24) & 0xFFFFFull), rk = (int)((d >> 44) & 0xFFFFFull);
                        const ItemGeo g = geometry(q, pi, rj, rk);
                        const double nx_ = S.fn[q][0], ny_ = S.fn[q][1], nz_ = S.fn[q][2];
                        const double hs = g.hs, rnx = 1.0 / nx_;
                        const int o = S.loff[q], m = S.loff[q + 1] - o;
                        const Reg Rg = region_integrals<VPL, useH>(S, o, m, g.Y0, g.Z0, h[1], h[2], hs, g.e, ny_, nz_, g.X, rnx);
                        const double G = hs * Rg.G;
                        if constexpr (!useH) {
                            if (Rg.A != 0.0) {
                                // full voxels below the face's x minimum, within the cell's own range
                                const int64_t iend = g.mm < i0[0] + bx ? g.mm : i0[0] + bx;
                                for (int64_t i = i0[0]; i < iend; ++i) emit(i, g.jj, g.kk, hs * h[0] * Rg.A);
                                emit(g.mm, g.jj, g.kk, G);
                                // the planes with the face entirely above them over R (classified
                                // with the same geometry and bound, so none is queued as well)
                                const double cy_ = -hs * ny_ * h[1], cz_ = -hs * nz_ * h[2];
                                const int npl = S.fpl[q][1];
#pragma unroll 1
                                for (int p = 1; p <= npl; ++p) {
                                    // geometry(q, p, rj, rk)'s X and e, the same expressions
                                    const int64_t mp = (int64_t)S.fpl[q][0] + p - 1;
                                    const double Xp = mp * h[0] + del[0] - g0[0];
                                    const double ep = S.fn[q][3] - S.fn[q][0] * Xp - S.fn[q][1] * g.Y0 - S.fn[q][2] * g.Z0;
                                    if (hs * ep + fmin(0.0, cy_) + fmin(0.0, cz_) < 0.0) break;
                                    const double Gp = hs * (Rg.G + (g.X - Xp) * Rg.A);
                                    emit(mp - 1, g.jj, g.kk, -Gp);
                                    emit(mp, g.jj, g.kk, Gp);
                                }
                            }
                        } else {
                            emit(g.mm - 1, g.jj, g.kk, -G);
                            emit(g.mm, g.jj, g.kk, G);
                        }
                    }
                    head[w] += take;
                    qn[w] -= take;
                    wave_sync();
                }
            };
            for (int base = 0; base < nitem; base += 64) {
                const int item = base + lane;
                bool need = false;
                int kind = 0;
                uint64_t desc = 0;
                if (item < nitem) {
                    int lo = 0, hi = nf - 1;
                    while (lo < hi) {
                        int mid = (lo + hi + 1) >> 1;
                        if (S.ipre[mid] <= item) lo = mid; else hi = mid - 1;
                    }
                    const int q = lo;
                    int pi, rj;
                    const int r = divmod_small(item - S.ipre[q], 1 + S.fpl[q][1], pi);
                    const int rk = divmod_small(r, S.frect[q][1], rj);
                    const ItemGeo g = geometry(q, pi, rj, rk);
                    const double cy_ = -g.hs * S.fn[q][1] * h[1], cz_ = -g.hs * S.fn[q][2] * h[2];
                    const double above_max = g.hs * g.e + fmax(0.0, cy_) + fmax(0.0, cz_);
                    const double above_min = g.hs * g.e + fmin(0.0, cy_) + fmin(0.0, cz_);
                    need = pi == 0 || (above_max > 0.0 && above_min < 0.0);
                    kind = pi == 0 ? 0 : 1;
                    desc = (uint64_t)q | ((uint64_t)pi << 8) | ((uint64_t)rj << 24) | ((uint64_t)rk << 44);
                }
                const uint64_t n0 = __ballot(need && kind == 0), n1 = __ballot(need && kind == 1);
                if (need) {
                    const uint64_t nb = kind == 0 ? n0 : n1;
                    S.iq[kind][(head[kind] + qn[kind] + __popcll(nb & lt)) & 127] = desc;
                }
                qn[0] += __popcll(n0);
                qn[1] += __popcll(n1);
                const bool last = base + 64 >= nitem;
                integrate(std::integral_constant<bool, false>(), last);
                integrate(std::integral_constant<bool, true>(), last);
            }
            wave_sync();
            for (int t = lane; t < nacc; t += 64) {
                const double v = S.acc[t];
                if (v != 0.0) {
                    const int64_t lk = t % bz, lj = (t / bz) % by, li = t / (by * bz);
                    const int64_t g = (wrap1(i0[0] + li, dims[0]) * dims[1] + wrap1(i0[1] + lj, dims[1])) * dims[2] +
                                      wrap1(i0[2] + lk, dims[2]);
                    unsafeAtomicAdd(&A.grid[g], v * vscale);
                }
            }
        }
    }
}

template <typename PT4, int VPL, bool RETRY>
__global__ void __launch_bounds__(256) k_grid(GridArgs A) {
    extern __shared__ char smem[];
    grid_body<PT4, VPL, RETRY>(A, smem, (int)(threadIdx.x >> 6));
}

// The normal deposit and, in the first n_large blocks (one wavefront each), the large kernel
// over the clip's retry queue, so that the few slow cells next to halos overlap the bulk.
template <typename PT4>
__global__ void __launch_bounds__(256) k_grid_fused(GridArgs A) {
    extern __shared__ char smem[];
    if ((int)blockIdx.x < A.n_large) {
        if ((threadIdx.x >> 6) != 0) return;
        grid_body<PT4, 4, true>(A, smem, 0);
    } else {
        grid_body<PT4, 1, false>(A, smem, (int)(threadIdx.x >> 6));
    }
}

// ---------------------------------------------------------------- nearest-particle sampling
// A cheaper grid (the paper lists grid variants as future work): every sample point takes the
// value of the particle nearest to it (periodic minimum image, FP64 squared distances
// ex*ex + ey*ey + ez*ez; ties to the smaller global id), i.e. of the Voronoi cell that contains
// it.  A voxel averages the sub^3 points at its sub-cell centres.
//
// The tessellation is already built, so each cell claims its points: a wavefront per cell walks
// the sample points within R of its seed (R its largest vertex distance) and claims a point
// when the seed is nearer than every facet neighbour (or as near, with the smaller global id).
// In exact arithmetic the cell is the intersection of its facet half-spaces, so the one cell
// holding a point claims it; the comparisons are the reference's own squared distances, and
// the claims go through a 64-bit atomic minimum on (global id, sorted index).  A point no cell
// claims (rounding at a boundary, or a cell with more candidate points or facets than a wave takes)
// is found by its own exact search.  With several points per voxel a cell's sphere holds
// sub^3 times as many candidates, and tiles of points do better: one wavefront takes a 4 x 4 x 4
// tile (a lane each) and scans one candidate list for the tile, the particles of the Morton
// cells covering the tile widened by r, staged through LDS 64 at a time; a lane is done when its
// best distance is below its distance to the sides of the covered cells less two key quanta,
// otherwise r doubles, and a tile whose region holds more than VT_SAMPLE_DENSE particles lets
// every lane search on its own through finer cells.  The minimum-image shift uses rint(e / L)
// with 1 / L precomputed; it can round differently from the quotient only near |e| = L / 2,
// where no nearest particle lies.
#define VT_CLAIM_MAX 65536  // candidate points above which a cell leaves its points to the search
#define VT_SAMPLE_DENSE 4096  // tiles: candidates above which a tile's lanes search on their own
#define VT_CLAIM_NBR 160    // facet neighbours staged per cell (the large clip kernel keeps at most 136)

struct SampleArgs {
    const void *spos;
    const uint64_t *skey;
    const int32_t *tab;
    const int32_t *sgid;
    const int32_t *srow;
    const DevItem *items;
    const int32_t *cells;       // cell slot -> sorted index of its seed
    const uint8_t *cstat;
    const double *crad;         // largest vertex distance per cell
    const int64_t *crow;        // facet list: stage_ids[crow .. crow + ccnt)
    const int32_t *ccnt;
    const int32_t *stage_ids;
    int64_t ncells;
    const double *value;
    double *grid;
    int32_t *nearest;           // global id per voxel (of its last point), or null
    unsigned long long *slot;   // per sample point: (global id << 32) | sorted index, ~0 unclaimed
    int nx, ny, nz, sub;
    double r0;                  // tiles: first widening (the mean inter-particle distance)
};

// sample point (fine index f along axis a): voxel f / sub, sub-cell f % sub, at the sub-cell centre
__device__ __forceinline__ double sample_coord(const DevItem &it, int a, int dim, int sub, int64_t f) {
    const double h = it.L[a] / dim;
    return it.lo[a] + ((double)(f / sub) + ((double)(f % sub) + 0.5) / (double)sub) * h;
}

// the same for f < 2^22 (the quotient by the float reciprocal, corrected)
__device__ __forceinline__ double sample_coord32(const DevItem &it, int a, int dim, int sub, int f) {
    const double h = it.L[a] / dim;
    int rem;
    const int vox = divmod_small(f, sub, rem);
    return it.lo[a] + ((double)vox + ((double)rem + 0.5) / (double)sub) * h;
}

// i in [-n, 2n) to [0, n)
__device__ __forceinline__ int wrap_once(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

struct SampleMem {
    int32_t rb[512];    // covering cells: range starts
    int32_t rp[513];    // prefix of range lengths
    double px[64], py[64], pz[64];
    int32_t pg[64], pj[64];
};

__device__ __forceinline__ int32_t lower_key(const uint64_t *skey, int32_t a, int32_t c, uint64_t k) {
    while (a < c) {
        const int32_t mid = (a + c) >> 1;
        if (skey[mid] < k) a = mid + 1; else c = mid;
    }
    return a;
}

// sorted-index range of Morton cell m at level l (dense table at levels <= T, binary search below)
__device__ __forceinline__ void morton_range(const SampleArgs &A, const DevItem &it, int l, uint64_t m, int32_t &b,
                                             int32_t &e) {
    if (l <= it.T) {
        const int sh = 3 * (it.T - l);
        b = A.tab[it.tab_off + (int64_t)(m << sh)];
        e = A.tab[it.tab_off + (int64_t)((m + 1) << sh)];
    } else {
        const uint64_t mT = m >> (3 * (l - it.T));
        const int32_t lo = A.tab[it.tab_off + (int64_t)mT], hi = A.tab[it.tab_off + (int64_t)mT + 1];
        const int sh = 3 * (VT_MORTON_BITS - l);
        b = lower_key(A.skey, lo, hi, m << sh);
        e = lower_key(A.skey, b, hi, (m + 1) << sh);
    }
}

// One point's nearest particle by its own search (used where a tile's region is dense): from the
// point's Morton cell (coarsened while empty, refined while it holds more than 32 particles),
// shells of cells at growing Chebyshev distance k until the best distance is below the point's
// distance to the sides of the (2k+1)^3 block less two key quanta.
template <typename PT4>
__device__ int32_t nearest_particle(const SampleArgs &A, const DevItem &it, const double q[3], const double invL[3],
                                    int32_t &bg) {
    int64_t qq[3];
    for (int a = 0; a < 3; ++a) qq[a] = vt_qclamp(vt_qraw(q[a], it.lo[a], it.inv_res));
    auto cell_at = [&](int l) -> uint64_t {
        const int sh = VT_MORTON_BITS - l;
        return vt_morton((uint64_t)qq[0] >> sh, (uint64_t)qq[1] >> sh, (uint64_t)qq[2] >> sh);
    };
    int l = it.T;
    int32_t b, e;
    morton_range(A, it, l, cell_at(l), b, e);
    while (e == b && l > 1) {
        --l;
        morton_range(A, it, l, cell_at(l), b, e);
    }
    while (e - b > 32 && l < VT_MORTON_BITS) {
        int32_t b2, e2;
        morton_range(A, it, l + 1, cell_at(l + 1), b2, e2);
        if (e2 == b2) break;
        ++l;
        b = b2;
        e = e2;
    }
    const double quantum = it.S / (double)(1 << VT_MORTON_BITS);
    const double side = it.S / (double)(1ll << l);
    const int64_t ncl = 1ll << l;
    const int sh = VT_MORTON_BITS - l;
    const int64_t cq[3] = {qq[0] >> sh, qq[1] >> sh, qq[2] >> sh};
    // the point's distance to the nearest side of its own cell
    double edge = 1e300;
    for (int a = 0; a < 3; ++a) {
        const double b0 = it.lo[a] + (double)cq[a] * side;
        edge = fmin(edge, fmin(q[a] - b0, b0 + side - q[a]));
    }
    double best = 1e300;
    int32_t bj = -1;
    bg = 0x7FFFFFFF;
    for (int k = 0;; ++k) {
        for (int dx = -k; dx <= k; ++dx)
            for (int dy = -k; dy <= k; ++dy)
                for (int dz = -k; dz <= k; ++dz) {
                    if (max(abs(dx), max(abs(dy), abs(dz))) != k) continue;
                    const uint64_t cx = (uint64_t)(((cq[0] + dx) % ncl + ncl) % ncl);
                    const uint64_t cy = (uint64_t)(((cq[1] + dy) % ncl + ncl) % ncl);
                    const uint64_t cz = (uint64_t)(((cq[2] + dz) % ncl + ncl) % ncl);
                    int32_t cb, ce;
                    morton_range(A, it, l, vt_morton(cx, cy, cz), cb, ce);
                    for (int32_t j = cb; j < ce; ++j) {
                        double px, py, pz;
                        gpos<PT4>(A.spos, j, px, py, pz);
                        double ex = px - q[0], ey = py - q[1], ez = pz - q[2];
                        ex -= it.L[0] * rint(ex * invL[0]);
                        ey -= it.L[1] * rint(ey * invL[1]);
                        ez -= it.L[2] * rint(ez * invL[2]);
                        const double d2 = ex * ex + ey * ey + ez * ez;
                        const int32_t gj = A.sgid[j];
                        if (d2 < best || (d2 == best && gj < bg)) {
                            best = d2;
                            bg = gj;
                            bj = j;
                        }
                    }
                }
        const double reach = (double)k * side + edge - 2.0 * quantum;
        if (bj >= 0 && reach > 0.0 && best < reach * reach) break;
        if (2 * k + 1 >= ncl) break;  // the block covers the whole box
    }
    return bj;
}

// One wavefront per cell: the facet neighbours are staged in LDS once (nearest first when
// there are at most 64), and the lanes take the cell's candidate points 64 at a time.
struct ClaimMem {
    double px[VT_CLAIM_NBR], py[VT_CLAIM_NBR], pz[VT_CLAIM_NBR];
    int32_t pg[VT_CLAIM_NBR];
};

template <typename PT4>
__global__ void __launch_bounds__(256) k_sample_claim(SampleArgs A) {
    __shared__ ClaimMem Ms[4];
    ClaimMem &M = Ms[threadIdx.x >> 6];
    const int lane = threadIdx.x & 63;
    const DevItem it = uniform_item(A.items[0]);
    const int sub = A.sub;
    const int dims[3] = {A.nx, A.ny, A.nz};
    const int64_t F[3] = {(int64_t)A.nx * sub, (int64_t)A.ny * sub, (int64_t)A.nz * sub};
    const double invL[3] = {1.0 / it.L[0], 1.0 / it.L[1], 1.0 / it.L[2]};
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t c = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); c < A.ncells; c += nwaves) {
        if (A.cstat[c] & VT_CELL_FAILED) continue;
        const int32_t cnt = A.ccnt[c];
        if (cnt > VT_CLAIM_NBR) continue;   // left to the search
        const int32_t j0 = A.cells[c];
        const int32_t gi = A.sgid[j0];
        double x[3];
        gpos<PT4>(A.spos, j0, x[0], x[1], x[2]);
        const double R = A.crad[c] * (1.0 + 1e-9) + 1e-12 * it.S;
        const double R2 = R * R;
        if (!(R2 < 1e300)) continue;   // not a finite radius: the points go to the search
        int64_t f0[3], nf[3];
        bool ok = true;
        for (int a = 0; a < 3; ++a) {
            const double hf = it.L[a] / (double)F[a];
            f0[a] = (int64_t)floor((x[a] - R - it.lo[a]) / hf - 0.5) - 1;
            nf[a] = (int64_t)floor((x[a] + R - it.lo[a]) / hf - 0.5) + 2 - f0[a];
            if (nf[a] > F[a]) {   // the cell spans the period along a: every point once
                f0[a] = 0;
                nf[a] = F[a];
            }
            ok = ok && nf[a] >= 1;
        }
        const int64_t ncand = nf[0] * nf[1] * nf[2];
        if (!ok || ncand > VT_CLAIM_MAX) continue;
        // one correction brings every candidate index into [0, F)
        for (int a = 0; a < 3; ++a) ok = ok && F[a] < (1 << 29) && f0[a] >= -F[a] && f0[a] + nf[a] <= 2 * F[a];
        if (!ok) continue;
        const int64_t row = A.crow[c];
        if (cnt <= 64) {
            // nearest neighbours first: a point outside the cell fails on one of them early
            double px = 0.0, py = 0.0, pz = 0.0;
            int32_t pg = 0;
            uint64_t key[1] = {~0ull};
            if (lane < cnt) {
                const int32_t j = A.stage_ids[row + lane];
                gpos<PT4>(A.spos, j, px, py, pz);
                pg = A.sgid[j];
                double ex = px - x[0], ey = py - x[1], ez = pz - x[2];
                ex -= it.L[0] * rint(ex * invL[0]);
                ey -= it.L[1] * rint(ey * invL[1]);
                ez -= it.L[2] * rint(ez * invL[2]);
                key[0] = ((uint64_t)__float_as_uint((float)(ex * ex + ey * ey + ez * ez)) << 32) | (uint64_t)lane;
            }
            bitonic_u64<1>(key);
            const int src = (int)(key[0] & 63ull);
            const double sx_ = __shfl(px, src), sy_ = __shfl(py, src), sz_ = __shfl(pz, src);
            const int32_t sg_ = __shfl(pg, src);
            if (lane < cnt) {
                M.px[lane] = sx_;
                M.py[lane] = sy_;
                M.pz[lane] = sz_;
                M.pg[lane] = sg_;
            }
        } else {
            for (int k = lane; k < cnt; k += 64) {
                const int32_t j = A.stage_ids[row + k];
                gpos<PT4>(A.spos, j, M.px[k], M.py[k], M.pz[k]);
                M.pg[k] = A.sgid[j];
            }
        }
        wave_sync();
        const unsigned long long mine = ((unsigned long long)(uint32_t)gi << 32) | (uint32_t)j0;
        for (int64_t base = 0; base < ncand; base += 64) {
            const int64_t m = base + lane;
            if (m < ncand) {
                // 32-bit index arithmetic: the candidate's offsets, then one period's correction
                // (a periodic cell is less than a quarter period across)
                int t, v;
                const int r = divmod_small((int)m, (int)nf[2], t);
                const int u = divmod_small(r, (int)nf[1], v);
                const int w0 = wrap_once((int)f0[0] + u, (int)F[0]);
                const int w1 = wrap_once((int)f0[1] + v, (int)F[1]);
                const int w2 = wrap_once((int)f0[2] + t, (int)F[2]);
                const double q0 = sample_coord32(it, 0, dims[0], sub, w0);
                const double q1 = sample_coord32(it, 1, dims[1], sub, w1);
                const double q2 = sample_coord32(it, 2, dims[2], sub, w2);
                double e0 = x[0] - q0, e1 = x[1] - q1, e2 = x[2] - q2;
                e0 -= it.L[0] * rint(e0 * invL[0]);
                e1 -= it.L[1] * rint(e1 * invL[1]);
                e2 -= it.L[2] * rint(e2 * invL[2]);
                const double d2 = e0 * e0 + e1 * e1 + e2 * e2;
                if (d2 <= R2) {
                    bool win = true;
                    for (int32_t k = 0; k < cnt && win; ++k) {
                        double ex = M.px[k] - q0, ey = M.py[k] - q1, ez = M.pz[k] - q2;
                        ex -= it.L[0] * rint(ex * invL[0]);
                        ey -= it.L[1] * rint(ey * invL[1]);
                        ez -= it.L[2] * rint(ez * invL[2]);
                        const double dj = ex * ex + ey * ey + ez * ez;
                        win = !(dj < d2 || (dj == d2 && M.pg[k] < gi));
                    }
                    if (win) atomicMin(&A.slot[((int64_t)w0 * F[1] + w1) * F[2] + w2], mine);
                }
            }
        }
        wave_sync();
    }
}

template <typename PT4>
__global__ void __launch_bounds__(256) k_sample_tiles(SampleArgs A) {
    extern __shared__ char smem[];
    SampleMem &S = *reinterpret_cast<SampleMem *>(smem + (size_t)(threadIdx.x >> 6) * sizeof(SampleMem));
    const int lane = threadIdx.x & 63;
    const uint64_t lt = (1ull << lane) - 1ull;
    const DevItem it = uniform_item(A.items[0]);
    const int sub = A.sub;
    const int64_t fd[3] = {(int64_t)A.nx * sub, (int64_t)A.ny * sub, (int64_t)A.nz * sub};
    const int64_t ntile[3] = {(fd[0] + 3) / 4, (fd[1] + 3) / 4, (fd[2] + 3) / 4};
    const int64_t n_tiles = ntile[0] * ntile[1] * ntile[2];
    const int dims[3] = {A.nx, A.ny, A.nz};
    const double quantum = it.S / (double)(1 << VT_MORTON_BITS);
    const double invL[3] = {1.0 / it.L[0], 1.0 / it.L[1], 1.0 / it.L[2]};
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t t = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); t < n_tiles; t += nwaves) {
        const int64_t tz = t % ntile[2], ty = (t / ntile[2]) % ntile[1], tx = t / (ntile[1] * ntile[2]);
        const int64_t f[3] = {tx * 4 + (lane >> 4), ty * 4 + ((lane >> 2) & 3), tz * 4 + (lane & 3)};
        const bool valid = f[0] < fd[0] && f[1] < fd[1] && f[2] < fd[2];
        // the sample point: voxel i, sub-cell s (the reference's expression)
        double q[3], tlo[3], thi[3];
        for (int a = 0; a < 3; ++a) {
            const double h = it.L[a] / dims[a];
            const int64_t fa = valid ? f[a] : 0;
            q[a] = it.lo[a] + ((double)(fa / sub) + ((double)(fa % sub) + 0.5) / (double)sub) * h;
            // the tile's extent: its first and last points along a
            const int64_t f0 = (a == 0 ? tx : a == 1 ? ty : tz) * 4;
            const int64_t f1 = min(f0 + 3, fd[a] - 1);
            tlo[a] = it.lo[a] + ((double)(f0 / sub) + ((double)(f0 % sub) + 0.5) / (double)sub) * h;
            thi[a] = it.lo[a] + ((double)(f1 / sub) + ((double)(f1 % sub) + 0.5) / (double)sub) * h;
        }
        double best = 1e300;
        int32_t bg = 0x7FFFFFFF, bj = -1;
        for (double r = A.r0;; r *= 2.0) {
            // covering Morton cells: side c >= r (coarser while more than 512 would be needed)
            int l = 0;
            double c = it.S;
            while (l < VT_MORTON_BITS && 0.5 * c >= r) {
                c *= 0.5;
                ++l;
            }
            int64_t a0[3], na[3];
            bool whole[3];
            for (;;) {
                const int64_t ncl = 1ll << l;
                for (int a = 0; a < 3; ++a) {
                    int64_t i0 = (int64_t)floor((tlo[a] - r - it.lo[a]) / c);
                    int64_t i1 = (int64_t)floor((thi[a] + r - it.lo[a]) / c);
                    whole[a] = i1 - i0 + 1 >= ncl;
                    if (whole[a]) {
                        i0 = 0;
                        i1 = ncl - 1;
                    }
                    a0[a] = i0;
                    na[a] = i1 - i0 + 1;
                }
                if (na[0] * na[1] * na[2] <= 512 || l == 0) break;
                --l;
                c *= 2.0;
            }
            // the lane's reach: its distance to the nearest side of the covered cells (axes not
            // covered whole), less two key quanta for the rounding of particle keys
            double reach = 1e300;
            for (int a = 0; a < 3; ++a)
                if (!whole[a]) {
                    const double b0 = it.lo[a] + (double)a0[a] * c, b1 = it.lo[a] + (double)(a0[a] + na[a]) * c;
                    reach = fmin(reach, fmin(q[a] - b0, b1 - q[a]));
                }
            reach -= 2.0 * quantum;
            const int64_t ncl = 1ll << l;
            const int ncells = (int)(na[0] * na[1] * na[2]);
            int count = 0;
            for (int base = 0; base < ncells; base += 64) {
                const int k = base + lane;
                int32_t cb = 0, ce = 0;
                if (k < ncells) {
                    const int64_t u[3] = {a0[0] + k % na[0], a0[1] + (k / na[0]) % na[1], a0[2] + k / (na[0] * na[1])};
                    const uint64_t cx = (uint64_t)((u[0] % ncl + ncl) % ncl), cy = (uint64_t)((u[1] % ncl + ncl) % ncl),
                                   cz = (uint64_t)((u[2] % ncl + ncl) % ncl);
                    morton_range(A, it, l, vt_morton(cx, cy, cz), cb, ce);
                }
                const bool keep = ce > cb;
                const uint64_t km = __ballot(keep);
                if (keep) {
                    const int slot = count + __popcll(km & lt);
                    S.rb[slot] = cb;
                    S.rp[slot] = ce - cb;
                }
                count += __popcll(km);
            }
            wave_sync();
            int carry = 0;
            for (int base = 0; base < count; base += 64) {
                const int k = base + lane;
                const int len = k < count ? S.rp[k] : 0;
                int tot;
                const int pre = wave_excl_scan(len, &tot);
                if (k < count) S.rp[k] = carry + pre;
                carry += tot;
            }
            if (lane == 0) S.rp[count] = carry;
            wave_sync();
            const int total = carry;
            if (total > VT_SAMPLE_DENSE) {
                // a dense region: every lane searches on its own, through finer cells
                if (valid) bj = nearest_particle<PT4>(A, it, q, invL, bg);
                break;
            }
            for (int c0 = 0; c0 < total; c0 += 64) {
                const int fi = c0 + lane;
                if (fi < total) {
                    int lo = 0, hi = count - 1;
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (S.rp[mid] <= fi) lo = mid; else hi = mid - 1;
                    }
                    const int32_t j = S.rb[lo] + (fi - S.rp[lo]);
                    double px, py, pz;
                    gpos<PT4>(A.spos, j, px, py, pz);
                    S.px[lane] = px;
                    S.py[lane] = py;
                    S.pz[lane] = pz;
                    S.pg[lane] = A.sgid[j];
                    S.pj[lane] = j;
                }
                wave_sync();
                const int nc = min(64, total - c0);
                for (int k = 0; k < nc; ++k) {
                    double ex = S.px[k] - q[0], ey = S.py[k] - q[1], ez = S.pz[k] - q[2];
                    ex -= it.L[0] * rint(ex * invL[0]);
                    ey -= it.L[1] * rint(ey * invL[1]);
                    ez -= it.L[2] * rint(ez * invL[2]);
                    const double d2 = ex * ex + ey * ey + ez * ez;
                    const int32_t gj = S.pg[k];
                    if (d2 < best || (d2 == best && gj < bg)) {
                        best = d2;
                        bg = gj;
                        bj = S.pj[k];
                    }
                }
                wave_sync();
            }
            const bool done = (whole[0] && whole[1] && whole[2]) || (bj >= 0 && reach > 0.0 && best < reach * reach);
            if (__ballot(valid && !done) == 0ull) break;
        }
        if (valid) A.slot[(f[0] * fd[1] + f[1]) * fd[2] + f[2]] = ((unsigned long long)(uint32_t)bg << 32) | (uint32_t)bj;
    }
}

// Points no cell claimed get their own exact search; with one point per voxel the voxel's
// value is written here too.
template <typename PT4>
__global__ void k_sample_fixup(SampleArgs A) {
    const int sub = A.sub;
    const int64_t F[3] = {(int64_t)A.nx * sub, (int64_t)A.ny * sub, (int64_t)A.nz * sub};
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= F[0] * F[1] * F[2]) return;
    unsigned long long s = A.slot[p];
    if (s == ~0ull) {
        const DevItem it = uniform_item(A.items[0]);
        const int dims[3] = {A.nx, A.ny, A.nz};
        const int64_t f[3] = {p / (F[1] * F[2]), (p / F[2]) % F[1], p % F[2]};
        double q[3];
        for (int a = 0; a < 3; ++a) q[a] = sample_coord(it, a, dims[a], sub, f[a]);
        const double invL[3] = {1.0 / it.L[0], 1.0 / it.L[1], 1.0 / it.L[2]};
        int32_t bg;
        const int32_t bj = nearest_particle<PT4>(A, it, q, invL, bg);
        s = ((unsigned long long)(uint32_t)bg << 32) | (uint32_t)bj;
        A.slot[p] = s;
    }
    if (sub == 1) {
        const int32_t bj = (int32_t)(s & 0xFFFFFFFFull);
        A.grid[p] = A.value[A.srow[bj]];
        if (A.nearest) A.nearest[p] = (int32_t)(s >> 32);
    }
}

__global__ void k_fill_u64(unsigned long long *p, int64_t n, unsigned long long v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// sub > 1: each voxel averages its sub^3 points in the reference's order
__global__ void k_sample_average(SampleArgs A) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nv = (int64_t)A.nx * A.ny * A.nz;
    if (v >= nv) return;
    const int sub = A.sub;
    const int64_t iz = v % A.nz, iy = (v / A.nz) % A.ny, ix = v / ((int64_t)A.ny * A.nz);
    const int64_t fy = (int64_t)A.ny * sub, fz = (int64_t)A.nz * sub;
    double acc = 0.0;
    unsigned long long last = 0;
    for (int s0 = 0; s0 < sub; ++s0)
        for (int s1 = 0; s1 < sub; ++s1)
            for (int s2 = 0; s2 < sub; ++s2) {
                last = A.slot[((ix * sub + s0) * fy + (iy * sub + s1)) * fz + (iz * sub + s2)];
                acc += A.value[A.srow[(int32_t)(last & 0xFFFFFFFFull)]];
            }
    A.grid[v] = acc / (double)(sub * sub * sub);
    if (A.nearest) A.nearest[v] = (int32_t)(last >> 32);
}

hipError_t vt_launch_grid_sample(vt_ctx *c, const double *value, int nx, int ny, int nz, int sub, double *grid,
                                 int32_t *nearest) {
    SampleArgs a;
    a.spos = c->spos;
    a.skey = c->skey;
    a.tab = c->tab;
    a.sgid = c->sgid;
    a.srow = c->srow;
    a.items = c->items;
    a.cells = c->cells;
    a.cstat = c->cstat;
    a.crad = c->crad;
    a.crow = c->crow;
    a.ccnt = c->ccnt;
    a.stage_ids = c->stage_ids;
    a.ncells = c->n_owned;
    a.value = value;
    a.grid = grid;
    a.nearest = nearest;
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    a.sub = sub;
    // one 64-bit slot per sample point, kept by the context (samp_fine counts int32 words)
    const int64_t nfine = (int64_t)nx * ny * nz * sub * sub * sub;
    if (2 * nfine > c->cap_samp) {
        if (c->samp_fine) (void)hipFree(c->samp_fine);
        c->samp_fine = nullptr;
        c->cap_samp = 0;
        hipError_t e = hipMalloc((void **)&c->samp_fine, sizeof(unsigned long long) * (size_t)nfine);
        if (e != hipSuccess) return e;
        c->cap_samp = 2 * nfine;
    }
    a.slot = (unsigned long long *)c->samp_fine;
    const DevItem &it0 = c->h_items[0];
    a.r0 = cbrt(it0.L[0] * it0.L[1] * it0.L[2] / (double)c->n_total);
    const int tpb = 256;
    int ncu = 0;
    if (sub > 1) {
        // several points per voxel: tiles of points sharing one candidate list
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device);
        if (ncu <= 0) ncu = 256;
        const size_t lds = sizeof(SampleMem) * 4;
        const int64_t tiles = ((int64_t)nx * sub + 3) / 4 * (((int64_t)ny * sub + 3) / 4) * (((int64_t)nz * sub + 3) / 4);
        int64_t blocks = (tiles + 3) / 4;
        if (blocks > (int64_t)ncu * 64) blocks = (int64_t)ncu * 64;
        if (c->dtype == VT_F32)
            k_sample_tiles<float4><<<(unsigned)blocks, 256, lds, c->stream>>>(a);
        else
            k_sample_tiles<double4><<<(unsigned)blocks, 256, lds, c->stream>>>(a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const int64_t nv = (int64_t)nx * ny * nz;
        k_sample_average<<<(nv + tpb - 1) / tpb, tpb, 0, c->stream>>>(a);
        return hipGetLastError();
    }
    // one point per voxel: the cells claim their points
    k_fill_u64<<<(nfine + tpb - 1) / tpb, tpb, 0, c->stream>>>(a.slot, nfine, ~0ull);
    hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device);
    if (ncu <= 0) ncu = 256;
    int64_t cblocks = (a.ncells + 3) / 4;
    if (cblocks > (int64_t)ncu * 32) cblocks = (int64_t)ncu * 32;
    if (cblocks < 1) cblocks = 1;
    if (c->dtype == VT_F32) {
        k_sample_claim<float4><<<(unsigned)cblocks, tpb, 0, c->stream>>>(a);
        k_sample_fixup<float4><<<(nfine + tpb - 1) / tpb, tpb, 0, c->stream>>>(a);
    } else {
        k_sample_claim<double4><<<(unsigned)cblocks, tpb, 0, c->stream>>>(a);
        k_sample_fixup<double4><<<(nfine + tpb - 1) / tpb, tpb, 0, c->stream>>>(a);
    }
    return hipGetLastError();
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
    int64_t blocks = RETRY ? (int64_t)ncu : (int64_t)ncu * 16 / wpb;
    kern<<<dim3((unsigned)blocks), dim3(64 * wpb), lds, c->stream>>>(a);
    return hipGetLastError();
}

template <typename PT4>
static hipError_t launch_grid_fused(vt_ctx *c, GridArgs &a) {
    const size_t l1 = sizeof(GridMem<1>) * 4, l4 = sizeof(GridMem<4>);
    const size_t lds = l1 > l4 ? l1 : l4;
    auto kern = k_grid_fused<PT4>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    int ncu = 0;
    hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device);
    if (ncu <= 0) ncu = 256;
    a.n_large = ncu;
    a.seg = 1;
    const int64_t blocks = (int64_t)ncu + (int64_t)ncu * 16 / 4;
    kern<<<dim3((unsigned)blocks), dim3(256), lds, c->stream>>>(a);
    return hipGetLastError();
}

// The normal kernel with the large one over the clip's retry queue in one launch, then the large
// kernel over the cells the normal one handed over.
template <typename PT4>
static hipError_t launch_grid_all(vt_ctx *c, GridArgs &a) {
    hipError_t e = launch_grid_fused<PT4>(c, a);
    if (e == hipSuccess) e = vt_launch_zero_u32(c->counters + CTR_GRID, 1, c->stream);
    if (e != hipSuccess) return e;
    a.seg = 2;
    a.n_large = 0;
    return launch_grid_one<PT4, 4, true>(c, a, 1);
}

hipError_t vt_launch_grid(vt_ctx *c, const double *value, int nx, int ny, int nz, double *grid) {
    const int64_t ng = (int64_t)nx * ny * nz;
    k_zero_f64<<<(ng + 255) / 256, 256, 0, c->stream>>>(grid, ng);
    hipError_t ez = vt_launch_zero_u32(c->counters + CTR_GRID, CTR_GRID_Q - CTR_GRID + 1, c->stream);
    if (ez != hipSuccess) return ez;
    GridArgs a;
    a.spos = c->spos;
    a.items = c->items;
    a.cells = c->cells;
    a.ncells = c->n_owned;
    a.queue = c->queue;
    a.queue_cap = c->cap_retry;
    a.gqueue = c->gqueue;
    a.gqueue_cap = c->cap_retry;
    a.crow = c->crow;
    a.ccnt = c->ccnt;
    a.cstat = c->cstat;
    a.cvol = c->cvol;
    a.crad = c->crad;
    a.ctopo = c->ctopo;
    a.cnf = c->cnf;
    a.cnv = c->cnv;
    a.npos = c->n_total;
    a.stage_ids = c->stage_ids;
    a.srow = c->srow;
    a.value = value;
    a.counters = c->counters;
    a.grid = grid;
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    a.seg = 0;
    a.n_large = 0;
    return c->dtype == VT_F32 ? launch_grid_all<float4>(c, a) : launch_grid_all<double4>(c, a);
}

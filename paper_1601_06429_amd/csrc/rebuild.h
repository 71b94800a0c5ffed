// rebuild.h -- a computed cell rebuilt as a wave-resident polytope, for the kernels that need
// its full geometry after the build (grid deposit, structure output).
//
// The fast clip kernel leaves a topology record per cell: the tag of every face (a sorted
// particle index, or -1 .. -6 for the walls -x, +x, -y, +y, -z, +z of the seed-relative box)
// and, per vertex, the ranks of its three faces.  Every face plane follows from its tag and
// every vertex is the intersection of its three planes, computed in the same order as the clip
// kernel computes it, so the rebuilt vertices are the clip kernel's own.  A cell without a
// record (cells of the large clip kernel, cells of more than VT_TOPO_FACES faces) is clipped
// again from its facet list.  A record that exists but fails a check (a tag or rank out of
// range, repeated ranks, a vertex that is not finite) can only come from a fault in the clip
// kernel: it is counted (CTR_REC_REJECT), the device status takes VT_DEV_TOPOLOGY so that
// vt_query reports it, and the cell is still rebuilt from its facets.
#pragma once
#include "poly.h"

// a double held by lane l (l the same in every lane)
__device__ __forceinline__ double readlane_d(double x, int l) {
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    const uint64_t lo = readlane_u32((uint32_t)u, l), hi = readlane_u32((uint32_t)(u >> 32), l);
    return __longlong_as_double((long long)((hi << 32) | lo));
}

template <typename PT4>
__device__ __forceinline__ void gpos(const void *spos, int32_t j, double &x, double &y, double &z) {
    PT4 p = ((const PT4 *)spos)[j];
    x = (double)p.x;
    y = (double)p.y;
    z = (double)p.z;
}

// where a cell's geometry is kept after the build
struct CellSrc {
    const void *spos;          // sorted positions
    const int32_t *ctopo;      // topology records (VT_TOPO_STRIDE words per cell)
    const int32_t *cnf;        // faces in the record (0: no record)
    const int32_t *cnv;        // vertices of the cell
    int64_t npos;              // sorted particles (bound of a record's face tags)
    const int64_t *crow;       // facet list of the cell: stage_ids[crow .. crow + ccnt)
    const int32_t *ccnt;
    const int32_t *stage_ids;
    uint32_t *counters;
};

enum { REBUILD_OK = 0, REBUILD_OVERFLOW = 1, REBUILD_FAILED = 2 };

// Rebuild cell c (seed at (sx, sy, sz), box [blo, bhi] relative to the seed) into P and SP.
// Face slots carry their tags in SP.ptag.  The normal kernel (VPL = 1, RETRY false) takes the
// record when there is one and otherwise applies the facets nearest first; the large kernel
// applies them in stored order.  Returns REBUILD_OVERFLOW when the normal kernel runs out of
// vertex slots (the cell belongs to the large kernel) and REBUILD_FAILED when a clip fails.
template <typename PT4, int VPL, bool RETRY>
__device__ __forceinline__ int rebuild_cell(const CellSrc &R, const DevItem &it, PolyMem<double, VPL> &SP,
                                            Poly<double, VPL> &P, int32_t c, double sx, double sy, double sz,
                                            const double blo[3], const double bhi[3]) {
    const int lane = lane_id();
    const uint64_t mybit = 1ull << lane;
    bool bad = false, over = false, have = false;
    if constexpr (!RETRY && VPL == 1) {
        const int nf = R.cnf[c], nv = R.cnv[c];
        bool rejected = nf != 0;  // a record exists; cleared once it passes every check
        if (nf >= 4 && nf <= VT_TOPO_FACES && nv >= 4 && nv <= 64) {
            const int64_t tb = (int64_t)c * VT_TOPO_STRIDE;
            bool ok = true;
            if (lane < nf) {
                const int32_t tag = R.ctopo[tb + lane];
                P4<double> p;
                if (tag >= 0 && (int64_t)tag < R.npos) {
                    double qx, qy, qz;
                    gpos<PT4>(R.spos, tag, qx, qy, qz);
                    qx -= sx;
                    qy -= sy;
                    qz -= sz;
                    if (it.periodic) {
                        qx -= it.L[0] * rint(qx * (1.0 / it.L[0]));
                        qy -= it.L[1] * rint(qy * (1.0 / it.L[1]));
                        qz -= it.L[2] * rint(qz * (1.0 / it.L[2]));
                    }
                    p.x = qx;
                    p.y = qy;
                    p.z = qz;
                    p.d = 0.5 * (qx * qx + qy * qy + qz * qz);
                } else if (tag < 0 && tag >= -6) {
                    const int b = -1 - tag, a = b >> 1;
                    const bool pos = b & 1;
                    p.x = (a == 0) ? (pos ? 1.0 : -1.0) : 0.0;
                    p.y = (a == 1) ? (pos ? 1.0 : -1.0) : 0.0;
                    p.z = (a == 2) ? (pos ? 1.0 : -1.0) : 0.0;
                    p.d = pos ? bhi[a] : -blo[a];
                } else {
                    ok = false;
                    p.x = p.y = p.z = p.d = 0.0;
                }
                SP.pl64[lane] = p;
                SP.ptag[lane] = tag;
                SP.fm[lane][0] = 0ull;
            }
            uint32_t t = 0, k0 = 0, k1 = 0, k2 = 0;
            if (lane < nv) {
                t = (uint32_t)R.ctopo[tb + VT_TOPO_FACES + lane];
                k0 = t & 0xFFu;
                k1 = (t >> 8) & 0xFFu;
                k2 = (t >> 16) & 0xFFu;
                if ((t >> 24) || k0 >= (uint32_t)nf || k1 >= (uint32_t)nf || k2 >= (uint32_t)nf || k0 == k1 ||
                    k1 == k2 || k0 == k2)
                    ok = false;
            }
            if (__ballot(!ok) == 0ull) {
                wave_sync();
                double x = 0.0, y = 0.0, z = 0.0;
                if (lane < nv) {
                    intersect3<double>(SP.pl64[k0], SP.pl64[k1], SP.pl64[k2], x, y, z);
                    atomicOr((unsigned long long *)&SP.fm[k0][0], (unsigned long long)mybit);
                    atomicOr((unsigned long long *)&SP.fm[k1][0], (unsigned long long)mybit);
                    atomicOr((unsigned long long *)&SP.fm[k2][0], (unsigned long long)mybit);
                }
                const bool fin = isfinite(x) && isfinite(y) && isfinite(z);
                if (__ballot(!fin) == 0ull) {
                    P.vx[0] = x;
                    P.vy[0] = y;
                    P.vz[0] = z;
                    P.vt[0] = t;
                    P.alive[0] = nv == 64 ? ~0ull : ((1ull << nv) - 1ull);
                    P.fa[0] = (1ull << nf) - 1ull;
                    have = true;
                    rejected = false;
                }
                wave_sync();
            }
        }
        if (rejected && lane == 0) {
            atomicAdd(&R.counters[CTR_REC_REJECT], 1u);
            atomicOr(&R.counters[CTR_STATUS], VT_DEV_TOPOLOGY);
        }
    }
    // otherwise from the facets: loaded lane-parallel; the normal kernel applies them nearest
    // first (the cell then stays close to its final size, so 64 vertices suffice), the large
    // kernel in stored order
    if (!have) P.init_box(SP, blo, bhi);
    const int64_t row = R.crow[c];
    const int32_t cnt = have ? 0 : R.ccnt[c];
    for (int32_t t0 = 0; t0 < cnt && !bad && !over; t0 += 64) {
        const int32_t t = t0 + lane;
        double qx = 0.0, qy = 0.0, qz = 0.0;
        int32_t qj = -1;
        uint64_t key = ~0ull;
        if (t < cnt) {
            qj = R.stage_ids[row + t];
            gpos<PT4>(R.spos, qj, qx, qy, qz);
            qx -= sx;
            qy -= sy;
            qz -= sz;
            if (it.periodic) {
                qx -= it.L[0] * rint(qx / it.L[0]);
                qy -= it.L[1] * rint(qy / it.L[1]);
                qz -= it.L[2] * rint(qz / it.L[2]);
            }
            const float d2f = (float)(qx * qx + qy * qy + qz * qz);
            key = RETRY ? (uint64_t)lane : (((uint64_t)__float_as_uint(d2f) << 32) | (uint64_t)lane);
        }
        if (!RETRY) {
            uint64_t kk[1] = {key};
            bitonic_u64<1>(kk);
            key = kk[0];
        }
        const int nin = min(64, cnt - t0);
        for (int i = 0; i < nin; ++i) {
            const int src = (int)(readlane_u32((uint32_t)(key & 0xFFFFFFFFull), i) & 63u);
            P4<double> p;
            p.x = __shfl(qx, src);
            p.y = __shfl(qy, src);
            p.z = __shfl(qz, src);
            p.d = 0.5 * (p.x * p.x + p.y * p.y + p.z * p.z);
            const int32_t j = __shfl(qj, src);
            const int rc = P.clip(SP, p, j);
            if (rc == CLIP_OVERFLOW && !RETRY) {
                over = true;
                break;
            }
            if (rc < 0) {
                if (lane == 0) atomicOr(&R.counters[CTR_DEBUG], 1u << (-rc));
                bad = true;
                break;
            }
        }
    }
    return over ? REBUILD_OVERFLOW : bad ? REBUILD_FAILED : REBUILD_OK;
}

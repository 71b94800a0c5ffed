// poly.h -- a convex cell held by one wavefront, and the bisector clip.
//
// The cell (a convex polytope around the seed, seed at the origin) is held in
// its dual form.  Each vertex is the triple (a, b, c) of the planes meeting
// there, counter-clockwise seen from outside; lanes own vertices (VPL per
// lane) with positions in registers.  For every plane slot f the LDS keeps a
// bit mask of the vertices on it, so the vertex across the edge (a, b) of
// vertex v is the single other bit of mask[a] & mask[b].  Clipping by plane p:
//   1. the lanes evaluate the side value of their vertices; a ballot gives the
//      clipped set M;
//   2. each clipped vertex looks at its three edges; an edge whose twin vertex
//      is kept is cut and yields the new vertex (a, b, p), the intersection of
//      the three planes, with the orientation of the clipped vertex;
//   3. new vertices go to free lanes (ranked by popcounts), the masks are
//      updated, and faces left without vertices release their plane slot.
// A vertex position is always the intersection of its own three planes, so any
// predicate can be re-evaluated in FP64 from the plane triple alone.
//
// T = double: FP64 arithmetic.  T = float: FP32 arithmetic; a side value within
// its error bound of zero is decided in FP64 from the FP64 planes, which is the
// FP64 path's own computation, so both paths take the same decisions.
#pragma once

#include <type_traits>

#include "vt_internal.h"

// ------------------------------------------------------------------ wave helpers
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// orders LDS accesses of the lanes of one wavefront
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t readlane_u32(uint32_t x, int l) {
    return (uint32_t)__builtin_amdgcn_readlane((int)x, l);
}

// values that are equal in every lane, moved to scalar registers
__device__ __forceinline__ int uni_i(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ double uni_d(double x) {
    long long b = __double_as_longlong(x);
    int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffff));
    int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)(unsigned)hi << 32) | (unsigned)lo);
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
    for (int o = 32; o > 0; o >>= 1) {
        T u = __shfl_xor(v, o);
        v = u > v ? u : v;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_min(T v) {
    for (int o = 32; o > 0; o >>= 1) {
        T u = __shfl_xor(v, o);
        v = u < v ? u : v;
    }
    return v;
}

__device__ __forceinline__ double wave_sum_d(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ int wave_sum_i(int v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Reductions whose cross-lane steps stay in the VALU: DPP moves within rows of 16 lanes (swap
// neighbours, swap pairs, mirror within 8, mirror within 16), then the gfx950 row swaps, which
// leave every lane holding its own value and its partner's 16 and 32 lanes away (in one order or
// the other: the operation is commutative, so either serves).  The result is in every lane.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    const uint64_t lo = dpp_u32<CTRL>((uint32_t)u), hi = dpp_u32<CTRL>((uint32_t)(u >> 32));
    return __longlong_as_double((long long)((hi << 32) | lo));
}
template <bool ROW32>
__device__ __forceinline__ void row_swap_d(double x, double &a, double &b) {
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = (uint32_t)u, hi = (uint32_t)(u >> 32);
    uint32_t alo, blo, ahi, bhi;
    if constexpr (ROW32) {
        auto rl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        auto rh = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        alo = rl[0], blo = rl[1], ahi = rh[0], bhi = rh[1];
    } else {
        auto rl = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        auto rh = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        alo = rl[0], blo = rl[1], ahi = rh[0], bhi = rh[1];
    }
    a = __longlong_as_double((long long)(((uint64_t)ahi << 32) | alo));
    b = __longlong_as_double((long long)(((uint64_t)bhi << 32) | blo));
}
enum { DPP_XOR1 = 0xB1, DPP_XOR2 = 0x4E, DPP_HALF_MIRROR = 0x141, DPP_MIRROR = 0x140 };
template <bool MAX>
__device__ __forceinline__ double wave_ext_d(double v) {
    auto op = [](double a, double b) { return MAX ? fmax(a, b) : fmin(a, b); };
    v = op(v, dpp_d<DPP_XOR1>(v));
    v = op(v, dpp_d<DPP_XOR2>(v));
    v = op(v, dpp_d<DPP_HALF_MIRROR>(v));
    v = op(v, dpp_d<DPP_MIRROR>(v));
    double a, b;
    row_swap_d<false>(v, a, b);
    v = op(a, b);
    row_swap_d<true>(v, a, b);
    return op(a, b);
}
__device__ __forceinline__ double wave_max_x(double v) { return wave_ext_d<true>(v); }
__device__ __forceinline__ double wave_min_x(double v) { return wave_ext_d<false>(v); }
// bitwise OR over the wave by the same steps (moves only; the result in every lane)
__device__ __forceinline__ uint64_t wave_or_u64(uint64_t v) {
    auto D = [](uint64_t x) { return __longlong_as_double((long long)x); };
    auto U = [](double x) { return (uint64_t)__double_as_longlong(x); };
    v |= U(dpp_d<DPP_XOR1>(D(v)));
    v |= U(dpp_d<DPP_XOR2>(D(v)));
    v |= U(dpp_d<DPP_HALF_MIRROR>(D(v)));
    v |= U(dpp_d<DPP_MIRROR>(D(v)));
    double a, b;
    row_swap_d<false>(D(v), a, b);
    v = U(a) | U(b);
    row_swap_d<true>(D(v), a, b);
    return U(a) | U(b);
}

// The value of lane l ^ J, without LDS: DPP for J < 16 (neighbour and pair swaps within quads;
// for 4 and 8, shifts within the row whose bank mask picks the lanes that read upwards or
// downwards), the gfx950 row swaps for 16 and 32 (each lane then holds its own value and its
// partner's: the one that differs from its own, or either when they are equal).
template <int J>
__device__ __forceinline__ uint32_t xor_lane_u32(uint32_t x) {
    if constexpr (J == 1) {
        return dpp_u32<DPP_XOR1>(x);
    } else if constexpr (J == 2) {
        return dpp_u32<DPP_XOR2>(x);
    } else if constexpr (J == 4 || J == 8) {
        constexpr int SHL = 0x100 + J, SHR = 0x110 + J;
        constexpr int LOW = J == 4 ? 0x5 : 0x3;  // banks (4 lanes each) whose lanes have bit J clear
        const int up = __builtin_amdgcn_update_dpp((int)x, (int)x, SHL, 0xF, LOW, false);
        return (uint32_t)__builtin_amdgcn_update_dpp(up, (int)x, SHR, 0xF, 0xF ^ LOW, false);
    } else {
        static_assert(J == 16 || J == 32, "lane distance");
        uint32_t a, b;
        if constexpr (J == 16) {
            auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
            a = r[0];
            b = r[1];
        } else {
            auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
            a = r[0];
            b = r[1];
        }
        return a != x ? a : b;
    }
}

// one compare-exchange stage of a bitonic network at lane distance J (size: the merge size)
template <int J>
__device__ __forceinline__ uint32_t bitonic_step(uint32_t k, int e, int size, bool last) {
    const uint32_t o = xor_lane_u32<J>(k);
    const bool up = (e & size) == 0 || last;
    const bool lower = (e & J) == 0;
    const uint32_t mn = k < o ? k : o, mx = k < o ? o : k;
    return (lower == up) ? mn : mx;
}
template <int J>
__device__ __forceinline__ void bitonic_merge(uint32_t &k, int e, int size, bool last) {
    k = bitonic_step<J>(k, e, size, last);
    if constexpr (J > 1) bitonic_merge<J / 2>(k, e, size, last);
}

// bitonic64 / bitonic128 with the cross-lane steps above (same networks, same results)
__device__ __forceinline__ uint32_t bitonic64_x(uint32_t k) {
    const int l = lane_id();
    bitonic_merge<1>(k, l, 2, false);
    bitonic_merge<2>(k, l, 4, false);
    bitonic_merge<4>(k, l, 8, false);
    bitonic_merge<8>(k, l, 16, false);
    bitonic_merge<16>(k, l, 32, false);
    bitonic_merge<32>(k, l, 64, true);
    return k;
}
__device__ __forceinline__ void bitonic128_x(uint32_t &k0, uint32_t &k1) {
    const int l = lane_id();
#define VT_BM2(J, SIZE)                          \
    bitonic_merge<J>(k0, l, SIZE, false);        \
    bitonic_merge<J>(k1, 64 + l, SIZE, false);
    VT_BM2(1, 2)
    VT_BM2(2, 4)
    VT_BM2(4, 8)
    VT_BM2(8, 16)
    VT_BM2(16, 32)
    VT_BM2(32, 64)
#undef VT_BM2
    // size 128: the exchange at distance 64 is between the two registers, then distances 32 .. 1
    const uint32_t mn = k0 < k1 ? k0 : k1, mx = k0 < k1 ? k1 : k0;
    k0 = mn;
    k1 = mx;
    bitonic_merge<32>(k0, l, 128, false);
    bitonic_merge<32>(k1, 64 + l, 128, false);
}

// a double held by lane l (l the same in every lane)
__device__ __forceinline__ double readlane_dbl(double x, int l) {
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    const uint64_t lo = readlane_u32((uint32_t)u, l), hi = readlane_u32((uint32_t)(u >> 32), l);
    return __longlong_as_double((long long)((hi << 32) | lo));
}

// An item's fields, read once into scalar registers (the item must be the same for the whole
// wavefront): through a reference the compiler reloads them from memory at every use, since the
// kernel's own stores might alias them, and waits on each load.
__device__ __forceinline__ DevItem uniform_item(const DevItem &g) {
    DevItem it;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        it.lo[a] = uni_d(g.lo[a]);
        it.L[a] = uni_d(g.L[a]);
    }
    it.S = uni_d(g.S);
    it.inv_res = uni_d(g.inv_res);
    it.start = g.start;
    it.count = g.count;
    it.n_owned = g.n_owned;
    it.owned_base = g.owned_base;
    const int64_t to = g.tab_off;
    it.tab_off = ((int64_t)uni_i((int)(to >> 32)) << 32) | (int64_t)(uint32_t)uni_i((int)(uint32_t)to);
    it.T = uni_i(g.T);
    it.periodic = uni_i(g.periodic);
    it.walls = uni_i(g.walls);
    it.pad = 0;
    return it;
}

// exclusive prefix sum over the wave
__device__ __forceinline__ int wave_excl_scan(int v, int *total) {
    int l = lane_id();
    int x = v;
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o);
        if (l >= o) x += y;
    }
    *total = __shfl(x, 63);
    return x - v;
}

// bitonic sort of 64 keys (one per lane), ascending by lane
__device__ __forceinline__ uint32_t bitonic64(uint32_t k) {
    int l = lane_id();
    for (int size = 2; size <= 64; size <<= 1) {
        for (int j = size >> 1; j > 0; j >>= 1) {
            uint32_t o = (uint32_t)__shfl_xor((int)k, j);
            bool up = (l & size) == 0 || size == 64;
            bool lower = (l & j) == 0;
            uint32_t mn = k < o ? k : o, mx = k < o ? o : k;
            k = (lower == up) ? mn : mx;
        }
    }
    return k;
}

// bitonic sort of 128 keys (element e = s * 64 + lane)
__device__ __forceinline__ void bitonic128(uint32_t &k0, uint32_t &k1) {
    int l = lane_id();
    for (int size = 2; size <= 128; size <<= 1) {
        for (int j = size >> 1; j > 0; j >>= 1) {
            if (j == 64) {
                uint32_t mn = k0 < k1 ? k0 : k1, mx = k0 < k1 ? k1 : k0;
                k0 = mn;
                k1 = mx;
                continue;
            }
            uint32_t o0 = (uint32_t)__shfl_xor((int)k0, j);
            uint32_t o1 = (uint32_t)__shfl_xor((int)k1, j);
            bool lower = (l & j) == 0;
            bool up0 = ((l & size) == 0);
            bool up1 = (((64 + l) & size) == 0);
            uint32_t mn0 = k0 < o0 ? k0 : o0, mx0 = k0 < o0 ? o0 : k0;
            uint32_t mn1 = k1 < o1 ? k1 : o1, mx1 = k1 < o1 ? o1 : k1;
            k0 = (lower == up0) ? mn0 : mx0;
            k1 = (lower == up1) ? mn1 : mx1;
        }
    }
}

// bitonic sort of 64*N 64-bit keys, element e = s * 64 + lane
template <int N>
__device__ __forceinline__ void bitonic_u64(uint64_t (&k)[N]) {
    int l = lane_id();
    const int total = 64 * N;
    for (int size = 2; size <= total; size <<= 1) {
        for (int j = size >> 1; j > 0; j >>= 1) {
            if (j >= 64) {
                int js = j >> 6;
#pragma unroll
                for (int s = 0; s < N; ++s) {
                    int p = s ^ js;
                    if (p > s) {
                        int e = s * 64 + l;
                        bool up = (e & size) == 0;
                        uint64_t a = k[s], b = k[p];
                        uint64_t mn = a < b ? a : b, mx = a < b ? b : a;
                        k[s] = up ? mn : mx;
                        k[p] = up ? mx : mn;
                    }
                }
            } else {
#pragma unroll
                for (int s = 0; s < N; ++s) {
                    uint64_t o = (uint64_t)__shfl_xor((long long)k[s], j);
                    int e = s * 64 + l;
                    bool up = (e & size) == 0;
                    bool lower = (l & j) == 0;
                    uint64_t mn = k[s] < o ? k[s] : o, mx = k[s] < o ? o : k[s];
                    k[s] = (lower == up) ? mn : mx;
                }
            }
        }
    }
}

// ------------------------------------------------------------------ geometry
template <typename T>
struct P4 {
    T x, y, z, d;  // half-space n.y <= d
};

__device__ __forceinline__ double fmad(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float fmad(float a, float b, float c) { return fmaf(a, b, c); }

template <typename T>
__device__ __forceinline__ void cross3(T ax, T ay, T az, T bx, T by, T bz, T &cx, T &cy, T &cz) {
    cx = fmad(ay, bz, -(az * by));
    cy = fmad(az, bx, -(ax * bz));
    cz = fmad(ax, by, -(ay * bx));
}

// FP64 1/x from the hardware reciprocal refined by two Newton steps (within an ulp or so of the
// correctly rounded quotient, at half the instructions and latency of the IEEE divide).
__device__ __forceinline__ double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(e, r, r);
    e = fma(-x, r, 1.0);
    return fma(e, r, r);
}
// FP32 (mixed path) keeps the IEEE quotient, which its vertex error bounds assume
__device__ __forceinline__ float recip(float x) { return 1.0f / x; }

// Intersection of three planes by Cramer's rule, with explicit FMAs (the
// library is built without FP contraction) so every kernel rounds it alike.
template <typename T>
__device__ __forceinline__ T intersect3(const P4<T> &a, const P4<T> &b, const P4<T> &c, T &x, T &y, T &z) {
    T bcx, bcy, bcz, cax, cay, caz, abx, aby, abz;
    cross3(b.x, b.y, b.z, c.x, c.y, c.z, bcx, bcy, bcz);
    cross3(c.x, c.y, c.z, a.x, a.y, a.z, cax, cay, caz);
    cross3(a.x, a.y, a.z, b.x, b.y, b.z, abx, aby, abz);
    T det = fmad(a.x, bcx, fmad(a.y, bcy, a.z * bcz));
    T inv = recip(det);
    x = fmad(a.d, bcx, fmad(b.d, cax, c.d * abx)) * inv;
    y = fmad(a.d, bcy, fmad(b.d, cay, c.d * aby)) * inv;
    z = fmad(a.d, bcz, fmad(b.d, caz, c.d * abz)) * inv;
    return det;
}

template <typename T>
__device__ __forceinline__ T side(T x, T y, T z, const P4<T> &p) {
    return fmad(x, p.x, fmad(y, p.y, z * p.z)) - p.d;
}

// ------------------------------------------------------------------ per-wave LDS
// NF face slots (at most 64 * VPL): a simple polytope with V vertices has V / 2 + 2 faces, so a
// kernel bounded to 64 vertices needs 34 and may hold fewer slots than 64 to save LDS.
template <typename T, int VPL, int NF = 64 * VPL>
struct PolyMem {
    static_assert(NF <= 64 * VPL && NF >= 8, "face slots");
    static constexpr int PMAX = NF;
    static constexpr int VMAX = 64 * VPL;
    static constexpr bool MIXED = std::is_same<T, float>::value;
    P4<double> pl64[PMAX];             // planes in FP64 (walls: unit normal, d = distance)
    P4<float> pl32[MIXED ? PMAX : 1];  // planes in FP32 (mixed path)
    float plh[MIXED ? PMAX : 1];       // plane distance from the seed (mixed error bound)
    float pln[MIXED ? PMAX : 1];       // |n| (mixed error bound)
    int32_t ptag[PMAX];                // generating particle (sorted index), or < 0 for walls
    uint64_t fm[PMAX][VPL];            // vertices on each plane
    T st[VMAX][3];                     // new-vertex staging
    uint32_t stt[VMAX];
    float ste[MIXED ? VMAX : 1];
};

enum { CLIP_NONE = 0, CLIP_CUT = 1, CLIP_OVERFLOW = -1, CLIP_CORRUPT = -2, CLIP_EMPTY = -3 };

template <typename T, int VPL, int NF = 64 * VPL>
struct Poly {
    using Mem = PolyMem<T, VPL, NF>;
    static constexpr bool MIXED = Mem::MIXED;
    static constexpr int PMAX = Mem::PMAX;
    static constexpr float U32 = 5.9604645e-08f;  // 2^-24

    T vx[VPL], vy[VPL], vz[VPL];
    uint32_t vt[VPL];
    float ve[VPL];     // position error bound (mixed)
    uint64_t alive[VPL], fa[VPL];
    double R2;         // squared largest vertex distance (conservative)

    // The box [blo, bhi] (seed-relative) with wall tags -1 .. -6 (-x,+x,-y,+y,-z,+z).
    __device__ void init_box(Mem &S, const double blo[3], const double bhi[3], int32_t tag_base = -1) {
        const int lane = lane_id();
        if (lane < 6) {
            int a = lane >> 1;
            bool pos = lane & 1;
            P4<double> p;
            p.x = (a == 0) ? (pos ? 1.0 : -1.0) : 0.0;
            p.y = (a == 1) ? (pos ? 1.0 : -1.0) : 0.0;
            p.z = (a == 2) ? (pos ? 1.0 : -1.0) : 0.0;
            p.d = pos ? bhi[a] : -blo[a];
            S.pl64[lane] = p;
            if constexpr (MIXED) {
                P4<float> q;
                q.x = (float)p.x;
                q.y = (float)p.y;
                q.z = (float)p.z;
                q.d = (float)p.d;
                S.pl32[lane] = q;
                S.plh[lane] = (float)fabs(p.d);
                S.pln[lane] = 1.0f;
            }
            S.ptag[lane] = tag_base - lane;
        }
#pragma unroll
        for (int s = 0; s < VPL; ++s) {
            vx[s] = vy[s] = vz[s] = T(0);
            vt[s] = 0;
            ve[s] = 0.f;
            alive[s] = 0;
            fa[s] = 0;
        }
        // vertex k (lanes 0..7) is corner (k&1, k&2, k&4); faces counter-clockwise from outside
        if (lane < 8) {
            int ix = lane & 1, iy = (lane >> 1) & 1, iz = (lane >> 2) & 1;
            vx[0] = (T)(ix ? bhi[0] : blo[0]);
            vy[0] = (T)(iy ? bhi[1] : blo[1]);
            vz[0] = (T)(iz ? bhi[2] : blo[2]);
            uint32_t X = ix ? 1 : 0, Y = iy ? 3 : 2, Z = iz ? 5 : 4;
            int neg = (1 - ix) + (1 - iy) + (1 - iz);
            vt[0] = (neg & 1) ? (X | (Z << 8) | (Y << 16)) : (X | (Y << 8) | (Z << 16));
            if constexpr (MIXED) {
                float r = sqrtf((float)(vx[0] * vx[0] + vy[0] * vy[0] + vz[0] * vz[0]));
                ve[0] = 4.f * U32 * r;
            }
        }
        alive[0] = 0xFFull;
        fa[0] = 0x3Full;
        for (int r = 0; r < VPL; ++r) {
            int f = r * 64 + lane;
            uint64_t m = 0;
            if (f < 6) {
                int a = f >> 1;
                bool pos = f & 1;
                for (int k = 0; k < 8; ++k)
                    if ((((k >> a) & 1) != 0) == pos) m |= 1ull << k;
            }
            if (f < PMAX)
                for (int s2 = 0; s2 < VPL; ++s2) S.fm[f][s2] = (s2 == 0) ? m : 0ull;
        }
        double hx = fmax(-blo[0], bhi[0]), hy = fmax(-blo[1], bhi[1]), hz = fmax(-blo[2], bhi[2]);
        R2 = (hx * hx + hy * hy + hz * hz) * (1.0 + 1e-12);
        wave_sync();
    }

    __device__ void update_r2() {
        const uint64_t mybit = 1ull << lane_id();
        double r2l = 0.0;
#pragma unroll
        for (int s = 0; s < VPL; ++s) {
            if (alive[s] & mybit) {
                double x = (double)vx[s], y = (double)vy[s], z = (double)vz[s];
                double d = x * x + y * y + z * z;
                if constexpr (MIXED) {
                    double rr = sqrt(d) * (1.0 + 1e-6) + (double)ve[s];
                    d = rr * rr;
                }
                r2l = fmax(r2l, d);
            }
        }
        R2 = uni_d(wave_max_x(r2l) * (1.0 + 1e-12));
    }

    // Clip by {y : p.y <= p.d} (p64 in FP64); `tag` identifies the plane.
    __device__ int clip(Mem &S, const P4<double> &p64, int32_t tag) {
        const int lane = lane_id();
        const uint64_t lt = lanemask_lt();
        const uint64_t mybit = 1ull << lane;
        P4<T> p;
        p.x = (T)p64.x;
        p.y = (T)p64.y;
        p.z = (T)p64.z;
        p.d = (T)p64.d;
        float pnorm = 0.f, ph = 0.f;
        if constexpr (MIXED) {
            pnorm = sqrtf(p.x * p.x + p.y * p.y + p.z * p.z);
            ph = fabsf(p.d) / pnorm;
        }
        // 1. side test
        bool out[VPL];
        uint64_t Mk[VPL];
        bool any = false, all = true;
#pragma unroll
        for (int s = 0; s < VPL; ++s) {
            bool al = (alive[s] & mybit) != 0;
            T sv = side<T>(vx[s], vy[s], vz[s], p);
            bool o = sv > T(0);
            if constexpr (MIXED) {
                float vn = sqrtf(vx[s] * vx[s] + vy[s] * vy[s] + vz[s] * vz[s]);
                float bound = pnorm * (ve[s] + 32.f * U32 * (ph + vn));
                if (al && fabsf(sv) <= bound) {
                    P4<double> qa = S.pl64[vt[s] & 0xFF], qb = S.pl64[(vt[s] >> 8) & 0xFF],
                               qc = S.pl64[(vt[s] >> 16) & 0xFF];
                    double wx, wy, wz;
                    intersect3<double>(qa, qb, qc, wx, wy, wz);
                    o = side<double>(wx, wy, wz, p64) > 0.0;
                }
            }
            out[s] = al && o;
            Mk[s] = __ballot(out[s]);
            any |= Mk[s] != 0;
            all &= Mk[s] == alive[s];
        }
        if (!any) return CLIP_NONE;
        if (all) return CLIP_EMPTY;
        // 2. slot for the new face
        int q = -1;
#pragma unroll
        for (int s = 0; s < VPL; ++s)
            if (q < 0 && ~fa[s] != 0ull) q = s * 64 + __builtin_ctzll(~fa[s]);
        if (q < 0 || q >= PMAX) return CLIP_OVERFLOW;
        // 3. cut edges: an edge of a clipped vertex whose twin vertex is kept
        int nbv[VPL];
        uint32_t emask[VPL];
        bool bad = false;
#pragma unroll
        for (int s = 0; s < VPL; ++s) {
            nbv[s] = 0;
            emask[s] = 0;
            if (out[s]) {
                const uint32_t t = vt[s];
                const int f0 = t & 0xFF, f1 = (t >> 8) & 0xFF, f2 = (t >> 16) & 0xFF;
                uint64_t m0[VPL], m1[VPL], m2[VPL];
#pragma unroll
                for (int ww = 0; ww < VPL; ++ww) {
                    m0[ww] = S.fm[f0][ww];
                    m1[ww] = S.fm[f1][ww];
                    m2[ww] = S.fm[f2][ww];
                }
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    bool nonzero = false, keptTwin = true;
#pragma unroll
                    for (int ww = 0; ww < VPL; ++ww) {
                        uint64_t x = (e == 0) ? (m0[ww] & m1[ww]) : (e == 1) ? (m1[ww] & m2[ww]) : (m2[ww] & m0[ww]);
                        if (ww == s) x &= ~mybit;
                        nonzero |= x != 0;
                        if (x & Mk[ww]) keptTwin = false;
                    }
                    if (!nonzero) bad = true;
                    if (nonzero && keptTwin) {
                        emask[s] |= 1u << e;
                        nbv[s]++;
                    }
                }
            }
        }
        if (__ballot(bad) != 0) return CLIP_CORRUPT;
        int pre_s[VPL];
        int NB = 0;
#pragma unroll
        for (int s = 0; s < VPL; ++s) {
            uint64_t b1 = __ballot(nbv[s] & 1), b2 = __ballot(nbv[s] & 2);
            pre_s[s] = NB + __popcll(b1 & lt) + 2 * __popcll(b2 & lt);
            NB += __popcll(b1) + 2 * __popcll(b2);
        }
        int nfree = 0;
#pragma unroll
        for (int s = 0; s < VPL; ++s) nfree += __popcll(~alive[s] | Mk[s]);
        if (NB > nfree) return CLIP_OVERFLOW;
        if (lane == 0) {
            S.pl64[q] = p64;
            if constexpr (MIXED) {
                S.pl32[q] = p;
                S.plh[q] = ph;
                S.pln[q] = pnorm;
            }
            S.ptag[q] = tag;
        }
        // 4. remove the clipped vertices from every face mask (the edge masks above were
        //    read first; LDS operations of one wavefront execute in order), noting which
        //    faces keep a vertex: those and the new face are the faces alive afterwards
        wave_sync();
        uint64_t keep[VPL];
#pragma unroll
        for (int r = 0; r < VPL; ++r) {
            const int f = r * 64 + lane;
            bool kept = false;
            if (fa[r] & mybit) {
#pragma unroll
                for (int ww = 0; ww < VPL; ++ww) {
                    const uint64_t m = S.fm[f][ww] & ~Mk[ww];
                    S.fm[f][ww] = m;
                    kept |= m != 0ull;
                }
            }
            keep[r] = __ballot(kept);
        }
        // 5. cut edges -> staging triples (a, b, p) in rank order
#pragma unroll
        for (int s = 0; s < VPL; ++s) {
            if (emask[s]) {
                const uint32_t t = vt[s];
                const int fx[3] = {(int)(t & 0xFF), (int)((t >> 8) & 0xFF), (int)((t >> 16) & 0xFF)};
                int k = pre_s[s];
                for (int e = 0; e < 3; ++e)
                    if (emask[s] & (1u << e))
                        S.stt[k++] = (uint32_t)fx[e] | ((uint32_t)fx[(e + 1) % 3] << 8) | ((uint32_t)q << 16);
            }
        }
        wave_sync();
        // 6. the r-th free lane takes the r-th new vertex: it computes the vertex itself as
        //    the intersection of its three planes, and joins the masks of its two old faces
        int rank0 = 0;
#pragma unroll
        for (int s = 0; s < VPL; ++s) {
            const uint64_t F = ~alive[s] | Mk[s];
            const int r = rank0 + __popcll(F & lt);
            const bool got = ((F & mybit) != 0) && r < NB;
            if (got) {
                const uint32_t t = S.stt[r];
                const int fa_ = t & 0xFF, fb_ = (t >> 8) & 0xFF;
                T wx, wy, wz;
                if constexpr (MIXED) {
                    const P4<float> pa = S.pl32[fa_], pb = S.pl32[fb_];
                    const float det = intersect3<float>(pa, pb, p, wx, wy, wz);
                    const float kap = S.pln[fa_] * S.pln[fb_] * pnorm / fabsf(det);
                    const float wn = sqrtf(wx * wx + wy * wy + wz * wz);
                    float err = 16.f * U32 * (kap * (S.plh[fa_] + S.plh[fb_] + ph + wn) + wn);
                    if (!(err < 1e30f)) err = 1e30f;
                    ve[s] = err;
                } else {
                    const P4<double> pa = S.pl64[fa_], pb = S.pl64[fb_];
                    intersect3<double>(pa, pb, p64, wx, wy, wz);
                }
                vx[s] = wx;
                vy[s] = wy;
                vz[s] = wz;
                vt[s] = t;
                atomicOr((unsigned long long *)&S.fm[fa_][s], (unsigned long long)mybit);
                atomicOr((unsigned long long *)&S.fm[fb_][s], (unsigned long long)mybit);
            }
            const uint64_t nm = __ballot(got);
            alive[s] = (alive[s] & ~Mk[s]) | nm;
            if (lane == 0) S.fm[q][s] = nm;
            rank0 += __popcll(F);
        }
        wave_sync();
        // 7. faces alive: those that kept a vertex, and the new one
#pragma unroll
        for (int r = 0; r < VPL; ++r) fa[r] = keep[r] | ((q >> 6) == r ? (1ull << (q & 63)) : 0ull);
        // R2 is left as it was: an upper bound (the cell only shrinks); callers
        // refresh it with update_r2() when they need the tighter value
        return CLIP_CUT;
    }

    __device__ int nvertices() const {
        int n = 0;
#pragma unroll
        for (int s = 0; s < VPL; ++s) n += __popcll(alive[s]);
        return n;
    }

    // FP64 position of this lane's vertex in slot s (recomputed from the planes on the mixed path)
    __device__ void pos64(const Mem &S, int s, double &x, double &y, double &z) const {
        if constexpr (MIXED) {
            P4<double> qa = S.pl64[vt[s] & 0xFF], qb = S.pl64[(vt[s] >> 8) & 0xFF], qc = S.pl64[(vt[s] >> 16) & 0xFF];
            intersect3<double>(qa, qb, qc, x, y, z);
        } else {
            x = (double)vx[s];
            y = (double)vy[s];
            z = (double)vz[s];
        }
    }

    // Volume in FP64 without walking faces: the cone over face f from the seed
    // is the sum of tetrahedra (seed, F_f, u, next_f(u)) over the vertices u of f,
    // with F_f the foot of the seed on plane f; next_f(u) is the vertex that
    // follows u counter-clockwise on f.  vp/vtri: LDS scratch of VMAX entries.
    __device__ double volume(const Mem &S, double (*vp)[3]) const {
        const int lane = lane_id();
        const uint64_t mybit = 1ull << lane;
#pragma unroll
        for (int s = 0; s < VPL; ++s) {
            if (alive[s] & mybit) {
                double x, y, z;
                pos64(S, s, x, y, z);
                vp[s * 64 + lane][0] = x;
                vp[s * 64 + lane][1] = y;
                vp[s * 64 + lane][2] = z;
            }
        }
        wave_sync();
        double acc = 0.0;
#pragma unroll
        for (int s = 0; s < VPL; ++s) {
            if (!(alive[s] & mybit)) continue;
            const int u = s * 64 + lane;
            const uint32_t t = vt[s];
            const int f[3] = {(int)(t & 0xFF), (int)((t >> 8) & 0xFF), (int)((t >> 16) & 0xFF)};
            const double *pu = vp[u];
            for (int k = 0; k < 3; ++k) {
                // on face f[k] the next vertex shares f[k] and f[k+2] (the face before f[k] in the triple)
                const int fk = f[k], fc = f[(k + 2) % 3];
                int w = -1;
#pragma unroll
                for (int ww = 0; ww < VPL; ++ww) {
                    uint64_t x = S.fm[fk][ww] & S.fm[fc][ww];
                    if (ww == s) x &= ~mybit;
                    if (w < 0 && x) w = ww * 64 + __builtin_ctzll(x);
                }
                if (w < 0) continue;
                const double *pw = vp[w];
                const P4<double> &pl = S.pl64[fk];
                double nn = pl.x * pl.x + pl.y * pl.y + pl.z * pl.z;
                double sc = pl.d / nn;
                double Fx = pl.x * sc, Fy = pl.y * sc, Fz = pl.z * sc;
                double cx = pu[1] * pw[2] - pu[2] * pw[1];
                double cy = pu[2] * pw[0] - pu[0] * pw[2];
                double cz = pu[0] * pw[1] - pu[1] * pw[0];
                acc += (Fx * cx + Fy * cy + Fz * cz) / 6.0;
            }
        }
        return wave_sum_d(acc);
    }
};

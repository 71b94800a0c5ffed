// sort.hip -- particle ordering for the neighbour search.
//
// Each world (item) is quantised on a 2^16 grid over a cube of side S, and its
// particles are sorted along the Morton curve (key = item << 48 | morton48) by
// an LSD radix sort with 8-bit digits.  A Morton cell at level l is then a
// contiguous range of the sorted arrays; a dense table at level T (8^T cells,
// about one particle per cell) gives these ranges directly for l <= T, and a
// binary search inside a level-T cell gives them for l > T.  This replaces the
// search structure the paper gets from Qhull (section 2) with one whose memory
// accesses are contiguous ranges.
#include "vt_internal.h"

#define SORT_THREADS 256
#define SORT_ITEMS 16
#define SORT_TILE (SORT_THREADS * SORT_ITEMS)

// ------------------------------------------------------------------ scan
#define SCAN_THREADS 256
#define SCAN_ITEMS 16
#define SCAN_TILE (SCAN_THREADS * SCAN_ITEMS)

int64_t vt_scan_tmp_elems(int64_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 1; }

template <typename T>
__device__ T block_exclusive_scan(T v, T *lds, T *total) {
    // Hillis-Steele over the block (256 threads) in LDS
    int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int off = 1; off < SCAN_THREADS; off <<= 1) {
        T x = (t >= off) ? lds[t - off] : T(0);
        __syncthreads();
        lds[t] += x;
        __syncthreads();
    }
    T incl = lds[t];
    *total = lds[SCAN_THREADS - 1];
    __syncthreads();
    return incl - v;
}

template <typename T>
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_reduce(const T *in, int64_t n, int64_t *sums) {
    __shared__ int64_t lds[SCAN_THREADS];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int64_t acc = 0;
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t k = base + (int64_t)i * SCAN_THREADS + threadIdx.x;
        if (k < n) acc += (int64_t)in[k];
    }
    int64_t tot;
    block_exclusive_scan<int64_t>(acc, lds, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// single block: exclusive scan of the block sums (nb <= SCAN_THREADS * 64)
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_top(int64_t *sums, int64_t nb) {
    __shared__ int64_t lds[SCAN_THREADS];
    const int per = 64;
    int64_t base = (int64_t)threadIdx.x * per;
    int64_t acc = 0;
    for (int i = 0; i < per; ++i)
        if (base + i < nb) acc += sums[base + i];
    int64_t tot;
    int64_t off = block_exclusive_scan<int64_t>(acc, lds, &tot);
    for (int i = 0; i < per; ++i)
        if (base + i < nb) {
            int64_t x = sums[base + i];
            sums[base + i] = off;
            off += x;
        }
    if (threadIdx.x == 0) sums[nb] = tot;
}

template <typename T>
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_down(const T *in, T *out, int64_t n, const int64_t *sums,
                                                            int write_total, int64_t nb) {
    __shared__ int64_t lds[SCAN_THREADS];
    __shared__ T tile[SCAN_TILE];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t k = base + (int64_t)i * SCAN_THREADS + threadIdx.x;
        tile[i * SCAN_THREADS + threadIdx.x] = (k < n) ? in[k] : T(0);
    }
    __syncthreads();
    // each thread scans SCAN_ITEMS consecutive elements of the tile
    int64_t acc = 0;
    T loc[SCAN_ITEMS];
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        loc[i] = tile[threadIdx.x * SCAN_ITEMS + i];
        acc += (int64_t)loc[i];
    }
    int64_t tot;
    int64_t off = block_exclusive_scan<int64_t>(acc, lds, &tot) + sums[blockIdx.x];
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        tile[threadIdx.x * SCAN_ITEMS + i] = (T)off;
        off += (int64_t)loc[i];
    }
    __syncthreads();
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t k = base + (int64_t)i * SCAN_THREADS + threadIdx.x;
        if (k < n) out[k] = tile[i * SCAN_THREADS + threadIdx.x];
    }
    if (write_total && blockIdx.x == 0 && threadIdx.x == 0) out[n] = (T)sums[nb];
}

// a scan of at most one tile: the block's own prefix, and the total, in one launch
template <typename T>
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_single(const T *in, T *out, int64_t n) {
    __shared__ int64_t lds[SCAN_THREADS];
    const int t = threadIdx.x;
    int64_t acc = 0;
    T loc[SCAN_ITEMS];
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        const int64_t k = (int64_t)t * SCAN_ITEMS + i;
        loc[i] = k < n ? in[k] : T(0);
        acc += (int64_t)loc[i];
    }
    int64_t tot;
    int64_t off = block_exclusive_scan<int64_t>(acc, lds, &tot);
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        const int64_t k = (int64_t)t * SCAN_ITEMS + i;
        if (k < n) out[k] = (T)off;
        off += (int64_t)loc[i];
    }
    if (t == 0) out[n] = (T)tot;
}

template <typename T>
static hipError_t scan_impl(const T *in, T *out, int64_t n, int64_t *tmp, hipStream_t s) {
    int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 0) nb = 1;
    if (nb > SCAN_THREADS * 64) return hipErrorInvalidValue;
    if (nb == 1) {
        k_scan_single<T><<<1, SCAN_THREADS, 0, s>>>(in, out, n);
        return hipGetLastError();
    }
    k_scan_reduce<T><<<nb, SCAN_THREADS, 0, s>>>(in, n, tmp);
    k_scan_top<<<1, SCAN_THREADS, 0, s>>>(tmp, nb);
    k_scan_down<T><<<nb, SCAN_THREADS, 0, s>>>(in, out, n, tmp, 1, nb);
    return hipGetLastError();
}

// exclusive scan: out[0..n] with out[n] = total; in and out must not overlap
hipError_t vt_launch_scan_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *tmp, hipStream_t s) {
    return scan_impl<int64_t>(in, out, n, tmp, s);
}
hipError_t vt_launch_scan_i32(const int32_t *in, int32_t *out, int64_t n, int64_t *tmp, hipStream_t s) {
    return scan_impl<int32_t>(in, out, n, tmp, s);
}

__global__ void k_zero_u32(uint32_t *p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

hipError_t vt_launch_zero_u32(uint32_t *p, int64_t n, hipStream_t s) {
    k_zero_u32<<<(n + 255) / 256, 256, 0, s>>>(p, n);
    return hipGetLastError();
}

// ------------------------------------------------------------------ keys
__device__ __forceinline__ int find_item(const DevItem *items, int n_items, int64_t p) {
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (items[mid].start <= p) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <typename PT>
__global__ void k_keys(const PT *pos, int64_t n, const DevItem *items, int n_items, uint64_t *keys, uint32_t *vals) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int b = find_item(items, n_items, p);
    const DevItem &it = items[b];
    uint64_t q[3];
    for (int a = 0; a < 3; ++a) {
        double x = (double)pos[3 * p + a];
        if (it.periodic) x -= it.L[a] * floor((x - it.lo[a]) / it.L[a]);
        q[a] = (uint64_t)vt_qclamp(vt_qraw(x, it.lo[a], it.inv_res));
    }
    keys[p] = ((uint64_t)b << VT_LOCAL_KEY_BITS) | vt_morton(q[0], q[1], q[2]);
    vals[p] = (uint32_t)p;
}

// ------------------------------------------------------------------ radix sort
__global__ void __launch_bounds__(SORT_THREADS) k_radix_hist(const uint64_t *keys, int64_t n, int shift,
                                                             int32_t *hist, int nblocks) {
    __shared__ int32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * SORT_TILE;
    for (int i = 0; i < SORT_ITEMS; ++i) {
        int64_t k = base + (int64_t)i * SORT_THREADS + threadIdx.x;
        if (k < n) atomicAdd(&h[(keys[k] >> shift) & 255u], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one tile.  Keys are ranked in index order: round-major, then wave, then lane;
// lanes holding the same digit are found with eight ballots.  The tile is first reordered by digit
// in LDS (its digit counts are the histogram's, their prefix the digits' starts in the tile), then
// written out in that order: consecutive threads write consecutive slots of each digit's run (16
// keys per digit on average), not one scattered slot each.  Thread t brings digit t's count in the
// tile and its global offset.
__device__ __forceinline__ void radix_scatter_tile(const uint64_t *kin, const uint32_t *vin, uint64_t *kout,
                                                   uint32_t *vout, int64_t n, int shift, int64_t base,
                                                   int32_t count_t, int64_t offset_t) {
    __shared__ int32_t running[256];   // next slot of each digit in the reordered tile
    __shared__ int64_t gbase[256];     // the digit's global offset minus its start in the tile
    __shared__ int32_t wcnt[SORT_THREADS / 64][256];
    __shared__ int32_t scan_lds[SORT_THREADS];
    __shared__ uint64_t lkey[SORT_TILE];
    __shared__ uint32_t lval[SORT_TILE];
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    {
        int32_t tot;
        const int32_t start = block_exclusive_scan<int32_t>(count_t, scan_lds, &tot);
        running[t] = start;
        gbase[t] = offset_t - start;
    }
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int i = 0; i < SORT_ITEMS; ++i) {
        for (int ww = 0; ww < SORT_THREADS / 64; ++ww) wcnt[ww][t] = 0;
        __syncthreads();
        int64_t k = base + (int64_t)i * SORT_THREADS + t;
        bool valid = k < n;
        uint64_t key = valid ? kin[k] : 0ull;
        uint32_t val = valid ? vin[k] : 0u;
        uint32_t d = (uint32_t)(key >> shift) & 255u;
        uint64_t match = __ballot(valid);
        for (int bit = 0; bit < 8; ++bit) {
            uint64_t b = __ballot(valid && ((d >> bit) & 1u));
            match &= ((d >> bit) & 1u) ? b : ~b;
        }
        int rank = __popcll(match & lt);
        if (valid && rank == 0) wcnt[w][d] = __popcll(match);
        __syncthreads();
        int pre = 0;
        for (int ww = 0; ww < w; ++ww) pre += wcnt[ww][d];
        if (valid) {
            const int slot = running[d] + pre + rank;
            lkey[slot] = key;
            lval[slot] = val;
        }
        __syncthreads();
        int add = 0;
        for (int ww = 0; ww < SORT_THREADS / 64; ++ww) add += wcnt[ww][t];
        running[t] += add;
        __syncthreads();
    }
    const int64_t left = n - base;
    const int cnt = left < (int64_t)SORT_TILE ? (int)left : SORT_TILE;
    for (int idx = t; idx < cnt; idx += SORT_THREADS) {
        const uint64_t key = lkey[idx];
        const int64_t pos = gbase[(uint32_t)(key >> shift) & 255u] + idx;
        kout[pos] = key;
        vout[pos] = lval[idx];
    }
}

__global__ void __launch_bounds__(SORT_THREADS) k_radix_scatter(const uint64_t *kin, const uint32_t *vin,
                                                                uint64_t *kout, uint32_t *vout, int64_t n,
                                                                int shift, const int32_t *counts,
                                                                const int32_t *offs, int nblocks) {
    const int t = threadIdx.x;
    radix_scatter_tile(kin, vin, kout, vout, n, shift, (int64_t)blockIdx.x * SORT_TILE,
                       counts[(int64_t)t * nblocks + blockIdx.x], (int64_t)offs[(int64_t)t * nblocks + blockIdx.x]);
}

// The whole sort of at most one tile (SORT_TILE keys) in one block: every pass's histogram, digit
// offsets and scatter, the passes ping-ponging between the two buffers (a pass reads what the
// block wrote in the one before, after a block barrier).  Small inputs then take one launch
// instead of five per pass.
__global__ void __launch_bounds__(SORT_THREADS) k_radix_tile(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1,
                                                             int64_t n, int key_bits) {
    __shared__ int32_t h[256];
    __shared__ int32_t scan_h[SORT_THREADS];
    const int t = threadIdx.x;
    uint64_t *kin = k0, *kout = k1;
    uint32_t *vin = v0, *vout = v1;
    for (int shift = 0; shift < key_bits; shift += 8) {
        h[t] = 0;
        __syncthreads();
        for (int i = 0; i < SORT_ITEMS; ++i) {
            const int64_t k = (int64_t)i * SORT_THREADS + t;
            if (k < n) atomicAdd(&h[(kin[k] >> shift) & 255u], 1);
        }
        __syncthreads();
        const int32_t cnt = h[t];
        int32_t tot;
        const int32_t off = block_exclusive_scan<int32_t>(cnt, scan_h, &tot);
        radix_scatter_tile(kin, vin, kout, vout, n, shift, 0, cnt, (int64_t)off);
        __syncthreads();
        uint64_t *tk = kin;
        kin = kout;
        kout = tk;
        uint32_t *tv = vin;
        vin = vout;
        vout = tv;
    }
}

// ------------------------------------------------------------------ sorted arrays
template <typename PT, typename PT4>
__global__ void k_sorted_gather(const PT *pos, const int32_t *gid, const uint32_t *order, int64_t n,
                                const DevItem *items, int n_items, PT4 *spos, int32_t *sgid, int32_t *srow,
                                int32_t *sorig) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int64_t p = order[j];
    int b = find_item(items, n_items, p);
    const DevItem &it = items[b];
    PT4 v;
    double x[3];
    for (int a = 0; a < 3; ++a) {
        x[a] = (double)pos[3 * p + a];
        if (it.periodic) {
            x[a] -= it.L[a] * floor((x[a] - it.lo[a]) / it.L[a]);
            if (x[a] >= it.lo[a] + it.L[a]) x[a] = it.lo[a];  // a value that rounds up to the top wall wraps to lo
        }
    }
    v.x = (decltype(v.x))x[0];
    v.y = (decltype(v.x))x[1];
    v.z = (decltype(v.x))x[2];
    v.w = 0;
    spos[j] = v;
    sgid[j] = gid ? gid[p] : (int32_t)p;
    int64_t k = p - it.start;
    srow[j] = (k < it.n_owned) ? (int32_t)(it.owned_base + k) : -1;
    sorig[j] = (int32_t)p;
}

// level-T table: tab[off + c] = first sorted index whose level-T cell is >= c.  The entries from
// particle j's predecessor's cell (exclusive) to its own take j, and the last particle of an item
// also fills the rest of the item's table.  A wavefront's 64 consecutive particles own one
// contiguous stretch of the table.  When the stretch is short its lanes write it together, entry
// by entry (the value of an entry is the first of the 64 whose cell reaches it, found by a binary
// search over their cells), so the writes are coalesced however unevenly the particles fill the
// cells.  Otherwise (empty regions: voids, the part of a cuboid item's Morton cube outside the item,
// the end of an item's table) each lane writes its own run if it is short, and lists a long run
// as pieces of at most VT_TAB_PIECE entries (slots reserved once per wavefront), which k_level_fill
// writes a wavefront per piece; runs that find the list full are written by their own lane.
#define VT_TAB_STRETCH 2048
#define VT_TAB_SHORT 64
#define VT_TAB_PIECE 4096
__device__ __forceinline__ int64_t tab_pieces(int64_t len) {
    return len > VT_TAB_SHORT ? (len + VT_TAB_PIECE - 1) / VT_TAB_PIECE : 0;
}

// Each lane's runs (its own and, for an item's last particle, the tail): short ones written here,
// long ones listed in slots reserved for the whole wavefront with one atomic; a lane whose slots do
// not all fit writes its runs itself and leaves its slots below the capacity as empty pieces.
__device__ __forceinline__ void tab_runs(int32_t *tab, int64_t loA, int64_t lenA, int32_t vA, int64_t loB, int64_t lenB,
                                         int32_t vB, uint64_t *pieces, int64_t piece_cap, uint32_t *counters) {
    const int64_t pa = tab_pieces(lenA), pb = tab_pieces(lenB), mine = pa + pb;
    // inclusive prefix of the lanes' piece counts, then one reservation for the wavefront
    const int lane = (int)(threadIdx.x & 63);
    int64_t pre = mine;
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t y = (int64_t)__shfl_up((long long)pre, o);
        if (lane >= o) pre += y;
    }
    const int64_t total = (int64_t)__shfl((long long)pre, 63);
    pre -= mine;
    int64_t base = 0;
    if (total > 0) {
        if (lane == 0) base = (int64_t)atomicAdd(&counters[CTR_TAB_PIECES], (uint32_t)total);
        base = (int64_t)__shfl((long long)base, 0);
    }
    const int64_t k0 = base + pre;
    const bool fits = k0 + mine <= piece_cap;
    if (!fits)
        for (int64_t q = k0; q < k0 + mine && q < piece_cap; ++q) {
            pieces[2 * q] = 0;
            pieces[2 * q + 1] = 0;
        }
    auto put = [&](int64_t lo, int64_t len, int32_t v, int64_t np, int64_t k) {
        if (np == 0 || !fits) {
            for (int64_t x = 0; x < len; ++x) tab[lo + x] = v;
            return;
        }
        for (int64_t q = 0; q < np; ++q) {
            const int64_t a = q * VT_TAB_PIECE, m = len - a < VT_TAB_PIECE ? len - a : VT_TAB_PIECE;
            pieces[2 * (k + q)] = (uint64_t)(lo + a);
            pieces[2 * (k + q) + 1] = ((uint64_t)m << 32) | (uint64_t)(uint32_t)v;
        }
    };
    if (lenA > 0) put(loA, lenA, vA, pa, k0);
    if (lenB > 0) put(loB, lenB, vB, pb, k0 + pa);
}

__global__ void __launch_bounds__(256) k_level_table(const uint64_t *skey, int64_t n, const DevItem *items,
                                                     int n_items, int32_t *tab, uint64_t *pieces, int64_t piece_cap,
                                                     uint32_t *counters) {
    __shared__ int64_t cells[4][64];
    const int lane = (int)(threadIdx.x & 63), wv = (int)(threadIdx.x >> 6);
    const int64_t jw = (int64_t)blockIdx.x * blockDim.x + wv * 64;  // the wavefront's first particle
    if (jw >= n) return;
    const int64_t j = jw + lane;
    const bool valid = j < n;
    const uint64_t lmask = (1ull << VT_LOCAL_KEY_BITS) - 1;
    int b = valid ? find_item(items, n_items, j) : -1;
    int64_t c = INT64_MAX, cprev = -1;
    if (valid) {
        const DevItem &it = items[b];
        const int sh = 3 * (VT_MORTON_BITS - it.T);
        c = (int64_t)((skey[j] & lmask) >> sh);
        cprev = (j == it.start) ? -1 : (int64_t)((skey[j - 1] & lmask) >> sh);
    }
    const int b0 = __shfl(b, 0);
    const uint64_t vm = __ballot(valid);
    const int last = 63 - __builtin_clzll(vm);
    const int64_t x0 = (int64_t)__shfl((long long)cprev, 0) + 1, x1 = (int64_t)__shfl((long long)c, last);
    if (__ballot(valid && b != b0) != 0 || x1 - x0 + 1 > VT_TAB_STRETCH) {
        // the wavefront spans two items, or its stretch is long: each lane its own runs
        int64_t loA = 0, lenA = 0, loB = 0, lenB = 0;
        int32_t vB = 0;
        if (valid) {
            const DevItem &it = items[b];
            loA = it.tab_off + cprev + 1;
            lenA = c - cprev;
            if (j == it.start + it.count - 1) {
                loB = it.tab_off + c + 1;
                lenB = (1ll << (3 * it.T)) - c;
                vB = (int32_t)(it.start + it.count);
            }
        }
        tab_runs(tab, loA, lenA, (int32_t)j, loB, lenB, vB, pieces, piece_cap, counters);
        return;
    }
    const DevItem &it = items[b0];
    cells[wv][lane] = c;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int64_t x = x0 + lane; x <= x1; x += 64) {
        int lo = 0, hi = last;  // the first particle whose cell is >= x (cells ascend; the last one's is x1)
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (cells[wv][mid] >= x) hi = mid; else lo = mid + 1;
        }
        tab[it.tab_off + x] = (int32_t)(jw + lo);
    }
    if (jw + last == it.start + it.count - 1) {
        // the item's tail, from the lane of its last particle
        const bool mine = lane == last;
        tab_runs(tab, 0, 0, 0, mine ? it.tab_off + x1 + 1 : 0, mine ? (1ll << (3 * it.T)) - x1 : 0,
                 (int32_t)(it.start + it.count), pieces, piece_cap, counters);
    }
}

// the listed pieces, a wavefront per piece
__global__ void __launch_bounds__(256) k_level_fill(const uint64_t *pieces, int64_t piece_cap, const uint32_t *counters,
                                                    int32_t *tab) {
    const int64_t np = min((int64_t)counters[CTR_TAB_PIECES], piece_cap);
    const int lane = (int)(threadIdx.x & 63);
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t p = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); p < np; p += nw) {
        const int64_t lo = (int64_t)pieces[2 * p];
        const uint64_t w = pieces[2 * p + 1];
        const int64_t m = (int64_t)(w >> 32);
        const int32_t v = (int32_t)(uint32_t)w;
        for (int64_t x = lane; x < m; x += 64) tab[lo + x] = v;
    }
}

__global__ void k_owned_flags(const int32_t *srow, int64_t n, int32_t *flag) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) flag[j] = srow[j] >= 0 ? 1 : 0;
}

__global__ void k_owned_compact(const int32_t *srow, const int32_t *scan, int64_t n, int32_t *cells,
                                int32_t *row2cell) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int32_t r = srow[j];
    if (r >= 0) {
        int32_t c = scan[j];
        cells[c] = (int32_t)j;
        row2cell[r] = c;
    }
}

hipError_t vt_launch_sort(vt_ctx *c, const void *pos, const int32_t *gid) {
    hipStream_t s = c->stream;
    const int64_t n = c->n_total;
    const int nb = (int)((n + SORT_TILE - 1) / SORT_TILE);
    const int tpb = 256;
    const int64_t grid = (n + tpb - 1) / tpb;
    if (c->dtype == VT_F32)
        k_keys<float><<<grid, tpb, 0, s>>>((const float *)pos, n, c->items, c->n_items, c->keys[0], c->vals[0]);
    else
        k_keys<double><<<grid, tpb, 0, s>>>((const double *)pos, n, c->items, c->n_items, c->keys[0], c->vals[0]);
    int cur = 0;
    if (nb == 1) {
        // one tile: the whole radix sort in one block
        k_radix_tile<<<1, SORT_THREADS, 0, s>>>(c->keys[0], c->vals[0], c->keys[1], c->vals[1], n, c->key_bits);
        cur = ((c->key_bits + 7) / 8) & 1;
    }
    for (int shift = 0; nb > 1 && shift < c->key_bits; shift += 8) {
        k_radix_hist<<<nb, SORT_THREADS, 0, s>>>(c->keys[cur], n, shift, c->hist, nb);
        hipError_t e = vt_launch_scan_i32(c->hist, c->hist + (int64_t)256 * nb, (int64_t)256 * nb, c->scan_tmp, s);
        if (e != hipSuccess) return e;
        k_radix_scatter<<<nb, SORT_THREADS, 0, s>>>(c->keys[cur], c->vals[cur], c->keys[cur ^ 1], c->vals[cur ^ 1], n,
                                                   shift, c->hist, c->hist + (int64_t)256 * nb, nb);
        cur ^= 1;
    }
    c->skey = c->keys[cur];
    if (c->dtype == VT_F32)
        k_sorted_gather<float, float4><<<grid, tpb, 0, s>>>((const float *)pos, gid, c->vals[cur], n, c->items,
                                                            c->n_items, (float4 *)c->spos, c->sgid, c->srow, c->sorig);
    else
        k_sorted_gather<double, double4><<<grid, tpb, 0, s>>>((const double *)pos, gid, c->vals[cur], n, c->items,
                                                              c->n_items, (double4 *)c->spos, c->sgid, c->srow,
                                                              c->sorig);
    // long runs of the table are listed in the spare key buffer (free until the compaction below)
    uint64_t *pieces = c->keys[cur ^ 1];
    const int64_t piece_cap = (n + 1) / 2;
    k_level_table<<<grid, tpb, 0, s>>>(c->skey, n, c->items, c->n_items, c->tab, pieces, piece_cap, c->counters);
    k_level_fill<<<1024, tpb, 0, s>>>(pieces, piece_cap, c->counters, c->tab);
    // owned cells in Morton order (flags -> scan -> compact); the flag array reuses vals[cur^1]
    int32_t *flag = (int32_t *)c->vals[cur ^ 1];
    int32_t *scan = (int32_t *)c->keys[cur ^ 1];
    k_owned_flags<<<grid, tpb, 0, s>>>(c->srow, n, flag);
    hipError_t e = vt_launch_scan_i32(flag, scan, n, c->scan_tmp, s);
    if (e != hipSuccess) return e;
    k_owned_compact<<<grid, tpb, 0, s>>>(c->srow, scan, n, c->cells, c->row2cell);
    return hipGetLastError();
}

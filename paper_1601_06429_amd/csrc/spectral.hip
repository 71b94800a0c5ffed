// spectral.hip -- second-derivative tensors of a periodic grid field, for the tidal-tensor and
// Hessian analysis the paper lists as future grid outputs (section 4):
//   tidal:   T_ij = d_i d_j phi,  laplacian(phi) = delta,  delta = f / mean(f) - 1
//            -> T_ij(k) = k_i k_j / |k|^2 * f(k) / mean(f)   (k != 0; 0 at k = 0)
//   Hessian: H_ij = d_i d_j f  ->  H_ij(k) = -k_i k_j f(k)
// with k_a = 2 pi m / L_a, m the signed frequency index.  A mixed component (i != j) is set to
// zero on the Nyquist plane of either of its axes, where the sign of k is ambiguous; this keeps
// every multiplier even in k, so every component is real.
//
// The 3D FFT is three passes of 1D transforms, one per axis.  A block takes B whole lines of
// length N (B N up to 2048 complex values, 32 KB of LDS, plus N / 2 twiddles; a line of 4096 is
// a block of its own) chosen so that its loads and stores are coalesced: lines along the
// contiguous axis are taken consecutively, lines along the other axes side by side.  Blocks of
// 32 KB leave room for four per CU; blocks of 64 KB, two, and took 27% longer at 256^3.  Each
// line is transformed in LDS by an in-place radix-2 decimation in time (loaded in bit-reversed
// order), two stages per pass over the LDS; the twiddles are computed once per block with
// sincospi in FP64.  Two real components go through one inverse transform as the real and
// imaginary parts of one complex field.
#include <mutex>

#include "vt_internal.h"

#define FFT_TPB 256
#define FFT_LDS 2048   // complex values per block (lines of up to 4096 take one block each)

// element i of line l of the transform along `axis` of an n0 x n1 x n2 array (n2 contiguous)
__device__ __forceinline__ int64_t line_elem(int axis, int64_t l, int64_t i, int n1, int n2) {
    if (axis == 2) return l * n2 + i;
    if (axis == 1) return (l / n2) * ((int64_t)n1 * n2) + (l % n2) + i * n2;
    return l + i * ((int64_t)n1 * n2);
}

// v times the twiddle t = (cos, sin)
__device__ __forceinline__ double2 bmul(double2 v, double2 t) {
    return make_double2(v.x * t.x - v.y * t.y, v.x * t.y + v.y * t.x);
}

__global__ void __launch_bounds__(FFT_TPB) k_fft(double2 *data, int n0, int n1, int n2, int axis, int logn, int B,
                                               double sign) {
    extern __shared__ double2 sl[];
    const int N = 1 << logn;
    const int64_t l0 = (int64_t)blockIdx.x * B;
    const int total = B * N;
    // twiddles exp(sign 2 pi i m / N), m < N / 2; stage s takes m = k N / 2^s, the same argument
    // k / 2^(s-1) as evaluating it in the stage
    double2 *tw = sl + total;
    for (int m = threadIdx.x; m < N / 2; m += FFT_TPB) {
        double sn, cs;
        sincospi(sign * 2.0 * (double)m / (double)N, &sn, &cs);
        tw[m] = make_double2(cs, sn);
    }
    // load in bit-reversed order within each line; consecutive threads take consecutive
    // addresses (along the line for the contiguous axis, across lines otherwise)
    for (int t = threadIdx.x; t < total; t += FFT_TPB) {
        int l, i;
        if (axis == 2) {
            l = t >> logn;
            i = t & (N - 1);
        } else {
            l = t % B;
            i = t / B;
        }
        const int r = (int)(__brev((unsigned)i) >> (32 - logn));
        sl[l * N + r] = data[line_elem(axis, l0 + l, i, n1, n2)];
    }
    __syncthreads();
    // stages s and s + 1 together: a thread takes the four points k, k + h, k + 2h, k + 3h of a
    // block of 4h (h = 2^(s-1)) through both radix-2 stages in registers, each point through
    // the same butterflies as stage by stage
    int s = 1;
    for (; s + 1 <= logn; s += 2) {
        const int h = 1 << (s - 1);
        for (int b = threadIdx.x; b < total / 4; b += FFT_TPB) {
            const int l = b >> (logn - 2);
            const int j = b & (N / 4 - 1);
            const int k = j & (h - 1);
            const int i0 = l * N + ((j >> (s - 1)) << (s + 1)) + k;
            const double2 a = sl[i0], bb = sl[i0 + h], c = sl[i0 + 2 * h], d = sl[i0 + 3 * h];
            const double2 t1 = tw[k << (logn - s)];
            const double2 t2 = tw[k << (logn - s - 1)], t3 = tw[(k + h) << (logn - s - 1)];
            const double2 wb = bmul(bb, t1), wd = bmul(d, t1);
            const double2 a1 = make_double2(a.x + wb.x, a.y + wb.y), b1 = make_double2(a.x - wb.x, a.y - wb.y);
            const double2 c1 = make_double2(c.x + wd.x, c.y + wd.y), d1 = make_double2(c.x - wd.x, c.y - wd.y);
            const double2 wc = bmul(c1, t2), wd1 = bmul(d1, t3);
            sl[i0] = make_double2(a1.x + wc.x, a1.y + wc.y);
            sl[i0 + 2 * h] = make_double2(a1.x - wc.x, a1.y - wc.y);
            sl[i0 + h] = make_double2(b1.x + wd1.x, b1.y + wd1.y);
            sl[i0 + 3 * h] = make_double2(b1.x - wd1.x, b1.y - wd1.y);
        }
        __syncthreads();
    }
    if (s == logn) {   // an odd number of stages: the last one alone
        const int half = 1 << (s - 1);
        for (int b = threadIdx.x; b < total / 2; b += FFT_TPB) {
            const int l = b >> (logn - 1);
            const int j = b & (N / 2 - 1);
            const int k = j & (half - 1);
            const int i0 = l * N + ((j >> (s - 1)) << s) + k;
            const int i1 = i0 + half;
            const double2 u = sl[i0];
            const double2 w = bmul(sl[i1], tw[k << (logn - s)]);
            sl[i0] = make_double2(u.x + w.x, u.y + w.y);
            sl[i1] = make_double2(u.x - w.x, u.y - w.y);
        }
        __syncthreads();
    }
    for (int t = threadIdx.x; t < total; t += FFT_TPB) {
        int l, i;
        if (axis == 2) {
            l = t >> logn;
            i = t & (N - 1);
        } else {
            l = t % B;
            i = t / B;
        }
        data[line_elem(axis, l0 + l, i, n1, n2)] = sl[l * N + i];
    }
}

__global__ void k_real_to_complex(const double *f, double2 *F, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) F[i] = make_double2(f[i], 0.0);
}

struct SpecArgs {
    const double2 *F;   // transform of the field
    double2 *G;         // out: F * (M_a + i M_b)
    int n[3];
    double L[3];
    int kind;           // VT_TENSOR_*
    int ca, cb;         // components (0..5: xx, yy, zz, xy, xz, yz)
};

__device__ __forceinline__ double multiplier(const SpecArgs &A, int comp, const double k[3], const bool nyq[3],
                                             double k2, double inv_mean) {
    const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
    const int i = ia[comp], j = ib[comp];
    if (i != j && (nyq[i] || nyq[j])) return 0.0;
    const double kk = k[i] * k[j];
    if (A.kind == VT_TENSOR_TIDAL) return k2 > 0.0 ? kk / k2 * inv_mean : 0.0;
    return -kk;
}

__global__ void k_spectral(SpecArgs A) {
    const int64_t ntot = (int64_t)A.n[0] * A.n[1] * A.n[2];
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ntot) return;
    const int64_t m2 = e % A.n[2], m1 = (e / A.n[2]) % A.n[1], m0 = e / ((int64_t)A.n[1] * A.n[2]);
    const int64_t m[3] = {m0, m1, m2};
    double k[3];
    bool nyq[3];
    double k2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        const int64_t s = m[a] < A.n[a] / 2 ? m[a] : m[a] - A.n[a];
        nyq[a] = 2 * m[a] == A.n[a];
        k[a] = 2.0 * M_PI * (double)s / A.L[a];
        k2 += k[a] * k[a];
    }
    const double inv_mean = (double)ntot / A.F[0].x;
    const double ma = multiplier(A, A.ca, k, nyq, k2, inv_mean);
    const double mb = A.cb >= 0 ? multiplier(A, A.cb, k, nyq, k2, inv_mean) : 0.0;
    const double2 f = A.F[e];
    // (ma + i mb) f
    A.G[e] = make_double2(ma * f.x - mb * f.y, ma * f.y + mb * f.x);
}

__global__ void k_unpack(const double2 *G, double *oa, double *ob, int64_t n, double scale) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double2 g = G[i];
    oa[i] = g.x * scale;
    if (ob) ob[i] = g.y * scale;
}

static hipError_t fft3(double2 *d, const int n[3], double sign, hipStream_t s) {
    for (int axis = 2; axis >= 0; --axis) {
        const int N = n[axis];
        int logn = 0;
        while ((1 << logn) < N) ++logn;
        const int64_t nlines = ((int64_t)n[0] * n[1] * n[2]) / N;
        int B = N >= FFT_LDS ? 1 : FFT_LDS / N;
        if (B > nlines) B = (int)nlines;
        const size_t lds = sizeof(double2) * ((size_t)B * N + N / 2);
        hipError_t e = hipFuncSetAttribute((const void *)k_fft, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        k_fft<<<dim3((unsigned)(nlines / B)), dim3(FFT_TPB), lds, s>>>(d, n[0], n[1], n[2], axis, logn, B, sign);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// The transforms of one call: the grid's spectrum F and the work array G (ntot complex values
// each, both fully written before they are read).
static hipError_t grid_tensor_into(vt_ctx *c, const double *grid, int nx, int ny, int nz, int kind, double *out,
                                   double2 *F, double2 *G) {
    const int64_t ntot = (int64_t)nx * ny * nz;
    const int n[3] = {nx, ny, nz};
    const unsigned nb = (unsigned)((ntot + 255) / 256);
    k_real_to_complex<<<nb, 256, 0, c->stream>>>(grid, F, ntot);
    hipError_t e = fft3(F, n, -1.0, c->stream);
    if (e != hipSuccess) return e;
    SpecArgs a;
    a.F = F;
    a.G = G;
    for (int k = 0; k < 3; ++k) {
        a.n[k] = n[k];
        a.L[k] = c->h_items[0].L[k];
    }
    a.kind = kind;
    const double scale = 1.0 / (double)ntot;
    for (int p = 0; p < 3; ++p) {
        a.ca = 2 * p;
        a.cb = 2 * p + 1;
        k_spectral<<<nb, 256, 0, c->stream>>>(a);
        e = fft3(G, n, 1.0, c->stream);
        if (e != hipSuccess) return e;
        k_unpack<<<nb, 256, 0, c->stream>>>(G, out + a.ca * ntot, out + a.cb * ntot, ntot, scale);
    }
    return hipGetLastError();
}

hipError_t vt_launch_grid_tensor(vt_ctx *c, const double *grid, int nx, int ny, int nz, int kind, double *out) {
    const int64_t ntot = (int64_t)nx * ny * nz;
    if (c->cap_spec < ntot) {
        (void)hipFree(c->spec_buf);
        c->spec_buf = nullptr;
        c->cap_spec = 0;
        hipError_t e = hipMalloc(&c->spec_buf, sizeof(double2) * 2 * (size_t)ntot);
        if (e != hipSuccess) return e;
        c->cap_spec = ntot;
    }
    double2 *F = (double2 *)c->spec_buf;
    return grid_tensor_into(c, grid, nx, ny, nz, kind, out, F, F + ntot);
}

// ---------------------------------------------------------------- allocation-free variant
// Scratch for vt_grid_tensor_noalloc: the two complex work arrays of a grid of at most
// VT_NOALLOC_TENSOR_POINTS points (64 MiB), one copy per device, held until the process ends.
// In host code `scratch` names a host-side stand-in; kernels get the device address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) double2 scratch[2 * (size_t)VT_NOALLOC_TENSOR_POINTS];

#define VT_MAX_DEVICES 64
static void *g_scratch_ptr[VT_MAX_DEVICES];
static std::mutex g_scratch_mu;

// the calling thread's current device's copy of `scratch` (looked up once per device)
static hipError_t scratch_address(double2 **ptr) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= VT_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *ptr = (double2 *)g_scratch_ptr[dev];
    return hipSuccess;
}

hipError_t vt_launch_grid_tensor_noalloc(vt_ctx *c, const double *grid, int nx, int ny, int nz, int kind,
                                         double *out) {
    const int64_t ntot = (int64_t)nx * ny * nz;
    if (ntot > VT_NOALLOC_TENSOR_POINTS) return hipErrorInvalidValue;
    double2 *F = nullptr;
    hipError_t e = scratch_address(&F);
    if (e != hipSuccess) return e;
    return grid_tensor_into(c, grid, nx, ny, nz, kind, out, F, F + ntot);
}

void vt_spec_free(vt_ctx *c) {
    (void)hipFree(c->spec_buf);
    c->spec_buf = nullptr;
    c->cap_spec = 0;
}

// tune_kernels.hip -- small kernels used only by the autotuner and by the
// slice-count rule: a deterministic operand fill, |op(A)||op(B)| on the
// leading components, and the per-entry error ratio of two P-component
// results; and the throughput probes that measure the FP64 vector and INT8
// matrix-core peaks the GEMM kernels are compared with.
#pragma clang fp contract(off)

#include "internal.hpp"
#include "mp_arith.hpp"

namespace mpg {

__device__ __forceinline__ uint64_t mix64(uint64_t x) {
    // splitmix64 finaliser
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

__device__ __forceinline__ double unit_sym(uint64_t h) {
    // 53 random bits -> [-1, 1)
    return (double)(h >> 11) * 0x1.0p-52 - 1.0;
}

// P-component numbers with leading part in [-1, 1) and each further component
// below half an ulp of the one before (non-overlapping).
__global__ void fill_kernel(int P, double* X, int64_t plane, int64_t ps, uint64_t seed) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < plane; i += stride) {
        double prev = unit_sym(mix64(seed * 0x100000001B3ull + (uint64_t)i));
        X[i] = prev;
        for (int p = 1; p < P; ++p) {
            const double v = unit_sym(mix64((seed + p) * 0x9E3779B97F4A7C15ull ^ (uint64_t)i));
            const double half_ulp = prev == 0.0 ? 0.0 : ldexp(1.0, ilogb(prev) - 53);
            prev = half_ulp * v;
            X[p * ps + i] = prev;
        }
    }
}

int launch_fill(int P, double* X, int64_t plane, int64_t ps, uint64_t seed, hipStream_t st) {
    int64_t blocks = (plane + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, st, P, X, plane, ps, seed);
    return (int)hipGetLastError();
}

// out[i + j m] = sum_l |op(A)_il| |op(B)_lj| on leading components (binary64).
__global__ void absdot_kernel(GemmArgs g, double* out) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.m * g.n) return;
    const int64_t i = idx % g.m, j = idx / g.m;
    double acc = 0.0;
    for (int64_t l = 0; l < g.k; ++l) {
        const double a = g.ta ? g.A[l + i * g.lda] : g.A[i + l * g.lda];
        const double b = g.tb ? g.B[j + l * g.ldb] : g.B[l + j * g.ldb];
        acc = acc + fabs(a) * fabs(b);
    }
    out[idx] = acc;
}

int launch_absdot(const GemmArgs& g, double* out, hipStream_t st) {
    const int64_t blocks = (g.m * g.n + 255) / 256;
    hipLaunchKernelGGL(absdot_kernel, dim3((unsigned)blocks), dim3(256), 0, st, g, out);
    return (int)hipGetLastError();
}

template <int P>
__global__ void diff_ratio_kernel(int64_t m, int64_t n, const double* Cs, const double* Cr,
                                  int64_t ld, int64_t ps, const double* absab, double scale,
                                  double* out) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= m * n) return;
    const int64_t i = idx % m, j = idx / m;
    mp<P> a, b;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        a.c[p] = Cs[p * ps + i + j * ld];
        b.c[p] = -Cr[p * ps + i + j * ld];
    }
    const double d = fabs(add(a, b).c[0]);
    const double base = absab[idx];
    out[idx] = base > 0.0 ? d * scale / base : (d == 0.0 ? 0.0 : HUGE_VAL);
}

int launch_diff_ratio(int P, int64_t m, int64_t n, const double* Cs, const double* Cr, int64_t ld,
                      int64_t ps, const double* absab, double scale, double* out, hipStream_t st) {
    const int64_t blocks = (m * n + 255) / 256;
    const dim3 gr((unsigned)blocks), bl(256);
    if (P == 2) hipLaunchKernelGGL(diff_ratio_kernel<2>, gr, bl, 0, st, m, n, Cs, Cr, ld, ps, absab, scale, out);
    else if (P == 3) hipLaunchKernelGGL(diff_ratio_kernel<3>, gr, bl, 0, st, m, n, Cs, Cr, ld, ps, absab, scale, out);
    else hipLaunchKernelGGL(diff_ratio_kernel<4>, gr, bl, 0, st, m, n, Cs, Cr, ld, ps, absab, scale, out);
    return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Peak probes.  Each thread (FP64) or wave (MFMA) runs 8 or 4 independent
// chains so that issue, not latency, limits the rate; the results are summed
// into out[] only to keep the chains alive.
// ---------------------------------------------------------------------------

// OP 0: fma(x, b, c); 1: x + c; 2: x * b.  Values stay near 1 (no overflow,
// no subnormals).
template <int OP>
__global__ __launch_bounds__(256) void probe_fp64_kernel(double* out, int iters, double b, double c) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double x[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = 1.0 + 1e-3 * (double)((id + i) & 1023);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if (OP == 0) x[i] = __builtin_fma(x[i], b, c);
            else if (OP == 1) x[i] = x[i] + c;
            else x[i] = x[i] * b;
        }
        c = -c;      // keeps the add chains bounded
    }
    double sum = 0.0;
#pragma unroll
    for (int i = 0; i < 8; ++i) sum = sum + x[i];
    out[id] = sum;
}

typedef int v4i_t __attribute__((ext_vector_type(4)));
typedef int v16i_t __attribute__((ext_vector_type(16)));

__global__ __launch_bounds__(256) void probe_mfma_i8_kernel(double* out, int iters) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // non-zero bytes in both operands (the matrix cores do the full work)
    const int l = (int)threadIdx.x;
    const v4i_t a = {0x11223344 ^ l, 0x55667788 ^ (l << 8), 0x0f1e2d3c ^ (l << 16), 0x4b5a6978 ^ l};
    const v4i_t b = {0x13579bdf ^ (l << 4), 0x2468ace0 ^ l, 0x7f6e5d4c ^ (l << 12), 0x3b2a1908 ^ (l << 20)};
    v16i_t acc0 = v16i_t{0}, acc1 = v16i_t{0}, acc2 = v16i_t{0}, acc3 = v16i_t{0};
    for (int it = 0; it < iters; ++it) {
        acc0 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(b, a, acc1, 0, 0, 0);
        acc2 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, a, acc2, 0, 0, 0);
        acc3 = __builtin_amdgcn_mfma_i32_32x32x32_i8(b, b, acc3, 0, 0, 0);
    }
    double sum = 0.0;
#pragma unroll
    for (int v = 0; v < 16; ++v) sum = sum + (double)(acc0[v] ^ acc1[v] ^ acc2[v] ^ acc3[v]);
    out[id] = sum;
}

// Streaming copy dst[i] = src[i], i < n, with the non-temporal hints of the
// element-wise kernels: the HBM bandwidth such a stream reaches.
__global__ __launch_bounds__(256) void probe_copy_kernel(const double* __restrict__ src,
                                                          double* __restrict__ dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

int launch_probe_copy(const double* src, double* dst, int64_t n, double* bytes, hipStream_t st) {
    hipLaunchKernelGGL(probe_copy_kernel, dim3(16384), dim3(256), 0, st, src, dst, n);
    *bytes = 16.0 * (double)n;
    return (int)hipGetLastError();
}

// Launches probe `which` (0 FP64 FMA, 1 FP64 add, 2 FP64 mul, 3 INT8 MFMA
// 32x32x32) over `blocks` x 256 threads into out[blocks * 256]; *ops is the
// work of one launch (flops for FMA: 2 per FMA; operations otherwise).
int launch_probe(int which, double* out, int blocks, int iters, double* ops, hipStream_t st) {
    const double threads = (double)blocks * 256.0;
    switch (which) {
    case 0:
        hipLaunchKernelGGL(probe_fp64_kernel<0>, dim3(blocks), dim3(256), 0, st, out, iters, 0.999999, 1e-3);
        *ops = threads * iters * 8.0 * 2.0;
        break;
    case 1:
        hipLaunchKernelGGL(probe_fp64_kernel<1>, dim3(blocks), dim3(256), 0, st, out, iters, 0.999999, 1e-3);
        *ops = threads * iters * 8.0;
        break;
    case 2:
        hipLaunchKernelGGL(probe_fp64_kernel<2>, dim3(blocks), dim3(256), 0, st, out, iters, 0.999999, 1e-3);
        *ops = threads * iters * 8.0;
        break;
    default:
        hipLaunchKernelGGL(probe_mfma_i8_kernel, dim3(blocks), dim3(256), 0, st, out, iters);
        *ops = threads / 64.0 * iters * 4.0 * (32.0 * 32.0 * 32.0 * 2.0);
        break;
    }
    return (int)hipGetLastError();
}

}  // namespace mpg

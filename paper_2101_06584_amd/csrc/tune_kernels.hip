// tune_kernels.hip -- small kernels used only by the autotuner and by the
// slice-count rule: a deterministic operand fill, |op(A)||op(B)| on the
// leading components, and the per-entry error ratio of two P-component
// results.
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

}  // namespace mpg

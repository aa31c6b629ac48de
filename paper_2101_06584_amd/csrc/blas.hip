// blas.hip -- BLAS-1/2 in DD / TD / QD on component planes: axpy, a dot
// product in a fixed 64-ary tree order, and gemv (the GEMM with one column).
//
// axpy:  y_i = ADD(MUL(alpha, x_i), y_i); a stream, HBM-bound.
// dot:   the n products are taken in blocks of 64 consecutive terms, each
//        block summed from zero in ascending order; the block sums are again
//        taken 64 at a time and summed the same way until one value is left
//        (one kernel pass per level, partial sums in the caller's workspace).
//        The order is fixed, so the result is reproducible bit for bit; for
//        n <= 64 it is the sequential chain.
// gemv:  y = alpha op(A) x + beta y with one ascending chain per entry of y,
//        then the plain GEMM's epilogue: the same bits as the GEMM with a
//        single column.  The chains' multiplications are formed by other
//        waves of the workgroup (see gemv_chain_kernel), so a chain's lane
//        only adds.
#pragma clang fp contract(off)

#include "internal.hpp"
#include "mp_arith.hpp"

namespace mpg {

static constexpr int kDotFanin = 64;

struct Scal {
    double v[4];
};

template <int P>
__device__ __forceinline__ mp<P> scal(const Scal& s) {
    mp<P> r;
#pragma unroll
    for (int c = 0; c < P; ++c) r.c[c] = s.v[c];
    return r;
}

template <int P>
__global__ __launch_bounds__(256) void axpy_kernel(int64_t n, Scal alpha, const double* __restrict__ x,
                                                   int64_t sx, double* __restrict__ y, int64_t sy) {
    const mp<P> a = scal<P>(alpha);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        mp<P> xv, yv;
#pragma unroll
        for (int c = 0; c < P; ++c) {
            xv.c[c] = __builtin_nontemporal_load(x + c * sx + i);
            yv.c[c] = __builtin_nontemporal_load(y + c * sy + i);
        }
        const mp<P> r = add(mul(a, xv), yv);
#pragma unroll
        for (int c = 0; c < P; ++c) __builtin_nontemporal_store(r.c[c], y + c * sy + i);
    }
}

// Leaf level: out[b] (P doubles, node-major) = ascending sum of the products
// x_i y_i, i in [64 b, min(64 b + 64, n)).  Each wave owns 32 consecutive
// blocks (lane L < 32 sums block b0 + L).  Per round of 16 positions, the
// whole wave forms the 512 products of the round from coalesced 128-byte
// runs (16 lanes per block: full cache lines) into LDS, then every lane
// L < 32 adds its block's 16 products in order.  The products and the order
// of the sum are those of the plain sequential loop.
static constexpr int kDotRound = 16;
static constexpr int kDotBlocks = 32;             // blocks per wave

template <int P>
__global__ __launch_bounds__(256) void dot_leaf_kernel(int64_t n, const double* __restrict__ x, int64_t sx,
                                                       const double* __restrict__ y, int64_t sy,
                                                       double* __restrict__ out, int64_t cnt) {
    // per wave: [32 blocks][kDotRound + 1 (pad)][P]
    __shared__ double prod[4][kDotBlocks * (kDotRound + 1) * P];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double* pw = prod[wave];
    const int64_t b0 = ((int64_t)blockIdx.x * 4 + wave) * kDotBlocks;   // first block of this wave
    if (b0 >= cnt) return;                                                // whole wave past the end
    const int64_t b = b0 + lane;                                          // summed by lanes < 32
    mp<P> acc = mp_zero<P>();
    for (int j0 = 0; j0 < kDotFanin; j0 += kDotRound) {
        // products: lane handles (block b0 + 4 q + lane / 16, position j0 + lane % 16), q = 0..7
        // loads first (indices past the end read element n - 1 and their
        // products are never summed), then the products
        mp<P> xv[8], yv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int bl = 4 * q + (lane >> 4), pos = lane & 15;
            const int64_t i = min((b0 + bl) * kDotFanin + j0 + pos, n - 1);
#pragma unroll
            for (int c = 0; c < P; ++c) {
                xv[q].c[c] = x[c * sx + i];
                yv[q].c[c] = y[c * sy + i];
            }
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int bl = 4 * q + (lane >> 4), pos = lane & 15;
            const mp<P> pr = mul(xv[q], yv[q]);
#pragma unroll
            for (int c = 0; c < P; ++c) pw[(bl * (kDotRound + 1) + pos) * P + c] = pr.c[c];
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        // sums: this lane's block, positions j0 .. j0 + 15 that exist
        if (lane < kDotBlocks) {
#pragma unroll
            for (int pos = 0; pos < kDotRound; ++pos) {
                const int64_t i = b * kDotFanin + j0 + pos;
                if (b < cnt && i < n) {
                    mp<P> v;
#pragma unroll
                    for (int c = 0; c < P; ++c) v.c[c] = pw[(lane * (kDotRound + 1) + pos) * P + c];
                    acc = add(acc, v);
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    }
    if (lane < kDotBlocks && b < cnt) {
#pragma unroll
        for (int c = 0; c < P; ++c) out[b * P + c] = acc.c[c];
    }
}

// Higher levels: out[b] = ascending sum of in[64 b .. min(64 b + 64, cnt_in)).
template <int P>
__global__ __launch_bounds__(256) void dot_node_kernel(int64_t cnt_in, const double* __restrict__ in,
                                                       double* __restrict__ out, int64_t cnt) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= cnt) return;
    mp<P> acc = mp_zero<P>();
    const int64_t i0 = b * kDotFanin, i1 = min(cnt_in, i0 + kDotFanin);
    for (int64_t i = i0; i < i1; ++i) {
        mp<P> v;
#pragma unroll
        for (int c = 0; c < P; ++c) v.c[c] = in[i * P + c];
        acc = add(acc, v);
    }
#pragma unroll
    for (int c = 0; c < P; ++c) out[b * P + c] = acc.c[c];
}

template <int P>
__global__ void dot_zero_kernel(double* out) {
    if (threadIdx.x < P) out[threadIdx.x] = 0.0;
}

// y = alpha op(A) x + beta y over `rows` entries; element (i, l) of op(A) at
// A[t ? l + i lda : i + l lda] (component planes at sa).  az: alpha == 0 or
// inner == 0 (then y = beta y, or 0 when beta == 0).
template <int P>
__global__ __launch_bounds__(256) void gemv_kernel(int64_t rows, int64_t inner, int t, Scal alpha,
                                                   const double* __restrict__ A, int64_t lda, int64_t sa,
                                                   const double* __restrict__ x, int64_t sx, Scal beta,
                                                   double* __restrict__ y, int64_t sy, int az) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    const mp<P> al = scal<P>(alpha), be = scal<P>(beta);
    const bool beta_zero = mp_is_zero(be);
    mp<P> r;
    if (az) {
        r = mp_zero<P>();
        if (!beta_zero) {
            mp<P> yo;
#pragma unroll
            for (int c = 0; c < P; ++c) yo.c[c] = y[c * sy + i];
            r = mul(be, yo);
        }
    } else {
        // the chain is sequential, so the loads of 8 steps are issued first
        // to overlap their latency (one thread per row leaves few waves)
        constexpr int UN = 8;
        mp<P> acc = mp_zero<P>();
        int64_t l = 0;
        for (; l + UN <= inner; l += UN) {
            mp<P> a[UN], b[UN];
#pragma unroll
            for (int u = 0; u < UN; ++u) {
                const int64_t off = t ? (l + u) + i * lda : i + (l + u) * lda;
#pragma unroll
                for (int c = 0; c < P; ++c) {
                    a[u].c[c] = A[c * sa + off];
                    b[u].c[c] = x[c * sx + l + u];
                }
            }
#pragma unroll
            for (int u = 0; u < UN; ++u) acc = add(acc, mul(a[u], b[u]));
        }
        for (; l < inner; ++l) {
            const int64_t off = t ? l + i * lda : i + l * lda;
            mp<P> a, b;
#pragma unroll
            for (int c = 0; c < P; ++c) {
                a.c[c] = A[c * sa + off];
                b.c[c] = x[c * sx + l];
            }
            acc = add(acc, mul(a, b));
        }
        r = mul(al, acc);
        if (!beta_zero) {
            mp<P> yo;
#pragma unroll
            for (int c = 0; c < P; ++c) yo.c[c] = y[c * sy + i];
            r = add(r, mul(be, yo));
        }
    }
#pragma unroll
    for (int c = 0; c < P; ++c) y[c * sy + i] = r.c[c];
}

// gemv with the products off the chains.  A workgroup owns 64 entries of y:
// wave 0 runs their 64 chains and only adds; waves 1-3 form the products of
// the next block of LB steps (64 x LB of them, 64 LB / 192 per thread) into
// LDS.  Blocks alternate between two buffers with one barrier per block: the
// chain wave adds block b - 1 while the others multiply block b, having
// loaded its operands into registers before the previous barrier, so the
// loads overlap the additions.  Lanes of the product waves run along
// whichever index of op(A) is contiguous.  LB is larger for the cheaper
// additions (DD 48, TD 36, QD 24), the LDS buffers 100-112 KiB.
template <int P>
struct GemvCfg {
    static constexpr int LB = P == 2 ? 48 : P == 3 ? 36 : 24;
    static constexpr int PER = 64 * LB / 192;          // products per producer thread
    static_assert(64 * LB % 192 == 0, "whole products per thread");
};
constexpr int kGemvRowPad = 65;          // 64 rows + 1: spreads the 'T' writes over banks

template <int P>
__global__ __launch_bounds__(256) void gemv_chain_kernel(int64_t rows, int64_t inner, int t, Scal alpha,
                                                         const double* __restrict__ A, int64_t lda,
                                                         int64_t sa, const double* __restrict__ x,
                                                         int64_t sx, Scal beta, double* __restrict__ y,
                                                         int64_t sy) {
    constexpr int LB = GemvCfg<P>::LB, PER = GemvCfg<P>::PER;
    __shared__ double prod[2][LB][P][kGemvRowPad];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    const int64_t nblk = (inner + LB - 1) / LB;
    const int pt = tid - 64;                              // producer thread 0..191
    // operands of the producer's next block, loaded a block ahead
    double av[PER][P], xv[PER][P];
    auto load_block = [&](int64_t b) __attribute__((always_inline)) {
        const int64_t l0 = b * LB;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int idx = pt + 192 * j;
            const int r = t ? idx / LB : (idx & 63);
            const int lb = t ? idx % LB : (idx >> 6);
            const int64_t i = i0 + r, l = l0 + lb;
            const bool ok = i < rows && l < inner;
            const int64_t off = t ? l + i * lda : i + l * lda;
#pragma unroll
            for (int c = 0; c < P; ++c) {
                av[j][c] = ok ? A[c * sa + off] : 0.0;
                xv[j][c] = ok ? x[c * sx + l] : 0.0;
            }
        }
    };
    if (wave > 0 && nblk > 0) load_block(0);
    mp<P> acc = mp_zero<P>();
    for (int64_t b = 0; b <= nblk; ++b) {
        if (wave > 0) {
            if (b < nblk) {
#pragma unroll
                for (int j = 0; j < PER; ++j) {
                    const int idx = pt + 192 * j;
                    const int r = t ? idx / LB : (idx & 63);
                    const int lb = t ? idx % LB : (idx >> 6);
                    mp<P> a, xx;
#pragma unroll
                    for (int c = 0; c < P; ++c) {
                        a.c[c] = av[j][c];
                        xx.c[c] = xv[j][c];
                    }
                    const mp<P> p = mul(a, xx);
#pragma unroll
                    for (int c = 0; c < P; ++c) prod[b & 1][lb][c][r] = p.c[c];
                }
                if (b + 1 < nblk) load_block(b + 1);
            }
        } else if (b > 0) {
            const int64_t l0 = (b - 1) * LB;
            const int cnt = (int)((inner - l0) < LB ? (inner - l0) : LB);
            for (int lb = 0; lb < cnt; ++lb) {
                mp<P> p;
#pragma unroll
                for (int c = 0; c < P; ++c) p.c[c] = prod[(b - 1) & 1][lb][c][lane];
                acc = add(acc, p);
            }
        }
        __syncthreads();
    }
    const int64_t i = i0 + lane;
    if (wave != 0 || i >= rows) return;
    const mp<P> al = scal<P>(alpha), be = scal<P>(beta);
    mp<P> r = mul(al, acc);
    if (!mp_is_zero(be)) {
        mp<P> yo;
#pragma unroll
        for (int c = 0; c < P; ++c) yo.c[c] = y[c * sy + i];
        r = add(r, mul(be, yo));
    }
#pragma unroll
    for (int c = 0; c < P; ++c) y[c * sy + i] = r.c[c];
}

static Scal to_scal(int P, const double* v) {
    Scal s{};
    for (int c = 0; c < P; ++c) s.v[c] = v[c];
    return s;
}

int launch_axpy(int P, int64_t n, const double* alpha, const double* x, int64_t sx, double* y, int64_t sy,
                hipStream_t st) {
    if (n <= 0) return 0;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 256 * 64) blocks = 256 * 64;
    const dim3 gr((unsigned)blocks), bl(256);
    const Scal a = to_scal(P, alpha);
    if (P == 2) hipLaunchKernelGGL(axpy_kernel<2>, gr, bl, 0, st, n, a, x, sx, y, sy);
    else if (P == 3) hipLaunchKernelGGL(axpy_kernel<3>, gr, bl, 0, st, n, a, x, sx, y, sy);
    else hipLaunchKernelGGL(axpy_kernel<4>, gr, bl, 0, st, n, a, x, sx, y, sy);
    return (int)hipGetLastError();
}

size_t dot_workspace_bytes(int P, int64_t n) {
    // every level's partial sums, node-major
    size_t d = 0;
    for (int64_t cnt = (n + kDotFanin - 1) / kDotFanin; cnt > 1; cnt = (cnt + kDotFanin - 1) / kDotFanin)
        d += (size_t)cnt * P;
    return d * 8;
}

template <int P>
static int dot_t(int64_t n, const double* x, int64_t sx, const double* y, int64_t sy, double* result,
                 double* ws, hipStream_t st) {
    if (n <= 0) {
        hipLaunchKernelGGL(dot_zero_kernel<P>, dim3(1), dim3(64), 0, st, result);
        return (int)hipGetLastError();
    }
    int64_t cnt = (n + kDotFanin - 1) / kDotFanin;
    double* out = cnt == 1 ? result : ws;
    // 4 waves of 32 blocks per workgroup
    const int64_t per_wg = 4 * kDotBlocks;
    if ((cnt + per_wg - 1) / per_wg > 0x7fffffffLL) return (int)hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(dot_leaf_kernel<P>, dim3((unsigned)((cnt + per_wg - 1) / per_wg)), dim3(256), 0, st, n,
                       x, sx, y, sy, out, cnt);
    double* in = out;
    double* free_at = ws + cnt * P;
    while (cnt > 1) {
        const int64_t next = (cnt + kDotFanin - 1) / kDotFanin;
        double* dst = next == 1 ? result : free_at;
        hipLaunchKernelGGL(dot_node_kernel<P>, dim3((unsigned)((next + 255) / 256)), dim3(256), 0, st, cnt,
                           (const double*)in, dst, next);
        in = dst;
        free_at += next * P;
        cnt = next;
    }
    return (int)hipGetLastError();
}

int launch_dot(int P, int64_t n, const double* x, int64_t sx, const double* y, int64_t sy, double* result,
               void* ws, hipStream_t st) {
    if (P == 2) return dot_t<2>(n, x, sx, y, sy, result, (double*)ws, st);
    if (P == 3) return dot_t<3>(n, x, sx, y, sy, result, (double*)ws, st);
    return dot_t<4>(n, x, sx, y, sy, result, (double*)ws, st);
}

int launch_gemv(int P, int t, int64_t rows, int64_t inner, const double* alpha, const double* A, int64_t lda,
                int64_t sa, const double* x, int64_t sx, const double* beta, double* y, int64_t sy, int az,
                hipStream_t st) {
    if (rows <= 0) return 0;
    const Scal al = to_scal(P, alpha), be = to_scal(P, beta);
    if (!az) {                                 // the chains with their products formed alongside
        const int64_t wgs = (rows + 63) / 64;
        if (wgs > 0x7fffffffLL) return (int)hipErrorInvalidConfiguration;
        const dim3 gr((unsigned)wgs), bl(256);
        if (P == 2) hipLaunchKernelGGL(gemv_chain_kernel<2>, gr, bl, 0, st, rows, inner, t, al, A, lda, sa, x, sx, be, y, sy);
        else if (P == 3) hipLaunchKernelGGL(gemv_chain_kernel<3>, gr, bl, 0, st, rows, inner, t, al, A, lda, sa, x, sx, be, y, sy);
        else hipLaunchKernelGGL(gemv_chain_kernel<4>, gr, bl, 0, st, rows, inner, t, al, A, lda, sa, x, sx, be, y, sy);
        return (int)hipGetLastError();
    }
    const int64_t blocks = (rows + 255) / 256;
    if (blocks > 0x7fffffffLL) return (int)hipErrorInvalidConfiguration;
    const dim3 gr((unsigned)blocks), bl(256);
    if (P == 2) hipLaunchKernelGGL(gemv_kernel<2>, gr, bl, 0, st, rows, inner, t, al, A, lda, sa, x, sx, be, y, sy, az);
    else if (P == 3) hipLaunchKernelGGL(gemv_kernel<3>, gr, bl, 0, st, rows, inner, t, al, A, lda, sa, x, sx, be, y, sy, az);
    else hipLaunchKernelGGL(gemv_kernel<4>, gr, bl, 0, st, rows, inner, t, al, A, lda, sa, x, sx, be, y, sy, az);
    return (int)hipGetLastError();
}

}  // namespace mpg

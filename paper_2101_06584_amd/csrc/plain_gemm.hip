// plain_gemm.hip -- FP64-VALU error-free-transformation GEMM for gfx950:
// C = alpha op(A) op(B) + beta C in DD / TD / QD on component planes.
//
// Method: eqn (1) of Sec. 3 with the DD/TD/QD additions and multiplications of
// Algorithms 1-6.  Each output entry keeps one running P-component sum over
// k in ascending order, so the result is bitwise independent of the tiling
// (the paper's blocking with n_min = 32 likewise leaves each entry's chain
// intact).  Tiles of op(A) and op(B) are staged through LDS one component
// plane at a time; every thread owns a TM x TN block of P-component
// accumulators.
//
// Also here: the element-wise vector kernels (Sec. 2.5's DD/TD/QD vector add
// and multiply), the alpha == 0 / k == 0 scaling kernel and the persistent
// batched kernel that reuses the same tile routine.
#pragma clang fp contract(off)

#include "internal.hpp"
#include "mp_arith.hpp"
#include "tile_order.hpp"

namespace mpg {

// ---------------------------------------------------------------------------
// Tile routine
// ---------------------------------------------------------------------------

template <int P, int TX, int TY, int TM, int TN, int BK, int V = 0>
struct PlainTile {
    static constexpr int BM = TX * TM;
    static constexpr int BN = TY * TN;
    static constexpr int NT = TX * TY;
    static constexpr int LDS_DOUBLES = P * BK * (BM + BN);

    // Stage the k-tile [k0, k0 + BK) of op(A) rows [m0, m0 + BM) and op(B)
    // columns [n0, n0 + BN) into LDS, zero-filling outside the matrices.
    __device__ static void stage(const GemmArgs& g, int64_t m0, int64_t n0, int64_t k0,
                                 double* As, double* Bs) {
        const int tid = threadIdx.x;
        for (int idx = tid; idx < BM * BK; idx += NT) {
            int i, l;
            if (!g.ta) { i = idx % BM; l = idx / BM; }
            else       { l = idx % BK; i = idx / BK; }
            const int64_t gi = m0 + i, gl = k0 + l;
            const bool ok = (gi < g.m) && (gl < g.k);
            const int64_t off = g.ta ? (gl + gi * g.lda) : (gi + gl * g.lda);
#pragma unroll
            for (int p = 0; p < P; ++p)
                As[(p * BK + l) * BM + i] = ok ? g.A[p * g.sa + off] : 0.0;
        }
        for (int idx = tid; idx < BN * BK; idx += NT) {
            int j, l;
            if (g.tb) { j = idx % BN; l = idx / BN; }
            else      { l = idx % BK; j = idx / BK; }
            const int64_t gj = n0 + j, gl = k0 + l;
            const bool ok = (gj < g.n) && (gl < g.k);
            const int64_t off = g.tb ? (gj + gl * g.ldb) : (gl + gj * g.ldb);
#pragma unroll
            for (int p = 0; p < P; ++p)
                Bs[(p * BK + l) * BN + j] = ok ? g.B[p * g.sb + off] : 0.0;
        }
    }

    // Rows rb + r RS (r < TM) and columns cb + c CS (c < TN) of the tile.
    template <int RS, int CS>
    __device__ static void step(const double* As, const double* Bs, int kk, int rb, int cb,
                                mp<P> (&acc)[TM][TN]) {
        mp<P> a[TM], b[TN];
#pragma unroll
        for (int r = 0; r < TM; ++r)
#pragma unroll
            for (int p = 0; p < P; ++p) a[r].c[p] = As[(p * BK + kk) * BM + rb + r * RS];
#pragma unroll
        for (int c = 0; c < TN; ++c)
#pragma unroll
            for (int p = 0; p < P; ++p) b[c].c[p] = Bs[(p * BK + kk) * BN + cb + c * CS];
        tile_mac_v<V, TM, TN>(acc, a, b);
    }

    // Thread-to-entry maps.  The default interleaves a thread's TM rows TX
    // apart and its TN columns TY apart.  The wave-quadrant map (16 x 16
    // threads, four waves) gives each wave one quadrant of the tile, its 64
    // lanes as 8 x 8 with TM rows and TN columns 8 apart; on a tile that
    // overhangs the matrix a wave whose quadrant lies wholly outside it skips
    // the k loop.  Either way each entry keeps its own ascending chain.
    static constexpr bool kQuadOk = (TX == 16 && TY == 16);

    template <bool QUAD = false>
    __device__ static void run(const GemmArgs& g, const mp<P>& alpha, const mp<P>& beta,
                               int64_t m0, int64_t n0, double* lds) {
        constexpr bool Q = QUAD && kQuadOk;
        constexpr int RS = Q ? 8 : TX, CS = Q ? 8 : TY;
        double* As = lds;
        double* Bs = lds + P * BK * BM;
        const int tid = threadIdx.x;
        int rb, cb;
        bool busy = true;   // this wave has entries inside the matrix
        if constexpr (Q) {
            const int w = tid >> 6, lane = tid & 63;
            const int qr = (w & 1) * (BM / 2), qc = (w >> 1) * (BN / 2);
            rb = qr + (lane & 7);
            cb = qc + (lane >> 3);
            busy = (m0 + qr < g.m) && (n0 + qc < g.n);
        } else {
            rb = tid % TX;
            cb = tid / TX;
        }
        mp<P> acc[TM][TN];
#pragma unroll
        for (int r = 0; r < TM; ++r)
#pragma unroll
            for (int c = 0; c < TN; ++c) acc[r][c] = mp_zero<P>();

        // alpha == 0 or k == 0: C = beta C (0 when beta == 0); nothing at all
        // when additionally beta == 1
        const bool az = (g.k == 0) || mp_is_zero(alpha);
        const bool beta_zero = mp_is_zero(beta);
        bool beta_one = beta.c[0] == 1.0;
#pragma unroll
        for (int p = 1; p < P; ++p) beta_one = beta_one && (beta.c[p] == 0.0);
        if (az && beta_one) return;

        const int64_t kend = az ? 0 : g.k;
        for (int64_t k0 = 0; k0 < kend; k0 += BK) {
            stage(g, m0, n0, k0, As, Bs);
            __syncthreads();
            const int64_t rem = g.k - k0;
            if (busy && rem >= BK) {
#pragma unroll 2
                for (int kk = 0; kk < BK; ++kk) step<RS, CS>(As, Bs, kk, rb, cb, acc);
            } else if (busy) {
                const int kb = (int)rem;
                for (int kk = 0; kk < kb; ++kk) step<RS, CS>(As, Bs, kk, rb, cb, acc);
            }
            __syncthreads();
        }

#pragma unroll
        for (int r = 0; r < TM; ++r)
#pragma unroll
            for (int c = 0; c < TN; ++c) {
                const int64_t i = m0 + rb + r * RS, j = n0 + cb + c * CS;
                if (i < g.m && j < g.n) {
                    const int64_t off = i + j * g.ldc;
                    mp<P> t;
                    if (az) {
                        t = mp_zero<P>();
                        if (!beta_zero) {
                            mp<P> co;
#pragma unroll
                            for (int p = 0; p < P; ++p) co.c[p] = g.C[p * g.sc + off];
                            t = mul_v<V>(beta, co);
                        }
                    } else {
                        t = mul_v<V>(alpha, acc[r][c]);
                        if (!beta_zero) {
                            mp<P> co;
#pragma unroll
                            for (int p = 0; p < P; ++p) co.c[p] = g.C[p * g.sc + off];
                            t = add_v<V>(t, mul_v<V>(beta, co));
                        }
                    }
#pragma unroll
                    for (int p = 0; p < P; ++p) g.C[p * g.sc + off] = t.c[p];
                }
            }
    }
};

template <int P>
__device__ __forceinline__ mp<P> load_scalar(const double* v) {
    mp<P> r;
#pragma unroll
    for (int p = 0; p < P; ++p) r.c[p] = v[p];
    return r;
}

// Waves per SIMD that a tile's register budget is held to (1: no bound).
// The DD 64 x 64 tile takes 180 registers unbounded, which leaves two waves
// per SIMD; at 168 a third wave hides the LDS reads and the staging.
template <int P, int TM, int TN>
constexpr int plain_waves_per_eu() { return (P == 2 && TM * TN >= 16) ? 3 : 1; }

template <int P, int TX, int TY, int TM, int TN, int BK, int V = 0>
__global__ __launch_bounds__(TX * TY) __attribute__((amdgpu_waves_per_eu(plain_waves_per_eu<P, TM, TN>())))
void plain_gemm_kernel(GemmArgs g) {
    using T = PlainTile<P, TX, TY, TM, TN, BK, V>;
    __shared__ double lds[T::LDS_DOUBLES];
    int64_t tm, tn;
    if (!xcd_tile_coords<8>(blockIdx.x, (g.m + T::BM - 1) / T::BM, (g.n + T::BN - 1) / T::BN, tm, tn))
        return;
    const mp<P> alpha = load_scalar<P>(g.alpha);
    const mp<P> beta = load_scalar<P>(g.beta);
    T::run(g, alpha, beta, tm * T::BM, tn * T::BN, lds);
}

// Strided batch of equal-shape products (Strassen's leaves): problem z =
// blockIdx.y uses A + z zA, B + z zB, C + z zC; alpha and beta from g.
template <int P, int TX, int TY, int TM, int TN, int BK>
__global__ __launch_bounds__(TX * TY) __attribute__((amdgpu_waves_per_eu(plain_waves_per_eu<P, TM, TN>())))
void plain_gemm_strided_kernel(GemmArgs g, int64_t zA, int64_t zB, int64_t zC) {
    using T = PlainTile<P, TX, TY, TM, TN, BK>;
    __shared__ double lds[T::LDS_DOUBLES];
    int64_t tm, tn;
    if (!xcd_tile_coords<8>(blockIdx.x, (g.m + T::BM - 1) / T::BM, (g.n + T::BN - 1) / T::BN, tm, tn))
        return;
    const int64_t z = blockIdx.y;
    g.A += z * zA;
    g.B += z * zB;
    g.C += z * zC;
    const mp<P> alpha = load_scalar<P>(g.alpha);
    const mp<P> beta = load_scalar<P>(g.beta);
    T::run(g, alpha, beta, tm * T::BM, tn * T::BN, lds);
}

// ---------------------------------------------------------------------------
// Persistent batched kernel: one launch, many GEMMs, a global tile queue.
// ---------------------------------------------------------------------------

struct BatchDesc {
    GemmArgs g;
    int64_t tile_begin;    // first global tile index of this problem
    int64_t tiles_m;       // tiles along m
};

template <int P, int TX, int TY, int TM, int TN, int BK>
__global__ __launch_bounds__(TX * TY) void batch_gemm_kernel(const BatchDesc* __restrict__ desc, int64_t count,
                                                             int64_t total_tiles, unsigned* counter) {
    using T = PlainTile<P, TX, TY, TM, TN, BK>;
    __shared__ double lds[T::LDS_DOUBLES];
    __shared__ int64_t s_tile;
    for (;;) {
        if (threadIdx.x == 0) s_tile = (int64_t)atomicAdd(counter, 1u);
        __syncthreads();
        const int64_t t = s_tile;
        __syncthreads();
        if (t >= total_tiles) break;   // every wave of the block sees the same t
        // last problem whose tile_begin <= t
        int64_t lo = 0, hi = count - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (desc[mid].tile_begin <= t) lo = mid; else hi = mid - 1;
        }
        const BatchDesc& d = desc[lo];
        const int64_t local = t - d.tile_begin;
        const int64_t tm = local % d.tiles_m, tn = local / d.tiles_m;
        const mp<P> alpha = load_scalar<P>(d.g.alpha);
        const mp<P> beta = load_scalar<P>(d.g.beta);
        T::template run<true>(d.g, alpha, beta, tm * T::BM, tn * T::BN, lds);
    }
}

__global__ void reset_counter_kernel(unsigned* counter) { *counter = 0u; }

// ---------------------------------------------------------------------------
// alpha == 0 or k == 0: C = beta C, or 0 when beta == 0 (C then not read).
// ---------------------------------------------------------------------------

template <int P, int V = 0>
__global__ void scale_kernel(GemmArgs g) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.m * g.n) return;
    const int64_t i = idx % g.m, j = idx / g.m;
    const int64_t off = i + j * g.ldc;
    const mp<P> beta = load_scalar<P>(g.beta);
    mp<P> t = mp_zero<P>();
    if (!mp_is_zero(beta)) {
        mp<P> co;
#pragma unroll
        for (int p = 0; p < P; ++p) co.c[p] = g.C[p * g.sc + off];
        t = mul_v<V>(beta, co);
    }
#pragma unroll
    for (int p = 0; p < P; ++p) g.C[p * g.sc + off] = t.c[p];
}

// ---------------------------------------------------------------------------
// Element-wise r = x + y or x * y over component planes (Sec. 2.5).
// ---------------------------------------------------------------------------

template <int P, int OP>
__global__ void vec_kernel(int64_t n, const double* __restrict__ x, int64_t sx,
                           const double* __restrict__ y, int64_t sy, double* __restrict__ r,
                           int64_t sr) {
    // a pure stream: every byte is used once, so loads and stores carry the
    // non-temporal hint (keeps the caches for other work, and measured a few
    // percent faster than plain accesses)
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        mp<P> a, b;
#pragma unroll
        for (int p = 0; p < P; ++p) {
            a.c[p] = __builtin_nontemporal_load(x + p * sx + i);
            b.c[p] = __builtin_nontemporal_load(y + p * sy + i);
        }
        mp<P> o;
        if constexpr (OP == 0) o = add(a, b);
        else if constexpr (OP == 1) o = mul(a, b);
        else if constexpr (OP == 2) o = add_v<1>(a, b);    // TD only: Algorithm 3
        else o = mul_v<2>(a, b);                           // TD only: TDmulq
#pragma unroll
        for (int p = 0; p < P; ++p) __builtin_nontemporal_store(o.c[p], r + p * sr + i);
    }
}

// ---------------------------------------------------------------------------
// Configuration table and launchers.
// ---------------------------------------------------------------------------

// Tile configurations (P, id, TX, TY, TM, TN, BK); the single list below
// generates the config table and both dispatch switches.
#define MPG_PLAIN_LIST(X)          \
    X(2, 0, 16, 16, 4, 4, 16)      \
    X(2, 1, 16, 16, 2, 2, 16)      \
    X(2, 2, 16, 16, 4, 2, 16)      \
    X(2, 3, 16, 8, 4, 4, 16)       \
    X(3, 0, 16, 16, 2, 2, 16)      \
    X(3, 1, 16, 16, 4, 2, 16)      \
    X(3, 2, 16, 16, 1, 2, 16)      \
    X(3, 3, 16, 16, 1, 1, 16)      \
    X(4, 0, 16, 16, 2, 2, 16)      \
    X(4, 1, 16, 16, 1, 2, 16)      \
    X(4, 2, 16, 16, 2, 1, 16)      \
    X(4, 3, 16, 16, 1, 1, 16)

PlainConfig plain_config(int P, int id) {
#define MPG_CFG(PP, ID, TX, TY, TM, TN, BK) \
    if (P == PP && id == ID) return PlainConfig{TX, TY, TM, TN, BK};
    MPG_PLAIN_LIST(MPG_CFG)
#undef MPG_CFG
    return PlainConfig{0, 0, 0, 0, 0};
}

uint32_t fnv1a(uint32_t h, int v) {
    for (int b = 0; b < 4; ++b) {
        h ^= (uint32_t)(v >> (8 * b)) & 255u;
        h *= 16777619u;
    }
    return h;
}

uint32_t plain_config_signature(int P) {
    uint32_t h = 2166136261u;
    for (int id = 0; id < kPlainConfigs; ++id) {
        const PlainConfig c = plain_config(P, id);
        for (int v : {c.tx, c.ty, c.tm, c.tn, c.bk}) h = fnv1a(h, v);
    }
    return h;
}

int plain_default_config(int P, int64_t m, int64_t n, int64_t k) {
    (void)k;
    // small problems: smaller tiles so the grid still covers the 256 CUs
    const int64_t mn = m * n;
    if (P == 2) return mn >= (int64_t)1536 * 1536 ? 0 : 1;
    if (P == 3) return mn >= (int64_t)1024 * 1024 ? 0 : 2;
    return mn >= (int64_t)1024 * 1024 ? 0 : 1;
}

template <int P, int TX, int TY, int TM, int TN, int BK, int V = 0>
static int launch_plain_t(const GemmArgs& g, hipStream_t st) {
    using T = PlainTile<P, TX, TY, TM, TN, BK, V>;
    const int64_t grid = xcd_grid(((g.m + T::BM - 1) / T::BM) * ((g.n + T::BN - 1) / T::BN));
    if (grid > 0x7fffffffLL) return (int)hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((plain_gemm_kernel<P, TX, TY, TM, TN, BK, V>), dim3((unsigned)grid), dim3(T::NT),
                       0, st, g);
    return (int)hipGetLastError();
}

template <int P, int TX, int TY, int TM, int TN, int BK>
static int launch_batch_t(int64_t count, int64_t total, const void* desc, unsigned* counter,
                          int grid, hipStream_t st) {
    using T = PlainTile<P, TX, TY, TM, TN, BK>;
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, st, counter);
    hipLaunchKernelGGL((batch_gemm_kernel<P, TX, TY, TM, TN, BK>), dim3(grid), dim3(T::NT), 0, st,
                       (const BatchDesc*)desc, count, total, counter);
    return (int)hipGetLastError();
}

template <int P, int TX, int TY, int TM, int TN, int BK>
static int launch_plain_strided_t(const GemmArgs& g, int64_t batch, int64_t zA, int64_t zB, int64_t zC,
                                  hipStream_t st) {
    using T = PlainTile<P, TX, TY, TM, TN, BK>;
    const int64_t grid = xcd_grid(((g.m + T::BM - 1) / T::BM) * ((g.n + T::BN - 1) / T::BN));
    if (grid > 0x7fffffffLL || batch > 65535) return (int)hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((plain_gemm_strided_kernel<P, TX, TY, TM, TN, BK>),
                       dim3((unsigned)grid, (unsigned)batch), dim3(T::NT), 0, st, g, zA, zB, zC);
    return (int)hipGetLastError();
}

int launch_plain_strided(int P, int cfg, const GemmArgs& g, int64_t batch, int64_t zA, int64_t zB,
                         int64_t zC, hipStream_t st) {
#define MPG_CASE(PP, ID, TX, TY, TM, TN, BK) \
    if (P == PP && cfg == ID) return launch_plain_strided_t<PP, TX, TY, TM, TN, BK>(g, batch, zA, zB, zC, st);
    MPG_PLAIN_LIST(MPG_CASE)
#undef MPG_CASE
    return (int)hipErrorInvalidValue;
}

int launch_plain(int P, int cfg, const GemmArgs& g, hipStream_t st) {
#define MPG_CASE(PP, ID, TX, TY, TM, TN, BK) \
    if (P == PP && cfg == ID) return launch_plain_t<PP, TX, TY, TM, TN, BK>(g, st);
    MPG_PLAIN_LIST(MPG_CASE)
#undef MPG_CASE
    return (int)hipErrorInvalidValue;
}

int launch_batch(int P, int cfg, int64_t count, int64_t total_tiles, const void* desc,
                 unsigned* counter, int grid, hipStream_t st) {
#define MPG_CASE(PP, ID, TX, TY, TM, TN, BK)                                                \
    if (P == PP && cfg == ID)                                                               \
        return launch_batch_t<PP, TX, TY, TM, TN, BK>(count, total_tiles, desc, counter, grid, st);
    MPG_PLAIN_LIST(MPG_CASE)
#undef MPG_CASE
    return (int)hipErrorInvalidValue;
}

int batch_max_grid(int P, int cfg) {
    // enough resident workgroups to cover every CU a few times over; blocks
    // beyond residency simply find the queue drained and exit
    (void)P;
    (void)cfg;
    return 256 * 4;
}

size_t batch_desc_bytes(int64_t count) { return (size_t)count * sizeof(BatchDesc); }

int64_t batch_build_desc(int P, int cfg, int64_t count, const GemmArgs* probs, const int64_t* order,
                         void* host_buf) {
    const PlainConfig c = plain_config(P, cfg);
    const int64_t BM = c.tx * c.tm, BN = c.ty * c.tn;
    BatchDesc* d = (BatchDesc*)host_buf;
    int64_t tiles = 0;
    for (int64_t q = 0; q < count; ++q) {
        const GemmArgs& g = probs[order ? order[q] : q];
        d[q].g = g;
        d[q].tile_begin = tiles;
        d[q].tiles_m = (g.m + BM - 1) / BM;
        tiles += d[q].tiles_m * ((g.n + BN - 1) / BN);
    }
    return tiles;
}

// TD with the other operations of Sec. 2.3 (variant bit 0: the accurate
// addition, bit 1: TDmulq), on TD tile configuration 0.
int launch_plain_td_variant(int variant, const GemmArgs& g, hipStream_t st) {
    switch (variant) {
    case 1: return launch_plain_t<3, 16, 16, 2, 2, 16, 1>(g, st);
    case 2: return launch_plain_t<3, 16, 16, 2, 2, 16, 2>(g, st);
    case 3: return launch_plain_t<3, 16, 16, 2, 2, 16, 3>(g, st);
    default: return (int)hipErrorInvalidValue;
    }
}

int launch_scale_td_variant(int variant, const GemmArgs& g, hipStream_t st) {
    const int64_t blocks = (g.m * g.n + 255) / 256;
    if (blocks > 0x7fffffffLL) return (int)hipErrorInvalidConfiguration;
    const dim3 gr((unsigned)blocks), bl(256);
    if (variant & 2) hipLaunchKernelGGL((scale_kernel<3, 2>), gr, bl, 0, st, g);
    else hipLaunchKernelGGL((scale_kernel<3, 0>), gr, bl, 0, st, g);
    return (int)hipGetLastError();
}

int launch_scale(int P, const GemmArgs& g, hipStream_t st) {
    const int64_t total = g.m * g.n;
    const int64_t blocks = (total + 255) / 256;
    if (blocks > 0x7fffffffLL) return (int)hipErrorInvalidConfiguration;
    if (P == 2) hipLaunchKernelGGL(scale_kernel<2>, dim3((unsigned)blocks), dim3(256), 0, st, g);
    else if (P == 3) hipLaunchKernelGGL(scale_kernel<3>, dim3((unsigned)blocks), dim3(256), 0, st, g);
    else hipLaunchKernelGGL(scale_kernel<4>, dim3((unsigned)blocks), dim3(256), 0, st, g);
    return (int)hipGetLastError();
}

int launch_vec(int P, int op, int64_t n, const double* x, int64_t sx, const double* y, int64_t sy,
               double* r, int64_t sr, hipStream_t st) {
    if (n <= 0) return 0;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 256 * 64) blocks = 256 * 64;
    const dim3 gr((unsigned)blocks), bl(256);
#define MPG_VEC(PP, OO) hipLaunchKernelGGL((vec_kernel<PP, OO>), gr, bl, 0, st, n, x, sx, y, sy, r, sr)
    if (P == 2) { if (op == 0) MPG_VEC(2, 0); else MPG_VEC(2, 1); }
    else if (P == 3) {
        if (op == 0) MPG_VEC(3, 0);
        else if (op == 1) MPG_VEC(3, 1);
        else if (op == 2) MPG_VEC(3, 2);
        else MPG_VEC(3, 3);
    }
    else { if (op == 0) MPG_VEC(4, 0); else MPG_VEC(4, 1); }
#undef MPG_VEC
    return (int)hipGetLastError();
}

}  // namespace mpg

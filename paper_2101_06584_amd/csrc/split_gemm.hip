// split_gemm.hip -- the split ("Ozaki-style") form of the DD/TD/QD product on
// gfx950: operands cut into signed 7-bit integer digits whose products run
// exactly on the INT8 matrix cores, then recombined into P components.
//
// Pipeline (each stage one kernel, all on the caller's stream):
//  1. scale exponents: E_i for every row of op(A), F_j for every column of
//     op(B): largest |leading component| M = f 2^e (f in [1/2,1)) -> e + 1, so
//     each entry divided by 2^E lies in (-1/2, 1/2);
//  2. slicing: x = value / 2^E becomes s digits d_1..d_s in [-64, 64] with
//     x = sum_p d_p 2^(-7p) + r, |r| <= 2^(-7s-1)(1 + 2^-40): per digit, the
//     remainder's components are re-summed with VecSum (exact), the digit is
//     rint of the leading component times 2^(7p), and the digit is subtracted
//     exactly from that component;
//  3. anti-diagonal sums S_d = sum_{p+q=d} DA_p DB_q^T, d = 2..s+1, exact in
//     int32 (|S_d| <= s k 2^12 < 2^31 for s k < 2^19) with
//     v_mfma_i32_32x32x32_i8;
//  4. recombination: groups of four consecutive diagonals are folded exactly
//     (Horner in base 2^7, < 2^53 in magnitude, so exact in binary64), scaled
//     by 2^(E_i + F_j - 7 d_last) and accumulated with the precision's own
//     addition (Algorithm 1 / TDaddq / Algorithm 5) from the least significant
//     group up; then the alpha/beta epilogue of the plain form.
// Every stage is deterministic, so results are reproducible bit for bit.
#pragma clang fp contract(off)

#include "internal.hpp"
#include "mp_arith.hpp"

namespace mpg {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

static constexpr int kTileK = 64;          // k bytes per pipeline step
static constexpr int kLdsPad = 16;         // row padding (bytes) against bank conflicts
static constexpr int kSliceTile = 32;      // slicing kernel: 32 rows x 32 k per block

static inline int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }
static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// {bm, bn}: output tile of one MFMA workgroup (4 waves in 2 x 2).
static const SplitConfig kSplit[kSplitConfigs] = {{128, 128}, {64, 64}};

SplitConfig split_config(int id) { return kSplit[id]; }

int split_layout(int P, int64_t m, int64_t n, int64_t k, int s, int cfg, size_t* offE, size_t* offF,
                 size_t* offDA, size_t* offDB, size_t* offS, int64_t* Mp_, int64_t* Np_,
                 int64_t* Kp_) {
    (void)P;
    const SplitConfig c = kSplit[cfg];
    const int64_t Mp = round_up(m > 0 ? m : 1, c.bm);
    const int64_t Np = round_up(n > 0 ? n : 1, c.bn);
    const int64_t Kp = round_up(k > 0 ? k : 1, kTileK);
    size_t off = 0;
    *offE = off;  off = align256(off + sizeof(int32_t) * Mp);
    *offF = off;  off = align256(off + sizeof(int32_t) * Np);
    *offDA = off; off = align256(off + (size_t)s * Mp * Kp);
    *offDB = off; off = align256(off + (size_t)s * Np * Kp);
    *offS = off;  off = align256(off + sizeof(int32_t) * (size_t)s * Np * Mp);
    *Mp_ = Mp;
    *Np_ = Np;
    *Kp_ = Kp;
    return (int)0;
}

size_t split_workspace_bytes(int P, int64_t m, int64_t n, int64_t k, int s, int cfg) {
    size_t oE, oF, oA, oB, oS;
    int64_t Mp, Np, Kp;
    split_layout(P, m, n, k, s, cfg, &oE, &oF, &oA, &oB, &oS, &Mp, &Np, &Kp);
    return align256(oS + sizeof(int32_t) * (size_t)s * Np * Mp);
}

// ---------------------------------------------------------------------------
// Stage 1: scale exponents of "rows" r of a matrix whose element (r, l) sits
// at X[r * rs + l * ls] (rows of op(A): rs, ls = 1, lda for 'N', lda, 1 for
// 'T'; columns of op(B): ldb, 1 for 'N', 1, ldb for 'T').  Rows >= count get 0.
// ---------------------------------------------------------------------------

__device__ __forceinline__ int32_t scale_exponent(double M) {
    if (M == 0.0) return 0;
    int e;
    (void)frexp(M, &e);
    return e + 1;
}

// Lanes along rows (coalesced when rows are contiguous, rs == 1).
__global__ __launch_bounds__(256) void exponent_rows_kernel(const double* __restrict__ X,
                                                            int64_t rs, int64_t ls, int64_t count,
                                                            int64_t padded, int64_t k,
                                                            int32_t* __restrict__ E) {
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const int64_t r = (int64_t)blockIdx.x * 64 + lane;
    double M = 0.0;
    if (r < count)
        for (int64_t l = grp; l < k; l += 4) M = fmax(M, fabs(X[r * rs + l * ls]));
    red[grp][lane] = M;
    __syncthreads();
    if (grp == 0 && r < padded) {
        M = fmax(fmax(red[0][lane], red[1][lane]), fmax(red[2][lane], red[3][lane]));
        E[r] = (r < count) ? scale_exponent(M) : 0;
    }
}

// One wave per row, lanes along l (coalesced when l is contiguous, ls == 1).
__global__ __launch_bounds__(256) void exponent_rows_wave_kernel(const double* __restrict__ X,
                                                                 int64_t rs, int64_t ls,
                                                                 int64_t count, int64_t padded,
                                                                 int64_t k,
                                                                 int32_t* __restrict__ E) {
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= padded) return;
    double M = 0.0;
    if (r < count)
        for (int64_t l = lane; l < k; l += 64) M = fmax(M, fabs(X[r * rs + l * ls]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) M = fmax(M, __shfl_xor(M, off, 64));
    if (lane == 0) E[r] = (r < count) ? scale_exponent(M) : 0;
}

// ---------------------------------------------------------------------------
// Stage 2: digits.  Output plane p (0-based digit p+1) of D: D[p][r][l] with
// row length Kp; zero outside count x k.  Each block stages a 32 x 32 tile of
// the P component planes through LDS so that both the reads (along whichever
// index is contiguous) and the byte-plane writes (along l) are coalesced.
// ---------------------------------------------------------------------------

template <int P>
__device__ __forceinline__ void vec_sum_inplace(double (&r)[P]) {
    double s = r[P - 1];
#pragma unroll
    for (int i = P - 2; i >= 0; --i) two_sum(r[i], s, s, r[i + 1]);
    r[0] = s;
}

template <int P>
__global__ __launch_bounds__(256) void slice_kernel(const double* __restrict__ X, int64_t rs,
                                                    int64_t ls, int64_t ps, int64_t count,
                                                    int64_t k, const int32_t* __restrict__ E,
                                                    int s, int8_t* __restrict__ D, int64_t Rp,
                                                    int64_t Kp) {
    __shared__ double tile[P][kSliceTile][kSliceTile + 1];
    const int64_t r0 = (int64_t)blockIdx.y * kSliceTile;
    const int64_t l0 = (int64_t)blockIdx.x * kSliceTile;
    const int t = threadIdx.x;
    const bool rows_contig = (rs == 1);
    // load: 1024 entries, 4 per thread
#pragma unroll
    for (int it = 0; it < 4; ++it) {
        const int e = t + 256 * it;
        const int a = e % kSliceTile, b = e / kSliceTile;
        const int rr = rows_contig ? a : b;        // fastest index follows memory
        const int ll = rows_contig ? b : a;
        const int64_t gr = r0 + rr, gl = l0 + ll;
        const bool ok = gr < count && gl < k;
#pragma unroll
        for (int p = 0; p < P; ++p)
            tile[p][rr][ll] = ok ? X[p * ps + gr * rs + gl * ls] : 0.0;
    }
    __syncthreads();
#pragma unroll 1
    for (int it = 0; it < 4; ++it) {
        const int e = t + 256 * it;
        const int ll = e % kSliceTile, rr = e / kSliceTile;
        const int64_t gr = r0 + rr, gl = l0 + ll;
        if (gr >= Rp || gl >= Kp) continue;
        const int32_t Ei = (gr < count) ? E[gr] : 0;
        double rem[P];
#pragma unroll
        for (int p = 0; p < P; ++p) rem[p] = ldexp(tile[p][rr][ll], -Ei);
        int8_t* out = D + gr * Kp + gl;
        const int64_t plane = Rp * Kp;
        for (int p = 1; p <= s; ++p) {
            vec_sum_inplace<P>(rem);
            const double y = ldexp(rem[0], 7 * p);
            const double d = rint(y);
            rem[0] = ldexp(y - d, -7 * p);
            out[(int64_t)(p - 1) * plane] = (int8_t)(int)d;
        }
    }
}

// ---------------------------------------------------------------------------
// Stage 3: anti-diagonal sums on the INT8 matrix cores.
//
// Workgroup = 4 waves in 2 x 2, each wave a (BM/2) x (BN/2) block of 32 x 32
// MFMA tiles.  The flat step sequence (d, p, k-tile) for d = 2..s+1,
// p = 1..d-1 (q = d - p), k-tile = 0..Kp/64-1 is double-buffered through LDS
// (A_p rows and B_q columns, K contiguous, 64 + 16 bytes per row).  When a
// diagonal's last step is done the int32 accumulators are written to S_d.
//
// v_mfma_i32_32x32x32_i8: lane L supplies A row (L % 32) and B column (L % 32),
// 16 consecutive k bytes starting at 16 (L / 32) of the 32-wide k step (the
// same k bytes for A and B, so every k is paired with itself); the result
// element (row, col) with col = L % 32 and row = 8 (v / 4) + 4 (L / 32) + v % 4
// is held in accumulator register v.
// ---------------------------------------------------------------------------

template <int BM, int BN>
struct DiagTile {
    static constexpr int WM = BM / 2, WN = BN / 2;      // wave block
    static constexpr int FM = WM / 32, FN = WN / 32;    // MFMA tiles per wave
    static constexpr int ROW = kTileK + kLdsPad;        // LDS row bytes
    static constexpr int A_BYTES = BM * ROW, B_BYTES = BN * ROW;
    static constexpr int A_CHUNKS = BM * kTileK / 16;   // 16-byte chunks per tile
    static constexpr int B_CHUNKS = BN * kTileK / 16;
    static constexpr int A_PER_T = (A_CHUNKS + 255) / 256;
    static constexpr int B_PER_T = (B_CHUNKS + 255) / 256;
};

// Tile order: blocks dispatched to the same XCD (blockIdx % 8) take
// consecutive logical tiles, and logical tiles walk 8-row groups so a
// run of them shares op(A) row panels and op(B) column panels in that
// XCD's L2.
__device__ __forceinline__ bool diag_tile_coords(int64_t tiles_m, int64_t tiles_n, int64_t& tm,
                                                 int64_t& tn) {
    const int64_t total = tiles_m * tiles_n;
    const int64_t per_xcd = (total + 7) / 8;
    const int64_t bid = blockIdx.x;
    const int64_t logical = (bid % 8) * per_xcd + bid / 8;
    if (logical >= total) return false;
    const int64_t GM = 8;
    const int64_t group = logical / (GM * tiles_n);
    const int64_t first_m = group * GM;
    const int64_t gsize = (tiles_m - first_m) < GM ? (tiles_m - first_m) : GM;
    const int64_t in_group = logical - group * GM * tiles_n;
    tm = first_m + in_group % gsize;
    tn = in_group / gsize;
    return true;
}

template <int BM, int BN>
__global__ __launch_bounds__(256) void diag_mfma_kernel(const int8_t* __restrict__ DA,
                                                        const int8_t* __restrict__ DB,
                                                        int32_t* __restrict__ S, int64_t Mp,
                                                        int64_t Np, int64_t Kp, int s) {
    using T = DiagTile<BM, BN>;
    __shared__ __attribute__((aligned(16))) int8_t As[2][T::A_BYTES];
    __shared__ __attribute__((aligned(16))) int8_t Bs[2][T::B_BYTES];

    int64_t tm, tn;
    if (!diag_tile_coords(Mp / BM, Np / BN, tm, tn)) return;
    const int64_t m0 = tm * BM, n0 = tn * BN;
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int64_t ktiles = Kp / kTileK;
    const int64_t planeA = Mp * Kp, planeB = Np * Kp;

    v4i ra[T::A_PER_T], rb[T::B_PER_T];

    auto gload = [&](int p, int q, int64_t kt) {
        const int8_t* a = DA + (int64_t)(p - 1) * planeA + m0 * Kp + kt * kTileK;
        const int8_t* b = DB + (int64_t)(q - 1) * planeB + n0 * Kp + kt * kTileK;
#pragma unroll
        for (int h = 0; h < T::A_PER_T; ++h) {
            const int c = t + 256 * h;
            if (c < T::A_CHUNKS)
                ra[h] = *(const v4i*)(a + (int64_t)(c >> 2) * Kp + (c & 3) * 16);
        }
#pragma unroll
        for (int h = 0; h < T::B_PER_T; ++h) {
            const int c = t + 256 * h;
            if (c < T::B_CHUNKS)
                rb[h] = *(const v4i*)(b + (int64_t)(c >> 2) * Kp + (c & 3) * 16);
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int h = 0; h < T::A_PER_T; ++h) {
            const int c = t + 256 * h;
            if (c < T::A_CHUNKS) *(v4i*)(&As[buf][(c >> 2) * T::ROW + (c & 3) * 16]) = ra[h];
        }
#pragma unroll
        for (int h = 0; h < T::B_PER_T; ++h) {
            const int c = t + 256 * h;
            if (c < T::B_CHUNKS) *(v4i*)(&Bs[buf][(c >> 2) * T::ROW + (c & 3) * 16]) = rb[h];
        }
    };

    v16i acc[T::FM][T::FN];
#pragma unroll
    for (int i = 0; i < T::FM; ++i)
#pragma unroll
        for (int j = 0; j < T::FN; ++j) acc[i][j] = v16i{0};

    // step cursor
    int d = 2, p = 1;
    int64_t kt = 0;
    gload(p, d - p, kt);
    sstore(0);
    __syncthreads();
    int buf = 0;
    for (;;) {
        // successor step
        int nd = d, np = p;
        int64_t nkt = kt + 1;
        if (nkt == ktiles) {
            nkt = 0;
            ++np;
            if (np == nd) { ++nd; np = 1; }
        }
        const bool has_next = nd <= s + 1;
        if (has_next) gload(np, nd - np, nkt);

        // MFMAs on the current buffer
#pragma unroll
        for (int ks = 0; ks < kTileK / 32; ++ks) {
            v4i fa[T::FM], fb[T::FN];
            const int kb = ks * 32 + (lane >> 5) * 16;
#pragma unroll
            for (int i = 0; i < T::FM; ++i)
                fa[i] = *(const v4i*)(&As[buf][(wm * T::WM + i * 32 + (lane & 31)) * T::ROW + kb]);
#pragma unroll
            for (int j = 0; j < T::FN; ++j)
                fb[j] = *(const v4i*)(&Bs[buf][(wn * T::WN + j * 32 + (lane & 31)) * T::ROW + kb]);
#pragma unroll
            for (int i = 0; i < T::FM; ++i)
#pragma unroll
                for (int j = 0; j < T::FN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[i], fb[j], acc[i][j], 0, 0, 0);
        }

        // end of a diagonal: write S_d and clear the accumulators
        if (nd != d) {
            int32_t* Sd = S + (int64_t)(d - 2) * Np * Mp;
#pragma unroll
            for (int i = 0; i < T::FM; ++i)
#pragma unroll
                for (int j = 0; j < T::FN; ++j) {
                    const int64_t col = n0 + wn * T::WN + j * 32 + (lane & 31);
                    const int64_t rowb = m0 + wm * T::WM + i * 32 + 4 * (lane >> 5);
#pragma unroll
                    for (int v4 = 0; v4 < 4; ++v4) {
                        v4i o = {acc[i][j][4 * v4 + 0], acc[i][j][4 * v4 + 1], acc[i][j][4 * v4 + 2],
                                 acc[i][j][4 * v4 + 3]};
                        *(v4i*)(Sd + col * Mp + rowb + 8 * v4) = o;
                    }
                    acc[i][j] = v16i{0};
                }
        }
        if (!has_next) break;
        sstore(buf ^ 1);
        __syncthreads();
        buf ^= 1;
        d = nd;
        p = np;
        kt = nkt;
    }
}

// ---------------------------------------------------------------------------
// Stage 4: recombination and epilogue, one thread per entry (i fastest).
// ---------------------------------------------------------------------------

template <int P>
__global__ __launch_bounds__(256) void recombine_kernel(GemmArgs g, const int32_t* __restrict__ E,
                                                        const int32_t* __restrict__ F,
                                                        const int32_t* __restrict__ S, int s,
                                                        int64_t Mp, int64_t Np) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.m * g.n) return;
    const int64_t i = idx % g.m, j = idx / g.m;
    const int32_t ef = E[i] + F[j];
    const int64_t plane = Np * Mp;
    const int32_t* Sij = S + j * Mp + i;
    mp<P> acc = mp_zero<P>();
    const int G = (s + 3) / 4;
    for (int gi = G - 1; gi >= 0; --gi) {
        const int d0 = 2 + 4 * gi;
        const int d1 = (d0 + 3 < s + 1) ? d0 + 3 : s + 1;
        int64_t x = 0;
        for (int dd = d0; dd <= d1; ++dd) x = x * 128 + (int64_t)Sij[(int64_t)(dd - 2) * plane];
        mp<P> term = mp_zero<P>();
        term.c[0] = ldexp((double)x, ef - 7 * d1);
        acc = add(acc, term);
    }
    mp<P> alpha, beta;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        alpha.c[p] = g.alpha[p];
        beta.c[p] = g.beta[p];
    }
    const int64_t off = i + j * g.ldc;
    mp<P> t = mul(alpha, acc);
    if (!mp_is_zero(beta)) {
        mp<P> co;
#pragma unroll
        for (int p = 0; p < P; ++p) co.c[p] = g.C[p * g.sc + off];
        t = add(t, mul(beta, co));
    }
#pragma unroll
    for (int p = 0; p < P; ++p) g.C[p * g.sc + off] = t.c[p];
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------

static int launch_exponents(const double* X, int64_t rs, int64_t ls, int64_t count, int64_t padded,
                            int64_t k, int32_t* E, hipStream_t st) {
    if (rs == 1) {
        const int64_t blocks = (padded + 63) / 64;
        hipLaunchKernelGGL(exponent_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, st, X, rs, ls,
                           count, padded, k, E);
    } else {
        const int64_t blocks = (padded + 3) / 4;
        hipLaunchKernelGGL(exponent_rows_wave_kernel, dim3((unsigned)blocks), dim3(256), 0, st, X, rs,
                           ls, count, padded, k, E);
    }
    return (int)hipGetLastError();
}

static int launch_slices(int P, const double* X, int64_t rs, int64_t ls, int64_t ps, int64_t count,
                         int64_t k, const int32_t* E, int s, int8_t* D, int64_t Rp, int64_t Kp,
                         hipStream_t st) {
    const dim3 grid((unsigned)(Kp / kSliceTile), (unsigned)(Rp / kSliceTile));
    if (P == 2)
        hipLaunchKernelGGL(slice_kernel<2>, grid, dim3(256), 0, st, X, rs, ls, ps, count, k, E, s, D, Rp, Kp);
    else if (P == 3)
        hipLaunchKernelGGL(slice_kernel<3>, grid, dim3(256), 0, st, X, rs, ls, ps, count, k, E, s, D, Rp, Kp);
    else
        hipLaunchKernelGGL(slice_kernel<4>, grid, dim3(256), 0, st, X, rs, ls, ps, count, k, E, s, D, Rp, Kp);
    return (int)hipGetLastError();
}

static int launch_diag(int cfg, const int8_t* DA, const int8_t* DB, int32_t* S, int64_t Mp,
                       int64_t Np, int64_t Kp, int s, hipStream_t st) {
    const SplitConfig c = kSplit[cfg];
    const int64_t tiles = (Mp / c.bm) * (Np / c.bn);
    const int64_t grid = (tiles + 7) / 8 * 8;
    if (grid > 0x7fffffffLL) return (int)hipErrorInvalidConfiguration;
    if (cfg == 0)
        hipLaunchKernelGGL((diag_mfma_kernel<128, 128>), dim3((unsigned)grid), dim3(256), 0, st, DA, DB,
                           S, Mp, Np, Kp, s);
    else
        hipLaunchKernelGGL((diag_mfma_kernel<64, 64>), dim3((unsigned)grid), dim3(256), 0, st, DA, DB, S,
                           Mp, Np, Kp, s);
    return (int)hipGetLastError();
}

static int launch_recombine(int P, const GemmArgs& g, const int32_t* E, const int32_t* F,
                            const int32_t* S, int s, int64_t Mp, int64_t Np, hipStream_t st) {
    const int64_t blocks = (g.m * g.n + 255) / 256;
    if (blocks > 0x7fffffffLL) return (int)hipErrorInvalidConfiguration;
    if (P == 2)
        hipLaunchKernelGGL(recombine_kernel<2>, dim3((unsigned)blocks), dim3(256), 0, st, g, E, F, S, s, Mp, Np);
    else if (P == 3)
        hipLaunchKernelGGL(recombine_kernel<3>, dim3((unsigned)blocks), dim3(256), 0, st, g, E, F, S, s, Mp, Np);
    else
        hipLaunchKernelGGL(recombine_kernel<4>, dim3((unsigned)blocks), dim3(256), 0, st, g, E, F, S, s, Mp, Np);
    return (int)hipGetLastError();
}

// Runs stages 1..last.  Caller has validated arguments, checked the
// workspace size and handled quick returns / alpha == 0 / k == 0.
int launch_split_stages(int P, int s, int cfg, int last, const GemmArgs& g, void* ws,
                        hipStream_t st) {
    size_t oE, oF, oA, oB, oS;
    int64_t Mp, Np, Kp;
    split_layout(P, g.m, g.n, g.k, s, cfg, &oE, &oF, &oA, &oB, &oS, &Mp, &Np, &Kp);
    char* base = (char*)ws;
    int32_t* E = (int32_t*)(base + oE);
    int32_t* F = (int32_t*)(base + oF);
    int8_t* DA = (int8_t*)(base + oA);
    int8_t* DB = (int8_t*)(base + oB);
    int32_t* S = (int32_t*)(base + oS);
    // rows of op(A): element (i, l) at A[i*rs + l*ls]
    const int64_t a_rs = g.ta ? g.lda : 1, a_ls = g.ta ? 1 : g.lda;
    // columns of op(B): element (j, l) = op(B)(l, j)
    const int64_t b_rs = g.tb ? 1 : g.ldb, b_ls = g.tb ? g.ldb : 1;
    int rc;
    if ((rc = launch_exponents(g.A, a_rs, a_ls, g.m, Mp, g.k, E, st))) return rc;
    if ((rc = launch_exponents(g.B, b_rs, b_ls, g.n, Np, g.k, F, st))) return rc;
    if (last <= 1) return 0;
    if ((rc = launch_slices(P, g.A, a_rs, a_ls, g.sa, g.m, g.k, E, s, DA, Mp, Kp, st))) return rc;
    if ((rc = launch_slices(P, g.B, b_rs, b_ls, g.sb, g.n, g.k, F, s, DB, Np, Kp, st))) return rc;
    if (last <= 2) return 0;
    if ((rc = launch_diag(cfg, DA, DB, S, Mp, Np, Kp, s, st))) return rc;
    if (last <= 3) return 0;
    return launch_recombine(P, g, E, F, S, s, Mp, Np, st);
}

int launch_split(int P, int s, int cfg, const GemmArgs& g, void* ws, size_t ws_bytes,
                 hipStream_t st) {
    (void)ws_bytes;
    return launch_split_stages(P, s, cfg, 4, g, ws, st);
}

}  // namespace mpg

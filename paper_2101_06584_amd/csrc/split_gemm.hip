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
//  4. exact recombination: X = sum_d S_d 128^(s+1-d) as an exact multi-limb
//     integer, X 2^(E_i + F_j - 7 (s+1)) rounded once into P components
//     (round to nearest, ties to even, of the value and then of each exact
//     remainder); then the alpha/beta epilogue of the plain form.
// Every stage is deterministic, so results are reproducible bit for bit.
#pragma clang fp contract(off)

#include <utility>

#include "internal.hpp"
#include "exact_round.hpp"
#include "lds_dma.hpp"
#include "mp_arith.hpp"
#include "tile_order.hpp"

namespace mpg {

static constexpr int kSliceTile = 32;      // slicing kernel: 32 rows x 32 k per block

static inline int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }
static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// {bm, bn, g}: output tile of one MFMA workgroup (4 waves in 2 x 2) and the
// number of diagonals accumulated at once (the LDS ring depth is fixed per
// configuration in launch_diag).
static const SplitConfig kSplit[kSplitConfigs] = {{128, 128, 2}, {64, 64, 8}, {128, 64, 4},
                                                  {64, 64, 4}};

SplitConfig split_config(int id) { return kSplit[id]; }

uint32_t split_config_signature() {
    uint32_t h = 2166136261u;
    for (const SplitConfig& c : kSplit)
        for (int v : {c.bm, c.bn, c.g}) h = fnv1a(h, v);
    return h;
}

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
    off = align256(off + sizeof(uint64_t) * (Mp + Np));      // row maxima (stage 1)
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

// Rows contiguous (rs == 1): lanes along rows, so every load is coalesced;
// k is cut into chunks of kExpChunk so that the grid fills the chip, and the
// chunk maxima meet in a per-row atomic maximum of the bit patterns (for
// non-negative binary64 values their order as unsigned integers), which does
// not depend on the order of the updates.
constexpr int kExpChunk = 256;

__global__ __launch_bounds__(256) void exponent_clear_kernel(unsigned long long* __restrict__ mx,
                                                             int64_t count) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < count) mx[r] = 0ull;
}

__global__ __launch_bounds__(256) void exponent_rows_kernel(const double* __restrict__ X,
                                                            int64_t ls, int64_t count, int64_t k,
                                                            unsigned long long* __restrict__ mx) {
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const int64_t r = (int64_t)blockIdx.x * 64 + lane;
    const int64_t l0 = (int64_t)blockIdx.y * kExpChunk;
    const int64_t l1 = (l0 + kExpChunk < k) ? l0 + kExpChunk : k;
    double M = 0.0;
    if (r < count) {
#pragma unroll 8
        for (int64_t l = l0 + grp; l < l1; l += 4) M = fmax(M, fabs(X[r + l * ls]));
    }
    red[grp][lane] = M;
    __syncthreads();
    if (grp == 0 && r < count) {
        M = fmax(fmax(red[0][lane], red[1][lane]), fmax(red[2][lane], red[3][lane]));
        if (M != 0.0) atomicMax(mx + r, (unsigned long long)__double_as_longlong(M));
    }
}

__global__ __launch_bounds__(256) void exponent_finish_kernel(const unsigned long long* __restrict__ mx,
                                                              int64_t count, int64_t padded,
                                                              int32_t* __restrict__ E) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < padded) E[r] = (r < count) ? scale_exponent(__longlong_as_double((long long)mx[r])) : 0;
}

// One wave per row, lanes along l (coalesced when l is contiguous, ls == 1).
// Both operands in one launch: blockIdx.y picks the matrix.
struct RowSet {
    const double* X;
    int64_t rs, ls, count, padded;
    int32_t* E;
};

__global__ __launch_bounds__(256) void exponent_rows_wave_kernel(RowSet a, RowSet b, int64_t k) {
    const RowSet o = blockIdx.y ? b : a;
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= o.padded) return;
    double M = 0.0;
    if (r < o.count)
        for (int64_t l = lane; l < k; l += 64) M = fmax(M, fabs(o.X[r * o.rs + l * o.ls]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) M = fmax(M, __shfl_xor(M, off, 64));
    if (lane == 0) o.E[r] = (r < o.count) ? scale_exponent(M) : 0;
}

// Exponents of a batch of residue-form problems: block b of the launch is
// block b - b[0] of its problem, the first ceil(Mp / 4) covering op(A)'s
// rows (four rows a block, a wave a row), the rest op(B)'s columns.
__global__ __launch_bounds__(256) void exponent_rows_batch_kernel(const CrtBatchItem* __restrict__ items,
                                                                  int64_t count) {
    const int64_t bid = blockIdx.x;
    const CrtBatchItem& it = items[crt_batch_find(items, count, bid, 0)];
    const GemmArgs& g = it.g;
    const int64_t local = bid - it.b[0], a_blocks = (it.Mp + 3) / 4;
    const bool second = local >= a_blocks;
    const RowSet o = second ? RowSet{g.B, g.tb ? 1 : g.ldb, g.tb ? g.ldb : 1, g.n, it.Np, it.F}
                            : RowSet{g.A, g.ta ? g.lda : 1, g.ta ? 1 : g.lda, g.m, it.Mp, it.E};
    const int lane = threadIdx.x & 63;
    const int64_t r = (second ? local - a_blocks : local) * 4 + (threadIdx.x >> 6);
    if (r >= o.padded) return;
    double M = 0.0;
    if (r < o.count)
        for (int64_t l = lane; l < g.k; l += 64) M = fmax(M, fabs(o.X[r * o.rs + l * o.ls]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) M = fmax(M, __shfl_xor(M, off, 64));
    if (lane == 0) o.E[r] = (r < o.count) ? scale_exponent(M) : 0;
}

// ---------------------------------------------------------------------------
// Stage 2: digits.  Digit p (1-based) of entry (r, l) goes to
// D[((p-1) * (Kp/64) + l/64) * Rp * 64 + r * 64 + l % 64]: per digit plane,
// k-tiles of 64 are outermost, so the 64-byte k-slices of all rows of one
// k-tile are contiguous and a workgroup's tile (BM rows x 64) is one block.
// Zero outside count x k.  Each block stages a 32 x 32 tile of the P
// component planes through LDS so that both the reads (along whichever index
// is contiguous) and the byte-plane writes (along l) are coalesced.
// ---------------------------------------------------------------------------

template <int P>
__device__ __forceinline__ void vec_sum_inplace(double (&r)[P]) {
    double s = r[P - 1];
#pragma unroll
    for (int i = P - 2; i >= 0; --i) two_sum(r[i], s, s, r[i + 1]);
    r[0] = s;
}

// One operand of the slicing pass: element (r, l) of component p at
// X[p ps + r rs + l ls]; E its exponents; D its digit planes, Rp padded rows.
struct SliceOperand {
    const double* X;
    int64_t rs, ls, ps, count;
    const int32_t* E;
    int8_t* D;
    int64_t Rp;
};

// Both operands in one launch: blockIdx.z picks op(A) (0) or op(B) (1);
// row blocks past an operand's padded rows have no work.
template <int P>
__global__ __launch_bounds__(256) void slice_kernel(SliceOperand oa, SliceOperand ob, int64_t k, int s,
                                                    int64_t Kp) {
    const SliceOperand o = blockIdx.z ? ob : oa;
    const double* __restrict__ X = o.X;
    const int64_t rs = o.rs, ls = o.ls, ps = o.ps, count = o.count, Rp = o.Rp;
    const int32_t* __restrict__ E = o.E;
    int8_t* __restrict__ D = o.D;
    const int64_t r0 = (int64_t)blockIdx.y * kSliceTile;
    if (r0 >= Rp) return;                         // the whole block: before the barrier
    __shared__ double tile[P][kSliceTile][kSliceTile + 1];
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
        int8_t* out = D + (gl / kTileK) * Rp * kTileK + gr * kTileK + (gl % kTileK);
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
// One workgroup (4 waves in 2 x 2) owns a BM x BN block of every S_d and
// accumulates G diagonals at once: diagonals are processed in groups
// [d0, d1] (d1 = min(d0 + G - 1, s + 1)).  Within a group and a 64-wide
// k-tile the pairs (p, q) are visited with p descending from d1 - 1 to 1: the
// step for p brings in digit slice A_p and the single new slice B_{d1 - p};
// its pairs are (p, d1 - p - j), j = 0..G-1 (while q >= 1 and d1 - j >= d0),
// and B_{d1-p-j} is exactly the slice of j steps earlier.  Each wave keeps
// the B fragments of the last G steps in a register window, so a step reads
// one A and one B fragment from LDS and feeds up to G pairs; the accumulator
// of pair j is always diagonal d1 - j.
//
// Staging: the tiles of a step (BM x 64 and BN x 64 bytes) are copied from
// HBM straight into LDS by 16-byte direct-to-LDS loads, D steps deep in a
// ring, so no register holds data in flight; a wave waits for its own copies
// of the step it computes (vector-memory counter) and then meets the others
// at a barrier.  A 16-byte chunk c of tile row r sits at LDS chunk
// c ^ ((r / 4) mod 4) of that row: a direct-to-LDS load writes 64 consecutive
// chunks, so each lane gathers the global chunk that belongs to its slot, and
// the fragment reads below (32 rows, one chunk each) hit distinct banks.
//
// v_mfma_i32_32x32x32_i8: lane L supplies A row (L % 32) and B column (L % 32),
// 16 consecutive k bytes starting at 16 (L / 32) of the 32-wide k step (the
// same k bytes for A and B, so every k is paired with itself); the result
// element (row, col) with col = L % 32 and row = 8 (v / 4) + 4 (L / 32) + v % 4
// is held in accumulator register v.
// ---------------------------------------------------------------------------

template <int BM, int BN, int G, int D>
struct DiagDma {
    static constexpr int WM = BM / 2, WN = BN / 2;       // wave block
    static constexpr int FM = WM / 32, FN = WN / 32;     // MFMA tiles per wave
    static constexpr int KS = kTileK / 32;               // MFMA k-substeps per step
    static constexpr int A_BYTES = BM * kTileK, B_BYTES = BN * kTileK;
    static constexpr int STAGE = A_BYTES + B_BYTES;
    static constexpr int A_LOADS = A_BYTES / 4096, B_LOADS = B_BYTES / 4096;  // per thread
    static constexpr int PER_STEP = A_LOADS + B_LOADS;   // vector-memory ops per step
    static constexpr int LDS_BYTES = D * STAGE;
    static_assert(A_BYTES % 4096 == 0 && B_BYTES % 4096 == 0, "tiles split into 1 KiB wave copies");
    static_assert(PER_STEP * (D - 2) <= 63, "vector-memory counter range");
};

template <typename F, int... I>
__device__ __forceinline__ bool diag_unrolled(F&& f, std::integer_sequence<int, I...>) {
    return (... || f(std::integral_constant<int, I>{}));
}

constexpr int gcd_c(int a, int b) { return b == 0 ? a : gcd_c(b, a % b); }

// Steps of one pass (group with top diagonal d1, one k-tile): d1 - 1 real
// steps, padded to a multiple of u.
__device__ __forceinline__ int pass_len(int d1, int u) { return (d1 - 1 + u - 1) / u * u; }

template <int BM, int BN, int G, int D>
__global__ __launch_bounds__(256, 2) void diag_mfma_kernel(const int8_t* __restrict__ DA,
                                                           const int8_t* __restrict__ DB,
                                                           int32_t* __restrict__ S, int64_t Mp,
                                                           int64_t Np, int64_t Kp, int s) {
    using T = DiagDma<BM, BN, G, D>;
    // every pass is a multiple of U steps, so the window slot (step % G) and
    // the ring slot (step % D) are compile-time constants in an unrolled block
    constexpr int U = G / gcd_c(G, D) * D;
    __shared__ __attribute__((aligned(1024))) int8_t lds[T::LDS_BYTES];

    int64_t tm, tn;
    // groups of 4 tile rows per XCD: 1-2% faster than 2, 8 or 16 at n = 4096 and 8192
    if (!xcd_tile_coords<4>(blockIdx.x, Mp / BM, Np / BN, tm, tn)) return;
    const int64_t m0 = tm * BM, n0 = tn * BN;
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int wave_lds = __builtin_amdgcn_readfirstlane(wave) * 1024;
    const int nkt = (int)(Kp / kTileK);
    const int last_d = s + 1;

    // byte strides between digit slices and between k-tiles of one slice
    const int64_t sliceA = (int64_t)nkt * Mp * kTileK, sliceB = (int64_t)nkt * Np * kTileK;
    const int64_t ktA = Mp * kTileK, ktB = Np * kTileK;
    const int8_t* const A0 = DA + m0 * kTileK;
    const int8_t* const B0 = DB + n0 * kTileK;

    // global byte offset (within a tile) that this lane copies for its h-th
    // 1 KiB slot: LDS chunk u = t + 256 h -> row u / 4, LDS slot u % 4,
    // global chunk (u % 4) ^ ((row / 4) % 4)
    constexpr int NL = T::A_LOADS > T::B_LOADS ? T::A_LOADS : T::B_LOADS;
    int gofs[NL];
#pragma unroll
    for (int h = 0; h < NL; ++h) {
        const int u = t + 256 * h;
        const int r = u >> 2;
        gofs[h] = r * kTileK + (((u & 3) ^ ((r >> 2) & 3)) << 4);
    }
    // LDS offsets of this lane's fragments (relative to a stage)
    int aofs[T::KS][T::FM], bofs[T::KS][T::FN];
#pragma unroll
    for (int ks = 0; ks < T::KS; ++ks) {
#pragma unroll
        for (int i = 0; i < T::FM; ++i) aofs[ks][i] = swz(wm * T::WM + i * 32 + (lane & 31), 2 * ks + (lane >> 5));
#pragma unroll
        for (int jj = 0; jj < T::FN; ++jj)
            bofs[ks][jj] = T::A_BYTES + swz(wn * T::WN + jj * 32 + (lane & 31), 2 * ks + (lane >> 5));
    }

    // Fetch cursor: step fr of the pass (fd1, fkt) of length fL, and the
    // addresses of its tiles.  Step r of a pass copies A_p, p = d1 - 1 - r,
    // and B_{r+1}; the slice tile (digit p, k-tile kt) of rows m0.. is the
    // contiguous block at DA + ((p-1) nkt + kt) Mp 64 + m0 64.  Padding steps
    // re-copy the last real tiles, and past the last pass the cursor starts
    // over, so every step issues the same number of copies (all in bounds).
    int fd1 = min(G + 1, last_d), fr = 0, fkt = 0;
    int fL = pass_len(fd1, U);
    const int8_t* fa = A0 + (int64_t)(fd1 - 2) * sliceA;
    const int8_t* fb = B0;
    auto fnext = [&]() __attribute__((always_inline)) {
        if (++fr < fL) {
            if (fr <= fd1 - 2) {
                fa -= sliceA;
                fb += sliceB;
            }
            return;
        }
        fr = 0;
        if (++fkt == nkt) {
            fkt = 0;
            fd1 = (fd1 == last_d) ? min(G + 1, last_d) : min(fd1 + G, last_d);
            fL = pass_len(fd1, U);
        }
        fa = A0 + (int64_t)(fd1 - 2) * sliceA + (int64_t)fkt * ktA;
        fb = B0 + (int64_t)fkt * ktB;
    };
    // copies of one fill into ring slot R: op(A)'s (part 0) and op(B)'s (part
    // 1, which then moves the cursor), or both (part 2)
    auto issue = [&](auto rslot, auto partc) __attribute__((always_inline)) {
        constexpr int R = decltype(rslot)::value, part = decltype(partc)::value;
        int8_t* la = lds + R * T::STAGE + wave_lds;
        if constexpr (part != 1) {
#pragma unroll
            for (int h = 0; h < T::A_LOADS; ++h)
                __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(fa + gofs[h]),
                                                 (__attribute__((address_space(3))) void*)(la + 4096 * h), 16, 0, 0);
        }
        if constexpr (part != 0) {
#pragma unroll
            for (int h = 0; h < T::B_LOADS; ++h)
                __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(fb + gofs[h]),
                                                 (__attribute__((address_space(3))) void*)(la + T::A_BYTES + 4096 * h),
                                                 16, 0, 0);
            fnext();
        }
    };

    v16i acc[G][T::FM][T::FN];
#pragma unroll
    for (int j = 0; j < G; ++j)
#pragma unroll
        for (int i = 0; i < T::FM; ++i)
#pragma unroll
            for (int jj = 0; jj < T::FN; ++jj) acc[j][i][jj] = v16i{0};
    v4i wb[G][T::KS][T::FN];   // B fragments of the last G steps, slot = step % G

    // prologue: steps 0 .. D-2 into ring slots 0 .. D-2 (a pass has >= D steps)
    static_for<D - 1>([&](auto r) __attribute__((always_inline)) { issue(r, std::integral_constant<int, 2>{}); });

    // compute cursor: pass (cd0, cd1, ckt) of length cL, block start r0
    int cd0 = 2, cd1 = min(G + 1, last_d), ckt = 0;
    int cL = pass_len(cd1, U);
    for (;;) {
        const int gsz = cd1 - cd0 + 1;
        for (int r0 = 0; r0 < cL; r0 += U) {
            static_for<U>([&](auto rrc) __attribute__((always_inline)) {
                constexpr int rr = decltype(rrc)::value;
                constexpr int W = rr % G, R = rr % D, RF = (rr + D - 1) % D;
                // this step's tiles are in; every wave is past the previous
                // step, whose ring slot RF is refilled now
                wait_vm_barrier<T::PER_STEP * (D - 2)>();

                const int8_t* st = lds + R * T::STAGE;
                v4i fa_[T::KS][T::FM];
#pragma unroll
                for (int ks = 0; ks < T::KS; ++ks) {
#pragma unroll
                    for (int i = 0; i < T::FM; ++i) fa_[ks][i] = *(const v4i*)(st + aofs[ks][i]);
#pragma unroll
                    for (int jj = 0; jj < T::FN; ++jj) wb[W][ks][jj] = *(const v4i*)(st + bofs[ks][jj]);
                }
                // step r: pairs (p, r + 1 - j), j < nv, with p = d1 - 1 - r;
                // pair j uses the B fragments of j steps earlier and adds to
                // S_{d1 - j}; padding steps (p < 1) have none
                const int r = r0 + rr;
                const int nv = (r <= cd1 - 2) ? min(gsz, r + 1) : 0;
                static_for<G>([&](auto jc) __attribute__((always_inline)) {
                    constexpr int j = decltype(jc)::value;
                    if (j < nv) {
#pragma unroll
                        for (int ks = 0; ks < T::KS; ++ks)
#pragma unroll
                            for (int i = 0; i < T::FM; ++i)
#pragma unroll
                                for (int jj = 0; jj < T::FN; ++jj)
                                    acc[j][i][jj] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                                        fa_[ks][i], wb[(W - j + G) % G][ks][jj], acc[j][i][jj], 0, 0, 0);
                    }
                    // the next fill's copies after this step's first MFMAs
                    // rather than in a burst before them
                    if constexpr (G == 1)
                        issue(std::integral_constant<int, RF>{}, std::integral_constant<int, 2>{});
                    else if constexpr (j < 2)
                        issue(std::integral_constant<int, RF>{}, std::integral_constant<int, j>{});
                });
            });
        }
        if (++ckt < nkt) continue;

        // end of a group: write S_d for its diagonals, clear the accumulators
#pragma unroll
        for (int j = 0; j < G; ++j) {
            if (j < gsz) {
                int32_t* Sd = S + (int64_t)(cd1 - j - 2) * Np * Mp;
#pragma unroll
                for (int i = 0; i < T::FM; ++i)
#pragma unroll
                    for (int jj = 0; jj < T::FN; ++jj) {
                        const int64_t col = n0 + wn * T::WN + jj * 32 + (lane & 31);
                        const int64_t rowb = m0 + wm * T::WM + i * 32 + 4 * (lane >> 5);
#pragma unroll
                        for (int v4 = 0; v4 < 4; ++v4) {
                            v4i o = {acc[j][i][jj][4 * v4 + 0], acc[j][i][jj][4 * v4 + 1],
                                     acc[j][i][jj][4 * v4 + 2], acc[j][i][jj][4 * v4 + 3]};
                            *(v4i*)(Sd + col * Mp + rowb + 8 * v4) = o;
                        }
                    }
            }
#pragma unroll
            for (int i = 0; i < T::FM; ++i)
#pragma unroll
                for (int jj = 0; jj < T::FN; ++jj) acc[j][i][jj] = v16i{0};
        }
        // the stores share the vector-memory counter with the copies: drain
        // it so the counts in the waits stay exact
        wait_vm_all();
        if (cd1 == last_d) break;
        cd0 = cd1 + 1;
        cd1 = min(cd0 + G - 1, last_d);
        cL = pass_len(cd1, U);
        ckt = 0;
    }
    // the copies run ahead of the last step: let them land before the
    // workgroup's LDS is released
    wait_vm_all();
}

// ---------------------------------------------------------------------------
// Stage 4: exact recombination and epilogue, one thread per entry (i fastest).
// X = sum_{d=2}^{s+1} S_d 128^(s+1-d) is formed exactly in K 32-bit limbs
// (two's complement): the diagonals are folded from the most significant
// one down in groups of up to four, aligned to the least significant end, so
// that every group but the top one holds four; a group's Horner value
// |x| <= (2^31 - 1)(128^4 - 1)/127 < 2^53 is exact in int64, and each full
// group enters as X = X 2^28 + x.  Its magnitude is rounded once into the P
// components of X 2^(E_i + F_j - 7 (s+1)), then the epilogue.
// |X| < 2^(24.01 + 7 s), so K limbs hold s <= (32 K - 25.01) / 7.
// ---------------------------------------------------------------------------

template <int K>
constexpr int recombine_max_slices() { return (32 * K - 26) / 7; }

template <int P, int K>
__global__ __launch_bounds__(256) void recombine_kernel(GemmArgs g, const int32_t* __restrict__ E,
                                                        const int32_t* __restrict__ F,
                                                        const int32_t* __restrict__ S, int s,
                                                        int64_t Mp, int64_t Np) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.m * g.n) return;
    const int64_t i = idx % g.m, j = idx / g.m;
    const int64_t plane = Np * Mp;
    const int32_t* Sij = S + j * Mp + i;
    const int G = (s + 3) / 4;
    const int top = s - 4 * (G - 1);          // diagonals in the top group
    int64_t x = 0;
    for (int d = 2; d <= top + 1; ++d) x = x * 128 + (int64_t)Sij[(int64_t)(d - 2) * plane];
    uint32_t w[K];
    w[0] = (uint32_t)x;
    w[1] = (uint32_t)((uint64_t)x >> 32);
#pragma unroll
    for (int l = 2; l < K; ++l) w[l] = x < 0 ? 0xffffffffu : 0u;
    for (int d0 = top + 2; d0 <= s + 1; d0 += 4) {
        x = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) x = x * 128 + (int64_t)Sij[(int64_t)(d0 + u - 2) * plane];
#pragma unroll
        for (int l = K - 1; l >= 1; --l) w[l] = (w[l] << 28) | (w[l - 1] >> 4);
        w[0] <<= 28;
        const uint32_t ext = x < 0 ? 0xffffffffu : 0u;
        uint64_t c = (uint64_t)w[0] + (uint32_t)x;
        w[0] = (uint32_t)c;
        c = (uint64_t)w[1] + (uint32_t)((uint64_t)x >> 32) + (c >> 32);
        w[1] = (uint32_t)c;
#pragma unroll
        for (int l = 2; l < K; ++l) {
            c = (uint64_t)w[l] + ext + (c >> 32);
            w[l] = (uint32_t)c;
        }
    }
    double sg = 1.0;
    if (w[K - 1] >> 31) {
        uint64_t c = 1;
#pragma unroll
        for (int l = 0; l < K; ++l) {
            c += (uint64_t)(~w[l]);
            w[l] = (uint32_t)c;
            c >>= 32;
        }
        sg = -1.0;
    }
    double comp[P];
    limbs_to_components<P, K>(w, sg, E[i] + F[j] - 7 * (s + 1), comp);

    mp<P> acc, alpha, beta;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        acc.c[p] = comp[p];
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

// contiguous rows: k-chunked maxima (three launches) pay off on large
// operands; up to 2^18 entries one wave per row (strided loads) is one
// launch and the same maxima
static bool exponents_chunked(int64_t rs, int64_t count, int64_t k) {
    return rs == 1 && count * k > ((int64_t)1 << 18);
}

static int launch_exponents(const double* X, int64_t rs, int64_t ls, int64_t count, int64_t padded,
                            int64_t k, int32_t* E, uint64_t* mx, hipStream_t st) {
    if (exponents_chunked(rs, count, k)) {
        const int64_t cb = (count + 255) / 256, pb = (padded + 255) / 256;
        const int64_t chunks = (k + kExpChunk - 1) / kExpChunk;
        if (chunks > 65535) return (int)hipErrorInvalidConfiguration;
        unsigned long long* m = (unsigned long long*)mx;
        if (cb > 0) {
            hipLaunchKernelGGL(exponent_clear_kernel, dim3((unsigned)cb), dim3(256), 0, st, m, count);
            if (chunks > 0)
                hipLaunchKernelGGL(exponent_rows_kernel, dim3((unsigned)((count + 63) / 64), (unsigned)chunks),
                                   dim3(256), 0, st, X, ls, count, k, m);
        }
        hipLaunchKernelGGL(exponent_finish_kernel, dim3((unsigned)pb), dim3(256), 0, st, m, count, padded, E);
    } else {
        const int64_t blocks = (padded + 3) / 4;
        if (blocks > 0x7fffffffLL) return (int)hipErrorInvalidConfiguration;
        const RowSet o{X, rs, ls, count, padded, E};
        if (blocks > 0)
            hipLaunchKernelGGL(exponent_rows_wave_kernel, dim3((unsigned)blocks), dim3(256), 0, st, o, o, k);
    }
    return (int)hipGetLastError();
}

// Exponents of op(A)'s rows and op(B)'s columns; when neither takes the
// chunked path, one launch covers both (they then run side by side).
static int launch_exponents_pair(const double* A, int64_t a_rs, int64_t a_ls, int64_t m, int64_t Mp,
                                 const double* B, int64_t b_rs, int64_t b_ls, int64_t n, int64_t Np,
                                 int64_t k, int32_t* E, int32_t* F, uint64_t* mx, hipStream_t st) {
    if (exponents_chunked(a_rs, m, k) || exponents_chunked(b_rs, n, k)) {
        int rc = launch_exponents(A, a_rs, a_ls, m, Mp, k, E, mx, st);
        return rc ? rc : launch_exponents(B, b_rs, b_ls, n, Np, k, F, mx + Mp, st);
    }
    const int64_t blocks = ((Mp > Np ? Mp : Np) + 3) / 4;
    if (blocks > 0x7fffffffLL) return (int)hipErrorInvalidConfiguration;
    if (blocks > 0)
        hipLaunchKernelGGL(exponent_rows_wave_kernel, dim3((unsigned)blocks, 2), dim3(256), 0, st,
                           RowSet{A, a_rs, a_ls, m, Mp, E}, RowSet{B, b_rs, b_ls, n, Np, F}, k);
    return (int)hipGetLastError();
}

int launch_row_exponents_batch(const CrtBatchItem* d_items, int64_t count, int64_t blocks, hipStream_t st) {
    if (blocks > 0x7fffffffLL) return (int)hipErrorInvalidConfiguration;
    if (blocks > 0)
        hipLaunchKernelGGL(exponent_rows_batch_kernel, dim3((unsigned)blocks), dim3(256), 0, st, d_items, count);
    return (int)hipGetLastError();
}

int launch_row_exponents(const double* A, int64_t a_rs, int64_t a_ls, int64_t m, int64_t Mp,
                         const double* B, int64_t b_rs, int64_t b_ls, int64_t n, int64_t Np,
                         int64_t k, int32_t* E, int32_t* F, uint64_t* mx, hipStream_t st) {
    return launch_exponents_pair(A, a_rs, a_ls, m, Mp, B, b_rs, b_ls, n, Np, k, E, F, mx, st);
}

static int launch_slices(int P, const SliceOperand& a, const SliceOperand& b, int64_t k, int s, int64_t Kp,
                         hipStream_t st) {
    const int64_t rows = (a.Rp > b.Rp ? a.Rp : b.Rp) / kSliceTile;
    if (Kp / kSliceTile > 0x7fffffffLL || rows > 65535) return (int)hipErrorInvalidConfiguration;
    if (rows == 0 || Kp == 0) return 0;
    const dim3 grid((unsigned)(Kp / kSliceTile), (unsigned)rows, 2);
    if (P == 2)
        hipLaunchKernelGGL(slice_kernel<2>, grid, dim3(256), 0, st, a, b, k, s, Kp);
    else if (P == 3)
        hipLaunchKernelGGL(slice_kernel<3>, grid, dim3(256), 0, st, a, b, k, s, Kp);
    else
        hipLaunchKernelGGL(slice_kernel<4>, grid, dim3(256), 0, st, a, b, k, s, Kp);
    return (int)hipGetLastError();
}

static int launch_diag(int cfg, const int8_t* DA, const int8_t* DB, int32_t* S, int64_t Mp,
                       int64_t Np, int64_t Kp, int s, hipStream_t st) {
    const SplitConfig c = kSplit[cfg];
    const int64_t grid = xcd_grid((Mp / c.bm) * (Np / c.bn));
    if (grid > 0x7fffffffLL) return (int)hipErrorInvalidConfiguration;
#define MPG_DIAG(BM, BN, G, D)                                                                   \
    hipLaunchKernelGGL((diag_mfma_kernel<BM, BN, G, D>), dim3((unsigned)grid), dim3(256), 0, st, DA, DB, \
                       S, Mp, Np, Kp, s)
    // ring depths: at most 64 KiB of LDS per workgroup, so two fit on a CU
    switch (cfg) {
    case 0: MPG_DIAG(128, 128, 2, 4); break;
    case 1: MPG_DIAG(64, 64, 8, 8); break;
    case 2: MPG_DIAG(128, 64, 4, 4); break;
    default: MPG_DIAG(64, 64, 4, 4); break;
    }
#undef MPG_DIAG
    return (int)hipGetLastError();
}

template <int P>
static int launch_recombine_p(dim3 grid, const GemmArgs& g, const int32_t* E, const int32_t* F,
                              const int32_t* S, int s, int64_t Mp, int64_t Np, hipStream_t st) {
#define MPG_REC(K) \
    hipLaunchKernelGGL((recombine_kernel<P, K>), grid, dim3(256), 0, st, g, E, F, S, s, Mp, Np)
    if (s <= recombine_max_slices<4>()) MPG_REC(4);
    else if (s <= recombine_max_slices<6>()) MPG_REC(6);
    else if (s <= recombine_max_slices<8>()) MPG_REC(8);
    else MPG_REC(10);
#undef MPG_REC
    return (int)hipGetLastError();
}

static_assert(recombine_max_slices<10>() >= 40, "ten limbs hold the largest slice count");

static int launch_recombine(int P, const GemmArgs& g, const int32_t* E, const int32_t* F,
                            const int32_t* S, int s, int64_t Mp, int64_t Np, hipStream_t st) {
    const int64_t blocks = (g.m * g.n + 255) / 256;
    if (blocks > 0x7fffffffLL) return (int)hipErrorInvalidConfiguration;
    if (s > recombine_max_slices<10>()) return (int)hipErrorInvalidValue;
    const dim3 grid((unsigned)blocks);
    if (P == 2) return launch_recombine_p<2>(grid, g, E, F, S, s, Mp, Np, st);
    if (P == 3) return launch_recombine_p<3>(grid, g, E, F, S, s, Mp, Np, st);
    return launch_recombine_p<4>(grid, g, E, F, S, s, Mp, Np, st);
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
    uint64_t* MX = (uint64_t*)(base + align256(oF + sizeof(int32_t) * Np));   // Mp + Np row maxima
    // rows of op(A): element (i, l) at A[i*rs + l*ls]
    const int64_t a_rs = g.ta ? g.lda : 1, a_ls = g.ta ? 1 : g.lda;
    // columns of op(B): element (j, l) = op(B)(l, j)
    const int64_t b_rs = g.tb ? 1 : g.ldb, b_ls = g.tb ? g.ldb : 1;
    int rc;
    if ((rc = launch_exponents_pair(g.A, a_rs, a_ls, g.m, Mp, g.B, b_rs, b_ls, g.n, Np, g.k, E, F, MX,
                                    st)))
        return rc;
    if (last <= 1) return 0;
    const SliceOperand sa{g.A, a_rs, a_ls, g.sa, g.m, E, DA, Mp};
    const SliceOperand sb{g.B, b_rs, b_ls, g.sb, g.n, F, DB, Np};
    if ((rc = launch_slices(P, sa, sb, g.k, s, Kp, st))) return rc;
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

// crt_gemm.hip -- the residue (Chinese-remainder) form of the split product
// on gfx950.  The operands are scaled and cut into the same signed 7-bit
// digits as the split form, which define integers
//   A'_il = sum_p d_p(a_il) 128^(s-p),   B'_lj likewise,
// and the exact integer C'_ij = sum_l A'_il B'_lj is obtained from its
// residues modulo N pairwise coprime moduli m_t <= 256: one INT8 matrix
// product per modulus instead of one per digit pair.  The value is
// C'_ij 2^(E_i + F_j - 14 s), rounded to P components by repeated round to
// nearest (ties to even) of the exact remainder, then the alpha/beta
// epilogue.  This is the full square of digit pairs, not the split form's
// triangle, so the result is the exactly rounded product of the truncated
// operands.
//
// Pipeline (each stage one kernel, all on the caller's stream):
//  1. scale exponents E_i, F_j (shared with the split form);
//  2. residues: per entry the digits d_1..d_s (the split form's arithmetic),
//     folded in pairs c = 128 d_p + d_(p+1) and weighted by 2^(14e) mod m_t,
//     reduced to a signed byte congruent to A' u_t (rows of op(A)) or B'
//     (columns of op(B)) modulo m_t, where u_t = (M/m_t)^-1 mod m_t and M is
//     the product of the N moduli;
//  3. one INT8 matrix-core product per modulus (|sum| <= k 2^14 < 2^31, exact
//     in int32), reduced on the way out to y_t = C' u_t mod m_t in [0, m_t)
//     and stored as one byte per entry;
//  4. reconstruction: C' = sum_t y_t (M/m_t) - q M with q the nearest integer
//     to sum_t y_t / m_t (the 32-bit limbs of the sum are exact in binary64),
//     then the exact rounding into P components and the epilogue.
// N is the smallest count with M > 2 max|C'| (max|C'| = k (64 (128^s - 1) /
// 127)^2), so C' is the representative in (-M/2, M/2).
#pragma clang fp contract(off)

#include <cmath>

#include "internal.hpp"
#include "lds_dma.hpp"
#include "mp_arith.hpp"
#include "tile_order.hpp"

namespace mpg {

namespace {

constexpr int kNumModuli = 49;
constexpr int kLimbs = 11;          // 32-bit limbs: the product of all moduli has 342 bits
constexpr int kMaxPairs = 18;       // digit pairs for s <= 35

// Greedy pairwise coprime moduli from 256 down: every m <= 256 coprime to
// all larger ones taken so far.  Their product reaches 2^341.87.
constexpr int kModuli[kNumModuli] = {256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 217, 211,
                                     199, 197, 193, 191, 181, 179, 173, 167, 163, 157, 151, 149, 139,
                                     137, 131, 127, 113, 109, 107, 103, 101, 97,  89,  83,  79,  73,
                                     71,  67,  61,  59,  53,  47,  43,  41,  37,  29};

// Prefix products M_N (N = 0..49) and the cofactors M_N / m_t (t < N) as
// little-endian 32-bit limbs; row N (N - 1) / 2 + t of W holds M_N / m_t.
struct CrtTables {
    uint32_t M[kNumModuli + 1][kLimbs];
    uint32_t W[kNumModuli * (kNumModuli + 1) / 2][kLimbs];
    double inv[kNumModuli];          // 1 / m_t, rounded to nearest
    int mod[kNumModuli];             // m_t
};

constexpr CrtTables make_crt_tables() {
    CrtTables t{};
    uint32_t prod[kLimbs] = {1};
    for (int N = 0; N <= kNumModuli; ++N) {
        for (int l = 0; l < kLimbs; ++l) t.M[N][l] = prod[l];
        for (int i = 0; i < N; ++i) {              // exact long division by m_i
            uint64_t rem = 0;
            for (int l = kLimbs - 1; l >= 0; --l) {
                const uint64_t cur = (rem << 32) | prod[l];
                t.W[N * (N - 1) / 2 + i][l] = (uint32_t)(cur / (uint64_t)kModuli[i]);
                rem = cur % (uint64_t)kModuli[i];
            }
        }
        if (N < kNumModuli) {
            uint64_t carry = 0;
            for (int l = 0; l < kLimbs; ++l) {
                const uint64_t cur = (uint64_t)prod[l] * (uint64_t)kModuli[N] + carry;
                prod[l] = (uint32_t)cur;
                carry = cur >> 32;
            }
        }
    }
    for (int i = 0; i < kNumModuli; ++i) {
        t.inv[i] = 1.0 / (double)kModuli[i];
        t.mod[i] = kModuli[i];
    }
    return t;
}

__device__ const CrtTables kCrtDev = make_crt_tables();

const CrtTables& crt_host_tables() {
    static constexpr CrtTables t = make_crt_tables();
    return t;
}

// Per-operand digit-pair weights, passed by value: w[e][t] congruent to
// 2^(14 e) (times u_t for op(A)) modulo m_t, in [-128, 127]; zero for t >= N.
struct CrtWeights {
    int8_t w[kMaxPairs][kNumModuli];
};

// Output tile (bm x bn) and LDS ring depth of the per-modulus product.
struct CrtConfig {
    int bm, bn;
};
constexpr CrtConfig kCrt[kCrtConfigs] = {{128, 128}, {64, 64}};

inline int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct CrtLayout {
    int64_t Mp, Np, Kp;
    size_t oE, oF, oRA, oRB, oY, total;
};

CrtLayout crt_layout(int64_t m, int64_t n, int64_t k, int N, int cfg) {
    const CrtConfig c = kCrt[cfg];
    CrtLayout L;
    L.Mp = round_up(m > 0 ? m : 1, c.bm);
    L.Np = round_up(n > 0 ? n : 1, c.bn);
    L.Kp = round_up(k > 0 ? k : 1, kTileK);
    size_t off = 0;
    L.oE = off;  off = align256(off + sizeof(int32_t) * L.Mp);
    L.oF = off;  off = align256(off + sizeof(int32_t) * L.Np);
    L.oRA = off; off = align256(off + (size_t)N * L.Mp * L.Kp);
    L.oRB = off; off = align256(off + (size_t)N * L.Np * L.Kp);
    L.oY = off;  off = align256(off + (size_t)N * L.Mp * L.Np);
    L.total = off;
    return L;
}

// ---------------------------------------------------------------------------
// Stage 2: residues.  Block (kt, row tile) handles 16 rows x 64 k; thread t
// owns row t / 16 and the four k entries 4 (t % 16) .. + 3, so that one
// 32-bit store per modulus writes its four residue bytes.  Residue plane t
// has the digit planes' layout: byte (r, l) at
// R[((t (Kp/64) + l/64) Rp + r) 64 + l % 64].
// ---------------------------------------------------------------------------

constexpr int kResRows = 16;

template <int P>
__device__ __forceinline__ void vec_sum_desc(double (&r)[P]) {
    double s = r[P - 1];
#pragma unroll
    for (int i = P - 2; i >= 0; --i) two_sum(r[i], s, s, r[i + 1]);
    r[0] = s;
}

// digit p of the remainder r (the split form's slicing step)
template <int P>
__device__ __forceinline__ int next_digit(double (&r)[P], int p) {
    vec_sum_desc<P>(r);
    const double y = ldexp(r[0], 7 * p);
    const double d = rint(y);
    r[0] = ldexp(y - d, -7 * p);
    return (int)d;
}

// A value congruent to a modulo MOD in [-128, 127], for |a| < 2^24.2: the
// quotient from a single-precision reciprocal is off by at most one, so
// |a - q MOD| <= 0.62 MOD and one correction brings large moduli in range.
template <int MOD>
__device__ __forceinline__ int reduce_byte(int a) {
    constexpr float inv = 1.0f / (float)MOD;
    const int q = (int)rintf((float)a * inv);
    int r = a - __mul24(q, MOD);
    if constexpr (MOD > 190) {
        r = r > 127 ? r - MOD : r;
        r = r < -128 ? r + MOD : r;
    }
    return r;
}

template <int P, int NB>
__global__ __launch_bounds__(256) void crt_residue_kernel(const double* __restrict__ X, int64_t rs,
                                                          int64_t ls, int64_t ps, int64_t count,
                                                          int64_t k, const int32_t* __restrict__ E,
                                                          int s, int N, CrtWeights wt,
                                                          int8_t* __restrict__ R, int64_t Rp,
                                                          int64_t Kp) {
    __shared__ double tile[P][kResRows][kTileK + 1];
    const int64_t kt = blockIdx.x;
    const int64_t r0 = (int64_t)blockIdx.y * kResRows;
    const int64_t l0 = kt * kTileK;
    const int t = threadIdx.x;
    const bool rows_contig = (rs == 1);
#pragma unroll
    for (int it = 0; it < 4; ++it) {
        const int e = t + 256 * it;
        const int rr = rows_contig ? (e % kResRows) : (e / kTileK);   // fastest index follows memory
        const int ll = rows_contig ? (e / kResRows) : (e % kTileK);
        const int64_t gr = r0 + rr, gl = l0 + ll;
        const bool ok = gr < count && gl < k;
#pragma unroll
        for (int p = 0; p < P; ++p) tile[p][rr][ll] = ok ? X[p * ps + gr * rs + gl * ls] : 0.0;
    }
    __syncthreads();

    const int rr = t >> 4, lq = t & 15;
    const int64_t gr = r0 + rr;
    const int32_t Ei = (gr < count) ? E[gr] : 0;
    // digit pairs (p, p + 1) from p = start; digit 0 is zero when s is odd
    const int start = (s & 1) ? 0 : 1;
    const int npairs = (s + 1 - start) / 2;
    uint32_t word[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) word[i] = 0;
#pragma unroll 1
    for (int e4 = 0; e4 < 4; ++e4) {
        double rem[P];
#pragma unroll
        for (int p = 0; p < P; ++p) rem[p] = ldexp(tile[p][rr][4 * lq + e4], -Ei);
        int acc[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) acc[i] = 0;
        int p = start;
#pragma unroll 1
        for (int g = 0; g < npairs; ++g, p += 2) {
            const int d1 = (p == 0) ? 0 : next_digit<P>(rem, p);
            const int d2 = next_digit<P>(rem, p + 1);
            const int c = d1 * 128 + d2;              // |c| <= 8256
            const int8_t* w = wt.w[npairs - 1 - g];
#pragma unroll
            for (int i = 0; i < NB; ++i) acc[i] = __mul24(c, (int)w[i]) + acc[i];
        }
        static_for<NB>([&](auto ic) __attribute__((always_inline)) {
            constexpr int i = decltype(ic)::value;
            const int r = reduce_byte<kModuli[i]>(acc[i]);
            word[i] |= (uint32_t)(r & 255) << (8 * e4);
        });
    }
    if (gr >= Rp) return;
    const int64_t nkt = Kp / kTileK;
    uint8_t* out = (uint8_t*)R + (kt * Rp + gr) * kTileK + 4 * lq;
#pragma unroll
    for (int i = 0; i < NB; ++i)
        if (i < N) *(uint32_t*)(out + (int64_t)i * nkt * Rp * kTileK) = word[i];
}

// ---------------------------------------------------------------------------
// Stage 3: one INT8 product per modulus on the matrix cores.
//
// One workgroup (4 waves in 2 x 2) owns a BM x BN output tile and walks the
// steps (modulus t, k-tile kt) in order t nkt + kt; since residue planes are
// stored modulus-major and k-tile-major, the tiles of step u sit at
// RA + u Mp 64 + m0 64 and RB + u Np 64 + n0 64.  Tiles are staged D steps
// deep through LDS by 16-byte direct-to-LDS copies (the split form's scheme:
// swizzled 64-byte rows, a wave waits for its own copies and then meets the
// others at a barrier).  After the last k-tile of a modulus the int32 sums
// are reduced to y = sum mod m_t in [0, m_t) (exactly, in binary64), four
// consecutive rows packed per 32-bit store into plane t of Y (column-major,
// Y[(t Np + col) Mp + row]), and the accumulators cleared.
// ---------------------------------------------------------------------------

template <int BM, int BN, int D>
struct CrtDma {
    static constexpr int WM = BM / 2, WN = BN / 2;
    static constexpr int FM = WM / 32, FN = WN / 32;
    static constexpr int KS = kTileK / 32;
    static constexpr int A_BYTES = BM * kTileK, B_BYTES = BN * kTileK;
    static constexpr int STAGE = A_BYTES + B_BYTES;
    static constexpr int A_LOADS = A_BYTES / 4096, B_LOADS = B_BYTES / 4096;
    static constexpr int PER_STEP = A_LOADS + B_LOADS;
    static constexpr int LDS_BYTES = D * STAGE;
    static_assert(A_BYTES % 4096 == 0 && B_BYTES % 4096 == 0, "tiles split into 1 KiB wave copies");
    static_assert(PER_STEP * (D - 2) <= 63, "vector-memory counter range");
    static_assert(LDS_BYTES <= 65536, "two workgroups per CU");
};

template <int BM, int BN, int D>
__global__ __launch_bounds__(256, 2) void crt_mfma_kernel(const int8_t* __restrict__ RA,
                                                          const int8_t* __restrict__ RB,
                                                          uint8_t* __restrict__ Y, int64_t Mp,
                                                          int64_t Np, int64_t Kp, int N) {
    using T = CrtDma<BM, BN, D>;
    __shared__ __attribute__((aligned(1024))) int8_t lds[T::LDS_BYTES];

    int64_t tm, tn;
    if (!xcd_tile_coords<8>(blockIdx.x, Mp / BM, Np / BN, tm, tn)) return;
    const int64_t m0 = tm * BM, n0 = tn * BN;
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int wave_lds = __builtin_amdgcn_readfirstlane(wave) * 1024;
    const int nkt = (int)(Kp / kTileK);
    const int steps = N * nkt;
    const int64_t stepA = Mp * kTileK, stepB = Np * kTileK;

    // this lane's global byte offset within a tile for its h-th 1 KiB slot
    // (LDS chunk u = t + 256 h -> row u / 4, global chunk (u % 4) ^ ((row / 4) % 4))
    constexpr int NL = T::A_LOADS > T::B_LOADS ? T::A_LOADS : T::B_LOADS;
    int gofs[NL];
#pragma unroll
    for (int h = 0; h < NL; ++h) {
        const int u = t + 256 * h;
        const int r = u >> 2;
        gofs[h] = r * kTileK + (((u & 3) ^ ((r >> 2) & 3)) << 4);
    }
    int aofs[T::KS][T::FM], bofs[T::KS][T::FN];
#pragma unroll
    for (int ks = 0; ks < T::KS; ++ks) {
#pragma unroll
        for (int i = 0; i < T::FM; ++i) aofs[ks][i] = swz(wm * T::WM + i * 32 + (lane & 31), 2 * ks + (lane >> 5));
#pragma unroll
        for (int jj = 0; jj < T::FN; ++jj)
            bofs[ks][jj] = T::A_BYTES + swz(wn * T::WN + jj * 32 + (lane & 31), 2 * ks + (lane >> 5));
    }

    // fetch cursor: the next step to copy; past the last step it stays on the
    // last tiles (re-copied into slots no step reads), so every step issues
    // the same number of copies, all in bounds
    const int8_t* fa = RA + m0 * kTileK;
    const int8_t* fb = RB + n0 * kTileK;
    int fstep = 0, fslot = 0;
    auto issue = [&]() __attribute__((always_inline)) {
        int8_t* la = lds + fslot * T::STAGE + wave_lds;
#pragma unroll
        for (int h = 0; h < T::A_LOADS; ++h) copy16_to_lds(fa + gofs[h], la + 4096 * h);
#pragma unroll
        for (int h = 0; h < T::B_LOADS; ++h) copy16_to_lds(fb + gofs[h], la + T::A_BYTES + 4096 * h);
        if (++fstep < steps) {
            fa += stepA;
            fb += stepB;
        }
        fslot = (fslot + 1 == D) ? 0 : fslot + 1;
    };

    v16i acc[T::FM][T::FN];
#pragma unroll
    for (int i = 0; i < T::FM; ++i)
#pragma unroll
        for (int jj = 0; jj < T::FN; ++jj) acc[i][jj] = v16i{0};

    for (int r = 0; r < D - 1; ++r) issue();

    int cslot = 0, kt = 0, mod = 0;
    for (int u = 0; u < steps; ++u) {
        // step u's tiles are in; every wave is past step u - 1, whose slot is
        // refilled now
        wait_vm_barrier<T::PER_STEP * (D - 2)>();
        issue();
        const int8_t* st = lds + cslot * T::STAGE;
        cslot = (cslot + 1 == D) ? 0 : cslot + 1;
        v4i fa_[T::KS][T::FM], fb_[T::KS][T::FN];
#pragma unroll
        for (int ks = 0; ks < T::KS; ++ks) {
#pragma unroll
            for (int i = 0; i < T::FM; ++i) fa_[ks][i] = *(const v4i*)(st + aofs[ks][i]);
#pragma unroll
            for (int jj = 0; jj < T::FN; ++jj) fb_[ks][jj] = *(const v4i*)(st + bofs[ks][jj]);
        }
#pragma unroll
        for (int ks = 0; ks < T::KS; ++ks)
#pragma unroll
            for (int i = 0; i < T::FM; ++i)
#pragma unroll
                for (int jj = 0; jj < T::FN; ++jj)
                    acc[i][jj] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa_[ks][i], fb_[ks][jj], acc[i][jj], 0, 0, 0);
        if (++kt < nkt) continue;

        // last k-tile of modulus `mod`: reduce, store, clear
        const int mt = kCrtDev.mod[mod];
        const double md = (double)mt, inv = kCrtDev.inv[mod];
        uint8_t* Yt = Y + (int64_t)mod * Np * Mp;
#pragma unroll
        for (int i = 0; i < T::FM; ++i)
#pragma unroll
            for (int jj = 0; jj < T::FN; ++jj) {
                const int64_t col = n0 + wn * T::WN + jj * 32 + (lane & 31);
                const int64_t rowb = m0 + wm * T::WM + i * 32 + 4 * (lane >> 5);
#pragma unroll
                for (int v4 = 0; v4 < 4; ++v4) {
                    uint32_t word = 0;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        // |x| < 2^31: the rounded quotient is off by at most one
                        const double x = (double)acc[i][jj][4 * v4 + q];
                        int y = (int)fma(-rint(x * inv), md, x);
                        y += (y < 0) ? mt : 0;
                        word |= (uint32_t)y << (8 * q);
                    }
                    *(uint32_t*)(Yt + col * Mp + rowb + 8 * v4) = word;
                }
                acc[i][jj] = v16i{0};
            }
        // the stores share the vector-memory counter with the copies: drain
        // it so the counts in the waits stay exact
        wait_vm_all();
        kt = 0;
        ++mod;
    }
    // the copies run ahead of the last step: let them land before the
    // workgroup's LDS is released
    wait_vm_all();
}

// ---------------------------------------------------------------------------
// Stage 4: reconstruction, rounding and epilogue, one thread per entry (i
// fastest).  K 32-bit limbs hold M_N (M_N < 2^(32 K)).
// ---------------------------------------------------------------------------

// Components c_0..c_{P-1} of w 2^e (w: K-limb magnitude, sign sg): c_0 = RN
// of the value, then RN of the exact remainder, and so on (ties to even).
template <int P, int K>
__device__ __forceinline__ void limbs_to_components(uint32_t (&w)[K], double sg, int e, double* c) {
#pragma unroll
    for (int q = 0; q < P; ++q) {
        int h = -1;                                     // top set bit
#pragma unroll
        for (int l = K - 1; l >= 0; --l)
            if (h < 0 && w[l] != 0u) h = 32 * l + 31 - __builtin_clz(w[l]);
        if (h < 0) {
            c[q] = 0.0;
            continue;
        }
        if (h <= 52) {                                  // exact: the rest is zero
            const uint64_t v = (uint64_t)w[0] | ((uint64_t)w[1] << 32);
            c[q] = sg * ldexp((double)v, e);
#pragma unroll
            for (int l = 0; l < K; ++l) w[l] = 0u;
            continue;
        }
        const int sh = h - 52;
        // bits [sh - 11, sh + 53) as one 64-bit window (the top 53 are the
        // significand, then the guard bit), sticky bits below it
        const int base = sh - 11;
        uint64_t win = 0;
        bool below = false;
#pragma unroll
        for (int l = 0; l < K; ++l) {
            const int a = 32 * l - base;                // position of limb l's bit 0 in the window
            if (a >= 64) continue;
            if (a >= 0) {
                win |= (uint64_t)w[l] << a;
            } else if (a > -32) {
                win |= (uint64_t)(w[l] >> (-a));
                below = below || (w[l] & ((1u << (-a)) - 1u)) != 0u;
            } else {
                below = below || w[l] != 0u;
            }
        }
        uint64_t v = win >> 11;
        const bool guard = ((win >> 10) & 1u) != 0u;
        const bool sticky = below || (win & 0x3ffu) != 0u;
        const bool up = guard && (sticky || (v & 1u));
        v += up ? 1u : 0u;
        c[q] = sg * ldexp((double)v, sh + e);
        // remainder: the bits below sh; after rounding up, 2^sh minus them
        // with the sign flipped
#pragma unroll
        for (int l = 0; l < K; ++l) {
            const int a = 32 * l;
            if (a >= sh) w[l] = 0u;
            else if (a + 32 > sh) w[l] &= (1u << (sh - a)) - 1u;
        }
        if (up) {
            uint64_t carry = 1;
#pragma unroll
            for (int l = 0; l < K; ++l) {
                const uint64_t t = (uint64_t)(~w[l]) + carry;
                w[l] = (uint32_t)t;
                carry = t >> 32;
            }
#pragma unroll
            for (int l = 0; l < K; ++l) {
                const int a = 32 * l;
                if (a >= sh) w[l] = 0u;
                else if (a + 32 > sh) w[l] &= (1u << (sh - a)) - 1u;
            }
            sg = -sg;
        }
    }
}

template <int P, int K>
__global__ __launch_bounds__(256) void crt_recombine_kernel(GemmArgs g, const int32_t* __restrict__ E,
                                                            const int32_t* __restrict__ F,
                                                            const uint8_t* __restrict__ Y, int N,
                                                            int s, int64_t Mp, int64_t Np) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.m * g.n) return;
    const int64_t i = idx % g.m, j = idx / g.m;
    const int64_t plane = Mp * Np;
    const uint8_t* yp = Y + j * Mp + i;
    const int row0 = N * (N - 1) / 2;

    // S = sum_t y_t (M / m_t) limb by limb (each limb sum < 2^46, exact) and
    // f = sum_t y_t / m_t, whose nearest integer q gives C' = S - q M
    double L[K];
#pragma unroll
    for (int l = 0; l < K; ++l) L[l] = 0.0;
    double f = 0.0;
    for (int t = 0; t < N; ++t) {
        const double y = (double)yp[t * plane];
        f = fma(y, kCrtDev.inv[t], f);
        const uint32_t* w = kCrtDev.W[row0 + t];
#pragma unroll
        for (int l = 0; l < K; ++l) L[l] = fma(y, (double)w[l], L[l]);
    }
    const double q = rint(f);
#pragma unroll
    for (int l = 0; l < K; ++l) L[l] = fma(-q, (double)kCrtDev.M[N][l], L[l]);

    // carries: two's complement K-limb C', then sign and magnitude
    uint32_t w[K];
    int64_t carry = 0;
#pragma unroll
    for (int l = 0; l < K; ++l) {
        const int64_t v = (int64_t)L[l] + carry;
        w[l] = (uint32_t)v;
        carry = v >> 32;
    }
    double sg = 1.0;
    if (carry < 0) {
        uint64_t c1 = 1;
#pragma unroll
        for (int l = 0; l < K; ++l) {
            const uint64_t t = (uint64_t)(~w[l]) + c1;
            w[l] = (uint32_t)t;
            c1 = t >> 32;
        }
        sg = -1.0;
    }
    double comp[P];
    limbs_to_components<P, K>(w, sg, E[i] + F[j] - 14 * s, comp);

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

int inverse_mod(int a, int m) {          // a^-1 mod m for gcd(a, m) = 1, m <= 256
    for (int x = 1; x < m; ++x)
        if ((a * x) % m == 1) return x;
    return 0;
}

int8_t sym_byte(int v, int m) { return (int8_t)(v >= 128 ? v - m : v); }   // v in [0, m)

// Digit-pair weights 16384^e mod m_t (times u_t when `scaled`).
CrtWeights crt_weights(int N, int npairs, bool scaled) {
    CrtWeights W{};
    for (int t = 0; t < N; ++t) {
        const int m = kModuli[t];
        int u = 1;
        if (scaled) {
            int cof = 1;                                // (M_N / m_t) mod m_t
            for (int j = 0; j < N; ++j)
                if (j != t) cof = cof * (kModuli[j] % m) % m;
            u = inverse_mod(cof, m);
        }
        int pw = u % m;
        for (int e = 0; e < npairs; ++e) {
            W.w[e][t] = sym_byte(pw, m);
            pw = pw * (16384 % m) % m;
        }
    }
    return W;
}

int limbs_for(int N) {
    int top = 0;
    for (int l = 0; l < kLimbs; ++l)
        if (crt_host_tables().M[N][l]) top = l + 1;
    return top <= 4 ? 4 : top <= 6 ? 6 : top <= 8 ? 8 : 11;
}

int residue_bucket(int N) { return N <= 16 ? 16 : N <= 24 ? 24 : N <= 32 ? 32 : N <= 40 ? 40 : 49; }

template <int P>
int launch_residues_p(int NB, dim3 grid, hipStream_t st, const double* X, int64_t rs, int64_t ls,
                      int64_t ps, int64_t count, int64_t k, const int32_t* E, int s, int N,
                      const CrtWeights& w, int8_t* R, int64_t Rp, int64_t Kp) {
#define MPG_RES(NBV)                                                                                  \
    hipLaunchKernelGGL((crt_residue_kernel<P, NBV>), grid, dim3(256), 0, st, X, rs, ls, ps, count, k, E, \
                       s, N, w, R, Rp, Kp)
    switch (NB) {
    case 16: MPG_RES(16); break;
    case 24: MPG_RES(24); break;
    case 32: MPG_RES(32); break;
    case 40: MPG_RES(40); break;
    default: MPG_RES(49); break;
    }
#undef MPG_RES
    return (int)hipGetLastError();
}

int launch_residues(int P, const double* X, int64_t rs, int64_t ls, int64_t ps, int64_t count,
                    int64_t k, const int32_t* E, int s, int N, const CrtWeights& w, int8_t* R,
                    int64_t Rp, int64_t Kp, hipStream_t st) {
    const dim3 grid((unsigned)(Kp / kTileK), (unsigned)(Rp / kResRows));
    const int NB = residue_bucket(N);
    if (P == 2) return launch_residues_p<2>(NB, grid, st, X, rs, ls, ps, count, k, E, s, N, w, R, Rp, Kp);
    if (P == 3) return launch_residues_p<3>(NB, grid, st, X, rs, ls, ps, count, k, E, s, N, w, R, Rp, Kp);
    return launch_residues_p<4>(NB, grid, st, X, rs, ls, ps, count, k, E, s, N, w, R, Rp, Kp);
}

int launch_crt_mfma(int cfg, const int8_t* RA, const int8_t* RB, uint8_t* Y, int64_t Mp, int64_t Np,
                    int64_t Kp, int N, hipStream_t st) {
    const CrtConfig c = kCrt[cfg];
    const int64_t grid = xcd_grid((Mp / c.bm) * (Np / c.bn));
    if (grid > 0x7fffffffLL) return (int)hipErrorInvalidConfiguration;
    if (cfg == 0)
        hipLaunchKernelGGL((crt_mfma_kernel<128, 128, 4>), dim3((unsigned)grid), dim3(256), 0, st, RA, RB,
                           Y, Mp, Np, Kp, N);
    else
        hipLaunchKernelGGL((crt_mfma_kernel<64, 64, 8>), dim3((unsigned)grid), dim3(256), 0, st, RA, RB, Y,
                           Mp, Np, Kp, N);
    return (int)hipGetLastError();
}

template <int P>
int launch_crt_recombine_p(int K, dim3 grid, hipStream_t st, const GemmArgs& g, const int32_t* E,
                           const int32_t* F, const uint8_t* Y, int N, int s, int64_t Mp, int64_t Np) {
#define MPG_REC(KV) \
    hipLaunchKernelGGL((crt_recombine_kernel<P, KV>), grid, dim3(256), 0, st, g, E, F, Y, N, s, Mp, Np)
    switch (K) {
    case 4: MPG_REC(4); break;
    case 6: MPG_REC(6); break;
    case 8: MPG_REC(8); break;
    default: MPG_REC(11); break;
    }
#undef MPG_REC
    return (int)hipGetLastError();
}

}  // namespace

int crt_moduli_count(int64_t k, int s) {
    if (k <= 0 || k > 131071 || s < 1 || (s + 1) / 2 > kMaxPairs) return 0;
    // log2 of max|C'| = k (64 (128^s - 1) / 127)^2, then one bit for the sign
    // and a margin far above the rounding of these logarithms
    const double amax = 6.0 + 7.0 * s + std::log1p(-std::ldexp(1.0, -7 * s)) / std::log(2.0) -
                        std::log2(127.0);
    const double need = 1.0 + std::log2((double)k) + 2.0 * amax + 0.01;
    double bits = 0.0;
    for (int N = 1; N <= kNumModuli; ++N) {
        bits += std::log2((double)kModuli[N - 1]);
        if (bits > need) return N;
    }
    return 0;
}

size_t crt_workspace_bytes(int P, int64_t m, int64_t n, int64_t k, int s, int cfg) {
    (void)P;
    const int N = crt_moduli_count(k, s);
    if (N == 0) return 0;
    return crt_layout(m, n, k, N, cfg).total;
}

// Caller has validated arguments, the slice count (crt_moduli_count > 0), the
// workspace size and handled quick returns / alpha == 0 / k == 0.
int launch_crt(int P, int s, int cfg, const GemmArgs& g, void* ws, hipStream_t st) {
    const int N = crt_moduli_count(g.k, s);
    if (N == 0) return (int)hipErrorInvalidValue;
    const CrtLayout L = crt_layout(g.m, g.n, g.k, N, cfg);
    char* base = (char*)ws;
    int32_t* E = (int32_t*)(base + L.oE);
    int32_t* F = (int32_t*)(base + L.oF);
    int8_t* RA = (int8_t*)(base + L.oRA);
    int8_t* RB = (int8_t*)(base + L.oRB);
    uint8_t* Y = (uint8_t*)(base + L.oY);
    const int64_t a_rs = g.ta ? g.lda : 1, a_ls = g.ta ? 1 : g.lda;
    const int64_t b_rs = g.tb ? 1 : g.ldb, b_ls = g.tb ? g.ldb : 1;
    const int start = (s & 1) ? 0 : 1;
    const int npairs = (s + 1 - start) / 2;
    const CrtWeights wa = crt_weights(N, npairs, true);
    const CrtWeights wb = crt_weights(N, npairs, false);
    int rc;
    if ((rc = launch_row_exponents(g.A, a_rs, a_ls, g.m, L.Mp, g.k, E, st))) return rc;
    if ((rc = launch_row_exponents(g.B, b_rs, b_ls, g.n, L.Np, g.k, F, st))) return rc;
    if ((rc = launch_residues(P, g.A, a_rs, a_ls, g.sa, g.m, g.k, E, s, N, wa, RA, L.Mp, L.Kp, st))) return rc;
    if ((rc = launch_residues(P, g.B, b_rs, b_ls, g.sb, g.n, g.k, F, s, N, wb, RB, L.Np, L.Kp, st))) return rc;
    if ((rc = launch_crt_mfma(cfg, RA, RB, Y, L.Mp, L.Np, L.Kp, N, st))) return rc;
    const int64_t blocks = (g.m * g.n + 255) / 256;
    if (blocks > 0x7fffffffLL) return (int)hipErrorInvalidConfiguration;
    const dim3 grid((unsigned)blocks);
    const int K = limbs_for(N);
    if (P == 2) return launch_crt_recombine_p<2>(K, grid, st, g, E, F, Y, N, s, L.Mp, L.Np);
    if (P == 3) return launch_crt_recombine_p<3>(K, grid, st, g, E, F, Y, N, s, L.Mp, L.Np);
    return launch_crt_recombine_p<4>(K, grid, st, g, E, F, Y, N, s, L.Mp, L.Np);
}

}  // namespace mpg

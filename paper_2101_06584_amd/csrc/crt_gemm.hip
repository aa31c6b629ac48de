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

#include <algorithm>
#include <cmath>

#include "internal.hpp"
#include "lds_dma.hpp"
#include "exact_round.hpp"
#include "mp_arith.hpp"
#include "tile_order.hpp"

namespace mpg {

namespace {

constexpr int kNumModuli = 49;
constexpr int kLimbs = 11;          // 32-bit limbs: the product of all moduli has 342 bits
constexpr int kMaxCrtDigits = 24;  // one level: 14 s + log2 k - 1 < 342 bits needs s <= 24
constexpr int kCrtTileK = 32;       // k bytes per residue tile row and per product step

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
    double Md[kNumModuli + 1][kLimbs];                       // M as binary64 limbs
    double Wd[kNumModuli * (kNumModuli + 1) / 2][kLimbs];    // W as binary64 limbs
    // the one-level reconstruction's constants for N moduli:
    // kc[N][l] = 128 sum_q B'_{4l+q} 256^q with B'_c = sum_{t<N} (byte c of
    // W_t - 128), and r[N][l] = 2^(32 l) / M_N (M_N rounded to binary64)
    double kc[kNumModuli + 1][kLimbs];
    double r[kNumModuli + 1][kLimbs];
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
    for (int r = 0; r <= kNumModuli; ++r)
        for (int l = 0; l < kLimbs; ++l) t.Md[r][l] = (double)t.M[r][l];
    for (int r = 0; r < kNumModuli * (kNumModuli + 1) / 2; ++r)
        for (int l = 0; l < kLimbs; ++l) t.Wd[r][l] = (double)t.W[r][l];
    for (int N = 1; N <= kNumModuli; ++N) {
        const int row0 = N * (N - 1) / 2;
        for (int l = 0; l < kLimbs; ++l) {
            double kc = 0.0, p256 = 1.0;
            for (int q = 0; q < 4; ++q, p256 *= 256.0) {
                int64_t b = 0;
                for (int i = 0; i < N; ++i) b += (int64_t)((t.W[row0 + i][l] >> (8 * q)) & 255u) - 128;
                kc += 128.0 * (double)b * p256;
            }
            t.kc[N][l] = kc;
        }
        double md = 0.0;
        for (int l = kLimbs - 1; l >= 0; --l) md = md * 4294967296.0 + (double)t.M[N][l];
        double pw = 1.0 / md;                       // times 2^32 per limb: exact scalings
        for (int l = 0; l < kLimbs; ++l, pw *= 4294967296.0) t.r[N][l] = pw;
    }
    return t;
}

__device__ const CrtTables kCrtDev = make_crt_tables();

const CrtTables& crt_host_tables() {
    static constexpr CrtTables t = make_crt_tables();
    return t;
}

// Per-operand digit weights, passed by value: w[t][p] congruent to
// 128^(s - 1 - p) (times u_t for op(A)) modulo m_t, in [-128, 127]; zero for
// p >= s and t >= N.  The kernels' two MFMA groups span 64 moduli; rows past
// the table are zero.  Both operands' tables travel in one launch's
// arguments (2 x 1568 bytes).
struct CrtWeights {
    int8_t w[kNumModuli][32];
};

// One operand of the residue pass: row r of the matrix whose element (r, l)
// of component p sits at X[p ps + r rs + l ls]; E its row exponents; R its
// residue planes, Rp padded rows.
struct ResOperand {
    const double* X;
    int64_t rs, ls, ps, count;
    const int32_t* E;
    int8_t* R;
    int64_t Rp;
};
// the residue kernel's arguments (plus the runtime's hidden ones) stay
// within the 4 KiB a launch may carry
static_assert(2 * sizeof(CrtWeights) + 2 * sizeof(ResOperand) + 64 <= 3584, "residue kernel arguments");

// Output tile (bm x bn) of the per-modulus product and workgroups per CU.
struct CrtConfig {
    int bm, bn, per_cu;
};
constexpr CrtConfig kCrt[kCrtConfigs] = {{256, 256, 1}, {256, 128, 2}, {128, 128, 2}};

inline int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct CrtLayout {
    int64_t Mp, Np, Kp;
    size_t oE, oF, oMX, oRA, oRB, oY, total;
};

// kalign: 2 kTileK by default (the wide kernel takes an even number of
// 64-byte steps per modulus); the others need whole 64-byte residue segments.
CrtLayout crt_layout(int64_t m, int64_t n, int64_t k, int N, int cfg, int kalign = 2 * kTileK) {
    const CrtConfig c = kCrt[cfg];
    CrtLayout L;
    L.Mp = round_up(m > 0 ? m : 1, c.bm);
    L.Np = round_up(n > 0 ? n : 1, c.bn);
    L.Kp = round_up(k > 0 ? k : 1, kalign);
    size_t off = 0;
    L.oE = off;  off = align256(off + sizeof(int32_t) * L.Mp);
    L.oF = off;  off = align256(off + sizeof(int32_t) * L.Np);
    L.oMX = off; off = align256(off + sizeof(uint64_t) * (L.Mp + L.Np));
    L.oRA = off; off = align256(off + (size_t)N * L.Mp * L.Kp);
    L.oRB = off; off = align256(off + (size_t)N * L.Np * L.Kp);
    L.oY = off;  off = align256(off + (size_t)N * L.Mp * L.Np);
    L.total = off;
    return L;
}

// ---------------------------------------------------------------------------
// Stage 2: residues.  Block (64-wide k segment, row tile) stages 16 rows x 64
// k of the P component planes through LDS (loads coalesced along whichever
// index is contiguous); wave w then takes rows 4 w .. 4 w + 3 one at a time,
// lane L the entry (r, l) with l = 64 segment + L.  The lane computes the
// entry's digits d_1..d_s (the split form's slicing arithmetic) into bytes
// 0..s-1 of eight dwords.  The weighted sums a_t = sum_p d_p w_pt, with w_pt
// congruent to 128^(s-p) (times u_t for op(A)) modulo m_t in [-128, 127], are
// the product of the 64 x 32 digit block with the 32 x 32 weight block of
// each group of 32 moduli: two INT8 MFMAs per group (|a_t| <= 24 64 128 <
// 2^18, exact).  Each a_t is reduced to a residue of magnitude <= m_t / 2
// in single precision (exact: |a_t| < 2^24, and the rounded quotient errs by
// far less than 1/2), stored as its low byte.
// Residue plane t is cut into 32-byte k-tiles:
// byte (r, l) at R[((t (Kp/32) + l/32) Rp + r) 32 + l % 32].
// A block's share of one plane is two runs of 512 bytes (its 16 rows of two
// k-tiles).  Each group of 32 moduli is gathered plane by plane in LDS (the
// input tile's space, free once the remainders are in registers) and then
// written as those runs, 16 bytes per lane, so that no store scatters its
// lanes over 32 planes.
// ---------------------------------------------------------------------------

constexpr int kResRows = 16;
constexpr int kStagePlane = 2 * kResRows * kCrtTileK + 16;   // bytes per staged plane (16 B pad)
constexpr int kStageBytes = 32 * kStagePlane;

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

// Weight fragments of one lane for the residue MFMAs: modulus 32 cg +
// lane % 32, digits 16 (lane / 32) .. + 15 of table wt, split into the two
// levels' sets when SETS = 3, and the lane's moduli for the reduction.  A
// macro, so that the tables are read where the kernel's arguments live
// (passed through a function they would be copied to private memory).
#define MPG_CRT_WEIGHT_FRAGMENTS(wt, shi, lane, bw, mf, invm)                                   \
    for (int cg = 0; cg < NG; ++cg) {                                                           \
        const int tt = 32 * cg + ((lane) & 31);                                                 \
        v4i row = v4i{0, 0, 0, 0};                                                              \
        if (tt < kNumModuli) {                                                                  \
            const uint32_t* wp = (const uint32_t*)(wt)->w[tt] + 4 * ((lane) >> 5);               \
            row = v4i{(int)wp[0], (int)wp[1], (int)wp[2], (int)wp[3]};                          \
        }                                                                                       \
        if constexpr (SETS == 1) {                                                              \
            bw[0][cg] = row;                                                                    \
        } else {                                                                                \
            v4i hi_mask;                                                                        \
            _Pragma("unroll") for (int c = 0; c < 4; ++c) {                                     \
                uint32_t mk = 0u;                                                               \
                _Pragma("unroll") for (int j = 0; j < 4; ++j)                                   \
                    mk |= (16 * ((lane) >> 5) + 4 * c + j < (shi)) ? (0xffu << (8 * j)) : 0u;   \
                hi_mask[c] = (int)mk;                                                           \
            }                                                                                   \
            bw[0][cg] = row & hi_mask;                                                          \
            bw[1][cg] = row & ~hi_mask;                                                         \
            bw[2][cg] = row;                                                                    \
        }                                                                                       \
        const int m = tt < kNumModuli ? kCrtDev.mod[tt] : 1;                                    \
        mf[cg] = (float)m;                                                                      \
        invm[cg] = 1.0f / (float)m;                                                             \
    }

// One block of the residue pass: k segment `seg` (64 wide) of row block
// `rowblk` (16 rows) of operand o, with this lane's weight fragments bw and
// moduli mf, invm (MPG_CRT_WEIGHT_FRAGMENTS).
template <int P, int NG, int SETS>
__device__ __forceinline__ void crt_residue_block(const ResOperand& o, const v4i (&bw)[SETS][NG],
                                                  const float (&mf)[NG], const float (&invm)[NG], int64_t k,
                                                  int s, int N, int64_t Kp, int64_t seg, int64_t rowblk) {
    const double* __restrict__ X = o.X;
    const int64_t rs = o.rs, ls = o.ls, ps = o.ps, count = o.count, Rp = o.Rp;
    const int32_t* __restrict__ E = o.E;
    int8_t* __restrict__ R = o.R;
    const int64_t r0 = rowblk * kResRows;
    if (r0 >= Rp) return;                         // the whole block: before any barrier
    const int64_t l0 = seg * kTileK;
    const int t = threadIdx.x;
    const int64_t nkt = Kp / kCrtTileK;
    if (r0 >= count || l0 >= k) {
        // padding only: every residue is zero (wave w writes planes w, w + 4, ..)
        const int lane = t & 63, wave = t >> 6;
        const int st_kt = lane >> 5, st_row = (lane >> 1) & 15, st_half = lane & 1;
        for (int plane = wave; plane < SETS * N; plane += 4)
            *(v4i*)(R + (((int64_t)plane * nkt + 2 * seg + st_kt) * Rp + r0 + st_row) * kCrtTileK + 16 * st_half) =
                v4i{0, 0, 0, 0};
        return;
    }
    constexpr int kTileBytes = P * kResRows * (kTileK + 1) * 8;
    __shared__ __align__(16) uint8_t lds[kTileBytes > kStageBytes ? kTileBytes : kStageBytes];
    double (*tile)[kResRows][kTileK + 1] = reinterpret_cast<double (*)[kResRows][kTileK + 1]>(lds);
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

    const int lane = t & 63, wave = t >> 6;
    // the remainders of the wave's four rows, then the tile's space is free
    double rem[4][P];
#pragma unroll
    for (int rw = 0; rw < 4; ++rw) {
        const int64_t gr = r0 + wave * 4 + rw;
        const int32_t Ei = (gr < count) ? E[gr] : 0;
#pragma unroll
        for (int p = 0; p < P; ++p) rem[rw][p] = ldexp(tile[p][wave * 4 + rw][lane], -Ei);
    }
    __syncthreads();
    // the digits, the four rows' chains interleaved
    uint32_t dg[4][8];
#pragma unroll
    for (int rw = 0; rw < 4; ++rw)
#pragma unroll
        for (int i = 0; i < 8; ++i) dg[rw][i] = 0u;
#pragma unroll
    for (int p = 1; p <= 32; ++p)                 // 32 digit bytes per entry
        if (p <= s) {
#pragma unroll
            for (int rw = 0; rw < 4; ++rw)
                dg[rw][(p - 1) / 4] |= ((uint32_t)next_digit<P>(rem[rw], p) & 255u) << (8 * ((p - 1) % 4));
        }
    // A fragments: lane L < 32 gives digits 0..15 of entry L (first MFMA) or
    // of entry L + 32 (second), lane L >= 32 digits 16..31 of entry L - 32
    // (first) or L (second); the halves trade through a lane swap
    v4i a1[4], a2[4];
#pragma unroll
    for (int rw = 0; rw < 4; ++rw) {
        const v4i lo = {(int)dg[rw][0], (int)dg[rw][1], (int)dg[rw][2], (int)dg[rw][3]};
        const v4i hi = {(int)dg[rw][4], (int)dg[rw][5], (int)dg[rw][6], (int)dg[rw][7]};
        const bool low = lane < 32;
        const v4i x = low ? hi : lo;
        v4i xs;
#pragma unroll
        for (int c = 0; c < 4; ++c) xs[c] = __shfl_xor(x[c], 32, 64);
        a1[rw] = low ? lo : xs;
        a2[rw] = low ? xs : hi;
    }
    // the 16 B chunk c of a staged plane holds k-tile c / 32, row (c / 2) % 16,
    // bytes 16 (c % 2) .. + 15
    const int st_kt = lane >> 5, st_row = (lane >> 1) & 15, st_half = lane & 1;
#pragma unroll
    for (int cg = 0; cg < NG; ++cg)
#pragma unroll
        for (int set = 0; set < SETS; ++set) {
            const int tt = 32 * cg + (lane & 31);
#pragma unroll
            for (int rw = 0; rw < 4; ++rw) {
                v16i acc[2];
                acc[0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1[rw], bw[set][cg], v16i{0}, 0, 0, 0);
                acc[1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a2[rw], bw[set][cg], v16i{0}, 0, 0, 0);
                if (tt >= N) continue;
                uint8_t* plane = lds + (lane & 31) * kStagePlane;
#pragma unroll
                for (int eg = 0; eg < 2; ++eg)
#pragma unroll
                    for (int v4 = 0; v4 < 4; ++v4) {
                        uint32_t bits[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            // |r| <= m / 2: a byte for m < 256; for m = 256
                            // the low byte of r is congruent all the same.  r
                            // is an integer far below 2^22, so 1.5 2^23 + r is
                            // exact and its bit pattern is 0x4b400000 + r: the
                            // low byte is r mod 256
                            const float a = (float)acc[eg][4 * v4 + q];
                            const float r = fmaf(-rintf(a * invm[cg]), mf[cg], a);
                            bits[q] = __float_as_uint(r + 0x1.8p23f);
                        }
                        // the four low bytes in order: (0, 1) and (2, 3) pairwise, then both pairs
                        const uint32_t word = __builtin_amdgcn_perm(__builtin_amdgcn_perm(bits[3], bits[2], 0x0c0c0400u),
                                                                    __builtin_amdgcn_perm(bits[1], bits[0], 0x0c0c0400u),
                                                                    0x05040100u);
                        // entries 32 eg + 8 v4 + 4 (lane / 32) + 0..3 of row 4 wave + rw
                        *(uint32_t*)(plane + (eg * kResRows + wave * 4 + rw) * kCrtTileK + 8 * v4 +
                                     4 * (lane >> 5)) = word;
                    }
            }
            __syncthreads();
            const int nplanes = N - 32 * cg < 32 ? N - 32 * cg : 32;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int pl = 4 * i + wave;
                if (pl < nplanes) {
                    const v4i v = *(const v4i*)(lds + pl * kStagePlane + 16 * lane);
                    const int64_t plane = (int64_t)set * N + 32 * cg + pl;
                    *(v4i*)(R + ((plane * nkt + 2 * seg + st_kt) * Rp + r0 + st_row) * kCrtTileK + 16 * st_half) = v;
                }
            }
            __syncthreads();
        }
}

// Both operands in one launch: blockIdx.z = 0 takes op(A) with weights wa,
// 1 op(B) with wb; blockIdx.y beyond an operand's padded rows has no work.
template <int P, int NG, int SETS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void crt_residue_kernel(
    ResOperand oa, ResOperand ob, CrtWeights wa, CrtWeights wb, int64_t k, int s, int N, int shi,
    int64_t Kp) {
    const bool second = blockIdx.z != 0;
    const ResOperand o = second ? ob : oa;
    if ((int64_t)blockIdx.y * kResRows >= o.Rp) return;
    const CrtWeights* __restrict__ wt = second ? &wb : &wa;
    const int lane = threadIdx.x & 63;
    v4i bw[SETS][NG];
    float mf[NG], invm[NG];
#pragma unroll
    MPG_CRT_WEIGHT_FRAGMENTS(wt, shi, lane, bw, mf, invm)
    crt_residue_block<P, NG, SETS>(o, bw, mf, invm, k, s, N, Kp, blockIdx.x, blockIdx.y);
}

// ---------------------------------------------------------------------------
// Stage 3: one INT8 product per modulus on the matrix cores.
//
// One workgroup (WGM x WGN waves) owns a BM x BN output tile and walks the
// steps (modulus t, k-tile kt) in order t (Kp/32) + kt; since residue planes
// are stored modulus-major and k-tile-major, the tiles of step u are the
// contiguous blocks at RA + (u Mp + m0) 32 and RB + (u Np + n0) 32.  They are
// staged D steps deep through LDS by 16-byte direct-to-LDS copies: a wave
// waits for its own copies of the step it computes (vector-memory counter)
// and then meets the others at a barrier, so no register holds data in
// flight.  The 16-byte half c of tile row r sits at LDS half c ^ ((r / 8) % 2)
// of that row, so that the fragment reads (32 rows, one half each) hit
// distinct banks.  After the last k-tile of a modulus the int32 sums are
// reduced to y = sum mod m_t in [0, m_t) (exactly, in binary64), four
// consecutive rows packed per 32-bit store into plane t of Y (column-major,
// Y[(t Np + col) Mp + row]), and the accumulators cleared.
// ---------------------------------------------------------------------------

// Entries 4 v4 .. 4 v4 + 3 of accumulator x reduced modulo m = md (inv = 1/m
// rounded), four residues in [0, m) packed into a word.  The quotient is
// floor(x inv + 2^-20): for |x| < 2^31 the two roundings in fma(x, inv, c)
// err by less than 2^-21 together, and the fraction of x / m is 0 or lies
// in [1/m, 1 - 1/m] with 1/m >= 2^-8, so the offset keeps exact multiples
// on their quotient and carries no other value past the next integer;
// x - q m is then exact and in [0, m).
__device__ __forceinline__ uint32_t reduce_word(const v16i& x, int v4, double md, double inv) {
    uint32_t word = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double xd = (double)x[4 * v4 + q];
        const double quo = floor(fma(xd, inv, 0x1p-20));
        word |= (uint32_t)(int)fma(-quo, md, xd) << (8 * q);
    }
    return word;
}

// Reduced residues of 32 x 32 accumulator tile x into its place in a plane
// (column-major, rows contiguous).  Lane L holds rows 8 v4 + 4 (L / 32) + 0..3
// of column L % 32 in word v4; two lane swaps (upper half of the first
// operand with lower half of the second) leave lane L < 32 with rows 0..15
// and lane L + 32 with rows 16..31 of its column, so each lane writes one
// 16-byte run instead of four 4-byte words.  p: the lane's own first row
// (row 4 (L / 32) of its column); hi = L / 32.
__device__ __forceinline__ void store_tile(uint8_t* p, const v16i& x, double md, double inv, int hi) {
    const uint32_t w0 = reduce_word(x, 0, md, inv), w1 = reduce_word(x, 1, md, inv);
    const uint32_t w2 = reduce_word(x, 2, md, inv), w3 = reduce_word(x, 3, md, inv);
    const auto s02 = __builtin_amdgcn_permlane32_swap(w0, w2, false, false);   // (w0 | w2), (w0' | w2')
    const auto s13 = __builtin_amdgcn_permlane32_swap(w1, w3, false, false);
    *(v4i*)(p + 12 * hi) = v4i{(int)s02[0], (int)s02[1], (int)s13[0], (int)s13[1]};
}

// The product kernels issue each fill's copies one at a time between the
// step's MFMAs rather than in a burst before them (the wide kernel after
// MFMAs kCopyFirst, kCopyFirst + kCopyGap, ...).
constexpr int kCopyFirst = 8, kCopyGap = 2;

template <int BM, int BN, int WGM, int WGN, int D>
struct CrtDma {
    static constexpr int NT = 64 * WGM * WGN;             // threads
    static constexpr int WM = BM / WGM, WN = BN / WGN;    // wave block
    static constexpr int FM = WM / 32, FN = WN / 32;      // MFMA tiles per wave
    static constexpr int A_BYTES = BM * kCrtTileK, B_BYTES = BN * kCrtTileK;
    static constexpr int STAGE = A_BYTES + B_BYTES;
    static constexpr int ROUND = NT * 16;                 // bytes one copy instruction moves
    static constexpr int A_LOADS = A_BYTES / ROUND, B_LOADS = B_BYTES / ROUND;
    static constexpr int PER_STEP = A_LOADS + B_LOADS;
    static constexpr int LDS_BYTES = D * STAGE;
    static_assert(A_BYTES % ROUND == 0 && B_BYTES % ROUND == 0, "tiles split into whole copy rounds");
    static_assert(WM % 32 == 0 && WN % 32 == 0, "wave block of 32 x 32 MFMA tiles");
    static_assert(PER_STEP * (D - 2) <= 63, "vector-memory counter range");
    static_assert(LDS_BYTES <= 163840, "160 KiB of LDS per CU");
};

// LDS offset of 16-byte half c of row r in a 32-byte-row tile.  A 128-bit
// LDS read is served 16 lanes at a time from 64 four-byte banks; lanes read
// 16 consecutive rows, so the four-bank group 2 r + position must differ
// across them: the halves swap every 8 rows.
__device__ __forceinline__ int swz32(int r, int c) { return r * kCrtTileK + ((c ^ ((r >> 3) & 1)) << 4); }

// Output tile (tm, tn) over planes mod0 .. mod1 - 1.
template <int BM, int BN, int WGM, int WGN, int D>
__device__ __forceinline__ void crt_mfma_block(const int8_t* __restrict__ RA, const int8_t* __restrict__ RB,
                                               uint8_t* __restrict__ Y, int64_t Mp, int64_t Np, int64_t Kp,
                                               int Nmod, int64_t tm, int64_t tn, int mod0, int mod1) {
    using T = CrtDma<BM, BN, WGM, WGN, D>;
    __shared__ __attribute__((aligned(1024))) int8_t lds[T::LDS_BYTES];

    const int64_t m0 = tm * BM, n0 = tn * BN;
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int wm = wave % WGM, wn = wave / WGM;
    const int wave_lds = __builtin_amdgcn_readfirstlane(wave) * 1024;
    const int nkt = (int)(Kp / kCrtTileK);
    const int steps = (mod1 - mod0) * nkt;
    const int64_t stepA = Mp * kCrtTileK, stepB = Np * kCrtTileK;

    // this lane's global byte offset within a tile for its h-th copy round:
    // LDS half u = t + NT h is row u / 2, position u % 2, which holds global
    // half (u % 2) ^ ((row / 8) % 2)
    constexpr int NL = T::A_LOADS > T::B_LOADS ? T::A_LOADS : T::B_LOADS;
    int gofs[NL];
#pragma unroll
    for (int h = 0; h < NL; ++h) {
        const int u = t + T::NT * h;
        const int r = u >> 1;
        gofs[h] = r * kCrtTileK + (((u & 1) ^ ((r >> 3) & 1)) << 4);
    }
    int aofs[T::FM], bofs[T::FN];
#pragma unroll
    for (int i = 0; i < T::FM; ++i) aofs[i] = swz32(wm * T::WM + i * 32 + (lane & 31), lane >> 5);
#pragma unroll
    for (int jj = 0; jj < T::FN; ++jj) bofs[jj] = T::A_BYTES + swz32(wn * T::WN + jj * 32 + (lane & 31), lane >> 5);

    // fetch cursor: the next step to copy; past the last step it stays on the
    // last tiles (re-copied into slots no step reads), so every step issues
    // the same number of copies, all in bounds
    const int8_t* fa = RA + (int64_t)mod0 * nkt * stepA + m0 * kCrtTileK;
    const int8_t* fb = RB + (int64_t)mod0 * nkt * stepB + n0 * kCrtTileK;
    int fstep = 0, fslot = 0;
    // copy c of a fill (A rounds first, then B); the last one moves the cursor
    auto issue_part = [&](auto cc) __attribute__((always_inline)) {
        constexpr int c = decltype(cc)::value;
        int8_t* la = lds + fslot * T::STAGE + wave_lds;
        if constexpr (c < T::A_LOADS) copy16_to_lds(fa + gofs[c], la + T::ROUND * c);
        else copy16_to_lds(fb + gofs[c - T::A_LOADS], la + T::A_BYTES + T::ROUND * (c - T::A_LOADS));
        if constexpr (c == T::PER_STEP - 1) {
            if (++fstep < steps) {
                fa += stepA;
                fb += stepB;
            }
            fslot = (fslot + 1 == D) ? 0 : fslot + 1;
        }
    };
    auto issue = [&]() __attribute__((always_inline)) {
        static_for<T::PER_STEP>([&](auto c) __attribute__((always_inline)) { issue_part(c); });
    };

    v16i acc[T::FM][T::FN];
#pragma unroll
    for (int i = 0; i < T::FM; ++i)
#pragma unroll
        for (int jj = 0; jj < T::FN; ++jj) acc[i][jj] = v16i{0};

    for (int r = 0; r < D - 1; ++r) issue();

    int cslot = 0, kt = 0, mod = mod0;
    for (int u = 0; u < steps; ++u) {
        // step u's tiles are in; every wave is past step u - 1, whose slot is
        // refilled now
        wait_vm_barrier<T::PER_STEP * (D - 2)>();
        const int8_t* st = lds + cslot * T::STAGE;
        cslot = (cslot + 1 == D) ? 0 : cslot + 1;
        v4i fa_[T::FM], fb_[T::FN];
#pragma unroll
        for (int i = 0; i < T::FM; ++i) fa_[i] = *(const v4i*)(st + aofs[i]);
#pragma unroll
        for (int jj = 0; jj < T::FN; ++jj) fb_[jj] = *(const v4i*)(st + bofs[jj]);
        // the next fill's copies one after each MFMA (the rest after the last)
        static_for<T::FM * T::FN>([&](auto qc) __attribute__((always_inline)) {
            constexpr int q = decltype(qc)::value, i = q / T::FN, jj = q % T::FN;
            acc[i][jj] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa_[i], fb_[jj], acc[i][jj], 0, 0, 0);
            if constexpr (q < T::PER_STEP) issue_part(std::integral_constant<int, q>{});
            if constexpr (q == T::FM * T::FN - 1)
                static_for<T::PER_STEP>([&](auto c) __attribute__((always_inline)) {
                    if constexpr (decltype(c)::value > q) issue_part(c);
                });
        });
        if (++kt < nkt) continue;

        // last k-tile of modulus `mod`: reduce, store, clear
        // plane `mod` is modulus mod % Nmod of its residue set
        const int mi = mod % Nmod;
        const double md = (double)kCrtDev.mod[mi], inv = kCrtDev.inv[mi];
        uint8_t* Yt = Y + (int64_t)mod * Np * Mp;
#pragma unroll
        for (int i = 0; i < T::FM; ++i)
#pragma unroll
            for (int jj = 0; jj < T::FN; ++jj) {
                const int64_t col = n0 + wn * T::WN + jj * 32 + (lane & 31);
                const int64_t rowb = m0 + wm * T::WM + i * 32 + 4 * (lane >> 5);
                store_tile(Yt + col * Mp + rowb, acc[i][jj], md, inv, lane >> 5);
                acc[i][jj] = v16i{0};
            }
        // no drain: the waits stay sufficient with stores outstanding (see
        // the wide kernel)
        kt = 0;
        ++mod;
    }
    // the copies run ahead of the last step: let them land before the
    // workgroup's LDS is released
    wait_vm_all();
}

// The same product with one more wave that does all the copying: it waits
// (on its own counter) for step u's copies, meets the others at the step's
// barrier and then refills the slot step u - 1 used.  The WGM x WGN MFMA
// waves issue no loads: they wait only for their LDS reads, and the stores
// of each modulus's residues never hold up a later step.  With the copies
// in every wave, those stores share the counter with the copies in flight,
// so the first step of each modulus waits for the whole ring.  That matters
// on short k panels (a few steps per modulus: the batched form, 11% there);
// on long ones the single-call kernels measured the same or slower with the
// extra wave, so they keep the copies in the MFMA waves.
template <int BM, int BN, int WGM, int WGN, int D>
struct CrtDmaCw {
    static constexpr int NW = WGM * WGN;                  // MFMA waves; wave NW copies
    static constexpr int WM = BM / WGM, WN = BN / WGN;
    static constexpr int FM = WM / 32, FN = WN / 32;
    static constexpr int A_BYTES = BM * kCrtTileK, B_BYTES = BN * kCrtTileK;
    static constexpr int STAGE = A_BYTES + B_BYTES;
    static constexpr int A_LOADS = A_BYTES / 1024, B_LOADS = B_BYTES / 1024;   // 1 KiB per copy instruction
    static constexpr int PER_STEP = A_LOADS + B_LOADS;
    static constexpr int LDS_BYTES = D * STAGE;
    static_assert(A_BYTES % 1024 == 0 && B_BYTES % 1024 == 0, "tiles split into whole copies");
    static_assert(WM % 32 == 0 && WN % 32 == 0, "wave block of 32 x 32 MFMA tiles");
    static_assert(PER_STEP * (D - 2) <= 63, "vector-memory counter range");
    static_assert(LDS_BYTES <= 163840, "160 KiB of LDS per CU");
};

template <int BM, int BN, int WGM, int WGN, int D>
__device__ __forceinline__ void crt_mfma_block_cw(const int8_t* __restrict__ RA, const int8_t* __restrict__ RB,
                                                  uint8_t* __restrict__ Y, int64_t Mp, int64_t Np, int64_t Kp,
                                                  int Nmod, int64_t tm, int64_t tn, int mod0, int mod1) {
    using T = CrtDmaCw<BM, BN, WGM, WGN, D>;
    __shared__ __attribute__((aligned(1024))) int8_t lds[T::LDS_BYTES];

    const int64_t m0 = tm * BM, n0 = tn * BN;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nkt = (int)(Kp / kCrtTileK);
    const int steps = (mod1 - mod0) * nkt;
    const int64_t stepA = Mp * kCrtTileK, stepB = Np * kCrtTileK;

    if (wave == T::NW) {
        // copy h of a step: LDS half u = 64 h + lane of its tile is row u / 2,
        // position u % 2, which holds global half (u % 2) ^ ((row / 8) % 2)
        const int r0 = lane >> 1;
        const int gofs = r0 * kCrtTileK + (((lane & 1) ^ ((r0 >> 3) & 1)) << 4);   // rows 32 h + r0: same swap
        const int8_t* fa = RA + (int64_t)mod0 * nkt * stepA + m0 * kCrtTileK + gofs;
        const int8_t* fb = RB + (int64_t)mod0 * nkt * stepB + n0 * kCrtTileK + gofs;
        int fstep = 0, fslot = 0;
        // past the last step the cursor stays on the last tiles (copied into
        // slots no step reads), so every step issues the same copies
        auto issue = [&]() __attribute__((always_inline)) {
            int8_t* la = lds + fslot * T::STAGE;
#pragma unroll
            for (int h = 0; h < T::A_LOADS; ++h) copy16_to_lds(fa + h * 32 * kCrtTileK, la + 1024 * h);
#pragma unroll
            for (int h = 0; h < T::B_LOADS; ++h) copy16_to_lds(fb + h * 32 * kCrtTileK, la + T::A_BYTES + 1024 * h);
            if (++fstep < steps) {
                fa += stepA;
                fb += stepB;
            }
            fslot = (fslot + 1 == D) ? 0 : fslot + 1;
        };
        for (int r = 0; r < D - 1; ++r) issue();
        for (int u = 0; u < steps; ++u) {
            wait_vm_barrier<T::PER_STEP * (D - 2)>();    // step u landed; step u - 1's slot is free
            issue();
        }
        wait_vm_all();                                   // before the workgroup's LDS is released
        return;
    }

    const int wm = wave % WGM, wn = wave / WGM;
    int aofs[T::FM], bofs[T::FN];
#pragma unroll
    for (int i = 0; i < T::FM; ++i) aofs[i] = swz32(wm * T::WM + i * 32 + (lane & 31), lane >> 5);
#pragma unroll
    for (int jj = 0; jj < T::FN; ++jj) bofs[jj] = T::A_BYTES + swz32(wn * T::WN + jj * 32 + (lane & 31), lane >> 5);
    v16i acc[T::FM][T::FN];
#pragma unroll
    for (int i = 0; i < T::FM; ++i)
#pragma unroll
        for (int jj = 0; jj < T::FN; ++jj) acc[i][jj] = v16i{0};

    int cslot = 0, kt = 0, mod = mod0;
    for (int u = 0; u < steps; ++u) {
        wait_lds_barrier();
        const int8_t* st = lds + cslot * T::STAGE;
        cslot = (cslot + 1 == D) ? 0 : cslot + 1;
        v4i fa_[T::FM], fb_[T::FN];
#pragma unroll
        for (int i = 0; i < T::FM; ++i) fa_[i] = *(const v4i*)(st + aofs[i]);
#pragma unroll
        for (int jj = 0; jj < T::FN; ++jj) fb_[jj] = *(const v4i*)(st + bofs[jj]);
#pragma unroll
        for (int i = 0; i < T::FM; ++i)
#pragma unroll
            for (int jj = 0; jj < T::FN; ++jj)
                acc[i][jj] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa_[i], fb_[jj], acc[i][jj], 0, 0, 0);
        if (++kt < nkt) continue;

        // last k-tile of modulus `mod` (modulus mod % Nmod of its residue
        // set): reduce, store, clear
        const int mi = mod % Nmod;
        const double md = (double)kCrtDev.mod[mi], inv = kCrtDev.inv[mi];
        uint8_t* Yt = Y + (int64_t)mod * Np * Mp;
#pragma unroll
        for (int i = 0; i < T::FM; ++i)
#pragma unroll
            for (int jj = 0; jj < T::FN; ++jj) {
                const int64_t col = n0 + wn * T::WN + jj * 32 + (lane & 31);
                const int64_t rowb = m0 + wm * T::WM + i * 32 + 4 * (lane >> 5);
                store_tile(Yt + col * Mp + rowb, acc[i][jj], md, inv, lane >> 5);
                acc[i][jj] = v16i{0};
            }
        kt = 0;
        ++mod;
    }
}

template <int BM, int BN, int WGM, int WGN, int D>
__global__ __launch_bounds__(64 * WGM * WGN, 2) void crt_mfma_kernel(const int8_t* __restrict__ RA,
                                                                     const int8_t* __restrict__ RB,
                                                                     uint8_t* __restrict__ Y, int64_t Mp,
                                                                     int64_t Np, int64_t Kp, int N,
                                                                     int Nmod, int mods) {
    int64_t tm, tn;
    if (!xcd_tile_coords<8>(blockIdx.x, Mp / BM, Np / BN, tm, tn)) return;
    // this workgroup's planes: mod0 .. mod1 - 1 (blockIdx.y < ceil(N / mods))
    const int mod0 = (int)blockIdx.y * mods;
    const int mod1 = mod0 + mods < N ? mod0 + mods : N;
    crt_mfma_block<BM, BN, WGM, WGN, D>(RA, RB, Y, Mp, Np, Kp, Nmod, tm, tn, mod0, mod1);
}

// Wide variant: a 256 x 256 tile, four waves in 2 x 2 with 128 x 128 each
// (sixteen 32 x 32 accumulators, one wave per SIMD), which halves the LDS
// bytes read per MAC against 128 x 64 wave blocks.  With one wave per SIMD
// nothing else hides the LDS latency, so the fragments of step u + 1 are
// read while the MFMAs of step u run (two register buffers, the loop
// unrolled by two), and the ring is read one step ahead: at the top of step
// u the copies of step u + 1 must have landed and every wave must be done
// reading step u's slot, which step u + D then refills.

// One 32-byte k-tile per step (16 MFMAs per wave between barriers); the
// ring holds D steps.
struct WideCfg {
    static constexpr int NT = 256, BM = 256, BN = 256, WM = 128, WN = 128, FM = 4, FN = 4;
    static constexpr int SUB = BM * kCrtTileK;            // one operand's k-tile: 8 KiB
    static constexpr int B_OFF = SUB;
    static constexpr int STAGE = 2 * SUB;
    static constexpr int ROUND = NT * 16;
    static constexpr int LOADS = SUB / ROUND;             // copy rounds per operand k-tile
    static constexpr int PER_STEP = 2 * LOADS;
    static constexpr int D = 8;
    static constexpr int LDS_BYTES = D * STAGE;
    static_assert(SUB % ROUND == 0, "whole copy rounds");
    static_assert(PER_STEP * (D - 1) <= 63, "vector-memory counter range");
    static_assert(LDS_BYTES <= 163840, "160 KiB of LDS per CU");
};

__global__ __launch_bounds__(256, 1) void crt_mfma_wide_kernel(const int8_t* __restrict__ RA,
                                                               const int8_t* __restrict__ RB,
                                                               uint8_t* __restrict__ Y, int64_t Mp,
                                                               int64_t Np, int64_t Kp, int N,
                                                               int Nmod, int mods) {
    using W = WideCfg;
    constexpr int D = W::D;
    __shared__ __attribute__((aligned(1024))) int8_t lds[W::LDS_BYTES];

    int64_t tm, tn;
    if (!xcd_tile_coords<8>(blockIdx.x, Mp / 256, Np / 256, tm, tn)) return;
    const int64_t m0 = tm * 256, n0 = tn * 256;
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int wm = wave % 2, wn = wave / 2;
    const int wave_lds = __builtin_amdgcn_readfirstlane(wave) * 1024;
    const int spm = (int)(Kp / kCrtTileK);        // steps per modulus, even (Kp % 64 == 0)
    // this workgroup's planes: mod0 .. mod1 - 1 (blockIdx.y < ceil(N / mods))
    const int mod0 = (int)blockIdx.y * mods;
    const int mod1 = mod0 + mods < N ? mod0 + mods : N;
    const int steps = (mod1 - mod0) * spm;
    const int64_t tileA = Mp * kCrtTileK, tileB = Np * kCrtTileK;

    int gofs[W::LOADS];
#pragma unroll
    for (int h = 0; h < W::LOADS; ++h) {
        const int u = t + W::NT * h;
        const int r = u >> 1;
        gofs[h] = r * kCrtTileK + (((u & 1) ^ ((r >> 3) & 1)) << 4);
    }
    int aofs[W::FM], bofs[W::FN];
#pragma unroll
    for (int i = 0; i < W::FM; ++i) aofs[i] = swz32(wm * W::WM + i * 32 + (lane & 31), lane >> 5);
#pragma unroll
    for (int jj = 0; jj < W::FN; ++jj) bofs[jj] = W::B_OFF + swz32(wn * W::WN + jj * 32 + (lane & 31), lane >> 5);

    const int8_t* fa = RA + (int64_t)mod0 * spm * tileA + m0 * kCrtTileK;
    const int8_t* fb = RB + (int64_t)mod0 * spm * tileB + n0 * kCrtTileK;
    int fstep = 0, fslot = 0;
    // the whole fill of one step (the prologue)
    auto issue = [&]() __attribute__((always_inline)) {
        int8_t* la = lds + fslot * W::STAGE + wave_lds;
#pragma unroll
        for (int h = 0; h < W::LOADS; ++h) {
            copy16_to_lds(fa + gofs[h], la + W::ROUND * h);
            copy16_to_lds(fb + gofs[h], la + W::B_OFF + W::ROUND * h);
        }
        if (++fstep < steps) {
            fa += tileA;
            fb += tileB;
        }
        fslot = (fslot + 1 == D) ? 0 : fslot + 1;
    };
    // one copy of that fill (in the loop): A round c / 2 for even c, B for
    // odd; the last one moves the cursor
    auto issue_part = [&](auto cc) __attribute__((always_inline)) {
        constexpr int c = decltype(cc)::value, h = c / 2;
        int8_t* la = lds + fslot * W::STAGE + wave_lds;
        if constexpr (c % 2 == 0) copy16_to_lds(fa + gofs[h], la + W::ROUND * h);
        else copy16_to_lds(fb + gofs[h], la + W::B_OFF + W::ROUND * h);
        if constexpr (c == 2 * W::LOADS - 1) {
            if (++fstep < steps) {
                fa += tileA;
                fb += tileB;
            }
            fslot = (fslot + 1 == D) ? 0 : fslot + 1;
        }
    };

    // each modulus's first step starts its accumulators from zero (no
    // clearing pass after the stores)
    v16i acc[W::FM][W::FN];
    v4i fra[2][W::FM], frb[2][W::FN];

    // prologue: steps 0 .. D-1 in flight, step 0 landed, its fragments read
    for (int r = 0; r < D; ++r) issue();
    wait_vm_barrier<W::PER_STEP * (D - 1)>();
#pragma unroll
    for (int i = 0; i < W::FM; ++i) fra[0][i] = *(const v4i*)(lds + aofs[i]);
#pragma unroll
    for (int jj = 0; jj < W::FN; ++jj) frb[0][jj] = *(const v4i*)(lds + bofs[jj]);

    auto step = [&](auto curc, auto firstc, int u) __attribute__((always_inline)) {
        constexpr int cur = decltype(curc)::value, nxt = 1 - cur;
        constexpr bool first = decltype(firstc)::value;   // a modulus's first step
        // keep each step's MFMAs after its barrier: hoisted above it they
        // would wait on the fragment reads just issued for them
        __builtin_amdgcn_sched_barrier(0);
        wait_vm_barrier<W::PER_STEP * (D - 2)>();
        // the next step's eight fragment reads, one after each of the first
        // eight MFMAs: issued in a burst they stall the wave (measured 2-3 %
        // on the whole product at n = 4096); then the copies of step u + D
        // into step u's slot, one after each of MFMAs kCopyFirst,
        // kCopyFirst + kCopyGap, ...
        const int8_t* st = lds + ((u + 1) % D) * W::STAGE;
        static_for<W::FM * W::FN>([&](auto qc) {
            constexpr int q = decltype(qc)::value, i = q / W::FN, jj = q % W::FN;
            acc[i][jj] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fra[cur][i], frb[cur][jj],
                                                               first ? v16i{0} : acc[i][jj], 0, 0, 0);
            if constexpr (q < W::FM) fra[nxt][q] = *(const v4i*)(st + aofs[q]);
            else if constexpr (q < W::FM + W::FN) frb[nxt][q - W::FM] = *(const v4i*)(st + bofs[q - W::FM]);
            if constexpr (q >= kCopyFirst && (q - kCopyFirst) % kCopyGap == 0 &&
                          (q - kCopyFirst) / kCopyGap < 2 * W::LOADS)
                issue_part(std::integral_constant<int, (q - kCopyFirst) / kCopyGap>{});
            __builtin_amdgcn_sched_barrier(0);
        });
    };
    const int64_t ybase = (n0 + wn * W::WN + (lane & 31)) * Mp + m0 + wm * W::WM + 4 * (lane >> 5);
    int u = 0;
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using First = std::integral_constant<bool, true>;
    using Next = std::integral_constant<bool, false>;
    for (int mod = mod0; mod < mod1; ++mod) {
        step(I0{}, First{}, u);
        step(I1{}, Next{}, u + 1);
        u += 2;
        for (int kk = 2; kk < spm; kk += 2, u += 2) {
            step(I0{}, Next{}, u);
            step(I1{}, Next{}, u + 1);
        }
        // plane `mod` is modulus mod % Nmod of its residue set
        const int mi = mod % Nmod;
        const double md = (double)kCrtDev.mod[mi], inv = kCrtDev.inv[mi];
        // this lane's first byte in plane `mod`; the tiles are uniform offsets from it
        uint8_t* Yl = Y + (int64_t)mod * Np * Mp + ybase;
#pragma unroll
        for (int i = 0; i < W::FM; ++i)
#pragma unroll
            for (int jj = 0; jj < W::FN; ++jj) {
                const int64_t tofs = (int64_t)(jj * 32) * Mp + i * 32;
                store_tile(Yl + tofs, acc[i][jj], md, inv, lane >> 5);
                __builtin_amdgcn_sched_barrier(0);      // one accumulator's temporaries at a time
            }
        // no drain here: the stores share the vector-memory counter with the
        // copies, and "at most N outstanding" with stores among them still
        // means the copies older than the N most recent operations have
        // landed (copies complete in order among themselves), so the waits
        // stay sufficient; they only wait longer while stores are pending
    }
    // the copies run ahead of the last step: let them land before the
    // workgroup's LDS is released
    wait_vm_all();
}

// ---------------------------------------------------------------------------
// Stage 4: reconstruction, rounding and epilogue.  K 32-bit limbs hold M_N
// (M_N < 2^(32 K)).
// ---------------------------------------------------------------------------

// One entry: the limb sums L (exact), the quotient estimate f; C' in
// two's complement, its magnitude rounded into P components, the epilogue.
template <int P, int K>
__device__ __forceinline__ void crt_finish_entry(const GemmArgs& g, double (&L)[K], double f, int N,
                                                 int e, int64_t i, int64_t j) {
    const double q = rint(f);
#pragma unroll
    for (int l = 0; l < K; ++l) L[l] = fma(-q, kCrtDev.Md[N][l], L[l]);
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
    limbs_to_components<P, K>(w, sg, e, comp);

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

// Rows of a reconstruction block (two columns of them) and the largest
// modulus count per level of the two-level reconstruction.
constexpr int kRec3Rows = 128;
constexpr int kRec3MaxN = 33;

// One level: S = sum_t y_t W_t with the cofactors W_t = M / m_t in K 32-bit
// limbs, limb sums L_l = sum_t y_t W_t[l] (each < 2^46), q = nearest integer
// to S / M, C' = S - q M.  The limb sums run on the matrix cores: with
// y' = y - 128 and b' = b - 128 (signed bytes) for the bytes b_tc of W_t
// (byte c of its limbs), sum_t y_t b_tc = Z_c + 128 (Y + B'_c), where
// Z_c = sum_t y'_t b'_tc is one INT8 product (digit column c x entry, the
// moduli as inner dimension; rows of moduli t >= N are zero), Y = sum_t y_t
// (byte sums) and B'_c = sum_t b'_tc (per N, from the host, folded into kc).
// So L_l = sum_q (Z_{4l+q} + 128 Y) 256^q + kc_l, every part an integer below
// 2^47, exact in binary64; q from S / M = sum_l L_l r_l with r_l = 2^(32 l) /
// M (S / M lies at least 0.003 from a half-integer, and the error of this sum
// is below 2^-45).  Block b takes rows 128 (b % (Mp / 128))
// .. + 127 of two columns; their N planes' bytes come into LDS by 16-byte
// direct-to-LDS copies.  Wave w forms entries 64 w .. 64 w + 63 in two groups
// of 32; lane L ends with entry 64 w + L (the two halves of the wave trade
// the limbs of opposite parity).
// Matrix-core limb sums for K limbs and NKB blocks of 32 moduli.
template <int K, int NKB>
struct LimbMfma {
    static constexpr int NCB = (4 * K + 31) / 32;     // blocks of 32 digit columns
    static constexpr int kCols = 32 * NCB, kMods = 32 * NKB;
};

// The cofactor bytes b'_tc of W_t = M_N / m_t in LDS, digit column major
// (bt[c][t], zero for t >= N; limb l is columns 4 l .. 4 l + 3), then this
// lane's A fragments: digit column 32 cb + L % 32, moduli 32 kb + 16 (L / 32)
// + 0..15.  Also waits for the caller's direct-to-LDS copies; ends on a
// barrier past which LDS is complete.
template <int K, int NKB>
__device__ __forceinline__ void cofactor_fragments(uint8_t* bt, int N, int tid,
                                                   v4i (&af)[LimbMfma<K, NKB>::NCB][NKB]) {
    using LM = LimbMfma<K, NKB>;
    const int lane = tid & 63, hi = lane >> 5;
#pragma unroll
    for (int o = 16 * tid; o < LM::kCols * LM::kMods; o += 16 * 256) *(v4i*)(bt + o) = v4i{0, 0, 0, 0};
    __syncthreads();
    const uint32_t* wrow = kCrtDev.W[N * (N - 1) / 2];
    for (int e = tid; e < N * K; e += 256) {
        const int t = e / K, l = e % K;
        const uint32_t w = wrow[t * kLimbs + l] ^ 0x80808080u;
#pragma unroll
        for (int q = 0; q < 4; ++q) bt[(4 * l + q) * LM::kMods + t] = (uint8_t)(w >> (8 * q));
    }
    wait_vm_all();
    __syncthreads();
#pragma unroll
    for (int cb = 0; cb < LM::NCB; ++cb)
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb)
            af[cb][kb] = *(const v4i*)(bt + (32 * cb + (lane & 31)) * LM::kMods + 32 * kb + 16 * hi);
}

// Limb sums L_l = sum_{t<N} y_t W_t[l] of entry 64 w + L for the residue
// bytes of N planes in LDS (plane t at ysl + 256 t, entry e at byte e; planes
// t >= N are read but masked).  Entries 64 w + 32 grp + L % 32 of the two
// groups are the columns of the B fragments; the two halves of the wave
// then trade limbs of opposite parity so that lane L holds entry 64 w + L.
template <int K, int NKB>
__device__ __forceinline__ void limb_sums(const uint8_t* ysl, const v4i (&af)[LimbMfma<K, NKB>::NCB][NKB],
                                          int N, int tid, const double* __restrict__ kcs, double (&L)[K]) {
    using LM = LimbMfma<K, NKB>;
    constexpr int NCB = LM::NCB;
    const int lane = tid & 63, wave = tid >> 6, hi = lane >> 5;
    v16i acc[2][NCB];
    uint32_t ysum[2];
#pragma unroll
    for (int grp = 0; grp < 2; ++grp) {
        const int eb = 64 * wave + 32 * grp + (lane & 31);
        uint32_t sum = 0u;
        v4i bf[NKB];
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb) {
            uint32_t w4[4] = {0u, 0u, 0u, 0u};
#pragma unroll
            for (int jj = 0; jj < 16; ++jj) {
                const int t = 32 * kb + 16 * hi + jj;
                const uint32_t y = ysl[t * 2 * kRec3Rows + eb];
                w4[jj / 4] |= (t < N ? y : 0u) << (8 * (jj % 4));
            }
#pragma unroll
            for (int d = 0; d < 4; ++d) sum = __builtin_amdgcn_sad_u8(w4[d], 0u, sum);
            bf[kb] = v4i{(int)(w4[0] ^ 0x80808080u), (int)(w4[1] ^ 0x80808080u), (int)(w4[2] ^ 0x80808080u),
                         (int)(w4[3] ^ 0x80808080u)};
        }
        ysum[grp] = sum;
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            acc[grp][cb] = v16i{0};
#pragma unroll
            for (int kb = 0; kb < NKB; ++kb)
                acc[grp][cb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af[cb][kb], bf[kb], acc[grp][cb], 0, 0, 0);
        }
    }
    // this lane's limbs of each group: value 4 v + q of column block cb is
    // digit column 32 cb + 8 v + 4 (L / 32) + q, so limb 8 cb + 2 v + L / 32
    double lh[2][4 * NCB];
#pragma unroll
    for (int grp = 0; grp < 2; ++grp) {
        const uint32_t yt = ysum[grp] + (uint32_t)__shfl_xor((int)ysum[grp], 32, 64);
        const double yk = 128.0 * 16843009.0 * (double)yt;         // 128 Y (1 + 256 + 256^2 + 256^3)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int le = 8 * cb + 2 * v;               // even limb; this lane's is le + hi
                if (le >= K) continue;
                const double kc = hi ? (le + 1 < K ? kcs[le + 1] : 0.0) : kcs[le];
                const v16i& a = acc[grp][cb];
                double z = fma((double)a[4 * v + 3], 256.0, (double)a[4 * v + 2]);
                z = fma(z, 256.0, (double)a[4 * v + 1]);
                z = fma(z, 256.0, (double)a[4 * v]);
                lh[grp][4 * cb + v] = z + yk + kc;
            }
    }
    // lanes L < 32 keep group 0 (entry 64 w + L), lanes L >= 32 group 1
    // (entry 64 w + L as well): trade the limbs of the other parity
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int le = 8 * cb + 2 * v;
            if (le >= K) continue;
            const double mine = hi ? lh[1][4 * cb + v] : lh[0][4 * cb + v];
            const double other = __shfl_xor(hi ? lh[0][4 * cb + v] : lh[1][4 * cb + v], 32, 64);
            L[le] = hi ? other : mine;
            if (le + 1 < K) L[le + 1] = hi ? mine : other;
        }
}

// Copies the residue bytes of `planes` planes for rows i0 .. i0 + 127 of
// columns j0, j0 + 1 into LDS (plane p at ys + 256 p: column 0's 128 bytes,
// then column 1's) with 16-byte direct-to-LDS copies, all in flight.
template <int MAXP>
__device__ __forceinline__ void stage_residue_bytes(uint8_t* ys, const uint8_t* Y, int planes, int64_t plane,
                                                    int64_t Mp, int64_t i0, int64_t j0, int64_t n, int tid) {
    constexpr int kChunks = MAXP * 2 * kRec3Rows / 16;
    const int lane = tid & 63;
    // chunk c = 256 u + tid: plane c / 16, column (c / 8) % 2, bytes 16 (c % 8) ..
    const int nch = planes * 2 * kRec3Rows / 16;
#pragma unroll
    for (int u = 0; u < (kChunks + 255) / 256; ++u) {
        const int c = 256 * u + tid;
        const int64_t col = j0 + ((c >> 3) & 1);
        if (c < nch && col < n)
            copy16_to_lds((const int8_t*)(Y + (int64_t)(c >> 4) * plane + col * Mp + i0 + 16 * (c & 7)),
                          (int8_t*)(ys + 16 * (c - lane)));
    }
}

// Block `blk` of the reconstruction: rows (blk % (Mp / 128)) 128 .. + 127
// of columns 2 (blk / (Mp / 128)) and the next.
template <int P, int K, int NKB>
__device__ __forceinline__ void crt_recombine_block(const GemmArgs& g, const int32_t* __restrict__ E,
                                                    const int32_t* __restrict__ F, const uint8_t* __restrict__ Y,
                                                    int N, int s, int64_t Mp, int64_t Np,
                                                    int64_t blk) {
    using LM = LimbMfma<K, NKB>;
    // room for 32 NKB planes: the fragments read every slot (bytes of planes
    // t >= N are stale and masked), which keeps the reads free of branches
    __shared__ __align__(16) uint8_t ys[32 * NKB * 2 * kRec3Rows];
    __shared__ __align__(16) uint8_t bt[LM::kCols * LM::kMods];
    const int64_t tiles = Mp / kRec3Rows;
    const int64_t i0 = (blk % tiles) * kRec3Rows, j0 = 2 * (blk / tiles);
    const int tid = threadIdx.x;
    stage_residue_bytes<kNumModuli>(ys, Y, N, Mp * Np, Mp, i0, j0, g.n, tid);
    v4i af[LM::NCB][NKB];
    cofactor_fragments<K, NKB>(bt, N, tid, af);
    double L[K];
    limb_sums<K, NKB>(ys, af, N, tid, kCrtDev.kc[N], L);
    const int64_t i = i0 + (tid & (kRec3Rows - 1)), j = j0 + tid / kRec3Rows;
    if (i >= g.m || j >= g.n) return;
    double f = 0.0;
#pragma unroll
    for (int l = 0; l < K; ++l) f = fma(L[l], kCrtDev.r[N][l], f);
    crt_finish_entry<P, K>(g, L, f, N, E[i] + F[j] - 14 * s, i, j);
}

template <int P, int K, int NKB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void crt_recombine_mfma_kernel(GemmArgs g, const int32_t* __restrict__ E,
                                                                 const int32_t* __restrict__ F,
                                                                 const uint8_t* __restrict__ Y, int N, int s,
                                                                 int64_t Mp, int64_t Np) {
    crt_recombine_block<P, K, NKB>(g, E, F, Y, N, s, Mp, Np, blockIdx.x);
}

// Two levels (digit integers cut into a high and a low half, A' = A_h 2^w +
// A_l with w = 7 SLO): the products hh = A_h B_h, ll = A_l B_l and
// ss = (A_h + A_l)(B_h + B_l) come as three sets of N residue planes and are
// reconstructed one after the other; then C' = hh 2^(2w) + (ss - hh - ll) 2^w
// + ll, formed exactly in 16 limbs (two's complement), and rounded as above.
constexpr int kLimbsC = 16;           // C' below 2^511: up to 32 digits

// c += sign * (x, sign-extended by ext) * 2^SH, modulo 2^512; K-limb x.
template <int SIGN, int SH, int K>
__device__ __forceinline__ void add_shifted(uint32_t (&c)[kLimbsC], const uint32_t (&x)[K], uint32_t ext) {
    constexpr int ws = SH / 32, bs = SH % 32;
    uint64_t carry = SIGN > 0 ? 0u : 1u;          // subtraction adds ~y + 1
#pragma unroll
    for (int d = 0; d < kLimbsC; ++d) {
        const int i = d - ws;
        const uint32_t cur = i < 0 ? 0u : (i < K ? x[i] : ext);
        const uint32_t prev = i - 1 < 0 ? 0u : (i - 1 < K ? x[i - 1] : ext);
        uint32_t y = bs == 0 ? cur : ((cur << bs) | (prev >> ((32 - bs) & 31)));
        if (SIGN < 0) y = ~y;
        const uint64_t t = (uint64_t)c[d] + y + carry;
        c[d] = (uint32_t)t;
        carry = t >> 32;
    }
}

// Block b takes rows 128 (b % (Mp / 128)) .. + 127 of two columns; it first
// copies their 3N planes' bytes (256 per plane) into LDS with 16-byte
// direct-to-LDS copies, all in flight at once; the limb sums of each set run
// on the matrix cores as in the one-level kernel (the same N moduli in every
// set), and thread t finishes entry (row t % 128, column t / 128).

template <int P, int SLO, int NKB>
__device__ __forceinline__ void crt_recombine3_block(const GemmArgs& g, const int32_t* __restrict__ E,
                                                     const int32_t* __restrict__ F,
                                                     const uint8_t* __restrict__ Y, int N, int s, int64_t Mp,
                                                     int64_t Np, int64_t blk) {
    constexpr int K = 8;                          // each partial below 2^255 (N <= 33)
    constexpr int w = 7 * SLO;
    using LM = LimbMfma<K, NKB>;
    // the last set's fragments read 32 NKB plane slots from 2N on
    __shared__ __align__(16) uint8_t ys[(2 * kRec3MaxN + 32 * NKB) * 2 * kRec3Rows];
    __shared__ __align__(16) uint8_t bt[LM::kCols * LM::kMods];
    const int64_t tiles = Mp / kRec3Rows;
    const int64_t i0 = (blk % tiles) * kRec3Rows, j0 = 2 * (blk / tiles);
    const int tid = threadIdx.x;
    stage_residue_bytes<3 * kRec3MaxN>(ys, Y, 3 * N, Mp * Np, Mp, i0, j0, g.n, tid);
    v4i af[LM::NCB][NKB];
    cofactor_fragments<K, NKB>(bt, N, tid, af);
    const int64_t i = i0 + (tid & (kRec3Rows - 1)), j = j0 + tid / kRec3Rows;
    uint32_t c[kLimbsC];
#pragma unroll
    for (int l = 0; l < kLimbsC; ++l) c[l] = 0u;
    static_for<3>([&](auto setc) __attribute__((always_inline)) {
        constexpr int set = decltype(setc)::value;     // 0: hh, 1: ll, 2: ss
        double L[K];
        limb_sums<K, NKB>(ys + set * N * 2 * kRec3Rows, af, N, tid, kCrtDev.kc[N], L);
        double f = 0.0;
#pragma unroll
        for (int l = 0; l < K; ++l) f = fma(L[l], kCrtDev.r[N][l], f);
        const double q = rint(f);
        uint32_t x[K];
        int64_t carry = 0;
#pragma unroll
        for (int l = 0; l < K; ++l) {
            const int64_t v = (int64_t)fma(-q, kCrtDev.Md[N][l], L[l]) + carry;
            x[l] = (uint32_t)v;
            carry = v >> 32;
        }
        const uint32_t ext = carry < 0 ? 0xffffffffu : 0u;
        if constexpr (set == 0) {
            add_shifted<+1, 2 * w, K>(c, x, ext);
            add_shifted<-1, w, K>(c, x, ext);
        } else if constexpr (set == 1) {
            add_shifted<+1, 0, K>(c, x, ext);
            add_shifted<-1, w, K>(c, x, ext);
        } else {
            add_shifted<+1, w, K>(c, x, ext);
        }
    });
    if (i >= g.m || j >= g.n) return;
    double sg = 1.0;
    if (c[kLimbsC - 1] >> 31) {
        uint64_t c1 = 1;
#pragma unroll
        for (int l = 0; l < kLimbsC; ++l) {
            const uint64_t t = (uint64_t)(~c[l]) + c1;
            c[l] = (uint32_t)t;
            c1 = t >> 32;
        }
        sg = -1.0;
    }
    double comp[P];
    limbs_to_components<P, kLimbsC>(c, sg, E[i] + F[j] - 14 * s, comp);
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

template <int P, int SLO, int NKB>
__global__ __launch_bounds__(256) void crt_recombine3_kernel(GemmArgs g, const int32_t* __restrict__ E,
                                                             const int32_t* __restrict__ F,
                                                             const uint8_t* __restrict__ Y, int N,
                                                             int s, int64_t Mp, int64_t Np) {
    crt_recombine3_block<P, SLO, NKB>(g, E, F, Y, N, s, Mp, Np, blockIdx.x);
}

// ---------------------------------------------------------------------------
// The four stages over a batch of problems (CrtBatchItem: each problem's
// arguments, workspace regions and first block per stage).  A block finds
// its problem by binary search over the block prefixes and runs the single
// call's block body on it; every problem has the same N moduli, s digits and
// levels (one, or two for QD: 3 N planes), and 128 x 128 product tiles.
// ---------------------------------------------------------------------------

// Stage 2: per problem (Kp / 64) (Mp / 16 + Np / 16) blocks, the k segment
// fastest, op(A)'s row blocks first.  SETS = 3: two levels (QD), halves of
// shi and s - shi digits.
template <int P, int NG, int SETS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void crt_residue_batch_kernel(
    const CrtBatchItem* __restrict__ items, int64_t count, CrtWeights wa, CrtWeights wb, int s, int N, int shi) {
    const int64_t bid = blockIdx.x;
    const CrtBatchItem& it = items[crt_batch_find(items, count, bid, 1)];
    const int64_t local = bid - it.b[1], segs = it.Kp / kTileK, ra = it.Mp / kResRows;
    const int64_t seg = local % segs, rb = local / segs;
    const bool second = rb >= ra;
    const GemmArgs& g = it.g;
    const ResOperand o = second ? ResOperand{g.B, g.tb ? 1 : g.ldb, g.tb ? g.ldb : 1, g.sb, g.n, it.F, it.RB, it.Np}
                                : ResOperand{g.A, g.ta ? g.lda : 1, g.ta ? 1 : g.lda, g.sa, g.m, it.E, it.RA, it.Mp};
    const CrtWeights* __restrict__ wt = second ? &wb : &wa;
    const int lane = threadIdx.x & 63;
    v4i bw[SETS][NG];
    float mf[NG], invm[NG];
#pragma unroll
    MPG_CRT_WEIGHT_FRAGMENTS(wt, shi, lane, bw, mf, invm)
    crt_residue_block<P, NG, SETS>(o, bw, mf, invm, g.k, s, N, it.Kp, seg, second ? rb - ra : rb);
}

// Stage 3: per problem (Mp / 128) (Np / 128) tiles times `groups` workgroups
// of `mods` of its `planes` planes each (plane t: modulus t % N); the tile
// fastest, row tiles before column tiles.  Block b works on XCD b % 8's
// range, so a problem's tiles share an L2.
__global__ __launch_bounds__(320, 2) void crt_mfma_batch_kernel(const CrtBatchItem* __restrict__ items,
                                                                int64_t count, int N, int planes, int mods,
                                                                CrtXcdRanges xr) {
    const int x = (int)(blockIdx.x % kXcds);
    const int64_t bid = xr.xcd[x] + blockIdx.x / kXcds;
    if (bid >= xr.xcd[x + 1]) return;
    const CrtBatchItem& it = items[crt_batch_find(items, count, bid, 2)];
    const int64_t local = bid - it.b[2], tms = it.Mp / 128, tiles = tms * (it.Np / 128);
    const int64_t tile = local % tiles;
    const int mod0 = (int)(local / tiles) * mods;
    const int mod1 = mod0 + mods < planes ? mod0 + mods : planes;
    crt_mfma_block_cw<128, 128, 2, 2, 8>(it.RA, it.RB, it.Y, it.Mp, it.Np, it.Kp, N, tile % tms, tile / tms, mod0,
                                         mod1);
}

// Stage 4: per problem (Mp / 128) ceil(n / 2) blocks, as in the single call.
template <int P, int K, int NKB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void crt_recombine_batch_kernel(
    const CrtBatchItem* __restrict__ items, int64_t count, int N, int s) {
    const int64_t bid = blockIdx.x;
    const CrtBatchItem& it = items[crt_batch_find(items, count, bid, 3)];
    crt_recombine_block<P, K, NKB>(it.g, it.E, it.F, it.Y, N, s, it.Mp, it.Np, bid - it.b[3]);
}

// The same with two levels (QD): the three sets' planes follow one another.
template <int P, int SLO, int NKB>
__global__ __launch_bounds__(256) void crt_recombine3_batch_kernel(const CrtBatchItem* __restrict__ items,
                                                                   int64_t count, int N, int s) {
    const int64_t bid = blockIdx.x;
    const CrtBatchItem& it = items[crt_batch_find(items, count, bid, 3)];
    crt_recombine3_block<P, SLO, NKB>(it.g, it.E, it.F, it.Y, N, s, it.Mp, it.Np, bid - it.b[3]);
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

// Digit weights mod m_t (times u_t when `scaled`): byte p (digit p + 1) gets
// 128^(shi - 1 - p) for p < shi (the high half, or the whole integer when
// shi = s) and 128^(s - 1 - p) for the low half p >= shi.
CrtWeights crt_weights(int N, int s, int shi, bool scaled) {
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
        for (int half = 0; half < 2; ++half) {
            const int lo = half ? shi : 0, hi = half ? s : shi;   // bytes [lo, hi)
            int pw = u % m;                             // weight of byte hi - 1
            for (int p = hi - 1; p >= lo; --p) {
                W.w[t][p] = sym_byte(pw, m);
                pw = pw * (128 % m) % m;
            }
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

int launch_residues(int P, int sets, const ResOperand& a, const ResOperand& b, const CrtWeights& wa,
                    const CrtWeights& wb, int64_t k, int s, int N, int shi, int64_t Kp, hipStream_t st) {
    const int64_t rows = (a.Rp > b.Rp ? a.Rp : b.Rp) / kResRows;
    if (Kp / kTileK > 0x7fffffffLL || rows > 65535) return (int)hipErrorInvalidConfiguration;
    if (rows == 0 || Kp == 0) return 0;
    const dim3 grid((unsigned)(Kp / kTileK), (unsigned)rows, 2);
#define MPG_RES(PV, NGV, SV)                                                                     \
    hipLaunchKernelGGL((crt_residue_kernel<PV, NGV, SV>), grid, dim3(256), 0, st, a, b, wa, wb, k, s, N, \
                       shi, Kp)
    const bool two = N > 32;
    if (sets == 3) {                             // two levels: QD only
        if (two) MPG_RES(4, 2, 3); else MPG_RES(4, 1, 3);
    } else if (P == 2) {
        if (two) MPG_RES(2, 2, 1); else MPG_RES(2, 1, 1);
    } else if (P == 3) {
        if (two) MPG_RES(3, 2, 1); else MPG_RES(3, 1, 1);
    } else {
        if (two) MPG_RES(4, 2, 1); else MPG_RES(4, 1, 1);
    }
#undef MPG_RES
    return (int)hipGetLastError();
}

// Workgroups per output tile: with fewer tiles than workgroup slots on the
// chip the planes are shared out over several workgroups per tile (each
// writes its own planes), so that small products still fill the CUs.
struct CrtGroups {
    int groups, mods;                              // grid.y, planes per workgroup
};
CrtGroups crt_groups(int64_t tiles, int per_cu, int planes) {
    const int64_t slots = 256 * (int64_t)per_cu;
    int64_t g = tiles > 0 ? (slots + tiles - 1) / tiles : 1;
    g = g < 1 ? 1 : (g > planes ? planes : g);
    const int mods = (int)((planes + g - 1) / g);
    return {(planes + mods - 1) / mods, mods};
}

int launch_crt_mfma(int cfg, const int8_t* RA, const int8_t* RB, uint8_t* Y, int64_t Mp, int64_t Np,
                    int64_t Kp, int N, int Nmod, hipStream_t st) {
    const CrtConfig c = kCrt[cfg];
    const int64_t tiles = (Mp / c.bm) * (Np / c.bn);
    const int64_t grid = xcd_grid(tiles);
    if (grid > 0x7fffffffLL) return (int)hipErrorInvalidConfiguration;
    const CrtGroups gr = crt_groups(tiles, c.per_cu, N);
    const dim3 blocks((unsigned)grid, (unsigned)gr.groups);
    // ring depths: the LDS of one CU (160 KiB) holds one wide workgroup's
    // ring or two of the others
    if (cfg == 0)
        hipLaunchKernelGGL(crt_mfma_wide_kernel, blocks, dim3(256), 0, st, RA, RB, Y, Mp, Np, Kp, N, Nmod,
                           gr.mods);
    else if (cfg == 1)
        hipLaunchKernelGGL((crt_mfma_kernel<256, 128, 2, 2, 6>), blocks, dim3(256), 0, st, RA, RB, Y, Mp, Np,
                           Kp, N, Nmod, gr.mods);
    else
        hipLaunchKernelGGL((crt_mfma_kernel<128, 128, 2, 2, 8>), blocks, dim3(256), 0, st, RA, RB, Y, Mp, Np,
                           Kp, N, Nmod, gr.mods);
    return (int)hipGetLastError();
}

template <int P>
int launch_crt_recombine_p(int K, dim3 grid, hipStream_t st, const GemmArgs& g, const int32_t* E,
                           const int32_t* F, const uint8_t* Y, int N, int s, int64_t Mp, int64_t Np) {
#define MPG_REC(KV, NKB)                                                                                      \
    hipLaunchKernelGGL((crt_recombine_mfma_kernel<P, KV, NKB>), grid, dim3(256), 0, st, g, E, F, Y, N, s, Mp, \
                       Np)
    if (N > 2 * 32) return (int)hipErrorInvalidValue;
    switch (K) {
    case 4: MPG_REC(4, 1); break;
    case 6: MPG_REC(6, 1); break;
    case 8:
        if (N > 32) MPG_REC(8, 2); else MPG_REC(8, 1);
        break;
    default: MPG_REC(11, 2); break;
    }
#undef MPG_REC
    return (int)hipGetLastError();
}

constexpr int kBatchCfg = 2;        // 128 x 128 product tiles, two workgroups per CU

}  // namespace

size_t crt_batch_item_bytes(int64_t m, int64_t n, int64_t k, int planes) {
    return crt_layout(m, n, k, planes, kBatchCfg, kTileK).total;
}

int crt_batch_plan(const CrtPlan& pl, int64_t count, const GemmArgs* gs, void* ws, CrtBatchItem* items,
                   CrtBatchInfo* info) {
    const int N = pl.N;
    if (N <= 0 || N > kNumModuli || (pl.sets == 3 && N > kRec3MaxN)) return MPGEMM_ERR_UNSUPPORTED;
    const int planes = N * pl.sets;
    CrtBatchInfo in{};
    in.N = N;
    in.sets = pl.sets;
    in.shi = pl.shi;
    in.slo = pl.slo;
    int64_t tiles = 0;
    for (int64_t q = 0; q < count; ++q) {
        const CrtLayout L = crt_layout(gs[q].m, gs[q].n, gs[q].k, planes, kBatchCfg, kTileK);
        tiles += (L.Mp / 128) * (L.Np / 128);
    }
    const CrtGroups gr = crt_groups(tiles, kCrt[kBatchCfg].per_cu, planes);
    in.mods = gr.mods;
    in.groups = gr.groups;
    size_t off = 0;
    int64_t pos = 0, widest = 0;
    for (int x = 0; x < kXcds; ++x) {
        in.ranges.xcd[x] = in.blocks[2];
        for (int64_t q = x; q < count; q += kXcds, ++pos) {
            const GemmArgs& g = gs[q];
            const CrtLayout L = crt_layout(g.m, g.n, g.k, planes, kBatchCfg, kTileK);
            if (items) {
                char* base = (char*)ws + off;
                CrtBatchItem& it = items[pos];
                it.g = g;
                it.E = (int32_t*)(base + L.oE);
                it.F = (int32_t*)(base + L.oF);
                it.RA = (int8_t*)(base + L.oRA);
                it.RB = (int8_t*)(base + L.oRB);
                it.Y = (uint8_t*)(base + L.oY);
                it.Mp = L.Mp;
                it.Np = L.Np;
                it.Kp = L.Kp;
                for (int f = 0; f < 4; ++f) it.b[f] = in.blocks[f];
            }
            in.blocks[0] += L.Mp / 4 + L.Np / 4;
            in.blocks[1] += (L.Kp / kTileK) * (L.Mp / kResRows + L.Np / kResRows);
            in.blocks[2] += (L.Mp / 128) * (L.Np / 128) * gr.groups;
            in.blocks[3] += L.Mp / kRec3Rows * ((g.n + 1) / 2);
            off += L.total;                          // each total is a multiple of 256
        }
        widest = std::max<int64_t>(widest, in.blocks[2] - in.ranges.xcd[x]);
    }
    in.ranges.xcd[kXcds] = in.blocks[2];
    in.ws_bytes = off;
    in.grid2 = widest * kXcds;
    for (int f = 0; f < 4; ++f)
        if (in.blocks[f] > 0x7fffffffLL) return MPGEMM_ERR_UNSUPPORTED;
    if (in.grid2 > 0x7fffffffLL) return MPGEMM_ERR_UNSUPPORTED;
    if (info) *info = in;
    return 0;
}

int launch_crt_batch(int P, int s, const CrtBatchInfo& info, const CrtBatchItem* d_items, int64_t count,
                     hipStream_t st) {
    const int N = info.N, planes = N * info.sets;
    if (count <= 0) return 0;
    if (info.sets == 3 && P != 4) return (int)hipErrorInvalidValue;
    int rc;
    if ((rc = launch_row_exponents_batch(d_items, count, info.blocks[0], st))) return rc;
    const CrtWeights wa = crt_weights(N, s, info.shi, true);
    const CrtWeights wb = crt_weights(N, s, info.shi, false);
    const dim3 g1((unsigned)info.blocks[1]);
#define MPG_RESB(PV, NGV, SV)                                                                            \
    hipLaunchKernelGGL((crt_residue_batch_kernel<PV, NGV, SV>), g1, dim3(256), 0, st, d_items, count, wa, wb, s, \
                       N, info.shi)
    const bool two = N > 32;
    if (info.sets == 3) {
        if (two) MPG_RESB(4, 2, 3); else MPG_RESB(4, 1, 3);
    } else if (P == 2) {
        if (two) MPG_RESB(2, 2, 1); else MPG_RESB(2, 1, 1);
    } else if (P == 3) {
        if (two) MPG_RESB(3, 2, 1); else MPG_RESB(3, 1, 1);
    } else {
        if (two) MPG_RESB(4, 2, 1); else MPG_RESB(4, 1, 1);
    }
#undef MPG_RESB
    if ((rc = (int)hipGetLastError())) return rc;
    hipLaunchKernelGGL(crt_mfma_batch_kernel, dim3((unsigned)info.grid2), dim3(320), 0, st, d_items, count, N,
                       planes, info.mods, info.ranges);
    if ((rc = (int)hipGetLastError())) return rc;
    const dim3 g3((unsigned)info.blocks[3]);
    if (info.sets == 3) {
#define MPG_REC3B(SL, NKB) \
    hipLaunchKernelGGL((crt_recombine3_batch_kernel<4, SL, NKB>), g3, dim3(256), 0, st, d_items, count, N, s)
#define MPG_REC3BN(SL) \
    if (N > 32) MPG_REC3B(SL, 2); else MPG_REC3B(SL, 1)
        switch (info.slo) {
        case 12: MPG_REC3BN(12); break;
        case 13: MPG_REC3BN(13); break;
        case 14: MPG_REC3BN(14); break;
        case 15: MPG_REC3BN(15); break;
        default: MPG_REC3BN(16); break;
        }
#undef MPG_REC3BN
#undef MPG_REC3B
        return (int)hipGetLastError();
    }
    const int K = limbs_for(N);
#define MPG_RECB(PV, KV, NKB) \
    hipLaunchKernelGGL((crt_recombine_batch_kernel<PV, KV, NKB>), g3, dim3(256), 0, st, d_items, count, N, s)
#define MPG_RECBP(PV)                                      \
    switch (K) {                                           \
    case 4: MPG_RECB(PV, 4, 1); break;                     \
    case 6: MPG_RECB(PV, 6, 1); break;                     \
    case 8:                                                \
        if (N > 32) MPG_RECB(PV, 8, 2); else MPG_RECB(PV, 8, 1); \
        break;                                             \
    default: MPG_RECB(PV, 11, 2); break;                   \
    }
    if (P == 2) { MPG_RECBP(2) } else if (P == 3) { MPG_RECBP(3) } else { MPG_RECBP(4) }
#undef MPG_RECBP
#undef MPG_RECB
    return (int)hipGetLastError();
}

uint32_t crt_config_signature() {
    uint32_t h = 2166136261u;
    for (const CrtConfig& c : kCrt)
        for (int v : {c.bm, c.bn, c.per_cu}) h = fnv1a(h, v);
    return h;
}

int crt_default_config(int64_t m, int64_t n) {
    // rounds of resident workgroups times one workgroup's time (its tile
    // over its share of the planes, 32 taken as typical), with the measured
    // relative throughput of each tile shape per CU
    const double eff[kCrtConfigs] = {1.0, 0.9, 0.6};
    int best = 0;
    double best_cost = 0.0;
    for (int c = 0; c < kCrtConfigs; ++c) {
        const int64_t tiles = ((m + kCrt[c].bm - 1) / kCrt[c].bm) * ((n + kCrt[c].bn - 1) / kCrt[c].bn);
        const int64_t slots = 256 * kCrt[c].per_cu;
        const CrtGroups gr = crt_groups(tiles, kCrt[c].per_cu, 32);
        const double rounds = (double)((tiles * gr.groups + slots - 1) / slots);
        const double cost = rounds * kCrt[c].bm * kCrt[c].bn * gr.mods * kCrt[c].per_cu / eff[c];
        if (c == 0 || cost < best_cost) {
            best = c;
            best_cost = cost;
        }
    }
    return best;
}

// log2 of the largest |digit integer| with d digits: 64 (128^d - 1) / 127
static double log2_amax(int d) {
    return 6.0 + 7.0 * d + std::log1p(-std::ldexp(1.0, -7 * d)) / std::log(2.0) - std::log2(127.0);
}

// Smallest N whose modulus product exceeds 2^need, 0 if none.
static int moduli_for_bits(double need) {
    double bits = 0.0;
    for (int N = 1; N <= kNumModuli; ++N) {
        bits += std::log2((double)kModuli[N - 1]);
        if (bits > need) return N;
    }
    return 0;
}

int crt_moduli_count(int64_t k, int s) {
    if (k <= 0 || k > 131071 || s < 1 || s > kMaxCrtDigits) return 0;
    // max|C'| = k amax(s)^2, one bit for the sign, and a margin far above the
    // rounding of these logarithms
    return moduli_for_bits(1.0 + std::log2((double)k) + 2.0 * log2_amax(s) + 0.01);
}

CrtPlan crt_plan(int P, int64_t k, int s) {
    CrtPlan pl{0, 1, s, 0};
    pl.N = crt_moduli_count(k, s);
    if (pl.N > 0 || P != 4 || s < 2 * 12 + 1 || s > 2 * 16 || k <= 0 || k > 131071) return pl;
    // two levels: halves of shi and slo digits; the largest of the three
    // products is ss, with |A_h + A_l| <= amax(shi) + amax(slo)
    pl.sets = 3;
    pl.shi = (s + 1) / 2;
    pl.slo = s / 2;
    const double a = log2_amax(pl.shi), b = log2_amax(pl.slo);
    const double asum = a + std::log2(1.0 + std::exp2(b - a));
    pl.N = moduli_for_bits(1.0 + std::log2((double)k) + 2.0 * asum + 0.01);
    if (pl.N > 33) pl.N = 0;                      // partials kept in 8 limbs
    return pl;
}

int crt_products(int P, int64_t k, int s) {
    const CrtPlan pl = crt_plan(P, k, s);
    return pl.N * pl.sets;
}

size_t crt_workspace_bytes(int P, int64_t m, int64_t n, int64_t k, int s, int cfg) {
    const CrtPlan pl = crt_plan(P, k, s);
    if (pl.N == 0) return 0;
    return crt_layout(m, n, k, pl.N * pl.sets, cfg).total;
}

// Caller has validated arguments, the plan (crt_products > 0), the workspace
// size and handled quick returns / alpha == 0 / k == 0.
int launch_crt(int P, int s, int cfg, const GemmArgs& g, void* ws, hipStream_t st) {
    const CrtPlan pl = crt_plan(P, g.k, s);
    const int N = pl.N;
    if (N == 0) return (int)hipErrorInvalidValue;
    const CrtLayout L = crt_layout(g.m, g.n, g.k, N * pl.sets, cfg);
    char* base = (char*)ws;
    int32_t* E = (int32_t*)(base + L.oE);
    int32_t* F = (int32_t*)(base + L.oF);
    int8_t* RA = (int8_t*)(base + L.oRA);
    int8_t* RB = (int8_t*)(base + L.oRB);
    uint8_t* Y = (uint8_t*)(base + L.oY);
    const int64_t a_rs = g.ta ? g.lda : 1, a_ls = g.ta ? 1 : g.lda;
    const int64_t b_rs = g.tb ? 1 : g.ldb, b_ls = g.tb ? g.ldb : 1;
    const CrtWeights wa = crt_weights(N, s, pl.shi, true);
    const CrtWeights wb = crt_weights(N, s, pl.shi, false);
    int rc;
    uint64_t* MX = (uint64_t*)(base + L.oMX);
    if ((rc = launch_row_exponents(g.A, a_rs, a_ls, g.m, L.Mp, g.B, b_rs, b_ls, g.n, L.Np, g.k, E, F, MX,
                                   st)))
        return rc;
    const ResOperand oa{g.A, a_rs, a_ls, g.sa, g.m, E, RA, L.Mp};
    const ResOperand ob{g.B, b_rs, b_ls, g.sb, g.n, F, RB, L.Np};
    if ((rc = launch_residues(P, pl.sets, oa, ob, wa, wb, g.k, s, N, pl.shi, L.Kp, st))) return rc;
    if ((rc = launch_crt_mfma(cfg, RA, RB, Y, L.Mp, L.Np, L.Kp, N * pl.sets, N, st))) return rc;
    if (pl.sets == 3) {
        if (N > kRec3MaxN) return (int)hipErrorInvalidValue;
        const int64_t blocks = L.Mp / kRec3Rows * ((g.n + 1) / 2);
        if (blocks > 0x7fffffffLL) return (int)hipErrorInvalidConfiguration;
        const dim3 grid((unsigned)blocks);
#define MPG_REC3(SL, NKB)                                                                                    \
    hipLaunchKernelGGL((crt_recombine3_kernel<4, SL, NKB>), grid, dim3(256), 0, st, g, E, F, Y, N, s, L.Mp, \
                       L.Np)
#define MPG_REC3N(SL) \
    if (N > 32) MPG_REC3(SL, 2); else MPG_REC3(SL, 1)
        switch (pl.slo) {
        case 12: MPG_REC3N(12); break;
        case 13: MPG_REC3N(13); break;
        case 14: MPG_REC3N(14); break;
        case 15: MPG_REC3N(15); break;
        default: MPG_REC3N(16); break;
        }
#undef MPG_REC3N
#undef MPG_REC3
        return (int)hipGetLastError();
    }
    const int64_t blocks = L.Mp / kRec3Rows * ((g.n + 1) / 2);
    if (blocks > 0x7fffffffLL) return (int)hipErrorInvalidConfiguration;
    const dim3 grid((unsigned)blocks);
    const int K = limbs_for(N);
    if (P == 2) return launch_crt_recombine_p<2>(K, grid, st, g, E, F, Y, N, s, L.Mp, L.Np);
    if (P == 3) return launch_crt_recombine_p<3>(K, grid, st, g, E, F, Y, N, s, L.Mp, L.Np);
    return launch_crt_recombine_p<4>(K, grid, st, g, E, F, Y, N, s, L.Mp, L.Np);
}

}  // namespace mpg

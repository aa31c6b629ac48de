// exact_round.hpp -- rounding an exact multi-limb integer into P binary64
// components, shared by the two split forms' recombination kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpg {

// Components c_0..c_{P-1} of w 2^e (w: K-limb magnitude, sign sg): c_0 = RN
// of the value, then RN of the exact remainder, and so on (ties to even).
// Branch-free: the top nonzero limb and the two below it are gathered by
// selects into a 96-bit window, normalised by its leading zeros; its top 53
// bits are the significand, then the guard bit, the rest and all lower limbs
// the sticky bit.  Values below 2^53 need no case of their own: the window
// then reaches below bit 0, where everything reads as zero.
template <int P, int K>
__device__ __forceinline__ void limbs_to_components(uint32_t (&w)[K], double sg, int e, double* c) {
#pragma unroll
    for (int q = 0; q < P; ++q) {
        // one ascending pass: at the top nonzero limb L, hi/mid/lo = limbs
        // L, L-1, L-2 and below = OR of limbs 0..L-3 (run holds that OR)
        int L = -1;
        uint32_t hi = 0u, mid = 0u, lo = 0u, below = 0u, run = 0u;
#pragma unroll
        for (int l = 0; l < K; ++l) {
            const bool nz = w[l] != 0u;
            L = nz ? l : L;
            hi = nz ? w[l] : hi;
            mid = nz ? (l >= 1 ? w[l - 1] : 0u) : mid;
            lo = nz ? (l >= 2 ? w[l - 2] : 0u) : lo;
            below = nz ? run : below;
            if (l >= 2) run |= w[l - 2];
        }
        const int z = __clz(hi | 1u);                   // leading zeros of hi (nonzero when L >= 0)
        const uint64_t hm = ((uint64_t)hi << 32) | mid;
        // (hi:mid:lo) << z: the top 64 bits and the 32 left over
        const uint64_t win = (z == 0) ? hm : ((hm << z) | (uint64_t)(lo >> (32 - z)));
        const uint32_t rest = lo << z;
        const int h = 32 * L + 31 - z;                  // top set bit
        const int sh = h - 52;                          // exponent of the significand's last bit
        uint64_t v = win >> 11;
        const bool guard = ((win >> 10) & 1u) != 0u;
        const bool sticky = (win & 0x3ffu) != 0u || rest != 0u || below != 0u;
        const bool up = guard && (sticky || (v & 1u));
        v += up ? 1u : 0u;
        c[q] = (L < 0) ? 0.0 : sg * ldexp((double)v, sh + e);
        if (q == P - 1) break;
        // remainder: the bits below sh; after rounding up, 2^sh minus them
        // with the sign flipped (a value below 2^53 leaves nothing): limbs
        // below sh / 32 whole, limb sh / 32 its low sh % 32 bits, none above
        const int sl = sh >> 5;                         // floor(sh / 32); negative below 2^53
        const uint32_t part = (1u << (sh & 31)) - 1u;
        uint32_t mask[K];
#pragma unroll
        for (int l = 0; l < K; ++l) {
            mask[l] = (l < sl) ? 0xffffffffu : (l == sl) ? part : 0u;
            w[l] &= mask[l];
        }
        uint32_t carry = 1u;
#pragma unroll
        for (int l = 0; l < K; ++l) {
            const uint64_t t = (uint64_t)(~w[l]) + carry;
            const uint32_t nl = (uint32_t)t & mask[l];
            carry = (uint32_t)(t >> 32);
            w[l] = up ? nl : w[l];
        }
        sg = up ? -sg : sg;
    }
}

}  // namespace mpg

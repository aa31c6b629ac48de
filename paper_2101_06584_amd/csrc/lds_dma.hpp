// lds_dma.hpp -- device helpers shared by the INT8 matrix-core kernels: the
// swizzled 64-byte-row LDS tile layout fed by 16-byte direct-to-LDS copies,
// the counter waits that order those copies, and compile-time loops.
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

namespace mpg {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

static constexpr int kTileK = 64;          // k bytes per pipeline step (and k-tile width)

template <int N, typename F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {   // f(0), ..., f(N - 1) as constants
    static_for_impl<N>(f, std::make_integer_sequence<int, N>{});
}

// LDS offset of 16-byte chunk c (0..3) of tile row r (64-byte rows).
__device__ __forceinline__ int swz(int r, int c) { return r * kTileK + ((c ^ ((r >> 2) & 3)) << 4); }

// Wait until at most N vector-memory operations of this wave are pending and
// its LDS reads are done, then meet the other waves; a compiler barrier too.
template <int N>
__device__ __forceinline__ void wait_vm_barrier() {
    static_assert(N >= 0 && N <= 63, "vmcnt range");
    asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" ::"n"(N) : "memory");
}

__device__ __forceinline__ void wait_vm_all() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Wait for this wave's LDS reads, then meet the other waves (no wait on its
// vector-memory operations: its global stores stay in flight).
__device__ __forceinline__ void wait_lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// One 16-byte direct-to-LDS copy: lane L of the wave writes LDS bytes
// [lds + 16 L, lds + 16 L + 16) (lds uniform across the wave).
__device__ __forceinline__ void copy16_to_lds(const int8_t* g, int8_t* lds) {
    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)g,
                                     (__attribute__((address_space(3))) void*)lds, 16, 0, 0);
}

}  // namespace mpg

// Small device helpers shared by the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace jac {

template <typename R, int V>
struct alignas(16) Chunk {
    R v[V];
};

// Typed access at a byte offset from a (wave-uniform) base pointer, so the
// compiler can use the scalar-base + 32-bit vector-offset addressing form.
template <typename X>
__device__ __forceinline__ const X &at(const void *base, uint32_t byte_off) {
    return *reinterpret_cast<const X *>(reinterpret_cast<const char *>(base) + byte_off);
}
template <typename X>
__device__ __forceinline__ X &at_mut(void *base, uint32_t byte_off) {
    return *reinterpret_cast<X *>(reinterpret_cast<char *>(base) + byte_off);
}

// 16-byte store with the non-temporal hint (the line is not kept in the
// caches on its way to memory).
template <typename X>
__device__ __forceinline__ void store_nt16(X *p, const X &v) {
    static_assert(sizeof(X) == 16, "16-byte stores only");
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    u32x4 t;
    __builtin_memcpy(&t, &v, 16);
    __builtin_nontemporal_store(t, reinterpret_cast<u32x4 *>(p));
}

// Whole-wave lane shifts through DPP (wave_shr:1 / wave_shl:1).  All 64
// lanes must be active.
// shift_up: lane i receives src of lane i-1; lane 0 keeps `old`.
__device__ __forceinline__ float shift_up(float old, float src) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(src),
                                                      0x138, 0xf, 0xf, false));
}
// shift_down: lane i receives src of lane i+1; lane 63 keeps `old`.
__device__ __forceinline__ float shift_down(float old, float src) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(src),
                                                      0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ double shift_up(double old, double src) {
    const long long o = __double_as_longlong(old), s = __double_as_longlong(src);
    const int lo = __builtin_amdgcn_update_dpp((int)o, (int)s, 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(s >> 32), 0x138, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double shift_down(double old, double src) {
    const long long o = __double_as_longlong(old), s = __double_as_longlong(src);
    const int lo = __builtin_amdgcn_update_dpp((int)o, (int)s, 0x130, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(s >> 32), 0x130, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Shifts within each 16-lane row of the wave through DPP (row_shr:1 /
// row_shl:1).  All 64 lanes must be active.
// row_shift_up: lane i receives src of lane i-1 of its row; the row's first
// lane keeps `old`.
__device__ __forceinline__ float row_shift_up(float old, float src) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(src),
                                                      0x111, 0xf, 0xf, false));
}
// row_shift_down: lane i receives src of lane i+1 of its row; the row's last
// lane keeps `old`.
__device__ __forceinline__ float row_shift_down(float old, float src) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(src),
                                                      0x101, 0xf, 0xf, false));
}
__device__ __forceinline__ double row_shift_up(double old, double src) {
    const long long o = __double_as_longlong(old), s = __double_as_longlong(src);
    const int lo = __builtin_amdgcn_update_dpp((int)o, (int)s, 0x111, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(s >> 32), 0x111, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double row_shift_down(double old, double src) {
    const long long o = __double_as_longlong(old), s = __double_as_longlong(src);
    const int lo = __builtin_amdgcn_update_dpp((int)o, (int)s, 0x101, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(s >> 32), 0x101, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Deterministic wave-wide FP64 sum (fixed xor-butterfly order).
__device__ __forceinline__ double wave_sum(double a) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
    return a;
}

// Workgroup renumbering for the 8 XCDs (each with its own L2): the hardware
// deals workgroups round-robin, so physical workgroup p runs on XCD p % 8.
// The returned logical numbering gives each XCD one contiguous range, so
// work items with adjacent logical numbers share an L2.
__device__ __forceinline__ int xcd_logical_block(int p, int nblocks) {
    const int q = nblocks >> 3, rem = nblocks & 7;
    const int x = p & 7;
    return x * q + (x < rem ? x : rem) + (p >> 3);
}

}  // namespace jac

// Device helpers shared by the GPU kernels of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lnf {

// Map a workgroup id onto a tile id so that the workgroups one XCD receives
// (the dispatcher deals them out round-robin, id mod 8) form one contiguous
// range of tiles.  Neighbouring tiles then run on the same XCD and their
// overlapping halos are served by that XCD's L2 instead of HBM.
__device__ __forceinline__ int xcd_tile(int b, int total)
{
    constexpr int kX = 8;
    const int q = total / kX, rem = total % kX;
    const int xcd = b % kX, idx = b / kX;
    return xcd * q + min(xcd, rem) + idx;
}

// The thread index for a tile of a loop that runs several tiles per
// workgroup: through an empty asm, so that the values a tile derives from it
// are computed per tile instead of being hoisted out of the loop, where they
// would stay live (and spill) across all of it.  Kernels that run one tile
// pass threadIdx.x itself.
__device__ __forceinline__ int tile_tid()
{
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    return tid;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

// ---- buffer resources -------------------------------------------------------
// A raw buffer resource holds a 64-bit base and a byte size in SGPRs, so the
// per-lane address is a 32-bit byte offset (no 64-bit VALU address math), and
// any access at or beyond `bytes` is dropped by the hardware.
using rsrc_t = __amdgpu_buffer_rsrc_t;
using lds_void_t = __attribute__((address_space(3))) void;

__device__ __forceinline__ rsrc_t make_rsrc(const void* base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                             0x00020000);
}

template <typename T>
__device__ __forceinline__ uint32_t buffer_load(rsrc_t r, uint32_t voff);
template <>
__device__ __forceinline__ uint32_t buffer_load<uint8_t>(rsrc_t r, uint32_t voff)
{
    return __builtin_amdgcn_raw_buffer_load_b8(r, voff, 0, 0);
}
template <>
__device__ __forceinline__ uint32_t buffer_load<uint16_t>(rsrc_t r, uint32_t voff)
{
    return __builtin_amdgcn_raw_buffer_load_b16(r, voff, 0, 0);
}

// Output stores are non-temporal (cache policy bit 1, "nt" on gfx950): every
// output voxel is written once and not read again by the kernel, so its lines
// stream through L2 instead of evicting the input rows that neighbouring
// tiles' halos still need.  On the 512^3 MEAN9 benchmark at r = 3 the reads
// per launch (FETCH_SIZE) fell from 432 to 357 MB and the rate rose by 10-15 %.
constexpr int kStoreNT = 2;

template <typename T>
__device__ __forceinline__ void buffer_store(uint32_t v, rsrc_t r, uint32_t voff, uint32_t soff);
template <>
__device__ __forceinline__ void buffer_store<uint8_t>(uint32_t v, rsrc_t r, uint32_t voff,
                                                      uint32_t soff)
{
    __builtin_amdgcn_raw_buffer_store_b8((uint8_t)v, r, voff, soff, kStoreNT);
}
template <>
__device__ __forceinline__ void buffer_store<uint16_t>(uint32_t v, rsrc_t r, uint32_t voff,
                                                       uint32_t soff)
{
    __builtin_amdgcn_raw_buffer_store_b16((uint16_t)v, r, voff, soff, kStoreNT);
}

// Direct buffer -> LDS load of one element per lane (LDS DMA).  The element is
// zero-extended to 32 bits and written to LDS at dst + 4 * lane, where dst is
// wave-uniform; the load bypasses VGPRs and completes asynchronously (vmcnt).
template <typename T>
__device__ __forceinline__ void buffer_load_lds(rsrc_t r, void* dst_wave, uint32_t voff);
template <>
__device__ __forceinline__ void buffer_load_lds<uint8_t>(rsrc_t r, void* dst_wave, uint32_t voff)
{
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_void_t*)dst_wave, 1, voff, 0, 0, 0);
}
template <>
__device__ __forceinline__ void buffer_load_lds<uint16_t>(rsrc_t r, void* dst_wave, uint32_t voff)
{
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_void_t*)dst_wave, 2, voff, 0, 0, 0);
}

// LDS DMA of two adjacent elements per lane (the byte offset must be a multiple
// of 2 * sizeof(T)): a uint16 pair fills the 32-bit LDS word, a uint8 pair
// lands zero-extended in its low 16 bits.
template <typename T>
__device__ __forceinline__ void buffer_load_lds_pair(rsrc_t r, void* dst_wave, uint32_t voff);
template <>
__device__ __forceinline__ void buffer_load_lds_pair<uint8_t>(rsrc_t r, void* dst_wave,
                                                              uint32_t voff)
{
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_void_t*)dst_wave, 2, voff, 0, 0, 0);
}
template <>
__device__ __forceinline__ void buffer_load_lds_pair<uint16_t>(rsrc_t r, void* dst_wave,
                                                               uint32_t voff)
{
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_void_t*)dst_wave, 4, voff, 0, 0, 0);
}

// Wait for this wave's outstanding vector-memory operations (including LDS DMA).
__device__ __forceinline__ void wait_vmem() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Workgroup barrier that orders LDS traffic only.  __syncthreads() also
// fences global memory, which makes every wave wait for all its outstanding
// loads and stores (vmcnt 0) first; here only this wave's LDS operations are
// waited for, so global loads, stores and LDS DMA stay in flight across it.
// The empty asm statements keep the compiler from moving memory accesses
// across the barrier.
__device__ __forceinline__ void barrier_lds()
{
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Wait until at most N of this wave's vector-memory operations are outstanding.
// They retire in issue order (loads, stores and LDS DMA alike), so every
// operation issued before the last N has then completed.
template <int N>
__device__ __forceinline__ void wait_vmem_le()
{
    static_assert(N >= 0 && N <= 63, "vmcnt is a 6-bit counter");
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// round(S / d) for an odd divisor d < 2^20, in two instructions: one fp64
// fma forms S * (1/d) + 2^52 with a single rounding.  Between 2^52 and 2^53
// the fp64 spacing is 1, so that rounding is to the nearest integer, and the
// low 32 bits of the result's encoding are that integer (the mantissa of
// 2^52 + q is q).  S/d is never a half-integer (odd d), so it lies at least
// 1/(2d) from every rounding boundary, while S * fl(1/d) differs from S/d by
// less than S/d * 2^-53 < 2^-21 <= 1/(2d) for S < 2^32: the nearest integer
// of S * fl(1/d) is the correctly rounded S/d.
__device__ __forceinline__ uint32_t round_div_odd(uint32_t s, double inv_d)
{
    const double t = __builtin_fma((double)s, inv_d, 4503599627370496.0);  // + 2^52
    return (uint32_t)__builtin_bit_cast(uint64_t, t);
}

}  // namespace lnf

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

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

// round(S / d) for an odd divisor d, as trunc(S * (1/d) + 1/2) in fp64.
// (2S + d) / (2d) is never an integer (odd over even), so it lies at least
// 1/(2d) from every integer, while the fp64 error is below 2^-52 * S/d; with
// S < 2^30 and d < 2^14 the truncation is therefore exact.
__device__ __forceinline__ uint32_t round_div_odd(uint32_t s, double inv_d)
{
    return (uint32_t)__builtin_fma((double)s, inv_d, 0.5);
}

}  // namespace lnf

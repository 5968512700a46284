// MINVAR9 tile body at the paper's cluster geometry (cubes, diagonal offset
// r): the per-plane cluster tile of plane_tile.h.  Shared by the
// single-volume kernel and the multi-volume batch kernel.
#pragma once

#include "plane_tile.h"

namespace lnf {

template <int R>
using MV9Shape = PTShape<R, R, kClusterBox, kRuleMinVar9>;
template <int R, typename T>
using MV9Smem = PTSmem<R, R, kClusterBox, kRuleMinVar9, T>;

// dn = n, invn = 1/n.
template <int R, typename T, bool GATE>
__device__ __forceinline__ void minvar9_tile(MV9Smem<R, T>& sm, const T* __restrict__ in,
                                             T* __restrict__ out, Geom g, int x0, int y0, int z0,
                                             int z1, uint32_t gate, double dn, double invn)
{
    plane_tile<R, R, kClusterBox, kRuleMinVar9, T, GATE>(sm, in, out, g, x0, y0, z0, z1, gate, dn,
                                                         invn);
}

}  // namespace lnf

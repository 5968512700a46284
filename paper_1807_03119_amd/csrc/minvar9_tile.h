// MINVAR9 tile body at the paper's cluster geometry (cubes, diagonal offset
// r): the per-plane cluster tile of plane_tile.h.  Shared by the
// single-volume kernel and the multi-volume batch kernel.
#pragma once

#include "plane_tile.h"

namespace lnf {

// WT: the wide-tile variant (64 x 16 outputs, 512 threads, up to r = 3).
template <int R, bool WT = false>
using MV9Shape = PTShape<R, R, kClusterBox, kRuleMinVar9, WT>;
template <int R, typename T, bool WT = false>
using MV9Smem = PTSmem<R, R, kClusterBox, kRuleMinVar9, T, WT>;

// dn = n, invn = 1/n.
template <int R, typename T, bool GATE, bool WT = false>
__device__ __forceinline__ void minvar9_tile(MV9Smem<R, T, WT>& sm, const T* __restrict__ in,
                                             T* __restrict__ out, Geom g, int x0, int y0, int z0,
                                             int z1, uint32_t gate, double dn, double invn,
                                             int tid)
{
    plane_tile<R, R, kClusterBox, kRuleMinVar9, T, GATE, WT>(sm, in, out, g, x0, y0, z0, z1, gate,
                                                             dn, invn, tid);
}

}  // namespace lnf

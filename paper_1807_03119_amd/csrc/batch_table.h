// Job table of a batch launch (lnf_filter_batch): the volumes of each class of
// equal (radius, voxel type), their tile grids, and the device-side walk from a
// class tile index to a volume and its tile.  Shared by the batch kernels of
// batch.hip and the geometry-variant kernels of cluster.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_common.h"
#include "lnf.h"
#include "lnf_internal.h"

namespace lnf {

struct BatchJobDesc {
    const void* in;
    void* out;
    int nx, ny, nz;
    int tiles_x, tiles_y, zs, tile_begin;  // tile_begin: first tile in its class
    int pairs;                             // MEAN9 stages element pairs (mean9_pairs_ok)
};

// Queue mode keeps each XCD's counter in a 128-byte line of its own: device-scope
// atomics from several XCDs on one line serialise.
constexpr int kCounterStride = 32;  // unsigned words

struct BatchClass {
    int total;       // tiles in this class
    int njobs;       // jobs in this class
    int job_begin;   // index of its first job in `jobs`
    int variant;     // tile variant of the class
    // queue mode: tiles handed out so far from each XCD's range (uploaded as 0)
    unsigned next[kXcds * kCounterStride];
};

constexpr int kClasses = 2 * LNF_RADIUS_MAX;  // (radius, voxel type)

// A launchable class kernel: function, block size.
struct ClassKernel {
    const void* fn = nullptr;
    int threads = 0;
};

// The kernel of a geometry-variant class (cluster.hip): launched with the
// arguments (table, class, nullptr, nullptr, Geom{}, 0, 0, 0, total, gate, dn,
// inv) over `total` workgroups; TX x TY output tiles.
struct GeomClassKernel {
    ClassKernel k;
    int tx, ty;
    double dn, inv;
};
GeomClassKernel geometry_class_kernel(int rule, uint32_t geom, int dtype, int r);

// Class of a (radius, dtype) pair.
constexpr int batch_class(int r, int dtype) { return 2 * (r - 1) + (dtype == LNF_U16 ? 1 : 0); }

struct BatchTable {
    BatchClass c[kClasses];
    BatchJobDesc jobs[LNF_BATCH_MAX];
};

// Job of class tile t: the last job whose first tile is <= t (uniform per
// workgroup, so these are scalar loads).
__device__ __forceinline__ const BatchJobDesc& job_of(const BatchTable* tab, const BatchClass& c,
                                                      int t)
{
    int lo = c.job_begin, hi = c.job_begin + c.njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab->jobs[mid].tile_begin <= t) lo = mid;
        else hi = mid - 1;
    }
    return tab->jobs[lo];
}

// Runs body(job, x0, y0, z0, z1, tid) on tiles of class `cls` with TX x TY
// output tiles.  Grid mode: workgroup b takes class tile b (XCD-aware order).
// Queue mode (the grid is the resident workgroups, not the tiles): the class's
// tiles are cut into one contiguous range per XCD, as xcd_tile does, so
// neighbouring tiles, which share halo rows, run on one XCD and its L2
// (workgroups reach the XCDs round-robin by id).  The workgroups of an XCD deal
// all but about one round of its range out among themselves by stride; the
// rest they take one tile at a time from the range's counter, and then take
// what is left of the other ranges from their counters in turn.  tile_tid is
// the thread index; s_t is one LDS word.
template <int TX, int TY, bool QUEUE, typename F>
__device__ __forceinline__ void for_class_tiles(BatchTable* tab, int cls, int* s_t, F&& body)
{
    const int total = tab->c[cls].total;
    auto run = [&](int t, int tid) {
        const BatchJobDesc d = job_of(tab, tab->c[cls], t);
        const int local = t - d.tile_begin;
        const int bx = local % d.tiles_x;
        const int rest = local / d.tiles_x;
        const int by = rest % d.tiles_y;
        const int bz = rest / d.tiles_y;
        const int z0 = bz * d.zs;
        body(d, bx * TX, by * TY, z0, min(z0 + d.zs, d.nz), tid);
    };
    if constexpr (!QUEUE) {
        run(xcd_tile(blockIdx.x, total), (int)threadIdx.x);
    } else {
        const int home = (int)(blockIdx.x % kXcds), w = (int)(blockIdx.x / kXcds);
        const int q = total / kXcds, rem = total % kXcds;
        for (int h = 0; h < kXcds; ++h) {
            const int x = (home + h) % kXcds;
            const int lo = x * q + min(x, rem), n = q + (x < rem ? 1 : 0);
            const int gx = ((int)gridDim.x - x + kXcds - 1) / kXcds;  // workgroups of XCD x
            const int ns = gx > 0 ? max(n / gx - 1, 0) * gx : 0;       // tiles dealt by stride
            if (h == 0)
                for (int i = w; i < ns; i += gx) run(lo + i, tile_tid());
            for (;;) {
                if (threadIdx.x == 0) *s_t = (int)atomicAdd(&tab->c[cls].next[x * kCounterStride], 1u);
                __syncthreads();
                const int i = ns + *s_t;
                __syncthreads();  // every thread has read s_t before it is written again
                if (i >= n) break;
                run(lo + i, tile_tid());
            }
        }
    }
}

}  // namespace lnf

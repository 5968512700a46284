// MINVAR9: every voxel becomes the rounded mean of the least-variance cluster
// among the nine of the paper's method (cluster geometry: Section "Our Method"
// and the nine-cluster figure).  The selection rule is not in the paper: the
// variance numerator n*q_k - s_k^2 (s_k = sum, q_k = sum of squares, n voxels)
// is minimised, the lowest cluster index winning ties.
//
// Each cluster statistic is a box sum B = box^3 E (and Q = box^3 E^2) taken at
// the cluster's centre, so the kernel computes B and Q once for every centre
// position it needs and gathers the nine values per output voxel.  Sums of
// squares are kept in fp64, which holds every integer below 2^53 exactly: the
// largest one here is n*q <= 729 * 729 * 65535^2 < 2^52, so n*q - s^2 is exact.
#include "device_common.h"
#include "lnf_internal.h"

namespace lnf {
namespace {

constexpr int kThreads = 256;

// Output tile 32 (x) x 8 (y), streaming `zs` slices in z.  Per input slice:
//   1. stage the raw (32+4r) x (8+4r) slice tile in LDS, prefetch the next;
//   2. x-pass: box sums of E and E^2 over 2r+1 columns for every cluster-centre
//      column of the (32+2r) wide region, on all 8+4r rows;
//   3. y-pass + z-window: each thread owns up to NCI centre columns of the
//      (32+2r) x (8+2r) region; it forms the 2D box sums and keeps a register
//      ring of the last 2r+1 of them to slide box_z, and writes the finished
//      3D sums B, Q of slice zi-r into an LDS ring of 2r+1 planes;
//   4. gather: once planes zi-3r .. zi-r exist, each thread takes the nine
//      (B, Q) pairs of output (x, y, zi-2r), selects, rounds and stores.
template <int R, typename T, bool GATE>
__global__ __launch_bounds__(kThreads) void minvar9_planes_32x8(
    const T* __restrict__ in, T* __restrict__ out, Geom g, int zs, int tiles_x, int tiles_y,
    int total, uint32_t gate, double dn, double invn)
{
    constexpr int TX = 32, TY = 8, H = 2 * R;
    constexpr int LX = TX + 2 * H, LY = TY + 2 * H;  // raw tile
    constexpr int GX = TX + 2 * R, GY = TY + 2 * R;  // cluster-centre region
    constexpr int NRAW = LX * LY;
    constexpr int NLOAD = (NRAW + kThreads - 1) / kThreads;
    constexpr int NFULL = NRAW / kThreads;
    constexpr int NXP = LY * GX;
    constexpr int NXI = (NXP + kThreads - 1) / kThreads;
    constexpr int NCOL = GX * GY;
    constexpr int NCI = (NCOL + kThreads - 1) / kThreads;
    constexpr int P = 2 * R + 1;  // ring period and number of planes
    static_assert(TX * TY == kThreads, "one output column per thread");

    __shared__ uint32_t s_raw[NRAW];
    __shared__ uint32_t s_bx[NXP];
    __shared__ double s_qx[NXP];
    __shared__ uint32_t s_bs[P][NCOL];
    __shared__ double s_bq[P][NCOL];

    const int tid = threadIdx.x;
    const int tile = xcd_tile(blockIdx.x, total);
    const int bx = tile % tiles_x;
    const int rest = tile / tiles_x;
    const int by = rest % tiles_y;
    const int bz = rest / tiles_y;
    const int x0 = bx * TX, y0 = by * TY, z0 = bz * zs;
    const int z1 = min(z0 + zs, g.nz);
    const size_t plane = (size_t)g.nx * g.ny;

    int off[NLOAD];
#pragma unroll
    for (int i = 0; i < NLOAD; ++i) {
        const int e = min(tid + i * kThreads, NRAW - 1);
        const int row = e / LX, col = e - row * LX;
        off[i] = clampi(y0 - H + row, 0, g.ny - 1) * g.nx + clampi(x0 - H + col, 0, g.nx - 1);
    }
    const bool last_ok = tid + (NLOAD - 1) * kThreads < NRAW;
    uint32_t v[NLOAD];
    auto load = [&](int zi) {
        const T* base = in + (size_t)clampi(zi, 0, g.nz - 1) * plane;
#pragma unroll
        for (int i = 0; i < NLOAD; ++i) v[i] = base[off[i]];
    };

    uint32_t pring[P][NCI];
    double qring[P][NCI];
    uint32_t bsum[NCI];
    double qsum[NCI];
#pragma unroll
    for (int j = 0; j < NCI; ++j) {
        bsum[j] = 0;
        qsum[j] = 0.0;
#pragma unroll
        for (int u = 0; u < P; ++u) {
            pring[u][j] = 0;
            qring[u][j] = 0.0;
        }
    }

    const int ox = tid % TX, oy = tid / TX;
    const int ns = (z1 - z0) + 2 * H;
    load(z0 - H);
    for (int kb = 0; kb < ns; kb += P) {
#pragma unroll
        for (int u = 0; u < P; ++u) {
            const int k = kb + u;
            if (k >= ns) break;
            // 1. stage
#pragma unroll
            for (int i = 0; i < NLOAD; ++i)
                if (i < NFULL || last_ok) s_raw[tid + i * kThreads] = v[i];
            if (k + 1 < ns) load(z0 - H + k + 1);
            __syncthreads();

            // 2. x-pass: centre column c of the region is raw column c + r
#pragma unroll
            for (int j = 0; j < NXI; ++j) {
                const int it = tid + j * kThreads;
                if (it < NXP) {
                    const int row = it / GX, col = it - row * GX;
                    const uint32_t* rp = s_raw + row * LX + col;
                    uint32_t b = 0;
                    double q = 0.0;
#pragma unroll
                    for (int t = 0; t <= 2 * R; ++t) {
                        const uint32_t e = rp[t];
                        b += e;
                        q = __builtin_fma((double)e, (double)e, q);
                    }
                    s_bx[it] = b;
                    s_qx[it] = q;
                }
            }
            __syncthreads();

            // 3. y-pass + z-window; region row gy covers x-pass rows gy .. gy+2r
#pragma unroll
            for (int j = 0; j < NCI; ++j) {
                const int it = tid + j * kThreads;
                if (it < NCOL) {
                    const int gy = it / GX, gx = it - gy * GX;
                    uint32_t b = 0;
                    double q = 0.0;
#pragma unroll
                    for (int t = 0; t <= 2 * R; ++t) {
                        b += s_bx[(gy + t) * GX + gx];
                        q += s_qx[(gy + t) * GX + gx];
                    }
                    bsum[j] += b - pring[u][j];
                    qsum[j] += q - qring[u][j];
                    pring[u][j] = b;
                    qring[u][j] = q;
                    s_bs[u][it] = bsum[j];  // 3D sums centred on slice z0 - 2r + k - r
                    s_bq[u][it] = qsum[j];
                }
            }
            __syncthreads();

            // 4. gather for output slice z = zi - 2r
            if (k >= 2 * H) {
                const int z = z0 + k - 2 * H;
                uint32_t best_s = 0;
                double best_v = 0.0;
#pragma unroll
                for (int kk = 0; kk < 9; ++kk) {
                    int dx = 0, dy = 0, slot = (u + R + 1) % P;  // plane of z
                    if (kk > 0) {
                        const int jj = kk - 1;
                        dx = (jj & 1) ? R : -R;
                        dy = (jj & 2) ? R : -R;
                        slot = (jj & 4) ? u : (u + 1) % P;  // z + r, z - r
                    }
                    const int idx = (oy + R + dy) * GX + (ox + R + dx);
                    const uint32_t s = s_bs[slot][idx];
                    const double ds = (double)s;
                    const double var = __builtin_fma(dn, s_bq[slot][idx], -ds * ds);
                    if (kk == 0 || var < best_v) {
                        best_v = var;
                        best_s = s;
                    }
                }
                uint32_t o = round_div_odd(best_s, invn);
                if (GATE && o < gate) o = 0;
                const int x = x0 + ox, y = y0 + oy;
                if (x < g.nx && y < g.ny) out[(size_t)z * plane + (size_t)y * g.nx + x] = (T)o;
            }
        }
    }
}

template <int R, typename T>
hipError_t launch_planes(const void* in, void* out, Geom g, uint32_t gate, int zs, hipStream_t s)
{
    const int tiles_x = (g.nx + 31) / 32, tiles_y = (g.ny + 7) / 8;
    if (zs <= 0) zs = default_zs(tiles_x * tiles_y, g.nz, 2048);
    const int nzs = (g.nz + zs - 1) / zs;
    const int total = tiles_x * tiles_y * nzs;
    const int n = (2 * R + 1) * (2 * R + 1) * (2 * R + 1);
    const T* pin = static_cast<const T*>(in);
    T* pout = static_cast<T*>(out);
    if (gate)
        hipLaunchKernelGGL((minvar9_planes_32x8<R, T, true>), dim3(total), dim3(kThreads), 0, s,
                           pin, pout, g, zs, tiles_x, tiles_y, total, gate, (double)n, 1.0 / n);
    else
        hipLaunchKernelGGL((minvar9_planes_32x8<R, T, false>), dim3(total), dim3(kThreads), 0, s,
                           pin, pout, g, zs, tiles_x, tiles_y, total, gate, (double)n, 1.0 / n);
    return hipGetLastError();
}

template <typename T>
hipError_t dispatch_r(const void* in, void* out, int r, Geom g, uint32_t gate, TileCfg cfg,
                      hipStream_t s)
{
    switch (r) {
    case 1: return launch_planes<1, T>(in, out, g, gate, cfg.zs, s);
    case 2: return launch_planes<2, T>(in, out, g, gate, cfg.zs, s);
    case 3: return launch_planes<3, T>(in, out, g, gate, cfg.zs, s);
    case 4: return launch_planes<4, T>(in, out, g, gate, cfg.zs, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

int minvar9_variants() { return 1; }

void minvar9_tile_shape(int variant, int* tx, int* ty)
{
    (void)variant;
    *tx = 32;
    *ty = 8;
}

hipError_t launch_minvar9(const void* in, void* out, int dtype, int r, Geom g, uint32_t gate,
                          TileCfg cfg, hipStream_t s)
{
    if (dtype == LNF_U8) return dispatch_r<uint8_t>(in, out, r, g, gate, cfg, s);
    return dispatch_r<uint16_t>(in, out, r, g, gate, cfg, s);
}

}  // namespace lnf

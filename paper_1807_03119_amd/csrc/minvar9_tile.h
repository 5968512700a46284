// MINVAR9 tile body: one workgroup filters a 32 x 8 column of output voxels
// over the z-range [z0, z1).  Shared by the single-volume kernel and the
// persistent batch kernel.
//
// The selection rule is not in the paper (its cluster geometry is: Section
// "Our Method" and the nine-cluster figure): the variance numerator
// n*q_k - s_k^2 (s_k = sum, q_k = sum of squares, n voxels) is minimised, the
// lowest cluster index winning ties, and the winner's rounded mean is written.
// Each cluster statistic is a box sum B = box^3 E (and Q = box^3 E^2) at the
// cluster's centre, so B and Q are computed once per centre position and
// gathered nine times.  Sums of squares are fp64, exact for every integer below
// 2^53: the largest value here is n*q <= 729 * 729 * 65535^2 < 2^52.
//
// Per input slice:
//   1. stage the raw (32+4r) x (8+4r) slice tile in LDS (loads of slice k+1
//      are issued into registers before slice k is processed, and stay in
//      flight across the slice's LDS-only barriers);
//   2. x-pass: box sums of E and E^2 over 2r+1 columns for every cluster-centre
//      column of the (32+2r) wide region, on all 8+4r rows, as prefix-sum
//      differences over 8-wide row segments;
//   3. y-pass + z-window: each thread owns up to NCI centre columns of the
//      (32+2r) x (8+2r) region; it forms the 2D box sums and keeps a register
//      ring of the last 2r+1 of them to slide box_z, and writes the finished
//      3D sums B, Q of slice zi-r into an LDS ring of 2r+1 planes;
//   4. gather: once planes zi-3r .. zi-r exist, each thread takes the nine
//      (B, Q) pairs of output (x, y, zi-2r), selects, rounds and stores.
#pragma once

#include "device_common.h"
#include "lnf_internal.h"

namespace lnf {

template <int R>
struct MV9Shape {
    static constexpr int THREADS = 256;
    static constexpr int TX = 32, TY = 8, H = 2 * R;
    static constexpr int LX = TX + 2 * H, LY = TY + 2 * H;  // raw tile
    static constexpr int GX = TX + 2 * R, GY = TY + 2 * R;  // cluster-centre region
    static constexpr int NRAW = LX * LY;
    static constexpr int NLOAD = (NRAW + THREADS - 1) / THREADS;
    static constexpr int NFULL = NRAW / THREADS;
    static constexpr int NXP = LY * GX;
    static constexpr int XS = 8;                           // x-pass positions per thread
    static constexpr int NXS = (GX + XS - 1) / XS;         // x-pass segments per row
    static constexpr int LXP = NXS * XS + 2 * R;           // raw row pitch (tail padded)
    static_assert(LY * NXS <= THREADS, "x-pass: one thread per row segment");
    static constexpr int NCOL = GX * GY;
    static constexpr int NCI = (NCOL + THREADS - 1) / THREADS;
    static constexpr int P = 2 * R + 1;  // ring period and number of planes
    static_assert(TX * TY == THREADS, "one output column per thread");
};

template <int R>
struct MV9Smem {
    using S = MV9Shape<R>;
    double qx[S::NXP];
    double bq[S::P][S::NCOL];
    uint32_t raw[S::LY * S::LXP];
    uint32_t bx[S::NXP];
    uint32_t bs[S::P][S::NCOL];
};

template <int R, typename T, bool GATE>
__device__ __forceinline__ void minvar9_tile(MV9Smem<R>& sm, const T* __restrict__ in,
                                             T* __restrict__ out, Geom g, int x0, int y0, int z0,
                                             int z1, uint32_t gate, double dn, double invn)
{
    using S = MV9Shape<R>;
    constexpr int TX = S::TX, H = S::H, LX = S::LX, GX = S::GX, P = S::P;
    constexpr int kThreads = S::THREADS;
    const int tid = threadIdx.x;
    const size_t plane = (size_t)g.nx * g.ny;
    const uint32_t pbytes = (uint32_t)(plane * sizeof(T));

    uint32_t off[S::NLOAD];
    int lidx[S::NLOAD];  // padded LDS index of each staged element
#pragma unroll
    for (int i = 0; i < S::NLOAD; ++i) {
        const int e = min(tid + i * kThreads, S::NRAW - 1);
        const int row = e / LX, col = e - row * LX;
        off[i] = (uint32_t)(clampi(y0 - H + row, 0, g.ny - 1) * g.nx +
                            clampi(x0 - H + col, 0, g.nx - 1)) * (uint32_t)sizeof(T);
        lidx[i] = row * S::LXP + col;
    }
    const bool last_ok = tid + (S::NLOAD - 1) * kThreads < S::NRAW;
    uint32_t v[S::NLOAD];
    auto load = [&](int zi) {
        const rsrc_t rs = make_rsrc(in + (size_t)clampi(zi, 0, g.nz - 1) * plane, pbytes);
#pragma unroll
        for (int i = 0; i < S::NLOAD; ++i) v[i] = buffer_load<T>(rs, off[i]);
    };

    uint32_t pring[P][S::NCI];
    double qring[P][S::NCI];
    uint32_t bsum[S::NCI];
    double qsum[S::NCI];
#pragma unroll
    for (int j = 0; j < S::NCI; ++j) {
        bsum[j] = 0;
        qsum[j] = 0.0;
#pragma unroll
        for (int u = 0; u < P; ++u) {
            pring[u][j] = 0;
            qring[u][j] = 0.0;
        }
    }

    // the tail of each padded raw row is read by the last x-pass segment but
    // only feeds discarded positions; keep it defined
    if constexpr (S::LXP > LX) {
        constexpr int PAD = S::LXP - LX;
        for (int i = tid; i < S::LY * PAD; i += kThreads) sm.raw[(i / PAD) * S::LXP + LX + i % PAD] = 0;
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
            for (int i = 0; i < S::NLOAD; ++i)
                if (i < S::NFULL || last_ok) sm.raw[lidx[i]] = v[i];
            if (k + 1 < ns) load(z0 - H + k + 1);
            barrier_lds();

            // 2. x-pass: centre column c of the region is raw column c + r; each
            //    thread runs prefix sums over an 8-wide segment (+2r halo)
            {
                const int row = tid / S::NXS, seg = tid % S::NXS;
                if (row < S::LY) {
                    constexpr int W = S::XS + 2 * R;
                    const uint32_t* rp = sm.raw + row * S::LXP + seg * S::XS;
                    uint32_t cb[W];
                    double cq[W];
                    cb[0] = rp[0];
                    cq[0] = (double)rp[0] * (double)rp[0];
#pragma unroll
                    for (int i = 1; i < W; ++i) {
                        const uint32_t e = rp[i];
                        cb[i] = cb[i - 1] + e;
                        cq[i] = __builtin_fma((double)e, (double)e, cq[i - 1]);
                    }
#pragma unroll
                    for (int m = 0; m < S::XS; ++m) {
                        const int c = seg * S::XS + m;
                        if (c < GX) {
                            sm.bx[row * GX + c] = cb[m + 2 * R] - (m ? cb[m - 1] : 0u);
                            sm.qx[row * GX + c] = cq[m + 2 * R] - (m ? cq[m - 1] : 0.0);
                        }
                    }
                }
            }
            barrier_lds();

            // 3. y-pass + z-window; region row gy covers x-pass rows gy .. gy+2r
#pragma unroll
            for (int j = 0; j < S::NCI; ++j) {
                const int it = tid + j * kThreads;
                if (it < S::NCOL) {
                    const int gy = it / GX, gx = it - gy * GX;
                    uint32_t b = 0;
                    double q = 0.0;
#pragma unroll
                    for (int t = 0; t <= 2 * R; ++t) {
                        b += sm.bx[(gy + t) * GX + gx];
                        q += sm.qx[(gy + t) * GX + gx];
                    }
                    bsum[j] += b - pring[u][j];
                    qsum[j] += q - qring[u][j];
                    pring[u][j] = b;
                    qring[u][j] = q;
                    sm.bs[u][it] = bsum[j];  // 3D sums centred on slice z0 - 2r + k - r
                    sm.bq[u][it] = qsum[j];
                }
            }
            barrier_lds();

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
                    const uint32_t s = sm.bs[slot][idx];
                    const double ds = (double)s;
                    const double var = __builtin_fma(dn, sm.bq[slot][idx], -ds * ds);
                    if (kk == 0 || var < best_v) {
                        best_v = var;
                        best_s = s;
                    }
                }
                uint32_t o = round_div_odd(best_s, invn);
                if (GATE && o < gate) o = 0;
                const int x = x0 + ox, y = y0 + oy;
                if (x < g.nx && y < g.ny) {
                    const rsrc_t wr = make_rsrc(out + (size_t)z * plane, pbytes);
                    buffer_store<T>(o, wr, (uint32_t)(y * g.nx + x) * (uint32_t)sizeof(T), 0);
                }
            }
        }
    }
}

}  // namespace lnf

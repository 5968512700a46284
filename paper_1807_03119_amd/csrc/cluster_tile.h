// Cluster-gather tile for the geometry variants of the nine-cluster filter:
// cubic clusters or eq. 2's cross clusters (three axis lines of 2r+1 voxels
// through the centre, the centre counted on each line), with the eight
// diagonal clusters at (+-D, +-D, +-D).  Both rules (MEAN9, MINVAR9).
//
// One workgroup filters a TX x TY column of output voxels over [z0, z1), in
// two steps per input slice:
//   - cluster sums G (and sums of squares Q for MINVAR9) at every cluster
//     centre of the (TX+2D) x (TY+2D) region, for the centre plane r slices
//     behind the newest input slice.  Cubes: x-line sums of the staged raw rows,
//     then column sums over 2r+1 rows, then a register ring sliding the z
//     window.  Crosses: the x-line and y-line through the centre (taken r
//     slices late from a register ring) plus the z-line, a running sum of the
//     centre column over the last 2r+1 slices;
//   - the planes of G (and Q) stay in an LDS ring of 2D+1 planes; once the
//     planes z-D .. z+D exist, each output voxel gathers its nine clusters and
//     applies the rule, rounding and gate.
// Sums of squares are fp64, exact below 2^53 (the largest is under 2^46).
#pragma once

#include "device_common.h"
#include "lnf_internal.h"

namespace lnf {

constexpr int kClusterBox = 0, kClusterCross = 1;
// rules of the tile
constexpr int kRuleMean9 = 0, kRuleMinVar9 = 1;

template <int R, int D, bool VAR>
struct CTDims {
    // LDS bytes of a TX x TY tile (the rings dominate)
    static constexpr long bytes(int tx, int ty)
    {
        const long gx = tx + 2 * D, gy = ty + 2 * D, ly = gy + 2 * R;
        const long nxs = (gx + 7) / 8, lxp = nxs * 8 + 2 * R;
        const long ncol = gx * gy, np = 2 * D + 1;
        return ly * lxp * 4 + ly * gx * (VAR ? 12 : 4) + np * ncol * (VAR ? 12 : 4);
    }
    static constexpr long kMax = 150 * 1024;  // leave room for the compiler's own LDS
    static constexpr int TX = bytes(32, 8) <= kMax ? 32 : bytes(16, 8) <= kMax ? 16 : 8;
    static constexpr int TY = bytes(TX, 8) <= kMax ? 8 : 4;
    static_assert(bytes(TX, TY) <= kMax, "cluster tile does not fit in LDS");
};

template <int R, int D, int SHAPE, bool VAR>
struct CTShape {
    static constexpr int THREADS = 256;
    static constexpr int TX = CTDims<R, D, VAR>::TX, TY = CTDims<R, D, VAR>::TY;
    static constexpr int H = R + D;                          // raw halo
    static constexpr int GX = TX + 2 * D, GY = TY + 2 * D;   // cluster-centre region
    static constexpr int LX = GX + 2 * R, LY = GY + 2 * R;   // raw tile
    static constexpr int NRAW = LX * LY;
    static constexpr int NLOAD = (NRAW + THREADS - 1) / THREADS;
    static constexpr int XS = 8;                             // x-pass centres per work item
    static constexpr int NXS = (GX + XS - 1) / XS;
    static constexpr int LXP = NXS * XS + 2 * R;             // raw row pitch (tail padded)
    static constexpr int NXW = LY * NXS;                     // x-pass work items
    static constexpr int NCOL = GX * GY;
    static constexpr int NCI = (NCOL + THREADS - 1) / THREADS;
    static constexpr int P = 2 * R + 1;                      // register-ring period
    static constexpr int NP = 2 * D + 1;                     // LDS planes kept for the gather
    static constexpr int M = 2 * R + 1;
    static constexpr int N = SHAPE == kClusterBox ? M * M * M : 3 * M;  // voxels per cluster
    static_assert(TX * TY <= THREADS, "one output column per thread");
};

template <int R, int D, int SHAPE, bool VAR>
struct CTSmem {
    using S = CTShape<R, D, SHAPE, VAR>;
    double qx[VAR ? S::LY * S::GX : 1];
    double gq[VAR ? S::NP : 1][VAR ? S::NCOL : 1];
    uint32_t raw[S::LY * S::LXP];
    uint32_t bx[S::LY * S::GX];
    uint32_t gs[S::NP][S::NCOL];
};

template <int R, int D, int SHAPE, int RULE, typename T, bool VAR = RULE == kRuleMinVar9>
__device__ __forceinline__ void cluster_tile(CTSmem<R, D, SHAPE, VAR>& sm,
                                             const T* __restrict__ in, T* __restrict__ out,
                                             Geom g, int x0, int y0, int z0, int z1,
                                             uint32_t gate)
{
    using S = CTShape<R, D, SHAPE, VAR>;
    constexpr int TX = S::TX, TY = S::TY, H = S::H, LX = S::LX, GX = S::GX, P = S::P;
    constexpr int NP = S::NP, THREADS = S::THREADS;
    const int tid = threadIdx.x;
    const size_t plane = (size_t)g.nx * g.ny;
    const uint32_t pbytes = (uint32_t)(plane * sizeof(T));

    // staging: each lane's raw elements, coordinates clamped into the volume
    uint32_t off[S::NLOAD];
    int lidx[S::NLOAD];
#pragma unroll
    for (int i = 0; i < S::NLOAD; ++i) {
        const int e = min(tid + i * THREADS, S::NRAW - 1);
        const int row = e / LX, col = e - row * LX;
        off[i] = (uint32_t)(clampi(y0 - H + row, 0, g.ny - 1) * g.nx +
                            clampi(x0 - H + col, 0, g.nx - 1)) * (uint32_t)sizeof(T);
        lidx[i] = row * S::LXP + col;
    }
    const bool last_ok = tid + (S::NLOAD - 1) * THREADS < S::NRAW;
    uint32_t v[S::NLOAD];
    auto load = [&](int zi) {
        const rsrc_t rs = make_rsrc(in + (size_t)clampi(zi, 0, g.nz - 1) * plane, pbytes);
#pragma unroll
        for (int i = 0; i < S::NLOAD; ++i) v[i] = buffer_load<T>(rs, off[i]);
    };
    // the padded tail of each raw row feeds only discarded x-pass outputs
    if constexpr (S::LXP > LX) {
        constexpr int PAD = S::LXP - LX;
        for (int i = tid; i < S::LY * PAD; i += THREADS)
            sm.raw[(i / PAD) * S::LXP + LX + i % PAD] = 0;
    }

    // z-window rings, per centre column owned by this thread
    constexpr int NR = SHAPE == kClusterBox ? 1 : 2;  // box: B; cross: centre value, x+y lines
    uint32_t ring[P][S::NCI][NR];
    double qring[VAR ? P : 1][S::NCI][NR];
    uint32_t zsum[S::NCI];
    double zsq[S::NCI];
#pragma unroll
    for (int j = 0; j < S::NCI; ++j) {
        zsum[j] = 0;
        zsq[j] = 0.0;
#pragma unroll
        for (int u = 0; u < P; ++u)
#pragma unroll
            for (int c = 0; c < NR; ++c) {
                ring[u][j][c] = 0;
                if constexpr (VAR) qring[u][j][c] = 0.0;
            }
    }

    const int ox = tid % TX, oy = tid / TX;
    const bool gathers = tid < TX * TY;
    const int ns = (z1 - z0) + 2 * H;  // input slices z0-H .. z1-1+H
    const double invn = 1.0 / S::N, inv9n = 1.0 / (9.0 * S::N);
    load(z0 - H);
    for (int kb = 0; kb < ns; kb += P) {
#pragma unroll
        for (int u = 0; u < P; ++u) {
            const int k = kb + u;
            if (k >= ns) break;
            // 1. stage slice k; prefetch slice k+1 into registers
#pragma unroll
            for (int i = 0; i < S::NLOAD; ++i)
                if (i < S::NLOAD - 1 || last_ok) sm.raw[lidx[i]] = v[i];
            if (k + 1 < ns) load(z0 - H + k + 1);
            barrier_lds();

            // 2. x-lines: sums over 2r+1 raw columns for every centre column
            for (int w = tid; w < S::NXW; w += THREADS) {
                const int row = w / S::NXS, seg = w % S::NXS;
                constexpr int W = S::XS + 2 * R;
                const uint32_t* rp = sm.raw + row * S::LXP + seg * S::XS;
                uint32_t cb[W];
                double cq[VAR ? W : 1];
                cb[0] = rp[0];
                if constexpr (VAR) cq[0] = (double)rp[0] * (double)rp[0];
#pragma unroll
                for (int i = 1; i < W; ++i) {
                    const uint32_t e = rp[i];
                    cb[i] = cb[i - 1] + e;
                    if constexpr (VAR) cq[i] = __builtin_fma((double)e, (double)e, cq[i - 1]);
                }
#pragma unroll
                for (int m = 0; m < S::XS; ++m) {
                    const int c = seg * S::XS + m;
                    if (c < GX) {
                        sm.bx[row * GX + c] = cb[m + 2 * R] - (m ? cb[m - 1] : 0u);
                        if constexpr (VAR) sm.qx[row * GX + c] = cq[m + 2 * R] - (m ? cq[m - 1] : 0.0);
                    }
                }
            }
            barrier_lds();

            // 3. cluster sums of centre plane zc = (slice k) - r into LDS slot zc mod NP
            const int slot = (k - R + 4 * NP) % NP;
#pragma unroll
            for (int j = 0; j < S::NCI; ++j) {
                const int it = tid + j * THREADS;
                if (it < S::NCOL) {
                    const int gy = it / GX, gx = it - gy * GX;
                    uint32_t G;
                    double Q = 0.0;
                    if constexpr (SHAPE == kClusterBox) {
                        uint32_t b = 0;
                        double q = 0.0;
#pragma unroll
                        for (int t = 0; t <= 2 * R; ++t) {
                            b += sm.bx[(gy + t) * GX + gx];
                            if constexpr (VAR) q += sm.qx[(gy + t) * GX + gx];
                        }
                        zsum[j] += b - ring[u][j][0];
                        ring[u][j][0] = b;
                        G = zsum[j];
                        if constexpr (VAR) {
                            zsq[j] += q - qring[u][j][0];
                            qring[u][j][0] = q;
                            Q = zsq[j];
                        }
                    } else {
                        // centre value and the x- and y-lines of this slice
                        const uint32_t e = sm.raw[(gy + R) * S::LXP + gx + R];
                        uint32_t xy = sm.bx[(gy + R) * GX + gx];
                        double xyq = 0.0;
                        if constexpr (VAR) xyq = sm.qx[(gy + R) * GX + gx];
#pragma unroll
                        for (int t = 0; t <= 2 * R; ++t) {
                            const uint32_t c = sm.raw[(gy + t) * S::LXP + gx + R];
                            xy += c;
                            if constexpr (VAR) xyq = __builtin_fma((double)c, (double)c, xyq);
                        }
                        zsum[j] += e - ring[u][j][0];  // z-line: centre column, last 2r+1 slices
                        ring[u][j][0] = e;
                        ring[u][j][1] = xy;
                        G = zsum[j] + ring[(u + P - R) % P][j][1];  // x+y lines, r slices back
                        if constexpr (VAR) {
                            const double eq = (double)e * (double)e;
                            zsq[j] += eq - qring[u][j][0];
                            qring[u][j][0] = eq;
                            qring[u][j][1] = xyq;
                            Q = zsq[j] + qring[(u + P - R) % P][j][1];
                        }
                    }
                    sm.gs[slot][it] = G;
                    if constexpr (VAR) sm.gq[slot][it] = Q;
                }
            }
            barrier_lds();

            // 4. gather for output slice z = zc - D, once planes z-D .. z+D exist
            if (k >= 2 * H && gathers) {
                const int z = z0 + k - 2 * H;
                const int s0 = (k - R - D + 4 * NP) % NP;       // plane z
                const int sm1 = (k - R - 2 * D + 4 * NP) % NP;  // plane z - D
                const int sp1 = slot;                           // plane z + D
                uint32_t o;
                if constexpr (!VAR) {
                    uint32_t tot = sm.gs[s0][(oy + D) * GX + ox + D];
#pragma unroll
                    for (int kk = 1; kk < 9; ++kk) {
                        const int jj = kk - 1;
                        const int cx = ox + ((jj & 1) ? 2 * D : 0);
                        const int cy = oy + ((jj & 2) ? 2 * D : 0);
                        tot += sm.gs[(jj & 4) ? sp1 : sm1][cy * GX + cx];
                    }
                    o = round_div_odd(tot, inv9n);
                } else {
                    const double dn = (double)S::N;
                    uint32_t best_s = 0;
                    double best_v = 0.0;
#pragma unroll
                    for (int kk = 0; kk < 9; ++kk) {
                        int idx = (oy + D) * GX + ox + D, sl = s0;
                        if (kk > 0) {
                            const int jj = kk - 1;
                            idx = (oy + ((jj & 2) ? 2 * D : 0)) * GX + ox + ((jj & 1) ? 2 * D : 0);
                            sl = (jj & 4) ? sp1 : sm1;
                        }
                        const uint32_t s = sm.gs[sl][idx];
                        const double ds = (double)s;
                        const double var = __builtin_fma(dn, sm.gq[sl][idx], -ds * ds);
                        if (kk == 0 || var < best_v) {
                            best_v = var;
                            best_s = s;
                        }
                    }
                    o = round_div_odd(best_s, invn);
                }
                if (o < gate) o = 0;
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

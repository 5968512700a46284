// Streaming MEAN9 tile body: one workgroup filters a TX x TY column of output
// voxels over the z-range [z0, z1).  Shared by the single-volume kernel and the
// persistent batch kernel.
//
// Arithmetic (paper, Section "Our Method", eqs. 2-3): the sum S over the nine
// clusters is box_x box_y box_z E + c_x c_y c_z E, with box = ones on [-r, r]
// and c = ones on [-2r, 2r] plus one more at the centre (the two diagonal
// clusters of an axis overlap there).  Everything is exact uint32.
//
// Pipeline per input slice k, in issue order within one iteration (one
// barrier per iteration):
//   - stores of the output slice finished in the previous iteration;
//   - LDS reads of everything the iteration consumes: this thread's raw row
//     segment of slice k and its px / qx column of slice k-1;
//   - y-pass of slice k-1: each thread owns one column and four rows, forms
//     P = box_y px and Q = c_y qx from prefix sums, and pushes them into a
//     register ring of the last 4r+2 slices; the ring keeps the running sums
//     B = sum of P over [z-r, z+r] and W = sum of Q over [z-2r, z+2r] for the
//     output slice z, two r behind the newest slice, and S = B + W + Q(z);
//     out = round(S / 9n) (fp64, exact), gate;
//   - LDS DMA: the raw (TX+4r) x (TY+4r) tile of slice k+PF is loaded straight
//     from HBM into LDS (one element per lane, zero-extended to 32 bits), its
//     coordinates clamped into the volume per lane; PF+1 raw buffers form a
//     ring, so each slice has PF iterations to arrive;
//   - x-pass of slice k: each thread takes an 8-wide row segment, forms prefix
//     sums over its 8+4r raw values and writes px = box_x E and qx = c_x E.
// px and qx are double-buffered, so the x-pass of slice k overlaps the y-pass
// of slice k-1.  Every iteration issues exactly NLOAD loads and YO stores (no
// branch around any of them: masked-off stores go to an offset the buffer's
// range check drops), so the wait for slice k+1 at the end of iteration k is
// a partial one that leaves the younger PF-1 iterations' operations in flight.
#pragma once

#include "device_common.h"
#include "lnf_internal.h"

namespace lnf {

#ifndef LNF_M9_PREFETCH
#define LNF_M9_PREFETCH 2
#endif

// PK: the raw tile is staged as element pairs, one 32-bit LDS word per pair
// (uint16: both halves; uint8: the low two bytes), loaded by one LDS DMA per
// lane.  That halves the DMA instructions and the LDS bytes of the staging and
// of the x-pass reads.  It needs an even nx (pairs never straddle a row end), a
// volume base aligned to a pair, and a tile whose halo stays inside the volume
// in x (a pair cannot be clamped element by element); tiles at an x face are
// staged element-wise.
template <int R, int TY, int TXW = 64, bool PK = false>
struct M9Shape {
    static constexpr int TX = TXW;
    static constexpr int YO = 4;                    // output rows per thread
    static constexpr int THREADS = TX * TY / YO;    // one thread per column x YO rows
    static constexpr int H = 2 * R;                 // halo: cluster radius + offset
    static constexpr int EPW = PK ? 2 : 1;          // raw elements per LDS word
    static constexpr int LXE = TX + 4 * R;          // raw elements per tile row
    static constexpr int LXW = LXE / EPW;           // LDS words holding them (LXE even)
    // Raw row pitch in words: padded to 4 mod 8, so that eight consecutive
    // rows start in eight different groups of four LDS banks (the x-pass reads
    // 16 bytes per lane, eight lanes per bank cycle).  The padding words repeat
    // the row's last word and are never used.
    static constexpr int LX = LXW + (12 - LXW % 8) % 8;
    static constexpr int LY = TY + 2 * H;
    static constexpr int NRAW = LX * LY;            // staged words per slice
    static constexpr int NLOAD = (NRAW + THREADS - 1) / THREADS;
    static constexpr int PXP = TX + 4;              // padded px/qx row pitch (words)
    static constexpr int D = 4 * R + 2;             // ring period (even)
    static constexpr int SEG = 8, NSEG = TX / SEG, SW = SEG + 4 * R;
    static constexpr int SWW = SW / EPW;            // words an x-pass segment reads
    static constexpr int XR = (LY + 7) / 8 * 8;     // x-pass row slots (multiple of 8)
    static constexpr int NPV = YO + 2 * R, NQV = YO + 4 * R;
    static constexpr int PF = LNF_M9_PREFETCH;       // slices staged ahead of the x-pass
    static constexpr int NRB = PF + 1;               // raw slice buffers (a ring)
    // vector-memory operations issued after a slice's loads, up to the wait
    // that needs that slice: PF-1 iterations of (NLOAD loads + YO stores)
    static constexpr int VMWAIT = (PF - 1) * (NLOAD + YO);
    static_assert(PF >= 1 && VMWAIT <= 63, "prefetch depth out of range");
    static_assert(XR * NSEG <= THREADS, "x-pass: one thread per row segment");
    static_assert(D % 2 == 0, "buffer parity must be static in the unrolled ring");
    static_assert(LX % 4 == 0 && (SEG / EPW) % 4 == 0, "x-pass reads 16-byte aligned rows");
    static_assert(SWW % 2 == 0 && LXE % 2 == 0, "x-pass reads whole 8-byte pieces");
};

// BOX: the box term alone (the paper's mean filter, eq. 4): no qx, no Q ring.
template <int R, int TY, int TXW = 64, bool PK = false, bool BOX = false>
struct M9Smem {
    using S = M9Shape<R, TY, TXW, PK>;
    uint32_t raw[S::NRB][S::NLOAD * S::THREADS];
    uint32_t px[2][S::LY * S::PXP];
    uint32_t qx[BOX ? 1 : 2][BOX ? 1 : S::LY * S::PXP];
};

// inv_div: 1/(9n), or 1/n with BOX.
template <int R, int TY, typename T, bool GATE, int TXW, bool PK, bool BOX = false>
__device__ __forceinline__ void mean9_tile_body(M9Smem<R, TY, TXW, PK, BOX>& sm,
                                                const T* __restrict__ in, T* __restrict__ out,
                                                Geom g, int x0, int y0, int z0, int z1,
                                                uint32_t gate, double inv9n)
{
    using S = M9Shape<R, TY, TXW, PK>;
    constexpr int H = S::H, LX = S::LX, D = S::D, TX = S::TX, PXP = S::PXP, YO = S::YO;
    constexpr int EPW = S::EPW;
    const int tid = threadIdx.x;
    // wave index as a scalar, so the LDS DMA destinations are scalar arithmetic
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const size_t plane = (size_t)g.nx * g.ny;
    const uint32_t pbytes = (uint32_t)(plane * sizeof(T));

    // byte offsets (within a slice) of the raw words this lane stages
    uint32_t off[S::NLOAD];
#pragma unroll
    for (int i = 0; i < S::NLOAD; ++i) {
        const int e = min(tid + i * S::THREADS, S::NRAW - 1);
        const int row = e / LX;
        // padding words re-read the row's last word: no extra cache lines
        const int col = min(e - row * LX, S::LXW - 1);
        const int gy = clampi(y0 - H + row, 0, g.ny - 1);
        const int gx = clampi(x0 - H + EPW * col, 0, g.nx - EPW);  // even when PK
        off[i] = (uint32_t)(gy * g.nx + gx) * (uint32_t)sizeof(T);
    }
    // every lane issues all NLOAD loads (lanes past the tile reload its last
    // word into unused LDS words), so the count per stage is fixed
    auto stage = [&](int zi, int slot) {
        const rsrc_t rs = make_rsrc(in + (size_t)clampi(zi, 0, g.nz - 1) * plane, pbytes);
#pragma unroll
        for (int i = 0; i < S::NLOAD; ++i) {
            if constexpr (PK)
                buffer_load_lds_pair<T>(rs, &sm.raw[slot][i * S::THREADS + wave * 64], off[i]);
            else
                buffer_load_lds<T>(rs, &sm.raw[slot][i * S::THREADS + wave * 64], off[i]);
        }
    };

    const int xq = tid % TX;
    // x-pass mapping: consecutive lanes take consecutive rows of one segment
    // (bank-conflict free with the padded pitch).  Row slots are padded to a
    // multiple of 8; surplus lanes and threads redo the last row or segment and
    // write the same values, so the x-pass needs no divergent branch.
    const int xrow = min(tid % S::XR, S::LY - 1);
    const int xseg = min(tid / S::XR, S::NSEG - 1);
    auto half = [](uint32_t w, int h) -> uint32_t {
        return h ? (w >> (8 * sizeof(T))) : (w & ((1u << (8 * sizeof(T))) - 1u));
    };
    // x-pass, part 1: this thread's raw row segment, read from LDS at the top
    // of the iteration so the reads overlap the y-pass
    uint32_t xw[S::SWW];
    auto xload = [&](int slot) {
        const uint32_t* rp = sm.raw[slot] + xrow * LX + xseg * (S::SEG / EPW);
#pragma unroll
        for (int i = 0; i < S::SWW; i += 4) {
            if (i + 4 <= S::SWW) {
                const uint4 t4 = *reinterpret_cast<const uint4*>(rp + i);
                xw[i] = t4.x;
                xw[i + 1] = t4.y;
                xw[i + 2] = t4.z;
                xw[i + 3] = t4.w;
            } else {
                const uint2 t2 = *reinterpret_cast<const uint2*>(rp + i);
                xw[i] = t2.x;
                xw[i + 1] = t2.y;
            }
        }
    };
    // x-pass, part 2: prefix sums over the segment, px and qx written to LDS;
    // el(i) is raw element i of the segment
    auto xsums = [&](int buf, auto el) {
        uint32_t pp[S::SEG], qq[S::SEG], c[S::SW];
        c[0] = el(0);
#pragma unroll
        for (int i = 1; i < S::SW; ++i) c[i] = c[i - 1] + el(i);
#pragma unroll
        for (int m = 0; m < S::SEG; ++m) {
            if constexpr (!BOX) qq[m] = c[m + 4 * R] - (m ? c[m - 1] : 0u) + el(m + 2 * R);
            pp[m] = c[m + 3 * R] - c[m + R - 1];
        }
        uint32_t* pd = sm.px[buf] + xrow * PXP + xseg * S::SEG;
#pragma unroll
        for (int m = 0; m < S::SEG; m += 4) {
            *reinterpret_cast<uint4*>(pd + m) = make_uint4(pp[m], pp[m + 1], pp[m + 2], pp[m + 3]);
            if constexpr (!BOX) {
                uint32_t* qd = sm.qx[buf] + xrow * PXP + xseg * S::SEG;
                *reinterpret_cast<uint4*>(qd + m) =
                    make_uint4(qq[m], qq[m + 1], qq[m + 2], qq[m + 3]);
            }
        }
    };
    auto xpass = [&](int buf) {
        if constexpr (PK) {
            xsums(buf, [&](int i) -> uint32_t { return half(xw[i / 2], i & 1); });
        } else {
            xsums(buf, [&](int i) -> uint32_t { return xw[i]; });
        }
    };

    // Value of px (Q = false) or qx (Q = true) at x-pass row `row`, column xq.
    auto xval = [&](int pb, bool q, int row) -> uint32_t {
        if constexpr (BOX) return sm.px[pb][row * PXP + xq];
        else return (q ? sm.qx[pb] : sm.px[pb])[row * PXP + xq];
    };

    // y-pass / ring ownership: column xq, rows yg*YO .. yg*YO+YO-1
    const int yg = tid / TX;
    const int xo = x0 + xq, ybase = y0 + yg * YO;
    const uint32_t voff = (uint32_t)((size_t)ybase * g.nx + xo) * (uint32_t)sizeof(T);
    const uint32_t rowb = (uint32_t)g.nx * (uint32_t)sizeof(T);
    // per-row store offsets; rows or columns outside the volume get the plane
    // size, which the range check of the store's buffer resource drops
    uint32_t soff[YO];
#pragma unroll
    for (int m = 0; m < YO; ++m)
        soff[m] = (xo < g.nx && ybase + m < g.ny) ? voff + (uint32_t)m * rowb : pbytes;

    uint32_t pr[D][YO], qr[D][YO], bacc[YO], wacc[YO];
#pragma unroll
    for (int m = 0; m < YO; ++m) {
        bacc[m] = wacc[m] = 0;
#pragma unroll
        for (int u = 0; u < D; ++u) pr[u][m] = qr[u][m] = 0;
    }

    // The y-pass of the first iteration reads px/qx buffer 1 before any x-pass
    // wrote it; zeros there push zeros into the (zero) ring, so the loop body
    // needs no branch.  Likewise the x-pass and the staging run
    // in every iteration (the extra ones at the end read clamped slices and
    // their results are never used).  The loop body is then one basic block
    // the compiler can interleave.
    for (int i = tid; i < S::LY * PXP; i += S::THREADS) {
        sm.px[1][i] = 0;
        if constexpr (!BOX) sm.qx[1][i] = 0;
    }
    const int ns = (z1 - z0) + 2 * H;  // input slices z0-2r .. z1-1+2r
    // the YO stores of output slice zo; zo < 0 stores to an empty buffer
    // resource (every access dropped), so each call issues exactly YO stores
    auto store_out = [&](int zo, const uint32_t(&o)[YO]) {
        const rsrc_t wr = make_rsrc(out + (size_t)max(zo, 0) * plane, zo >= 0 ? pbytes : 0u);
#pragma unroll
        for (int m = 0; m < YO; ++m) buffer_store<T>(o[m], wr, soff[m], 0u);
    };
    // prologue: slices 0 .. PF-1, each but the first preceded by YO (dropped)
    // stores so the operation pattern matches the loop's
    stage(z0 - H, 0);
#pragma unroll
    for (int p = 1; p < S::PF; ++p) {
        store_out(-1, bacc);
        stage(z0 - H + p, p);
    }
    wait_vmem_le<S::VMWAIT>();
    barrier_lds();
    // iteration k: x-pass of slice k, y-pass of slice k-1, z-window and output
    // of slice k-2 (the z-window work needs no LDS data, so it runs while the
    // iteration's LDS reads are in flight)
    const int nk = ns + 1;
    for (int kb = 0; kb <= nk; kb += D) {
#pragma unroll
        for (int u = 0; u < D; ++u) {
            const int k = kb + u;
            if (k > nk) break;
            xload(k % S::NRB);
            const int buf = u & 1;  // == k & 1 because D is even
            const int pb = buf ^ 1;
            uint32_t pv[S::NPV], qv[S::NQV];
#pragma unroll
            for (int i = 0; i < S::NPV; ++i) pv[i] = xval(pb, false, yg * YO + R + i);
            if constexpr (!BOX) {
#pragma unroll
                for (int i = 0; i < S::NQV; ++i) qv[i] = xval(pb, true, yg * YO + i);
            }
            {
                // z-window of slice j = k-2, whose P and Q entered the ring in
                // the previous iteration; it reads slot j+1 (Q of slice j-4r-1)
                // before the y-pass below overwrites it with slice k-1
                const int uj = (u + D - 2) % D;
                uint32_t o[YO];
#pragma unroll
                for (int m = 0; m < YO; ++m) {
                    bacc[m] += pr[(uj + D - R) % D][m] - pr[(uj + R + 1) % D][m];
                    if constexpr (BOX) {
                        o[m] = round_div_odd(bacc[m], inv9n);
                    } else {
                        wacc[m] += qr[uj][m] - qr[(uj + 1) % D][m];
                        const uint32_t Ssum = bacc[m] + wacc[m] + qr[(uj + D - 2 * R) % D][m];
                        o[m] = round_div_odd(Ssum, inv9n);
                    }
                    if (GATE && o[m] < gate) o[m] = 0;
                }
                store_out((k - 2 >= 2 * H) ? z0 + k - 2 - 2 * H : -1, o);
            }
            {
                // y-pass of slice k-1 into ring slot k-1
                const int uy = (u + D - 1) % D;
                uint32_t cp[S::NPV], cq[S::NQV];
                cp[0] = pv[0];
#pragma unroll
                for (int i = 1; i < S::NPV; ++i) cp[i] = cp[i - 1] + pv[i];
#pragma unroll
                for (int m = 0; m < YO; ++m) pr[uy][m] = cp[m + 2 * R] - (m ? cp[m - 1] : 0u);
                if constexpr (!BOX) {
                    cq[0] = qv[0];
#pragma unroll
                    for (int i = 1; i < S::NQV; ++i) cq[i] = cq[i - 1] + qv[i];
#pragma unroll
                    for (int m = 0; m < YO; ++m)
                        qr[uy][m] = cq[m + 4 * R] - (m ? cq[m - 1] : 0u) + qv[m + 2 * R];
                }
            }
            // slice i lives in raw slot i mod NRB: slice k+PF takes the slot
            // slice k-1 used, read in the previous iteration
            stage(z0 - H + k + S::PF, (k + S::PF) % S::NRB);
            xpass(buf);
            wait_vmem_le<S::VMWAIT>();  // slice k+1 has landed
            barrier_lds();
        }
    }
    // drain the staging of the slices past the end before the LDS is reused
    wait_vmem();
    barrier_lds();
}

// LDS for either staging; a kernel that may run both holds the union.
template <int R, int TY, int TXW = 64, bool BOX = false>
union M9SmemAny {
    M9Smem<R, TY, TXW, false, BOX> e;  // element-wise staging
    M9Smem<R, TY, TXW, true, BOX> p;   // paired staging
};

// One tile; `pairs` (mean9_pairs_ok for the volume) selects paired staging
// for the tiles whose x halo stays inside the volume.
template <int R, int TY, typename T, bool GATE, int TXW = 64, bool BOX = false>
__device__ __forceinline__ void mean9_tile(M9SmemAny<R, TY, TXW, BOX>& sm, bool pairs,
                                           const T* __restrict__ in, T* __restrict__ out, Geom g,
                                           int x0, int y0, int z0, int z1, uint32_t gate,
                                           double inv_div)
{
    constexpr int H = 2 * R, LXE = TXW + 4 * R;
    if (pairs && x0 - H >= 0 && x0 - H + LXE <= g.nx)
        mean9_tile_body<R, TY, T, GATE, TXW, true, BOX>(sm.p, in, out, g, x0, y0, z0, z1, gate,
                                                        inv_div);
    else
        mean9_tile_body<R, TY, T, GATE, TXW, false, BOX>(sm.e, in, out, g, x0, y0, z0, z1, gate,
                                                         inv_div);
}

}  // namespace lnf

// Streaming MEAN9 tile body: one workgroup filters a TX x TY column of output
// voxels over the z-range [z0, z1).  Shared by the single-volume kernel, the
// mean filter and the batch kernel.
//
// Arithmetic (paper, Section "Our Method", eqs. 2-3): the sum S over the nine
// clusters is box_x box_y box_z E + c_x c_y c_z E, with box = ones on [-r, r]
// and c = ones on [-2r, 2r] plus one more at the centre (the two diagonal
// clusters of an axis overlap there).  Per axis c = box shifted by -r plus box
// shifted by +r.  Everything is exact uint32.
//
// Per input slice s the x- and y-passes give the plane sums
//   P(s) = box_y box_x E(s),   Q(s) = c_y c_x E(s)
// at each output column.  Along z, c_z = box_z shifted by -r plus by +r, so
//   S(z) = sum_{t=z-r..z+r} P(t) + sum_{t=z-r..z+r} Q(t-r) + sum_{t=z-r..z+r} Q(t+r)
//        = sum_{t=z..z+2r} G(t),   G(t) = P(t-r) + Q(t) + Q(t-2r),
// a running box of 2r+1 slices of one quantity.  A value of P is kept r
// slices, of Q 2r slices and of G 2r+1 slices: 5r+1 registers per output
// column, in a register ring of D = 2r+2 slots indexed statically by the
// unrolled loop (the allocator keeps only the live values).
//
// Pipeline per iteration k (one barrier per iteration):
//   - LDS reads of this thread's raw row segment of slice k and of its x-pass
//     column of slice k-1;
//   - y-pass of slice k-1 (each thread owns one column and YO = 4 rows; prefix
//     sums), G, the running sum, out = round(S / 9n) (fp64, exact), gate and
//     the stores of output slice k-1-4r;
//   - LDS DMA of the raw (TX+4r) x (TY+4r) tile of slice k+PF straight from
//     HBM into LDS, coordinates clamped into the volume per lane; NRB = PF+1
//     raw buffers form a ring, so each slice has PF iterations to arrive;
//   - x-pass of slice k: each thread takes an 8-wide row segment and forms
//     px = box_x E and qx = c_x E from prefix sums over its 8+4r raw values.
// The x-pass results are double-buffered, so the x-pass of slice k overlaps
// the y-pass of slice k-1.  Every iteration issues exactly NLOAD loads and YO
// stores (masked-off stores go to an offset the buffer's range check drops),
// so the wait for slice k+1 at the end of iteration k is a partial one that
// leaves the younger PF-1 iterations' operations in flight.
//
// Modes:
//   kM9Packed  px <= qx, and when qx < 2^16 both fit one LDS word px | qx<<16.
//              The x-pass stores half as much and a y-pass thread loads 4+4r
//              words instead of (4+2r) + (4+4r): its px rows lie inside its qx
//              rows.  Whether qx < 2^16 depends on the data (always for values
//              up to 65535 / (4r+2): uint8, or 12-bit data up to r = 3), so
//              the x-pass ORs together every qx it forms; at the end of each
//              block of D slices the workgroup checks the OR, and a tile that
//              saw qx >= 2^16 stops: the caller filters it again in kM9Exact
//              from the first output slice that may hold a wrong value on.
//              Exact for every input.
//   kM9Exact   px and qx in separate uint32 LDS words.
//   kM9Box     the box term alone (the paper's mean filter, eq. 4): px only,
//              S(z) = sum_{t=z-r..z+r} P(t).
#pragma once

#include "device_common.h"
#include "lnf_internal.h"

namespace lnf {

constexpr int kM9Exact = 0, kM9Packed = 1, kM9Box = 2;

// Tile geometry.  PK: the raw tile is staged as element pairs, one 32-bit LDS
// word per pair (uint16: both halves; uint8: the low two bytes), loaded by one
// LDS DMA per lane.  That halves the DMA instructions and the LDS bytes of the
// staging and of the x-pass reads.  It needs an even nx (pairs never straddle
// a row end), a volume base aligned to a pair, and a tile whose halo stays
// inside the volume in x (a pair cannot be clamped element by element); tiles
// at an x face are staged element-wise.
template <int R, int TY, int TXW = 64, bool PK = false>
struct M9Geo {
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
    static constexpr int RAWW = NLOAD * THREADS;    // words of one raw buffer
    static constexpr int PXP = TX + 4;              // padded x-pass row pitch (words)
    static constexpr int XPW = (LY + 1) * PXP;      // words of one x-pass buffer
    static constexpr int D = 2 * R + 2;             // ring period and unroll (even)
    static constexpr int SEG = 8, NSEG = TX / SEG, SW = SEG + 4 * R;
    static constexpr int SWW = SW / EPW;            // words an x-pass segment reads
    static constexpr int XR = (LY + 7) / 8 * 8;     // x-pass row slots (multiple of 8)
    static constexpr int NPV = YO + 2 * R, NQV = YO + 4 * R;
    static_assert(XR * NSEG <= THREADS, "x-pass: one thread per row segment");
    static_assert(D % 2 == 0, "buffer parity must be static in the unrolled ring");
    static_assert(LX % 4 == 0 && (SEG / EPW) % 4 == 0, "x-pass reads 16-byte aligned rows");
    static_assert(SWW % 2 == 0 && LXE % 2 == 0, "x-pass reads whole 8-byte pieces");
};

// LDS one workgroup may use: three 256-thread workgroups per CU (160 KiB).
constexpr int kM9LdsBudget = 53 * 1024;

// Waves per SIMD the tile kernels are compiled for: three up to r = 3 (the
// tile body fits 168 VGPRs there), two at r = 4 and for 512-thread
// workgroups (one of those per CU holds two waves per SIMD).
template <int R, int THREADS>
constexpr int m9_waves()
{
    return (R <= 3 && THREADS <= 256) ? 3 : 2;
}

template <int R, int TY, int TXW, bool PK, int MODE>
struct M9Shape : M9Geo<R, TY, TXW, PK> {
    using G = M9Geo<R, TY, TXW, PK>;
    static constexpr int XBUFS = MODE == kM9Exact ? 4 : 2;  // px (and qx), double-buffered
    static constexpr int bytes_for(int nrb) { return 4 * (XBUFS * G::XPW + nrb * G::RAWW) + 16; }
    // Raw buffers: the largest count up to 5 that divides the unroll (so a
    // slice's buffer index is static), keeps the partial wait within the 6-bit
    // counter and fits the budget (the least, 2, if none does).
    static constexpr int pick_nrb()
    {
        for (int n = 5; n > 2; --n)
            if (G::D % n == 0 && (n - 2) * (G::NLOAD + G::YO) <= 63 &&
                bytes_for(n) <= kM9LdsBudget)
                return n;
        return 2;
    }
    static constexpr int NRB = pick_nrb();
    static constexpr int PF = NRB - 1;  // slices staged ahead of the x-pass
    // vector-memory operations issued after a slice's loads, up to the wait
    // that needs that slice: PF-1 iterations of (NLOAD loads + YO stores)
    static constexpr int VMWAIT = (PF - 1) * (G::NLOAD + G::YO);
    static_assert(G::D % NRB == 0 && VMWAIT <= 63, "raw ring");
};

template <int R, int TY, int TXW, bool PK, int MODE>
struct M9Smem {
    using S = M9Shape<R, TY, TXW, PK, MODE>;
    uint32_t raw[S::NRB][S::RAWW];
    // x-pass results; the extra row LY takes the surplus x-pass lanes' stores,
    // so no two lanes of a store hit the same address
    uint32_t px[2][S::XPW];
    uint32_t qx[MODE == kM9Exact ? 2 : 1][MODE == kM9Exact ? S::XPW : 1];
    uint32_t flag;  // kM9Packed: some x-pass of the tile formed qx >= 2^16
};

// Whether packed mode can see qx >= 2^16 for this element type and radius.
template <typename T, int R>
constexpr bool m9_packed_may_overflow()
{
    return (uint64_t)(4 * R + 2) * ((1u << (8 * sizeof(T))) - 1u) >= 65536u;
}

// inv_div: 1/(9n), or 1/n with kM9Box.  Returns z1 when every output slice
// of [z0, z1) is final.  A kM9Packed tile that stopped because some qx did
// not fit 16 bits returns the first output slice that may be wrong instead:
// the slices before it are final, and the rest must be filtered again in
// kM9Exact from that slice on.
template <int R, int TY, typename T, bool GATE, int TXW, bool PK, int MODE>
__device__ __forceinline__ int mean9_tile_body(M9Smem<R, TY, TXW, PK, MODE>& sm,
                                                const T* __restrict__ in, T* __restrict__ out,
                                                Geom g, int x0, int y0, int z0, int z1,
                                                uint32_t gate, double inv_div, int tid)
{
    using S = M9Shape<R, TY, TXW, PK, MODE>;
    constexpr bool kBox = MODE == kM9Box, kPQ = MODE == kM9Packed;
    constexpr bool kCheck = kPQ && m9_packed_may_overflow<T, R>();
    constexpr int H = S::H, LX = S::LX, D = S::D, TX = S::TX, PXP = S::PXP, YO = S::YO;
    constexpr int EPW = S::EPW, NRB = S::NRB, PF = S::PF;
    // output slice of iteration k: z0 + k - 1 - LAG
    constexpr int LAG = kBox ? 3 * R : 4 * R;
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
    // multiple of 8; surplus lanes redo the last row (no divergent branch) and
    // store to the spare row LY.
    const int xrow = min(tid % S::XR, S::LY - 1);
    const int xroww = (tid % S::XR < S::LY) ? xrow : S::LY;
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
    // OR of every qx this thread formed (kM9Packed: must stay below 2^16)
    uint32_t qor = 0;
    // x-pass, part 2: prefix sums over the segment, results written to LDS;
    // el(i) is raw element i of the segment
    auto xsums = [&](int buf, auto el) {
        uint32_t pp[S::SEG], qq[S::SEG], c[S::SW];
        c[0] = el(0);
#pragma unroll
        for (int i = 1; i < S::SW; ++i) c[i] = c[i - 1] + el(i);
#pragma unroll
        for (int m = 0; m < S::SEG; ++m) {
            if constexpr (!kBox) qq[m] = c[m + 4 * R] - (m ? c[m - 1] : 0u) + el(m + 2 * R);
            pp[m] = c[m + 3 * R] - c[m + R - 1];
        }
        if constexpr (kPQ) {
#pragma unroll
            for (int m = 0; m < S::SEG; ++m) {
                if constexpr (kCheck) qor |= qq[m];
                pp[m] |= qq[m] << 16;
            }
        }
        uint32_t* pd = sm.px[buf] + xroww * PXP + xseg * S::SEG;
#pragma unroll
        for (int m = 0; m < S::SEG; m += 4) {
            *reinterpret_cast<uint4*>(pd + m) = make_uint4(pp[m], pp[m + 1], pp[m + 2], pp[m + 3]);
            if constexpr (MODE == kM9Exact) {
                uint32_t* qd = sm.qx[buf] + xroww * PXP + xseg * S::SEG;
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

    // ring slots of P, Q and G (slice s in slot s mod D) and the running sum
    uint32_t pr[D][YO], qr[D][YO], gr[D][YO], acc[YO];
#pragma unroll
    for (int m = 0; m < YO; ++m) {
        acc[m] = 0;
#pragma unroll
        for (int u = 0; u < D; ++u) pr[u][m] = qr[u][m] = gr[u][m] = 0;
    }

    // The y-pass of the first iteration reads x-pass buffer 1 before any
    // x-pass wrote it: zeros there give zero plane sums.  The staging and the
    // passes run in every iteration (the extra ones at the end read clamped
    // slices and their results are never stored), so the unrolled block is
    // one basic block the compiler can interleave.
    for (int i = tid; i < S::LY * PXP; i += S::THREADS) {
        sm.px[1][i] = 0;
        if constexpr (MODE == kM9Exact) sm.qx[1][i] = 0;
    }
    if constexpr (kCheck) {
        if (tid == 0) sm.flag = 0;
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
    for (int p = 1; p < PF; ++p) {
        store_out(-1, acc);
        stage(z0 - H + p, p);
    }
    wait_vmem_le<S::VMWAIT>();
    barrier_lds();
    int zdone = z1;
    // iteration k: x-pass of slice k, y-pass of slice k-1 and its outputs;
    // whole blocks of D iterations (no exit inside the unrolled block)
    for (int kb = 0; kb <= ns; kb += D) {
#pragma unroll
        for (int u = 0; u < D; ++u) {
            const int k = kb + u;
            xload(u % NRB);  // slice k, staged PF iterations ago (k mod NRB)
            const int buf = u & 1;  // == k & 1 because D is even
            const int pb = buf ^ 1;
            uint32_t pv[S::NPV], qv[S::NQV];
            if constexpr (kPQ) {
                // one word per row: px in the low half, qx in the high half;
                // the px rows yg*YO+R .. are rows R .. of the qx range
                uint32_t wv[S::NQV];
#pragma unroll
                for (int i = 0; i < S::NQV; ++i) wv[i] = sm.px[pb][(yg * YO + i) * PXP + xq];
#pragma unroll
                for (int i = 0; i < S::NQV; ++i) qv[i] = wv[i] >> 16;
#pragma unroll
                for (int i = 0; i < S::NPV; ++i) pv[i] = wv[i + R] & 0xffffu;
            } else {
#pragma unroll
                for (int i = 0; i < S::NPV; ++i) pv[i] = sm.px[pb][(yg * YO + R + i) * PXP + xq];
                if constexpr (MODE == kM9Exact) {
#pragma unroll
                    for (int i = 0; i < S::NQV; ++i) qv[i] = sm.qx[pb][(yg * YO + i) * PXP + xq];
                }
            }
            {
                // y-pass of slice s = k-1 into ring slot us; slot (us+1) mod D
                // holds slice s-2r-1, the one that leaves the running sum
                const int us = (u + D - 1) % D;
                uint32_t cp[S::NPV], o[YO];
                cp[0] = pv[0];
#pragma unroll
                for (int i = 1; i < S::NPV; ++i) cp[i] = cp[i - 1] + pv[i];
#pragma unroll
                for (int m = 0; m < YO; ++m) pr[us][m] = cp[m + 2 * R] - (m ? cp[m - 1] : 0u);
                if constexpr (kBox) {
#pragma unroll
                    for (int m = 0; m < YO; ++m) {
                        acc[m] += pr[us][m] - pr[(us + 1) % D][m];
                        o[m] = round_div_odd(acc[m], inv_div);
                    }
                } else {
                    uint32_t cq[S::NQV];
                    cq[0] = qv[0];
#pragma unroll
                    for (int i = 1; i < S::NQV; ++i) cq[i] = cq[i - 1] + qv[i];
#pragma unroll
                    for (int m = 0; m < YO; ++m) {
                        qr[us][m] = cq[m + 4 * R] - (m ? cq[m - 1] : 0u) + qv[m + 2 * R];
                        gr[us][m] = pr[(us + D - R) % D][m] + qr[us][m] + qr[(us + 2) % D][m];
                        acc[m] += gr[us][m] - gr[(us + 1) % D][m];
                        o[m] = round_div_odd(acc[m], inv_div);
                    }
                }
#pragma unroll
                for (int m = 0; m < YO; ++m)
                    if (GATE && o[m] < gate) o[m] = 0;
                const int zo = z0 + k - 1 - LAG;
                store_out((zo >= z0 && zo < z1) ? zo : -1, o);
            }
            // slice k+PF takes the buffer slice k-1 used, read in the previous
            // iteration
            stage(z0 - H + k + PF, (u + PF) % NRB);
            xpass(buf);
            wait_vmem_le<S::VMWAIT>();  // slice k+1 has landed
            barrier_lds();
        }
        if constexpr (kCheck) {
            // block end: publish any qx >= 2^16 formed so far, then stop the
            // whole workgroup if some thread saw one.  The previous check
            // cleared the x-passes of iterations before kb, and the outputs of
            // iteration k read the x-pass of iteration k-1 only, so outputs of
            // iterations up to kb are final
            if (qor >> 16) sm.flag = 1;
            barrier_lds();
            if (sm.flag) {
                zdone = max(z0, z0 + kb - 1 - LAG);
                break;
            }
        }
    }
    // drain the staging of the slices past the end before the LDS is reused
    wait_vmem();
    barrier_lds();
    return zdone;
}

// Whether packed mode can stop, so that a kernel needs the unpacked bodies.
template <typename T, int R, bool BOX>
constexpr bool m9_needs_exact()
{
    return !BOX && m9_packed_may_overflow<T, R>();
}

// LDS of every body a kernel runs: packed (or box) mode with paired and
// element-wise staging, and the unpacked fallback where packed mode can stop
// (where it cannot, those members repeat the packed layouts).
template <int R, int TY, int TXW, typename T, bool BOX = false>
union M9SmemAny {
    static constexpr int kMode = BOX ? kM9Box : kM9Packed;
    static constexpr int kFallback = m9_needs_exact<T, R, BOX>() ? kM9Exact : kMode;
    M9Smem<R, TY, TXW, true, kMode> p;
    M9Smem<R, TY, TXW, false, kMode> e;
    M9Smem<R, TY, TXW, true, kFallback> px;
    M9Smem<R, TY, TXW, false, kFallback> ex;
};

// One tile; `pairs` (mean9_pairs_ok for the volume) selects paired staging
// for the tiles whose x halo stays inside the volume.  MEAN9 runs packed and,
// where that can stop, unpacked from the first slice a stopped packed run
// left unfinished.
// tid: threadIdx.x (see tile_tid for loops over several tiles).
template <int R, int TY, typename T, bool GATE, int TXW = 64, bool BOX = false>
__device__ __forceinline__ void mean9_tile(M9SmemAny<R, TY, TXW, T, BOX>& sm, bool pairs,
                                           const T* __restrict__ in, T* __restrict__ out, Geom g,
                                           int x0, int y0, int z0, int z1, uint32_t gate,
                                           double inv_div, int tid)
{
    constexpr int H = 2 * R, LXE = TXW + 4 * R;
    constexpr int kMode = BOX ? kM9Box : kM9Packed;
    if (pairs && x0 - H >= 0 && x0 - H + LXE <= g.nx) {
        const int zr = mean9_tile_body<R, TY, T, GATE, TXW, true, kMode>(
            sm.p, in, out, g, x0, y0, z0, z1, gate, inv_div, tid);
        if constexpr (m9_needs_exact<T, R, BOX>())
            if (zr < z1)
                mean9_tile_body<R, TY, T, GATE, TXW, true, kM9Exact>(sm.px, in, out, g, x0, y0, zr,
                                                                     z1, gate, inv_div, tid);
    } else {
        const int zr = mean9_tile_body<R, TY, T, GATE, TXW, false, kMode>(
            sm.e, in, out, g, x0, y0, z0, z1, gate, inv_div, tid);
        if constexpr (m9_needs_exact<T, R, BOX>())
            if (zr < z1)
                mean9_tile_body<R, TY, T, GATE, TXW, false, kM9Exact>(sm.ex, in, out, g, x0, y0,
                                                                      zr, z1, gate, inv_div, tid);
    }
}

}  // namespace lnf

// Fused finest levels ("head"): levels j and j+1 of a multi-level transform in
// one launch, the low-low band between them kept in LDS.
//
// The finest levels carry almost all the bytes. Run one launch each, level j
// writes its low-low band to HBM and level j+1 reads it straight back, and
// each launch pays its own ramp-up and drain. Here one workgroup computes
// level j over a window of 2-quad-per-lane rows (the one-level kernels'
// register tile and lifting code), keeps the scaled low-low values its window
// produces correctly in LDS, and computes level j+1 from them over the
// co-located coarser window; it writes both levels' detail bands and level
// j+1's low-low band. The same per-quad arithmetic runs on the same values as
// in one-level launches (the intermediate band is FP32 in both), so results
// are bit-identical to them.
//
// Geometry, with a halo unit RG = 2 quads (at least the number of lifting
// pairs of either wavelet), in quads of each level:
//   forward: the coarser window is 62 x H2 quads (lanes 0..61, each one quad,
//     H2 rows over the wavefronts), of which the centre 58 x (H2 - 2 RG) is
//     owned. It reads the low-low values of 124 x 2 H2 finer quads, the part
//     of the finer 128 x NR1 window (one halo lane and RG halo rows on each
//     side) that the finer lifting computes correctly; so NR1 = 2 H2 + 2 RG.
//     The finer level writes the bands of its 116 x 2 (H2 - 2 RG) quads that
//     map to the owned coarser block.
//   inverse: the finer window is 120 x NR1 quads (lanes 0..59; lanes 60..63
//     carry nothing useful), of which the centre 116 x (NR1 - 2 RG) is written.
//     It needs the finer low-low band over its whole window, i.e. coarser
//     outputs over 60 x NR1/2 quads; the coarser window adds RG on each side:
//     64 x (NR1/2 + 2 RG) quads.
// Outside the image each level reads its input through the whole-sample
// symmetric extension (forward) or the per-phase extension of the
// coefficients (inverse), as the one-level kernels do; the mirrored
// positions of every value that reaches a written output fall inside the
// region held in LDS, and reads for other lanes are clamped into it.
#pragma once

#include "dwt2_tail.hpp"

namespace dwt2 {

template <int ROWS, int WAVES>
struct HeadGeom {
    static constexpr int RG = 2;
    static constexpr int NR1 = WAVES * ROWS;              // finer window rows
    static_assert(NR1 % 2 == 0, "whole coarser rows");
    // forward
    static constexpr int FH2 = (NR1 - 2 * RG) / 2;        // coarser window rows
    static constexpr int FOX2 = 62 - 2 * RG;              // coarser owned columns
    static constexpr int FOY2 = FH2 - 2 * RG;             // coarser owned rows
    static constexpr int FROWS2 = (FH2 + WAVES - 1) / WAVES;
    static_assert(FOY2 > 0, "forward head window too short");
    // inverse
    static constexpr int IOX1 = 116;                      // finer owned columns
    static constexpr int IOY1 = NR1 - 2 * RG;             // finer owned rows
    static constexpr int IH2 = NR1 / 2 + 2 * RG;          // coarser window rows
    static constexpr int IROWS2 = (IH2 + WAVES - 1) / WAVES;
};

struct FwdHead {
    FwdParams l1;             // level j: input and detail bands (its ll is unused)
    FwdParams l2;             // level j+1: detail bands and low-low output (its in is unused)
    int32_t tiles_x, tiles_y; // owned blocks of level j+1
};

struct InvHead {
    InvParams l2;             // level j+1: low-low and detail bands (its out is unused)
    InvParams l1;             // level j: detail bands and output (its ll is unused)
    int32_t tiles_x, tiles_y; // owned blocks of level j
};

// Position p of an LDS axis of n values starting at p0, clamped into it.
__device__ __forceinline__ int lds_at(int p, int p0, int n) { return min(max(p - p0, 0), n - 1); }

// Wavefronts per SIMD that the register allocation must allow. Two head
// workgroups share a CU (their LDS fits twice), which takes WAVES/2 per SIMD,
// i.e. at most 80 VGPRs for 12 wavefronts. Left free, forward heads with
// 16-bit input come out at 80-81 (the separable FP16 one and the BF16 ones at
// 81) and then run one workgroup per CU (about 35% slower); those
// instantiations are held to the budget. The FP32 ones fit as they are and
// keep the allocation the workgroup size alone implies.
template <int SCH, int WAVES, typename TIN>
constexpr int kFwdHeadWavesPerSimd = sizeof(TIN) == 2 ? (2 * WAVES + 3) / 4 : (WAVES + 3) / 4;
template <int WAVES>
constexpr int kInvHeadWavesPerSimd = (WAVES + 3) / 4;
// The batched heads (which read their parameters from the plan, one more
// register or so) are all held to the two-workgroup budget.
template <int WAVES>
constexpr int kTableHeadWavesPerSimd = (2 * WAVES + 3) / 4;

// LDS of a head workgroup: the mailbox serves the finer level's exchanges, then
// the coarser level's (smaller); ll1 holds the level j low-low band as the four
// components of the level j+1 quads, [phase][row][column].
template <int WAVES, int H2>
struct HeadLds {
    Mailbox<2, WAVES> box;
    float ll1[4][H2][64];
};

template <int ROWS, int WAVES>
using FwdHeadLds = HeadLds<WAVES, HeadGeom<ROWS, WAVES>::FH2>;
template <int ROWS, int WAVES>
using InvHeadLds = HeadLds<WAVES, HeadGeom<ROWS, WAVES>::IH2>;

// Levels j and j+1 of forward head tile t (row-major over tiles_x x tiles_y).
// Wavefronts below the coarser level's window return early, after passing its
// barriers.
template <int WV, int SCH, int ROWS, int WAVES, typename TIN, typename TLL, typename TB>
__device__ __forceinline__ void fwd_head_tile(const FwdHead &hd, const int t,
                                              FwdHeadLds<ROWS, WAVES> &lds) {
    using G = HeadGeom<ROWS, WAVES>;
    using L = Wavelet<WV>;
    constexpr int RG = G::RG, H2 = G::FH2, R2 = G::FROWS2, NR1 = G::NR1;
    Mailbox<2, WAVES> &box = lds.box;
    float(&ll1)[4][H2][64] = lds.ll1;
    const float sLL = (float)(L::ZL * L::ZL), sHL = (float)(L::ZL * L::ZH);
    const float sHH = (float)(L::ZH * L::ZH);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ty = t / hd.tiles_x, tx = t - ty * hd.tiles_x;
    const int ox2 = tx * G::FOX2, oy2 = ty * G::FOY2;   // owned block of level j+1

    // ---- level j: window of 128 x NR1 quads, two per lane
    {
        const FwdParams &p1 = hd.l1;
        const int qx = 2 * (ox2 - RG - 1 + lane);       // the lane's first quad column
        const int qy0 = 2 * oy2 - 3 * RG + wave * ROWS; // its first quad row
        Quads<ROWS, 2> q;
        fwd_load_at<2, ROWS, TIN>(q, p1, qx, qy0);
        {
            Exchange<ROWS, 2, WAVES> x{&box, wave, lane, 0};
            lift_forward<WV, SCH>(q, x);
        }
        // correct low-low values (lanes 1..62, rows RG..NR1-RG-1) into LDS
        if (lane >= 1 && lane <= 62) {
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const int rr = wave * ROWS + r - RG;
                if (rr >= 0 && rr < 2 * H2) {
                    const int ph = 2 * (rr & 1);
                    ll1[ph][rr >> 1][lane - 1] = q.a[r][0] * sLL;
                    ll1[ph + 1][rr >> 1][lane - 1] = q.a[r][1] * sLL;
                }
            }
        }
        __syncthreads();   // the low-low band is in LDS; every level j exchange is done
        // detail bands of the quads under the owned level j+1 block, issued
        // after the barrier so that no wavefront waits there for another's
        // store addressing
        const bool own_x = lane >= RG + 1 && lane < RG + 1 + G::FOX2 && qx + 2 <= p1.nqx;
        TB *hl = static_cast<TB *>(p1.hl);
        TB *lh = static_cast<TB *>(p1.lh);
        TB *hh = static_cast<TB *>(p1.hh);
        const uint32_t bb = (uint32_t)p1.nqx * (uint32_t)sizeof(TB);
        const uint32_t off = own_x ? (uint32_t)qx * (uint32_t)sizeof(TB) : kNoAccess;
        int64_t rowo = (int64_t)qy0 * p1.band_pitch;   // band row qy0 + r, stepped
#pragma unroll
        for (int r = 0; r < ROWS; ++r, rowo += p1.band_pitch) {
            const int wr = wave * ROWS + r;
            const int gy = qy0 + r;
            if (wr < 3 * RG || wr >= 3 * RG + 2 * G::FOY2 || gy >= p1.nqy) continue;
            const float vb[2] = {q.b[r][0] * sHL, q.b[r][1] * sHL};
            const float vc[2] = {q.c[r][0] * sHL, q.c[r][1] * sHL};
            const float vd[2] = {q.d[r][0] * sHH, q.d[r][1] * sHH};
            if (p1.vec_band) {
                store_vec<TB, 2>(make_rsrc(hl + rowo, bb), off, vb);
                store_vec<TB, 2>(make_rsrc(lh + rowo, bb), off, vc);
                store_vec<TB, 2>(make_rsrc(hh + rowo, bb), off, vd);
            } else {
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    const uint32_t oi = own_x ? off + (uint32_t)(i * sizeof(TB)) : kNoAccess;
                    store_elem<TB>(make_rsrc(hl + rowo, bb), oi, vb[i]);
                    store_elem<TB>(make_rsrc(lh + rowo, bb), oi, vc[i]);
                    store_elem<TB>(make_rsrc(hh + rowo, bb), oi, vd[i]);
                }
            }
        }
    }

    // ---- level j+1: window of 62 x H2 quads, one per lane, R2 rows per wavefront
    const FwdParams &p2 = hd.l2;
    if (wave * R2 >= H2) {   // below the window: pass the lifting's barriers
        idle_through_lifting<WV>();
        return;
    }
    const int c0 = ox2 - RG, r0 = oy2 - RG;             // LDS origin, level j+1 quads
    const int X = c0 + lane;
    const int xe = mirror(2 * X, p2.w), xo = mirror(2 * X + 1, p2.w);
    const int ce = lds_at(xe >> 1, c0, 62), co = lds_at(xo >> 1, c0, 62);
    Quads<R2, 1> q;
    const int Y0 = r0 + wave * R2;
    if (Y0 >= 0 && 2 * (Y0 + R2) <= p2.h) {
        // all rows inside the level (wavefront-uniform): no row is mirrored
#pragma unroll
        for (int r = 0; r < R2; ++r) {
            const int ry = lds_at(Y0 + r, r0, H2);
            q.a[r][0] = ll1[xe & 1][ry][ce];
            q.b[r][0] = ll1[xo & 1][ry][co];
            q.c[r][0] = ll1[2 + (xe & 1)][ry][ce];
            q.d[r][0] = ll1[2 + (xo & 1)][ry][co];
        }
    } else {
#pragma unroll
        for (int r = 0; r < R2; ++r) {
            const int Y = Y0 + r;
            const int ye = mirror(2 * Y, p2.h), yo = mirror(2 * Y + 1, p2.h);
            const int re = lds_at(ye >> 1, r0, H2), ro = lds_at(yo >> 1, r0, H2);
            const int pe = 2 * (ye & 1), po = 2 * (yo & 1);
            q.a[r][0] = ll1[pe + (xe & 1)][re][ce];
            q.b[r][0] = ll1[pe + (xo & 1)][re][co];
            q.c[r][0] = ll1[po + (xe & 1)][ro][ce];
            q.d[r][0] = ll1[po + (xo & 1)][ro][co];
        }
    }
    {
        Exchange<R2, 1, WAVES> x{reinterpret_cast<Mailbox<1, WAVES> *>(&box), wave, lane, 0};
        lift_forward<WV, SCH>(q, x);
    }
    const bool own_x = lane >= RG && lane < RG + G::FOX2 && X < p2.nqx;
    const uint32_t ob = own_x ? (uint32_t)X * (uint32_t)sizeof(TB) : kNoAccess;
    const uint32_t ol = own_x ? (uint32_t)X * (uint32_t)sizeof(TLL) : kNoAccess;
    int64_t rb = (int64_t)(r0 + wave * R2) * p2.band_pitch;   // row r0 + wr, stepped
    int64_t rl = (int64_t)(r0 + wave * R2) * p2.ll_pitch;
#pragma unroll
    for (int r = 0; r < R2; ++r, rb += p2.band_pitch, rl += p2.ll_pitch) {
        const int wr = wave * R2 + r;
        const int gy = r0 + wr;
        if (wr < RG || wr >= RG + G::FOY2 || gy >= p2.nqy) continue;   // wavefront-uniform
        store_elem<TB>(row_at<TB>(p2.hl, rb, p2.nqx), ob, q.b[r][0] * sHL);
        store_elem<TB>(row_at<TB>(p2.lh, rb, p2.nqx), ob, q.c[r][0] * sHL);
        store_elem<TB>(row_at<TB>(p2.hh, rb, p2.nqx), ob, q.d[r][0] * sHH);
        store_elem<TLL>(row_at<TLL>(p2.ll, rl, p2.nqx), ol, q.a[r][0] * sLL);
    }
}

// Levels j+1 and j of inverse head tile t (row-major over tiles_x x tiles_y).
template <int WV, int SCH, int ROWS, int WAVES, typename TLL, typename TB, typename TOUT>
__device__ __forceinline__ void inv_head_tile(const InvHead &hd, const int t,
                                              InvHeadLds<ROWS, WAVES> &lds) {
    using G = HeadGeom<ROWS, WAVES>;
    using L = Wavelet<WV>;
    constexpr int RG = G::RG, H2 = G::IH2, R2 = G::IROWS2, NR1 = G::NR1;
    Mailbox<2, WAVES> &box = lds.box;     // level j+1 exchanges (smaller), then level j's
    float(&ll1)[4][H2][64] = lds.ll1;     // level j low-low as level j+1 output quads
    const float uLL = (float)(1.0 / (L::ZL * L::ZL)), uHL = (float)(1.0 / (L::ZL * L::ZH));
    const float uHH = (float)(1.0 / (L::ZH * L::ZH));
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ty = t / hd.tiles_x, tx = t - ty * hd.tiles_x;
    const int ox1 = tx * G::IOX1, oy1 = ty * G::IOY1;    // owned block of level j
    const int wx1 = ox1 - 2, wy1 = oy1 - RG;             // level j window origin (even)
    const int c0 = wx1 / 2 - RG, r0 = wy1 / 2 - RG;      // level j+1 window origin

    // ---- level j+1: window of 64 x H2 quads, one per lane, R2 rows per wavefront
    if (wave * R2 < H2) {
        Quads<R2, 1> q;
        inv_load_at<1, R2, TLL, TB>(q, hd.l2, c0 + lane, r0 + wave * R2);
#pragma unroll
        for (int r = 0; r < R2; ++r) {
            q.a[r][0] *= uLL; q.b[r][0] *= uHL; q.c[r][0] *= uHL; q.d[r][0] *= uHH;
        }
        {
            Exchange<R2, 1, WAVES> x{reinterpret_cast<Mailbox<1, WAVES> *>(&box), wave, lane, 0};
            lift_inverse<WV, SCH>(q, x);
        }
#pragma unroll
        for (int r = 0; r < R2; ++r) {
            const int wr = wave * R2 + r;
            if (wr < H2) {
                ll1[0][wr][lane] = q.a[r][0];
                ll1[1][wr][lane] = q.b[r][0];
                ll1[2][wr][lane] = q.c[r][0];
                ll1[3][wr][lane] = q.d[r][0];
            }
        }
    } else {
        idle_through_lifting<WV>();
    }
    __syncthreads();   // the low-low band is in LDS; every level j+1 exchange is done

    // ---- level j: window of 120 x NR1 quads, two per lane (lanes 60..63 idle)
    const InvParams &p1 = hd.l1;
    const int qx = wx1 + 2 * lane;
    const int qy0 = wy1 + wave * ROWS;
    Quads<ROWS, 2> q;
    inv_load_at<2, ROWS, TB, TB, false>(q, p1, qx, qy0);
    {
        // the low-low coefficient of quad (i, j) is the extended low phase
        int cx[2], px[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int xe = mirror(2 * (qx + i), p1.w) >> 1;
            cx[i] = lds_at(xe >> 1, c0, 64);
            px[i] = xe & 1;
        }
        if (qy0 >= 0 && 2 * (qy0 + ROWS) <= p1.h) {
            // all rows inside the level (wavefront-uniform): quad row gy's low
            // phase is row gy of the coarser output
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const int gy = qy0 + r;
                const int ry = lds_at(gy >> 1, r0, H2);
                const int py = 2 * (gy & 1);
#pragma unroll
                for (int i = 0; i < 2; ++i) q.a[r][i] = ll1[py + px[i]][ry][cx[i]];
            }
        } else {
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const int ye = mirror(2 * (qy0 + r), p1.h) >> 1;
                const int ry = lds_at(ye >> 1, r0, H2);
                const int py = 2 * (ye & 1);
#pragma unroll
                for (int i = 0; i < 2; ++i) q.a[r][i] = ll1[py + px[i]][ry][cx[i]];
            }
        }
    }
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            q.a[r][i] *= uLL; q.b[r][i] *= uHL; q.c[r][i] *= uHL; q.d[r][i] *= uHH;
        }
    }
    {
        Exchange<ROWS, 2, WAVES> x{&box, wave, lane, 0};
        lift_inverse<WV, SCH>(q, x);
    }
    const bool own_x = lane >= 1 && lane < 1 + G::IOX1 / 2;
    TOUT *out = static_cast<TOUT *>(p1.out);
    const int px0 = 2 * qx;
    const bool full_x = own_x && p1.vec_out && px0 + 4 <= p1.w;
    const uint32_t rb = (uint32_t)p1.w * (uint32_t)sizeof(TOUT);
    int64_t ro = (int64_t)(2 * qy0) * p1.out_pitch;   // pixel row 2 (qy0 + r), stepped
#pragma unroll
    for (int r = 0; r < ROWS; ++r, ro += 2 * p1.out_pitch) {
        const int wr = wave * ROWS + r;
        const int gy = qy0 + r;
        if (wr < RG || wr >= RG + G::IOY1 || gy >= p1.nqy) continue;   // wavefront-uniform
        const float e[4] = {q.a[r][0], q.b[r][0], q.a[r][1], q.b[r][1]};
        const float o[4] = {q.c[r][0], q.d[r][0], q.c[r][1], q.d[r][1]};
        TOUT *r0p = out + ro;
        TOUT *r1p = r0p + p1.out_pitch;
        if (p1.vec_out) {
            const uint32_t off = full_x ? (uint32_t)px0 * (uint32_t)sizeof(TOUT) : kNoAccess;
            if (p1.stream_out) {
                store_vec<TOUT, 4, kStoreStream>(make_rsrc(r0p, rb), off, e);
                store_vec<TOUT, 4, kStoreStream>(make_rsrc(r1p, rb), off, o);
            } else {
                store_vec<TOUT, 4>(make_rsrc(r0p, rb), off, e);
                store_vec<TOUT, 4>(make_rsrc(r1p, rb), off, o);
            }
        } else if (own_x) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (px0 + k < p1.w) {
                    r0p[px0 + k] = from_float<TOUT>(e[k]);
                    r1p[px0 + k] = from_float<TOUT>(o[k]);
                }
            }
        }
    }
}

// One workgroup per tile of one image.
template <int WV, int SCH, int ROWS, int WAVES, typename TIN, typename TLL, typename TB>
__global__ __launch_bounds__(64 * WAVES, (kFwdHeadWavesPerSimd<SCH, WAVES, TIN>)) void fwd_head_kernel(
    FwdHead hd) {
    __shared__ FwdHeadLds<ROWS, WAVES> lds;
    fwd_head_tile<WV, SCH, ROWS, WAVES, TIN, TLL, TB>(hd, block_tile(), lds);
}

template <int WV, int SCH, int ROWS, int WAVES, typename TLL, typename TB, typename TOUT>
__global__ __launch_bounds__(64 * WAVES, kInvHeadWavesPerSimd<WAVES>) void inv_head_kernel(InvHead hd) {
    __shared__ InvHeadLds<ROWS, WAVES> lds;
    inv_head_tile<WV, SCH, ROWS, WAVES, TLL, TB, TOUT>(hd, block_tile(), lds);
}

// Heads of a planned batch: the tiles of every image in one launch, each
// image's parameters in the device copy of the plan. A workgroup walks the
// tiles t = its id, id + gridDim.x, ... below `total` (several when the grid is
// capped at the resident workgroups), with a barrier between tiles, which
// share the LDS.
template <int WV, int SCH, int ROWS, int WAVES, typename TIN, typename TLL, typename TB>
__global__ __launch_bounds__(64 * WAVES, kTableHeadWavesPerSimd<WAVES>) void fwd_head_table_kernel(
    TableLaunch<FwdHead> tl) {
    __shared__ FwdHeadLds<ROWS, WAVES> lds;
    for (int t = block_tile(); t < tl.total; t += gridDim.x) {
        const int i = __builtin_amdgcn_readfirstlane(tl.img[t]);
        const FwdHead hd = tl.params[i];
        fwd_head_tile<WV, SCH, ROWS, WAVES, TIN, TLL, TB>(hd, t - tl.start[i], lds);
        __syncthreads();
    }
}

template <int WV, int SCH, int ROWS, int WAVES, typename TLL, typename TB, typename TOUT>
__global__ __launch_bounds__(64 * WAVES, kTableHeadWavesPerSimd<WAVES>) void inv_head_table_kernel(
    TableLaunch<InvHead> tl) {
    __shared__ InvHeadLds<ROWS, WAVES> lds;
    for (int t = block_tile(); t < tl.total; t += gridDim.x) {
        const int i = __builtin_amdgcn_readfirstlane(tl.img[t]);
        const InvHead hd = tl.params[i];
        inv_head_tile<WV, SCH, ROWS, WAVES, TLL, TB, TOUT>(hd, t - tl.start[i], lds);
        __syncthreads();
    }
}

// Heads of independent images in one launch, with their parameters in the
// kernel arguments (continuous batching: a different set every call), as the
// level batches: up to kHeadBatchMax heads of one set of storage types;
// tile_start[i] is the first global tile of head i (tile_start[n] the total).
// One workgroup per tile.
constexpr int kHeadBatchMax = 18;

struct FwdHeadBatch {
    int32_t n;
    int32_t tile_start[kHeadBatchMax + 1];
    FwdHead h[kHeadBatchMax];
};
struct InvHeadBatch {
    int32_t n;
    int32_t tile_start[kHeadBatchMax + 1];
    InvHead h[kHeadBatchMax];
};
static_assert(sizeof(FwdHeadBatch) <= 4096 && sizeof(InvHeadBatch) <= 4096,
              "kernel argument limit");

template <int WV, int SCH, int ROWS, int WAVES, typename TIN, typename TLL, typename TB>
__global__ __launch_bounds__(64 * WAVES, kTableHeadWavesPerSimd<WAVES>) void fwd_head_batch_kernel(
    FwdHeadBatch bt) {
    __shared__ FwdHeadLds<ROWS, WAVES> lds;
    const int t = block_tile();
    const int i = batch_image(bt, t);
    fwd_head_tile<WV, SCH, ROWS, WAVES, TIN, TLL, TB>(bt.h[i], t - bt.tile_start[i], lds);
}

template <int WV, int SCH, int ROWS, int WAVES, typename TLL, typename TB, typename TOUT>
__global__ __launch_bounds__(64 * WAVES, kTableHeadWavesPerSimd<WAVES>) void inv_head_batch_kernel(
    InvHeadBatch bt) {
    __shared__ InvHeadLds<ROWS, WAVES> lds;
    const int t = block_tile();
    const int i = batch_image(bt, t);
    inv_head_tile<WV, SCH, ROWS, WAVES, TLL, TB, TOUT>(bt.h[i], t - bt.tile_start[i], lds);
}

}  // namespace dwt2

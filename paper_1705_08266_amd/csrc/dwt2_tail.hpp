// Fused coarse levels ("tail"): the last F levels of a multi-level transform
// in one launch.
//
// The coarse levels of a pyramid are too small to fill the GPU; launched one
// by one, each costs a kernel start plus a full load-lift-store latency
// chain. Here one workgroup owns a square block of the coarsest fused level
// and computes every fused level for the region that block depends on (a
// halo pyramid): the finest fused level is read from HBM once, the low-low
// band of each intermediate level stays in LDS in FP32, and only the bands
// the workgroup owns are written. The lifting itself is the register-tile
// code of the one-level kernels (same per-quad arithmetic on the same values),
// so the results are bit-identical to running the levels one at a time.
//
// Regions, in quads of level m (forward: m = 0 is the finest fused level).
// An output quad depends on the input quads within R = number of lifting
// pairs on each side. Forward: to produce the owned block of level m+1
// extended by e[m+1], level m must produce its owned block extended by
// e[m] = 2 e[m+1] + 2R (its low-low band is the next level's input at half
// the resolution); e[F-1] = 0. Inverse (m = 0 is the coarsest level):
// e[m] = ceil((e[m+1] + R) / 2). Outside the image, every level reads its
// input through the whole-sample symmetric extension; the mirrored positions
// always fall inside the region held in LDS.
#pragma once

#include "dwt2_kernels.hpp"

namespace dwt2 {

constexpr int kTailMax = 3;                       // most fused levels per launch
// Few workgroups run at once in a tail launch, so each level pass is bound by
// instruction latency: 16 wavefronts of 4 quad rows keep more work in flight
// than 8 of 8 rows.
constexpr int kTailQPL = 1, kTailRows = 4, kTailWaves = 16;
constexpr int kTailWin = 64;                      // register window: 64 x 64 quads
constexpr int kTailBufSide = 60;                  // LDS region: up to 60 x 60 values
constexpr int kTailBuf = kTailBufSide * kTailBufSide;

struct FwdTail {
    FwdParams lv[kTailMax];   // lv[0].in: input of the finest fused level; lv[F-1].ll: final LL
    int32_t F;                // number of fused levels, 2..kTailMax
    int32_t B;                // owned block side at the coarsest fused level, in quads
    int32_t blocks_x;         // blocks along x (the grid is blocks_x * blocks_y)
    int32_t e[kTailMax];      // region extension per level, quads
};

struct InvTail {
    InvParams lv[kTailMax];   // lv[0]: coarsest fused level (reads the pyramid's LL);
                              // lv[F-1]: finest (writes `out`)
    int32_t F, B, blocks_x;
    int32_t e[kTailMax];
};

// Workgroup barriers in one lifting sequence (one per vertical exchange).
template <int WV>
constexpr int kLiftBarriers = 2 * Wavelet<WV>::NPAIRS;

// Wavefronts whose rows lie below a level's window skip that level's work
// but pass the same barriers. Their stale mailbox slots feed only the rows
// within the lifting radius of the window's lower edge, which are never
// stored, as at the window edge itself.
template <int WV>
__device__ __forceinline__ void idle_through_lifting() {
#pragma unroll
    for (int k = 0; k < kLiftBarriers<WV>; ++k) __syncthreads();
}

struct Region {
    int ox0, ox1, oy0, oy1;   // owned quads (clipped to the level)
    int cx0, cx1, cy0, cy1;   // computed quads: owned plus extension (clipped)
};

__device__ __forceinline__ Region tail_region(int bx, int by, int side, int ext, int nqx,
                                              int nqy) {
    Region g;
    g.ox0 = bx * side; g.oy0 = by * side;
    g.ox1 = min(g.ox0 + side, nqx); g.oy1 = min(g.oy0 + side, nqy);
    g.cx0 = max(g.ox0 - ext, 0); g.cy0 = max(g.oy0 - ext, 0);
    g.cx1 = min(g.ox0 + side + ext, nqx); g.cy1 = min(g.oy0 + side + ext, nqy);
    return g;
}

// Offset of position p in an LDS region axis of n values starting at p0,
// clamped into the region: lanes outside the computed area read some held
// value, and their results are never stored.
__device__ __forceinline__ int clamp_to(int p, int p0, int n) {
    return min(max(p - p0, 0), n - 1);
}

// Wavefront-uniform buffer resource of one row of `n` elements of T.
template <typename T>
__device__ __forceinline__ rsrc_t row_rsrc(const void *base, int64_t row, int64_t pitch, int n) {
    return make_rsrc(static_cast<const T *>(base) + row * pitch,
                     (uint32_t)n * (uint32_t)sizeof(T));
}

// The same for a row whose element offset (row times pitch) the caller keeps:
// loops over consecutive rows step the offset by the pitch instead of
// multiplying per row.
template <typename T>
__device__ __forceinline__ rsrc_t row_at(const void *base, int64_t off, int n) {
    return make_rsrc(static_cast<const T *>(base) + off, (uint32_t)n * (uint32_t)sizeof(T));
}

// F (the number of fused levels) is a template parameter so that the level
// loop unrolls and every level's parameters load at kernel start.
template <int WV, int SCH, int F, typename TIN, typename TLL, typename TB>
__global__ __launch_bounds__(64 * kTailWaves) void fwd_tail_kernel(FwdTail t) {
    constexpr int QPL = kTailQPL, ROWS = kTailRows, WAVES = kTailWaves;
    constexpr int R = Wavelet<WV>::NPAIRS;
    using L = Wavelet<WV>;
    __shared__ Mailbox<QPL, WAVES> box;
    __shared__ float llbuf[2][kTailBuf];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // XCD-contiguous block numbering: neighbouring blocks, whose halo
    // pyramids overlap, run on the same XCD and share its L2
    const int blk = block_tile();
    const int bx = blk % t.blocks_x, by = blk / t.blocks_x;
    const float sLL = (float)(L::ZL * L::ZL), sHL = (float)(L::ZL * L::ZH);
    const float sHH = (float)(L::ZH * L::ZH);
    int px0 = 0, py0 = 0, pw = 1, ph = 1;       // previous level's LL region in LDS
#pragma unroll
    for (int m = 0; m < F; ++m) {
        const FwdParams &prm = t.lv[m];
        const Region g = tail_region(bx, by, t.B << (F - 1 - m), t.e[m], prm.nqx, prm.nqy);
        const int qx = g.cx0 - R + lane;          // the lane's quad column
        const int qy0 = g.cy0 - R + wave * ROWS;  // its first quad row
        const int cw = g.cx1 - g.cx0;
        if (wave * ROWS >= (g.cy1 - g.cy0) + 2 * R) {   // below this level's window
            idle_through_lifting<WV>();
            px0 = g.cx0; py0 = g.cy0; pw = cw; ph = g.cy1 - g.cy0;
            __syncthreads();
            continue;
        }
        Quads<ROWS, QPL> q;
        if (m == 0) {
            fwd_load_at<QPL, ROWS, TIN>(q, prm, qx, qy0);
        } else {
            // the level input is the previous level's LL, held in LDS for its
            // computed region
            const float *src = llbuf[(m - 1) & 1];
            const int xe = clamp_to(mirror(2 * qx, prm.w), px0, pw);
            const int xo = clamp_to(mirror(2 * qx + 1, prm.w), px0, pw);
            const bool inside = qy0 >= 0 && 2 * (qy0 + ROWS) <= prm.h;   // wavefront-uniform
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const int y = 2 * (qy0 + r);
                const int ye = clamp_to(inside ? y : mirror(y, prm.h), py0, ph) * pw;
                const int yo = clamp_to(inside ? y + 1 : mirror(y + 1, prm.h), py0, ph) * pw;
                q.a[r][0] = src[ye + xe]; q.b[r][0] = src[ye + xo];
                q.c[r][0] = src[yo + xe]; q.d[r][0] = src[yo + xo];
            }
        }
        Exchange<ROWS, QPL, WAVES> x{&box, wave, lane, 0};
        lift_forward<WV, SCH>(q, x);
        const bool last = m == F - 1;
        float *dst = llbuf[m & 1];
        // lanes outside the owned columns store nowhere
        const uint32_t ob = (qx >= g.ox0 && qx < g.ox1) ? (uint32_t)qx * sizeof(TB) : kNoAccess;
        const uint32_t ol = (qx >= g.ox0 && qx < g.ox1) ? (uint32_t)qx * sizeof(TLL) : kNoAccess;
        const bool comp_x = qx >= g.cx0 && qx < g.cx1;
        int64_t rb = (int64_t)qy0 * prm.band_pitch, rl = (int64_t)qy0 * prm.ll_pitch;
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int gy = qy0 + r;
            const float va = q.a[r][0] * sLL;
            if (gy >= g.oy0 && gy < g.oy1) {   // wavefront-uniform
                store_elem<TB>(row_at<TB>(prm.hl, rb, prm.nqx), ob, q.b[r][0] * sHL);
                store_elem<TB>(row_at<TB>(prm.lh, rb, prm.nqx), ob, q.c[r][0] * sHL);
                store_elem<TB>(row_at<TB>(prm.hh, rb, prm.nqx), ob, q.d[r][0] * sHH);
                if (last) store_elem<TLL>(row_at<TLL>(prm.ll, rl, prm.nqx), ol, va);
            }
            if (!last && comp_x && gy >= g.cy0 && gy < g.cy1)
                dst[(gy - g.cy0) * cw + (qx - g.cx0)] = va;
            rb += prm.band_pitch; rl += prm.ll_pitch;
        }
        px0 = g.cx0; py0 = g.cy0; pw = cw; ph = g.cy1 - g.cy0;
        __syncthreads();   // this level's LL is complete before the next level reads it
    }
}

template <int WV, int SCH, int F, typename TLL, typename TB, typename TOUT>
__global__ __launch_bounds__(64 * kTailWaves) void inv_tail_kernel(InvTail t) {
    constexpr int QPL = kTailQPL, ROWS = kTailRows, WAVES = kTailWaves;
    constexpr int R = Wavelet<WV>::NPAIRS;
    using L = Wavelet<WV>;
    __shared__ Mailbox<QPL, WAVES> box;
    __shared__ float pxbuf[2][kTailBuf];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // XCD-contiguous block numbering: neighbouring blocks, whose halo
    // pyramids overlap, run on the same XCD and share its L2
    const int blk = block_tile();
    const int bx = blk % t.blocks_x, by = blk / t.blocks_x;
    const float uLL = (float)(1.0 / (L::ZL * L::ZL)), uHL = (float)(1.0 / (L::ZL * L::ZH));
    const float uHH = (float)(1.0 / (L::ZH * L::ZH));
    int px0 = 0, py0 = 0, pw = 1, ph = 1;       // previous level's output region in LDS
#pragma unroll
    for (int m = 0; m < F; ++m) {
        const InvParams &prm = t.lv[m];
        const Region g = tail_region(bx, by, t.B << m, t.e[m], prm.nqx, prm.nqy);
        const int qx = g.cx0 - R + lane;
        const int qy0 = g.cy0 - R + wave * ROWS;
        const int cw = 2 * (g.cx1 - g.cx0);
        if (wave * ROWS >= (g.cy1 - g.cy0) + 2 * R) {   // below this level's window
            idle_through_lifting<WV>();
            px0 = 2 * g.cx0; py0 = 2 * g.cy0; pw = cw; ph = 2 * (g.cy1 - g.cy0);
            __syncthreads();
            continue;
        }
        Quads<ROWS, QPL> q;
        if (m == 0) {
            inv_load_at<QPL, ROWS, TLL, TB>(q, prm, qx, qy0);
        } else {
            // LL from the previous (coarser) level's output in LDS; the detail
            // bands from the pyramid. Each phase is extended on its own grid.
            const float *src = pxbuf[(m - 1) & 1];
            const int xe = mirror(2 * qx, prm.w) >> 1;
            const int xo = (mirror(2 * qx + 1, prm.w) - 1) >> 1;
            const int xl = clamp_to(xe, px0, pw);
            const uint32_t oe = (uint32_t)xe * sizeof(TB), oo = (uint32_t)xo * sizeof(TB);
            if (qy0 >= 0 && 2 * (qy0 + ROWS) <= prm.h) {
                // all rows inside the level (wavefront-uniform): both phases of
                // quad row gy are band row gy
                int64_t rb = (int64_t)qy0 * prm.band_pitch;
#pragma unroll
                for (int r = 0; r < ROWS; ++r) {
                    q.a[r][0] = src[clamp_to(qy0 + r, py0, ph) * pw + xl];
                    q.b[r][0] = load_elem<TB>(row_at<TB>(prm.hl, rb, prm.nqx), oo);
                    q.c[r][0] = load_elem<TB>(row_at<TB>(prm.lh, rb, prm.nqx), oe);
                    q.d[r][0] = load_elem<TB>(row_at<TB>(prm.hh, rb, prm.nqx), oo);
                    rb += prm.band_pitch;
                }
            } else {
#pragma unroll
                for (int r = 0; r < ROWS; ++r) {
                    const int gy = qy0 + r;
                    const int ye = mirror(2 * gy, prm.h) >> 1;
                    const int yo = (mirror(2 * gy + 1, prm.h) - 1) >> 1;
                    q.a[r][0] = src[clamp_to(ye, py0, ph) * pw + xl];
                    q.b[r][0] = load_elem<TB>(row_rsrc<TB>(prm.hl, ye, prm.band_pitch, prm.nqx), oo);
                    q.c[r][0] = load_elem<TB>(row_rsrc<TB>(prm.lh, yo, prm.band_pitch, prm.nqx), oe);
                    q.d[r][0] = load_elem<TB>(row_rsrc<TB>(prm.hh, yo, prm.band_pitch, prm.nqx), oo);
                }
            }
        }
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            q.a[r][0] *= uLL; q.b[r][0] *= uHL; q.c[r][0] *= uHL; q.d[r][0] *= uHH;
        }
        Exchange<ROWS, QPL, WAVES> x{&box, wave, lane, 0};
        lift_inverse<WV, SCH>(q, x);
        const bool last = m == F - 1;
        float *dst = pxbuf[m & 1];
        const uint32_t oo = (qx >= g.ox0 && qx < g.ox1) ? 2u * (uint32_t)qx * sizeof(TOUT)
                                                        : kNoAccess;
        const bool comp_x = qx >= g.cx0 && qx < g.cx1;
        int64_t ro = (int64_t)(2 * qy0) * prm.out_pitch;   // pixel row 2 gy
#pragma unroll
        for (int r = 0; r < ROWS; ++r, ro += 2 * prm.out_pitch) {
            const int gy = qy0 + r;
            if (last) {
                if (gy >= g.oy0 && gy < g.oy1) {   // wavefront-uniform
                    const rsrc_t r0 = row_at<TOUT>(prm.out, ro, prm.w);
                    const rsrc_t r1 = row_at<TOUT>(prm.out, ro + prm.out_pitch, prm.w);
                    if (prm.vec_out) {
                        const float e[2] = {q.a[r][0], q.b[r][0]};
                        const float o[2] = {q.c[r][0], q.d[r][0]};
                        store_vec<TOUT, 2>(r0, oo, e);
                        store_vec<TOUT, 2>(r1, oo, o);
                    } else {
                        store_elem<TOUT>(r0, oo, q.a[r][0]);
                        store_elem<TOUT>(r0, oo + (uint32_t)sizeof(TOUT), q.b[r][0]);
                        store_elem<TOUT>(r1, oo, q.c[r][0]);
                        store_elem<TOUT>(r1, oo + (uint32_t)sizeof(TOUT), q.d[r][0]);
                    }
                }
            } else if (comp_x && gy >= g.cy0 && gy < g.cy1) {
                float *p0 = dst + (2 * (gy - g.cy0)) * cw + 2 * (qx - g.cx0);
                p0[0] = q.a[r][0]; p0[1] = q.b[r][0];
                p0[cw] = q.c[r][0]; p0[cw + 1] = q.d[r][0];
            }
        }
        px0 = 2 * g.cx0; py0 = 2 * g.cy0; pw = cw; ph = 2 * (g.cy1 - g.cy0);
        __syncthreads();   // this level's output is complete before the next level reads it
    }
}

}  // namespace dwt2

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
constexpr int kTailQPL = 1, kTailRows = 8, kTailWaves = 8;
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

// Index into an LDS region of `pw` x `ph` values with origin (x0, y0), with
// the position clamped into the region: lanes outside the computed area read
// some held value, and their results are never stored.
__device__ __forceinline__ int region_index(int x, int y, int x0, int y0, int pw, int ph) {
    const int cx = min(max(x - x0, 0), pw - 1);
    const int cy = min(max(y - y0, 0), ph - 1);
    return cy * pw + cx;
}

template <int WV, int SCH, typename TIN, typename TLL, typename TB>
__global__ __launch_bounds__(64 * kTailWaves) void fwd_tail_kernel(FwdTail t) {
    constexpr int QPL = kTailQPL, ROWS = kTailRows, WAVES = kTailWaves;
    constexpr int R = Wavelet<WV>::NPAIRS;
    using L = Wavelet<WV>;
    __shared__ Mailbox<QPL, WAVES> box;
    __shared__ float llbuf[2][kTailBuf];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int bx = blockIdx.x % t.blocks_x, by = blockIdx.x / t.blocks_x;
    const float sLL = (float)(L::ZL * L::ZL), sHL = (float)(L::ZL * L::ZH);
    const float sHH = (float)(L::ZH * L::ZH);
    int px0 = 0, py0 = 0, pw = 1, ph = 1;       // previous level's LL region in LDS
    for (int m = 0; m < t.F; ++m) {
        const FwdParams &prm = t.lv[m];
        const Region g = tail_region(bx, by, t.B << (t.F - 1 - m), t.e[m], prm.nqx, prm.nqy);
        const int qx = g.cx0 - R + lane;          // the lane's quad column
        const int qy0 = g.cy0 - R + wave * ROWS;  // its first quad row
        Quads<ROWS, QPL> q;
        if (m == 0) {
            fwd_load_at<QPL, ROWS, TIN>(q, prm, qx, qy0);
        } else {
            const float *src = llbuf[(m - 1) & 1];
            const int xe = mirror(2 * qx, prm.w), xo = mirror(2 * qx + 1, prm.w);
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const int ye = mirror(2 * (qy0 + r), prm.h);
                const int yo = mirror(2 * (qy0 + r) + 1, prm.h);
                q.a[r][0] = src[region_index(xe, ye, px0, py0, pw, ph)];
                q.b[r][0] = src[region_index(xo, ye, px0, py0, pw, ph)];
                q.c[r][0] = src[region_index(xe, yo, px0, py0, pw, ph)];
                q.d[r][0] = src[region_index(xo, yo, px0, py0, pw, ph)];
            }
        }
        Exchange<ROWS, QPL, WAVES> x{&box, wave, lane, 0};
        lift_forward<WV, SCH>(q, x);
        const bool last = m == t.F - 1;
        const bool own_x = qx >= g.ox0 && qx < g.ox1;
        const bool comp_x = qx >= g.cx0 && qx < g.cx1;
        const int cw = g.cx1 - g.cx0;
        float *dst = llbuf[m & 1];
        TB *hl = static_cast<TB *>(prm.hl);
        TB *lh = static_cast<TB *>(prm.lh);
        TB *hh = static_cast<TB *>(prm.hh);
        TLL *llg = static_cast<TLL *>(prm.ll);
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int gy = qy0 + r;
            const float va = q.a[r][0] * sLL, vb = q.b[r][0] * sHL;
            const float vc = q.c[r][0] * sHL, vd = q.d[r][0] * sHH;
            if (own_x && gy >= g.oy0 && gy < g.oy1) {
                const int64_t ob = (int64_t)gy * prm.band_pitch + qx;
                hl[ob] = from_float<TB>(vb);
                lh[ob] = from_float<TB>(vc);
                hh[ob] = from_float<TB>(vd);
                if (last) llg[(int64_t)gy * prm.ll_pitch + qx] = from_float<TLL>(va);
            }
            if (!last && comp_x && gy >= g.cy0 && gy < g.cy1)
                dst[(gy - g.cy0) * cw + (qx - g.cx0)] = va;
        }
        px0 = g.cx0; py0 = g.cy0; pw = cw; ph = g.cy1 - g.cy0;
        __syncthreads();   // this level's LL is complete before the next level reads it
    }
}

template <int WV, int SCH, typename TLL, typename TB, typename TOUT>
__global__ __launch_bounds__(64 * kTailWaves) void inv_tail_kernel(InvTail t) {
    constexpr int QPL = kTailQPL, ROWS = kTailRows, WAVES = kTailWaves;
    constexpr int R = Wavelet<WV>::NPAIRS;
    using L = Wavelet<WV>;
    __shared__ Mailbox<QPL, WAVES> box;
    __shared__ float pxbuf[2][kTailBuf];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int bx = blockIdx.x % t.blocks_x, by = blockIdx.x / t.blocks_x;
    const float uLL = (float)(1.0 / (L::ZL * L::ZL)), uHL = (float)(1.0 / (L::ZL * L::ZH));
    const float uHH = (float)(1.0 / (L::ZH * L::ZH));
    int px0 = 0, py0 = 0, pw = 1, ph = 1;       // previous level's output region in LDS
    for (int m = 0; m < t.F; ++m) {
        const InvParams &prm = t.lv[m];
        const Region g = tail_region(bx, by, t.B << m, t.e[m], prm.nqx, prm.nqy);
        const int qx = g.cx0 - R + lane;
        const int qy0 = g.cy0 - R + wave * ROWS;
        Quads<ROWS, QPL> q;
        if (m == 0) {
            inv_load_at<QPL, ROWS, TLL, TB>(q, prm, qx, qy0);
        } else {
            // LL from the previous (coarser) level's output in LDS; the detail
            // bands from the pyramid. Each phase is extended on its own grid.
            const float *src = pxbuf[(m - 1) & 1];
            const TB *hl = static_cast<const TB *>(prm.hl);
            const TB *lh = static_cast<const TB *>(prm.lh);
            const TB *hh = static_cast<const TB *>(prm.hh);
            const int xe = mirror(2 * qx, prm.w) >> 1;
            const int xo = (mirror(2 * qx + 1, prm.w) - 1) >> 1;
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const int gy = qy0 + r;
                const int ye = mirror(2 * gy, prm.h) >> 1;
                const int yo = (mirror(2 * gy + 1, prm.h) - 1) >> 1;
                q.a[r][0] = src[region_index(xe, ye, px0, py0, pw, ph)];
                q.b[r][0] = to_float(hl[(int64_t)ye * prm.band_pitch + xo]);
                q.c[r][0] = to_float(lh[(int64_t)yo * prm.band_pitch + xe]);
                q.d[r][0] = to_float(hh[(int64_t)yo * prm.band_pitch + xo]);
            }
        }
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            q.a[r][0] *= uLL; q.b[r][0] *= uHL; q.c[r][0] *= uHL; q.d[r][0] *= uHH;
        }
        Exchange<ROWS, QPL, WAVES> x{&box, wave, lane, 0};
        lift_inverse<WV, SCH>(q, x);
        const bool last = m == t.F - 1;
        const int cw = 2 * (g.cx1 - g.cx0);
        float *dst = pxbuf[m & 1];
        TOUT *out = static_cast<TOUT *>(prm.out);
        const bool own_x = qx >= g.ox0 && qx < g.ox1;
        const bool comp_x = qx >= g.cx0 && qx < g.cx1;
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int gy = qy0 + r;
            if (last) {
                if (own_x && gy >= g.oy0 && gy < g.oy1) {
                    TOUT *r0 = out + (int64_t)(2 * gy) * prm.out_pitch + 2 * qx;
                    TOUT *r1 = r0 + prm.out_pitch;
                    r0[0] = from_float<TOUT>(q.a[r][0]); r0[1] = from_float<TOUT>(q.b[r][0]);
                    r1[0] = from_float<TOUT>(q.c[r][0]); r1[1] = from_float<TOUT>(q.d[r][0]);
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

// Streaming one-level 2-D DWT kernels for gfx950.
//
// One wavefront walks down a vertical strip of the level, one quad row at a
// time. Lane l owns QPL consecutive quads of every row; the HXL lanes at each
// edge of the wavefront are the horizontal lifting halo. Each lifting step of
// the level (Sec. 2 separable steps or Sec. 3 non-separable steps) is applied
// to a row as soon as the rows it reads are ready:
//   * a "down" step (T_P, T_P^V) reads the row below at the previous stage,
//     so it runs one row behind the step before it;
//   * an "up" step (S_U, S_U^V) reads the row above at the previous stage;
//     that row already moved on, so its two components the step reads (c, d)
//     are saved just before the step is applied to it;
//   * a horizontal step (T_P^H, S_U^H) needs only DPP lane shifts.
// After the last step the row that entered LAG rows earlier is finished and
// is written out. Rows live in one ring of D register slots from the moment
// they are prefetched until they are written, so a strip segment of any
// length costs no LDS, no barrier and no register copies, and its vertical
// halo (one row per lifting pair at each end) is paid once per segment
// instead of once per tile.
#pragma once

#include "dwt2_device.hpp"
#include "dwt2_kernels.hpp"

namespace dwt2 {

enum : int { K_T = 0, K_S = 1, K_TH = 2, K_TV = 3, K_SH = 4, K_SV = 5 };

// The lifting steps of one level, in execution order.
template <int WV, int SCH, bool INV>
struct StepList {
    using L = Wavelet<WV>;
    static constexpr int NP = L::NPAIRS;
    static constexpr int PER = SCH == NONSEP ? 2 : 4;
    static constexpr int N = NP * PER;
    __host__ __device__ static constexpr int kind(int k) {
        const int f = INV ? N - 1 - k : k;
        const int sub = f % PER;
        if (SCH == NONSEP) return sub == 0 ? K_T : K_S;
        return sub == 0 ? K_TH : sub == 1 ? K_TV : sub == 2 ? K_SH : K_SV;
    }
    __host__ __device__ static constexpr double coef(int k) {
        const int f = INV ? N - 1 - k : k;
        const int pair = f / PER, sub = f % PER;
        const bool predict = SCH == NONSEP ? sub == 0 : sub < 2;
        const double c = predict ? L::p(pair) : L::u(pair);
        return INV ? -c : c;
    }
    __host__ __device__ static constexpr bool down(int k) {
        return kind(k) == K_T || kind(k) == K_TV;
    }
    __host__ __device__ static constexpr bool up(int k) {
        return kind(k) == K_S || kind(k) == K_SV;
    }
    // rows behind the newest row at which step k runs
    __host__ __device__ static constexpr int lag(int k) {
        int l = 0;
        for (int i = 0; i <= k; ++i) l += down(i) ? 1 : 0;
        return l;
    }
    __host__ __device__ static constexpr int up_slot(int k) {
        int n = 0;
        for (int i = 0; i < k; ++i) n += up(i) ? 1 : 0;
        return n;
    }
    static constexpr int LAG = lag(N - 1);
    static constexpr int NUP = up_slot(N);
};

template <int QPL>
struct Row {
    float a[QPL], b[QPL], c[QPL], d[QPL];
};

template <int QPL>
struct Saved {
    float c[QPL], d[QPL];
};

// ---- one step on one row --------------------------------------------------------
// Non-separable T_P with the constant split: spatial T_{P1} (right and lower
// neighbours, pre-step values) then T^H_{P0}, T^V_{P0} on the own quad.
template <int QPL>
__device__ __forceinline__ void row_nonsep_predict(Row<QPL> &x, const Row<QPL> &dn, float p) {
    const float pp = p * p;
    const float aR = from_right(x.a[0]);
    const float cR = from_right(x.c[0]);
    const float adR = from_right(dn.a[0]);
#pragma unroll
    for (int i = 0; i < QPL; ++i) {
        const int j = (i + 1 < QPL) ? i + 1 : i;
        const float ar = (i + 1 < QPL) ? x.a[j] : aR;
        const float cr = (i + 1 < QPL) ? x.c[j] : cR;
        const float adr = (i + 1 < QPL) ? dn.a[j] : adR;
        const float a = x.a[i];
        float b = fmaf(p, ar, x.b[i]);
        float c = fmaf(p, dn.a[i], x.c[i]);
        float d = fmaf(p, cr, x.d[i]);
        d = fmaf(p, dn.b[i], d);
        d = fmaf(pp, adr, d);
        b = fmaf(p, a, b);
        d = fmaf(p, c, d);
        c = fmaf(p, a, c);
        d = fmaf(p, b, d);
        x.b[i] = b; x.c[i] = c; x.d[i] = d;
    }
}

// Non-separable S_U with the constant split: spatial S_{U1} (left and upper
// neighbours, pre-step values) then S^H_{U0}, S^V_{U0} on the own quad.
template <int QPL>
__device__ __forceinline__ void row_nonsep_update(Row<QPL> &x, const Saved<QPL> &up, float u) {
    const float uu = u * u;
    const float bL = from_left(x.b[QPL - 1]);
    const float dL = from_left(x.d[QPL - 1]);
    const float duL = from_left(up.d[QPL - 1]);
#pragma unroll
    for (int i = QPL - 1; i >= 0; --i) {
        const int j = (i > 0) ? i - 1 : i;
        const float bl = (i > 0) ? x.b[j] : bL;
        const float dl = (i > 0) ? x.d[j] : dL;
        const float dul = (i > 0) ? up.d[j] : duL;
        const float d = x.d[i];
        float a = fmaf(u, bl, x.a[i]);
        a = fmaf(u, up.c[i], a);
        a = fmaf(uu, dul, a);
        float b = fmaf(u, up.d[i], x.b[i]);
        float c = fmaf(u, dl, x.c[i]);
        a = fmaf(u, b, a);
        c = fmaf(u, d, c);
        a = fmaf(u, c, a);
        b = fmaf(u, d, b);
        x.a[i] = a; x.b[i] = b; x.c[i] = c;
    }
}

// Separable T^H_P: b += P a, d += P c.
template <int QPL>
__device__ __forceinline__ void row_sep_predict_h(Row<QPL> &x, float p) {
    const float aR = from_right(x.a[0]);
    const float cR = from_right(x.c[0]);
#pragma unroll
    for (int i = 0; i < QPL; ++i) {
        const int j = (i + 1 < QPL) ? i + 1 : i;
        const float ar = (i + 1 < QPL) ? x.a[j] : aR;
        const float cr = (i + 1 < QPL) ? x.c[j] : cR;
        x.b[i] = fmaf(p, ar, fmaf(p, x.a[i], x.b[i]));
        x.d[i] = fmaf(p, cr, fmaf(p, x.c[i], x.d[i]));
    }
}

// Separable T^V_P: c += P* a, d += P* b.
template <int QPL>
__device__ __forceinline__ void row_sep_predict_v(Row<QPL> &x, const Row<QPL> &dn, float p) {
#pragma unroll
    for (int i = 0; i < QPL; ++i) {
        x.c[i] = fmaf(p, dn.a[i], fmaf(p, x.a[i], x.c[i]));
        x.d[i] = fmaf(p, dn.b[i], fmaf(p, x.b[i], x.d[i]));
    }
}

// Separable S^H_U: a += U b, c += U d.
template <int QPL>
__device__ __forceinline__ void row_sep_update_h(Row<QPL> &x, float u) {
    const float bL = from_left(x.b[QPL - 1]);
    const float dL = from_left(x.d[QPL - 1]);
#pragma unroll
    for (int i = QPL - 1; i >= 0; --i) {
        const int j = (i > 0) ? i - 1 : i;
        const float bl = (i > 0) ? x.b[j] : bL;
        const float dl = (i > 0) ? x.d[j] : dL;
        x.a[i] = fmaf(u, bl, fmaf(u, x.b[i], x.a[i]));
        x.c[i] = fmaf(u, dl, fmaf(u, x.d[i], x.c[i]));
    }
}

// Separable S^V_U: a += U* c, b += U* d.
template <int QPL>
__device__ __forceinline__ void row_sep_update_v(Row<QPL> &x, const Saved<QPL> &up, float u) {
#pragma unroll
    for (int i = 0; i < QPL; ++i) {
        x.a[i] = fmaf(u, up.c[i], fmaf(u, x.c[i], x.a[i]));
        x.b[i] = fmaf(u, up.d[i], fmaf(u, x.d[i], x.b[i]));
    }
}

// Apply steps K.. of the list for the iteration whose newest row sits in ring
// slot S0. Step k works on the row that entered lag(k) iterations earlier
// (slot S0 - lag(k) mod D); an up step reads the pair its predecessor row
// saved (parity of that row) and saves its own pair for the row below.
// PAR is the parity of the newest row.
template <typename SL, int K, int S0, int PAR, int QPL, int D, int NS>
__device__ __forceinline__ void run_steps(Row<QPL> (&ring)[D], Saved<QPL> (&saved)[NS][2]) {
    if constexpr (K < SL::N) {
        constexpr int kind = SL::kind(K);
        constexpr int l = SL::lag(K);
        constexpr int slot = (S0 - l + D) % D;
        constexpr int below = (S0 - l + 1 + D) % D;
        constexpr int par = (PAR + l) & 1;      // parity of the row the step works on
        const float c = (float)SL::coef(K);
        if constexpr (kind == K_T) {
            row_nonsep_predict(ring[slot], ring[below], c);
        } else if constexpr (kind == K_TV) {
            row_sep_predict_v(ring[slot], ring[below], c);
        } else if constexpr (kind == K_TH) {
            row_sep_predict_h(ring[slot], c);
        } else if constexpr (kind == K_SH) {
            row_sep_update_h(ring[slot], c);
        } else {
            constexpr int s = SL::up_slot(K);
#pragma unroll
            for (int i = 0; i < QPL; ++i) {
                saved[s][par].c[i] = ring[slot].c[i];
                saved[s][par].d[i] = ring[slot].d[i];
            }
            if constexpr (kind == K_S)
                row_nonsep_update(ring[slot], saved[s][par ^ 1], c);
            else
                row_sep_update_v(ring[slot], saved[s][par ^ 1], c);
        }
        run_steps<SL, K + 1, S0, PAR>(ring, saved);
    }
}

// Geometry of a streaming configuration.
template <int WV, int QPL>
struct StreamGeom {
    static constexpr int NP = Wavelet<WV>::NPAIRS;
    static constexpr int HXL = (NP + QPL - 1) / QPL;      // halo lanes per side
    static constexpr int OX = (64 - 2 * HXL) * QPL;        // output quads per strip
};

// ---- row access ---------------------------------------------------------------
// Each row of a 2-D buffer is a wave-uniform buffer resource; lanes address it
// with 32-bit byte offsets. Accesses that must not happen are not branched
// around: a row outside the range a segment may touch gets a zero-length
// resource, and a lane that must not write (the horizontal halo, quads past
// the level edge) gets an offset beyond every row, so the hardware bounds
// check drops them. The loop body then has no branches, which lets the
// compiler keep the prefetched loads in flight across iterations.
//
// FastIO serves wavefronts whose whole window lies inside the level (one
// vector access per pixel row and lane); EdgeIO serves the others, gathering
// every sample through the symmetric extension with per-lane offsets computed
// once, since a column's mirror image does not depend on the row.

template <int WV, int QPL, typename TIN, typename TLL, typename TB>
struct FwdFastIO {
    const FwdParams &prm;
    uint32_t in_off, out_off;   // lane byte offsets in an input / band row
    int y_hi;                   // last row the segment may load
    int o_lo, o_hi;             // rows [o_lo, o_hi) are written

    __device__ __forceinline__ FwdFastIO(const FwdParams &p, int qx0, bool store_lane, int yh,
                                         int ol, int oh)
        : prm(p), y_hi(yh), o_lo(ol), o_hi(oh) {
        in_off = (uint32_t)(2 * qx0) * (uint32_t)sizeof(TIN);
        out_off = store_lane ? (uint32_t)qx0 * (uint32_t)sizeof(TB) : kNoAccess;
    }
    __device__ __forceinline__ void load(Row<QPL> &r, int y) const {
        const TIN *in = static_cast<const TIN *>(prm.in);
        const uint32_t rb = y <= y_hi ? (uint32_t)prm.w * (uint32_t)sizeof(TIN) : 0u;
        const int yc = min(y, y_hi);
        float e[2 * QPL], o[2 * QPL];
        load_vec<TIN, 2 * QPL>(make_rsrc(in + (int64_t)(2 * yc) * prm.in_pitch, rb), in_off, e);
        load_vec<TIN, 2 * QPL>(make_rsrc(in + (int64_t)(2 * yc + 1) * prm.in_pitch, rb), in_off, o);
#pragma unroll
        for (int i = 0; i < QPL; ++i) {
            r.a[i] = e[2 * i]; r.b[i] = e[2 * i + 1];
            r.c[i] = o[2 * i]; r.d[i] = o[2 * i + 1];
        }
    }
    __device__ __forceinline__ void store(const Row<QPL> &r, int yo) const {
        using L = Wavelet<WV>;
        const bool ok = yo >= o_lo && yo < o_hi;
        const int yc = min(max(yo, 0), prm.nqy - 1);
        float va[QPL], vb[QPL], vc[QPL], vd[QPL];
#pragma unroll
        for (int i = 0; i < QPL; ++i) {
            va[i] = r.a[i] * (float)(L::ZL * L::ZL);
            vb[i] = r.b[i] * (float)(L::ZL * L::ZH);
            vc[i] = r.c[i] * (float)(L::ZL * L::ZH);
            vd[i] = r.d[i] * (float)(L::ZH * L::ZH);
        }
        const uint32_t lb = ok ? (uint32_t)prm.nqx * (uint32_t)sizeof(TLL) : 0u;
        const uint32_t bb = ok ? (uint32_t)prm.nqx * (uint32_t)sizeof(TB) : 0u;
        const int64_t ob = (int64_t)yc * prm.band_pitch;
        const uint32_t loff = out_off == kNoAccess ? kNoAccess
                                                   : out_off / (uint32_t)sizeof(TB) * (uint32_t)sizeof(TLL);
        store_vec<TLL, QPL>(make_rsrc(static_cast<TLL *>(prm.ll) + (int64_t)yc * prm.ll_pitch, lb), loff, va);
        store_vec<TB, QPL>(make_rsrc(static_cast<TB *>(prm.hl) + ob, bb), out_off, vb);
        store_vec<TB, QPL>(make_rsrc(static_cast<TB *>(prm.lh) + ob, bb), out_off, vc);
        store_vec<TB, QPL>(make_rsrc(static_cast<TB *>(prm.hh) + ob, bb), out_off, vd);
    }
};

template <int WV, int QPL, typename TIN, typename TLL, typename TB>
struct FwdEdgeIO {
    const FwdParams &prm;
    uint32_t xe[QPL], xo[QPL];            // mirrored even / odd column byte offsets
    uint32_t sl[QPL], sb[QPL];            // store offsets (LL row, band row) or kNoAccess
    int y_hi, o_lo, o_hi;

    __device__ __forceinline__ FwdEdgeIO(const FwdParams &p, int qx0, bool store_lane, int yh,
                                         int ol, int oh)
        : prm(p), y_hi(yh), o_lo(ol), o_hi(oh) {
#pragma unroll
        for (int i = 0; i < QPL; ++i) {
            xe[i] = (uint32_t)mirror(2 * (qx0 + i), p.w) * (uint32_t)sizeof(TIN);
            xo[i] = (uint32_t)mirror(2 * (qx0 + i) + 1, p.w) * (uint32_t)sizeof(TIN);
            const bool w = store_lane && qx0 + i >= 0 && qx0 + i < p.nqx;
            sl[i] = w ? (uint32_t)(qx0 + i) * (uint32_t)sizeof(TLL) : kNoAccess;
            sb[i] = w ? (uint32_t)(qx0 + i) * (uint32_t)sizeof(TB) : kNoAccess;
        }
    }
    __device__ __forceinline__ void load(Row<QPL> &r, int y) const {
        const TIN *in = static_cast<const TIN *>(prm.in);
        const uint32_t rb = y <= y_hi ? (uint32_t)prm.w * (uint32_t)sizeof(TIN) : 0u;
        const int yc = min(y, y_hi);
        const rsrc_t r0 = make_rsrc(in + (int64_t)mirror(2 * yc, prm.h) * prm.in_pitch, rb);
        const rsrc_t r1 = make_rsrc(in + (int64_t)mirror(2 * yc + 1, prm.h) * prm.in_pitch, rb);
#pragma unroll
        for (int i = 0; i < QPL; ++i) {
            r.a[i] = load_elem<TIN>(r0, xe[i]); r.b[i] = load_elem<TIN>(r0, xo[i]);
            r.c[i] = load_elem<TIN>(r1, xe[i]); r.d[i] = load_elem<TIN>(r1, xo[i]);
        }
    }
    __device__ __forceinline__ void store(const Row<QPL> &r, int yo) const {
        using L = Wavelet<WV>;
        const bool ok = yo >= o_lo && yo < o_hi;
        const int yc = min(max(yo, 0), prm.nqy - 1);
        const uint32_t lb = ok ? (uint32_t)prm.nqx * (uint32_t)sizeof(TLL) : 0u;
        const uint32_t bb = ok ? (uint32_t)prm.nqx * (uint32_t)sizeof(TB) : 0u;
        const int64_t ob = (int64_t)yc * prm.band_pitch;
        const rsrc_t rl = make_rsrc(static_cast<TLL *>(prm.ll) + (int64_t)yc * prm.ll_pitch, lb);
        const rsrc_t r1 = make_rsrc(static_cast<TB *>(prm.hl) + ob, bb);
        const rsrc_t r2 = make_rsrc(static_cast<TB *>(prm.lh) + ob, bb);
        const rsrc_t r3 = make_rsrc(static_cast<TB *>(prm.hh) + ob, bb);
#pragma unroll
        for (int i = 0; i < QPL; ++i) {
            store_elem<TLL>(rl, sl[i], r.a[i] * (float)(L::ZL * L::ZL));
            store_elem<TB>(r1, sb[i], r.b[i] * (float)(L::ZL * L::ZH));
            store_elem<TB>(r2, sb[i], r.c[i] * (float)(L::ZL * L::ZH));
            store_elem<TB>(r3, sb[i], r.d[i] * (float)(L::ZH * L::ZH));
        }
    }
};

template <int WV, int QPL>
__device__ __forceinline__ void unscale(Row<QPL> &r) {
    using L = Wavelet<WV>;
    const float uLL = (float)(1.0 / (L::ZL * L::ZL)), uHL = (float)(1.0 / (L::ZL * L::ZH));
    const float uHH = (float)(1.0 / (L::ZH * L::ZH));
#pragma unroll
    for (int i = 0; i < QPL; ++i) {
        r.a[i] *= uLL; r.b[i] *= uHL; r.c[i] *= uHL; r.d[i] *= uHH;
    }
}

template <int WV, int QPL, typename TLL, typename TB, typename TOUT>
struct InvFastIO {
    const InvParams &prm;
    uint32_t ll_off, b_off, out_off;
    int y_hi, o_lo, o_hi;

    __device__ __forceinline__ InvFastIO(const InvParams &p, int qx0, bool store_lane, int yh,
                                         int ol, int oh)
        : prm(p), y_hi(yh), o_lo(ol), o_hi(oh) {
        ll_off = (uint32_t)qx0 * (uint32_t)sizeof(TLL);
        b_off = (uint32_t)qx0 * (uint32_t)sizeof(TB);
        out_off = store_lane ? (uint32_t)(2 * qx0) * (uint32_t)sizeof(TOUT) : kNoAccess;
    }
    __device__ __forceinline__ void load(Row<QPL> &r, int y) const {
        const bool ok = y <= y_hi;
        const int yc = min(y, y_hi);
        const uint32_t lb = ok ? (uint32_t)prm.nqx * (uint32_t)sizeof(TLL) : 0u;
        const uint32_t bb = ok ? (uint32_t)prm.nqx * (uint32_t)sizeof(TB) : 0u;
        const int64_t ob = (int64_t)yc * prm.band_pitch;
        load_vec<TLL, QPL>(make_rsrc(static_cast<const TLL *>(prm.ll) + (int64_t)yc * prm.ll_pitch, lb),
                           ll_off, r.a);
        load_vec<TB, QPL>(make_rsrc(static_cast<const TB *>(prm.hl) + ob, bb), b_off, r.b);
        load_vec<TB, QPL>(make_rsrc(static_cast<const TB *>(prm.lh) + ob, bb), b_off, r.c);
        load_vec<TB, QPL>(make_rsrc(static_cast<const TB *>(prm.hh) + ob, bb), b_off, r.d);
        unscale<WV, QPL>(r);
    }
    __device__ __forceinline__ void store(const Row<QPL> &r, int yo) const {
        const bool ok = yo >= o_lo && yo < o_hi;
        const int yc = min(max(yo, 0), prm.nqy - 1);
        const uint32_t rb = ok ? (uint32_t)prm.w * (uint32_t)sizeof(TOUT) : 0u;
        float e[2 * QPL], o[2 * QPL];
#pragma unroll
        for (int i = 0; i < QPL; ++i) {
            e[2 * i] = r.a[i]; e[2 * i + 1] = r.b[i];
            o[2 * i] = r.c[i]; o[2 * i + 1] = r.d[i];
        }
        TOUT *r0 = static_cast<TOUT *>(prm.out) + (int64_t)(2 * yc) * prm.out_pitch;
        store_vec<TOUT, 2 * QPL>(make_rsrc(r0, rb), out_off, e);
        store_vec<TOUT, 2 * QPL>(make_rsrc(r0 + prm.out_pitch, rb), out_off, o);
    }
};

template <int WV, int QPL, typename TLL, typename TB, typename TOUT>
struct InvEdgeIO {
    const InvParams &prm;
    uint32_t le[QPL], bo[QPL], be[QPL];   // LL (even col), odd-col and even-col band offsets
    uint32_t se[QPL], so[QPL];            // output offsets of the even / odd pixel, or kNoAccess
    int y_hi, o_lo, o_hi;

    __device__ __forceinline__ InvEdgeIO(const InvParams &p, int qx0, bool store_lane, int yh,
                                         int ol, int oh)
        : prm(p), y_hi(yh), o_lo(ol), o_hi(oh) {
#pragma unroll
        for (int i = 0; i < QPL; ++i) {
            const uint32_t xe = (uint32_t)(mirror(2 * (qx0 + i), p.w) >> 1);
            const uint32_t xo = (uint32_t)((mirror(2 * (qx0 + i) + 1, p.w) - 1) >> 1);
            le[i] = xe * (uint32_t)sizeof(TLL);
            be[i] = xe * (uint32_t)sizeof(TB);
            bo[i] = xo * (uint32_t)sizeof(TB);
            const bool w = store_lane && qx0 + i >= 0 && qx0 + i < p.nqx;
            se[i] = w ? (uint32_t)(2 * (qx0 + i)) * (uint32_t)sizeof(TOUT) : kNoAccess;
            so[i] = w ? (uint32_t)(2 * (qx0 + i) + 1) * (uint32_t)sizeof(TOUT) : kNoAccess;
        }
    }
    __device__ __forceinline__ void load(Row<QPL> &r, int y) const {
        const bool ok = y <= y_hi;
        const int yc = min(y, y_hi);
        const int ye = mirror(2 * yc, prm.h) >> 1;
        const int yo = (mirror(2 * yc + 1, prm.h) - 1) >> 1;
        const uint32_t lb = ok ? (uint32_t)prm.nqx * (uint32_t)sizeof(TLL) : 0u;
        const uint32_t bb = ok ? (uint32_t)prm.nqx * (uint32_t)sizeof(TB) : 0u;
        const rsrc_t rl = make_rsrc(static_cast<const TLL *>(prm.ll) + (int64_t)ye * prm.ll_pitch, lb);
        const rsrc_t rh = make_rsrc(static_cast<const TB *>(prm.hl) + (int64_t)ye * prm.band_pitch, bb);
        const rsrc_t rv = make_rsrc(static_cast<const TB *>(prm.lh) + (int64_t)yo * prm.band_pitch, bb);
        const rsrc_t rd = make_rsrc(static_cast<const TB *>(prm.hh) + (int64_t)yo * prm.band_pitch, bb);
#pragma unroll
        for (int i = 0; i < QPL; ++i) {
            r.a[i] = load_elem<TLL>(rl, le[i]);
            r.b[i] = load_elem<TB>(rh, bo[i]);
            r.c[i] = load_elem<TB>(rv, be[i]);
            r.d[i] = load_elem<TB>(rd, bo[i]);
        }
        unscale<WV, QPL>(r);
    }
    __device__ __forceinline__ void store(const Row<QPL> &r, int yo) const {
        const bool ok = yo >= o_lo && yo < o_hi;
        const int yc = min(max(yo, 0), prm.nqy - 1);
        const uint32_t rb = ok ? (uint32_t)prm.w * (uint32_t)sizeof(TOUT) : 0u;
        TOUT *r0 = static_cast<TOUT *>(prm.out) + (int64_t)(2 * yc) * prm.out_pitch;
        const rsrc_t s0 = make_rsrc(r0, rb), s1 = make_rsrc(r0 + prm.out_pitch, rb);
#pragma unroll
        for (int i = 0; i < QPL; ++i) {
            store_elem<TOUT>(s0, se[i], r.a[i]); store_elem<TOUT>(s0, so[i], r.b[i]);
            store_elem<TOUT>(s1, se[i], r.c[i]); store_elem<TOUT>(s1, so[i], r.d[i]);
        }
    }
};

// ---- the streaming pipeline, shared by both directions -----------------------------
// Iteration i brings row y_first + i (loaded earlier into ring slot i mod D)
// into the pipeline, runs every step on the rows in flight, writes the row
// that entered LAG iterations earlier and refills its slot with the row
// D - LAG iterations ahead. The loop is unrolled by D (even), so ring slots
// and the parity of the saved pairs are compile-time constants; iterations
// past the segment end compute on zero rows whose stores are dropped.
template <typename SL, int QPL, int D, int NS, int K, typename IO>
__device__ __forceinline__ void stream_iters(Row<QPL> (&ring)[D], Saved<QPL> (&saved)[NS][2],
                                             int y, const IO &io) {
    if constexpr (K < D) {
        constexpr int LAG = SL::LAG;
        run_steps<SL, 0, K, K & 1>(ring, saved);
        constexpr int fin = (K - LAG + D) % D;
        io.store(ring[fin], y + K - LAG);
        io.load(ring[fin], y + K + D - LAG);
        // keep iterations in program order: a row's lifting must not be
        // hoisted next to the loads of rows it does not need yet, which
        // would make the loop wait for the whole prefetch ring
        __builtin_amdgcn_sched_barrier(0);
        stream_iters<SL, QPL, D, NS, K + 1>(ring, saved, y, io);
    }
}

template <typename SL, int QPL, int D, typename IO>
__device__ __forceinline__ void stream_segment(int y0, int y_end_out, const IO &io) {
    constexpr int LAG = SL::LAG;
    constexpr int NS = SL::NUP > 0 ? SL::NUP : 1;
    static_assert(D % 2 == 0 && D >= LAG + 2, "ring too small for the pipeline");
    const int y_first = y0 - SL::NUP;              // rows above y0 whose lifting is needed
    const int n_iter = (y_end_out - y0) + SL::NUP + LAG;

    Row<QPL> ring[D];
    Saved<QPL> saved[NS][2];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        if (k < D - LAG) {
            io.load(ring[k], y_first + k);
        } else {
#pragma unroll
            for (int i = 0; i < QPL; ++i) ring[k].a[i] = ring[k].b[i] = ring[k].c[i] = ring[k].d[i] = 0.f;
        }
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
#pragma unroll
        for (int p = 0; p < 2; ++p) {
#pragma unroll
            for (int i = 0; i < QPL; ++i) { saved[s][p].c[i] = 0.f; saved[s][p].d[i] = 0.f; }
        }
    }
    // The first block is peeled so that the loop is entered with the same
    // loads and stores in flight as at its back edge; the waits the compiler
    // derives then only cover the row each iteration consumes.
    stream_iters<SL, QPL, D, NS, 0>(ring, saved, y_first, io);
    for (int ib = D; ib < n_iter; ib += D)
        stream_iters<SL, QPL, D, NS, 0>(ring, saved, y_first + ib, io);
}

// Each wavefront of the workgroup processes one segment; tasks are numbered
// row-major over (segment row, strip), so each XCD sweeps a horizontal band. prm.tiles_x = strips, prm.tiles_y = segments
// per strip, prm.seg = output rows per segment.
template <int WV, int SCH, int QPL, int D, int WAVES, typename TIN, typename TLL, typename TB>
__global__ __launch_bounds__(64 * WAVES) void fwd_stream_kernel(FwdParams prm) {
    using SL = StepList<WV, SCH, false>;
    using GM = StreamGeom<WV, QPL>;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform per wavefront
    const int task = xcd_contiguous_tile(blockIdx.x, gridDim.x) * WAVES + wave;
    if (task >= prm.tiles_x * prm.tiles_y) return;
    const int sy = task / prm.tiles_x;             // row-major over (segment, strip)
    const int sx = task - sy * prm.tiles_x;
    const int qx0 = sx * GM::OX + (lane - GM::HXL) * QPL;
    const int y0 = sy * prm.seg;
    const int y_end = min(y0 + prm.seg, prm.nqy);
    const int y_hi = y_end - 1 + SL::LAG;            // last row the pipeline needs
    const bool store_lane = lane >= GM::HXL && lane < 64 - GM::HXL;
    const int wx0 = sx * GM::OX - GM::HXL * QPL;     // first quad column of the wavefront
    const bool fast = prm.vec_in && prm.vec_ll && prm.vec_band && wx0 >= 0 &&
                      wx0 + 64 * QPL <= prm.nqx && y0 - SL::NUP >= 0 && y_hi < prm.nqy;
    if (fast) {
        const FwdFastIO<WV, QPL, TIN, TLL, TB> io(prm, qx0, store_lane, y_hi, y0, y_end);
        stream_segment<SL, QPL, D>(y0, y_end, io);
    } else {
        const FwdEdgeIO<WV, QPL, TIN, TLL, TB> io(prm, qx0, store_lane, y_hi, y0, y_end);
        stream_segment<SL, QPL, D>(y0, y_end, io);
    }
}

template <int WV, int SCH, int QPL, int D, int WAVES, typename TLL, typename TB, typename TOUT>
__global__ __launch_bounds__(64 * WAVES) void inv_stream_kernel(InvParams prm) {
    using SL = StepList<WV, SCH, true>;
    using GM = StreamGeom<WV, QPL>;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform per wavefront
    const int task = xcd_contiguous_tile(blockIdx.x, gridDim.x) * WAVES + wave;
    if (task >= prm.tiles_x * prm.tiles_y) return;
    const int sy = task / prm.tiles_x;             // row-major over (segment, strip)
    const int sx = task - sy * prm.tiles_x;
    const int qx0 = sx * GM::OX + (lane - GM::HXL) * QPL;
    const int y0 = sy * prm.seg;
    const int y_end = min(y0 + prm.seg, prm.nqy);
    const int y_hi = y_end - 1 + SL::LAG;
    const bool store_lane = lane >= GM::HXL && lane < 64 - GM::HXL;
    const int wx0 = sx * GM::OX - GM::HXL * QPL;
    const bool fast = prm.vec_ll && prm.vec_band && prm.vec_out && wx0 >= 0 &&
                      wx0 + 64 * QPL <= prm.nqx && y0 - SL::NUP >= 0 && y_hi < prm.nqy;
    if (fast) {
        const InvFastIO<WV, QPL, TLL, TB, TOUT> io(prm, qx0, store_lane, y_hi, y0, y_end);
        stream_segment<SL, QPL, D>(y0, y_end, io);
    } else {
        const InvEdgeIO<WV, QPL, TLL, TB, TOUT> io(prm, qx0, store_lane, y_hi, y0, y_end);
        stream_segment<SL, QPL, D>(y0, y_end, io);
    }
}

}  // namespace dwt2

// One-level forward and inverse 2-D DWT kernels for gfx950.
//
// One launch computes one level: each workgroup reads its window of the level
// input once from HBM (coalesced vector loads straight into registers, the
// lifting halo included), runs every lifting step of the level in registers
// (non-separable: S_U | T_P per lifting pair, Sec. 3; separable:
// S_U^V | S_U^H | T_P^V | T_P^H, Sec. 2), scales, and writes the centre of
// the window: the four bands (forward) or the interleaved pixels (inverse).
#pragma once

#include "dwt2_device.hpp"

namespace dwt2 {

// Parameters of one forward level. The input is w x h pixels (even), the
// outputs are nqx x nqy = (w/2) x (h/2) quads per band.
struct FwdParams {
    const void *in;
    int64_t in_pitch;
    void *ll;
    int64_t ll_pitch;
    void *hl, *lh, *hh;
    int64_t band_pitch;
    int32_t w, h, nqx, nqy;
    int32_t tiles_x, tiles_y;
    int32_t vec_in, vec_ll, vec_band;   // 1 when vector accesses are aligned
};

struct InvParams {
    const void *ll;
    int64_t ll_pitch;
    const void *hl, *lh, *hh;
    int64_t band_pitch;
    void *out;
    int64_t out_pitch;
    int32_t w, h, nqx, nqy;
    int32_t tiles_x, tiles_y;
    uint8_t vec_ll, vec_band, vec_out;   // 1 when vector accesses are aligned
    uint8_t stream_out;                  // 1: vector output stores are non-temporal
};

// Geometry of a tile configuration. The horizontal halo is one lane's worth
// of quads on each side (>= the number of lifting pairs), which keeps every
// lane's loads and stores aligned to its vector width; the vertical halo is
// one quad row per lifting pair.
template <int WV, int QPL, int ROWS, int WAVES>
struct TileGeom {
    static constexpr int NP = Wavelet<WV>::NPAIRS;
    static constexpr int HX = QPL;
    static constexpr int HY = NP;
    static constexpr int OX = 64 * QPL - 2 * HX;
    static constexpr int OY = WAVES * ROWS - 2 * HY;
    static_assert(HX >= NP, "horizontal halo must cover the lifting support");
    static_assert(OY > 0, "tile too short for the lifting halo");
};

// The hardware hands consecutive workgroup ids to the 8 XCDs in turn. Remap
// the ids so that the workgroups of one XCD are numbered contiguously; with
// contiguous tile runs per workgroup, each XCD then works on one contiguous
// region of the image and the halo rows shared by neighbouring tiles stay in
// that XCD's L2.
__device__ __forceinline__ int xcd_contiguous_tile(int b, int n) {
    const int per = n >> 3, rem = n & 7;
    const int xcd = b & 7, idx = b >> 3;
    return xcd * per + (xcd < rem ? xcd : rem) + idx;
}

// Tiles are numbered row-major; with the XCD-contiguous block numbering each
// XCD sweeps one horizontal band of the level, so the rows it has in flight
// are few and whole (DRAM page locality), and horizontally adjacent tiles,
// which share partial cache lines at their edges, meet in the same L2.
__device__ __forceinline__ int block_tile() {
    return xcd_contiguous_tile(blockIdx.x, gridDim.x);
}

// ---- forward: load / store of one tile ----------------------------------------
// Column access of one lane at the level edge. A lane reads E consecutive
// elements starting at column x0; outside [0, n) each element stands for its
// symmetric-extension mirror. The mirrored columns of E consecutive positions
// lie within E consecutive indices, so two aligned E-element vector loads
// (at `base` and base + E) cover them and a per-lane select rebuilds the
// lane's values. Lanes inside the level read their E elements with the first
// load alone (the second is dropped by the buffer hardware). Every lane
// issues the same loads, so no load sits in a divergent or lane-dependent
// branch: the loads of all rows stay in flight together.
template <int E>
struct EdgeCols {
    uint32_t off_a, off_b;   // byte offsets of the two loads (kNoAccess: none)
    int sel[E];              // element k comes from index sel[k] of the 2E loaded
    bool plain;              // the lane reads its own E columns unchanged

    // m[k]: the column element k stands for (in [0, n)); plain: m[k] = x0 + k.
    template <typename T>
    __device__ __forceinline__ static EdgeCols from(const int (&m)[E], int x0, bool plain) {
        EdgeCols c;
        int lo = m[0];
#pragma unroll
        for (int k = 1; k < E; ++k) lo = min(lo, m[k]);
        c.plain = plain;
        const int base = plain ? x0 : (lo & ~(E - 1));
        c.off_a = (uint32_t)base * (uint32_t)sizeof(T);
        c.off_b = plain ? kNoAccess : (uint32_t)(base + E) * (uint32_t)sizeof(T);
#pragma unroll
        for (int k = 0; k < E; ++k) c.sel[k] = plain ? k : m[k] - base;
        return c;
    }
};

// Element i of the 2E values (a, b), as a bitwise select: exact, and kept in
// registers (a select chain over a runtime index would be lowered to an
// indexed access).
template <int E>
__device__ __forceinline__ float pick(const float (&a)[E], const float (&b)[E], int i) {
    uint32_t r = 0;
#pragma unroll
    for (int k = 0; k < E; ++k) r |= __float_as_uint(a[k]) & (0u - (uint32_t)(i == k));
#pragma unroll
    for (int k = 0; k < E; ++k) r |= __float_as_uint(b[k]) & (0u - (uint32_t)(i == E + k));
    return __uint_as_float(r);
}

// Completes the loads of `n` rows for the lanes of an edge wavefront: the
// second vector of each row, then the per-lane select. `v[r]` holds the
// first vector on entry and the lane's elements on exit.
template <typename T, int E, int N>
__device__ __forceinline__ void fix_cols(const rsrc_t (&rows)[N], const EdgeCols<E> &c,
                                         float (&v)[N][E]) {
    float b[N][E];
#pragma unroll
    for (int r = 0; r < N; ++r) load_vec<T, E>(rows[r], c.off_b, b[r]);
#pragma unroll
    for (int r = 0; r < N; ++r) {
        float a[E];
#pragma unroll
        for (int k = 0; k < E; ++k) a[k] = v[r][k];
#pragma unroll
        for (int k = 0; k < E; ++k) v[r][k] = pick<E>(a, b[r], c.sel[k]);
    }
}

// The lane's quads start at quad column qx0 and quad row qy0 of the level;
// positions outside the level are read through the symmetric extension.
template <int QPL, int ROWS, typename TIN>
__device__ __forceinline__ void fwd_load_at(Quads<ROWS, QPL> &q, const FwdParams &prm, int qx0,
                                            int qy0) {
    const TIN *in = static_cast<const TIN *>(prm.in);
    const int px0 = 2 * qx0;
    // vector loads need aligned rows whose length is a multiple of the lane's
    // E elements, so that no vector is partly outside the row
    if (!prm.vec_in || (prm.w & (2 * QPL - 1)) != 0) {   // else one element at a time
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const TIN *r0 = in + (int64_t)mirror(2 * (qy0 + r), prm.h) * prm.in_pitch;
            const TIN *r1 = in + (int64_t)mirror(2 * (qy0 + r) + 1, prm.h) * prm.in_pitch;
#pragma unroll
            for (int i = 0; i < QPL; ++i) {
                const int xe = mirror(px0 + 2 * i, prm.w);
                const int xo = mirror(px0 + 2 * i + 1, prm.w);
                q.a[r][i] = to_float(r0[xe]); q.b[r][i] = to_float(r0[xo]);
                q.c[r][i] = to_float(r1[xe]); q.d[r][i] = to_float(r1[xo]);
            }
        }
        return;
    }
    int m[2 * QPL];
#pragma unroll
    for (int k = 0; k < 2 * QPL; ++k) m[k] = mirror(px0 + k, prm.w);
    const EdgeCols<2 * QPL> cols = EdgeCols<2 * QPL>::template from<TIN>(
        m, px0, px0 >= 0 && px0 + 2 * QPL <= prm.w);
    const uint32_t rb = (uint32_t)prm.w * (uint32_t)sizeof(TIN);
    // all rows' first vectors, then (edge wavefronts only) the completion
    rsrc_t rows[2 * ROWS];
    float v[2 * ROWS][2 * QPL];
    if (2 * qy0 >= 0 && 2 * (qy0 + ROWS) <= prm.h) {
        // all rows inside the level (wavefront-uniform): step the row pointer
        // instead of mirroring and multiplying per row, so that the loads
        // issue sooner
        const TIN *p = in + (int64_t)(2 * qy0) * prm.in_pitch;
#pragma unroll
        for (int r = 0; r < 2 * ROWS; ++r) {
            rows[r] = make_rsrc(p, rb);
            load_vec<TIN, 2 * QPL>(rows[r], cols.off_a, v[r]);
            p += prm.in_pitch;
        }
    } else {
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int py = 2 * (qy0 + r);
            rows[2 * r] = make_rsrc(in + (int64_t)mirror(py, prm.h) * prm.in_pitch, rb);
            rows[2 * r + 1] = make_rsrc(in + (int64_t)mirror(py + 1, prm.h) * prm.in_pitch, rb);
            load_vec<TIN, 2 * QPL>(rows[2 * r], cols.off_a, v[2 * r]);
            load_vec<TIN, 2 * QPL>(rows[2 * r + 1], cols.off_a, v[2 * r + 1]);
        }
    }
    if (!wave_all(cols.plain)) fix_cols<TIN>(rows, cols, v);
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
#pragma unroll
        for (int i = 0; i < QPL; ++i) {
            q.a[r][i] = v[2 * r][2 * i]; q.b[r][i] = v[2 * r][2 * i + 1];
            q.c[r][i] = v[2 * r + 1][2 * i]; q.d[r][i] = v[2 * r + 1][2 * i + 1];
        }
    }
}

template <int QPL, int ROWS, typename G, typename TIN>
__device__ __forceinline__ void fwd_load(Quads<ROWS, QPL> &q, const FwdParams &prm, int t,
                                         int lane, int wave) {
    const int ty = t / prm.tiles_x, tx = t - (t / prm.tiles_x) * prm.tiles_x;
    fwd_load_at<QPL, ROWS, TIN>(q, prm, tx * G::OX - G::HX + lane * QPL,
                                ty * G::OY - G::HY + wave * ROWS);
}

template <int WV, int QPL, int ROWS, int WAVES, typename G, typename TLL, typename TB>
__device__ __forceinline__ void fwd_store(const Quads<ROWS, QPL> &q, const FwdParams &prm, int t,
                                          int lane, int wave) {
    using L = Wavelet<WV>;
    const float sLL = (float)(L::ZL * L::ZL), sHL = (float)(L::ZL * L::ZH);
    const float sHH = (float)(L::ZH * L::ZH);
    if (lane == 0 || lane == 63) return;   // halo lanes
    const int ty = t / prm.tiles_x, tx = t - (t / prm.tiles_x) * prm.tiles_x;
    const int qx0 = tx * G::OX - G::HX + lane * QPL;
    const int qy0 = ty * G::OY - G::HY + wave * ROWS;
    TLL *ll = static_cast<TLL *>(prm.ll);
    TB *hl = static_cast<TB *>(prm.hl);
    TB *lh = static_cast<TB *>(prm.lh);
    TB *hh = static_cast<TB *>(prm.hh);
    const bool full_x = qx0 + QPL <= prm.nqx;
    // element offsets of row qy0 + r, stepped
    int64_t rowb = (int64_t)qy0 * prm.band_pitch, rowl = (int64_t)qy0 * prm.ll_pitch;
#pragma unroll
    for (int r = 0; r < ROWS; ++r, rowb += prm.band_pitch, rowl += prm.ll_pitch) {
        const int wr = wave * ROWS + r;
        const int gy = qy0 + r;
        if (wr < G::HY || wr >= WAVES * ROWS - G::HY || gy >= prm.nqy) continue;
        float va[QPL], vb[QPL], vc[QPL], vd[QPL];
#pragma unroll
        for (int i = 0; i < QPL; ++i) {
            va[i] = q.a[r][i] * sLL; vb[i] = q.b[r][i] * sHL;
            vc[i] = q.c[r][i] * sHL; vd[i] = q.d[r][i] * sHH;
        }
        const int64_t ob = rowb + qx0;
        const int64_t ol = rowl + qx0;
        if (full_x && prm.vec_ll) {
            store_vec<TLL, QPL>(make_rsrc(ll + rowl, (uint32_t)prm.nqx * (uint32_t)sizeof(TLL)),
                                (uint32_t)qx0 * (uint32_t)sizeof(TLL), va);
        } else {
#pragma unroll
            for (int i = 0; i < QPL; ++i)
                if (qx0 + i < prm.nqx) ll[ol + i] = from_float<TLL>(va[i]);
        }
        if (full_x && prm.vec_band) {
            const uint32_t bb = (uint32_t)prm.nqx * (uint32_t)sizeof(TB);
            const uint32_t off = (uint32_t)qx0 * (uint32_t)sizeof(TB);
            const int64_t rowo = rowb;
            store_vec<TB, QPL>(make_rsrc(hl + rowo, bb), off, vb);
            store_vec<TB, QPL>(make_rsrc(lh + rowo, bb), off, vc);
            store_vec<TB, QPL>(make_rsrc(hh + rowo, bb), off, vd);
        } else {
#pragma unroll
            for (int i = 0; i < QPL; ++i) {
                if (qx0 + i < prm.nqx) {
                    hl[ob + i] = from_float<TB>(vb[i]);
                    lh[ob + i] = from_float<TB>(vc[i]);
                    hh[ob + i] = from_float<TB>(vd[i]);
                }
            }
        }
    }
}

// One tile of a forward level: load, lift, store. All waves of the
// workgroup call it with the same tile (it contains workgroup barriers).
template <int WV, int SCH, int QPL, int ROWS, int WAVES, typename TIN, typename TLL, typename TB>
__device__ __forceinline__ void fwd_tile(const FwdParams &prm, int t, Mailbox<QPL, WAVES> &box,
                                         int lane, int wave) {
    using G = TileGeom<WV, QPL, ROWS, WAVES>;
    Quads<ROWS, QPL> q;
    fwd_load<QPL, ROWS, G, TIN>(q, prm, t, lane, wave);
    if constexpr (SCH == NONSEP_LDS || SCH == SEP_LDS) {
        __shared__ HBox<ROWS, WAVES> hb;
        LdsExchange<ROWS, QPL, WAVES> x{&box, &hb, wave, lane, 0};
        lift_forward<WV, SCH>(q, x);
    } else {
        Exchange<ROWS, QPL, WAVES> x{&box, wave, lane, 0};
        lift_forward<WV, SCH>(q, x);
    }
    fwd_store<WV, QPL, ROWS, WAVES, G, TLL, TB>(q, prm, t, lane, wave);
}

// One tile per workgroup.
template <int WV, int SCH, int QPL, int ROWS, int WAVES, typename TIN, typename TLL, typename TB>
__global__ __launch_bounds__(64 * WAVES) void fwd_level_kernel(FwdParams prm) {
    __shared__ Mailbox<QPL, WAVES> box;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform per wavefront
    fwd_tile<WV, SCH, QPL, ROWS, WAVES, TIN, TLL, TB>(prm, block_tile(), box, lane, wave);
}

// ---- inverse ---------------------------------------------------------------------
// Outside the level, each polyphase component is extended through the
// symmetric extension of the pixel grid it lives on: quad (i, j) component b
// stands for pixel (2i+1, 2j), and so on.
// WITH_LL false: the detail bands only (q.a is left as it is).
template <int QPL, int ROWS, typename TLL, typename TB, bool WITH_LL = true>
__device__ __forceinline__ void inv_load_at(Quads<ROWS, QPL> &q, const InvParams &prm, int qx0,
                                            int qy0) {
    const TLL *ll = static_cast<const TLL *>(prm.ll);
    const TB *hl = static_cast<const TB *>(prm.hl);
    const TB *lh = static_cast<const TB *>(prm.lh);
    const TB *hh = static_cast<const TB *>(prm.hh);
    // quad (i, j)'s even phase stands for pixel 2i, its odd phase for 2i+1
    int xe[QPL], xo[QPL];
#pragma unroll
    for (int i = 0; i < QPL; ++i) {
        xe[i] = mirror(2 * (qx0 + i), prm.w) >> 1;
        xo[i] = (mirror(2 * (qx0 + i) + 1, prm.w) - 1) >> 1;
    }
    if (!(prm.vec_ll && prm.vec_band) || (prm.nqx & (QPL - 1)) != 0) {   // one at a time
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int gy = qy0 + r;
            const int ye = mirror(2 * gy, prm.h) >> 1;
            const int yo = (mirror(2 * gy + 1, prm.h) - 1) >> 1;
#pragma unroll
            for (int i = 0; i < QPL; ++i) {
                if constexpr (WITH_LL) q.a[r][i] = to_float(ll[(int64_t)ye * prm.ll_pitch + xe[i]]);
                q.b[r][i] = to_float(hl[(int64_t)ye * prm.band_pitch + xo[i]]);
                q.c[r][i] = to_float(lh[(int64_t)yo * prm.band_pitch + xe[i]]);
                q.d[r][i] = to_float(hh[(int64_t)yo * prm.band_pitch + xo[i]]);
            }
        }
        return;
    }
    const bool plain = qx0 >= 0 && qx0 + QPL <= prm.nqx;
    const EdgeCols<QPL> ce = EdgeCols<QPL>::template from<TB>(xe, qx0, plain);
    const EdgeCols<QPL> co = EdgeCols<QPL>::template from<TB>(xo, qx0, plain);
    const EdgeCols<QPL> cl = EdgeCols<QPL>::template from<TLL>(xe, qx0, plain);
    const uint32_t bb = (uint32_t)prm.nqx * (uint32_t)sizeof(TB);
    const uint32_t lb = (uint32_t)prm.nqx * (uint32_t)sizeof(TLL);
    rsrc_t rl[ROWS], rh[ROWS], rv[ROWS], rd[ROWS];   // LL, HL, LH, HH rows
    if (qy0 >= 0 && 2 * (qy0 + ROWS) <= prm.h) {
        // all rows inside the level (wavefront-uniform): both phases of quad
        // row gy are band row gy; step the row pointers
        const TLL *pl = ll + (int64_t)qy0 * prm.ll_pitch;
        const int64_t ob = (int64_t)qy0 * prm.band_pitch;
        const TB *ph = hl + ob, *pv = lh + ob, *pd = hh + ob;
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            if constexpr (WITH_LL) rl[r] = make_rsrc(pl, lb);
            rh[r] = make_rsrc(ph, bb);
            rv[r] = make_rsrc(pv, bb);
            rd[r] = make_rsrc(pd, bb);
            if constexpr (WITH_LL) load_vec<TLL, QPL>(rl[r], cl.off_a, q.a[r]);
            load_vec<TB, QPL>(rh[r], co.off_a, q.b[r]);
            load_vec<TB, QPL>(rv[r], ce.off_a, q.c[r]);
            load_vec<TB, QPL>(rd[r], co.off_a, q.d[r]);
            pl += prm.ll_pitch; ph += prm.band_pitch; pv += prm.band_pitch; pd += prm.band_pitch;
        }
    } else {
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int gy = qy0 + r;
            const int64_t ye = mirror(2 * gy, prm.h) >> 1;
            const int64_t yo = (mirror(2 * gy + 1, prm.h) - 1) >> 1;
            if constexpr (WITH_LL) rl[r] = make_rsrc(ll + ye * prm.ll_pitch, lb);
            rh[r] = make_rsrc(hl + ye * prm.band_pitch, bb);
            rv[r] = make_rsrc(lh + yo * prm.band_pitch, bb);
            rd[r] = make_rsrc(hh + yo * prm.band_pitch, bb);
            if constexpr (WITH_LL) load_vec<TLL, QPL>(rl[r], cl.off_a, q.a[r]);
            load_vec<TB, QPL>(rh[r], co.off_a, q.b[r]);
            load_vec<TB, QPL>(rv[r], ce.off_a, q.c[r]);
            load_vec<TB, QPL>(rd[r], co.off_a, q.d[r]);
        }
    }
    if (!wave_all(plain)) {
        if constexpr (WITH_LL) fix_cols<TLL>(rl, cl, q.a);
        fix_cols<TB>(rh, co, q.b);
        fix_cols<TB>(rv, ce, q.c);
        fix_cols<TB>(rd, co, q.d);
    }
}

template <int QPL, int ROWS, typename G, typename TLL, typename TB>
__device__ __forceinline__ void inv_load(Quads<ROWS, QPL> &q, const InvParams &prm, int t,
                                         int lane, int wave) {
    const int ty = t / prm.tiles_x, tx = t - (t / prm.tiles_x) * prm.tiles_x;
    inv_load_at<QPL, ROWS, TLL, TB>(q, prm, tx * G::OX - G::HX + lane * QPL,
                                    ty * G::OY - G::HY + wave * ROWS);
}

template <int QPL, int ROWS, int WAVES, typename G, typename TOUT>
__device__ __forceinline__ void inv_store(const Quads<ROWS, QPL> &q, const InvParams &prm, int t,
                                          int lane, int wave) {
    if (lane == 0 || lane == 63) return;   // halo lanes
    const int ty = t / prm.tiles_x, tx = t - (t / prm.tiles_x) * prm.tiles_x;
    const int qx0 = tx * G::OX - G::HX + lane * QPL;
    const int qy0 = ty * G::OY - G::HY + wave * ROWS;
    TOUT *out = static_cast<TOUT *>(prm.out);
    const int px0 = 2 * qx0;
    const bool full_x = prm.vec_out && px0 + 2 * QPL <= prm.w;
    int64_t ro = (int64_t)(2 * qy0) * prm.out_pitch;   // pixel row 2 (qy0 + r), stepped
#pragma unroll
    for (int r = 0; r < ROWS; ++r, ro += 2 * prm.out_pitch) {
        const int wr = wave * ROWS + r;
        const int gy = qy0 + r;
        if (wr < G::HY || wr >= WAVES * ROWS - G::HY || gy >= prm.nqy) continue;
        float e[2 * QPL], o[2 * QPL];
#pragma unroll
        for (int i = 0; i < QPL; ++i) {
            e[2 * i] = q.a[r][i]; e[2 * i + 1] = q.b[r][i];
            o[2 * i] = q.c[r][i]; o[2 * i + 1] = q.d[r][i];
        }
        TOUT *r0 = out + ro;
        TOUT *r1 = r0 + prm.out_pitch;
        if (full_x) {
            const uint32_t rb = (uint32_t)prm.w * (uint32_t)sizeof(TOUT);
            const uint32_t off = (uint32_t)px0 * (uint32_t)sizeof(TOUT);
            if (prm.stream_out) {
                store_vec<TOUT, 2 * QPL, kStoreStream>(make_rsrc(r0, rb), off, e);
                store_vec<TOUT, 2 * QPL, kStoreStream>(make_rsrc(r1, rb), off, o);
            } else {
                store_vec<TOUT, 2 * QPL>(make_rsrc(r0, rb), off, e);
                store_vec<TOUT, 2 * QPL>(make_rsrc(r1, rb), off, o);
            }
        } else {
#pragma unroll
            for (int k = 0; k < 2 * QPL; ++k) {
                if (px0 + k < prm.w) {
                    r0[px0 + k] = from_float<TOUT>(e[k]);
                    r1[px0 + k] = from_float<TOUT>(o[k]);
                }
            }
        }
    }
}

template <int WV, int SCH, int QPL, int ROWS, int WAVES, typename TLL, typename TB, typename TOUT>
__device__ __forceinline__ void inv_tile(const InvParams &prm, int t, Mailbox<QPL, WAVES> &box,
                                         int lane, int wave) {
    using G = TileGeom<WV, QPL, ROWS, WAVES>;
    using L = Wavelet<WV>;
    const float uLL = (float)(1.0 / (L::ZL * L::ZL)), uHL = (float)(1.0 / (L::ZL * L::ZH));
    const float uHH = (float)(1.0 / (L::ZH * L::ZH));
    Quads<ROWS, QPL> q;
    inv_load<QPL, ROWS, G, TLL, TB>(q, prm, t, lane, wave);
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
#pragma unroll
        for (int i = 0; i < QPL; ++i) {
            q.a[r][i] *= uLL; q.b[r][i] *= uHL; q.c[r][i] *= uHL; q.d[r][i] *= uHH;
        }
    }
    if constexpr (SCH == NONSEP_LDS || SCH == SEP_LDS) {
        __shared__ HBox<ROWS, WAVES> hb;
        LdsExchange<ROWS, QPL, WAVES> x{&box, &hb, wave, lane, 0};
        lift_inverse<WV, SCH>(q, x);
    } else {
        Exchange<ROWS, QPL, WAVES> x{&box, wave, lane, 0};
        lift_inverse<WV, SCH>(q, x);
    }
    inv_store<QPL, ROWS, WAVES, G, TOUT>(q, prm, t, lane, wave);
}

template <int WV, int SCH, int QPL, int ROWS, int WAVES, typename TLL, typename TB, typename TOUT>
__global__ __launch_bounds__(64 * WAVES) void inv_level_kernel(InvParams prm) {
    __shared__ Mailbox<QPL, WAVES> box;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform per wavefront
    inv_tile<WV, SCH, QPL, ROWS, WAVES, TLL, TB, TOUT>(prm, block_tile(), box, lane, wave);
}

// ---- single levels of many images, parameters in the kernel arguments -----------
// Up to kBatchMax level jobs of one size class per launch (continuous
// batching: a different set of jobs every call, so nothing is planned ahead);
// their level parameters travel in the kernel arguments, and tile_start[i] is
// the first global tile index of job i (tile_start[n] is the total). One
// workgroup per tile.
constexpr int kBatchMax = 36;

struct FwdBatch {
    int32_t n;
    int32_t tile_start[kBatchMax + 1];
    FwdParams p[kBatchMax];
};
struct InvBatch {
    int32_t n;
    int32_t tile_start[kBatchMax + 1];
    InvParams p[kBatchMax];
};
static_assert(sizeof(FwdBatch) <= 4096 && sizeof(InvBatch) <= 4096, "kernel argument limit");

// Image owning global tile t (wave-uniform; the table is in kernel arguments).
template <typename B>
__device__ __forceinline__ int batch_image(const B &bt, int t) {
    int lo = 0, hi = bt.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (bt.tile_start[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <int WV, int SCH, int QPL, int ROWS, int WAVES, typename TIN, typename TLL, typename TB>
__global__ __launch_bounds__(64 * WAVES) void fwd_batch_kernel(FwdBatch bt) {
    __shared__ Mailbox<QPL, WAVES> box;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int total = bt.tile_start[bt.n];
    for (int t = block_tile(); t < total; t += gridDim.x) {
        const int i = batch_image(bt, t);
        fwd_tile<WV, SCH, QPL, ROWS, WAVES, TIN, TLL, TB>(bt.p[i], t - bt.tile_start[i], box, lane,
                                                          wave);
    }
}

template <int WV, int SCH, int QPL, int ROWS, int WAVES, typename TLL, typename TB, typename TOUT>
__global__ __launch_bounds__(64 * WAVES) void inv_batch_kernel(InvBatch bt) {
    __shared__ Mailbox<QPL, WAVES> box;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int total = bt.tile_start[bt.n];
    for (int t = block_tile(); t < total; t += gridDim.x) {
        const int i = batch_image(bt, t);
        inv_tile<WV, SCH, QPL, ROWS, WAVES, TLL, TB, TOUT>(bt.p[i], t - bt.tile_start[i], box, lane,
                                                           wave);
    }
}

// ---- batches planned in a device table ------------------------------------------
// One launch covers every image of one level that uses one tile configuration,
// however many: the per-image level parameters and a tile -> image map sit in
// a table in device memory that the host planned once (a graph captures only
// the launches). Global tile t belongs to image img[t] and is that image's
// tile t - start[img[t]].
template <typename P>
struct TableLaunch {
    const int32_t *img;     // [total] image of each tile (index into params)
    const int32_t *start;   // [images] first global tile of each image
    const P *params;        // [images]
    int32_t total;          // tiles of the launch
};

// Every workgroup walks the tiles t = its id, id + gridDim.x, ... below
// `total`: one tile each when the grid has one workgroup per tile, several
// when the grid is capped at the resident workgroups (persistent).
template <int WV, int SCH, int QPL, int ROWS, int WAVES, typename TIN, typename TLL, typename TB>
__global__ __launch_bounds__(64 * WAVES) void fwd_table_kernel(TableLaunch<FwdParams> tl) {
    __shared__ Mailbox<QPL, WAVES> box;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int t = block_tile(); t < tl.total; t += gridDim.x) {
        const int i = __builtin_amdgcn_readfirstlane(tl.img[t]);
        const FwdParams prm = tl.params[i];
        fwd_tile<WV, SCH, QPL, ROWS, WAVES, TIN, TLL, TB>(prm, t - tl.start[i], box, lane, wave);
    }
}

template <int WV, int SCH, int QPL, int ROWS, int WAVES, typename TLL, typename TB, typename TOUT>
__global__ __launch_bounds__(64 * WAVES) void inv_table_kernel(TableLaunch<InvParams> tl) {
    __shared__ Mailbox<QPL, WAVES> box;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int t = block_tile(); t < tl.total; t += gridDim.x) {
        const int i = __builtin_amdgcn_readfirstlane(tl.img[t]);
        const InvParams prm = tl.params[i];
        inv_tile<WV, SCH, QPL, ROWS, WAVES, TLL, TB, TOUT>(prm, t - tl.start[i], box, lane, wave);
    }
}

}  // namespace dwt2

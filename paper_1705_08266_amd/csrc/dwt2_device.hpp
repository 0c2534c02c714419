// Device-side building blocks of the 2-D lifting DWT for gfx950 (CDNA4).
//
// Data layout in registers. A workgroup owns a window of quads: 64 lanes per
// wavefront along x, each lane holding QPL consecutive quads of a quad row,
// and ROWS quad rows per lane; WAVES wavefronts are stacked along y. A quad is
// the 2x2 polyphase block (a, b, c, d) = (x[2j][2i], x[2j][2i+1],
// x[2j+1][2i], x[2j+1][2i+1]), the paper's components 1..4 (Sec. 2).
//
// Neighbour exchange. Horizontal neighbours of the first/last quad of a lane
// come from the adjacent lane through DPP wavefront shifts (no LDS, no
// barrier); vertical neighbours inside a lane's rows are registers; the rows
// on the boundary between two wavefronts go through a small double-buffered
// LDS mailbox, one workgroup barrier per exchange. Window edges read
// don't-care values; the lifting halo around the written centre absorbs them.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace dwt2 {

enum : int { CDF97 = 0, CDF53 = 1 };
// NONSEP_LDS and SEP_LDS are the same schemes with every neighbour exchange
// going through LDS and a workgroup barrier, horizontal ones included (the
// paper's local-memory design), instead of DPP lane shifts.
enum : int { NONSEP = 0, SEP = 1, NONSEP_LDS = 2, SEP_LDS = 3 };
enum : int { DT_F32 = 0, DT_F16 = 1, DT_BF16 = 2 };

// ---- lifting constants ------------------------------------------------------
// CDF 9/7: two pairs (alpha, beta), (gamma, delta) and the scaling K; CDF 5/3:
// one pair (-1/2, 1/4). Predicts P(z) = p (1 + z), updates U(z) = u (1 + 1/z).
// Unit-gain scaling: low phase * 1/K, high phase * K/2 (5/3: 1 and 1/2).
template <int WV> struct Wavelet;

template <> struct Wavelet<CDF97> {
    static constexpr int NPAIRS = 2;
    static constexpr double K = 1.230174104914001;
    __host__ __device__ static constexpr double p(int k) { return k == 0 ? -1.586134342059924 : 0.882911075530934; }
    __host__ __device__ static constexpr double u(int k) { return k == 0 ? -0.052980118572961 : 0.443506852043971; }
    static constexpr double ZL = 1.0 / K;
    static constexpr double ZH = K / 2.0;
};

template <> struct Wavelet<CDF53> {
    static constexpr int NPAIRS = 1;
    __host__ __device__ static constexpr double p(int) { return -0.5; }
    __host__ __device__ static constexpr double u(int) { return 0.25; }
    static constexpr double ZL = 1.0;
    static constexpr double ZH = 0.5;
};

// ---- storage types ----------------------------------------------------------
struct bf16_t { uint16_t bits; };

template <typename T> struct Storage;
template <> struct Storage<float> {
    static constexpr int code = DT_F32;
    __device__ static float decode(uint32_t v) { return __uint_as_float(v); }
};
template <> struct Storage<__half> {
    static constexpr int code = DT_F16;
    __device__ static float decode(uint32_t v) {
        return __half2float(__ushort_as_half((unsigned short)v));
    }
};
template <> struct Storage<bf16_t> {
    static constexpr int code = DT_BF16;
    __device__ static float decode(uint32_t v) { return __uint_as_float(v << 16); }
};

__device__ __forceinline__ float to_float(float v) { return v; }
__device__ __forceinline__ float to_float(__half v) { return __half2float(v); }
__device__ __forceinline__ float to_float(bf16_t v) { return __uint_as_float((uint32_t)v.bits << 16); }

// Round-to-nearest-even conversions from FP32.
template <typename T> __device__ __forceinline__ T from_float(float v);
template <> __device__ __forceinline__ float from_float<float>(float v) { return v; }
// The value is pinned in an FP32 register first: otherwise the compiler may
// fuse the multiply that produced it into an FMA with FP16 output (one
// rounding instead of FP32-then-FP16), and results would depend on the
// kernel configuration.
template <> __device__ __forceinline__ __half from_float<__half>(float v) {
    asm volatile("" : "+v"(v));
    return __float2half_rn(v);
}
template <> __device__ __forceinline__ bf16_t from_float<bf16_t>(float v) {
    uint32_t u = __float_as_uint(v);
    bf16_t r;
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) {
        r.bits = 0x7fc0;                       // quiet NaN
    } else {
        u += 0x7fffu + ((u >> 16) & 1u);       // round half to even
        r.bits = (uint16_t)(u >> 16);
    }
    return r;
}

template <typename T> __device__ __forceinline__ uint32_t bits_of(T v);
template <> __device__ __forceinline__ uint32_t bits_of<float>(float v) { return __float_as_uint(v); }
template <> __device__ __forceinline__ uint32_t bits_of<__half>(__half v) { return (uint32_t)__half_as_ushort(v); }
template <> __device__ __forceinline__ uint32_t bits_of<bf16_t>(bf16_t v) { return v.bits; }

// ---- vector row access through buffer resources ---------------------------------
// A row of a 2-D buffer is described by a wave-uniform buffer resource (base
// pointer and byte length); each lane addresses it with a 32-bit byte offset.
// The hardware checks every access against the length: reads past the end
// return zero and writes past the end are dropped.
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;   // raw (untyped) buffer, gfx9 family

__device__ __forceinline__ rsrc_t make_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                             kRsrcWord3);
}

// Cache policy of a buffer store (the instruction's cache-policy operand).
// kStoreStream sets the non-temporal bit: the written lines go out to memory
// without being kept in the caches for reuse, for output that no later step
// of the transform reads.
constexpr int kStoreCached = 0, kStoreStream = 2;

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Raw 32-bit words of an access of W words.
template <int W>
__device__ __forceinline__ void buf_load_words(rsrc_t r, uint32_t off, uint32_t (&w)[W]) {
    static_assert(W == 1 || W == 2 || W == 4 || W == 8, "access width");
    if constexpr (W == 1) {
        w[0] = __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0);
    } else if constexpr (W == 2) {
        u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0);
        w[0] = v.x; w[1] = v.y;
    } else {
#pragma unroll
        for (int h = 0; h < W / 4; ++h) {
            u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)(off + 16u * h), 0, 0);
            w[4 * h] = v.x; w[4 * h + 1] = v.y; w[4 * h + 2] = v.z; w[4 * h + 3] = v.w;
        }
    }
}

template <int W, int POLICY = kStoreCached>
__device__ __forceinline__ void buf_store_words(rsrc_t r, uint32_t off, const uint32_t (&w)[W]) {
    static_assert(W == 1 || W == 2 || W == 4 || W == 8, "access width");
    if constexpr (W == 1) {
        __builtin_amdgcn_raw_buffer_store_b32(w[0], r, (int)off, 0, POLICY);
    } else if constexpr (W == 2) {
        u32x2 v; v.x = w[0]; v.y = w[1];
        __builtin_amdgcn_raw_buffer_store_b64(v, r, (int)off, 0, POLICY);
    } else {
#pragma unroll
        for (int h = 0; h < W / 4; ++h) {
            u32x4 v; v.x = w[4 * h]; v.y = w[4 * h + 1]; v.z = w[4 * h + 2]; v.w = w[4 * h + 3];
            __builtin_amdgcn_raw_buffer_store_b128(v, r, (int)(off + 16u * h), 0, POLICY);
        }
    }
}

// One element of type T at byte offset `off` (reads past the end give 0).
template <typename T>
__device__ __forceinline__ float load_elem(rsrc_t r, uint32_t off) {
    if constexpr (sizeof(T) == 4) {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
    } else {
        return Storage<T>::decode((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, 0));
    }
}

template <typename T>
__device__ __forceinline__ void store_elem(rsrc_t r, uint32_t off, float v) {
    if constexpr (sizeof(T) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)off, 0, 0);
    } else {
        __builtin_amdgcn_raw_buffer_store_b16((unsigned short)bits_of<T>(from_float<T>(v)), r,
                                              (int)off, 0, 0);
    }
}

// A byte offset that every buffer resource of this library rejects: rows
// are shorter than 2 GiB, so a store at this offset is dropped.
constexpr uint32_t kNoAccess = 0x80000000u;

// N consecutive elements of type T (2 to 32 bytes) at byte offset `off`.
template <typename T, int N>
__device__ __forceinline__ void load_vec(rsrc_t r, uint32_t off, float (&out)[N]) {
    constexpr int BYTES = N * (int)sizeof(T);
    if constexpr (BYTES == 2) {
        out[0] = load_elem<T>(r, off);
    } else {
        static_assert(BYTES % 4 == 0, "whole words");
        uint32_t w[BYTES / 4];
        buf_load_words<BYTES / 4>(r, off, w);
        if constexpr (sizeof(T) == 4) {
#pragma unroll
            for (int e = 0; e < N; ++e) out[e] = __uint_as_float(w[e]);
        } else {
#pragma unroll
            for (int e = 0; e < N; ++e)
                out[e] = Storage<T>::decode((w[e / 2] >> (16 * (e & 1))) & 0xffffu);
        }
    }
}

template <typename T, int N, int POLICY = kStoreCached>
__device__ __forceinline__ void store_vec(rsrc_t r, uint32_t off, const float (&in)[N]) {
    constexpr int BYTES = N * (int)sizeof(T);
    if constexpr (BYTES == 2) {
        store_elem<T>(r, off, in[0]);
    } else {
        static_assert(BYTES % 4 == 0, "whole words");
        uint32_t w[BYTES / 4];
        if constexpr (sizeof(T) == 4) {
#pragma unroll
            for (int e = 0; e < N; ++e) w[e] = __float_as_uint(in[e]);
        } else {
#pragma unroll
            for (int e = 0; e < N; e += 2)
                w[e / 2] = bits_of<T>(from_float<T>(in[e])) |
                           (bits_of<T>(from_float<T>(in[e + 1])) << 16);
        }
        buf_store_words<BYTES / 4, POLICY>(r, off, w);
    }
}

// ---- boundary ---------------------------------------------------------------
// Whole-sample symmetric extension of an n-sample axis (n >= 2), periodic
// with period 2n-2: the index of the sample that position x stands for.
__device__ __forceinline__ int mirror(int x, int n) {
    if (x < 0) x = -x;                 // the extension is even about 0
    if (x < n) return x;
    const int period = 2 * n - 2;
    if (x >= period) x %= period;      // only for windows wider than the level
    return x < n ? x : period - x;
}

// True when every lane of the wavefront has `c` set: a wavefront-uniform
// branch condition. Loads of the two paths then never share an exec mask,
// so the vector path's loads of all rows stay in flight together.
__device__ __forceinline__ bool wave_all(bool c) {
    return __builtin_amdgcn_ballot_w64(!c) == 0;
}

// ---- cross-lane shifts (DPP, wavefront-wide) ----------------------------------
// from_right(v): lane l receives lane l+1's v (lane 63 receives 0).
// from_left(v):  lane l receives lane l-1's v (lane 0 receives 0).
// The zero for the lane without a source comes from the bound-control bit,
// not from the instruction's old value, so no register has to be zeroed
// before each shift.
__device__ __forceinline__ float from_right(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_left(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, true));
}

// ---- the register tile --------------------------------------------------------
template <int ROWS, int QPL>
struct Quads {
    float a[ROWS][QPL], b[ROWS][QPL], c[ROWS][QPL], d[ROWS][QPL];
};

// Mailbox between vertically adjacent wavefronts. Two buffers alternate so
// that one barrier per exchange suffices: the writes of exchange k+1 go to the
// buffer last read in exchange k-1, which every wave finished before it
// passed the barrier of exchange k.
template <int QPL, int WAVES>
struct Mailbox {
    float v[2][WAVES][2][QPL][64];
};

template <int ROWS, int QPL, int WAVES>
struct Exchange {
    Mailbox<QPL, WAVES> *box;
    int wave, lane, buf;

    // Every wave sends its first row's (x, y) up and receives the first row of
    // the wave below it (the row after its last row).
    __device__ __forceinline__ void from_below(const float (&x0)[QPL], const float (&y0)[QPL],
                                               float (&xo)[QPL], float (&yo)[QPL]) {
        if constexpr (WAVES == 1) {
#pragma unroll
            for (int i = 0; i < QPL; ++i) { xo[i] = x0[i]; yo[i] = y0[i]; }
        } else {
#pragma unroll
            for (int i = 0; i < QPL; ++i) {
                box->v[buf][wave][0][i][lane] = x0[i];
                box->v[buf][wave][1][i][lane] = y0[i];
            }
            __syncthreads();
            const int src = (wave + 1 < WAVES) ? wave + 1 : wave;
#pragma unroll
            for (int i = 0; i < QPL; ++i) {
                xo[i] = box->v[buf][src][0][i][lane];
                yo[i] = box->v[buf][src][1][i][lane];
            }
            buf ^= 1;
        }
    }

    // Every wave sends its last row's (x, y) down and receives the last row of
    // the wave above it (the row before its first row).
    __device__ __forceinline__ void from_above(const float (&xl)[QPL], const float (&yl)[QPL],
                                               float (&xo)[QPL], float (&yo)[QPL]) {
        if constexpr (WAVES == 1) {
#pragma unroll
            for (int i = 0; i < QPL; ++i) { xo[i] = xl[i]; yo[i] = yl[i]; }
        } else {
#pragma unroll
            for (int i = 0; i < QPL; ++i) {
                box->v[buf][wave][0][i][lane] = xl[i];
                box->v[buf][wave][1][i][lane] = yl[i];
            }
            __syncthreads();
            const int src = (wave > 0) ? wave - 1 : wave;
#pragma unroll
            for (int i = 0; i < QPL; ++i) {
                xo[i] = box->v[buf][src][0][i][lane];
                yo[i] = box->v[buf][src][1][i][lane];
            }
            buf ^= 1;
        }
    }
};

// ---- non-separable steps (Sec. 3) ---------------------------------------------
// T_P:  b += P a;  c += P* a;  d += P P* a + P* b + P c   (pre-step values)
// computed as the spatial T_{P1} with P1 = p z (right and lower neighbours),
// followed on the unit's own quad by T^H_{P0} then T^V_{P0} with P0 = p.
// Rows run top to bottom and quads left to right, so every neighbour read
// (row below, quad to the right) still holds its pre-step value.
template <int ROWS, int QPL, int WAVES>
__device__ __forceinline__ void nonsep_predict(Quads<ROWS, QPL> &q, Exchange<ROWS, QPL, WAVES> &x,
                                               float p) {
    const float pp = p * p;
    float na[QPL], nb[QPL];
    x.from_below(q.a[0], q.b[0], na, nb);
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        constexpr int dummy = 0; (void)dummy;
        float ad[QPL], bd[QPL];
#pragma unroll
        for (int i = 0; i < QPL; ++i) {
            ad[i] = (r + 1 < ROWS) ? q.a[(r + 1 < ROWS) ? r + 1 : r][i] : na[i];
            bd[i] = (r + 1 < ROWS) ? q.b[(r + 1 < ROWS) ? r + 1 : r][i] : nb[i];
        }
        const float aR = from_right(q.a[r][0]);
        const float cR = from_right(q.c[r][0]);
        const float adR = from_right(ad[0]);
#pragma unroll
        for (int i = 0; i < QPL; ++i) {
            const float ar = (i + 1 < QPL) ? q.a[r][(i + 1 < QPL) ? i + 1 : i] : aR;
            const float cr = (i + 1 < QPL) ? q.c[r][(i + 1 < QPL) ? i + 1 : i] : cR;
            const float adr = (i + 1 < QPL) ? ad[(i + 1 < QPL) ? i + 1 : i] : adR;
            const float a = q.a[r][i];
            float b = fmaf(p, ar, q.b[r][i]);
            float c = fmaf(p, ad[i], q.c[r][i]);
            float d = fmaf(p, cr, q.d[r][i]);
            d = fmaf(p, bd[i], d);
            d = fmaf(pp, adr, d);
            b = fmaf(p, a, b);      // T^H_{P0}
            d = fmaf(p, c, d);
            c = fmaf(p, a, c);      // T^V_{P0}
            d = fmaf(p, b, d);
            q.b[r][i] = b; q.c[r][i] = c; q.d[r][i] = d;
        }
    }
}

// S_U:  a += U b + U* c + U U* d;  b += U* d;  c += U d   (pre-step values)
// computed as the spatial S_{U1} with U1 = u / z (left and upper neighbours),
// followed by S^H_{U0} then S^V_{U0} with U0 = u. Rows run bottom to top and
// quads right to left so neighbour reads see pre-step values.
template <int ROWS, int QPL, int WAVES>
__device__ __forceinline__ void nonsep_update(Quads<ROWS, QPL> &q, Exchange<ROWS, QPL, WAVES> &x,
                                              float u) {
    const float uu = u * u;
    float pc[QPL], pd[QPL];
    x.from_above(q.c[ROWS - 1], q.d[ROWS - 1], pc, pd);
#pragma unroll
    for (int r = ROWS - 1; r >= 0; --r) {
        float cu[QPL], du[QPL];
#pragma unroll
        for (int i = 0; i < QPL; ++i) {
            cu[i] = (r > 0) ? q.c[(r > 0) ? r - 1 : r][i] : pc[i];
            du[i] = (r > 0) ? q.d[(r > 0) ? r - 1 : r][i] : pd[i];
        }
        const float bL = from_left(q.b[r][QPL - 1]);
        const float dL = from_left(q.d[r][QPL - 1]);
        const float duL = from_left(du[QPL - 1]);
#pragma unroll
        for (int i = QPL - 1; i >= 0; --i) {
            const float bl = (i > 0) ? q.b[r][(i > 0) ? i - 1 : i] : bL;
            const float dl = (i > 0) ? q.d[r][(i > 0) ? i - 1 : i] : dL;
            const float dul = (i > 0) ? du[(i > 0) ? i - 1 : i] : duL;
            const float d = q.d[r][i];
            float a = fmaf(u, bl, q.a[r][i]);
            a = fmaf(u, cu[i], a);
            a = fmaf(uu, dul, a);
            float b = fmaf(u, du[i], q.b[r][i]);
            float c = fmaf(u, dl, q.c[r][i]);
            a = fmaf(u, b, a);      // S^H_{U0}
            c = fmaf(u, d, c);
            a = fmaf(u, c, a);      // S^V_{U0}
            b = fmaf(u, d, b);
            q.a[r][i] = a; q.b[r][i] = b; q.c[r][i] = c;
        }
    }
}

// ---- separable steps (Sec. 2) -------------------------------------------------
// T^H_P: b += P a, d += P c.  Horizontal only: DPP exchange, no barrier.
template <int ROWS, int QPL>
__device__ __forceinline__ void sep_predict_h(Quads<ROWS, QPL> &q, float p) {
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const float aR = from_right(q.a[r][0]);
        const float cR = from_right(q.c[r][0]);
#pragma unroll
        for (int i = 0; i < QPL; ++i) {
            const float ar = (i + 1 < QPL) ? q.a[r][(i + 1 < QPL) ? i + 1 : i] : aR;
            const float cr = (i + 1 < QPL) ? q.c[r][(i + 1 < QPL) ? i + 1 : i] : cR;
            q.b[r][i] = fmaf(p, ar, fmaf(p, q.a[r][i], q.b[r][i]));
            q.d[r][i] = fmaf(p, cr, fmaf(p, q.c[r][i], q.d[r][i]));
        }
    }
}

// T^V_P: c += P* a, d += P* b.  Vertical: one mailbox exchange.
template <int ROWS, int QPL, int WAVES>
__device__ __forceinline__ void sep_predict_v(Quads<ROWS, QPL> &q, Exchange<ROWS, QPL, WAVES> &x,
                                              float p) {
    float na[QPL], nb[QPL];
    x.from_below(q.a[0], q.b[0], na, nb);
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
#pragma unroll
        for (int i = 0; i < QPL; ++i) {
            const float ad = (r + 1 < ROWS) ? q.a[(r + 1 < ROWS) ? r + 1 : r][i] : na[i];
            const float bd = (r + 1 < ROWS) ? q.b[(r + 1 < ROWS) ? r + 1 : r][i] : nb[i];
            q.c[r][i] = fmaf(p, ad, fmaf(p, q.a[r][i], q.c[r][i]));
            q.d[r][i] = fmaf(p, bd, fmaf(p, q.b[r][i], q.d[r][i]));
        }
    }
}

// S^H_U: a += U b, c += U d.
template <int ROWS, int QPL>
__device__ __forceinline__ void sep_update_h(Quads<ROWS, QPL> &q, float u) {
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const float bL = from_left(q.b[r][QPL - 1]);
        const float dL = from_left(q.d[r][QPL - 1]);
#pragma unroll
        for (int i = 0; i < QPL; ++i) {
            const float bl = (i > 0) ? q.b[r][(i > 0) ? i - 1 : i] : bL;
            const float dl = (i > 0) ? q.d[r][(i > 0) ? i - 1 : i] : dL;
            q.a[r][i] = fmaf(u, bl, fmaf(u, q.b[r][i], q.a[r][i]));
            q.c[r][i] = fmaf(u, dl, fmaf(u, q.d[r][i], q.c[r][i]));
        }
    }
}

// S^V_U: a += U* c, b += U* d.
template <int ROWS, int QPL, int WAVES>
__device__ __forceinline__ void sep_update_v(Quads<ROWS, QPL> &q, Exchange<ROWS, QPL, WAVES> &x,
                                             float u) {
    float pc[QPL], pd[QPL];
    x.from_above(q.c[ROWS - 1], q.d[ROWS - 1], pc, pd);
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
#pragma unroll
        for (int i = 0; i < QPL; ++i) {
            const float cu = (r > 0) ? q.c[(r > 0) ? r - 1 : r][i] : pc[i];
            const float du = (r > 0) ? q.d[(r > 0) ? r - 1 : r][i] : pd[i];
            q.a[r][i] = fmaf(u, cu, fmaf(u, q.c[r][i], q.a[r][i]));
            q.b[r][i] = fmaf(u, du, fmaf(u, q.d[r][i], q.b[r][i]));
        }
    }
}

// ---- every exchange through LDS (ablation of the DPP lane shifts) ------------
// Per-row edge values of each lane, double-buffered like the mailbox; one
// exchange publishes, passes one workgroup barrier and reads.
template <int ROWS, int WAVES>
struct HBox {
    float v[2][WAVES][2][ROWS][64];
};

template <int ROWS, int QPL, int WAVES>
struct LdsExchange {
    Mailbox<QPL, WAVES> *box;
    HBox<ROWS, WAVES> *hb;
    int wave, lane, buf;
};

// T_P with the right neighbours (a, c of the next lane's first quad, and the
// row below) and the lower row read from LDS after one barrier.
template <int ROWS, int QPL, int WAVES>
__device__ __forceinline__ void nonsep_predict_lds(Quads<ROWS, QPL> &q,
                                                   LdsExchange<ROWS, QPL, WAVES> &x, float p) {
    const float pp = p * p;
    const int b = x.buf, w = x.wave, l = x.lane;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        x.hb->v[b][w][0][r][l] = q.a[r][0];
        x.hb->v[b][w][1][r][l] = q.c[r][0];
    }
#pragma unroll
    for (int i = 0; i < QPL; ++i) {
        x.box->v[b][w][0][i][l] = q.a[0][i];
        x.box->v[b][w][1][i][l] = q.b[0][i];
    }
    __syncthreads();
    const int src = (w + 1 < WAVES) ? w + 1 : w;
    const int rl = l < 63 ? l + 1 : l;      // the window's last lane reads itself
    float na[QPL], nb[QPL];
#pragma unroll
    for (int i = 0; i < QPL; ++i) {
        na[i] = x.box->v[b][src][0][i][l];
        nb[i] = x.box->v[b][src][1][i][l];
    }
    float aR[ROWS], cR[ROWS], adR[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        aR[r] = x.hb->v[b][w][0][r][rl];
        cR[r] = x.hb->v[b][w][1][r][rl];
        adR[r] = (r + 1 < ROWS) ? x.hb->v[b][w][0][(r + 1 < ROWS) ? r + 1 : r][rl]
                                : x.box->v[b][src][0][0][rl];
    }
    x.buf ^= 1;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        float ad[QPL], bd[QPL];
#pragma unroll
        for (int i = 0; i < QPL; ++i) {
            ad[i] = (r + 1 < ROWS) ? q.a[(r + 1 < ROWS) ? r + 1 : r][i] : na[i];
            bd[i] = (r + 1 < ROWS) ? q.b[(r + 1 < ROWS) ? r + 1 : r][i] : nb[i];
        }
#pragma unroll
        for (int i = 0; i < QPL; ++i) {
            const float ar = (i + 1 < QPL) ? q.a[r][(i + 1 < QPL) ? i + 1 : i] : aR[r];
            const float cr = (i + 1 < QPL) ? q.c[r][(i + 1 < QPL) ? i + 1 : i] : cR[r];
            const float adr = (i + 1 < QPL) ? ad[(i + 1 < QPL) ? i + 1 : i] : adR[r];
            const float a = q.a[r][i];
            float bv = fmaf(p, ar, q.b[r][i]);
            float c = fmaf(p, ad[i], q.c[r][i]);
            float d = fmaf(p, cr, q.d[r][i]);
            d = fmaf(p, bd[i], d);
            d = fmaf(pp, adr, d);
            bv = fmaf(p, a, bv);    // T^H_{P0}
            d = fmaf(p, c, d);
            c = fmaf(p, a, c);      // T^V_{P0}
            d = fmaf(p, bv, d);
            q.b[r][i] = bv; q.c[r][i] = c; q.d[r][i] = d;
        }
    }
}

// S_U with the left neighbours (b, d of the previous lane's last quad, and the
// row above) and the upper row read from LDS after one barrier.
template <int ROWS, int QPL, int WAVES>
__device__ __forceinline__ void nonsep_update_lds(Quads<ROWS, QPL> &q,
                                                  LdsExchange<ROWS, QPL, WAVES> &x, float u) {
    const float uu = u * u;
    const int b = x.buf, w = x.wave, l = x.lane;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        x.hb->v[b][w][0][r][l] = q.b[r][QPL - 1];
        x.hb->v[b][w][1][r][l] = q.d[r][QPL - 1];
    }
#pragma unroll
    for (int i = 0; i < QPL; ++i) {
        x.box->v[b][w][0][i][l] = q.c[ROWS - 1][i];
        x.box->v[b][w][1][i][l] = q.d[ROWS - 1][i];
    }
    __syncthreads();
    const int src = (w > 0) ? w - 1 : w;
    const int ll = l > 0 ? l - 1 : l;       // the window's first lane reads itself
    float pc[QPL], pd[QPL];
#pragma unroll
    for (int i = 0; i < QPL; ++i) {
        pc[i] = x.box->v[b][src][0][i][l];
        pd[i] = x.box->v[b][src][1][i][l];
    }
    float bL[ROWS], dL[ROWS], duL[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        bL[r] = x.hb->v[b][w][0][r][ll];
        dL[r] = x.hb->v[b][w][1][r][ll];
        duL[r] = (r > 0) ? x.hb->v[b][w][1][(r > 0) ? r - 1 : r][ll]
                         : x.box->v[b][src][1][QPL - 1][ll];
    }
    x.buf ^= 1;
#pragma unroll
    for (int r = ROWS - 1; r >= 0; --r) {
        float cu[QPL], du[QPL];
#pragma unroll
        for (int i = 0; i < QPL; ++i) {
            cu[i] = (r > 0) ? q.c[(r > 0) ? r - 1 : r][i] : pc[i];
            du[i] = (r > 0) ? q.d[(r > 0) ? r - 1 : r][i] : pd[i];
        }
#pragma unroll
        for (int i = QPL - 1; i >= 0; --i) {
            const float bl = (i > 0) ? q.b[r][(i > 0) ? i - 1 : i] : bL[r];
            const float dl = (i > 0) ? q.d[r][(i > 0) ? i - 1 : i] : dL[r];
            const float dul = (i > 0) ? du[(i > 0) ? i - 1 : i] : duL[r];
            const float d = q.d[r][i];
            float a = fmaf(u, bl, q.a[r][i]);
            a = fmaf(u, cu[i], a);
            a = fmaf(uu, dul, a);
            float bv = fmaf(u, du[i], q.b[r][i]);
            float c = fmaf(u, dl, q.c[r][i]);
            a = fmaf(u, bv, a);     // S^H_{U0}
            c = fmaf(u, d, c);
            a = fmaf(u, c, a);      // S^V_{U0}
            bv = fmaf(u, d, bv);
            q.a[r][i] = a; q.b[r][i] = bv; q.c[r][i] = c;
        }
    }
}

// T^H_P through LDS: one barrier.
template <int ROWS, int QPL, int WAVES>
__device__ __forceinline__ void sep_predict_h_lds(Quads<ROWS, QPL> &q,
                                                  LdsExchange<ROWS, QPL, WAVES> &x, float p) {
    const int b = x.buf, w = x.wave, l = x.lane;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        x.hb->v[b][w][0][r][l] = q.a[r][0];
        x.hb->v[b][w][1][r][l] = q.c[r][0];
    }
    __syncthreads();
    const int rl = l < 63 ? l + 1 : l;
    float aR[ROWS], cR[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        aR[r] = x.hb->v[b][w][0][r][rl];
        cR[r] = x.hb->v[b][w][1][r][rl];
    }
    x.buf ^= 1;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
#pragma unroll
        for (int i = 0; i < QPL; ++i) {
            const float ar = (i + 1 < QPL) ? q.a[r][(i + 1 < QPL) ? i + 1 : i] : aR[r];
            const float cr = (i + 1 < QPL) ? q.c[r][(i + 1 < QPL) ? i + 1 : i] : cR[r];
            q.b[r][i] = fmaf(p, ar, fmaf(p, q.a[r][i], q.b[r][i]));
            q.d[r][i] = fmaf(p, cr, fmaf(p, q.c[r][i], q.d[r][i]));
        }
    }
}

// S^H_U through LDS: one barrier.
template <int ROWS, int QPL, int WAVES>
__device__ __forceinline__ void sep_update_h_lds(Quads<ROWS, QPL> &q,
                                                 LdsExchange<ROWS, QPL, WAVES> &x, float u) {
    const int b = x.buf, w = x.wave, l = x.lane;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        x.hb->v[b][w][0][r][l] = q.b[r][QPL - 1];
        x.hb->v[b][w][1][r][l] = q.d[r][QPL - 1];
    }
    __syncthreads();
    const int ll = l > 0 ? l - 1 : l;
    float bL[ROWS], dL[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        bL[r] = x.hb->v[b][w][0][r][ll];
        dL[r] = x.hb->v[b][w][1][r][ll];
    }
    x.buf ^= 1;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
#pragma unroll
        for (int i = 0; i < QPL; ++i) {
            const float bl = (i > 0) ? q.b[r][(i > 0) ? i - 1 : i] : bL[r];
            const float dl = (i > 0) ? q.d[r][(i > 0) ? i - 1 : i] : dL[r];
            q.a[r][i] = fmaf(u, bl, fmaf(u, q.b[r][i], q.a[r][i]));
            q.c[r][i] = fmaf(u, dl, fmaf(u, q.d[r][i], q.c[r][i]));
        }
    }
}

// The vertical separable steps on the LDS exchange's mailbox (same parity).
template <int ROWS, int QPL, int WAVES>
__device__ __forceinline__ Exchange<ROWS, QPL, WAVES> as_exchange(LdsExchange<ROWS, QPL, WAVES> &x) {
    return Exchange<ROWS, QPL, WAVES>{x.box, x.wave, x.lane, x.buf};
}

// ---- whole lifting sequences --------------------------------------------------
template <int WV, int SCH, int ROWS, int QPL, int WAVES>
__device__ __forceinline__ void lift_forward(Quads<ROWS, QPL> &q, LdsExchange<ROWS, QPL, WAVES> &x) {
    using L = Wavelet<WV>;
#pragma unroll
    for (int k = 0; k < L::NPAIRS; ++k) {
        const float p = (float)L::p(k), u = (float)L::u(k);
        if constexpr (SCH == NONSEP_LDS) {
            nonsep_predict_lds(q, x, p);
            nonsep_update_lds(q, x, u);
        } else {
            sep_predict_h_lds(q, x, p);
            Exchange<ROWS, QPL, WAVES> v = as_exchange(x);
            sep_predict_v(q, v, p);
            x.buf = v.buf;
            sep_update_h_lds(q, x, u);
            v = as_exchange(x);
            sep_update_v(q, v, u);
            x.buf = v.buf;
        }
    }
}

template <int WV, int SCH, int ROWS, int QPL, int WAVES>
__device__ __forceinline__ void lift_inverse(Quads<ROWS, QPL> &q, LdsExchange<ROWS, QPL, WAVES> &x) {
    using L = Wavelet<WV>;
#pragma unroll
    for (int k = L::NPAIRS - 1; k >= 0; --k) {
        const float p = -(float)L::p(k), u = -(float)L::u(k);
        if constexpr (SCH == NONSEP_LDS) {
            nonsep_update_lds(q, x, u);
            nonsep_predict_lds(q, x, p);
        } else {
            Exchange<ROWS, QPL, WAVES> v = as_exchange(x);
            sep_update_v(q, v, u);
            x.buf = v.buf;
            sep_update_h_lds(q, x, u);
            v = as_exchange(x);
            sep_predict_v(q, v, p);
            x.buf = v.buf;
            sep_predict_h_lds(q, x, p);
        }
    }
}

template <int WV, int SCH, int ROWS, int QPL, int WAVES>
__device__ __forceinline__ void lift_forward(Quads<ROWS, QPL> &q, Exchange<ROWS, QPL, WAVES> &x) {
    using L = Wavelet<WV>;
#pragma unroll
    for (int k = 0; k < L::NPAIRS; ++k) {
        const float p = (float)L::p(k), u = (float)L::u(k);
        if constexpr (SCH == NONSEP) {
            nonsep_predict(q, x, p);
            nonsep_update(q, x, u);
        } else {
            sep_predict_h(q, p);
            sep_predict_v(q, x, p);
            sep_update_h(q, u);
            sep_update_v(q, x, u);
        }
    }
}

// The inverse undoes each step with the negated filter, in reverse order.
template <int WV, int SCH, int ROWS, int QPL, int WAVES>
__device__ __forceinline__ void lift_inverse(Quads<ROWS, QPL> &q, Exchange<ROWS, QPL, WAVES> &x) {
    using L = Wavelet<WV>;
#pragma unroll
    for (int k = L::NPAIRS - 1; k >= 0; --k) {
        const float p = -(float)L::p(k), u = -(float)L::u(k);
        if constexpr (SCH == NONSEP) {
            nonsep_update(q, x, u);
            nonsep_predict(q, x, p);
        } else {
            sep_update_v(q, x, u);
            sep_update_h(q, u);
            sep_predict_v(q, x, p);
            sep_predict_h(q, p);
        }
    }
}

}  // namespace dwt2

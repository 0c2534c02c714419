// C ABI of the 2-D DWT library: argument checking, level planning, launches.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <algorithm>
#include <cstring>
#include <atomic>
#include <mutex>
#include <type_traits>
#include <vector>

#include "dwt2.h"
#include "dwt2_table.hpp"

namespace dwt2 {

int resident_blocks(const void *kernel, int block_threads) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1024;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block_threads, 0) !=
            hipSuccess ||
        per_cu <= 0)
        per_cu = 1;
    return cus * per_cu;
}

}  // namespace dwt2

namespace {

using namespace dwt2;

thread_local int g_last_hip_error = 0;

int hip_fail(hipError_t e) {
    g_last_hip_error = (int)e;
    return DWT2_ERR_HIP;
}

size_t elem_size(int dt) { return dt == DWT2_F32 ? 4 : 2; }
bool valid_dtype(int dt) { return dt == DWT2_F32 || dt == DWT2_F16 || dt == DWT2_BF16; }
bool valid_wavelet(int w) { return w == DWT2_CDF97 || w == DWT2_CDF53; }
bool valid_scheme(int s) { return s >= DWT2_NONSEPARABLE && s <= DWT2_SEPARABLE_LDS; }
// The exchange ablation schemes: FP32 level kernels of 2-D tile configurations.
bool lds_scheme(int s) { return s == DWT2_NONSEPARABLE_LDS || s == DWT2_SEPARABLE_LDS; }
bool lds_scheme_ok(int dt0, int dt1, int dt2) {
    return dt0 == DWT2_F32 && dt1 == DWT2_F32 && dt2 == DWT2_F32;
}

// The bytes of a rows x cols buffer with row starts `pitch` bytes apart:
// {base + r * pitch + c : 0 <= r < rows, 0 <= c < row_bytes}.
struct Region {
    uintptr_t base;
    int64_t rows, row_bytes, pitch;
    uintptr_t lo() const { return base; }
    uintptr_t hi() const {   // one past the last byte
        return rows > 0 ? base + (uintptr_t)((rows - 1) * pitch + row_bytes) : base;
    }
};
Region region_of(const void *p, int64_t rows, int64_t cols, int64_t pitch, int dt) {
    const int64_t es = (int64_t)elem_size(dt);
    return {(uintptr_t)p, rows, cols * es, pitch * es};
}
// A contiguous byte range as a one-row region.
Region bytes_region(const void *p, size_t n) {
    return {(uintptr_t)p, n > 0 ? 1 : 0, (int64_t)n, (int64_t)n};
}

// True when two regions share a byte. Regions with the same pitch (the bands
// of one Mallat array, sub-images of one tensor) are tested exactly: bytes
// a.base + r1 p + c1 and b.base + r2 p + c2 coincide when, for k = r1 - r2,
// c1 - c2 = d - k p with d = b.base - a.base; since c1 - c2 lies in
// (-b.row_bytes, a.row_bytes) and both row lengths are at most p, only the two
// k next to d / p can qualify; a contiguous range counts as one row of the
// other region's pitch. Other pairs are tested by their byte spans, which may
// refuse interleaved buffers of different pitches.
bool regions_overlap(Region a, Region b) {
    if (a.rows <= 0 || b.rows <= 0 || a.row_bytes <= 0 || b.row_bytes <= 0) return false;
    if (!(a.lo() < b.hi() && b.lo() < a.hi())) return false;
    // a single row (a contiguous range) takes the other region's pitch
    if (a.rows == 1) a.pitch = b.pitch;
    if (b.rows == 1) b.pitch = a.pitch;
    const int64_t p = a.pitch;
    if (p != b.pitch || a.row_bytes > p || b.row_bytes > p || (a.rows > 1 && p <= 0))
        return true;   // the byte spans overlap
    if (a.rows == 1 && b.rows == 1) return true;
    const int64_t d = (int64_t)(b.base - a.base);   // two's complement difference
    int64_t k0 = d / p;
    if (d % p != 0 && d < 0) --k0;                   // floor(d / p)
    for (int64_t k = k0; k <= k0 + 1; ++k) {
        if (k < -(b.rows - 1) || k > a.rows - 1) continue;
        const int64_t c = d - k * p;                 // c1 - c2
        if (c > -b.row_bytes && c < a.row_bytes) return true;
    }
    return false;
}

// One buffer access of a batched call: which image (or job) makes it, and
// whether it writes.
struct Access {
    Region r;
    int owner;
    bool write;
};

// True when some buffer written for one image (job) shares a byte with any
// buffer another image (job) reads or writes: such calls would race. Sorted
// by start address, each access is tested only against the accesses whose
// byte spans begin inside its own.
bool cross_conflict(std::vector<Access> &v) {
    std::sort(v.begin(), v.end(),
              [](const Access &x, const Access &y) { return x.r.lo() < y.r.lo(); });
    for (size_t i = 0; i < v.size(); ++i)
        for (size_t j = i + 1; j < v.size() && v[j].r.lo() < v[i].r.hi(); ++j)
            if (v[i].owner != v[j].owner && (v[i].write || v[j].write) &&
                regions_overlap(v[i].r, v[j].r))
                return true;
    return false;
}

bool aligned(const void *p, int64_t pitch, int dt, int vec_elems) {
    size_t bytes = (size_t)vec_elems * elem_size(dt);
    if (bytes > 16) bytes = 16;
    return ((uintptr_t)p % bytes) == 0 && ((size_t)pitch * elem_size(dt)) % bytes == 0;
}

int pairs_of(int wavelet) { return wavelet == DWT2_CDF97 ? 2 : 1; }

// Output quads per tile along x and y: the window minus the lifting halo
// (one lane's quads on each side; one quad row per lifting pair above and
// below).
int out_x(int tile, int wavelet) {
    (void)wavelet;
    return 64 * kTiles[tile].qpl - 2 * kTiles[tile].qpl;
}
int out_y(int tile, int wavelet) {
    return kTiles[tile].waves * kTiles[tile].rows - 2 * pairs_of(wavelet);
}

// Tile grid of one level.
struct Plan {
    int tiles_x, tiles_y;
};
Plan plan_level(int tile, int wavelet, int nqx, int nqy) {
    const int ox = out_x(tile, wavelet), oy = out_y(tile, wavelet);
    return {(nqx + ox - 1) / ox, (nqy + oy - 1) / oy};
}

// Configuration choice for one level: the 128 x 16-quad window held by 8
// wavefronts of 2 quad rows was the fastest measured configuration from
// 1024^2 to 4096^2 levels in both directions with FP32 storage (more
// wavefronts with fewer rows each keep more loads in flight per workgroup
// than 4 of 4 rows). With 16-bit storage each lane moves half the bytes per
// row, and above 2048^2 pixels 4 wavefronts of 4 rows measured faster.
int pick_tile(int width, int height, int wavelet, int storage) {
    (void)wavelet;
    if (storage != DWT2_F32 && (int64_t)width * height > (int64_t)2048 * 2048) return 1;
    return 0;
}

// Sizes of reconstructed image (bytes) that dwt2_inverse writes with
// non-temporal stores. Nothing in the transform reads its output again, and
// streaming it keeps the 256 MiB Infinity Cache for the bands the inverse
// reads; that measured faster from 32 MiB up to the cache's size. Smaller
// images stay cached for whatever consumes them next; beyond the cache's size
// there is nothing left to protect, and cached stores measured as fast or
// faster.
constexpr int64_t kStreamOutMinBytes = (int64_t)32 << 20;
constexpr int64_t kStreamOutMaxBytes = (int64_t)256 << 20;

const FwdTable &fwd_table(int dt) {
    return dt == DWT2_F32 ? kFwdF32 : dt == DWT2_F16 ? kFwdF16 : kFwdBF16;
}
const InvTable &inv_table(int dt) {
    return dt == DWT2_F32 ? kInvF32 : dt == DWT2_F16 ? kInvF16 : kInvBF16;
}
const FwdBatchTable &fwd_batch_table(int dt) {
    return dt == DWT2_F32 ? kFwdBatchF32 : dt == DWT2_F16 ? kFwdBatchF16 : kFwdBatchBF16;
}
const InvBatchTable &inv_batch_table(int dt) {
    return dt == DWT2_F32 ? kInvBatchF32 : dt == DWT2_F16 ? kInvBatchF16 : kInvBatchBF16;
}

const FwdTailTable &fwd_tail_table(int dt) {
    return dt == DWT2_F32 ? kFwdTailF32 : dt == DWT2_F16 ? kFwdTailF16 : kFwdTailBF16;
}
const InvTailTable &inv_tail_table(int dt) {
    return dt == DWT2_F32 ? kInvTailF32 : dt == DWT2_F16 ? kInvTailF16 : kInvTailBF16;
}

const FwdHeadTable &fwd_head_table(int dt) {
    return dt == DWT2_F32 ? kFwdHeadF32 : dt == DWT2_F16 ? kFwdHeadF16 : kFwdHeadBF16;
}
const InvHeadTable &inv_head_table(int dt) {
    return dt == DWT2_F32 ? kInvHeadF32 : dt == DWT2_F16 ? kInvHeadF16 : kInvHeadBF16;
}

static_assert(DWT2_TAIL_MAX == kTailMax, "header and kernels agree on the fused depth");

// First fused level (1-based) of an L-level transform, or levels + 1 when no
// level is fused. With explicit tiles the DWT2_TILE_TAIL entries must form a
// suffix of 2..kTailMax levels (else -1).
int tail_start(int W, int H, int levels, const int32_t *tiles) {
    if (tiles) {   // (head entries are validated separately)
        int k = levels + 1;
        while (k > 1 && tiles[k - 2] == DWT2_TILE_TAIL) --k;
        for (int j = 1; j < k; ++j)
            if (tiles[j - 1] == DWT2_TILE_TAIL) return -1;
        const int F = levels + 1 - k;
        if (F == 0) return k;
        return (F >= 2 && F <= kTailMax) ? k : -1;
    }
    int k = levels + 1;
    while (k > 1 && levels + 2 - k <= kTailMax &&
           (int64_t)(W >> (k - 2)) * (int64_t)(H >> (k - 2)) <= DWT2_TAIL_AUTO_PIXELS)
        --k;
    return levels + 1 - k >= 2 ? k : levels + 1;
}

// True when levels 1 and 2 run as one fused launch (dwt2_head.hpp): when
// asked for with DWT2_TILE_HEAD in tiles[0] and tiles[1], or by default when
// there are two or more levels and the fused tail starts at level 3 or later
// (k: first tail level). The exchange-ablation schemes never fuse.
bool use_head(int levels, const int32_t *tiles, int k, int scheme) {
    if (lds_scheme(scheme) || levels < 2) return false;
    if (tiles) return tiles[0] == DWT2_TILE_HEAD;
    return k >= 3;
}

// Block side and region extensions of a fused tail (see dwt2_tail.hpp).
// Forward: level m = 0 is the finest; inverse: m = 0 is the coarsest.
struct TailPlan {
    int B, e[kTailMax];
};

// Compute units of the current device (queried once per device).
int device_cus() {
    static std::atomic<int> cus[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int n = cus[dev].load(std::memory_order_relaxed);
    if (n <= 0) {
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            n <= 0)
            n = 256;
        cus[dev].store(n, std::memory_order_relaxed);
    }
    return n;
}

// Block side of a tail whose block-owning level has nqx x nqy quads, given the
// largest side that fits (fit): the smallest side whose grid still has at most
// one workgroup per CU, and at least 2. Each workgroup's latency chain shortens with its
// region, and the tail runs in one round, so up to that point smaller blocks
// are faster; beyond it workgroups share CUs. Measured on both directions at
// 2048^2 to 8192^2 (e.g. 4096^2, three levels: 11.9 -> 11.0 us forward with
// 256 instead of 225 workgroups); the results do not depend on the block.
int tail_block(int fit, int nqx, int nqy) {
    const int64_t cus = device_cus();
    int B = fit;
    while (B > 2 && (int64_t)((nqx + B - 2) / (B - 1)) * ((nqy + B - 2) / (B - 1)) <= cus) --B;
    return B;
}

TailPlan plan_fwd_tail(int F, int wavelet, int nqx_last, int nqy_last) {
    const int R = wavelet == DWT2_CDF97 ? 2 : 1;
    TailPlan t;
    t.e[F - 1] = 0;
    for (int m = F - 2; m >= 0; --m) t.e[m] = 2 * t.e[m + 1] + 2 * R;
    int B = 1 << 30;
    for (int m = 0; m < F; ++m) {
        int lim = kTailWin - 2 * R;                       // the register window
        if (m < F - 1 && lim > kTailBufSide) lim = kTailBufSide;   // the LDS region
        const int b = (lim - 2 * t.e[m]) >> (F - 1 - m);
        if (b < B) B = b;
    }
    t.B = tail_block(B, nqx_last, nqy_last);
    return t;
}

TailPlan plan_inv_tail(int F, int wavelet, int nqx_first, int nqy_first) {
    const int R = wavelet == DWT2_CDF97 ? 2 : 1;
    TailPlan t;
    t.e[F - 1] = 0;
    for (int m = F - 2; m >= 0; --m) t.e[m] = (t.e[m + 1] + R + 1) / 2;
    int B = 1 << 30;
    for (int m = 0; m < F; ++m) {
        int b = (kTailWin - 2 * R - 2 * t.e[m]) >> m;
        if (m < F - 1) {
            const int bl = (kTailBufSide / 2 - 2 * t.e[m]) >> m;   // output pixels in LDS
            if (bl < b) b = bl;
        }
        if (b < B) B = b;
    }
    // The largest block leaves most of the GPU idle (100 workgroups for the
    // three-level tail at 4096^2): as the forward, the smallest block whose
    // grid fits one workgroup per CU (4096^2: 10.4 -> 9.6 us against the
    // earlier cap of 28 quads at the finest level).
    t.B = tail_block(B, nqx_first, nqy_first);
    return t;
}

// Size class of a level whose input is width x height pixels.
int size_class(int width, int height) {
    const int64_t px = (int64_t)width * height;
    if (px <= 128 * 128) return 0;
    if (px <= 512 * 512) return 1;
    if (px <= 2048 * 2048) return 2;
    return 3;
}
// Default tile per size class and storage type (the same choice as
// pick_tile for a level of that class).
int class_tile(int cls, int storage) {
    return (cls == DWT2_SIZE_CLASSES - 1 && storage != DWT2_F32) ? 1 : 0;
}

int check_level_dims(int32_t width, int32_t height) {
    if (width < 2 || height < 2 || (width & 1) || (height & 1)) return DWT2_ERR_INVALID_ARG;
    return DWT2_OK;
}

FwdParams fwd_params(const void *in, int64_t in_pitch, int in_dt, int width, int height, void *ll,
                     int64_t ll_pitch, int ll_dt, void *hl, void *lh, void *hh,
                     int64_t band_pitch, int band_dt, int wavelet, int tile) {
    const int nqx = width / 2, nqy = height / 2;
    FwdParams p;
    p.in = in; p.in_pitch = in_pitch;
    p.ll = ll; p.ll_pitch = ll_pitch;
    p.hl = hl; p.lh = lh; p.hh = hh; p.band_pitch = band_pitch;
    p.w = width; p.h = height; p.nqx = nqx; p.nqy = nqy;
    const Plan pl = plan_level(tile, wavelet, nqx, nqy);
    p.tiles_x = pl.tiles_x; p.tiles_y = pl.tiles_y;
    const int q = kTiles[tile].qpl;
    p.vec_in = aligned(in, in_pitch, in_dt, 2 * q);
    p.vec_ll = aligned(ll, ll_pitch, ll_dt, q);
    p.vec_band = aligned(hl, band_pitch, band_dt, q) && aligned(lh, band_pitch, band_dt, q) &&
                 aligned(hh, band_pitch, band_dt, q);
    return p;
}

InvParams inv_params(const void *ll, int64_t ll_pitch, int ll_dt, const void *hl, const void *lh,
                     const void *hh, int64_t band_pitch, int band_dt, void *out,
                     int64_t out_pitch, int out_dt, int width, int height, int wavelet,
                     int tile) {
    const int nqx = width / 2, nqy = height / 2;
    InvParams p;
    p.ll = ll; p.ll_pitch = ll_pitch;
    p.hl = hl; p.lh = lh; p.hh = hh; p.band_pitch = band_pitch;
    p.out = out; p.out_pitch = out_pitch;
    p.w = width; p.h = height; p.nqx = nqx; p.nqy = nqy;
    const Plan pl = plan_level(tile, wavelet, nqx, nqy);
    p.tiles_x = pl.tiles_x; p.tiles_y = pl.tiles_y;
    const int q = kTiles[tile].qpl;
    p.vec_ll = aligned(ll, ll_pitch, ll_dt, q);
    p.vec_band = aligned(hl, band_pitch, band_dt, q) && aligned(lh, band_pitch, band_dt, q) &&
                 aligned(hh, band_pitch, band_dt, q);
    p.vec_out = aligned(out, out_pitch, out_dt, 2 * q);
    p.stream_out = 0;
    return p;
}

int fwd_level(const void *in, int64_t in_pitch, int in_dt, int width, int height,
              void *ll, int64_t ll_pitch, int ll_dt, void *hl, void *lh, void *hh,
              int64_t band_pitch, int band_dt, int wavelet, int scheme, int tile,
              hipStream_t stream) {
    if (tile < 0) tile = pick_tile(width, height, wavelet, in_dt);
    const FwdParams p = fwd_params(in, in_pitch, in_dt, width, height, ll, ll_pitch, ll_dt, hl, lh,
                                   hh, band_pitch, band_dt, wavelet, tile);
    const FwdLauncher f =
        lds_scheme(scheme)
            ? kFwdLds[wavelet][scheme - DWT2_NONSEPARABLE_LDS][tile]
            : fwd_table(band_dt)[wavelet][scheme][in_dt == DWT2_F32][ll_dt == DWT2_F32][tile];
    const hipError_t e = f(p, stream);
    return e == hipSuccess ? DWT2_OK : hip_fail(e);
}

int inv_level(const void *ll, int64_t ll_pitch, int ll_dt, const void *hl, const void *lh,
              const void *hh, int64_t band_pitch, int band_dt, void *out, int64_t out_pitch,
              int out_dt, int width, int height, int wavelet, int scheme, int tile,
              hipStream_t stream, bool stream_out = false) {
    if (tile < 0) tile = pick_tile(width, height, wavelet, out_dt);
    InvParams p = inv_params(ll, ll_pitch, ll_dt, hl, lh, hh, band_pitch, band_dt, out,
                             out_pitch, out_dt, width, height, wavelet, tile);
    p.stream_out = stream_out;
    const InvLauncher f =
        lds_scheme(scheme)
            ? kInvLds[wavelet][scheme - DWT2_NONSEPARABLE_LDS][tile]
            : inv_table(band_dt)[wavelet][scheme][ll_dt == DWT2_F32][out_dt == DWT2_F32][tile];
    const hipError_t e = f(p, stream);
    return e == hipSuccess ? DWT2_OK : hip_fail(e);
}

// Checks shared by the one-level entry points. `a` is the full-resolution
// buffer (input of the forward, output of the inverse).
int check_level_args(const void *a, int64_t a_pitch, int a_dt, int32_t width, int32_t height,
                     const void *ll, int64_t ll_pitch, int ll_dt, const void *hl,
                     const void *lh, const void *hh, int64_t band_pitch, int band_dt,
                     int32_t wavelet, int32_t scheme, int32_t tile) {
    if (!a || !ll || !hl || !lh || !hh) return DWT2_ERR_INVALID_ARG;
    if (check_level_dims(width, height)) return DWT2_ERR_INVALID_ARG;
    if (!valid_dtype(a_dt) || !valid_dtype(ll_dt) || !valid_dtype(band_dt) ||
        !valid_wavelet(wavelet) || !valid_scheme(scheme))
        return DWT2_ERR_UNSUPPORTED;
    if (tile >= kNumTiles) return DWT2_ERR_UNSUPPORTED;
    if (lds_scheme(scheme) && !lds_scheme_ok(a_dt, ll_dt, band_dt)) return DWT2_ERR_UNSUPPORTED;
    // The full-resolution and LL buffers are either FP32 or the band type.
    if ((a_dt != band_dt && a_dt != DWT2_F32) || (ll_dt != band_dt && ll_dt != DWT2_F32))
        return DWT2_ERR_INVALID_ARG;
    const int nqx = width / 2, nqy = height / 2;
    if (a_pitch < width || ll_pitch < nqx || band_pitch < nqx) return DWT2_ERR_INVALID_ARG;
    // no two of the five buffers may share a byte
    const Region r[5] = {region_of(a, height, width, a_pitch, a_dt),
                         region_of(ll, nqy, nqx, ll_pitch, ll_dt),
                         region_of(hl, nqy, nqx, band_pitch, band_dt),
                         region_of(lh, nqy, nqx, band_pitch, band_dt),
                         region_of(hh, nqy, nqx, band_pitch, band_dt)};
    for (int i = 0; i < 5; ++i)
        for (int j = i + 1; j < 5; ++j)
            if (regions_overlap(r[i], r[j])) return DWT2_ERR_INVALID_ARG;
    return DWT2_OK;
}

// Checks shared by the multi-level entry points.
int check_multi(const void *x, const dwt2_desc *xd, const void *y, const dwt2_desc *yd,
                int32_t wavelet, int32_t levels, int32_t boundary, int32_t scheme,
                const int32_t *tiles, const void *ws, size_t ws_bytes) {
    if (!x || !xd || !y || !yd) return DWT2_ERR_INVALID_ARG;
    if (!valid_wavelet(wavelet) || !valid_scheme(scheme) ||
        boundary != DWT2_EXT_WHOLE_SAMPLE_SYMMETRIC || !valid_dtype(xd->dtype) ||
        !valid_dtype(yd->dtype))
        return DWT2_ERR_UNSUPPORTED;
    if (levels < 1 || levels > 16) return DWT2_ERR_INVALID_ARG;
    const int32_t W = xd->width, H = xd->height;
    if (yd->width != W || yd->height != H || yd->dtype != xd->dtype) return DWT2_ERR_INVALID_ARG;
    if (W < 2 || H < 2) return DWT2_ERR_INVALID_ARG;
    if ((W % (1 << levels)) != 0 || (H % (1 << levels)) != 0) return DWT2_ERR_INVALID_ARG;
    if (xd->pitch < W || yd->pitch < W) return DWT2_ERR_INVALID_ARG;
    if (tiles) {
        for (int j = 0; j < levels; ++j) {
            if (tiles[j] == DWT2_TILE_HEAD) {   // levels 1 and 2 only, both marked
                if (j > 1 || levels < 2 || tiles[0] != DWT2_TILE_HEAD ||
                    tiles[1] != DWT2_TILE_HEAD)
                    return DWT2_ERR_UNSUPPORTED;
                continue;
            }
            if (tiles[j] < DWT2_TILE_TAIL || tiles[j] >= kNumTiles) return DWT2_ERR_UNSUPPORTED;
        }
        const int k = tail_start(W, H, levels, tiles);
        if (k < 0 || (tiles[0] == DWT2_TILE_HEAD && k < 3)) return DWT2_ERR_UNSUPPORTED;
    }
    if (lds_scheme(scheme)) {   // no fused tail; FP32 2-D tiles only
        if (xd->dtype != DWT2_F32) return DWT2_ERR_UNSUPPORTED;
        for (int j = 0; tiles && j < levels; ++j)
            if (tiles[j] == DWT2_TILE_TAIL || tiles[j] == DWT2_TILE_HEAD)
                return DWT2_ERR_UNSUPPORTED;
    }
    const Region sx = region_of(x, H, W, xd->pitch, xd->dtype);
    const Region sy = region_of(y, H, W, yd->pitch, yd->dtype);
    if (regions_overlap(sx, sy)) return DWT2_ERR_INVALID_ARG;
    const size_t need = dwt2_workspace_bytes(W, H, levels, DWT2_F32);
    if (need > 0) {
        if (!ws || ws_bytes < need) return DWT2_ERR_WORKSPACE;
        const Region sw = bytes_region(ws, need);
        if (regions_overlap(sw, sx) || regions_overlap(sw, sy)) return DWT2_ERR_INVALID_ARG;
    }
    return DWT2_OK;
}

// Checks one batch image (same rules as the multi-level entry points).
int check_batch_image(const dwt2_image &im, int32_t dtype, int32_t levels) {
    const dwt2_desc a{im.width, im.height, im.src_pitch, (dwt2_dtype)dtype};
    const dwt2_desc b{im.width, im.height, im.dst_pitch, (dwt2_dtype)dtype};
    return check_multi(im.src, &a, im.dst, &b, DWT2_CDF97, levels, DWT2_EXT_WHOLE_SAMPLE_SYMMETRIC,
                       DWT2_NONSEPARABLE, nullptr, im.workspace, im.workspace_bytes);
}

// Images of one batch that write a buffer another image reads or writes.
bool batch_images_conflict(const dwt2_image *images, int n, int dtype, int levels) {
    std::vector<Access> v;
    v.reserve(3 * (size_t)(n > 0 ? n : 0));
    for (int i = 0; i < n; ++i) {
        const dwt2_image &im = images[i];
        v.push_back({region_of(im.src, im.height, im.width, im.src_pitch, dtype), i, false});
        v.push_back({region_of(im.dst, im.height, im.width, im.dst_pitch, dtype), i, true});
        v.push_back({bytes_region(im.workspace,
                                  dwt2_workspace_bytes(im.width, im.height, levels, DWT2_F32)),
                     i, true});
    }
    return cross_conflict(v);
}

// ---- planned batches ---------------------------------------------------------
// A plan is one byte image, valid both on the host (read by dwt2_batch_run for
// the launch shapes) and, copied, in device memory (read by the kernels): a
// header, one PlanLaunch per launch, then per launch the tile -> image map,
// each image's first tile and the images' level parameters. Offsets are from
// the start of the plan; sections are 256-byte aligned.
constexpr uint32_t kPlanMagic = 0x42545744u;   // "DWTB"
constexpr int32_t kPlanVersion = 2;

struct PlanHeader {
    uint32_t magic;
    int32_t version;
    int32_t n, levels, inverse, dtype, wavelet, nlaunch;
    uint64_t bytes;
};
struct PlanLaunch {
    int32_t level;          // 1-based; a head launch (levels 1 and 2) has level 1
    int32_t tile;           // tile configuration, or DWT2_TILE_HEAD
    int32_t f32_a, f32_b;   // operand types, as indexed in the single-level tables
    int32_t images;         // images in this launch
    int32_t total;          // tiles in this launch
    uint64_t off_img, off_start, off_params;
};

const PlanLaunch *plan_launches(const PlanHeader *h) {
    return reinterpret_cast<const PlanLaunch *>(reinterpret_cast<const char *>(h) +
                                                sizeof(PlanHeader));
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

const FwdHeadPlanTable &fwd_head_plan_table(int dt) {
    return dt == DWT2_F32 ? kFwdHeadPlanF32 : dt == DWT2_F16 ? kFwdHeadPlanF16 : kFwdHeadPlanBF16;
}
const InvHeadPlanTable &inv_head_plan_table(int dt) {
    return dt == DWT2_F32 ? kInvHeadPlanF32 : dt == DWT2_F16 ? kInvHeadPlanF16 : kInvHeadPlanBF16;
}

const FwdTableTable &fwd_plan_table(int dt) {
    return dt == DWT2_F32 ? kFwdPlanF32 : dt == DWT2_F16 ? kFwdPlanF16 : kFwdPlanBF16;
}
const InvTableTable &inv_plan_table(int dt) {
    return dt == DWT2_F32 ? kInvPlanF32 : dt == DWT2_F16 ? kInvPlanF16 : kInvPlanBF16;
}

// Structural checks of a host plan before its launches are read.
int check_plan(const void *plan, size_t bytes, const PlanHeader **out) {
    if (!plan || bytes < sizeof(PlanHeader)) return DWT2_ERR_INVALID_ARG;
    const PlanHeader *h = static_cast<const PlanHeader *>(plan);
    if (h->magic != kPlanMagic || h->version != kPlanVersion || h->bytes != bytes)
        return DWT2_ERR_INVALID_ARG;
    if (!valid_dtype(h->dtype) || !valid_wavelet(h->wavelet) || h->levels < 1 ||
        h->levels > 16 || h->nlaunch < 0 || h->n < 0)
        return DWT2_ERR_INVALID_ARG;
    if (sizeof(PlanHeader) + (size_t)h->nlaunch * sizeof(PlanLaunch) > bytes)
        return DWT2_ERR_INVALID_ARG;
    const PlanLaunch *L = plan_launches(h);
    for (int k = 0; k < h->nlaunch; ++k) {
        const PlanLaunch &l = L[k];
        const bool head = l.tile == DWT2_TILE_HEAD;
        const size_t psize = head ? (h->inverse ? sizeof(InvHead) : sizeof(FwdHead))
                                  : (h->inverse ? sizeof(InvParams) : sizeof(FwdParams));
        if (head ? (l.level != 1 || h->levels < 2) : (l.tile < 0 || l.tile >= kNumTiles))
            return DWT2_ERR_INVALID_ARG;
        if (l.level < 1 || l.level > h->levels || (l.f32_a | l.f32_b) & ~1 || l.images < 1 ||
            l.images > h->n || l.total < 1)
            return DWT2_ERR_INVALID_ARG;
        if (l.off_img + 4 * (uint64_t)l.total > bytes ||
            l.off_start + 4 * (uint64_t)l.images > bytes ||
            l.off_params + psize * (uint64_t)l.images > bytes)
            return DWT2_ERR_INVALID_ARG;
    }
    *out = h;
    return DWT2_OK;
}

// Plans an L-level batched transform: for each level (forward 1..L, inverse
// L..1) and each tile configuration its images' size classes use, one launch.
// With DWT2_PLAN_HEAD and L >= 2, levels 1 and 2 of every image are one head
// launch instead (planned at level 1).
int build_plan(const dwt2_image *images, int32_t n, int32_t dtype, int32_t wavelet,
               int32_t levels, int32_t inverse, int32_t boundary, const int32_t *class_tiles,
               int32_t flags, std::vector<unsigned char> &out) {
    if (n < 1 || !images) return DWT2_ERR_INVALID_ARG;
    if (!valid_dtype(dtype) || !valid_wavelet(wavelet) ||
        boundary != DWT2_EXT_WHOLE_SAMPLE_SYMMETRIC || (inverse != 0 && inverse != 1) ||
        (flags & ~DWT2_PLAN_HEAD))
        return DWT2_ERR_UNSUPPORTED;
    const bool fuse_head = (flags & DWT2_PLAN_HEAD) && levels >= 2;
    if (levels < 1 || levels > 16) return DWT2_ERR_INVALID_ARG;
    int ctile[DWT2_SIZE_CLASSES];
    for (int c = 0; c < DWT2_SIZE_CLASSES; ++c) {
        ctile[c] = class_tiles ? class_tiles[c] : class_tile(c, dtype);
        if (ctile[c] < 0 || ctile[c] >= kNumTiles) return DWT2_ERR_UNSUPPORTED;
    }
    for (int i = 0; i < n; ++i) {
        const int st = check_batch_image(images[i], dtype, levels);
        if (st) return st;
    }
    if (batch_images_conflict(images, n, dtype, levels)) return DWT2_ERR_INVALID_ARG;

    const size_t es = elem_size(dtype);
    struct Group {
        PlanLaunch l;
        std::vector<int32_t> img, start;
        std::vector<FwdParams> fp;
        std::vector<InvParams> ip;
        std::vector<FwdHead> fh;
        std::vector<InvHead> ih;
    };
    std::vector<Group> groups;
    // one head launch over every image: levels 1 and 2, as dwt2_forward /
    // dwt2_inverse plan them (the level-2 low-low band in the workspace unless
    // it is the last level's)
    auto add_head = [&]() -> int {
        Group G;
        G.l = PlanLaunch{};
        G.l.level = 1;
        G.l.tile = DWT2_TILE_HEAD;
        const int ll2_f32 = levels > 2 || dtype == DWT2_F32;
        G.l.f32_a = inverse ? ll2_f32 : dtype == DWT2_F32;
        G.l.f32_b = inverse ? dtype == DWT2_F32 : ll2_f32;
        for (int i = 0; i < n; ++i) {
            const dwt2_image &im = images[i];
            const int W = im.width, H = im.height;
            float *ws0 = static_cast<float *>(im.workspace);
            float *ws1 = ws0 + (size_t)(W / 2) * (H / 2);
            int tiles;
            if (inverse) {
                const char *cb = static_cast<const char *>(im.src);
                const int64_t cp = im.src_pitch;
                InvHead hd;
                hd.l2 = inv_params(levels == 2 ? im.src : (const void *)ws1,
                                   levels == 2 ? cp : W / 4, levels == 2 ? dtype : DWT2_F32,
                                   cb + (size_t)(W / 4) * es, cb + (size_t)((int64_t)(H / 4) * cp) * es,
                                   cb + (size_t)((int64_t)(H / 4) * cp + W / 4) * es, cp, dtype,
                                   ws0, W / 2, DWT2_F32, W / 2, H / 2, wavelet, 0);
                hd.l1 = inv_params(ws0, W / 2, DWT2_F32, cb + (size_t)(W / 2) * es,
                                   cb + (size_t)((int64_t)(H / 2) * cp) * es,
                                   cb + (size_t)((int64_t)(H / 2) * cp + W / 2) * es, cp, dtype,
                                   im.dst, im.dst_pitch, dtype, W, H, wavelet, 0);
                hd.tiles_x = (hd.l1.nqx + FwdHeadGeom::IOX1 - 1) / FwdHeadGeom::IOX1;
                hd.tiles_y = (hd.l1.nqy + FwdHeadGeom::IOY1 - 1) / FwdHeadGeom::IOY1;
                tiles = hd.tiles_x * hd.tiles_y;
                G.ih.push_back(hd);
            } else {
                char *cb = static_cast<char *>(im.dst);
                const int64_t cp = im.dst_pitch;
                FwdHead hd;
                hd.l1 = fwd_params(im.src, im.src_pitch, dtype, W, H, ws0, W / 2, DWT2_F32,
                                   cb + (size_t)(W / 2) * es, cb + (size_t)((int64_t)(H / 2) * cp) * es,
                                   cb + (size_t)((int64_t)(H / 2) * cp + W / 2) * es, cp, dtype,
                                   wavelet, 0);
                hd.l2 = fwd_params(ws0, W / 2, DWT2_F32, W / 2, H / 2,
                                   levels == 2 ? im.dst : (void *)ws1, levels == 2 ? cp : W / 4,
                                   levels == 2 ? dtype : DWT2_F32, cb + (size_t)(W / 4) * es,
                                   cb + (size_t)((int64_t)(H / 4) * cp) * es,
                                   cb + (size_t)((int64_t)(H / 4) * cp + W / 4) * es, cp, dtype,
                                   wavelet, 0);
                hd.tiles_x = (hd.l2.nqx + FwdHeadGeom::FOX2 - 1) / FwdHeadGeom::FOX2;
                hd.tiles_y = (hd.l2.nqy + FwdHeadGeom::FOY2 - 1) / FwdHeadGeom::FOY2;
                tiles = hd.tiles_x * hd.tiles_y;
                G.fh.push_back(hd);
            }
            G.start.push_back((int32_t)G.img.size());
            if ((int64_t)G.img.size() + tiles > (int64_t)INT32_MAX) return DWT2_ERR_INVALID_ARG;
            G.img.insert(G.img.end(), (size_t)tiles, (int32_t)i);
        }
        groups.push_back(std::move(G));
        return DWT2_OK;
    };
    for (int step = 0; step < levels; ++step) {
        const int j = inverse ? levels - step : step + 1;
        if (fuse_head && j <= 2) {   // the head launch, planned once at level 2 (inverse) or 1
            if (j == (inverse ? 2 : 1)) {
                const int st = add_head();
                if (st) return st;
            }
            continue;
        }
        const int first = (int)groups.size();
        for (int i = 0; i < n; ++i) {
            const dwt2_image &im = images[i];
            const int W = im.width, H = im.height;
            const int w = W >> (j - 1), h = H >> (j - 1);
            const int tile = ctile[size_class(w, h)];
            int g = first;
            while (g < (int)groups.size() && groups[g].l.tile != tile) ++g;
            if (g == (int)groups.size()) {
                Group ng;
                ng.l = PlanLaunch{};
                ng.l.level = j;
                ng.l.tile = tile;
                if (inverse) {
                    ng.l.f32_a = j == levels ? dtype == DWT2_F32 : 1;   // LL input
                    ng.l.f32_b = j == 1 ? dtype == DWT2_F32 : 1;        // level output
                } else {
                    ng.l.f32_a = j == 1 ? dtype == DWT2_F32 : 1;        // level input
                    ng.l.f32_b = j == levels ? dtype == DWT2_F32 : 1;   // LL output
                }
                groups.push_back(ng);
            }
            Group &G = groups[g];
            float *ws0 = static_cast<float *>(im.workspace);
            float *ws[2] = {ws0, ws0 ? ws0 + (size_t)(W / 2) * (H / 2) : nullptr};
            int tiles;
            if (inverse) {
                const char *cbase = static_cast<const char *>(im.src);
                const int64_t cp = im.src_pitch;
                const void *ll = j == levels ? im.src : (const void *)ws[(j - 1) & 1];
                const InvParams p = inv_params(
                    ll, j == levels ? cp : w / 2, j == levels ? dtype : DWT2_F32,
                    cbase + (size_t)(w / 2) * es, cbase + (size_t)((int64_t)(h / 2) * cp) * es,
                    cbase + (size_t)((int64_t)(h / 2) * cp + w / 2) * es, cp, dtype,
                    j == 1 ? im.dst : (void *)ws[(j - 2) & 1], j == 1 ? im.dst_pitch : w,
                    j == 1 ? dtype : DWT2_F32, w, h, wavelet, tile);
                tiles = p.tiles_x * p.tiles_y;
                G.ip.push_back(p);
            } else {
                char *cbase = static_cast<char *>(im.dst);
                const int64_t cp = im.dst_pitch;
                const FwdParams p = fwd_params(
                    j == 1 ? im.src : (const void *)ws[(j - 2) & 1], j == 1 ? im.src_pitch : w,
                    j == 1 ? dtype : DWT2_F32, w, h,
                    j == levels ? im.dst : (void *)ws[(j - 1) & 1], j == levels ? cp : w / 2,
                    j == levels ? dtype : DWT2_F32, cbase + (size_t)(w / 2) * es,
                    cbase + (size_t)((int64_t)(h / 2) * cp) * es,
                    cbase + (size_t)((int64_t)(h / 2) * cp + w / 2) * es, cp, dtype, wavelet,
                    tile);
                tiles = p.tiles_x * p.tiles_y;
                G.fp.push_back(p);
            }
            const int local = (int)G.start.size();
            G.start.push_back((int32_t)G.img.size());
            if ((int64_t)G.img.size() + tiles > (int64_t)INT32_MAX) return DWT2_ERR_INVALID_ARG;
            G.img.insert(G.img.end(), (size_t)tiles, (int32_t)local);
        }
    }
    // lay out: header, launches, then per launch its three arrays
    size_t off = align256(sizeof(PlanHeader) + groups.size() * sizeof(PlanLaunch));
    for (Group &G : groups) {
        G.l.images = (int32_t)G.start.size();
        G.l.total = (int32_t)G.img.size();
        G.l.off_img = off;
        off = align256(off + 4 * G.img.size());
        G.l.off_start = off;
        off = align256(off + 4 * G.start.size());
        G.l.off_params = off;
        off = align256(off + sizeof(InvParams) * G.ip.size() + sizeof(FwdParams) * G.fp.size() +
                       sizeof(InvHead) * G.ih.size() + sizeof(FwdHead) * G.fh.size());
    }
    out.assign(off, 0);
    PlanHeader h{kPlanMagic, kPlanVersion, n, levels, inverse, dtype, wavelet,
                 (int32_t)groups.size(), (uint64_t)off};
    std::memcpy(out.data(), &h, sizeof h);
    for (size_t k = 0; k < groups.size(); ++k) {
        const Group &G = groups[k];
        std::memcpy(out.data() + sizeof(PlanHeader) + k * sizeof(PlanLaunch), &G.l,
                    sizeof(PlanLaunch));
        std::memcpy(out.data() + G.l.off_img, G.img.data(), 4 * G.img.size());
        std::memcpy(out.data() + G.l.off_start, G.start.data(), 4 * G.start.size());
        unsigned char *prm = out.data() + G.l.off_params;
        if (!G.ih.empty()) std::memcpy(prm, G.ih.data(), sizeof(InvHead) * G.ih.size());
        if (!G.fh.empty()) std::memcpy(prm, G.fh.data(), sizeof(FwdHead) * G.fh.size());
        if (!G.ip.empty()) std::memcpy(prm, G.ip.data(), sizeof(InvParams) * G.ip.size());
        if (!G.fp.empty()) std::memcpy(prm, G.fp.data(), sizeof(FwdParams) * G.fp.size());
    }
    return DWT2_OK;
}

int record(const hipEvent_t *events, int idx, hipStream_t s) {
    if (!events) return DWT2_OK;
    const hipError_t e = hipEventRecord(events[idx], s);
    return e == hipSuccess ? DWT2_OK : hip_fail(e);
}

}  // namespace

namespace {

// Workspace of dwt2_forward_no_alloc: a device array of the library's own,
// one copy per GPU (the code object's data), never allocated or freed by a
// call. Host code uses it only through the address hipGetSymbolAddress
// returns on each device: the array's name is a host-side stand-in.
static __device__ __align__(256) unsigned char scratch[DWT2_STATIC_WORKSPACE_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices] = {};

// Address of `scratch` on the current device, looked up on the first call on
// that device (with the device current) and kept.
int scratch_on_current_device(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e);
    if (dev < 0 || dev >= kMaxDevices) return DWT2_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e);
        if (!p) return hip_fail(hipErrorInvalidSymbol);
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return DWT2_OK;
}

}  // namespace

extern "C" {

int dwt2_forward_no_alloc(const void *src, const dwt2_desc *src_d, void *coef,
                          const dwt2_desc *coef_d, dwt2_wavelet wavelet, int32_t levels,
                          dwt2_boundary boundary, dwt2_scheme scheme, hipStream_t stream) {
    // every argument check that needs no workspace, then the size limit
    int st = check_multi(src, src_d, coef, coef_d, wavelet, levels, boundary, scheme, nullptr,
                         nullptr, 0);
    if (st != DWT2_OK && st != DWT2_ERR_WORKSPACE) return st;
    if (dwt2_workspace_bytes(src_d->width, src_d->height, levels, src_d->dtype) >
        DWT2_STATIC_WORKSPACE_BYTES)
        return DWT2_ERR_WORKSPACE;
    void *ws = nullptr;
    if ((st = scratch_on_current_device(&ws))) return st;
    return dwt2_forward_ex(src, src_d, coef, coef_d, wavelet, levels, boundary, scheme, ws,
                           DWT2_STATIC_WORKSPACE_BYTES, nullptr, nullptr, stream);
}

int dwt2_version(void) { return 100; }

const char *dwt2_status_string(int status) {
    switch (status) {
        case DWT2_OK: return "ok";
        case DWT2_ERR_INVALID_ARG: return "invalid argument";
        case DWT2_ERR_UNSUPPORTED: return "unsupported wavelet, scheme, boundary, dtype or tile";
        case DWT2_ERR_WORKSPACE: return "workspace too small";
        case DWT2_ERR_HIP: return "HIP launch failed";
        default: return "unknown status";
    }
}

int dwt2_last_hip_error(void) { return g_last_hip_error; }

size_t dwt2_workspace_bytes(int32_t width, int32_t height, int32_t levels, dwt2_dtype dtype) {
    if (!valid_dtype(dtype)) return 0;
    if (width < 2 || height < 2 || levels < 1 || levels > 16) return 0;
    if ((width % (1 << levels)) != 0 || (height % (1 << levels)) != 0) return 0;
    if (levels == 1) return 0;
    size_t n = (size_t)(width / 2) * (size_t)(height / 2);
    if (levels >= 3) n += (size_t)(width / 4) * (size_t)(height / 4);
    return n * sizeof(float);
}

int dwt2_fused_levels(int32_t width, int32_t height, int32_t levels) {
    if (levels < 1 || levels > 16 || width < 2 || height < 2 ||
        (width % (1 << levels)) != 0 || (height % (1 << levels)) != 0)
        return DWT2_ERR_INVALID_ARG;
    return levels + 1 - tail_start(width, height, levels, nullptr);
}

int dwt2_head_levels(int32_t width, int32_t height, int32_t levels) {
    if (levels < 1 || levels > 16 || width < 2 || height < 2 ||
        (width % (1 << levels)) != 0 || (height % (1 << levels)) != 0)
        return DWT2_ERR_INVALID_ARG;
    return use_head(levels, nullptr, tail_start(width, height, levels, nullptr), 0) ? 2 : 0;
}

int dwt2_tile_config_count(void) { return kNumTiles; }

int dwt2_tile_config_info(int32_t tile, dwt2_wavelet wavelet, int32_t *quads_per_lane, int32_t *rows,
                          int32_t *waves, int32_t *ox, int32_t *oy) {
    if (tile < 0 || tile >= kNumTiles || !valid_wavelet(wavelet)) return DWT2_ERR_UNSUPPORTED;
    if (quads_per_lane) *quads_per_lane = kTiles[tile].qpl;
    if (rows) *rows = kTiles[tile].rows;
    if (waves) *waves = kTiles[tile].waves;
    if (ox) *ox = out_x(tile, wavelet);
    if (oy) *oy = out_y(tile, wavelet);
    return DWT2_OK;
}

int dwt2_default_tile(int32_t width, int32_t height, dwt2_wavelet wavelet, dwt2_scheme scheme,
                      dwt2_dtype dtype) {
    (void)scheme;
    if (check_level_dims(width, height) || !valid_wavelet(wavelet)) return DWT2_ERR_INVALID_ARG;
    return pick_tile(width, height, wavelet, valid_dtype(dtype) ? dtype : DWT2_F32);
}

int dwt2_forward_level(const void *in, int64_t in_pitch, dwt2_dtype in_dtype, int32_t width,
                       int32_t height, void *ll, int64_t ll_pitch, dwt2_dtype ll_dtype, void *hl,
                       void *lh, void *hh, int64_t band_pitch, dwt2_dtype band_dtype,
                       dwt2_wavelet wavelet, dwt2_scheme scheme, int32_t tile, hipStream_t stream) {
    const int st = check_level_args(in, in_pitch, in_dtype, width, height, ll, ll_pitch,
                                    ll_dtype, hl, lh, hh, band_pitch, band_dtype, wavelet,
                                    scheme, tile);
    if (st) return st;
    return fwd_level(in, in_pitch, in_dtype, width, height, ll, ll_pitch, ll_dtype, hl, lh, hh,
                     band_pitch, band_dtype, wavelet, scheme, tile, stream);
}

int dwt2_inverse_level(const void *ll, int64_t ll_pitch, dwt2_dtype ll_dtype, const void *hl,
                       const void *lh, const void *hh, int64_t band_pitch, dwt2_dtype band_dtype,
                       void *out, int64_t out_pitch, dwt2_dtype out_dtype, int32_t width,
                       int32_t height, dwt2_wavelet wavelet, dwt2_scheme scheme, int32_t tile,
                       hipStream_t stream) {
    const int st = check_level_args(out, out_pitch, out_dtype, width, height, ll, ll_pitch,
                                    ll_dtype, hl, lh, hh, band_pitch, band_dtype, wavelet,
                                    scheme, tile);
    if (st) return st;
    return inv_level(ll, ll_pitch, ll_dtype, hl, lh, hh, band_pitch, band_dtype, out, out_pitch,
                     out_dtype, width, height, wavelet, scheme, tile, stream);
}

int dwt2_forward(const void *src, const dwt2_desc *src_d, void *coef, const dwt2_desc *coef_d,
                 dwt2_wavelet wavelet, int32_t levels, dwt2_boundary boundary,
                 dwt2_scheme scheme, void *workspace, size_t workspace_bytes,
                 hipStream_t stream) {
    return dwt2_forward_ex(src, src_d, coef, coef_d, wavelet, levels, boundary, scheme,
                           workspace, workspace_bytes, nullptr, nullptr, stream);
}

int dwt2_forward_ex(const void *src, const dwt2_desc *src_d, void *coef, const dwt2_desc *coef_d,
                    dwt2_wavelet wavelet, int32_t levels, dwt2_boundary boundary,
                    dwt2_scheme scheme, void *workspace, size_t workspace_bytes,
                    const int32_t *tiles, const hipEvent_t *level_events, hipStream_t stream) {
    int st = check_multi(src, src_d, coef, coef_d, wavelet, levels, boundary, scheme, tiles,
                         workspace, workspace_bytes);
    if (st) return st;
    const hipStream_t s = stream;
    const int32_t W = src_d->width, H = src_d->height, T = src_d->dtype;
    const size_t es = elem_size(T);
    float *ws[2] = {static_cast<float *>(workspace),
                    workspace ? static_cast<float *>(workspace) + (size_t)(W / 2) * (H / 2)
                              : nullptr};
    char *cbase = static_cast<char *>(coef);
    const int64_t cp = coef_d->pitch;
    const int k = lds_scheme(scheme) ? levels + 1 : tail_start(W, H, levels, tiles);
    const bool head = use_head(levels, tiles, k, scheme);
    FwdTail tail;
    FwdHead hd;
    for (int j = 1; j <= levels; ++j) {
        const int w = W >> (j - 1), h = H >> (j - 1);
        const void *in = j == 1 ? src : (const void *)ws[(j - 2) & 1];
        const int64_t in_pitch = j == 1 ? src_d->pitch : w;
        const int in_dt = j == 1 ? T : DWT2_F32;
        void *hl = cbase + (size_t)(w / 2) * es;
        void *lh = cbase + (size_t)((int64_t)(h / 2) * cp) * es;
        void *hh = cbase + (size_t)((int64_t)(h / 2) * cp + w / 2) * es;
        void *ll = j == levels ? (void *)coef : (void *)ws[(j - 1) & 1];
        const int64_t ll_pitch = j == levels ? cp : w / 2;
        const int ll_dt = j == levels ? T : DWT2_F32;
        if (j >= k) {   // fused: parameters only (the kernel reads in of the first, ll of the last)
            tail.lv[j - k] = fwd_params(in, in_pitch, in_dt, w, h, ll, ll_pitch, ll_dt, hl, lh,
                                        hh, cp, T, wavelet, 0);
            tail.lv[j - k].vec_in = aligned(in, in_pitch, in_dt, 2);
            continue;
        }
        if (head && j <= 2) {   // levels 1 and 2: one launch once both are planned
            (j == 1 ? hd.l1 : hd.l2) = fwd_params(in, in_pitch, in_dt, w, h, ll, ll_pitch, ll_dt,
                                                  hl, lh, hh, cp, T, wavelet, 0);
            if (j == 1) continue;
            hd.tiles_x = (hd.l2.nqx + FwdHeadGeom::FOX2 - 1) / FwdHeadGeom::FOX2;
            hd.tiles_y = (hd.l2.nqy + FwdHeadGeom::FOY2 - 1) / FwdHeadGeom::FOY2;
            if ((st = record(level_events, 0, s))) return st;
            const hipError_t e =
                fwd_head_table(T)[wavelet][scheme][T == DWT2_F32][levels > 2 || T == DWT2_F32](
                    hd, s);
            if (e != hipSuccess) return hip_fail(e);
            for (int ev = 1; ev <= 3; ++ev)
                if ((st = record(level_events, ev, s))) return st;
            continue;
        }
        const int tile = tiles ? tiles[j - 1] : -1;
        if ((st = record(level_events, 2 * (j - 1), s))) return st;
        st = fwd_level(in, in_pitch, in_dt, w, h, ll, ll_pitch, ll_dt, hl, lh, hh, cp, T, wavelet,
                       scheme, tile, s);
        if (st) return st;
        if ((st = record(level_events, 2 * (j - 1) + 1, s))) return st;
    }
    if (k <= levels) {
        const int F = levels + 1 - k;
        const TailPlan pl = plan_fwd_tail(F, wavelet, tail.lv[F - 1].nqx, tail.lv[F - 1].nqy);
        tail.F = F;
        tail.B = pl.B;
        for (int m = 0; m < F; ++m) tail.e[m] = pl.e[m];
        const FwdParams &last = tail.lv[F - 1];
        tail.blocks_x = (last.nqx + pl.B - 1) / pl.B;
        const int grid = tail.blocks_x * ((last.nqy + pl.B - 1) / pl.B);
        if ((st = record(level_events, 2 * (k - 1), s))) return st;
        const hipError_t e =
            fwd_tail_table(T)[wavelet][scheme][F - 2][k > 1 || T == DWT2_F32](tail, grid, s);
        if (e != hipSuccess) return hip_fail(e);
        if ((st = record(level_events, 2 * (k - 1) + 1, s))) return st;
        for (int j = k + 1; j <= levels; ++j) {
            if ((st = record(level_events, 2 * (j - 1), s))) return st;
            if ((st = record(level_events, 2 * (j - 1) + 1, s))) return st;
        }
    }
    return DWT2_OK;
}

int dwt2_inverse(const void *coef, const dwt2_desc *coef_d, void *dst, const dwt2_desc *dst_d,
                 dwt2_wavelet wavelet, int32_t levels, dwt2_boundary boundary,
                 dwt2_scheme scheme, void *workspace, size_t workspace_bytes,
                 hipStream_t stream) {
    return dwt2_inverse_ex(coef, coef_d, dst, dst_d, wavelet, levels, boundary, scheme,
                           workspace, workspace_bytes, nullptr, nullptr, stream);
}

int dwt2_inverse_ex(const void *coef, const dwt2_desc *coef_d, void *dst, const dwt2_desc *dst_d,
                    dwt2_wavelet wavelet, int32_t levels, dwt2_boundary boundary,
                    dwt2_scheme scheme, void *workspace, size_t workspace_bytes,
                    const int32_t *tiles, const hipEvent_t *level_events, hipStream_t stream) {
    int st = check_multi(coef, coef_d, dst, dst_d, wavelet, levels, boundary, scheme, tiles,
                         workspace, workspace_bytes);
    if (st) return st;
    const hipStream_t s = stream;
    const int32_t W = coef_d->width, H = coef_d->height, T = coef_d->dtype;
    const size_t es = elem_size(T);
    float *ws[2] = {static_cast<float *>(workspace),
                    workspace ? static_cast<float *>(workspace) + (size_t)(W / 2) * (H / 2)
                              : nullptr};
    const char *cbase = static_cast<const char *>(coef);
    const int64_t cp = coef_d->pitch;
    const int k = lds_scheme(scheme) ? levels + 1 : tail_start(W, H, levels, tiles);
    const bool head = use_head(levels, tiles, k, scheme);
    InvTail tail;
    InvHead hd;
    for (int j = levels; j >= 1; --j) {
        const int w = W >> (j - 1), h = H >> (j - 1);
        const void *ll = j == levels ? coef : (const void *)ws[(j - 1) & 1];
        const int64_t ll_pitch = j == levels ? cp : w / 2;
        const int ll_dt = j == levels ? T : DWT2_F32;
        const void *hl = cbase + (size_t)(w / 2) * es;
        const void *lh = cbase + (size_t)((int64_t)(h / 2) * cp) * es;
        const void *hh = cbase + (size_t)((int64_t)(h / 2) * cp + w / 2) * es;
        void *out = j == 1 ? dst : (void *)ws[(j - 2) & 1];
        const int64_t out_pitch = j == 1 ? dst_d->pitch : w;
        const int out_dt = j == 1 ? T : DWT2_F32;
        if (j >= k) {   // fused: collected here, launched once after the loop body below
            InvParams &p = tail.lv[levels - j];
            p = inv_params(ll, ll_pitch, ll_dt, hl, lh, hh, cp, T, out, out_pitch, out_dt, w, h,
                           wavelet, 0);
            p.vec_ll = aligned(ll, ll_pitch, ll_dt, 1);
            p.vec_band = aligned(hl, cp, T, 1) && aligned(lh, cp, T, 1) && aligned(hh, cp, T, 1);
            p.vec_out = aligned(out, out_pitch, out_dt, 2);
            if (j > k) continue;
            const int F = levels + 1 - k;
            const TailPlan pl = plan_inv_tail(F, wavelet, tail.lv[0].nqx, tail.lv[0].nqy);
            tail.F = F;
            tail.B = pl.B;
            for (int m = 0; m < F; ++m) tail.e[m] = pl.e[m];
            const InvParams &first = tail.lv[0];
            tail.blocks_x = (first.nqx + pl.B - 1) / pl.B;
            const int grid = tail.blocks_x * ((first.nqy + pl.B - 1) / pl.B);
            if ((st = record(level_events, 2 * (levels - 1), s))) return st;
            const hipError_t e =
                inv_tail_table(T)[wavelet][scheme][F - 2][k > 1 || T == DWT2_F32](tail, grid, s);
            if (e != hipSuccess) return hip_fail(e);
            if ((st = record(level_events, 2 * (levels - 1) + 1, s))) return st;
            for (int jj = levels - 1; jj >= k; --jj) {
                if ((st = record(level_events, 2 * (jj - 1), s))) return st;
                if ((st = record(level_events, 2 * (jj - 1) + 1, s))) return st;
            }
            continue;
        }
        // the reconstructed image is the transform's last write
        const int64_t image_bytes = (int64_t)W * H * (int64_t)es;
        const bool stream_out = j == 1 && image_bytes >= kStreamOutMinBytes &&
                                image_bytes <= kStreamOutMaxBytes;
        if (head && j <= 2) {   // levels 2 and 1: one launch once both are planned
            (j == 2 ? hd.l2 : hd.l1) = inv_params(ll, ll_pitch, ll_dt, hl, lh, hh, cp, T, out,
                                                  out_pitch, out_dt, w, h, wavelet, 0);
            if (j == 2) continue;
            hd.l1.stream_out = stream_out;
            hd.tiles_x = (hd.l1.nqx + FwdHeadGeom::IOX1 - 1) / FwdHeadGeom::IOX1;
            hd.tiles_y = (hd.l1.nqy + FwdHeadGeom::IOY1 - 1) / FwdHeadGeom::IOY1;
            if ((st = record(level_events, 0, s))) return st;
            const hipError_t e =
                inv_head_table(T)[wavelet][scheme][levels > 2 || T == DWT2_F32][T == DWT2_F32](
                    hd, s);
            if (e != hipSuccess) return hip_fail(e);
            for (int ev = 1; ev <= 3; ++ev)
                if ((st = record(level_events, ev, s))) return st;
            continue;
        }
        const int tile = tiles ? tiles[j - 1] : -1;
        if ((st = record(level_events, 2 * (j - 1), s))) return st;
        st = inv_level(ll, ll_pitch, ll_dt, hl, lh, hh, cp, T, out, out_pitch, out_dt, w, h,
                       wavelet, scheme, tile, s, stream_out);
        if (st) return st;
        if ((st = record(level_events, 2 * (j - 1) + 1, s))) return st;
    }
    return DWT2_OK;
}

}  // extern "C"

extern "C" {

int dwt2_size_class(int32_t width, int32_t height) {
    if (width < 2 || height < 2) return DWT2_ERR_INVALID_ARG;
    return size_class(width, height);
}

int dwt2_batch_plan_bytes(const dwt2_image *images, int32_t n, dwt2_dtype dtype,
                          dwt2_wavelet wavelet, int32_t levels, int32_t inverse,
                          dwt2_boundary boundary, const int32_t *class_tiles, int32_t flags,
                          size_t *bytes) {
    if (!bytes) return DWT2_ERR_INVALID_ARG;
    std::vector<unsigned char> plan;
    const int st = build_plan(images, n, dtype, wavelet, levels, inverse, boundary, class_tiles,
                              flags, plan);
    if (st) return st;
    *bytes = plan.size();
    return DWT2_OK;
}

int dwt2_batch_plan(const dwt2_image *images, int32_t n, dwt2_dtype dtype, dwt2_wavelet wavelet,
                    int32_t levels, int32_t inverse, dwt2_boundary boundary,
                    const int32_t *class_tiles, int32_t flags, void *plan, size_t plan_bytes) {
    if (!plan) return DWT2_ERR_INVALID_ARG;
    std::vector<unsigned char> v;
    const int st = build_plan(images, n, dtype, wavelet, levels, inverse, boundary, class_tiles,
                              flags, v);
    if (st) return st;
    if (plan_bytes < v.size()) return DWT2_ERR_WORKSPACE;
    std::memcpy(plan, v.data(), v.size());
    return DWT2_OK;
}

int dwt2_batch_launches(const void *plan, size_t plan_bytes, int32_t *launches,
                        int32_t *per_level) {
    const PlanHeader *h = nullptr;
    const int st = check_plan(plan, plan_bytes, &h);
    if (st) return st;
    if (launches) *launches = h->nlaunch;
    if (per_level) {
        for (int j = 0; j < h->levels; ++j) per_level[j] = 0;
        const PlanLaunch *L = plan_launches(h);
        for (int k = 0; k < h->nlaunch; ++k) ++per_level[L[k].level - 1];
    }
    return DWT2_OK;
}

int dwt2_batch_run(const void *plan, size_t plan_bytes, const void *plan_device,
                   dwt2_scheme scheme, int32_t flags, hipStream_t stream) {
    const PlanHeader *h = nullptr;
    int st = check_plan(plan, plan_bytes, &h);
    if (st) return st;
    if (!plan_device) return DWT2_ERR_INVALID_ARG;
    if (!valid_scheme(scheme) || lds_scheme(scheme)) return DWT2_ERR_UNSUPPORTED;
    if (flags & ~DWT2_BATCH_PERSISTENT) return DWT2_ERR_UNSUPPORTED;
    const bool persistent = (flags & DWT2_BATCH_PERSISTENT) != 0;
    const char *dev = static_cast<const char *>(plan_device);
    const PlanLaunch *L = plan_launches(h);
    for (int k = 0; k < h->nlaunch; ++k) {
        const PlanLaunch &l = L[k];
        hipError_t e;
        if (l.tile == DWT2_TILE_HEAD && h->inverse) {
            TableLaunch<InvHead> tl{reinterpret_cast<const int32_t *>(dev + l.off_img),
                                    reinterpret_cast<const int32_t *>(dev + l.off_start),
                                    reinterpret_cast<const InvHead *>(dev + l.off_params),
                                    l.total};
            e = inv_head_plan_table(h->dtype)[h->wavelet][scheme][l.f32_a][l.f32_b](
                tl, persistent, stream);
        } else if (l.tile == DWT2_TILE_HEAD) {
            TableLaunch<FwdHead> tl{reinterpret_cast<const int32_t *>(dev + l.off_img),
                                    reinterpret_cast<const int32_t *>(dev + l.off_start),
                                    reinterpret_cast<const FwdHead *>(dev + l.off_params),
                                    l.total};
            e = fwd_head_plan_table(h->dtype)[h->wavelet][scheme][l.f32_a][l.f32_b](
                tl, persistent, stream);
        } else if (h->inverse) {
            TableLaunch<InvParams> tl{reinterpret_cast<const int32_t *>(dev + l.off_img),
                                      reinterpret_cast<const int32_t *>(dev + l.off_start),
                                      reinterpret_cast<const InvParams *>(dev + l.off_params),
                                      l.total};
            e = inv_plan_table(h->dtype)[h->wavelet][scheme][l.f32_a][l.f32_b][l.tile](
                tl, persistent, stream);
        } else {
            TableLaunch<FwdParams> tl{reinterpret_cast<const int32_t *>(dev + l.off_img),
                                      reinterpret_cast<const int32_t *>(dev + l.off_start),
                                      reinterpret_cast<const FwdParams *>(dev + l.off_params),
                                      l.total};
            e = fwd_plan_table(h->dtype)[h->wavelet][scheme][l.f32_a][l.f32_b][l.tile](
                tl, persistent, stream);
        }
        if (e != hipSuccess) return hip_fail(e);
    }
    return DWT2_OK;
}

}  // extern "C"

namespace {

// Jobs of one launch group share size class and storage types.
struct JobKey {
    int cls, full_dt, ll_dt, band_dt;
    bool operator==(const JobKey &o) const {
        return cls == o.cls && full_dt == o.full_dt && ll_dt == o.ll_dt && band_dt == o.band_dt;
    }
};

template <bool INV>
int level_batch(const dwt2_level_job *jobs, int32_t n, int32_t wavelet, int32_t scheme,
                const int32_t *class_tiles, hipStream_t stream) {
    if (n < 0 || (n > 0 && !jobs)) return DWT2_ERR_INVALID_ARG;
    if (!valid_wavelet(wavelet) || !valid_scheme(scheme) || lds_scheme(scheme))
        return DWT2_ERR_UNSUPPORTED;
    int ctile[DWT2_SIZE_CLASSES];
    for (int c = 0; c < DWT2_SIZE_CLASSES; ++c) {
        ctile[c] = class_tiles ? class_tiles[c] : -1;   // -1: by storage, per group below
        if (class_tiles && (ctile[c] < 0 || ctile[c] >= kNumTiles)) return DWT2_ERR_UNSUPPORTED;
    }
    for (int i = 0; i < n; ++i) {
        const dwt2_level_job &j = jobs[i];
        const int st = check_level_args(j.full, j.full_pitch, j.full_dtype, j.width, j.height,
                                        j.ll, j.ll_pitch, j.ll_dtype, j.hl, j.lh, j.hh,
                                        j.band_pitch, j.band_dtype, wavelet, scheme, 0);
        if (st) return st;
    }
    {   // the forward writes the bands and reads `full`; the inverse the reverse
        std::vector<Access> v;
        v.reserve(5 * (size_t)(n > 0 ? n : 0));
        for (int i = 0; i < n; ++i) {
            const dwt2_level_job &j = jobs[i];
            const int nqx = j.width / 2, nqy = j.height / 2;
            v.push_back({region_of(j.full, j.height, j.width, j.full_pitch, j.full_dtype), i, INV});
            v.push_back({region_of(j.ll, nqy, nqx, j.ll_pitch, j.ll_dtype), i, !INV});
            v.push_back({region_of(j.hl, nqy, nqx, j.band_pitch, j.band_dtype), i, !INV});
            v.push_back({region_of(j.lh, nqy, nqx, j.band_pitch, j.band_dtype), i, !INV});
            v.push_back({region_of(j.hh, nqy, nqx, j.band_pitch, j.band_dtype), i, !INV});
        }
        if (cross_conflict(v)) return DWT2_ERR_INVALID_ARG;
    }
    const hipStream_t s = stream;
    std::vector<JobKey> keys(n > 0 ? n : 1);
    std::vector<char> done(n > 0 ? n : 1);
    for (int i = 0; i < n; ++i) {
        keys[i] = {size_class(jobs[i].width, jobs[i].height), jobs[i].full_dtype, jobs[i].ll_dtype,
                   jobs[i].band_dtype};
        done[i] = false;
    }
    int st = DWT2_OK;
    // one group per distinct key, in order of first appearance
    for (int g = 0; g < n && st == DWT2_OK; ++g) {
        if (done[g]) continue;
        const JobKey key = keys[g];
        const int tile = ctile[key.cls] >= 0 ? ctile[key.cls] : class_tile(key.cls, key.full_dt);
        typename std::conditional<INV, InvBatch, FwdBatch>::type b;
        b.n = 0;
        b.tile_start[0] = 0;
        for (int i = g; i <= n && st == DWT2_OK; ++i) {
            if (i < n && !done[i] && keys[i] == key) {
                const dwt2_level_job &j = jobs[i];
                if constexpr (INV) {
                    b.p[b.n] = inv_params(j.ll, j.ll_pitch, j.ll_dtype, j.hl, j.lh, j.hh,
                                          j.band_pitch, j.band_dtype, j.full, j.full_pitch,
                                          j.full_dtype, j.width, j.height, wavelet, tile);
                } else {
                    b.p[b.n] = fwd_params(j.full, j.full_pitch, j.full_dtype, j.width, j.height,
                                          j.ll, j.ll_pitch, j.ll_dtype, j.hl, j.lh, j.hh,
                                          j.band_pitch, j.band_dtype, wavelet, tile);
                }
                b.tile_start[b.n + 1] = b.tile_start[b.n] + b.p[b.n].tiles_x * b.p[b.n].tiles_y;
                ++b.n;
                done[i] = true;
            }
            if (b.n > 0 && (b.n == kBatchMax || i == n)) {
                hipError_t e;
                if constexpr (INV)
                    e = inv_batch_table(key.band_dt)[wavelet][scheme][key.ll_dt == DWT2_F32]
                                       [key.full_dt == DWT2_F32][tile](b, s);
                else
                    e = fwd_batch_table(key.band_dt)[wavelet][scheme][key.full_dt == DWT2_F32]
                                       [key.ll_dt == DWT2_F32][tile](b, s);
                if (e != hipSuccess) st = hip_fail(e);
                b.n = 0;
            }
        }
    }
    return st;
}

// Head level batches: jobs[2i] is the finer level j and jobs[2i+1] the
// coarser level j+1 of pair i, each a level job as in the level batches. The
// band between them (the finer job's ll, the coarser job's full) stays in LDS
// in FP32 and is not accessed, so it must be that one FP32 buffer.
struct HeadKey {
    int band_dt, a_f32, b_f32;
    bool operator==(const HeadKey &o) const {
        return band_dt == o.band_dt && a_f32 == o.a_f32 && b_f32 == o.b_f32;
    }
};

const FwdHeadBatchTable &fwd_head_batch_table(int dt) {
    return dt == DWT2_F32 ? kFwdHeadBatchF32 : dt == DWT2_F16 ? kFwdHeadBatchF16 : kFwdHeadBatchBF16;
}
const InvHeadBatchTable &inv_head_batch_table(int dt) {
    return dt == DWT2_F32 ? kInvHeadBatchF32 : dt == DWT2_F16 ? kInvHeadBatchF16 : kInvHeadBatchBF16;
}

template <bool INV>
int head_batch(const dwt2_level_job *jobs, int32_t n, int32_t wavelet, int32_t scheme,
               hipStream_t stream) {
    if (n < 0 || (n > 0 && !jobs)) return DWT2_ERR_INVALID_ARG;
    if (!valid_wavelet(wavelet) || !valid_scheme(scheme) || lds_scheme(scheme))
        return DWT2_ERR_UNSUPPORTED;
    for (int i = 0; i < 2 * n; ++i) {
        const dwt2_level_job &j = jobs[i];
        const int st = check_level_args(j.full, j.full_pitch, j.full_dtype, j.width, j.height,
                                        j.ll, j.ll_pitch, j.ll_dtype, j.hl, j.lh, j.hh,
                                        j.band_pitch, j.band_dtype, wavelet, scheme, 0);
        if (st) return st;
    }
    for (int i = 0; i < n; ++i) {
        const dwt2_level_job &f = jobs[2 * i], &c = jobs[2 * i + 1];
        if (c.width != f.width / 2 || c.height != f.height / 2 || f.ll != c.full ||
            f.ll_pitch != c.full_pitch || f.ll_dtype != DWT2_F32 || c.full_dtype != DWT2_F32 ||
            f.band_dtype != c.band_dtype)
            return DWT2_ERR_INVALID_ARG;
    }
    {   // the buffers each pair touches: the forward reads the finer `full` and
        // writes both levels' bands and the coarser ll; the inverse the reverse
        std::vector<Access> v;
        v.reserve(8 * (size_t)(n > 0 ? n : 0));
        for (int i = 0; i < n; ++i) {
            const dwt2_level_job &f = jobs[2 * i], &c = jobs[2 * i + 1];
            const int fx = f.width / 2, fy = f.height / 2, cx = c.width / 2, cy = c.height / 2;
            v.push_back({region_of(f.full, f.height, f.width, f.full_pitch, f.full_dtype), 2 * i,
                         INV});
            v.push_back({region_of(f.hl, fy, fx, f.band_pitch, f.band_dtype), 2 * i, !INV});
            v.push_back({region_of(f.lh, fy, fx, f.band_pitch, f.band_dtype), 2 * i, !INV});
            v.push_back({region_of(f.hh, fy, fx, f.band_pitch, f.band_dtype), 2 * i, !INV});
            v.push_back({region_of(c.ll, cy, cx, c.ll_pitch, c.ll_dtype), 2 * i + 1, !INV});
            v.push_back({region_of(c.hl, cy, cx, c.band_pitch, c.band_dtype), 2 * i + 1, !INV});
            v.push_back({region_of(c.lh, cy, cx, c.band_pitch, c.band_dtype), 2 * i + 1, !INV});
            v.push_back({region_of(c.hh, cy, cx, c.band_pitch, c.band_dtype), 2 * i + 1, !INV});
        }
        if (cross_conflict(v)) return DWT2_ERR_INVALID_ARG;
    }
    std::vector<HeadKey> keys(n > 0 ? n : 1);
    std::vector<char> done(n > 0 ? n : 1);
    for (int i = 0; i < n; ++i) {
        const dwt2_level_job &f = jobs[2 * i], &c = jobs[2 * i + 1];
        keys[i] = INV ? HeadKey{f.band_dtype, c.ll_dtype == DWT2_F32, f.full_dtype == DWT2_F32}
                      : HeadKey{f.band_dtype, f.full_dtype == DWT2_F32, c.ll_dtype == DWT2_F32};
        done[i] = false;
    }
    int st = DWT2_OK;
    for (int g = 0; g < n && st == DWT2_OK; ++g) {   // one group per distinct key
        if (done[g]) continue;
        const HeadKey key = keys[g];
        typename std::conditional<INV, InvHeadBatch, FwdHeadBatch>::type b;
        b.n = 0;
        b.tile_start[0] = 0;
        for (int i = g; i <= n && st == DWT2_OK; ++i) {
            if (i < n && !done[i] && keys[i] == key) {
                const dwt2_level_job &f = jobs[2 * i], &c = jobs[2 * i + 1];
                int tiles;
                if constexpr (INV) {
                    InvHead &hd = b.h[b.n];
                    hd.l2 = inv_params(c.ll, c.ll_pitch, c.ll_dtype, c.hl, c.lh, c.hh,
                                       c.band_pitch, c.band_dtype, c.full, c.full_pitch,
                                       c.full_dtype, c.width, c.height, wavelet, 0);
                    hd.l1 = inv_params(f.ll, f.ll_pitch, f.ll_dtype, f.hl, f.lh, f.hh,
                                       f.band_pitch, f.band_dtype, f.full, f.full_pitch,
                                       f.full_dtype, f.width, f.height, wavelet, 0);
                    hd.tiles_x = (hd.l1.nqx + FwdHeadGeom::IOX1 - 1) / FwdHeadGeom::IOX1;
                    hd.tiles_y = (hd.l1.nqy + FwdHeadGeom::IOY1 - 1) / FwdHeadGeom::IOY1;
                    tiles = hd.tiles_x * hd.tiles_y;
                } else {
                    FwdHead &hd = b.h[b.n];
                    hd.l1 = fwd_params(f.full, f.full_pitch, f.full_dtype, f.width, f.height,
                                       f.ll, f.ll_pitch, f.ll_dtype, f.hl, f.lh, f.hh,
                                       f.band_pitch, f.band_dtype, wavelet, 0);
                    hd.l2 = fwd_params(c.full, c.full_pitch, c.full_dtype, c.width, c.height,
                                       c.ll, c.ll_pitch, c.ll_dtype, c.hl, c.lh, c.hh,
                                       c.band_pitch, c.band_dtype, wavelet, 0);
                    hd.tiles_x = (hd.l2.nqx + FwdHeadGeom::FOX2 - 1) / FwdHeadGeom::FOX2;
                    hd.tiles_y = (hd.l2.nqy + FwdHeadGeom::FOY2 - 1) / FwdHeadGeom::FOY2;
                    tiles = hd.tiles_x * hd.tiles_y;
                }
                if ((int64_t)b.tile_start[b.n] + tiles > (int64_t)INT32_MAX) {
                    st = DWT2_ERR_INVALID_ARG;
                    break;
                }
                b.tile_start[b.n + 1] = b.tile_start[b.n] + tiles;
                ++b.n;
                done[i] = true;
            }
            if (b.n > 0 && (b.n == kHeadBatchMax || i == n)) {
                hipError_t e;
                if constexpr (INV)
                    e = inv_head_batch_table(key.band_dt)[wavelet][scheme][key.a_f32][key.b_f32](
                        b, stream);
                else
                    e = fwd_head_batch_table(key.band_dt)[wavelet][scheme][key.a_f32][key.b_f32](
                        b, stream);
                if (e != hipSuccess) st = hip_fail(e);
                b.n = 0;
            }
        }
    }
    return st;
}

}  // namespace

extern "C" {

int dwt2_forward_level_batch(const dwt2_level_job *jobs, int32_t n, dwt2_wavelet wavelet,
                             dwt2_scheme scheme, const int32_t *class_tiles, hipStream_t stream) {
    return level_batch<false>(jobs, n, wavelet, scheme, class_tiles, stream);
}

int dwt2_inverse_level_batch(const dwt2_level_job *jobs, int32_t n, dwt2_wavelet wavelet,
                             dwt2_scheme scheme, const int32_t *class_tiles, hipStream_t stream) {
    return level_batch<true>(jobs, n, wavelet, scheme, class_tiles, stream);
}

int dwt2_forward_head_batch(const dwt2_level_job *jobs, int32_t n, dwt2_wavelet wavelet,
                            dwt2_scheme scheme, hipStream_t stream) {
    return head_batch<false>(jobs, n, wavelet, scheme, stream);
}

int dwt2_inverse_head_batch(const dwt2_level_job *jobs, int32_t n, dwt2_wavelet wavelet,
                            dwt2_scheme scheme, hipStream_t stream) {
    return head_batch<true>(jobs, n, wavelet, scheme, stream);
}

}  // extern "C"

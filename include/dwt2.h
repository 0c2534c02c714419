/*
 * dwt2.h - 2-D discrete wavelet transform on AMD Instinct MI355X (gfx950).
 *
 * The library computes the single-scale and multi-level 2-D CDF 9/7 and
 * CDF 5/3 forward and inverse DWT with the non-separable lifting scheme of
 * Barina, Kula, Matysek and Zemcik, "Accelerating Discrete Wavelet
 * Transforms on GPUs": each horizontal and vertical predict (update) pair of
 * the separable lifting scheme is merged into one spatial step T_P (S_U) on a
 * 2x2 polyphase quad (Sec. 3), with the constant parts P0, U0 split off and
 * applied to the unit's own quad without a barrier (Sec. 3, "optimization").
 * The separable lifting scheme (Sec. 2) is available as a baseline.
 *
 * Problem statement (Sec. 2): the 2-D transform splits the image into a
 * quadruple of coefficient bands per level. Conventions, where the paper is
 * silent:
 *   - pixel (0,0) is an even/even sample; quad (i,j) holds
 *     a = x[2j][2i] -> LL, b = x[2j][2i+1] -> HL, c = x[2j+1][2i] -> LH,
 *     d = x[2j+1][2i+1] -> HH;
 *   - boundary: whole-sample symmetric extension (x[-k] = x[k],
 *     x[N-1+k] = x[N-1-k]), periodic with period 2N-2, so any N >= 2 works;
 *   - scaling: unit gain (low-pass DC gain 1, high-pass Nyquist gain 1);
 *   - multi-level: dyadic recursion on LL, written in the Mallat layout
 *     inside one W x H coefficient buffer: after level j, LL_j is the
 *     (W/2^j) x (H/2^j) top-left block, HL_j is to its right, LH_j below it
 *     and HH_j diagonally below-right.
 *
 * Arithmetic is FP32. Storage of the image and the coefficients may be FP32,
 * FP16 or BF16; intermediate low-low bands between levels stay FP32 in the
 * caller's workspace.
 *
 * Memory and threading
 *   - All buffer pointers are DEVICE pointers on the current HIP device.
 *   - The caller owns every buffer. The library allocates and frees no device
 *     memory (the batch entry points use host-side scratch for their launch
 *     descriptors), keeps no global mutable state except a thread-local last
 *     HIP error and per-process caches of device properties (compute-unit
 *     and occupancy counts), and never synchronises: every call enqueues
 *     work on `stream` (a hipStream_t; NULL = the default stream) and
 *     returns.
 *   - Argument errors are detected before anything is enqueued. Faults during
 *     execution surface at the caller's next synchronisation of `stream`.
 *   - Calls on different streams that use disjoint buffers may overlap.
 */
#ifndef DWT2_H
#define DWT2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* HIP's stream and event handles (the same declarations as the HIP runtime's
 * own headers, so this header needs no HIP include; C11 or C++). */
typedef struct ihipStream_t *hipStream_t;
typedef struct ihipEvent_t *hipEvent_t;

/* Status codes returned by every entry point that can fail. */
typedef enum {
    DWT2_OK = 0,
    DWT2_ERR_INVALID_ARG = -1,  /* null pointer, bad size, overlap, mismatch */
    DWT2_ERR_UNSUPPORTED = -2,  /* unknown enum value or tile id */
    DWT2_ERR_WORKSPACE = -3,    /* workspace smaller than required */
    DWT2_ERR_HIP = -4           /* a HIP launch failed; see dwt2_last_hip_error */
} dwt2_status;

/* The two wavelets the paper evaluates (Sec. 4): CDF 9/7 (two lifting pairs)
 * and CDF 5/3 (one pair). */
typedef enum { DWT2_CDF97 = 0, DWT2_CDF53 = 1 } dwt2_wavelet;

/* Only whole-sample symmetric extension is defined. */
typedef enum { DWT2_EXT_WHOLE_SAMPLE_SYMMETRIC = 0 } dwt2_boundary;

/* Storage type of a buffer; arithmetic is always FP32. */
typedef enum { DWT2_F32 = 0, DWT2_F16 = 1, DWT2_BF16 = 2 } dwt2_dtype;

/* Lifting scheme.
 *   NONSEPARABLE: the spatial steps T_P and S_U of Sec. 3, two per lifting
 *     pair, with the constant parts P0 and U0 applied without a barrier.
 *   SEPARABLE: the horizontal and vertical steps T_P^H, T_P^V, S_U^H, S_U^V
 *     of Sec. 2, four per lifting pair.
 * Both move horizontal neighbours between lanes of a wavefront (no barrier)
 * and vertical ones through LDS with one workgroup barrier per step.
 *   NONSEPARABLE_LDS, SEPARABLE_LDS: the same steps with every neighbour
 *     exchange through LDS and a barrier, the setting of Sec. 3 in which
 *     every step synchronises. They measure the barrier count and support
 *     FP32 single-image calls only (no fused levels, no batches). */
typedef enum {
    DWT2_NONSEPARABLE = 0,
    DWT2_SEPARABLE = 1,
    DWT2_NONSEPARABLE_LDS = 2,
    DWT2_SEPARABLE_LDS = 3
} dwt2_scheme;

/* A 2-D buffer: `height` rows of `width` elements, row starts `pitch`
 * elements apart (pitch >= width), elements of type `dtype`. */
typedef struct {
    int32_t width;
    int32_t height;
    int64_t pitch;
    dwt2_dtype dtype;
} dwt2_desc;

/* Bytes of workspace that an L-level transform of a width x height image of
 * storage type `dtype` needs. The low-low band between two levels is kept in
 * FP32 whatever the storage type (intermediate rounding to 16 bits would
 * double the error of the deep levels), in two ping-pong buffers:
 * (W/2)(H/2) floats for L >= 2, plus (W/4)(H/4) for L >= 3. Returns 0 for
 * L = 1 and for invalid sizes or dtypes. */
size_t dwt2_workspace_bytes(int32_t width, int32_t height, int32_t levels, dwt2_dtype dtype);

/* Forward L-level 2-D DWT (Sec. 2, problem statement: each level splits its
 * input into the LL, HL, LH and HH bands; the lifting steps are those of
 * Sec. 3 for NONSEPARABLE and Sec. 2 for SEPARABLE).
 *   src    : the image, described by *src_d (read only, device memory).
 *   coef   : the Mallat-layout coefficients, described by *coef_d; same
 *            width, height and dtype as the image. Must not overlap src.
 *   wavelet, boundary, scheme : enum values above.
 *   levels : 1..16; width and height must be divisible by 2^levels.
 *   workspace, workspace_bytes : device scratch of at least
 *            dwt2_workspace_bytes(width, height, levels, dtype) bytes; may be
 *            NULL when that is 0. Must not overlap src or coef.
 *   stream : the HIP stream to enqueue on (NULL: the default stream).
 * The library picks each level's tile configuration and fuses the trailing
 * levels whose input has at most DWT2_TAIL_AUTO_PIXELS pixels into one
 * launch (dwt2_fused_levels). Returns a dwt2_status; on an error nothing is
 * enqueued. */
int dwt2_forward(const void *src, const dwt2_desc *src_d, void *coef, const dwt2_desc *coef_d,
                 dwt2_wavelet wavelet, int32_t levels, dwt2_boundary boundary,
                 dwt2_scheme scheme, void *workspace, size_t workspace_bytes,
                 hipStream_t stream);

/* Inverse L-level 2-D DWT: coef (Mallat layout, read only) -> dst. The exact
 * reverse of dwt2_forward: per level, the lifting steps undone in reverse
 * order with negated coefficients (Sec. 2 and 3 define the forward steps; the
 * paper does not spell out the inverse). Arguments as for dwt2_forward. When
 * dst holds 32 MiB to 256 MiB, the finest level writes it with non-temporal
 * stores (the values are the same; the lines are not kept in the GPU
 * caches). */
int dwt2_inverse(const void *coef, const dwt2_desc *coef_d, void *dst, const dwt2_desc *dst_d,
                 dwt2_wavelet wavelet, int32_t levels, dwt2_boundary boundary,
                 dwt2_scheme scheme, void *workspace, size_t workspace_bytes,
                 hipStream_t stream);

/* ---- a forward call that allocates nothing --------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * transform as dwt2_forward, with the workspace taken from a library-owned
 * array of DWT2_STATIC_WORKSPACE_BYTES bytes in device memory. Each GPU the
 * library runs on holds its own copy of that array from the library's load
 * until the process ends. The call allocates and frees nothing (on its first
 * call on a device it looks up the array's address there).
 *   Arguments, results and errors as for dwt2_forward, plus
 *   DWT2_ERR_WORKSPACE when dwt2_workspace_bytes(width, height, levels,
 *   dtype) exceeds DWT2_STATIC_WORKSPACE_BYTES (e.g. 16384^2 with L >= 2).
 *   Every call on one GPU shares that GPU's array: calls that may overlap in
 *   time on one GPU (different streams, or host threads enqueueing
 *   concurrently) race on it and give wrong results. Each call overwrites
 *   every byte of the array it reads, so no state carries over between
 *   calls. */
#define DWT2_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
int dwt2_forward_no_alloc(const void *src, const dwt2_desc *src_d, void *coef,
                          const dwt2_desc *coef_d, dwt2_wavelet wavelet, int32_t levels,
                          dwt2_boundary boundary, dwt2_scheme scheme, hipStream_t stream);

/* Tile id that marks a level as part of the fused tail launch. */
#define DWT2_TILE_TAIL (-2)
/* Tile id that marks levels 1 and 2 as one fused launch (the "head"). */
#define DWT2_TILE_HEAD (-3)
#define DWT2_TAIL_MAX 3
#define DWT2_TAIL_AUTO_PIXELS (1 << 22)

/* Number of trailing levels that dwt2_forward and dwt2_inverse fuse into
 * one launch (0 when none; never 1). Multi-scale fusion is the paper's
 * outlook (Sec. 5). Returns DWT2_ERR_INVALID_ARG for sizes the transform
 * rejects. */
int dwt2_fused_levels(int32_t width, int32_t height, int32_t levels);

/* Number of leading levels (0 or 2) that dwt2_forward and dwt2_inverse run
 * as one launch: levels 1 and 2 are fused, their low-low band kept on chip,
 * whenever there are two or more levels and the fused tail starts at level 3
 * or later (Sec. 5 names fusing several consecutive steps as a way to cut
 * memory traffic). Returns DWT2_ERR_INVALID_ARG for sizes the transform
 * rejects. */
int dwt2_head_levels(int32_t width, int32_t height, int32_t levels);

/* dwt2_forward (dwt2_inverse) with two tuning and timing hooks; results are
 * identical to the plain calls.
 *   tiles : NULL to let the library choose, else `levels` tile ids
 *           (0 <= id < dwt2_tile_config_count()), one per level, or
 *           DWT2_TILE_TAIL for each of the last 2..DWT2_TAIL_MAX levels:
 *           those run fused in one launch (one workgroup computes every
 *           fused level for its block; intermediate low-low bands stay in
 *           LDS), or DWT2_TILE_HEAD for both levels 1 and 2 (fused the same
 *           way; the tail must then start at level 3 or later). Entry j
 *           belongs to level j+1.
 *   level_events : NULL, or 2*levels events; events [2j] and [2j+1] are
 *           recorded on `stream` before and after the launch of level j+1.
 *           For fused tail levels the first fused level's pair brackets the
 *           fused launch and the other fused levels' pairs are both recorded
 *           after it; a fused head is bracketed by level 1's pair, and level
 *           2's pair is recorded after it. */
int dwt2_forward_ex(const void *src, const dwt2_desc *src_d, void *coef, const dwt2_desc *coef_d,
                    dwt2_wavelet wavelet, int32_t levels, dwt2_boundary boundary,
                    dwt2_scheme scheme, void *workspace, size_t workspace_bytes,
                    const int32_t *tiles, const hipEvent_t *level_events, hipStream_t stream);
int dwt2_inverse_ex(const void *coef, const dwt2_desc *coef_d, void *dst, const dwt2_desc *dst_d,
                    dwt2_wavelet wavelet, int32_t levels, dwt2_boundary boundary,
                    dwt2_scheme scheme, void *workspace, size_t workspace_bytes,
                    const int32_t *tiles, const hipEvent_t *level_events, hipStream_t stream);

/* One forward level, one kernel launch (the building block of dwt2_forward;
 * Sec. 2: one level of the 2-D transform).
 *   in    : level input, width x height (both even), pitch in_pitch, in_dtype.
 *   ll    : (width/2) x (height/2) low-low output, pitch ll_pitch, ll_dtype.
 *   hl, lh, hh : the three detail bands, each (width/2) x (height/2), sharing
 *           pitch band_pitch and band_dtype.
 *   tile  : a tile configuration id, or < 0 to let the library choose.
 * The input and LL are FP32 or the band type. No two of the five buffers may
 * overlap. */
int dwt2_forward_level(const void *in, int64_t in_pitch, dwt2_dtype in_dtype,
                       int32_t width, int32_t height,
                       void *ll, int64_t ll_pitch, dwt2_dtype ll_dtype,
                       void *hl, void *lh, void *hh, int64_t band_pitch,
                       dwt2_dtype band_dtype,
                       dwt2_wavelet wavelet, dwt2_scheme scheme, int32_t tile,
                       hipStream_t stream);

/* One inverse level: four bands of (width/2) x (height/2) -> out
 * (width x height). Arguments as for dwt2_forward_level. */
int dwt2_inverse_level(const void *ll, int64_t ll_pitch, dwt2_dtype ll_dtype,
                       const void *hl, const void *lh, const void *hh,
                       int64_t band_pitch, dwt2_dtype band_dtype,
                       void *out, int64_t out_pitch, dwt2_dtype out_dtype,
                       int32_t width, int32_t height,
                       dwt2_wavelet wavelet, dwt2_scheme scheme, int32_t tile,
                       hipStream_t stream);

/* Kernel configurations ("tiles") compiled into the library: a workgroup of
 * `waves` wavefronts stacked vertically; each lane owns `quads_per_lane`
 * consecutive quads of a row and `rows` quad rows. Of the
 * (64*quads_per_lane) x (waves*rows) quad window the centre out_x x out_y
 * quads are written; the rest is the lifting halo. Returns DWT2_OK or
 * DWT2_ERR_UNSUPPORTED; null out-pointers are skipped. */
int dwt2_tile_config_count(void);
int dwt2_tile_config_info(int32_t tile, dwt2_wavelet wavelet, int32_t *quads_per_lane,
                          int32_t *rows, int32_t *waves, int32_t *out_x, int32_t *out_y);

/* The tile id the library picks for one level whose full-resolution side
 * (the forward's input, the inverse's output) is width x height pixels of
 * `dtype` storage. */
int dwt2_default_tile(int32_t width, int32_t height, dwt2_wavelet wavelet,
                      dwt2_scheme scheme, dwt2_dtype dtype);

/* ---- batches of images ---------------------------------------------------
 * Many images of one storage type, wavelet and level count, planned once and
 * run as few launches: each level is one launch over every image whose size
 * class uses the same tile configuration (one launch per level with the
 * default configurations of FP32 storage), and with DWT2_PLAN_HEAD levels 1
 * and 2 are one launch over every image (fusing consecutive levels, Sec. 5,
 * as the default chain of dwt2_forward does). Not a topic of the paper, which
 * transforms one image at a time: batching serves many uneven images.
 *
 * dwt2_batch_plan writes a plan (a byte image in host memory, of
 * dwt2_batch_plan_bytes bytes): per launch, a tile -> image map and every
 * image's level parameters, with the images' device pointers. The caller
 * copies it byte for byte into device memory (e.g. hipMemcpy) and passes both
 * copies to dwt2_batch_run, which reads the launch shapes from the host copy
 * while the kernels read the device copy. The launches hold nothing but
 * pointers into the device copy, so a captured HIP graph of dwt2_batch_run
 * replays the whole batch. Both copies must stay unchanged while launches
 * that use them may run, and the device copy must equal the host copy (the
 * library cannot check device memory; a differing copy gives wrong results or
 * faults). */
typedef struct {
    const void *src;        /* forward: image; inverse: Mallat coefficients */
    int64_t src_pitch;      /* elements */
    void *dst;              /* forward: Mallat coefficients; inverse: image */
    int64_t dst_pitch;      /* elements */
    void *workspace;        /* scratch of dwt2_workspace_bytes(width, height, levels, dtype) */
    size_t workspace_bytes;
    int32_t width, height;  /* divisible by 2^levels */
} dwt2_image;

#define DWT2_SIZE_CLASSES 4

/* Size class of one level whose input is width x height pixels:
 * 0: <= 128^2, 1: <= 512^2, 2: <= 2048^2, 3: larger. DWT2_ERR_INVALID_ARG
 * for sizes below 2. */
int dwt2_size_class(int32_t width, int32_t height);

/* Plan flag: with two or more levels, levels 1 and 2 of every image run as
 * one launch of the fused head (the level-1 low-low band stays on chip, as in
 * dwt2_forward's default chain), planned at level 1; the tile configurations
 * then serve levels 3 and beyond. No effect with one level. */
#define DWT2_PLAN_HEAD 1

/* Bytes of the plan of an L-level forward (inverse = 0) or inverse
 * (inverse = 1) transform of images[0..n), n >= 1, in *bytes. Each image is
 * checked as by dwt2_forward (dwt2_inverse); src and dst of one image must
 * not overlap, and no image may write a buffer another image reads or writes
 * (images may share a source). class_tiles: NULL for the library's choice,
 * else DWT2_SIZE_CLASSES tile configuration ids, the one used for the levels
 * of each size class. flags: 0 or DWT2_PLAN_HEAD (others:
 * DWT2_ERR_UNSUPPORTED). Returns a dwt2_status. */
int dwt2_batch_plan_bytes(const dwt2_image *images, int32_t n, dwt2_dtype dtype,
                          dwt2_wavelet wavelet, int32_t levels, int32_t inverse,
                          dwt2_boundary boundary, const int32_t *class_tiles, int32_t flags,
                          size_t *bytes);

/* Writes the plan into plan[0..plan_bytes) (host memory): DWT2_ERR_WORKSPACE
 * if plan_bytes is too small, else as dwt2_batch_plan_bytes. */
int dwt2_batch_plan(const dwt2_image *images, int32_t n, dwt2_dtype dtype, dwt2_wavelet wavelet,
                    int32_t levels, int32_t inverse, dwt2_boundary boundary,
                    const int32_t *class_tiles, int32_t flags, void *plan, size_t plan_bytes);

/* Number of launches of a plan, in total and (per_level: NULL or `levels`
 * entries) per level, index j for level j+1; a head launch counts at level
 * 1, and level 2 then has none. */
int dwt2_batch_launches(const void *plan, size_t plan_bytes, int32_t *launches,
                        int32_t *per_level);

/* Grid of dwt2_batch_run: one workgroup per tile (flags 0), or
 * DWT2_BATCH_PERSISTENT: at most as many workgroups as fit on the device at
 * once, each walking several tiles. Results are identical. */
#define DWT2_BATCH_PERSISTENT 1

/* Enqueues the planned transform on `stream`: plan (host memory, plan_bytes
 * bytes as written by dwt2_batch_plan) and plan_device (its device copy).
 * Launches run level after level in stream order. Returns a dwt2_status;
 * nothing is enqueued if the host plan is malformed or an argument invalid. */
int dwt2_batch_run(const void *plan, size_t plan_bytes, const void *plan_device,
                   dwt2_scheme scheme, int32_t flags, hipStream_t stream);

/* One level of one image, as given to dwt2_forward_level (forward) or
 * dwt2_inverse_level (inverse): `full` is the width x height buffer (the
 * level input of a forward, the level output of an inverse), ll the
 * (width/2) x (height/2) low band, hl/lh/hh the detail bands sharing
 * band_pitch. */
typedef struct {
    void *full;  int64_t full_pitch; dwt2_dtype full_dtype;
    void *ll;    int64_t ll_pitch;   dwt2_dtype ll_dtype;
    void *hl, *lh, *hh; int64_t band_pitch; dwt2_dtype band_dtype;
    int32_t width, height;
} dwt2_level_job;

/* Many independent single levels in few launches: jobs are grouped by size
 * class and storage types, and each group runs as batched launches of up to
 * 36 jobs. Forward jobs read `full` and write ll/hl/lh/hh; inverse jobs read
 * ll/hl/lh/hh and write `full`. Every job is checked as by the single-level
 * entry points; no job may write a buffer another job of the call reads or
 * writes. For continuous batching: each call advances every active request
 * by one level. Returns a dwt2_status; nothing is enqueued on an error. */
int dwt2_forward_level_batch(const dwt2_level_job *jobs, int32_t n,
                             dwt2_wavelet wavelet, dwt2_scheme scheme,
                             const int32_t *class_tiles, hipStream_t stream);
int dwt2_inverse_level_batch(const dwt2_level_job *jobs, int32_t n,
                             dwt2_wavelet wavelet, dwt2_scheme scheme,
                             const int32_t *class_tiles, hipStream_t stream);

/* Two consecutive levels j and j+1 of many independent images in few
 * launches of the fused head (levels fused as Sec. 5 suggests; the same
 * arithmetic as two level jobs, bit for bit): n pairs, jobs[2i] the finer
 * level j and jobs[2i+1] the coarser level j+1 of pair i, each a level job as
 * above. The forward reads jobs[2i].full and writes both levels' bands and
 * jobs[2i+1].ll; the inverse reads jobs[2i+1].ll and both levels' bands and
 * writes jobs[2i].full. The band between the two levels stays on chip in
 * FP32 and is not accessed: jobs[2i].ll and jobs[2i+1].full must be the same
 * FP32 buffer (equal pointer and pitch), jobs[2i+1] must be half the size of
 * jobs[2i] in each dimension, and both levels share one band storage type;
 * else DWT2_ERR_INVALID_ARG. Pairs are grouped by storage types into launches
 * of up to 18. Every job is checked as by the level batches, and no pair may
 * write a buffer another pair (or the pair's other level) reads or writes.
 * Returns a dwt2_status; nothing is enqueued on an argument error. */
int dwt2_forward_head_batch(const dwt2_level_job *jobs, int32_t n, dwt2_wavelet wavelet,
                            dwt2_scheme scheme, hipStream_t stream);
int dwt2_inverse_head_batch(const dwt2_level_job *jobs, int32_t n, dwt2_wavelet wavelet,
                            dwt2_scheme scheme, hipStream_t stream);

/* Human-readable text of a status code (static storage). */
const char *dwt2_status_string(int status);

/* hipError_t behind the most recent DWT2_ERR_HIP on this thread. */
int dwt2_last_hip_error(void);

/* Library ABI version (major*100 + minor). */
int dwt2_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DWT2_H */

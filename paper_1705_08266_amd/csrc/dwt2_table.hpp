// Launch table: one launcher per (wavelet, scheme, storage types, config).
#pragma once

#include <array>
#include <utility>

#include "dwt2_kernels.hpp"
#include "dwt2_head.hpp"
#include "dwt2_tail.hpp"

namespace dwt2 {

// A compiled 2-D tile configuration: a workgroup of `waves` wavefronts stacked
// vertically, each lane holding `qpl` consecutive quads of a row and `rows`
// quad rows; the window is (64 qpl) x (waves rows) quads, one per workgroup.
struct TileCfg {
    int qpl;
    int rows;
    int waves;
};

constexpr TileCfg kTiles[] = {
    {2, 2, 8},   // 0: 128 x 16 window, 512 threads (FP32 default)
    {2, 4, 4},   // 1: 128 x 16, 256 threads (16-bit default above 2048^2)
    {2, 3, 8},   // 2: 128 x 24, 512 threads
    {2, 8, 1},   // 3: 128 x 8, one wavefront (no workgroup barriers)
};
constexpr int kNumTiles = (int)(sizeof(kTiles) / sizeof(kTiles[0]));

// A launcher takes the level parameters (grid fields filled in by the host
// planner) and launches its kernel.
using FwdLauncher = hipError_t (*)(const FwdParams &, hipStream_t);
using InvLauncher = hipError_t (*)(const InvParams &, hipStream_t);

template <int WV, int SCH, int T, typename TIN, typename TLL, typename TB>
hipError_t launch_fwd(const FwdParams &p, hipStream_t s) {
    constexpr TileCfg c = kTiles[T];
    hipLaunchKernelGGL((fwd_level_kernel<WV, SCH, c.qpl, c.rows, c.waves, TIN, TLL, TB>),
                       dim3(p.tiles_x * p.tiles_y), dim3(64 * c.waves), 0, s, p);
    return hipGetLastError();
}

template <int WV, int SCH, int T, typename TLL, typename TB, typename TOUT>
hipError_t launch_inv(const InvParams &p, hipStream_t s) {
    constexpr TileCfg c = kTiles[T];
    hipLaunchKernelGGL((inv_level_kernel<WV, SCH, c.qpl, c.rows, c.waves, TLL, TB, TOUT>),
                       dim3(p.tiles_x * p.tiles_y), dim3(64 * c.waves), 0, s, p);
    return hipGetLastError();
}

// Level jobs with parameters in the kernel arguments: one workgroup per tile.
using FwdBatchLauncher = hipError_t (*)(const FwdBatch &, hipStream_t);
using InvBatchLauncher = hipError_t (*)(const InvBatch &, hipStream_t);

template <int WV, int SCH, int T, typename TIN, typename TLL, typename TB>
hipError_t launch_fwd_batch(const FwdBatch &b, hipStream_t s) {
    constexpr TileCfg c = kTiles[T];
    const int total = b.tile_start[b.n];
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL((fwd_batch_kernel<WV, SCH, c.qpl, c.rows, c.waves, TIN, TLL, TB>),
                       dim3(total), dim3(64 * c.waves), 0, s, b);
    return hipGetLastError();
}

template <int WV, int SCH, int T, typename TLL, typename TB, typename TOUT>
hipError_t launch_inv_batch(const InvBatch &b, hipStream_t s) {
    constexpr TileCfg c = kTiles[T];
    const int total = b.tile_start[b.n];
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL((inv_batch_kernel<WV, SCH, c.qpl, c.rows, c.waves, TLL, TB, TOUT>),
                       dim3(total), dim3(64 * c.waves), 0, s, b);
    return hipGetLastError();
}

// Workgroups of `kernel` that fit on the current device at once.
int resident_blocks(const void *kernel, int block_threads);

// Planned batches: one launch over a device table. `persistent` caps the grid
// at the workgroups that fit on the device at once (each then walks several
// tiles); otherwise the grid has one workgroup per tile.
using FwdTableLauncher = hipError_t (*)(const TableLaunch<FwdParams> &, bool, hipStream_t);
using InvTableLauncher = hipError_t (*)(const TableLaunch<InvParams> &, bool, hipStream_t);

template <int WV, int SCH, int T, typename TIN, typename TLL, typename TB>
hipError_t launch_fwd_table(const TableLaunch<FwdParams> &tl, bool persistent, hipStream_t s) {
    constexpr TileCfg c = kTiles[T];
    const auto k = fwd_table_kernel<WV, SCH, c.qpl, c.rows, c.waves, TIN, TLL, TB>;
    int grid = tl.total;
    if (persistent) {
        static const int resident = resident_blocks((const void *)k, 64 * c.waves);
        grid = grid < resident ? grid : resident;
    }
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k, dim3(grid), dim3(64 * c.waves), 0, s, tl);
    return hipGetLastError();
}

template <int WV, int SCH, int T, typename TLL, typename TB, typename TOUT>
hipError_t launch_inv_table(const TableLaunch<InvParams> &tl, bool persistent, hipStream_t s) {
    constexpr TileCfg c = kTiles[T];
    const auto k = inv_table_kernel<WV, SCH, c.qpl, c.rows, c.waves, TLL, TB, TOUT>;
    int grid = tl.total;
    if (persistent) {
        static const int resident = resident_blocks((const void *)k, 64 * c.waves);
        grid = grid < resident ? grid : resident;
    }
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k, dim3(grid), dim3(64 * c.waves), 0, s, tl);
    return hipGetLastError();
}

template <int WV, int SCH, typename TIN, typename TLL, typename TB, int... I>
constexpr std::array<FwdTableLauncher, kNumTiles> fwd_table_tiles(std::integer_sequence<int, I...>) {
    return {&launch_fwd_table<WV, SCH, I, TIN, TLL, TB>...};
}
template <int WV, int SCH, typename TLL, typename TB, typename TOUT, int... I>
constexpr std::array<InvTableLauncher, kNumTiles> inv_table_tiles(std::integer_sequence<int, I...>) {
    return {&launch_inv_table<WV, SCH, I, TLL, TB, TOUT>...};
}

// Index [wavelet][scheme][first operand is FP32][second operand is FP32]
// [config], as for the single-level tables.
using FwdTableTable = std::array<std::array<std::array<std::array<std::array<FwdTableLauncher, kNumTiles>, 2>, 2>, 2>, 2>;
using InvTableTable = std::array<std::array<std::array<std::array<std::array<InvTableLauncher, kNumTiles>, 2>, 2>, 2>, 2>;

template <typename T, int WV, int SCH>
constexpr std::array<std::array<std::array<FwdTableLauncher, kNumTiles>, 2>, 2> fwd_table_types() {
    using S = std::make_integer_sequence<int, kNumTiles>;
    return {{{fwd_table_tiles<WV, SCH, T, T, T>(S{}), fwd_table_tiles<WV, SCH, T, float, T>(S{})},
             {fwd_table_tiles<WV, SCH, float, T, T>(S{}), fwd_table_tiles<WV, SCH, float, float, T>(S{})}}};
}
template <typename T, int WV, int SCH>
constexpr std::array<std::array<std::array<InvTableLauncher, kNumTiles>, 2>, 2> inv_table_types() {
    using S = std::make_integer_sequence<int, kNumTiles>;
    return {{{inv_table_tiles<WV, SCH, T, T, T>(S{}), inv_table_tiles<WV, SCH, T, T, float>(S{})},
             {inv_table_tiles<WV, SCH, float, T, T>(S{}), inv_table_tiles<WV, SCH, float, T, float>(S{})}}};
}
template <typename T>
constexpr FwdTableTable make_fwd_table_table() {
    return {{{fwd_table_types<T, CDF97, NONSEP>(), fwd_table_types<T, CDF97, SEP>()},
             {fwd_table_types<T, CDF53, NONSEP>(), fwd_table_types<T, CDF53, SEP>()}}};
}
template <typename T>
constexpr InvTableTable make_inv_table_table() {
    return {{{inv_table_types<T, CDF97, NONSEP>(), inv_table_types<T, CDF97, SEP>()},
             {inv_table_types<T, CDF53, NONSEP>(), inv_table_types<T, CDF53, SEP>()}}};
}

template <int WV, int SCH, typename TIN, typename TLL, typename TB, int... I>
constexpr std::array<FwdBatchLauncher, kNumTiles> fwd_batch_tiles(std::integer_sequence<int, I...>) {
    return {&launch_fwd_batch<WV, SCH, I, TIN, TLL, TB>...};
}
template <int WV, int SCH, typename TLL, typename TB, typename TOUT, int... I>
constexpr std::array<InvBatchLauncher, kNumTiles> inv_batch_tiles(std::integer_sequence<int, I...>) {
    return {&launch_inv_batch<WV, SCH, I, TLL, TB, TOUT>...};
}

template <int WV, int SCH, typename TIN, typename TLL, typename TB, int... I>
constexpr std::array<FwdLauncher, kNumTiles> fwd_tiles(std::integer_sequence<int, I...>) {
    return {&launch_fwd<WV, SCH, I, TIN, TLL, TB>...};
}
template <int WV, int SCH, typename TLL, typename TB, typename TOUT, int... I>
constexpr std::array<InvLauncher, kNumTiles> inv_tiles(std::integer_sequence<int, I...>) {
    return {&launch_inv<WV, SCH, I, TLL, TB, TOUT>...};
}

// Per storage type T of the user-visible buffers: index [wavelet][scheme]
// [first operand is FP32][second operand is FP32][config], where for the
// forward the operands are (level input, LL output) and for the inverse
// (LL input, level output); the other one of each pair is T. Intermediate
// levels use FP32.
using FwdTable = std::array<std::array<std::array<std::array<std::array<FwdLauncher, kNumTiles>, 2>, 2>, 2>, 2>;
using InvTable = std::array<std::array<std::array<std::array<std::array<InvLauncher, kNumTiles>, 2>, 2>, 2>, 2>;

template <typename T, int WV, int SCH>
constexpr std::array<std::array<std::array<FwdLauncher, kNumTiles>, 2>, 2> fwd_types() {
    using S = std::make_integer_sequence<int, kNumTiles>;
    return {{{fwd_tiles<WV, SCH, T, T, T>(S{}), fwd_tiles<WV, SCH, T, float, T>(S{})},
             {fwd_tiles<WV, SCH, float, T, T>(S{}), fwd_tiles<WV, SCH, float, float, T>(S{})}}};
}
template <typename T, int WV, int SCH>
constexpr std::array<std::array<std::array<InvLauncher, kNumTiles>, 2>, 2> inv_types() {
    using S = std::make_integer_sequence<int, kNumTiles>;
    return {{{inv_tiles<WV, SCH, T, T, T>(S{}), inv_tiles<WV, SCH, T, T, float>(S{})},
             {inv_tiles<WV, SCH, float, T, T>(S{}), inv_tiles<WV, SCH, float, T, float>(S{})}}};
}

using FwdBatchTable = std::array<std::array<std::array<std::array<std::array<FwdBatchLauncher, kNumTiles>, 2>, 2>, 2>, 2>;
using InvBatchTable = std::array<std::array<std::array<std::array<std::array<InvBatchLauncher, kNumTiles>, 2>, 2>, 2>, 2>;

template <typename T, int WV, int SCH>
constexpr std::array<std::array<std::array<FwdBatchLauncher, kNumTiles>, 2>, 2> fwd_batch_types() {
    using S = std::make_integer_sequence<int, kNumTiles>;
    return {{{fwd_batch_tiles<WV, SCH, T, T, T>(S{}), fwd_batch_tiles<WV, SCH, T, float, T>(S{})},
             {fwd_batch_tiles<WV, SCH, float, T, T>(S{}), fwd_batch_tiles<WV, SCH, float, float, T>(S{})}}};
}
template <typename T, int WV, int SCH>
constexpr std::array<std::array<std::array<InvBatchLauncher, kNumTiles>, 2>, 2> inv_batch_types() {
    using S = std::make_integer_sequence<int, kNumTiles>;
    return {{{inv_batch_tiles<WV, SCH, T, T, T>(S{}), inv_batch_tiles<WV, SCH, T, T, float>(S{})},
             {inv_batch_tiles<WV, SCH, float, T, T>(S{}), inv_batch_tiles<WV, SCH, float, T, float>(S{})}}};
}
template <typename T>
constexpr FwdBatchTable make_fwd_batch_table() {
    return {{{fwd_batch_types<T, CDF97, NONSEP>(), fwd_batch_types<T, CDF97, SEP>()},
             {fwd_batch_types<T, CDF53, NONSEP>(), fwd_batch_types<T, CDF53, SEP>()}}};
}
template <typename T>
constexpr InvBatchTable make_inv_batch_table() {
    return {{{inv_batch_types<T, CDF97, NONSEP>(), inv_batch_types<T, CDF97, SEP>()},
             {inv_batch_types<T, CDF53, NONSEP>(), inv_batch_types<T, CDF53, SEP>()}}};
}

template <typename T>
constexpr FwdTable make_fwd_table() {
    return {{{fwd_types<T, CDF97, NONSEP>(), fwd_types<T, CDF97, SEP>()},
             {fwd_types<T, CDF53, NONSEP>(), fwd_types<T, CDF53, SEP>()}}};
}
template <typename T>
constexpr InvTable make_inv_table() {
    return {{{inv_types<T, CDF97, NONSEP>(), inv_types<T, CDF97, SEP>()},
             {inv_types<T, CDF53, NONSEP>(), inv_types<T, CDF53, SEP>()}}};
}

// Fused tails. Forward index [wavelet][scheme][fused levels - 2][input of the
// finest fused level is FP32]; inverse [wavelet][scheme][fused levels - 2]
// [output of the finest fused level is FP32]. The pyramid (bands and the
// coarsest LL) is in the storage type.
using FwdTailLauncher = hipError_t (*)(const FwdTail &, int, hipStream_t);
using InvTailLauncher = hipError_t (*)(const InvTail &, int, hipStream_t);

template <int WV, int SCH, int F, typename TIN, typename T>
hipError_t launch_fwd_tail(const FwdTail &t, int grid, hipStream_t s) {
    hipLaunchKernelGGL((fwd_tail_kernel<WV, SCH, F, TIN, T, T>), dim3(grid),
                       dim3(64 * kTailWaves), 0, s, t);
    return hipGetLastError();
}
template <int WV, int SCH, int F, typename T, typename TOUT>
hipError_t launch_inv_tail(const InvTail &t, int grid, hipStream_t s) {
    hipLaunchKernelGGL((inv_tail_kernel<WV, SCH, F, T, T, TOUT>), dim3(grid),
                       dim3(64 * kTailWaves), 0, s, t);
    return hipGetLastError();
}

static_assert(kTailMax == 3, "tail tables cover 2 and 3 fused levels");
using FwdTailTable = std::array<std::array<std::array<std::array<FwdTailLauncher, 2>, 2>, 2>, 2>;
using InvTailTable = std::array<std::array<std::array<std::array<InvTailLauncher, 2>, 2>, 2>, 2>;

template <typename T, int WV, int SCH>
constexpr std::array<std::array<FwdTailLauncher, 2>, 2> fwd_tail_depths() {
    return {{{&launch_fwd_tail<WV, SCH, 2, T, T>, &launch_fwd_tail<WV, SCH, 2, float, T>},
             {&launch_fwd_tail<WV, SCH, 3, T, T>, &launch_fwd_tail<WV, SCH, 3, float, T>}}};
}
template <typename T, int WV, int SCH>
constexpr std::array<std::array<InvTailLauncher, 2>, 2> inv_tail_depths() {
    return {{{&launch_inv_tail<WV, SCH, 2, T, T>, &launch_inv_tail<WV, SCH, 2, T, float>},
             {&launch_inv_tail<WV, SCH, 3, T, T>, &launch_inv_tail<WV, SCH, 3, T, float>}}};
}
template <typename T>
constexpr FwdTailTable make_fwd_tail_table() {
    return {{{fwd_tail_depths<T, CDF97, NONSEP>(), fwd_tail_depths<T, CDF97, SEP>()},
             {fwd_tail_depths<T, CDF53, NONSEP>(), fwd_tail_depths<T, CDF53, SEP>()}}};
}
template <typename T>
constexpr InvTailTable make_inv_tail_table() {
    return {{{inv_tail_depths<T, CDF97, NONSEP>(), inv_tail_depths<T, CDF97, SEP>()},
             {inv_tail_depths<T, CDF53, NONSEP>(), inv_tail_depths<T, CDF53, SEP>()}}};
}

// Fused finest levels (head). Forward index [wavelet][scheme][level j's input
// is FP32][level j+1's low-low output is FP32]; inverse [wavelet][scheme]
// [level j+1's low-low input is FP32][level j's output is FP32]. The detail
// bands are in the storage type; the band between the two levels is FP32 in
// LDS. One configuration: 12 wavefronts of 4 quad rows.
constexpr int kHeadRows = 4, kHeadWaves = 12;
using FwdHeadGeom = HeadGeom<kHeadRows, kHeadWaves>;
using FwdHeadLauncher = hipError_t (*)(const FwdHead &, hipStream_t);
using InvHeadLauncher = hipError_t (*)(const InvHead &, hipStream_t);

template <int WV, int SCH, typename TIN, typename TLL, typename T>
hipError_t launch_fwd_head(const FwdHead &h, hipStream_t s) {
    hipLaunchKernelGGL((fwd_head_kernel<WV, SCH, kHeadRows, kHeadWaves, TIN, TLL, T>),
                       dim3(h.tiles_x * h.tiles_y), dim3(64 * kHeadWaves), 0, s, h);
    return hipGetLastError();
}
template <int WV, int SCH, typename TLL, typename T, typename TOUT>
hipError_t launch_inv_head(const InvHead &h, hipStream_t s) {
    hipLaunchKernelGGL((inv_head_kernel<WV, SCH, kHeadRows, kHeadWaves, TLL, T, TOUT>),
                       dim3(h.tiles_x * h.tiles_y), dim3(64 * kHeadWaves), 0, s, h);
    return hipGetLastError();
}

using FwdHeadTable = std::array<std::array<std::array<std::array<FwdHeadLauncher, 2>, 2>, 2>, 2>;
using InvHeadTable = std::array<std::array<std::array<std::array<InvHeadLauncher, 2>, 2>, 2>, 2>;

template <typename T, int WV, int SCH>
constexpr std::array<std::array<FwdHeadLauncher, 2>, 2> fwd_head_types() {
    return {{{&launch_fwd_head<WV, SCH, T, T, T>, &launch_fwd_head<WV, SCH, T, float, T>},
             {&launch_fwd_head<WV, SCH, float, T, T>, &launch_fwd_head<WV, SCH, float, float, T>}}};
}
template <typename T, int WV, int SCH>
constexpr std::array<std::array<InvHeadLauncher, 2>, 2> inv_head_types() {
    return {{{&launch_inv_head<WV, SCH, T, T, T>, &launch_inv_head<WV, SCH, T, T, float>},
             {&launch_inv_head<WV, SCH, float, T, T>, &launch_inv_head<WV, SCH, float, T, float>}}};
}
template <typename T>
constexpr FwdHeadTable make_fwd_head_table() {
    return {{{fwd_head_types<T, CDF97, NONSEP>(), fwd_head_types<T, CDF97, SEP>()},
             {fwd_head_types<T, CDF53, NONSEP>(), fwd_head_types<T, CDF53, SEP>()}}};
}
template <typename T>
constexpr InvHeadTable make_inv_head_table() {
    return {{{inv_head_types<T, CDF97, NONSEP>(), inv_head_types<T, CDF97, SEP>()},
             {inv_head_types<T, CDF53, NONSEP>(), inv_head_types<T, CDF53, SEP>()}}};
}

// Heads of a planned batch: one launch over the head tiles of every image,
// indexed as the single-image head tables. `persistent` caps the grid at the
// workgroups that fit on the device at once.
using FwdHeadTableLauncher = hipError_t (*)(const TableLaunch<FwdHead> &, bool, hipStream_t);
using InvHeadTableLauncher = hipError_t (*)(const TableLaunch<InvHead> &, bool, hipStream_t);

template <int WV, int SCH, typename TIN, typename TLL, typename T>
hipError_t launch_fwd_head_table(const TableLaunch<FwdHead> &tl, bool persistent, hipStream_t s) {
    const auto k = fwd_head_table_kernel<WV, SCH, kHeadRows, kHeadWaves, TIN, TLL, T>;
    int grid = tl.total;
    if (persistent) {
        static const int resident = resident_blocks((const void *)k, 64 * kHeadWaves);
        grid = grid < resident ? grid : resident;
    }
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k, dim3(grid), dim3(64 * kHeadWaves), 0, s, tl);
    return hipGetLastError();
}
template <int WV, int SCH, typename TLL, typename T, typename TOUT>
hipError_t launch_inv_head_table(const TableLaunch<InvHead> &tl, bool persistent, hipStream_t s) {
    const auto k = inv_head_table_kernel<WV, SCH, kHeadRows, kHeadWaves, TLL, T, TOUT>;
    int grid = tl.total;
    if (persistent) {
        static const int resident = resident_blocks((const void *)k, 64 * kHeadWaves);
        grid = grid < resident ? grid : resident;
    }
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k, dim3(grid), dim3(64 * kHeadWaves), 0, s, tl);
    return hipGetLastError();
}

using FwdHeadPlanTable = std::array<std::array<std::array<std::array<FwdHeadTableLauncher, 2>, 2>, 2>, 2>;
using InvHeadPlanTable = std::array<std::array<std::array<std::array<InvHeadTableLauncher, 2>, 2>, 2>, 2>;

template <typename T, int WV, int SCH>
constexpr std::array<std::array<FwdHeadTableLauncher, 2>, 2> fwd_head_plan_types() {
    return {{{&launch_fwd_head_table<WV, SCH, T, T, T>, &launch_fwd_head_table<WV, SCH, T, float, T>},
             {&launch_fwd_head_table<WV, SCH, float, T, T>,
              &launch_fwd_head_table<WV, SCH, float, float, T>}}};
}
template <typename T, int WV, int SCH>
constexpr std::array<std::array<InvHeadTableLauncher, 2>, 2> inv_head_plan_types() {
    return {{{&launch_inv_head_table<WV, SCH, T, T, T>, &launch_inv_head_table<WV, SCH, T, T, float>},
             {&launch_inv_head_table<WV, SCH, float, T, T>,
              &launch_inv_head_table<WV, SCH, float, T, float>}}};
}
template <typename T>
constexpr FwdHeadPlanTable make_fwd_head_plan_table() {
    return {{{fwd_head_plan_types<T, CDF97, NONSEP>(), fwd_head_plan_types<T, CDF97, SEP>()},
             {fwd_head_plan_types<T, CDF53, NONSEP>(), fwd_head_plan_types<T, CDF53, SEP>()}}};
}
template <typename T>
constexpr InvHeadPlanTable make_inv_head_plan_table() {
    return {{{inv_head_plan_types<T, CDF97, NONSEP>(), inv_head_plan_types<T, CDF97, SEP>()},
             {inv_head_plan_types<T, CDF53, NONSEP>(), inv_head_plan_types<T, CDF53, SEP>()}}};
}

// Head level batches (kernel-argument tables), indexed as the single-image
// head tables.
using FwdHeadBatchLauncher = hipError_t (*)(const FwdHeadBatch &, hipStream_t);
using InvHeadBatchLauncher = hipError_t (*)(const InvHeadBatch &, hipStream_t);

template <int WV, int SCH, typename TIN, typename TLL, typename T>
hipError_t launch_fwd_head_batch(const FwdHeadBatch &b, hipStream_t s) {
    const int grid = b.tile_start[b.n];
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL((fwd_head_batch_kernel<WV, SCH, kHeadRows, kHeadWaves, TIN, TLL, T>),
                       dim3(grid), dim3(64 * kHeadWaves), 0, s, b);
    return hipGetLastError();
}
template <int WV, int SCH, typename TLL, typename T, typename TOUT>
hipError_t launch_inv_head_batch(const InvHeadBatch &b, hipStream_t s) {
    const int grid = b.tile_start[b.n];
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL((inv_head_batch_kernel<WV, SCH, kHeadRows, kHeadWaves, TLL, T, TOUT>),
                       dim3(grid), dim3(64 * kHeadWaves), 0, s, b);
    return hipGetLastError();
}

using FwdHeadBatchTable = std::array<std::array<std::array<std::array<FwdHeadBatchLauncher, 2>, 2>, 2>, 2>;
using InvHeadBatchTable = std::array<std::array<std::array<std::array<InvHeadBatchLauncher, 2>, 2>, 2>, 2>;

template <typename T, int WV, int SCH>
constexpr std::array<std::array<FwdHeadBatchLauncher, 2>, 2> fwd_head_batch_types() {
    return {{{&launch_fwd_head_batch<WV, SCH, T, T, T>, &launch_fwd_head_batch<WV, SCH, T, float, T>},
             {&launch_fwd_head_batch<WV, SCH, float, T, T>,
              &launch_fwd_head_batch<WV, SCH, float, float, T>}}};
}
template <typename T, int WV, int SCH>
constexpr std::array<std::array<InvHeadBatchLauncher, 2>, 2> inv_head_batch_types() {
    return {{{&launch_inv_head_batch<WV, SCH, T, T, T>, &launch_inv_head_batch<WV, SCH, T, T, float>},
             {&launch_inv_head_batch<WV, SCH, float, T, T>,
              &launch_inv_head_batch<WV, SCH, float, T, float>}}};
}
template <typename T>
constexpr FwdHeadBatchTable make_fwd_head_batch_table() {
    return {{{fwd_head_batch_types<T, CDF97, NONSEP>(), fwd_head_batch_types<T, CDF97, SEP>()},
             {fwd_head_batch_types<T, CDF53, NONSEP>(), fwd_head_batch_types<T, CDF53, SEP>()}}};
}
template <typename T>
constexpr InvHeadBatchTable make_inv_head_batch_table() {
    return {{{inv_head_batch_types<T, CDF97, NONSEP>(), inv_head_batch_types<T, CDF97, SEP>()},
             {inv_head_batch_types<T, CDF53, NONSEP>(), inv_head_batch_types<T, CDF53, SEP>()}}};
}

// The exchange ablation (NONSEP_LDS, SEP_LDS): FP32 level kernels only, index [wavelet][scheme - NONSEP_LDS][config].
using FwdLdsTable = std::array<std::array<std::array<FwdLauncher, kNumTiles>, 2>, 2>;
using InvLdsTable = std::array<std::array<std::array<InvLauncher, kNumTiles>, 2>, 2>;

template <int WV, int SCH, int T>
hipError_t launch_fwd_lds(const FwdParams &p, hipStream_t s) {
    return launch_fwd<WV, SCH, T, float, float, float>(p, s);
}
template <int WV, int SCH, int T>
hipError_t launch_inv_lds(const InvParams &p, hipStream_t s) {
    return launch_inv<WV, SCH, T, float, float, float>(p, s);
}
template <int WV, int SCH, int... I>
constexpr std::array<FwdLauncher, kNumTiles> fwd_lds_tiles(std::integer_sequence<int, I...>) {
    return {&launch_fwd_lds<WV, SCH, I>...};
}
template <int WV, int SCH, int... I>
constexpr std::array<InvLauncher, kNumTiles> inv_lds_tiles(std::integer_sequence<int, I...>) {
    return {&launch_inv_lds<WV, SCH, I>...};
}
inline constexpr FwdLdsTable make_fwd_lds_table() {
    using S = std::make_integer_sequence<int, kNumTiles>;
    return {{{fwd_lds_tiles<CDF97, NONSEP_LDS>(S{}), fwd_lds_tiles<CDF97, SEP_LDS>(S{})},
             {fwd_lds_tiles<CDF53, NONSEP_LDS>(S{}), fwd_lds_tiles<CDF53, SEP_LDS>(S{})}}};
}
inline constexpr InvLdsTable make_inv_lds_table() {
    using S = std::make_integer_sequence<int, kNumTiles>;
    return {{{inv_lds_tiles<CDF97, NONSEP_LDS>(S{}), inv_lds_tiles<CDF97, SEP_LDS>(S{})},
             {inv_lds_tiles<CDF53, NONSEP_LDS>(S{}), inv_lds_tiles<CDF53, SEP_LDS>(S{})}}};
}

// Defined in one translation unit per storage type and direction.
extern FwdTable kFwdF32, kFwdF16, kFwdBF16;
extern InvTable kInvF32, kInvF16, kInvBF16;
extern FwdBatchTable kFwdBatchF32, kFwdBatchF16, kFwdBatchBF16;
extern InvBatchTable kInvBatchF32, kInvBatchF16, kInvBatchBF16;
extern FwdTableTable kFwdPlanF32, kFwdPlanF16, kFwdPlanBF16;
extern InvTableTable kInvPlanF32, kInvPlanF16, kInvPlanBF16;
extern FwdTailTable kFwdTailF32, kFwdTailF16, kFwdTailBF16;
extern FwdHeadTable kFwdHeadF32, kFwdHeadF16, kFwdHeadBF16;
extern InvHeadTable kInvHeadF32, kInvHeadF16, kInvHeadBF16;
extern FwdHeadPlanTable kFwdHeadPlanF32, kFwdHeadPlanF16, kFwdHeadPlanBF16;
extern InvHeadPlanTable kInvHeadPlanF32, kInvHeadPlanF16, kInvHeadPlanBF16;
extern FwdHeadBatchTable kFwdHeadBatchF32, kFwdHeadBatchF16, kFwdHeadBatchBF16;
extern InvHeadBatchTable kInvHeadBatchF32, kInvHeadBatchF16, kInvHeadBatchBF16;
extern InvTailTable kInvTailF32, kInvTailF16, kInvTailBF16;
extern FwdLdsTable kFwdLds;
extern InvLdsTable kInvLds;

}  // namespace dwt2

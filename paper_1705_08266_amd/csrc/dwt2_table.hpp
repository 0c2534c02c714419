// Launch table: one launcher per (wavelet, scheme, storage types, tile).
#pragma once

#include <array>
#include <utility>

#include "dwt2_kernels.hpp"

namespace dwt2 {

struct TileCfg {
    int qpl;    // quads per lane along x
    int rows;   // quad rows per lane
    int waves;  // wavefronts stacked along y
};

// Compiled tile shapes. Window = (64*qpl) x (waves*rows) quads.
constexpr TileCfg kTiles[] = {
    {2, 8, 4},    // 0: 128 x 32 window, 256 threads
    {2, 4, 4},    // 1: 128 x 16
    {4, 4, 4},    // 2: 256 x 16
    {2, 16, 4},   // 3: 128 x 64
    {2, 8, 8},    // 4: 128 x 64, 512 threads
    {2, 8, 1},    // 5: 128 x 8, one wavefront, no barriers
    {4, 8, 4},    // 6: 256 x 32
    {2, 4, 8},    // 7: 128 x 32, 512 threads
};
constexpr int kNumTiles = (int)(sizeof(kTiles) / sizeof(kTiles[0]));

using FwdLauncher = hipError_t (*)(const FwdParams &, int grid, hipStream_t);
using InvLauncher = hipError_t (*)(const InvParams &, int grid, hipStream_t);

template <int WV, int SCH, int T, typename TIN, typename TLL, typename TB>
hipError_t launch_fwd(const FwdParams &p, int grid, hipStream_t s) {
    constexpr TileCfg c = kTiles[T];
    hipLaunchKernelGGL((fwd_level_kernel<WV, SCH, c.qpl, c.rows, c.waves, TIN, TLL, TB>),
                       dim3(grid), dim3(64 * c.waves), 0, s, p);
    return hipGetLastError();
}

template <int WV, int SCH, int T, typename TLL, typename TB, typename TOUT>
hipError_t launch_inv(const InvParams &p, int grid, hipStream_t s) {
    constexpr TileCfg c = kTiles[T];
    hipLaunchKernelGGL((inv_level_kernel<WV, SCH, c.qpl, c.rows, c.waves, TLL, TB, TOUT>),
                       dim3(grid), dim3(64 * c.waves), 0, s, p);
    return hipGetLastError();
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
// [first operand is FP32][second operand is FP32][tile], where for the forward
// the operands are (level input, LL output) and for the inverse (LL input,
// level output); the other one of each pair is T. Intermediate levels use FP32.
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

// Defined in one translation unit per storage type.
extern FwdTable kFwdF32, kFwdF16, kFwdBF16;
extern InvTable kInvF32, kInvF16, kInvBF16;

}  // namespace dwt2

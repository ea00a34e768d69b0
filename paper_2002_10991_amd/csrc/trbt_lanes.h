// trbt_lanes.h -- sums across the lanes of one 64-wide wavefront on gfx950
// without a trip through LDS: DPP moves within 16-lane rows, then the
// lane-swap instructions across rows and halves.  Every lane gets the sum,
// in the same order of additions in every lane.
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>

// x from another lane of the same 16-lane row, by a DPP move of each 32-bit
// half (a VALU operation: no trip through the LDS crossbar)
template <int CTRL>
__device__ inline double dpp_f64(double x)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// sum over a 16-lane row, in every lane of the row: pairs within quads, then
// quads within half rows, then half rows (quad_perm [1,0,3,2], [2,3,0,1],
// row_half_mirror, row_mirror)
__device__ inline double row_sum(double x)
{
    x += dpp_f64<0xB1>(x);
    x += dpp_f64<0x4E>(x);
    x += dpp_f64<0x141>(x);
    x += dpp_f64<0x140>(x);
    return x;
}

// x plus x of the lane 16 apart (W = 16: rows 0/1 and 2/3) or 32 apart
// (W = 32: the two halves), by the gfx950 lane-swap instructions (VALU, no
// trip through the LDS crossbar).  Swapping two copies of x exchanges rows
// 1 and 3 of the first with rows 0 and 2 of the second (W = 16), or the
// upper half of the first with the lower half of the second (W = 32), so in
// both lanes of a pair the first copy holds the lower lane's x and the
// second the upper lane's: the sum is the same, in the same order, in both.
template <int W>
__device__ inline double swap_add(double x)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = (uint32_t)u, hi = (uint32_t)(u >> 32);
    uint32_t l0, l1, h0, h1;
    if constexpr (W == 16) {
        const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        l0 = l[0], l1 = l[1], h0 = h[0], h1 = h[1];
    } else {
        static_assert(W == 32, "lane distance 16 or 32");
        const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        l0 = l[0], l1 = l[1], h0 = h[0], h1 = h[1];
    }
    const double a = __builtin_bit_cast(double, ((uint64_t)h0 << 32) | l0);
    const double b = __builtin_bit_cast(double, ((uint64_t)h1 << 32) | l1);
    return a + b;
}

// sum over all 64 lanes, in every lane: rows by DPP, then rows 0/1 and
// 2/3, then the two halves
__device__ inline double wave_sum(double x) { return swap_add<32>(swap_add<16>(row_sum(x))); }

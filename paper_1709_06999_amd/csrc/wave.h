// wave.h -- reductions and scans across the 64 lanes of a wave, by DPP lane
// permutations inside rows of 16 lanes and lane reads across the four rows.
//
// Every helper must be called with the whole wave active (uniform control
// flow); every lane gets the result.  The combination order is fixed, so the
// results are bitwise repeatable.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gal {

// DPP controls (GFX9 encoding)
constexpr int DPP_QUAD_XOR1 = 0xB1;       // quad_perm [1, 0, 3, 2]
constexpr int DPP_QUAD_XOR2 = 0x4E;       // quad_perm [2, 3, 0, 1]
constexpr int DPP_ROW_HALF_MIRROR = 0x141;  // lane j of 8 <- 7 - j
constexpr int DPP_ROW_MIRROR = 0x140;     // lane j of 16 <- 15 - j
constexpr int DPP_ROW_SHR1 = 0x111;       // lane j of 16 <- j - 1 (0 at j = 0)
constexpr int DPP_ROW_SHR2 = 0x112;
constexpr int DPP_ROW_SHR4 = 0x114;
constexpr int DPP_ROW_SHR8 = 0x118;

// the value of another lane of the same row; a lane whose source lies
// outside its row gets 0
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int x) {
    return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const int lo = dpp_i32<CTRL>((int)(uint32_t)b), hi = dpp_i32<CTRL>((int)(uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

__device__ __forceinline__ double read_lane(double x, int lane) {
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// butterfly inside each row of 16: afterwards every lane of a row holds the
// row's combination
#define GAL_ROW_REDUCE(x, OP, DPP)                   \
    x = OP(x, DPP<DPP_QUAD_XOR1>(x));                \
    x = OP(x, DPP<DPP_QUAD_XOR2>(x));                \
    x = OP(x, DPP<DPP_ROW_HALF_MIRROR>(x));          \
    x = OP(x, DPP<DPP_ROW_MIRROR>(x))

__device__ __forceinline__ int op_min(int a, int b) { return a < b ? a : b; }
__device__ __forceinline__ int op_max(int a, int b) { return a > b ? a : b; }
__device__ __forceinline__ double op_add(double a, double b) { return a + b; }

__device__ __forceinline__ int wave_min(int x) {
    GAL_ROW_REDUCE(x, op_min, dpp_i32);
    const int a = __builtin_amdgcn_readlane(x, 0), b = __builtin_amdgcn_readlane(x, 16);
    const int c = __builtin_amdgcn_readlane(x, 32), d = __builtin_amdgcn_readlane(x, 48);
    return op_min(op_min(a, b), op_min(c, d));
}
__device__ __forceinline__ int wave_max(int x) {
    GAL_ROW_REDUCE(x, op_max, dpp_i32);
    const int a = __builtin_amdgcn_readlane(x, 0), b = __builtin_amdgcn_readlane(x, 16);
    const int c = __builtin_amdgcn_readlane(x, 32), d = __builtin_amdgcn_readlane(x, 48);
    return op_max(op_max(a, b), op_max(c, d));
}
// sum over the 64 lanes: rows of 16 by butterflies, then (r0 + r1) + (r2 + r3)
__device__ __forceinline__ double wave_sum(double x) {
    GAL_ROW_REDUCE(x, op_add, dpp_f64);
    return (read_lane(x, 0) + read_lane(x, 16)) + (read_lane(x, 32) + read_lane(x, 48));
}
#undef GAL_ROW_REDUCE

// The same sum through LDS lane permutes (xor butterflies over 64 lanes).
// Slower alone, but its steps are asynchronous: in a loop that reduces one
// value per iteration, the next iteration's independent work overlaps them.
__device__ __forceinline__ double wave_sum_permute(double x) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// exclusive prefix sum over the lanes in lane order: a scan inside each row
// of 16 (shifts by 1, 2, 4, 8), then the totals of the rows before
__device__ __forceinline__ double wave_excl_scan(double x) {
    double s = x;
    s += dpp_f64<DPP_ROW_SHR1>(s);
    s += dpp_f64<DPP_ROW_SHR2>(s);
    s += dpp_f64<DPP_ROW_SHR4>(s);
    s += dpp_f64<DPP_ROW_SHR8>(s);          // inclusive scan within the row
    const double e = dpp_f64<DPP_ROW_SHR1>(s);  // exclusive within the row
    const double t0 = read_lane(s, 15), t1 = read_lane(s, 31), t2 = read_lane(s, 47);
    const int row = (int)(threadIdx.x & 63) >> 4;
    const double base = row == 0 ? 0.0 : (row == 1 ? t0 : (row == 2 ? t0 + t1 : (t0 + t1) + t2));
    return base + e;
}

}  // namespace gal

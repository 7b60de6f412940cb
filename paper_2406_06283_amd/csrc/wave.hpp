// Wave-level reductions on data-parallel-primitive (DPP) lane moves.
//
// A 64-lane wave is four rows of 16 lanes.  Within a row the butterfly runs on DPP moves, which
// are ALU operations (quad permutations, then the half-row and row mirrors); the four row results
// are then read with v_readlane and combined in row order.  Every lane ends with the same bits, and
// the summation order is fixed, so results are deterministic.  (Cross-lane shuffles by index
// permute through the LDS unit and cost a round trip per step.)
#pragma once

#include <hip/hip_runtime.h>

namespace hkg {

constexpr int DPP_QUAD_XOR1 = 0xB1;       // quad_perm [1, 0, 3, 2]
constexpr int DPP_QUAD_XOR2 = 0x4E;       // quad_perm [2, 3, 0, 1]
constexpr int DPP_ROW_MIRROR = 0x140;     // lane i <- lane 15 - i within the row
constexpr int DPP_ROW_HALF_MIRROR = 0x141; // lane i <- lane 7 - i within each half row

// A workgroup barrier that first waits for this wave's LDS operations to complete
// (s_waitcnt lgkmcnt(0), the other counters left as they are).  The compiler does not always emit
// that wait before the barrier of __syncthreads() when the LDS stores come from a loop's previous
// iteration; another wave can then read a slot after the barrier before the store has landed.
__device__ __forceinline__ void sync_lds() {
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __syncthreads();
}

template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
    return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xf, 0xf, false);
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = dpp_i32<CTRL>((int)b);
    const int hi = dpp_i32<CTRL>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
    return __int_as_float(dpp_i32<CTRL>(__float_as_int(v)));
}

template <int CTRL, typename T>
__device__ __forceinline__ T dpp_move(T v) {
    if constexpr (sizeof(T) == 8) return dpp_f64<CTRL>(v);
    else return dpp_f32<CTRL>(v);
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ float readlane_f32(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

template <typename T>
__device__ __forceinline__ T readlane_any(T v, int lane) {
    if constexpr (sizeof(T) == 8) return readlane_f64(v, lane);
    else return readlane_f32(v, lane);
}

// sum over the 16 lanes of each row; every lane of the row gets the row's sum
__device__ __forceinline__ double row_sum16(double v) {
    v += dpp_f64<DPP_QUAD_XOR1>(v);
    v += dpp_f64<DPP_QUAD_XOR2>(v);
    v += dpp_f64<DPP_ROW_HALF_MIRROR>(v);
    v += dpp_f64<DPP_ROW_MIRROR>(v);
    return v;
}

// sum over the 64 lanes; every lane gets the same value
__device__ __forceinline__ double wave_sum64(double v) {
    v = row_sum16(v);
    return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// max / min over the 64 lanes; every lane gets the result
__device__ __forceinline__ double wave_max64(double v) {
    v = fmax(v, dpp_f64<DPP_QUAD_XOR1>(v));
    v = fmax(v, dpp_f64<DPP_QUAD_XOR2>(v));
    v = fmax(v, dpp_f64<DPP_ROW_HALF_MIRROR>(v));
    v = fmax(v, dpp_f64<DPP_ROW_MIRROR>(v));
    return fmax(fmax(readlane_f64(v, 0), readlane_f64(v, 16)), fmax(readlane_f64(v, 32), readlane_f64(v, 48)));
}

__device__ __forceinline__ double wave_min64(double v) {
    v = fmin(v, dpp_f64<DPP_QUAD_XOR1>(v));
    v = fmin(v, dpp_f64<DPP_QUAD_XOR2>(v));
    v = fmin(v, dpp_f64<DPP_ROW_HALF_MIRROR>(v));
    v = fmin(v, dpp_f64<DPP_ROW_MIRROR>(v));
    return fmin(fmin(readlane_f64(v, 0), readlane_f64(v, 16)), fmin(readlane_f64(v, 32), readlane_f64(v, 48)));
}

// arg-max of |value| candidates (v, idx): larger v wins, ties go to the smaller idx
template <typename T>
__device__ __forceinline__ void argmax_pick(T &v, int &idx, T ov, int oi) {
    if (ov > v || (ov == v && oi < idx)) {
        v = ov;
        idx = oi;
    }
}

template <int CTRL, typename T>
__device__ __forceinline__ void argmax_dpp_step(T &v, int &idx) {
    const T ov = dpp_move<CTRL>(v);
    const int oi = dpp_i32<CTRL>(idx);
    argmax_pick(v, idx, ov, oi);
}

// arg-max within each 16-lane row; every lane of the row gets the row's winner
template <typename T>
__device__ __forceinline__ void argmax_row16(T &v, int &idx) {
    argmax_dpp_step<DPP_QUAD_XOR1>(v, idx);
    argmax_dpp_step<DPP_QUAD_XOR2>(v, idx);
    argmax_dpp_step<DPP_ROW_HALF_MIRROR>(v, idx);
    argmax_dpp_step<DPP_ROW_MIRROR>(v, idx);
}

// arg-max over the 64 lanes; every lane gets the winner (rows combined in order 0..3)
template <typename T>
__device__ __forceinline__ void argmax_wave64(T &v, int &idx) {
    argmax_row16(v, idx);
    T bv = readlane_any(v, 0);
    int bi = __builtin_amdgcn_readlane(idx, 0);
#pragma unroll
    for (int r = 1; r < 4; ++r) argmax_pick(bv, bi, readlane_any(v, 16 * r), __builtin_amdgcn_readlane(idx, 16 * r));
    v = bv;
    idx = bi;
}

}  // namespace hkg

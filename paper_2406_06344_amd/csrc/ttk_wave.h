// Cross-lane reductions for 64-wide waves without LDS traffic: DPP row
// rotations (row_ror by 8, 4, 2, 1 within each row of 16 lanes) give every
// lane its row's result, and the four rows of a wave are combined from lanes
// 0, 16, 32 and 48 by v_readlane.  Every lane of the wave (or of the row, for
// the row16 forms) must be active.
#pragma once

#include <hip/hip_runtime.h>

namespace ttk {

template <int N>
__device__ inline double row_ror(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x120 + N, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x120 + N, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int N>
__device__ inline int row_ror_i(int x) {
  return __builtin_amdgcn_update_dpp(0, x, 0x120 + N, 0xF, 0xF, false);
}

// any DPP lane permutation of a double (CTRL: the DPP control word)
template <int CTRL>
__device__ inline double dpp_d(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ inline double readlane_d(double x, int lane) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// sum / max over each row of 16 lanes, in every lane of the row
__device__ inline double row16_sum(double v) {
  v += row_ror<8>(v);
  v += row_ror<4>(v);
  v += row_ror<2>(v);
  v += row_ror<1>(v);
  return v;
}
// sum over each group of 32 lanes (two DPP rows), the same value in every
// lane of the group: the row sums, then the other row's by a lane swap
__device__ inline double row32_sum(double v) {
  v = row16_sum(v);
  return v + __shfl_xor(v, 16, 64);
}
// sum over each group of 8 lanes (half a row), the same value in every lane
// of the group: neighbour swap and pair swap within quads (quad_perm
// [1,0,3,2] and [2,3,0,1]), then the other quad by row_half_mirror
__device__ inline double row8_sum(double v) {
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  v += dpp_d<0x141>(v);
  return v;
}
__device__ inline double row16_max(double v) {
  v = fmax(v, row_ror<8>(v));
  v = fmax(v, row_ror<4>(v));
  v = fmax(v, row_ror<2>(v));
  v = fmax(v, row_ror<1>(v));
  return v;
}
__device__ inline int row16_min_i(int v) {
  v = min(v, row_ror_i<8>(v));
  v = min(v, row_ror_i<4>(v));
  v = min(v, row_ror_i<2>(v));
  v = min(v, row_ror_i<1>(v));
  return v;
}

// sum / max / min over the whole wave, uniform result in every lane
__device__ inline double wave64_sum(double v) {
  v = row16_sum(v);
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}
__device__ inline double wave64_max(double v) {
  v = row16_max(v);
  return fmax(fmax(readlane_d(v, 0), readlane_d(v, 16)), fmax(readlane_d(v, 32), readlane_d(v, 48)));
}
__device__ inline int wave64_min_i(int v) {
  v = row16_min_i(v);
  return min(min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
             min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

}  // namespace ttk

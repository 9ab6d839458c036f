// Deterministic FP64 sums across a wavefront (fixed order, no LDS).
#pragma once
#include <hip/hip_runtime.h>

namespace lbm {

// Lane 15 of every row of 16 lanes gets the row's total: DPP row shifts,
// without the LDS crossbar, in a fixed order.
__device__ __forceinline__ double row_sum16(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
#define WAVE_SUM_STEP(CTRL)                                                              \
  {                                                                                      \
    const int l2 = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xf, 0xf, false);            \
    const int h2 = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xf, 0xf, false);            \
    const double t = __hiloint2double(h2, l2) + __hiloint2double(hi, lo);                \
    lo = __double2loint(t);                                                              \
    hi = __double2hiint(t);                                                              \
  }
  WAVE_SUM_STEP(0x111)  // row_shr:1
  WAVE_SUM_STEP(0x112)  // row_shr:2
  WAVE_SUM_STEP(0x114)  // row_shr:4
  WAVE_SUM_STEP(0x118)  // row_shr:8
#undef WAVE_SUM_STEP
  return __hiloint2double(hi, lo);
}

// Sum of a double over the 64 lanes of a wavefront: the four row totals of
// row_sum16 read out and added in a fixed order (deterministic). Every lane
// returns the wavefront total.
__device__ __forceinline__ double wave_sum(double v) {
  const double rs = row_sum16(v);
  const int lo = __double2loint(rs), hi = __double2hiint(rs);
  double tot = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r)
    tot += __hiloint2double(__builtin_amdgcn_readlane(hi, 16 * r + 15), __builtin_amdgcn_readlane(lo, 16 * r + 15));
  return tot;
}

// The wavefront totals of N values per lane (N <= 16) for a workgroup of
// one wavefront, lane j < N returning the total of value j: the same sums as
// wave_sum(v[j]) in lane j, to the bit, with far fewer instructions. Each
// row total is the balanced pairwise tree that row_sum16 leaves in lane 15
// ((v15 + v14) + (v13 + v12)) + ..., evaluated here by lane 4j + r from the
// values staged in LDS, and the four row totals are added in wave_sum's
// order, starting from 0. sm: LDS of N * 64 + N * 4 doubles.
template <int N>
__device__ __forceinline__ double wave_sums_lds(const double (&v)[N], double* sm) {
  static_assert(N <= 16, "at most 16 values");
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < N; ++j) sm[j * 64 + lane] = v[j];
  __syncthreads();
  if (lane < 4 * N) {
    const double* x = sm + (lane >> 2) * 64 + 16 * (lane & 3);
    double a[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = x[15 - 2 * i] + x[14 - 2 * i];
    const double r = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    sm[N * 64 + lane] = r;
  }
  __syncthreads();
  double tot = 0.0;
  if (lane < N) {
#pragma unroll
    for (int r = 0; r < 4; ++r) tot += sm[N * 64 + 4 * lane + r];
  }
  return tot;
}

}  // namespace lbm

// Device helpers of the single-pulse search (boxcar matched filter over each
// dedispersed series, the detection step that dedispersion feeds in the
// real-time pipeline of Section 1 of Sclocco et al., arXiv 1601.01165).
//
// Definition (the same as the dedisp_detect entry point documents):
//   B_w(t)  = sum of y[t .. t + w) over full windows, w = 1, 2, 4, ..., 32
//   S/N_w   = (max_t B_w(t) - w mean) / (std sqrt(w)), mean and std (ddof 0)
//             over the whole series
//   result  = the width with the largest S/N (ties: the narrower) and the
//             first t reaching that width's maximum.
//
// The series is cut into time tiles that overlap: tile k computes the samples
// [k step, k step + ST) but owns only the window starts [k step, (k+1) step),
// with ST - step >= 31, so each window that starts in a tile ends inside it.
// A tile reduces its owned windows to one record per (series, tile): per
// width the largest sum and its first start, plus the FP64 sum and sum of
// squares of its owned samples.  A second kernel merges the records of a
// series in tile order.  In a tile each lane owns a run of L consecutive
// starts and reads the 32 samples after its run as look-ahead.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace dd {

// Sum of a double over the 64 lanes of a wave (fixed butterfly order; lane 0
// holds the same value on every run).
__device__ __forceinline__ double det_wave_sum(double x) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
  return x;
}

__device__ __forceinline__ int det_wave_max(int x) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x = max(x, __shfl_xor(x, m, 64));
  return x;
}

__device__ __forceinline__ float det_wave_maxf(float x) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x = fmaxf(x, __shfl_xor(x, m, 64));
  return x;
}

__device__ __forceinline__ int det_wave_min(int x) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x = min(x, __shfl_xor(x, m, 64));
  return x;
}

// Float series.  v[0 .. L + 32) holds the lane's run and its look-ahead, with
// -inf at positions past the end of the series, so a window that reaches
// them sums to -inf and never wins.  Boxcar sums by doubling,
// B_2w(i) = B_w(i) + B_w(i + w), the order the record merge and the unfused
// search share.  owned: the lane's starts belong to this tile; lim: starts
// i < lim hold samples of the series (MASK = false when lim >= L).  Per width
// the lane's largest sum and its first start (-1 and -inf when none).
template <int L, bool MASK>
__device__ __forceinline__ void det_lane_f32(float* v, bool owned, int lim, float* bval, int* bidx, double& s1,
                                             double& s2) {
  s1 = 0.0;
  s2 = 0.0;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const double y = (double)v[i];
    const bool ok = !MASK || i < lim;
    s1 += ok ? y : 0.0;
    s2 = ok ? fma(y, y, s2) : s2;
  }
#pragma unroll
  for (int k = 0; k < kDetNW; ++k) {
    const int w = 1 << k;
    if (k > 0) {
      const int h = w >> 1;
#pragma unroll
      for (int i = 0; i < L + kDetLook - w; ++i) v[i] = v[i] + v[i + h];
    }
    float best = -INFINITY;
    int at = -1;
#pragma unroll
    for (int i = 0; i < L; ++i) {
      if (v[i] > best) {
        best = v[i];
        at = i;
      }
    }
    bval[k] = owned ? best : -INFINITY;
    bidx[k] = owned ? at : -1;
  }
  if (!owned) {
    s1 = 0.0;
    s2 = 0.0;
  }
}

// Merge the lanes' results of one series in one tile and write its record.
// lane_pos0: tile-relative position of the lane's first start; t0: the
// tile's first sample.
__device__ __forceinline__ void det_commit_f32(DetRec* rec, const float* bval, const int* bidx, double s1, double s2,
                                               int lane_pos0, int t0) {
  const int lane = threadIdx.x & 63;
  int val[kDetNW], pos[kDetNW];
#pragma unroll
  for (int k = 0; k < kDetNW; ++k) {
    const float m = det_wave_maxf(bval[k]);
    // lanes hold consecutive runs, so the lowest lane with the maximum holds its first start
    const uint64_t hit = __ballot(bidx[k] >= 0 && bval[k] == m);
    int p = -1;
    if (hit) {
      const int l0 = __builtin_ctzll(hit);
      p = t0 + __builtin_amdgcn_readlane(lane_pos0 + bidx[k], l0);
    }
    val[k] = __float_as_int(m);
    pos[k] = p;
  }
  s1 = det_wave_sum(s1);
  s2 = det_wave_sum(s2);
  if (lane == 0) {
    int4* r = reinterpret_cast<int4*>(rec);
    r[0] = make_int4(val[0], val[1], val[2], val[3]);
    r[1] = make_int4(val[4], val[5], pos[0], pos[1]);
    r[2] = make_int4(pos[2], pos[3], pos[4], pos[5]);
    double2 s;
    s.x = s1;
    s.y = s2;
    *reinterpret_cast<double2*>(r + 3) = s;
  }
}

// Integer series (uint8 input: exact sums).  v[0 .. L + 32) holds the run and
// look-ahead scaled by 2^IB (y << IB).  With prefix sums P over v, the key
//   P(i + w) - (P(i) - (L - 1 - i)) = (B_w(i) << IB) + (L - 1 - i)
// orders windows by sum and, for equal sums, the earlier start first, so one
// integer max per window finds both.  Starts outside the tile's owned range
// or past the series end get P(i) := 2^30 and prefix entries past the end
// -2^30, which makes every key that touches them negative (the host limits
// sums to keep |P| < 2^30).  Per width the lane's largest key (negative: none).
template <int L, int IB, bool MASK>
__device__ __forceinline__ void det_lane_int(const int* v, bool owned, int lim, int* key, double& s1, double& s2) {
  int s1i = 0;
  s2 = 0.0;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const int y = v[i] >> IB;
    const bool ok = !MASK || i < lim;
    s1i += ok ? y : 0;
    const double yd = (double)(ok ? y : 0);
    s2 = fma(yd, yd, s2);
  }
  s1 = owned ? (double)s1i : 0.0;
  if (!owned) s2 = 0.0;
#pragma unroll
  for (int k = 0; k < kDetNW; ++k) key[k] = INT32_MIN;
  // One pass over the prefix sums P(j), j = 0 .. L + 31: P(j) closes the
  // window of width w that starts at j - w, so only the L start terms stay
  // live, not the whole prefix.
  int Q[L];
  int P = 0;
#pragma unroll
  for (int j = 0; j < L + kDetLook; ++j) {
    if (j < L) {
      const bool start_ok = owned && (!MASK || j < lim);
      Q[j] = start_ok ? P - (L - 1 - j) : (1 << 30);
    }
    const int Pj = (MASK && j > lim) ? -(1 << 30) : P;
#pragma unroll
    for (int k = 0; k < kDetNW; ++k) {
      const int i = j - (1 << k);
      if (i >= 0 && i < L) key[k] = max(key[k], Pj - Q[i]);
    }
    if (j + 1 < L + kDetLook) P += v[j];
  }
}

template <int L, int IB>
__device__ __forceinline__ void det_commit_int(DetRec* rec, const int* key, double s1, double s2, int lane_pos0,
                                               int t0) {
  const int lane = threadIdx.x & 63;
  int val[kDetNW], pos[kDetNW];
#pragma unroll
  for (int k = 0; k < kDetNW; ++k) {
    const int m = key[k] >> IB;  // the sum; negative: no window
    const int mm = det_wave_max(m);
    int p = -1;
    if (mm >= 0) {
      const uint64_t hit = __ballot(m == mm);
      const int l0 = __builtin_ctzll(hit);
      const int kk = __builtin_amdgcn_readlane(key[k], l0);
      p = t0 + __builtin_amdgcn_readlane(lane_pos0, l0) + (L - 1 - (kk & (L - 1)));
    }
    val[k] = mm;
    pos[k] = p;
  }
  s1 = det_wave_sum(s1);
  s2 = det_wave_sum(s2);
  if (lane == 0) {
    int4* r = reinterpret_cast<int4*>(rec);
    r[0] = make_int4(val[0], val[1], val[2], val[3]);
    r[1] = make_int4(val[4], val[5], pos[0], pos[1]);
    r[2] = make_int4(pos[2], pos[3], pos[4], pos[5]);
    double2 s;
    s.x = s1;
    s.y = s2;
    *reinterpret_cast<double2*>(r + 3) = s;
  }
}

}  // namespace dd

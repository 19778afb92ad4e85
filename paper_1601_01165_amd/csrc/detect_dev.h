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
// starts and takes the 32 samples after its run from the lanes above.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace dd {

// Reductions over the 64 lanes of a wave with DPP row shifts and row
// broadcasts (no LDS traffic): shifts by 1, 2, 4 and 8 lanes leave each
// 16-lane row's result in its lane 15, broadcasting lane 15 into rows 1 and 3
// and then lane 31 into rows 2 and 3 leaves the wave's result in lane 63,
// which is read as a scalar.  Each step is one in-place DPP instruction: it
// writes only the lanes whose source lane is in range and whose row is
// enabled, the others keep their value.  A vector result read through DPP
// needs two wait states, hence the s_nop before each step.
#define DET_DPP_STEPS(OP)                                                   \
  "s_nop 1\n\t" OP " %0, %0, %0 row_shr:1 row_mask:0xf bank_mask:0xf\n\t"    \
  "s_nop 1\n\t" OP " %0, %0, %0 row_shr:2 row_mask:0xf bank_mask:0xf\n\t"    \
  "s_nop 1\n\t" OP " %0, %0, %0 row_shr:4 row_mask:0xf bank_mask:0xf\n\t"    \
  "s_nop 1\n\t" OP " %0, %0, %0 row_shr:8 row_mask:0xf bank_mask:0xf\n\t"    \
  "s_nop 1\n\t" OP " %0, %0, %0 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t" \
  "s_nop 1\n\t" OP " %0, %0, %0 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t" \
  "s_nop 1"

__device__ __forceinline__ int det_wave_max(int x) {
  asm volatile(DET_DPP_STEPS("v_max_i32_dpp") : "+v"(x));
  return __builtin_amdgcn_readlane(x, 63);
}

__device__ __forceinline__ int det_wave_min(int x) {
  asm volatile(DET_DPP_STEPS("v_min_i32_dpp") : "+v"(x));
  return __builtin_amdgcn_readlane(x, 63);
}

__device__ __forceinline__ float det_wave_maxf(float x) {
  asm volatile(DET_DPP_STEPS("v_max_f32_dpp") : "+v"(x));
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

// Lanes whose DPP source is out of range or whose row is masked take `old`.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ int det_dpp(int old, int x) {
  return __builtin_amdgcn_update_dpp(old, x, CTRL, ROWMASK, 0xf, false);
}

template <int CTRL, int ROWMASK>
__device__ __forceinline__ double det_dpp_d(double x) {
  const int lo = det_dpp<CTRL, ROWMASK>(0, __double2loint(x));
  const int hi = det_dpp<CTRL, ROWMASK>(0, __double2hiint(x));
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double det_wave_sum(double x) {
  x += det_dpp_d<0x111, 0xf>(x);
  x += det_dpp_d<0x112, 0xf>(x);
  x += det_dpp_d<0x114, 0xf>(x);
  x += det_dpp_d<0x118, 0xf>(x);
  x += det_dpp_d<0x142, 0xa>(x);
  x += det_dpp_d<0x143, 0xc>(x);
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), 63),
                          __builtin_amdgcn_readlane(__double2loint(x), 63));
}

// The lane one higher's copy of x (DPP wave shift); lane 63 gets `old`.
__device__ __forceinline__ int det_next_lane(int old, int x) {
  return __builtin_amdgcn_update_dpp(old, x, 0x130, 0xf, 0xf, false);
}

// Float series.  v[0 .. L) holds the lane's run; the look-ahead v[L .. L + 32)
// is filled from the lanes above (position L + k of this lane is position k
// of the next lane), lane 63's from -inf.  Positions past the end of the
// series must hold -inf, so a window that reaches them sums to -inf and
// never wins.  Boxcar sums by doubling, B_2w(i) = B_w(i) + B_w(i + w).
// owned: the lane's starts belong to this tile; lim: starts i < lim hold
// samples of the series (MASK = false when lim >= L).  Per width the lane's
// largest sum and its first start (-inf and -1 when none).
template <int L, bool MASK>
__device__ __forceinline__ void det_lane_f32(float* v, bool owned, int lim, float* bval, int* bidx, double& s1,
                                             double& s2) {
#pragma unroll
  for (int j = L; j < L + kDetLook; ++j)
    v[j] = __int_as_float(det_next_lane(__float_as_int(-INFINITY), __float_as_int(v[j - L])));
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

// Integer series (uint8 input: exact sums).  v[0 .. L) holds the lane's run
// scaled by 2^IB (y << IB).  With E(j) the sum of the first j values from the
// lane's first start on (its own prefix for j <= L, then E(j) = E(L) + the
// next lane's E(j - L)), the key
//   E(i + w) - (E(i) - (L - 1 - i)) = (B_w(i) << IB) + (L - 1 - i)
// orders windows by sum and, for equal sums, the earlier start first, so one
// integer max per window finds both.  Starts past the series end get
// E(i) := 2^30 and entries past the end -2^30, which makes every key that
// touches them negative (the host limits sums to keep |E| < 2^30); lanes
// whose starts lie outside the tile's owned range report no window.  One pass in order of j: E(j) closes the window of width w
// that starts at j - w, so only the L start terms and the entries the next
// look-ahead step reads stay live.  Per width the lane's largest key
// (negative: none).
template <int L, int IB, bool MASK>
__device__ __forceinline__ void det_lane_int(const int* v, bool owned, int lim, bool s2_u32, int* key, double& s1,
                                             double& s2) {
  int s1i = 0;
  if (s2_u32) {
    // every y < 2^24 and the lane's sum of squares < 2^32 (the host checks)
    uint32_t q = 0;
#pragma unroll
    for (int i = 0; i < L; ++i) {
      const uint32_t y = (!MASK || i < lim) ? (uint32_t)(v[i] >> IB) : 0u;
      s1i += (int)y;
      q += __umul24(y, y);
    }
    s2 = (double)q;
  } else {
    s2 = 0.0;
#pragma unroll
    for (int i = 0; i < L; ++i) {
      const int y = (!MASK || i < lim) ? v[i] >> IB : 0;
      s1i += y;
      const double yd = (double)y;
      s2 = fma(yd, yd, s2);
    }
  }
  s1 = owned ? (double)s1i : 0.0;
  if (!owned) s2 = 0.0;
#pragma unroll
  for (int k = 0; k < kDetNW; ++k) key[k] = INT32_MIN;
  int E[L + kDetLook];
  int Q[L];
  E[0] = 0;
#pragma unroll
  for (int j = 0; j < L + kDetLook; ++j) {
    if (j > 0) {
      const int e = j <= L ? E[j - 1] + v[j - 1] : E[L] + det_next_lane(0, E[j - L]);
      E[j] = (MASK && j > lim) ? -(1 << 30) : e;
    }
    if (j < L) Q[j] = (!MASK || j < lim) ? E[j] - (L - 1 - j) : (1 << 30);
#pragma unroll
    for (int k = 0; k < kDetNW; ++k) {
      const int i = j - (1 << k);
      if (i >= 0 && i < L) key[k] = max(key[k], E[j] - Q[i]);
    }
  }
  // starts outside the tile's owned range: no window
#pragma unroll
  for (int k = 0; k < kDetNW; ++k) key[k] = owned ? key[k] : INT32_MIN;
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

// gfx950 kernels of the single-pulse search that do not dedisperse: the
// search over stored rows (the unfused path) and the merge of the per-tile
// records into one result per series.  The definition of the search and the
// tile records are in detect_dev.h.
#include <math.h>

#include "detect_dev.h"
#include "internal.h"

namespace dd {

// One wave per row and time tile; each lane loads its run of kDetRowsRun
// starts (-inf past the row end) and takes the look-ahead from the lanes
// above.
template <bool I32>
__global__ __launch_bounds__(256) void detect_rows_kernel(const void* __restrict__ rows, int64_t stride, int nrows,
                                                          int nsamp, int ntiles, DetRec* __restrict__ recs) {
  constexpr int L = kDetRowsRun;
  constexpr int ST = kDetRowsTile;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tt = blockIdx.x % ntiles;
  const int r = (blockIdx.x / ntiles) * 4 + wave;
  if (r >= nrows) return;  // whole waves; no block barrier follows
  const int t0 = tt * kDetRowsStep;
  const int nvalid = min(ST, nsamp - t0);
  const int pos0 = L * lane;
  const int lim = nvalid - pos0;    // the lane's starts that hold samples
  const int avail = nsamp - t0 - pos0;  // samples of the row from the lane's first start on
  float v[L + kDetLook];
  if (I32) {
    const int32_t* src = static_cast<const int32_t*>(rows) + (int64_t)r * stride + t0 + pos0;
    if (avail >= L) {
#pragma unroll
      for (int i4 = 0; i4 < L / 4; ++i4) {
        const int4 x = reinterpret_cast<const int4*>(src)[i4];
        v[4 * i4 + 0] = (float)x.x;
        v[4 * i4 + 1] = (float)x.y;
        v[4 * i4 + 2] = (float)x.z;
        v[4 * i4 + 3] = (float)x.w;
      }
    } else {
#pragma unroll
      for (int i = 0; i < L; ++i) v[i] = i < avail ? (float)src[i] : -INFINITY;
    }
  } else {
    const float* src = static_cast<const float*>(rows) + (int64_t)r * stride + t0 + pos0;
    if (avail >= L) {
#pragma unroll
      for (int i4 = 0; i4 < L / 4; ++i4) {
        const float4 x = reinterpret_cast<const float4*>(src)[i4];
        v[4 * i4 + 0] = x.x;
        v[4 * i4 + 1] = x.y;
        v[4 * i4 + 2] = x.z;
        v[4 * i4 + 3] = x.w;
      }
    } else {
#pragma unroll
      for (int i = 0; i < L; ++i) v[i] = i < avail ? src[i] : -INFINITY;
    }
  }
  float bval[kDetNW];
  int bidx[kDetNW];
  double s1, s2;
  const bool owned = pos0 < kDetRowsStep;
  if (nvalid < ST)
    det_lane_f32<L, true>(v, owned, lim, bval, bidx, s1, s2);
  else
    det_lane_f32<L, false>(v, owned, lim, bval, bidx, s1, s2);
  det_commit_f32(recs + (int64_t)r * ntiles + tt, bval, bidx, s1, s2, pos0, t0);
}

// One wave per series: lane k takes tiles k, k + 64, ... in order (keeping
// the first of equal sums), then the lanes merge (largest sum, then smallest
// start), the moments are summed in a fixed order, and lane 0 scores the
// widths:  S/N_w = (max B_w - w mean) / (std sqrt(w)), 0 when std == 0.
template <bool INT_VALS>
__global__ __launch_bounds__(256) void det_finish_kernel(const DetRec* __restrict__ recs, int nseries, int ntiles,
                                                         int nsamp, int nwidth, double* __restrict__ snr,
                                                         int32_t* __restrict__ width, int32_t* __restrict__ start,
                                                         double* __restrict__ mean, double* __restrict__ stdv) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int sidx = blockIdx.x * 4 + wave;
  if (sidx >= nseries) return;
  const DetRec* R = recs + (int64_t)sidx * ntiles;
  float bf[kDetNW];
  int bi[kDetNW], bp[kDetNW];
#pragma unroll
  for (int k = 0; k < kDetNW; ++k) {
    bf[k] = -INFINITY;
    bi[k] = INT32_MIN;
    bp[k] = -1;
  }
  double s1 = 0.0, s2 = 0.0;
  for (int t = lane; t < ntiles; t += 64) {
    const DetRec rec = R[t];
#pragma unroll
    for (int k = 0; k < kDetNW; ++k) {
      if (rec.pos[k] < 0) continue;
      if (INT_VALS) {
        if (bp[k] < 0 || rec.val[k] > bi[k]) {
          bi[k] = rec.val[k];
          bp[k] = rec.pos[k];
        }
      } else {
        const float f = __int_as_float(rec.val[k]);
        if (bp[k] < 0 || f > bf[k]) {
          bf[k] = f;
          bp[k] = rec.pos[k];
        }
      }
    }
    s1 += rec.s1;
    s2 += rec.s2;
  }
  s1 = det_wave_sum(s1);
  s2 = det_wave_sum(s2);
  double m[kDetNW];
  int p[kDetNW];
#pragma unroll
  for (int k = 0; k < kDetNW; ++k) {
    if (INT_VALS) {
      const int mm = det_wave_max(bp[k] >= 0 ? bi[k] : INT32_MIN);
      p[k] = det_wave_min(bp[k] >= 0 && bi[k] == mm ? bp[k] : INT32_MAX);
      m[k] = (double)mm;
    } else {
      const float mm = det_wave_maxf(bp[k] >= 0 ? bf[k] : -INFINITY);
      p[k] = det_wave_min(bp[k] >= 0 && bf[k] == mm ? bp[k] : INT32_MAX);
      m[k] = (double)mm;
    }
  }
  if (lane != 0) return;
  const double n = (double)nsamp;
  const double mu = s1 / n;
  double var = (s2 - s1 * mu) / n;
  if (!(var > 0.0)) var = 0.0;
  const double sd = sqrt(var);
  double best = 0.0;
  int bw = -1, bs = -1;
  for (int k = 0; k < nwidth && k < kDetNW; ++k) {
    if (p[k] == INT32_MAX) continue;  // no window of this width fits
    const double w = (double)(1 << k);
    const double sn = sd > 0.0 ? (m[k] - w * mu) / (sd * sqrt(w)) : 0.0;
    if (bw < 0 || sn > best) {
      best = sn;
      bw = 1 << k;
      bs = p[k];
    }
  }
  snr[sidx] = best;
  width[sidx] = bw;
  start[sidx] = bs;
  if (mean) mean[sidx] = mu;
  if (stdv) stdv[sidx] = sd;
}

hipError_t launch_detect_rows(const void* rows, bool i32, int64_t stride, int nrows, int nsamp, int ntiles,
                              DetRec* recs, hipStream_t s) {
  const int64_t nblk = (int64_t)ntiles * ((nrows + 3) / 4);
  if (nrows < 1 || ntiles < 1 || nblk > 0x7fffffff) return hipErrorInvalidConfiguration;
  const dim3 grid((unsigned)nblk);
  if (i32)
    hipLaunchKernelGGL((detect_rows_kernel<true>), grid, dim3(256), 0, s, rows, stride, nrows, nsamp, ntiles, recs);
  else
    hipLaunchKernelGGL((detect_rows_kernel<false>), grid, dim3(256), 0, s, rows, stride, nrows, nsamp, ntiles, recs);
  return hipGetLastError();
}

hipError_t launch_det_finish(const DetRec* recs, bool int_vals, int nseries, int ntiles, int nsamp, int nwidth,
                             double* snr, int32_t* width, int32_t* start, double* mean, double* stdv, hipStream_t s) {
  if (nseries < 1 || ntiles < 1) return hipErrorInvalidConfiguration;
  const dim3 grid((unsigned)((nseries + 3) / 4));
  if (int_vals)
    hipLaunchKernelGGL((det_finish_kernel<true>), grid, dim3(256), 0, s, recs, nseries, ntiles, nsamp, nwidth, snr,
                       width, start, mean, stdv);
  else
    hipLaunchKernelGGL((det_finish_kernel<false>), grid, dim3(256), 0, s, recs, nseries, ntiles, nsamp, nwidth, snr,
                       width, start, mean, stdv);
  return hipGetLastError();
}

}  // namespace dd

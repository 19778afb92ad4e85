// gfx950 kernels for brute-force incoherent dedispersion.
//
// Forward map (Sclocco et al., arXiv 1601.01165, Section 2.1, Algorithm 1):
//   out[b][r][t] = sum over input rows c, ascending, of w[c] * in[b][c][t + delta(r, c)]
// with r a DM trial and c a channel.  The adjoint is the same map with the
// roles swapped (r a channel, c a DM trial, delay' = pad - delay, input rows
// read as zero outside the output range), so one tile engine serves both.
//
// Parallel structure (Section 2.2): each work item owns (output row, time)
// pairs; a block owns a tile of output rows x time samples, so the input rows
// it needs are shared by all its rows (the paper's DM-direction reuse through
// local memory).  On gfx950:
//   * a block stages, for cc input rows at a time, the window
//     [t0 + stage_base(c), t0 + stage_base(c) + stage_len(c)) of each row into
//     LDS with 16-byte loads (all 16-byte aligned);
//   * each wave owns dpw output rows and 64*tp samples, each lane tp
//     consecutive samples.  Per input row the lane copies its window of
//     samples from LDS into registers once (16-byte LDS reads) and every one
//     of its dpw rows adds tp window registers, selected through VGPR index
//     mode with the row's delay offset (see gen_win_asm.py).  One LDS byte
//     thus feeds several adds, which is what keeps the add units busy: an LDS
//     read per add would cap the rate at the LDS bandwidth.
//   * blocks are remapped so that the blocks of one time tile run on the same
//     XCD, sharing that XCD's L2 for the input window.
//   * accumulation order per output is ascending input row with one rounding
//     per term, the order of Algorithm 1, so the FP32 results are those of a
//     sequential FP32 loop.
#include <algorithm>

#include "detect_dev.h"
#include "internal.h"

namespace dd {

typedef float v16f __attribute__((ext_vector_type(16)));
#include "win_asm.inc"

#define LDS_AS __attribute__((address_space(3)))

// Blocks are dispatched round-robin over the 8 XCDs.  Give each XCD a
// contiguous range of work items (time-major, output rows fastest).
__device__ __forceinline__ int xcd_remap(int L, int N) {
  const int q = N >> 3, r = N & 7;
  const int x = L & 7, k = L >> 3;
  return (x < r) ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// The lane index, recomputed where it is used: the asm keeps the compiler
// from hoisting lane-dependent offsets out of loops and holding them in
// registers the small register windows cannot spare.
__device__ __forceinline__ int lane_fresh() {
  int l;
  asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(l));
  return l;
}

// A pointer the compiler must keep in SGPRs (its value is wave-uniform).
template <typename T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return reinterpret_cast<T*>(((uint64_t)hi << 32) | lo);
}

// Wave-uniform scalar loads (wait included) of a table entry and a weight.
typedef int32_t ent2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ ent2_t sload_entry2(const int32_t* p) {
  ent2_t r;
  asm volatile("s_load_dwordx2 %0, %1, 0x0\n\ts_waitcnt lgkmcnt(0)" : "=s"(r) : "s"(p));
  return r;
}
__device__ __forceinline__ ent4_t sload_entry4(const int32_t* p) {
  ent4_t r;
  asm volatile("s_load_dwordx4 %0, %1, 0x0\n\ts_waitcnt lgkmcnt(0)" : "=s"(r) : "s"(p));
  return r;
}
__device__ __forceinline__ ent8_t sload_entry8(const int32_t* p) {
  ent8_t r;
  asm volatile("s_load_dwordx8 %0, %1, 0x0\n\ts_waitcnt lgkmcnt(0)" : "=s"(r) : "s"(p));
  return r;
}
template <typename E>
__device__ __forceinline__ E sload_entry_t(const int32_t* p);
template <>
__device__ __forceinline__ ent4_t sload_entry_t<ent4_t>(const int32_t* p) {
  return sload_entry4(p);
}
template <>
__device__ __forceinline__ ent8_t sload_entry_t<ent8_t>(const int32_t* p) {
  return sload_entry8(p);
}
template <>
__device__ __forceinline__ ent16_t sload_entry_t<ent16_t>(const int32_t* p) {
  ent16_t r;
  asm volatile("s_load_dwordx16 %0, %1, 0x0\n\ts_waitcnt lgkmcnt(0)" : "=s"(r) : "s"(p));
  return r;
}
// Scalar buffer loads (reads past the resource's range return zero), wait included.
__device__ __forceinline__ ent8_t sbload8(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
  ent8_t r;
  asm volatile("s_buffer_load_dwordx8 %0, %1, %2\n\ts_waitcnt lgkmcnt(0)" : "=s"(r) : "s"(rs), "s"(off));
  return r;
}
__device__ __forceinline__ ent16_t sbload16(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
  ent16_t r;
  asm volatile("s_buffer_load_dwordx16 %0, %1, %2\n\ts_waitcnt lgkmcnt(0)" : "=s"(r) : "s"(rs), "s"(off));
  return r;
}
__device__ __forceinline__ ent4_t sbload4(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
  ent4_t r;
  asm volatile("s_buffer_load_dwordx4 %0, %1, %2\n\ts_waitcnt lgkmcnt(0)" : "=s"(r) : "s"(rs), "s"(off));
  return r;
}
template <typename E>
__device__ __forceinline__ E sbload_t(__amdgpu_buffer_rsrc_t rs, uint32_t off);
template <>
__device__ __forceinline__ ent4_t sbload_t<ent4_t>(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
  return sbload4(rs, off);
}
template <>
__device__ __forceinline__ ent8_t sbload_t<ent8_t>(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
  return sbload8(rs, off);
}
template <>
__device__ __forceinline__ ent16_t sbload_t<ent16_t>(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
  return sbload16(rs, off);
}
__device__ __forceinline__ float sload_f32(const float* p) {
  float r;
  asm volatile("s_load_dword %0, %1, 0x0\n\ts_waitcnt lgkmcnt(0)" : "=s"(r) : "s"(p));
  return r;
}

// ---------------------------------------------------------------------------
// FP32 tile engine with the register window.
// ---------------------------------------------------------------------------

// Stage input rows [c0, c0 + ncc) into LDS.  Wave w copies rows w, w + NWAVE, ...
// With weights each staged sample is the FP32 product w[c] * x (the weight is
// a gain on the channel's data), so the sums themselves are plain adds.
template <int NWAVE, int ROWCAP, bool WEIGHTED>
__device__ __forceinline__ void stage_f32(int wave, float4* lds4, const float* in, const TileArgs& a, const int32_t* blk,
                                          int c0, int ncc, int t0) {
  const int lane = lane_fresh();
  for (int cl = wave; cl < ncc; cl += NWAVE) {
    const int sb = blk[2 * (c0 + cl)];
    const int sl = blk[2 * (c0 + cl) + 1];
    const float wc = WEIGHTED ? a.w_in[c0 + cl] : 1.f;
    const float* src = in + (int64_t)(c0 + cl) * a.in_stride + a.in_shift;
    const int u0 = t0 + sb;
    float4* dst = lds4 + cl * (ROWCAP / 4);
    const int nv = sl >> 2;
#pragma unroll 4
    for (int v = lane; v < nv; v += 64) {
      const int u = u0 + 4 * v;
      float4 x;
      if (u >= a.in_lo && u + 4 <= a.in_hi) {
        x = *reinterpret_cast<const float4*>(src + u);
      } else {
        x.x = (u + 0 >= a.in_lo && u + 0 < a.in_hi) ? src[u + 0] : 0.f;
        x.y = (u + 1 >= a.in_lo && u + 1 < a.in_hi) ? src[u + 1] : 0.f;
        x.z = (u + 2 >= a.in_lo && u + 2 < a.in_hi) ? src[u + 2] : 0.f;
        x.w = (u + 3 >= a.in_lo && u + 3 < a.in_hi) ? src[u + 3] : 0.f;
      }
      if (WEIGHTED) {
        x.x = wc * x.x;
        x.y = wc * x.y;
        x.z = wc * x.z;
        x.w = wc * x.w;
      }
      dst[v] = x;
    }
  }
}

// Asynchronous form: 16-byte buffer loads that write LDS directly (no VGPR
// round trip), completed by `s_waitcnt vmcnt(0)`.  Each row gets a buffer
// resource covering its valid range, so positions outside it read as zero
// without a branch (the adjoint relies on this for its virtual padding).
template <int NWAVE, int ROWCAP>
__device__ __forceinline__ void stage_f32_async(int wave, float4* lds4, const float* in, const TileArgs& a,
                                                const int32_t* blk, int c0, int ncc, int t0) {
  // whole 64-lane loads stay inside the row's LDS slot
  static_assert(ROWCAP % 256 == 0, "LDS rows hold a multiple of 64 float4");
  const int lane = lane_fresh();
  for (int cl = wave; cl < ncc; cl += NWAVE) {
    const ent2_t bl = sload_entry2(blk + 2 * (c0 + cl));
    const int sb = bl[0];
    const int sl = bl[1];
    const float* base = in + (int64_t)(c0 + cl) * a.in_stride + a.in_lo + a.in_shift;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (a.in_hi - a.in_lo) * 4, 0x00020000);
    const int u0 = t0 + sb - a.in_lo;
    const int nv = sl >> 2;
    for (int v0 = 0; v0 < nv; v0 += 64) {
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (LDS_AS void*)(lds4 + cl * (ROWCAP / 4) + v0), 16,
                                               (u0 + 4 * (v0 + lane)) * 4, 0, 0, 0);
    }
  }
}

// Entries {stage base, stage length} of the rows wave w stages for the pass
// starting at input row c0 (rows w, w + NWAVE, ...): lane 2k holds the base
// of the wave's k-th row, lane 2k + 1 its length and lane 32 + k its weight
// (float bits; weighted kernels only).  A vector load, issued a pass ahead:
// the per-pass wait for the staged rows covers it, so staging never stalls on
// a scalar-cache miss.
template <int NWAVE, int CC>
__device__ __forceinline__ int32_t stage_entries(int wave, const int32_t* blk, const float* w, int rows_in, int c0) {
  constexpr int RPW = (CC + NWAVE - 1) / NWAVE;
  static_assert(2 * RPW <= 32, "entries and weights share one VGPR");
  const int lane = lane_fresh();
  if (lane < 32) {
    const int cl = wave + (lane >> 1) * NWAVE;
    if (lane < 2 * RPW && cl < CC && c0 + cl < rows_in) return blk[2 * (c0 + cl) + (lane & 1)];
  } else if (w) {
    const int cl = wave + (lane - 32) * NWAVE;
    if (lane - 32 < RPW && cl < CC && c0 + cl < rows_in) return __float_as_int(w[c0 + cl]);
  }
  return 0;
}

// Weighted kernels, asynchronous staging: once this wave's rows of a pass
// have landed, scale them in place by their channel's weight (FP32 product,
// the weight being a gain on the data), before the barrier that publishes the
// pass.  `ent` holds the pass's entries and weights (stage_entries).
template <int NWAVE, int ROWCAP>
__device__ __forceinline__ void scale_rows(int wave, float4* lds4, int32_t ent, int ncc) {
  for (int k = 0, cl = wave; cl < ncc; ++k, cl += NWAVE) {
    const int lane = lane_fresh();
    const int sl = __builtin_amdgcn_readlane(ent, 2 * k + 1);
    const float wc = __int_as_float(__builtin_amdgcn_readlane(ent, 32 + k));
    float4* row = lds4 + cl * (ROWCAP / 4);
    for (int v = lane; v < (sl >> 2); v += 64) {
      float4 x = row[v];
      x.x = wc * x.x;
      x.y = wc * x.y;
      x.z = wc * x.z;
      x.w = wc * x.w;
      row[v] = x;
    }
  }
}

// stage_f32_async with the entries from stage_entries (no scalar loads).
template <int NWAVE, int ROWCAP>
__device__ __forceinline__ void stage_f32_async_pre(int wave, float4* lds4, const float* in, const TileArgs& a, int32_t ent,
                                                    int c0, int ncc, int t0) {
  static_assert(ROWCAP % 256 == 0, "LDS rows hold a multiple of 64 float4");
  for (int k = 0, cl = wave; cl < ncc; ++k, cl += NWAVE) {
    const int lane = lane_fresh();
    const int sb = __builtin_amdgcn_readlane(ent, 2 * k);
    const int sl = __builtin_amdgcn_readlane(ent, 2 * k + 1);
    const float* base = in + (int64_t)(c0 + cl) * a.in_stride + a.in_lo + a.in_shift;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (a.in_hi - a.in_lo) * 4, 0x00020000);
    const int u0 = t0 + sb - a.in_lo;
    const int nv = sl >> 2;
    for (int v0 = 0; v0 < nv; v0 += 64) {
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (LDS_AS void*)(lds4 + cl * (ROWCAP / 4) + v0), 16,
                                               (u0 + 4 * (v0 + lane)) * 4, 0, 0, 0);
    }
  }
}

// After the asynchronous loads of a pass have landed: rewrite the one 16-byte
// chunk per row that straddles the end of the valid range (valid elements
// from memory, the rest zero), whatever the hardware returned for it.  Only
// the adjoint's range can end off a 16-byte boundary.
template <int NWAVE, int ROWCAP>
__device__ __forceinline__ void fix_tail_async(int wave, float4* lds4, const float* in, const TileArgs& a,
                                               const int32_t* blk, int c0, int ncc, int t0) {
  if ((a.in_hi & 3) == 0) return;
  const int lane = lane_fresh();
  const int hi4 = a.in_hi & ~3;
  for (int cl = wave; cl < ncc; cl += NWAVE) {
    const ent2_t bl = sload_entry2(blk + 2 * (c0 + cl));
    const int v = (hi4 - (t0 + bl[0])) >> 2;
    if (lane == 0 && v >= 0 && 4 * v < bl[1]) {
      const float* src = in + (int64_t)(c0 + cl) * a.in_stride + a.in_shift;
      float4 x;
      x.x = src[hi4];
      x.y = (hi4 + 1 < a.in_hi) ? src[hi4 + 1] : 0.f;
      x.z = (hi4 + 2 < a.in_hi) ? src[hi4 + 2] : 0.f;
      x.w = 0.f;
      lds4[cl * (ROWCAP / 4) + v] = x;
    }
  }
}

// Store a finished tile (adjoint: scaled by w_out, with the wave's partial
// sums of x * G for the weight gradient).
template <int TP, int DPW, int NWAVE, bool ADJ>
__device__ __forceinline__ void win_store(int wave, const TileArgs& a, const v16f* acc, int tt, int rt, int beam) {
  constexpr int DT = NWAVE * DPW;
  const int t0 = tt * 64 * TP;
  const int lane = lane_fresh();
  float* out = static_cast<float*>(a.out);
  const int tl = t0 + lane * TP;
#pragma unroll
  for (int jj = 0; jj < DPW; ++jj) {
    const int r = rt * DT + wave * DPW + jj;
    if (r >= a.rows_out) break;
    const float scale = (ADJ && a.w_out) ? a.w_out[r] : 1.f;
    double gw = 0.0;
    const float* xrow = nullptr;
    if (ADJ && a.partial) xrow = a.x + (int64_t)beam * a.x_beam_stride + (int64_t)r * a.x_stride;
    float* orow = out ? out + (int64_t)beam * a.out_beam_stride + (int64_t)r * a.out_stride : nullptr;
#pragma unroll
    for (int i4 = 0; i4 < TP / 4; ++i4) {
      const int e0 = jj * TP + 4 * i4;
      float4 v;
      v.x = acc[(e0 + 0) / 16][(e0 + 0) % 16];
      v.y = acc[(e0 + 1) / 16][(e0 + 1) % 16];
      v.z = acc[(e0 + 2) / 16][(e0 + 2) % 16];
      v.w = acc[(e0 + 3) / 16][(e0 + 3) % 16];
      const int t = tl + 4 * i4;
      if (ADJ && xrow) {
        if (t + 4 <= a.nout) {
          const float4 xv = *reinterpret_cast<const float4*>(xrow + t);
          gw += (double)xv.x * (double)v.x;
          gw += (double)xv.y * (double)v.y;
          gw += (double)xv.z * (double)v.z;
          gw += (double)xv.w * (double)v.w;
        } else {
          if (t + 0 < a.nout) gw += (double)xrow[t + 0] * (double)v.x;
          if (t + 1 < a.nout) gw += (double)xrow[t + 1] * (double)v.y;
          if (t + 2 < a.nout) gw += (double)xrow[t + 2] * (double)v.z;
          if (t + 3 < a.nout) gw += (double)xrow[t + 3] * (double)v.w;
        }
      }
      if (orow) {
        if (ADJ) {
          v.x *= scale;
          v.y *= scale;
          v.z *= scale;
          v.w *= scale;
        }
        if (t + 4 <= a.nout) {
          *reinterpret_cast<float4*>(orow + t) = v;
        } else {
          if (t + 0 < a.nout) orow[t + 0] = v.x;
          if (t + 1 < a.nout) orow[t + 1] = v.y;
          if (t + 2 < a.nout) orow[t + 2] = v.z;
          if (t + 3 < a.nout) orow[t + 3] = v.w;
        }
      }
    }
    if (ADJ && xrow) {
      // Fixed-order reduction over the 64 lanes of the wave.
#pragma unroll
      for (int m = 32; m >= 1; m >>= 1) gw += __shfl_xor(gw, m, 64);
      if (lane == 0) a.partial[((size_t)beam * a.n_time_tiles + tt) * a.rows_out + r] = gw;
    }
  }
}


// Single-pulse search in place of the store: each lane's TP consecutive
// samples of a row are its run of window starts; the look-ahead comes from
// the lanes above (DPP), so the rows never leave the registers.  Samples past
// the series end read as -inf.
template <int TP, int DPW, int NWAVE>
__device__ __forceinline__ void det_store_f32(int wave, const TileArgs& a, const v16f* acc, int tt, int rt, int beam, int t0) {
  constexpr int ST = 64 * TP;
  constexpr int DT = NWAVE * DPW;
  const int lane = lane_fresh();
  const int nvalid = min(ST, a.det_nsamp - t0);
  const int pos0 = TP * lane;
  const bool owned = pos0 < a.tile_step;
  const int lim = nvalid - pos0;
#pragma unroll
  for (int jj = 0; jj < DPW; ++jj) {
    const int r = rt * DT + wave * DPW + jj;
    if (r >= a.rows_out) break;
    float v[TP + kDetLook];
#pragma unroll
    for (int i = 0; i < TP; ++i) v[i] = acc[(jj * TP + i) / 16][(jj * TP + i) % 16];
    float bval[kDetNW];
    int bidx[kDetNW];
    double s1, s2;
    if (nvalid < ST) {
#pragma unroll
      for (int i = 0; i < TP; ++i) v[i] = i < lim ? v[i] : -INFINITY;
      det_lane_f32<TP, true>(v, owned, lim, bval, bidx, s1, s2);
    } else {
      det_lane_f32<TP, false>(v, owned, lim, bval, bidx, s1, s2);
    }
    det_commit_f32(a.det + ((int64_t)beam * a.rows_out + r) * a.n_time_tiles + tt, bval, bidx, s1, s2, pos0, t0);
  }
}

// NBUF = 1: synchronous staging through registers, one LDS buffer.
// NBUF = 2: asynchronous LDS loads into two buffers; the rows of pass p + 1
// are in flight while pass p is summed.
template <int TP, int DPW, int NWAVE, int NWIN, int CC, int ROWCAP, int NBUF, bool WEIGHTED, bool ADJ,
          bool DET = false, int JMP = 0>
__device__ __forceinline__ void win_tile(int wave, const TileArgs& a, int tt, int rt, int beam, float4* lds4) {
  constexpr int ST = 64 * TP;
  constexpr int DT = NWAVE * DPW;
  constexpr int NACC = TP * DPW / 16;
  constexpr int WI = EntT<DPW>::ints;
  tt = __builtin_amdgcn_readfirstlane(tt);
  rt = __builtin_amdgcn_readfirstlane(rt);
  const int t0 = DET ? tt * a.tile_step : tt * ST;
  const int wt = rt * NWAVE + wave;
  const float* in = static_cast<const float*>(a.in) + (int64_t)beam * a.in_beam_stride;
  const int32_t* __restrict__ blk = uniform_ptr(a.blk + (size_t)rt * a.rows_in * 2);
  const int32_t* __restrict__ wav = uniform_ptr(a.wav + (size_t)wt * a.rows_in * WI);
  const float* w_in = WEIGHTED ? a.w_in : nullptr;
  const uint32_t lds_base = (uint32_t)(uintptr_t)(LDS_AS float4*)(lds4);

  v16f acc[NACC];
#pragma unroll
  for (int q = 0; q < NACC; ++q) acc[q] = (v16f)(0.f);

  // The wave's table entry of the current input row lives in SGPRs; each
  // step fetches the next row's through a buffer resource (reads past the
  // last row return zero), advancing the byte offset itself.  Weights were
  // applied when the rows were staged, so the steps only add.
  typedef typename EntT<DPW>::type E;
  const __amdgpu_buffer_rsrc_t trs =
      __builtin_amdgcn_make_buffer_rsrc((void*)wav, (short)0, a.rows_in * WI * 4, 0x00020000);
  const __amdgpu_buffer_rsrc_t wrs = __builtin_amdgcn_make_buffer_rsrc(nullptr, (short)0, 0, 0x00020000);
  uint32_t toff = WI * 4, woff = 4;
  E ea = sload_entry_t<E>(wav), eb;
  float wa = 0.f, wb = 0.f;
  const int npass = (a.rows_in + CC - 1) / CC;
  int32_t stg = 0;      // staging entries (and weights) of the next pass (NBUF = 2)
  int32_t stg_cur = 0;  // those of the pass being summed (weighted kernels)
  // Adjoint: the input rows (DM trials) of the passes at either end may stage
  // windows that all miss the valid samples [in_lo, in_hi) of the output
  // gradient (only zeros would be added); the tile runs from its first to
  // its last pass that meets them (all passes when no span table is given).
  int p_lo = 0, p_hi = npass - 1;
  if constexpr (ADJ) {
    if (a.span) {
      const int32_t* sp = uniform_ptr(a.span + (size_t)rt * npass * 2);
      auto live = [&](int q) {
        const ent2_t e = sload_entry2(sp + 2 * q);
        return t0 + e[0] < a.in_hi && t0 + e[1] > a.in_lo;
      };
      while (p_lo <= p_hi && !live(p_lo)) ++p_lo;
      while (p_hi > p_lo && !live(p_hi)) --p_hi;
      if (p_lo > 0) {
        toff = (uint32_t)((p_lo * CC + 1) * WI * 4);
        ea = sbload_t<E>(trs, (uint32_t)(p_lo * CC * WI * 4));
      }
    }
  }
  if (NBUF == 2 && p_lo <= p_hi) {
    __syncthreads();  // a previous tile of this block is done with the LDS rows
    stage_f32_async<NWAVE, ROWCAP>(wave, lds4 + (p_lo & 1) * CC * (ROWCAP / 4), in, a, blk, p_lo * CC,
                                   min(CC, a.rows_in - p_lo * CC), t0);
    if (WEIGHTED) stg_cur = stage_entries<NWAVE, CC>(wave, blk, w_in, a.rows_in, p_lo * CC);
    if (p_lo < p_hi) stg = stage_entries<NWAVE, CC>(wave, blk, w_in, a.rows_in, (p_lo + 1) * CC);
  }
  for (int p = p_lo; p <= p_hi; ++p) {
    const int c0 = p * CC;
    const int ncc = min(CC, a.rows_in - c0);
    const int bufrow = NBUF == 2 ? (p & 1) * CC : 0;
    if (NBUF == 1) {
      __syncthreads();  // the previous pass is done with the LDS rows
      stage_f32<NWAVE, ROWCAP, WEIGHTED>(wave, lds4, in, a, blk, c0, ncc, t0);
      __syncthreads();
    } else {
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this wave's rows of pass p have landed
      fix_tail_async<NWAVE, ROWCAP>(wave, lds4 + (p & 1) * CC * (ROWCAP / 4), in, a, blk, c0, ncc, t0);
      if (WEIGHTED) scale_rows<NWAVE, ROWCAP>(wave, lds4 + (p & 1) * CC * (ROWCAP / 4), stg_cur, ncc);
      __syncthreads();  // every wave's have; every wave is done with pass p - 1
      if (p + 1 <= p_hi)
        stage_f32_async_pre<NWAVE, ROWCAP>(wave, lds4 + ((p + 1) & 1) * CC * (ROWCAP / 4), in, a, stg, c0 + CC,
                                           min(CC, a.rows_in - c0 - CC), t0);
      if (WEIGHTED) stg_cur = stg;
      if (p + 2 <= p_hi) stg = stage_entries<NWAVE, CC>(wave, blk, w_in, a.rows_in, c0 + 2 * CC);
    }
    // LDS byte address of this lane's window in the pass's first row slot
    uint32_t row = lds_base + (uint32_t)(lane_fresh() * TP * 4) + (uint32_t)(bufrow * ROWCAP * 4);
    if constexpr (JMP) {
      // the whole pass in one block, each row's DM slots branching into static adds
      static_assert(HasJmpPass<TP, DPW, NWIN, CC>::value, "no jump-form pass for this shape");
      JmpPass<TP, DPW, NWIN, CC, false, JMP == 2, ROWCAP>::run(acc, row, ncc, ea, trs, toff, wa, wrs, woff);
    } else if constexpr (HasWinPass<TP, DPW, NWIN, CC>::value) {
      // the whole pass in one block, index mode on throughout
      WinPass<TP, DPW, NWIN, CC, false, ROWCAP>::run(acc, row, ncc, ea, trs, toff, wa, wrs, woff);
    } else {
      // two rows per iteration with the entry registers swapping roles, so
      // the next row's entry needs no copy
      int cl = 0;
      for (; cl + 1 < ncc; cl += 2) {
        win_step<TP, DPW, NWIN, false>(acc, row + (uint32_t)ea[0] * 4u, ea, eb, trs, toff, wa, wb, wrs, woff);
        row += ROWCAP * 4;
        win_step<TP, DPW, NWIN, false>(acc, row + (uint32_t)eb[0] * 4u, eb, ea, trs, toff, wb, wa, wrs, woff);
        row += ROWCAP * 4;
      }
      if (cl < ncc) {
        win_step<TP, DPW, NWIN, false>(acc, row + (uint32_t)ea[0] * 4u, ea, eb, trs, toff, wa, wb, wrs, woff);
        ea = eb;
        wa = wb;
      }
    }
  }

  if constexpr (DET)
    det_store_f32<TP, DPW, NWAVE>(wave, a, acc, tt, rt, beam, t0);
  else
    win_store<TP, DPW, NWAVE, ADJ>(wave, a, acc, tt, rt, beam);
}

// Waves per SIMD that a jump-form variant's registers allow (its accumulators
// start at JmpAcc0, the window follows them), asked of the compiler so that it
// keeps the rest of the kernel within that budget; 1 (no request) otherwise,
// and for the search epilogue, whose registers would otherwise spill.
template <int TP, int DPW, int NWIN, int CC, int JMP, bool DET = false>
constexpr int win_waves_per_eu() {
  if constexpr (JMP != 0 && !DET) {
    constexpr int regs = (JmpAcc0<TP, DPW, NWIN, CC>::value + TP * DPW + NWIN + 7) / 8 * 8;
    return 512 / regs > 8 ? 8 : 512 / regs;
  } else {
    return 1;
  }
}

template <int TP, int DPW, int NWAVE, int NWIN, int CC, int ROWCAP, int NBUF, bool WEIGHTED, bool ADJ,
          bool DET = false, int JMP = 0>
__global__ __launch_bounds__(64 * NWAVE)
__attribute__((amdgpu_waves_per_eu(win_waves_per_eu<TP, DPW, NWIN, CC, JMP, DET>()))) void win_kernel(TileArgs a) {
  __shared__ float4 lds4[NBUF * CC * ROWCAP / 4];
  const int nblk = a.n_time_tiles * a.n_row_tiles;
  const int W = xcd_remap(blockIdx.x, nblk);
  // Forward: the row tiles of one time tile run on one XCD (they share its
  // input window in that L2).  Adjoint: the time tiles of one row tile do
  // instead, so that the passes skipped near both ends of the output (see
  // win_tile) are spread over every XCD rather than idling the first and last.
  const int tt = ADJ ? W % a.n_time_tiles : W / a.n_row_tiles;
  const int rt = ADJ ? W / a.n_time_tiles : W % a.n_row_tiles;
  win_tile<TP, DPW, NWAVE, NWIN, CC, ROWCAP, NBUF, WEIGHTED, ADJ, DET, JMP>(wave_id(), a, tt, rt, blockIdx.y, lds4);
}

// Persistent form for batches of beams.  The work table is split into one
// queue per XCD (all row tiles of a (beam, time tile) in the same queue, so
// the blocks sharing that input window share that XCD's L2).  Blocks are
// dispatched round-robin over the XCDs, so block i drains queue i % NXCD
// first and then helps the others, in order, until every queue is empty.
// Every beam shares the variant; per-beam pointers and tables come from its
// descriptor.  The counters (one per queue, 128 bytes apart) are cleared by a
// separate kernel before each launch.
template <int TP, int DPW, int NWAVE, int NWIN, int CC, int ROWCAP, int NBUF, bool WEIGHTED, int JMP>
__global__ __launch_bounds__(64 * NWAVE) __attribute__((amdgpu_waves_per_eu(win_waves_per_eu<TP, DPW, NWIN, CC, JMP>())))
void win_persistent(const BeamDesc* __restrict__ beams,
                                                             const int32_t* __restrict__ order,
                                                             const int32_t* __restrict__ qoff, int* counters) {
  __shared__ float4 lds4[NBUF * CC * ROWCAP / 4];
  __shared__ int s_tile;
  const int home = blockIdx.x % kNumXcd;
  const int wave = wave_id();
  for (int qi = 0; qi < kNumXcd; ++qi) {
    const int q = (home + qi) % kNumXcd;
    const int q0 = qoff[q], n = qoff[q + 1] - q0;
    for (;;) {
      __syncthreads();  // everyone is done with s_tile and the LDS rows
      if (wave == 0 && lane_fresh() == 0) s_tile = atomicAdd(counters + q * kCounterStride, 1);
      __syncthreads();
      const int k = __builtin_amdgcn_readfirstlane(s_tile);
      if (k >= n) break;
      const int b = order[2 * (q0 + k)];
      const int local = order[2 * (q0 + k) + 1];
      const TileArgs& a = beams[b].a;
      const int tt = local / a.n_row_tiles, rt = local % a.n_row_tiles;
      win_tile<TP, DPW, NWAVE, NWIN, CC, ROWCAP, NBUF, WEIGHTED, false, false, JMP>(wave, a, tt, rt, 0, lds4);
    }
  }
}

__global__ void zero_counter_kernel(int* c) {
  if (threadIdx.x < kNumXcd) c[threadIdx.x * kCounterStride] = 0;
}

// ---------------------------------------------------------------------------
// uint8 -> int32 tile engine.  Lane l owns 4 consecutive samples in each of
// Q groups spaced 256 samples apart, so its LDS reads of one group are
// consecutive across lanes (no bank conflicts).  Per (input row, output row)
// the lane reads the dword holding its 4 samples and the next one, aligns
// them by the delay's byte offset and adds the 4 bytes into 4 int32
// accumulators.  The output store is the dominant traffic, written with
// non-temporal 16-byte stores.
// ---------------------------------------------------------------------------
template <int NWAVE, int ROWCAP>
__device__ __forceinline__ void stage_u8(uint4* lds, const uint8_t* in, const TileArgs& a, const int32_t* blk, int c0,
                                         int ncc, int t0) {
  const int wave = wave_id(), lane = threadIdx.x & 63;
  for (int cl = wave; cl < ncc; cl += NWAVE) {
    const int sb = blk[2 * (c0 + cl)];
    const int sl = blk[2 * (c0 + cl) + 1];
    const uint8_t* src = in + (int64_t)(c0 + cl) * a.in_stride;
    const int u0 = t0 + sb;
    uint4* dst = lds + cl * (ROWCAP / 16);
    const int nv = sl >> 4;
#pragma unroll 2
    for (int v = lane; v < nv; v += 64) {
      const int u = u0 + 16 * v;
      uint4 x;
      if (u + 16 <= a.in_hi) {
        x = *reinterpret_cast<const uint4*>(src + u);
      } else {
        uint32_t wv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          uint32_t acc = 0;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int uu = u + 4 * q + k;
            const uint32_t byte = (uu < a.in_hi) ? (uint32_t)src[uu] : 0u;
            acc |= byte << (8 * k);
          }
          wv[q] = acc;
        }
        x = make_uint4(wv[0], wv[1], wv[2], wv[3]);
      }
      dst[v] = x;
    }
  }
}

// Staging of four byte-shifted copies of each row: copy s holds row[k + s]
// at position k, so a dword holding four consecutive samples starting at any
// byte offset o is the aligned dword (o >> 2) of copy o & 3.  The copies need
// a byte shift, so the data passes through registers: load() fetches a pass's
// bytes into registers, store() writes the shifted copies to LDS.  The kernel calls load() for pass p + 1 before it
// sums pass p, so the global loads are in flight during the adds.
// With fewer rows than waves, the G = NWAVE / CC waves of a row take its
// 16-byte chunks in turn (wave w: row w mod CC, chunks lane + 64 (w / CC +
// G i)), so that every wave stages and each holds fewer chunks.
template <int NWAVE, int CC, int ROWCAP, typename E>
struct ShiftStage {
  static constexpr int G = CC < NWAVE ? NWAVE / CC : 1;  // waves per row
  static_assert(CC >= NWAVE || NWAVE % CC == 0, "rows per pass must divide the waves");
  static constexpr int RPW = (CC + NWAVE - 1) / NWAVE;        // rows staged per wave
  static constexpr int VPL = (ROWCAP / 16 + 64 * G - 1) / (64 * G);  // 16-byte chunks per lane per row
  uint32_t d[RPW][VPL][5];
  int nv[RPW];

  static __device__ __forceinline__ int row_of(int wave, int r) { return G > 1 ? wave % CC : wave + r * NWAVE; }
  static __device__ __forceinline__ int chunk_of(int wave, int lane, int i) {
    return G > 1 ? lane + 64 * (wave / CC + G * i) : lane + 64 * i;
  }

  __device__ __forceinline__ void load(const uint8_t* in, const TileArgs& a, const int32_t* blk, const int32_t* wav,
                                       int c0, int ncc, int t0) {
    const int wave = wave_id(), lane = threadIdx.x & 63;
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      const int cl = row_of(wave, r);
      nv[r] = 0;
      if (cl < ncc) {
        const ent2_t bl = sload_entry2(blk + 2 * (c0 + cl));
        const uint8_t* src = in + (int64_t)(c0 + cl) * a.in_stride;
        const int u0 = t0 + bl[0];
        nv[r] = bl[1] >> 4;
#pragma unroll
        for (int i = 0; i < VPL; ++i) {
          const int v = chunk_of(wave, lane, i);
          const int u = u0 + 16 * v;
          if (v < nv[r]) {
            if (u + 20 <= a.in_hi) {
              const uint4 x = *reinterpret_cast<const uint4*>(src + u);
              d[r][i][0] = x.x;
              d[r][i][1] = x.y;
              d[r][i][2] = x.z;
              d[r][i][3] = x.w;
              d[r][i][4] = *reinterpret_cast<const uint32_t*>(src + u + 16);
            } else {
#pragma unroll
              for (int q = 0; q < 5; ++q) {
                uint32_t w = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                  const int uu = u + 4 * q + k;
                  w |= (uu < a.in_hi ? (uint32_t)src[uu] : 0u) << (8 * k);
                }
                d[r][i][q] = w;
              }
            }
          }
        }
      }
    }
    (void)wav;
  }

  __device__ __forceinline__ void store(uint4* lds, int ncc) const {
    const int wave = wave_id(), lane = threadIdx.x & 63;
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      const int cl = row_of(wave, r);
#pragma unroll
      for (int i = 0; i < VPL; ++i) {
        const int v = chunk_of(wave, lane, i);
        if (v < nv[r]) {
          const uint32_t* x = d[r][i];
          lds[(0 * CC + cl) * (ROWCAP / 16) + v] = make_uint4(x[0], x[1], x[2], x[3]);
#pragma unroll
          for (int sh = 1; sh < 4; ++sh) {
            lds[(sh * CC + cl) * (ROWCAP / 16) + v] =
                make_uint4(__builtin_amdgcn_alignbyte(x[1], x[0], sh), __builtin_amdgcn_alignbyte(x[2], x[1], sh),
                           __builtin_amdgcn_alignbyte(x[3], x[2], sh), __builtin_amdgcn_alignbyte(x[4], x[3], sh));
          }
        }
      }
    }
    (void)ncc;
  }
};

// Asynchronous staging of one pass: the rows (16-byte buffer loads writing
// LDS directly; positions past the row end read as zero) and this wave's
// table entries for the pass (one 16-byte entry per lane, lanes past the
// pass read zero into the slack of the per-wave table slot).
template <int NWAVE, int ROWCAP>
__device__ __forceinline__ void stage_u8_async(uint4* lds, ent4_t* tabw, const uint8_t* in, const TileArgs& a,
                                               const int32_t* blk, const int32_t* wav, int c0, int ncc, int t0) {
  const int wave = wave_id(), lane = threadIdx.x & 63;
  for (int cl = wave; cl < ncc; cl += NWAVE) {
    const ent2_t bl = sload_entry2(blk + 2 * (c0 + cl));
    const uint8_t* row = in + (int64_t)(c0 + cl) * a.in_stride;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void*)row, (short)0, a.in_hi, 0x00020000);
    const int u0 = t0 + bl[0];
    const int nv = bl[1] >> 4;
    for (int v0 = 0; v0 < nv; v0 += 64) {
      if (v0 + lane < nv)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (LDS_AS void*)(lds + cl * (ROWCAP / 16) + v0), 16,
                                                 u0 + 16 * (v0 + lane), 0, 0, 0);
    }
  }
  const __amdgpu_buffer_rsrc_t rt =
      __builtin_amdgcn_make_buffer_rsrc((void*)(wav + (size_t)c0 * 4), (short)0, ncc * 16, 0x00020000);
  __builtin_amdgcn_raw_ptr_buffer_load_lds(rt, (LDS_AS void*)tabw, 16, lane * 16, 0, 0, 0);
}

// One block walks `tiles_per_block` consecutive time tiles of one DM tile.
// NBUF = 1: synchronous staging; NBUF = 2: the rows of the next (time tile,
// pass) step are loaded into the second buffer while the current one is
// summed, and the finished tile's stores drain behind the next tile's work.
template <int Q, int DPW, int NWAVE, int CC, int ROWCAP, int NBUF>
__global__ __launch_bounds__(64 * NWAVE) void u8_kernel(TileArgs a) {
  constexpr int ST = 256 * Q;
  constexpr int DT = NWAVE * DPW;
  constexpr int WI = 4;  // packed 16-bit offsets, DPW <= 8
  static_assert(DPW <= 8, "uint8 variants pack at most 8 offsets");
  typedef ent4_t E;
  __shared__ uint4 lds[NBUF * CC * ROWCAP / 16];
  __shared__ E tab[NBUF][NWAVE][NBUF == 2 ? 64 : CC];
  const int tpb = NBUF == 2 ? a.tiles_per_block : 1;
  const int ngroups = (a.n_time_tiles + tpb - 1) / tpb;
  const int nblk = ngroups * a.n_row_tiles;
  const int W = xcd_remap(blockIdx.x, nblk);
  const int grp = W / a.n_row_tiles, rt = W % a.n_row_tiles;
  const int tt0 = grp * tpb;
  const int ntile = min(tpb, a.n_time_tiles - tt0);
  const int beam = blockIdx.y;
  const int wave = wave_id(), lane = threadIdx.x & 63;
  const int wt = rt * NWAVE + wave;
  const uint8_t* in = static_cast<const uint8_t*>(a.in) + (int64_t)beam * a.in_beam_stride;
  const int32_t* blk = uniform_ptr(a.blk + (size_t)rt * a.rows_in * 2);
  const int32_t* __restrict__ wav = uniform_ptr(a.wav + (size_t)wt * a.rows_in * WI);
  const uint32_t* lds32 = reinterpret_cast<const uint32_t*>(lds);
  int32_t* out = static_cast<int32_t*>(a.out) + (int64_t)beam * a.out_beam_stride;
  const int npass = (a.rows_in + CC - 1) / CC;
  const int nsteps = ntile * npass;

  int acc[DPW][Q][4];
#pragma unroll
  for (int j = 0; j < DPW; ++j)
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[j][q][k] = 0;

  if (NBUF == 2) stage_u8_async<NWAVE, ROWCAP>(lds, tab[0][wave], in, a, blk, wav, 0, min(CC, a.rows_in), tt0 * ST);
  for (int s = 0; s < nsteps; ++s) {
    const int k = s / npass, p = s - k * npass;
    const int t0 = (tt0 + k) * ST;
    const int c0 = p * CC;
    const int ncc = min(CC, a.rows_in - c0);
    const int buf = NBUF == 2 ? (s & 1) : 0;
    if (NBUF == 1) {
      // The wave's offsets for the rows of a pass are copied into LDS with
      // the rows.
      __syncthreads();
      stage_u8<NWAVE, ROWCAP>(lds, in, a, blk, c0, ncc, t0);
      if (lane < ncc) tab[0][wave][lane] = *reinterpret_cast<const E*>(wav + (size_t)(c0 + lane) * WI);
      __syncthreads();
    } else {
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
      if (s + 1 < nsteps) {
        const int k1 = (s + 1) / npass, p1 = s + 1 - k1 * npass;
        stage_u8_async<NWAVE, ROWCAP>(lds + ((s + 1) & 1) * CC * (ROWCAP / 16), tab[(s + 1) & 1][wave], in, a, blk,
                                      wav, p1 * CC, min(CC, a.rows_in - p1 * CC), (tt0 + k1) * ST);
      }
    }
    const uint32_t* rows = lds32 + buf * CC * (ROWCAP / 4);
    E cur = tab[buf][wave][0];
    for (int cl = 0; cl < ncc; ++cl) {
      // each step reads the next row's entry (a broadcast LDS read) one step
      // ahead of its use
      const E nxt = tab[buf][wave][min(cl + 1, ncc - 1)];
      const uint32_t* row = rows + cl * (ROWCAP / 4);
      uint32_t cw[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) cw[q] = (uint32_t)__builtin_amdgcn_readfirstlane(cur[q]);
#pragma unroll
      for (int jj = 0; jj < DPW; ++jj) {
        const uint32_t o = (cw[jj >> 1] >> (16 * (jj & 1))) & 0xFFFFu;
        const uint32_t sh = o & 3u;
        const uint32_t* pr = row + (o >> 2) + lane;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const uint32_t d0 = pr[64 * q];
          const uint32_t d1 = pr[64 * q + 1];
          const uint32_t v = __builtin_amdgcn_alignbyte(d1, d0, sh);
          acc[jj][q][0] += (int)(v & 0xFFu);
          acc[jj][q][1] += (int)((v >> 8) & 0xFFu);
          acc[jj][q][2] += (int)((v >> 16) & 0xFFu);
          acc[jj][q][3] += (int)(v >> 24);
        }
      }
      cur = nxt;
    }
    if (p == npass - 1) {
#pragma unroll
      for (int jj = 0; jj < DPW; ++jj) {
        const int r = rt * DT + wave * DPW + jj;
        if (r < a.rows_out) {
          int32_t* orow = out + (int64_t)r * a.out_stride;
#pragma unroll
          for (int q = 0; q < Q; ++q) {
            const int t = t0 + 4 * lane + 256 * q;
            if (t + 4 <= a.nout) {
              __builtin_nontemporal_store(acc[jj][q][0], orow + t + 0);
              __builtin_nontemporal_store(acc[jj][q][1], orow + t + 1);
              __builtin_nontemporal_store(acc[jj][q][2], orow + t + 2);
              __builtin_nontemporal_store(acc[jj][q][3], orow + t + 3);
            } else {
#pragma unroll
              for (int e = 0; e < 4; ++e)
                if (t + e < a.nout) orow[t + e] = acc[jj][q][e];
            }
          }
        }
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[jj][q][e] = 0;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// uint8 -> int32 tile engine on byte-shifted rows.  Each input row is staged
// as four copies shifted by 0..3 bytes (ShiftStage), so the four samples
// a lane needs at any delay are one aligned LDS dword: one 4-byte LDS read
// per 4 adds.  The table gives, per (wave tile, input row), each output row's
// dword offset into the staged copies, so a read costs one address add.
// For a dword v = (b0, b1, b2, b3) the lane keeps two sums over rows:
//   E += v & 0x00FF00FF     (16-bit lanes: sum b0, sum b2)
//   U += v >> 8             (sum b1 + 2^8 sum b2 + 2^16 sum b3)
// four two-operand integer operations, which issue at the full rate, per 4
// adds.  Over at most 256 rows neither overflows, and
//   sum b0 = E & 0xFFFF, sum b2 = E >> 16, U - 2^8 sum b2 = sum b1 + 2^16 sum b3.
// WIDE variants move these into int32 sums every 256 input rows; the others
// accept at most 256 input rows.  Sums are exact integers, so the order does
// not matter.
// ---------------------------------------------------------------------------
template <int Q, int DPW, int NWAVE, int CC, int ROWCAP, bool WIDE, bool DET>
__device__ __forceinline__ void u8s_tile(const TileArgs& a) {
  constexpr int ST = 256 * Q;
  constexpr int DT = NWAVE * DPW;
  constexpr int WI = DPW <= 4 ? 4 : 8;  // ints per table entry
  static_assert(DPW == 2 || DPW == 4 || DPW == 8, "unsupported rows per wave");
  static_assert(256 % CC == 0, "a flush every 256 rows must fall on a pass boundary");
  typedef typename std::conditional<(WI == 4), ent4_t, ent8_t>::type E;
  constexpr int LDS_STAGE = 4 * CC * ROWCAP / 16;
  constexpr int LDS_DET = DET ? NWAVE * ST / 4 : 0;
  __shared__ uint4 lds[LDS_STAGE > LDS_DET ? LDS_STAGE : LDS_DET];
  const int nblk = a.n_time_tiles * a.n_row_tiles;
  const int W = xcd_remap(blockIdx.x, nblk);
  const int tt = W / a.n_row_tiles, rt = W % a.n_row_tiles;
  const int beam = blockIdx.y;
  const int wave = wave_id(), lane = threadIdx.x & 63;
  const int wt = rt * NWAVE + wave;
  const int t0 = DET ? tt * a.tile_step : tt * ST;
  const uint8_t* in = static_cast<const uint8_t*>(a.in) + (int64_t)beam * a.in_beam_stride;
  const int32_t* blk = uniform_ptr(a.blk + (size_t)rt * a.rows_in * 2);
  const int32_t* __restrict__ wav = uniform_ptr(a.wav + (size_t)wt * a.rows_in * WI);
  const uint32_t* lds32 = reinterpret_cast<const uint32_t*>(lds) + lane;
  int32_t* out = static_cast<int32_t*>(a.out) + (int64_t)beam * a.out_beam_stride;
  const int npass = (a.rows_in + CC - 1) / CC;

  uint32_t ev[DPW][Q], hi[DPW][Q];
  int acc[WIDE ? DPW : 1][WIDE ? Q : 1][4];
#pragma unroll
  for (int j = 0; j < DPW; ++j)
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      ev[j][q] = hi[j][q] = 0u;
      if (WIDE)
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[WIDE ? j : 0][WIDE ? q : 0][k] = 0;
    }

  // the four sample sums of (output row j, dword q) from the packed sums
  auto unpack = [&](int j, int q, int* s4) {
    const uint32_t s2 = ev[j][q] >> 16;
    const uint32_t u = hi[j][q] - (s2 << 8);
    s4[0] = (int)(ev[j][q] & 0xFFFFu);
    s4[1] = (int)(u & 0xFFFFu);
    s4[2] = (int)s2;
    s4[3] = (int)(u >> 16);
  };

  // this wave's table entries, read with scalar loads (past the last row: zero)
  const __amdgpu_buffer_rsrc_t trs =
      __builtin_amdgcn_make_buffer_rsrc((void*)wav, (short)0, a.rows_in * WI * 4, 0x00020000);
  constexpr int NI = CC * WI;  // ints of one pass's entries
  static_assert(NI == 8 || NI % 16 == 0, "a pass's entries are loaded in 8- or 16-int pieces");
  ShiftStage<NWAVE, CC, ROWCAP, E> stage;
  stage.load(in, a, blk, wav, 0, min(CC, a.rows_in), t0);
  for (int p = 0; p < npass; ++p) {
    const int c0 = p * CC;
    const int ncc = min(CC, a.rows_in - c0);
    int32_t off[NI];
    if constexpr (NI == 8) {
      const ent8_t x = sbload8(trs, (uint32_t)(c0 * WI * 4));
#pragma unroll
      for (int k = 0; k < 8; ++k) off[k] = x[k];
    } else {
#pragma unroll
      for (int k0 = 0; k0 < NI; k0 += 16) {
        const ent16_t x = sbload16(trs, (uint32_t)((c0 * WI + k0) * 4));
#pragma unroll
        for (int k = 0; k < 16; ++k) off[k0 + k] = x[k];
      }
    }
    __syncthreads();  // every wave is done with pass p - 1's rows
    stage.store(lds, ncc);
    __syncthreads();
    if (p + 1 < npass) stage.load(in, a, blk, wav, c0 + CC, min(CC, a.rows_in - c0 - CC), t0);
#pragma unroll
    for (int cl = 0; cl < CC; ++cl) {
      if (cl >= ncc) break;
#pragma unroll
      for (int jj = 0; jj < DPW; ++jj) {
        const uint32_t* pr = reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(lds32) + off[cl * WI + jj]);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const uint32_t v = pr[64 * q];
          ev[jj][q] += v & 0x00FF00FFu;
          hi[jj][q] += v >> 8;
        }
      }
    }
    if (WIDE && (((p + 1) * CC) % 256 == 0 || p == npass - 1)) {
#pragma unroll
      for (int j = 0; j < DPW; ++j)
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          int s4[4];
          unpack(j, q, s4);
#pragma unroll
          for (int k = 0; k < 4; ++k) acc[WIDE ? j : 0][WIDE ? q : 0][k] += s4[k];
          ev[j][q] = hi[j][q] = 0u;
        }
    }
  }

  if constexpr (DET) {
    // Single-pulse search in place of the store (see detect_dev.h): each
    // wave passes its rows one at a time through its own LDS slot, scaled by
    // 2^IB for the keys, to give every lane L consecutive samples (the
    // 16-byte chunks are XOR-swizzled within groups of eight so that both
    // the writes and the reads are free of bank conflicts); the look-ahead
    // comes from the lanes above.
    constexpr int L = 4 * Q;
    constexpr int IB = Q == 2 ? 3 : Q == 4 ? 4 : 5;
    static_assert((1 << IB) == L, "a lane's run is a power of two");
    __syncthreads();  // every wave is done with the staged rows
    int4* slot = reinterpret_cast<int4*>(lds) + wave * (ST / 4);
    const int nvalid = min(ST, a.det_nsamp - t0);
    const int pos0 = L * lane;
    const bool owned = pos0 < a.tile_step;
    const int lim = nvalid - pos0;
#pragma unroll
    for (int jj = 0; jj < DPW; ++jj) {
      const int r = rt * DT + wave * DPW + jj;
      if (r >= a.rows_out) break;
      __builtin_amdgcn_sched_barrier(0);  // one row at a time: keeps the search's registers to one row's
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        int s4[4];
        if (WIDE) {
#pragma unroll
          for (int e = 0; e < 4; ++e) s4[e] = acc[WIDE ? jj : 0][WIDE ? q : 0][e];
        } else {
          unpack(jj, q, s4);
        }
        const int m = lane + 64 * q;  // chunk of samples 4m .. 4m + 3
        slot[m ^ ((m >> 2) & 7)] = make_int4(s4[0] << IB, s4[1] << IB, s4[2] << IB, s4[3] << IB);
      }
      __builtin_amdgcn_wave_barrier();
      int v[L];
#pragma unroll
      for (int c = 0; c < L / 4; ++c) {
        const int m = (L / 4) * lane + c;
        const int4 x = slot[m ^ ((m >> 2) & 7)];
        v[4 * c + 0] = x.x;
        v[4 * c + 1] = x.y;
        v[4 * c + 2] = x.z;
        v[4 * c + 3] = x.w;
      }
      int key[kDetNW];
      double s1, s2;
      if (nvalid < ST)
        det_lane_int<L, IB, true>(v, owned, lim, a.det_s2_u32 != 0, key, s1, s2);
      else
        det_lane_int<L, IB, false>(v, owned, lim, a.det_s2_u32 != 0, key, s1, s2);
      det_commit_int<L, IB>(a.det + ((int64_t)beam * a.rows_out + r) * a.n_time_tiles + tt, key, s1, s2, pos0, t0);
      __builtin_amdgcn_wave_barrier();
    }
    return;
  }

#pragma unroll
  for (int jj = 0; jj < DPW; ++jj) {
    const int r = rt * DT + wave * DPW + jj;
    if (r < a.rows_out) {
      int32_t* orow = out + (int64_t)r * a.out_stride;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        int s4[4];
        if (WIDE) {
#pragma unroll
          for (int e = 0; e < 4; ++e) s4[e] = acc[WIDE ? jj : 0][WIDE ? q : 0][e];
        } else {
          unpack(jj, q, s4);
        }
        const int t = t0 + 4 * lane + 256 * q;
        if (t + 4 <= a.nout) {
          __builtin_nontemporal_store(s4[0], orow + t + 0);
          __builtin_nontemporal_store(s4[1], orow + t + 1);
          __builtin_nontemporal_store(s4[2], orow + t + 2);
          __builtin_nontemporal_store(s4[3], orow + t + 3);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (t + e < a.nout) orow[t + e] = s4[e];
        }
      }
    }
  }
}

// WPE > 0 asks the compiler to fit WPE waves per SIMD (512 / WPE registers),
// so that as many blocks as the LDS allows stay resident on a CU.
template <int Q, int DPW, int NWAVE, int CC, int ROWCAP, bool WIDE, int WPE>
__global__ __launch_bounds__(64 * NWAVE) __attribute__((amdgpu_waves_per_eu(WPE > 0 ? WPE : 1))) void u8s_kernel(
    TileArgs a) {
  u8s_tile<Q, DPW, NWAVE, CC, ROWCAP, WIDE, false>(a);
}

// With the single-pulse search in the epilogue (no occupancy request: the
// search needs its registers).
template <int Q, int DPW, int NWAVE, int CC, int ROWCAP, bool WIDE>
__global__ __launch_bounds__(64 * NWAVE) void u8s_det_kernel(TileArgs a) {
  u8s_tile<Q, DPW, NWAVE, CC, ROWCAP, WIDE, true>(a);
}

// ---------------------------------------------------------------------------
// Direct kernels: one work item per (output row, sample), one-dimensional
// blocks along time, every term read straight from global memory.  This is
// the paper's "generically tuned" form (Section 5: no DM-direction reuse) and
// the fallback for plans whose delay spans fit no tiled variant.
// ---------------------------------------------------------------------------
template <bool WEIGHTED>
__global__ __launch_bounds__(256) void direct_f32_kernel(const float* __restrict__ in, int64_t in_stride,
                                                         int64_t in_beam_stride, const int32_t* __restrict__ delta,
                                                         int nchan, const float* __restrict__ w, float* out,
                                                         int64_t out_stride, int64_t out_beam_stride, int nsamp,
                                                         int ntb) {
  const int j = blockIdx.x / ntb;
  const int t = (blockIdx.x - j * ntb) * 256 + threadIdx.x;
  const int b = blockIdx.y;
  if (t >= nsamp) return;
  const int32_t* drow = delta + (size_t)j * nchan;
  const float* src = in + (int64_t)b * in_beam_stride + t;
  float acc = 0.f;
  for (int c = 0; c < nchan; ++c) {
    const float x = src[(int64_t)c * in_stride + drow[c]];
    const float term = WEIGHTED ? w[c] * x : x;  // the weighted sample, rounded
    acc = acc + term;
  }
  out[(int64_t)b * out_beam_stride + (int64_t)j * out_stride + t] = acc;
}

__global__ __launch_bounds__(256) void direct_u8_kernel(const uint8_t* __restrict__ in, int64_t in_stride,
                                                        int64_t in_beam_stride, const int32_t* __restrict__ delta,
                                                        int nchan, int32_t* out, int64_t out_stride,
                                                        int64_t out_beam_stride, int nsamp, int ntb) {
  const int j = blockIdx.x / ntb;
  const int t = (blockIdx.x - j * ntb) * 256 + threadIdx.x;
  const int b = blockIdx.y;
  if (t >= nsamp) return;
  const int32_t* drow = delta + (size_t)j * nchan;
  const uint8_t* src = in + (int64_t)b * in_beam_stride + t;
  int32_t acc = 0;
  for (int c = 0; c < nchan; ++c) acc += (int32_t)src[(int64_t)c * in_stride + drow[c]];
  out[(int64_t)b * out_beam_stride + (int64_t)j * out_stride + t] = acc;
}

// Direct adjoint: one work item per (channel, input sample), summing over
// DM trials in ascending order; block partial sums of x * G for grad_w.
__global__ __launch_bounds__(256) void direct_adjoint_kernel(const float* __restrict__ g, int64_t g_stride,
                                                             int64_t g_beam_stride, const int32_t* __restrict__ delta,
                                                             int nchan, int ndm, int nsamp, int nin,
                                                             const float* __restrict__ w, float* grad_in,
                                                             int64_t gi_stride, int64_t gi_beam_stride,
                                                             const float* __restrict__ x, int64_t x_stride,
                                                             int64_t x_beam_stride, double* partial, int ntb) {
  __shared__ double red[256];
  const int c = blockIdx.x / ntb;
  const int tb = blockIdx.x - c * ntb;
  const int t = tb * 256 + threadIdx.x;
  const int b = blockIdx.y;
  float acc = 0.f;
  if (t < nin) {
    const float* gb = g + (int64_t)b * g_beam_stride;
    for (int j = 0; j < ndm; ++j) {
      const int s = t - delta[(size_t)j * nchan + c];
      if (s >= 0 && s < nsamp) acc = acc + gb[(int64_t)j * g_stride + s];
    }
    if (grad_in) grad_in[(int64_t)b * gi_beam_stride + (int64_t)c * gi_stride + t] = (w ? w[c] : 1.f) * acc;
  }
  if (partial) {
    double p = 0.0;
    if (t < nin) p = (double)x[(int64_t)b * x_beam_stride + (int64_t)c * x_stride + t] * (double)acc;
    red[threadIdx.x] = p;
    __syncthreads();
    for (int m = 128; m >= 1; m >>= 1) {
      if ((int)threadIdx.x < m) red[threadIdx.x] += red[threadIdx.x + m];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[((size_t)b * ntb + tb) * nchan + c] = red[0];
  }
}

// grad_w[c] = sum over parts p (ascending) of partial[p][c].
__global__ __launch_bounds__(256) void reduce_gradw_kernel(const double* __restrict__ partial, int nparts, int nchan,
                                                           float* grad_w) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= nchan) return;
  double s = 0.0;
  for (int p = 0; p < nparts; ++p) s += partial[(size_t)p * nchan + c];
  grad_w[c] = (float)s;
}

// ---------------------------------------------------------------------------
// Variant tables and launchers.
// ---------------------------------------------------------------------------
// (index, TP samples per lane, DPW rows per wave, NWAVE, NWIN window registers,
//  CC rows per LDS pass, ROWCAP floats per LDS row, NBUF LDS buffers, JMP)
// JMP = 1: each row's DM slots branch into static blocks of adds (JmpPass)
// instead of indexing the window registers; JMP = 2: the same, every row
// reading the whole window (no per-row read-count branches).
// A lane owns TP consecutive samples; TP/4 odd (12, 20, 28, 36) keeps its
// 16-byte LDS reads free of bank conflicts.
#define F32_VARIANTS(X)                                          \
  X(0, 12, 4, 4, 36, 8, 1024, 1, 0)   /* 16 DMs x 768             */ \
  X(1, 12, 4, 4, 48, 8, 1024, 1, 0)   /* 16 DMs x 768, wide spans */ \
  X(2, 8, 8, 4, 64, 8, 1024, 1, 0)    /* 32 DMs x 512             */ \
  X(3, 16, 8, 4, 72, 8, 2048, 1, 0)   /* 32 DMs x 1024            */ \
  X(4, 8, 4, 4, 48, 16, 1024, 1, 0)   /* 16 DMs x 512             */ \
  X(5, 16, 4, 4, 64, 8, 2048, 1, 0)   /* 16 DMs x 1024            */ \
  X(6, 12, 4, 4, 36, 4, 1024, 2, 0)   /* 16 DMs x 768, async      */ \
  X(7, 12, 8, 4, 56, 4, 1024, 2, 0)   /* 32 DMs x 768, async      */ \
  X(8, 20, 4, 4, 44, 4, 1536, 2, 0)   /* 16 DMs x 1280, async     */ \
  X(9, 12, 4, 8, 36, 4, 1024, 2, 0)   /* 32 DMs x 768, async      */ \
  X(10, 12, 8, 8, 56, 4, 1280, 2, 0)  /* 64 DMs x 768, async      */ \
  X(11, 12, 4, 4, 48, 4, 1024, 2, 0)  /* 16 DMs x 768, async      */ \
  X(12, 8, 8, 4, 64, 4, 1024, 2, 0)   /* 32 DMs x 512, async      */ \
  X(13, 20, 8, 4, 56, 4, 1536, 2, 0)  /* 32 DMs x 1280, async     */ \
  X(14, 28, 4, 4, 48, 4, 2048, 2, 0)  /* 16 DMs x 1792, async     */ \
  X(15, 20, 8, 8, 56, 4, 1792, 2, 0)  /* 64 DMs x 1280, async     */ \
  X(16, 28, 4, 8, 48, 4, 2048, 2, 0)  /* 32 DMs x 1792, async     */ \
  X(17, 20, 8, 8, 56, 8, 1792, 2, 0)  /* 64 DMs x 1280, async     */ \
  X(18, 20, 8, 4, 56, 6, 1536, 2, 0)  /* 32 DMs x 1280, async     */ \
  X(19, 20, 4, 6, 44, 4, 1536, 2, 1)  /* 24 DMs x 1280, jump      */ \
  X(20, 20, 4, 4, 44, 4, 1536, 2, 1)  /* 16 DMs x 1280, jump      */ \
  X(21, 20, 4, 12, 44, 4, 1792, 2, 1) /* 48 DMs x 1280, jump      */ \
  X(22, 20, 8, 4, 56, 6, 1536, 2, 1)  /* 32 DMs x 1280, jump      */ \
  X(23, 20, 8, 8, 56, 4, 1792, 2, 1)  /* 64 DMs x 1280, jump      */ \
  X(24, 28, 4, 4, 48, 4, 2048, 2, 1)  /* 16 DMs x 1792, jump      */ \
  X(25, 28, 4, 8, 48, 4, 2048, 2, 1)  /* 32 DMs x 1792, jump      */ \
  X(26, 12, 4, 8, 36, 4, 1024, 2, 1)  /* 32 DMs x 768, jump       */ \
  X(27, 12, 4, 12, 36, 4, 1024, 2, 1) /* 48 DMs x 768, jump       */ \
  X(28, 20, 8, 4, 56, 6, 1536, 2, 2)  /* 32 DMs x 1280, jump full */ \
  X(29, 20, 4, 12, 44, 4, 1792, 2, 2) /* 48 DMs x 1280, jump full */ \
  X(30, 20, 4, 4, 44, 4, 1536, 2, 2)  /* 16 DMs x 1280, jump full */ \
  X(31, 20, 8, 8, 56, 4, 1792, 2, 2)  /* 64 DMs x 1280, jump full */ \
  X(32, 20, 4, 8, 40, 6, 1536, 2, 1)  /* 32 DMs x 1280, jump, 4 waves/SIMD */ \
  X(33, 20, 4, 4, 40, 3, 1536, 2, 1)  /* 16 DMs x 1280, jump, 4 waves/SIMD */ \
  X(34, 20, 4, 16, 40, 8, 1792, 2, 1) /* 64 DMs x 1280, jump, 4 waves/SIMD */ \
  X(35, 20, 4, 16, 40, 10, 1792, 2, 1) /* 64 DMs x 1280, jump, 4 waves/SIMD */ \
  X(36, 20, 4, 16, 40, 8, 1792, 2, 2) /* 64 DMs x 1280, jump full, 4 waves/SIMD */ \
  X(37, 20, 4, 16, 44, 10, 1792, 2, 1) /* 64 DMs x 1280, jump, 4 waves/SIMD */ \
  X(38, 20, 4, 16, 44, 8, 1792, 2, 1) /* 64 DMs x 1280, jump, 4 waves/SIMD */

// (index, Q dwords per lane, DPW, NWAVE, CC rows per LDS pass, ROWCAP bytes)
#define U8_VARIANTS(X)                                      \
  X(0, 4, 4, 4, 16, 2048, 1) /* 16 DMs x 1024          */   \
  X(1, 4, 2, 4, 32, 1536, 1) /*  8 DMs x 1024          */   \
  X(2, 2, 4, 4, 16, 1536, 1) /* 16 DMs x 512           */   \
  X(3, 4, 4, 4, 32, 2048, 1) /* 16 DMs x 1024          */   \
  X(4, 2, 2, 4, 32, 1024, 1) /*  8 DMs x 512           */   \
  X(5, 4, 8, 4, 16, 4096, 1) /* 32 DMs x 1024          */   \
  X(6, 4, 4, 8, 16, 4096, 1) /* 32 DMs x 1024          */   \
  X(7, 2, 4, 4, 16, 1152, 2) /* 16 DMs x 512, async    */   \
  X(8, 4, 4, 4, 16, 1664, 2) /* 16 DMs x 1024, async   */   \
  X(9, 4, 4, 8, 8, 2304, 2)  /* 32 DMs x 1024, async   */   \
  X(10, 2, 8, 4, 16, 1792, 2) /* 32 DMs x 512, async   */   \
  X(11, 2, 4, 4, 32, 1152, 2) /* 16 DMs x 512, async   */

// Byte-shifted variants: (index, Q, DPW, NWAVE, CC, ROWCAP bytes per copy,
// WIDE, waves per SIMD asked of the compiler or 0)
#define U8S_VARIANTS(X)                                          \
  X(12, 4, 4, 4, 4, 1792, false, 0) /* 16 DMs x 1024      */    \
  X(13, 2, 4, 8, 4, 1792, false, 0) /* 32 DMs x 512       */    \
  X(14, 4, 4, 8, 8, 2304, false, 0) /* 32 DMs x 1024      */    \
  X(15, 4, 8, 4, 4, 2304, false, 0) /* 32 DMs x 1024      */    \
  X(16, 4, 4, 8, 4, 2304, false, 0) /* 32 DMs x 1024      */    \
  X(17, 4, 4, 4, 2, 1792, false, 0) /* 16 DMs x 1024      */    \
  X(18, 4, 4, 4, 4, 1792, true, 0)  /* 16 DMs x 1024, wide */   \
  X(19, 4, 4, 8, 4, 2304, true, 0)  /* 32 DMs x 1024, wide */   \
  X(20, 8, 4, 8, 4, 3328, false, 0) /* 32 DMs x 2048      */    \
  X(21, 4, 8, 8, 4, 3584, false, 0) /* 64 DMs x 1024      */    \
  X(22, 4, 4, 16, 4, 3584, false, 8) /* 64 DMs x 1024, 2 blocks/CU */

const std::vector<Variant>& variants_f32() {
  static const std::vector<Variant> v = [] {
    std::vector<Variant> r;
#define MAKE_F32(ID, TP, DPW, NW, NWIN, CC, RC, NB, JMP)                                                    \
  r.push_back(Variant{JMP == 2 ? "win_tp" #TP "_dpw" #DPW "_nw" #NW "_win" #NWIN "_cc" #CC "_buf" #NB "_jmpf"   \
                      : JMP    ? "win_tp" #TP "_dpw" #DPW "_nw" #NW "_win" #NWIN "_cc" #CC "_buf" #NB "_jmp"    \
                               : "win_tp" #TP "_dpw" #DPW "_nw" #NW "_win" #NWIN "_cc" #CC "_buf" #NB,         \
                      KIND_WIN_F32, TP, DPW, NW, NWIN, CC, RC, NB, ID, 0, JMP});
    F32_VARIANTS(MAKE_F32)
#undef MAKE_F32
    return r;
  }();
  return v;
}

const std::vector<Variant>& variants_u8() {
  static const std::vector<Variant> v = [] {
    std::vector<Variant> r;
#define MAKE_U8(ID, Q, DPW, NW, CC, RC, NB)                                                                 \
  r.push_back(Variant{"u8_q" #Q "_dpw" #DPW "_nw" #NW "_cc" #CC "_buf" #NB, KIND_TILE_U8, Q, DPW, NW, 0, CC, RC, NB, \
                      ID});
    U8_VARIANTS(MAKE_U8)
#undef MAKE_U8
#define MAKE_U8S(ID, Q, DPW, NW, CC, RC, WIDE, WPE)                                                          \
  r.push_back(Variant{WIDE        ? "u8s_q" #Q "_dpw" #DPW "_nw" #NW "_cc" #CC "_wide"                          \
                      : WPE > 0   ? "u8s_q" #Q "_dpw" #DPW "_nw" #NW "_cc" #CC "_o" #WPE                        \
                                  : "u8s_q" #Q "_dpw" #DPW "_nw" #NW "_cc" #CC,                                 \
                      KIND_TILE_U8, Q, DPW, NW, 0, CC, RC, 1, ID, WIDE ? 2 : 1});
    U8S_VARIANTS(MAKE_U8S)
#undef MAKE_U8S
    return r;
  }();
  return v;
}

hipError_t launch_tiled(const Variant& v, const TileArgs& a, int nbeam, bool adjoint, hipStream_t s) {
  // uint8 double-buffered blocks walk tiles_per_block time tiles each
  const int tpb = (v.kind == KIND_TILE_U8 && v.nbuf == 2) ? a.tiles_per_block : 1;
  if (tpb < 1) return hipErrorInvalidConfiguration;
  const int64_t nblk = (int64_t)((a.n_time_tiles + tpb - 1) / tpb) * a.n_row_tiles;
  if (nblk < 1 || nblk > 0x7fffffff || nbeam < 1 || nbeam > 65535) return hipErrorInvalidConfiguration;
  const dim3 grid((unsigned)nblk, (unsigned)nbeam);
  const dim3 block(64 * v.nwave);
  const bool weighted = adjoint ? false : (a.w_in != nullptr);
  if (v.kind == KIND_WIN_F32) {
#define LAUNCH_F32(ID, TP, DPW, NW, NWIN, CC, RC, NB, JMP)                                                      \
  if (v.id == ID) {                                                                                             \
    if (adjoint)                                                                                                \
      hipLaunchKernelGGL((win_kernel<TP, DPW, NW, NWIN, CC, RC, NB, false, true, false, JMP>), grid, block, 0, s, \
                         a);                                                                                    \
    else if (weighted)                                                                                          \
      hipLaunchKernelGGL((win_kernel<TP, DPW, NW, NWIN, CC, RC, NB, true, false, false, JMP>), grid, block, 0, s, \
                         a);                                                                                    \
    else                                                                                                        \
      hipLaunchKernelGGL((win_kernel<TP, DPW, NW, NWIN, CC, RC, NB, false, false, false, JMP>), grid, block, 0,   \
                         s, a);                                                                                 \
    return hipGetLastError();                                                                                   \
  }
    F32_VARIANTS(LAUNCH_F32)
#undef LAUNCH_F32
  } else {
#define LAUNCH_U8(ID, Q, DPW, NW, CC, RC, NB)                                          \
  if (v.id == ID) {                                                                    \
    hipLaunchKernelGGL((u8_kernel<Q, DPW, NW, CC, RC, NB>), grid, block, 0, s, a);     \
    return hipGetLastError();                                                          \
  }
    U8_VARIANTS(LAUNCH_U8)
#undef LAUNCH_U8
#define LAUNCH_U8S(ID, Q, DPW, NW, CC, RC, WIDE, WPE)                                       \
  if (v.id == ID) {                                                                         \
    hipLaunchKernelGGL((u8s_kernel<Q, DPW, NW, CC, RC, WIDE, WPE>), grid, block, 0, s, a);  \
    return hipGetLastError();                                                          \
  }
    U8S_VARIANTS(LAUNCH_U8S)
#undef LAUNCH_U8S
  }
  return hipErrorInvalidDeviceFunction;
}

// Variants with the single-pulse search in their epilogue: the FP32 window
// variants from 13 on (asynchronous staging, the fastest ones) and every
// byte-shifted uint8 variant.
bool detect_fusable(const Variant& v) {
  return v.kind == KIND_WIN_F32 ? (v.id >= 13 && v.nbuf == 2) : v.mode >= 1;
}

int det_step(const Variant& v) {
  const int run = v.kind == KIND_WIN_F32 ? v.tp : 4 * v.tp;  // window starts per lane
  return v.st() - run * ((kDetLook - 1 + run - 1) / run);
}

hipError_t launch_detect(const Variant& v, const TileArgs& a, int nbeam, hipStream_t s) {
  if (!detect_fusable(v)) return hipErrorInvalidDeviceFunction;
  const int64_t nblk = (int64_t)a.n_time_tiles * a.n_row_tiles;
  if (nblk < 1 || nblk > 0x7fffffff || nbeam < 1 || nbeam > 65535) return hipErrorInvalidConfiguration;
  const dim3 grid((unsigned)nblk, (unsigned)nbeam);
  const dim3 block(64 * v.nwave);
  if (v.kind == KIND_WIN_F32) {
#define LAUNCH_DF(ID, TP, DPW, NW, NWIN, CC, RC, NB, JMP)                                                   \
  if constexpr (ID >= 13 && NB == 2) {                                                                        \
    if (v.id == ID) {                                                                                         \
      if (a.w_in)                                                                                             \
        hipLaunchKernelGGL((win_kernel<TP, DPW, NW, NWIN, CC, RC, NB, true, false, true, JMP>), grid, block, 0, \
                           s, a);                                                                             \
      else                                                                                                    \
        hipLaunchKernelGGL((win_kernel<TP, DPW, NW, NWIN, CC, RC, NB, false, false, true, JMP>), grid, block,   \
                           0, s, a);                                                                          \
      return hipGetLastError();                                                                               \
    }                                                                                                         \
  }
    F32_VARIANTS(LAUNCH_DF)
#undef LAUNCH_DF
  } else {
#define LAUNCH_DU8(ID, Q, DPW, NW, CC, RC, WIDE, WPE)                                     \
  if (v.id == ID) {                                                                       \
    hipLaunchKernelGGL((u8s_det_kernel<Q, DPW, NW, CC, RC, WIDE>), grid, block, 0, s, a);   \
    return hipGetLastError();                                                             \
  }
    U8S_VARIANTS(LAUNCH_DU8)
#undef LAUNCH_DU8
  }
  return hipErrorInvalidDeviceFunction;
}

hipError_t launch_batched(const Variant& v, const BeamDesc* d_beams, bool weighted, const int32_t* d_order,
                          const int32_t* d_qoff, int* d_counter, int grid, hipStream_t s) {
  const dim3 block(64 * v.nwave);
#define LAUNCH_P(ID, TP, DPW, NW, NWIN, CC, RC, NB, JMP)                                                    \
  if (v.id == ID) {                                                                                          \
    if (weighted)                                                                                            \
      hipLaunchKernelGGL((win_persistent<TP, DPW, NW, NWIN, CC, RC, NB, true, JMP>), dim3(grid), block, 0, s,  \
                         d_beams, d_order, d_qoff, d_counter);                                               \
    else                                                                                                     \
      hipLaunchKernelGGL((win_persistent<TP, DPW, NW, NWIN, CC, RC, NB, false, JMP>), dim3(grid), block, 0, s, \
                         d_beams, d_order, d_qoff, d_counter);                                               \
    return hipGetLastError();                                                                                \
  }
  if (v.kind == KIND_WIN_F32) {
    F32_VARIANTS(LAUNCH_P)
  }
#undef LAUNCH_P
  return hipErrorInvalidDeviceFunction;
}

int batched_blocks_per_cu(const Variant& v) {
  int n = 0;
#define OCC_P(ID, TP, DPW, NW, NWIN, CC, RC, NB, JMP)                                                            \
  if (v.id == ID) {                                                                                              \
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, win_persistent<TP, DPW, NW, NWIN, CC, RC, NB, false, JMP>, \
                                                     64 * NW, 0) != hipSuccess)                                   \
      n = 1;                                                                                                     \
    return n > 0 ? n : 1;                                                                                        \
  }
  if (v.kind == KIND_WIN_F32) {
    F32_VARIANTS(OCC_P)
  }
#undef OCC_P
  return 1;
}

// 32-bit integer hash (a murmur3-style finaliser) of the word index.
__device__ __forceinline__ uint32_t hash32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

__global__ void fill_random_kernel(uint32_t* p, size_t nwords, bool f32, uint32_t seed) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nwords; i += (size_t)gridDim.x * blockDim.x) {
    const uint32_t h = hash32((uint32_t)i * 2654435761u + seed);
    p[i] = f32 ? __float_as_uint((float)(h >> 8) * (1.f / 8388608.f) - 1.f) : h;
  }
}

hipError_t launch_fill_random(void* p, size_t nbytes, bool f32, uint32_t seed, hipStream_t s) {
  const size_t nwords = nbytes / 4;  // a tail of < 4 bytes keeps its contents
  if (nwords == 0) return hipSuccess;
  const size_t blocks = std::min<size_t>((nwords + 255) / 256, 65536);
  hipLaunchKernelGGL(fill_random_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t*)p, nwords, f32, seed);
  return hipGetLastError();
}

hipError_t launch_zero_counter(int* d_counter, hipStream_t s) {
  hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(64), 0, s, d_counter);
  return hipGetLastError();
}

hipError_t launch_direct_f32(const float* in, int64_t in_stride, int64_t in_beam_stride, const int32_t* delta,
                             int nchan, int ndm, const float* w, float* out, int64_t out_stride,
                             int64_t out_beam_stride, int nsamp, int nbeam, hipStream_t s) {
  const int ntb = (nsamp + 255) / 256;
  const int64_t gx = (int64_t)ntb * ndm;
  if (gx > 0x7fffffff || nbeam > 65535) return hipErrorInvalidConfiguration;
  if (w)
    hipLaunchKernelGGL(direct_f32_kernel<true>, dim3((unsigned)gx, nbeam), dim3(256), 0, s, in, in_stride,
                       in_beam_stride, delta, nchan, w, out, out_stride, out_beam_stride, nsamp, ntb);
  else
    hipLaunchKernelGGL(direct_f32_kernel<false>, dim3((unsigned)gx, nbeam), dim3(256), 0, s, in, in_stride,
                       in_beam_stride, delta, nchan, w, out, out_stride, out_beam_stride, nsamp, ntb);
  return hipGetLastError();
}

hipError_t launch_direct_u8(const uint8_t* in, int64_t in_stride, int64_t in_beam_stride, const int32_t* delta,
                            int nchan, int ndm, int32_t* out, int64_t out_stride, int64_t out_beam_stride,
                            int nsamp, int nbeam, hipStream_t s) {
  const int ntb = (nsamp + 255) / 256;
  const int64_t gx = (int64_t)ntb * ndm;
  if (gx > 0x7fffffff || nbeam > 65535) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(direct_u8_kernel, dim3((unsigned)gx, nbeam), dim3(256), 0, s, in, in_stride, in_beam_stride,
                     delta, nchan, out, out_stride, out_beam_stride, nsamp, ntb);
  return hipGetLastError();
}

hipError_t launch_direct_adjoint(const float* g, int64_t g_stride, int64_t g_beam_stride, const int32_t* delta,
                                 int nchan, int ndm, int nsamp, int nin, const float* w, float* grad_in,
                                 int64_t gi_stride, int64_t gi_beam_stride, const float* x, int64_t x_stride,
                                 int64_t x_beam_stride, double* partial, int nbeam, hipStream_t s) {
  const int ntb = (nin + 255) / 256;
  const int64_t gx = (int64_t)ntb * nchan;
  if (gx > 0x7fffffff || nbeam > 65535) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(direct_adjoint_kernel, dim3((unsigned)gx, nbeam), dim3(256), 0, s, g, g_stride, g_beam_stride,
                     delta, nchan, ndm, nsamp, nin, w, grad_in, gi_stride, gi_beam_stride, x, x_stride, x_beam_stride,
                     partial, ntb);
  return hipGetLastError();
}

hipError_t launch_reduce_gradw(const double* partial, int nparts, int nchan, float* grad_w, hipStream_t s) {
  hipLaunchKernelGGL(reduce_gradw_kernel, dim3((nchan + 255) / 256), dim3(256), 0, s, partial, nparts, nchan, grad_w);
  return hipGetLastError();
}

}  // namespace dd

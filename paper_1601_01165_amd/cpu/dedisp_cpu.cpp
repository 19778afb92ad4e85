// Tuned multi-core CPU dedispersion (the declarations and the contract are in
// include/dedisp_cpu.h).  The paper compares its GPU kernels with an OpenMP
// implementation on CPUs and Xeon Phi (Section 5); this is that comparator:
// register tiles of dt DM trials x tt samples, SIMD across samples (each SIMD
// lane keeps Algorithm 1's ascending channel order, so results equal a
// sequential loop), OpenMP over blocks of DM trials x samples, channels in
// blocks whose rows stay in L1 while all the block's register tiles use them.
//
// The file is compiled once per instruction set (DDCPU_NS names the copy,
// with -mavx512f / -mavx2 -mfma / nothing) plus once with DDCPU_DISPATCH for
// the C entry points, which pick the widest copy the CPU supports.
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "../../include/dedisp_cpu.h"

namespace {
struct Cfg {
  int dt, tt;
};
constexpr Cfg kCfgs[] = {{1, 64}, {2, 64}, {4, 32}, {4, 64}, {4, 128}, {8, 32}, {8, 64}};
constexpr int kNumCfgs = sizeof(kCfgs) / sizeof(kCfgs[0]);
constexpr int kDmBlock = 64;     // DM trials per OpenMP work item
constexpr int kTimeBlock = 256;  // samples per OpenMP work item
constexpr int kChanBlock = 256;   // channels summed per pass over a work item's register tiles
}  // namespace

#ifndef DDCPU_DISPATCH

namespace DDCPU_NS {

// One register tile: DT DM trials (rows d0 .. d0 + nd - 1) x nt samples from
// t0, channels [c0, c1).  The partial sums live in `out` between channel
// blocks (exact: they are stored and reloaded as the same type).
template <int DT, int TT, bool WEIGHTED, typename TI, typename TA>
static inline void tile(const TI* in, int64_t is, const int32_t* delta, int nchan, int c0, int c1, int d0, int nd,
                        const float* w, TA* out, int64_t os, int t0, int nt) {
  TA acc[DT][TT];
  for (int d = 0; d < DT; ++d)
    for (int t = 0; t < TT; ++t) acc[d][t] = TA(0);
  if (c0 > 0)
    for (int d = 0; d < nd; ++d) std::memcpy(acc[d], out + (int64_t)(d0 + d) * os + t0, sizeof(TA) * nt);
  const int32_t* drow[DT];
  for (int d = 0; d < DT; ++d) drow[d] = delta + (int64_t)(d0 + std::min(d, nd - 1)) * nchan;
  if (nt == TT) {
    for (int c = c0; c < c1; ++c) {
      const TI* row = in + c * is + t0;
      const float wc = WEIGHTED ? w[c] : 1.f;
      for (int d = 0; d < DT; ++d) {
        const TI* src = row + drow[d][c];
#pragma omp simd
        for (int t = 0; t < TT; ++t) {
          if (WEIGHTED)
            acc[d][t] = acc[d][t] + wc * (TA)src[t];
          else
            acc[d][t] = acc[d][t] + (TA)src[t];
        }
      }
    }
  } else {
    for (int c = c0; c < c1; ++c) {
      const TI* row = in + c * is + t0;
      const float wc = WEIGHTED ? w[c] : 1.f;
      for (int d = 0; d < DT; ++d) {
        const TI* src = row + drow[d][c];
        for (int t = 0; t < nt; ++t) {
          if (WEIGHTED)
            acc[d][t] = acc[d][t] + wc * (TA)src[t];
          else
            acc[d][t] = acc[d][t] + (TA)src[t];
        }
      }
    }
  }
  for (int d = 0; d < nd; ++d) std::memcpy(out + (int64_t)(d0 + d) * os + t0, acc[d], sizeof(TA) * nt);
}

// OpenMP over (beam, DM block, time block); inside, channels in blocks of
// kChanBlock so the rows a block reads stay in L1 while every register tile
// of the work item consumes them.
template <int DT, int TT, bool WEIGHTED, typename TI, typename TA>
static void run(int nbeam, int nchan, int ndm, int nsamp, const TI* in, int64_t is, const int32_t* delta,
                const float* w, TA* out, int64_t os) {
  const int ndb = (ndm + kDmBlock - 1) / kDmBlock;
  const int ntb = (nsamp + kTimeBlock - 1) / kTimeBlock;
  const int64_t items = (int64_t)nbeam * ndb * ntb;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t k = 0; k < items; ++k) {
    const int b = (int)(k / ((int64_t)ndb * ntb));
    const int rem = (int)(k % ((int64_t)ndb * ntb));
    const int db = rem / ntb, tb = rem % ntb;
    const TI* inb = in + (int64_t)b * nchan * is;
    TA* outb = out + (int64_t)b * ndm * os;
    const int dlo = db * kDmBlock, dhi = std::min(ndm, dlo + kDmBlock);
    const int tlo = tb * kTimeBlock, thi = std::min(nsamp, tlo + kTimeBlock);
    for (int c0 = 0; c0 < nchan; c0 += kChanBlock) {
      const int c1 = std::min(nchan, c0 + kChanBlock);
      for (int d0 = dlo; d0 < dhi; d0 += DT)
        for (int t0 = tlo; t0 < thi; t0 += TT)
          tile<DT, TT, WEIGHTED, TI, TA>(inb, is, delta, nchan, c0, c1, d0, std::min(DT, dhi - d0), w, outb, os, t0,
                                         std::min(TT, thi - t0));
    }
  }
}

template <bool WEIGHTED, typename TI, typename TA>
static void dispatch_cfg(int cfg, int nbeam, int nchan, int ndm, int nsamp, const TI* in, int64_t is,
                         const int32_t* delta, const float* w, TA* out, int64_t os) {
  switch (cfg) {
#define CASE(I)                                                                                              \
  case I:                                                                                                    \
    run<kCfgs[I].dt, kCfgs[I].tt, WEIGHTED, TI, TA>(nbeam, nchan, ndm, nsamp, in, is, delta, w, out, os);    \
    break;
    CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6)
#undef CASE
    default:
      break;
  }
}

void forward_f32(int nbeam, int nchan, int ndm, int nsamp, const float* in, int64_t is, const int32_t* delta,
                 const float* w, float* out, int64_t os, int cfg) {
  if (w)
    dispatch_cfg<true, float, float>(cfg, nbeam, nchan, ndm, nsamp, in, is, delta, w, out, os);
  else
    dispatch_cfg<false, float, float>(cfg, nbeam, nchan, ndm, nsamp, in, is, delta, nullptr, out, os);
}

void forward_u8(int nbeam, int nchan, int ndm, int nsamp, const uint8_t* in, int64_t is, const int32_t* delta,
                int32_t* out, int64_t os, int cfg) {
  dispatch_cfg<false, uint8_t, int32_t>(cfg, nbeam, nchan, ndm, nsamp, in, is, delta, nullptr, out, os);
}

}  // namespace DDCPU_NS

#else  // DDCPU_DISPATCH

#include <omp.h>

#define DECL(NS)                                                                                              \
  namespace NS {                                                                                              \
  void forward_f32(int, int, int, int, const float*, int64_t, const int32_t*, const float*, float*, int64_t,   \
                   int);                                                                                      \
  void forward_u8(int, int, int, int, const uint8_t*, int64_t, const int32_t*, int32_t*, int64_t, int);        \
  }
DECL(ddcpu_avx512)
DECL(ddcpu_avx2)
DECL(ddcpu_generic)
#undef DECL

namespace {
int isa_level() {
  static const int lvl = [] {
    __builtin_cpu_init();
    if (__builtin_cpu_supports("avx512f")) return 2;
    if (__builtin_cpu_supports("avx2") && __builtin_cpu_supports("fma")) return 1;
    return 0;
  }();
  return lvl;
}

bool valid(int nbeam, int nchan, int ndm, int nsamp, const void* in, int64_t is, const int32_t* delta,
           const void* out, int64_t os, int cfg) {
  if (nbeam < 1 || nchan < 1 || ndm < 1 || nsamp < 1 || !in || !delta || !out) return false;
  if (cfg < 0 || cfg >= kNumCfgs || os < nsamp) return false;
  int32_t mx = 0;
  for (int64_t i = 0; i < (int64_t)ndm * nchan; ++i) {
    if (delta[i] < 0) return false;
    mx = std::max(mx, delta[i]);
  }
  return is >= (int64_t)nsamp + mx;
}
}  // namespace

extern "C" {

int ddcpu_forward_f32(int32_t nbeam, int32_t nchan, int32_t ndm, int32_t nsamp, const float* in, int64_t in_stride,
                      const int32_t* delta, const float* w, float* out, int64_t out_stride, int32_t cfg) {
  if (!valid(nbeam, nchan, ndm, nsamp, in, in_stride, delta, out, out_stride, cfg)) return 1;
  const int l = isa_level();
  if (l == 2)
    ddcpu_avx512::forward_f32(nbeam, nchan, ndm, nsamp, in, in_stride, delta, w, out, out_stride, cfg);
  else if (l == 1)
    ddcpu_avx2::forward_f32(nbeam, nchan, ndm, nsamp, in, in_stride, delta, w, out, out_stride, cfg);
  else
    ddcpu_generic::forward_f32(nbeam, nchan, ndm, nsamp, in, in_stride, delta, w, out, out_stride, cfg);
  return 0;
}

int ddcpu_forward_u8(int32_t nbeam, int32_t nchan, int32_t ndm, int32_t nsamp, const uint8_t* in, int64_t in_stride,
                     const int32_t* delta, int32_t* out, int64_t out_stride, int32_t cfg) {
  if (!valid(nbeam, nchan, ndm, nsamp, in, in_stride, delta, out, out_stride, cfg)) return 1;
  const int l = isa_level();
  if (l == 2)
    ddcpu_avx512::forward_u8(nbeam, nchan, ndm, nsamp, in, in_stride, delta, out, out_stride, cfg);
  else if (l == 1)
    ddcpu_avx2::forward_u8(nbeam, nchan, ndm, nsamp, in, in_stride, delta, out, out_stride, cfg);
  else
    ddcpu_generic::forward_u8(nbeam, nchan, ndm, nsamp, in, in_stride, delta, out, out_stride, cfg);
  return 0;
}

int32_t ddcpu_num_configs(void) { return kNumCfgs; }

int ddcpu_config(int32_t i, int32_t* dt, int32_t* tt) {
  if (i < 0 || i >= kNumCfgs || !dt || !tt) return 1;
  *dt = kCfgs[i].dt;
  *tt = kCfgs[i].tt;
  return 0;
}

int32_t ddcpu_num_threads(void) { return omp_get_max_threads(); }

const char* ddcpu_isa(void) {
  const int l = isa_level();
  return l == 2 ? "avx512f" : l == 1 ? "avx2" : "generic";
}

}  // extern "C"

#endif

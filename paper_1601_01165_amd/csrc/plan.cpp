// Host side of the dedispersion library: plans, delay tables, tile tables,
// argument validation and the forward / adjoint entry points of the C-ABI.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <climits>
#include <atomic>
#include <cstdio>
#include <functional>
#include <map>
#include <mutex>
#include <thread>
#include <limits>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

namespace dd {

static thread_local std::string g_last_error;

dedisp_status fail(dedisp_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

dedisp_status hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return DEDISP_E_HIP;
}

// ---------------------------------------------------------------------------
// Delay table (Section 2, Equation 1; computed ahead of time, Section 2.1).
//   f_h = highest channel frequency
//   k   = 4150 * DM * (1/f^2 - 1/f_h^2) seconds, f in MHz
//   delta = floor(k / tsamp + 1/2)
// ---------------------------------------------------------------------------
static dedisp_status build_delay_table(int nchan, const double* f, double tsamp, int ndm, const double* dm,
                                       std::vector<int32_t>& out, int& max_delay) {
  double fh = f[0];
  for (int c = 0; c < nchan; ++c) {
    if (!(f[c] > 0.0) || !std::isfinite(f[c])) return fail(DEDISP_E_INVALID, "channel frequency must be > 0 and finite");
    fh = std::max(fh, f[c]);
  }
  const double inv_fh2 = 1.0 / (fh * fh);
  out.assign((size_t)nchan * ndm, 0);
  max_delay = 0;
  for (int j = 0; j < ndm; ++j) {
    if (!(dm[j] >= 0.0) || !std::isfinite(dm[j])) return fail(DEDISP_E_INVALID, "DM must be >= 0 and finite");
    for (int c = 0; c < nchan; ++c) {
      const double kdelay = 4150.0 * dm[j] * (1.0 / (f[c] * f[c]) - inv_fh2);
      const double x = std::floor(kdelay / tsamp + 0.5);
      if (!(x >= 0.0) || x > 2147483647.0) return fail(DEDISP_E_SHAPE, "a delay does not fit in int32");
      out[(size_t)j * nchan + c] = (int32_t)x;
      max_delay = std::max(max_delay, (int)x);
    }
  }
  return DEDISP_OK;
}

// ---------------------------------------------------------------------------
// Tile tables.  `delay(r, c)` is the delay of output row r for input row c.
// Output rows are grouped in block tiles of v.dt() rows and wave tiles of
// v.dpw rows; rows past the end repeat the last row (their results are not
// stored).
// ---------------------------------------------------------------------------
// Runs f(i) for i in [0, n) on the host's cores (the tables of large plans
// and batches are built per block row tile, independently).
template <class F>
static void parallel_for(int n, F&& f) {
  const int nt = std::min<int>(n, std::max(1u, std::min(16u, std::thread::hardware_concurrency())));
  if (nt <= 1 || n < 4) {
    for (int i = 0; i < n; ++i) f(i);
    return;
  }
  std::atomic<int> next(0);
  std::vector<std::thread> th;
  th.reserve(nt);
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&]() {
      for (int i; (i = next.fetch_add(1)) < n;) f(i);
    });
  for (auto& x : th) x.join();
}

template <class DelayFn>
static bool build_tables(const Variant& v, int rows_out, int rows_in, const DelayFn& delay, std::vector<int32_t>& blk,
                         std::vector<int32_t>& wav, int& n_row_tiles, int& max_stage, std::string& why) {
  const int DT = v.dt(), DPW = v.dpw, NW = v.nwave, WI = v.wav_ints();
  if (v.kind == KIND_TILE_U8 && v.mode == 1 && rows_in > 256) {
    why = "more than 256 input rows overflow its packed sums";
    return false;
  }
  n_row_tiles = (rows_out + DT - 1) / DT;
  const int n_wave_tiles = n_row_tiles * NW;
  blk.assign((size_t)n_row_tiles * rows_in * 2, 0);
  wav.assign((size_t)n_wave_tiles * rows_in * WI, 0);
  std::vector<int> stage_max(n_row_tiles, 0);
  std::atomic<int> bad(0);  // 1: window span, 2: LDS row, 3: 16-bit offset
  parallel_for(n_row_tiles, [&](int rt) {
    std::vector<int> d(DT);
    int smax = 0;
    for (int c = 0; c < rows_in && !bad.load(std::memory_order_relaxed); ++c) {
      for (int k = 0; k < DT; ++k) d[k] = delay(std::min(rt * DT + k, rows_out - 1), c);
      if (v.kind == KIND_WIN_F32) {
        const int bmin = *std::min_element(d.begin(), d.end());
        const int sbase = bmin & ~3;
        int need = 0;
        for (int w = 0; w < NW; ++w) {
          const int* dw = &d[w * DPW];
          const int wmin = *std::min_element(dw, dw + DPW);
          const int ws = (wmin - sbase) & ~3;
          int maxo = 0;
          int32_t* e = &wav[(((size_t)(rt * NW + w)) * rows_in + c) * WI];
          for (int j = 0; j < DPW; ++j) {
            const int o = dw[j] - sbase - ws;
            if (o < 0 || o > v.nwin - v.tp) {
              bad.store(1);
              return;
            }
            maxo = std::max(maxo, o);
            e[2 + j] = v.jmp ? o * (4 * v.tp + 4) : o;
          }
          const int nl = std::max(v.tp / 4 + 1, (v.tp + maxo + 3) / 4);
          e[0] = ws;
          e[1] = nl;
          // full-window variants read all nwin samples of every row
          need = std::max(need, ws + 63 * v.tp + (v.jmp == 2 ? v.nwin : 4 * nl));
        }
        need = (need + 3) & ~3;
        if (need > v.rowcap) {
          bad.store(2);
          return;
        }
        blk[((size_t)rt * rows_in + c) * 2 + 0] = sbase;
        blk[((size_t)rt * rows_in + c) * 2 + 1] = need;
        smax = std::max(smax, need);
      } else {
        const int bmin = *std::min_element(d.begin(), d.end());
        const int sbase = bmin & ~15;
        int need = 0;
        for (int w = 0; w < NW; ++w) {
          const int* dw = &d[w * DPW];
          int32_t* e = &wav[(((size_t)(rt * NW + w)) * rows_in + c) * WI];
          for (int j = 0; j < DPW; ++j) {
            const int o = dw[j] - sbase;
            if (o < 0 || o > 65535) {
              bad.store(3);
              return;
            }
            if (v.mode == 0) {
              e[j / 2] |= (int32_t)((uint32_t)o << (16 * (j % 2)));
            } else {
              // byte offset into the staged copies: copy o & 3, row slot c % cc, dword o >> 2
              e[j] = 4 * (((o & 3) * v.cc + c % v.cc) * (v.rowcap / 4) + (o >> 2));
            }
            need = std::max(need, (o & ~3) + 256 * v.tp + 4);
          }
        }
        need = (need + 15) & ~15;
        if (need > v.rowcap) {
          bad.store(2);
          return;
        }
        blk[((size_t)rt * rows_in + c) * 2 + 0] = sbase;
        blk[((size_t)rt * rows_in + c) * 2 + 1] = need;
        smax = std::max(smax, need);
      }
    }
    stage_max[rt] = smax;
  });
  switch (bad.load()) {
    case 1: why = "delay span within a wave exceeds the register window"; return false;
    case 2: why = "delay span within a block exceeds the LDS row"; return false;
    case 3: why = "delay span exceeds the 16-bit offset range"; return false;
    default: break;
  }
  max_stage = 0;
  for (int m : stage_max) max_stage = std::max(max_stage, m);
  return true;
}

static void free_tables(Tables& t) {
  if (t.d_blk) (void)hipFree(t.d_blk);
  if (t.d_wav) (void)hipFree(t.d_wav);
  if (t.d_span) (void)hipFree(t.d_span);
  t = Tables();
}

void drop_spare_tables(dedisp_plan p, int dir, int keep) {
  std::map<int, Tables>& m = dir == 0 ? p->fwd_f32 : dir == 1 ? p->fwd_u8 : p->adj_f32;
  for (auto it = m.begin(); it != m.end();) {
    const int vi = it->first;
    const bool chosen = vi == keep || (dir == 0 && (vi == p->var_f32 || vi == p->var_det_f32)) ||
                        (dir == 1 && (vi == p->var_u8 || vi == p->var_det_u8)) || (dir == 2 && vi == p->var_adj);
    if (chosen || it->second.pins > 0) {
      ++it;
      continue;
    }
    free_tables(it->second);
    it = m.erase(it);
  }
}

// Build and upload the tables of variant `vi` in direction `dir`
// (0 = forward f32, 1 = forward u8, 2 = adjoint f32).
dedisp_status ensure_tables(dedisp_plan p, int dir, int vi, Tables** out) {
  std::map<int, Tables>& m = dir == 0 ? p->fwd_f32 : dir == 1 ? p->fwd_u8 : p->adj_f32;
  auto it = m.find(vi);
  if (it != m.end()) {
    if (out) *out = &it->second;
    return DEDISP_OK;
  }
  const std::vector<Variant>& vs = dir == 1 ? variants_u8() : variants_f32();
  if (vi < 0 || vi >= (int)vs.size()) return fail(DEDISP_E_INVALID, "variant index out of range");
  const Variant& v = vs[vi];
  std::vector<int32_t> blk, wav;
  int nrt = 0, maxs = 0;
  std::string why;
  bool ok;
  const int C = p->nchan, D = p->ndm;
  const int32_t* del = p->delay.data();
  if (dir == 2) {
    const int pad = p->adj_pad;
    ok = build_tables(v, C, D, [&](int r, int c) { return pad - del[(size_t)c * C + r]; }, blk, wav, nrt, maxs, why);
  } else {
    ok = build_tables(v, D, C, [&](int r, int c) { return del[(size_t)r * C + c]; }, blk, wav, nrt, maxs, why);
  }
  if (!ok) return fail(DEDISP_E_UNTUNED, std::string(v.name) + ": " + why);
  // The adjoint's input rows (DM trials) reach outside the output gradient's
  // samples for part of the time tiles: the span of each pass's staged
  // windows lets the kernel skip passes that would add only zeros.
  std::vector<int32_t> span;
  if (dir == 2) {
    const int rows_in = D, npass = (rows_in + v.cc - 1) / v.cc;
    span.assign((size_t)nrt * npass * 2, 0);
    for (int rt = 0; rt < nrt; ++rt)
      for (int q = 0; q < npass; ++q) {
        int smin = INT32_MAX, emax = INT32_MIN;
        for (int c = q * v.cc; c < std::min(rows_in, (q + 1) * v.cc); ++c) {
          const int32_t* b = &blk[((size_t)rt * rows_in + c) * 2];
          smin = std::min(smin, b[0]);
          emax = std::max(emax, b[0] + b[1]);
        }
        span[((size_t)rt * npass + q) * 2 + 0] = smin;
        span[((size_t)rt * npass + q) * 2 + 1] = emax;
      }
  }
  Tables t;
  t.variant = vi;
  t.n_row_tiles = nrt;
  t.n_wave_tiles = nrt * v.nwave;
  t.max_stage = maxs;
  t.bytes = (blk.size() + wav.size() + span.size()) * sizeof(int32_t);
  hipError_t e = hipMalloc(&t.d_blk, blk.size() * sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc(&t.d_wav, wav.size() * sizeof(int32_t));
  if (e == hipSuccess && !span.empty()) e = hipMalloc(&t.d_span, span.size() * sizeof(int32_t));
  if (e == hipSuccess) e = hipMemcpy(t.d_blk, blk.data(), blk.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(t.d_wav, wav.data(), wav.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess && !span.empty())
    e = hipMemcpy(t.d_span, span.data(), span.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    free_tables(t);
    return e == hipErrorOutOfMemory ? fail(DEDISP_E_NOMEM, "device allocation of tile tables failed")
                                    : hip_fail(e, "uploading tile tables");
  }
  auto res = m.emplace(vi, t);
  if (out) *out = &res.first->second;
  return DEDISP_OK;
}

// Variant preference when nothing was tuned, fastest first as measured on
// MI355X: forward FP32 on the 1024-channel, 2048-DM beam; forward uint8 on the
// 32-channel, 2048-DM beam; the adjoint on 32 beams of 1024 channels and
// 1024 DMs.  Variants with wide register windows or int32 sums come last:
// they fit the widest delay spans and the most channels.
const std::vector<int>& default_order(int dir) {
  static const std::vector<int> f32 = {35, 34, 37, 38, 36, 32, 33, 22, 28, 21, 29, 31, 23, 30, 19, 20, 25, 24, 27, 26, 15, 18, 13,
                                       17, 9,  8,  16, 6,  14, 11, 7,  12, 10, 2,  3,  0,  1,  5,  4};
  static const std::vector<int> u8 = {22, 16, 20, 15, 21, 12, 13, 17, 14, 18, 6, 2, 0, 5, 19, 9, 3, 4, 1, 8, 7, 10, 11};
  static const std::vector<int> adj = {37, 38, 26, 27, 32, 34, 35, 36, 33, 19, 21, 29, 20, 30, 9, 8, 6, 11, 12, 7, 10, 13, 22, 28,
                                       18, 15, 23, 31, 17, 16, 25, 24, 14, 2, 3, 1, 0, 5, 4};
  return dir == 1 ? u8 : dir == 2 ? adj : f32;
}

// Default variant choice: the first of the preference order whose tables
// build (else -1, the direct kernel).
static int default_variant(dedisp_plan p, int dir) {
  for (int vi : default_order(dir))
    if (ensure_tables(p, dir, vi, nullptr) == DEDISP_OK) return vi;
  return -1;
}

static bool aligned16(const void* ptr) { return ((uintptr_t)ptr & 15u) == 0; }

// The uint8 and adjoint kernels are chosen (and their tables built) on first
// use or by dedisp_plan_prepare; -2 marks "not chosen yet".
static void ensure_chosen(dedisp_plan p, int dir) {
  int& v = dir == 0 ? p->var_f32 : dir == 1 ? p->var_u8 : p->var_adj;
  if (v == -2) v = default_variant(p, dir);
}

// Scratch of the allocation-free adjoint (dedisp_adjoint_noalloc): the
// per-tile FP64 partial sums of the weight gradient.  Every GPU the library
// runs on holds its own copy until the process ends.  Host code never uses
// the array's name as an address: the device address of the current
// device's copy comes from scratch_address().
constexpr size_t kNoAllocScratchBytes = DEDISP_ADJOINT_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

// Device address of the current device's scratch, looked up once per device
// (at plan creation, with that device current); nullptr with the error set
// if the lookup fails.
static void* scratch_address(int device) {
  static std::mutex mu;
  static std::map<int, void*> addr;
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(device);
  if (it != addr.end()) return it->second;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hip_fail(e == hipSuccess ? hipErrorInvalidSymbol : e, "looking up the adjoint scratch array");
    return nullptr;
  }
  addr[device] = ptr;
  return ptr;
}

// The adjoint's launches with the partial-sum buffer given (null when no
// weight gradient is asked for).  With may_allocate false the plan's chosen
// adjoint variant and its tables must exist already (nothing is built).
static dedisp_status adjoint_impl(dedisp_plan p, int32_t nbeam, int32_t nsamp, int32_t nin, const float* d_g,
                                  int64_t g_stride, const float* d_w, const float* d_in, int64_t in_stride,
                                  float* d_grad_in, int64_t gi_stride, float* d_grad_w, double* partial,
                                  hipStream_t s, bool may_allocate) {
  hipError_t e;
  int nparts;
  if (may_allocate) {
    ensure_chosen(p, 2);
  } else if (p->var_adj == -2) {
    return fail(DEDISP_E_INVALID, "the adjoint kernel is not chosen yet: call dedisp_plan_prepare first");
  }
  const int vi = p->var_adj;
  if (vi < 0) {
    e = launch_direct_adjoint(d_g, g_stride, g_stride * p->ndm, p->d_delay, p->nchan, p->ndm, nsamp, nin, d_w,
                              d_grad_in, gi_stride, gi_stride * p->nchan, d_in, in_stride, in_stride * p->nchan,
                              partial, nbeam, s);
    if (e != hipSuccess) return hip_fail(e, "launching the direct adjoint kernel");
    nparts = nbeam * ((nin + 255) / 256);
  } else {
    Tables* t = nullptr;
    if (may_allocate) {
      dedisp_status st = ensure_tables(p, 2, vi, &t);
      if (st != DEDISP_OK) return st;
    } else {
      auto it = p->adj_f32.find(vi);
      if (it == p->adj_f32.end())
        return fail(DEDISP_E_INVALID, "the adjoint tile tables are not built: call dedisp_plan_prepare first");
      t = &it->second;
    }
    const Variant& v = variants_f32()[vi];
    TileArgs a = {};
    a.in = d_g;
    a.in_stride = g_stride;
    a.in_beam_stride = g_stride * p->ndm;
    a.in_shift = -p->adj_pad;
    a.in_lo = p->adj_pad;
    a.in_hi = p->adj_pad + nsamp;
    a.rows_in = p->ndm;
    a.rows_out = p->nchan;
    a.nout = nin;
    a.n_time_tiles = (nin + v.st() - 1) / v.st();
    a.n_row_tiles = t->n_row_tiles;
    a.blk = t->d_blk;
    a.wav = t->d_wav;
    a.span = t->d_span;
    a.w_in = nullptr;
    a.out = d_grad_in;
    a.out_stride = gi_stride;
    a.out_beam_stride = gi_stride * p->nchan;
    a.w_out = d_w;
    a.x = d_in;
    a.x_stride = in_stride;
    a.x_beam_stride = in_stride * p->nchan;
    a.partial = partial;
    e = launch_tiled(v, a, nbeam, true, s);
    if (e != hipSuccess) return hip_fail(e, "launching the tiled adjoint kernel");
    nparts = nbeam * a.n_time_tiles;
  }
  if (d_grad_w) {
    e = launch_reduce_gradw(partial, nparts, p->nchan, d_grad_w, s);
    if (e != hipSuccess) return hip_fail(e, "launching the grad_w reduction");
  }
  return DEDISP_OK;
}

// Argument checks shared by both adjoint entry points.
static dedisp_status adjoint_check(dedisp_plan p, int32_t nbeam, int32_t nsamp, int32_t nin, const float* d_g,
                                   int64_t g_stride, const float* d_w, const float* d_in, int64_t in_stride,
                                   float* d_grad_in, int64_t gi_stride, float* d_grad_w) {
  if (!p) return fail(DEDISP_E_INVALID, "plan is NULL");
  if (nbeam < 1 || nsamp < 1 || nin < 1) return fail(DEDISP_E_INVALID, "nbeam, nsamp and nin must be >= 1");
  if (nbeam > kMaxBeams) return fail(DEDISP_E_SHAPE, "at most 65535 beams per call");
  if (!d_g) return fail(DEDISP_E_INVALID, "output gradient is NULL");
  if (d_grad_w && !d_in) return fail(DEDISP_E_INVALID, "grad_w needs the forward input");
  if (g_stride < nsamp) return fail(DEDISP_E_SHAPE, "g_stride < nsamp");
  if (d_grad_in && gi_stride < nin) return fail(DEDISP_E_SHAPE, "gi_stride < nin");
  if (d_in && in_stride < nin) return fail(DEDISP_E_SHAPE, "in_stride < nin");
  if ((int64_t)nsamp + p->max_delay > nin) return fail(DEDISP_E_SHAPE, "nin < nsamp + max_delay");
  if (nin > kMaxRow || g_stride > kMaxRow || (d_in && in_stride > kMaxRow) || (d_grad_in && gi_stride > kMaxRow))
    return fail(DEDISP_E_SHAPE, "rows longer than 2^29 samples are not supported");
  if (!aligned16(d_g) || (g_stride * 4) % 16 || (d_grad_in && (!aligned16(d_grad_in) || (gi_stride * 4) % 16)) ||
      (d_in && (!aligned16(d_in) || (in_stride * 4) % 16)) || (d_w && ((uintptr_t)d_w & 3)))
    return fail(DEDISP_E_ALIGN, "pointers and row byte sizes must be multiples of 16 bytes");
  return DEDISP_OK;
}

}  // namespace dd

using namespace dd;

extern "C" {

const char* dedisp_status_string(dedisp_status s) {
  switch (s) {
    case DEDISP_OK: return "ok";
    case DEDISP_E_INVALID: return "invalid argument";
    case DEDISP_E_SHAPE: return "invalid shape or stride";
    case DEDISP_E_DTYPE: return "unsupported data type";
    case DEDISP_E_ALIGN: return "misaligned pointer or row";
    case DEDISP_E_NOMEM: return "out of memory";
    case DEDISP_E_HIP: return "HIP runtime error";
    case DEDISP_E_UNTUNED: return "no kernel variant fits";
    case DEDISP_E_WORKSPACE: return "workspace too small";
  }
  return "unknown status";
}

const char* dedisp_last_error(void) { return g_last_error.c_str(); }

dedisp_status dedisp_plan_create(dedisp_plan* plan, int32_t nchan, const double* freq_mhz, double tsamp_s,
                                 int32_t ndm, const double* dm) {
  if (!plan) return fail(DEDISP_E_INVALID, "plan pointer is NULL");
  *plan = nullptr;
  if (nchan < 1 || ndm < 1) return fail(DEDISP_E_INVALID, "nchan and ndm must be >= 1");
  if (!freq_mhz || !dm) return fail(DEDISP_E_INVALID, "frequency or DM array is NULL");
  if (!(tsamp_s > 0.0) || !std::isfinite(tsamp_s)) return fail(DEDISP_E_INVALID, "tsamp must be > 0 and finite");
  dedisp_plan p = new (std::nothrow) dedisp_plan_s();
  if (!p) return fail(DEDISP_E_NOMEM, "host allocation failed");
  p->nchan = nchan;
  p->ndm = ndm;
  p->tsamp = tsamp_s;
  p->freq.assign(freq_mhz, freq_mhz + nchan);
  p->dm.assign(dm, dm + ndm);
  dedisp_status st = build_delay_table(nchan, freq_mhz, tsamp_s, ndm, dm, p->delay, p->max_delay);
  if (st != DEDISP_OK) {
    delete p;
    return st;
  }
  p->adj_pad = (p->max_delay + 3) & ~3;
  hipError_t e = hipGetDevice(&p->device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&p->ncu, hipDeviceAttributeMultiprocessorCount, p->device);
  if (e == hipSuccess && p->ncu < 1) p->ncu = 1;
  if (e == hipSuccess) e = hipMalloc(&p->d_delay, p->delay.size() * sizeof(int32_t));
  if (e == hipSuccess)
    e = hipMemcpy(p->d_delay, p->delay.data(), p->delay.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    st = hip_fail(e, "uploading the delay table");
    dedisp_plan_destroy(p);
    return st;
  }
  // the allocation-free adjoint's scratch on this device, looked up once
  if (!scratch_address(p->device)) {
    st = DEDISP_E_HIP;
    dedisp_plan_destroy(p);
    return st;
  }
  p->var_f32 = default_variant(p, 0);
  *plan = p;
  return DEDISP_OK;
}

dedisp_status dedisp_compute_delays(int32_t nchan, const double* freq_mhz, double tsamp_s, int32_t ndm,
                                    const double* dm, int32_t* host, int32_t* max_delay) {
  if (nchan < 1 || ndm < 1) return fail(DEDISP_E_INVALID, "nchan and ndm must be >= 1");
  if (!freq_mhz || !dm || !host) return fail(DEDISP_E_INVALID, "an array pointer is NULL");
  if (!(tsamp_s > 0.0) || !std::isfinite(tsamp_s)) return fail(DEDISP_E_INVALID, "tsamp must be > 0 and finite");
  std::vector<int32_t> t;
  int md = 0;
  dedisp_status st = build_delay_table(nchan, freq_mhz, tsamp_s, ndm, dm, t, md);
  if (st != DEDISP_OK) return st;
  memcpy(host, t.data(), t.size() * sizeof(int32_t));
  if (max_delay) *max_delay = md;
  return DEDISP_OK;
}

dedisp_status dedisp_plan_destroy(dedisp_plan p) {
  if (!p) return DEDISP_OK;
  for (auto* m : {&p->fwd_f32, &p->fwd_u8, &p->adj_f32})
    for (auto& kv : *m) free_tables(kv.second);
  if (p->d_delay) (void)hipFree(p->d_delay);
  delete p;
  return DEDISP_OK;
}

dedisp_status dedisp_plan_info(dedisp_plan p, int32_t* nchan, int32_t* ndm, int32_t* max_delay) {
  if (!p) return fail(DEDISP_E_INVALID, "plan is NULL");
  if (nchan) *nchan = p->nchan;
  if (ndm) *ndm = p->ndm;
  if (max_delay) *max_delay = p->max_delay;
  return DEDISP_OK;
}

dedisp_status dedisp_plan_delays(dedisp_plan p, int32_t* host) {
  if (!p || !host) return fail(DEDISP_E_INVALID, "plan or output is NULL");
  memcpy(host, p->delay.data(), p->delay.size() * sizeof(int32_t));
  return DEDISP_OK;
}

int32_t dedisp_variant_count(dedisp_dtype t) {
  return t == DEDISP_U8 ? (int32_t)variants_u8().size() : t == DEDISP_F32 ? (int32_t)variants_f32().size() : 0;
}

const char* dedisp_variant_name(dedisp_dtype t, int32_t i) {
  if (t == DEDISP_U8 && i >= 0 && i < (int)variants_u8().size()) return variants_u8()[i].name;
  if (t == DEDISP_F32 && i >= 0 && i < (int)variants_f32().size()) return variants_f32()[i].name;
  return nullptr;
}

dedisp_status dedisp_plan_set_variant(dedisp_plan p, dedisp_dtype t, int32_t vi) {
  if (!p) return fail(DEDISP_E_INVALID, "plan is NULL");
  if (t != DEDISP_F32 && t != DEDISP_U8) return fail(DEDISP_E_DTYPE, "dtype must be F32 or U8");
  const int dir = t == DEDISP_U8 ? 1 : 0;
  if (vi >= 0) {
    dedisp_status st = ensure_tables(p, dir, vi, nullptr);
    if (st != DEDISP_OK) return st;
  } else if (vi != -1) {
    return fail(DEDISP_E_INVALID, "variant must be >= -1");
  }
  (t == DEDISP_U8 ? p->var_u8 : p->var_f32) = vi;
  return DEDISP_OK;
}

int32_t dedisp_plan_variant(dedisp_plan p, dedisp_dtype t) {
  if (!p) return -2;
  ensure_chosen(p, t == DEDISP_U8 ? 1 : 0);
  return t == DEDISP_U8 ? p->var_u8 : p->var_f32;
}

dedisp_status dedisp_plan_set_adjoint_variant(dedisp_plan p, int32_t vi) {
  if (!p) return fail(DEDISP_E_INVALID, "plan is NULL");
  if (vi >= 0) {
    dedisp_status st = ensure_tables(p, 2, vi, nullptr);
    if (st != DEDISP_OK) return st;
  } else if (vi != -1) {
    return fail(DEDISP_E_INVALID, "variant must be >= -1");
  }
  p->var_adj = vi;
  return DEDISP_OK;
}

int32_t dedisp_plan_adjoint_variant(dedisp_plan p) {
  if (!p) return -2;
  ensure_chosen(p, 2);
  return p->var_adj;
}

dedisp_status dedisp_plan_prepare(dedisp_plan p, dedisp_dtype t, int32_t adjoint) {
  if (!p) return fail(DEDISP_E_INVALID, "plan is NULL");
  if (t != DEDISP_F32 && t != DEDISP_U8) return fail(DEDISP_E_DTYPE, "dtype must be F32 or U8");
  if (adjoint && t != DEDISP_F32) return fail(DEDISP_E_DTYPE, "the adjoint is float32 only");
  const int dir = adjoint ? 2 : (t == DEDISP_U8 ? 1 : 0);
  ensure_chosen(p, dir);
  const int v = dir == 0 ? p->var_f32 : dir == 1 ? p->var_u8 : p->var_adj;
  return v < 0 ? DEDISP_OK : ensure_tables(p, dir, v, nullptr);
}

dedisp_status dedisp_execute(dedisp_plan p, int32_t nbeam, int32_t nsamp, const void* d_in, dedisp_dtype in_type,
                             int64_t in_stride, const float* d_w, void* d_out, dedisp_dtype out_type,
                             int64_t out_stride, void* stream) {
  if (!p) return fail(DEDISP_E_INVALID, "plan is NULL");
  if (nbeam < 1 || nsamp < 1) return fail(DEDISP_E_INVALID, "nbeam and nsamp must be >= 1");
  if (nbeam > kMaxBeams) return fail(DEDISP_E_SHAPE, "at most 65535 beams per call");
  if (!d_in || !d_out) return fail(DEDISP_E_INVALID, "input or output pointer is NULL");
  const bool f32 = in_type == DEDISP_F32 && out_type == DEDISP_F32;
  const bool u8 = in_type == DEDISP_U8 && out_type == DEDISP_I32;
  if (!f32 && !u8) return fail(DEDISP_E_DTYPE, "supported pairs: F32->F32, U8->I32");
  if (u8 && d_w) return fail(DEDISP_E_DTYPE, "weights are not supported for uint8 input");
  if (in_stride < (int64_t)nsamp + p->max_delay) return fail(DEDISP_E_SHAPE, "in_stride < nsamp + max_delay");
  if (out_stride < nsamp) return fail(DEDISP_E_SHAPE, "out_stride < nsamp");
  if (in_stride > kMaxRow || (int64_t)nsamp + p->max_delay > kMaxRow)
    return fail(DEDISP_E_SHAPE, "rows longer than 2^29 samples are not supported");
  const int esz = u8 ? 1 : 4;
  if (!aligned16(d_in) || !aligned16(d_out) || (in_stride * esz) % 16 || (out_stride * 4) % 16 ||
      (d_w && ((uintptr_t)d_w & 3)))
    return fail(DEDISP_E_ALIGN, "pointers and row byte sizes must be multiples of 16 bytes");
  hipStream_t s = (hipStream_t)stream;
  ensure_chosen(p, u8 ? 1 : 0);
  const int vi = u8 ? p->var_u8 : p->var_f32;
  hipError_t e;
  if (vi < 0) {
    if (u8)
      e = launch_direct_u8((const uint8_t*)d_in, in_stride, in_stride * p->nchan, p->d_delay, p->nchan, p->ndm,
                           (int32_t*)d_out, out_stride, out_stride * p->ndm, nsamp, nbeam, s);
    else
      e = launch_direct_f32((const float*)d_in, in_stride, in_stride * p->nchan, p->d_delay, p->nchan, p->ndm, d_w,
                            (float*)d_out, out_stride, out_stride * p->ndm, nsamp, nbeam, s);
    return e == hipSuccess ? DEDISP_OK : hip_fail(e, "launching the direct kernel");
  }
  const int dir = u8 ? 1 : 0;
  Tables* t = nullptr;
  dedisp_status st = ensure_tables(p, dir, vi, &t);
  if (st != DEDISP_OK) return st;
  const Variant& v = (u8 ? variants_u8() : variants_f32())[vi];
  TileArgs a = {};
  a.in = d_in;
  a.in_stride = in_stride;
  a.in_beam_stride = in_stride * p->nchan;
  a.in_shift = 0;
  a.in_lo = 0;
  a.in_hi = (int)in_stride;
  a.rows_in = p->nchan;
  a.rows_out = p->ndm;
  a.nout = nsamp;
  a.n_time_tiles = (nsamp + v.st() - 1) / v.st();
  a.n_row_tiles = t->n_row_tiles;
  // blocks that walk several time tiles: about six per CU in total
  a.tiles_per_block = (int)std::max<int64_t>(
      1, std::min<int64_t>(a.n_time_tiles, (int64_t)a.n_time_tiles * a.n_row_tiles * nbeam / (6 * p->ncu)));
  a.blk = t->d_blk;
  a.wav = t->d_wav;
  a.w_in = d_w;
  a.out = d_out;
  a.out_stride = out_stride;
  a.out_beam_stride = out_stride * p->ndm;
  e = launch_tiled(v, a, nbeam, false, s);
  return e == hipSuccess ? DEDISP_OK : hip_fail(e, "launching the tiled kernel");
}

size_t dedisp_adjoint_workspace_bytes(dedisp_plan p, int32_t nbeam, int32_t nin) {
  if (!p || nbeam < 1 || nin < 1) return 0;
  // Enough for the direct kernel (256-sample parts) and every tiled variant.
  const int64_t parts = (int64_t)nbeam * ((nin + 255) / 256);
  return (size_t)parts * p->nchan * sizeof(double);
}

dedisp_status dedisp_adjoint(dedisp_plan p, int32_t nbeam, int32_t nsamp, int32_t nin, const float* d_g,
                             int64_t g_stride, const float* d_w, const float* d_in, int64_t in_stride,
                             float* d_grad_in, int64_t gi_stride, float* d_grad_w, void* d_ws, size_t ws_bytes,
                             void* stream) {
  dedisp_status st =
      adjoint_check(p, nbeam, nsamp, nin, d_g, g_stride, d_w, d_in, in_stride, d_grad_in, gi_stride, d_grad_w);
  if (st != DEDISP_OK) return st;
  if (!d_grad_in && !d_grad_w) return DEDISP_OK;
  if (d_grad_w) {
    if (!d_ws) return fail(DEDISP_E_WORKSPACE, "workspace is NULL");
    if (ws_bytes < dedisp_adjoint_workspace_bytes(p, nbeam, nin)) return fail(DEDISP_E_WORKSPACE, "workspace too small");
    if ((uintptr_t)d_ws & 7) return fail(DEDISP_E_ALIGN, "workspace must be 8-byte aligned");
  }
  return adjoint_impl(p, nbeam, nsamp, nin, d_g, g_stride, d_w, d_in, in_stride, d_grad_in, gi_stride, d_grad_w,
                      d_grad_w ? (double*)d_ws : nullptr, (hipStream_t)stream, true);
}

size_t dedisp_adjoint_noalloc_bytes(dedisp_plan p, int32_t nbeam, int32_t nin) {
  if (!p || nbeam < 1 || nin < 1 || p->var_adj == -2) return 0;
  const int vi = p->var_adj;
  // one FP64 partial sum per channel and (beam, time part): 256-sample parts
  // for the direct kernel, the variant's time tiles otherwise
  const int64_t part = vi < 0 ? 256 : variants_f32()[vi].st();
  return (size_t)nbeam * (size_t)((nin + part - 1) / part) * (size_t)p->nchan * sizeof(double);
}

dedisp_status dedisp_adjoint_noalloc(dedisp_plan p, int32_t nbeam, int32_t nsamp, int32_t nin, const float* d_g,
                                     int64_t g_stride, const float* d_w, const float* d_in, int64_t in_stride,
                                     float* d_grad_in, int64_t gi_stride, float* d_grad_w, void* stream) {
  dedisp_status st =
      adjoint_check(p, nbeam, nsamp, nin, d_g, g_stride, d_w, d_in, in_stride, d_grad_in, gi_stride, d_grad_w);
  if (st != DEDISP_OK) return st;
  if (!d_grad_in && !d_grad_w) return DEDISP_OK;
  if (p->var_adj == -2)
    return fail(DEDISP_E_INVALID, "the adjoint kernel is not chosen yet: call dedisp_plan_prepare first");
  double* partial = nullptr;
  if (d_grad_w) {
    const size_t need = dedisp_adjoint_noalloc_bytes(p, nbeam, nin);
    if (need > kNoAllocScratchBytes)
      return fail(DEDISP_E_WORKSPACE, "the weight gradient's partial sums (" + std::to_string(need) +
                                          " bytes) exceed the fixed scratch of " +
                                          std::to_string(kNoAllocScratchBytes) + " bytes; use dedisp_adjoint");
    int dev = 0;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "querying the current device");
    if (dev != p->device) return fail(DEDISP_E_INVALID, "the plan belongs to another device");
    partial = static_cast<double*>(scratch_address(dev));
    if (!partial) return DEDISP_E_HIP;
  }
  return adjoint_impl(p, nbeam, nsamp, nin, d_g, g_stride, d_w, d_in, in_stride, d_grad_in, gi_stride, d_grad_w,
                      partial, (hipStream_t)stream, false);
}

}  // extern "C"

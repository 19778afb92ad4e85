// Host side of the single-pulse search (boxcar S/N over every dedispersed
// series, the detection step of the real-time pipeline of Section 1): the
// fused path runs a tile kernel whose epilogue searches the tile instead of
// storing it, then merges the per-tile records; the unfused path searches
// stored rows.  The definition is documented with dedisp_detect.
#include <string>

#include "internal.h"

namespace dd {
dedisp_status ensure_tables(dedisp_plan p, int dir, int vi, Tables** out);

// Keys of the uint8 search hold (window sum << IB) in 31 bits: prefix sums over
// a lane's run and look-ahead must stay below 2^30.
static bool u8_sums_fit(const Variant& v, int nchan) {
  const int run = 4 * v.tp;
  const double scale = (double)run;  // 2^IB == run
  return (double)(run + kDetLook - 1) * 255.0 * nchan * scale < (double)(1 << 30);
}

static bool det_fits(dedisp_plan p, bool u8, int vi) {
  const std::vector<Variant>& vs = u8 ? variants_u8() : variants_f32();
  if (vi < 0 || vi >= (int)vs.size()) return false;
  const Variant& v = vs[vi];
  if (!detect_fusable(v)) return false;
  if (u8 && !u8_sums_fit(v, p->nchan)) return false;
  return ensure_tables(p, u8 ? 1 : 0, vi, nullptr) == DEDISP_OK;
}

// The variant of the search for this plan and dtype: the one set or tuned
// (-1: unfused); otherwise the first that fits from a preference list
// (fastest first as measured on MI355X with the search fused: FP32 on the
// 1024-channel, 2048-DM beam, uint8 on the 32-channel, 2048-DM beam), else -1.
static int det_variant(dedisp_plan p, bool u8) {
  const int set = u8 ? p->var_det_u8 : p->var_det_f32;
  if (set >= -1) return set;
  auto fits = [&](int vi) { return det_fits(p, u8, vi); };
  static const int pref_f32[] = {16, 14, 18, 13, 15, 17};
  static const int pref_u8[] = {14, 16, 15, 12, 17, 18, 20, 13, 21, 19};
  if (u8) {
    for (int vi : pref_u8)
      if (fits(vi)) return vi;
  } else {
    for (int vi : pref_f32)
      if (fits(vi)) return vi;
  }
  return -1;
}

static size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

static int64_t rows_tiles(int nsamp) { return (nsamp + kDetRowsStep - 1) / kDetRowsStep; }

static size_t rows_ws(int64_t nrows, int nsamp) { return (size_t)nrows * rows_tiles(nsamp) * sizeof(DetRec); }

// Unfused fallback: forward into the workspace, then the row search.
static size_t fallback_ws(dedisp_plan p, int nbeam, int nsamp) {
  const int64_t nrows = (int64_t)nbeam * p->ndm;
  const size_t rows = round_up((size_t)nrows * round_up(nsamp, 4) * 4, 256);
  return rows + rows_ws(nrows, nsamp);
}

}  // namespace dd

using namespace dd;

extern "C" {

size_t dedisp_detect_workspace_bytes(dedisp_plan p, dedisp_dtype in_type, int32_t nbeam, int32_t nsamp) {
  if (!p || nbeam < 1 || nsamp < 1 || (in_type != DEDISP_F32 && in_type != DEDISP_U8)) return 0;
  const bool u8 = in_type == DEDISP_U8;
  const int vi = det_variant(p, u8);
  if (vi < 0) return fallback_ws(p, nbeam, nsamp);
  const Variant& v = (u8 ? variants_u8() : variants_f32())[vi];
  const int64_t ntiles = (nsamp + det_step(v) - 1) / det_step(v);
  return (size_t)nbeam * p->ndm * ntiles * sizeof(DetRec);
}

int32_t dedisp_detect_variant(dedisp_plan p, dedisp_dtype in_type) {
  if (!p || (in_type != DEDISP_F32 && in_type != DEDISP_U8)) return -1;
  return det_variant(p, in_type == DEDISP_U8);
}

static dedisp_status check_outputs(int32_t nwidth, const double* d_snr, const int32_t* d_width,
                                   const int32_t* d_start) {
  if (nwidth < 1 || nwidth > kDetNW) return fail(DEDISP_E_INVALID, "nwidth must be in [1, 6]");
  if (!d_snr || !d_width || !d_start) return fail(DEDISP_E_INVALID, "snr, width and start must not be NULL");
  return DEDISP_OK;
}

dedisp_status dedisp_detect(dedisp_plan p, int32_t nbeam, int32_t nsamp, const void* d_in, dedisp_dtype in_type,
                            int64_t in_stride, const float* d_w, int32_t nwidth, double* d_snr, int32_t* d_width,
                            int32_t* d_start, double* d_mean, double* d_std, void* d_ws, size_t ws_bytes,
                            void* stream) {
  if (!p) return fail(DEDISP_E_INVALID, "plan is NULL");
  if (nbeam < 1 || nsamp < 1) return fail(DEDISP_E_INVALID, "nbeam and nsamp must be >= 1");
  if (nbeam > kMaxBeams) return fail(DEDISP_E_SHAPE, "at most 65535 beams per call");
  if (!d_in) return fail(DEDISP_E_INVALID, "input pointer is NULL");
  dedisp_status st = check_outputs(nwidth, d_snr, d_width, d_start);
  if (st != DEDISP_OK) return st;
  const bool u8 = in_type == DEDISP_U8;
  if (!u8 && in_type != DEDISP_F32) return fail(DEDISP_E_DTYPE, "input must be F32 or U8");
  if (u8 && d_w) return fail(DEDISP_E_DTYPE, "weights are not supported for uint8 input");
  if (in_stride < (int64_t)nsamp + p->max_delay) return fail(DEDISP_E_SHAPE, "in_stride < nsamp + max_delay");
  if (in_stride > kMaxRow || (int64_t)nsamp + p->max_delay > kMaxRow)
    return fail(DEDISP_E_SHAPE, "rows longer than 2^29 samples are not supported");
  const int esz = u8 ? 1 : 4;
  if (((uintptr_t)d_in & 15u) || (in_stride * esz) % 16 || (d_w && ((uintptr_t)d_w & 3)))
    return fail(DEDISP_E_ALIGN, "pointers and row byte sizes must be multiples of 16 bytes");
  if (!d_ws) return fail(DEDISP_E_WORKSPACE, "workspace is NULL");
  if ((uintptr_t)d_ws & 15u) return fail(DEDISP_E_ALIGN, "workspace must be 16-byte aligned");
  if (ws_bytes < dedisp_detect_workspace_bytes(p, in_type, nbeam, nsamp))
    return fail(DEDISP_E_WORKSPACE, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  const int64_t nseries = (int64_t)nbeam * p->ndm;
  if (nseries > 0x7ffffff0) return fail(DEDISP_E_SHAPE, "too many series");
  const int vi = det_variant(p, u8);
  hipError_t e;
  if (vi < 0) {
    // unfused (no variant with the search in its epilogue fits, or the
    // unfused path was set or tuned): dedisperse into the workspace, then
    // search the stored rows
    const int64_t stride = round_up(nsamp, 4);
    void* rows = d_ws;
    DetRec* recs = (DetRec*)((char*)d_ws + round_up((size_t)nseries * stride * 4, 256));
    st = dedisp_execute(p, nbeam, nsamp, d_in, in_type, in_stride, d_w, rows, u8 ? DEDISP_I32 : DEDISP_F32, stride,
                        stream);
    if (st != DEDISP_OK) return st;
    const int ntiles = (int)rows_tiles(nsamp);
    e = launch_detect_rows(rows, u8, stride, (int)nseries, nsamp, ntiles, recs, s);
    if (e != hipSuccess) return hip_fail(e, "launching the row search");
    e = launch_det_finish(recs, false, (int)nseries, ntiles, nsamp, nwidth, d_snr, d_width, d_start, d_mean, d_std,
                          s);
    return e == hipSuccess ? DEDISP_OK : hip_fail(e, "launching the record merge");
  }
  Tables* t = nullptr;
  st = ensure_tables(p, u8 ? 1 : 0, vi, &t);
  if (st != DEDISP_OK) return st;
  const Variant& v = (u8 ? variants_u8() : variants_f32())[vi];
  const int step = det_step(v);
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
  a.n_time_tiles = (nsamp + step - 1) / step;
  a.n_row_tiles = t->n_row_tiles;
  a.tiles_per_block = 1;
  a.blk = t->d_blk;
  a.wav = t->d_wav;
  a.w_in = d_w;
  a.out = nullptr;
  a.tile_step = step;
  a.det_nsamp = nsamp;
  // a lane's sum of squares in 32 bits: run * (255 * nchan)^2 < 2^32
  a.det_s2_u32 = u8 && (double)(4 * v.tp) * (255.0 * p->nchan) * (255.0 * p->nchan) < 4294967296.0;
  a.det = (DetRec*)d_ws;
  e = launch_detect(v, a, nbeam, s);
  if (e != hipSuccess) return hip_fail(e, "launching the fused search");
  e = launch_det_finish(a.det, u8, (int)nseries, a.n_time_tiles, nsamp, nwidth, d_snr, d_width, d_start, d_mean,
                        d_std, s);
  return e == hipSuccess ? DEDISP_OK : hip_fail(e, "launching the record merge");
}

dedisp_status dedisp_plan_set_detect_variant(dedisp_plan p, dedisp_dtype in_type, int32_t vi) {
  if (!p) return fail(DEDISP_E_INVALID, "plan is NULL");
  if (in_type != DEDISP_F32 && in_type != DEDISP_U8) return fail(DEDISP_E_DTYPE, "dtype must be F32 or U8");
  const bool u8 = in_type == DEDISP_U8;
  const int n = (int)(u8 ? variants_u8() : variants_f32()).size();
  if (vi < -2 || vi >= n) return fail(DEDISP_E_INVALID, "variant index out of range");
  if (vi >= 0 && !det_fits(p, u8, vi)) return fail(DEDISP_E_UNTUNED, "variant has no search epilogue or does not fit");
  (u8 ? p->var_det_u8 : p->var_det_f32) = vi;
  return DEDISP_OK;
}

dedisp_status dedisp_detect_autotune(dedisp_plan p, int32_t nbeam, int32_t nsamp, dedisp_dtype in_type, int32_t nwidth,
                                     float* ms, int32_t n) {
  if (!p) return fail(DEDISP_E_INVALID, "plan is NULL");
  if (nbeam < 1 || nsamp < 1) return fail(DEDISP_E_INVALID, "nbeam and nsamp must be >= 1");
  if (in_type != DEDISP_F32 && in_type != DEDISP_U8) return fail(DEDISP_E_DTYPE, "dtype must be F32 or U8");
  if (nwidth < 1 || nwidth > kDetNW) return fail(DEDISP_E_INVALID, "nwidth must be in [1, 6]");
  const bool u8 = in_type == DEDISP_U8;
  const int nv = (int)(u8 ? variants_u8() : variants_f32()).size();
  const int esz = u8 ? 1 : 4;
  const int64_t q = 16 / esz;
  const int64_t in_stride = ((int64_t)nsamp + p->max_delay + q - 1) / q * q;
  const int64_t nseries = (int64_t)nbeam * p->ndm;
  // the unfused path needs the most workspace
  const size_t ws_bytes = fallback_ws(p, nbeam, nsamp);
  void *d_in = nullptr, *d_ws = nullptr, *d_res = nullptr;
  hipError_t e = hipMalloc(&d_in, (size_t)nbeam * p->nchan * in_stride * esz);
  if (e == hipSuccess) e = hipMalloc(&d_ws, ws_bytes);
  if (e == hipSuccess) e = hipMalloc(&d_res, (size_t)nseries * 16);
  if (e == hipSuccess) e = launch_fill_random(d_in, (size_t)nbeam * p->nchan * in_stride * esz, !u8, 1601u, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    if (d_in) (void)hipFree(d_in);
    if (d_ws) (void)hipFree(d_ws);
    if (d_res) (void)hipFree(d_res);
    return e == hipErrorOutOfMemory ? fail(DEDISP_E_NOMEM, "autotune scratch allocation failed")
                                    : hip_fail(e, "autotune scratch");
  }
  double* snr = (double*)d_res;
  int32_t* wid = (int32_t*)(snr + nseries);
  int32_t* start = wid + nseries;
  hipStream_t s;
  hipEvent_t e0, e1;
  (void)hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  int& var = u8 ? p->var_det_u8 : p->var_det_f32;
  const int saved = var;
  std::vector<float> times(nv + 1, -1.f);
  int best = -2;
  float best_ms = 1e30f;
  for (int vi = -1; vi < nv; ++vi) {
    if (vi >= 0 && !det_fits(p, u8, vi)) continue;
    var = vi;
    const float t = median_ms(
        [&]() {
          return dedisp_detect(p, nbeam, nsamp, d_in, in_type, in_stride, nullptr, nwidth, snr, wid, start, nullptr,
                               nullptr, d_ws, ws_bytes, s) == DEDISP_OK
                     ? hipSuccess
                     : hipErrorUnknown;
        },
        s, 3, e0, e1);
    times[vi < 0 ? nv : vi] = t;
    if (t > 0 && t < best_ms) {
      best_ms = t;
      best = vi;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(s);
  (void)hipFree(d_in);
  (void)hipFree(d_ws);
  (void)hipFree(d_res);
  if (ms)
    for (int i = 0; i < n && i <= nv; ++i) ms[i] = times[i];
  if (best == -2) {
    var = saved;
    return fail(DEDISP_E_UNTUNED, "no search path ran");
  }
  var = best;
  return DEDISP_OK;
}

size_t dedisp_detect_rows_workspace_bytes(int32_t nrows, int32_t nsamp) {
  if (nrows < 1 || nsamp < 1) return 0;
  return rows_ws(nrows, nsamp);
}

dedisp_status dedisp_detect_rows(int32_t nrows, int32_t nsamp, const void* d_rows, dedisp_dtype type, int64_t stride,
                                 int32_t nwidth, double* d_snr, int32_t* d_width, int32_t* d_start, double* d_mean,
                                 double* d_std, void* d_ws, size_t ws_bytes, void* stream) {
  if (nrows < 1 || nsamp < 1) return fail(DEDISP_E_INVALID, "nrows and nsamp must be >= 1");
  if (!d_rows) return fail(DEDISP_E_INVALID, "rows pointer is NULL");
  dedisp_status st = check_outputs(nwidth, d_snr, d_width, d_start);
  if (st != DEDISP_OK) return st;
  if (type != DEDISP_F32 && type != DEDISP_I32) return fail(DEDISP_E_DTYPE, "rows must be F32 or I32");
  if (stride < nsamp) return fail(DEDISP_E_SHAPE, "stride < nsamp");
  if (stride > kMaxRow) return fail(DEDISP_E_SHAPE, "rows longer than 2^29 samples are not supported");
  if (((uintptr_t)d_rows & 15u) || (stride * 4) % 16)
    return fail(DEDISP_E_ALIGN, "pointers and row byte sizes must be multiples of 16 bytes");
  if (!d_ws) return fail(DEDISP_E_WORKSPACE, "workspace is NULL");
  if ((uintptr_t)d_ws & 15u) return fail(DEDISP_E_ALIGN, "workspace must be 16-byte aligned");
  if (ws_bytes < rows_ws(nrows, nsamp)) return fail(DEDISP_E_WORKSPACE, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  const int ntiles = (int)rows_tiles(nsamp);
  DetRec* recs = (DetRec*)d_ws;
  hipError_t e = launch_detect_rows(d_rows, type == DEDISP_I32, stride, nrows, nsamp, ntiles, recs, s);
  if (e != hipSuccess) return hip_fail(e, "launching the row search");
  e = launch_det_finish(recs, false, nrows, ntiles, nsamp, nwidth, d_snr, d_width, d_start, d_mean, d_std, s);
  return e == hipSuccess ? DEDISP_OK : hip_fail(e, "launching the record merge");
}

}  // extern "C"

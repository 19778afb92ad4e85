// Batched execution of many independent beams (the multi-beam use of
// Section 5.1): one persistent launch walks a device work table of every
// tile of every beam, largest tiles first, and is captured once into a HIP
// graph that later calls replay.
#include <algorithm>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "internal.h"

namespace dd {
dedisp_status ensure_tables(dedisp_plan p, int dir, int vi, Tables** out);
int autotune_batch_variant(const std::vector<dedisp_plan>& plans, const std::vector<int32_t>& nsamp,
                           const std::vector<const float*>& d_in, const std::vector<int64_t>& in_stride,
                           const std::vector<const float*>& d_w, const std::vector<float*>& d_out,
                           const std::vector<int64_t>& out_stride);
}  // namespace dd

using namespace dd;

struct dedisp_batch_s {
  int nbeam = 0;
  int variant = -1;
  std::vector<dedisp_plan> plans;
  std::vector<int32_t> nsamp;
  std::vector<const float*> d_in;
  std::vector<int64_t> in_stride;
  std::vector<const float*> d_w;
  std::vector<float*> d_out;
  std::vector<int64_t> out_stride;
  BeamDesc* d_beams = nullptr;
  int32_t* d_order = nullptr;
  int* d_counter = nullptr;
  int64_t ntiles = 0;
  int grid = 0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

static void batch_free(dedisp_batch b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->d_beams) (void)hipFree(b->d_beams);
  if (b->d_order) (void)hipFree(b->d_order);
  if (b->d_counter) (void)hipFree(b->d_counter);
  delete b;
}

// Validate one beam the way dedisp_execute does.
static dedisp_status check_beam(int i, dedisp_plan p, int32_t ns, const float* in, int64_t is, const float* w,
                                const float* out, int64_t os) {
  const std::string at = "beam " + std::to_string(i) + ": ";
  if (!p) return fail(DEDISP_E_INVALID, at + "plan is NULL");
  if (ns < 1) return fail(DEDISP_E_INVALID, at + "nsamp must be >= 1");
  if (!in || !out) return fail(DEDISP_E_INVALID, at + "input or output pointer is NULL");
  if (is < (int64_t)ns + p->max_delay) return fail(DEDISP_E_SHAPE, at + "in_stride < nsamp + max_delay");
  if (os < ns) return fail(DEDISP_E_SHAPE, at + "out_stride < nsamp");
  if (is > kMaxRow || (int64_t)ns + p->max_delay > kMaxRow)
    return fail(DEDISP_E_SHAPE, at + "rows longer than 2^29 samples are not supported");
  if (((uintptr_t)in & 15) || ((uintptr_t)out & 15) || (is * 4) % 16 || (os * 4) % 16 || ((uintptr_t)w & 3))
    return fail(DEDISP_E_ALIGN, at + "pointers and row byte sizes must be multiples of 16 bytes");
  return DEDISP_OK;
}

// Build the beam descriptors and the work table for variant vi.
static dedisp_status build_work(dedisp_batch b, int vi) {
  const Variant& v = variants_f32()[vi];
  std::vector<BeamDesc> beams(b->nbeam);
  std::vector<int64_t> cost(b->nbeam);
  int64_t total = 0;
  for (int i = 0; i < b->nbeam; ++i) {
    dedisp_plan p = b->plans[i];
    Tables* t = nullptr;
    dedisp_status st = ensure_tables(p, 0, vi, &t);
    if (st != DEDISP_OK) return st;
    TileArgs& a = beams[i].a;
    a = TileArgs{};
    a.in = b->d_in[i];
    a.in_stride = b->in_stride[i];
    a.in_beam_stride = 0;
    a.in_shift = 0;
    a.in_lo = 0;
    a.in_hi = (int)b->in_stride[i];
    a.rows_in = p->nchan;
    a.rows_out = p->ndm;
    a.nout = b->nsamp[i];
    a.n_time_tiles = (b->nsamp[i] + v.st() - 1) / v.st();
    a.n_row_tiles = t->n_row_tiles;
    a.blk = t->d_blk;
    a.wav = t->d_wav;
    a.w_in = b->d_w[i];
    a.out = b->d_out[i];
    a.out_stride = b->out_stride[i];
    a.out_beam_stride = 0;
    beams[i].tile_begin = total;
    total += (int64_t)a.n_time_tiles * a.n_row_tiles;
    cost[i] = p->nchan;  // a tile costs ~ rows_in * tile area
  }
  if (total > 0x7fffffff) return fail(DEDISP_E_SHAPE, "too many tiles in one batch");
  for (int i = 0; i < b->nbeam; ++i)
    if ((b->d_w[i] != nullptr) != (b->d_w[0] != nullptr))
      return fail(DEDISP_E_INVALID, "weights must be given for all beams or none");
  // Work table: (beam, local tile) pairs, beams with the costliest tiles first;
  // within a beam, time-major with output-row tiles fastest.
  std::vector<int> ord(b->nbeam);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return cost[x] > cost[y]; });
  std::vector<int32_t> order;
  order.reserve((size_t)total * 2);
  for (int i : ord) {
    const int64_t n = (int64_t)beams[i].a.n_time_tiles * beams[i].a.n_row_tiles;
    for (int64_t k = 0; k < n; ++k) {
      order.push_back(i);
      order.push_back((int32_t)k);
    }
  }
  b->ntiles = total;
  hipError_t e = hipMalloc(&b->d_beams, sizeof(BeamDesc) * b->nbeam);
  if (e == hipSuccess) e = hipMalloc(&b->d_order, sizeof(int32_t) * order.size());
  if (e == hipSuccess) e = hipMalloc(&b->d_counter, sizeof(int) * 64);
  if (e == hipSuccess) e = hipMemcpy(b->d_beams, beams.data(), sizeof(BeamDesc) * b->nbeam, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->d_order, order.data(), sizeof(int32_t) * order.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(b->d_counter, 0, sizeof(int) * 64);
  if (e != hipSuccess) return hip_fail(e, "uploading the batch work table");
  int dev = 0, ncu = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_fail(e, "querying the device");
  b->grid = ncu * batched_blocks_per_cu(v);
  b->variant = vi;
  return DEDISP_OK;
}

extern "C" {

dedisp_status dedisp_batch_create(dedisp_batch* out, int32_t nbeam, const dedisp_plan* plans, const int32_t* nsamp,
                                  const float* const* d_in, const int64_t* in_stride, const float* const* d_w,
                                  float* const* d_out, const int64_t* out_stride, int32_t tune) {
  if (!out) return fail(DEDISP_E_INVALID, "batch pointer is NULL");
  *out = nullptr;
  if (nbeam < 1) return fail(DEDISP_E_INVALID, "nbeam must be >= 1");
  if (!plans || !nsamp || !d_in || !in_stride || !d_out || !out_stride)
    return fail(DEDISP_E_INVALID, "a per-beam array is NULL");
  dedisp_batch b = new (std::nothrow) dedisp_batch_s();
  if (!b) return fail(DEDISP_E_NOMEM, "host allocation failed");
  b->nbeam = nbeam;
  for (int i = 0; i < nbeam; ++i) {
    const float* w = d_w ? d_w[i] : nullptr;
    dedisp_status st = check_beam(i, plans[i], nsamp[i], d_in[i], in_stride[i], w, d_out[i], out_stride[i]);
    if (st != DEDISP_OK) {
      batch_free(b);
      return st;
    }
    b->plans.push_back(plans[i]);
    b->nsamp.push_back(nsamp[i]);
    b->d_in.push_back(d_in[i]);
    b->in_stride.push_back(in_stride[i]);
    b->d_w.push_back(w);
    b->d_out.push_back(d_out[i]);
    b->out_stride.push_back(out_stride[i]);
  }
  // Variant: the tuned choice, or the first default that fits every beam.
  int vi = -1;
  if (tune) vi = autotune_batch_variant(b->plans, b->nsamp, b->d_in, b->in_stride, b->d_w, b->d_out, b->out_stride);
  if (vi < 0) {
    static const int pref[] = {0, 1, 2, 4, 3, 5};
    for (int k : pref) {
      bool ok = true;
      for (int i = 0; i < nbeam && ok; ++i) ok = ensure_tables(b->plans[i], 0, k, nullptr) == DEDISP_OK;
      if (ok) {
        vi = k;
        break;
      }
    }
  }
  if (vi < 0) {
    batch_free(b);
    return fail(DEDISP_E_UNTUNED, "no tiled variant fits every beam of the batch");
  }
  dedisp_status st = build_work(b, vi);
  if (st != DEDISP_OK) {
    batch_free(b);
    return st;
  }
  hipError_t e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    batch_free(b);
    return hip_fail(e, "creating the capture stream");
  }
  *out = b;
  return DEDISP_OK;
}

dedisp_status dedisp_execute_batched(dedisp_batch b, void* stream) {
  if (!b) return fail(DEDISP_E_INVALID, "batch is NULL");
  const Variant& v = variants_f32()[b->variant];
  hipError_t e;
  if (!b->exec) {
    // Capture [clear counter, persistent kernel] once on a private stream.
    e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "beginning graph capture");
    hipError_t e1 = launch_zero_counter(b->d_counter, b->cap_stream);
    hipError_t e2 = launch_batched(v, b->d_beams, b->d_w[0] != nullptr, b->d_order, b->ntiles, b->d_counter,
                                   b->grid, b->cap_stream);
    e = hipStreamEndCapture(b->cap_stream, &b->graph);
    if (e1 != hipSuccess) return hip_fail(e1, "capturing the counter reset");
    if (e2 != hipSuccess) return hip_fail(e2, "capturing the persistent kernel");
    if (e != hipSuccess) return hip_fail(e, "ending graph capture");
    e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      b->exec = nullptr;
      return hip_fail(e, "instantiating the graph");
    }
  }
  e = hipGraphLaunch(b->exec, (hipStream_t)stream);
  return e == hipSuccess ? DEDISP_OK : hip_fail(e, "launching the graph");
}

dedisp_status dedisp_execute_per_beam(dedisp_batch b, void* stream) {
  if (!b) return fail(DEDISP_E_INVALID, "batch is NULL");
  for (int i = 0; i < b->nbeam; ++i) {
    dedisp_status st = dedisp_execute(b->plans[i], 1, b->nsamp[i], b->d_in[i], DEDISP_F32, b->in_stride[i], b->d_w[i],
                                      b->d_out[i], DEDISP_F32, b->out_stride[i], stream);
    if (st != DEDISP_OK) return st;
  }
  return DEDISP_OK;
}

dedisp_status dedisp_batch_destroy(dedisp_batch b) {
  batch_free(b);
  return DEDISP_OK;
}

}  // extern "C"

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
  int32_t* d_qoff = nullptr;  // kNumXcd + 1 queue offsets into d_order (in pairs)
  int nqueue = 1;             // queues in use: 1 (one global order) or kNumXcd (one per XCD)
  int* d_counter = nullptr;
  int64_t ntiles = 0;
  int grid = 0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

static void drop_work(dedisp_batch b);

static void batch_free(dedisp_batch b) {
  if (!b) return;
  drop_work(b);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
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

// Free the work table, descriptors and captured graph of the current variant.
static void drop_work(dedisp_batch b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->d_beams) (void)hipFree(b->d_beams);
  if (b->d_order) (void)hipFree(b->d_order);
  if (b->d_qoff) (void)hipFree(b->d_qoff);
  if (b->d_counter) (void)hipFree(b->d_counter);
  b->exec = nullptr;
  b->graph = nullptr;
  b->d_beams = nullptr;
  b->d_order = nullptr;
  b->d_qoff = nullptr;
  b->d_counter = nullptr;
  b->variant = -1;
}

// Build the beam descriptors and the work table for variant vi, dealt over
// b->nqueue queues.
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
  // Work table: (beam, local tile) pairs, beams with the costliest tiles first.
  // Each (beam, time tile) group, with its row tiles in order, goes to one
  // queue; groups are dealt round-robin over the nqueue queues in use (the
  // others stay empty).
  std::vector<int> ord(b->nbeam);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return cost[x] > cost[y]; });
  std::vector<std::vector<int32_t>> qs(kNumXcd);
  int64_t g = 0;
  for (int i : ord) {
    const TileArgs& a = beams[i].a;
    for (int tt = 0; tt < a.n_time_tiles; ++tt, ++g) {
      std::vector<int32_t>& q = qs[g % b->nqueue];
      for (int rt = 0; rt < a.n_row_tiles; ++rt) {
        q.push_back(i);
        q.push_back(tt * a.n_row_tiles + rt);
      }
    }
  }
  std::vector<int32_t> order, qoff(kNumXcd + 1, 0);
  order.reserve((size_t)total * 2);
  for (int q = 0; q < kNumXcd; ++q) {
    order.insert(order.end(), qs[q].begin(), qs[q].end());
    qoff[q + 1] = (int32_t)(order.size() / 2);
  }
  b->ntiles = total;
  hipError_t e = hipMalloc(&b->d_beams, sizeof(BeamDesc) * b->nbeam);
  if (e == hipSuccess) e = hipMalloc(&b->d_order, sizeof(int32_t) * order.size());
  if (e == hipSuccess) e = hipMalloc(&b->d_qoff, sizeof(int32_t) * qoff.size());
  if (e == hipSuccess) e = hipMalloc(&b->d_counter, sizeof(int) * kNumXcd * kCounterStride);
  if (e == hipSuccess) e = hipMemcpy(b->d_beams, beams.data(), sizeof(BeamDesc) * b->nbeam, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->d_order, order.data(), sizeof(int32_t) * order.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->d_qoff, qoff.data(), sizeof(int32_t) * qoff.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(b->d_counter, 0, sizeof(int) * kNumXcd * kCounterStride);
  if (e != hipSuccess) return hip_fail(e, "uploading the batch work table");
  int dev = 0, ncu = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_fail(e, "querying the device");
  b->grid = ncu * batched_blocks_per_cu(v);
  b->variant = vi;
  return DEDISP_OK;
}

// The batch's auto-tuning (Sections 2.2 and 4.1, applied to the whole
// batch): time the persistent launch of every variant that fits every beam
// on the batch's own buffers (their outputs are overwritten by the real run)
// and return the fastest, or -1; then time the winner with one queue per XCD
// and keep that split if it is faster.  Leaves the batch without a work
// table.
static int tune_batch(dedisp_batch b) {
  const std::vector<Variant>& vs = variants_f32();
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return -1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    (void)hipStreamDestroy(s);
    return -1;
  }
  int best = -1;
  float best_ms = 1e30f;
  for (int vi = 0; vi < (int)vs.size(); ++vi) {
    bool ok = true;
    for (int i = 0; i < b->nbeam && ok; ++i) ok = ensure_tables(b->plans[i], 0, vi, nullptr) == DEDISP_OK;
    if (!ok) continue;
    drop_work(b);
    b->nqueue = 1;
    if (build_work(b, vi) != DEDISP_OK) continue;
    const bool weighted = b->d_w[0] != nullptr;
    const float ms = median_ms(
        [&]() {
          const hipError_t r = launch_zero_counter(b->d_counter, s);
          return r == hipSuccess
                     ? launch_batched(vs[vi], b->d_beams, weighted, b->d_order, b->d_qoff, b->d_counter, b->grid, s)
                     : r;
        },
        s, 2, e0, e1);
    if (ms > 0 && ms < best_ms) {
      best_ms = ms;
      best = vi;
    }
  }
  // the best variant with one queue per XCD as well
  if (best >= 0) {
    drop_work(b);
    b->nqueue = kNumXcd;
    float ms = -1.f;
    if (build_work(b, best) == DEDISP_OK) {
      const bool weighted = b->d_w[0] != nullptr;
      ms = median_ms(
          [&]() {
            const hipError_t r = launch_zero_counter(b->d_counter, s);
            return r == hipSuccess ? launch_batched(vs[best], b->d_beams, weighted, b->d_order, b->d_qoff,
                                                    b->d_counter, b->grid, s)
                                   : r;
          },
          s, 2, e0, e1);
    }
    if (!(ms > 0 && ms < best_ms)) b->nqueue = 1;
  }
  drop_work(b);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(s);
  return best;
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
  if (tune) vi = tune_batch(b);
  if (vi < 0) {
    for (int k : default_order(0)) {
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
  if (b->variant < 0) return fail(DEDISP_E_INVALID, "batch has no work table (a variant change failed)");
  const Variant& v = variants_f32()[b->variant];
  hipError_t e;
  if (!b->exec) {
    // Capture [clear counter, persistent kernel] once on a private stream.
    e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "beginning graph capture");
    hipError_t e1 = launch_zero_counter(b->d_counter, b->cap_stream);
    hipError_t e2 = launch_batched(v, b->d_beams, b->d_w[0] != nullptr, b->d_order, b->d_qoff, b->d_counter,
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

dedisp_status dedisp_batch_set_variant(dedisp_batch b, int32_t variant) {
  if (!b) return fail(DEDISP_E_INVALID, "batch is NULL");
  if (variant < 0 || variant >= (int32_t)variants_f32().size())
    return fail(DEDISP_E_INVALID, "variant index out of range");
  for (int i = 0; i < b->nbeam; ++i) {
    dedisp_status st = ensure_tables(b->plans[i], 0, variant, nullptr);
    if (st != DEDISP_OK) return st;
  }
  const hipError_t e = hipDeviceSynchronize();  // no replay of the old graph is in flight
  if (e != hipSuccess) return hip_fail(e, "synchronizing before a variant change");
  drop_work(b);
  return build_work(b, variant);
}

int32_t dedisp_batch_variant(dedisp_batch b) { return b ? b->variant : -1; }

dedisp_status dedisp_batch_destroy(dedisp_batch b) {
  batch_free(b);
  return DEDISP_OK;
}

}  // extern "C"

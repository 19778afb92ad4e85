// Batched execution of many independent beams (the multi-beam use of
// Section 5.1): one persistent launch walks a device work table of every
// tile of every beam, largest tiles first, and is captured once into a HIP
// graph that later calls replay.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "internal.h"

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
  hipEvent_t done = nullptr;  // recorded after every replay
  bool launched = false;
  int cache_hit = 0;
};

static void drop_work(dedisp_batch b);

// Wait until no replay of the batch's graph is in flight.
static hipError_t wait_idle(dedisp_batch b) {
  if (!b->launched || !b->done) return hipSuccess;
  const hipError_t e = hipEventSynchronize(b->done);
  if (e == hipSuccess) b->launched = false;
  return e;
}

static void batch_free(dedisp_batch b) {
  if (!b) return;
  (void)wait_idle(b);
  drop_work(b);
  if (b->done) (void)hipEventDestroy(b->done);
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

// Pin (+1) or unpin (-1) the tile tables of variant vi in every beam's plan.
static void pin_tables(dedisp_batch b, int vi, int by) {
  for (int i = 0; i < b->nbeam; ++i) {
    auto it = b->plans[i]->fwd_f32.find(vi);
    if (it != b->plans[i]->fwd_f32.end()) it->second.pins += by;
  }
}

// Free the work table, descriptors and captured graph of the current variant.
static void drop_work(dedisp_batch b) {
  if (b->variant >= 0) pin_tables(b, b->variant, -1);
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
  pin_tables(b, vi, +1);  // the descriptors point at these tables
  return DEDISP_OK;
}

// The batch's auto-tuning (Sections 2.2 and 4.1, applied to the whole
// batch): time the persistent launch of every variant that fits every beam
// on the batch's own buffers (their outputs are overwritten by the real run)
// and return the fastest, or -1; then time the winner with one queue per XCD
// and keep that split if it is faster.  Leaves the batch without a work
// table.
static int tune_batch(dedisp_batch b, float* best_out) {
  const std::vector<Variant>& vs = variants_f32();
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return -1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    (void)hipStreamDestroy(s);
    return -1;
  }
  const bool weighted = b->d_w[0] != nullptr;
  // one variant (with nq queues) timed on the batch's buffers, its tables
  // freed afterwards unless something else holds them; -1 if it does not fit
  auto time_variant = [&](int vi, int nq, int reps) {
    float ms = -1.f;
    bool ok = true;
    for (int i = 0; i < b->nbeam && ok; ++i) ok = ensure_tables(b->plans[i], 0, vi, nullptr) == DEDISP_OK;
    drop_work(b);
    b->nqueue = nq;
    if (ok && build_work(b, vi) == DEDISP_OK)
      ms = median_ms(
          [&]() {
            const hipError_t r = launch_zero_counter(b->d_counter, s);
            return r == hipSuccess
                       ? launch_batched(vs[vi], b->d_beams, weighted, b->d_order, b->d_qoff, b->d_counter, b->grid, s)
                       : r;
          },
          s, reps, e0, e1);
    drop_work(b);
    for (int i = 0; i < b->nbeam; ++i) drop_spare_tables(b->plans[i], 0, -3);
    return ms;
  };
  // every variant once, then the three fastest again, more carefully
  std::vector<std::pair<float, int>> first;
  for (int vi = 0; vi < (int)vs.size(); ++vi) {
    const float ms = time_variant(vi, 1, 1);
    if (ms > 0) first.push_back({ms, vi});
  }
  std::sort(first.begin(), first.end());
  int best = -1;
  float best_ms = 1e30f;
  for (size_t k = 0; k < first.size() && k < 3; ++k) {
    const float ms = time_variant(first[k].second, 1, 3);
    if (ms > 0 && ms < best_ms) {
      best_ms = ms;
      best = first[k].second;
    }
  }
  // the best variant with one queue per XCD as well
  int nq = 1;
  if (best >= 0) {
    const float ms = time_variant(best, kNumXcd, 3);
    if (ms > 0 && ms < best_ms) {
      best_ms = ms;
      nq = kNumXcd;
    }
  }
  b->nqueue = nq;
  if (best_out) *best_out = best_ms;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(s);
  return best;
}

// Tune-cache key of a batch: the device, the weights flag and the multiset of
// beam set-ups (channels, DM trials, output length rounded up to a power of
// two, delay-table hash), hashed in sorted order.
static std::string batch_cache_key(dedisp_batch b) {
  std::vector<std::string> items;
  for (int i = 0; i < b->nbeam; ++i) {
    int bucket = 1;
    while (bucket < b->nsamp[i]) bucket <<= 1;
    char buf[96];
    snprintf(buf, sizeof(buf), "%d/%d/%d/%016llx", b->plans[i]->nchan, b->plans[i]->ndm, bucket,
             (unsigned long long)delay_table_hash(b->plans[i]));
    items.push_back(buf);
  }
  std::sort(items.begin(), items.end());
  uint64_t h = 1469598103934665603ull;
  for (const std::string& it : items)
    for (char c : it + ";") {
      h ^= (unsigned char)c;
      h *= 1099511628211ull;
    }
  char key[192];
  snprintf(key, sizeof(key), "%s|batch|f32|w%d|n%d|h%016llx", tune_device_name().c_str(), b->d_w[0] != nullptr,
           b->nbeam, (unsigned long long)h);
  return key;
}

// Cached choice "variant name" or "variant name|q8" (one queue per XCD).
static int parse_cached(const std::string& v, int& nqueue) {
  std::string name = v;
  nqueue = 1;
  const size_t bar = v.find('|');
  if (bar != std::string::npos) {
    name = v.substr(0, bar);
    if (v.substr(bar + 1) == "q8") nqueue = kNumXcd;
  }
  const std::vector<Variant>& vs = variants_f32();
  for (int i = 0; i < (int)vs.size(); ++i)
    if (name == vs[i].name) return i;
  return -1;
}

extern "C" {

dedisp_status dedisp_batch_create(dedisp_batch* out, int32_t nbeam, const dedisp_plan* plans, const int32_t* nsamp,
                                  const void* const* d_in, dedisp_dtype in_t, const int64_t* in_stride,
                                  const float* const* d_w, void* const* d_out, const int64_t* out_stride, int32_t tune,
                                  const char* tune_cache) {
  if (!out) return fail(DEDISP_E_INVALID, "batch pointer is NULL");
  *out = nullptr;
  if (nbeam < 1) return fail(DEDISP_E_INVALID, "nbeam must be >= 1");
  if (!plans || !nsamp || !d_in || !in_stride || !d_out || !out_stride)
    return fail(DEDISP_E_INVALID, "a per-beam array is NULL");
  if (in_t != DEDISP_F32) return fail(DEDISP_E_DTYPE, "batches take float32 input only");
  dedisp_batch b = new (std::nothrow) dedisp_batch_s();
  if (!b) return fail(DEDISP_E_NOMEM, "host allocation failed");
  b->nbeam = nbeam;
  for (int i = 0; i < nbeam; ++i) {
    const float* w = d_w ? d_w[i] : nullptr;
    const float* xin = static_cast<const float*>(d_in[i]);
    float* xout = static_cast<float*>(d_out[i]);
    dedisp_status st = check_beam(i, plans[i], nsamp[i], xin, in_stride[i], w, xout, out_stride[i]);
    if (st != DEDISP_OK) {
      batch_free(b);
      return st;
    }
    b->plans.push_back(plans[i]);
    b->nsamp.push_back(nsamp[i]);
    b->d_in.push_back(xin);
    b->in_stride.push_back(in_stride[i]);
    b->d_w.push_back(w);
    b->d_out.push_back(xout);
    b->out_stride.push_back(out_stride[i]);
  }
  for (int i = 1; i < nbeam; ++i)
    if ((b->d_w[i] != nullptr) != (b->d_w[0] != nullptr)) {
      batch_free(b);
      return fail(DEDISP_E_INVALID, "weights must be given for all beams or none");
    }
  // Variant: the cached or tuned choice, or the first default that fits every beam.
  int vi = -1;
  if (tune) {
    const std::string key = batch_cache_key(b);
    std::string hit;
    if (tune_cache_lookup(tune_cache, key, hit)) {
      int nq = 1;
      const int ci = parse_cached(hit, nq);
      bool ok = ci >= 0;
      for (int i = 0; i < nbeam && ok; ++i) ok = ensure_tables(b->plans[i], 0, ci, nullptr) == DEDISP_OK;
      if (ok) {
        vi = ci;
        b->nqueue = nq;
        b->cache_hit = 1;
      }
    }
    if (vi < 0) {
      float ms = -1.f;
      vi = tune_batch(b, &ms);
      if (vi >= 0)
        tune_cache_store(tune_cache, key,
                         std::string(variants_f32()[vi].name) + (b->nqueue == kNumXcd ? "|q8" : ""), ms);
    }
  }
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
  // tables the search built for other variants
  for (int i = 0; i < nbeam; ++i) drop_spare_tables(b->plans[i], 0, vi);
  dedisp_status st = build_work(b, vi);
  if (st != DEDISP_OK) {
    batch_free(b);
    return st;
  }
  hipError_t e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
  if (e != hipSuccess) {
    batch_free(b);
    return hip_fail(e, "creating the capture stream");
  }
  *out = b;
  return DEDISP_OK;
}

int32_t dedisp_batch_queues(dedisp_batch b) { return b ? b->nqueue : 0; }

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
  if (e != hipSuccess) return hip_fail(e, "launching the graph");
  e = hipEventRecord(b->done, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "recording the replay's completion event");
  b->launched = true;
  return DEDISP_OK;
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
  const hipError_t e = wait_idle(b);  // no replay of the old graph is in flight
  if (e != hipSuccess) return hip_fail(e, "waiting for the batch before a variant change");
  drop_work(b);
  return build_work(b, variant);
}

dedisp_status dedisp_batch_set_queues(dedisp_batch b, int32_t nqueue) {
  if (!b) return fail(DEDISP_E_INVALID, "batch is NULL");
  if (nqueue != 1 && nqueue != kNumXcd) return fail(DEDISP_E_INVALID, "nqueue must be 1 or 8");
  const int vi = b->variant;
  if (vi < 0) return fail(DEDISP_E_INVALID, "batch has no work table");
  const hipError_t e = wait_idle(b);
  if (e != hipSuccess) return hip_fail(e, "waiting for the batch before a queue change");
  drop_work(b);
  b->nqueue = nqueue;
  return build_work(b, vi);
}

int32_t dedisp_batch_variant(dedisp_batch b) { return b ? b->variant : -1; }

int32_t dedisp_batch_cache_hit(dedisp_batch b) { return b ? b->cache_hit : -1; }

dedisp_status dedisp_batch_destroy(dedisp_batch b) {
  batch_free(b);
  return DEDISP_OK;
}

}  // extern "C"

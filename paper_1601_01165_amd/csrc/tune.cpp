// Auto-tuning.  The paper tries every meaningful combination of its tuning
// parameters and keeps the fastest, per platform, set-up and DM count
// (Section 2.2, Section 3, Section 4.1).  Here the search runs over the
// kernel variants compiled into the library (plus the direct kernel), timed
// with HIP events on the plan's real delay tables, and the winner is kept in
// the plan and in an optional JSON cache file.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "internal.h"

namespace dd {

// FNV-1a over the delay table: two plans with equal tables share tuning.
uint64_t delay_table_hash(dedisp_plan p) {
  uint64_t h = 1469598103934665603ull;
  const unsigned char* b = reinterpret_cast<const unsigned char*>(p->delay.data());
  const size_t n = p->delay.size() * sizeof(int32_t);
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

std::string tune_device_name() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string s = prop.gcnArchName;
  return s.substr(0, s.find(':'));
}

static std::string cache_key(dedisp_plan p, dedisp_dtype t, int nbeam, int nsamp) {
  // Samples are bucketed by powers of two: tuning depends on the tile count,
  // not on the exact length.
  int bucket = 1;
  while (bucket < nsamp) bucket <<= 1;
  char buf[256];
  snprintf(buf, sizeof(buf), "%s|%s|c%d|d%d|s%d|b%d|h%016llx", tune_device_name().c_str(), t == DEDISP_U8 ? "u8" : "f32",
           p->nchan, p->ndm, bucket, nbeam, (unsigned long long)delay_table_hash(p));
  return buf;
}

// Cache file: a JSON object, one entry per line:
//   "key": {"variant": "name", "ms": 1.234},
bool tune_cache_lookup(const char* path, const std::string& key, std::string& variant) {
  if (!path) return false;
  std::ifstream f(path);
  if (!f) return false;
  std::string line;
  const std::string pat = "\"" + key + "\": {\"variant\": \"";
  while (std::getline(f, line)) {
    size_t k = line.find(pat);
    if (k == std::string::npos) continue;
    size_t s = k + pat.size();
    size_t e = line.find('"', s);
    if (e == std::string::npos) return false;
    variant = line.substr(s, e - s);
    return true;
  }
  return false;
}

void tune_cache_store(const char* path, const std::string& key, const std::string& variant, float ms) {
  if (!path) return;
  std::vector<std::string> entries;
  {
    std::ifstream f(path);
    std::string line;
    const std::string pat = "\"" + key + "\":";
    while (f && std::getline(f, line)) {
      if (line.find("\": {\"variant\"") == std::string::npos) continue;
      if (line.find(pat) != std::string::npos) continue;
      while (!line.empty() && (line.back() == ',' || line.back() == ' ')) line.pop_back();
      entries.push_back(line);
    }
  }
  char buf[512];
  snprintf(buf, sizeof(buf), "  \"%s\": {\"variant\": \"%s\", \"ms\": %.6f}", key.c_str(), variant.c_str(), ms);
  entries.push_back(buf);
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream f(tmp);
    f << "{\n";
    for (size_t i = 0; i < entries.size(); ++i) f << entries[i] << (i + 1 < entries.size() ? ",\n" : "\n");
    f << "}\n";
  }
  (void)rename(tmp.c_str(), path);
}

// Time in ms per launch of fn.  A first timed launch warms up and sizes the
// groups: launches shorter than kGroupMs run back to back in groups of about
// kGroupMs (after one such group as a further warm-up), so that the GPU is
// timed busy, as in a pipeline, and not recovering from the idle gap of a
// per-launch wait.  Returns the median over `reps` groups of the group mean.
static constexpr float kGroupMs = 2.0f;

float median_ms(const std::function<hipError_t()>& fn, hipStream_t s, int reps, hipEvent_t e0, hipEvent_t e1) {
  auto timed = [&](int n, float& ms) {
    if (hipEventRecord(e0, s) != hipSuccess) return false;
    for (int i = 0; i < n; ++i)
      if (fn() != hipSuccess) return false;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return false;
    return hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
  };
  float t1 = 0.f;
  if (!timed(1, t1)) return -1.f;
  const int n = t1 >= kGroupMs ? 1 : std::min(64, (int)std::ceil(kGroupMs / std::max(t1, 1e-3f)));
  float ms = 0.f;
  if (n > 1 && !timed(n, ms)) return -1.f;
  std::vector<float> t;
  for (int r = 0; r < reps; ++r) {
    if (!timed(n, ms)) return -1.f;
    t.push_back(ms / n);
  }
  std::sort(t.begin(), t.end());
  return t[t.size() / 2];
}

// Last search of each plan and dtype: times per variant (-1 = does not fit),
// the last entry being the direct kernel.
static std::vector<float>& last_times(dedisp_plan p, dedisp_dtype t) {
  static thread_local std::vector<std::pair<std::pair<dedisp_plan, int>, std::vector<float>>> store;
  for (auto& kv : store)
    if (kv.first.first == p && kv.first.second == (int)t) return kv.second;
  store.push_back({{p, (int)t}, {}});
  return store.back().second;
}

}  // namespace dd

using namespace dd;

extern "C" {

dedisp_status dedisp_autotune(dedisp_plan p, int32_t nbeam, int32_t nsamp, dedisp_dtype t, const char* cache_path) {
  if (!p) return fail(DEDISP_E_INVALID, "plan is NULL");
  if (nbeam < 1 || nsamp < 1) return fail(DEDISP_E_INVALID, "nbeam and nsamp must be >= 1");
  if (t != DEDISP_F32 && t != DEDISP_U8) return fail(DEDISP_E_DTYPE, "dtype must be F32 or U8");
  const bool u8 = t == DEDISP_U8;
  const std::vector<Variant>& vs = u8 ? variants_u8() : variants_f32();
  const std::string key = cache_key(p, t, nbeam, nsamp);
  std::string hit;
  if (tune_cache_lookup(cache_path, key, hit)) {
    if (hit == "direct") return dedisp_plan_set_variant(p, t, -1);
    for (int i = 0; i < (int)vs.size(); ++i)
      if (hit == vs[i].name && dedisp_plan_set_variant(p, t, i) == DEDISP_OK) return DEDISP_OK;
  }
  const int esz = u8 ? 1 : 4;
  const int64_t q = 16 / esz;
  const int64_t in_stride = ((int64_t)nsamp + p->max_delay + q - 1) / q * q;
  const int64_t out_stride = ((int64_t)nsamp + 3) / 4 * 4;
  void* d_in = nullptr;
  void* d_out = nullptr;
  hipError_t e = hipMalloc(&d_in, (size_t)nbeam * p->nchan * in_stride * esz);
  if (e == hipSuccess) e = hipMalloc(&d_out, (size_t)nbeam * p->ndm * out_stride * 4);
  // noise-like input: the clock under load, and so the timings, depend on the data
  if (e == hipSuccess) e = launch_fill_random(d_in, (size_t)nbeam * p->nchan * in_stride * esz, !u8, 1601u, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    if (d_in) (void)hipFree(d_in);
    if (d_out) (void)hipFree(d_out);
    return e == hipErrorOutOfMemory ? fail(DEDISP_E_NOMEM, "autotune scratch allocation failed")
                                    : hip_fail(e, "autotune scratch");
  }
  hipStream_t s;
  hipEvent_t e0, e1;
  (void)hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const dedisp_dtype out_t = u8 ? DEDISP_I32 : DEDISP_F32;
  std::vector<float>& times = last_times(p, t);
  times.assign(vs.size() + 1, -1.f);
  const int saved = u8 ? p->var_u8 : p->var_f32;
  const int dir = u8 ? 1 : 0;
  auto time_variant = [&](int vi, int reps) {
    if (dedisp_plan_set_variant(p, t, vi) != DEDISP_OK) return -1.f;
    return median_ms(
        [&]() {
          return dedisp_execute(p, nbeam, nsamp, d_in, t, in_stride, nullptr, d_out, out_t, out_stride, s) == DEDISP_OK
                     ? hipSuccess
                     : hipErrorUnknown;
        },
        s, reps, e0, e1);
  };
  // every variant once (its tables freed again), then the three fastest
  // more carefully
  std::vector<std::pair<float, int>> first;
  for (int vi = -1; vi < (int)vs.size(); ++vi) {
    const float ms = time_variant(vi, 1);
    times[vi < 0 ? vs.size() : (size_t)vi] = ms;
    if (ms > 0) first.push_back({ms, vi});
    (u8 ? p->var_u8 : p->var_f32) = saved;
    drop_spare_tables(p, dir, -3);
  }
  std::sort(first.begin(), first.end());
  int best = -2;
  float best_ms = 1e30f;
  for (size_t k = 0; k < first.size() && k < 3; ++k) {
    const int vi = first[k].second;
    const float ms = time_variant(vi, 3);
    times[vi < 0 ? vs.size() : (size_t)vi] = ms;
    if (ms > 0 && ms < best_ms) {
      best_ms = ms;
      best = vi;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(s);
  (void)hipFree(d_in);
  (void)hipFree(d_out);
  if (best == -2) {
    (void)dedisp_plan_set_variant(p, t, saved);
    return fail(DEDISP_E_UNTUNED, "no variant ran");
  }
  dedisp_status st = dedisp_plan_set_variant(p, t, best);
  if (st != DEDISP_OK) return st;
  drop_spare_tables(p, dir, best);
  tune_cache_store(cache_path, key, best < 0 ? "direct" : vs[best].name, best_ms);
  return DEDISP_OK;
}

dedisp_status dedisp_autotune_adjoint(dedisp_plan p, int32_t nbeam, int32_t nsamp, float* ms, int32_t n) {
  if (!p) return fail(DEDISP_E_INVALID, "plan is NULL");
  if (nbeam < 1 || nsamp < 1) return fail(DEDISP_E_INVALID, "nbeam and nsamp must be >= 1");
  const std::vector<Variant>& vs = variants_f32();
  const int64_t nin = ((int64_t)nsamp + p->max_delay + 3) / 4 * 4;
  const int64_t gs = ((int64_t)nsamp + 3) / 4 * 4;
  const size_t ws_bytes = dedisp_adjoint_workspace_bytes(p, nbeam, (int32_t)nin);
  float *d_g = nullptr, *d_x = nullptr, *d_gi = nullptr, *d_gw = nullptr;
  void* d_ws = nullptr;
  hipError_t e = hipMalloc(&d_g, (size_t)nbeam * p->ndm * gs * 4);
  if (e == hipSuccess) e = hipMalloc(&d_x, (size_t)nbeam * p->nchan * nin * 4);
  if (e == hipSuccess) e = hipMalloc(&d_gi, (size_t)nbeam * p->nchan * nin * 4);
  if (e == hipSuccess) e = hipMalloc(&d_gw, (size_t)p->nchan * 4);
  if (e == hipSuccess) e = hipMalloc(&d_ws, std::max<size_t>(ws_bytes, 16));
  if (e == hipSuccess) e = launch_fill_random(d_g, (size_t)nbeam * p->ndm * gs * 4, true, 1602u, nullptr);
  if (e == hipSuccess) e = launch_fill_random(d_x, (size_t)nbeam * p->nchan * nin * 4, true, 1603u, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  auto release = [&]() {
    for (void* q : {(void*)d_g, (void*)d_x, (void*)d_gi, (void*)d_gw, d_ws})
      if (q) (void)hipFree(q);
  };
  if (e != hipSuccess) {
    release();
    return e == hipErrorOutOfMemory ? fail(DEDISP_E_NOMEM, "autotune scratch allocation failed")
                                    : hip_fail(e, "autotune scratch");
  }
  hipStream_t s;
  hipEvent_t e0, e1;
  (void)hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const int saved = p->var_adj;
  std::vector<float> times(vs.size() + 1, -1.f);
  auto time_variant = [&](int vi, int reps) {
    if (dedisp_plan_set_adjoint_variant(p, vi) != DEDISP_OK) return -1.f;
    return median_ms(
        [&]() {
          return dedisp_adjoint(p, nbeam, nsamp, (int32_t)nin, d_g, gs, nullptr, d_x, nin, d_gi, nin, d_gw, d_ws,
                                ws_bytes, s) == DEDISP_OK
                     ? hipSuccess
                     : hipErrorUnknown;
        },
        s, reps, e0, e1);
  };
  std::vector<std::pair<float, int>> first;
  for (int vi = -1; vi < (int)vs.size(); ++vi) {
    const float t = time_variant(vi, 1);
    times[vi < 0 ? vs.size() : (size_t)vi] = t;
    if (t > 0) first.push_back({t, vi});
    p->var_adj = saved;
    drop_spare_tables(p, 2, -3);
  }
  std::sort(first.begin(), first.end());
  int best = -2;
  float best_ms = 1e30f;
  for (size_t k = 0; k < first.size() && k < 3; ++k) {
    const int vi = first[k].second;
    const float t = time_variant(vi, 3);
    times[vi < 0 ? vs.size() : (size_t)vi] = t;
    if (t > 0 && t < best_ms) {
      best_ms = t;
      best = vi;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(s);
  release();
  if (ms)
    for (int32_t i = 0; i < n && i <= (int32_t)vs.size(); ++i) ms[i] = times[i];
  if (best == -2) {
    (void)dedisp_plan_set_adjoint_variant(p, saved);
    return fail(DEDISP_E_UNTUNED, "no adjoint variant ran");
  }
  const dedisp_status st = dedisp_plan_set_adjoint_variant(p, best);
  if (st == DEDISP_OK) drop_spare_tables(p, 2, best);
  return st;
}

int32_t dedisp_autotune_times(dedisp_plan p, dedisp_dtype t, float* ms, int32_t n) {
  if (!p || !ms) return 0;
  std::vector<float>& times = last_times(p, t);
  const int32_t k = std::min<int32_t>(n, (int32_t)times.size());
  for (int32_t i = 0; i < k; ++i) ms[i] = times[i];
  return k;
}

}  // extern "C"

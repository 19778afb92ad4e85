// Internal declarations shared by the host code and the kernels of the
// dedispersion library.  Not part of the C-ABI (include/dedisp.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <map>
#include <string>
#include <vector>

#include "../../include/dedisp.h"

namespace dd {

// ---------------------------------------------------------------------------
// Kernel variants.  The paper tunes five parameters per platform and set-up
// (Section 2.2): work-items per work-group in time and in DM, elements per
// work-item in time and in DM, and local memory versus cache.  On gfx950 the
// corresponding knobs are: samples per lane (tp), output rows per wave (dpw),
// waves per block (nwave), the register window length (nwin), input rows
// staged in LDS per pass (cc) and the LDS row capacity (rowcap); the direct
// kernel is the "no local memory, no reuse" end of the space.
// ---------------------------------------------------------------------------
enum Kind { KIND_WIN_F32 = 0, KIND_TILE_U8 = 1 };

// Longest row (samples) accepted: row byte sizes must fit a 32-bit buffer
// range, and sample indices an int, with room for tile overhang.
constexpr int64_t kMaxRow = (int64_t)1 << 29;
// Most beams one call takes: beams are the y dimension of the launch grid.
constexpr int kMaxBeams = 65535;

struct Variant {
  const char* name;
  int kind;
  int tp;      // f32: samples per lane; u8: dwords (4 samples each) per lane
  int dpw;     // output rows per wave
  int nwave;   // waves per block
  int nwin;    // f32: window registers (0 for u8)
  int cc;      // input rows per LDS pass
  int rowcap;  // LDS row capacity (f32: elements, u8: bytes)
  int nbuf;    // LDS buffers: 1 = synchronous staging, 2 = asynchronous double buffering
  int id;      // index in the variant list
  // u8 only: 0 = one LDS copy per row, int32 sums; 1 = four byte-shifted copies, packed sums (at most
  // 256 input rows); 2 = as 1, flushed to int32 sums every 256 rows
  int mode = 0;
  // f32 only: 1 = each row's DM slots branch into static blocks of adds; the table then holds block byte
  // offsets o * (4 * tp + 4) in place of the window offsets o
  int jmp = 0;
  int st() const { return kind == KIND_WIN_F32 ? 64 * tp : 256 * tp; }
  int dt() const { return nwave * dpw; }
  // ints per wave-table entry: f32 {win_start, nl, one offset per row} padded to 4/8/16; u8 packed u16
  // offsets (mode 0) or one LDS byte offset per row (byte-shifted modes)
  int wav_ints() const {
    if (kind == KIND_WIN_F32) return dpw + 2 <= 4 ? 4 : dpw + 2 <= 8 ? 8 : 16;
    return mode == 0 ? 4 : (dpw <= 4 ? 4 : 8);
  }
};

const std::vector<Variant>& variants_f32();
const std::vector<Variant>& variants_u8();
// Variant indices in order of preference when nothing was tuned (dir: 0 forward
// FP32, 1 forward uint8, 2 adjoint); every index of the direction's list appears.
const std::vector<int>& default_order(int dir);

// Host-built tile tables for one variant on one delay matrix.
//   blk[row_tile][rows_in]            {stage_base, stage_len}
//   wav[wave_tile][rows_in][wav_ints] f32: {win_start, nl, offset of each row...} (jump form: offset times
//                                      the block size)
//                                      u8:  {packed u16 offsets...} or {LDS byte offset of each row...}
struct Tables {
  int variant = -1;
  int n_row_tiles = 0;
  int n_wave_tiles = 0;
  int max_stage = 0;
  int32_t* d_blk = nullptr;
  int32_t* d_wav = nullptr;
  int32_t* d_span = nullptr;  // adjoint: per (row tile, pass) {least stage base, greatest stage end}
  size_t bytes = 0;
  int pins = 0;  // batches whose work table points at these tables (never freed while pinned)
};

// Single-pulse search (detect_dev.h): boxcar widths 1, 2, ..., 2^(kDetNW - 1);
// each lane reads kDetLook samples past its run of window starts.
constexpr int kDetNW = 6;
constexpr int kDetLook = 32;

// One record per (series, time tile): per width the largest window sum
// (int32 for uint8 input, float bits otherwise) and its first start (-1: no
// window), and the FP64 sum and sum of squares of the tile's owned samples.
struct DetRec {
  int32_t val[kDetNW];
  int32_t pos[kDetNW];
  double s1, s2;
};
static_assert(sizeof(DetRec) == 64, "records are 64 bytes");

// Arguments of the tiled kernels (passed by value).
struct TileArgs {
  const void* in;            // input rows of beam 0
  int64_t in_stride;         // elements per input row
  int64_t in_beam_stride;    // elements per beam
  int in_shift;              // global index = virtual position + in_shift
  int in_lo, in_hi;          // valid virtual positions [lo, hi); others read as 0
  int rows_in;
  int rows_out;
  int nout;                  // output samples per row
  int n_time_tiles;
  int n_row_tiles;
  int tiles_per_block;       // time tiles walked by one block (uint8 double-buffered kernels)
  const int32_t* blk;
  const int32_t* wav;
  const int32_t* span;       // adjoint: per (row tile, pass) {least stage base, greatest stage end}, or null
  const float* w_in;         // per input-row weight or null
  void* out;
  int64_t out_stride;
  int64_t out_beam_stride;
  const float* w_out;        // per output-row scale or null (adjoint: w[c])
  // weight-gradient partials (adjoint only)
  const float* x;            // forward input rows [beam][rows_out][x_stride] or null
  int64_t x_stride;
  int64_t x_beam_stride;
  double* partial;           // [beam][n_time_tiles][rows_out]
  // single-pulse search launches only
  int tile_step;             // samples between time tiles = window starts owned by a tile
  int det_nsamp;             // samples of each dedispersed series
  int det_s2_u32;            // uint8: a lane's sum of squares fits 32 bits
  DetRec* det;               // [beam][rows_out][n_time_tiles]
};

// One beam of a batched launch.
struct BeamDesc {
  TileArgs a;                // in/out pointers already offset for the beam
  int64_t tile_begin;        // first global tile index of this beam
};

// Launchers (engine.hip).  Each returns hipSuccess or the launch error.
hipError_t launch_tiled(const Variant& v, const TileArgs& a, int nbeam, bool adjoint, hipStream_t s);
hipError_t launch_direct_f32(const float* in, int64_t in_stride, int64_t in_beam_stride, const int32_t* delta,
                             int nchan, int ndm, const float* w, float* out, int64_t out_stride,
                             int64_t out_beam_stride, int nsamp, int nbeam, hipStream_t s);
hipError_t launch_direct_u8(const uint8_t* in, int64_t in_stride, int64_t in_beam_stride, const int32_t* delta,
                            int nchan, int ndm, int32_t* out, int64_t out_stride, int64_t out_beam_stride,
                            int nsamp, int nbeam, hipStream_t s);
hipError_t launch_direct_adjoint(const float* g, int64_t g_stride, int64_t g_beam_stride, const int32_t* delta,
                                 int nchan, int ndm, int nsamp, int nin, const float* w, float* grad_in,
                                 int64_t gi_stride, int64_t gi_beam_stride, const float* x, int64_t x_stride,
                                 int64_t x_beam_stride, double* partial, int nbeam, hipStream_t s);
hipError_t launch_reduce_gradw(const double* partial, int nparts, int nchan, float* grad_w, hipStream_t s);
// Persistent launch over a work table of (beam, local tile) pairs split into
// kNumXcd queues: queue q is order[2*qoff[q] .. 2*qoff[q+1]); d_counter holds
// kNumXcd counters kCounterStride ints apart.
constexpr int kNumXcd = 8;
constexpr int kCounterStride = 32;
hipError_t launch_batched(const Variant& v, const BeamDesc* d_beams, bool weighted, const int32_t* d_order,
                          const int32_t* d_qoff, int* d_counter, int grid, hipStream_t s);
hipError_t launch_zero_counter(int* d_counter, hipStream_t s);

// Single-pulse search.  detect_fusable: the variant has a kernel with the
// search in its epilogue; det_step: window starts owned by one of its time
// tiles (its tile length minus the lane runs that cover kDetLook - 1 samples).
bool detect_fusable(const Variant& v);
int det_step(const Variant& v);
hipError_t launch_detect(const Variant& v, const TileArgs& a, int nbeam, hipStream_t s);
// Unfused search over stored rows (float32, or int32 searched in float32).
constexpr int kDetRowsRun = 16;                              // starts per lane
constexpr int kDetRowsTile = 64 * kDetRowsRun;               // samples per tile
constexpr int kDetRowsStep = kDetRowsTile - 2 * kDetRowsRun;  // owned starts per tile
hipError_t launch_detect_rows(const void* rows, bool i32, int64_t stride, int nrows, int nsamp, int ntiles,
                              DetRec* recs, hipStream_t s);
// Merge the records of each series (tile order) into its result.
hipError_t launch_det_finish(const DetRec* recs, bool int_vals, int nseries, int ntiles, int nsamp, int nwidth,
                             double* snr, int32_t* width, int32_t* start, double* mean, double* stdv, hipStream_t s);
int batched_blocks_per_cu(const Variant& v);

// Tile tables of a plan (plan.cpp): build or find (dir 0 forward FP32, 1
// forward uint8, 2 adjoint); free those of direction dir other than `keep`,
// the plan's chosen variants and pinned ones.
dedisp_status ensure_tables(dedisp_plan p, int dir, int vi, Tables** out);
void drop_spare_tables(dedisp_plan p, int dir, int keep);

// Timing (tune.cpp): ms per launch of fn, the median over `reps` groups of
// back-to-back launches (about 2 ms per group, one launch for longer ones)
// after a warm-up; -1 if a launch fails.
float median_ms(const std::function<hipError_t()>& fn, hipStream_t s, int reps, hipEvent_t e0, hipEvent_t e1);

// Tuning cache (tune.cpp): a JSON file of {"key": {"variant": "...", "ms": t}}
// lines.  The device's architecture name, a hash of a plan's delay table.
std::string tune_device_name();
uint64_t delay_table_hash(dedisp_plan p);
bool tune_cache_lookup(const char* path, const std::string& key, std::string& value);
void tune_cache_store(const char* path, const std::string& key, const std::string& value, float ms);

// Fill nbytes of device memory with seeded pseudo-random data (f32: values in
// [-1, 1); otherwise bytes), for timing on realistic inputs.
hipError_t launch_fill_random(void* p, size_t nbytes, bool f32, uint32_t seed, hipStream_t s);

// Errors (plan.cpp).
dedisp_status fail(dedisp_status st, const std::string& msg);
dedisp_status hip_fail(hipError_t e, const char* what);

}  // namespace dd

// The plan object.
struct dedisp_plan_s {
  int device = 0;
  int ncu = 256;                    // compute units of the device
  int nchan = 0, ndm = 0, max_delay = 0;
  double tsamp = 0;
  std::vector<double> freq, dm;
  std::vector<int32_t> delay;       // [ndm][nchan]
  int32_t* d_delay = nullptr;       // device copy [ndm][nchan]
  // adjoint view: out rows = channels, in rows = DMs, delay' = pad - delay
  int adj_pad = 0;                  // max_delay rounded up to a multiple of 4
  std::map<int, dd::Tables> fwd_f32, fwd_u8, adj_f32;
  int var_f32 = -2, var_u8 = -2, var_adj = -2;  // -1 = direct kernel, -2 = not chosen yet
  int var_det_f32 = -2, var_det_u8 = -2;         // single-pulse search: -1 = unfused, -2 = automatic
};

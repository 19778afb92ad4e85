/* Tuned multi-core CPU dedispersion: the comparison baseline the paper runs
 * beside its GPU kernels (Sclocco et al., arXiv 1601.01165, Section 5, the
 * OpenMP implementation on CPUs and Xeon Phi), built with OpenMP and SIMD
 * across output samples, its tile shape chosen by timing.  Separate library
 * (libdedisp_cpu.so), host memory only, no GPU.
 *
 * The sum is the one of Algorithm 1 (Section 2.1): for every beam b, DM
 * trial j and output sample t,
 *     out[b][j][t] = sum over channels c, ascending, of w[c] * in[b][c][t + delta[j][c]]
 * with the weighted sample w[c] * x rounded, then added with one rounding (a plain add when w is NULL),
 * so FP32 results equal a sequential loop bit for bit; uint8 input sums into
 * int32 exactly.
 *
 * Layouts (all host pointers, owned by the caller):
 *   in    [nbeam][nchan][in_stride], in_stride >= nsamp + max(delta)
 *   delta [ndm][nchan] int32 sample delays (Section 2, Equation 1)
 *   w     [nchan] or NULL
 *   out   [nbeam][ndm][out_stride], out_stride >= nsamp
 * The tile shape is configuration `cfg` (0 <= cfg < ddcpu_num_configs()):
 * dt DM trials x tt samples per register tile.
 * Return: 0 on success, 1 for invalid arguments (NULL pointer, sizes < 1,
 * strides too small, cfg out of range, a negative delay). */
#ifndef DEDISP_CPU_H
#define DEDISP_CPU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

int ddcpu_forward_f32(int32_t nbeam, int32_t nchan, int32_t ndm, int32_t nsamp, const float* in, int64_t in_stride,
                      const int32_t* delta, const float* w, float* out, int64_t out_stride, int32_t cfg);

int ddcpu_forward_u8(int32_t nbeam, int32_t nchan, int32_t ndm, int32_t nsamp, const uint8_t* in, int64_t in_stride,
                     const int32_t* delta, int32_t* out, int64_t out_stride, int32_t cfg);

/* Number of tile configurations, and the shape of configuration i (0 on success). */
int32_t ddcpu_num_configs(void);
int ddcpu_config(int32_t i, int32_t* dt, int32_t* tt);

/* OpenMP threads the forward calls use. */
int32_t ddcpu_num_threads(void);

/* Instruction set the forward calls run with ("avx512f", "avx2" or "generic"). */
const char* ddcpu_isa(void);

#ifdef __cplusplus
}
#endif

#endif

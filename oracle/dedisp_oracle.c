/*
 * Plain CPU oracle for brute-force incoherent dedispersion.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It shares
 * no source, header, table or helper with the GPU library.
 *
 * Source: Sclocco, van Leeuwen, Bal, van Nieuwpoort, "Real-Time Dedispersion
 * for Fast Radio Transient Surveys, using Auto Tuning on Many-Core
 * Accelerators" (arXiv 1601.01165).
 *
 *   - Delay law: Section 2, Equation 1.  Delays are computed ahead of time
 *     (Section 2.1).
 *   - Forward dedispersion: the sum that Section 2.1 (Algorithm 1) defines,
 *     out[dm][t] = sum over channels of in[chan][t + delta[dm][chan]], with
 *     every output receiving its terms in ascending channel order.  Data are
 *     single precision (Section 2.1), so each output is an FP32 sum with one
 *     rounding per term; an FP64 twin gives the exact value and the error
 *     scale.  The loops run per output row: the row is cleared, then each
 *     channel's shifted input row is added into it.
 *   - Adjoint: the transpose of Algorithm 1's linear map (not in the paper;
 *     derived from it), in gather form and in scatter form.
 *
 * Parity pins (all in the CPU test suite): Equation 1 checked against
 * hand-derived delays and its invariants; forward against a dense-matrix brute
 * force, channel-sum, constant, ramp, one-hot and copy special cases,
 * linearity, and pulse recovery; adjoint against the dot-product identity and
 * a dense transpose; grad_w against finite differences of the linear map.
 *
 * Build: plain C99 with OpenMP over independent output rows only (each output
 * keeps the sequential channel order), -O2 -fno-fast-math -ffp-contract=off.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <omp.h>

/* ------------------------------------------------------------------------ */
/* Delay table, Section 2 Equation 1.                                        */
/*   k = 4150 * DM * (1/f_i^2 - 1/f_h^2)  seconds, f in MHz, f_h the highest */
/*   frequency of the band.  The paper indexes input[chan][sample + delta]  */
/*   with an integer delta and does not say how k/t_samp becomes an integer; */
/*   this oracle rounds to nearest with halves going up: floor(x + 0.5).     */
/* ------------------------------------------------------------------------ */

/* Unrounded delay in samples, x = k / tsamp.  Returns 0 on success, -1 on an
 * invalid argument. */
int oracle_delay_samples(int nchan, const double* freq_mhz, double tsamp_s, int ndm, const double* dm,
                         double* x_out /* [ndm][nchan] */) {
  if (nchan < 1 || ndm < 1 || !(tsamp_s > 0.0) || !freq_mhz || !dm || !x_out) return -1;
  double fh = freq_mhz[0];
  for (int c = 0; c < nchan; ++c) {
    if (!(freq_mhz[c] > 0.0) || !isfinite(freq_mhz[c])) return -1;
    if (freq_mhz[c] > fh) fh = freq_mhz[c];
  }
  for (int j = 0; j < ndm; ++j) {
    if (!(dm[j] >= 0.0) || !isfinite(dm[j])) return -1;
    for (int c = 0; c < nchan; ++c) {
      double f = freq_mhz[c];
      double k = 4150.0 * dm[j] * (1.0 / (f * f) - 1.0 / (fh * fh));
      x_out[(size_t)j * nchan + c] = k / tsamp_s;
    }
  }
  return 0;
}

/* Integer delay table delta[dm][chan].  Returns 0, or -1 on an invalid
 * argument or a delay that does not fit in int32. */
int oracle_delay_table(int nchan, const double* freq_mhz, double tsamp_s, int ndm, const double* dm,
                       int32_t* delta /* [ndm][nchan] */) {
  if (nchan < 1 || ndm < 1 || !(tsamp_s > 0.0) || !freq_mhz || !dm || !delta) return -1;
  double fh = freq_mhz[0];
  for (int c = 0; c < nchan; ++c) {
    if (!(freq_mhz[c] > 0.0) || !isfinite(freq_mhz[c])) return -1;
    if (freq_mhz[c] > fh) fh = freq_mhz[c];
  }
  for (int j = 0; j < ndm; ++j) {
    if (!(dm[j] >= 0.0) || !isfinite(dm[j])) return -1;
    for (int c = 0; c < nchan; ++c) {
      double f = freq_mhz[c];
      double k = 4150.0 * dm[j] * (1.0 / (f * f) - 1.0 / (fh * fh));
      double x = floor(k / tsamp_s + 0.5);
      if (!(x >= 0.0) || x > 2147483647.0) return -1;
      delta[(size_t)j * nchan + c] = (int32_t)x;
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Forward dedispersion, Section 2.1 Algorithm 1.                            */
/*   out[b][dm][sample] = sum over chan ascending of                         */
/*                        w[chan] * in[b][chan][sample + delta[dm][chan]]    */
/* The weight w is an extension (absent from Algorithm 1): a per-channel    */
/* gain applied to the data before dedispersion, so each term is the FP32    */
/* product w * x (rounded), then added to the FP32 sum (rounded); w == NULL  */
/* means every weight is 1, i.e. the plain FP32 adds of Algorithm 1.         */
/* Layouts: in [nbeam][nchan][in_stride], out [nbeam][ndm][out_stride].      */
/* The caller guarantees in_stride >= nsamp + max delta.                     */
/* ------------------------------------------------------------------------ */

void oracle_forward_f32(int nbeam, int nchan, int ndm, int nsamp, const float* in, int64_t in_stride,
                        const int32_t* delta, const float* w, float* out, int64_t out_stride) {
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
  for (int b = 0; b < nbeam; ++b) {
    for (int j = 0; j < ndm; ++j) {
      float* row = out + ((size_t)b * ndm + j) * out_stride;
      for (int t = 0; t < nsamp; ++t) row[t] = 0.0f;
      for (int c = 0; c < nchan; ++c) {
        /* channel c's input row, shifted by its delay at DM trial j */
        const float* src = in + ((size_t)b * nchan + c) * in_stride + delta[(size_t)j * nchan + c];
        if (w) {
          const float wc = w[c];
          for (int t = 0; t < nsamp; ++t) {
            const float term = wc * src[t]; /* the weighted sample, rounded */
            row[t] = row[t] + term;
          }
        } else {
          for (int t = 0; t < nsamp; ++t) row[t] = row[t] + src[t];
        }
      }
    }
  }
}

/* Same sum in FP64 (exact for the test data sizes used), plus the error
 * scale sum |w * x| that bounds the FP32 summation error. */
void oracle_forward_f64(int nbeam, int nchan, int ndm, int nsamp, const double* in, int64_t in_stride,
                        const int32_t* delta, const double* w, double* out, double* absout, int64_t out_stride) {
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
  for (int b = 0; b < nbeam; ++b) {
    for (int j = 0; j < ndm; ++j) {
      double* row = out + ((size_t)b * ndm + j) * out_stride;
      double* arow = absout ? absout + ((size_t)b * ndm + j) * out_stride : NULL;
      for (int t = 0; t < nsamp; ++t) {
        row[t] = 0.0;
        if (arow) arow[t] = 0.0;
      }
      for (int c = 0; c < nchan; ++c) {
        const double* src = in + ((size_t)b * nchan + c) * in_stride + delta[(size_t)j * nchan + c];
        const double wc = w ? w[c] : 1.0;
        for (int t = 0; t < nsamp; ++t) {
          row[t] += wc * src[t];
          if (arow) arow[t] += fabs(wc * src[t]);
        }
      }
    }
  }
}

/* The same sum on 8-bit unsigned input with a 32-bit integer accumulator
 * (unit weights; exact). */
void oracle_forward_u8(int nbeam, int nchan, int ndm, int nsamp, const uint8_t* in, int64_t in_stride,
                       const int32_t* delta, int32_t* out, int64_t out_stride) {
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
  for (int b = 0; b < nbeam; ++b) {
    for (int j = 0; j < ndm; ++j) {
      int32_t* row = out + ((size_t)b * ndm + j) * out_stride;
      for (int t = 0; t < nsamp; ++t) row[t] = 0;
      for (int c = 0; c < nchan; ++c) {
        const uint8_t* src = in + ((size_t)b * nchan + c) * in_stride + delta[(size_t)j * nchan + c];
        for (int t = 0; t < nsamp; ++t) row[t] += (int32_t)src[t];
      }
    }
  }
}

/* Selected outputs, one by one, for checks at sizes where the full output is
 * too costly on the CPU.  Point p is (beam[p], dm[p], sample[p]).  Writes the
 * FP32 sum (channels ascending, each weighted sample rounded, then each add
 * rounded) and the FP64 error scale sum |w * x|. */
void oracle_forward_points_f32(int nchan, const float* in, int64_t in_stride, int64_t beam_stride,
                               const int32_t* delta, const float* w, int64_t npts, const int32_t* pb,
                               const int32_t* pdm, const int32_t* ps, float* out, double* absout) {
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < npts; ++p) {
    const float* inb = in + (size_t)pb[p] * beam_stride;
    const int32_t* drow = delta + (size_t)pdm[p] * nchan;
    float acc = 0.0f;
    double a = 0.0;
    for (int chan = 0; chan < nchan; ++chan) {
      float x = inb[(size_t)chan * in_stride + ps[p] + drow[chan]];
      if (w) {
        const float term = w[chan] * x;
        acc = acc + term;
        a += fabs((double)w[chan] * (double)x);
      } else {
        acc = acc + x;
        a += fabs((double)x);
      }
    }
    out[p] = acc;
    if (absout) absout[p] = a;
  }
}

void oracle_forward_points_u8(int nchan, const uint8_t* in, int64_t in_stride, int64_t beam_stride,
                              const int32_t* delta, int64_t npts, const int32_t* pb, const int32_t* pdm,
                              const int32_t* ps, int32_t* out) {
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < npts; ++p) {
    const uint8_t* inb = in + (size_t)pb[p] * beam_stride;
    const int32_t* drow = delta + (size_t)pdm[p] * nchan;
    int32_t acc = 0;
    for (int chan = 0; chan < nchan; ++chan) acc += (int32_t)inb[(size_t)chan * in_stride + ps[p] + drow[chan]];
    out[p] = acc;
  }
}

/* ------------------------------------------------------------------------ */
/* Adjoint (transpose of the Algorithm 1 map, with weights).                 */
/* For output gradient g[b][dm][s] (s < nsamp), the input gradient is        */
/*   grad_in[b][chan][t] = w[chan] * G[b][chan][t],                          */
/*   G[b][chan][t] = sum over dm ascending with 0 <= t - delta[dm][chan]     */
/*                   < nsamp of g[b][dm][t - delta[dm][chan]],               */
/* for every t < nin (the input row length in use).  Terms whose output      */
/* sample falls outside [0, nsamp) contribute nothing.                       */
/* Gather form: one G element at a time.                                     */
/* ------------------------------------------------------------------------ */

void oracle_adjoint_gather_f32(int nbeam, int nchan, int ndm, int nsamp, int nin, const float* g, int64_t g_stride,
                               const int32_t* delta, const float* w, float* grad_in, int64_t gi_stride) {
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
  for (int b = 0; b < nbeam; ++b) {
    for (int chan = 0; chan < nchan; ++chan) {
      const float* gb = g + (size_t)b * ndm * g_stride;
      float* gi = grad_in + ((size_t)b * nchan + chan) * gi_stride;
      float wc = w ? w[chan] : 1.0f;
      for (int t = 0; t < nin; ++t) {
        float acc = 0.0f;
        for (int dmi = 0; dmi < ndm; ++dmi) {
          int s = t - delta[(size_t)dmi * nchan + chan];
          if (s >= 0 && s < nsamp) acc = acc + gb[(size_t)dmi * g_stride + s];
        }
        gi[t] = wc * acc;
      }
    }
  }
}

/* Scatter form: walk the forward loops (dm, sample, chan) and push each
 * output gradient to the input element it read.  For a fixed input element
 * the contributions arrive in ascending dm order, the same order as the
 * gather form.  G_tmp must hold nbeam*nchan*gi_stride floats. */
void oracle_adjoint_scatter_f32(int nbeam, int nchan, int ndm, int nsamp, int nin, const float* g, int64_t g_stride,
                                const int32_t* delta, const float* w, float* grad_in, int64_t gi_stride,
                                float* g_tmp) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int b = 0; b < nbeam; ++b) {
    float* gt = g_tmp + (size_t)b * nchan * gi_stride;
    for (size_t i = 0; i < (size_t)nchan * gi_stride; ++i) gt[i] = 0.0f;
    const float* gb = g + (size_t)b * ndm * g_stride;
    for (int dmi = 0; dmi < ndm; ++dmi)
      for (int sample = 0; sample < nsamp; ++sample)
        for (int chan = 0; chan < nchan; ++chan) {
          size_t idx = (size_t)chan * gi_stride + sample + delta[(size_t)dmi * nchan + chan];
          gt[idx] = gt[idx] + gb[(size_t)dmi * g_stride + sample];
        }
    for (int chan = 0; chan < nchan; ++chan) {
      float wc = w ? w[chan] : 1.0f;
      for (int t = 0; t < nin; ++t) grad_in[((size_t)b * nchan + chan) * gi_stride + t] = wc * gt[(size_t)chan * gi_stride + t];
    }
  }
}

/* FP64 adjoint twin: G64 = sum of g over the same index set, in FP64, and the
 * scale sum |g| over that set. */
void oracle_adjoint_gather_f64(int nbeam, int nchan, int ndm, int nsamp, int nin, const double* g, int64_t g_stride,
                               const int32_t* delta, double* G, double* absG, int64_t gi_stride) {
#pragma omp parallel for collapse(2) schedule(dynamic, 1)
  for (int b = 0; b < nbeam; ++b) {
    for (int chan = 0; chan < nchan; ++chan) {
      const double* gb = g + (size_t)b * ndm * g_stride;
      size_t o = ((size_t)b * nchan + chan) * gi_stride;
      for (int t = 0; t < nin; ++t) {
        double acc = 0.0, a = 0.0;
        for (int dmi = 0; dmi < ndm; ++dmi) {
          int s = t - delta[(size_t)dmi * nchan + chan];
          if (s >= 0 && s < nsamp) {
            acc += gb[(size_t)dmi * g_stride + s];
            a += fabs(gb[(size_t)dmi * g_stride + s]);
          }
        }
        G[o + t] = acc;
        if (absG) absG[o + t] = a;
      }
    }
  }
}

/* Gradient of sum_b,dm,s g[b][dm][s] * out[b][dm][s] with respect to the
 * channel weights, straight from the forward definition:
 *   grad_w[chan] = sum_b sum_dm sum_s g[b][dm][s] * in[b][chan][s + delta[dm][chan]]
 * accumulated in FP64, with the scale sum |g * in| alongside. */
void oracle_grad_w(int nbeam, int nchan, int ndm, int nsamp, const float* in, int64_t in_stride, const float* g,
                   int64_t g_stride, const int32_t* delta, double* grad_w, double* abs_grad_w) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int chan = 0; chan < nchan; ++chan) {
    double s = 0.0, a = 0.0;
    for (int b = 0; b < nbeam; ++b) {
      const float* inrow = in + ((size_t)b * nchan + chan) * in_stride;
      const float* gb = g + (size_t)b * ndm * g_stride;
      for (int dmi = 0; dmi < ndm; ++dmi) {
        int d = delta[(size_t)dmi * nchan + chan];
        for (int sample = 0; sample < nsamp; ++sample) {
          double p = (double)gb[(size_t)dmi * g_stride + sample] * (double)inrow[sample + d];
          s += p;
          a += fabs(p);
        }
      }
    }
    grad_w[chan] = s;
    if (abs_grad_w) abs_grad_w[chan] = a;
  }
}

int oracle_num_threads(void) { return omp_get_max_threads(); }

/*
 * FP64 CPU oracle for Pulscan's boxcar search (White et al. 2024,
 * "Pulscan: Binary pulsar detection using unmatched filters on NVIDIA GPUs").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with
 * the GPU library: it is a plain, slow, obviously correct restatement of what
 * the paper computes, in double precision, so the GPU path can be checked
 * against it.
 *
 * Steps, in the paper's order:
 *   1. per-block robust normalisation of the real and imaginary parts
 *      (section 2.2.3, the "Normalised Data" equation; the GPU median of
 *      medians of section 2.5 and the appendix algorithm "Median of Medians
 *      Normalisation"; the exact median of the CPU version, section 2.5);
 *   2. power = re^2 + im^2 (section 2.2.3);
 *   3. unit boxcars of every width 1..zmax (section 2.2.5);
 *   4. per-chunk maxima for every width (appendix algorithm "Boxcar Filtering
 *      Process");
 *   5. significance: chi-square survival with 2w degrees of freedom,
 *      Bonferroni correction, Gaussian-equivalent sigma (section 2.2.3);
 *   optionally, between steps 2 and 3, harmonic summing (section 2.3 and the
 *      appendix algorithm "Harmonic Sum Decimation"): stage H searches the
 *      sum of the power decimated by 1..H, with H(H+1) w degrees of freedom.
 *
 * Readings where the paper is silent or garbled (each is listed in the
 * design notes):
 *   - widths are 1..zmax; the paper's z is width - 1; dof = 2 * width;
 *   - the MAD is the median of |x - median| (the appendix writes
 *     "chunk - median"; section 2.2.3 defines the MAD);
 *   - the MAD scale is 1 / Phi^-1(3/4) = 1.482602218505602 (the appendix
 *     rounds it to 1.4826);
 *   - a block with MAD = 0 normalises to 0;
 *   - the last block, when nbins is not a multiple of the block, takes its
 *     statistics over the last `block` bins [n - block, n);
 *   - a window exists only when it fits: i + w <= n (output length n - k + 1
 *     in section 2.2.5);
 *   - argmax ties go to the smallest bin;
 *   - ntrials defaults to nbins * (number of searched widths); with harmonic
 *     summing, per stage, to the stage's length times the searched widths;
 *   - harmonic stage H has floor(n / H) bins (the bounds of the decimation
 *     algorithm), is chunked and searched like the power itself, and its
 *     candidates' bins are the stage's (the fundamental's) r-bins;
 *   - logarithms are natural.
 *
 * Parity of every function here is pinned by the CPU tests against
 * brute force, library routines (numpy, scipy) and the paper's worked
 * recursion example; none is "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* 1 / Phi^-1(3/4): makes the MAD a consistent estimator of a Gaussian's
 * standard deviation (section 2.2.3). */
#define ORACLE_MAD_SCALE 1.482602218505602

#define ORACLE_NORM_MOM 0
#define ORACLE_NORM_EXACT 1

/* ------------------------------------------------------------------------ */
/* Medians                                                                   */
/* ------------------------------------------------------------------------ */

static void sort_small(double *v, int n) {
  for (int i = 1; i < n; ++i) {
    double x = v[i];
    int j = i - 1;
    while (j >= 0 && v[j] > x) {
      v[j + 1] = v[j];
      --j;
    }
    v[j + 1] = x;
  }
}

/* Median of four values: the mean of the two middle order statistics.  The
 * appendix's local_median writes the same number as (a+b+c+d-min-max)/2. */
double oracle_med4(double a, double b, double c, double d) {
  double v[4] = {a, b, c, d};
  sort_small(v, 4);
  return 0.5 * (v[1] + v[2]);
}

/* Median of medians of n = 4^k values (section 2.5, appendix "Median of
 * Medians Normalisation"): at stride s = n/4, n/16, ..., 1 every position
 * t < s is replaced by the median of the four values at t, t+s, t+2s, t+3s;
 * the result is the value left at position 0.  `work` holds n doubles. */
double oracle_mom(const double *x, int64_t n, double *work) {
  memcpy(work, x, (size_t)n * sizeof(double));
  for (int64_t s = n / 4; s >= 1; s /= 4)
    for (int64_t t = 0; t < s; ++t)
      work[t] = oracle_med4(work[t], work[t + s], work[t + 2 * s], work[t + 3 * s]);
  return work[0];
}

static int cmp_double(const void *a, const void *b) {
  double x = *(const double *)a, y = *(const double *)b;
  return (x > y) - (x < y);
}

/* Textbook median (the CPU version's exact selection, section 2.5): the
 * middle order statistic, or the mean of the two middle ones for even n. */
double oracle_exact_median(const double *x, int64_t n, double *work) {
  memcpy(work, x, (size_t)n * sizeof(double));
  qsort(work, (size_t)n, sizeof(double), cmp_double);
  if (n & 1) return work[n / 2];
  return 0.5 * (work[n / 2 - 1] + work[n / 2]);
}

static int is_power_of_4(int64_t n) {
  if (n < 1) return 0;
  while (n % 4 == 0) n /= 4;
  return n == 1;
}

/* ------------------------------------------------------------------------ */
/* Step 1-2: normalisation and power                                         */
/* ------------------------------------------------------------------------ */

/* Statistics window of block k: [kB, kB + B), or [n - B, n) for a block that
 * runs past the end of the spectrum. */
static int64_t stats_start(int64_t k, int64_t block, int64_t n) {
  int64_t s = k * block;
  if (s + block > n) s = n - block;
  return s;
}

/* Normalise the real and imaginary parts of `spec` (interleaved float pairs,
 * n bins) block by block (section 2.2.3):
 *     v' = (v - median) / (MAD * 1.482602218505602),   MAD = median(|v - median|)
 * with the median of medians (mode 0) or the exact median (mode 1).
 * Outputs re_out, im_out (n doubles each) and, if non-null, stats with four
 * doubles per block: median_re, mad_re, median_im, mad_im.
 * Returns 0, or -1 on invalid arguments. */
int oracle_normalise(const float *spec, int64_t n, int64_t block, int mode, double *re_out,
                     double *im_out, double *stats) {
  if (!spec || !re_out || !im_out || n < 1 || block < 1 || block > n) return -1;
  if (mode == ORACLE_NORM_MOM && !is_power_of_4(block)) return -1;
  if (mode != ORACLE_NORM_MOM && mode != ORACLE_NORM_EXACT) return -1;
  int64_t nblocks = (n + block - 1) / block;
  int fail = 0;
#pragma omp parallel
  {
    double *v = (double *)malloc((size_t)block * sizeof(double));
    double *d = (double *)malloc((size_t)block * sizeof(double));
    double *work = (double *)malloc((size_t)block * sizeof(double));
    if (!v || !d || !work) {
#pragma omp atomic write
      fail = 1;
    } else {
#pragma omp for schedule(static)
      for (int64_t k = 0; k < nblocks; ++k) {
        int64_t s0 = stats_start(k, block, n);
        int64_t lo = k * block, hi = (k + 1) * block < n ? (k + 1) * block : n;
        for (int comp = 0; comp < 2; ++comp) {
          for (int64_t t = 0; t < block; ++t) v[t] = (double)spec[2 * (s0 + t) + comp];
          double med = mode == ORACLE_NORM_MOM ? oracle_mom(v, block, work)
                                               : oracle_exact_median(v, block, work);
          for (int64_t t = 0; t < block; ++t) d[t] = fabs(v[t] - med);
          double mad = mode == ORACLE_NORM_MOM ? oracle_mom(d, block, work)
                                               : oracle_exact_median(d, block, work);
          double *out = comp == 0 ? re_out : im_out;
          for (int64_t i = lo; i < hi; ++i) {
            double x = (double)spec[2 * i + comp];
            out[i] = mad > 0.0 ? (x - med) / (mad * ORACLE_MAD_SCALE) : 0.0;
          }
          if (stats) {
            stats[4 * k + 2 * comp] = med;
            stats[4 * k + 2 * comp + 1] = mad;
          }
        }
      }
    }
    free(v);
    free(d);
    free(work);
  }
  return fail ? -1 : 0;
}

/* Power of each bin, re^2 + im^2: chi-square with 2 dof under Gaussian
 * noise (section 2.2.3). */
void oracle_power(const double *re, const double *im, int64_t n, double *P) {
  for (int64_t i = 0; i < n; ++i) P[i] = re[i] * re[i] + im[i] * im[i];
}

/* ------------------------------------------------------------------------ */
/* Step 3-4: boxcars and per-chunk maxima                                    */
/* ------------------------------------------------------------------------ */

/* Unit boxcar of width w (section 2.2.5): Y_w[i] = P[i] + ... + P[i+w-1] for
 * i = 0 .. n-w (n - w + 1 outputs).  Summed left to right. */
void oracle_boxcar(const double *P, int64_t n, int w, double *Y) {
  for (int64_t i = 0; i + w <= n; ++i) {
    double s = 0.0;
    for (int j = 0; j < w; ++j) s += P[i + j];
    Y[i] = s;
  }
}

/* Per-chunk maxima of every boxcar (appendix "Boxcar Filtering Process"):
 * chunk c covers window starts i in [c*chunk, min((c+1)*chunk, n)); for each
 * width w = 1..zmax, M[c*zmax + w-1] is the largest Y_w[i] over the starts of
 * the chunk whose window fits (i + w <= n) and I[...] the smallest such i
 * attaining it.  A chunk with no fitting window of width w gets M = -inf and
 * I = -1.  For each start the widths are built up one bin at a time,
 * Y_w[i] = Y_{w-1}[i] + P[i+w-1] (the recursion of section 2.2.5). */
void oracle_chunk_maxima(const double *P, int64_t n, int zmax, int64_t chunk, double *M,
                         int64_t *I) {
  int64_t nchunks = (n + chunk - 1) / chunk;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t c = 0; c < nchunks; ++c) {
    double *m = M + c * zmax;
    int64_t *ix = I + c * zmax;
    for (int w = 0; w < zmax; ++w) {
      m[w] = -INFINITY;
      ix[w] = -1;
    }
    int64_t lo = c * chunk, hi = lo + chunk < n ? lo + chunk : n;
    for (int64_t i = lo; i < hi; ++i) {
      double s = 0.0;
      for (int w = 1; w <= zmax && i + w <= n; ++w) {
        s += P[i + w - 1];
        if (s > m[w - 1]) { /* strict: the first (smallest) i keeps a tie */
          m[w - 1] = s;
          ix[w - 1] = i;
        }
      }
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Step 5: significance                                                      */
/* ------------------------------------------------------------------------ */

/* log of the survival function of chi-square with 2w degrees of freedom
 * (section 2.2.3: a width-w boxcar of chi^2(2) powers is chi^2(2w)).  For
 * even dof the survival function has the closed form
 *     P(X > x) = exp(-x/2) * sum_{k=0}^{w-1} (x/2)^k / k!,
 * evaluated here in log space (log-sum-exp over the terms). */
double oracle_log_sf_chi2_2w(double x, int w) {
  if (!(x > 0.0)) return 0.0;
  double y = 0.5 * x, ly = log(y);
  double mx = -INFINITY;
  for (int k = 0; k < w; ++k) {
    double a = k * ly - lgamma(k + 1.0);
    if (a > mx) mx = a;
  }
  double s = 0.0;
  for (int k = 0; k < w; ++k) s += exp(k * ly - lgamma(k + 1.0) - mx);
  return -y + mx + log(s);
}

/* log of the standard normal upper tail, log Phi_c(s).  Direct through erfc
 * while it does not underflow; beyond s = 30 the asymptotic series
 *     Phi_c(s) = phi(s)/s * (1 - 1/s^2 + 3/s^4 - 15/s^6 + ...)
 * (Abramowitz & Stegun 26.2.12), whose omitted terms are below 1e-16 there. */
double oracle_log_norm_sf(double s) {
  if (s < 30.0) return log(0.5 * erfc(s / sqrt(2.0)));
  double inv2 = 1.0 / (s * s), term = 1.0, sum = 1.0;
  for (int k = 1; k <= 8; ++k) {
    term *= -(2.0 * k - 1.0) * inv2;
    sum += term;
  }
  return -0.5 * s * s - log(s) - 0.5 * log(2.0 * M_PI) + log(sum);
}

/* Gaussian-equivalent sigma of a log upper-tail probability: the s with
 * log Phi_c(s) = logp (section 2.2.3, last step).  logp >= 0 gives -inf.
 * Bisection: log Phi_c is strictly decreasing. */
double oracle_sigma_from_logp(double logp) {
  if (!(logp < 0.0)) return -INFINITY;
  double lo = -40.0, hi = 40.0;
  while (oracle_log_norm_sf(hi) > logp) hi *= 2.0;
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid == lo || mid == hi) break;
    if (oracle_log_norm_sf(mid) > logp)
      lo = mid;
    else
      hi = mid;
  }
  return 0.5 * (lo + hi);
}

/* Bonferroni-corrected log p of a width-w boxcar power:
 * min(0, log P(chi^2(2w) > power) + ln ntrials) (section 2.2.3). */
double oracle_log_p_corrected(double power, int w, double ntrials) {
  double lp = oracle_log_sf_chi2_2w(power, w) + log(ntrials);
  return lp < 0.0 ? lp : 0.0;
}

/* Gaussian-equivalent, Bonferroni-corrected significance of a width-w power. */
double oracle_candidate_sigma(double power, int w, double ntrials) {
  return oracle_sigma_from_logp(oracle_log_p_corrected(power, w, ntrials));
}

/* The power T at which the corrected significance of width w equals sigma:
 * the inverse of oracle_candidate_sigma in its first argument, by bisection
 * on log p (monotone in the power). */
double oracle_power_for_sigma(double sigma, int w, double ntrials) {
  double target = oracle_log_norm_sf(sigma);
  double lo = 0.0, hi = 2.0 * w + 10.0;
  while (oracle_log_p_corrected(hi, w, ntrials) > target) hi *= 2.0;
  for (int it = 0; it < 400; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid == lo || mid == hi) break;
    if (oracle_log_p_corrected(mid, w, ntrials) > target)
      lo = mid;
    else
      hi = mid;
  }
  return hi;
}

/* ------------------------------------------------------------------------ */
/* The whole search                                                          */
/* ------------------------------------------------------------------------ */

typedef struct {
  int64_t chunk;  /* chunk index */
  int64_t bin;    /* window start (left edge), 0-based */
  int32_t width;  /* 1..zmax */
  int32_t harm;   /* harmonic stage H the window was found on (1: the power itself) */
  double power;   /* Y_width[bin] */
  double sigma;   /* Bonferroni-corrected Gaussian-equivalent sigma */
  double logp;    /* corrected log p */
} oracle_candidate;

/* Widths searched for candidates (all are summed): every width (mode 0), or
 * the logarithmic z sampling of section 4.1.3 (mode 1), whose list runs
 * z = 1, 2, 4, 8, ... and ends at z-max: the widths whose drift z = w - 1 is
 * a power of two, plus the widest width zmax itself. */
int oracle_width_is_searched(int w, int zmax, int width_search) {
  if (w < 1 || w > zmax) return 0;
  if (width_search == 1) {
    int z = w - 1;
    return w == zmax || (z > 0 && (z & (z - 1)) == 0);
  }
  return 1;
}

/* Harmonic summing (section 2.3; appendix algorithm "Harmonic Sum
 * Decimation").  Decimating the power spectrum by h sums h adjacent,
 * non-overlapping bins, D_h[r] = P[h r] + ... + P[h r + h - 1].  Stage H adds
 * D_1 .. D_H aligned at bin 0 over their common length m = floor(n / H):
 *     S_H[r] = D_1[r] + D_2[r] + ... + D_H[r],   r = 0 .. m - 1,
 * which is chi-square with 2 + 4 + ... + 2H = H(H+1) degrees of freedom under
 * the noise model.  Writes S (m doubles) and returns m. */
int64_t oracle_harmonic_sum(const double *P, int64_t n, int H, double *S) {
  if (H < 1) return 0;
  int64_t m = n / H;
  for (int64_t r = 0; r < m; ++r) {
    double s = 0.0;
    for (int h = 1; h <= H; ++h) {
      double d = 0.0;
      for (int j = 0; j < h; ++j) d += P[(int64_t)h * r + j];
      s += d;
    }
    S[r] = s;
  }
  return m;
}

/* Location a candidate reports (section 2.4, "Approximate r-bin location"):
 * the exact r-bin of its window's left edge, or, in the R-Block variant
 * (rblock > 0), only the index of the rblock-bin block holding that edge,
 * floor(bin / rblock).  The candidate itself (its chunk, width, power and
 * significance) is the same in both variants. */
int64_t oracle_rblock_index(int64_t bin, int64_t rblock) {
  return rblock > 0 ? bin / rblock : bin;
}

/* Search one power series (one harmonic stage): per-chunk maxima of every
 * width, significance with H(H+1) w degrees of freedom (a width-w boxcar of
 * chi^2(H(H+1)) values), and emission of the maxima of searched widths whose
 * corrected significance reaches the threshold, in (chunk, width) order.
 * Appends to out (at most cap - *count entries) and advances *count by the
 * number found. */
static int search_stage(const double *S, int64_t m, int H, int zmax, int64_t chunk,
                        double sigma_thresh, double ntrials, int width_search, int64_t rblock,
                        int64_t cap, oracle_candidate *out, int64_t *count, double *M_out,
                        int64_t *I_out) {
  int64_t nchunks = (m + chunk - 1) / chunk;
  double *M = M_out ? M_out : (double *)malloc((size_t)(nchunks * zmax) * sizeof(double));
  int64_t *I = I_out ? I_out : (int64_t *)malloc((size_t)(nchunks * zmax) * sizeof(int64_t));
  double *lp = (double *)malloc((size_t)(nchunks * zmax) * sizeof(double));
  int ok = M && I && lp;
  if (ok) {
    const int dof_half = H * (H + 1) / 2;  /* chi^2(2 w dof_half) */
    oracle_chunk_maxima(S, m, zmax, chunk, M, I);
    double lthresh = oracle_log_norm_sf(sigma_thresh);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t e = 0; e < nchunks * zmax; ++e) {
      int w = (int)(e % zmax) + 1;
      lp[e] = I[e] >= 0 ? oracle_log_p_corrected(M[e], w * dof_half, ntrials) : 0.0;
    }
    for (int64_t e = 0; e < nchunks * zmax; ++e) {
      if (I[e] < 0 || !oracle_width_is_searched((int)(e % zmax) + 1, zmax, width_search))
        continue;
      if (!(lp[e] <= lthresh) || !(lp[e] < 0.0)) continue;
      if (*count < cap && out) {
        oracle_candidate *o = &out[*count];
        o->chunk = e / zmax;
        o->bin = oracle_rblock_index(I[e], rblock);
        o->width = (int32_t)(e % zmax) + 1;
        o->harm = H;
        o->power = M[e];
        o->logp = lp[e];
        o->sigma = oracle_sigma_from_logp(lp[e]);
      }
      ++*count;
    }
  }
  if (!M_out) free(M);
  if (!I_out) free(I);
  free(lp);
  return ok ? 0 : -1;
}

/* Run the whole search on one spectrum: normalisation, power, and for each
 * harmonic stage H = 1 .. numharm (numharm <= 1: the power alone) the
 * boxcars, per-chunk maxima and threshold.  Emits, in (stage, chunk, width)
 * order, every per-chunk maximum of a searched width whose corrected
 * significance reaches sigma_thresh.  ntrials <= 0 means, per stage, the
 * stage's length times the number of searched widths.  rblock > 0 reports
 * each candidate's r-block index instead of its r-bin.  Writes at most `cap`
 * candidates to `out` and returns the total count, or -1 on invalid
 * arguments or allocation failure.  If M_out / I_out are non-null they
 * receive the (nchunks x zmax) maxima tables of stage 1 and P_out the
 * normalised power. */
int64_t oracle_search_harm(const float *spec, int64_t n, int zmax, int64_t chunk,
                           double sigma_thresh, int64_t norm_block, int mode, double ntrials,
                           int width_search, int numharm, int64_t rblock, int64_t cap,
                           oracle_candidate *out, double *M_out, int64_t *I_out, double *P_out) {
  if (!spec || n < 1 || zmax < 1 || chunk < 1 || rblock < 0) return -1;
  if (numharm < 1) numharm = 1;
  if (norm_block <= 0) norm_block = chunk;
  if (norm_block > n || zmax > n) return -1;
  int searched = 0;
  for (int w = 1; w <= zmax; ++w) searched += oracle_width_is_searched(w, zmax, width_search);
  if (searched == 0) searched = 1;
  double *re = (double *)malloc((size_t)n * sizeof(double));
  double *im = (double *)malloc((size_t)n * sizeof(double));
  double *P = P_out ? P_out : (double *)malloc((size_t)n * sizeof(double));
  double *S = numharm > 1 ? (double *)malloc((size_t)(n / 2 + 1) * sizeof(double)) : NULL;
  int64_t count = -1;
  if (!re || !im || !P || (numharm > 1 && !S)) goto done;
  if (oracle_normalise(spec, n, norm_block, mode, re, im, NULL) != 0) goto done;
  oracle_power(re, im, n, P);
  count = 0;
  for (int H = 1; H <= numharm; ++H) {
    const double *X = P;
    int64_t m = n;
    if (H > 1) {
      m = oracle_harmonic_sum(P, n, H, S);
      X = S;
    }
    if (m < 1) break;
    double nt = ntrials > 0.0 ? ntrials : (double)m * searched;
    if (search_stage(X, m, H, zmax, chunk, sigma_thresh, nt, width_search, rblock, cap, out,
                     &count, H == 1 ? M_out : NULL, H == 1 ? I_out : NULL) != 0) {
      count = -1;
      goto done;
    }
  }
done:
  free(re);
  free(im);
  if (!P_out) free(P);
  free(S);
  return count;
}

/* The search without harmonic summing (numharm = 1). */
int64_t oracle_search(const float *spec, int64_t n, int zmax, int64_t chunk, double sigma_thresh,
                      int64_t norm_block, int mode, double ntrials, int width_search, int64_t cap,
                      oracle_candidate *out, double *M_out, int64_t *I_out, double *P_out) {
  return oracle_search_harm(spec, n, zmax, chunk, sigma_thresh, norm_block, mode, ntrials,
                            width_search, 1, 0, cap, out, M_out, I_out, P_out);
}

/* Number of OpenMP threads a parallel region of this library uses. */
int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void oracle_set_num_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}

/*
 * Drives the FP64 oracle's entry points on small synthetic spectra so that a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer checks their
 * memory accesses and arithmetic: ragged lengths, both normalisations,
 * harmonic stages, logarithmic width sampling, R-Block indices, output
 * truncation, the optional tables, extreme significance arguments and the
 * rejected argument combinations.  Prints "ok <checks>" and exits 0, or
 * prints what failed and exits 1.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
  int64_t chunk;
  int64_t bin;
  int32_t width;
  int32_t harm;
  double power;
  double sigma;
  double logp;
} oracle_candidate;

double oracle_med4(double a, double b, double c, double d);
double oracle_mom(const double *x, int64_t n, double *work);
double oracle_exact_median(const double *x, int64_t n, double *work);
int oracle_normalise(const float *spec, int64_t n, int64_t block, int mode, double *re_out,
                     double *im_out, double *stats);
void oracle_power(const double *re, const double *im, int64_t n, double *P);
void oracle_boxcar(const double *P, int64_t n, int w, double *Y);
void oracle_chunk_maxima(const double *P, int64_t n, int zmax, int64_t chunk, double *M,
                         int64_t *I);
double oracle_log_sf_chi2_2w(double x, int w);
double oracle_log_norm_sf(double s);
double oracle_sigma_from_logp(double logp);
double oracle_log_p_corrected(double power, int w, double ntrials);
double oracle_candidate_sigma(double power, int w, double ntrials);
double oracle_power_for_sigma(double sigma, int w, double ntrials);
int oracle_width_is_searched(int w, int zmax, int width_search);
int64_t oracle_harmonic_sum(const double *P, int64_t n, int H, double *S);
int64_t oracle_rblock_index(int64_t bin, int64_t rblock);
int64_t oracle_search_harm(const float *spec, int64_t n, int zmax, int64_t chunk,
                           double sigma_thresh, int64_t norm_block, int mode, double ntrials,
                           int width_search, int numharm, int64_t rblock, int64_t cap,
                           oracle_candidate *out, double *M_out, int64_t *I_out, double *P_out);
int64_t oracle_search(const float *spec, int64_t n, int zmax, int64_t chunk, double sigma_thresh,
                      int64_t norm_block, int mode, double ntrials, int width_search, int64_t cap,
                      oracle_candidate *out, double *M_out, int64_t *I_out, double *P_out);

static int checks = 0, failures = 0;
static void expect(int ok, const char *what) {
  ++checks;
  if (!ok) {
    ++failures;
    printf("FAILED: %s\n", what);
  }
}

/* 64-bit linear congruential generator and Box-Muller pairs */
static uint64_t state = 0x9E3779B97F4A7C15ull;
static double uniform01(void) {
  state = state * 6364136223846793005ull + 1442695040888963407ull;
  return ((state >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}
static void gaussian_spectrum(float *x, int64_t n) {
  for (int64_t i = 0; i < n; ++i) {
    double r = sqrt(-2.0 * log(uniform01())), t = 2.0 * M_PI * uniform01();
    x[2 * i] = (float)(r * cos(t));
    x[2 * i + 1] = (float)(r * sin(t));
  }
}
/* a boxcar tone of `w` bins starting at bin `b`, amplitude `a` */
static void add_tone(float *x, int64_t n, int64_t b, int w, float a) {
  for (int64_t i = b; i < b + w && i < n; ++i) x[2 * i] += a;
}

static void run_search(const float *x, int64_t n, int zmax, int64_t chunk, int64_t block,
                       int mode, int ws, int numharm, int64_t rblock, int64_t cap) {
  int64_t nch = (n + chunk - 1) / chunk;
  oracle_candidate *out = (oracle_candidate *)malloc((size_t)(cap > 0 ? cap : 1) * sizeof *out);
  double *M = (double *)malloc((size_t)(nch * zmax) * sizeof(double));
  int64_t *I = (int64_t *)malloc((size_t)(nch * zmax) * sizeof(int64_t));
  double *P = (double *)malloc((size_t)n * sizeof(double));
  int64_t c = oracle_search_harm(x, n, zmax, chunk, 6.0, block, mode, 0.0, ws, numharm, rblock,
                                 cap, out, M, I, P);
  expect(c >= 0, "search returns a count");
  int64_t shown = c < cap ? c : cap;
  for (int64_t i = 0; i < shown; ++i) {
    expect(out[i].width >= 1 && out[i].width <= zmax && out[i].harm >= 1 &&
               out[i].harm <= (numharm < 1 ? 1 : numharm) && out[i].chunk >= 0 &&
               out[i].chunk < nch && isfinite(out[i].power) && out[i].sigma >= 6.0 - 1e-9,
           "candidate fields in range");
  }
  for (int64_t e = 0; e < nch * zmax; ++e)
    expect(I[e] == -1 ? M[e] == -INFINITY : (I[e] >= 0 && I[e] + e % zmax + 1 <= n),
           "table entry consistent");
  int64_t c2 = oracle_search(x, n, zmax, chunk, 6.0, block, mode, 0.0, ws, 0, NULL, NULL, NULL,
                             NULL);
  if (numharm <= 1 && rblock == 0) expect(c2 == c, "counting call agrees");
  free(out);
  free(M);
  free(I);
  free(P);
}

int main(void) {
  /* medians */
  double v[1025], work[1025];
  for (int i = 0; i < 1025; ++i) v[i] = uniform01();
  expect(oracle_med4(1, 2, 3, 4) == 2.5, "med4");
  for (int64_t n = 1; n <= 1025; n += 64) expect(isfinite(oracle_exact_median(v, n, work)), "median");
  for (int64_t n = 1; n <= 1024; n *= 4) expect(isfinite(oracle_mom(v, n, work)), "mom");

  /* normalisation with a ragged tail, both modes, invalid arguments */
  const int64_t n = 10000 + 37;
  float *x = (float *)malloc((size_t)(2 * n) * sizeof(float));
  gaussian_spectrum(x, n);
  add_tone(x, n, 1000, 12, 3.0f);
  add_tone(x, n, n - 20, 20, 2.0f);
  double *re = (double *)malloc((size_t)n * sizeof(double));
  double *im = (double *)malloc((size_t)n * sizeof(double));
  double *st = (double *)malloc((size_t)(4 * ((n + 63) / 64)) * sizeof(double));
  double *P = (double *)malloc((size_t)n * sizeof(double));
  expect(oracle_normalise(x, n, 256, 0, re, im, st) == 0, "normalise mom");
  expect(oracle_normalise(x, n, 100, 1, re, im, st) == 0, "normalise exact");
  expect(oracle_normalise(x, n, 100, 0, re, im, st) == -1, "mom needs 4^k blocks");
  expect(oracle_normalise(x, n, n + 1, 1, re, im, st) == -1, "block beyond n");
  expect(oracle_normalise(x, n, 64, 2, re, im, st) == -1, "unknown mode");
  oracle_power(re, im, n, P);

  /* boxcars, maxima, harmonic sums */
  double *Y = (double *)malloc((size_t)n * sizeof(double));
  for (int w = 1; w <= 40; w += 13) oracle_boxcar(P, n, w, Y);
  const int zmax = 50;
  const int64_t chunk = 256, nch = (n + chunk - 1) / chunk;
  double *M = (double *)malloc((size_t)(nch * zmax) * sizeof(double));
  int64_t *I = (int64_t *)malloc((size_t)(nch * zmax) * sizeof(int64_t));
  oracle_chunk_maxima(P, n, zmax, chunk, M, I);
  double *S = (double *)malloc((size_t)n * sizeof(double)); /* stage 1 has n bins */
  for (int H = 1; H <= 8; ++H) expect(oracle_harmonic_sum(P, n, H, S) == n / H, "stage length");
  expect(oracle_harmonic_sum(P, n, 0, S) == 0, "stage 0");

  /* significance over wide argument ranges */
  for (int w = 1; w <= 4096; w *= 2) {
    for (double p = 0.0; p < 20000.0; p = p * 3.0 + 0.5) {
      double l = oracle_log_sf_chi2_2w(p, w);
      expect(l <= 1e-12 && !isnan(l), "log sf (rounding may leave it a few ulp above 0)");
      double s = oracle_candidate_sigma(p, w, 1e8);
      expect(!isnan(s), "sigma");
    }
    double t = oracle_power_for_sigma(6.0, w, 1e8);
    expect(t > 0.0 && isfinite(t), "threshold");
  }
  for (double s = -10.0; s <= 60.0; s += 0.75) expect(!isnan(oracle_log_norm_sf(s)), "norm sf");
  for (double lp = -2000.0; lp < 0.0; lp = lp * 0.7 + 0.01)
    expect(!isnan(oracle_sigma_from_logp(lp)), "sigma from log p");
  for (int w = 0; w <= 70; ++w) (void)oracle_width_is_searched(w, 64, w & 1);
  expect(oracle_rblock_index(1000, 64) == 15 && oracle_rblock_index(1000, 0) == 1000, "rblock");

  /* whole searches */
  run_search(x, n, 50, 256, 256, 0, 0, 1, 0, 10000);
  run_search(x, n, 64, 512, 1024, 0, 1, 1, 0, 10000);
  run_search(x, n, 33, 256, 100, 1, 0, 1, 0, 10000);
  run_search(x, n, 40, 256, 256, 0, 0, 3, 0, 10000);
  run_search(x, n, 50, 256, 256, 0, 0, 1, 32, 10000);
  run_search(x, n, 50, 256, 256, 0, 0, 1, 0, 3);
  run_search(x, 4096, 4096, 4096, 4096, 0, 0, 1, 0, 100);
  expect(oracle_search(x, n, 0, 256, 6.0, 256, 0, 0.0, 0, 0, NULL, NULL, NULL, NULL) == -1,
         "zmax 0 rejected");
  expect(oracle_search(x, n, 50, 0, 6.0, 256, 0, 0.0, 0, 0, NULL, NULL, NULL, NULL) == -1,
         "chunk 0 rejected");
  expect(oracle_search(NULL, n, 50, 256, 6.0, 256, 0, 0.0, 0, 0, NULL, NULL, NULL, NULL) == -1,
         "null spectrum rejected");

  free(x);
  free(re);
  free(im);
  free(st);
  free(P);
  free(Y);
  free(M);
  free(I);
  free(S);
  if (failures) return 1;
  printf("ok %d\n", checks);
  return 0;
}

// Significance on the device, in FP64, and the passes after the bank: the
// per-width power thresholds, the scan of the per-tile candidate counts, and
// the emission of the candidates in canonical order with their
// Gaussian-equivalent sigma (section 2.2.3: a width-w boxcar of chi^2(2)
// powers is chi^2(2w); its survival probability is Bonferroni-corrected for
// the number of trials and converted to the normal quantile).
#include <float.h>

#include "internal.hpp"

namespace pulscan {

// log P(chi^2(2w) > x).  For even dof the survival function is
// exp(-x/2) * sum_{k<w} (x/2)^k / k!; the sum is taken relative to its largest
// term (at k = min(w-1, floor(x/2))) so that neither tail of it overflows.
// log(k!) for an integer k: Stirling's series for k >= 16 (terms through
// 1/x^7, error below 1e-16 relative there), a table below (the values of
// log k! rounded to double).
__constant__ double kLogFactorialSmall[16] = {
    0.0, 0.0, 0.6931471805599453, 1.791759469228055, 3.1780538303479458, 4.787491742782046,
    6.579251212010101, 8.525161361065415, 10.60460290274525, 12.801827480081469,
    15.104412573075516, 17.502307845873887, 19.987214495661885, 22.552163853123425,
    25.19122118273868, 27.89927138384089};

__device__ double log_factorial(uint32_t k) {
  if (k < 16) return kLogFactorialSmall[k];
  const double x = (double)k + 1.0, ix = 1.0 / x, ix2 = ix * ix;
  const double series =
      ix * (1.0 / 12.0 - ix2 * (1.0 / 360.0 - ix2 * (1.0 / 1260.0 - ix2 * (1.0 / 1680.0))));
  return (x - 0.5) * log(x) - x + 0.91893853320467274178 + series;
}

__device__ double log_sf_chi2_even(double x, uint32_t w) {
  if (!(x > 0.0)) return 0.0;
  const double y = 0.5 * x;
  const uint32_t kp = (y >= (double)(w - 1)) ? w - 1 : (uint32_t)floor(y);
  const double log_peak = (double)kp * log(y) - log_factorial(kp);
  // Terms are taken several at a time: the products of the ratios do not
  // depend on the running term, so the dependent chain advances one
  // multiplication per step (one candidate per thread, few threads: the
  // chain's latency is the kernel's time).  Below the peak, where the long
  // runs are, eight terms a step; above it, four.
  double acc = 1.0, r = 1.0;
  const double iy = 1.0 / y;
  uint32_t k = kp;
  for (; k >= 8; k -= 8) {  // terms below the peak shrink by k / y
    double a[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = (double)(k - j) * iy;
    const double b12 = a[0] * a[1], b34 = a[2] * a[3], b56 = a[4] * a[5], b78 = a[6] * a[7];
    const double b1234 = b12 * b34, b5678 = b56 * b78;
    const double p3 = b12 * a[2], p5 = b1234 * a[4], p6 = b1234 * b56;
    const double p7 = p6 * a[6], p8 = b1234 * b5678;
    const double s14 = (r * a[0] + r * b12) + (r * p3 + r * b1234);
    const double s58 = (r * p5 + r * p6) + (r * p7 + r * p8);
    acc += s14 + s58;
    r *= p8;
    if (r < 1e-18 * acc) break;
  }
  if (k < 8 && !(r < 1e-18 * acc)) {
    for (; k >= 1; --k) {
      r *= (double)k * iy;
      acc += r;
    }
  }
  r = 1.0;
  k = kp + 1;
  for (; k + 3 < w; k += 4) {  // terms above the peak shrink by y / k
    const double a1 = y / (double)k, a2 = y / (double)(k + 1);
    const double a3 = y / (double)(k + 2), a4 = y / (double)(k + 3);
    const double b12 = a1 * a2, b123 = b12 * a3, b1234 = b12 * (a3 * a4);
    const double r1 = r * a1, r2 = r * b12, r3 = r * b123, r4 = r * b1234;
    acc += (r1 + r2) + (r3 + r4);
    r = r4;
    if (r < 1e-18 * acc) break;
  }
  if (k + 3 >= w && !(r < 1e-18 * acc)) {
    for (; k < w; ++k) {
      r *= y / (double)k;
      acc += r;
    }
  }
  return -y + log_peak + log(acc);
}

// log of the chi^2(2w) density.
__device__ double log_pdf_chi2_even(double x, uint32_t w) {
  return (double)(w - 1) * log(0.5 * x) - 0.5 * x - M_LN2 - log_factorial(w - 1);
}

// log Phi_c(s), the standard normal upper tail.  For s > 0 the scaled
// complementary error function keeps it finite far into the tail:
// Phi_c(s) = exp(-s^2/2) erfcx(s / sqrt 2) / 2.
__device__ double log_norm_sf(double s) {
  if (s > 0.0) return -0.5 * s * s + log(0.5 * erfcx(s * M_SQRT1_2));
  return log(0.5 * erfc(s * M_SQRT1_2));
}

// log Phi_c(s) and its derivative -phi(s) / Phi_c(s) together (one erfcx).
__device__ void log_norm_sf_d(double s, double &f, double &df) {
  if (s > 0.0) {
    const double ex = erfcx(s * M_SQRT1_2);
    f = -0.5 * s * s + log(0.5 * ex);
    df = -M_SQRT2 / (sqrt(M_PI) * ex);
  } else {
    f = log(0.5 * erfc(s * M_SQRT1_2));
    df = -exp(-0.5 * s * s - 0.5 * log(2.0 * M_PI) - f);
  }
}

// The s with log Phi_c(s) = L (L < 0); -inf for L >= 0.  Halley's method on
// f(s) = log Phi_c(s) - L, a concave, decreasing function; the start solves
// the tail's leading terms, -s^2/2 - ln(s sqrt(2 pi)) = L.  The second
// derivative comes with the first: with h = -f' (the inverse Mills ratio),
// f'' = -h (h - s) = f' (-f' - s).
__device__ __forceinline__ double sigma_from_logp(double L) {
  if (!(L < 0.0)) return -INFINITY;
  double s = 0.0;
  if (L < -1.0) {
    // the tail's asymptotic form, log Q(s) ~ -s^2/2 - log(s sqrt(2 pi)) +
    // log(1 - 1/s^2 + 3/s^4), solved by two fixed-point steps from the
    // leading term, leaves Newton a few digits to add
    s = sqrt(-2.0 * L);
    s = sqrt(fmax(-2.0 * L - 2.0 * log(s * 2.5066282746310002), 1.0));
    if (s > 2.0) {
      const double q = 1.0 / (s * s);
      s = sqrt(fmax(-2.0 * L - 2.0 * log(s * 2.5066282746310002) + 2.0 * log1p(q * (3.0 * q - 1.0)),
                    1.0));
    }
  }
  // Halley's iteration converges cubically: a step of at most 1e-4 (relative
  // to max(1, s)) leaves an error of order 1e-12, so it ends the iteration.
  // From the start's error (below 5e-5 relative for L <= -20, i.e. s >= 6)
  // that is the first step; closer to the body of the distribution a few
  // more (the result is reported in FP32).
  for (int it = 0; it < 200; ++it) {
    double f, df;
    log_norm_sf_d(s, f, df);
    const double g = f - L, d2 = df * (-df - s);
    const double step = 2.0 * g * df / (2.0 * df * df - g * d2);
    s -= step;
    if (fabs(step) <= 1e-4 * fmax(1.0, fabs(s))) break;
  }
  return s;
}

// The power x at which the corrected significance of a width-w boxcar
// reaches sigma: log P(chi^2(2w) > x) = log Phi_c(sigma) - ln(ntrials).
// Newton on the concave, decreasing log survival function (after its first
// step every iterate lies above the root and they fall to it).  The start is
// the Wilson-Hilferty approximation, whose cube root of chi^2(k) / k is
// normal with mean 1 - 2/(9k) and variance 2/(9k), taken at the normal
// quantile of the same tail probability: within 1e-3 of the root at k = 400
// and 6 sigma, half the iterations of a start at the mean.
__device__ double power_threshold(double sigma, uint32_t w, double ntrials) {
  const double target = log_norm_sf(sigma) - log(ntrials);
  if (!(target < 0.0)) return 0.0;
  const double k = 2.0 * (double)w, c = 2.0 / (9.0 * k);
  const double r = 1.0 - c + sigma_from_logp(target) * sqrt(c);
  double x = r > 0.0 ? k * (r * r * r) : k;
  for (int it = 0; it < 400; ++it) {
    const double ls = log_sf_chi2_even(x, w);
    const double f = ls - target;
    const double df = -exp(log_pdf_chi2_even(x, w) - ls);
    double nx = x - f / df;
    if (!(nx > 0.0)) nx = 0.5 * x;
    const double step = nx - x;
    x = nx;
    if (fabs(step) <= 1e-15 * x) break;
  }
  return x;
}

// Smallest FP32 value >= t, so that "power >= threshold" in FP32 means the
// FP64 condition on the same power.
__device__ float round_up_f32(double t) {
  float f = (float)t;
  if ((double)f < t) f = nextafterf(f, INFINITY);
  return f;
}

__global__ void threshold_kernel(const ThreshJob *__restrict__ jobs, ThreshJob single, double sigma,
                                 int width_search, int debug) {
  const ThreshJob jb = jobs ? jobs[blockIdx.y] : single;
  const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x + 1;
  if (w > jb.zc) return;
  float out;
  if (!width_searched(w, jb.zmax, width_search))
    out = INFINITY;
  else if (debug)
    out = -FLT_MAX;
  else
    out = round_up_f32(power_threshold(sigma, w * jb.dofmul, jb.ntrials));
  jb.thr[w - 1] = out;
}

hipError_t launch_thresholds(const ThreshJob *jobs_dev, const ThreshJob &single, int njobs,
                             uint32_t zc_max, double sigma, int width_search, int debug,
                             hipStream_t stream) {
  dim3 grid((zc_max + 63) / 64, njobs);
  hipLaunchKernelGGL(threshold_kernel, grid, dim3(64), 0, stream, jobs_dev, single, sigma,
                     width_search, debug);
  return hipGetLastError();
}

// The FP32 boxcar power of the window [bin, bin + w) of a series: its powers
// recomputed from the raw spectrum with its blocks' statistics exactly as the
// bank kernel normalises them (or read, for a power series), summed in
// increasing order.  The re-check of the FP16-stored search.
__device__ float power32_window(const SpecDesc &d, uint32_t B, int from_power, uint32_t bin,
                                uint32_t w) {
  float acc = 0.f;
  if (from_power) {
    const float *P = reinterpret_cast<const float *>(d.x);
    for (uint32_t j = bin; j < bin + w; ++j) acc += P[j];
    return acc;
  }
  for (uint32_t j = bin; j < bin + w; ++j) {
    const float *st = d.aux + 4 * (size_t)(j / B);
    const float med_re = st[0], mad_re = st[1], med_im = st[2], mad_im = st[3];
    const float inv_re = mad_re > 0.f ? 1.0f / (mad_re * kMadScale) : 0.f;
    const float inv_im = mad_im > 0.f ? 1.0f / (mad_im * kMadScale) : 0.f;
    const float2 x = d.x[j];
    const float a = fmaf(x.x, inv_re, -med_re * inv_re);
    const float c = fmaf(x.y, inv_im, -med_im * inv_im);
    acc += fmaf(a, a, c * c);
  }
  return acc;
}

// ---------------------------------------------------------------------------
// Emit: pool entry f (tile, rank) goes to its canonical place, the tile's
// exclusive prefix plus its rank, with its Gaussian-equivalent sigma.

// One wave per workgroup: the few candidate chains of a search then run on
// as many CUs as there are waves, none sharing a CU's instruction fetch.
constexpr int kEmitThreads = 64;

__global__ __launch_bounds__(kEmitThreads) void emit_kernel(EmitParams p, SpecDesc single) {
  // Each thread's significance is a long dependent chain: the entry's
  // prefix is loaded before it and used only after it.
  // The first pool entry is requested before the candidate count arrives: the
  // pool holds pool_cap entries, so the read is in bounds, and its value is
  // used only when the entry lies below the count.
  const uint64_t stride = (uint64_t)gridDim.x * kEmitThreads;
  const uint64_t f0 = (uint64_t)blockIdx.x * kEmitThreads + threadIdx.x;
  if (*p.overflow == 2u) {
    // a count was lost (the search reports PULSCAN_EHIP): re-arm what the
    // late workgroups left behind instead of placing anything
    if (p.tile_word)
      for (uint64_t i = f0; i < p.ntiles; i += stride) p.tile_word[i] = 0ull;
    if (f0 == 0) *p.pool_head = 0u;
    return;
  }
  if (f0 >= p.pool_cap) return;
  const StageEntry e0 = p.pool[f0];
  const unsigned long long total = *p.total;
  const uint64_t lim = total < p.pool_cap ? total : p.pool_cap;
  for (uint64_t f = f0; f < lim; f += stride) {
    const StageEntry e = f == f0 ? e0 : p.pool[f];
    const uint64_t dest = (uint64_t)p.tile_prefix[e.unit] + e.rank +
                          (p.span_prefix ? p.span_prefix[e.unit / kScanSpan] : 0u);
    const SpecDesc &d = p.nspec > 1 ? p.descs[e.spec] : single;
    const uint32_t w = e.width;
    double lp = log_sf_chi2_even((double)e.power, w * d.dofmul) + log(d.ntrials);
    float pw = e.power;
    bool recheck = false;
    // within the FP16 re-check band, sigma < sigma_req + band, i.e. (sigma
    // falling as log p rises) log p above log Q(sigma_req + band); or from
    // saturated FP16 input: the FP32 power decides
    if (p.fp16 && (lp > log_norm_sf((double)p.sigma + kRecheckBand) || !(pw < kRecheckPower))) {
      recheck = true;
      pw = power32_window(d, p.block, p.from_power, e.bin, w);
      lp = log_sf_chi2_even((double)pw, w * d.dofmul) + log(d.ntrials);
    }
    const double lpc = lp < 0.0 ? lp : 0.0;
    const double sg = sigma_from_logp(lpc);
    const bool keep = !recheck || sg >= (double)p.sigma;
    pulscan_candidate c;
    c.spectrum = d.spec_id;
    c.bin = p.rblock ? e.bin / p.rblock : e.bin;
    c.width = w;
    c.power = pw;
    c.sigma = keep ? (float)sg : NAN;
    c.chunk = e.bin / p.chunk;
    c.harmonics = d.harm;
    c.logp = (float)lpc;
    if (dest < p.capacity) p.out[dest] = c;
  }
}

hipError_t launch_emit(const EmitParams &p, const SpecDesc &single, uint32_t grid,
                       hipStream_t stream) {
  hipLaunchKernelGGL(emit_kernel, dim3(grid), dim3(kEmitThreads), 0, stream, p, single);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Final pass over a canonical candidate list: drops the entries the FP32
// re-check rejected (sigma NaN) and, with `best`, keeps of each (spectrum,
// stage, chunk) only its highest-sigma entry (the first on ties).  Each key
// is one contiguous run of the list.  One workgroup walks the list in rounds
// of kFinThreads; ranks come from ballots, so the order is kept.

constexpr int kFinThreads = 1024;

__device__ __forceinline__ bool same_key(const pulscan_candidate &a, const pulscan_candidate &b) {
  return a.spectrum == b.spectrum && a.harmonics == b.harmonics && a.chunk == b.chunk;
}

__global__ __launch_bounds__(kFinThreads) void finalize_kernel(
    const pulscan_candidate *__restrict__ all, const unsigned long long *__restrict__ total_p,
    uint64_t all_cap, pulscan_candidate *__restrict__ out, uint64_t capacity,
    unsigned long long *count, unsigned long long *count2, const uint32_t *overflow, int best) {
  __shared__ uint32_t wave_cnt[kFinThreads / 64];
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const unsigned long long tot = *total_p;
  const uint64_t n = tot < all_cap ? tot : all_cap;
  uint64_t kept = 0;
  for (uint64_t base = 0; base < n; base += kFinThreads) {
    const uint64_t i = base + tid;
    bool emit = false;
    uint64_t pick = i;
    if (i < n) {
      if (!best) {
        emit = !isnan(all[i].sigma);
      } else if (i == 0 || !same_key(all[i - 1], all[i])) {
        // run head: the best surviving entry of the run
        for (uint64_t j = i; j < n && same_key(all[i], all[j]); ++j) {
          if (isnan(all[j].sigma)) continue;
          if (!emit || all[j].sigma > all[pick].sigma) pick = j;
          emit = true;
        }
      }
    }
    const unsigned long long mask = __ballot(emit);
    if (lane == 0) wave_cnt[wave] = (uint32_t)__popcll(mask);
    __syncthreads();
    uint64_t before = 0, here = 0;
    for (uint32_t v = 0; v < kFinThreads / 64; ++v) {
      before += v < wave ? wave_cnt[v] : 0u;
      here += wave_cnt[v];
    }
    if (emit) {
      const uint64_t rank = kept + before + (uint64_t)__popcll(mask & ((1ull << lane) - 1ull));
      if (rank < capacity) out[rank] = all[pick];
    }
    kept += here;
    __syncthreads();
  }
  if (tid == 0) {
    *count = kept;
    if (count2) *count2 = count_word(kept, *overflow);
  }
}

hipError_t launch_finalize(const pulscan_candidate *all, const unsigned long long *total,
                           uint64_t all_cap, pulscan_candidate *out, uint64_t capacity,
                           unsigned long long *count, unsigned long long *count2,
                           const uint32_t *overflow, int best, hipStream_t stream) {
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kFinThreads), 0, stream, all, total, all_cap,
                     out, capacity, count, count2, overflow, best);
  return hipGetLastError();
}

}  // namespace pulscan

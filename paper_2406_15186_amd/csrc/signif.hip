// Significance on the device, in FP64: per-width power thresholds and the
// finalising pass that orders the staged candidates and attaches their
// Gaussian-equivalent sigma (section 2.2.3: a width-w boxcar of chi^2(2)
// powers is chi^2(2w); its survival probability is Bonferroni-corrected for
// the number of trials and converted to the normal quantile).
#include <float.h>

#include "internal.hpp"

namespace pulscan {

// log P(chi^2(2w) > x).  For even dof the survival function is
// exp(-x/2) * sum_{k<w} (x/2)^k / k!; the sum is taken relative to its largest
// term (at k = min(w-1, floor(x/2))) so that neither tail of it overflows.
__device__ double log_sf_chi2_even(double x, uint32_t w) {
  if (!(x > 0.0)) return 0.0;
  const double y = 0.5 * x;
  const uint32_t kp = (y >= (double)(w - 1)) ? w - 1 : (uint32_t)floor(y);
  const double log_peak = (double)kp * log(y) - lgamma((double)kp + 1.0);
  double acc = 1.0, r = 1.0;
  for (uint32_t k = kp; k >= 1; --k) {  // terms below the peak shrink by k / y
    r *= (double)k / y;
    acc += r;
    if (r < 1e-18 * acc) break;
  }
  r = 1.0;
  for (uint32_t k = kp + 1; k < w; ++k) {  // terms above the peak shrink by y / k
    r *= y / (double)k;
    acc += r;
    if (r < 1e-18 * acc) break;
  }
  return -y + log_peak + log(acc);
}

// log of the chi^2(2w) density.
__device__ double log_pdf_chi2_even(double x, uint32_t w) {
  return (double)(w - 1) * log(0.5 * x) - 0.5 * x - M_LN2 - lgamma((double)w);
}

// log Phi_c(s), the standard normal upper tail.  For s > 0 the scaled
// complementary error function keeps it finite far into the tail:
// Phi_c(s) = exp(-s^2/2) erfcx(s / sqrt 2) / 2.
__device__ double log_norm_sf(double s) {
  if (s > 0.0) return -0.5 * s * s + log(0.5 * erfcx(s * M_SQRT1_2));
  return log(0.5 * erfc(s * M_SQRT1_2));
}

// d/ds log Phi_c(s) = -phi(s) / Phi_c(s).
__device__ double dlog_norm_sf(double s) {
  if (s > 0.0) return -M_SQRT2 / (sqrt(M_PI) * erfcx(s * M_SQRT1_2));
  return -exp(-0.5 * s * s - 0.5 * log(2.0 * M_PI) - log_norm_sf(s));
}

// The s with log Phi_c(s) = L (L < 0); -inf for L >= 0.  Newton's method on a
// concave, decreasing function converges from either side of the root.
__device__ double sigma_from_logp(double L) {
  if (!(L < 0.0)) return -INFINITY;
  double s = (L < -1.0) ? sqrt(-2.0 * L) : 0.0;
  for (int it = 0; it < 200; ++it) {
    const double step = (log_norm_sf(s) - L) / dlog_norm_sf(s);
    s -= step;
    if (fabs(step) <= 1e-14 * fmax(1.0, fabs(s))) break;
  }
  return s;
}

// The power x at which the corrected significance of a width-w boxcar
// reaches sigma: log P(chi^2(2w) > x) = log Phi_c(sigma) - ln(ntrials).
// Newton on the concave, decreasing log survival function.
__device__ double power_threshold(double sigma, uint32_t w, double ntrials) {
  const double target = log_norm_sf(sigma) - log(ntrials);
  if (!(target < 0.0)) return 0.0;
  double x = 2.0 * (double)w;
  for (int it = 0; it < 400; ++it) {
    const double f = log_sf_chi2_even(x, w) - target;
    const double df = -exp(log_pdf_chi2_even(x, w) - log_sf_chi2_even(x, w));
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
  if (w > jb.zmax || !width_searched(w, width_search))
    out = INFINITY;
  else if (debug)
    out = -FLT_MAX;
  else
    out = round_up_f32(power_threshold(sigma, w, jb.ntrials));
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

// ---------------------------------------------------------------------------
// Finalise: one workgroup per spectrum.

constexpr int kFinThreads = 1024;

__device__ unsigned long long block_sum(unsigned long long v, unsigned long long *red) {
  // wave sum, then across the 16 waves of the workgroup
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  unsigned long long t = 0;
  for (int i = 0; i < kFinThreads / 64; ++i) t += red[i];
  return t;
}

// In-place ascending bitonic sort of n (a power of two) 64-bit keys by the
// whole workgroup.
__device__ void bitonic_sort(uint64_t *a, uint32_t n) {
  for (uint32_t k = 2; k <= n; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = threadIdx.x; i < n; i += kFinThreads) {
        const uint32_t l = i ^ j;
        if (l > i) {
          const uint64_t x = a[i], y = a[l];
          const bool up = (i & k) == 0;
          if ((x > y) == up) {
            a[i] = y;
            a[l] = x;
          }
        }
      }
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(kFinThreads) void finalise_kernel(FinalParams p, SpecDesc single) {
  __shared__ uint64_t keys[kSortLds];
  __shared__ unsigned long long red[kFinThreads / 64];
  const int s = blockIdx.x;
  const SpecDesc d = p.descs ? p.descs[s] : single;

  unsigned long long before = 0, all = 0;
  for (int i = threadIdx.x; i < p.nspec; i += kFinThreads) {
    const unsigned long long c = p.counts[i];
    all += c;
    if (i < s) before += c;
  }
  before = block_sum(before, red);
  all = block_sum(all, red);
  if (threadIdx.x == 0) {
    p.counts_next[s] = 0;
    if (s == 0) {
      if (p.total) *p.total = all;
      if (p.total2) *p.total2 = all;
    }
  }
  unsigned long long cnt = p.counts[s];
  if (cnt > d.stage_cap) cnt = d.stage_cap;
  if (cnt == 0) return;

  uint32_t n2 = 1;
  while (n2 < cnt) n2 <<= 1;
  uint64_t *a = n2 <= (uint32_t)kSortLds ? keys : p.sort_scratch + 2 * d.stage_off;
  const StageEntry *st = p.stage + d.stage_off;
  for (uint32_t i = threadIdx.x; i < n2; i += kFinThreads)
    a[i] = i < cnt ? (((uint64_t)st[i].key << 32) | i) : ~0ull;
  __syncthreads();
  bitonic_sort(a, n2);

  for (uint32_t j = threadIdx.x; j < cnt; j += kFinThreads) {
    const unsigned long long pos = before + j;
    if (pos >= p.capacity) break;
    const StageEntry e = st[(uint32_t)(a[j] & 0xFFFFFFFFull)];
    const double lp = log_sf_chi2_even((double)e.power, e.width) + log(d.ntrials);
    pulscan_candidate c;
    c.spectrum = (uint32_t)s;
    c.bin = e.bin;
    c.width = e.width;
    c.power = e.power;
    c.sigma = (float)sigma_from_logp(lp < 0.0 ? lp : 0.0);
    c.chunk = e.key / d.zmax;
    p.out[pos] = c;
  }
}

hipError_t launch_finalise(const FinalParams &p, const SpecDesc &single, hipStream_t stream) {
  hipLaunchKernelGGL(finalise_kernel, dim3(p.nspec), dim3(kFinThreads), 0, stream, p, single);
  return hipGetLastError();
}

}  // namespace pulscan

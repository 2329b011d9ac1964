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
// Scan of the per-tile counts: one workgroup.  Thread t sums a contiguous
// run of tiles, the run totals are scanned in LDS, and each thread writes the
// prefixes of its run.

constexpr int kScanThreads = 1024;

__global__ __launch_bounds__(kScanThreads) void scan_kernel(ScanParams p) {
  __shared__ uint32_t part[kScanThreads];
  const uint64_t T = p.total_tiles;
  const uint64_t per = (T + kScanThreads - 1) / kScanThreads;
  const uint64_t lo = (uint64_t)threadIdx.x * per;
  const uint64_t hi = lo + per < T ? lo + per : T;
  uint32_t sum = 0;
  for (uint64_t t = lo; t < hi; ++t) sum += p.tile_count[t];
  part[threadIdx.x] = sum;
  __syncthreads();
  // Hillis-Steele inclusive scan of the run totals
  for (int o = 1; o < kScanThreads; o <<= 1) {
    const uint32_t v = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t run = threadIdx.x ? part[threadIdx.x - 1] : 0u;
  for (uint64_t t = lo; t < hi; ++t) {
    p.tile_prefix[t] = run;
    run += p.tile_count[t];
  }
  if (threadIdx.x == kScanThreads - 1) {
    const uint32_t total = part[kScanThreads - 1];
    p.tile_prefix[T] = total;
    if (p.total) *p.total = total;
    if (p.total2) *p.total2 = total;
    *p.overflow = *p.pool_head > p.pool_cap ? 1u : 0u;
    *p.pool_head = 0u;
  }
}

hipError_t launch_scan(const ScanParams &p, hipStream_t stream) {
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(kScanThreads), 0, stream, p);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Emit: candidate f of the canonical order (tile order, then the tile's own
// (chunk, width) order) is found by binary search over the tile prefixes.

constexpr int kEmitThreads = 256;

__global__ __launch_bounds__(kEmitThreads) void emit_kernel(EmitParams p, SpecDesc single) {
  const uint64_t T = p.total_tiles;
  const uint64_t total = p.tile_prefix[T];
  const uint64_t lim = total < p.capacity ? total : p.capacity;
  const uint64_t stride = (uint64_t)gridDim.x * kEmitThreads;
  for (uint64_t f = (uint64_t)blockIdx.x * kEmitThreads + threadIdx.x; f < lim; f += stride) {
    // largest t with tile_prefix[t] <= f (that tile holds candidate f)
    uint64_t lo = 0, hi = T - 1;
    while (lo < hi) {
      const uint64_t mid = (lo + hi + 1) >> 1;
      if (p.tile_prefix[mid] <= f)
        lo = mid;
      else
        hi = mid - 1;
    }
    const uint64_t t = lo;
    const uint64_t idx = (uint64_t)p.tile_pos[t] + (f - p.tile_prefix[t]);
    if (idx >= p.pool_cap) continue;  // lost to a staging overflow (reported)
    int s = 0;
    if (p.nspec > 1) {
      int a = 0, b = p.nspec - 1;
      while (a < b) {
        const int mid = (a + b + 1) >> 1;
        if (p.descs[mid].tile_begin <= t)
          a = mid;
        else
          b = mid - 1;
      }
      s = a;
    }
    const double ntrials = p.nspec > 1 ? p.descs[s].ntrials : single.ntrials;
    const StageEntry e = p.pool[idx];
    const double lp = log_sf_chi2_even((double)e.power, e.width) + log(ntrials);
    pulscan_candidate c;
    c.spectrum = (uint32_t)s;
    c.bin = e.bin;
    c.width = e.width;
    c.power = e.power;
    c.sigma = (float)sigma_from_logp(lp < 0.0 ? lp : 0.0);
    c.chunk = e.chunk;
    p.out[f] = c;
  }
}

hipError_t launch_emit(const EmitParams &p, const SpecDesc &single, uint32_t grid,
                       hipStream_t stream) {
  hipLaunchKernelGGL(emit_kernel, dim3(grid), dim3(kEmitThreads), 0, stream, p, single);
  return hipGetLastError();
}

}  // namespace pulscan

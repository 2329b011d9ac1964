// Harmonic summing (section 2.3; appendix algorithm "Harmonic Sum
// Decimation").  Decimating a power series by h sums h adjacent,
// non-overlapping bins, D_h[r] = P[h r] + ... + P[h r + h - 1]; stage H adds
// D_1 .. D_H aligned at bin 0 over their common length floor(n / H):
//   S_H[r] = S_{H-1}[r] + D_H[r],   S_1 = P,
// chi-square with H(H+1) degrees of freedom under the noise model.  One
// thread per r builds every stage that has bin r, so each stage's output is
// written with unit stride and the h-bin groups a warp reads are contiguous.
#include "internal.hpp"

namespace pulscan {

constexpr int kHarmThreads = 256;

__global__ __launch_bounds__(kHarmThreads) void harmonic_kernel(const HarmJob *__restrict__ jobs,
                                                                HarmJob single) {
  const HarmJob jb = jobs ? jobs[blockIdx.y] : single;
  const uint64_t stride = (uint64_t)gridDim.x * kHarmThreads;
  for (uint64_t r = (uint64_t)blockIdx.x * kHarmThreads + threadIdx.x; r < jb.n / 2; r += stride) {
    float s = jb.P[r];
    uint64_t off = 0;
    for (uint32_t H = 2; H <= jb.numharm; ++H) {
      const uint64_t m = jb.n / H;
      if (r >= m) break;
      const float *g = jb.P + (uint64_t)H * r;
      float d = g[0];
      for (uint32_t j = 1; j < H; ++j) d += g[j];
      s += d;
      jb.S[off + r] = s;
      off += m;
    }
  }
}

hipError_t launch_harmonics(const HarmJob *jobs_dev, const HarmJob &single, int njobs,
                            uint32_t n_max, hipStream_t stream) {
  const uint64_t work = n_max / 2;
  uint64_t blocks = (work + kHarmThreads - 1) / kHarmThreads;
  if (blocks > 4096) blocks = 4096;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(harmonic_kernel, dim3((uint32_t)blocks, njobs), dim3(kHarmThreads), 0, stream,
                     jobs_dev, single);
  return hipGetLastError();
}

}  // namespace pulscan

// The fused boxcar-bank kernel: one pass over each tile of a spectrum does
// normalisation, power, the boxcar bank of every width and the per-chunk
// maxima with the threshold test.
//
//  * Normalisation (section 2.2.3; section 2.5 and the appendix algorithm
//    "Median of Medians Normalisation"): one wave per block of B = 64*EPL bins.
//    Lane l holds elements l + 64m, so the first levels of the median-of-4
//    tree (strides B/4, B/16, ... down to 64) stay inside a lane and the last
//    three (16, 4, 1 lanes) use cross-lane moves (permlane swaps and DPP row
//    shifts).  The real and imaginary trees run interleaved.
//  * Power (section 2.2.3): re'^2 + im'^2, written to LDS only.  The tile
//    holds its T bins plus a halo of up to zmax - 1 bins from the next blocks
//    (normalised with those blocks' own statistics).
//  * Bank (section 2.2.5): each lane owns K consecutive window starts.  A
//    running upper bound first finds the first width block in which any of
//    the wave's windows could reach its threshold (powers are non-negative,
//    so a lane's union window bounds all its windows); a wave that cannot
//    reach any threshold is done.  Otherwise the wave runs the exact
//    recursion Y_w = Y_{w-1} + P[i+w-1] in registers from width 1, testing
//    the thresholds from that block on.  Both routes give the same result.
//  * Per-chunk maxima (appendix algorithm "Boxcar Filtering Process"): a lane
//    compares the maximum of its K sums with the width's threshold; when it
//    reaches it, the lane finds its first bin attaining that maximum and
//    merges (power, bin) into the chunk's LDS slot for the width with one
//    64-bit atomic max (larger power wins, then the smaller bin).  Without a
//    threshold (tables mode) every maximum is merged.
//  * Extraction: the tile's non-empty slots are compacted in (chunk, width)
//    order into one run of the staging pool (ballot + popcount ranks).
#include <float.h>

#include "internal.hpp"

namespace pulscan {

// Row pitch (floats) of the power tile for K bins per lane: the 64 lane
// columns plus 64/K pad words, so that the bank's reads (64 consecutive
// words of a row) and the normalisation's writes (lane l -> row l % K,
// column l / K) both fall on distinct banks.
template <int K>
__host__ __device__ constexpr int pitch_of() {
  return K == 1 ? 64 : 64 + 64 / K;
}

// Twice the median of four values: the two middle values of four are
// max(min(a,b), min(c,d)) and min(max(a,b), max(c,d)).  Carrying the factor
// 2 through the tree and removing it with one exact power-of-two scale at the
// end rounds exactly as halving at every level would.
__device__ __forceinline__ float m4x2(float a, float b, float c, float d) {
  return fmaxf(fminf(a, b), fminf(c, d)) + fminf(fmaxf(a, b), fmaxf(c, d));
}

template <int CTRL>
__device__ __forceinline__ float dpp_row(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}
constexpr int kRowShl1 = 0x101, kRowShl2 = 0x102, kRowShl3 = 0x103;
constexpr int kRowShl4 = 0x104, kRowShl8 = 0x108, kRowShl12 = 0x10C;

// Lane l (l < 16 in each half-wave) receives lane l + 16's value.
__device__ __forceinline__ float from_plus16(float x) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false,
                                                  false);
  return __uint_as_float(r[1]);
}
// Lane l (l < 32) receives lane l + 32's value.
__device__ __forceinline__ float from_plus32(float x) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false,
                                                  false);
  return __uint_as_float(r[1]);
}

template <int EPL>
constexpr int log4_of() {
  return EPL == 1 ? 0 : EPL == 4 ? 1 : EPL == 16 ? 2 : 3;
}

// Medians of medians of two sets of 64*EPL values of one wave (lane l holds
// element l + 64m of each in a[m], b[m]); a and b are consumed.  The results
// are wave-uniform.
template <int EPL>
__device__ __forceinline__ void wave_mom2(float (&a)[EPL], float (&b)[EPL], float &ra, float &rb) {
#pragma unroll
  for (int cnt = EPL; cnt >= 4; cnt /= 4) {
    const int q = cnt / 4;
#pragma unroll
    for (int m = 0; m < q; ++m) {
      a[m] = m4x2(a[m], a[m + q], a[m + 2 * q], a[m + 3 * q]);
      b[m] = m4x2(b[m], b[m + q], b[m + 2 * q], b[m + 3 * q]);
    }
  }
  float x = a[0], y = b[0];
  {  // stride 16 lanes: lane l < 16 combines lanes l, l+16, l+32, l+48
    const float x1 = from_plus16(x), y1 = from_plus16(y);
    const float x2 = from_plus32(x), y2 = from_plus32(y);
    const float x3 = from_plus32(x1), y3 = from_plus32(y1);
    x = m4x2(x, x1, x2, x3);
    y = m4x2(y, y1, y2, y3);
  }
  // stride 4 lanes, then 1, inside each row of 16
  x = m4x2(x, dpp_row<kRowShl4>(x), dpp_row<kRowShl8>(x), dpp_row<kRowShl12>(x));
  y = m4x2(y, dpp_row<kRowShl4>(y), dpp_row<kRowShl8>(y), dpp_row<kRowShl12>(y));
  x = m4x2(x, dpp_row<kRowShl1>(x), dpp_row<kRowShl2>(x), dpp_row<kRowShl3>(x));
  y = m4x2(y, dpp_row<kRowShl1>(y), dpp_row<kRowShl2>(y), dpp_row<kRowShl3>(y));
  // every level doubled the value: undo log4(EPL) + 3 doublings exactly
  constexpr float scale = 1.0f / (float)(1 << (log4_of<EPL>() + 3));
  ra = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x))) * scale;
  rb = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(y))) * scale;
}

// The same for one set of values (the trees of blocks of 1024 bins or more
// run one at a time to stay within the register budget of 4 waves per SIMD).
template <int EPL>
__device__ __forceinline__ float wave_mom1(float (&a)[EPL]) {
#pragma unroll
  for (int cnt = EPL; cnt >= 4; cnt /= 4) {
    const int q = cnt / 4;
#pragma unroll
    for (int m = 0; m < q; ++m) a[m] = m4x2(a[m], a[m + q], a[m + 2 * q], a[m + 3 * q]);
  }
  float x = a[0];
  {
    const float x1 = from_plus16(x);
    x = m4x2(x, x1, from_plus32(x), from_plus32(x1));
  }
  x = m4x2(x, dpp_row<kRowShl4>(x), dpp_row<kRowShl8>(x), dpp_row<kRowShl12>(x));
  x = m4x2(x, dpp_row<kRowShl1>(x), dpp_row<kRowShl2>(x), dpp_row<kRowShl3>(x));
  constexpr float scale = 1.0f / (float)(1 << (log4_of<EPL>() + 3));
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x))) * scale;
}

// Order-preserving map of a float to a 32-bit unsigned integer and back.
__device__ __forceinline__ uint32_t ord_f32(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float unord_f32(uint32_t o) {
  const uint32_t u = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
  return __uint_as_float(u);
}

// LDS address of tile-relative bin i.  Bins are grouped in segments of 64*K;
// within a segment, bin L*K + j (lane L, j < K) sits at row j, column L of a
// K-row array, so the 64 lanes of a wave reading "their" j-th bin hit 64
// consecutive words.  Group L of segment g (its K bins) is group g*64 + L.
template <int K>
__device__ __forceinline__ uint32_t paddr(uint32_t i) {
  constexpr uint32_t SEG = 64 * K;
  const uint32_t g = i / SEG, r = i % SEG;
  return g * (K * pitch_of<K>()) + (r % K) * pitch_of<K>() + r / K;
}

template <int K>
__device__ __forceinline__ float max_of(const float (&s)[K]) {
  if constexpr (K == 1) {
    return s[0];
  } else if constexpr (K == 2) {
    return fmaxf(s[0], s[1]);
  } else if constexpr (K == 4) {
    return fmaxf(fmaxf(s[0], s[1]), fmaxf(s[2], s[3]));
  } else if constexpr (K == 8) {
    const float a = fmaxf(fmaxf(s[0], s[1]), s[2]);
    const float b = fmaxf(fmaxf(s[3], s[4]), s[5]);
    return fmaxf(fmaxf(a, b), fmaxf(s[6], s[7]));
  } else {
    const float a = fmaxf(fmaxf(s[0], s[1]), s[2]);
    const float b = fmaxf(fmaxf(s[3], s[4]), s[5]);
    const float c = fmaxf(fmaxf(s[6], s[7]), s[8]);
    const float d = fmaxf(fmaxf(s[9], s[10]), s[11]);
    const float e = fmaxf(fmaxf(s[12], s[13]), s[14]);
    const float f = fmaxf(fmaxf(a, b), c);
    const float g = fmaxf(fmaxf(d, e), s[15]);
    return fmaxf(f, g);
  }
}

// The raw amplitudes of one normalisation block, loaded by one wave.  Lane l
// holds elements l + 64m of the block's statistics window: the block itself,
// or the last B bins of the spectrum for its last, partial block.
template <int EPL>
struct BlockData {
  float re[EPL], im[EPL];
  uint32_t own;  // first bin of block b
  uint32_t s0;   // first bin of its statistics window
  bool last;
};

template <int EPL>
__device__ __forceinline__ void load_block(const float2 *__restrict__ x, uint32_t n, uint32_t b,
                                           uint32_t lane, BlockData<EPL> &bd) {
  constexpr uint32_t B = 64 * EPL;
  bd.own = b * B;
  bd.last = bd.own + B > n;
  bd.s0 = bd.last ? n - B : bd.own;
#pragma unroll
  for (int m = 0; m < EPL; ++m) {
    const float2 v = x[bd.s0 + lane + 64 * m];
    bd.re[m] = v.x;
    bd.im[m] = v.y;
  }
}

// Normalise a loaded block and write its power into the tile's LDS array for
// every bin of the block that the tile needs (tile-relative index below
// `need`).  Executed by one whole wave.
template <int K, int EPL>
__device__ __forceinline__ void normalise_block(BlockData<EPL> &bd, uint32_t b, uint32_t t0,
                                                uint32_t need, uint32_t T, float *Pl,
                                                uint32_t lane, float *P_out, float *stats_out) {
  constexpr uint32_t B = 64 * EPL;
  constexpr int PITCH = pitch_of<K>();
  float(&re)[EPL] = bd.re;
  float(&im)[EPL] = bd.im;
  const uint32_t own = bd.own, s0 = bd.s0;
  float med_re, med_im, mad_re, mad_im;
  if constexpr (EPL >= 16) {
    float w[EPL];
#pragma unroll
    for (int m = 0; m < EPL; ++m) w[m] = re[m];
    med_re = wave_mom1<EPL>(w);
#pragma unroll
    for (int m = 0; m < EPL; ++m) w[m] = im[m];
    med_im = wave_mom1<EPL>(w);
#pragma unroll
    for (int m = 0; m < EPL; ++m) w[m] = fabsf(re[m] - med_re);
    mad_re = wave_mom1<EPL>(w);
#pragma unroll
    for (int m = 0; m < EPL; ++m) w[m] = fabsf(im[m] - med_im);
    mad_im = wave_mom1<EPL>(w);
  } else {
    float wa[EPL], wb[EPL];
#pragma unroll
    for (int m = 0; m < EPL; ++m) {
      wa[m] = re[m];
      wb[m] = im[m];
    }
    wave_mom2<EPL>(wa, wb, med_re, med_im);
#pragma unroll
    for (int m = 0; m < EPL; ++m) {
      wa[m] = fabsf(re[m] - med_re);
      wb[m] = fabsf(im[m] - med_im);
    }
    wave_mom2<EPL>(wa, wb, mad_re, mad_im);
  }
  const float inv_re = mad_re > 0.f ? 1.0f / (mad_re * kMadScale) : 0.f;
  const float inv_im = mad_im > 0.f ? 1.0f / (mad_im * kMadScale) : 0.f;
  const float off_re = -med_re * inv_re, off_im = -med_im * inv_im;
  if ((EPL % K) == 0 && !bd.last && own + B - t0 <= need && !P_out) {
    // whole block needed and aligned to the segments: addresses are a lane
    // base plus compile-time offsets
    const uint32_t c0 = (own - t0) / 64;
    const uint32_t base = (c0 / K) * (K * PITCH) + (lane % K) * PITCH + lane / K;
#pragma unroll
    for (int m = 0; m < EPL; ++m) {
      const float a = fmaf(re[m], inv_re, off_re);
      const float c = fmaf(im[m], inv_im, off_im);
      Pl[base + (m / K) * (K * PITCH) + (64 / K) * (m % K)] = fmaf(a, a, c * c);
    }
  } else {
#pragma unroll
    for (int m = 0; m < EPL; ++m) {
      const uint32_t t = s0 + lane + 64 * m;
      if (t >= own && t - t0 < need) {
        const float a = fmaf(re[m], inv_re, off_re);
        const float c = fmaf(im[m], inv_im, off_im);
        const float P = fmaf(a, a, c * c);
        Pl[paddr<K>(t - t0)] = P;
        if (P_out && t - t0 < T) P_out[t] = P;
      }
    }
  }
  if (stats_out && lane == 0 && own >= t0 && own < t0 + T) {
    stats_out[4 * (size_t)b + 0] = med_re;
    stats_out[4 * (size_t)b + 1] = mad_re;
    stats_out[4 * (size_t)b + 2] = med_im;
    stats_out[4 * (size_t)b + 3] = mad_im;
  }
}

// A wave-uniform pointer in the constant address space: loads through it
// with uniform indices become scalar loads into SGPRs.
typedef __attribute__((address_space(4))) const float *const_fptr;
__device__ __forceinline__ const_fptr uniform_const(const float *p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (const_fptr)(((uint64_t)hi << 32) | lo);
}

// The exact bank over one segment of 64*K window starts (segment g of the
// tile), lane l owning starts g*64K + l*K .. +K-1: the running sums of
// section 2.2.5 for every width, and from width block `first` on, the
// per-lane maximum, the threshold test and the merge into the chunk's slot.
template <int K>
__device__ __forceinline__ void bank_dense(const float *__restrict__ Pl, uint32_t g, uint32_t lane,
                                           const_fptr thr, uint32_t zmax, uint32_t zc,
                                           uint32_t first, unsigned long long *slot_row,
                                           uint32_t bin0) {
  constexpr int PITCH = pitch_of<K>();
  float s[K], q[2 * K];
#pragma unroll
  for (int k = 0; k < K; ++k) s[k] = 0.f;
  {
    const float *bp = Pl + g * (K * PITCH) + lane;
#pragma unroll
    for (int v = 0; v < K; ++v) q[v] = bp[v * PITCH];
  }
  for (uint32_t wb = 0; wb < zc; wb += K) {
    // q[j] = P[start + wb + j], j < 2K: fetch the upper half
    {
      const uint32_t L = lane + wb / K + 1;
      const float *bp = Pl + (g + (L >> 6)) * (K * PITCH) + (L & 63);
#pragma unroll
      for (int v = 0; v < K; ++v) q[K + v] = bp[v * PITCH];
    }
    if (wb < first * K) {
      // widths below the first block that can reach a threshold: sums only
#pragma unroll
      for (int u = 0; u < K; ++u)
#pragma unroll
        for (int k = 0; k < K; ++k) s[k] += q[k + u];
    } else {
      float Tv[K];  // this block's thresholds (scalar loads)
#pragma unroll
      for (int u = 0; u < K; ++u) Tv[u] = thr[wb + u];
#pragma unroll
      for (int u = 0; u < K; ++u) {
#pragma unroll
        for (int k = 0; k < K; ++k) s[k] += q[k + u];  // width wb+u+1
        const float m = max_of<K>(s);
        if (m >= Tv[u]) {
          const uint32_t w = wb + u + 1;
          if (w <= zmax) {
            uint32_t kk = K - 1;
#pragma unroll
            for (int k = K - 2; k >= 0; --k) kk = (s[k] == m) ? (uint32_t)k : kk;
            const unsigned long long key =
                ((unsigned long long)ord_f32(m) << 32) | (0xFFFFFFFFu - (bin0 + kk));
            atomicMax(&slot_row[w - 1], key);
          }
        }
      }
    }
#pragma unroll
    for (int v = 0; v < K; ++v) q[v] = q[K + v];
  }
}

// Safety factor of the pruning bound.  A sum of m non-negative FP32 terms,
// in any order, is at least (1 - m u) times the exact sum and a width-w FP32
// boxcar at most (1 + w u) times its exact sum (u = 2^-24); for zmax <= 4096
// the ratio of the two stays above 1 - 2^-10, so comparing a union sum with
// T * (1 - 2^-10) never skips a window whose FP32 boxcar reaches T.
constexpr float kBoundSlack = 1.0f - 1.0f / 1024.0f;
constexpr int kSub = 4;  // widths per bound check inside the first width block

// The first width block in which one of this lane's windows might reach its
// threshold, or `nblk` if none can.  Powers are non-negative, so every window
// of width <= w starting at one of the lane's K starts lies in the lane's
// first w + K - 1 bins, whose sum bounds them all.  The first block (widths
// 1..K, the lowest thresholds) is checked every kSub widths from the powers
// themselves; later blocks add one K-bin group sum per block.
// CLAMP: the tile holds -inf past the end of the spectrum; count those as 0.
template <int K, bool CLAMP>
__device__ __forceinline__ uint32_t bound_lane(const float *__restrict__ Pl,
                                               const float *__restrict__ Sg, uint32_t g,
                                               uint32_t lane, const float *__restrict__ Tb1,
                                               const float *__restrict__ Tb, uint32_t nblk) {
  constexpr int PITCH = pitch_of<K>();
  constexpr int S = K < kSub ? K : kSub;
  float q[2 * K];
  {
    const float *bp = Pl + g * (K * PITCH) + lane;
#pragma unroll
    for (int v = 0; v < K; ++v) q[v] = bp[v * PITCH];
    const uint32_t L = lane + 1;
    const float *bq = Pl + (g + (L >> 6)) * (K * PITCH) + (L & 63);
#pragma unroll
    for (int v = 0; v < K - 1; ++v) q[K + v] = bq[v * PITCH];
  }
  if (CLAMP) {
#pragma unroll
    for (int j = 0; j < 2 * K - 1; ++j) q[j] = fmaxf(q[j], 0.f);
  }
  float U = 0.f;
#pragma unroll
  for (int j = 0; j < K - 1; ++j) U += q[j];
  bool hit = false;
#pragma unroll
  for (int u = 0; u < K; ++u) {
    U += q[K - 1 + u];
    if ((u + 1) % S == 0) hit = hit || (U >= Tb1[u / S]);
  }
  uint32_t fl = hit ? 0u : nblk;
  const uint32_t own = g * 64 + lane;
  U = Sg[own] + Sg[own + 1];
  for (uint32_t b = 1; b < nblk; ++b) {
    if (__ballot(fl == nblk) == 0ull) break;  // every lane already flagged
    U += Sg[own + b + 1];
    if (fl == nblk && U >= Tb[b]) fl = b;
  }
  return fl;
}

// Exact evaluation of KF consecutive window starts [st, st + KF) of the tile
// (one work item of the cooperative pass): the running sums of section 2.2.5
// from width 1, with the threshold test from width wfirst + 1 on.  Every
// lane of the wave steps through the same widths; `valid` lanes merge their
// maxima into the slots.
template <int K, int KF>
__device__ __forceinline__ void eval_starts(const float *__restrict__ Pl, uint32_t st, bool valid,
                                            uint32_t wfirst, const_fptr thr, uint32_t zmax,
                                            uint32_t zc, unsigned long long *slot_row,
                                            uint32_t bin0) {
  constexpr int PITCH = pitch_of<K>();
  float s[KF], q[2 * KF];
#pragma unroll
  for (int k = 0; k < KF; ++k) s[k] = 0.f;
  {
    const uint32_t a = paddr<K>(st);  // KF | st and KF | K: the group stays in one column
#pragma unroll
    for (int v = 0; v < KF; ++v) q[v] = Pl[a + v * PITCH];
  }
  for (uint32_t wb = 0; wb < zc; wb += KF) {
    {
      const uint32_t a = paddr<K>(st + wb + KF);
#pragma unroll
      for (int v = 0; v < KF; ++v) q[KF + v] = Pl[a + v * PITCH];
    }
#pragma unroll
    for (int u = 0; u < KF; ++u) {
#pragma unroll
      for (int k = 0; k < KF; ++k) s[k] += q[k + u];  // width wb+u+1
      const uint32_t w = wb + u + 1;
      const float Tw = thr[wb + u];
      float m = s[0];
#pragma unroll
      for (int k = 1; k < KF; ++k) m = fmaxf(m, s[k]);
      if (valid && w > wfirst && m >= Tw && w <= zmax) {
        uint32_t kk = KF - 1;
#pragma unroll
        for (int k = KF - 2; k >= 0; --k) kk = (s[k] == m) ? (uint32_t)k : kk;
        const unsigned long long key =
            ((unsigned long long)ord_f32(m) << 32) | (0xFFFFFFFFu - (bin0 + kk));
        atomicMax(&slot_row[w - 1], key);
      }
    }
#pragma unroll
    for (int v = 0; v < KF; ++v) q[v] = q[KF + v];
  }
}

template <int EPL>
constexpr int threads_for() {
  return EPL >= 64 ? 256 : kMaxThreads;  // 4096-bin blocks need the whole register file
}
// Waves per SIMD the register allocation must allow: 4 lets two 8-wave
// workgroups share a CU.
template <int EPL>
constexpr int waves_per_eu_for() {
  return EPL >= 64 ? 1 : 4;
}

template <int K, int EPL>
__global__ __launch_bounds__(threads_for<EPL>(), waves_per_eu_for<EPL>()) void bank_kernel(
    BankParams p) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ uint32_t wave_sum[kMaxThreads / 64];
  __shared__ uint32_t tile_base;
  __shared__ uint32_t any_dense;
  __shared__ uint32_t n_items;
  constexpr uint32_t SEG = 64 * K;
  constexpr uint32_t B = 64 * EPL;
  constexpr int PITCH = pitch_of<K>();
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t nw = blockDim.x >> 6, nthr = blockDim.x;
  const uint32_t T = p.tile, C = p.chunk;
  const uint32_t chunks_per_tile = T / C;
  // LDS: slots (chunks_per_tile x zmax_max, 64-bit) | thresholds (zc_max) |
  // first-block bound thresholds (4) | per-block bound thresholds |
  // K-bin group sums | power tile
  unsigned long long *slots = reinterpret_cast<unsigned long long *>(lds_raw);
  float *Tl = reinterpret_cast<float *>(slots + (size_t)chunks_per_tile * p.zmax_max);
  float *Tb1 = Tl + p.zc_max_pad;
  float *Tb = Tb1 + 4;
  float *Sg = Tb + p.zc_max_pad / K + 4;
  uint32_t *items = reinterpret_cast<uint32_t *>(Sg + p.nseg_lds * 64);  // T / K entries
  float *Pl = reinterpret_cast<float *>(items + T / K);

  // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a
  // contiguous run of tiles so the halo a tile shares with its neighbour is
  // read through the same L2.
  uint64_t first_tile = blockIdx.x;
  if ((gridDim.x & 7) == 0) first_tile = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);

  for (uint64_t tg = first_tile; tg < p.total_tiles; tg += gridDim.x) {
    int sidx = 0;
    if (p.nspec > 1) {
      int lo = 0, hi = p.nspec - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (p.descs[mid].tile_begin <= tg)
          lo = mid;
        else
          hi = mid - 1;
      }
      sidx = lo;
    }
    const SpecDesc d = p.nspec > 1 ? p.descs[sidx] : p.single;
    const uint32_t t0 = (uint32_t)(tg - d.tile_begin) * T;
    const uint32_t n = d.n, zmax = d.zmax, zc = d.zc;
    const uint32_t rem = n - t0;
    const uint32_t need = min(T + zmax - 1, rem);
    const uint32_t nblk = zc / K;
    const uint32_t span = T + zc;  // tile bins the bank and the bound read
    const uint32_t bfirst = t0 / B, blast = (t0 + need - 1) / B;

    // --- set-up and power --------------------------------------------------
    // the wave's first block is requested before anything else so that its
    // memory latency overlaps the set-up
    BlockData<EPL> bd;
    const bool have = !p.from_power && bfirst + wave <= blast;
    if (have) load_block<EPL>(d.x, n, bfirst + wave, lane, bd);
    if (threadIdx.x == 0) {
      any_dense = 0u;
      n_items = 0u;
    }
    for (uint32_t i = threadIdx.x; i < chunks_per_tile * zmax; i += nthr) slots[i] = 0ull;
    for (uint32_t i = threadIdx.x; i < zc; i += nthr) Tl[i] = d.thr[i];
    if (threadIdx.x < 4) {
      constexpr int S = K < kSub ? K : kSub;
      float m = INFINITY;
      if (threadIdx.x * S < (uint32_t)K)
        for (int u = 0; u < S; ++u) m = fminf(m, d.thr[threadIdx.x * S + u]);
      Tb1[threadIdx.x] = m * kBoundSlack;
    }
    for (uint32_t i = threadIdx.x; i < nblk; i += nthr) {
      float m = d.thr[i * K];
      for (int u = 1; u < K; ++u) m = fminf(m, d.thr[i * K + u]);
      Tb[i] = m * kBoundSlack;
    }
    // bins past the spectrum's end are -inf (no window may contain them);
    // halo bins beyond what any width <= zmax reads are 0 (read only by the
    // unrecorded widths zmax+1..zc and by the pruning bound)
    for (uint32_t i = need + threadIdx.x; i < span; i += nthr)
      Pl[paddr<K>(i)] = i < rem ? 0.f : -INFINITY;
    if (p.from_power) {
      const float *pw = reinterpret_cast<const float *>(d.x);
      for (uint32_t i = threadIdx.x; i < need; i += nthr) Pl[paddr<K>(i)] = pw[t0 + i];
    } else if (have) {
      const bool dbg = p.mode == kModeTables;
      float *po = dbg ? p.P_out : nullptr;
      float *so = dbg ? p.stats_out : nullptr;
      normalise_block<K, EPL>(bd, bfirst + wave, t0, need, T, Pl, lane, po, so);
      for (uint32_t b = bfirst + wave + nw; b <= blast; b += nw) {
        load_block<EPL>(d.x, n, b, lane, bd);
        normalise_block<K, EPL>(bd, b, t0, need, T, Pl, lane, po, so);
      }
    }
    __syncthreads();

    // --- bank ----------------------------------------------------------------
    const bool prune = !p.dense && p.mode != kModeTables;
    const bool clamp = rem < span;
    if (prune) {
      // K-bin group sums of the whole span (inputs of the pruning bound)
      const uint32_t ngroups = span / K;
      for (uint32_t j = threadIdx.x; j < ngroups; j += nthr) {
        const float *cp = Pl + (j >> 6) * (K * PITCH) + (j & 63);
        float a = 0.f;
        if (clamp) {
#pragma unroll
          for (int v = 0; v < K; ++v) a += fmaxf(cp[v * PITCH], 0.f);
        } else {
#pragma unroll
          for (int v = 0; v < K; ++v) a += cp[v * PITCH];
        }
        Sg[j] = a;
      }
      __syncthreads();
    }
    const uint32_t nseg_tile = T / SEG;
    const const_fptr thr = uniform_const(d.thr);
    if (prune) {
      // each lane's first width block that might reach a threshold; the
      // flagged lanes become work items of a cooperative exact pass
      for (uint32_t g = wave; g < nseg_tile; g += nw) {
        if (g * SEG >= rem) break;
        const uint32_t fl = clamp ? bound_lane<K, true>(Pl, Sg, g, lane, Tb1, Tb, nblk)
                                  : bound_lane<K, false>(Pl, Sg, g, lane, Tb1, Tb, nblk);
        const unsigned long long mask = __ballot(fl < nblk);
        if (mask) {
          uint32_t base = 0;
          if (lane == 0) base = atomicAdd(&n_items, (uint32_t)__popcll(mask));
          base = __shfl(base, 0, 64);
          if (fl < nblk)
            items[base + __popcll(mask & ((1ull << lane) - 1ull))] = ((g * 64 + lane) << 12) | fl;
        }
      }
      __syncthreads();
      constexpr int KF = K < 4 ? K : 4;
      const uint32_t nsub = n_items * (K / KF);
      if (threadIdx.x == 0 && nsub) any_dense = 1u;
      for (uint32_t r = 0; r < nsub; r += nthr) {
        const uint32_t j = r + threadIdx.x;
        const bool valid = j < nsub;
        const uint32_t it = valid ? items[j / (K / KF)] : 0u;
        const uint32_t st = (it >> 12) * K + (j % (K / KF)) * KF;  // tile-relative first start
        const uint32_t wfirst = (it & 0xFFFu) * K;
        eval_starts<K, KF>(Pl, valid ? st : 0u, valid, wfirst, thr, zmax, zc,
                           slots + (size_t)((valid ? st : 0u) / C) * zmax, t0 + st);
      }
    } else {
      for (uint32_t g = wave; g < nseg_tile; g += nw) {
        const uint32_t seg0 = g * SEG;
        if (seg0 >= rem) break;
        any_dense = 1u;
        bank_dense<K>(Pl, g, lane, thr, zmax, zc, 0u, slots + (size_t)(seg0 / C) * zmax,
                      t0 + seg0 + lane * K);
      }
    }
    __syncthreads();

    // --- extraction ----------------------------------------------------------
    const uint32_t chunk0 = t0 / C;
    const uint32_t nch = min(chunks_per_tile, d.nchunks - chunk0);
    const uint32_t nsl = nch * zmax;
    if (p.mode == kModeSearch && !any_dense) {
      // no wave evaluated a width block: no slot can hold a maximum
      if (threadIdx.x == 0) {
        p.tile_count[tg] = 0u;
        p.tile_pos[tg] = 0u;
      }
    } else if (p.mode == kModeSearch) {
      // stage the tile's maxima in slot order, i.e. (chunk, width) order:
      // count, reserve one run of the pool, then write with ordered ranks
      uint32_t mine = 0;
      for (uint32_t i = threadIdx.x; i < nsl; i += nthr) mine += slots[i] != 0ull ? 1u : 0u;
      for (int o = 32; o >= 1; o >>= 1) mine += __shfl_xor(mine, o, 64);
      if (lane == 0) wave_sum[wave] = mine;
      __syncthreads();
      if (threadIdx.x == 0) {
        uint32_t tot = 0;
        for (uint32_t v = 0; v < nw; ++v) tot += wave_sum[v];
        const uint32_t base = tot ? atomicAdd(p.pool_head, tot) : 0u;
        p.tile_count[tg] = tot;
        p.tile_pos[tg] = base;
        tile_base = base;
      }
      __syncthreads();
      uint32_t run = tile_base;
      for (uint32_t r = 0; r < nsl; r += nthr) {
        const uint32_t i = r + threadIdx.x;
        const unsigned long long key = i < nsl ? slots[i] : 0ull;
        const bool valid = key != 0ull;
        const unsigned long long mask = __ballot(valid);
        if (lane == 0) wave_sum[wave] = (uint32_t)__popcll(mask);
        __syncthreads();
        uint32_t before = 0, all = 0;
        for (uint32_t v = 0; v < nw; ++v) {
          before += v < wave ? wave_sum[v] : 0u;
          all += wave_sum[v];
        }
        if (valid) {
          const uint32_t pos = run + before + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
          if (pos < p.pool_cap) {
            const uint32_t cl = i / zmax, w = i - cl * zmax + 1;
            StageEntry e;
            e.chunk = chunk0 + cl;
            e.bin = 0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull);
            e.power = unord_f32((uint32_t)(key >> 32));
            e.width = w;
            p.pool[pos] = e;
          }
        }
        run += all;
        __syncthreads();
      }
    } else {
      for (uint32_t i = threadIdx.x; i < nsl; i += nthr) {
        const unsigned long long key = slots[i];
        const size_t o = (size_t)chunk0 * zmax + i;
        p.M[o] = key ? unord_f32((uint32_t)(key >> 32)) : -INFINITY;
        p.I[o] = key ? 0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull) : 0xFFFFFFFFu;
      }
    }
    __syncthreads();
  }
}

template <int K>
static size_t lds_need_k(uint32_t T, uint32_t C, uint32_t zmax_max, uint32_t *nseg,
                         uint32_t *zc_pad) {
  const uint32_t zc = round_widths(zmax_max, K);
  const uint32_t segb = 64u * (uint32_t)K;
  *nseg = (T + zc + segb - 1) / segb;
  *zc_pad = (zc + 3) / 4 * 4;
  return (size_t)(T / C) * zmax_max * 8u              // slots
         + (size_t)(*zc_pad) * 4u                     // thresholds
         + (4 + (size_t)(*zc_pad) / K + 4) * 4u       // bound thresholds
         + (size_t)(*nseg) * 64u * 4u                 // group sums
         + (size_t)(T / K) * 4u                       // cooperative work items
         + (size_t)(*nseg) * K * pitch_of<K>() * 4u;  // power tile
}

static size_t lds_need(int K, uint32_t T, uint32_t C, uint32_t zmax_max, uint32_t *nseg,
                       uint32_t *zc_pad) {
  switch (K) {
    case 1: return lds_need_k<1>(T, C, zmax_max, nseg, zc_pad);
    case 2: return lds_need_k<2>(T, C, zmax_max, nseg, zc_pad);
    case 4: return lds_need_k<4>(T, C, zmax_max, nseg, zc_pad);
    case 8: return lds_need_k<8>(T, C, zmax_max, nseg, zc_pad);
    default: return lds_need_k<16>(T, C, zmax_max, nseg, zc_pad);
  }
}

static uint64_t gcd_u(uint64_t a, uint64_t b) {
  while (b) {
    const uint64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}
static uint64_t lcm_u(uint64_t a, uint64_t b) { return a / gcd_u(a, b) * b; }

constexpr size_t kLdsBudget = 64 * 1024;
constexpr uint32_t kMaxWaves = 8;

bool choose_geometry(uint32_t C, uint32_t B, uint32_t zmax_max, uint64_t n_hint, Geometry *g) {
  if (C == 0 || C % 64 != 0 || C > (uint32_t)kMaxTile) return false;
  if (B != 64 && B != 256 && B != 1024 && B != 4096) return false;
  if (zmax_max == 0 || zmax_max > 4096) return false;
  int K = 16;
  while (K > 1 && (C / 64) % (uint32_t)K != 0) K /= 2;
  const uint64_t L0 = lcm_u(lcm_u(C, B), 64ull * K);
  if (L0 > (uint64_t)kMaxTile) return false;
  const uint32_t halo = (zmax_max - 1 + B - 1) / B;  // blocks beyond the tile
  const uint32_t wmax = B == 4096 ? 4u : kMaxWaves;
  uint32_t nseg = 0, zcp = 0;
  // largest tile (a multiple of L0) whose blocks plus halo blocks give every
  // wave one block, that fits in LDS and leaves enough tiles to fill the GPU
  uint64_t T = 0;
  for (uint64_t t = L0; t <= (uint64_t)kMaxTile; t += L0) {
    if (t / B + halo > wmax && t > L0) break;
    if (lds_need(K, (uint32_t)t, C, zmax_max, &nseg, &zcp) > kLdsBudget) break;
    if (t > L0 && n_hint / t < 256) break;
    T = t;
  }
  if (T == 0) return false;
  g->K = K;
  g->EPL = (int)(B / 64);
  uint32_t nw = (uint32_t)(T / B) + halo;
  g->waves = (int)(nw < 1 ? 1 : (nw > wmax ? wmax : nw));
  g->tile = (uint32_t)T;
  g->lds_bytes = lds_need(K, g->tile, C, zmax_max, &nseg, &zcp);
  g->nseg_lds = nseg;
  g->zc_max_pad = zcp;
  return true;
}

template <int K>
static hipError_t launch_k(int EPL, uint64_t grid, uint32_t threads, size_t lds,
                           const BankParams &p, hipStream_t stream) {
  switch (EPL) {
    case 1:
      hipLaunchKernelGGL((bank_kernel<K, 1>), dim3((uint32_t)grid), dim3(threads), lds, stream, p);
      break;
    case 4:
      hipLaunchKernelGGL((bank_kernel<K, 4>), dim3((uint32_t)grid), dim3(threads), lds, stream, p);
      break;
    case 16:
      hipLaunchKernelGGL((bank_kernel<K, 16>), dim3((uint32_t)grid), dim3(threads), lds, stream, p);
      break;
    case 64:
      hipLaunchKernelGGL((bank_kernel<K, 64>), dim3((uint32_t)grid), dim3(threads), lds, stream, p);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_bank(const Geometry &g, const BankParams &p, uint64_t grid, hipStream_t stream) {
  if (grid == 0) return hipSuccess;
  const uint32_t threads = 64u * (uint32_t)g.waves;
  switch (g.K) {
    case 1: return launch_k<1>(g.EPL, grid, threads, g.lds_bytes, p, stream);
    case 2: return launch_k<2>(g.EPL, grid, threads, g.lds_bytes, p, stream);
    case 4: return launch_k<4>(g.EPL, grid, threads, g.lds_bytes, p, stream);
    case 8: return launch_k<8>(g.EPL, grid, threads, g.lds_bytes, p, stream);
    case 16: return launch_k<16>(g.EPL, grid, threads, g.lds_bytes, p, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pulscan

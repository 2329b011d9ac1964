// The streaming bank kernel: persistent workgroups, each taking contiguous
// ranges of normalisation blocks, do normalisation, power, the boxcar bank of
// every width, the per-chunk maxima with the threshold test and the staging
// of the candidates, reading every bin of a range from HBM once.
//
//  * Ranges.  A launch is cut into nseg ranges.  Workgroup w takes range w,
//    then the next range that no workgroup has taken (a counter in global
//    memory), so that the workgroups a batch's series slow down (a larger
//    zmax, a tone's flagged lanes, a busier CU) take fewer ranges and every
//    workgroup ends within about one range of the others; the ranges shrink
//    along the launch, so that the last ones taken are short.  Launches
//    below about 67 M bins use one equal range per workgroup.
//  * Streaming.  A workgroup's range (a run of blocks of one or more series)
//    is taken a batch of kStreamBatch blocks at a time, one block per wave.
//    The next batch's loads are in flight (in registers) while the current
//    one is normalised and searched, and the one after is requested as soon
//    as a batch has been normalised (batch 1 only once batch 0 is in).
//    Every issue is the same number of unconditional loads, so that the
//    compiler's wait counts never hold one batch for the next.  Normalised
//    power goes to an LDS ring of blocks; a tile of blocks is searched once
//    the ring holds every bin its windows reach (zmax - 1 bins past its end,
//    `lag` blocks).
//  * Halo.  The windows of a range's last tile reach into the next range,
//    which another workgroup normalises.  That workgroup publishes the four
//    statistics of its first `lag` blocks as soon as it has them; the
//    neighbour then reads only the bins its windows need and normalises them
//    with those statistics (the same arithmetic, so the same bits).  A word
//    that does not arrive in time is recomputed from the block itself; with
//    several ranges per workgroup, neighbouring ranges run at unrelated
//    times and each range normalises its halo blocks itself.
//  * Normalisation (section 2.2.3; section 2.5 and the appendix algorithm
//    "Median of Medians Normalisation"): lane l of a wave holds elements
//    l + 64m of its block, so the first levels of the median-of-4 tree stay
//    in the lane and the last three cross lanes.  The cross-lane levels of
//    the real and imaginary trees run through one set of lane permutations
//    and DPP min/max operations.
//  * Bank (section 2.2.5, appendix algorithm "Boxcar Filtering Process"): as
//    in the tiled kernel, a per-lane upper bound on K starts' windows finds
//    the first width block that might reach a threshold.  Flagged lanes are
//    evaluated exactly, width-parallel, in units of 64 widths shared by the
//    waves (exact_unit), in the canonical FP32 order that the dense route
//    (eval_unit over every lane) also follows, so the two agree bit for bit.
//  * Staging: each tile's (chunk, width) maxima that reach their thresholds
//    are staged in order with their rank in the workgroup's range; the last
//    workgroup scans the ranges' counts.
//
// This translation unit is built without NaN semantics (inputs are finite;
// bins past a series' end are -inf), which lets the compiler fold the
// cross-lane moves into DPP min/max instructions.
#include <float.h>

#include "internal.hpp"
#include "mom.hpp"

namespace pulscan {

#define GAS __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ GAS T *gp(T *p) {
  return (GAS T *)p;
}
typedef float f32x2 __attribute__((ext_vector_type(2)));

// Row pitch (floats) of a ring segment of 64 K-bin groups: the 64 lane
// columns plus 64/K pad words, so that 64 lanes reading "their" j-th bin and
// the normalising wave's writes both fall on distinct banks (or two-way).
template <int K>
__host__ __device__ constexpr int spitch() {
  return 64 + 64 / K;
}
// Starts one exact-pass unit evaluates together (four: the unit's working
// set stays small beside the batch of loads in flight).
template <int K>
__host__ __device__ constexpr int sks() {
  return K < 4 ? K : 4;
}
// Width blocks per step of the bound.
constexpr int kSBoundBatch = 8;
// Safety factor of the pruning bound (see the tiled kernel): a union sum of
// non-negative FP32 terms compared with T (1 - 2^-10) never skips a window
// whose FP32 boxcar reaches T, for zmax <= 4096.
constexpr float kSBoundSlack = 1.0f - 1.0f / 1024.0f;
// s_waitcnt operand of "vmcnt(0)" on gfx9-family parts (vmcnt in bits 3:0
// and 15:14, expcnt 6:4 and lgkmcnt 11:8 left at their maxima)
constexpr int kWaitVm0 = 0x0F70;

// ---------------------------------------------------------------------------
// Median of medians: block_stats (mom.hpp)

// Normalised power (section 2.2.3): each component less its block's median,
// divided by its scaled MAD (0 when the MAD is 0), squared and summed.  The
// tiled kernel evaluates it in the same operations, x / s - med / s as one
// fused multiply-add, so the two kernels give the same power bit for bit.
struct Scales {
  float re, im, off_re, off_im;
};
__device__ __forceinline__ Scales scales_of(const BlockStats &s) {
  Scales c;
  c.re = s.mad_re > 0.f ? 1.0f / (s.mad_re * kMadScale) : 0.f;
  c.im = s.mad_im > 0.f ? 1.0f / (s.mad_im * kMadScale) : 0.f;
  c.off_re = -s.med_re * c.re;
  c.off_im = -s.med_im * c.im;
  return c;
}
__device__ __forceinline__ float power_of(float re, float im, const Scales &c) {
  const float a = fmaf(re, c.re, c.off_re), b = fmaf(im, c.im, c.off_im);
  return fmaf(a, a, b * b);
}

// Order-preserving map of a float to 32 bits and back.
__device__ __forceinline__ uint32_t sord(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float sunord(uint32_t o) {
  return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
}

// A wave-uniform 64-bit value in scalar registers (a division's result is
// computed in vector registers, where it would hold two of them).
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
  return ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32)) << 32) |
         __builtin_amdgcn_readfirstlane((uint32_t)v);
}

// threadIdx.x through an empty asm statement, so that each phase recomputes
// its lane addresses instead of keeping them live across the kernel.
__device__ __forceinline__ uint32_t ftid() {
  uint32_t t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// ---------------------------------------------------------------------------
// LDS views

template <int K>
struct Ring {
  float *P;          // power ring: segments of 64 groups x K bins, lane-major
  float *Sg;         // group sums, per ring group position (+ mirror)
  float *E[3];       // first-group partial sums E(3), E(7), E(15) (+ mirror)
  uint32_t NG;       // groups in the ring
  uint32_t mirror;   // entries repeated past NG
  // power address of bin j of the group at ring position q
  __device__ __forceinline__ float *bin(uint32_t q, uint32_t j) const {
    return P + (q >> 6) * (K * spitch<K>()) + j * spitch<K>() + (q & 63);
  }
  __device__ __forceinline__ uint32_t wrap(uint32_t q) const { return q >= NG ? q - NG : q; }
};

// Group sums of the groups [gi0, gi1) of the block at ring slot `slot`
// (block-relative group indices), each summed from zero in increasing order,
// and the partial sums over their first 3, 7 and 15 bins (the first width
// block's bound).  CLAMP counts -inf (past a series' end) as 0.
template <int K, int EPL, bool CLAMP>
__device__ __forceinline__ void group_sums(const Ring<K> &R, uint32_t slot, uint32_t gi1,
                                           uint32_t lane) {
  constexpr uint32_t GPB = 64 * EPL / K;
  for (uint32_t gi = lane; gi < gi1; gi += 64) {
    const uint32_t q = slot * GPB + gi;
    const float *c = R.bin(q, 0);
    float e = 0.f, e3 = 0.f, e7 = 0.f, e15 = 0.f;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      float v = c[j * spitch<K>()];
      if (CLAMP) v = fmaxf(v, 0.f);
      e = j == 0 ? v : e + v;
      if (j == 2) e3 = e;
      if (j == 6) e7 = e;
      if (j == 14) e15 = e;
    }
    R.Sg[q] = e;
    R.E[0][q] = e3;
    if (K >= 8) R.E[1][q] = e7;
    if (K >= 16) R.E[2][q] = e15;
    if (q < R.mirror) {
      R.Sg[q + R.NG] = e;
      R.E[0][q + R.NG] = e3;
      if (K >= 8) R.E[1][q + R.NG] = e7;
      if (K >= 16) R.E[2][q + R.NG] = e15;
    }
  }
}

// A block's ring slot with no spectrum behind it (past the series' end): the
// first `need` bins are -inf, their groups' sums 0.
template <int K, int EPL>
__device__ __forceinline__ void fill_past_end(const Ring<K> &R, uint32_t slot, uint32_t need,
                                              uint32_t lane) {
  constexpr uint32_t GPB = 64 * EPL / K;
  for (uint32_t r = lane; r < need; r += 64) {
    const uint32_t q = slot * GPB + r / K;
    *R.bin(q, r % K) = -INFINITY;
  }
  for (uint32_t gi = lane; gi < need / K; gi += 64) {
    const uint32_t q = slot * GPB + gi;
    R.Sg[q] = 0.f;
#pragma unroll
    for (int k = 0; k < (K >= 16 ? 3 : K >= 8 ? 2 : 1); ++k) R.E[k][q] = 0.f;
    if (q < R.mirror) {
      R.Sg[q + R.NG] = 0.f;
#pragma unroll
      for (int k = 0; k < (K >= 16 ? 3 : K >= 8 ? 2 : 1); ++k) R.E[k][q + R.NG] = 0.f;
    }
  }
}

__device__ __forceinline__ void lds_wait() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// ---------------------------------------------------------------------------
// Loads.  A block's raw data: lane l element m is bin s0 + l + 64m of the
// block's statistics window (the block, or the series' last B bins for a
// partial last block).  Power input: the block's own bins.

// What the kernel needs of a series descriptor, held by value.
struct Series {
  const float2 *x;
  const float *thr;
  uint64_t block_begin;
  uint32_t n, zmax, zc;
};

template <int EPL, bool FP>
struct Raw {
  f32x2 v[FP ? (EPL + 1) / 2 : EPL];  // power input packs two elements per slot
};

// A wave-uniform value passed through an empty asm statement, so that what
// is derived from it (load addresses, per-element conditions) is computed
// where it is used rather than hoisted out of the loop and kept live.
__device__ __forceinline__ uint32_t fresh_u(uint32_t v) {
  v = __builtin_amdgcn_readfirstlane(v);
  asm volatile("" : "+s"(v));
  return v;
}

// Loads of a block: unconditional, from one base address with immediate
// offsets, so that they stay in flight without branches around them.  A
// spectrum block reads its statistics window (the block, or the series' last
// B bins for a partial last block); a power block reads its own bins, indices
// clamped into the series for a partial last block (those values are never
// used).
template <int EPL, bool FP>
__device__ __forceinline__ void load_block(const Series &d, uint32_t k, Raw<EPL, FP> &r) {
  constexpr uint32_t B = 64 * EPL;
  const uint32_t lane = ftid() & 63;
  const uint32_t own = fresh_u(k * B), n = d.n;
  if constexpr (FP) {
    const GAS float *x = gp(reinterpret_cast<const float *>(d.x));
    if (own + B <= n) {
      const GAS float *xl = x + own + lane;
#pragma unroll
      for (int m = 0; m < EPL; ++m) {
        const float v = xl[64 * m];
        if (m & 1)
          r.v[m / 2].y = v;
        else
          r.v[m / 2].x = v;
      }
    } else {
#pragma unroll
      for (int m = 0; m < EPL; ++m) {
        const float v = x[min(own + lane + 64 * m, n - 1)];
        if (m & 1)
          r.v[m / 2].y = v;
        else
          r.v[m / 2].x = v;
      }
    }
  } else {
    const uint32_t s0 = own + B > n ? n - B : own;
    const GAS f32x2 *xl = gp(reinterpret_cast<const f32x2 *>(d.x)) + s0 + lane;
#pragma unroll
    for (int m = 0; m < EPL; ++m) r.v[m] = xl[64 * m];
  }
}

// The first `need` bins of block k (need a multiple of 64, at least 64): a
// halo block normalised with published statistics.  Unconditional loads,
// elements past `need` re-reading bin need - 1, so that every issue of a
// batch is the same number of loads (the compiler can then wait for one set
// while the next is in flight).  The series' partial last block is loaded
// whole (its statistics window), as the normalisation expects.
template <int EPL, bool FP>
__device__ __forceinline__ void load_prefix(const Series &d, uint32_t k, uint32_t need,
                                            Raw<EPL, FP> &r) {
  constexpr uint32_t B = 64 * EPL;
  const uint32_t own = fresh_u(k * B), n = d.n;
  const bool partial = own + B > n;
  if constexpr (FP) {
    if (partial) {
      load_block<EPL, FP>(d, k, r);
      return;
    }
  }
  const uint32_t s0 = partial ? n - B : own;
  const uint32_t lim = partial ? B : fresh_u(need);
  const uint32_t lane = ftid() & 63;
#pragma unroll
  for (int m = 0; m < EPL; ++m) {
    const uint32_t i = s0 + min(lane + 64u * m, lim - 1u);
    if constexpr (FP) {
      const float v = gp(reinterpret_cast<const float *>(d.x))[i];
      if (m & 1)
        r.v[m / 2].y = v;
      else
        r.v[m / 2].x = v;
    } else {
      r.v[m] = gp(reinterpret_cast<const f32x2 *>(d.x))[i];
    }
  }
}

// Where a block's normalisation results go besides the ring.
struct NormOut {
  float *P_out;       // tables mode: the normalised power (series bins)
  float *stats_out;   // tables mode: 4 floats per block
  unsigned long long *pub;  // non-null: publish the statistics (4 tagged words)
  uint32_t tag;
};

// Normalise block k of series d (raw data in r, loaded by load_block) or, with
// `given`, only its first `limit` bins with the given statistics (raw data
// from load_prefix); write the power of bins [0, limit) of the block into ring
// slot `slot`, -inf for bins past the series' end, and the block's group
// sums.  One whole wave.
template <int K, int EPL, bool FP>
__device__ __forceinline__ void normalise(const Series &d, uint32_t k, Raw<EPL, FP> &r,
                                          bool use_given, const BlockStats &given, uint32_t limit,
                                          const Ring<K> &R, uint32_t slot, const NormOut &o,
                                          uint32_t lane) {
  constexpr uint32_t B = 64 * EPL, SEG = 64 * K, GPB = B / K;
  constexpr int PITCH = spitch<K>();
  const uint32_t own = k * B, n = d.n;
  const bool partial = own + B > n;           // the series' last block, not whole
  const uint32_t s0 = (!FP && partial) ? n - B : own;
  float *base = R.P + slot * (B / SEG) * (K * PITCH);
  float P[EPL];
  if constexpr (FP) {
#pragma unroll
    for (int m = 0; m < EPL; ++m) P[m] = (m & 1) ? r.v[m / 2].y : r.v[m / 2].x;
  } else {
    float re[EPL], im[EPL];
#pragma unroll
    for (int m = 0; m < EPL; ++m) {
      re[m] = r.v[m].x;
      im[m] = r.v[m].y;
    }
    BlockStats st;
    if (use_given) {
      st = given;
    } else {
      st = block_stats<EPL>(re, im, lane);
      if (o.pub && lane < 4) {
        const float v = lane == 0 ? st.med_re : lane == 1 ? st.mad_re : lane == 2 ? st.med_im : st.mad_im;
        __hip_atomic_store(o.pub + lane, ((unsigned long long)o.tag << 32) | __float_as_uint(v),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      if (o.stats_out && lane == 0) {
        GAS float *so = gp(o.stats_out) + 4 * (size_t)k;
        so[0] = st.med_re;
        so[1] = st.mad_re;
        so[2] = st.med_im;
        so[3] = st.mad_im;
      }
    }
    const Scales c = scales_of(st);
#pragma unroll
    for (int m = 0; m < EPL; ++m) P[m] = power_of(re[m], im[m], c);
  }
  if (!partial && s0 == own && limit == B) {
    // a whole block: lane l element m is block bin l + 64m, at row l % K,
    // column l / K + (64/K)(m % K) of segment m / K
    float *lb = base + (lane % K) * PITCH + lane / K;
#pragma unroll
    for (int m = 0; m < EPL; ++m) lb[(m / K) * (K * PITCH) + (64 / K) * (m % K)] = P[m];
    if (o.P_out) {
#pragma unroll
      for (int m = 0; m < EPL; ++m) gp(o.P_out)[own + lane + 64 * m] = P[m];
    }
    lds_wait();
    group_sums<K, EPL, false>(R, slot, GPB, lane);
  } else {
    // a partial block, or the first bins of a halo block (rare): addresses
    // from fresh copies of the lane id and the bounds, so that the compiler
    // does not hoist them into the streaming loop
    const uint32_t ln = ftid() & 63, s0f = fresh_u(s0), ownf = fresh_u(own);
    const uint32_t lim = fresh_u(limit), nf = fresh_u(n);
    float *const bf = R.P + fresh_u(slot * (B / SEG) * (K * PITCH));
#pragma unroll
    for (int m = 0; m < EPL; ++m) {
      const uint32_t t = s0f + ln + 64 * m;
      if (t >= ownf && t - ownf < lim) {
        const uint32_t rr = t - ownf, sg = rr / SEG, rs = rr % SEG;
        bf[sg * (K * PITCH) + (rs % K) * PITCH + rs / K] = t < nf ? P[m] : -INFINITY;
        if (o.P_out && t < nf) gp(o.P_out)[t] = P[m];
      }
    }
    // bins past the end that no element covered
    for (uint32_t rr = (nf > ownf ? nf - ownf : 0) + ln; rr < lim; rr += 64) {
      const uint32_t sg = rr / SEG, rs = rr % SEG;
      bf[sg * (K * PITCH) + (rs % K) * PITCH + rs / K] = -INFINITY;
    }
    lds_wait();
    if (partial)
      group_sums<K, EPL, true>(R, slot, limit / K, lane);
    else
      group_sums<K, EPL, false>(R, slot, limit / K, lane);
  }
}

// ---------------------------------------------------------------------------
// The bank

// First width block in which one of lane L's windows might reach its
// threshold, or nblk if none can (powers are non-negative and thresholds
// rise with the width, so the lane's union window bounds every window of
// width <= (b+1) K from its K starts).  The first block is checked every few
// widths from the lane's group sum plus the next group's partial sums.
template <int K>
__device__ __forceinline__ uint32_t sbound(const Ring<K> &R, uint32_t q, const float *Tb1,
                                           const float *Tb, uint32_t nblk) {
  const float own = R.Sg[q];
  bool hit = own + R.E[0][q + 1] >= Tb1[0];
  if (K >= 8) hit |= own + R.E[1][q + 1] >= Tb1[1];
  if (K >= 16) hit |= own + R.E[2][q + 1] >= Tb1[2];
  float U = own + R.Sg[q + 1];
  bool later = false;
  for (uint32_t b = 1; b < nblk; b += kSBoundBatch) {
    float sg[kSBoundBatch], tb[kSBoundBatch];
#pragma unroll
    for (int k = 0; k < kSBoundBatch; ++k) {
      const uint32_t bb = min(b + k, nblk - 1);
      sg[k] = R.Sg[q + bb + 1];
      tb[k] = Tb[bb];
    }
#pragma unroll
    for (int k = 0; k < kSBoundBatch; ++k) {
      if (b + k < nblk) {
        U += sg[k];
        later |= U >= tb[k];
      }
    }
  }
  if (hit) return 0u;
  if (!later) return nblk;
  // rare: find the first block that passes
  U = own + R.Sg[q + 1];
  for (uint32_t b = 1; b < nblk; ++b) {
    U += R.Sg[q + b + 1];
    if (U >= Tb[b]) return b;
  }
  return nblk;
}

// Exact evaluation of width block b (widths bK+1 .. bK+K) for starts
// K0 .. K0+KS-1 of the lane whose group is at ring position q (series bin
// bin0 = its first start), merging each width's maximum that reaches its
// threshold into the chunk's slot (larger power wins, then the smaller bin).
//
// Canonical FP32 order of a boxcar, the tiled kernel's: a start keeps a
// running pair (hb, t) and each width adds the next bin to t, the window's
// sum being hb + t; when the window reaches the end of a K-bin group, hb
// takes that sum and t restarts from zero.  In closed form, with the window
// [s, s + w) ending at position p = s + w - 1 of the lane's groups:
//   * p < K (inside the lane's own group): the bins s..p summed from zero in
//     increasing order;
//   * otherwise, with the window ending in group g = p / K >= 1 at its
//     e = p % K + 1-th bin:  Y = HB(s, g) + E_g(e),  where HB(s, 1) = H_s
//     sums the own group's bins s..K-1 from zero in increasing order,
//     HB(s, g + 1) = HB(s, g) + Sg(g) adds group g's sum, and E_g(e) sums
//     group g's first e bins from zero in increasing order (a group sum Sg is
//     E_g(K)).
// Both kernels and both routes (dense and pruned) follow this order, so they
// agree bit for bit; any width block can be entered from the group sums
// alone.  (Sums of non-negative terms: every order is within (w - 1) u of
// the exact sum.)
template <int K, int K0>
__device__ __forceinline__ void eval_unit(const Ring<K> &R, uint32_t q, uint32_t b,
                                          const float *Tl, uint32_t zmax,
                                          unsigned long long *slot_row, uint32_t bin0) {
  constexpr int KS = sks<K>();
  constexpr int PITCH = spitch<K>();
  // H_s for s = K0 .. K0+KS-1, each from its own reads of the lane's bins
  // (the barrier keeps one chain's loads in flight at a time)
  const float *po = R.bin(q, 0);
  float H[KS];
#pragma unroll
  for (int k = 0; k < KS; ++k) {
    asm volatile("" ::: "memory");
    float v[K - K0];
#pragma unroll
    for (int j = K0 + k; j < K; ++j) v[j - K0] = po[j * PITCH];
    float h = v[k];
#pragma unroll
    for (int j = K0 + k + 1; j < K; ++j) h = h + v[j - K0];
    H[k] = h;
  }
  // prefix sums of the group after the window-end group's (EB: e = 1 .. K0+KS-1)
  constexpr int NB1 = K0 + KS - 1;
  float EB[NB1 > 0 ? NB1 : 1];
  {
    const float *pb = R.bin(R.wrap(q + b + 1), 0);
#pragma unroll
    for (int j = 0; j < NB1; ++j) {
      const float v = pb[j * PITCH];
      EB[j] = j == 0 ? v : EB[j - 1] + v;
    }
  }
  // each width's maximum over the KS starts, merged into the slot when it
  // reaches the width's threshold (first start attaining it)
  auto merge = [&](int u, const float (&y)[KS]) __attribute__((always_inline)) {
    float m = y[0];
#pragma unroll
    for (int k = 1; k < KS; ++k) m = fmaxf(m, y[k]);
    const uint32_t wi = b * K + u;
    if (m >= Tl[wi] && wi < zmax) {
      uint32_t kk = KS - 1;
#pragma unroll
      for (int k = KS - 2; k >= 0; --k) kk = y[k] == m ? (uint32_t)k : kk;
      const unsigned long long key =
          ((unsigned long long)sord(m) << 32) | (0xFFFFFFFFu - (bin0 + K0 + kk));
      atomicMax(&slot_row[wi], key);
    }
  };
  if (b == 0) {
    // in-group windows by the recursion; crossing ones from HB(s, 1) = H_s
    float own[K - K0];
#pragma unroll
    for (int j = K0; j < K; ++j) own[j - K0] = po[j * PITCH];
    float t[KS];
#pragma unroll
    for (int u = 0; u < K; ++u) {
      float y[KS];
#pragma unroll
      for (int k = 0; k < KS; ++k) {
        const int s = K0 + k;
        if (s + u < K) {
          t[k] = u == 0 ? own[s - K0] : t[k] + own[s + u - K0];
          y[k] = t[k];
        } else {
          y[k] = H[k] + EB[s + u - K];
        }
      }
      merge(u, y);
    }
  } else {
    // HB(s, b) and HB(s, b + 1)
    float hA[KS], hB[KS];
#pragma unroll
    for (int k = 0; k < KS; ++k) hA[k] = H[k];
    for (uint32_t j = 1; j < b; ++j) {
      const float sg = R.Sg[q + j];
#pragma unroll
      for (int k = 0; k < KS; ++k) hA[k] = hA[k] + sg;
    }
    {
      const float sg = R.Sg[q + b];
#pragma unroll
      for (int k = 0; k < KS; ++k) hB[k] = hA[k] + sg;
    }
    float EA[K];
    {
      const float *pa = R.bin(R.wrap(q + b), 0);
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const float v = pa[j * PITCH];
        EA[j] = j == 0 ? v : EA[j - 1] + v;
      }
    }
#pragma unroll
    for (int u = 0; u < K; ++u) {
      float y[KS];
#pragma unroll
      for (int k = 0; k < KS; ++k) {
        const int s = K0 + k;
        y[k] = s + u < K ? hA[k] + EA[s + u] : hB[k] + EB[s + u - K];
      }
      merge(u, y);
    }
  }
}

// Exact evaluation of the widths of one pass, w0 .. w0 + 63 (w0 = fb K + 1 +
// 64 pass), for the K starts of a flagged lane, by one wave, in the canonical
// order above (so bit for bit what eval_unit and the tiled kernel give).
// Thread t takes width w = w0 + t and runs over the lane's starts s: a window
// ending at p = s + w - 1 >= K in group g = p / K, at its e = p % K + 1-th
// bin, sums to HB(s, g) + E_g(e).  The unit first builds, in the wave's
// scratch, HB(s, g) for the groups the pass reaches (lane s runs its chain
// from H_s) and their prefix sums E_g (one lane per group), every chain with
// its reads issued together; a window then costs two LDS reads, a select and
// one addition.  Windows inside the lane's own group (p < K, first pass of
// the first width block only) are summed by the recursion from their start,
// one lane per start.  Each width's maximum over the starts (first start
// attaining it) that reaches the threshold is merged into the chunk's slot.
// A flagged lane's passes are independent units, so that the waves of the
// workgroup share them.

// Groups one pass of 64 widths reads, at most, and the scratch floats per
// wave (their prefix sums, then HB of those groups and of the one after).
template <int K>
__host__ __device__ constexpr int xgroups() {
  return (2 * K + 62) / K + 1;
}
template <int K>
__host__ __device__ constexpr int xs_floats() {
  return (xgroups<K>() * K + (xgroups<K>() + 1) * K + 15) / 16 * 16;
}

__device__ __forceinline__ unsigned long long slot_key(float y, uint32_t bin) {
  return ((unsigned long long)sord(y) << 32) | (0xFFFFFFFFu - bin);
}

template <int K>
__device__ __forceinline__ void exact_unit(const Ring<K> &R, uint32_t q, uint32_t fb,
                                           uint32_t pass, const float *Tl, uint32_t zmax,
                                           uint32_t nblk, unsigned long long *slot_row,
                                           uint32_t bin0, float *xs, uint32_t lane) {
  constexpr int PITCH = spitch<K>();
  constexpr int NG = xgroups<K>();
  float *const Q = xs;            // prefix sums of the unit's groups, flat by p
  float *const HBt = xs + NG * K;  // HB(s, g) at (g - glo) K + s
  const float *po = R.bin(q, 0);
  const uint32_t w0 = fb * K + 1 + 64 * pass;
  // groups glo..ghi hold every window end p >= K of the unit
  const uint32_t glo = (w0 - 1) / K > 1u ? (w0 - 1) / K : 1u;
  const uint32_t last = min(w0 + 63u, zmax);
  const uint32_t ghi = min((last + K - 2) / K, nblk);
  lds_wait();  // the previous unit's reads of the scratch are done
  // (the barriers below keep eight loads in flight at a time: the batch of
  // spectrum loads in flight holds many registers)
  if (lane < (uint32_t)K) {
    // H_s: lane s sums its group's bins s..K-1 from zero in increasing order
    float h = 0.f;
#pragma unroll
    for (int j0 = 0; j0 < K; j0 += 8) {
      asm volatile("" ::: "memory");
      float v[8];
#pragma unroll
      for (int k = 0; k < 8 && j0 + k < K; ++k) v[k] = po[(j0 + k) * PITCH];
#pragma unroll
      for (int k = 0; k < 8 && j0 + k < K; ++k) {
        const uint32_t j = j0 + k;
        if (j >= lane) h = j == lane ? v[k] : h + v[k];
      }
    }
    // HB(s, g) for g = 1 .. ghi + 1, kept for g >= glo
    float hb = h;
    for (uint32_t g0 = 1; g0 <= ghi + 1; g0 += 8) {
      asm volatile("" ::: "memory");
      float sg[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) sg[k] = R.Sg[q + min(g0 + k, ghi)];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const uint32_t g = g0 + k;
        if (g <= ghi + 1) {
          if (g >= glo) HBt[(g - glo) * K + lane] = hb;
          if (g <= ghi) hb = hb + sg[k];
        }
      }
    }
  }
  if (lane <= ghi - glo) {
    // prefix sums of group glo + lane, from zero in order
    const float *pg = R.bin(R.wrap(q + glo + lane), 0);
    float e = 0.f;
#pragma unroll
    for (int j0 = 0; j0 < K; j0 += 8) {
      asm volatile("" ::: "memory");
      float v[8];
#pragma unroll
      for (int k = 0; k < 8 && j0 + k < K; ++k) v[k] = pg[(j0 + k) * PITCH];
#pragma unroll
      for (int k = 0; k < 8 && j0 + k < K; ++k) {
        e = j0 + k == 0 ? v[0] : e + v[k];
        Q[lane * K + j0 + k] = e;
      }
    }
  }
  if (pass == 0 && fb == 0 && lane < (uint32_t)K) {
    // windows inside the own group: lane s sums from its start, in order
    // (zmax passes through an empty asm so that the K tests on it are made
    // here, not hoisted out of the workgroup's loops into K live masks)
    uint32_t zm = zmax;
    asm volatile("" : "+v"(zm));
    float t = 0.f;
#pragma unroll
    for (int u0 = 0; u0 < K; u0 += 8) {
      asm volatile("" ::: "memory");
      float v[8];
#pragma unroll
      for (int k = 0; k < 8 && u0 + k < K; ++k)
        v[k] = po[min(lane + u0 + k, (uint32_t)K - 1) * PITCH];
#pragma unroll
      for (int k = 0; k < 8 && u0 + k < K; ++k) {
        const int u = u0 + k;
        t = u == 0 ? v[0] : t + v[k];
        if (lane + u < (uint32_t)K && (uint32_t)u < zm && t >= Tl[u])
          atomicMax(&slot_row[u], slot_key(t, bin0 + lane));
      }
    }
  }
  lds_wait();
  const uint32_t w = w0 + lane;
  if (w <= last) {
    const uint32_t wm = w - 1, r = wm % K;
    const float *h0 = HBt + (wm / K - glo) * K;  // HB of the window's end group when s + r < K
    const float *qp = Q + (wm - glo * K);
    float m = -INFINITY;
    uint32_t best = 0;
    const bool head = w0 <= (uint32_t)K;  // uniform: windows inside the own group exist
#pragma unroll
    for (int s = 0; s < K; ++s) {
      if (s % 8 == 0 && s > 0) asm volatile("" ::: "memory");
      const float hb = s + r >= (uint32_t)K ? h0[K + s] : h0[s];
      const float y = hb + qp[s];
      const bool ok = !head || wm + s >= (uint32_t)K;
      if (ok && y > m) {
        m = y;
        best = (uint32_t)s;
      }
    }
    if (m >= Tl[wm]) atomicMax(&slot_row[wm], slot_key(m, bin0 + best));
  }
}

// ---------------------------------------------------------------------------
// The kernel

struct Shared {
  uint32_t items[3];  // flagged lanes of a tile (tile t counts in items[t % 3])
  uint32_t lost;
  uint32_t base;
  uint32_t next;      // the range taken next
  uint32_t wsum[kStreamWaves];
};

// Descriptors are read through the scalar cache (constant address space):
// wave-uniform values in scalar registers, whose loads are counted apart from
// the spectrum's vector loads, so that addresses built from them never wait
// for the spectrum.
#define CAS __attribute__((address_space(4)))
__device__ __forceinline__ Series series_at(const SpecDesc *descs, int s) {
  static_assert(sizeof(SpecDesc) % 8 == 0, "descriptor of whole words");
  constexpr int W = sizeof(SpecDesc) / 8;
  const CAS unsigned long long *g = (const CAS unsigned long long *)(descs + s);
  unsigned long long w[W];
#pragma unroll
  for (int k = 0; k < W; ++k) w[k] = g[k];
  SpecDesc d;
  __builtin_memcpy(&d, w, sizeof d);
  return Series{d.x, d.thr, d.block_begin, d.n, d.zmax, d.zc};
}

// Four waves per SIMD (two workgroups per CU): at most 128 registers.
// PRUNE: the pruned search (the hot path), compiled without the dense
// route and the table outputs; otherwise the dense search or the tables.
template <int K, int EPL, bool FP, bool PRUNE>
__global__ __launch_bounds__(kStreamThreads, 4) void stream_kernel(StreamParams p) {
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ Shared sh;
  constexpr uint32_t B = 64 * EPL, GPB = B / K;
  constexpr uint32_t NB = kStreamBatch;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const uint32_t nthr = kStreamThreads;
  // the launch's parameters as values (a reference to the argument, captured
  // by the lambdas below, would make the compiler copy it to scratch memory)
  const SpecDesc *descs = p.descs;
  const int nspec = p.nspec;
  const uint32_t nwg = p.nwg, C = p.chunk, spin = p.spin, pool_cap = p.pool_cap;
  // chunks tile the block (a power of two), so C is one: divisions by it are
  // shifts (a division by a runtime value would keep its reciprocal live)
  const uint32_t lgC = __builtin_ctz(C);
  const uint32_t RB = p.g.ring, lag = p.g.lag;
  // x mod RB, with RB through an empty asm at each use: the division's set-up
  // is then made there instead of its reciprocal held in a register
  auto ring_mod = [&](uint32_t x) __attribute__((always_inline)) {
    uint32_t rb = RB;
    asm volatile("" : "+s"(rb));
    return x % rb;
  };
  StageEntry *const pool = p.pool;
  uint32_t *const pool_head = p.pool_head;
  unsigned long long *const halo = p.halo;
  Ring<K> R;
  R.P = reinterpret_cast<float *>(lds);
  R.Sg = reinterpret_cast<float *>(lds + p.g.off_sg);
  R.NG = RB * GPB;
  R.mirror = p.g.mirror;
  {
    const uint32_t stride = R.NG + p.g.mirror;
    float *e = reinterpret_cast<float *>(lds + p.g.off_ep);
    R.E[0] = e;
    R.E[1] = e + stride;
    R.E[2] = e + 2 * stride;
  }
  unsigned long long *slots = reinterpret_cast<unsigned long long *>(lds + p.g.off_slots);
  float *Tl = reinterpret_cast<float *>(lds + p.g.off_tl);
  float *Tb1 = Tl + p.g.zc_pad;
  float *Tb = Tb1 + 4;
  uint32_t *items = reinterpret_cast<uint32_t *>(lds + p.g.off_items);

  const uint32_t wg = blockIdx.x;
  const uint32_t tag = *gp(p.gen) + 1u;
  const uint64_t units = p.total_blocks;
  const uint32_t nseg = p.nseg;
  const bool search = PRUNE || p.mode == kModeSearch;
  constexpr bool prune = PRUNE;
  NormOut no{};
  no.P_out = !PRUNE && p.mode == kModeTables ? p.P_out : nullptr;
  no.stats_out = !PRUNE && p.mode == kModeTables ? p.stats_out : nullptr;
  uint32_t tc = 0;        // tiles banked so far (uniform)
  if (threadIdx.x == 0) {
    sh.items[0] = 0u;
    sh.items[1] = 0u;
    sh.items[2] = 0u;
  }

  // the ranges of this workgroup, of the launch's nseg: range w first, then
  // the next one not yet taken (from the launch's counter) or, without a
  // counter, w + nwg, w + 2 nwg, ...  The counters alternate between
  // launches: launch tag t takes from seg_ctr[t & 1], whose last increments
  // may come after the scan, and the scan re-arms seg_ctr[(t + 1) & 1] for
  // the next launch.
  uint32_t *const seg_ctr = p.seg_ctr ? p.seg_ctr + (tag & 1u) : nullptr;
  for (uint32_t seg = wg; seg < nseg;) {
    // The range [g0, g1): with one range per workgroup, equal ones; with
    // several, ranges that shrink along the launch (range i starts at
    // units (i N + 3 (N^2 - (N - i)^2)) / 4N^2, N = nseg: the first about
    // 1.75 times the mean, the last a quarter of it), so that the ranges
    // taken last, which set how far apart the workgroups end, are short.
    // (The divisor goes through an empty asm: the division's set-up is then
    // made here, once per range, instead of held in registers across the
    // loop.  units 4N^2 stays below 2^64 for launches below 10^13 bins.)
    uint32_t ns = nseg;
    asm volatile("" : "+s"(ns));
    uint64_t g0, g1;
    if (nseg == nwg) {  // (not ns: the compiler would then divide by nwg)
      g0 = uniform64(units * seg / ns);
      g1 = uniform64(units * (seg + 1) / ns);
    } else {
      const uint64_t N = ns, r0 = N - seg, r1 = r0 - 1;
      g0 = uniform64(units * ((uint64_t)seg * N + 3 * (N * N - r0 * r0)) / (4 * N * N));
      g1 = uniform64(units * ((uint64_t)(seg + 1) * N + 3 * (N * N - r1 * r1)) / (4 * N * N));
    }
    uint32_t wg_count = 0;  // candidates staged so far in this range (uniform)

    // the series holding block g0
    int s = 0;
    if (nspec > 1) {
      int lo = 0, hi = nspec - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (((const CAS SpecDesc *)descs)[mid].block_begin <= g0)
          lo = mid;
        else
          hi = mid - 1;
      }
      s = lo;
    }
    uint64_t gc = g0;
    while (gc < g1 && s < nspec) {
      const Series d = nspec == 1 ? Series{p.single.x, p.single.thr, p.single.block_begin,
                                           p.single.n, p.single.zmax, p.single.zc}
                                  : series_at(descs, s);
      const uint32_t nbs = (d.n + B - 1) / B;
      if (gc < d.block_begin) gc = d.block_begin;
      if (gc >= g1) break;
      if (gc >= d.block_begin + nbs) {  // padding after the series
        ++s;
        continue;
      }
      const uint32_t a = (uint32_t)(gc - d.block_begin);
      const uint32_t b = (uint32_t)min(g1 - d.block_begin, (uint64_t)nbs);
      const uint32_t n = d.n, zmax = d.zmax, zc = d.zc, nblk = zc / K;
      const uint32_t lgs = (zc + B - 1) / B;       // halo blocks of this series
      // the previous range needs our first blocks; with several ranges per
      // workgroup the ranges' neighbours run at unrelated times, and each
      // range normalises its halo blocks itself (lag blocks against ranges
      // of kStreamRangeMin blocks on average)
      const bool publish = nseg == nwg && a > 0 && gc == g0;
      const bool consume = b < nbs;                // our last tile reaches into the next range
      const uint32_t zpub = min(lgs, b - a);

      // this series' first thresholds, then the first batch's loads (loads
      // complete in order, so the thresholds can be stored before the spectrum
      // arrives), then the set-up
      const float thr0 = threadIdx.x < zc ? gp(d.thr)[threadIdx.x] : 0.f;
      const uint32_t nbat = (b - a + NB - 1) / NB;
      Raw<EPL, FP> cur, nxt;
      // issue the loads of batch j into r: block a + jNB + wave, or, for
      // j == nbat, the halo block b + wave's first bins
      // Every wave issues the same number of loads on every path (a wave with
      // no block re-reads the range's last one, never used), so that waiting
      // for one set never waits for the next.
      auto issue = [&](uint32_t j, Raw<EPL, FP> &r) __attribute__((always_inline)) {
        if (j < nbat) {
          load_block<EPL, FP>(d, min(a + j * NB + wave, b - 1), r);
        } else {
          const bool halo = j == nbat && consume && wave < lgs && b + wave < nbs;
          const uint32_t need = halo ? min(B, (zc - wave * B + 63) / 64 * 64) : B;
          load_prefix<EPL, FP>(d, halo ? b + wave : b - 1, need, r);
        }
      };
      issue(0, cur);

      // thresholds of the series, and the bound's minima of them
      __syncthreads();
      if (threadIdx.x < zc) Tl[threadIdx.x] = thr0;
      if (zc > nthr) {  // zmax above 512 (uniform)
        for (uint32_t i = ftid() + nthr; i < zc; i += nthr) Tl[i] = gp(d.thr)[i];
      }
      __syncthreads();
      {
        // the first block's sub-ranges, widths 1..4, 5..8, 9..16 (those that
        // exist), and every width block
        const uint32_t tid = ftid();
        if (tid == 0) {
          float m0 = Tl[0], m1 = INFINITY, m2 = INFINITY;
  #pragma unroll
          for (int w = 1; w < K; ++w) {
            if (w < 4) m0 = fminf(m0, Tl[w]);
            else if (w < 8) m1 = fminf(m1, Tl[w]);
            else m2 = fminf(m2, Tl[w]);
          }
          Tb1[0] = m0 * kSBoundSlack;
          Tb1[1] = m1 * kSBoundSlack;
          Tb1[2] = m2 * kSBoundSlack;
        }
        for (uint32_t i = tid; i < nblk; i += nthr) {
          float m = Tl[i * K];
  #pragma unroll
          for (int u = 1; u < K; ++u) m = fminf(m, Tl[i * K + u]);
          Tb[i] = m * kSBoundSlack;
        }
      }

      // the halo's statistics words, published by the next range's workgroup
      const unsigned long long *hw = halo + (size_t)(seg + 1) * lag * 4;
      unsigned long long *pw = halo + (size_t)seg * lag * 4;

      uint32_t banked = a;
      no.tag = tag;

      // bank the tile of blocks [t0, t1)
      auto bank_tile = [&](uint32_t t0, uint32_t t1) __attribute__((always_inline)) {
        const uint32_t tb0 = t0 * B;
        const uint32_t tbins = min((t1 - t0) * B, n - tb0);   // window starts
        const uint32_t nlane = (tbins + K - 1) / K;            // lanes with starts
        const uint32_t gb = ring_mod(t0 - a) * GPB;             // ring position of the tile's group 0
        const uint32_t nch = (tbins + C - 1) >> lgC, chunk0 = tb0 >> lgC;
        const uint32_t nsl = nch * zmax;
        const uint32_t nbw = (zmax + K - 1) / K;               // width blocks
        // tile tc counts its flagged lanes in items[tc % 3].  After its first
        // barrier every thread has read tile tc-1's count, and no thread can
        // reach tile tc+2's counting before passing tile tc+1's first barrier,
        // which thread 0 reaches only after clearing items[(tc+2) % 3] here
        const uint32_t ci = tc % 3;
        uint32_t *cnt = &sh.items[ci];
        ++tc;
        if (prune) {
          const uint32_t tid = ftid(), ln = tid & 63, wv = tid >> 6;
          for (uint32_t sg = wv; sg * 64 < nlane; sg += kStreamWaves) {
            const uint32_t L = sg * 64 + ln;
            const uint32_t fl = L < nlane ? sbound<K>(R, R.wrap(gb + L), Tb1, Tb, nblk) : nblk;
            const unsigned long long mask = __ballot(fl < nblk);
            if (mask) {
              uint32_t base = 0;
              if (ln == 0) base = atomicAdd(cnt, (uint32_t)__popcll(mask));
              base = __shfl(base, 0, 64);
              if (fl < nblk) items[base + __popcll(mask & ((1ull << ln) - 1ull))] = (L << 12) | fl;
            }
          }
          __syncthreads();
          if (threadIdx.x == 0) sh.items[ci == 0 ? 2 : ci - 1] = 0u;
        }
        const uint32_t nitems = prune ? *cnt : nlane;
        if (nitems == 0) return;  // nothing evaluated: no candidate (uniform)
        {
          const uint32_t tid = ftid();
          for (uint32_t i = tid; i < nsl; i += nthr) slots[i] = 0ull;
          __syncthreads();
        }
        if constexpr (PRUNE) {
          // units (flagged lane, pass of 64 widths from its first flagged
          // width block), one per wave at a time; a lane's passes go to
          // consecutive waves
          float *xs = reinterpret_cast<float *>(lds + p.g.off_xs) + wave * xs_floats<K>();
          const uint32_t np = (zmax + 63) / 64;
          for (uint32_t u = wave; u < nitems * np; u += kStreamWaves) {
            const uint32_t it = items[u / np], pass = u % np, fb = it & 0xFFFu;
            if (fb * K + 1 + 64 * pass > zmax) continue;  // past the lane's widths (uniform)
            const uint32_t L = it >> 12;
            // the lane index taken afresh per unit: its masks and addresses are
            // rebuilt here rather than held across the workgroup's loops
            exact_unit<K>(R, R.wrap(gb + L), fb, pass, Tl, zmax, nblk,
                          slots + (size_t)((L * K) >> lgC) * zmax, tb0 + L * K, xs, ftid() & 63);
          }
        } else {
          // units (lane, width block, start group): lane-major pairs, every 64
          // pairs taken once per start group by whole waves
          const uint32_t tid = ftid();
          constexpr uint32_t NH = K / sks<K>();
          const uint32_t npairs = nitems * nbw;
          const uint32_t nrun = (npairs + 63) / 64 * 64 * NH;
          for (uint32_t r0 = 0; r0 < nrun; r0 += nthr) {
            const uint32_t j = r0 + tid;
            const uint32_t grp = j >> 6, half = grp % NH;
            const uint32_t u = (grp / NH) * 64 + (j & 63);
            const bool ok = j < nrun && u < npairs;
            const uint32_t it = ok ? (prune ? items[u / nbw] : ((u / nbw) << 12)) : 0u;
            const uint32_t bw = ok ? u % nbw : 0u;
            if (ok && bw >= (it & 0xFFFu)) {
              const uint32_t L = it >> 12;
              const uint32_t q = R.wrap(gb + L);
              unsigned long long *row = slots + (size_t)((L * K) >> lgC) * zmax;
              if constexpr (NH == 1) {
                eval_unit<K, 0>(R, q, bw, Tl, zmax, row, tb0 + L * K);
              } else {
                static_assert(NH == 4, "four start groups of four");
                if (half == 0)
                  eval_unit<K, 0>(R, q, bw, Tl, zmax, row, tb0 + L * K);
                else if (half == 1)
                  eval_unit<K, 4>(R, q, bw, Tl, zmax, row, tb0 + L * K);
                else if (half == 2)
                  eval_unit<K, 8>(R, q, bw, Tl, zmax, row, tb0 + L * K);
                else
                  eval_unit<K, 12>(R, q, bw, Tl, zmax, row, tb0 + L * K);
              }
            }
          }
        }
        __syncthreads();
        const uint32_t tid = ftid(), ln = tid & 63, wv = tid >> 6;
        if (search) {
          // stage the tile's maxima in slot order, i.e. (chunk, width) order
          const uint32_t per = (nsl + nthr - 1) / nthr;
          const uint32_t lo = min(tid * per, nsl), hi = min(lo + per, nsl);
          uint32_t mine = 0;
          for (uint32_t i = lo; i < hi; ++i) mine += slots[i] != 0ull ? 1u : 0u;
          uint32_t incl = mine;
  #pragma unroll
          for (int o = 1; o < 64; o <<= 1) {
            const uint32_t v = __shfl_up(incl, o, 64);
            if (ln >= (uint32_t)o) incl += v;
          }
          if (ln == 63) sh.wsum[wv] = incl;
          __syncthreads();
          uint32_t before = 0, tot = 0;
          for (uint32_t v = 0; v < (uint32_t)kStreamWaves; ++v) {
            before += v < wv ? sh.wsum[v] : 0u;
            tot += sh.wsum[v];
          }
          if (tid == 0) sh.base = tot ? atomicAdd(pool_head, tot) : 0u;
          __syncthreads();
          const uint32_t base = sh.base;
          uint32_t rank = before + incl - mine;
          for (uint32_t i = lo; i < hi; ++i) {
            const unsigned long long key = slots[i];
            if (key == 0ull) continue;
            const uint32_t pos = base + rank;
            if (pos < pool_cap) {
              const uint32_t cl = i / zmax, w = i - cl * zmax + 1;
              StageEntry e;
              e.unit = seg;
              e.rank = wg_count + rank;
              e.spec = (uint32_t)s;
              e.bin = 0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull);
              e.power = sunord((uint32_t)(key >> 32));
              e.width = w;
              pool[pos] = e;
            }
            ++rank;
          }
          wg_count += tot;
        } else {
          for (uint32_t i = tid; i < nsl; i += nthr) {
            const unsigned long long key = slots[i];
            const size_t o = (size_t)chunk0 * zmax + i;
            p.M[o] = key ? sunord((uint32_t)(key >> 32)) : -INFINITY;
            p.I[o] = key ? 0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull) : 0xFFFFFFFFu;
          }
        }
        __syncthreads();
      };

      // Step j normalises batch j (wave w: block a + jNB + w) and banks every
      // tile whose windows the ring then holds: up to f + NB - lgs, the
      // batch's end less the halo (the next batch overwrites the blocks before
      // f + NB - lag), and for the last batch up to b - lgs, so that the
      // halo's slots are free.  The halo step then normalises the first bins of
      // blocks b .. b+lgs-1 (wave w: block b + w) and banks up to b.  The next
      // batches' loads (or the halo's) are in flight while this one is
      // searched: the two register sets alternate.  Only the first two batches
      // are not requested together (issued together, they would arrive
      // interleaved, every workgroup's whole first pair at once, with nothing
      // to search in the meantime).
      auto step = [&](uint32_t j, Raw<EPL, FP> &r) __attribute__((always_inline)) {
        const uint32_t f = a + j * NB;
        const uint32_t k = f + wave;
        if (k < b) {
          NormOut o = no;
          o.pub = (publish && k - a < zpub) ? pw + 4 * (k - a) : nullptr;
          normalise<K, EPL, FP>(d, k, r, false, BlockStats{}, B, R, ring_mod(k - a), o, lane);
        }
        __syncthreads();
        const uint32_t ready = j + 1 == nbat ? (b > lgs ? b - lgs : 0u)
                                             : (f + NB > lgs ? f + NB - lgs : 0u);
        while (banked < ready) {
          const uint32_t t1 = min(banked + NB, ready);
          bank_tile(banked, t1);
          banked = t1;
        }
      };
      // batch 1 is requested once batch 0 has arrived (every load issued so
      // far); from then on batch j + 2 is requested as soon as batch j has been
      // normalised, so that two batches are in flight while batch j + 1 is
      // awaited
      __builtin_amdgcn_s_waitcnt(kWaitVm0);
      issue(1, nxt);
      uint32_t j = 0;
      while (true) {
        step(j, cur);
        if (j + 1 == nbat) break;  // the halo is in nxt
        issue(j + 2, cur);
        step(j + 1, nxt);
        if (j + 2 == nbat) {  // the halo is in cur
          nxt = cur;
          break;
        }
        issue(j + 3, nxt);
        j += 2;
      }
      {
        // the halo step
        const uint32_t k = b + wave;
        if (wave < lgs) {
          const uint32_t limit = min(B, (zc - wave * B + 63) / 64 * 64);
          const uint32_t slot = ring_mod(k - a);
          if (k >= nbs) {
            // no spectrum behind these bins
            fill_past_end<K, EPL>(R, slot, limit, lane);
          } else {
            BlockStats given{};
            bool use_given = false;
            if constexpr (!FP) {
              // the next range's published statistics, or our own
              unsigned long long v = 0;
              bool ok = false;
              // (the word's address from a fresh lane id, so that it is not
              // computed at the kernel's start and kept live)
              const uint32_t ln = ftid() & 63;
              if (ln < 4) {
                const unsigned long long *hwl = hw + 4 * wave + ln;
                for (uint32_t it = 0; it < (nseg == nwg ? spin : 0u); ++it) {
                  v = __hip_atomic_load(hwl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                  if ((uint32_t)(v >> 32) == tag) {
                    ok = true;
                    break;
                  }
                  __builtin_amdgcn_s_sleep(2);
                }
              }
              use_given = __ballot(ok) == 0xFull;
              if (use_given) {
                given.med_re = __uint_as_float(__builtin_amdgcn_readlane((uint32_t)v, 0));
                given.mad_re = __uint_as_float(__builtin_amdgcn_readlane((uint32_t)v, 1));
                given.med_im = __uint_as_float(__builtin_amdgcn_readlane((uint32_t)v, 2));
                given.mad_im = __uint_as_float(__builtin_amdgcn_readlane((uint32_t)v, 3));
              } else {
                load_block<EPL, FP>(d, k, nxt);
              }
            }
            normalise<K, EPL, FP>(d, k, nxt, use_given, given, limit, R, slot, NormOut{}, lane);
          }
        }
        __syncthreads();
        while (banked < b) {
          const uint32_t t1 = min(banked + NB, b);
          bank_tile(banked, t1);
          banked = t1;
        }
      }
      gc = d.block_begin + b;
      if (b == nbs) ++s;
      // every load of this series has been consumed: say so, so that the next
      // series' loads are not held back for ones that might be in flight
      __builtin_amdgcn_s_waitcnt(0);
    }

    // publish this range's count; the last workgroup scans every range's
    __syncthreads();
    if (threadIdx.x == 0) {
      // the pool reservations are complete before the count is published, so
      // the scan (which waits for every count) may re-arm the pool head
      __builtin_amdgcn_s_waitcnt(0);
      __hip_atomic_store(p.wg_word + seg, ((unsigned long long)tag << 32) | wg_count,
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      sh.next = seg_ctr ? nwg + atomicAdd(seg_ctr, 1u) : seg + nwg;
    }
    __syncthreads();
    seg = __builtin_amdgcn_readfirstlane(sh.next);
  }
  if (threadIdx.x == 0) sh.lost = 0u;
  if (wg != p.nwg - 1) return;
  __syncthreads();
  const uint32_t tid = threadIdx.x;
  const uint32_t per = (nseg + nthr - 1) / nthr;
  const uint32_t lo = min(tid * per, nseg), hi = min(lo + per, nseg);
  uint32_t mine = 0;
  bool lost = false;
  for (uint32_t i = lo; i < hi; ++i) {
    unsigned long long v = 0;
    bool ok = false;
    for (uint32_t it = 0; it < p.spin; ++it) {
      v = __hip_atomic_load(p.wg_word + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if ((uint32_t)(v >> 32) == tag) {
        ok = true;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    lost |= !ok;
    mine += ok ? (uint32_t)v : 0u;
  }
  if (lost) atomicOr(&sh.lost, 1u);
  uint32_t incl = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t v = __shfl_up(incl, o, 64);
    if (lane >= (uint32_t)o) incl += v;
  }
  if (lane == 63) sh.wsum[wave] = incl;
  __syncthreads();
  uint32_t run = 0, tot = 0;
  for (uint32_t v = 0; v < (uint32_t)kStreamWaves; ++v) {
    run += v < wave ? sh.wsum[v] : 0u;
    tot += sh.wsum[v];
  }
  run += incl - mine;
  for (uint32_t i = lo; i < hi; ++i) {
    p.wg_prefix[i] = run;
    run += (uint32_t)__hip_atomic_load(p.wg_word + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  if (tid == 0) {
    p.wg_prefix[nseg] = tot;
    if (search) {
      const uint32_t ovf = sh.lost ? 2u : (tot > p.pool_cap ? 1u : 0u);
      *p.total = tot;
      if (p.total2) *p.total2 = count_word(tot, ovf);
      *p.overflow = ovf;
    } else {
      *p.overflow = sh.lost ? 2u : 0u;
    }
    __hip_atomic_store(p.pool_head, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (p.seg_ctr)
      __hip_atomic_store(p.seg_ctr + ((tag + 1u) & 1u), 0u, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    *gp(p.gen) = tag;
  }
}

// ---------------------------------------------------------------------------
// Host side

// LDS per workgroup, beside its static shared memory: two workgroups share a
// CU's 160 KiB
constexpr size_t kStreamLdsMax = 80 * 1024 - 512;

static uint32_t up16(uint32_t v) { return (v + 15u) & ~15u; }

bool choose_stream_geometry(uint32_t C, uint32_t B, uint32_t zmax_max, bool from_power,
                            bool norm_exact, bool fp16, StreamGeometry *g) {
  if (norm_exact || fp16) return false;
  if (zmax_max == 0 || zmax_max > 4096 || C == 0 || C % 64 != 0) return false;
  int K = 16;
  while (K > 1 && (C / 64) % (uint32_t)K != 0) K /= 2;
  if (K != 16 && K != 4) return false;
  if (from_power) B = 1024;  // the streaming unit of power input
  if (B != 256 && B != 1024) return false;
  // a tile starts on a block boundary, so chunks must tile the block
  if (C > B || B % C != 0 || 64u * (uint32_t)K > B) return false;
  const uint32_t zc = (zmax_max + K - 1) / K * K;
  const uint32_t lag = (zc + B - 1) / B;
  if (lag > (uint32_t)kStreamBatch) return false;
  const uint32_t ring = kStreamBatch + lag;
  const uint32_t gpb = B / K, ng = ring * gpb;
  const uint32_t nblk = zc / K;
  const uint32_t mirror = nblk + 2;
  const uint32_t ne = K >= 16 ? 3 : K >= 8 ? 2 : 1;
  const uint32_t pitch = 64 + 64 / K;
  uint32_t off = 0;
  const uint32_t ring_bytes = ring * (B / (64 * K)) * K * pitch * 4;
  off = up16(ring_bytes);
  g->off_sg = off;
  off = up16(off + (ng + mirror) * 4);
  g->off_ep = off;
  off = up16(off + ne * (ng + mirror) * 4);
  g->off_slots = off;
  const uint32_t nch = kStreamBatch * B / C;
  off = up16(off + nch * zmax_max * 8);
  g->off_tl = off;
  g->zc_pad = (zc + 3) / 4 * 4;
  off = up16(off + (g->zc_pad + 4 + nblk + 4) * 4);
  g->off_items = off;
  off = up16(off + kStreamBatch * B / K * 4);
  g->off_xs = off;
  off = up16(off + kStreamWaves * (K == 16 ? xs_floats<16>() : xs_floats<4>()) * 4);
  if (off > kStreamLdsMax) return false;
  g->K = K;
  g->EPL = (int)(B / 64);
  g->lag = lag;
  g->ring = ring;
  g->mirror = mirror;
  g->zc_max = zc;
  g->lds_bytes = off;
  return true;
}

template <int K, int EPL, bool FP, bool PRUNE>
static const void *stream_fn() {
  return reinterpret_cast<const void *>(&stream_kernel<K, EPL, FP, PRUNE>);
}

template <bool PRUNE>
static const void *stream_entry_p(const StreamGeometry &g, bool fp) {
  if (g.K == 16 && g.EPL == 16)
    return fp ? stream_fn<16, 16, true, PRUNE>() : stream_fn<16, 16, false, PRUNE>();
  if (g.K == 4 && g.EPL == 16)
    return fp ? stream_fn<4, 16, true, PRUNE>() : stream_fn<4, 16, false, PRUNE>();
  if (g.K == 4 && g.EPL == 4)
    return fp ? stream_fn<4, 4, true, PRUNE>() : stream_fn<4, 4, false, PRUNE>();
  return nullptr;
}

static const void *stream_entry(const StreamGeometry &g, bool fp, bool prune) {
  return prune ? stream_entry_p<true>(g, fp) : stream_entry_p<false>(g, fp);
}

// Workgroups above 64 KiB of LDS must say so before they launch.
static bool allow_lds(const void *fn, size_t bytes) {
  if (bytes <= 64 * 1024) return true;
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) !=
      hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return true;
}

// Every workgroup of a launch must be resident at once (workgroups wait for
// their neighbours' words), so the occupancy is the smaller of the two
// instantiations'.
int stream_occupancy(const StreamGeometry &g, bool from_power) {
  int occ = 1 << 30;
  for (int pr = 0; pr < 2; ++pr) {
    const void *fn = stream_entry(g, from_power, pr != 0);
    if (!fn || !allow_lds(fn, g.lds_bytes)) return 0;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kStreamThreads, g.lds_bytes) !=
        hipSuccess) {
      (void)hipGetLastError();
      return 0;
    }
    occ = nb < occ ? nb : occ;
  }
  return occ;
}

hipError_t launch_stream(const StreamParams &p, hipStream_t stream) {
  const bool prune = p.mode == kModeSearch && !p.dense;
  const void *fn = stream_entry(p.g, p.from_power != 0, prune);
  if (!fn || !allow_lds(fn, p.g.lds_bytes)) return hipErrorInvalidValue;
  void *args[] = {const_cast<StreamParams *>(&p)};
  return hipLaunchKernel(fn, dim3(p.nwg), dim3(kStreamThreads), args, p.g.lds_bytes, stream);
}

}  // namespace pulscan

// The fused boxcar-bank kernel: one pass over each tile of a spectrum does
// normalisation, power, the boxcar bank of every width and the per-chunk
// maxima with the threshold test.
//
//  * Normalisation (section 2.2.3; section 2.5 and the appendix algorithm
//    "Median of Medians Normalisation", or the exact median of the CPU
//    version by a radix select): one wave per block of B = 64*EPL bins.
//    Lane l holds elements l + 64m, so the first levels of the median-of-4
//    tree (strides B/4, B/16, ... down to 64) stay inside a lane and the last
//    three (16, 4, 1 lanes) use cross-lane moves (permlane swaps and DPP row
//    shifts).  The real and imaginary trees run interleaved.
//  * Power (section 2.2.3): re'^2 + im'^2, written to LDS only.  The tile
//    holds its T bins plus a halo of up to zmax - 1 bins from the next blocks
//    (normalised with those blocks' own statistics).
//  * Bank (section 2.2.5): each lane owns K consecutive window starts.  A
//    running upper bound finds, per lane, the first width block in which one
//    of its windows could reach its threshold (powers are non-negative, so a
//    lane's union window bounds all its windows, and thresholds rise with
//    the width).  Lanes that can reach one are queued; the whole workgroup
//    then evaluates every (queued lane, width block) exactly, each unit
//    entering its block from the K-bin group sums.  The sums follow one
//    canonical FP32 order (see width_block) in both this pruned route and
//    the dense route, which evaluates everything; both give the same bits.
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
#include "mom.hpp"

namespace pulscan {

// Global-memory view of a pointer the kernels receive inside a structure.
// The compiler cannot infer the address space of such pointers, and generic
// (flat) accesses are also counted against the LDS wait counter, so every LDS
// wait would wait for outstanding spectrum loads too.
#define GLOBAL_AS __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ GLOBAL_AS T *glob(T *p) {
  return (GLOBAL_AS T *)p;
}
typedef float f32x2 __attribute__((ext_vector_type(2)));

// A series descriptor read from the device table as 64-bit words.
__device__ __forceinline__ SpecDesc load_desc(const SpecDesc *p) {
  static_assert(sizeof(SpecDesc) % 8 == 0, "descriptor of whole words");
  constexpr int W = sizeof(SpecDesc) / 8;
  const GLOBAL_AS unsigned long long *g = glob(reinterpret_cast<const unsigned long long *>(p));
  unsigned long long w[W];
#pragma unroll
  for (int k = 0; k < W; ++k) w[k] = g[k];
  SpecDesc d;
  __builtin_memcpy(&d, w, sizeof d);
  return d;
}

// Row pitch (floats) of the power tile for K bins per lane: the 64 lane
// columns plus 64/K pad words, so that the bank's reads (64 consecutive
// words of a row) and the normalisation's writes (lane l -> row l % K,
// column l / K) both fall on distinct banks.
template <int K>
__host__ __device__ constexpr int pitch_of() {
  return K == 1 ? 64 : 64 + 64 / K;
}

// Lane l of each row of 16 receives lane l + k's value (row_shl k); lanes
// whose source lies past the row's end read 0 (bound control), so no old
// value has to be set up.  Only lanes whose sources lie inside the row are
// used.
template <int CTRL>
__device__ __forceinline__ float dpp_row(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, true));
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
      if (cnt == EPL) {  // the inputs themselves (or their deviations)
        a[m] = m4x2(a[m], a[m + q], a[m + 2 * q], a[m + 3 * q]);
        b[m] = m4x2(b[m], b[m + q], b[m + 2 * q], b[m + 3 * q]);
      } else {
        a[m] = m4x2(a[m], a[m + q], a[m + 2 * q], a[m + 3 * q]);
        b[m] = m4x2(b[m], b[m + q], b[m + 2 * q], b[m + 3 * q]);
      }
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
// run one at a time to stay within the register budget).
template <int EPL, bool DEV>
__device__ __forceinline__ float wave_mom1(const float (&a)[EPL], float c) {
  // first level straight from the inputs (f(x) = x, or |x - c| for the MAD),
  // so the inputs need no working copy
  constexpr int Q = EPL / 4;
  float v[Q];
#pragma unroll
  for (int m = 0; m < Q; ++m) {
    float e[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) e[j] = DEV ? fabsf(a[m + j * Q] - c) : a[m + j * Q];
    v[m] = DEV ? m4x2(e[0], e[1], e[2], e[3]) : m4x2(e[0], e[1], e[2], e[3]);
  }
#pragma unroll
  for (int cnt = Q; cnt >= 4; cnt /= 4) {
    const int q = cnt / 4;
#pragma unroll
    for (int m = 0; m < q; ++m) v[m] = m4x2(v[m], v[m + q], v[m + 2 * q], v[m + 3 * q]);
  }
  float x = v[0];
  {
    const float x1 = from_plus16(x);
    x = m4x2(x, x1, from_plus32(x), from_plus32(x1));
  }
  x = m4x2(x, dpp_row<kRowShl4>(x), dpp_row<kRowShl8>(x), dpp_row<kRowShl12>(x));
  x = m4x2(x, dpp_row<kRowShl1>(x), dpp_row<kRowShl2>(x), dpp_row<kRowShl3>(x));
  constexpr float scale = 1.0f / (float)(1 << (log4_of<EPL>() + 3));
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x))) * scale;
}

// A power as stored in the LDS tile: FP32, or FP16 (round to nearest;
// values beyond the FP16 range become +inf, which the re-check catches).
template <typename PT>
__device__ __forceinline__ PT to_pt(float v) {
  return (PT)v;
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
__device__ __forceinline__ float unord_key(uint32_t o) { return unord_f32(o); }

// Exact median of the 64*EPL values f(a[m]) of one wave (lane l holds
// element l + 64m), f(x) = x or |x - c| for DEV: the mean of the two middle
// order statistics (the CPU version's median, section 2.5).  The lower one
// is found by a binary radix select on the order-preserving 32-bit keys,
// most significant bit first, counting with wave-wide sums; the upper one is
// the same value when it repeats, else the smallest key above it.
template <int EPL, bool DEV>
__device__ __forceinline__ uint32_t key_of(const float (&a)[EPL], int m, float c) {
  const float v = DEV ? fabsf(a[m] - c) : a[m];
  const uint32_t u = __float_as_uint(v);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = min(v, (uint32_t)__shfl_xor(v, o, 64));
  return v;
}

template <int EPL, bool DEV>
__device__ __forceinline__ float wave_median_exact(const float (&a)[EPL], float c) {
  constexpr uint32_t N = 64u * EPL;
  const uint32_t k = N / 2 - 1;  // rank (0-based) of the lower middle value
  uint32_t key[EPL];
#pragma unroll
  for (int m = 0; m < EPL; ++m) key[m] = key_of<EPL, DEV>(a, m, c);
  uint32_t prefix = 0, rank = k;
#pragma unroll 1
  for (int bit = 31; bit >= 0; --bit) {
    const uint32_t hi = bit == 31 ? 0u : (0xFFFFFFFFu << (bit + 1));
    const uint32_t b = 1u << bit;
    uint32_t cnt = 0;
#pragma unroll
    for (int m = 0; m < EPL; ++m) cnt += ((key[m] & hi) == prefix && !(key[m] & b)) ? 1u : 0u;
    cnt = wave_sum_u32(cnt);
    if (rank >= cnt) {
      rank -= cnt;
      prefix |= b;
    }
  }
  // prefix is the key of the k-th smallest; the (k+1)-th is equal to it when
  // more than k + 1 keys are <= it, else the least key above it
  uint32_t le = 0, above = 0xFFFFFFFFu;
#pragma unroll
  for (int m = 0; m < EPL; ++m) {
    le += key[m] <= prefix ? 1u : 0u;
    if (key[m] > prefix) above = min(above, key[m]);
  }
  le = wave_sum_u32(le);
  above = wave_min_u32(above);
  const uint32_t k2 = le >= k + 2 ? prefix : above;
  const float v1 = unord_key(prefix), v2 = unord_key(k2);
  const float med = 0.5f * (v1 + v2);
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(med)));
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
    const f32x2 v = glob(reinterpret_cast<const f32x2 *>(x))[bd.s0 + lane + 64 * m];
    bd.re[m] = v.x;
    bd.im[m] = v.y;
  }
}

// Normalise a loaded block and write its power into the tile's LDS array for
// every bin of the block that the tile needs (tile-relative index below
// `need`).  Executed by one whole wave.
template <int K, int EPL, typename PT, bool EXACT>
__device__ __forceinline__ void normalise_block(BlockData<EPL> &bd, uint32_t b, uint32_t t0,
                                                uint32_t need, uint32_t T, PT *Pl,
                                                uint32_t lane, float *P_out, float *stats_out) {
  constexpr uint32_t B = 64 * EPL;
  constexpr int PITCH = pitch_of<K>();
  float(&re)[EPL] = bd.re;
  float(&im)[EPL] = bd.im;
  const uint32_t own = bd.own, s0 = bd.s0;
  float med_re, med_im, mad_re, mad_im;
  if constexpr (EXACT) {
    // the exact median and MAD
    med_re = wave_median_exact<EPL, false>(re, 0.f);
    med_im = wave_median_exact<EPL, false>(im, 0.f);
    mad_re = wave_median_exact<EPL, true>(re, med_re);
    mad_im = wave_median_exact<EPL, true>(im, med_im);
  } else if constexpr (EPL == 4 || EPL == 16) {
    // the statistics of the streaming kernel, in the same operations
    const BlockStats st = block_stats<EPL>(re, im, lane);
    med_re = st.med_re;
    med_im = st.med_im;
    mad_re = st.mad_re;
    mad_im = st.mad_im;
  } else if constexpr (EPL >= 16) {
    med_re = wave_mom1<EPL, false>(re, 0.f);
    med_im = wave_mom1<EPL, false>(im, 0.f);
    mad_re = wave_mom1<EPL, true>(re, med_re);
    mad_im = wave_mom1<EPL, true>(im, med_im);
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
      Pl[base + (m / K) * (K * PITCH) + (64 / K) * (m % K)] = to_pt<PT>(fmaf(a, a, c * c));
    }
  } else {
#pragma unroll
    for (int m = 0; m < EPL; ++m) {
      const uint32_t t = s0 + lane + 64 * m;
      if (t >= own && t - t0 < need) {
        const float a = fmaf(re[m], inv_re, off_re);
        const float c = fmaf(im[m], inv_im, off_im);
        const float P = fmaf(a, a, c * c);
        Pl[paddr<K>(t - t0)] = to_pt<PT>(P);
        if (P_out && t - t0 < T) glob(P_out)[t] = P;
      }
    }
  }
  if (stats_out && lane == 0 && own >= t0 && own < t0 + T) {
    GLOBAL_AS float *st = glob(stats_out) + 4 * (size_t)b;
    st[0] = med_re;
    st[1] = mad_re;
    st[2] = med_im;
    st[3] = mad_im;
  }
}

// threadIdx.x passed through an empty asm statement.  Each phase of the bank
// kernel derives its lane addresses from its own copy, so the compiler
// recomputes them there instead of keeping them live (and spilled) across
// the whole kernel.
__device__ __forceinline__ uint32_t fresh_tid() {
  uint32_t t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
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

// Canonical FP32 order of a boxcar sum.  A tile is cut into groups of K
// bins (the bins one lane owns).  The window [i, i + w) is summed as
//   Y = hb + t,
// where t adds the bins of the window's last, unfinished group in increasing
// order starting from zero, and hb adds, in order, the partial sum of the
// first group (bins i .. end of i's group, increasing, from zero) and the
// sums of the whole groups in between (each added in increasing order from
// zero, exactly as the K-bin group sums of the pruning bound).  Carried from
// width to width this is the recursion of section 2.2.5 with one extra
// addition: t += P[i + w - 1], Y = hb + t, and when the window ends on a
// group boundary hb = Y, t = 0.  Any width block can be entered from the
// group sums alone, so the exact pass can split one lane's widths over many
// threads; the dense and the pruned routes both use this order and agree bit
// for bit.  (Sums of non-negative terms: every order is within (w-1) u of
// the exact sum, as the recursion's.)

// Starts handled together by one thread: a lane's K starts are taken KS at
// a time, which keeps the running state within the register budget of six
// waves per SIMD.
template <int K>
constexpr int ks_of() {
  return K < 8 ? K : 8;
}

// Load the KS + K - 1 powers P[b0 + k0 + wb + j] (j < KS + K - 1) that the
// starts k0 .. k0+KS-1 of lane L (b0 = L*K) read in width block wb+1 ..
// wb+K.  They lie in lane columns L + wb/K and L + wb/K + 1.
template <int K, typename PT>
__device__ __forceinline__ void load_window(const PT *__restrict__ Pl, uint32_t L, uint32_t wb,
                                            int k0, float (&q)[ks_of<K>() + K - 1]) {
  constexpr int PITCH = pitch_of<K>();
  constexpr int KS = ks_of<K>();
  const uint32_t La = L + wb / K, Lb = La + 1;
  const PT *pa = Pl + (La >> 6) * (K * PITCH) + (La & 63);
  const PT *pb = Pl + (Lb >> 6) * (K * PITCH) + (Lb & 63);
#pragma unroll
  for (int j = 0; j < KS + K - 1; ++j) {
    const int r = k0 + j;  // k0 is a multiple of KS, known at compile time after unrolling
    q[j] = r < K ? (float)pa[r * PITCH] : (float)pb[(r - K) * PITCH];
  }
}

// One width block wb+1 .. wb+K (wb a multiple of K) for starts k0 .. k0+KS-1
// of a lane: q[j] = P[b0 + k0 + wb + j], hb and t the state of those starts
// after width wb.  The maximum over the KS starts of each width is compared
// with the width's threshold Tv[u] and merged into the chunk's slot (larger
// power wins, then the smaller bin).
template <int K, typename TV>
__device__ __forceinline__ void width_block(const float (&q)[ks_of<K>() + K - 1],
                                            float (&hb)[ks_of<K>()], float (&t)[ks_of<K>()],
                                            int k0, const TV &Tv, uint32_t wb, uint32_t zmax,
                                            unsigned long long *slot_row, uint32_t bin0) {
  constexpr int KS = ks_of<K>();
#pragma unroll
  for (int u = 0; u < K; ++u) {
    const int c = K - 1 - u - k0;  // the start whose window ends on a group boundary
    float m = -INFINITY;
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      t[k] += q[k + u];
      const float y = hb[k] + t[k];
      m = fmaxf(m, y);
      if (k == c) {
        hb[k] = y;
        t[k] = 0.f;
      }
    }
    if (m >= Tv[u]) {
      const uint32_t w = wb + u + 1;
      if (w <= zmax) {
        // hb + t is each start's sum again (hb + 0 for the folded start)
        uint32_t kk = KS - 1;
#pragma unroll
        for (int k = KS - 2; k >= 0; --k) kk = (hb[k] + t[k] == m) ? (uint32_t)k : kk;
        const unsigned long long key =
            ((unsigned long long)ord_f32(m) << 32) | (0xFFFFFFFFu - (bin0 + k0 + kk));
        atomicMax(&slot_row[w - 1], key);
      }
    }
  }
}

// The exact bank over one segment of 64*K window starts (segment g of the
// tile), lane l owning starts g*64K + l*K .. +K-1: every width 1..zc in the
// canonical order, with the per-lane maximum, the threshold test and the
// merge into the chunk's slot for every width.
template <int K, typename PT>
__device__ __forceinline__ void bank_dense(const PT *__restrict__ Pl, uint32_t g, uint32_t lane,
                                           const_fptr thr, uint32_t zmax, uint32_t zc,
                                           unsigned long long *slot_row, uint32_t bin0) {
  constexpr int KS = ks_of<K>();
  const uint32_t L = g * 64 + lane;
#pragma unroll
  for (int k0 = 0; k0 < K; k0 += KS) {
    float hb[KS], t[KS], q[KS + K - 1];
#pragma unroll
    for (int k = 0; k < KS; ++k) hb[k] = t[k] = 0.f;
    for (uint32_t wb = 0; wb < zc; wb += K) {
      load_window<K, PT>(Pl, L, wb, k0, q);
      float Tv[K];  // this block's thresholds (scalar loads)
#pragma unroll
      for (int u = 0; u < K; ++u) Tv[u] = thr[wb + u];
      width_block<K>(q, hb, t, k0, Tv, wb, zmax, slot_row, bin0);
    }
  }
}

// Safety factor of the pruning bound.  A sum of m non-negative FP32 terms,
// in any order, is at least (1 - m u) times the exact sum and a width-w FP32
// boxcar at most (1 + w u) times its exact sum (u = 2^-24); for zmax <= 4096
// the ratio of the two stays above 1 - 2^-10, so comparing a union sum with
// T * (1 - 2^-10) never skips a window whose FP32 boxcar reaches T.
constexpr float kBoundSlack = 1.0f - 1.0f / 1024.0f;
// max(v, 0) of a power read from the tile (-inf past the spectrum's end),
// without the quieting of signalling NaNs that fmaxf of a loaded value gets
__device__ __forceinline__ float clamp0(float v) {
  return __builtin_amdgcn_fmed3f(v, 0.f, INFINITY);
}

constexpr int kBoundBatch = 8;  // width blocks per step of the bound's later blocks
constexpr int kSub = 4;  // widths per bound check inside the first width block

// The first width block in which one of this lane's windows might reach its
// threshold, or `nblk` if none can.  Powers are non-negative, so every window
// of width <= w starting at one of the lane's K starts lies in the lane's
// first w + K - 1 bins, whose sum bounds them all.  The first block (widths
// 1..K, the lowest thresholds) is checked every kSub widths, from the lane's
// group sum and the next group's powers; later blocks add one K-bin group
// sum per block.
// CLAMP: the tile holds -inf past the end of the spectrum; count those as 0.
template <int K, bool CLAMP, typename PT>
__device__ __forceinline__ uint32_t bound_lane(const PT *__restrict__ Pl,
                                               const float *__restrict__ Sg, uint32_t g,
                                               uint32_t lane, const float *__restrict__ Tb1,
                                               const float *__restrict__ Tb, uint32_t nblk) {
  constexpr int PITCH = pitch_of<K>();
  constexpr int S = K < kSub ? K : kSub;
  // the first K - 1 bins of the next lane's group
  const uint32_t L1 = lane + 1;
  const PT *bq = Pl + (g + (L1 >> 6)) * (K * PITCH) + (L1 & 63);
  // The lane's own K bins summed from zero in increasing order are its
  // group sum, Sg[own], exactly (the same order, the same clamp); the next
  // group's first K - 1 bins are added to it.  Every load is issued before
  // the sums use them.
  const uint32_t own = g * 64 + lane;
  float v[K > 1 ? K - 1 : 1];
#pragma unroll
  for (int u = 1; u < K; ++u) v[u - 1] = (float)bq[(u - 1) * PITCH];
  float t1[(K + S - 1) / S];
#pragma unroll
  for (int i = 0; i < (K + S - 1) / S; ++i) t1[i] = Tb1[i];
  float U = Sg[own];
  bool hit = false;
#pragma unroll
  for (int u = 0; u < K; ++u) {
    if (u > 0) U += CLAMP ? clamp0(v[u - 1]) : v[u - 1];
    if ((u + 1) % S == 0) hit |= U >= t1[u / S];
  }
  uint32_t fl = hit ? 0u : nblk;
  if (__ballot(fl == nblk) == 0ull) return fl;  // every lane already flagged
  // Whether any later block reaches its threshold: the largest U - Tb[b]
  // (U >= Tb[b] exactly when U - Tb[b] >= 0).  Blocks are taken kBoundBatch
  // at a time with their loads issued together (indices clamped to the last
  // block, whose terms are then not used).
  const float U1 = Sg[own] + Sg[own + 1];
  U = U1;
  float m = -INFINITY;
  for (uint32_t b = 1; b < nblk; b += kBoundBatch) {
    float sg[kBoundBatch], tb[kBoundBatch];
#pragma unroll
    for (int k = 0; k < kBoundBatch; ++k) {
      const uint32_t bb = min(b + k, nblk - 1);
      sg[k] = Sg[own + bb + 1];
      tb[k] = Tb[bb];
    }
#pragma unroll
    for (int k = 0; k < kBoundBatch; ++k) {
      if (b + k < nblk) {
        U += sg[k];
        m = fmaxf(m, U - tb[k]);
      }
    }
  }
  if (fl == nblk && m >= 0.f) {
    // the first such block: the same sums in the same order
    U = U1;
    for (uint32_t b = 1; b < nblk && fl == nblk; b += kBoundBatch) {
      float sg[kBoundBatch], tb[kBoundBatch];
#pragma unroll
      for (int k = 0; k < kBoundBatch; ++k) {
        const uint32_t bb = min(b + k, nblk - 1);
        sg[k] = Sg[own + bb + 1];
        tb[k] = Tb[bb];
      }
#pragma unroll
      for (int k = 0; k < kBoundBatch; ++k) {
        if (b + k < nblk) {
          U += sg[k];
          if (fl == nblk && U >= tb[k]) fl = b + k;
        }
      }
    }
  }
  return fl;
}

// Exact evaluation of width block b (widths bK+1 .. bK+K) for starts
// k0 .. k0+KS-1 of lane L of the tile (bins LK+k0 ..): one work unit of the
// cooperative pass.  The state of the canonical order after width bK is
// rebuilt from the group sums: the window of start s has crossed b group
// boundaries, so hb = H_s + Sg[L+1] + ... + Sg[L+b-1], with H_s the sum of
// bins LK+s .. LK+K-1, and t holds the first s bins of group L+b.  A window
// that already reaches past the spectrum's end (tile bin `rem`) is -inf, as
// the dense route's running sum would be.
template <int K, typename PT>
__device__ __forceinline__ void eval_unit(const PT *__restrict__ Pl,
                                          const float *__restrict__ Sg,
                                          const float *__restrict__ Tl, uint32_t L, uint32_t b,
                                          int k0, uint32_t rem, uint32_t zmax,
                                          unsigned long long *slot_row, uint32_t bin0) {
  constexpr int PITCH = pitch_of<K>();
  constexpr int KS = ks_of<K>();
  float hb[KS], t[KS], q[KS + K - 1];
  if (b == 0) {
#pragma unroll
    for (int k = 0; k < KS; ++k) hb[k] = t[k] = 0.f;
  } else {
    const PT *po = Pl + (L >> 6) * (K * PITCH) + (L & 63);
#pragma unroll
    for (int k = KS - 1; k >= 0; --k) {
      // H_s adds bins s .. K-1 in increasing order from zero
      float a = (float)po[(k0 + k) * PITCH];
#pragma unroll
      for (int v = k0 + k + 1; v < K; ++v) a += (float)po[v * PITCH];
      hb[k] = a;
    }
    for (uint32_t j = 1; j < b; ++j) {
      const float gs = Sg[L + j];
#pragma unroll
      for (int k = 0; k < KS; ++k) hb[k] += gs;
    }
    // t: the first s bins of group L+b, s = k0 + k
    const uint32_t Lg = L + b;
    const PT *pg = Pl + (Lg >> 6) * (K * PITCH) + (Lg & 63);
    float pre = 0.f;
#pragma unroll
    for (int v = 0; v < k0; ++v) pre += (float)pg[v * PITCH];
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      t[k] = pre;
      if (k + 1 < KS) pre += (float)pg[(k0 + k) * PITCH];
    }
#pragma unroll
    for (int k = 0; k < KS; ++k)
      if (L * K + k0 + k + b * K > rem) hb[k] = -INFINITY;
  }
  load_window<K, PT>(Pl, L, b * K, k0, q);
  width_block<K>(q, hb, t, k0, Tl + b * K, b * K, zmax, slot_row, bin0);
}

// Exclusive scan of the per-tile candidate counts by the workgroup of the
// last index, after its own tile (it is dispatched last, so its polls overlap
// the tiles still running; it holds one slot, so every other workgroup can
// still be dispatched while it waits).  Each tile publishes its count as one relaxed 64-bit word
// (kTilePublished | count); a word not yet published is waited for rather
// than fenced, so no tile pays for a device-wide release.  The scan clears
// every word it reads, so the next launch (or graph replay) starts from
// unpublished words without any per-launch tag.  Thread t sums a contiguous
// run of tiles, the run totals are scanned across the workgroup, and each
// thread writes its run's prefixes.  Also records the total and the staging
// overflow, and re-arms the pool head for the next launch.
__device__ __forceinline__ uint32_t tile_count_of(const BankParams &p, uint64_t i, bool &lost) {
  unsigned long long v = 0;
  for (uint32_t k = 0; k < p.spin; ++k) {  // p.spin polls per word before giving up
    v = __hip_atomic_load(p.tile_word + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (v & kTilePublished) return (uint32_t)v;
    __builtin_amdgcn_s_sleep(1);
  }
  lost = true;  // reported through the overflow flag
  return 0u;
}

__device__ void scan_tiles(const BankParams &p, uint32_t tid, uint32_t nthr, uint32_t *wave_sum,
                           uint32_t *lost_any) {
  const uint32_t lane = tid & 63, wave = tid >> 6, nw = nthr >> 6;
  const uint64_t T = p.total_tiles;
  const uint64_t per = (T + nthr - 1) / nthr;
  const uint64_t lo = min((uint64_t)tid * per, T), hi = min(lo + per, T);
  bool lost = false;
  uint32_t mine = 0;
  // the run's first R counts stay in registers; eight independent loads are
  // in flight at a time, and a word not yet published is then waited for on
  // its own
  constexpr int R = 8;
  uint32_t first[R];
  {
    unsigned long long v[R];
#pragma unroll
    for (int k = 0; k < R; ++k)
      v[k] = lo + k < hi ? __hip_atomic_load(p.tile_word + lo + k, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT)
                         : kTilePublished;
#pragma unroll
    for (int k = 0; k < R; ++k) {
      first[k] = (v[k] & kTilePublished) ? (uint32_t)v[k] : tile_count_of(p, lo + k, lost);
      mine += first[k];
    }
  }
  uint64_t i = lo + R;
  for (; i + 8 <= hi; i += 8) {
    unsigned long long v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
      v[k] = __hip_atomic_load(p.tile_word + i + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
    for (int k = 0; k < 8; ++k)
      mine += (v[k] & kTilePublished) ? (uint32_t)v[k] : tile_count_of(p, i + k, lost);
  }
  for (; i < hi; ++i) mine += tile_count_of(p, i, lost);
  if (lost) atomicOr(lost_any, 1u);
  uint32_t incl = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t v = __shfl_up(incl, o, 64);
    if (lane >= (uint32_t)o) incl += v;
  }
  if (lane == 63) wave_sum[wave] = incl;
  __syncthreads();
  uint32_t run = 0, tot = 0;
  for (uint32_t v = 0; v < nw; ++v) {
    run += v < wave ? wave_sum[v] : 0u;
    tot += wave_sum[v];
  }
  run += incl - mine;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    if (lo + k < hi) {
      p.tile_prefix[lo + k] = run;
      run += first[k];
      __hip_atomic_store(p.tile_word + lo + k, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  for (uint64_t j = lo + R; j < hi; ++j) {
    p.tile_prefix[j] = run;
    run += (uint32_t)__hip_atomic_load(p.tile_word + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(p.tile_word + j, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  if (tid == 0) {
    p.tile_prefix[T] = tot;
    const uint32_t ovf = *lost_any ? 2u : (tot > p.pool_cap ? 1u : 0u);
    *p.total = tot;
    if (p.total2) *p.total2 = count_word(tot, ovf);
    *p.overflow = ovf;
    __hip_atomic_store(p.pool_head, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <int EPL>
constexpr int threads_for() {
  return EPL >= 64 ? 256 : kMaxThreads;  // 4096-bin blocks need the whole register file
}
// Waves per SIMD the register allocation must allow: 6 lets three 8-wave
// workgroups share a CU.  The exact median keeps a block's keys in
// registers and settles for four.
template <int EPL, bool EXACT>
constexpr int waves_per_eu_for() {
  return EPL >= 64 ? 1 : EXACT ? 4 : 6;
}

template <int K, int EPL, typename PT, bool EXACT>
__global__ __launch_bounds__(threads_for<EPL>(), (waves_per_eu_for<EPL, EXACT>())) void bank_kernel(
    BankParams p) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ uint32_t wave_sum[kMaxThreads / 64];
  __shared__ uint32_t tile_base;
  __shared__ uint32_t any_dense;
  __shared__ uint32_t n_items;
  __shared__ uint32_t lost_any;
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
  PT *Pl = reinterpret_cast<PT *>(items + T / K);

  // One tile per workgroup, in index order.  (Workgroups are dealt
  // round-robin to the 8 XCDs, so neighbouring tiles run on different XCDs
  // and spread their reads over all of them; giving each XCD a contiguous
  // run of tiles, so that a tile's halo block is read through the L2 that
  // read it for its neighbour, measured slower.)
  const uint64_t first_tile = blockIdx.x;

  if (first_tile >= p.total_tiles) return;
  {
    const uint64_t tg = first_tile;
    int sidx = 0;
    if (p.nspec > 1) {
      int lo = 0, hi = p.nspec - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (glob(p.descs)[mid].tile_begin <= tg)
          lo = mid;
        else
          hi = mid - 1;
      }
      sidx = lo;
    }
    const SpecDesc d = p.nspec > 1 ? load_desc(p.descs + sidx) : p.single;
    const uint32_t t0 = (uint32_t)(tg - d.tile_begin) * T;
    const uint32_t n = d.n, zmax = d.zmax, zc = d.zc;
    const uint32_t rem = n - t0;
    const bool power_only = p.mode == kModePower;
    const uint32_t need = min(power_only ? T : T + zmax - 1, rem);
    const uint32_t nblk = zc / K;
    const uint32_t span = T + zc;  // tile bins the bank and the bound read
    const uint32_t bfirst = t0 / B, blast = (t0 + need - 1) / B;

    // --- set-up and power --------------------------------------------------
    // the wave's first block is requested before the rest of the set-up so
    // that its memory latency overlaps it
    {
    const uint32_t tid = fresh_tid(), lane = tid & 63, wave = tid >> 6;
    BlockData<EPL> bd;
    const bool have = !p.from_power && bfirst + wave <= blast;
    // the thresholds (one per thread) are requested with the block; the
    // bound's minima of them come later from LDS, so the set-up makes no
    // further round trip to memory
    const GLOBAL_AS float *gthr = glob(d.thr);
    const float thr_own = !power_only && tid < zc ? gthr[tid] : 0.f;
    if (have) load_block<EPL>(d.x, n, bfirst + wave, lane, bd);
    if (tid == 0) {
      any_dense = 0u;
      n_items = 0u;
    }
    if (!power_only) {
    // the pruned search clears the slots only once it has work items
    if (p.dense || p.mode == kModeTables)
      for (uint32_t i = tid; i < chunks_per_tile * zmax; i += nthr) slots[i] = 0ull;
    if (tid < zc) Tl[tid] = thr_own;
    for (uint32_t i = tid + nthr; i < zc; i += nthr) Tl[i] = gthr[i];
    }
    // bins past the spectrum's end are -inf (no window may contain them);
    // halo bins beyond what any width <= zmax reads are 0 (read only by the
    // unrecorded widths zmax+1..zc and by the pruning bound)
    for (uint32_t i = need + tid; i < span; i += nthr)
      Pl[paddr<K>(i)] = to_pt<PT>(i < rem ? 0.f : -INFINITY);
    if (p.from_power) {
      const float *pw = reinterpret_cast<const float *>(d.x);
      for (uint32_t i = tid; i < need; i += nthr) Pl[paddr<K>(i)] = to_pt<PT>(glob(pw)[t0 + i]);
    } else if (have) {
      const bool dbg = p.mode == kModeTables;
      float *po = power_only ? d.aux : dbg ? p.P_out : nullptr;
      // the half-precision search keeps every block's statistics for its
      // FP32 re-check of candidates near the threshold
      float *so = dbg ? p.stats_out : (p.mode == kModeSearch && sizeof(PT) == 2) ? d.aux : nullptr;
      for (uint32_t b = bfirst + wave; b <= blast; b += nw) {
        if (b != bfirst + wave) load_block<EPL>(d.x, n, b, lane, bd);
        normalise_block<K, EPL, PT, EXACT>(bd, b, t0, need, T, Pl, lane, po, so);
      }
    }
    }
    if (power_only) return;  // the power is written; nothing else to do
    __syncthreads();

    // --- bank ----------------------------------------------------------------
    const bool prune = !p.dense && p.mode != kModeTables;
    const bool clamp = rem < span;
    if (prune) {
      const uint32_t tid = fresh_tid();
      // K-bin group sums of the whole span (inputs of the pruning bound)
      const uint32_t ngroups = span / K;
      for (uint32_t j = tid; j < ngroups; j += nthr) {
        const PT *cp = Pl + (j >> 6) * (K * PITCH) + (j & 63);
        float a = 0.f;
        if (clamp) {
#pragma unroll
          for (int v = 0; v < K; ++v) a += clamp0((float)cp[v * PITCH]);
        } else {
#pragma unroll
          for (int v = 0; v < K; ++v) a += (float)cp[v * PITCH];
        }
        Sg[j] = a;
      }
      // the bound's thresholds: minima of the width thresholds (in LDS since
      // the set-up) over the first block's sub-blocks and over each block
      if (tid < 4) {
        constexpr int S = K < kSub ? K : kSub;
        float m = INFINITY;
        if (tid * S < (uint32_t)K)
          for (int u = 0; u < S; ++u) m = fminf(m, Tl[tid * S + u]);
        Tb1[tid] = m * kBoundSlack;
      }
      for (uint32_t i = tid; i < nblk; i += nthr) {
        float m = Tl[i * K];
        for (int u = 1; u < K; ++u) m = fminf(m, Tl[i * K + u]);
        Tb[i] = m * kBoundSlack;
      }
      __syncthreads();
    }
    const uint32_t nseg_tile = T / SEG;
    const const_fptr thr = uniform_const(d.thr);
    if (prune) {
      {
      const uint32_t tid = fresh_tid(), lane = tid & 63, wave = tid >> 6;
      // each lane's first width block that might reach a threshold; the
      // flagged lanes become work items of a cooperative exact pass
      for (uint32_t g = wave; g < nseg_tile; g += nw) {
        if (g * SEG >= rem) break;
        const uint32_t fl = clamp ? bound_lane<K, true, PT>(Pl, Sg, g, lane, Tb1, Tb, nblk)
                                  : bound_lane<K, false, PT>(Pl, Sg, g, lane, Tb1, Tb, nblk);
        const unsigned long long mask = __ballot(fl < nblk);
        if (mask) {
          uint32_t base = 0;
          if (lane == 0) base = atomicAdd(&n_items, (uint32_t)__popcll(mask));
          base = __shfl(base, 0, 64);
          if (fl < nblk)
            items[base + __popcll(mask & ((1ull << lane) - 1ull))] = ((g * 64 + lane) << 12) | fl;
        }
      }
      }
      __syncthreads();
      if (n_items) {
        const uint32_t tid = fresh_tid();
        for (uint32_t i = tid; i < chunks_per_tile * zmax; i += nthr) slots[i] = 0ull;
        __syncthreads();
      }
    }
    // With more than a quarter of its lanes flagged (a power series of many
    // degrees of freedom per bin, such as a harmonic stage, whose thresholds
    // sit close to its mean: the union windows reach them everywhere) the
    // tile takes the dense route, which evaluates every lane in the same
    // canonical order faster than per-lane work units.
    if (prune && n_items * 4u <= T / K) {
      // work units (flagged lane, width block, half of the lane's starts).
      // The (lane, block) pairs are lane-major, so that the lanes of a wave
      // share lanes' chunks but not widths and their slot merges rarely
      // collide; every 64 pairs are taken once per half by whole waves, so
      // that a wave runs one half's code only.
      const uint32_t tid = fresh_tid();
      const uint32_t nb = (zmax + K - 1) / K;
      constexpr uint32_t NH = K / ks_of<K>();  // start groups per lane
      const uint32_t npairs = n_items * nb;
      const uint32_t nrun = (npairs + 63) / 64 * 64 * NH;
      if (tid == 0 && npairs) any_dense = 1u;
      for (uint32_t r = 0; r < nrun; r += nthr) {
        const uint32_t j = r + tid;
        const uint32_t grp = j >> 6, half = grp % NH;
        const uint32_t u = (grp / NH) * 64 + (j & 63);
        const bool ok = j < nrun && u < npairs;
        const uint32_t it = ok ? items[u / nb] : 0u;
        const uint32_t b = ok ? u % nb : 0u;
        if (ok && b >= (it & 0xFFFu)) {
          const uint32_t L = it >> 12;
          unsigned long long *row = slots + (size_t)((L * K) / C) * zmax;
          if (NH == 1 || half == 0)
            eval_unit<K, PT>(Pl, Sg, Tl, L, b, 0, rem, zmax, row, t0 + L * K);
          else
            eval_unit<K, PT>(Pl, Sg, Tl, L, b, ks_of<K>(), rem, zmax, row, t0 + L * K);
        }
      }
    } else {
      const uint32_t tid = fresh_tid(), lane = tid & 63, wave = tid >> 6;
      for (uint32_t g = wave; g < nseg_tile; g += nw) {
        const uint32_t seg0 = g * SEG;
        if (seg0 >= rem) break;
        any_dense = 1u;
        bank_dense<K, PT>(Pl, g, lane, thr, zmax, zc, slots + (size_t)(seg0 / C) * zmax,
                      t0 + seg0 + lane * K);
      }
    }
    __syncthreads();

    {
    const uint32_t tid = fresh_tid(), lane = tid & 63, wave = tid >> 6;
    // --- extraction ----------------------------------------------------------
    const uint32_t chunk0 = t0 / C;
    const uint32_t nch = min(chunks_per_tile, d.nchunks - chunk0);
    const uint32_t nsl = nch * zmax;
    // the workgroup of the last index scans the per-tile counts
    const bool scanner = p.scan_in_kernel && blockIdx.x == gridDim.x - 1;
    if (p.mode == kModeSearch && !any_dense) {
      // nothing was evaluated, so nothing reached a threshold
      if (tid == 0) {
        __hip_atomic_store(p.tile_word + tg, kTilePublished, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        lost_any = 0u;
      }
      if (scanner) {
        __syncthreads();
        scan_tiles(p, tid, nthr, wave_sum, &lost_any);
      }
    } else if (p.mode == kModeSearch) {
      // stage the tile's maxima in slot order, i.e. (chunk, width) order:
      // thread t takes a contiguous run of slots; ranks come from a scan of
      // the run counts, one atomic reserves the tile's run of the pool
      const uint32_t per = (nsl + nthr - 1) / nthr;
      const uint32_t lo = min(tid * per, nsl), hi = min(lo + per, nsl);
      uint32_t mine = 0;
      for (uint32_t i = lo; i < hi; ++i) mine += slots[i] != 0ull ? 1u : 0u;
      uint32_t incl = mine;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t v = __shfl_up(incl, o, 64);
        if (lane >= (uint32_t)o) incl += v;
      }
      if (lane == 63) wave_sum[wave] = incl;
      __syncthreads();
      uint32_t before = 0, tot = 0;
      for (uint32_t v = 0; v < nw; ++v) {
        before += v < wave ? wave_sum[v] : 0u;
        tot += wave_sum[v];
      }
      if (tid == 0) {
        tile_base = tot ? atomicAdd(p.pool_head, tot) : 0u;
        // the pool reservation has been performed before the count is
        // published, so the scan (which waits for every count) may re-arm
        // the pool head
        __builtin_amdgcn_s_waitcnt(0);
        __hip_atomic_store(p.tile_word + tg, kTilePublished | tot, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        lost_any = 0u;
      }
      __syncthreads();
      uint32_t rank = before + incl - mine;
      for (uint32_t i = lo; i < hi; ++i) {
        const unsigned long long key = slots[i];
        if (key == 0ull) continue;
        const uint32_t pos = tile_base + rank;
        if (pos < p.pool_cap) {
          const uint32_t cl = i / zmax, w = i - cl * zmax + 1;
          StageEntry e;
          e.unit = (uint32_t)tg;
          e.rank = rank;
          e.spec = (uint32_t)sidx;
          e.bin = 0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull);
          e.power = unord_f32((uint32_t)(key >> 32));
          e.width = w;
          p.pool[pos] = e;
        }
        ++rank;
      }
      if (scanner) scan_tiles(p, tid, nthr, wave_sum, &lost_any);
    } else {
      for (uint32_t i = tid; i < nsl; i += nthr) {
        const unsigned long long key = slots[i];
        const size_t o = (size_t)chunk0 * zmax + i;
        p.M[o] = key ? unord_f32((uint32_t)(key >> 32)) : -INFINITY;
        p.I[o] = key ? 0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull) : 0xFFFFFFFFu;
      }
    }
    }
    __syncthreads();
  }
}

template <int K>
static size_t lds_need_k(uint32_t T, uint32_t C, uint32_t zmax_max, uint32_t *nseg,
                         uint32_t *zc_pad, uint32_t pbytes) {
  const uint32_t zc = round_widths(zmax_max, K);
  const uint32_t segb = 64u * (uint32_t)K;
  *nseg = (T + zc + segb - 1) / segb;
  *zc_pad = (zc + 3) / 4 * 4;
  return (size_t)(T / C) * zmax_max * 8u              // slots
         + (size_t)(*zc_pad) * 4u                     // thresholds
         + (4 + (size_t)(*zc_pad) / K + 4) * 4u       // bound thresholds
         + (size_t)(*nseg) * 64u * 4u                 // group sums
         + (size_t)(T / K) * 4u                       // cooperative work items
         + (size_t)(*nseg) * K * pitch_of<K>() * pbytes;  // power tile
}

static size_t lds_need(int K, uint32_t T, uint32_t C, uint32_t zmax_max, uint32_t *nseg,
                       uint32_t *zc_pad, uint32_t pbytes) {
  switch (K) {
    case 1: return lds_need_k<1>(T, C, zmax_max, nseg, zc_pad, pbytes);
    case 2: return lds_need_k<2>(T, C, zmax_max, nseg, zc_pad, pbytes);
    case 4: return lds_need_k<4>(T, C, zmax_max, nseg, zc_pad, pbytes);
    case 8: return lds_need_k<8>(T, C, zmax_max, nseg, zc_pad, pbytes);
    default: return lds_need_k<16>(T, C, zmax_max, nseg, zc_pad, pbytes);
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

constexpr size_t kLdsBudget = 64 * 1024;     // per workgroup
constexpr size_t kLdsPreferred = 53 * 1024;  // three workgroups share a CU's 160 KiB
constexpr uint32_t kMaxWaves = 8;

bool choose_geometry(uint32_t C, uint32_t B, uint32_t zmax_max, uint64_t n_hint, Geometry *g,
                     uint32_t tile, bool fp16) {
  const uint32_t pb = fp16 ? 2u : 4u;
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
  // wave one block, that leaves room for three workgroups per CU (the
  // smallest tile may use up to the per-workgroup budget) and enough tiles
  // to fill the GPU
  uint64_t T = 0;
  if (tile) {
    // a tile asked for (by the autotuner): it must be a multiple of L0 that
    // fits the wave and LDS limits
    if (tile % L0 != 0 || tile > (uint64_t)kMaxTile) return false;
    if (tile / B + halo > wmax && tile > L0) return false;
    if (lds_need(K, tile, C, zmax_max, &nseg, &zcp, pb) > kLdsBudget) return false;
    T = tile;
  }
  for (uint64_t t = L0; !tile && t <= (uint64_t)kMaxTile; t += L0) {
    if (t / B + halo > wmax && t > L0) break;
    const size_t lds = lds_need(K, (uint32_t)t, C, zmax_max, &nseg, &zcp, pb);
    if (lds > kLdsBudget || (lds > kLdsPreferred && t > L0)) break;
    if (t > L0 && n_hint / t < 256) break;
    T = t;
  }
  if (T == 0) return false;
  g->K = K;
  g->EPL = (int)(B / 64);
  uint32_t nw = (uint32_t)(T / B) + halo;
  g->waves = (int)(nw < 1 ? 1 : (nw > wmax ? wmax : nw));
  g->tile = (uint32_t)T;
  g->lds_bytes = lds_need(K, g->tile, C, zmax_max, &nseg, &zcp, pb);
  g->fp16 = fp16;
  g->nseg_lds = nseg;
  g->zc_max_pad = zcp;
  return true;
}

// Tiles the kernels can run for chunk C, block B and zmax_max: the multiples
// of the smallest legal tile that fit the wave and LDS limits.
std::vector<uint32_t> tile_choices(uint32_t C, uint32_t B, uint32_t zmax_max, bool fp16) {
  std::vector<uint32_t> out;
  Geometry g;
  if (!choose_geometry(C, B, zmax_max, ~0ull, &g, 0, fp16)) return out;
  const uint64_t L0 = lcm_u(lcm_u(C, B), 64ull * g.K);
  for (uint64_t t = L0; t <= (uint64_t)kMaxTile; t += L0) {
    Geometry h;
    if (!choose_geometry(C, B, zmax_max, ~0ull, &h, (uint32_t)t, fp16)) break;
    out.push_back((uint32_t)t);
  }
  return out;
}

template <int K, typename PT, bool EXACT>
static hipError_t launch_k(int EPL, uint64_t grid, uint32_t threads, size_t lds,
                           const BankParams &p, hipStream_t stream) {
  const dim3 gd((uint32_t)grid), bd(threads);
  switch (EPL) {
    case 1: hipLaunchKernelGGL((bank_kernel<K, 1, PT, EXACT>), gd, bd, lds, stream, p); break;
    case 4: hipLaunchKernelGGL((bank_kernel<K, 4, PT, EXACT>), gd, bd, lds, stream, p); break;
    case 16: hipLaunchKernelGGL((bank_kernel<K, 16, PT, EXACT>), gd, bd, lds, stream, p); break;
    case 64:
      // 4096-bin blocks: FP32 power and the median of medians only
      if (sizeof(PT) != 4 || EXACT) return hipErrorInvalidValue;
      hipLaunchKernelGGL((bank_kernel<K, 64, float, false>), gd, bd, lds, stream, p);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int K>
static hipError_t launch_pt(const Geometry &g, const BankParams &p, uint64_t grid,
                            uint32_t threads, hipStream_t stream) {
  if (p.norm_exact) {
    // the exact median keeps FP32 power
    if (g.fp16) return hipErrorInvalidValue;
    return launch_k<K, float, true>(g.EPL, grid, threads, g.lds_bytes, p, stream);
  }
  return g.fp16 ? launch_k<K, _Float16, false>(g.EPL, grid, threads, g.lds_bytes, p, stream)
                : launch_k<K, float, false>(g.EPL, grid, threads, g.lds_bytes, p, stream);
}

hipError_t launch_bank(const Geometry &g, const BankParams &p, uint64_t grid, hipStream_t stream) {
  if (grid == 0) return hipSuccess;
  const uint32_t threads = 64u * (uint32_t)g.waves;
  switch (g.K) {
    case 1: return launch_pt<1>(g, p, grid, threads, stream);
    case 2: return launch_pt<2>(g, p, grid, threads, stream);
    case 4: return launch_pt<4>(g, p, grid, threads, stream);
    case 8: return launch_pt<8>(g, p, grid, threads, stream);
    case 16: return launch_pt<16>(g, p, grid, threads, stream);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// Two-level scan of the per-tile counts of launches with many tiles.

constexpr int kBigThreads = 512;

__global__ __launch_bounds__(kBigThreads) void scan_span_kernel(BigScan s) {
  __shared__ uint32_t wave_sum[kBigThreads / 64];
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t base = (uint64_t)blockIdx.x * kScanSpan;
  constexpr uint32_t PER = kScanSpan / kBigThreads;
  uint32_t v[PER];
  uint32_t mine = 0;
#pragma unroll
  for (uint32_t k = 0; k < PER; ++k) {
    const uint64_t i = base + (uint64_t)tid * PER + k;
    uint32_t c = 0;
    if (i < s.total_tiles) {
      const unsigned long long w = s.tile_word[i];  // written by the previous kernel
      c = (uint32_t)w;
      if (!(w & kTilePublished)) atomicOr(s.lost, 1u);
      s.tile_word[i] = 0ull;
    }
    v[k] = c;
    mine += c;
  }
  uint32_t incl = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(incl, o, 64);
    if (lane >= (uint32_t)o) incl += t;
  }
  if (lane == 63) wave_sum[wave] = incl;
  __syncthreads();
  uint32_t run = 0, tot = 0;
  for (uint32_t w = 0; w < kBigThreads / 64; ++w) {
    run += w < wave ? wave_sum[w] : 0u;
    tot += wave_sum[w];
  }
  run += incl - mine;
#pragma unroll
  for (uint32_t k = 0; k < PER; ++k) {
    const uint64_t i = base + (uint64_t)tid * PER + k;
    if (i < s.total_tiles) s.tile_prefix[i] = run;
    run += v[k];
  }
  if (tid == 0) s.span_sum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kBigThreads) void scan_top_kernel(BigScan s, uint32_t nspan) {
  __shared__ uint32_t wave_sum[kBigThreads / 64];
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  uint32_t carry = 0;
  for (uint32_t b0 = 0; b0 < nspan; b0 += kBigThreads) {
    const uint32_t i = b0 + tid;
    const uint32_t v = i < nspan ? s.span_sum[i] : 0u;
    uint32_t incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t t = __shfl_up(incl, o, 64);
      if (lane >= (uint32_t)o) incl += t;
    }
    if (lane == 63) wave_sum[wave] = incl;
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (uint32_t w = 0; w < kBigThreads / 64; ++w) {
      before += w < wave ? wave_sum[w] : 0u;
      tot += wave_sum[w];
    }
    if (i < nspan) s.span_prefix[i] = carry + before + incl - v;
    carry += tot;
    __syncthreads();
  }
  if (tid == 0) {
    const uint32_t ovf = *s.lost ? 2u : (carry > s.pool_cap ? 1u : 0u);
    *s.total = carry;
    if (s.total2) *s.total2 = count_word(carry, ovf);
    *s.overflow = ovf;
    *s.lost = 0u;
    *s.pool_head = 0u;
  }
}

hipError_t launch_scan_big(const BigScan &s, hipStream_t stream) {
  const uint32_t nspan = (uint32_t)((s.total_tiles + kScanSpan - 1) / kScanSpan);
  hipLaunchKernelGGL(scan_span_kernel, dim3(nspan), dim3(kBigThreads), 0, stream, s);
  hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(kBigThreads), 0, stream, s, nspan);
  return hipGetLastError();
}

}  // namespace pulscan

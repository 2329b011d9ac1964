// Median-of-medians block statistics (section 2.2.3; section 2.5 and the
// appendix algorithm "Median of Medians Normalisation") shared by the two
// bank kernels, which must normalise with the same bits.  One wave holds a
// block of 64*EPL values, lane l holding elements l + 64m: the first levels
// of the median-of-4 tree (strides B/4 .. 64) stay inside a lane, the last
// three (16, 4 and 1 lanes) cross lanes, two trees (the real and imaginary
// parts) at a time through one set of lane permutations and DPP min/max
// operations.  Translation units that include this are built without NaN
// semantics, so that min/max of three values and the DPP row shifts fold
// into single instructions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pulscan {

// Twice the median of four values, i.e. the sum of the middle two.  With m
// the median of a, b, c and lo, hi their minimum and maximum, adding d
// leaves {m, median(lo, d, hi)} as the middle pair, so the result is one
// rounding of the sum of the same two values however they are picked.
// Carrying the factor 2 through the tree and removing it with one exact
// power-of-two scale at the end rounds exactly as halving at every level
// would.  Inputs are finite; built without NaN semantics the minimum and
// maximum of three become one v_min3 / v_max3 each (five VALU operations).
__device__ __forceinline__ float m4x2(float a, float b, float c, float d) {
  const float m = __builtin_amdgcn_fmed3f(a, b, c);
  const float lo = fminf(fminf(a, b), c), hi = fmaxf(fmaxf(a, b), c);
  return m + __builtin_amdgcn_fmed3f(lo, d, hi);
}

template <int CTRL>
__device__ __forceinline__ float sdpp(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, true));
}

// Inside each row of 16 lanes, lane l (for the lanes used) receives twice the
// median of x[l], x[l+S], x[l+2S], x[l+3S], as max(min(a, b), min(c, d)) +
// min(max(a, b), max(c, d)): the same two middle values as m4x2, so the same
// bits.  The row shifts fold into the min/max instructions.
template <int S>
__device__ __forceinline__ float row_m4x2(float x) {
  constexpr int C1 = 0x100 + S, C2 = 0x100 + 2 * S;
  const float lo = fminf(x, sdpp<C1>(x)), hi = fmaxf(x, sdpp<C1>(x));
  return fmaxf(lo, sdpp<C2>(lo)) + fminf(hi, sdpp<C2>(hi));
}

// The three cross-lane levels of two trees at once.  x holds tree A's 64
// values, y tree B's; the level over lanes l, l+16, l+32, l+48 regroups the
// values so that row 0 holds tree A's pairs (l, l+16) and row 1 its pairs
// (l+32, l+48), rows 2 and 3 tree B's, and finishes with one exchange of
// rows; the next two levels then run on rows 0 and 2 together.  Returns the
// wave-uniform results (each doubled at every level).
__device__ __forceinline__ void cross2(float x, float y, uint32_t lane, float &ra, float &rb) {
  const auto s1 = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false,
                                                   false);
  // rows: [A0-15, A16-31, B0-15, B16-31] and [A32-47, A48-63, B32-47, B48-63]
  const auto s2 = __builtin_amdgcn_permlane16_swap(s1[0], s1[1], false, false);
  // rows: [A0-15, A32-47, B0-15, B32-47] and [A16-31, A48-63, B16-31, B48-63]
  const float p = __uint_as_float(s2[0]), q = __uint_as_float(s2[1]);
  const float lo = fminf(p, q), hi = fmaxf(p, q);
  const auto s3 = __builtin_amdgcn_permlane16_swap(__float_as_uint(lo), __float_as_uint(hi), false,
                                                   false);
  // even rows: own low and the odd row's low; odd rows: the even row's high
  // and own high
  const float u = __uint_as_float(s3[0]), v = __uint_as_float(s3[1]);
  const float z = (lane & 16) ? fminf(u, v) : fmaxf(u, v);
  const auto s4 = __builtin_amdgcn_permlane16_swap(__float_as_uint(z), __float_as_uint(z), false,
                                                   false);
  float w = z + __uint_as_float(s4[1]);
  w = row_m4x2<4>(w);
  w = row_m4x2<1>(w);
  ra = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(w), 0));
  rb = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(w), 32));
}

// The in-lane levels of one tree over the lane's EPL values (or, with DEV,
// their distances |x - c| from c), doubled at each level.
template <int EPL, bool DEV>
__device__ __forceinline__ float lane_tree(const float (&v)[EPL], float c) {
  auto f = [c](float x) { return DEV ? fabsf(x - c) : x; };
  if constexpr (EPL == 4) {
    return m4x2(f(v[0]), f(v[1]), f(v[2]), f(v[3]));
  } else {
    float t[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) t[m] = m4x2(f(v[m]), f(v[m + 4]), f(v[m + 8]), f(v[m + 12]));
    return m4x2(t[0], t[1], t[2], t[3]);
  }
}

struct BlockStats {
  float med_re, mad_re, med_im, mad_im;
};

// Median-of-medians statistics of a block held as re[m], im[m] = element
// lane + 64m: the medians, then the medians of the distances from them.
template <int EPL>
__device__ __forceinline__ BlockStats block_stats(const float (&re)[EPL], const float (&im)[EPL],
                                                  uint32_t lane) {
  // log4(EPL) in-lane levels and three cross-lane levels, each doubling
  constexpr float scale = EPL == 16 ? 1.0f / 32.0f : 1.0f / 16.0f;
  BlockStats s;
  float a, b;
  cross2(lane_tree<EPL, false>(re, 0.f), lane_tree<EPL, false>(im, 0.f), lane, a, b);
  s.med_re = a * scale;
  s.med_im = b * scale;
  cross2(lane_tree<EPL, true>(re, s.med_re), lane_tree<EPL, true>(im, s.med_im), lane, a, b);
  s.mad_re = a * scale;
  s.mad_im = b * scale;
  return s;
}


}  // namespace pulscan

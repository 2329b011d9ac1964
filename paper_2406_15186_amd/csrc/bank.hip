// The fused boxcar-bank kernel: one pass over each tile of a spectrum does
// normalisation, power, the boxcar bank of every width and the per-chunk
// maxima with the threshold test.
//
//  * Normalisation (section 2.2.3; section 2.5 and the appendix algorithm
//    "Median of Medians Normalisation"): one wave per block of B = 64*EPL bins.
//    Lane l holds elements l + 64m, so the first levels of the median-of-4
//    tree (strides B/4, B/16, ... down to 64) stay inside a lane and the last
//    three (16, 4, 1) cross lanes.
//  * Power (section 2.2.3): re'^2 + im'^2, written to LDS only.  The tile
//    holds its T bins plus a halo of up to zmax - 1 bins from the next blocks
//    (normalised with those blocks' own statistics).
//  * Bank (section 2.2.5): each lane owns K consecutive window starts and
//    keeps their running sums Y_w = Y_{w-1} + P[i+w-1] in registers while w
//    steps through 1..zmax; the powers come from LDS, K per K widths.
//  * Per-chunk maxima (appendix algorithm "Boxcar Filtering Process"): a lane
//    compares the maximum of its K sums with the width's threshold; in the
//    rare case it reaches it, the lane finds its first bin attaining that
//    maximum and merges (power, bin) into the chunk's LDS slot for the width
//    with one 64-bit atomic max (larger power wins, then the smaller bin).
//    Without a threshold (tables mode) every maximum is merged.
//  * Extraction: non-empty slots are compacted (ballot + popcount) into the
//    spectrum's staging area; a separate pass orders them.
#include <float.h>

#include "internal.hpp"

namespace pulscan {

__device__ __forceinline__ float med4f(float a, float b, float c, float d) {
  // the two middle values of four are max(min(a,b), min(c,d)) and
  // min(max(a,b), max(c,d)); the median is their mean
  const float lo = fmaxf(fminf(a, b), fminf(c, d));
  const float hi = fminf(fmaxf(a, b), fmaxf(c, d));
  return (lo + hi) * 0.5f;
}

// Median of medians of the 64*EPL values of one wave, lane l holding
// element l + 64m in v[m].  v is consumed.  Every lane gets the result.
template <int EPL>
__device__ __forceinline__ float wave_mom(float (&v)[EPL]) {
#pragma unroll
  for (int cnt = EPL; cnt >= 4; cnt /= 4) {
    const int q = cnt / 4;
#pragma unroll
    for (int m = 0; m < q; ++m) v[m] = med4f(v[m], v[m + q], v[m + 2 * q], v[m + 3 * q]);
  }
  float x = v[0];
#pragma unroll
  for (int s = 16; s >= 1; s /= 4) {
    const float b = __shfl_down(x, s, 64);
    const float c = __shfl_down(x, 2 * s, 64);
    const float d = __shfl_down(x, 3 * s, 64);
    x = med4f(x, b, c, d);
  }
  return __shfl(x, 0, 64);
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
// K x 65 array, so the 64 lanes of a wave reading "their" j-th bin hit 64
// consecutive words.
template <int K>
__device__ __forceinline__ uint32_t paddr(uint32_t i) {
  constexpr uint32_t SEG = 64 * K;
  const uint32_t g = i / SEG, r = i % SEG;
  return g * (K * kRowPitch) + (r % K) * kRowPitch + r / K;
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

// Normalise block b of the spectrum and write its power into the tile's LDS
// array for every bin of the block that the tile needs (tile-relative index
// below `need`).  Executed by one whole wave.
template <int K, int EPL>
__device__ __forceinline__ void normalise_block(const float2 *__restrict__ x, uint32_t n, uint32_t b,
                                                uint32_t t0, uint32_t need, uint32_t T, float *Pl,
                                                uint32_t lane, float *P_out, float *stats_out) {
  constexpr uint32_t B = 64 * EPL;
  uint32_t s0 = b * B;
  if (s0 + B > n) s0 = n - B;  // the last, partial block uses the last B bins
  float re[EPL], im[EPL], w[EPL];
#pragma unroll
  for (int m = 0; m < EPL; ++m) {
    const float2 v = x[s0 + lane + 64 * m];
    re[m] = v.x;
    im[m] = v.y;
  }
#pragma unroll
  for (int m = 0; m < EPL; ++m) w[m] = re[m];
  const float med_re = wave_mom<EPL>(w);
#pragma unroll
  for (int m = 0; m < EPL; ++m) w[m] = fabsf(re[m] - med_re);
  const float mad_re = wave_mom<EPL>(w);
#pragma unroll
  for (int m = 0; m < EPL; ++m) w[m] = im[m];
  const float med_im = wave_mom<EPL>(w);
#pragma unroll
  for (int m = 0; m < EPL; ++m) w[m] = fabsf(im[m] - med_im);
  const float mad_im = wave_mom<EPL>(w);
  const float inv_re = mad_re > 0.f ? 1.0f / (mad_re * kMadScale) : 0.f;
  const float inv_im = mad_im > 0.f ? 1.0f / (mad_im * kMadScale) : 0.f;
  const uint32_t own = b * B;
#pragma unroll
  for (int m = 0; m < EPL; ++m) {
    const uint32_t t = s0 + lane + 64 * m;
    if (t >= own && t - t0 < need) {
      const float a = (re[m] - med_re) * inv_re;
      const float c = (im[m] - med_im) * inv_im;
      const float P = fmaf(a, a, c * c);
      Pl[paddr<K>(t - t0)] = P;
      if (P_out && t - t0 < T) P_out[t] = P;
    }
  }
  if (stats_out && lane == 0 && own >= t0 && own < t0 + T) {
    stats_out[4 * (size_t)b + 0] = med_re;
    stats_out[4 * (size_t)b + 1] = mad_re;
    stats_out[4 * (size_t)b + 2] = med_im;
    stats_out[4 * (size_t)b + 3] = mad_im;
  }
}

// The bank over one segment of 64*K window starts (segment g of the tile),
// lane l owning starts g*64K + l*K .. +K-1.  slot_row points at the chunk's
// slots (zmax entries); bin0 is the spectrum bin of the lane's first start.
template <int K>
__device__ __forceinline__ void bank_segment(const float *__restrict__ Pl, uint32_t g,
                                             uint32_t lane, const float *__restrict__ Tl,
                                             uint32_t zmax, uint32_t zc,
                                             unsigned long long *slot_row, uint32_t bin0) {
  float s[K], q[2 * K];
#pragma unroll
  for (int k = 0; k < K; ++k) s[k] = 0.f;
  {
    const float *bp = Pl + g * (K * kRowPitch) + lane;
#pragma unroll
    for (int v = 0; v < K; ++v) q[v] = bp[v * kRowPitch];
  }
  for (uint32_t wb = 0; wb < zc; wb += K) {
    // q[j] = P[start + wb + j], j < 2K: fetch the upper half
    {
      const uint32_t L = lane + wb / K + 1;
      const float *bp = Pl + (g + (L >> 6)) * (K * kRowPitch) + (L & 63);
#pragma unroll
      for (int v = 0; v < K; ++v) q[K + v] = bp[v * kRowPitch];
    }
    float Tv[K];  // this block's thresholds (same LDS word for every lane)
#pragma unroll
    for (int u = 0; u < K; ++u) Tv[u] = Tl[wb + u];
#pragma unroll
    for (int u = 0; u < K; ++u) {
#pragma unroll
      for (int k = 0; k < K; ++k) s[k] += q[k + u];  // width wb+u+1
      const float m = max_of<K>(s);
      const float Tw = Tv[u];
      if (m >= Tw) {
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
#pragma unroll
    for (int v = 0; v < K; ++v) q[v] = q[K + v];
  }
}

template <int K, int EPL>
__global__ __launch_bounds__(kThreads) void bank_kernel(BankParams p) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ uint32_t wave_sum[kWaves];
  __shared__ uint32_t tile_base;
  constexpr uint32_t SEG = 64 * K;
  constexpr uint32_t B = 64 * EPL;
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t T = p.tile, C = p.chunk;
  const uint32_t chunks_per_tile = T / C;
  // LDS: slots (chunks_per_tile x zmax_max, 64-bit) | thresholds (zc_max) | power tile
  unsigned long long *slots = reinterpret_cast<unsigned long long *>(lds_raw);
  float *Tl = reinterpret_cast<float *>(slots + (size_t)chunks_per_tile * p.zmax_max);
  float *Pl = Tl + p.zc_max_pad;
  const uint32_t plen = p.nseg_lds * K * kRowPitch;

  // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a
  // contiguous run of tiles so the halo a tile shares with its neighbour is
  // read through the same L2.
  uint64_t first = blockIdx.x;
  if ((gridDim.x & 7) == 0) first = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);

  for (uint64_t tg = first; tg < p.total_tiles; tg += gridDim.x) {
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
    const uint32_t n = d.n, zmax = d.zmax;
    const uint32_t rem = n - t0;
    const uint32_t need = min(T + zmax - 1, rem);

    for (uint32_t i = threadIdx.x; i < chunks_per_tile * zmax; i += kThreads) slots[i] = 0ull;
    for (uint32_t i = threadIdx.x; i < d.zc; i += kThreads) Tl[i] = d.thr[i];
    for (uint32_t i = threadIdx.x; i < plen; i += kThreads) Pl[i] = -INFINITY;
    __syncthreads();

    if (p.from_power) {
      const float *pw = reinterpret_cast<const float *>(d.x);
      for (uint32_t i = threadIdx.x; i < need; i += kThreads) Pl[paddr<K>(i)] = pw[t0 + i];
    } else {
      const bool dbg = p.mode == kModeTables;
      const uint32_t bfirst = t0 / B, blast = (t0 + need - 1) / B;
      for (uint32_t b = bfirst + wave; b <= blast; b += kWaves)
        normalise_block<K, EPL>(d.x, n, b, t0, need, T, Pl, lane, dbg ? p.P_out : nullptr,
                                dbg ? p.stats_out : nullptr);
    }
    __syncthreads();

    const uint32_t nseg_tile = T / SEG;
    for (uint32_t g = wave; g < nseg_tile; g += kWaves) {
      const uint32_t seg0 = g * SEG;
      if (seg0 >= rem) break;
      const uint32_t c_local = seg0 / C;
      bank_segment<K>(Pl, g, lane, Tl, zmax, d.zc, slots + (size_t)c_local * zmax,
                      t0 + seg0 + lane * K);
    }
    __syncthreads();

    const uint32_t chunk0 = t0 / C;
    const uint32_t nch = min(chunks_per_tile, d.nchunks - chunk0);
    const uint32_t nsl = nch * zmax;
    if (p.mode == kModeSearch) {
      // Stage the tile's maxima in slot order, i.e. (chunk, width) order:
      // count, reserve one run of the pool, then write with ordered ranks.
      uint32_t mine = 0;
      for (uint32_t i = threadIdx.x; i < nsl; i += kThreads) mine += slots[i] != 0ull ? 1u : 0u;
      for (int o = 32; o >= 1; o >>= 1) mine += __shfl_xor(mine, o, 64);
      if (lane == 0) wave_sum[wave] = mine;
      __syncthreads();
      if (threadIdx.x == 0) {
        uint32_t tot = 0;
        for (int v = 0; v < kWaves; ++v) tot += wave_sum[v];
        const uint32_t base = tot ? atomicAdd(p.pool_head, tot) : 0u;
        p.tile_count[tg] = tot;
        p.tile_pos[tg] = base;
        tile_base = base;
      }
      __syncthreads();
      uint32_t run = tile_base;
      for (uint32_t r = 0; r < nsl; r += kThreads) {
        const uint32_t i = r + threadIdx.x;
        const unsigned long long key = i < nsl ? slots[i] : 0ull;
        const bool valid = key != 0ull;
        const unsigned long long mask = __ballot(valid);
        if (lane == 0) wave_sum[wave] = (uint32_t)__popcll(mask);
        __syncthreads();
        uint32_t before = 0, all = 0;
        for (int v = 0; v < kWaves; ++v) {
          before += (uint32_t)v < wave ? wave_sum[v] : 0u;
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
      for (uint32_t i = threadIdx.x; i < nsl; i += kThreads) {
        const unsigned long long key = slots[i];
        const size_t o = (size_t)chunk0 * zmax + i;
        p.M[o] = key ? unord_f32((uint32_t)(key >> 32)) : -INFINITY;
        p.I[o] = key ? 0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull) : 0xFFFFFFFFu;
      }
    }
    __syncthreads();
  }
}

static size_t lds_need(uint32_t T, uint32_t C, uint32_t zmax_max, int K, uint32_t *nseg,
                       uint32_t *zc_pad) {
  const uint32_t zc = round_widths(zmax_max, K);
  const uint32_t segb = 64u * (uint32_t)K;
  *nseg = (T + zc + segb - 1) / segb;
  *zc_pad = (zc + 3) / 4 * 4;
  return (size_t)(T / C) * zmax_max * 8u + (size_t)(*zc_pad) * 4u +
         (size_t)(*nseg) * K * kRowPitch * 4u;
}

static uint32_t gcd_u(uint32_t a, uint32_t b) {
  while (b) {
    const uint32_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}
static uint64_t lcm_u(uint64_t a, uint64_t b) { return a / gcd_u((uint32_t)a, (uint32_t)b) * b; }

constexpr size_t kLdsBudget = 64 * 1024;

bool choose_geometry(uint32_t C, uint32_t B, uint32_t zmax_max, Geometry *g) {
  if (C == 0 || C % 64 != 0 || C > (uint32_t)kMaxTile) return false;
  if (B != 64 && B != 256 && B != 1024 && B != 4096) return false;
  int K = 16;
  while (K > 1 && (C / 64) % (uint32_t)K != 0) K /= 2;
  uint64_t T = lcm_u(lcm_u(64ull * K * kWaves, C), B);
  if (T > (uint64_t)kMaxTile) return false;
  uint32_t nseg = 0, zcp = 0;
  if (lds_need((uint32_t)T, C, zmax_max, K, &nseg, &zcp) > kLdsBudget) return false;
  while (T * 2 <= 4096 && lds_need((uint32_t)(T * 2), C, zmax_max, K, &nseg, &zcp) <= kLdsBudget)
    T *= 2;
  g->K = K;
  g->EPL = (int)(B / 64);
  g->tile = (uint32_t)T;
  g->lds_bytes = lds_need(g->tile, C, zmax_max, K, &nseg, &zcp);
  g->nseg_lds = nseg;
  g->zc_max_pad = zcp;
  return true;
}

template <int K>
static hipError_t launch_k(int EPL, uint64_t grid, size_t lds, const BankParams &p,
                           hipStream_t stream) {
  switch (EPL) {
    case 1:
      hipLaunchKernelGGL((bank_kernel<K, 1>), dim3((uint32_t)grid), dim3(kThreads), lds, stream, p);
      break;
    case 4:
      hipLaunchKernelGGL((bank_kernel<K, 4>), dim3((uint32_t)grid), dim3(kThreads), lds, stream, p);
      break;
    case 16:
      hipLaunchKernelGGL((bank_kernel<K, 16>), dim3((uint32_t)grid), dim3(kThreads), lds, stream, p);
      break;
    case 64:
      hipLaunchKernelGGL((bank_kernel<K, 64>), dim3((uint32_t)grid), dim3(kThreads), lds, stream, p);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_bank(const Geometry &g, const BankParams &p, uint64_t grid, hipStream_t stream) {
  if (grid == 0) return hipSuccess;
  switch (g.K) {
    case 1: return launch_k<1>(g.EPL, grid, g.lds_bytes, p, stream);
    case 2: return launch_k<2>(g.EPL, grid, g.lds_bytes, p, stream);
    case 4: return launch_k<4>(g.EPL, grid, g.lds_bytes, p, stream);
    case 8: return launch_k<8>(g.EPL, grid, g.lds_bytes, p, stream);
    case 16: return launch_k<16>(g.EPL, grid, g.lds_bytes, p, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pulscan

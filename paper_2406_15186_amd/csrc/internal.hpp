// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pulscan.h"

namespace pulscan {

// 1 / Phi^-1(3/4) rounded to FP32: scales a MAD to a Gaussian standard
// deviation (section 2.2.3).
constexpr float kMadScale = 1.482602218505602f;

constexpr int kWaves = 4;             // waves per workgroup of the bank kernel
constexpr int kThreads = 64 * kWaves;
constexpr int kRowPitch = 65;         // LDS row pitch (floats) of the power tile
constexpr int kMaxTile = 16384;       // bins per tile
constexpr int kSortLds = 8192;        // candidates sorted in LDS per spectrum

// One spectrum of a launch.  A device-resident array of these drives the
// bank and finalise kernels; a single search is a batch of one.
struct SpecDesc {
  const float2 *x;        // complex spectrum (or, from-power mode, float power)
  const float *thr;       // per-width thresholds, zc entries (+inf beyond zmax)
  uint64_t tile_begin;    // first global tile of this spectrum
  uint64_t stage_off;     // first staging entry of this spectrum
  uint64_t stage_cap;     // staging entries reserved (nchunks * zmax)
  double ntrials;         // Bonferroni factor
  uint32_t n;             // bins
  uint32_t zmax;          // widths 1..zmax
  uint32_t zc;            // zmax rounded up to the bank kernel's width block
  uint32_t nchunks;       // ceil(n / chunk)
};

// A staged candidate, written by the bank kernel in arbitrary order.
struct StageEntry {
  uint32_t key;    // chunk * zmax + (width - 1): unique within a spectrum
  uint32_t bin;    // window start
  float power;     // boxcar power
  uint32_t width;  // 1..zmax
};

enum BankMode : int {
  kModeSearch = 0,   // stage (chunk, width) maxima that reach the threshold
  kModeTables = 1,   // write every (chunk, width) maximum to M / I
};

// Launch-wide parameters of the bank kernel.
struct BankParams {
  const SpecDesc *descs;   // device table when nspec > 1
  SpecDesc single;         // the spectrum when nspec == 1
  int nspec;
  uint64_t total_tiles;
  uint32_t chunk;          // C
  uint32_t block;          // normalisation block B
  uint32_t tile;           // T bins per tile (multiple of C, B and 64*K*kWaves)
  uint32_t zmax_max;       // largest zmax of the batch (slot row stride bound)
  uint32_t nseg_lds;       // segments of 64*K bins held in LDS (tile + halo)
  int mode;                // BankMode
  int from_power;          // x holds float power; skip normalisation
  StageEntry *stage;       // search mode
  unsigned long long *stage_count;  // search mode: one counter per spectrum
  float *M;                // tables mode: nchunks x zmax (spectrum 0 only)
  uint32_t *I;
  float *P_out;            // tables mode, optional: normalised power
  float *stats_out;        // tables mode, optional: 4 floats per block
};

// Chosen launch geometry of a search.
struct Geometry {
  int K;          // bins per lane in the bank
  int EPL;        // normalisation elements per lane (block / 64)
  uint32_t tile;
  uint32_t nseg_lds;
  size_t lds_bytes;
};

// Geometry for chunk C, block B and the largest width zc (rounded); returns
// false when the kernels cannot run it (too large for LDS, bad sizes).
bool choose_geometry(uint32_t chunk, uint32_t block, uint32_t zmax_max, Geometry *g);

// Round zmax up to the width block of the bank kernel for K bins per lane.
inline uint32_t round_widths(uint32_t zmax, int K) { return (zmax + K - 1) / K * K; }

hipError_t launch_bank(const Geometry &g, const BankParams &p, uint64_t grid, hipStream_t stream);

// Per-width thresholds for nspec tables laid out at thr + s * zc_stride:
// thr[s][w-1] for w <= zmax[s] (searched), +inf otherwise; debug fills
// -FLT_MAX for every w <= zmax[s] (every maximum qualifies).
struct ThreshJob {
  float *thr;
  uint32_t zmax;
  uint32_t zc;
  double ntrials;
};
// jobs_dev == nullptr: one job, `single`.
hipError_t launch_thresholds(const ThreshJob *jobs_dev, const ThreshJob &single, int njobs,
                             uint32_t zc_max, double sigma, int width_search, int debug,
                             hipStream_t stream);

// Sort each spectrum's staged candidates into canonical order, compute their
// FP64 significance and write them out.  counts[s] are read, counts_next[s]
// cleared, *total (if non-null) receives the sum of counts.
struct FinalParams {
  const SpecDesc *descs;           // device table, or nullptr for one spectrum
  int nspec;
  const StageEntry *stage;
  const unsigned long long *counts;
  unsigned long long *counts_next;
  pulscan_candidate *out;
  uint64_t capacity;
  unsigned long long *total;       // device
  unsigned long long *total2;      // optional second device destination (caller's)
  uint64_t *sort_scratch;          // >= max stage_cap entries, for lists beyond kSortLds
};
hipError_t launch_finalise(const FinalParams &p, const SpecDesc &single, hipStream_t stream);

// Is width w searched under width_search?
__host__ __device__ inline bool width_searched(uint32_t w, int width_search) {
  if (width_search == PULSCAN_W_LOG2) {
    uint32_t z = w - 1;
    return z != 0 && (z & (z - 1)) == 0;
  }
  return true;
}

}  // namespace pulscan

// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "pulscan.h"

namespace pulscan {

// 1 / Phi^-1(3/4) rounded to FP32: scales a MAD to a Gaussian standard
// deviation (section 2.2.3).
constexpr float kMadScale = 1.482602218505602f;

constexpr int kMaxThreads = 512;      // threads per workgroup of the bank kernel (<= 8 waves)
constexpr int kMaxTile = 16384;       // bins per tile
constexpr uint32_t kPoolMax = 1u << 26;  // staging-pool entries per context (1 GiB)

// The caller's count word after a scan: the total, or the failure code of the
// scan's overflow flag (1: the staging pool overflowed, 2: a count was lost).
__host__ __device__ inline unsigned long long count_word(unsigned long long total,
                                                         uint32_t overflow) {
  return overflow == 2 ? PULSCAN_COUNT_LOST : overflow == 1 ? PULSCAN_COUNT_POOL_FULL : total;
}

// One searched series of a launch: a spectrum, or one harmonic stage of a
// spectrum (power input).  A device-resident array of these drives the bank
// and emit kernels; a single series is a batch of one.
struct SpecDesc {
  const float2 *x;        // complex spectrum (or, from-power mode, float power)
  const float *thr;       // per-width thresholds, zc entries (+inf beyond zmax)
  float *aux;             // power mode: where the normalised power goes; FP16
                          // search: the blocks' statistics (4 floats each)
  uint64_t tile_begin;    // first global tile of this series (tiled kernel)
  uint64_t block_begin;   // first global block of this series (streaming kernel)
  double ntrials;         // Bonferroni factor
  uint32_t n;             // bins
  uint32_t zmax;          // widths 1..zmax
  uint32_t zc;            // zmax rounded up to the bank kernel's width block
  uint32_t nchunks;       // ceil(n / chunk)
  uint32_t dofmul;        // degrees of freedom per width / 2: H(H+1)/2 for stage H
  uint32_t spec_id;       // spectrum index reported in candidates
  uint32_t harm;          // harmonic stage H reported in candidates
  uint32_t pad;
};

// A staged candidate.  Each unit of work (a tile of the tiled kernel, a
// workgroup's range of the streaming kernel) stages its own in canonical
// order; a candidate's place in the output is its unit's exclusive prefix
// plus its rank within the unit.
struct StageEntry {
  uint32_t unit;        // tile or workgroup index
  uint32_t rank;        // rank within the unit
  uint32_t spec;        // series index in the launch
  uint32_t bin;         // window start
  float power;          // boxcar power
  uint32_t width;       // boxcar width
};

enum BankMode : int {
  kModeSearch = 0,   // stage (chunk, width) maxima that reach the threshold
  kModeTables = 1,   // write every (chunk, width) maximum to M / I
  kModePower = 2,    // normalise only: each series' power to its desc.aux
};

// Launch-wide parameters of the bank kernel.
struct BankParams {
  const SpecDesc *descs;   // device table when nspec > 1
  SpecDesc single;         // the spectrum when nspec == 1
  int nspec;
  uint64_t total_tiles;
  uint32_t chunk;          // C
  uint32_t block;          // normalisation block B
  uint32_t tile;           // T bins per tile (multiple of C, B and 64*K*waves)
  uint32_t zmax_max;       // largest zmax of the batch (slot row stride bound)
  uint32_t nseg_lds;       // segments of 64*K bins held in LDS (tile + halo)
  uint32_t zc_max_pad;     // LDS floats reserved for the threshold table
  int mode;                // BankMode
  int from_power;          // x holds float power; skip normalisation
  int dense;               // 1: skip the pruning bound (every width block evaluated)
  int norm_exact;          // 1: exact median / MAD instead of the median of medians
  // search mode: candidate staging and the scan of the per-tile counts,
  // which the workgroup of the last index performs after its own tile
  StageEntry *pool;        // staging pool
  uint32_t pool_cap;       // entries in the pool
  uint32_t *pool_head;     // next free pool entry (re-armed to 0 by the scan)
  unsigned long long *tile_word;  // per tile: kTilePublished | candidates it staged
                                  // (0 until published; the scan clears it)
  uint32_t *tile_prefix;   // per tile: exclusive prefix of the counts; [total_tiles] = total
  unsigned long long *total;   // candidate count (device)
  unsigned long long *total2;  // optional second destination (the caller's)
  uint32_t *overflow;      // 1: the pool was too small; 2: a tile's count never arrived
  int scan_in_kernel;      // 1: the last tile scans the counts; 0: launch_scan_big does
  uint32_t spin;           // polls of a tile's count word before the scan gives up on it
  float *M;                // tables mode: nchunks x zmax (spectrum 0 only)
  uint32_t *I;
  float *P_out;            // tables mode, optional: normalised power
  float *stats_out;        // tables mode, optional: 4 floats per block
};

// A tile word holds this flag once the tile has published its count.
constexpr unsigned long long kTilePublished = 1ull << 32;

// Chosen launch geometry of a search.
struct Geometry {
  int K;          // bins per lane in the bank
  int EPL;        // normalisation elements per lane (block / 64)
  int waves;      // waves per workgroup
  uint32_t tile;
  uint32_t nseg_lds;
  uint32_t zc_max_pad;
  size_t lds_bytes;
  bool fp16;      // power tile stored in FP16
};

// Geometry for chunk C, block B, the largest zmax of the launch and the
// shortest spectrum (n_hint, to keep enough tiles); returns false when the
// kernels cannot run it (too large for LDS, bad sizes, zmax > 4096).  A
// non-zero `tile` asks for that tile instead of the heuristic choice.
bool choose_geometry(uint32_t chunk, uint32_t block, uint32_t zmax_max, uint64_t n_hint,
                     Geometry *g, uint32_t tile = 0, bool fp16 = false);
// Every tile choose_geometry accepts for these sizes, smallest first.
std::vector<uint32_t> tile_choices(uint32_t chunk, uint32_t block, uint32_t zmax_max,
                                   bool fp16 = false);

// Round zmax up to the width block of the bank kernel for K bins per lane.
inline uint32_t round_widths(uint32_t zmax, int K) { return (zmax + K - 1) / K * K; }

hipError_t launch_bank(const Geometry &g, const BankParams &p, uint64_t grid, hipStream_t stream);

// ---------------------------------------------------------------------------
// The streaming bank kernel: persistent workgroups, each owning a contiguous
// range of normalisation blocks of the launch's series (concatenated in
// order, each series padded to a whole number of alignment units).  A
// workgroup streams its range through an LDS ring of blocks: it normalises a
// batch of blocks while the next batch's loads are in flight, and searches
// the tile of blocks whose windows the ring now holds in full.

constexpr int kStreamWaves = 8;                       // waves per workgroup
constexpr int kStreamThreads = 64 * kStreamWaves;
constexpr int kStreamBatch = kStreamWaves;            // blocks normalised per batch
// A long launch is cut into up to kStreamRounds ranges per workgroup, of at
// least kStreamRangeMin blocks on average (the last ones a quarter of the
// mean); a workgroup that has finished a range takes the next one not yet
// taken, so that workgroups slowed by their series (zmax, flagged lanes) or
// by their CU take fewer, and all finish within about one range of each
// other
constexpr uint32_t kStreamRounds = 16;
constexpr uint64_t kStreamRangeMin = 64;
constexpr uint32_t kStreamSpin = 1u << 20;            // polls of a cross-workgroup word before giving up

struct StreamGeometry {
  int K;              // bins per lane of the bank (4 or 16)
  int EPL;            // normalisation elements per lane: block / 64 (4 or 16)
  uint32_t lag;       // halo blocks a tile needs beyond itself (max over the series)
  uint32_t ring;      // blocks in the LDS ring
  uint32_t mirror;    // group-sum entries repeated past the ring's end
  uint32_t zc_max;    // largest zmax rounded up to K
  uint32_t zc_pad;    // threshold floats reserved in LDS
  uint32_t off_sg, off_ep, off_slots, off_tl, off_items, off_xs;  // LDS byte offsets
  size_t lds_bytes;
};

struct StreamParams {
  const SpecDesc *descs;   // device table when nspec > 1
  SpecDesc single;         // the series when nspec == 1
  int nspec;
  uint64_t total_blocks;   // padded blocks of the whole launch
  uint32_t nwg;            // workgroups
  uint32_t nseg;           // ranges: workgroup w takes ranges w, w + nwg, ... (nseg >= nwg)
  uint32_t chunk;          // C
  uint32_t block;          // normalisation block B (the streaming unit of power input)
  uint32_t zmax_max;
  StreamGeometry g;
  int mode;                // kModeSearch or kModeTables
  int dense;               // 1: evaluate every width block
  int from_power;          // series are float power
  uint32_t spin;           // polls of a cross-workgroup word before giving up
  // candidate staging
  StageEntry *pool;
  uint32_t pool_cap;
  uint32_t *pool_head;     // re-armed to 0 by the scan
  unsigned long long *wg_word;   // per range: (tag << 32) | candidates staged
  uint32_t *wg_prefix;     // per range exclusive prefix; [nseg] = total
  uint32_t *gen;           // launch generation; tags are gen + 1
  uint32_t *seg_ctr;       // two range counters (launch tag parity), or null: ranges in turn
  unsigned long long *halo;      // per range: lag x 4 published statistics words
  unsigned long long *total;
  unsigned long long *total2;
  uint32_t *overflow;      // 1: pool too small; 2: a count never arrived
  // tables mode (series 0)
  float *M;
  uint32_t *I;
  float *P_out;
  float *stats_out;
};

// The geometry of the streaming kernel for these sizes, or false when it does
// not serve them (the tiled kernel then runs the search).
bool choose_stream_geometry(uint32_t chunk, uint32_t block, uint32_t zmax_max, bool from_power,
                            bool norm_exact, bool fp16, StreamGeometry *g);
// Workgroups resident per CU for this geometry (0 if it cannot launch).
int stream_occupancy(const StreamGeometry &g, bool from_power);
hipError_t launch_stream(const StreamParams &p, hipStream_t stream);

// Per-width thresholds for nspec tables laid out at thr + s * zc_stride:
// thr[s][w-1] for w <= zmax[s] (searched), +inf otherwise; debug fills
// -FLT_MAX for every w <= zmax[s] (every maximum qualifies).
struct ThreshJob {
  float *thr;
  uint32_t zmax;
  uint32_t zc;
  double ntrials;
  uint32_t dofmul;  // chi^2(2 w dofmul) for width w
  uint32_t pad;
};
// jobs_dev == nullptr: one job, `single`.
hipError_t launch_thresholds(const ThreshJob *jobs_dev, const ThreshJob &single, int njobs,
                             uint32_t zc_max, double sigma, int width_search, int debug,
                             hipStream_t stream);

// Scan of the per-tile counts for launches with many tiles (batches), in
// two kernels after the bank kernel: each workgroup scans kScanSpan tiles
// into tile_prefix (relative to its span) and writes the span's total; one
// workgroup scans the span totals into span_prefix, records the total and
// the overflow flag, and re-arms the pool head.  The span scan clears the
// tile words it reads.
constexpr uint32_t kScanSpan = 4096;
struct BigScan {
  unsigned long long *tile_word;
  uint32_t *tile_prefix;
  uint32_t *span_sum;
  uint32_t *span_prefix;
  uint64_t total_tiles;
  uint32_t *pool_head;
  uint32_t pool_cap;
  unsigned long long *total;
  unsigned long long *total2;
  uint32_t *overflow;
  uint32_t *lost;                  // set by a span that found a count missing
};
hipError_t launch_scan_big(const BigScan &s, hipStream_t stream);

// Candidate f of the staging pool goes to out[tile_prefix[unit] + rank]
// (when that is below capacity), with its FP64 significance.
struct EmitParams {
  const SpecDesc *descs;           // device table, or nullptr for one series
  int nspec;
  const StageEntry *pool;
  uint32_t pool_cap;
  const uint32_t *tile_prefix;     // per unit: exclusive prefix of the counts
  const uint32_t *span_prefix;     // non-null: tile_prefix is relative to its kScanSpan span
  const unsigned long long *total;
  uint32_t chunk;
  uint32_t rblock;                 // > 0: report bin / rblock
  pulscan_candidate *out;
  uint64_t capacity;
  int fp16;                        // FP16-stored search: re-check near the threshold
  int from_power;                  // the series are power (re-check reads them)
  uint32_t block;                  // normalisation block (re-check statistics)
  float sigma;                     // the requested threshold
  // After a lost count (overflow 2) the bank launch's late workgroups may
  // have published their words and reserved pool entries after the scan
  // re-armed them; emit, which runs once every workgroup has ended, then
  // places nothing and clears them for the next launch.
  const uint32_t *overflow;
  unsigned long long *tile_word;   // the tiled kernel's count words, or nullptr
  uint64_t ntiles;
  uint32_t *pool_head;
};
hipError_t launch_emit(const EmitParams &p, const SpecDesc &single, uint32_t grid,
                       hipStream_t stream);

// Final pass over the canonical list `all` (count *total, at most all_cap
// stored): entries with NaN sigma (rejected by the FP32 re-check) are
// dropped; with `best`, out[k] is the highest-sigma survivor of the k-th run
// of equal (spectrum, stage, chunk) (the first on ties).  The number written
// goes to *count and, if non-null, *count2.  One workgroup.
hipError_t launch_finalize(const pulscan_candidate *all, const unsigned long long *total,
                           uint64_t all_cap, pulscan_candidate *out, uint64_t capacity,
                           unsigned long long *count, unsigned long long *count2,
                           const uint32_t *overflow, int best,
                           hipStream_t stream);

// FP16 power storage: the bank compares against thresholds kRecheckBand sigma
// below the requested one, and every candidate below sigma + kRecheckBand
// (or whose FP16 sum reached kRecheckPower, where FP16 inputs may have
// saturated) is re-decided on its FP32 power.
constexpr float kRecheckBand = 0.5f;
constexpr float kRecheckPower = 60000.0f;

// Harmonic stages 2..numharm of one power series (section 2.3): S_H has
// floor(n / H) bins and starts at S + sum_{h=2}^{H-1} floor(n / h).
struct HarmJob {
  const float *P;
  float *S;
  uint32_t n;
  uint32_t numharm;
};
hipError_t launch_harmonics(const HarmJob *jobs_dev, const HarmJob &single, int njobs,
                            uint32_t n_max, hipStream_t stream);
inline uint64_t harmonic_offset(uint64_t n, uint32_t H) {
  uint64_t off = 0;
  for (uint32_t h = 2; h < H; ++h) off += n / h;
  return off;
}
constexpr int kMaxHarm = 16;

// The argument checks every search entry point applies to one spectrum
// (PULSCAN_OK, EINVAL or EUNSUPPORTED); *block gets the normalisation block.
int check_search_args(const void *x, uint64_t n, int zmax, int chunk, const pulscan_opts &o,
                      uint32_t *block);

// Is width w of a 1..zmax bank searched under width_search?  The
// logarithmic z sampling (section 4.1.3) searches z = w - 1 = 1, 2, 4, ...
// and the largest drift, i.e. the widest width zmax itself.
__host__ __device__ inline bool width_searched(uint32_t w, uint32_t zmax, int width_search) {
  if (w < 1 || w > zmax) return false;
  if (width_search == PULSCAN_W_LOG2) {
    const uint32_t z = w - 1;
    return w == zmax || (z != 0 && (z & (z - 1)) == 0);
  }
  return true;
}

}  // namespace pulscan

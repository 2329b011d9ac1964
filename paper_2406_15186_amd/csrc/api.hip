// C ABI of the boxcar search: argument checks, the context and its device
// memory, threshold caching and the launch sequence
//   thresholds (cached) -> fused bank kernel -> scan of tile counts -> emit
//   (canonical order + FP64 sigma).
#include <float.h>
#include <math.h>
#include <string.h>

#include <mutex>
#include <unordered_map>
#include <utility>
#include <vector>

#include "internal.hpp"

using namespace pulscan;

namespace {

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

// What a threshold table depends on.  Compared and hashed as bytes: every
// member is 4 or 8 bytes wide and the struct has no padding.
struct ThrKey {
  uint32_t zmax, zc, dofmul;
  int32_t ws, debug;
  float sigma;
  double ntrials;
  bool operator==(const ThrKey &o) const { return memcmp(this, &o, sizeof o) == 0; }
};
static_assert(sizeof(ThrKey) == 32, "no padding in the threshold key");
struct ThrKeyHash {
  size_t operator()(const ThrKey &k) const {
    // FNV-1a over the key's bytes
    const unsigned char *b = reinterpret_cast<const unsigned char *>(&k);
    uint64_t h = 1469598103934665603ull;
    for (size_t i = 0; i < sizeof k; ++i) h = (h ^ b[i]) * 1099511628211ull;
    return (size_t)h;
  }
};

// Device memory the threshold tables of a context occupy before the cache
// is emptied and refilled (a soft limit: one launch may exceed it).
constexpr size_t kThrCacheBytes = 64ull << 20;
constexpr size_t kThrArenaBytes = 1ull << 20;

}  // namespace

struct pulscan_ctx {
  int device = 0;
  DevBuf pool, tile_word, tile_prefix, counters, outbuf, descs, jobs;
  DevBuf allbuf, hpow, hsum, hjobs;  // best-per-chunk scratch; harmonic power, sums, jobs
  DevBuf tune_out;                   // autotuner: candidate output of its timing runs
  DevBuf stats;                      // FP16 search: per-block statistics for the re-check
  DevBuf span_sum, span_prefix;      // two-level scan of many tiles
  // threshold tables: key -> device table, carved from arenas that live
  // until the cache is emptied; thr_new lists the tables the last search
  // launch added (forgotten again if that launch never ran)
  std::unordered_map<ThrKey, float *, ThrKeyHash> thr_tab;
  std::vector<ThrKey> thr_new;
  std::vector<void *> thr_arenas;
  size_t thr_used = 0, thr_cap = 0, thr_bytes = 0;
  // what the device holds for batched launches (re-uploaded only on change)
  std::vector<HarmJob> last_hjobs;
  // autotuner: (batch signature) -> (chunk, tile)
  std::vector<std::pair<std::vector<uint64_t>, std::pair<uint32_t, uint32_t>>> tuned;
  // graph replay of the last graph-mode call
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  std::vector<uint64_t> graph_key;
  // bumped whenever device memory a captured graph may use is reallocated or
  // refilled with other contents (thresholds, descriptors, stage jobs)
  uint64_t epoch = 0;
  uint64_t graph_epoch = 0;
  // a search's bank kernel ran but its count scan was not launched: tile
  // words may be left published and the pool head advanced
  bool counts_dirty = false;
  // pinned staging of batched descriptors / threshold jobs
  void *pinned = nullptr;
  size_t pinned_bytes = 0;
  hipEvent_t pinned_ev = nullptr;
  bool pinned_pending = false;
  std::vector<SpecDesc> last_descs;  // what the device descriptor table holds
  DevBuf pdescs;                     // descriptor table of the power pass (harmonic mode)
  std::vector<SpecDesc> last_pdescs;
  // streaming kernel: per-workgroup counts and prefixes, the launch
  // generation and the published halo statistics
  DevBuf wg_word, wg_prefix, gen, halo, seg_ctr;
  int n_cu = 0;
  int kernel = PULSCAN_KERNEL_AUTO;  // which bank kernel serves a search (pulscan_ctx_set_kernel)
  int last_kernel = -1;              // the bank kernel of the last launch
  uint32_t spin = kStreamSpin;    // polls of a cross-workgroup word before giving up
  std::vector<std::pair<uint64_t, int>> occ;  // (geometry key, workgroups per CU)
  // kernel timing: every timing-th bank launch (0: off)
  int timing = 0;
  uint64_t timing_seen = 0;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_rec;
};

namespace {

// Device-resident counters of a search; zeroed when allocated.  The scan of
// the tile counts re-arms the pool head at the end of every search.
struct Counters {
  unsigned long long total;
  unsigned long long best;   // candidates kept by the final pass (best / re-check)
  uint32_t head;             // next free staging-pool entry
  uint32_t overflow;
  uint32_t lost;             // two-level scan: a tile's count was missing
  uint32_t pad;
};

// Launches with more tiles than this scan their counts in two kernels after
// the bank kernel instead of in its last workgroup.
constexpr uint64_t kInKernelScanMax = 4096;

#define HIP_TRY(call)                       \
  do {                                      \
    if ((call) != hipSuccess) {             \
      (void)hipGetLastError();              \
      return PULSCAN_EHIP;                  \
    }                                       \
  } while (0)

int grow(pulscan_ctx *ctx, DevBuf &b, size_t bytes, bool zero) {
  if (bytes == 0) bytes = 8;
  if (b.bytes >= bytes) return PULSCAN_OK;
  // a buffer may still be read by work queued earlier on any stream
  HIP_TRY(hipDeviceSynchronize());
  ++ctx->epoch;
  if (b.p) {
    HIP_TRY(hipFree(b.p));
    b.p = nullptr;
    b.bytes = 0;
  }
  size_t want = bytes + bytes / 4;
  if (hipMalloc(&b.p, want) != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return PULSCAN_ENOMEM;
  }
  b.bytes = want;
  if (zero) {
    HIP_TRY(hipMemset(b.p, 0, want));
  }
  return PULSCAN_OK;
}

int grow_pinned(pulscan_ctx *ctx, size_t bytes) {
  if (ctx->pinned_pending) {
    HIP_TRY(hipEventSynchronize(ctx->pinned_ev));
    ctx->pinned_pending = false;
  }
  if (ctx->pinned_bytes >= bytes) return PULSCAN_OK;
  if (ctx->pinned) {
    HIP_TRY(hipHostFree(ctx->pinned));
    ctx->pinned = nullptr;
    ctx->pinned_bytes = 0;
  }
  if (hipHostMalloc(&ctx->pinned, bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    ctx->pinned = nullptr;
    return PULSCAN_ENOMEM;
  }
  ctx->pinned_bytes = bytes;
  return PULSCAN_OK;
}

// Copy host bytes to device through the pinned staging buffer; the buffer is
// reused only after the copy has completed (an event guards it).
int upload(pulscan_ctx *ctx, void *dst, const void *src, size_t bytes, hipStream_t stream) {
  ++ctx->epoch;
  int st = grow_pinned(ctx, bytes);
  if (st) return st;
  memcpy(ctx->pinned, src, bytes);
  HIP_TRY(hipMemcpyAsync(dst, ctx->pinned, bytes, hipMemcpyHostToDevice, stream));
  HIP_TRY(hipEventRecord(ctx->pinned_ev, stream));
  ctx->pinned_pending = true;
  return PULSCAN_OK;
}

void drop_graph(pulscan_ctx *ctx);

// Empty the threshold cache (after the device has finished with its tables).
int thr_clear(pulscan_ctx *ctx) {
  HIP_TRY(hipDeviceSynchronize());
  drop_graph(ctx);
  for (void *p : ctx->thr_arenas) (void)hipFree(p);
  ctx->thr_arenas.clear();
  ctx->thr_tab.clear();
  ctx->thr_new.clear();
  ctx->thr_used = ctx->thr_cap = ctx->thr_bytes = 0;
  ++ctx->epoch;
  return PULSCAN_OK;
}

// Point every descriptor at its threshold table, reserving (and listing in
// *jobs, for the threshold kernel) the tables the cache does not hold yet.
// *zc_max gets the widest new table's width count.
int thr_reserve(pulscan_ctx *ctx, std::vector<SpecDesc> &descs, float sigma, int ws, int debug,
                std::vector<ThreshJob> *jobs, uint32_t *zc_max) {
  ctx->thr_new.clear();
  auto key_of = [&](const SpecDesc &d) {
    ThrKey k;
    memset(&k, 0, sizeof k);
    k.zmax = d.zmax;
    k.zc = d.zc;
    k.dofmul = d.dofmul;
    k.ws = ws;
    k.debug = debug;
    k.sigma = sigma;
    k.ntrials = d.ntrials;
    return k;
  };
  auto tab_bytes = [](uint32_t zc) { return ((size_t)zc * sizeof(float) + 255) & ~(size_t)255; };
  // bytes of the tables missing (an upper bound: duplicates counted)
  size_t need = 0;
  for (const SpecDesc &d : descs)
    if (!ctx->thr_tab.count(key_of(d))) need += tab_bytes(d.zc);
  if (need && ctx->thr_bytes && ctx->thr_bytes + need > kThrCacheBytes) {
    const int st = thr_clear(ctx);
    if (st) return st;
    need = 0;
    for (const SpecDesc &d : descs) need += tab_bytes(d.zc);
  }
  *zc_max = 0;
  for (SpecDesc &d : descs) {
    const ThrKey k = key_of(d);
    auto it = ctx->thr_tab.find(k);
    if (it != ctx->thr_tab.end()) {
      d.thr = it->second;
      continue;
    }
    const size_t b = tab_bytes(d.zc);
    if (ctx->thr_used + b > ctx->thr_cap) {
      const size_t sz = need > kThrArenaBytes ? need : kThrArenaBytes;
      void *p = nullptr;
      if (hipMalloc(&p, sz) != hipSuccess) {
        (void)hipGetLastError();
        return PULSCAN_ENOMEM;
      }
      ctx->thr_arenas.push_back(p);
      ctx->thr_bytes += sz;
      ctx->thr_used = 0;
      ctx->thr_cap = sz;
      ++ctx->epoch;
    }
    float *t = reinterpret_cast<float *>(static_cast<char *>(ctx->thr_arenas.back()) + ctx->thr_used);
    ctx->thr_used += b;
    need = need > b ? need - b : 0;
    ctx->thr_tab.emplace(k, t);
    ctx->thr_new.push_back(k);
    d.thr = t;
    jobs->push_back(ThreshJob{t, d.zmax, d.zc, d.ntrials, d.dofmul, 0u});
    *zc_max = d.zc > *zc_max ? d.zc : *zc_max;
  }
  return PULSCAN_OK;
}

// Forget the tables the last search launch reserved: their kernel never ran.
void thr_forget_new(pulscan_ctx *ctx) {
  for (const ThrKey &k : ctx->thr_new) ctx->thr_tab.erase(k);
  ctx->thr_new.clear();
}

bool is_pow4(uint64_t v) {
  if (v == 0) return false;
  while (v % 4 == 0) v /= 4;
  return v == 1;
}

uint32_t searched_widths(uint32_t zmax, int ws) {
  uint32_t c = 0;
  for (uint32_t w = 1; w <= zmax; ++w) c += width_searched(w, zmax, ws) ? 1u : 0u;
  return c;
}

// Checks shared by every search entry point.  Sets *block to the
// normalisation block.
int check_spectrum(const void *x, uint64_t n, int zmax, int chunk, const pulscan_opts &o,
                   uint32_t *block) {
  if (!x || zmax < 1 || chunk < 1 || n == 0 || n >= (1ull << 32)) return PULSCAN_EINVAL;
  if (o.norm != PULSCAN_NORM_MOM && o.norm != PULSCAN_NORM_EXACT) return PULSCAN_EINVAL;
  if (o.width_search != PULSCAN_W_ALL && o.width_search != PULSCAN_W_LOG2) return PULSCAN_EINVAL;
  if (o.norm_block < 0) return PULSCAN_EINVAL;
  if (!(o.ntrials == 0.0 || (isfinite(o.ntrials) && o.ntrials >= 1.0))) return PULSCAN_EINVAL;
  if (o.dense != 0 && o.dense != 1) return PULSCAN_EINVAL;
  if (o.numharm < 0 || o.numharm > kMaxHarm) return PULSCAN_EINVAL;
  if (o.best_per_chunk != 0 && o.best_per_chunk != 1) return PULSCAN_EINVAL;
  if (o.rblock < 0) return PULSCAN_EINVAL;
  if (o.graph != 0 && o.graph != 1) return PULSCAN_EINVAL;
  if (o.power_fp16 != 0 && o.power_fp16 != 1) return PULSCAN_EINVAL;
  const uint64_t B = o.norm_block > 0 ? (uint64_t)o.norm_block : (uint64_t)chunk;
  if (n < B || n < (uint64_t)zmax) return PULSCAN_EINVAL;
  if (o.norm == PULSCAN_NORM_MOM && !is_pow4(B)) return PULSCAN_EINVAL;
  // the kernels hold a block as 64 lanes x {1, 4, 16, 64} values
  if (o.norm == PULSCAN_NORM_EXACT && (!is_pow4(B) || B > 1024)) return PULSCAN_EUNSUPPORTED;
  if (B < 64 || B > 4096) return PULSCAN_EUNSUPPORTED;
  if (o.power_fp16 && (B == 4096 || o.norm == PULSCAN_NORM_EXACT)) return PULSCAN_EUNSUPPORTED;
  if (chunk % 64 != 0 || chunk > kMaxTile) return PULSCAN_EUNSUPPORTED;
  const uint64_t nchunks = (n + chunk - 1) / chunk;
  if (nchunks * (uint64_t)zmax >= (1ull << 32)) return PULSCAN_EUNSUPPORTED;
  *block = (uint32_t)B;
  return PULSCAN_OK;
}

int check_out(const pulscan_candidates *out, bool async) {
  if (!out) return PULSCAN_EINVAL;
  if (out->capacity > 0 && !out->data) return PULSCAN_EINVAL;
  if (async && (!out->on_device || !out->count_device)) return PULSCAN_EINVAL;
  return PULSCAN_OK;
}

hipEvent_t take_event(pulscan_ctx *ctx) {
  if (!ctx->ev_pool.empty()) {
    hipEvent_t e = ctx->ev_pool.back();
    ctx->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

struct SpecIn {
  const void *x;
  uint64_t n;
  uint32_t zmax;
  uint32_t dofmul = 1;     // chi^2(2 w dofmul) per width-w boxcar
  uint32_t spec_id = 0;    // reported spectrum index
  uint32_t harm = 1;       // reported harmonic stage
  float *aux = nullptr;    // power mode: output power
};

enum RunKind { kRunSearch, kRunTables, kRunPower };

struct RunArgs {
  RunKind kind = kRunSearch;
  bool from_power = false;  // the series are float power (no normalisation)
  uint32_t chunk = 0, block = 0;
  uint32_t tile = 0;        // 0: the heuristic tile; else the autotuner's
  float sigma = 0.f;
  pulscan_opts opts{};
  pulscan_candidates *out = nullptr;
  float *M = nullptr;
  uint32_t *I = nullptr;
  float *P_out = nullptr;
  float *stats_out = nullptr;
};

// What a synchronous search reads back once its launches are queued.
struct Pending {
  Counters *cnt = nullptr;
  bool best = false;     // the count comes from the final pass
  uint64_t cap = 0;      // entries of the destination the caller receives
  bool host = false;     // results go through ctx->outbuf to host memory
};

// Queue one fused launch of the bank kernel over a batch of series and, in
// search mode, the emission of the candidates and the best-per-chunk pass.
// Never waits on the device except to grow a buffer (which a call repeating
// an earlier one never does), so it can run under stream capture.
void drop_graph(pulscan_ctx *ctx);

// Whether the streaming kernel serves a launch it can run.  Both kernels give
// the same bits; in automatic mode the streaming kernel takes launches of
// spectra long enough to keep every resident workgroup streaming (at least
// kStreamAutoBlocks blocks each), where it reads each bin once, and the tiled
// kernel the rest, whose tiles start all at once.
constexpr uint64_t kStreamAutoBlocks = 64;
bool wants_stream(const pulscan_ctx *ctx, const std::vector<SpecIn> &specs, uint32_t block,
                  bool from_power, int occ) {
  if (ctx->kernel == PULSCAN_KERNEL_STREAM) return true;
  if (ctx->kernel == PULSCAN_KERNEL_TILED || from_power) return false;
  uint64_t blocks = 0;
  for (const SpecIn &s : specs) blocks += (s.n + block - 1) / block;
  return blocks >= kStreamAutoBlocks * (uint64_t)occ * (uint64_t)ctx->n_cu;
}

// Workgroups of the streaming kernel resident per CU for this geometry
// (cached per geometry).
int stream_occ(pulscan_ctx *ctx, const StreamGeometry &g, bool from_power) {
  const uint64_t key = ((uint64_t)g.lds_bytes << 16) | ((uint64_t)g.K << 8) |
                       ((uint64_t)g.EPL << 1) | (from_power ? 1u : 0u);
  for (auto &e : ctx->occ)
    if (e.first == key) return e.second;
  const int n = stream_occupancy(g, from_power);
  ctx->occ.emplace_back(key, n);
  return n;
}

int enqueue(pulscan_ctx *ctx, const std::vector<SpecIn> &specs, const RunArgs &a, Pending *pend) {
  hipStream_t stream = (hipStream_t)a.opts.stream;
  const int nspec = (int)specs.size();
  const bool search = a.kind == kRunSearch;
  const bool power_only = a.kind == kRunPower;
  const int ws = search ? a.opts.width_search : PULSCAN_W_ALL;

  uint32_t zmax_max = 0;
  uint64_t n_min = ~0ull;
  for (const SpecIn &s : specs) {
    zmax_max = s.zmax > zmax_max ? s.zmax : zmax_max;
    n_min = s.n < n_min ? s.n : n_min;
  }
  const bool fp16 = search && a.opts.power_fp16;
  const bool exact = a.opts.norm == PULSCAN_NORM_EXACT;
  // the streaming kernel serves what it can (search and tables), the tiled
  // kernel the rest (normalisation-only passes, the exact median, FP16
  // power, and sizes outside the streaming kernel's geometry)
  StreamGeometry sgeo{};
  int occ = 0;
  const bool sk = !power_only && a.tile == 0 &&
                  choose_stream_geometry(a.chunk, a.block, zmax_max, a.from_power, exact, fp16,
                                         &sgeo) &&
                  (occ = stream_occ(ctx, sgeo, a.from_power)) > 0 &&
                  wants_stream(ctx, specs, 64u * (uint32_t)sgeo.EPL, a.from_power, occ);
  Geometry g{};
  if (sk) {
    g.K = sgeo.K;
  } else if (!choose_geometry(a.chunk, a.block, zmax_max, n_min, &g, a.tile, fp16)) {
    return PULSCAN_EUNSUPPORTED;
  }
  const uint32_t sblock = sk ? 64u * (uint32_t)sgeo.EPL : 0u;
  // FP16 search on spectra: room for every block's statistics
  float *stats = nullptr;
  if (fp16 && !a.from_power) {
    uint64_t nb = 0;
    for (const SpecIn &s : specs) nb += (s.n + a.block - 1) / a.block;
    int st0 = grow(ctx, ctx->stats, nb * 4 * sizeof(float), false);
    if (st0) return st0;
    stats = static_cast<float *>(ctx->stats.p);
  }

  // descriptors
  std::vector<SpecDesc> descs(nspec);
  uint64_t tiles = 0, blocks = 0;
  uint32_t zc_max = 0;
  for (int s = 0; s < nspec; ++s) {
    SpecDesc &d = descs[s];
    d = SpecDesc{};
    d.x = reinterpret_cast<const float2 *>(specs[s].x);
    d.aux = specs[s].aux;
    if (stats) {
      d.aux = stats;
      stats += 4 * ((specs[s].n + a.block - 1) / a.block);
    }
    d.n = (uint32_t)specs[s].n;
    d.zmax = specs[s].zmax;
    d.zc = round_widths(d.zmax, g.K);
    d.nchunks = (uint32_t)((specs[s].n + a.chunk - 1) / a.chunk);
    d.dofmul = specs[s].dofmul;
    d.spec_id = specs[s].spec_id;
    d.harm = specs[s].harm;
    if (sk) {
      d.block_begin = blocks;
      blocks += (specs[s].n + sblock - 1) / sblock;
    } else {
      d.tile_begin = tiles;
      tiles += (specs[s].n + g.tile - 1) / g.tile;
    }
    if (a.opts.ntrials > 0.0) {
      d.ntrials = a.opts.ntrials;
    } else {
      const uint32_t sw = searched_widths(d.zmax, ws);
      d.ntrials = (double)d.n * (double)(sw ? sw : 1u);
    }
    zc_max = d.zc > zc_max ? d.zc : zc_max;
  }

  // thresholds: one cached device table per (zmax, ntrials, degrees of
  // freedom, sigma, width search, debug); the tables this launch lacks are
  // computed together, before the bank kernel, on the same stream
  int st = PULSCAN_OK;
  if (!power_only) {
    const int debug = search ? 0 : 1;
    // the FP16-stored search compares against thresholds kRecheckBand sigma lower
    const float tsig = fp16 ? a.sigma - kRecheckBand : a.sigma;
    std::vector<ThreshJob> jobs;
    uint32_t zc_new = 0;
    st = thr_reserve(ctx, descs, tsig, ws, debug, &jobs, &zc_new);
    if (st) return st;
    if (!jobs.empty()) {
      const ThreshJob *jobs_dev = nullptr;
      if (jobs.size() > 1) {
        st = grow(ctx, ctx->jobs, jobs.size() * sizeof(ThreshJob), false);
        if (st) return st;
        st = upload(ctx, ctx->jobs.p, jobs.data(), jobs.size() * sizeof(ThreshJob), stream);
        if (st) return st;
        jobs_dev = static_cast<const ThreshJob *>(ctx->jobs.p);
      }
      if (launch_thresholds(jobs_dev, jobs[0], (int)jobs.size(), zc_new, (double)tsig, ws, debug,
                            stream) != hipSuccess) {
        (void)hipGetLastError();
        thr_forget_new(ctx);
        return PULSCAN_EHIP;
      }
      ++ctx->epoch;
    }
  }

  BankParams bp{};
  bp.nspec = nspec;
  bp.single = descs[0];
  bp.total_tiles = tiles;
  bp.chunk = a.chunk;
  bp.block = a.block;
  bp.tile = g.tile;
  bp.zmax_max = zmax_max;
  bp.nseg_lds = g.nseg_lds;
  bp.zc_max_pad = g.zc_max_pad;
  bp.mode = search ? kModeSearch : power_only ? kModePower : kModeTables;
  bp.from_power = a.from_power ? 1 : 0;
  bp.dense = a.opts.dense ? 1 : 0;
  bp.norm_exact = a.opts.norm == PULSCAN_NORM_EXACT ? 1 : 0;
  bp.M = a.M;
  bp.I = a.I;
  bp.P_out = a.P_out;
  bp.stats_out = a.stats_out;

  // staging: a pool for the candidates and per-unit counts and offsets
  uint64_t worst = 0;
  for (const SpecDesc &d : descs) worst += (uint64_t)d.nchunks * d.zmax;
  if (worst >= (1ull << 32)) return PULSCAN_EUNSUPPORTED;
  const uint32_t pool_cap = (uint32_t)(worst < (uint64_t)kPoolMax ? (worst ? worst : 1) : kPoolMax);
  const bool best = search && a.opts.best_per_chunk;
  const bool fin = best || fp16;  // a final pass compacts the emitted list
  Counters *cnt = nullptr;
  // the streaming kernel's workgroups: as many as are resident, each range
  // at least a batch and the halo long
  const uint64_t min_range = sgeo.lag > (uint32_t)kStreamBatch ? sgeo.lag : (uint64_t)kStreamBatch;
  uint64_t nwg = 0, nseg = 0;
  if (sk) {
    nwg = (uint64_t)occ * (uint64_t)ctx->n_cu;
    const uint64_t by_size = blocks / min_range;
    nwg = by_size < nwg ? by_size : nwg;
    if (nwg < 1) nwg = 1;
    // long launches (a batch): several ranges per workgroup, taken in turn
    uint64_t rounds = blocks / (nwg * kStreamRangeMin);
    rounds = rounds > kStreamRounds ? kStreamRounds : rounds;
    nseg = nwg * (rounds > 1 ? rounds : 1);
  }
  if (search || sk) {
    st = grow(ctx, ctx->counters, sizeof(Counters), true);
    if (st) return st;
    cnt = static_cast<Counters *>(ctx->counters.p);
  }
  if (search) {
    st = grow(ctx, ctx->pool, (size_t)pool_cap * sizeof(StageEntry), false);
    if (st) return st;
    if (!sk) {
      st = grow(ctx, ctx->tile_word, tiles * sizeof(unsigned long long), true);
      if (st) return st;
      st = grow(ctx, ctx->tile_prefix, (tiles + 1) * sizeof(uint32_t), false);
      if (st) return st;
    }
    if (ctx->counts_dirty) {
      // re-arm what a failed launch left behind (never under capture: a
      // failure drops the graph, so the next call runs directly)
      if (ctx->tile_word.p)
        HIP_TRY(hipMemsetAsync(ctx->tile_word.p, 0, ctx->tile_word.bytes, stream));
      HIP_TRY(hipMemsetAsync(&cnt->head, 0, sizeof(cnt->head), stream));
      ctx->counts_dirty = false;
    }
    bp.pool = static_cast<StageEntry *>(ctx->pool.p);
    bp.pool_cap = pool_cap;
    bp.pool_head = &cnt->head;
    bp.tile_word = static_cast<unsigned long long *>(ctx->tile_word.p);
    bp.tile_prefix = static_cast<uint32_t *>(ctx->tile_prefix.p);
    bp.total = &cnt->total;
    bp.total2 = fin ? nullptr : reinterpret_cast<unsigned long long *>(a.out->count_device);
    bp.overflow = &cnt->overflow;
    bp.scan_in_kernel = tiles <= kInKernelScanMax ? 1 : 0;
    bp.spin = ctx->spin;
    if (!sk && !bp.scan_in_kernel) {
      const uint64_t nspan = (tiles + kScanSpan - 1) / kScanSpan;
      st = grow(ctx, ctx->span_sum, nspan * sizeof(uint32_t), false);
      if (st) return st;
      st = grow(ctx, ctx->span_prefix, nspan * sizeof(uint32_t), false);
      if (st) return st;
    }
  }
  if (sk) {
    st = grow(ctx, ctx->wg_word, nseg * sizeof(unsigned long long), true);
    if (st) return st;
    st = grow(ctx, ctx->wg_prefix, (nseg + 1) * sizeof(uint32_t), false);
    if (st) return st;
    st = grow(ctx, ctx->gen, sizeof(uint32_t), true);
    if (st) return st;
    st = grow(ctx, ctx->halo, nseg * sgeo.lag * 4 * sizeof(unsigned long long), true);
    if (st) return st;
    st = grow(ctx, ctx->seg_ctr, 2 * sizeof(uint32_t), true);
    if (st) return st;
  }

  if (nspec > 1) {
    // the power pass of harmonic mode keeps its own table, so that a call
    // repeating an earlier one re-uploads neither
    DevBuf &buf = power_only ? ctx->pdescs : ctx->descs;
    std::vector<SpecDesc> &last = power_only ? ctx->last_pdescs : ctx->last_descs;
    const bool same = last.size() == descs.size() &&
                      memcmp(last.data(), descs.data(), descs.size() * sizeof(SpecDesc)) == 0;
    if (!same) {
      st = grow(ctx, buf, descs.size() * sizeof(SpecDesc), false);
      if (st) return st;
      st = upload(ctx, buf.p, descs.data(), descs.size() * sizeof(SpecDesc), stream);
      if (st) return st;
      last = descs;
    }
    bp.descs = static_cast<const SpecDesc *>(buf.p);
  }

  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ctx->timing && !power_only && stream != ctx->cap_stream &&
      ctx->timing_seen++ % (uint64_t)ctx->timing == 0) {
    e0 = take_event(ctx);
    e1 = take_event(ctx);
    if (!e0 || !e1) return PULSCAN_EHIP;
    HIP_TRY(hipEventRecord(e0, stream));
  }
  if (sk) {
    StreamParams sp{};
    sp.descs = bp.descs;
    sp.single = descs[0];
    sp.nspec = nspec;
    sp.total_blocks = blocks;
    sp.nwg = (uint32_t)nwg;
    sp.nseg = (uint32_t)nseg;
    sp.chunk = a.chunk;
    sp.block = sblock;
    sp.zmax_max = zmax_max;
    sp.g = sgeo;
    sp.mode = search ? kModeSearch : kModeTables;
    sp.dense = a.opts.dense ? 1 : 0;
    sp.from_power = a.from_power ? 1 : 0;
    sp.spin = ctx->spin;
    sp.pool = bp.pool;
    sp.pool_cap = pool_cap;
    sp.pool_head = &cnt->head;
    sp.wg_word = static_cast<unsigned long long *>(ctx->wg_word.p);
    sp.wg_prefix = static_cast<uint32_t *>(ctx->wg_prefix.p);
    sp.gen = static_cast<uint32_t *>(ctx->gen.p);
    sp.seg_ctr = static_cast<uint32_t *>(ctx->seg_ctr.p);
    sp.halo = static_cast<unsigned long long *>(ctx->halo.p);
    sp.total = &cnt->total;
    sp.total2 = bp.total2;
    sp.overflow = &cnt->overflow;
    sp.M = a.M;
    sp.I = a.I;
    sp.P_out = a.P_out;
    sp.stats_out = a.stats_out;
    HIP_TRY(launch_stream(sp, stream));
    ctx->last_kernel = PULSCAN_KERNEL_STREAM;
  } else {
    HIP_TRY(launch_bank(g, bp, tiles, stream));
    ctx->last_kernel = PULSCAN_KERNEL_TILED;
  }
  if (e1) {
    HIP_TRY(hipEventRecord(e1, stream));
    ctx->ev_rec.emplace_back(e0, e1);
  }
  if (!search) return PULSCAN_OK;
  if (!sk && !bp.scan_in_kernel) {
    BigScan bs{};
    bs.tile_word = bp.tile_word;
    bs.tile_prefix = bp.tile_prefix;
    bs.span_sum = static_cast<uint32_t *>(ctx->span_sum.p);
    bs.span_prefix = static_cast<uint32_t *>(ctx->span_prefix.p);
    bs.total_tiles = tiles;
    bs.pool_head = bp.pool_head;
    bs.pool_cap = pool_cap;
    bs.total = bp.total;
    bs.total2 = bp.total2;
    bs.overflow = bp.overflow;
    bs.lost = &cnt->lost;
    if (launch_scan_big(bs, stream) != hipSuccess) {
      (void)hipGetLastError();
      ctx->counts_dirty = true;
      drop_graph(ctx);
      return PULSCAN_EHIP;
    }
  }

  // emit into the caller's device buffer, or into ours for a host copy; with
  // best_per_chunk everything goes to scratch first
  pulscan_candidates *out = a.out;
  pulscan_candidate *dst = out->data;
  uint64_t cap = out->capacity;
  if (!out->on_device) {
    if (cap > worst) cap = worst;
    st = grow(ctx, ctx->outbuf, (size_t)cap * sizeof(pulscan_candidate), false);
    if (st) return st;
    dst = static_cast<pulscan_candidate *>(ctx->outbuf.p);
  }
  EmitParams ep{};
  ep.descs = nspec > 1 ? bp.descs : nullptr;
  ep.nspec = nspec;
  ep.pool = bp.pool;
  ep.pool_cap = pool_cap;
  ep.tile_prefix = sk ? static_cast<const uint32_t *>(ctx->wg_prefix.p) : bp.tile_prefix;
  ep.span_prefix = (sk || bp.scan_in_kernel) ? nullptr
                                             : static_cast<const uint32_t *>(ctx->span_prefix.p);
  ep.total = bp.total;
  ep.chunk = a.chunk;
  ep.rblock = (uint32_t)a.opts.rblock;
  ep.out = dst;
  ep.capacity = cap;
  ep.fp16 = fp16 ? 1 : 0;
  ep.from_power = a.from_power ? 1 : 0;
  ep.block = a.block;
  ep.sigma = a.sigma;
  ep.overflow = &cnt->overflow;
  ep.tile_word = sk ? nullptr : bp.tile_word;
  ep.ntiles = sk ? 0 : tiles;
  ep.pool_head = &cnt->head;
  if (fin) {
    st = grow(ctx, ctx->allbuf, (size_t)pool_cap * sizeof(pulscan_candidate), false);
    if (st) return st;
    ep.out = static_cast<pulscan_candidate *>(ctx->allbuf.p);
    ep.capacity = pool_cap;
  }
  const uint64_t work = ep.capacity < worst ? ep.capacity : worst;
  const uint32_t egrid = (uint32_t)(work / 64 + 1 < 2048 ? work / 64 + 1 : 2048);
  HIP_TRY(launch_emit(ep, descs[0], egrid, stream));
  if (fin)
    HIP_TRY(launch_finalize(ep.out, bp.total, pool_cap, dst, cap, &cnt->best,
                            reinterpret_cast<unsigned long long *>(out->count_device),
                            &cnt->overflow, best ? 1 : 0, stream));
  if (pend) {
    pend->cnt = cnt;
    pend->best = fin;
    pend->cap = cap;
    pend->host = !out->on_device;
  }
  return PULSCAN_OK;
}

// Wait for a queued search and deliver its count (and host copy).
int finish(pulscan_ctx *ctx, const RunArgs &a, const Pending &pd) {
  hipStream_t stream = (hipStream_t)a.opts.stream;
  pulscan_candidates *out = a.out;
  Counters hc{};
  HIP_TRY(hipMemcpyAsync(&hc, pd.cnt, sizeof(hc), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  if (hc.overflow == 2) {
    // a count never arrived: its workgroup may have reserved pool entries or
    // published its word after the scan re-armed them, so the next launch
    // clears the counters first (directly, not from a captured graph)
    ctx->counts_dirty = true;
    drop_graph(ctx);
    return PULSCAN_EHIP;
  }
  if (hc.overflow) return PULSCAN_ENOMEM;
  const unsigned long long total = pd.best ? hc.best : hc.total;
  out->count = total;
  if (pd.host) {
    const uint64_t ncopy = total < pd.cap ? total : pd.cap;
    if (ncopy) {
      HIP_TRY(hipMemcpyAsync(out->data, ctx->outbuf.p, ncopy * sizeof(pulscan_candidate),
                             hipMemcpyDeviceToHost, stream));
      HIP_TRY(hipStreamSynchronize(stream));
    }
  }
  return total > out->capacity ? PULSCAN_EOVERFLOW : PULSCAN_OK;
}

// Harmonic summing: the normalised power of every spectrum is written once,
// stages 2..numharm are built from it, and all stages of all spectra are
// searched in one fused launch (power input), stage by stage in canonical
// order.
int enqueue_harmonics(pulscan_ctx *ctx, const std::vector<SpecIn> &specs, const RunArgs &a,
                      Pending *pend) {
  hipStream_t stream = (hipStream_t)a.opts.stream;
  const uint32_t nh = (uint32_t)a.opts.numharm;
  const int nspec = (int)specs.size();
  uint64_t pn = 0, sn = 0;
  uint32_t n_max = 0;
  for (const SpecIn &s : specs) {
    pn += s.n;
    sn += harmonic_offset(s.n, nh + 1);
    n_max = s.n > n_max ? (uint32_t)s.n : n_max;
  }
  int st = grow(ctx, ctx->hpow, pn * sizeof(float), false);
  if (st) return st;
  st = grow(ctx, ctx->hsum, (sn ? sn : 1) * sizeof(float), false);
  if (st) return st;
  float *P = static_cast<float *>(ctx->hpow.p);
  float *S = static_cast<float *>(ctx->hsum.p);

  // 1. normalised power of every spectrum
  std::vector<SpecIn> ps(specs);
  std::vector<HarmJob> jobs(nspec);
  uint64_t po = 0, so = 0;
  for (int s = 0; s < nspec; ++s) {
    ps[s].aux = P + po;
    jobs[s] = HarmJob{P + po, S + so, (uint32_t)specs[s].n, nh};
    po += specs[s].n;
    so += harmonic_offset(specs[s].n, nh + 1);
  }
  RunArgs ap = a;
  ap.kind = kRunPower;
  st = enqueue(ctx, ps, ap, nullptr);
  if (st) return st;

  // 2. stages 2..numharm
  const HarmJob *jobs_dev = nullptr;
  if (nspec > 1) {
    const bool same = ctx->last_hjobs.size() == jobs.size() &&
                      memcmp(ctx->last_hjobs.data(), jobs.data(), jobs.size() * sizeof(HarmJob)) == 0;
    if (!same) {
      st = grow(ctx, ctx->hjobs, jobs.size() * sizeof(HarmJob), false);
      if (st) return st;
      st = upload(ctx, ctx->hjobs.p, jobs.data(), jobs.size() * sizeof(HarmJob), stream);
      if (st) return st;
      ctx->last_hjobs = jobs;
    }
    jobs_dev = static_cast<const HarmJob *>(ctx->hjobs.p);
  }
  HIP_TRY(launch_harmonics(jobs_dev, jobs[0], nspec, n_max, stream));

  // 3. every stage of every spectrum, searched on its power
  std::vector<SpecIn> stages;
  for (int s = 0; s < nspec; ++s) {
    for (uint32_t H = 1; H <= nh; ++H) {
      const uint64_t m = specs[s].n / H;
      if (m == 0) break;
      SpecIn si{};
      si.x = H == 1 ? (const void *)jobs[s].P
                    : (const void *)(jobs[s].S + harmonic_offset(specs[s].n, H));
      si.n = m;
      si.zmax = specs[s].zmax;
      si.dofmul = H * (H + 1) / 2;
      si.spec_id = specs[s].spec_id;
      si.harm = H;
      stages.push_back(si);
    }
  }
  RunArgs as = a;
  as.from_power = true;
  return enqueue(ctx, stages, as, pend);
}

int enqueue_any(pulscan_ctx *ctx, const std::vector<SpecIn> &specs, const RunArgs &a,
                Pending *pend) {
  if (a.kind == kRunSearch && a.opts.numharm > 1) return enqueue_harmonics(ctx, specs, a, pend);
  return enqueue(ctx, specs, a, pend);
}

// Graph-mode key: everything a replay bakes in.
std::vector<uint64_t> graph_key_of(const std::vector<SpecIn> &specs, const RunArgs &a) {
  std::vector<uint64_t> k;
  k.push_back(specs.size());
  for (const SpecIn &s : specs) {
    k.push_back((uint64_t)(uintptr_t)s.x);
    k.push_back(s.n);
    k.push_back(s.zmax);
  }
  pulscan_opts o = a.opts;
  o.stream = nullptr;
  o.async = 0;
  const uint64_t *ow = reinterpret_cast<const uint64_t *>(&o);
  for (size_t i = 0; i < sizeof(o) / 8; ++i) k.push_back(ow[i]);
  uint32_t sb;
  memcpy(&sb, &a.sigma, 4);
  k.push_back(((uint64_t)a.chunk << 32) | a.block);
  k.push_back(((uint64_t)a.tile << 32) | sb);
  k.push_back((uint64_t)(uintptr_t)a.out->data);
  k.push_back(a.out->capacity);
  k.push_back((uint64_t)a.out->on_device);
  k.push_back((uint64_t)(uintptr_t)a.out->count_device);
  return k;
}

void drop_graph(pulscan_ctx *ctx) {
  if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
  ctx->graph_exec = nullptr;
  ctx->graph_key.clear();
}

// A search replayed from a captured graph: the first call with a given set
// of arguments runs normally (growing buffers and filling the caches), then
// its launches are captured on the context's own stream; later calls with
// the same arguments launch the graph on the caller's stream.
int run_graph(pulscan_ctx *ctx, const std::vector<SpecIn> &specs, const RunArgs &a) {
  hipStream_t stream = (hipStream_t)a.opts.stream;
  std::vector<uint64_t> key = graph_key_of(specs, a);
  Pending pd;
  if (!(ctx->graph_exec && key == ctx->graph_key && ctx->epoch == ctx->graph_epoch)) {
    drop_graph(ctx);
    int st = enqueue_any(ctx, specs, a, &pd);
    if (st) return st;
    HIP_TRY(hipStreamSynchronize(stream));
    RunArgs c = a;
    c.opts.stream = ctx->cap_stream;
    hipGraph_t graph = nullptr;
    const uint64_t before = ctx->epoch;
    HIP_TRY(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
    st = enqueue_any(ctx, specs, c, &pd);
    const hipError_t ce = hipStreamEndCapture(ctx->cap_stream, &graph);
    if (!st && ce == hipSuccess && ctx->epoch != before) st = PULSCAN_EHIP;  // cannot happen
    if (st || ce != hipSuccess) {
      (void)hipGetLastError();
      if (graph) (void)hipGraphDestroy(graph);
      // captured work never ran: forget what it would have put on the device
      thr_forget_new(ctx);
      ctx->last_descs.clear();
      ctx->last_pdescs.clear();
      ctx->last_hjobs.clear();
      ++ctx->epoch;
      return st ? st : PULSCAN_EHIP;
    }
    const hipError_t ie = hipGraphInstantiate(&ctx->graph_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) {
      (void)hipGetLastError();
      ctx->graph_exec = nullptr;
      return PULSCAN_EHIP;
    }
    ctx->graph_key = key;
    ctx->graph_epoch = ctx->epoch;
    // this call's results came from the direct run
    return a.opts.async ? PULSCAN_OK : finish(ctx, a, pd);
  }
  HIP_TRY(hipGraphLaunch(ctx->graph_exec, stream));
  if (a.opts.async) return PULSCAN_OK;
  // the same launches as the captured run: its buffers and flags
  pd.cnt = static_cast<Counters *>(ctx->counters.p);
  pd.best = a.opts.best_per_chunk != 0 || a.opts.power_fp16 != 0;
  pd.host = !a.out->on_device;
  uint64_t worst = 0;
  for (const SpecIn &s : specs)
    for (uint32_t H = 1; H <= (uint32_t)(a.opts.numharm > 1 ? a.opts.numharm : 1); ++H)
      worst += (s.n / H + a.chunk - 1) / a.chunk * (uint64_t)s.zmax;
  pd.cap = a.out->capacity;
  if (pd.host && pd.cap > worst) pd.cap = worst;
  return finish(ctx, a, pd);
}

int run(pulscan_ctx *ctx, std::vector<SpecIn> specs, const RunArgs &a) {
  HIP_TRY(hipSetDevice(ctx->device));
  for (size_t s = 0; s < specs.size(); ++s) specs[s].spec_id = (uint32_t)s;
  if (a.kind == kRunSearch && a.opts.graph) return run_graph(ctx, specs, a);
  Pending pd;
  int st = enqueue_any(ctx, specs, a, &pd);
  if (st) return st;
  if (a.kind != kRunSearch) {
    HIP_TRY(hipStreamSynchronize((hipStream_t)a.opts.stream));
    return PULSCAN_OK;
  }
  return a.opts.async ? PULSCAN_OK : finish(ctx, a, pd);
}

// Autotuner of the batched call with chunk 0: every (chunk, tile) the
// kernels accept, chunk from {256, 1024, 4096}, is timed on the batch itself
// (the second of two runs, the first warms the caches), and the fastest is
// kept for batches of the same signature.  The chunk changes what the search
// reports and is returned to the caller; the tile only changes the speed.
int autotune(pulscan_ctx *ctx, const std::vector<SpecIn> &specs, const RunArgs &a,
             uint32_t *chunk_out, uint32_t *tile_out) {
  std::vector<uint64_t> sig;
  uint64_t nsum = 0;
  uint32_t zmax_max = 0;
  for (const SpecIn &s : specs) {
    nsum += s.n;
    zmax_max = s.zmax > zmax_max ? s.zmax : zmax_max;
  }
  sig.push_back(specs.size());
  sig.push_back(nsum >> 20);
  sig.push_back(zmax_max);
  sig.push_back((uint64_t)a.opts.norm_block);
  sig.push_back((uint64_t)a.opts.numharm);
  sig.push_back((uint64_t)a.opts.width_search);
  sig.push_back((uint64_t)a.opts.dense);
  sig.push_back((uint64_t)a.opts.power_fp16);
  sig.push_back((uint64_t)a.opts.norm);
  sig.push_back((uint64_t)ctx->kernel);
  for (auto &e : ctx->tuned)
    if (e.first == sig) {
      *chunk_out = e.second.first;
      *tile_out = e.second.second;
      return PULSCAN_OK;
    }
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t stream = (hipStream_t)a.opts.stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  float best_ms = INFINITY;
  uint32_t best_c = 0, best_t = 0;
  int st = PULSCAN_OK;
  static const uint32_t chunks[] = {256, 1024, 4096};
  for (uint32_t C : chunks) {
    const uint32_t B = a.opts.norm_block > 0 ? (uint32_t)a.opts.norm_block : C;
    bool ok = true;
    uint64_t worst = 0;
    for (const SpecIn &s : specs) {
      uint32_t b = 0;
      if (check_spectrum(s.x, s.n, (int)s.zmax, (int)C, a.opts, &b) != PULSCAN_OK) ok = false;
      for (uint32_t H = 1; H <= (uint32_t)(a.opts.numharm > 1 ? a.opts.numharm : 1); ++H)
        worst += (s.n / H + C - 1) / C * (uint64_t)s.zmax;
    }
    if (!ok) continue;
    st = grow(ctx, ctx->tune_out, (size_t)(worst + 1) * sizeof(pulscan_candidate), false);
    if (st) break;
    Counters *cnt = nullptr;
    // where the streaming kernel serves the search it is the only candidate
    // (tile 0), so that a later call with the returned chunk and no tile
    // runs the same kernel and reports the same bits
    StreamGeometry sg{};
    const bool from_power = a.opts.numharm > 1;
    int socc = 0;
    const bool sk = choose_stream_geometry(C, B, zmax_max, from_power,
                                           a.opts.norm == PULSCAN_NORM_EXACT,
                                           a.opts.power_fp16 != 0, &sg) &&
                    (socc = stream_occ(ctx, sg, from_power)) > 0 &&
                    wants_stream(ctx, specs, 64u * (uint32_t)sg.EPL, from_power, socc);
    const std::vector<uint32_t> tiles =
        sk ? std::vector<uint32_t>{0u} : tile_choices(C, B, zmax_max, a.opts.power_fp16 != 0);
    for (uint32_t T : tiles) {
      RunArgs t = a;
      t.chunk = C;
      t.block = B;
      t.tile = T;
      pulscan_candidates o{};
      o.data = static_cast<pulscan_candidate *>(ctx->tune_out.p);
      o.capacity = worst + 1;
      o.on_device = 1;
      t.out = &o;
      t.opts.async = 1;
      t.opts.graph = 0;
      float ms = INFINITY;
      for (int rep = 0; rep < 2 && st == PULSCAN_OK; ++rep) {
        HIP_TRY(hipEventRecord(e0, stream));
        Pending pd;
        st = enqueue_any(ctx, specs, t, &pd);
        cnt = pd.cnt;
        HIP_TRY(hipEventRecord(e1, stream));
        HIP_TRY(hipEventSynchronize(e1));
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      }
      if (st == PULSCAN_EUNSUPPORTED) {
        st = PULSCAN_OK;
        continue;
      }
      if (st) break;
      (void)cnt;
      if (ms < best_ms) {
        best_ms = ms;
        best_c = C;
        best_t = T;
      }
    }
    if (st) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) return st;
  if (best_c == 0) return PULSCAN_EUNSUPPORTED;
  ctx->tuned.emplace_back(sig, std::make_pair(best_c, best_t));
  *chunk_out = best_c;
  *tile_out = best_t;
  return PULSCAN_OK;
}

std::mutex g_default_mu;
pulscan_ctx *g_default = nullptr;

}  // namespace

namespace pulscan {
int check_search_args(const void *x, uint64_t n, int zmax, int chunk, const pulscan_opts &o,
                      uint32_t *block) {
  return check_spectrum(x, n, zmax, chunk, o, block);
}
}  // namespace pulscan

extern "C" {

const char *pulscan_strerror(int status) {
  switch (status) {
    case PULSCAN_OK: return "ok";
    case PULSCAN_EINVAL: return "invalid argument";
    case PULSCAN_ENOMEM: return "out of memory";
    case PULSCAN_EOVERFLOW: return "more candidates than the output capacity";
    case PULSCAN_EHIP: return "HIP runtime error";
    case PULSCAN_EUNSUPPORTED: return "unsupported by the GPU kernels";
    default: return "unknown status";
  }
}

void pulscan_opts_default(pulscan_opts *o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->norm = PULSCAN_NORM_MOM;
  o->width_search = PULSCAN_W_ALL;
  o->numharm = 1;
}

int pulscan_ctx_create(pulscan_ctx **out, int device) {
  if (!out) return PULSCAN_EINVAL;
  *out = nullptr;
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return PULSCAN_EINVAL;
  HIP_TRY(hipSetDevice(device));
  pulscan_ctx *ctx = new (std::nothrow) pulscan_ctx();
  if (!ctx) return PULSCAN_ENOMEM;
  ctx->device = device;
  if (hipDeviceGetAttribute(&ctx->n_cu, hipDeviceAttributeMultiprocessorCount, device) !=
          hipSuccess ||
      hipEventCreateWithFlags(&ctx->pinned_ev, hipEventDisableTiming) != hipSuccess ||
      hipStreamCreate(&ctx->cap_stream) != hipSuccess) {
    (void)hipGetLastError();
    pulscan_ctx_destroy(ctx);
    return PULSCAN_EHIP;
  }
  *out = ctx;
  return PULSCAN_OK;
}

void pulscan_ctx_destroy(pulscan_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  drop_graph(ctx);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  for (void *p : ctx->thr_arenas) (void)hipFree(p);
  DevBuf *bufs[] = {&ctx->pool,   &ctx->tile_word, &ctx->tile_prefix,
                    &ctx->counters, &ctx->outbuf, &ctx->descs,  &ctx->jobs,
                    &ctx->allbuf, &ctx->hpow,   &ctx->hsum,     &ctx->hjobs,
                    &ctx->tune_out, &ctx->stats,  &ctx->pdescs,
                    &ctx->span_sum, &ctx->span_prefix, &ctx->wg_word, &ctx->wg_prefix,
                    &ctx->gen,      &ctx->halo,      &ctx->seg_ctr};
  for (DevBuf *b : bufs)
    if (b->p) (void)hipFree(b->p);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->pinned_ev) (void)hipEventDestroy(ctx->pinned_ev);
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  for (auto &pr : ctx->ev_rec) {
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  delete ctx;
}

int pulscan_search_ex(pulscan_ctx *ctx, const pulscan_complex *spectrum, size_t nbins, int zmax,
                      int chunk, float sigma_thresh, const pulscan_opts *opts,
                      pulscan_candidates *out) {
  pulscan_opts o;
  pulscan_opts_default(&o);
  if (opts) o = *opts;
  if (!ctx || !isfinite(sigma_thresh)) return PULSCAN_EINVAL;
  int st = check_out(out, o.async != 0);
  if (st) return st;
  uint32_t block = 0;
  st = check_spectrum(spectrum, nbins, zmax, chunk, o, &block);
  if (st) return st;
  RunArgs a;
  a.kind = kRunSearch;
  a.chunk = (uint32_t)chunk;
  a.block = block;
  a.sigma = sigma_thresh;
  a.opts = o;
  a.out = out;
  std::vector<SpecIn> specs{SpecIn{spectrum, (uint64_t)nbins, (uint32_t)zmax}};
  return run(ctx, specs, a);
}

int pulscan_search(const pulscan_complex *spectrum, size_t nbins, int zmax, int chunk,
                   float sigma_thresh, pulscan_candidates *out) {
  std::lock_guard<std::mutex> lock(g_default_mu);
  if (!g_default) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    int st = pulscan_ctx_create(&g_default, dev);
    if (st) return st;
  }
  pulscan_opts o;
  pulscan_opts_default(&o);
  return pulscan_search_ex(g_default, spectrum, nbins, zmax, chunk, sigma_thresh, &o, out);
}

int pulscan_search_batched(pulscan_ctx *ctx, int nspec, const pulscan_complex *const *spectra,
                           const uint64_t *nbins, const int32_t *zmax, int chunk,
                           float sigma_thresh, const pulscan_opts *opts, pulscan_candidates *out,
                           int *chunk_used) {
  pulscan_opts o;
  pulscan_opts_default(&o);
  if (opts) o = *opts;
  if (!ctx || nspec < 1 || !spectra || !nbins || !zmax || chunk < 0 || !isfinite(sigma_thresh))
    return PULSCAN_EINVAL;
  int st = check_out(out, o.async != 0);
  if (st) return st;
  std::vector<SpecIn> specs(nspec);
  for (int s = 0; s < nspec; ++s) {
    if (!spectra[s] || zmax[s] < 1 || nbins[s] == 0) return PULSCAN_EINVAL;
    specs[s] = SpecIn{spectra[s], nbins[s], (uint32_t)zmax[s]};
  }
  RunArgs a;
  a.kind = kRunSearch;
  a.sigma = sigma_thresh;
  a.opts = o;
  a.out = out;
  uint32_t c = (uint32_t)chunk, tile = 0;
  if (chunk == 0) {
    // validate at the default chunk first, so that argument errors are not
    // masked by the tuner's search over chunks
    for (int s = 0; s < nspec; ++s) {
      uint32_t b = 0;
      st = check_spectrum(spectra[s], nbins[s], zmax[s], 1024, o, &b);
      if (st == PULSCAN_EINVAL) return st;
    }
    st = autotune(ctx, specs, a, &c, &tile);
    if (st) return st;
  }
  uint32_t block = 0;
  for (int s = 0; s < nspec; ++s) {
    uint32_t b = 0;
    st = check_spectrum(spectra[s], nbins[s], zmax[s], (int)c, o, &b);
    if (st) return st;
    block = b;
  }
  if (chunk_used) *chunk_used = (int)c;
  a.chunk = c;
  a.block = block;
  a.tile = tile;
  return run(ctx, specs, a);
}

int pulscan_debug_tables(pulscan_ctx *ctx, const pulscan_complex *spectrum, size_t nbins,
                         int zmax, int chunk, const pulscan_opts *opts, float *M, uint32_t *I,
                         float *power, float *stats) {
  pulscan_opts o;
  pulscan_opts_default(&o);
  if (opts) o = *opts;
  o.async = 0;
  if (!ctx || !M || !I) return PULSCAN_EINVAL;
  uint32_t block = 0;
  int st = check_spectrum(spectrum, nbins, zmax, chunk, o, &block);
  if (st) return st;
  RunArgs a;
  a.kind = kRunTables;
  a.chunk = (uint32_t)chunk;
  a.block = block;
  a.opts = o;
  a.M = M;
  a.I = I;
  a.P_out = power;
  a.stats_out = stats;
  std::vector<SpecIn> specs{SpecIn{spectrum, (uint64_t)nbins, (uint32_t)zmax}};
  return run(ctx, specs, a);
}

int pulscan_debug_bank_from_power(pulscan_ctx *ctx, const float *power, size_t nbins, int zmax,
                                  int chunk, float *M, uint32_t *I) {
  if (!ctx || !power || !M || !I || zmax < 1 || chunk < 1 || nbins == 0 ||
      nbins >= (1ull << 32) || nbins < (size_t)zmax)
    return PULSCAN_EINVAL;
  if (chunk % 64 != 0 || chunk > kMaxTile) return PULSCAN_EUNSUPPORTED;
  const uint64_t nchunks = (nbins + chunk - 1) / chunk;
  if (nchunks * (uint64_t)zmax >= (1ull << 32)) return PULSCAN_EUNSUPPORTED;
  RunArgs a;
  a.kind = kRunTables;
  a.from_power = true;
  a.chunk = (uint32_t)chunk;
  a.block = 64;
  pulscan_opts_default(&a.opts);
  a.M = M;
  a.I = I;
  std::vector<SpecIn> specs{SpecIn{power, (uint64_t)nbins, (uint32_t)zmax}};
  return run(ctx, specs, a);
}

int pulscan_threshold_table(pulscan_ctx *ctx, int zmax, float sigma_thresh, double ntrials,
                            int width_search, float *T_host) {
  if (!ctx || zmax < 1 || !T_host || !isfinite(sigma_thresh) || !isfinite(ntrials) ||
      ntrials < 1.0)
    return PULSCAN_EINVAL;
  if (width_search != PULSCAN_W_ALL && width_search != PULSCAN_W_LOG2) return PULSCAN_EINVAL;
  HIP_TRY(hipSetDevice(ctx->device));
  DevBuf tmp;
  if (hipMalloc(&tmp.p, (size_t)zmax * sizeof(float)) != hipSuccess) {
    (void)hipGetLastError();
    return PULSCAN_ENOMEM;
  }
  ThreshJob job{static_cast<float *>(tmp.p), (uint32_t)zmax, (uint32_t)zmax, ntrials, 1u, 0u};
  int st = PULSCAN_OK;
  if (launch_thresholds(nullptr, job, 1, (uint32_t)zmax, (double)sigma_thresh, width_search, 0,
                        nullptr) != hipSuccess ||
      hipMemcpy(T_host, tmp.p, (size_t)zmax * sizeof(float), hipMemcpyDeviceToHost) !=
          hipSuccess) {
    (void)hipGetLastError();
    st = PULSCAN_EHIP;
  }
  (void)hipFree(tmp.p);
  return st;
}

int pulscan_ctx_set_timing(pulscan_ctx *ctx, int enable) {
  if (!ctx) return PULSCAN_EINVAL;
  if (enable < 0) return PULSCAN_EINVAL;
  ctx->timing = enable;
  ctx->timing_seen = 0;
  if (ctx->timing) {
    // create the events up front so that timed calls do not create any
    HIP_TRY(hipSetDevice(ctx->device));
    while (ctx->ev_pool.size() < 2048) {
      hipEvent_t e = nullptr;
      HIP_TRY(hipEventCreate(&e));
      ctx->ev_pool.push_back(e);
    }
  }
  return PULSCAN_OK;
}

int pulscan_ctx_set_kernel(pulscan_ctx *ctx, int kernel) {
  if (!ctx || (kernel != PULSCAN_KERNEL_STREAM && kernel != PULSCAN_KERNEL_TILED &&
               kernel != PULSCAN_KERNEL_AUTO))
    return PULSCAN_EINVAL;
  if (kernel != ctx->kernel) drop_graph(ctx);
  ctx->kernel = kernel;
  return PULSCAN_OK;
}

int pulscan_ctx_set_spin(pulscan_ctx *ctx, uint32_t polls) {
  if (!ctx || polls < 1) return PULSCAN_EINVAL;
  if (polls != ctx->spin) drop_graph(ctx);
  ctx->spin = polls;
  return PULSCAN_OK;
}

int pulscan_ctx_last_kernel(pulscan_ctx *ctx, int *kernel) {
  if (!ctx || !kernel) return PULSCAN_EINVAL;
  *kernel = ctx->last_kernel;
  return PULSCAN_OK;
}

int pulscan_ctx_kernel_time(pulscan_ctx *ctx, double *total_ms, uint64_t *launches) {
  if (!ctx || !total_ms || !launches) return PULSCAN_EINVAL;
  HIP_TRY(hipSetDevice(ctx->device));
  double sum = 0.0;
  int st = PULSCAN_OK;
  for (auto &pr : ctx->ev_rec) {
    float ms = 0.f;
    if (hipEventSynchronize(pr.second) != hipSuccess ||
        hipEventElapsedTime(&ms, pr.first, pr.second) != hipSuccess) {
      (void)hipGetLastError();
      st = PULSCAN_EHIP;
    }
    sum += ms;
    ctx->ev_pool.push_back(pr.first);
    ctx->ev_pool.push_back(pr.second);
  }
  *launches = ctx->ev_rec.size();
  *total_ms = sum;
  ctx->ev_rec.clear();
  return st;
}

}  // extern "C"

// pulscan_search_noalloc: the single-spectrum search for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).  It runs the same kernels as
// pulscan_search_ex (thresholds, the streaming bank kernel, emit) with every
// piece of scratch memory they need taken from one file-scope device array,
// `scratch`, which each GPU holds from the library's load until the process
// ends.  Nothing here calls hipMalloc, hipFree or an allocating library
// routine.
//
// Layout of `scratch` (byte offsets, each 256-aligned):
//   control  counters (total, head, overflow) and the launch generation
//   thr      one threshold table (zmax <= kNaMaxZ widths)
//   wg       per-workgroup count words and prefixes (<= kNaMaxWg workgroups)
//   halo     per-workgroup published halo statistics
//   pool     candidate staging (kNaPoolEntries entries)
#include <math.h>
#include <string.h>

#include <mutex>

#include "internal.hpp"

namespace pulscan {
namespace {

constexpr uint32_t kNaMaxZ = 4096;          // widths of the threshold table
constexpr uint32_t kNaMaxWg = 2048;         // streaming-kernel workgroups
constexpr uint32_t kNaMaxLag = kStreamBatch;  // halo blocks per workgroup
constexpr size_t kNaPoolEntries = 1u << 20;   // staged candidates per call

constexpr size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct NaCounters {
  unsigned long long total;
  uint32_t head;
  uint32_t overflow;
  uint32_t gen;
  uint32_t pad[3];
};

constexpr size_t kOffCtl = 0;
constexpr size_t kOffThr = align256(kOffCtl + sizeof(NaCounters));
constexpr size_t kOffWord = align256(kOffThr + kNaMaxZ * sizeof(float));
constexpr size_t kOffPrefix = align256(kOffWord + kNaMaxWg * sizeof(unsigned long long));
constexpr size_t kOffHalo = align256(kOffPrefix + (kNaMaxWg + 1) * sizeof(uint32_t));
constexpr size_t kOffPool =
    align256(kOffHalo + (size_t)kNaMaxWg * kNaMaxLag * 4 * sizeof(unsigned long long));
constexpr size_t kScratchBytes = align256(kOffPool + kNaPoolEntries * sizeof(StageEntry));
// the part that must start at zero: counters, generation, count and halo words
constexpr size_t kClearBytes = kOffPool;

}  // namespace

// Device-side home of every buffer the no-allocation search uses (about 25
// MiB per GPU).  In host code this name is a host-side stand-in: only the
// address hipGetSymbolAddress returns may be passed to kernels or copies.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// Fill n 32-bit words with zero: clears the control area with a kernel, which
// (unlike a memset node) replays correctly inside a captured graph.
__global__ void na_clear_kernel(uint32_t *p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// Re-arm the pool head and the overflow flag before a search (a search that
// gave up on a count may leave the head advanced).
__global__ void na_arm_kernel(NaCounters *c) {
  if (threadIdx.x == 0) {
    c->head = 0u;
    c->overflow = 0u;
  }
}

struct NaDevice {
  unsigned char *ptr = nullptr;  // device address of `scratch` on this GPU
  bool cleared = false;          // its control area has been cleared once
  int n_cu = 0;
};
constexpr int kNaMaxDevices = 64;
std::mutex g_na_mu;
NaDevice g_na[kNaMaxDevices];

// The scratch address of the current device, looked up once per device.
int na_device(int dev, NaDevice **out) {
  if (dev < 0 || dev >= kNaMaxDevices) return PULSCAN_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_na_mu);
  NaDevice &d = g_na[dev];
  if (!d.ptr) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return PULSCAN_EHIP;
    }
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        ncu < 1) {
      (void)hipGetLastError();
      return PULSCAN_EHIP;
    }
    d.ptr = static_cast<unsigned char *>(p);
    d.n_cu = ncu;
  }
  *out = &d;
  return PULSCAN_OK;
}

#define NA_TRY(call)                        \
  do {                                      \
    if ((call) != hipSuccess) {             \
      (void)hipGetLastError();              \
      return PULSCAN_EHIP;                  \
    }                                       \
  } while (0)

}  // namespace
}  // namespace pulscan

using namespace pulscan;

extern "C" int pulscan_search_noalloc(const pulscan_complex *spectrum, size_t nbins, int zmax,
                                      int chunk, float sigma_thresh, const pulscan_opts *opts,
                                      pulscan_candidates *out) {
  pulscan_opts o;
  pulscan_opts_default(&o);
  if (opts) o = *opts;
  if (!isfinite(sigma_thresh) || !out) return PULSCAN_EINVAL;
  if (out->capacity > 0 && !out->data) return PULSCAN_EINVAL;
  if (!out->on_device) return PULSCAN_EINVAL;  // a host copy would need a staging buffer
  if (o.async && !out->count_device) return PULSCAN_EINVAL;
  uint32_t block = 0;
  int st = check_search_args(spectrum, nbins, zmax, chunk, o, &block);
  if (st) return st;
  // what the scratch layout and the streaming kernel cover
  if (o.numharm > 1 || o.best_per_chunk || o.power_fp16 || o.graph ||
      o.norm != PULSCAN_NORM_MOM || (uint32_t)zmax > kNaMaxZ)
    return PULSCAN_EUNSUPPORTED;
  StreamGeometry g{};
  if (!choose_stream_geometry((uint32_t)chunk, block, (uint32_t)zmax, false, false, false, &g) ||
      g.lag > kNaMaxLag)
    return PULSCAN_EUNSUPPORTED;
  const int occ = stream_occupancy(g, false);
  if (occ < 1) return PULSCAN_EUNSUPPORTED;

  int dev = 0;
  NA_TRY(hipGetDevice(&dev));
  NaDevice *nd = nullptr;
  st = na_device(dev, &nd);
  if (st) return st;
  hipStream_t stream = (hipStream_t)o.stream;
  unsigned char *base = nd->ptr;
  NaCounters *ctl = reinterpret_cast<NaCounters *>(base + kOffCtl);
  if (!nd->cleared) {
    // once per device, ordered before this call's kernels.  Under stream
    // capture the clear becomes part of the caller's graph (each replay then
    // starts from cleared words, which is consistent) and is repeated by the
    // next call made outside a capture.
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    NA_TRY(hipStreamIsCapturing(stream, &cs));
    const size_t words = kClearBytes / 4;
    hipLaunchKernelGGL(na_clear_kernel, dim3(256), dim3(256), 0, stream,
                       reinterpret_cast<uint32_t *>(base), words);
    NA_TRY(hipGetLastError());
    if (cs == hipStreamCaptureStatusNone) nd->cleared = true;
  }
  hipLaunchKernelGGL(na_arm_kernel, dim3(1), dim3(64), 0, stream, ctl);
  NA_TRY(hipGetLastError());

  // the series
  const uint32_t n = (uint32_t)nbins;
  const uint32_t sblock = 64u * (uint32_t)g.EPL;
  SpecDesc d{};
  d.x = reinterpret_cast<const float2 *>(spectrum);
  d.n = n;
  d.zmax = (uint32_t)zmax;
  d.zc = round_widths(d.zmax, g.K);
  d.nchunks = (n + (uint32_t)chunk - 1) / (uint32_t)chunk;
  d.dofmul = 1;
  d.harm = 1;
  d.block_begin = 0;
  uint32_t sw = 0;
  for (uint32_t w = 1; w <= d.zmax; ++w) sw += width_searched(w, d.zmax, o.width_search) ? 1u : 0u;
  d.ntrials = o.ntrials > 0.0 ? o.ntrials : (double)n * (double)(sw ? sw : 1u);
  float *thr = reinterpret_cast<float *>(base + kOffThr);
  d.thr = thr;

  // thresholds, every call (no table cache without an allocation)
  ThreshJob job{thr, d.zmax, d.zc, d.ntrials, 1u, 0u};
  NA_TRY(launch_thresholds(nullptr, job, 1, d.zc, (double)sigma_thresh, o.width_search, 0,
                           stream));

  // the streaming bank kernel over the spectrum's blocks
  const uint64_t blocks = (n + sblock - 1) / sblock;
  const uint64_t min_range = g.lag > (uint32_t)kStreamBatch ? g.lag : (uint64_t)kStreamBatch;
  uint64_t nwg = (uint64_t)occ * (uint64_t)nd->n_cu;
  if (nwg > kNaMaxWg) nwg = kNaMaxWg;
  if (blocks / min_range < nwg) nwg = blocks / min_range;
  if (nwg < 1) nwg = 1;
  const uint64_t worst = (uint64_t)d.nchunks * d.zmax;
  const uint32_t pool_cap = (uint32_t)(worst < kNaPoolEntries ? (worst ? worst : 1) : kNaPoolEntries);
  StreamParams sp{};
  sp.descs = nullptr;
  sp.single = d;
  sp.nspec = 1;
  sp.total_blocks = blocks;
  sp.nwg = (uint32_t)nwg;
  sp.nseg = (uint32_t)nwg;  // one range per workgroup: the scratch holds nwg words
  sp.chunk = (uint32_t)chunk;
  sp.block = sblock;
  sp.zmax_max = d.zmax;
  sp.g = g;
  sp.mode = kModeSearch;
  sp.dense = o.dense ? 1 : 0;
  sp.from_power = 0;
  sp.spin = kStreamSpin;
  sp.pool = reinterpret_cast<StageEntry *>(base + kOffPool);
  sp.pool_cap = pool_cap;
  sp.pool_head = &ctl->head;
  sp.wg_word = reinterpret_cast<unsigned long long *>(base + kOffWord);
  sp.wg_prefix = reinterpret_cast<uint32_t *>(base + kOffPrefix);
  sp.gen = &ctl->gen;
  sp.halo = reinterpret_cast<unsigned long long *>(base + kOffHalo);
  sp.total = &ctl->total;
  sp.total2 = reinterpret_cast<unsigned long long *>(out->count_device);
  sp.overflow = &ctl->overflow;
  NA_TRY(launch_stream(sp, stream));

  // canonical placement and significance, into the caller's buffer
  EmitParams ep{};
  ep.descs = nullptr;
  ep.nspec = 1;
  ep.pool = sp.pool;
  ep.pool_cap = pool_cap;
  ep.tile_prefix = sp.wg_prefix;
  ep.span_prefix = nullptr;
  ep.total = &ctl->total;
  ep.chunk = (uint32_t)chunk;
  ep.rblock = (uint32_t)o.rblock;
  ep.out = out->data;
  ep.capacity = out->capacity;
  ep.fp16 = 0;
  ep.from_power = 0;
  ep.block = block;
  ep.sigma = sigma_thresh;
  ep.overflow = &ctl->overflow;
  ep.tile_word = nullptr;  // the streaming kernel's words carry the launch's tag
  ep.ntiles = 0;
  ep.pool_head = &ctl->head;
  const uint64_t work = out->capacity < worst ? out->capacity : worst;
  const uint32_t egrid = (uint32_t)(work / 64 + 1 < 2048 ? work / 64 + 1 : 2048);
  NA_TRY(launch_emit(ep, d, egrid, stream));
  if (o.async) return PULSCAN_OK;

  // synchronous: read the counters back (no staging buffer of ours)
  NaCounters hc{};
  NA_TRY(hipMemcpyAsync(&hc, ctl, sizeof hc, hipMemcpyDeviceToHost, stream));
  NA_TRY(hipStreamSynchronize(stream));
  if (hc.overflow == 2) return PULSCAN_EHIP;  // a workgroup's count never arrived
  out->count = hc.total;
  if (hc.overflow) return PULSCAN_ENOMEM;     // more than kNaPoolEntries candidates
  return hc.total > out->capacity ? PULSCAN_EOVERFLOW : PULSCAN_OK;
}

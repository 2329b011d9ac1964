/*
 * pulscan.h -- C ABI of the MI355X (gfx950) boxcar filter-bank search.
 *
 * The search is the hot path of Pulscan (White et al. 2024): complex
 * Fourier amplitudes are normalised block by block (median / MAD of the
 * real and imaginary parts, section 2.2.3, with the median of medians of
 * section 2.5 and the appendix algorithm "Median of Medians Normalisation"),
 * squared into power (section 2.2.3), filtered by unit boxcars of every width
 * 1..zmax (the recursion of section 2.2.5), reduced to per-chunk maxima for
 * every width (appendix algorithm "Boxcar Filtering Process"), and the maxima
 * whose Bonferroni-corrected Gaussian-equivalent significance reaches a
 * threshold are returned as candidates (section 2.2.3).
 *
 * Conventions shared by every entry point:
 *   - A width w covers bins [bin, bin + w); the paper's drift is z = w - 1
 *     and a width-w boxcar of chi^2(2) powers is chi^2(2w).
 *   - Windows exist only where they fit: bin + w <= nbins.
 *   - Chunk c holds the window starts [c*chunk, min((c+1)*chunk, nbins)).
 *     Each (chunk, width) yields at most one candidate: the largest boxcar
 *     power of that width starting in the chunk, at the smallest such bin.
 *   - The normalisation block defaults to the chunk.  The last, partial block
 *     takes its statistics over the last `block` bins.  A block whose MAD is
 *     0 normalises to 0.  The MAD scale is 1 / Phi^-1(3/4).
 *   - ntrials (the Bonferroni factor) defaults to nbins * (number of
 *     searched widths).
 *   - Harmonic summing (opts.numharm = Hmax > 1, section 2.3 and the
 *     appendix algorithm "Harmonic Sum Decimation"): stage H searches
 *     S_H[r] = sum_{h=1..H} (P[h r] + ... + P[h r + h - 1]) over its
 *     floor(nbins / H) bins exactly as the power itself (chunks, windows,
 *     maxima), with H(H+1) w degrees of freedom for a width-w boxcar and, by
 *     default, ntrials = floor(nbins / H) * searched widths.  Stage 1 is the
 *     power.
 *   - Candidates come out in canonical order: ascending (spectrum, harmonic
 *     stage, chunk, width).  Results are deterministic.
 *   - Inputs must be finite; NaN or infinite amplitudes give undefined
 *     candidates (no crash).
 *
 * Memory: spectra, tables and on_device candidate buffers are DEVICE
 * pointers owned by the caller, read-only for inputs and never retained
 * after the call returns (or, for asynchronous calls, after the stream
 * reaches the end of the call's work).  A context owns all scratch memory
 * (thresholds, candidate staging, counters) and grows it on demand.
 *
 * Errors: every entry point returns a pulscan_status; nothing is thrown.  On
 * any error other than PULSCAN_EOVERFLOW no output is written.
 *
 * Threads and streams: a context may be used by one host thread at a time,
 * and its calls must not overlap on different streams.  Calls run on the
 * stream given in the options (the null stream by default) and are ordered
 * after work already queued there.  The plain
 * pulscan_search uses an internal default context, created on the device
 * that is current at its first call.
 */
#ifndef PULSCAN_H
#define PULSCAN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PULSCAN_OK = 0,
  PULSCAN_EINVAL = -1,      /* invalid argument (null pointer, bad size, bad option)   */
  PULSCAN_ENOMEM = -2,      /* device or host allocation failed                          */
  PULSCAN_EOVERFLOW = -3,   /* more candidates than out->capacity (see pulscan_search)  */
  PULSCAN_EHIP = -4,        /* a HIP runtime call failed                                 */
  PULSCAN_EUNSUPPORTED = -5 /* valid for the method but outside what the kernels support */
} pulscan_status;

enum { PULSCAN_NORM_MOM = 0, PULSCAN_NORM_EXACT = 1 };
enum { PULSCAN_W_ALL = 0, PULSCAN_W_LOG2 = 1 };

/* One complex Fourier amplitude: interleaved real and imaginary parts, the
 * layout of a complex FP32 FFT output (the paper's .fft input, section 2.2.2). */
typedef struct {
  float re, im;
} pulscan_complex;

/* One candidate: a per-chunk maximum whose significance reached the threshold. */
typedef struct {
  uint32_t spectrum;  /* index in the batch; 0 for single-spectrum calls          */
  uint32_t bin;       /* left edge of the window, 0-based (the paper's r-bin), in
                         the searched series (harmonic stage H: the fundamental's
                         r-bin); with opts.rblock > 0, the r-block index
                         bin / rblock instead (section 2.4)                       */
  uint32_t width;     /* boxcar width 1..zmax; the paper's z-bin is width - 1     */
  float power;        /* boxcar power of the window, FP32                         */
  float sigma;        /* Bonferroni-corrected Gaussian-equivalent significance    */
  uint32_t chunk;     /* chunk index, bin / chunk (of the exact bin)              */
  uint32_t harmonics; /* harmonic stage H (1: the power itself), section 2.3      */
  float logp;         /* natural log of the Bonferroni-corrected p-value of which
                         sigma is the Gaussian equivalent (the log probability
                         of section 2.6), at most 0                              */
} pulscan_candidate;  /* 32 bytes */

/* Caller-owned candidate buffer. */
typedef struct {
  pulscan_candidate *data; /* capacity entries; host memory, or device if on_device */
  uint64_t capacity;
  uint64_t count;          /* out: the true number of candidates (may exceed capacity)
                              -- set by synchronous calls                            */
  int32_t on_device;       /* 1: data is a device pointer                             */
  int32_t reserved;
  uint64_t *count_device;  /* optional device pointer: receives the true count; the
                              only count an asynchronous call delivers, which
                              there also reports a failure on the device as one of
                              the PULSCAN_COUNT_* values below                        */
} pulscan_candidates;

/* Counts written to out->count_device when a search fails on the device (a
 * synchronous call returns the status instead): a workgroup's candidate count
 * never reached the scan (PULSCAN_EHIP), or more candidates than the staging
 * pool holds (PULSCAN_ENOMEM).  No real count comes near them. */
#define PULSCAN_COUNT_LOST 0xFFFFFFFFFFFFFFFFull
#define PULSCAN_COUNT_POOL_FULL 0xFFFFFFFFFFFFFFFEull

/* Options of the _ex and batched calls (fill with pulscan_opts_default). */
typedef struct {
  int32_t norm;         /* PULSCAN_NORM_MOM (default): median of medians (section
                           2.5); the GPU kernels support 4^k blocks of 64..4096
                           bins.  PULSCAN_NORM_EXACT: the exact median and MAD
                           (mean of the two middle values) of the CPU version,
                           by a radix select; blocks of 64, 256 or 1024 bins,
                           several times the normalisation work of MoM          */
  int32_t norm_block;   /* normalisation block in bins; 0 = chunk                    */
  double ntrials;       /* Bonferroni trials; 0 = nbins * searched widths            */
  int32_t width_search; /* PULSCAN_W_ALL (default): widths 1..zmax.
                           PULSCAN_W_LOG2: only widths w with z = w - 1 a power of
                           two (2, 3, 5, 9, 17, ...) and the widest width zmax,
                           section 4.1.3 (z = 1, 2, 4, ... z-max); every width
                           is still summed, the others are just not searched        */
  int32_t async;        /* 0 (default): wait for the stream and set out->count.
                           1: enqueue only; needs out->on_device and
                           out->count_device                                         */
  void *stream;         /* hipStream_t to run on; NULL = the null (default) stream */
  int32_t dense;        /* 0 (default): skip width blocks that a running upper bound
                           proves cannot reach their threshold (exact: the same
                           candidates).  1: evaluate every width block            */
  int32_t numharm;      /* harmonic stages searched, 1..16; 0 or 1 = the power only */
  int32_t best_per_chunk; /* 1: of the candidates of one (spectrum, stage, chunk),
                           keep only the one of highest sigma (the first in
                           canonical order on ties); count is then the number
                           of chunks kept                                          */
  int32_t rblock;       /* > 0: candidates report the r-block index bin / rblock in
                           place of the bin (section 2.4); 0 = exact bins         */
  int32_t graph;        /* 1: the context captures the call's launches in a HIP
                           graph and replays it for later calls with the same
                           arguments (spectra, sizes, options, output buffers);
                           a call with other arguments recaptures.  The first
                           call of a set runs directly                           */
  int32_t power_fp16;   /* 1: the bank keeps normalised power in FP16 (FP32 sums):
                           half the LDS, more workgroups per CU.  It compares
                           against thresholds 0.5 sigma lower, and every
                           candidate within 0.5 sigma of the threshold is
                           re-decided on its FP32 power, recomputed from the
                           spectrum; other candidates report FP16-based power
                           (relative error up to about 5e-4).  Not with 4096-bin
                           normalisation blocks                                  */
} pulscan_opts;

typedef struct pulscan_ctx pulscan_ctx;

/* Human-readable name of a status code. */
const char *pulscan_strerror(int status);

/* Default options: MoM normalisation, block = chunk, default ntrials, all widths,
 * synchronous, the null stream, pruned bank, no harmonic summing, every
 * candidate, exact bins. */
void pulscan_opts_default(pulscan_opts *opts);

/* Create a context on HIP device `device` (it becomes current for the calls
 * of this thread that use the context).  Returns EINVAL for a null ctx or a
 * bad device, EHIP if the runtime fails. */
int pulscan_ctx_create(pulscan_ctx **ctx, int device);

/* Release a context and all its device memory.  NULL is ignored. */
void pulscan_ctx_destroy(pulscan_ctx *ctx);

/* Search one spectrum (the four steps above) with default options on the
 * default context, synchronously (thread-safe: calls are serialised).
 *   spectrum      device pointer, nbins complex amplitudes
 *   nbins         >= max(chunk, zmax) and < 2^32
 *   zmax          largest boxcar width, >= 1
 *   chunk         bins per chunk (and per normalisation block): a power of 4 in
 *                 64..4096 with the default options
 *   sigma_thresh  emit a (chunk, width) maximum when its corrected sigma >= this
 *   out           candidates; out->count = true count.  If it exceeds
 *                 out->capacity, the first capacity candidates (canonical order)
 *                 are written and PULSCAN_EOVERFLOW is returned.            */
int pulscan_search(const pulscan_complex *spectrum, size_t nbins, int zmax, int chunk,
                   float sigma_thresh, pulscan_candidates *out);

/* pulscan_search on an explicit context with options (opts NULL = defaults).
 * The GPU kernels take chunk a multiple of 64 (at most 16384), zmax <= 4096
 * and a tile that fits in 64 KiB of LDS (chunk * zmax is the main term);
 * other valid shapes return PULSCAN_EUNSUPPORTED.  See pulscan_opts for the
 * normalisation block. */
int pulscan_search_ex(pulscan_ctx *ctx, const pulscan_complex *spectrum, size_t nbins, int zmax,
                      int chunk, float sigma_thresh, const pulscan_opts *opts,
                      pulscan_candidates *out);

/* Search nspec spectra of independent lengths and widths in one fused launch.
 *   spectra, nbins, zmax   host arrays of nspec entries (spectra[s] on device)
 *   chunk                  common chunk; 0 = chosen by the library from
 *                          {256, 1024, 4096}, the choice returned in *chunk_used
 *   opts.ntrials           applied per spectrum when non-zero; 0 = nbins[s] * widths
 * Candidates of all spectra are returned together, ordered by spectrum.
 * Validation is per spectrum as in pulscan_search_ex; one bad spectrum fails
 * the call. */
int pulscan_search_batched(pulscan_ctx *ctx, int nspec, const pulscan_complex *const *spectra,
                           const uint64_t *nbins, const int32_t *zmax, int chunk,
                           float sigma_thresh, const pulscan_opts *opts, pulscan_candidates *out,
                           int *chunk_used);

/* Dense per-chunk maxima for parity checks: the search without the threshold.
 *   M, I    device, nchunks x zmax (row = chunk): the maximum boxcar power of each
 *           (chunk, width) and its bin; -inf and 0xFFFFFFFF where no window fits
 *   power   optional device output, nbins normalised powers (NULL to skip)
 *   stats   optional device output, nblocks x 4: median_re, mad_re, median_im,
 *           mad_im of each normalisation block (NULL to skip)
 * Synchronous. */
int pulscan_debug_tables(pulscan_ctx *ctx, const pulscan_complex *spectrum, size_t nbins,
                         int zmax, int chunk, const pulscan_opts *opts, float *M, uint32_t *I,
                         float *power, float *stats);

/* The boxcar bank and per-chunk maxima alone, on a caller-supplied power
 * array (device, nbins floats >= 0), skipping normalisation: integer-valued
 * powers give exact sums.  M, I as in pulscan_debug_tables.  Synchronous. */
int pulscan_debug_bank_from_power(pulscan_ctx *ctx, const float *power, size_t nbins, int zmax,
                                  int chunk, float *M, uint32_t *I);

/* The per-width power thresholds the search compares against: T_host[w-1] is
 * the smallest FP32 power whose corrected sigma (width w, ntrials) reaches
 * sigma_thresh, for w = 1..zmax (+inf for widths not searched under
 * width_search).  Computed in FP64 on the device.  Synchronous. */
int pulscan_threshold_table(pulscan_ctx *ctx, int zmax, float sigma_thresh, double ntrials,
                            int width_search, float *T_host);

/* Kernel timing: with enable = N > 0, every N-th bank-kernel launch of the
 * context (the first, the N+1-th, ...) is bracketed by HIP events on its
 * stream; 0 turns timing off, negative values are PULSCAN_EINVAL.  Timing
 * one launch in N keeps the events' own cost out of most steps.
 * pulscan_ctx_kernel_time waits for the recorded launches, returns their
 * summed duration in milliseconds and their number, and clears the
 * record. */
int pulscan_ctx_set_timing(pulscan_ctx *ctx, int enable);
int pulscan_ctx_kernel_time(pulscan_ctx *ctx, double *total_ms, uint64_t *launches);

/* Which bank kernel the context launches.  Both kernels give the same
 * candidates bit for bit (the same arithmetic, the same FP32 summation order);
 * they differ in speed.  kernel = PULSCAN_KERNEL_AUTO (the default): the
 * streaming kernel (persistent workgroups, each reading a contiguous range of
 * normalisation blocks once) for launches of spectra with at least 64 blocks
 * per resident workgroup (a DM-trial batch, a served batch), the tiled kernel
 * (one workgroup per tile) for the rest; PULSCAN_KERNEL_STREAM: the streaming
 * kernel wherever it serves the search (not: FP16 power, the exact median,
 * shapes outside its geometry); PULSCAN_KERNEL_TILED: the tiled kernel
 * always.  EINVAL for other values. */
enum { PULSCAN_KERNEL_STREAM = 0, PULSCAN_KERNEL_TILED = 1, PULSCAN_KERNEL_AUTO = 2 };
int pulscan_ctx_set_kernel(pulscan_ctx *ctx, int kernel);
/* The bank kernel of the context's last launch (PULSCAN_KERNEL_STREAM or
 * PULSCAN_KERNEL_TILED; -1 before the first) into *kernel.  EINVAL on null. */
int pulscan_ctx_last_kernel(pulscan_ctx *ctx, int *kernel);

/* Polls of a word another workgroup publishes (a count, or the statistics of
 * a halo block) before a bank kernel gives up on it: a lost count makes the
 * search return PULSCAN_EHIP (and the context re-arms its counters before
 * its next launch), a lost statistics word (streaming kernel) is recomputed
 * from the spectrum.  Every kernel still runs to its end.  Default 2^20 (a
 * hundred milliseconds or more); a small value forces the give-up paths in
 * tests.  polls >= 1, else EINVAL. */
int pulscan_ctx_set_spin(pulscan_ctx *ctx, uint32_t polls);

/* The single-spectrum search of pulscan_search_ex for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  It calls no hipMalloc, hipFree or other
 * allocating routine and needs no context: every buffer its kernels use
 * (threshold table, candidate staging, counters, per-workgroup words) lives
 * in one static device array of about 25 MiB, which each GPU the library
 * runs on holds until the process ends.
 *   spectrum, nbins, zmax, chunk, sigma_thresh, opts: as pulscan_search_ex,
 *     on the device current at the call, on opts->stream.
 *   out: on_device must be 1 (the candidates go straight to out->data); with
 *     opts->async, out->count_device receives the count and the call returns
 *     once the work is queued; otherwise the call waits and sets out->count.
 * Limits (PULSCAN_EUNSUPPORTED beyond them, before any launch): the shapes
 * of the streaming bank kernel -- median-of-medians normalisation, chunk 256
 * with 256- or 1024-bin blocks or chunk 1024 with 1024-bin blocks, zmax at
 * most what one LDS ring holds (<= 4096) -- and numharm 1, no FP16 power, no
 * best_per_chunk, no library graph mode.  At most 2^20 candidates are staged per call: more
 * return PULSCAN_ENOMEM (out->count still gets the true total).  Other
 * errors as pulscan_search_ex; EINVAL for a host output buffer.
 * The thresholds are recomputed on every call (no table cache).  Every call
 * on a GPU shares that GPU's array: calls that overlap on one GPU (on two
 * streams or two host threads) race and give undefined results. */
int pulscan_search_noalloc(const pulscan_complex *spectrum, size_t nbins, int zmax, int chunk,
                           float sigma_thresh, const pulscan_opts *opts,
                           pulscan_candidates *out);

/* ---------------------------------------------------------------------- */
/* Serving: spectra searched as they arrive.                                */
/* ---------------------------------------------------------------------- */

/* A server owns a context, two streams (copies and searches), a device ring
 * of hbm_budget bytes for copies of host spectra, and a worker thread.  The
 * worker admits submitted spectra in arrival order while the bytes of the
 * admitted, unfinished spectra stay within hbm_budget (a spectrum larger
 * than what is free waits; one alone is always admitted), searches each
 * admitted set (at most max_batch spectra) in one batched launch while the
 * next set is being copied, and publishes every spectrum's candidates with
 * its timestamps. */
typedef struct pulscan_server pulscan_server;

typedef struct {
  uint64_t hbm_budget;     /* bytes of spectra in flight (default 4 GiB); 0 = half of
                              the device memory free when the server starts.  A
                              budget beyond the free device memory is refused     */
  int32_t max_batch;       /* spectra per launch (default 256)                        */
  int32_t chunk;           /* chunk of every search (default 1024)                    */
  float sigma_thresh;      /* default 6                                               */
  uint32_t max_candidates; /* per launch; further candidates are counted, dropped
                              and flagged PULSCAN_EOVERFLOW (default 2^20)            */
  pulscan_opts opts;       /* search options (async, graph and stream must be 0)     */
} pulscan_server_config;

typedef struct {
  int64_t ticket;          /* as returned by pulscan_server_submit                   */
  int32_t status;          /* PULSCAN_OK or the search's error                       */
  uint32_t count;          /* candidates in `candidates`                             */
  uint64_t total;          /* candidates found                                       */
  double t_submit;         /* seconds on the server's clock: submitted,              */
  double t_start;          /*   admitted (its set's launch queued),                  */
  double t_done;           /*   results on the host                                  */
  const pulscan_candidate *candidates; /* host, owned by the server, valid until
                              the next pulscan_server_poll; spectrum = 0          */
} pulscan_result;

/* Defaults as listed in pulscan_server_config. */
void pulscan_server_config_default(pulscan_server_config *cfg);

/* Create a server on `device`; EINVAL for bad settings, ENOMEM if the budget
 * exceeds the device's free memory or the server's buffers cannot be
 * allocated.  While it runs, a set is launched only when the device has at
 * least 256 MiB free for the search's scratch, else once the sets in flight
 * have finished (admission by free device memory). */
int pulscan_server_create(pulscan_server **srv, int device, const pulscan_server_config *cfg);

/* The server's budget in bytes (as configured, or taken from the free device
 * memory for hbm_budget = 0). */
int pulscan_server_budget(pulscan_server *srv, uint64_t *bytes);

/* Finish every submitted spectrum, stop the worker and free everything. */
void pulscan_server_destroy(pulscan_server *srv);

/* Queue one spectrum of nbins complex amplitudes and widths 1..zmax.
 * on_device = 0: host memory, copied by the server (pinned memory from
 * pulscan_host_alloc copies fastest); 1: device memory, searched in place.
 * The memory must stay valid and unchanged until the result is polled.
 * Returns the ticket (>= 0) or a negative pulscan_status.  Invalid
 * spectra (too short for the chunk, ...) are reported in their result. */
int64_t pulscan_server_submit(pulscan_server *srv, const pulscan_complex *spectrum,
                              uint64_t nbins, int32_t zmax, int32_t on_device);

/* Take up to max_results finished results, oldest first, waiting up to
 * wait_ms for the first one.  Returns how many were written. */
int pulscan_server_poll(pulscan_server *srv, pulscan_result *results, int max_results,
                        int wait_ms);

/* Spectra waiting, finished so far, launches made, bytes admitted now. */
int pulscan_server_stats(pulscan_server *srv, uint64_t *pending, uint64_t *completed,
                         uint64_t *batches, uint64_t *budget_used);

/* Pinned host memory for spectra (hipHostMalloc); free with pulscan_host_free. */
int pulscan_host_alloc(void **ptr, uint64_t bytes);
void pulscan_host_free(void *ptr);

#ifdef __cplusplus
}
#endif

#endif /* PULSCAN_H */

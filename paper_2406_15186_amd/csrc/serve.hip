// The serving runtime: a worker thread that admits spectra as they arrive,
// as far as a budget of device memory allows, searches each admitted set in
// one batched launch and hands back every request's candidates with its
// timestamps.  Host-resident spectra are copied into a device ring on a copy
// stream while the previous set is searched on the compute stream; device-
// resident spectra are searched in place.  Normalisation statistics and
// thresholds live on the device in the server's context, and candidates land
// in a device buffer per in-flight set before they are copied out.
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "internal.hpp"

namespace {

constexpr int kInFlight = 2;  // sets searched while the next is admitted and copied

struct Request {
  int64_t ticket = 0;
  const pulscan_complex *src = nullptr;  // caller's spectrum (host or device)
  bool on_device = false;
  uint64_t n = 0;
  int32_t zmax = 0;
  double t_submit = 0.0;
  uint64_t off = 0;    // ring offset of the device copy (host requests)
  uint64_t bytes = 0;  // bytes counted against the budget
};

struct Done {
  int64_t ticket;
  int32_t status;
  uint64_t total;
  double t_submit, t_start, t_done;
  std::vector<pulscan_candidate> cands;
};

struct Slot {
  std::vector<Request> reqs;
  pulscan_candidate *dev_out = nullptr;
  unsigned long long *dev_count = nullptr;
  hipEvent_t copied = nullptr, done = nullptr;
  int32_t status = PULSCAN_OK;
  double t_start = 0.0;
  bool busy = false;
  bool in_ring = false;   // some spectrum of the set was copied into the ring
  uint64_t ring_end = 0;  // ring head after this set's copies
};

double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct pulscan_server {
  int device = 0;
  pulscan_server_config cfg{};
  pulscan_ctx *ctx = nullptr;
  hipStream_t copy_stream = nullptr, compute_stream = nullptr;
  char *ring = nullptr;          // device copies of host spectra
  uint64_t ring_bytes = 0;
  uint64_t ring_head = 0, ring_tail = 0, ring_used = 0;
  uint64_t budget_used = 0;      // bytes of admitted, unfinished spectra
  Slot slots[kInFlight];
  int next_slot = 0;
  std::deque<int> order;         // in-flight slots, oldest first
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv, cv_done;
  std::deque<Request> pending;
  std::deque<Done> done;
  std::vector<Done> polled;      // results handed out by the last poll
  int64_t next_ticket = 0;
  bool stop = false;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  uint64_t completed = 0, batches = 0;
};

namespace {

// Place `bytes` in the ring (FIFO allocation, freed in the same order);
// false if it does not fit now.
bool ring_alloc(pulscan_server *s, uint64_t bytes, uint64_t *off) {
  const uint64_t a = (bytes + 255) & ~255ull;
  if (a > s->ring_bytes) return false;
  if (s->ring_used == 0) s->ring_head = s->ring_tail = 0;
  const uint64_t h = s->ring_head;
  // allocated bytes run from tail to head, past the end and round to 0 when
  // wrapped (head <= tail with something allocated)
  const bool wrapped = s->ring_used > 0 && h <= s->ring_tail;
  if (!wrapped) {
    if (h + a <= s->ring_bytes) {
      *off = h;
    } else if (a <= s->ring_tail) {
      *off = 0;  // wrap; the end of the ring stays unused this round
      s->ring_used += s->ring_bytes - h;
    } else {
      return false;
    }
  } else {
    if (h + a > s->ring_tail) return false;
    *off = h;
  }
  s->ring_head = *off + a;
  s->ring_used += a;
  return true;
}

void ring_release_to(pulscan_server *s, uint64_t end) {
  // everything up to `end` (a former head) is free again
  if (end >= s->ring_tail) {
    s->ring_used -= end - s->ring_tail;
  } else {
    s->ring_used -= (s->ring_bytes - s->ring_tail) + end;
  }
  s->ring_tail = end;
  if (s->ring_used == 0) s->ring_head = s->ring_tail = 0;
}

// Device memory a launch may need for its search's scratch (candidate pool,
// tile words, outputs) beyond what the server holds.
constexpr uint64_t kFreeReserve = 256ull << 20;

bool device_has_room() {
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
    (void)hipGetLastError();
    return true;  // no answer: do not hold the queue on it
  }
  return (uint64_t)free_b >= kFreeReserve;
}

// Copy the oldest in-flight set's results out and publish them.
void collect(pulscan_server *s) {
  const int k = s->order.front();
  s->order.pop_front();
  Slot &sl = s->slots[k];
  int st = sl.status;
  unsigned long long total = 0;
  std::vector<pulscan_candidate> all;
  if (st == PULSCAN_OK) {
    if (hipEventSynchronize(sl.done) != hipSuccess ||
        hipMemcpy(&total, sl.dev_count, sizeof(total), hipMemcpyDeviceToHost) != hipSuccess) {
      (void)hipGetLastError();
      st = PULSCAN_EHIP;
    } else if (total == PULSCAN_COUNT_LOST || total == PULSCAN_COUNT_POOL_FULL) {
      // the search failed on the device (a count never arrived, or the
      // staging pool overflowed)
      st = total == PULSCAN_COUNT_LOST ? PULSCAN_EHIP : PULSCAN_ENOMEM;
    } else {
      const uint64_t take = total < s->cfg.max_candidates ? total : s->cfg.max_candidates;
      all.resize(take);
      if (take && hipMemcpy(all.data(), sl.dev_out, take * sizeof(pulscan_candidate),
                            hipMemcpyDeviceToHost) != hipSuccess) {
        (void)hipGetLastError();
        st = PULSCAN_EHIP;
      }
    }
  }
  if (st != PULSCAN_OK) {
    // copies of a failed set may still be writing into its ring space
    (void)hipStreamSynchronize(s->copy_stream);
    (void)hipGetLastError();
  }
  const double t = now_s(s->t0);
  std::vector<Done> out(sl.reqs.size());
  for (size_t i = 0; i < sl.reqs.size(); ++i) {
    out[i].ticket = sl.reqs[i].ticket;
    out[i].status = st;
    out[i].total = 0;
    out[i].t_submit = sl.reqs[i].t_submit;
    out[i].t_start = sl.t_start;
    out[i].t_done = t;
  }
  if (st == PULSCAN_OK) {
    for (const pulscan_candidate &c : all) {
      if (c.spectrum < out.size()) {
        out[c.spectrum].cands.push_back(c);
        out[c.spectrum].cands.back().spectrum = 0;
      }
    }
    for (auto &d : out) d.total = d.cands.size();
    if (total > all.size())
      for (auto &d : out) d.status = PULSCAN_EOVERFLOW;
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    uint64_t bytes = 0;
    for (const Request &r : sl.reqs) bytes += r.bytes;
    s->budget_used -= bytes;
    // only sets that placed copies in the ring free ring space: a set of
    // device spectra may have recorded a head from before the ring was reset
    if (sl.in_ring) ring_release_to(s, sl.ring_end);
    for (auto &d : out) s->done.push_back(std::move(d));
    s->completed += sl.reqs.size();
  }
  sl.reqs.clear();
  sl.busy = false;
  s->cv_done.notify_all();
}

void work(pulscan_server *s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    // admit a set: FIFO, as long as the device budget and the ring allow
    std::vector<Request> set;
    // a further set only while the device keeps memory free for its search's
    // scratch, unless nothing is in flight (then it runs and fails alone)
    const bool slot_free = !s->slots[s->next_slot].busy && (s->order.empty() || device_has_room());
    if (slot_free) {
      while (!s->pending.empty() && (int)set.size() < s->cfg.max_batch) {
        Request &r = s->pending.front();
        if (s->budget_used + r.bytes > s->cfg.hbm_budget && !(set.empty() && s->order.empty()))
          break;
        if (!r.on_device && !ring_alloc(s, r.bytes, &r.off)) break;
        s->budget_used += r.bytes;
        set.push_back(r);
        s->pending.pop_front();
      }
    }
    if (!set.empty()) {
      Slot &sl = s->slots[s->next_slot];
      sl.busy = true;
      sl.in_ring = false;
      for (const Request &r : set) sl.in_ring = sl.in_ring || !r.on_device;
      sl.reqs = std::move(set);
      sl.ring_end = s->ring_head;
      sl.t_start = now_s(s->t0);
      const int k = s->next_slot;
      s->next_slot = (s->next_slot + 1) % kInFlight;
      lk.unlock();
      // copies, then one batched search on the compute stream
      std::vector<const pulscan_complex *> ptrs(sl.reqs.size());
      std::vector<uint64_t> ns(sl.reqs.size());
      std::vector<int32_t> zs(sl.reqs.size());
      bool copies = false;
      int st = PULSCAN_OK;
      for (size_t i = 0; i < sl.reqs.size() && st == PULSCAN_OK; ++i) {
        const Request &r = sl.reqs[i];
        ns[i] = r.n;
        zs[i] = r.zmax;
        if (r.on_device) {
          ptrs[i] = r.src;
        } else {
          pulscan_complex *dst = reinterpret_cast<pulscan_complex *>(s->ring + r.off);
          if (hipMemcpyAsync(dst, r.src, r.n * sizeof(pulscan_complex), hipMemcpyHostToDevice,
                             s->copy_stream) != hipSuccess)
            st = PULSCAN_EHIP;
          ptrs[i] = dst;
          copies = true;
        }
      }
      if (st == PULSCAN_OK && copies &&
          (hipEventRecord(sl.copied, s->copy_stream) != hipSuccess ||
           hipStreamWaitEvent(s->compute_stream, sl.copied, 0) != hipSuccess))
        st = PULSCAN_EHIP;
      if (st == PULSCAN_OK) {
        pulscan_opts o = s->cfg.opts;
        o.async = 1;
        o.graph = 0;
        o.stream = s->compute_stream;
        pulscan_candidates out{};
        out.data = sl.dev_out;
        out.capacity = s->cfg.max_candidates;
        out.on_device = 1;
        out.count_device = reinterpret_cast<uint64_t *>(sl.dev_count);
        st = pulscan_search_batched(s->ctx, (int)sl.reqs.size(), ptrs.data(), ns.data(),
                                    zs.data(), s->cfg.chunk, s->cfg.sigma_thresh, &o, &out,
                                    nullptr);
      }
      if (st == PULSCAN_OK && hipEventRecord(sl.done, s->compute_stream) != hipSuccess)
        st = PULSCAN_EHIP;
      if (st != PULSCAN_OK) (void)hipGetLastError();
      sl.status = st;
      lk.lock();
      s->order.push_back(k);
      ++s->batches;
      continue;
    }
    if (!s->order.empty()) {
      // nothing more can be admitted now (or the device is short of free
      // memory for another set's scratch): finish the oldest set
      lk.unlock();
      collect(s);
      lk.lock();
      continue;
    }
    if (s->stop) break;
    s->cv.wait(lk, [s] { return s->stop || !s->pending.empty(); });
  }
}

}  // namespace

extern "C" {

void pulscan_server_config_default(pulscan_server_config *c) {
  if (!c) return;
  memset(c, 0, sizeof(*c));
  c->hbm_budget = 4ull << 30;
  c->max_batch = 256;
  c->chunk = 1024;
  c->sigma_thresh = 6.0f;
  c->max_candidates = 1u << 20;
  pulscan_opts_default(&c->opts);
}

int pulscan_server_create(pulscan_server **out, int device, const pulscan_server_config *cfg) {
  if (!out || !cfg) return PULSCAN_EINVAL;
  *out = nullptr;
  if ((cfg->hbm_budget != 0 && cfg->hbm_budget < (1ull << 20)) || cfg->max_batch < 1 ||
      cfg->chunk < 64 || cfg->max_candidates < 1 || !(cfg->sigma_thresh == cfg->sigma_thresh))
    return PULSCAN_EINVAL;
  if (cfg->opts.async || cfg->opts.graph || cfg->opts.stream) return PULSCAN_EINVAL;
  // the budget against the device memory free now
  size_t free_b = 0, total_b = 0;
  if (hipSetDevice(device) != hipSuccess || hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
    (void)hipGetLastError();
    return PULSCAN_EHIP;
  }
  const uint64_t out_bytes =
      (uint64_t)kInFlight * ((uint64_t)cfg->max_candidates * sizeof(pulscan_candidate) + 256);
  uint64_t budget = cfg->hbm_budget;
  if (budget == 0) budget = ((uint64_t)free_b / 2) & ~255ull;
  if (budget < (1ull << 20) || budget + out_bytes > (uint64_t)free_b) return PULSCAN_ENOMEM;
  pulscan_server *s = new (std::nothrow) pulscan_server();
  if (!s) return PULSCAN_ENOMEM;
  s->device = device;
  s->cfg = *cfg;
  s->cfg.hbm_budget = budget;
  int st = pulscan_ctx_create(&s->ctx, device);
  if (st) {
    delete s;
    return st;
  }
  bool ok = hipSetDevice(device) == hipSuccess &&
            hipStreamCreate(&s->copy_stream) == hipSuccess &&
            hipStreamCreate(&s->compute_stream) == hipSuccess;
  // the ring places copies at 256-byte boundaries: sized to the budget rounded
  // up, so that every spectrum the budget admits also fits in it
  s->ring_bytes = (budget + 255) & ~255ull;
  ok = ok && hipMalloc(reinterpret_cast<void **>(&s->ring), s->ring_bytes) == hipSuccess;
  for (int k = 0; ok && k < kInFlight; ++k) {
    Slot &sl = s->slots[k];
    ok = hipMalloc(reinterpret_cast<void **>(&sl.dev_out),
                   (size_t)cfg->max_candidates * sizeof(pulscan_candidate)) == hipSuccess &&
         hipMalloc(reinterpret_cast<void **>(&sl.dev_count), sizeof(unsigned long long)) ==
             hipSuccess &&
         hipEventCreateWithFlags(&sl.copied, hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess;
  }
  if (!ok) {
    (void)hipGetLastError();
    pulscan_server_destroy(s);
    return PULSCAN_ENOMEM;
  }
  s->worker = std::thread(work, s);
  *out = s;
  return PULSCAN_OK;
}

void pulscan_server_destroy(pulscan_server *s) {
  if (!s) return;
  if (s->worker.joinable()) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stop = true;
    }
    s->cv.notify_all();
    s->worker.join();  // drains everything submitted before
  }
  (void)hipSetDevice(s->device);
  (void)hipDeviceSynchronize();
  for (Slot &sl : s->slots) {
    if (sl.dev_out) (void)hipFree(sl.dev_out);
    if (sl.dev_count) (void)hipFree(sl.dev_count);
    if (sl.copied) (void)hipEventDestroy(sl.copied);
    if (sl.done) (void)hipEventDestroy(sl.done);
  }
  if (s->ring) (void)hipFree(s->ring);
  if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
  if (s->compute_stream) (void)hipStreamDestroy(s->compute_stream);
  pulscan_ctx_destroy(s->ctx);
  delete s;
}

int64_t pulscan_server_submit(pulscan_server *s, const pulscan_complex *spectrum, uint64_t nbins,
                              int32_t zmax, int32_t on_device) {
  if (!s || !spectrum || nbins == 0 || zmax < 1) return PULSCAN_EINVAL;
  // what the search would reject, rejected here so that one bad spectrum
  // cannot fail the set it would have been searched with
  const uint64_t block = s->cfg.opts.norm_block > 0 ? (uint64_t)s->cfg.opts.norm_block
                                                    : (uint64_t)s->cfg.chunk;
  if (nbins < block || nbins < (uint64_t)s->cfg.chunk || nbins < (uint64_t)zmax ||
      nbins >= (1ull << 32) || zmax > 4096)
    return PULSCAN_EINVAL;
  Request r;
  r.src = spectrum;
  r.on_device = on_device != 0;
  r.n = nbins;
  r.zmax = zmax;
  r.bytes = nbins * sizeof(pulscan_complex);
  if (r.bytes > s->cfg.hbm_budget) return PULSCAN_EINVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return PULSCAN_EINVAL;
    r.ticket = s->next_ticket++;
    r.t_submit = now_s(s->t0);
    s->pending.push_back(r);
  }
  s->cv.notify_one();
  return r.ticket;
}

int pulscan_server_poll(pulscan_server *s, pulscan_result *res, int max_results, int wait_ms) {
  if (!s || (!res && max_results > 0) || max_results < 0) return PULSCAN_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done.empty() && wait_ms > 0)
    s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [s] { return !s->done.empty(); });
  s->polled.clear();
  int k = 0;
  while (k < max_results && !s->done.empty()) {
    s->polled.push_back(std::move(s->done.front()));
    s->done.pop_front();
    ++k;
  }
  for (int i = 0; i < k; ++i) {
    const Done &d = s->polled[i];
    res[i].ticket = d.ticket;
    res[i].status = d.status;
    res[i].count = (uint32_t)d.cands.size();
    res[i].total = d.total;
    res[i].t_submit = d.t_submit;
    res[i].t_start = d.t_start;
    res[i].t_done = d.t_done;
    res[i].candidates = d.cands.empty() ? nullptr : d.cands.data();
  }
  return k;
}

int pulscan_server_budget(pulscan_server *s, uint64_t *bytes) {
  if (!s || !bytes) return PULSCAN_EINVAL;
  *bytes = s->cfg.hbm_budget;
  return PULSCAN_OK;
}

int pulscan_server_stats(pulscan_server *s, uint64_t *pending, uint64_t *completed,
                         uint64_t *batches, uint64_t *budget_used) {
  if (!s) return PULSCAN_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (pending) *pending = s->pending.size();
  if (completed) *completed = s->completed;
  if (batches) *batches = s->batches;
  if (budget_used) *budget_used = s->budget_used;
  return PULSCAN_OK;
}

int pulscan_host_alloc(void **ptr, uint64_t bytes) {
  if (!ptr || bytes == 0) return PULSCAN_EINVAL;
  *ptr = nullptr;
  if (hipHostMalloc(ptr, bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    *ptr = nullptr;
    return PULSCAN_ENOMEM;
  }
  return PULSCAN_OK;
}

void pulscan_host_free(void *ptr) {
  if (ptr) (void)hipHostFree(ptr);
}

}  // extern "C"

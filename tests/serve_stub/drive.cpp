// Drives the serving runtime (compiled against the host stand-ins) through
// the scenarios of its CPU test: argv = budget_bytes max_batch nreq seed
// [edges].  Every request carries a distinct tag in its first amplitude; the
// program checks that each ticket comes back once, with its own tag, and
// prints "ok <requests> <launches>".  edges bit 0: every seventh request has
// the largest size the budget admits; bit 1: every eleventh request's search
// fails on the device, and it (with the others of its launch) must come back
// with PULSCAN_EHIP.
#include <stdio.h>
#include <stdlib.h>

#include <chrono>
#include <random>
#include <thread>
#include <vector>

#include "pulscan.h"

int main(int argc, char **argv) {
  if (argc < 5) return 2;
  pulscan_server_config cfg;
  pulscan_server_config_default(&cfg);
  cfg.hbm_budget = strtoull(argv[1], nullptr, 10);
  cfg.max_batch = atoi(argv[2]);
  cfg.chunk = 64;
  const int nreq = atoi(argv[3]);
  std::mt19937 rng(atoi(argv[4]));
  if (nreq == 0) {
    // creation only: report the status and the budget the server took
    pulscan_server *srv = nullptr;
    const int st = pulscan_server_create(&srv, 0, &cfg);
    uint64_t b = 0;
    if (st == PULSCAN_OK) {
      if (pulscan_server_budget(srv, &b) != PULSCAN_OK) return 12;
      pulscan_server_destroy(srv);
    }
    printf("create %d budget %llu\n", st, (unsigned long long)b);
    return 0;
  }
  pulscan_server *srv = nullptr;
  if (pulscan_server_create(&srv, 0, &cfg) != PULSCAN_OK) return 3;
  std::vector<std::vector<pulscan_complex>> data(nreq);
  std::vector<int64_t> ticket(nreq);
  const int edges = argc > 5 ? atoi(argv[5]) : 0;
  const uint64_t max_n = cfg.hbm_budget / sizeof(pulscan_complex);
  std::vector<int> failing(nreq, 0);
  for (int i = 0; i < nreq; ++i) {
    uint64_t n = 64 + rng() % (max_n > 64 ? max_n - 64 : 1);
    if ((edges & 1) && i % 7 == 0) n = max_n;
    data[i].resize(n);
    data[i][0].re = (float)i;
    failing[i] = (edges & 2) && i % 11 == 0;
    data[i][0].im = failing[i] ? -1.0f : 0.0f;
    ticket[i] = pulscan_server_submit(srv, data[i].data(), n, 1 + (int)(rng() % 32),
                                      (int)(rng() % 2));
    if (ticket[i] < 0) return 4;
    if (rng() % 4 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 300));
  }
  std::vector<int> seen(nreq, 0);
  int got = 0, failed = 0;
  auto t_end = std::chrono::steady_clock::now() + std::chrono::seconds(20);
  pulscan_result res[64];
  while (got < nreq) {
    if (std::chrono::steady_clock::now() > t_end) {
      printf("stuck after %d of %d\n", got, nreq);
      return 5;
    }
    int k = pulscan_server_poll(srv, res, 64, 20);
    for (int j = 0; j < k; ++j) {
      const int64_t t = res[j].ticket;
      if (t < 0 || t >= nreq || seen[t]) return 6;
      seen[t] = 1;
      ++got;
      if (res[j].status == PULSCAN_EHIP && (edges & 2)) {
        ++failed;  // a failing search, or one launched with it
        continue;
      }
      if (failing[t] || res[j].status != PULSCAN_OK || res[j].count != 1) return 7;
      if ((int64_t)res[j].candidates[0].bin != t) return 8;
      if (!(res[j].t_submit <= res[j].t_start && res[j].t_start <= res[j].t_done)) return 9;
    }
  }
  uint64_t pend = 0, done = 0, launches = 0, used = 0;
  pulscan_server_stats(srv, &pend, &done, &launches, &used);
  if (pend || done != (uint64_t)nreq || used) return 10;
  pulscan_server_destroy(srv);
  if ((edges & 2) && failed == 0) return 11;
  printf("ok %d %llu\n", nreq, (unsigned long long)launches);
  return 0;
}

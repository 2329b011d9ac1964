// Stand-ins for the context and the batched search used by the serving
// runtime's CPU test (see internal.hpp in this directory).
#include <stdlib.h>
#include <string.h>

#include "pulscan.h"

struct pulscan_ctx {
  int calls;
};

extern "C" {

void pulscan_opts_default(pulscan_opts *o) {
  memset(o, 0, sizeof(*o));
  o->numharm = 1;
}

int pulscan_ctx_create(pulscan_ctx **c, int) {
  *c = (pulscan_ctx *)calloc(1, sizeof(pulscan_ctx));
  return *c ? PULSCAN_OK : PULSCAN_ENOMEM;
}

void pulscan_ctx_destroy(pulscan_ctx *c) { free(c); }

int pulscan_search_batched(pulscan_ctx *ctx, int nspec, const pulscan_complex *const *spectra,
                           const uint64_t *nbins, const int32_t *zmax, int chunk, float,
                           const pulscan_opts *opts, pulscan_candidates *out, int *) {
  if (!ctx || nspec < 1 || !opts || !opts->async || !out->on_device || !out->count_device)
    return PULSCAN_EINVAL;
  ctx->calls++;
  uint64_t k = 0;
  bool fail = false;
  for (int s = 0; s < nspec; ++s) {
    if (nbins[s] < (uint64_t)chunk || zmax[s] < 1) return PULSCAN_EINVAL;
    // a negative imaginary part in bin 0 stands for a search that fails on
    // the device: the count word then carries the failure code
    fail = fail || spectra[s][0].im < 0.f;
    if (k < out->capacity) {
      pulscan_candidate c{};
      c.spectrum = (uint32_t)s;
      c.bin = (uint32_t)spectra[s][0].re;  // the spectrum's tag
      c.width = (uint32_t)zmax[s];
      c.power = (float)nbins[s];
      out->data[k] = c;
    }
    ++k;
  }
  *out->count_device = fail ? PULSCAN_COUNT_LOST : k;
  return PULSCAN_OK;
}

}  // extern "C"

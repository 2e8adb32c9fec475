// Library-wide entry points: version, error reporting, host-side counts.
#include <stdarg.h>
#include <stdio.h>

#include "common.h"

namespace tgs {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

int32_t hip_status(const char* where) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("%s: %s", where, hipGetErrorString(e));
    return TGS_ERR_HIP;
  }
  return TGS_OK;
}

}  // namespace tgs

extern "C" uint32_t tgs_version(void) { return TGS_ABI_VERSION; }

extern "C" const char* tgs_last_error(void) { return tgs::g_err; }

extern "C" int32_t tgs_pixels_per_tile(int32_t rate_permille) {
  if (rate_permille <= 0) return 1;
  int64_t n = (int64_t)rate_permille * tgs::kTilePixels / 1000;
  if (n < 1) n = 1;
  if (n > tgs::kTilePixels) n = tgs::kTilePixels;
  return (int32_t)n;
}

extern "C" int32_t tgs_sample_tile_count(int32_t height, int32_t width,
                                         const tgs_sample_params* sp) {
  if (height <= 0 || width <= 0 || sp == nullptr) return 0;
  const int32_t n_t = (int32_t)(tgs::ceil_div(width, tgs::kTile) * tgs::ceil_div(height, tgs::kTile));
  if (sp->n_tiles_sel < 0 || sp->n_tiles_sel >= n_t) return n_t;
  return sp->n_tiles_sel;
}

// fit_matvec / fit_matvec_batched: applications of the matrix-free operator.
#include <algorithm>
#include <cmath>

#include "fit_internal.h"
#include "stencil.h"
#include "tuning.h"

using namespace fit;

namespace fit {

template <class T>
static fit_status matvec_typed(const fit_grid* g, double omega, int scaling, const void* x,
                               void* y, hipStream_t s) {
  OpMatvec<T> op{(const T*)x, (T*)y};
  const TileShape t = tile_for(g, sizeof(T) == 8 ? FIT_C128 : FIT_C64);
  if (scaling == FIT_SCALE_SYM) return launch_stencil<T, MODE_MEC>(g->view, t, omega, op, s);
  if (scaling == FIT_SCALE_FACT) return launch_stencil<T, MODE_FACT>(g->view, t, omega, op, s);
  return launch_stencil<T, MODE_D>(g->view, t, omega, op, s);
}

}  // namespace fit

extern "C" fit_status fit_matvec(const fit_grid* g, double omega, int dtype, int scaling,
                                 const void* x_dev, void* y_dev, void* stream) {
  if (!g || !x_dev || !y_dev) {
    set_error("fit_matvec: NULL argument");
    return FIT_E_INVALID;
  }
  if (!(omega >= 0.0) || !std::isfinite(omega)) {
    set_error("fit_matvec: omega must be finite and >= 0");
    return FIT_E_INVALID;
  }
  if (scaling != FIT_SCALE_NONE && scaling != FIT_SCALE_SYM && scaling != FIT_SCALE_FACT) {
    set_error("fit_matvec: unknown scaling");
    return FIT_E_INVALID;
  }
  if (scaling != FIT_SCALE_NONE && omega == 0.0) {
    set_error("fit_matvec: FIT_SCALE_SYM and FIT_SCALE_FACT need omega > 0");
    return FIT_E_INVALID;
  }
  if (x_dev == y_dev) {
    set_error("fit_matvec: x and y must not alias");
    return FIT_E_INVALID;
  }
  DeviceScope dev(g->device);
  if (dtype == FIT_C128) return matvec_typed<double>(g, omega, scaling, x_dev, y_dev, (hipStream_t)stream);
  if (dtype == FIT_C64) return matvec_typed<float>(g, omega, scaling, x_dev, y_dev, (hipStream_t)stream);
  set_error("fit_matvec: unknown dtype");
  return FIT_E_INVALID;
}

namespace fit {
template <class T>
static fit_status matvec_batched_typed(const fit_grid* g, int nbatch, const double* omegas,
                                       int scaling, const void* x, void* y, hipStream_t s) {
  const TileShape t = tile_for(g, sizeof(T) == 8 ? FIT_C128 : FIT_C64);
  const int64_t stride = 2 * g->ne;  // T values per complex vector
  for (int b0 = 0; b0 < nbatch; b0 += BatchVecs<T>::kMax) {
    const int n = std::min(BatchVecs<T>::kMax, nbatch - b0);
    BatchVecs<T> a{};
    for (int b = 0; b < n; ++b) {
      a.x[b] = (const T*)x + (b0 + b) * stride;
      a.y[b] = (T*)y + (b0 + b) * stride;
      a.omega[b] = omegas[b0 + b];
    }
    const fit_status st = scaling == FIT_SCALE_SYM ? launch_stencil_batch<T, MODE_MEC>(g->view, t, a, n, s)
                                                   : launch_stencil_batch<T, MODE_D>(g->view, t, a, n, s);
    if (st != FIT_OK) return st;
  }
  return FIT_OK;
}
}  // namespace fit

extern "C" fit_status fit_matvec_batched(const fit_grid* g, int nbatch, const double* omegas,
                                         int dtype, int scaling, const void* x_dev, void* y_dev,
                                         void* stream) {
  if (!g || !omegas || !x_dev || !y_dev) {
    set_error("fit_matvec_batched: NULL argument");
    return FIT_E_INVALID;
  }
  if (nbatch < 1 || nbatch > 64) {
    set_error("fit_matvec_batched: nbatch must be in [1, 64]");
    return FIT_E_INVALID;
  }
  if (scaling != FIT_SCALE_NONE && scaling != FIT_SCALE_SYM) {
    set_error("fit_matvec_batched: unknown scaling");
    return FIT_E_INVALID;
  }
  for (int b = 0; b < nbatch; ++b) {
    if (!(omegas[b] >= 0.0) || !std::isfinite(omegas[b]) ||
        (scaling == FIT_SCALE_SYM && omegas[b] == 0.0)) {
      set_error("fit_matvec_batched: every omega must be finite, >= 0 (> 0 with FIT_SCALE_SYM)");
      return FIT_E_INVALID;
    }
  }
  if (dtype != FIT_C128 && dtype != FIT_C64) {
    set_error("fit_matvec_batched: unknown dtype");
    return FIT_E_INVALID;
  }
  const size_t bytes = (size_t)g->ne * (dtype == FIT_C128 ? 16 : 8) * nbatch;
  const char *xa = (const char*)x_dev, *ya = (const char*)y_dev;
  if (xa < ya + bytes && ya < xa + bytes) {
    set_error("fit_matvec_batched: x and y must not overlap");
    return FIT_E_INVALID;
  }
  DeviceScope dev(g->device);
  hipStream_t s = (hipStream_t)stream;
  if (dtype == FIT_C128) return matvec_batched_typed<double>(g, nbatch, omegas, scaling, x_dev, y_dev, s);
  return matvec_batched_typed<float>(g, nbatch, omegas, scaling, x_dev, y_dev, s);
}

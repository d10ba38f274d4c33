// fit_matvec: one application of the matrix-free operator.
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
  if (scaling != FIT_SCALE_NONE && scaling != FIT_SCALE_SYM) {
    set_error("fit_matvec: unknown scaling");
    return FIT_E_INVALID;
  }
  if (scaling == FIT_SCALE_SYM && omega == 0.0) {
    set_error("fit_matvec: FIT_SCALE_SYM needs omega > 0");
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

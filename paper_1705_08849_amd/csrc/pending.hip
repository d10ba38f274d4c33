// Entry points declared in fit.h whose implementation has not landed yet.
// Each reports FIT_E_UNSUPPORTED with a message.
#include "fit_internal.h"
#include "precond.h"

using namespace fit;

static fit_status unsupported(const char* name) {
  set_error(std::string(name) + ": not implemented in this build");
  return FIT_E_UNSUPPORTED;
}

extern "C" fit_status fit_precond_train(fit_grid* const*, int, const double*, int,
                                        const fit_precond_cfg*, fit_precond**) {
  return unsupported("fit_precond_train");
}
extern "C" fit_status fit_precond_create(const fit_precond_cfg*, int, fit_precond**) {
  return unsupported("fit_precond_create");
}
extern "C" fit_status fit_precond_save(const fit_precond*, void*, size_t*) {
  return unsupported("fit_precond_save");
}
extern "C" fit_status fit_precond_load(const void*, size_t, int, fit_precond**) {
  return unsupported("fit_precond_load");
}
extern "C" fit_status fit_precond_apply(fit_precond*, const fit_grid*, double, const void*, void*,
                                        void*) {
  return unsupported("fit_precond_apply");
}
extern "C" void fit_precond_destroy(fit_precond*) {}

namespace fit {
PrecondApply* precond_apply_of(fit_precond*, const fit_grid*, double) { return nullptr; }
}  // namespace fit

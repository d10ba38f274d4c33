// Right-preconditioner interface used by flexible GMRES.
#pragma once

#include "fit_internal.h"

namespace fit {

struct Ctx;

// z = M(v) for one vector of the grid in the solver's working precision
// (complex64 when f32, else complex128), enqueued on the solver's stream.
struct PrecondApply {
  virtual ~PrecondApply() {}
  virtual fit_status apply(Ctx& c, const void* v, void* z, bool f32) = 0;
};

// Adapter for a learned preconditioner object on grid g at omega (nullptr if
// the object cannot serve this grid).  The caller deletes the adapter.
PrecondApply* precond_apply_of(fit_precond* p, const fit_grid* g, double omega);

// Solver-generated residual -> error pairs (fit_precond_harvest): e and r
// hold npairs complex128 vectors of g back to back; *made receives how many
// were written (fewer if the solve ends before the last snapshot).
fit_status harvest_pairs(fit_grid* g, double omega, int port, int npairs, double tol, double* e,
                         double* r, int* made, int* iterations);

}  // namespace fit

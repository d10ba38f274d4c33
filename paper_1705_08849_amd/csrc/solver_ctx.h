// Host-side solver context: stream, reduction scratch, pinned mirrors,
// tiles and the small launch helpers shared by the solver drivers.
#pragma once

#include <algorithm>
#include <cmath>

#include "fit_internal.h"
#include "krylov.h"
#include "krylov_more.h"
#include "solver_kernels.h"
#include "stencil.h"
#include "tuning.h"

namespace fit {

// Block partial sums per block that the context's partials buffer holds
// (every reduction launched through it writes at most this many per block:
// the launches of the solvers' kernels and the operator launches, whose
// width launch_op_stencil_mode checks at compile time).
constexpr int kPartWidth = 4;

// ---------------------------------------------------------------------------
// Host-side solver context.
// ---------------------------------------------------------------------------
struct Ctx {
  fit_grid* g;
  hipStream_t s;
  double omega;
  int sym;
  int diag = 0;  // COCG: fit_diag kind of a stored diagonal preconditioner (0: none stored)
  // reduction scratch
  double* part;
  unsigned* cnt;
  RedOut* red;
  BiState* bst;
  GmState* gst;
  RedOut* h_red;   // pinned host mirrors
  BiState* h_bst;
  GmState* h_gst;
  CgState* cst = nullptr;
  CgState* h_cst = nullptr;
  TqState* tst = nullptr;
  TqState* h_tst = nullptr;
  int max_blocks;
  double bytes = 0.0;  // algorithmic bytes launched
  int matvecs = 0;
  // iterate snapshots of the first inner COCG solve (training pairs of the
  // learned preconditioner): every snap_stride iterations, eta * x of the
  // inner solve goes to snap + k * snap_ld, k < snap_cap
  double* snap = nullptr;
  int64_t snap_ld = 0;
  int snap_cap = 0, snap_stride = 0, snap_n = 0;
  bool snap_active = false;
  double inner_eta = 1.0;  // scale of the current inner solve's rhs (x_outer += eta d)
  // FGMRES with a learned preconditioner: stop as stalled when the restart
  // residual has not halved within this many cycles (0: never)
  int gm_stall_cycles = 0;
  int last_reason = 0;   // breakdown test of the last inner BiCGStab
  double last_rr = 0.0;  // its final recursive ||r||^2 (unit initial norm)
  TileShape tile128, tile64;
};

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

template <class T, class Op>
static fit_status launch_op_stencil_mode(Ctx& c, bool sym, const Op& op) {
  static_assert(Op::NRED <= kPartWidth, "the partials buffer holds kPartWidth sums per block");
  const TileShape t = sizeof(T) == 8 ? c.tile128 : c.tile64;
  if (sym) return launch_stencil<T, MODE_MEC>(c.g->view, t, c.omega, op, c.s);
  return launch_stencil<T, MODE_D>(c.g->view, t, c.omega, op, c.s);
}

static double node_bytes(const fit_grid* g, int vec_passes, size_t elem) {
  return (double)g->view.np * 3.0 * elem * vec_passes + (double)g->view.ncx * g->view.ncy * g->view.ncz;
}

// r = b - A x (unscaled complex128), ||r||^2 -> c.red->v[0]; optional c64 copy.
static fit_status residual(Ctx& c, const double* x, const double* b, double* r, float* r32,
                           double r32_scale) {
  OpResidual<double> op{x, b, r, r32, r32_scale, c.red, c.part, c.cnt};
  c.bytes += node_bytes(c.g, 2 + (r ? 1 : 0), 16) + (r32 ? (double)c.g->ne * 8 : 0.0);
  c.matvecs += 1;
  return launch_op_stencil_mode<double>(c, false, op);
}

template <class TI, class TO, int KIND>
static fit_status xform(Ctx& c, bool sym, bool inverse, const TI* in, TO* out, double factor,
                        bool reduce, uint64_t seed = kShadowSeed) {
  hipLaunchKernelGGL((node_xform_kernel<TI, TO, KIND>), dim3(pw_blocks(c.g->view.np)), dim3(256), 0,
                     c.s, c.g->view, c.omega, sym ? 1 : 0, inverse ? 1 : 0, in, out, factor,
                     reduce ? c.red : nullptr, c.part, c.cnt, seed);
  FIT_HIP(hipGetLastError());
  if (reduce) FIT_HIP(launch_finish<1>(c.part, pw_blocks(c.g->view.np), StoreSums<1>{c.red}, c.s));
  c.bytes += (double)c.g->ne * (sizeof(TI) + sizeof(TO)) * 2 * (KIND == XF_AXPY ? 1.5 : 1.0);
  return FIT_OK;
}

template <class T>
static fit_status vzero(Ctx& c, T* v, int64_t ncomplex) {
  hipLaunchKernelGGL(zero_kernel<T>, dim3(pw_blocks(2 * ncomplex)), dim3(256), 0, c.s, v,
                     2 * ncomplex);
  FIT_HIP(hipGetLastError());
  return FIT_OK;
}
template <class T>
static fit_status vcopy(Ctx& c, const T* a, T* b, int64_t ncomplex) {
  hipLaunchKernelGGL(copy_kernel<T>, dim3(pw_blocks(2 * ncomplex)), dim3(256), 0, c.s, a, b,
                     2 * ncomplex);
  FIT_HIP(hipGetLastError());
  return FIT_OK;
}

static fit_status sync_copy(Ctx& c, void* dst, const void* src, size_t bytes) {
  FIT_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, c.s));
  FIT_HIP(hipStreamSynchronize(c.s));
  return FIT_OK;
}

// Bump allocator over the grid's workspace arena.
struct Arena {
  char* base;
  size_t off = 0, cap;
  template <class P>
  P* take(size_t bytes) {
    P* p = (P*)(base + off);
    off += align_up(bytes, 256);
    return p;
  }
};

inline fit_status setup_ctx(Ctx& c, fit_grid* g, double omega, int sym, hipStream_t s) {
  c.g = g;
  c.s = s;
  c.omega = omega;
  c.sym = sym;
  c.tile128 = tile_for(g, FIT_C128);
  c.tile64 = tile_for(g, FIT_C64);
  const int b128 = launch_blocks(make_launch(g->view, c.tile128, omega));
  const int b64 = launch_blocks(make_launch(g->view, c.tile64, omega));
  // room for one update-kernel block per item (a grid-stride loop over
  // several items per block was 8 % slower on the 256x256x128 grid)
  const int b_upd = otf_shape(g->view, 1 << 30).blocks;
  c.max_blocks = std::max(std::max(std::max(b128, b64), b_upd), 4096);
  const size_t need = align_up(sizeof(double) * kPartWidth * (size_t)c.max_blocks, 256) + 256 +
                      align_up(sizeof(RedOut), 256) + align_up(sizeof(BiState), 256) +
                      align_up(sizeof(GmState), 256) + align_up(sizeof(CgState), 256) +
                      align_up(sizeof(TqState), 256);
  fit_status st = ensure_ws(g->red, need, g->device);
  if (st != FIT_OK) return st;
  char* p = (char*)g->red.ptr;
  c.part = (double*)p;
  p += align_up(sizeof(double) * kPartWidth * (size_t)c.max_blocks, 256);
  c.cnt = (unsigned*)p;
  p += 256;
  c.red = (RedOut*)p;
  p += align_up(sizeof(RedOut), 256);
  c.bst = (BiState*)p;
  p += align_up(sizeof(BiState), 256);
  c.gst = (GmState*)p;
  p += align_up(sizeof(GmState), 256);
  c.cst = (CgState*)p;
  p += align_up(sizeof(CgState), 256);
  c.tst = (TqState*)p;
  if (!g->pinned) {
    FIT_HIP(hipHostMalloc(&g->pinned, sizeof(RedOut) + sizeof(BiState) + sizeof(GmState) +
                                          sizeof(CgState) + sizeof(TqState) + 256));
  }
  char* hp = (char*)g->pinned;
  c.h_red = (RedOut*)hp;
  c.h_bst = (BiState*)(hp + sizeof(RedOut));
  c.h_gst = (GmState*)(hp + sizeof(RedOut) + sizeof(BiState));
  c.h_cst = (CgState*)(hp + sizeof(RedOut) + sizeof(BiState) + sizeof(GmState));
  c.h_tst = (TqState*)(hp + sizeof(RedOut) + sizeof(BiState) + sizeof(GmState) + sizeof(CgState));
  // ticket counter starts at zero; the red block's flag too
  FIT_HIP(hipMemsetAsync(c.cnt, 0, 256, s));
  FIT_HIP(hipMemsetAsync(c.red, 0, sizeof(RedOut), s));
  return FIT_OK;
}

}  // namespace fit

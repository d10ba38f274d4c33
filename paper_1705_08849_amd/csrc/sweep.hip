// fit_sweep: many independent systems A_g(omega) e = -j omega j advanced
// together (Sec. II: every frequency and excitation is its own system).
//
// The systems are solved in batches.  Each batch runs the mass-preconditioned
// COCG iteration (the same method and recurrences as fit_solve's COCG) for
// all of its systems at once: one iteration is four launches whatever the
// batch size -- one operator launch covering every system's tiles (the grids
// may differ; it also recomputes the preconditioner and applies the previous
// solution update, as in fit_solve), one finish launch with a block per
// system, one streaming residual-update launch and one more finish launch.  The loop of `check_every`
// iterations is captured once as a hipGraph and replayed.  Every system
// keeps its own scalars and done flag on the device, so a converged system
// drops out at once (its blocks return immediately); the graph is captured
// again for the survivors when fewer than half of the captured systems are
// still running.
//
// Precision: FIT_PREC_FP64 runs the iteration in complex128.  FIT_PREC_MIXED
// runs it in complex64 on the normalised residual with complex128 refinement
// (x += ||r|| d, true residual recomputed in complex128) and finishes any
// system whose complex64 refinement stalls in complex128.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <type_traits>
#include <vector>

#include "fit_internal.h"
#include "krylov.h"
#include "solver_ctx.h"
#include "solver_kernels.h"
#include "stencil.h"
#include "tuning.h"

namespace fit {
fit_status port_voltages_dev(const fit_grid* g, const void* x_dev, int nvec, double* out_dev,
                             hipStream_t s);
}

using namespace fit;

namespace {

constexpr int kMaxBatch = 64;
// systems advanced together per batch (at most kMaxBatch); set by
// fit_sweep_set_batch or fit_autotune_sweep, process-wide
std::atomic<int> g_sweep_batch{kMaxBatch};

// One system of the sweep.
struct Sys {
  fit_grid* g = nullptr;
  double omega = 0.0;
  const double* src = nullptr;  // impressed current (complex128)
  double* x = nullptr;          // field (complex128)
  double* b = nullptr;          // -j omega j
  double* r = nullptr;          // true residual b - A x (complex128)
  // inner iteration vectors, in the inner precision (sized for complex128)
  void *rin = nullptr, *d = nullptr, *ri = nullptr, *z = nullptr, *p[2] = {nullptr, nullptr},
       *q = nullptr, *m = nullptr;
  double* part = nullptr;
  unsigned* cnt = nullptr;
  RedOut* red = nullptr;
  CgState* st = nullptr;
  RedOut* h_red = nullptr;  // pinned
  int max_blocks = 0;
  // host bookkeeping
  double bnorm = 0.0, rnorm = 0.0, relres = 1.0, best_rel = 1.0;
  fit_status status = FIT_E_NOT_CONVERGED;
  int iters = 0, refin = 0, matvecs = 0, fell_back = 0, stall = 0;
  bool running = true;  // still refining
  double bytes = 0.0;
  // inner run
  int inner_done = kRunning, inner_iters = 0, best_at = 0;
  double best_rr = 0.0, q_inner = 0.5, eta = 0.0;
  bool m_ready = false;
};

Ctx ctx_of(Sys& y, hipStream_t s) {
  Ctx c{};
  c.g = y.g;
  c.s = s;
  c.omega = y.omega;
  c.sym = 0;
  c.part = y.part;
  c.cnt = y.cnt;
  c.red = y.red;
  c.bst = nullptr;
  c.gst = nullptr;
  c.h_red = y.h_red;
  c.h_bst = nullptr;
  c.h_gst = nullptr;
  c.cst = y.st;
  c.h_cst = nullptr;
  c.max_blocks = y.max_blocks;
  c.tile128 = tile_for(y.g, FIT_C128);
  c.tile64 = tile_for(y.g, FIT_C64);
  return c;
}

// z-chunk for grid g under the block shape t: the grid's tuned chunk when
// its tuned shape is t, else the default rule (>= ~1024 workgroups, zc >= 8).
int zc_for(const fit_grid* g, int dtype, TileShape t) {
  const TileShape tt = tile_for(g, dtype);
  if (tt.tx == t.tx && tt.ty == t.ty) return tt.zc;
  const long nbx = (g->view.nx + t.tx - 3) / (t.tx - 2), nby = (g->view.ny + t.ty - 3) / (t.ty - 2);
  int zc = std::min(g->view.nz, kMaxZChunk);
  while (zc > 8 && nbx * nby * ((g->view.nz + zc - 1) / zc) < 1024) zc = (zc + 1) / 2;
  return std::max(zc, 1);
}

// Upper bound on the workgroups of any operator launch a system of grid g
// makes (its own tiles, or any compiled shape under the batch rule), and of
// the streaming kernels.
int max_blocks_for(const fit_grid* g) {
  int mb = 8192;
  const TileShape shapes[] = {{64, 8, 0}, {48, 8, 0}, {32, 8, 0}, {32, 16, 0}};
  for (int dt : {(int)FIT_C128, (int)FIT_C64, (int)FIT_TILE_BATCHED_C128}) {
    mb = std::max(mb, launch_blocks(make_launch(g->view, tile_for(g, dt), 1.0)));
    for (TileShape t : shapes) {
      t.zc = zc_for(g, dt, t);
      mb = std::max(mb, launch_blocks(make_launch(g->view, t, 1.0)));
    }
  }
  return mb;
}

// Per-system device bytes (arena layout below).
size_t sys_bytes(const fit_grid* g, bool own_x, int max_blocks) {
  const size_t v = align_up((size_t)g->ne * 16, 256);
  return v * ((own_x ? 1 : 0) + 2 + 8) + align_up(sizeof(double) * 4 * (size_t)max_blocks, 256) +
         256 + align_up(sizeof(RedOut), 256) + align_up(sizeof(CgState), 256);
}

void carve(Sys& y, Arena& a, bool own_x) {
  const size_t v = (size_t)y.g->ne * 16;
  if (own_x) y.x = a.take<double>(v);
  y.b = a.take<double>(v);
  y.r = a.take<double>(v);
  y.rin = a.take<char>(v);
  y.d = a.take<char>(v);
  y.ri = a.take<char>(v);
  y.z = a.take<char>(v);
  y.p[0] = a.take<char>(v);
  y.p[1] = a.take<char>(v);
  y.q = a.take<char>(v);
  y.m = a.take<char>(v);
  y.part = a.take<double>(sizeof(double) * 4 * (size_t)y.max_blocks);
  y.cnt = a.take<unsigned>(256);
  y.red = a.take<RedOut>(sizeof(RedOut));
  y.st = a.take<CgState>(sizeof(CgState));
}

struct BatchGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~BatchGraph() { reset(); }
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
};

// Device-side launch tables of one captured batch, in precision T.
template <class T>
struct Tables {
  MultiItem<OpCocgPX<T>>* stencil[2] = {nullptr, nullptr};  // by parity
  FinishItem<OpFinish<OpCocgPX<T>>>* fin1[2] = {nullptr, nullptr};
  OtfItem<T>* upd[2] = {nullptr, nullptr};
  FinishItem<CocgFinish>* fin2 = nullptr;
  int n = 0, stencil_blocks = 0, upd_blocks = 0;
  TileShape shape{32, 8, 8};
};

// Builds and uploads the launch tables for the systems `act` (synchronous).
template <class T>
fit_status build_tables(std::vector<Sys*>& act, Tables<T>& t, void* dev_buf, hipStream_t s) {
  // tile-table key of the batched launches' block shape (complex128: the
  // sweep tuner's own entry, else the single-system shape)
  const int dtype = sizeof(T) == 8 ? FIT_TILE_BATCHED_C128 : FIT_C64;
  // one block shape for the launch: the largest grid's
  const Sys* big = act[0];
  for (Sys* y : act)
    if (y->g->ne > big->g->ne) big = y;
  t.shape = tile_for(big->g, dtype);
  const int n = (int)act.size();
  std::vector<MultiItem<OpCocgPX<T>>> st[2];
  std::vector<FinishItem<OpFinish<OpCocgPX<T>>>> f1[2];
  std::vector<OtfItem<T>> up[2];
  std::vector<FinishItem<CocgFinish>> f2;
  int sb = 0, ub = 0;
  for (int i = 0; i < n; ++i) {
    Sys& y = *act[i];
    TileShape ts = t.shape;
    ts.zc = zc_for(y.g, dtype, t.shape);
    const StencilLaunch L = make_launch(y.g->view, ts, y.omega);
    const int nb = launch_blocks(L);
    const int nu = otf_shape(y.g->view, y.max_blocks).blocks;
    if (nb > y.max_blocks || nu > y.max_blocks) {
      set_error("fit_sweep: internal launch larger than its partials buffer");
      return FIT_E_DEVICE;
    }
    for (int par = 0; par < 2; ++par) {
      T* p_old = (T*)y.p[par];
      T* p_new = (T*)y.p[par ^ 1];
      OpCocgPX<T> op{(const T*)y.ri, p_old, p_new, (T*)y.q, (T*)y.d, y.st, y.part,
                     (T)(y.omega * y.omega), {}, {}};
      st[par].push_back(MultiItem<OpCocgPX<T>>{y.g->view, L, op, sb, nb});
      f1[par].push_back(FinishItem<OpFinish<OpCocgPX<T>>>{y.part, nb, OpFinish<OpCocgPX<T>>{op}});
      up[par].push_back(OtfItem<T>{y.g->view, y.omega, (T*)y.ri, (const T*)y.q, y.st, y.part, ub, nu});
    }
    f2.push_back(FinishItem<CocgFinish>{y.part, nu, CocgFinish{y.st}});
    sb += nb;
    ub += nu;
  }
  t.n = n;
  t.stencil_blocks = sb;
  t.upd_blocks = ub;
  char* p = (char*)dev_buf;
  auto put = [&](auto& vec, auto*& dst) -> fit_status {
    using E = typename std::decay<decltype(vec)>::type::value_type;
    dst = (E*)p;
    const size_t bytes = sizeof(E) * vec.size();
    FIT_HIP(hipMemcpyAsync(p, vec.data(), bytes, hipMemcpyHostToDevice, s));
    p += align_up(bytes, 256);
    return FIT_OK;
  };
  fit_status e;
  for (int par = 0; par < 2; ++par) {
    if ((e = put(st[par], t.stencil[par])) != FIT_OK) return e;
    if ((e = put(f1[par], t.fin1[par])) != FIT_OK) return e;
    if ((e = put(up[par], t.upd[par])) != FIT_OK) return e;
  }
  if ((e = put(f2, t.fin2)) != FIT_OK) return e;
  FIT_HIP(hipStreamSynchronize(s));
  return FIT_OK;
}

template <class T>
size_t table_bytes(int n) {
  return 2 * (align_up(sizeof(MultiItem<OpCocgPX<T>>) * n, 256) +
              align_up(sizeof(FinishItem<OpFinish<OpCocgPX<T>>>) * n, 256) +
              align_up(sizeof(OtfItem<T>) * n, 256)) +
         align_up(sizeof(FinishItem<CocgFinish>) * n, 256) + 4096;
}

template <class T>
fit_status one_iter(const Tables<T>& t, int par, hipStream_t s) {
  fit_status e = launch_stencil_multi<T, MODE_D>(t.stencil[par], t.n, t.stencil_blocks, t.shape, s,
                                                sizeof(T) == 8 ? "sweep_cocg_step1_c128"
                                                               : "sweep_cocg_step1_c64");
  if (e != FIT_OK) return e;
  hipLaunchKernelGGL((finish_multi_kernel<2, OpFinish<OpCocgPX<T>>>), dim3(t.n), dim3(256), 0, s,
                     t.fin1[par]);
  FIT_HIP(hipGetLastError());
  const int tok = prof_begin(s);
  hipLaunchKernelGGL((pcocg_rupdate_otf_multi_kernel<T, kOtfZc>), dim3(t.upd_blocks), dim3(256), 0, s,
                     t.upd[par], t.n);
  FIT_HIP(hipGetLastError());
  prof_end(tok, s, sizeof(T) == 8 ? "sweep_cocg_update_c128" : "sweep_cocg_update_c64");
  hipLaunchKernelGGL((finish_multi_kernel<3, CocgFinish>), dim3(t.n), dim3(256), 0, s, t.fin2);
  FIT_HIP(hipGetLastError());
  return FIT_OK;
}

template <class T>
fit_status capture(const Tables<T>& t, int check_every, BatchGraph& bg) {
  bg.reset();
  hipStream_t cap = nullptr;
  FIT_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  hipError_t he = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  fit_status e = he == hipSuccess ? FIT_OK : hip_fail(he, "hipStreamBeginCapture");
  for (int k = 0; k < check_every && e == FIT_OK; ++k) e = one_iter<T>(t, k & 1, cap);
  if (he == hipSuccess) he = hipStreamEndCapture(cap, &bg.graph);
  (void)hipStreamDestroy(cap);
  if (e != FIT_OK) return e;
  if (he != hipSuccess) return hip_fail(he, "hipStreamEndCapture");
  he = hipGraphInstantiate(&bg.exec, bg.graph, nullptr, nullptr, 0);
  if (he != hipSuccess) return hip_fail(he, "hipGraphInstantiate");
  return FIT_OK;
}

// Starts one inner COCG run for system y on A d = rin (unit-norm rin in
// precision T), from d = 0, to the relative tolerance y.q_inner.
template <class T>
fit_status start_inner(Sys& y, int budget, hipStream_t s) {
  Ctx c = ctx_of(y, s);
  const int64_t ne = y.g->ne;
  fit_status e;
  if ((e = vzero<T>(c, (T*)y.d, ne)) != FIT_OK) return e;
  if ((e = vzero<T>(c, (T*)y.p[0], ne)) != FIT_OK) return e;
  if ((e = vcopy<T>(c, (const T*)y.rin, (T*)y.ri, ne)) != FIT_OK) return e;
  if (!y.m_ready) {
    hipLaunchKernelGGL(mass_inverse_kernel<T>, dim3((unsigned)pw_blocks(y.g->view.np)), dim3(256),
                       0, s, y.g->view, y.omega, (T*)y.m);
    FIT_HIP(hipGetLastError());
    y.m_ready = true;
  }
  CgState h{};
  h.tol2 = y.q_inner * y.q_inner;
  h.hscale = 1.0;
  h.max_iter = budget;
  h.done = kRunning;
  FIT_HIP(hipMemcpyAsync(y.st, &h, sizeof(CgState), hipMemcpyHostToDevice, s));
  const int nb = pw_blocks(ne);
  hipLaunchKernelGGL((pcocg_update_kernel<T, true>), dim3((unsigned)nb), dim3(256), 0, s, ne,
                     (T*)y.d, (T*)y.ri, (T*)y.z, (const T*)y.p[0], (const T*)y.q, (const T*)y.m,
                     y.st, y.part);
  FIT_HIP(hipGetLastError());
  FIT_HIP(launch_finish<3>(y.part, nb, PcocgInitFinish{y.st}, s));
  y.inner_done = kRunning;
  y.inner_iters = 0;
  y.best_rr = 1.0;
  y.best_at = 0;
  return FIT_OK;
}

// Refinement loop over the systems of one batch in inner precision T.
template <class T>
fit_status run_batch(std::vector<Sys*>& sys, double tol, const fit_solve_opts& o, void* table_buf,
                     CgState* h_states, hipStream_t s) {
  const bool f32 = sizeof(T) == 4;
  const int stall_window = f32 ? 4000 : 30000;
  std::vector<Sys*> act;
  fit_status e;
  for (;;) {
    // systems that take another refinement step
    act.clear();
    for (Sys* y : sys)
      if (y->running) act.push_back(y);
    if (act.empty()) return FIT_OK;
    int64_t ne_sum = 0;
    for (Sys* y : act) {
      Ctx c = ctx_of(*y, s);
      // inner right-hand side: r / ||r|| in precision T
      if ((e = xform<double, T, XF_SCALE>(c, false, false, y->r, (T*)y->rin, 1.0 / y->rnorm, false)) != FIT_OK)
        return e;
      y->eta = y->rnorm;
      const double rel = y->rnorm / y->bnorm;
      double q = 0.5 * tol / rel;
      if (f32) q = std::max(q, o.inner_tol);
      y->q_inner = std::min(q, 0.5);
      const int budget = o.max_iters - y->iters;
      if ((e = start_inner<T>(*y, std::max(budget, 1), s)) != FIT_OK) return e;
      ne_sum += y->g->ne;
    }
    int check_every = o.check_every;
    if (check_every <= 0) check_every = 2 * std::max(1, std::min(100, (int)(4e8 / (double)ne_sum)));
    if (check_every & 1) ++check_every;

    // inner iterations of all systems in lockstep
    std::vector<Sys*> run = act;
    Tables<T> tab;
    BatchGraph bg;
    int captured = 0;
    while (!run.empty()) {
      if (captured == 0 || 2 * (int)run.size() <= captured) {
        if ((e = build_tables<T>(run, tab, table_buf, s)) != FIT_OK) return e;
        if (o.use_graph && (e = capture<T>(tab, check_every, bg)) != FIT_OK) return e;
        captured = (int)run.size();
      }
      if (o.use_graph) {
        hipError_t he = hipGraphLaunch(bg.exec, s);
        if (he != hipSuccess) return hip_fail(he, "hipGraphLaunch");
      } else {
        for (int k = 0; k < check_every; ++k)
          if ((e = one_iter<T>(tab, k & 1, s)) != FIT_OK) return e;
      }
      // poll every running system's state
      for (size_t i = 0; i < run.size(); ++i)
        FIT_HIP(hipMemcpyAsync(&h_states[i], run[i]->st, sizeof(CgState), hipMemcpyDeviceToHost, s));
      FIT_HIP(hipStreamSynchronize(s));
      std::vector<Sys*> still;
      for (size_t i = 0; i < run.size(); ++i) {
        Sys& y = *run[i];
        const CgState& h = h_states[i];
        y.inner_iters = h.iter;
        if (h.done != kRunning) {
          y.inner_done = h.done;
          continue;
        }
        if (h.rr < 0.25 * y.best_rr) {
          y.best_rr = h.rr;
          y.best_at = h.iter;
        } else if (h.iter - y.best_at >= stall_window) {
          // stagnated: stop this system's inner run
          const int stop = kBreakdown;
          FIT_HIP(hipMemcpyAsync(&y.st->done, &stop, sizeof(int), hipMemcpyHostToDevice, s));
          FIT_HIP(hipStreamSynchronize(s));
          y.inner_done = kBreakdown;
          continue;
        }
        still.push_back(&y);
      }
      run.swap(still);
    }

    // the fused step leaves the last solution update pending
    for (Sys* yp : act) {
      hipLaunchKernelGGL(cocg_fixup_kernel<T>, dim3((unsigned)pw_blocks(yp->g->ne)), dim3(256), 0, s,
                         yp->g->ne, (T*)yp->d, (const T*)yp->p[0], (const T*)yp->p[1], yp->st);
      FIT_HIP(hipGetLastError());
    }
    // x += eta d, true residual, decisions
    for (Sys* yp : act) {
      Sys& y = *yp;
      Ctx c = ctx_of(y, s);
      y.iters += y.inner_iters;
      y.matvecs += y.inner_iters + 1;
      y.refin += 1;
      y.bytes += (double)y.inner_iters * ((double)y.g->view.np * 3.0 * sizeof(T) * 2 * 10);
      if (y.inner_done == kNan) {
        y.status = FIT_E_NAN;
        y.running = false;
        continue;
      }
      if ((e = xform<T, double, XF_AXPY>(c, false, false, (const T*)y.d, y.x, y.eta, false)) != FIT_OK)
        return e;
      if ((e = residual(c, y.x, y.b, y.r, nullptr, 0.0)) != FIT_OK) return e;
      if ((e = sync_copy(c, y.h_red, y.red, sizeof(RedOut))) != FIT_OK) return e;
      double rn = std::sqrt(y.h_red->v[0]);
      if (!std::isfinite(rn) || rn > y.rnorm) {
        // the correction made things worse: undo it and stop this precision
        if ((e = xform<T, double, XF_AXPY>(c, false, false, (const T*)y.d, y.x, -y.eta, false)) != FIT_OK)
          return e;
        if ((e = residual(c, y.x, y.b, y.r, nullptr, 0.0)) != FIT_OK) return e;
        if ((e = sync_copy(c, y.h_red, y.red, sizeof(RedOut))) != FIT_OK) return e;
        rn = std::sqrt(y.h_red->v[0]);
        y.relres = rn / y.bnorm;
        y.rnorm = rn;
        y.status = !std::isfinite(rn) ? FIT_E_NAN
                   : (y.inner_done == kMaxIter || y.iters >= o.max_iters) ? FIT_E_NOT_CONVERGED
                                                                          : FIT_E_BREAKDOWN;
        y.running = false;
        continue;
      }
      y.rnorm = rn;
      y.relres = rn / y.bnorm;
      if (rn <= tol * y.bnorm) {
        y.status = FIT_OK;
        y.running = false;
        continue;
      }
      if (y.relres < 0.5 * y.best_rel) {
        y.best_rel = y.relres;
        y.stall = 0;
      } else {
        ++y.stall;
      }
      if (y.inner_done == kMaxIter || y.iters >= o.max_iters || y.stall >= 4) {
        y.status = FIT_E_NOT_CONVERGED;
        y.running = false;
      }
    }
  }
}

}  // namespace

extern "C" fit_status fit_sweep(fit_grid* const* grids, int ngrids, const double* omegas, int nomega,
                                const void* const* sources_dev, int nrhs, double tol,
                                const fit_solve_opts* opts, double* port_v_host,
                                void* const* x_dev_opt, fit_solve_info* infos) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!grids || ngrids < 1 || !omegas || nomega < 1 || !sources_dev || nrhs < 1) {
    set_error("fit_sweep: NULL argument or empty sweep");
    return FIT_E_INVALID;
  }
  if (!(tol > 0.0) || !(tol < 1.0)) {
    set_error("fit_sweep: tol must be in (0, 1)");
    return FIT_E_INVALID;
  }
  for (int f = 0; f < nomega; ++f) {
    if (!(omegas[f] > 0.0) || !std::isfinite(omegas[f])) {
      set_error("fit_sweep: every omega must be finite and > 0");
      return FIT_E_INVALID;
    }
  }
  for (int gi = 0; gi < ngrids; ++gi) {
    if (!grids[gi] || !sources_dev[gi] || (x_dev_opt && !x_dev_opt[gi])) {
      set_error("fit_sweep: NULL grid, source or field buffer");
      return FIT_E_INVALID;
    }
    if (grids[gi]->device != grids[0]->device) {
      set_error("fit_sweep: all grids must live on one device");
      return FIT_E_INVALID;
    }
  }
  fit_solve_opts o{};
  if (opts) o = *opts;
  if (o.max_iters <= 0) o.max_iters = 100000;
  if (o.inner_tol <= 0.0) o.inner_tol = 1e-4;
  if (o.solver != FIT_COCG || (o.precision != FIT_PREC_FP64 && o.precision != FIT_PREC_MIXED)) {
    set_error("fit_sweep: the batched sweep runs COCG (opts.solver = FIT_COCG), FP64 or MIXED");
    return FIT_E_UNSUPPORTED;
  }
  DeviceScope dev(grids[0]->device);
  hipStream_t s = (hipStream_t)o.stream;

  // the system list, grid-major as in the output layout
  std::vector<Sys> all;
  all.reserve((size_t)ngrids * nomega * nrhs);
  for (int gi = 0; gi < ngrids; ++gi)
    for (int f = 0; f < nomega; ++f)
      for (int r = 0; r < nrhs; ++r) {
        Sys y;
        y.g = grids[gi];
        y.omega = omegas[f];
        y.src = (const double*)sources_dev[gi] + (size_t)r * 2 * grids[gi]->ne;
        if (x_dev_opt) y.x = (double*)x_dev_opt[gi] + ((size_t)f * nrhs + r) * 2 * grids[gi]->ne;
        y.max_blocks = max_blocks_for(y.g);
        all.push_back(y);
      }
  const int nsys = (int)all.size();
  const bool own_x = x_dev_opt == nullptr;

  // batches: consecutive systems within a device-memory budget
  size_t free_b = 0, total_b = 0;
  FIT_HIP(hipMemGetInfo(&free_b, &total_b));
  const size_t budget = std::max<size_t>(free_b / 2, (size_t)1 << 30);
  std::vector<std::pair<int, int>> batches;
  for (int i = 0; i < nsys;) {
    size_t used = 0;
    int j = i;
    const int cap = std::max(1, std::min<int>(kMaxBatch, g_sweep_batch.load()));
    while (j < nsys && j - i < cap) {
      const size_t need = sys_bytes(all[j].g, own_x, all[j].max_blocks);
      if (j > i && used + need > budget) break;
      used += need;
      ++j;
    }
    batches.push_back({i, j});
    i = j;
  }

  // port-voltage offsets: [g][f][r][p]
  std::vector<size_t> port_off(nsys + 1, 0);
  for (int i = 0; i < nsys; ++i) port_off[i + 1] = port_off[i] + (size_t)all[i].g->nports;

  void* pinned = nullptr;
  FIT_HIP(hipHostMalloc(&pinned, sizeof(RedOut) * kMaxBatch + sizeof(CgState) * kMaxBatch + 256));
  RedOut* h_red = (RedOut*)pinned;
  CgState* h_states = (CgState*)((char*)pinned + sizeof(RedOut) * kMaxBatch);
  double* d_ports = nullptr;
  void* arena = nullptr;
  fit_status result = FIT_OK;
  auto fail = [&](fit_status e) {
    result = e;
    return e;
  };
  std::vector<double> ports_host(2 * std::max<size_t>(port_off[nsys], 1), 0.0);
  if (port_off[nsys] > 0) {
    hipError_t he = hipMalloc(&d_ports, sizeof(double) * 2 * port_off[nsys]);
    if (he != hipSuccess) {
      (void)hipHostFree(pinned);
      return hip_fail(he, "hipMalloc(sweep ports)");
    }
  }
  size_t arena_bytes = 0;
  for (auto& bt : batches) {
    size_t need = table_bytes<double>(bt.second - bt.first) + 4096;
    for (int i = bt.first; i < bt.second; ++i) need += sys_bytes(all[i].g, own_x, all[i].max_blocks);
    arena_bytes = std::max(arena_bytes, need);
  }
  if (hipMalloc(&arena, arena_bytes) != hipSuccess) {
    (void)hipFree(d_ports);
    (void)hipHostFree(pinned);
    set_error("fit_sweep: out of device memory for the batch workspace");
    return FIT_E_NOMEM;
  }

  for (auto& bt : batches) {
    if (result != FIT_OK && result != FIT_E_NOT_CONVERGED && result != FIT_E_BREAKDOWN &&
        result != FIT_E_NAN)
      break;
    Arena a{(char*)arena, 0, arena_bytes};
    void* table_buf = a.take<char>(table_bytes<double>(bt.second - bt.first));
    std::vector<Sys*> sys;
    for (int i = bt.first; i < bt.second; ++i) {
      Sys& y = all[i];
      carve(y, a, own_x);
      y.h_red = &h_red[i - bt.first];
      sys.push_back(&y);
    }
    fit_status e = FIT_OK;
    // b = -j omega j, ||b||, masked-source check; x = 0, r = b
    for (Sys* yp : sys) {
      Sys& y = *yp;
      Ctx c = ctx_of(y, s);
      FIT_HIP(hipMemsetAsync(y.red, 0, sizeof(RedOut), s));
      if ((e = xform<double, double, XF_RHS>(c, false, false, y.src, y.b, 1.0, true)) != FIT_OK) break;
      if ((e = sync_copy(c, y.h_red, y.red, sizeof(RedOut))) != FIT_OK) break;
      if (y.h_red->flag) {
        set_error("fit_sweep: nonzero source on a masked edge");
        e = FIT_E_INVALID;
        break;
      }
      y.bnorm = std::sqrt(y.h_red->v[0]);
      if ((e = vzero<double>(c, y.x, y.g->ne)) != FIT_OK) break;
      if ((e = vcopy<double>(c, y.b, y.r, y.g->ne)) != FIT_OK) break;
      y.rnorm = y.bnorm;
      if (!std::isfinite(y.bnorm)) {
        y.status = FIT_E_NAN;
        y.running = false;
      } else if (y.bnorm == 0.0) {
        y.status = FIT_OK;
        y.relres = 0.0;
        y.running = false;
      }
    }
    if (e != FIT_OK) {
      fail(e);
      break;
    }
    if (o.precision == FIT_PREC_MIXED) {
      if ((e = run_batch<float>(sys, tol, o, table_buf, h_states, s)) != FIT_OK) {
        fail(e);
        break;
      }
      // complex64 stalled: continue in complex128 from the current x
      for (Sys* yp : sys) {
        Sys& y = *yp;
        if (y.status != FIT_OK && y.status != FIT_E_NAN && y.iters < o.max_iters) {
          y.running = true;
          y.fell_back = 1;
          y.m_ready = false;
          y.stall = 0;
          y.best_rel = y.relres;
        }
      }
    }
    if ((e = run_batch<double>(sys, tol, o, table_buf, h_states, s)) != FIT_OK) {
      fail(e);
      break;
    }
    for (Sys* yp : sys) {
      Sys& y = *yp;
      const int idx = (int)(yp - all.data());
      if (y.g->nports > 0 &&
          (e = port_voltages_dev(y.g, y.x, 1, d_ports + 2 * port_off[idx], s)) != FIT_OK)
        break;
      if (y.status != FIT_OK && result == FIT_OK) result = y.status;
    }
    if (e != FIT_OK) {
      fail(e);
      break;
    }
    FIT_HIP(hipStreamSynchronize(s));
  }
  const auto t1 = std::chrono::steady_clock::now();
  const double ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  if (port_off[nsys] > 0 && (result == FIT_OK || result == FIT_E_NOT_CONVERGED ||
                             result == FIT_E_BREAKDOWN || result == FIT_E_NAN)) {
    hipError_t he = hipMemcpy(ports_host.data(), d_ports, sizeof(double) * 2 * port_off[nsys],
                              hipMemcpyDeviceToHost);
    if (he != hipSuccess) result = hip_fail(he, "sweep ports copy");
    else if (port_v_host) std::memcpy(port_v_host, ports_host.data(), sizeof(double) * 2 * port_off[nsys]);
  }
  if (infos && result != FIT_E_INVALID) {
    for (int i = 0; i < nsys; ++i) {
      fit_solve_info inf{};
      inf.status = all[i].status;
      inf.iterations = all[i].iters;
      inf.refinements = all[i].refin;
      inf.fell_back = all[i].fell_back;
      inf.matvecs = all[i].matvecs;
      inf.true_relres = all[i].relres;
      inf.time_ms = ms;
      inf.bytes_moved = all[i].bytes;
      infos[i] = inf;
    }
  }
  (void)hipFree(arena);
  (void)hipFree(d_ports);
  (void)hipHostFree(pinned);
  if (result != FIT_OK && result != FIT_E_INVALID && result != FIT_E_NOMEM && result != FIT_E_DEVICE) {
    int bad = 0;
    for (auto& y : all) bad += y.status != FIT_OK;
    set_error("fit_sweep: " + std::to_string(bad) + " of " + std::to_string(nsys) +
              " systems did not reach tol");
  }
  return result;
}

// ---------------------------------------------------------------------------
// Systems per batch: a process-wide setting and its autotuner.
// ---------------------------------------------------------------------------
extern "C" fit_status fit_sweep_set_batch(int systems) {
  if (systems < 1 || systems > kMaxBatch) {
    set_error("fit_sweep_set_batch: systems must be in [1, 64]");
    return FIT_E_INVALID;
  }
  g_sweep_batch.store(systems);
  return FIT_OK;
}

namespace {
__global__ void mask_to_source_kernel(const uint8_t* mask, int64_t ne, int nrep, double* src) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne * nrep;
       e += (int64_t)gridDim.x * blockDim.x) {
    src[2 * e] = mask[e % ne] ? 1.0 : 0.0;
    src[2 * e + 1] = 0.0;
  }
}
}  // namespace

extern "C" fit_status fit_autotune_sweep(fit_grid* g, const double* omegas, int nomega, int iters,
                                         void* stream, int32_t* best_batch, double* best_rate) {
  if (!g || !omegas || nomega < 1 || nomega > 4096 || iters < 2) {
    set_error("fit_autotune_sweep: bad argument (NULL, nomega outside [1, 4096] or iters < 2)");
    return FIT_E_INVALID;
  }
  for (int f = 0; f < nomega; ++f)
    if (!(omegas[f] > 0.0) || !std::isfinite(omegas[f])) {
      set_error("fit_autotune_sweep: omegas must be finite and > 0");
      return FIT_E_INVALID;
    }
  DeviceScope dev(g->device);
  hipStream_t s = (hipStream_t)stream;
  // one right-hand side: 1 A on every free edge (the tuner times iterations,
  // it never converges at the tolerance below)
  uint8_t* mask = nullptr;
  double* src = nullptr;
  FIT_HIP(hipMalloc(&mask, g->ne));
  hipError_t he = hipMalloc(&src, (size_t)g->ne * 16);
  if (he != hipSuccess) {
    (void)hipFree(mask);
    return hip_fail(he, "hipMalloc(autotune_sweep)");
  }
  fit_status st = fit_edge_mask(g, mask, s);
  if (st == FIT_OK) {
    hipLaunchKernelGGL(mask_to_source_kernel, dim3(1024), dim3(256), 0, s, mask, g->ne, 1, src);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) st = FIT_E_DEVICE;
  }
  const int saved = g_sweep_batch.load();
  int best_b = saved;
  double best = -1.0;
  fit_grid* grids[1] = {g};
  const void* srcs[1] = {src};
  auto run = [&](int nf, int cap, double* secs, int64_t* sys_iters) -> fit_status {
    fit_solve_opts o{};
    o.solver = FIT_COCG;
    o.precision = FIT_PREC_FP64;
    o.max_iters = cap;
    o.check_every = iters;
    o.use_graph = 1;
    o.stream = stream;
    std::vector<fit_solve_info> infos((size_t)nf);
    const auto t0 = std::chrono::steady_clock::now();
    const fit_status e = fit_sweep(grids, 1, omegas, nf, srcs, 1, 1e-15, &o, nullptr, nullptr,
                                   infos.data());
    *secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *sys_iters = 0;
    for (auto& i : infos) *sys_iters += i.iterations;
    return (e == FIT_OK || e == FIT_E_NOT_CONVERGED || e == FIT_E_BREAKDOWN) ? FIT_OK : e;
  };
  if (st == FIT_OK) {  // warm-up: first-use allocations stay out of the timed pairs
    double w = 0.0;
    int64_t wi = 0;
    g_sweep_batch.store(4);
    st = run(std::min(nomega, 4), iters, &w, &wi);
  }
  // system-iterations per second of the batched iteration itself for batches
  // of b systems (the difference of two runs removes set-up and capture);
  // negative if the runs stopped early
  auto rate_of = [&](int b, double* rate) -> fit_status {
    g_sweep_batch.store(b);
    const int nf = std::min(nomega, b);
    double secs[2] = {0.0, 0.0};
    int64_t its[2] = {0, 0};
    for (int rep = 0; rep < 2; ++rep) {
      const fit_status e = run(nf, rep == 0 ? iters : 2 * iters, &secs[rep], &its[rep]);
      if (e != FIT_OK) return e;
    }
    *rate = its[1] > its[0] ? (double)(its[1] - its[0]) / std::max(secs[1] - secs[0], 1e-9) : -1.0;
    return FIT_OK;
  };
  // The complex128 block shape of the batched launches (every system of a
  // launch uses the largest grid's shape): the compiled shapes with z-chunks
  // of 4 and 8 planes, timed on batches of up to 16 systems; the best one is
  // stored under the batched key for the grid's dimensions (single solves
  // keep theirs).  Shapes that suit one system at a time leave a batch of
  // small grids too few workgroups per system.
  const TileShape saved_tile = tile_for(g, FIT_TILE_BATCHED_C128);
  TileShape best_t = saved_tile;
  double best_tr = -1.0;
  const TileShape cands[] = {{32, 16, 4}, {32, 16, 8}, {32, 8, 4}, {32, 8, 8},
                             {48, 8, 4}, {48, 8, 8}, {64, 8, 4}, {64, 8, 8}};
  for (const TileShape& t : cands) {
    if (st != FIT_OK) break;
    if (t.zc > g->view.nz) continue;
    if ((st = fit_tile_set(g, FIT_TILE_BATCHED_C128, t.tx, t.ty, t.zc)) != FIT_OK) break;
    double rate = -1.0;
    if ((st = rate_of(16, &rate)) != FIT_OK) break;
    if (rate > 0.0 && (best_tr < 0.0 || rate > 1.02 * best_tr)) {
      best_tr = rate;
      best_t = t;
    }
  }
  {
    const fit_status e = st == FIT_OK
                             ? fit_tile_set(g, FIT_TILE_BATCHED_C128, best_t.tx, best_t.ty, best_t.zc)
                             : fit_tile_set(g, FIT_TILE_BATCHED_C128, saved_tile.tx, saved_tile.ty, saved_tile.zc);
    if (st == FIT_OK) st = e;
  }
  // largest batch first: a smaller batch must be more than 2 % faster to
  // replace it (fewer batches mean fewer serial tails of slow systems)
  for (int b : {64, 32, 16, 8, 4}) {
    if (st != FIT_OK) break;
    if (b > nomega && b != 4 && b / 2 >= nomega) continue;
    double rate = -1.0;
    if ((st = rate_of(b, &rate)) != FIT_OK) break;
    if (rate < 0.0) continue;
    if (best < 0.0 || rate > 1.02 * best) {
      best = rate;
      best_b = b;
    }
  }
  (void)hipFree(mask);
  (void)hipFree(src);
  g_sweep_batch.store(st == FIT_OK ? best_b : saved);
  if (st != FIT_OK) return st;
  if (best_batch) *best_batch = best_b;
  if (best_rate) *best_rate = best;
  return FIT_OK;
}

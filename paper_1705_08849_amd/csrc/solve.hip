// fit_solve: BiCGStab, restarted GMRES(m) and flexible GMRES(m) around the
// matrix-free operator, in complex128 or in complex64 with complex128
// iterative refinement.  The iteration always stops on the true relative
// residual of the unscaled complex128 system.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "diag.h"
#include "fit_internal.h"
#include "krylov.h"
#include "precond.h"
#include "solver_ctx.h"
#include "solver_kernels.h"
#include "stencil.h"
#include "tuning.h"

namespace fit {


// ---------------------------------------------------------------------------
// BiCGStab on A_int x = r0 (A_int = S A S when sym), starting from x = 0.
// The caller supplies r0 in `r` (overwritten).  Returns the device done code
// through *done and the iteration count through *iters.
// ---------------------------------------------------------------------------
template <class T>
struct BiVecs {
  T *x, *r, *rh, *p[2], *v[2], *s, *t;
  T* xb = nullptr;  // BiCGStab: the iterate with the smallest residual seen at a poll
};

template <class T>
static fit_status bicgstab(Ctx& c, BiVecs<T>& V, double tol_rel, int max_iter, int check_every,
                           double hscale, double* hist_dev, int hist_len, int use_graph,
                           uint64_t shadow_seed, int* done, int* iters, double* rr_out) {
  const int64_t ne = c.g->ne;
  fit_status st;
  if ((st = vzero(c, V.x, ne)) != FIT_OK) return st;
  if ((st = vzero(c, V.p[0], ne)) != FIT_OK) return st;
  if ((st = vzero(c, V.v[0], ne)) != FIT_OK) return st;
  // Shadow vector: dense pseudo-random on the free edges, a fresh seed for
  // every restart.  (The textbook choice r_hat = r_0 collapses for
  // lumped-port sources: r_0 lives on a handful of edges and <r_hat, r_k>
  // soon vanishes relative to |r_k|.)
  if ((st = xform<T, T, XF_SHADOW>(c, false, false, V.r, V.rh, 1.0, false, shadow_seed)) != FIT_OK)
    return st;
  hipLaunchKernelGGL(dot_kernel<T>, dim3(pw_blocks(ne)), dim3(256), 0, c.s, V.rh, V.r, ne, c.red,
                     c.part, c.cnt);
  FIT_HIP(hipGetLastError());
  FIT_HIP(launch_finish<4>(c.part, pw_blocks(ne), StoreSums<4>{c.red}, c.s));
  if ((st = sync_copy(c, c.h_red, c.red, sizeof(RedOut))) != FIT_OK) return st;
  const cx<double> rho0{c.h_red->v[0], c.h_red->v[1]};
  const double rhrh = c.h_red->v[2];
  const double r0 = c.h_red->v[3];
  *iters = 0;
  *rr_out = r0;
  if (!(r0 > 0.0) || !std::isfinite(r0)) {
    *done = r0 == 0.0 ? kConverged : kNan;
    return FIT_OK;
  }
  BiState h{};
  h.rho = rho0;
  h.alpha = cx<double>{1.0, 0.0};
  h.omega = cx<double>{1.0, 0.0};
  h.beta = cx<double>{0.0, 0.0};
  h.rr = r0;
  h.rhrh = rhrh;
  h.tol2 = tol_rel * tol_rel * r0;
  h.hscale = hscale;
  h.iter = 0;
  h.max_iter = max_iter;
  h.done = kRunning;
  h.hist = hist_dev;
  h.hist_len = hist_len;
  FIT_HIP(hipMemcpyAsync(c.bst, &h, sizeof(BiState), hipMemcpyHostToDevice, c.s));

  const int64_t nb = pw_blocks(ne);
  auto one_iter = [&](int parity) -> fit_status {
    T* p_old = V.p[parity];
    T* p_new = V.p[parity ^ 1];
    T* v_old = V.v[parity];
    T* v_new = V.v[parity ^ 1];
    OpBicgP<T> k1{V.r, p_old, v_old, V.rh, p_new, v_new, c.bst, c.part, c.cnt, {}, {}};
    fit_status e = launch_op_stencil_mode<T>(c, c.sym, k1);
    if (e != FIT_OK) return e;
    OpBicgS<T> k2{V.r, v_new, V.s, V.t, c.bst, c.part, c.cnt, {}};
    e = launch_op_stencil_mode<T>(c, c.sym, k2);
    if (e != FIT_OK) return e;
    const int tok = prof_begin(c.s);
    hipLaunchKernelGGL(bicg_update_kernel<T>, dim3((unsigned)nb), dim3(256), 0, c.s, V.x, V.r,
                       p_new, V.s, V.t, V.rh, ne, c.bst, c.part, c.cnt);
    FIT_HIP(hipGetLastError());
    prof_end(tok, c.s, sizeof(T) == 8 ? "bicgstab_update_c128" : "bicgstab_update_c64");
    FIT_HIP(launch_finish<3>(c.part, (int)nb, BicgFinish{c.bst}, c.s));
    return FIT_OK;
  };
  const double per_iter_bytes = node_bytes(c.g, 17, sizeof(T)) + node_bytes(c.g, 0, 0) * 1.0;
  if (check_every <= 0) check_every = 2 * std::max(1, std::min(50, (int)(2e8 / (double)ne)));
  if (check_every & 1) ++check_every;  // ping-pong parity returns to 0

  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  if (use_graph) {
    // Capture on a private stream (the null stream cannot be captured); the
    // instantiated graph is then launched in order on the caller's stream.
    hipStream_t cap = nullptr;
    FIT_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    const hipStream_t user = c.s;
    c.s = cap;
    hipError_t he = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    fit_status e = he == hipSuccess ? FIT_OK : hip_fail(he, "hipStreamBeginCapture");
    for (int q = 0; q < check_every && e == FIT_OK; ++q) e = one_iter(q & 1);
    if (he == hipSuccess) he = hipStreamEndCapture(cap, &graph);
    c.s = user;
    (void)hipStreamDestroy(cap);
    if (e != FIT_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return e;
    }
    if (he != hipSuccess) return hip_fail(he, "hipStreamEndCapture");
    he = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
    if (he != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return hip_fail(he, "hipGraphInstantiate");
    }
  }
  int last_iter = 0;
  fit_status ret = FIT_OK;
  double best_rr = r0;
  int best_at = 0;
  bool stalled = false;
  const int stall_window = sizeof(T) == 4 ? 1500 : 6000;
  // smallest recursive residual seen at a poll, and whether V.xb holds it
  double kept_rr = r0;
  bool kept = false;
  for (;;) {
    if (use_graph) {
      hipError_t he = hipGraphLaunch(gexec, c.s);
      if (he != hipSuccess) {
        ret = hip_fail(he, "hipGraphLaunch");
        break;
      }
    } else {
      for (int q = 0; q < check_every; ++q)
        if ((ret = one_iter(q & 1)) != FIT_OK) break;
      if (ret != FIT_OK) break;
    }
    if ((ret = sync_copy(c, c.h_bst, c.bst, sizeof(BiState))) != FIT_OK) break;
    c.bytes += per_iter_bytes * (c.h_bst->iter - last_iter);
    c.matvecs += 2 * (c.h_bst->iter - last_iter);
    last_iter = c.h_bst->iter;
    if (c.h_bst->done != kRunning) break;
    if (V.xb && std::isfinite(c.h_bst->rr) && c.h_bst->rr < kept_rr) {
      if ((ret = vcopy(c, V.x, V.xb, ne)) != FIT_OK) break;
      c.bytes += (double)ne * sizeof(T) * 4;
      kept_rr = c.h_bst->rr;
      kept = true;
    }
    // Stagnation: no halving of the recursive residual within the window.
    // Stop here; the caller restarts from the current iterate with a fresh
    // shadow vector (or falls back to complex128 in the mixed form).
    if (c.h_bst->rr < 0.25 * best_rr) {
      best_rr = c.h_bst->rr;
      best_at = c.h_bst->iter;
    } else if (c.h_bst->iter - best_at >= stall_window) {
      stalled = true;
      break;
    }
  }
  if (gexec) (void)hipGraphExecDestroy(gexec);
  if (graph) (void)hipGraphDestroy(graph);
  if (ret != FIT_OK) return ret;
  *done = stalled ? kBreakdown : c.h_bst->done;
  c.last_reason = stalled ? 9 : c.h_bst->reason;
  double rr_end = c.h_bst->rr;
  // hand back the best iterate seen at a poll when the run ended worse
  // (a breakdown or a stall leaves the last iterate, not the best one)
  if (kept && *done != kConverged && !(rr_end <= kept_rr)) {
    fit_status e = vcopy(c, V.xb, V.x, ne);
    if (e != FIT_OK) return e;
    c.bytes += (double)ne * sizeof(T) * 4;
    rr_end = kept_rr;
  }
  c.last_rr = rr_end / r0;
  *iters = c.h_bst->iter;
  *rr_out = rr_end;
  // The last step ends with p in p[parity] where parity = iter & 1; after an
  // odd number of iterations the fresh p lives in p[1].  x and r are final.
  return FIT_OK;
}

// ---------------------------------------------------------------------------
// Restarted (F)GMRES(m) on A_int x = r0 from x = 0 (r0 in w0, overwritten).
// ---------------------------------------------------------------------------
template <class T>
struct GmVecs {
  T* x;
  T* V;   // (m+1) basis vectors, stride ldv complex
  T* Z;   // m preconditioned directions (FGMRES) or null
  T* W[2];
  int64_t ldv;
  double* mdpart;  // multi-dot partials (m+1) * nblk complex
};

template <class T>
static fit_status gmres(Ctx& c, GmVecs<T>& V, int m, double tol_rel, int max_iter,
                        double hscale, double* hist_dev, int hist_len, PrecondApply* pre,
                        const T* r0, const double* b128, int* done, int* iters, double* rel_est,
                        double r0norm_abs) {
  const int64_t ne = c.g->ne;
  fit_status st;
  if ((st = vzero(c, V.x, ne)) != FIT_OK) return st;
  // w0 = r0; beta = ||r0||
  if ((st = vcopy(c, r0, V.W[0], ne)) != FIT_OK) return st;
  if ((st = xform<T, T, XF_SCALE>(c, false, false, V.W[0], V.W[0], 1.0, true)) != FIT_OK) return st;
  if ((st = sync_copy(c, c.h_red, c.red, sizeof(RedOut))) != FIT_OK) return st;
  double beta = std::sqrt(c.h_red->v[0]);
  const double target = tol_rel * beta;
  int it = 0;
  *done = kRunning;
  const int nblk_md = (int)((ne + 256 * kMdPer - 1) / (256 * kMdPer));
  int cur = 0;
  double best_beta = beta;
  int cycle = 0, best_cycle = 0;
  while (true) {
    if (!(beta > 0.0)) {
      *done = beta == 0.0 ? kConverged : kNan;
      break;
    }
    GmState h;
    std::memset(&h, 0, sizeof(h));
    h.m = m;
    h.j = 0;
    h.k = 0;
    h.g[0] = cx<double>{beta, 0.0};
    h.vscale = 1.0 / beta;
    h.beta = beta;
    h.tol = target;
    h.hscale = hscale;
    h.iter = it;
    h.max_iter = max_iter;
    h.done = kRunning;
    h.hist = hist_dev;
    h.hist_len = hist_len;
    FIT_HIP(hipMemcpyAsync(c.gst, &h, sizeof(GmState), hipMemcpyHostToDevice, c.s));
    for (int j = 0; j < m; ++j) {
      T* vj = V.V + 2 * V.ldv * j;
      T* wcur = V.W[cur];
      T* wnext = V.W[cur ^ 1];
      if (pre) {
        // FGMRES: v_j = w * vscale (separately), z_j = M(v_j), w' = A z_j
        hipLaunchKernelGGL(gm_normalize_kernel<T>, dim3(pw_blocks(ne)), dim3(256), 0, c.s, wcur,
                           vj, ne, c.gst);
        FIT_HIP(hipGetLastError());
        T* zj = V.Z + 2 * V.ldv * j;
        if ((st = pre->apply(c, vj, zj, sizeof(T) == 4)) != FIT_OK) return st;
        OpGmresMv<T> mv{zj, nullptr, wnext, c.gst, T(1)};
        if ((st = launch_op_stencil_mode<T>(c, c.sym, mv)) != FIT_OK) return st;
        c.bytes += (double)ne * sizeof(T) * 2 * 3;
      } else {
        OpGmresMv<T> mv{wcur, vj, wnext, c.gst, T(1)};
        if ((st = launch_op_stencil_mode<T>(c, c.sym, mv)) != FIT_OK) return st;
      }
      c.matvecs += 1;
      c.bytes += node_bytes(c.g, 3, sizeof(T));
      // CGS2: two rounds of multi-dot + update
      for (int round = 0; round < 2; ++round) {
        hipLaunchKernelGGL(multidot_kernel<T>, dim3(nblk_md), dim3(256), 0, c.s, V.V, V.ldv,
                           j + 1, wnext, ne, V.mdpart, c.gst);
        FIT_HIP(hipGetLastError());
        hipLaunchKernelGGL(multidot_finish_kernel, dim3(j + 1), dim3(256), 0, c.s, V.mdpart,
                           nblk_md, c.gst, round);
        FIT_HIP(hipGetLastError());
        hipLaunchKernelGGL(multi_axpy_kernel<T>, dim3(pw_blocks(ne)), dim3(256), 0, c.s, V.V,
                           V.ldv, j + 1, wnext, ne, c.gst, round == 1 ? c.red : nullptr, c.part,
                           c.cnt);
        FIT_HIP(hipGetLastError());
        if (round == 1) FIT_HIP(launch_finish<1>(c.part, pw_blocks(ne), StoreSums<1>{c.red}, c.s));
        c.bytes += (double)ne * sizeof(T) * 2 * ((j + 2) + (j + 3));
      }
      hipLaunchKernelGGL(gmres_step_kernel, dim3(1), dim3(64), 0, c.s, c.gst, c.red);
      FIT_HIP(hipGetLastError());
      cur ^= 1;
      // Poll every few steps so converged cycles end early.
      if ((j & 7) == 7 || j == m - 1) {
        if ((st = sync_copy(c, c.h_gst, c.gst, sizeof(GmState))) != FIT_OK) return st;
        if (c.h_gst->done != kRunning) break;
      }
    }
    if ((st = sync_copy(c, c.h_gst, c.gst, sizeof(GmState))) != FIT_OK) return st;
    it = c.h_gst->iter;
    const int code = c.h_gst->done;
    const int k = c.h_gst->k;
    if (k > 0) {
      hipLaunchKernelGGL(gmres_solve_kernel, dim3(1), dim3(64), 0, c.s, c.gst);
      FIT_HIP(hipGetLastError());
      hipLaunchKernelGGL(gmres_update_kernel<T>, dim3(pw_blocks(ne)), dim3(256), 0, c.s, V.x,
                         pre ? V.Z : V.V, V.ldv, ne, c.gst);
      FIT_HIP(hipGetLastError());
      c.bytes += (double)ne * sizeof(T) * 2 * (k + 2);
    }
    *rel_est = std::sqrt(cabs2(c.h_gst->g[k])) / (beta > 0 ? beta : 1.0);
    if (code == kConverged || code == kNan || code == kMaxIter) {
      *done = code;
      break;
    }
    // restart: recompute the internal residual w = r0 - A_int x
    hipLaunchKernelGGL(gm_restart_prep_kernel, dim3(1), dim3(64), 0, c.s, c.gst);
    FIT_HIP(hipGetLastError());
    OpGmresMv<T> mv{V.x, nullptr, V.W[0], c.gst, T(1)};
    if ((st = launch_op_stencil_mode<T>(c, c.sym, mv)) != FIT_OK) return st;
    c.matvecs += 1;
    hipLaunchKernelGGL(sub_norm_kernel<T>, dim3(pw_blocks(ne)), dim3(256), 0, c.s, r0, V.W[0],
                       ne, c.red, c.part, c.cnt);
    FIT_HIP(hipGetLastError());
    FIT_HIP(launch_finish<1>(c.part, pw_blocks(ne), StoreSums<1>{c.red}, c.s));
    if ((st = sync_copy(c, c.h_red, c.red, sizeof(RedOut))) != FIT_OK) return st;
    cur = 0;
    beta = std::sqrt(c.h_red->v[0]);
    if (beta <= target) {
      *done = kConverged;
      break;
    }
    ++cycle;
    if (beta < 0.5 * best_beta) {
      best_beta = beta;
      best_cycle = cycle;
    } else if (c.gm_stall_cycles > 0 && cycle - best_cycle >= c.gm_stall_cycles) {
      *done = kBreakdown;  // stalled: the caller falls back
      c.last_reason = 9;
      break;
    }
  }
  *iters = it;
  (void)b128;
  (void)r0norm_abs;
  return FIT_OK;
}

// Identity right preconditioner (FGMRES without a learned model).
struct IdentityPrecond : PrecondApply {
  fit_status apply(Ctx& c, const void* v, void* z, bool f32) override {
    if (f32) return vcopy<float>(c, (const float*)v, (float*)z, c.g->ne);
    return vcopy<double>(c, (const double*)v, (double*)z, c.g->ne);
  }
};


// Inner solve in precision T on A_int d = rin (rin has unit norm), from d = 0.
// COCR vectors: x, r, p, q = A p, w = A r.
template <class T>
struct CrVecs {
  T *x, *r, *p, *q, *w;
};
// TFQMR vectors: the even and odd u and their products, w, v, d, shadow.
template <class T>
struct TqVecs {
  T *x, *w, *u0, *u1, *au0, *au1, *v, *d, *rh;
};
// CGS vectors: x, r, the shadow, u (then w = u + q), p, q, v (A p, then A w).
template <class T>
struct CgsVecs {
  T *x, *r, *rh, *u, *p, *q, *v;
};

template <class T>
struct Inner {
  int solver, m;
  BiVecs<T> bv;
  GmVecs<T> gv;
  CrVecs<T> cr;
  TqVecs<T> tq;
  CgsVecs<T> cg;
  T* rin;
  T* d;
  // true: the inner method applies the symmetric scaling itself (as a
  // preconditioner) and works on unscaled vectors
  bool own_scaling = false;
  int restarts = 0;  // inner solves started (BiCGStab: selects the shadow seed)
};

// COCG on A_int x = r (r overwritten), from x = 0; same driver structure as
// bicgstab(): fused kernels, device scalars, periodic host polls, optional
// captured graph, stagnation window.
template <class T>
static fit_status cocg(Ctx& c, BiVecs<T>& V, double tol_rel, int max_iter, int check_every,
                       double hscale, double* hist_dev, int hist_len, int use_graph, int* done,
                       int* iters) {
  const int64_t ne = c.g->ne;
  fit_status st;
  T* q = V.v[0];
  if ((st = vzero(c, V.x, ne)) != FIT_OK) return st;
  if ((st = vzero(c, V.p[0], ne)) != FIT_OK) return st;
  hipLaunchKernelGGL((dot_kernel<T, true>), dim3(pw_blocks(ne)), dim3(256), 0, c.s, V.r, V.r, ne,
                     c.red, c.part, c.cnt);
  FIT_HIP(hipGetLastError());
  FIT_HIP(launch_finish<4>(c.part, pw_blocks(ne), StoreSums<4>{c.red}, c.s));
  if ((st = sync_copy(c, c.h_red, c.red, sizeof(RedOut))) != FIT_OK) return st;
  const cx<double> rho0{c.h_red->v[0], c.h_red->v[1]};
  const double r0 = c.h_red->v[2];
  *iters = 0;
  if (!(r0 > 0.0) || !std::isfinite(r0)) {
    *done = r0 == 0.0 ? kConverged : kNan;
    return FIT_OK;
  }
  CgState h{};
  h.rho = rho0;
  h.beta = cx<double>{0.0, 0.0};
  h.alpha = cx<double>{0.0, 0.0};
  h.rr = r0;
  h.tol2 = tol_rel * tol_rel * r0;
  h.hscale = hscale / std::sqrt(r0);
  h.max_iter = max_iter;
  h.done = kRunning;
  h.hist = hist_dev;
  h.hist_len = hist_len;
  FIT_HIP(hipMemcpyAsync(c.cst, &h, sizeof(CgState), hipMemcpyHostToDevice, c.s));
  const int64_t nb = pw_blocks(ne);
  // With the symmetric scaling requested, COCG runs on the unscaled operator
  // preconditioned by M = S^2 (z = M r); the iterates equal those of COCG on
  // S A S, and the operator kernel needs no per-edge square roots.  A stored
  // diagonal (c.diag: the mass matrix, the paper's eq. (Precond) or Jacobi)
  // runs the unfused form instead: z = m .* r kept as a vector.
  const bool stored = c.diag != 0;
  const bool pre = !stored && c.sym != 0;
  T* z = V.s;
  T* mdiag = V.t;
  const int64_t nbn = nb;
  const OtfShape otf = otf_shape(c.g->view, c.max_blocks);
  if (stored) {
    hipLaunchKernelGGL(edge_diag_kernel<T>, dim3((unsigned)pw_blocks(c.g->view.np)), dim3(256), 0,
                       c.s, c.g->view, c.omega, c.diag, mdiag);
    FIT_HIP(hipGetLastError());
    // COCG's iterates do not change when M is scaled by a constant; scale m
    // to unit rms so that rho = r^T z keeps the magnitude of r^T r and the
    // breakdown test (|rho| against ||r||^2) means the same for every
    // diagonal (1/K_ee is ~1e-11 in SI units, 1/M_eps,c ~1e16)
    if ((st = xform<T, T, XF_SCALE>(c, false, false, mdiag, mdiag, 1.0, true)) != FIT_OK) return st;
    if ((st = sync_copy(c, c.h_red, c.red, sizeof(RedOut))) != FIT_OK) return st;
    const double m2 = c.h_red->v[0];
    if (!(m2 > 0.0) || !std::isfinite(m2)) {
      *done = kNan;
      return FIT_OK;
    }
    if ((st = xform<T, T, XF_SCALE>(c, false, false, mdiag, mdiag, std::sqrt((double)ne / m2), false)) != FIT_OK)
      return st;
    hipLaunchKernelGGL((pcocg_update_kernel<T, true>), dim3((unsigned)nbn), dim3(256), 0, c.s, ne,
                       V.x, V.r, z, V.p[0], q, mdiag, c.cst, c.part);
    FIT_HIP(hipGetLastError());
    FIT_HIP(launch_finish<3>(c.part, (int)nbn, PcocgInitFinish{c.cst}, c.s));
  }
  if (pre) {
    hipLaunchKernelGGL(mass_inverse_kernel<T>, dim3((unsigned)pw_blocks(c.g->view.np)), dim3(256),
                       0, c.s, c.g->view, c.omega, mdiag);
    FIT_HIP(hipGetLastError());
    hipLaunchKernelGGL((pcocg_update_kernel<T, true>), dim3((unsigned)nbn), dim3(256), 0, c.s, ne,
                       V.x, V.r, z, V.p[0], q, mdiag, c.cst, c.part);
    FIT_HIP(hipGetLastError());
    FIT_HIP(launch_finish<3>(c.part, (int)nbn, PcocgInitFinish{c.cst}, c.s));
  }
  auto one_iter = [&](int parity) -> fit_status {
    T* p_old = V.p[parity];
    T* p_new = V.p[parity ^ 1];
    fit_status e;
    if (pre) {
      // fused form: m recomputed in the operator launch, x updated one step late
      OpCocgPX<T> k1{V.r, p_old, p_new, q, V.x, c.cst, c.part, (T)(c.omega * c.omega), {}, {}};
      if ((e = launch_op_stencil_mode<T>(c, false, k1)) != FIT_OK) return e;
    } else {
      // p = z + beta p_old (z = r without a preconditioner), q = A p
      OpCocgP<T> k1{stored ? z : V.r, p_old, p_new, q, c.cst, c.part, c.cnt, {}};
      if ((e = launch_op_stencil_mode<T>(c, false, k1)) != FIT_OK) return e;
    }
    const int tok = prof_begin(c.s);
    if (stored) {
      hipLaunchKernelGGL((pcocg_update_kernel<T, false>), dim3((unsigned)nbn), dim3(256), 0, c.s,
                         ne, V.x, V.r, z, p_new, q, mdiag, c.cst, c.part);
    } else if (pre) {
      hipLaunchKernelGGL((pcocg_rupdate_otf_kernel<T, kOtfZc>), dim3((unsigned)otf.blocks), dim3(256),
                         0, c.s, c.g->view, c.omega, V.r, q, c.cst, c.part);
    } else {
      hipLaunchKernelGGL(cocg_update_kernel<T>, dim3((unsigned)nb), dim3(256), 0, c.s, V.x, V.r,
                         p_new, q, ne, c.cst, c.part, c.cnt);
    }
    FIT_HIP(hipGetLastError());
    prof_end(tok, c.s, sizeof(T) == 8 ? "cocg_update_c128" : "cocg_update_c64");
    FIT_HIP(launch_finish<3>(c.part, (int)(pre ? otf.blocks : nb), CocgFinish{c.cst}, c.s));
    return FIT_OK;
  };
  const double per_iter_bytes = node_bytes(c.g, stored ? 12 : (pre ? 9 : 10), sizeof(T));
  if (check_every <= 0) check_every = 2 * std::max(1, std::min(100, (int)(4e8 / (double)ne)));
  if (check_every & 1) ++check_every;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  if (use_graph) {
    hipStream_t cap = nullptr;
    FIT_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    const hipStream_t user = c.s;
    c.s = cap;
    hipError_t he = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    fit_status e = he == hipSuccess ? FIT_OK : hip_fail(he, "hipStreamBeginCapture");
    for (int k = 0; k < check_every && e == FIT_OK; ++k) e = one_iter(k & 1);
    if (he == hipSuccess) he = hipStreamEndCapture(cap, &graph);
    c.s = user;
    (void)hipStreamDestroy(cap);
    if (e != FIT_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return e;
    }
    if (he != hipSuccess) return hip_fail(he, "hipStreamEndCapture");
    he = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
    if (he != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return hip_fail(he, "hipGraphInstantiate");
    }
  }
  int last_iter = 0;
  fit_status ret = FIT_OK;
  double best_rr = r0;
  int best_at = 0;
  bool stalled = false;
  // COCG residuals oscillate by orders of magnitude before they fall; the
  // window is wide so only genuine stagnation ends the inner solve.
  const int stall_window = sizeof(T) == 4 ? 4000 : 30000;
  for (;;) {
    if (use_graph) {
      hipError_t he = hipGraphLaunch(gexec, c.s);
      if (he != hipSuccess) {
        ret = hip_fail(he, "hipGraphLaunch");
        break;
      }
    } else {
      for (int k = 0; k < check_every; ++k)
        if ((ret = one_iter(k & 1)) != FIT_OK) break;
      if (ret != FIT_OK) break;
    }
    if ((ret = sync_copy(c, c.h_cst, c.cst, sizeof(CgState))) != FIT_OK) break;
    c.bytes += per_iter_bytes * (c.h_cst->iter - last_iter);
    c.matvecs += c.h_cst->iter - last_iter;
    last_iter = c.h_cst->iter;
    if (c.h_cst->done != kRunning) break;
    if constexpr (sizeof(T) == 8) {
      // an iterate of the solve for the pair harvest (with the fused path x
      // lags one step: still an iterate of the same Krylov sequence)
      if (c.snap && c.snap_active && c.snap_n < c.snap_cap &&
          c.h_cst->iter >= (c.snap_n + 1) * c.snap_stride) {
        if ((ret = xform<T, double, XF_SCALE>(c, false, false, V.x, c.snap + c.snap_n * c.snap_ld,
                                              c.inner_eta, false)) != FIT_OK)
          break;
        ++c.snap_n;
      }
    }
    if (c.h_cst->rr < 0.25 * best_rr) {
      best_rr = c.h_cst->rr;
      best_at = c.h_cst->iter;
    } else if (c.h_cst->iter - best_at >= stall_window) {
      stalled = true;
      break;
    }
  }
  if (gexec) (void)hipGraphExecDestroy(gexec);
  if (graph) (void)hipGraphDestroy(graph);
  if (ret != FIT_OK) return ret;
  if (pre) {
    hipLaunchKernelGGL(cocg_fixup_kernel<T>, dim3((unsigned)nbn), dim3(256), 0, c.s, ne, V.x,
                       V.p[0], V.p[1], c.cst);
    FIT_HIP(hipGetLastError());
  }
  *done = stalled ? kBreakdown : c.h_cst->done;
  *iters = c.h_cst->iter;
  c.last_reason = stalled ? 9 : c.h_cst->reason;
  c.last_rr = c.h_cst->rr / r0;
  return FIT_OK;
}

// Host side of an iteration whose scalars live in device state S (fields
// iter, done, rr): replay check_every iterations (a captured graph or eager
// launches), read the state, count bytes and operator applications, and stop
// on a stop code or when the residual estimate has not fallen to a quarter
// within stall_window iterations (reported as a stall through *stalled).
template <class S, class F>
static fit_status poll_iterations(Ctx& c, F&& one_iter, int check_every, int use_graph, S* st_dev,
                                  S* st_host, double per_iter_bytes, int mv_per_iter,
                                  int stall_window, bool* stalled) {
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  if (use_graph) {
    hipStream_t cap = nullptr;
    FIT_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    const hipStream_t user = c.s;
    c.s = cap;
    hipError_t he = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    fit_status e = he == hipSuccess ? FIT_OK : hip_fail(he, "hipStreamBeginCapture");
    for (int k = 0; k < check_every && e == FIT_OK; ++k) e = one_iter();
    if (he == hipSuccess) he = hipStreamEndCapture(cap, &graph);
    c.s = user;
    (void)hipStreamDestroy(cap);
    if (e != FIT_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return e;
    }
    if (he != hipSuccess) return hip_fail(he, "hipStreamEndCapture");
    he = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
    if (he != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return hip_fail(he, "hipGraphInstantiate");
    }
  }
  int last_iter = 0, best_at = 0;
  double best_rr = -1.0;
  fit_status ret = FIT_OK;
  *stalled = false;
  for (;;) {
    if (use_graph) {
      const hipError_t he = hipGraphLaunch(gexec, c.s);
      if (he != hipSuccess) {
        ret = hip_fail(he, "hipGraphLaunch");
        break;
      }
    } else {
      for (int k = 0; k < check_every && ret == FIT_OK; ++k) ret = one_iter();
      if (ret != FIT_OK) break;
    }
    if ((ret = sync_copy(c, st_host, st_dev, sizeof(S))) != FIT_OK) break;
    c.bytes += per_iter_bytes * (st_host->iter - last_iter);
    c.matvecs += mv_per_iter * (st_host->iter - last_iter);
    last_iter = st_host->iter;
    if (st_host->done != kRunning) break;
    if (best_rr < 0.0 || st_host->rr < 0.25 * best_rr) {
      best_rr = st_host->rr;
      best_at = st_host->iter;
    } else if (st_host->iter - best_at >= stall_window) {
      *stalled = true;
      break;
    }
  }
  if (gexec) (void)hipGraphExecDestroy(gexec);
  if (graph) (void)hipGraphDestroy(graph);
  return ret;
}

// COCR (the paper's CR in complex symmetric form) on A_int x = r, from
// x = 0; r is overwritten.

template <class T>
static fit_status cocr(Ctx& c, CrVecs<T>& V, double tol_rel, int max_iter, int check_every,
                       double hscale, double* hist_dev, int hist_len, int use_graph, int* done,
                       int* iters) {
  const int64_t ne = c.g->ne;
  const int64_t nb = pw_blocks(ne);
  fit_status st;
  if ((st = vzero(c, V.x, ne)) != FIT_OK) return st;
  if ((st = vzero(c, V.p, ne)) != FIT_OK) return st;
  if ((st = vzero(c, V.q, ne)) != FIT_OK) return st;
  hipLaunchKernelGGL((dot_kernel<T, true>), dim3((unsigned)nb), dim3(256), 0, c.s, V.r, V.r, ne,
                     c.red, c.part, c.cnt);
  FIT_HIP(hipGetLastError());
  FIT_HIP(launch_finish<4>(c.part, (int)nb, StoreSums<4>{c.red}, c.s));
  if ((st = sync_copy(c, c.h_red, c.red, sizeof(RedOut))) != FIT_OK) return st;
  const double r0 = c.h_red->v[2];
  *iters = 0;
  if (!(r0 > 0.0) || !std::isfinite(r0)) {
    *done = r0 == 0.0 ? kConverged : kNan;
    return FIT_OK;
  }
  CgState h{};
  h.rr = r0;
  h.tol2 = tol_rel * tol_rel * r0;
  h.hscale = hscale / std::sqrt(r0);
  h.max_iter = max_iter;
  h.done = kRunning;
  h.hist = hist_dev;
  h.hist_len = hist_len;
  FIT_HIP(hipMemcpyAsync(c.cst, &h, sizeof(CgState), hipMemcpyHostToDevice, c.s));
  // w = A r, rho = r^T w
  OpCocrW<T> k0{V.r, V.w, c.cst, c.part, c.cnt, 1};
  if ((st = launch_op_stencil_mode<T>(c, c.sym, k0)) != FIT_OK) return st;
  auto one_iter = [&]() -> fit_status {
    const int tok = prof_begin(c.s);
    hipLaunchKernelGGL(cocr_pq_kernel<T>, dim3((unsigned)nb), dim3(256), 0, c.s, ne, V.r, V.w, V.p,
                       V.q, c.cst, c.part);
    FIT_HIP(hipGetLastError());
    FIT_HIP(launch_finish<2>(c.part, (int)nb, CocrAlphaFinish{c.cst}, c.s));
    hipLaunchKernelGGL(cocr_xr_kernel<T>, dim3((unsigned)nb), dim3(256), 0, c.s, ne, V.x, V.r, V.p,
                       V.q, c.cst, c.part);
    FIT_HIP(hipGetLastError());
    FIT_HIP(launch_finish<1>(c.part, (int)nb, CocrResFinish{c.cst}, c.s));
    prof_end(tok, c.s, sizeof(T) == 8 ? "cocr_update_c128" : "cocr_update_c64");
    OpCocrW<T> k1{V.r, V.w, c.cst, c.part, c.cnt, 0};
    return launch_op_stencil_mode<T>(c, c.sym, k1);
  };
  // operator 2 passes, p/q update 6, x/r update 6
  const double per_iter_bytes = node_bytes(c.g, 14, sizeof(T));
  if (check_every <= 0) check_every = 2 * std::max(1, std::min(100, (int)(4e8 / (double)ne)));
  bool stalled = false;
  const int stall_window = sizeof(T) == 4 ? 4000 : 30000;
  if ((st = poll_iterations(c, one_iter, check_every, use_graph, c.cst, c.h_cst, per_iter_bytes, 1,
                            stall_window, &stalled)) != FIT_OK)
    return st;
  *done = stalled ? kBreakdown : c.h_cst->done;
  *iters = c.h_cst->iter;
  c.last_reason = stalled ? 9 : c.h_cst->reason;
  c.last_rr = c.h_cst->rr / r0;
  return FIT_OK;
}

// TFQMR on A_int x = r0v from x = 0.

template <class T>
static fit_status tfqmr(Ctx& c, TqVecs<T>& V, const T* r0v, double tol_rel, int max_iter,
                        int check_every, double hscale, double* hist_dev, int hist_len,
                        int use_graph, uint64_t shadow_seed, int* done, int* iters) {
  const int64_t ne = c.g->ne;
  const int64_t nb = pw_blocks(ne);
  fit_status st;
  if ((st = vzero(c, V.x, ne)) != FIT_OK) return st;
  if ((st = vzero(c, V.d, ne)) != FIT_OK) return st;
  if ((st = vcopy(c, r0v, V.w, ne)) != FIT_OK) return st;
  if ((st = vcopy(c, r0v, V.u0, ne)) != FIT_OK) return st;
  // dense pseudo-random shadow vector (as for BiCGStab), rho = <rh, r0>
  if ((st = xform<T, T, XF_SHADOW>(c, false, false, V.w, V.rh, 1.0, false, shadow_seed)) != FIT_OK)
    return st;
  hipLaunchKernelGGL(dot_kernel<T>, dim3((unsigned)nb), dim3(256), 0, c.s, V.rh, V.w, ne, c.red,
                     c.part, c.cnt);
  FIT_HIP(hipGetLastError());
  FIT_HIP(launch_finish<4>(c.part, (int)nb, StoreSums<4>{c.red}, c.s));
  if ((st = sync_copy(c, c.h_red, c.red, sizeof(RedOut))) != FIT_OK) return st;
  const double r0 = c.h_red->v[3];
  *iters = 0;
  if (!(r0 > 0.0) || !std::isfinite(r0)) {
    *done = r0 == 0.0 ? kConverged : kNan;
    return FIT_OK;
  }
  TqState h{};
  h.rho = cx<double>{c.h_red->v[0], c.h_red->v[1]};
  h.tau = std::sqrt(r0);
  h.rr = r0;
  h.tol2 = tol_rel * tol_rel * r0;
  h.hscale = hscale / std::sqrt(r0);
  h.max_iter = max_iter;
  h.done = kRunning;
  h.hist = hist_dev;
  h.hist_len = hist_len;
  FIT_HIP(hipMemcpyAsync(c.tst, &h, sizeof(TqState), hipMemcpyHostToDevice, c.s));
  const int* dflag = &c.tst->done;
  {  // v = A u0, kept as A u0 too
    OpMatvecIf<T> mv{V.u0, V.au0, dflag};
    if ((st = launch_op_stencil_mode<T>(c, c.sym, mv)) != FIT_OK) return st;
    if ((st = vcopy(c, V.au0, V.v, ne)) != FIT_OK) return st;
  }
  auto one_iter = [&]() -> fit_status {
    fit_status e;
    const int tok = prof_begin(c.s);
    // even half-step: alpha = rho / <rh, v>; u1 = u0 - alpha v; w -= alpha A u0
    hipLaunchKernelGGL(tq_dot_kernel<T>, dim3((unsigned)nb), dim3(256), 0, c.s, ne, V.rh, V.v,
                       c.tst, c.part);
    FIT_HIP(hipGetLastError());
    FIT_HIP(launch_finish<2>(c.part, (int)nb, TqAlphaFinish{c.tst}, c.s));
    hipLaunchKernelGGL((tq_half_kernel<T, true>), dim3((unsigned)nb), dim3(256), 0, c.s, ne, V.u0,
                       V.u1, V.v, V.w, V.au0, V.d, c.tst, c.part);
    FIT_HIP(hipGetLastError());
    FIT_HIP(launch_finish<1>(c.part, (int)nb, TqStepFinish{c.tst}, c.s));
    hipLaunchKernelGGL((tq_x_kernel<T, false>), dim3((unsigned)nb), dim3(256), 0, c.s, ne, V.x,
                       V.d, V.rh, V.w, c.tst, c.part);
    FIT_HIP(hipGetLastError());
    prof_end(tok, c.s, sizeof(T) == 8 ? "tfqmr_update_c128" : "tfqmr_update_c64");
    // odd half-step: w -= alpha A u1, x update, rho' = <rh, w>, beta
    OpMatvecIf<T> m1{V.u1, V.au1, dflag};
    if ((e = launch_op_stencil_mode<T>(c, c.sym, m1)) != FIT_OK) return e;
    hipLaunchKernelGGL((tq_half_kernel<T, false>), dim3((unsigned)nb), dim3(256), 0, c.s, ne, V.u1,
                       V.u1, V.v, V.w, V.au1, V.d, c.tst, c.part);
    FIT_HIP(hipGetLastError());
    FIT_HIP(launch_finish<1>(c.part, (int)nb, TqStepFinish{c.tst}, c.s));
    hipLaunchKernelGGL((tq_x_kernel<T, true>), dim3((unsigned)nb), dim3(256), 0, c.s, ne, V.x, V.d,
                       V.rh, V.w, c.tst, c.part);
    FIT_HIP(hipGetLastError());
    FIT_HIP(launch_finish<2>(c.part, (int)nb, TqRhoFinish{c.tst}, c.s));
    // next u0 = w + beta u1, its product, and v = A u0 + beta (A u1 + beta v)
    hipLaunchKernelGGL(tq_u_kernel<T>, dim3((unsigned)nb), dim3(256), 0, c.s, ne, V.u0, V.w, V.u1,
                       c.tst);
    FIT_HIP(hipGetLastError());
    OpMatvecIf<T> m0{V.u0, V.au0, dflag};
    if ((e = launch_op_stencil_mode<T>(c, c.sym, m0)) != FIT_OK) return e;
    hipLaunchKernelGGL(tq_v_kernel<T>, dim3((unsigned)nb), dim3(256), 0, c.s, ne, V.v, V.au0,
                       V.au1, c.tst);
    FIT_HIP(hipGetLastError());
    return FIT_OK;
  };
  // two operator applications (4 passes) and about 27 vector passes
  const double per_iter_bytes = node_bytes(c.g, 31, sizeof(T));
  if (check_every <= 0) check_every = 2 * std::max(1, std::min(50, (int)(2e8 / (double)ne)));
  bool stalled = false;
  const int stall_window = sizeof(T) == 4 ? 1500 : 6000;
  if ((st = poll_iterations(c, one_iter, check_every, use_graph, c.tst, c.h_tst, per_iter_bytes, 2,
                            stall_window, &stalled)) != FIT_OK)
    return st;
  *done = stalled ? kBreakdown : c.h_tst->done;
  *iters = c.h_tst->iter;
  c.last_reason = stalled ? 9 : c.h_tst->reason;
  c.last_rr = c.h_tst->rr / r0;
  return FIT_OK;
}

// CGS on A_int x = r0v from x = 0.
template <class T>
static fit_status cgs(Ctx& c, CgsVecs<T>& V, const T* r0v, double tol_rel, int max_iter,
                      int check_every, double hscale, double* hist_dev, int hist_len,
                      int use_graph, uint64_t shadow_seed, int* done, int* iters) {
  const int64_t ne = c.g->ne;
  const int64_t nb = pw_blocks(ne);
  fit_status st;
  if ((st = vzero(c, V.x, ne)) != FIT_OK) return st;
  if ((st = vzero(c, V.p, ne)) != FIT_OK) return st;
  if ((st = vzero(c, V.q, ne)) != FIT_OK) return st;
  if ((st = vcopy(c, r0v, V.r, ne)) != FIT_OK) return st;
  if ((st = xform<T, T, XF_SHADOW>(c, false, false, V.r, V.rh, 1.0, false, shadow_seed)) != FIT_OK)
    return st;
  hipLaunchKernelGGL(dot_kernel<T>, dim3((unsigned)nb), dim3(256), 0, c.s, V.rh, V.r, ne, c.red,
                     c.part, c.cnt);
  FIT_HIP(hipGetLastError());
  FIT_HIP(launch_finish<4>(c.part, (int)nb, StoreSums<4>{c.red}, c.s));
  if ((st = sync_copy(c, c.h_red, c.red, sizeof(RedOut))) != FIT_OK) return st;
  const double r0 = c.h_red->v[3];
  *iters = 0;
  if (!(r0 > 0.0) || !std::isfinite(r0)) {
    *done = r0 == 0.0 ? kConverged : kNan;
    return FIT_OK;
  }
  TqState h{};
  h.rho = cx<double>{c.h_red->v[0], c.h_red->v[1]};
  h.beta = cx<double>{0.0, 0.0};
  h.rr = r0;
  h.tol2 = tol_rel * tol_rel * r0;
  h.hscale = hscale / std::sqrt(r0);
  h.max_iter = max_iter;
  h.done = kRunning;
  h.hist = hist_dev;
  h.hist_len = hist_len;
  FIT_HIP(hipMemcpyAsync(c.tst, &h, sizeof(TqState), hipMemcpyHostToDevice, c.s));
  const int* dflag = &c.tst->done;
  auto one_iter = [&]() -> fit_status {
    fit_status e;
    const int tok = prof_begin(c.s);
    hipLaunchKernelGGL(cgs_up_kernel<T>, dim3((unsigned)nb), dim3(256), 0, c.s, ne, V.r, V.u, V.p,
                       V.q, c.tst);
    FIT_HIP(hipGetLastError());
    prof_end(tok, c.s, sizeof(T) == 8 ? "cgs_update_c128" : "cgs_update_c64");
    OpMatvecIf<T> m1{V.p, V.v, dflag};
    if ((e = launch_op_stencil_mode<T>(c, c.sym, m1)) != FIT_OK) return e;
    hipLaunchKernelGGL(tq_dot_kernel<T>, dim3((unsigned)nb), dim3(256), 0, c.s, ne, V.rh, V.v,
                       c.tst, c.part);
    FIT_HIP(hipGetLastError());
    FIT_HIP(launch_finish<2>(c.part, (int)nb, TqAlphaFinish{c.tst}, c.s));
    hipLaunchKernelGGL(cgs_qw_kernel<T>, dim3((unsigned)nb), dim3(256), 0, c.s, ne, V.u, V.q, V.v,
                       c.tst);
    FIT_HIP(hipGetLastError());
    OpMatvecIf<T> m2{V.u, V.v, dflag};  // A w into v (v is free again)
    if ((e = launch_op_stencil_mode<T>(c, c.sym, m2)) != FIT_OK) return e;
    hipLaunchKernelGGL(cgs_xr_kernel<T>, dim3((unsigned)nb), dim3(256), 0, c.s, ne, V.x, V.r, V.u,
                       V.v, V.rh, c.tst, c.part);
    FIT_HIP(hipGetLastError());
    FIT_HIP(launch_finish<3>(c.part, (int)nb, CgsFinish{c.tst}, c.s));
    return FIT_OK;
  };
  // two operator applications (4 passes) and about 18 vector passes
  const double per_iter_bytes = node_bytes(c.g, 22, sizeof(T));
  if (check_every <= 0) check_every = 2 * std::max(1, std::min(50, (int)(2e8 / (double)ne)));
  bool stalled = false;
  const int stall_window = sizeof(T) == 4 ? 1500 : 6000;
  if ((st = poll_iterations(c, one_iter, check_every, use_graph, c.tst, c.h_tst, per_iter_bytes, 2,
                            stall_window, &stalled)) != FIT_OK)
    return st;
  *done = stalled ? kBreakdown : c.h_tst->done;
  *iters = c.h_tst->iter;
  c.last_reason = stalled ? 9 : c.h_tst->reason;
  c.last_rr = c.h_tst->rr / r0;
  return FIT_OK;
}

template <class T>
static size_t inner_bytes(int64_t ne, int solver, int m) {
  const size_t v = align_up((size_t)ne * 2 * sizeof(T), 256);
  if (solver == FIT_BICGSTAB) return 11 * v;
  if (solver == FIT_COCG) return 8 * v;
  if (solver == FIT_COCR) return 6 * v;
  if (solver == FIT_TFQMR) return 10 * v;
  if (solver == FIT_CGS) return 8 * v;
  const int nblk = (int)((ne + 256 * kMdPer - 1) / (256 * kMdPer));
  return (size_t)(2 * m + 5) * v + align_up(sizeof(double) * 2 * (size_t)(m + 1) * nblk, 256);
}

template <class T>
static void inner_carve(Arena& a, Inner<T>& in, int64_t ne, int solver, int m) {
  const size_t v = (size_t)ne * 2 * sizeof(T);
  in.solver = solver;
  in.m = m;
  in.rin = a.take<T>(v);
  if (solver == FIT_BICGSTAB) {
    in.bv.x = a.take<T>(v);
    in.bv.r = a.take<T>(v);
    in.bv.rh = a.take<T>(v);
    in.bv.p[0] = a.take<T>(v);
    in.bv.p[1] = a.take<T>(v);
    in.bv.v[0] = a.take<T>(v);
    in.bv.v[1] = a.take<T>(v);
    in.bv.s = a.take<T>(v);
    in.bv.t = a.take<T>(v);
    in.bv.xb = a.take<T>(v);
    in.d = in.bv.x;
  } else if (solver == FIT_COCG) {
    in.bv.x = a.take<T>(v);
    in.bv.r = a.take<T>(v);
    in.bv.p[0] = a.take<T>(v);
    in.bv.p[1] = a.take<T>(v);
    in.bv.v[0] = a.take<T>(v);
    in.bv.s = a.take<T>(v);  // z = M r of the mass-preconditioned form
    in.bv.t = a.take<T>(v);  // the diagonal M
    in.bv.rh = in.bv.v[1] = nullptr;
    in.d = in.bv.x;
    in.own_scaling = true;
  } else if (solver == FIT_COCR) {
    in.cr.x = a.take<T>(v);
    in.cr.r = a.take<T>(v);
    in.cr.p = a.take<T>(v);
    in.cr.q = a.take<T>(v);
    in.cr.w = a.take<T>(v);
    in.d = in.cr.x;
  } else if (solver == FIT_TFQMR) {
    in.tq.x = a.take<T>(v);
    in.tq.w = a.take<T>(v);
    in.tq.u0 = a.take<T>(v);
    in.tq.u1 = a.take<T>(v);
    in.tq.au0 = a.take<T>(v);
    in.tq.au1 = a.take<T>(v);
    in.tq.v = a.take<T>(v);
    in.tq.d = a.take<T>(v);
    in.tq.rh = a.take<T>(v);
    in.d = in.tq.x;
  } else if (solver == FIT_CGS) {
    in.cg.x = a.take<T>(v);
    in.cg.r = a.take<T>(v);
    in.cg.rh = a.take<T>(v);
    in.cg.u = a.take<T>(v);
    in.cg.p = a.take<T>(v);
    in.cg.q = a.take<T>(v);
    in.cg.v = a.take<T>(v);
    in.d = in.cg.x;
  } else {
    const size_t vv = align_up(v, 256);
    in.gv.ldv = (int64_t)(vv / (2 * sizeof(T)));
    in.gv.x = a.take<T>(v);
    in.gv.V = a.take<T>(vv * (m + 1));
    in.gv.Z = solver == FIT_FGMRES ? a.take<T>(vv * m) : nullptr;
    in.gv.W[0] = a.take<T>(v);
    in.gv.W[1] = a.take<T>(v);
    const int nblk = (int)((ne + 256 * kMdPer - 1) / (256 * kMdPer));
    in.gv.mdpart = a.take<double>(sizeof(double) * 2 * (size_t)(m + 1) * nblk);
    in.d = in.gv.x;
  }
}

template <class T>
static fit_status run_inner(Ctx& c, Inner<T>& in, double q, int max_iter, int check_every,
                            double hscale, double* hist, int hist_len, int use_graph,
                            PrecondApply* pre, int* done, int* iters) {
  double tmp = 0.0;
  if (in.solver == FIT_BICGSTAB) {
    fit_status st = vcopy<T>(c, in.rin, in.bv.r, c.g->ne);
    if (st != FIT_OK) return st;
    const uint64_t seed = kShadowSeed + (uint64_t)in.restarts++;
    return bicgstab<T>(c, in.bv, q, max_iter, check_every, hscale, hist, hist_len, use_graph,
                       seed, done, iters, &tmp);
  }
  if (in.solver == FIT_COCG) {
    fit_status st = vcopy<T>(c, in.rin, in.bv.r, c.g->ne);
    if (st != FIT_OK) return st;
    return cocg<T>(c, in.bv, q, max_iter, check_every, hscale, hist, hist_len, use_graph, done,
                   iters);
  }
  if (in.solver == FIT_COCR) {
    fit_status st = vcopy<T>(c, in.rin, in.cr.r, c.g->ne);
    if (st != FIT_OK) return st;
    return cocr<T>(c, in.cr, q, max_iter, check_every, hscale, hist, hist_len, use_graph, done,
                   iters);
  }
  if (in.solver == FIT_TFQMR) {
    const uint64_t seed = kShadowSeed + (uint64_t)in.restarts++;
    return tfqmr<T>(c, in.tq, in.rin, q, max_iter, check_every, hscale, hist, hist_len, use_graph,
                    seed, done, iters);
  }
  if (in.solver == FIT_CGS) {
    const uint64_t seed = kShadowSeed + (uint64_t)in.restarts++;
    return cgs<T>(c, in.cg, in.rin, q, max_iter, check_every, hscale, hist, hist_len, use_graph,
                  seed, done, iters);
  }
  return gmres<T>(c, in.gv, in.m, q, max_iter, hscale, hist, hist_len, pre, in.rin, nullptr,
                  done, iters, &tmp, 0.0);
}

}  // namespace fit

using namespace fit;

namespace {

// FIT_VERBOSE=1 in the environment prints one line per refinement step.
bool verbose() {
  static const bool v = [] {
    const char* e = std::getenv("FIT_VERBOSE");
    return e && *e && *e != '0';
  }();
  return v;
}

// Outer loop shared by both precisions: x += ||r|| S d with d from an inner
// solve on the scaled, normalised residual; stop on the true residual.
template <class T>
fit_status refine(Ctx& c, Inner<T>& in, const double* b, double bnorm, double* x, double* r,
                  const double* r_init, double rnorm_init, double tol, const fit_solve_opts& o,
                  double inner_tol, PrecondApply* pre, double* hist, fit_solve_info& info,
                  double* relres_out, int* total_iters) {
  const int64_t ne = c.g->ne;
  fit_status st;
  double rnorm = rnorm_init;  // residual of the incoming x
  const double* rcur = r_init;
  int iters = 0, refin = 0, stall = 0, breakdowns = 0;
  double best = 1.0;
  fit_status result = FIT_E_NOT_CONVERGED;
  // BiCGStab restarts with a fresh shadow vector until the iteration budget
  // is spent: a correction that does not lower the true residual is undone
  // and the next inner solve starts again from the best iterate.  Only a
  // long run of inner solves without halving the residual ends it early.
  const bool retry = in.solver == FIT_BICGSTAB || in.solver == FIT_TFQMR || in.solver == FIT_CGS;
  const int max_no_progress = retry ? (sizeof(T) == 4 ? 6 : 64) : 4;
  for (;;) {
    // inner rhs: S r scaled to unit norm, in precision T (S r = eta * rin)
    if ((st = xform<double, T, XF_SCALE>(c, c.sym && !in.own_scaling, false, rcur, in.rin, 1.0 / rnorm, true)) != FIT_OK)
      return st;
    if ((st = sync_copy(c, c.h_red, c.red, sizeof(RedOut))) != FIT_OK) return st;
    const double eta = rnorm * std::sqrt(c.h_red->v[0]);
    if (!(eta > 0.0) || !std::isfinite(eta)) {
      result = FIT_E_NAN;
      break;
    }
    if ((st = xform<T, T, XF_SCALE>(c, false, false, in.rin, in.rin, rnorm / eta, false)) != FIT_OK)
      return st;
    const double rel = rnorm / bnorm;
    double q = 0.5 * tol / rel;
    if (sizeof(T) == 4) q = std::max(q, inner_tol);
    q = std::min(q, 0.5);
    int done = 0, it = 0;
    const int budget = o.max_iters - iters;
    if (budget <= 0) break;
    c.inner_eta = eta;
    c.snap_active = refin == 0 && rcur == r_init;
    const int hoff = std::min(iters, o.resid_history_len);
    if ((st = run_inner<T>(c, in, q, budget, o.check_every, rel, hist ? hist + hoff : nullptr,
                           o.resid_history_len - hoff, o.use_graph, pre, &done, &it)) != FIT_OK)
      return st;
    iters += it;
    ++refin;
    if (done == kNan) {
      result = FIT_E_NAN;
      break;
    }
    // x += eta S d
    if ((st = xform<T, double, XF_AXPY>(c, c.sym && !in.own_scaling, false, in.d, x, eta, false)) != FIT_OK) return st;
    // true residual
    if ((st = residual(c, x, b, r, nullptr, 0.0)) != FIT_OK) return st;
    if ((st = sync_copy(c, c.h_red, c.red, sizeof(RedOut))) != FIT_OK) return st;
    double rn = std::sqrt(c.h_red->v[0]);
    if (verbose()) {
      std::fprintf(stderr,
                   "[fit] refinement %d (%s): inner exit %d (reason %d, inner relres %.2e) after "
                   "%d it (target %.1e), true relres %.3e\n",
                   refin, sizeof(T) == 4 ? "c64" : "c128", done, c.last_reason,
                   std::sqrt(c.last_rr), it, q, rn / bnorm);
    }
    if (!std::isfinite(rn) || rn > rnorm) {
      // The correction made things worse (an inner solve that broke down
      // early): undo it.  BiCGStab tries again with a new shadow vector;
      // the other methods would repeat the same iteration, so this
      // precision's refinement stops.
      if ((st = xform<T, double, XF_AXPY>(c, c.sym && !in.own_scaling, false, in.d, x, -eta, false)) != FIT_OK) return st;
      if ((st = residual(c, x, b, r, nullptr, 0.0)) != FIT_OK) return st;
      if ((st = sync_copy(c, c.h_red, c.red, sizeof(RedOut))) != FIT_OK) return st;
      rn = std::sqrt(c.h_red->v[0]);
      *relres_out = rn / bnorm;
      const bool budget_left = done != kMaxIter && iters < o.max_iters;
      if (std::isfinite(rn) && retry && budget_left && ++stall < max_no_progress) {
        rcur = r;
        rnorm = rn;
        continue;
      }
      if (!std::isfinite(rn))
        result = FIT_E_NAN;
      else if (!budget_left)
        result = FIT_E_NOT_CONVERGED;
      else
        result = FIT_E_BREAKDOWN;
      break;
    }
    rcur = r;
    *relres_out = rn / bnorm;
    if (rn <= tol * bnorm) {
      result = FIT_OK;
      rnorm = rn;
      break;
    }
    if (done == kBreakdown && c.gm_stall_cycles > 0) {
      result = FIT_E_BREAKDOWN;  // the learned preconditioner stalled: fall back
      rnorm = rn;
      break;
    }
    if (done == kBreakdown && in.solver == FIT_BICGSTAB) ++breakdowns;
    if (rn / bnorm < 0.5 * best) {
      best = rn / bnorm;
      stall = 0;
      breakdowns = 0;
    } else {
      ++stall;
    }
    rnorm = rn;
    if (done == kMaxIter || iters >= o.max_iters) {
      result = FIT_E_NOT_CONVERGED;
      break;
    }
    if (!retry && breakdowns >= 5) {
      result = FIT_E_BREAKDOWN;
      break;
    }
    if (stall >= max_no_progress) {
      result = retry ? FIT_E_BREAKDOWN : FIT_E_NOT_CONVERGED;
      break;
    }
  }
  info.refinements += refin;
  *total_iters = iters;
  (void)ne;
  return result;
}

}  // namespace

namespace fit {
// Iterates kept by a solve for the pair harvest (see Ctx::snap).
struct SnapRequest {
  double* buf;
  int64_t ld;
  int cap, stride;
  int made = 0;
};
}  // namespace fit

namespace {
fit_status solve_impl(fit_grid* g, double omega, const void* source_dev, double tol,
                      const fit_solve_opts* opts, void* x_dev, fit_solve_info* info,
                      SnapRequest* snap);
}  // namespace

extern "C" fit_status fit_solve(fit_grid* g, double omega, const void* source_dev, double tol,
                                const fit_solve_opts* opts, void* x_dev, fit_solve_info* info) {
  return solve_impl(g, omega, source_dev, tol, opts, x_dev, info, nullptr);
}

namespace {
fit_status solve_impl(fit_grid* g, double omega, const void* source_dev, double tol,
                      const fit_solve_opts* opts, void* x_dev, fit_solve_info* info,
                      SnapRequest* snap) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!g || !source_dev || !x_dev) {
    set_error("fit_solve: NULL argument");
    return FIT_E_INVALID;
  }
  if (!(omega > 0.0) || !std::isfinite(omega)) {
    set_error("fit_solve: omega must be finite and > 0");
    return FIT_E_INVALID;
  }
  if (!(tol > 0.0) || !(tol < 1.0)) {
    set_error("fit_solve: tol must be in (0, 1)");
    return FIT_E_INVALID;
  }
  fit_solve_opts o{};
  if (opts) o = *opts;
  if (o.restart == 0) o.restart = 30;
  if (o.max_iters <= 0) o.max_iters = 100000;
  if (o.solver < FIT_BICGSTAB || o.solver > FIT_CGS || o.restart < 1 ||
      o.restart > kMaxRestart || (o.precision != FIT_PREC_FP64 && o.precision != FIT_PREC_MIXED) ||
      (o.scaling != FIT_SCALE_NONE && o.scaling != FIT_SCALE_SYM) || o.resid_history_len < 0 ||
      (o.resid_history_len > 0 && !o.resid_history) || o.diag < FIT_DIAG_AUTO ||
      o.diag > FIT_DIAG_JACOBI) {
    set_error("fit_solve: invalid options");
    return FIT_E_INVALID;
  }
  if (o.diag != FIT_DIAG_AUTO && o.solver != FIT_COCG) {
    set_error("fit_solve: a stored diagonal preconditioner (opts.diag) is implemented for FIT_COCG only");
    return FIT_E_UNSUPPORTED;
  }
  if (o.inner_tol <= 0.0) o.inner_tol = 1e-4;
  DeviceScope dev(g->device);
  hipStream_t s = (hipStream_t)o.stream;
  Ctx c;
  fit_status st = setup_ctx(c, g, omega, o.scaling == FIT_SCALE_SYM, s);
  if (st != FIT_OK) return st;
  c.diag = o.diag;
  if (snap) {
    c.snap = snap->buf;
    c.snap_ld = snap->ld;
    c.snap_cap = snap->cap;
    c.snap_stride = std::max(1, snap->stride);
  }
  const bool learned = o.solver == FIT_FGMRES && o.precond != nullptr;
  if (learned) c.gm_stall_cycles = 10;

  const int64_t ne = g->ne;
  const size_t v128 = align_up((size_t)ne * 16, 256);
  const bool mixed = o.precision == FIT_PREC_MIXED;
  // The mixed form reserves room for a complex128 inner solve as well, so a
  // fallback carves the same arena (b, r and the residual history stay put).
  size_t in_bytes = mixed ? std::max(inner_bytes<float>(ne, o.solver, o.restart),
                                     inner_bytes<double>(ne, o.solver, o.restart))
                          : inner_bytes<double>(ne, o.solver, o.restart);
  // a learned FGMRES preconditioner can fall back to COCG in the same arena
  if (learned) in_bytes = std::max(in_bytes, inner_bytes<double>(ne, FIT_COCG, o.restart));
  const size_t hist_bytes = align_up(sizeof(double) * (size_t)std::max(o.resid_history_len, 1), 256);
  if ((st = ensure_ws(g->ws, 2 * v128 + in_bytes + hist_bytes + 4096, g->device)) != FIT_OK) return st;
  Arena a{(char*)g->ws.ptr, 0, g->ws.bytes};
  double* b = a.take<double>(v128);
  double* r = a.take<double>(v128);
  double* hist = o.resid_history_len > 0 ? a.take<double>(hist_bytes) : nullptr;
  double* x = (double*)x_dev;

  // b = -j omega j, ||b||^2, masked-source check
  FIT_HIP(hipMemsetAsync(c.red, 0, sizeof(RedOut), s));
  if ((st = xform<double, double, XF_RHS>(c, false, false, (const double*)source_dev, b, 1.0, true)) != FIT_OK)
    return st;
  if ((st = sync_copy(c, c.h_red, c.red, sizeof(RedOut))) != FIT_OK) return st;
  if (c.h_red->flag) {
    set_error("fit_solve: nonzero source on a masked edge");
    return FIT_E_INVALID;
  }
  const double bnorm = std::sqrt(c.h_red->v[0]);
  if ((st = vzero<double>(c, x, ne)) != FIT_OK) return st;
  fit_solve_info inf{};
  double relres = 1.0;
  int iters = 0;
  fit_status result;
  IdentityPrecond ident;
  PrecondApply* pre = nullptr;
  if (o.solver == FIT_FGMRES) {
    pre = &ident;
    if (o.precond) {
      pre = precond_apply_of(o.precond, g, omega);
      if (!pre) {
        set_error("fit_solve: the preconditioner cannot serve this grid (device mismatch or no memory)");
        return FIT_E_INVALID;
      }
    }
  }
  if (!std::isfinite(bnorm)) {
    result = FIT_E_NAN;
  } else if (bnorm == 0.0) {
    result = FIT_OK;
    relres = 0.0;
  } else if (mixed) {
    Inner<float> in;
    inner_carve<float>(a, in, ne, o.solver, o.restart);
    result = refine<float>(c, in, b, bnorm, x, r, b, bnorm, tol, o, o.inner_tol, pre, hist, inf,
                           &relres, &iters);
    if ((result == FIT_E_NOT_CONVERGED || result == FIT_E_BREAKDOWN || result == FIT_E_NAN) &&
        iters < o.max_iters) {
      // complex64 stagnated: continue in complex128 from the current x, in
      // the same arena (sized for it above): b, r and the history are kept
      inf.fell_back = 1;
      Arena a2{(char*)g->ws.ptr, 0, g->ws.bytes};
      (void)a2.take<double>(v128);
      (void)a2.take<double>(v128);
      if (hist) (void)a2.take<double>(hist_bytes);
      Inner<double> in2;
      inner_carve<double>(a2, in2, ne, o.solver, o.restart);
      fit_solve_opts o2 = o;
      o2.max_iters = o.max_iters - iters;
      const int hoff = std::min(iters, o.resid_history_len);
      o2.resid_history_len = o.resid_history_len - hoff;
      double* hist2 = (hist && o2.resid_history_len > 0) ? hist + hoff : nullptr;
      int it2 = 0;
      if ((st = residual(c, x, b, r, nullptr, 0.0)) != FIT_OK) return st;
      if ((st = sync_copy(c, c.h_red, c.red, sizeof(RedOut))) != FIT_OK) return st;
      result = refine<double>(c, in2, b, bnorm, x, r, r, std::sqrt(c.h_red->v[0]), tol, o2,
                              o.inner_tol, pre, hist2, inf, &relres, &it2);
      iters += it2;
    }
  } else {
    Inner<double> in;
    inner_carve<double>(a, in, ne, o.solver, o.restart);
    result = refine<double>(c, in, b, bnorm, x, r, b, bnorm, tol, o, o.inner_tol, pre, hist, inf,
                            &relres, &iters);
    if (learned && result != FIT_OK && result != FIT_E_NAN && iters < o.max_iters) {
      // The learned preconditioner stalled: finish with the plain method
      // (mass-preconditioned COCG, the symmetric scaling of eq. (e2t)) from
      // the current x, judged by the same true FP64 residual.
      inf.fell_back = 1;
      c.gm_stall_cycles = 0;
      c.sym = 1;
      c.diag = FIT_DIAG_AUTO;
      Arena a2{(char*)g->ws.ptr, 0, g->ws.bytes};
      (void)a2.take<double>(v128);
      (void)a2.take<double>(v128);
      if (hist) (void)a2.take<double>(hist_bytes);
      Inner<double> in2;
      inner_carve<double>(a2, in2, ne, FIT_COCG, o.restart);
      fit_solve_opts o2 = o;
      o2.solver = FIT_COCG;
      o2.max_iters = o.max_iters - iters;
      const int hoff = std::min(iters, o.resid_history_len);
      o2.resid_history_len = o.resid_history_len - hoff;
      double* hist2 = (hist && o2.resid_history_len > 0) ? hist + hoff : nullptr;
      if ((st = residual(c, x, b, r, nullptr, 0.0)) != FIT_OK) return st;
      if ((st = sync_copy(c, c.h_red, c.red, sizeof(RedOut))) != FIT_OK) return st;
      int it2 = 0;
      result = refine<double>(c, in2, b, bnorm, x, r, r, std::sqrt(c.h_red->v[0]), tol, o2,
                              o.inner_tol, nullptr, hist2, inf, &relres, &it2);
      iters += it2;
    }
  }
  if (snap) snap->made = c.snap_n;
  if (pre && pre != &ident) delete pre;
  if (hist && o.resid_history) {
    const int n = std::min(o.resid_history_len, iters);
    if (n > 0) FIT_HIP(hipMemcpyAsync(o.resid_history, hist, sizeof(double) * n, hipMemcpyDeviceToHost, s));
  }
  FIT_HIP(hipStreamSynchronize(s));
  const auto t1 = std::chrono::steady_clock::now();
  inf.status = result;
  inf.iterations = iters;
  inf.matvecs = c.matvecs;
  inf.true_relres = relres;
  inf.time_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  inf.bytes_moved = c.bytes;
  if (info) *info = inf;
  if (result != FIT_OK) {
    static const char* names[] = {"", "", "", "", "iteration cap reached", "Krylov breakdown",
                                  "NaN/Inf in the iteration", ""};
    set_error(std::string("fit_solve: ") + names[result] + " (relres " + std::to_string(relres) + ")");
  }
  return result;
}
}  // namespace

// ---------------------------------------------------------------------------
// Residual -> error pairs generated by the solver, for training the learned
// preconditioner: x* from a COCG solve to tol, then a second identical solve
// keeps its iterate x_k at npairs evenly spaced polls; e_k = x* - x_k and
// r_k = A(omega) e_k (equal to b - A x_k up to rounding).
// ---------------------------------------------------------------------------
namespace fit {
fit_status harvest_pairs(fit_grid* g, double omega, int port, int npairs, double tol, double* e,
                         double* r, int* made, int* iterations) {
  DeviceScope dev(g->device);
  const int64_t ne = g->ne;
  *made = 0;
  std::vector<double> hsrc((size_t)2 * ne, 0.0);
  const fit_port& q = (*g->host_ports)[port];
  for (int k = q.k0; k < q.k1; ++k)
    hsrc[2 * (3 * ((int64_t)q.i + (int64_t)g->view.nx * (q.j + (int64_t)g->view.ny * k)) + 2)] = 1.0;
  double *src = nullptr, *xs = nullptr, *xt = nullptr;
  auto cleanup = [&]() {
    (void)hipFree(src);
    (void)hipFree(xs);
    (void)hipFree(xt);
  };
  if (hipMalloc(&src, ne * 16) != hipSuccess || hipMalloc(&xs, ne * 16) != hipSuccess ||
      hipMalloc(&xt, ne * 16) != hipSuccess) {
    cleanup();
    set_error("fit_precond_harvest: out of device memory");
    return FIT_E_NOMEM;
  }
  fit_status st = FIT_OK;
  if (hipMemcpy(src, hsrc.data(), ne * 16, hipMemcpyHostToDevice) != hipSuccess) st = FIT_E_DEVICE;
  fit_solve_opts o{};
  o.solver = FIT_COCG;
  o.scaling = FIT_SCALE_SYM;
  o.max_iters = 200000;
  fit_solve_info i1{}, i2{};
  if (st == FIT_OK) st = solve_impl(g, omega, src, tol, &o, xs, &i1, nullptr);
  if (st == FIT_OK) {
    // snapshots every `stride` iterations, strictly before convergence; the
    // host polls (where snapshots are taken) at that spacing
    const int stride = std::max(2, i1.iterations / (npairs + 1)) & ~1;
    SnapRequest req{e, ne * 2, npairs, stride};
    fit_solve_opts o2 = o;
    o2.check_every = stride;
    st = solve_impl(g, omega, src, tol, &o2, xt, &i2, &req);
    *made = req.made;
  }
  if (iterations) *iterations = i1.iterations;
  if (st == FIT_OK) {
    Ctx c;
    st = setup_ctx(c, g, omega, 0, nullptr);
    for (int k = 0; k < *made && st == FIT_OK; ++k) {
      double* ek = e + (int64_t)k * ne * 2;
      double* rk = r + (int64_t)k * ne * 2;
      // e_k = x* - x_k, r_k = A e_k
      st = xform<double, double, XF_SCALE>(c, false, false, ek, ek, -1.0, false);
      if (st == FIT_OK) st = xform<double, double, XF_AXPY>(c, false, false, xs, ek, 1.0, false);
      OpMatvec<double> mv{ek, rk};
      if (st == FIT_OK) st = launch_stencil<double, MODE_D>(g->view, tile_for(g, FIT_C128), omega, mv, nullptr);
    }
    if (st == FIT_OK && hipDeviceSynchronize() != hipSuccess) st = FIT_E_DEVICE;
  }
  cleanup();
  return st;
}
}  // namespace fit

extern "C" fit_status fit_precond_harvest(fit_grid* g, double omega, int port, int npairs, double tol,
                                          void* e_dev, void* r_dev, int* made, int* iterations) {
  if (!g || !e_dev || !r_dev || !made || npairs < 1 || port < 0 || port >= g->nports ||
      !(omega > 0.0) || !std::isfinite(omega) || !(tol > 0.0) || !(tol < 1.0)) {
    set_error("fit_precond_harvest: bad argument (NULL, npairs < 1, port outside the grid's "
              "ports, omega <= 0 or tol outside (0, 1))");
    return FIT_E_INVALID;
  }
  return harvest_pairs(g, omega, port, npairs, tol, (double*)e_dev, (double*)r_dev, made,
                       iterations);
}

// ---------------------------------------------------------------------------
// Port voltages: u_p = sum of the edge voltages along port p (Sec. IV).
// ---------------------------------------------------------------------------
struct PortList {
  int n;
  int i[64], j[64], k0[64], k1[64];
};

__global__ void port_sum_kernel(GridView g, PortList pl, const double* x, int nvec, double* out) {
  __shared__ double lds[2 * 4];
  const int p = blockIdx.x, v = blockIdx.y;
  double acc[2] = {0.0, 0.0};
  const int64_t off = (int64_t)v * 3 * g.np;
  for (int k = pl.k0[p] + threadIdx.x; k < pl.k1[p]; k += blockDim.x) {
    const int64_t n = pl.i[p] + (int64_t)g.nx * (pl.j[p] + (int64_t)g.ny * k);
    const cx<double> e = ldc(x, off + 3 * n + 2);
    acc[0] += e.re;
    acc[1] += e.im;
  }
  block_reduce<2>(acc, lds);
  if (threadIdx.x == 0) {
    out[2 * ((int64_t)v * pl.n + p)] = acc[0];
    out[2 * ((int64_t)v * pl.n + p) + 1] = acc[1];
  }
}

namespace fit {
fit_status port_voltages_dev(const fit_grid* g, const void* x_dev, int nvec, double* out_dev,
                             hipStream_t s) {
  PortList pl{};
  pl.n = g->nports;
  for (int p = 0; p < g->nports; ++p) {
    const fit_port& q = (*g->host_ports)[p];
    pl.i[p] = q.i;
    pl.j[p] = q.j;
    pl.k0[p] = q.k0;
    pl.k1[p] = q.k1;
  }
  if (pl.n == 0 || nvec == 0) return FIT_OK;
  hipLaunchKernelGGL(port_sum_kernel, dim3(pl.n, nvec), dim3(64), 0, s, g->view, pl,
                     (const double*)x_dev, nvec, out_dev);
  FIT_HIP(hipGetLastError());
  return FIT_OK;
}
}  // namespace fit

extern "C" fit_status fit_port_voltages(const fit_grid* g, const void* x_dev, int nvec,
                                        double* out_host, void* stream) {
  if (!g || !x_dev || !out_host || nvec < 1) {
    set_error("fit_port_voltages: bad argument");
    return FIT_E_INVALID;
  }
  if (g->nports == 0) return FIT_OK;
  DeviceScope dev(g->device);
  hipStream_t s = (hipStream_t)stream;
  double* d = nullptr;
  const size_t bytes = sizeof(double) * 2 * (size_t)nvec * g->nports;
  FIT_HIP(hipMalloc(&d, bytes));
  fit_status st = port_voltages_dev(g, x_dev, nvec, d, s);
  if (st == FIT_OK) {
    hipError_t e = hipMemcpyAsync(out_host, d, bytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = hip_fail(e, "port voltages copy");
  }
  (void)hipFree(d);
  return st;
}

// ---------------------------------------------------------------------------
// Port voltages without any allocation: the per-call device buffer of
// fit_port_voltages is replaced by a file-scope device array.  Every GPU the
// library runs on holds its own copy of the array until the process ends; its
// address on a device is looked up once, with that device current, and kept.
// ---------------------------------------------------------------------------
namespace {
constexpr int kPortScratchValues = 65536;  // complex128 port sums per call (1 MiB)
constexpr int kMaxScratchDevices = 64;
static __device__ __align__(256) double scratch[2 * kPortScratchValues];

std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxScratchDevices] = {};

// The device address of `scratch` on `device` (which must be current).
fit_status scratch_for(int device, double** out) {
  if (device < 0 || device >= kMaxScratchDevices) {
    set_error("fit_port_voltages_noalloc: device ordinal outside the supported range");
    return FIT_E_INVALID;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[device] = (double*)ptr;
  }
  *out = g_scratch_ptr[device];
  return FIT_OK;
}
}  // namespace

extern "C" fit_status fit_port_voltages_noalloc(const fit_grid* g, const void* x_dev, int nvec,
                                                double* out_host, void* stream) {
  if (!g || !x_dev || !out_host || nvec < 1) {
    set_error("fit_port_voltages_noalloc: bad argument");
    return FIT_E_INVALID;
  }
  if (g->nports == 0) return FIT_OK;
  if ((int64_t)nvec * g->nports > kPortScratchValues) {
    set_error("fit_port_voltages_noalloc: nvec * nports exceeds the 65536 values of the static "
              "scratch array");
    return FIT_E_INVALID;
  }
  DeviceScope dev(g->device);
  double* d = nullptr;
  fit_status st = scratch_for(g->device, &d);
  if (st != FIT_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  // port_sum_kernel writes every one of the nvec * nports values, so nothing
  // left from an earlier call can reach the output
  st = port_voltages_dev(g, x_dev, nvec, d, s);
  if (st != FIT_OK) return st;
  const size_t bytes = sizeof(double) * 2 * (size_t)nvec * g->nports;
  hipError_t e = hipMemcpyAsync(out_host, d, bytes, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "port voltages copy");
  return FIT_OK;
}

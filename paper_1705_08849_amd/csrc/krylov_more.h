// Further Krylov methods of the paper's solver comparison (Sec. IV): the
// conjugate residual method in its complex symmetric form (COCR: Sogabe &
// Zhang 2007, CR recurrences with the unconjugated bilinear form), the
// transpose-free QMR method (TFQMR: Freund 1993) and conjugate gradients
// squared (CGS: Sonneveld 1989).  Both run on the
// internal operator of the solve (S A S with the symmetric scaling of
// eq. (e2t)) with device-resident scalars, like BiCGStab and COCG: each
// reduction ends in a one-block finish kernel that performs the scalar step,
// and every kernel returns at once after the iteration has stopped.
#pragma once

#include "fit_internal.h"
#include "krylov.h"
#include "reduce.h"
#include "stencil.h"

namespace fit {

__host__ __device__ __forceinline__ cx<double> cdiv_d(cx<double> a, cx<double> b) {
  const double b2 = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / b2, (a.im * b.re - a.re * b.im) / b2};
}

template <class T>
__device__ __forceinline__ cx<T> to_t(cx<double> a) {
  return cx<T>{(T)a.re, (T)a.im};
}

// ===========================================================================
// COCR on A x = r0 (A complex symmetric), from x = 0:
//   p = r, q = w = A r, rho = r^T w;
//   loop: alpha = rho / q^T q; x += alpha p; r -= alpha q;
//         w = A r; rho' = r^T w; beta = rho'/rho; p = r + beta p; q = w + beta q.
// Scalars in CgState (rho, alpha, beta, rr, iteration count, stop code).
// ===========================================================================

// Operator step: w = A r and r^T w (r read as the operator input).
template <class T>
struct OpCocrW {
  const T* r;
  T* w;
  CgState* st;
  double* part;
  unsigned* cnt;
  int init;  // first application: rho = r^T w, beta = 0
  struct Raw {
    cx<T> v[3];
  };
  static constexpr int NRED = 2;
  __device__ bool skip() const { return *(volatile int*)&st->done != kRunning; }
  __device__ void begin() {}
  __device__ void load(int64_t n, Raw& a) const {
#pragma unroll
    for (int k = 0; k < 3; ++k) a.v[k] = ldc(r, 3 * n + k);
  }
  __device__ void zero(Raw& a) const {
#pragma unroll
    for (int k = 0; k < 3; ++k) a.v[k] = cx<T>{T(0), T(0)};
  }
  __device__ void input(const Raw& a, cx<T> (&x)[3]) const {
#pragma unroll
    for (int k = 0; k < 3; ++k) x[k] = a.v[k];
  }
  __device__ void own_input(int64_t, const cx<T> (&)[3]) const {}
  __device__ void consume(int64_t n, const cx<T> (&y)[3], const cx<T> (&xr)[3], double* acc) const {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      stc(w, 3 * n + k, y[k]);
      const double ar = xr[k].re, ai = xr[k].im, yr = y[k].re, yi = y[k].im;
      acc[0] += ar * yr - ai * yi;  // r^T w, unconjugated
      acc[1] += ar * yi + ai * yr;
    }
  }
  __host__ __device__ double* partials() const { return part; }
  __device__ unsigned* counter() const { return cnt; }
  __device__ void finalize(const double* s) const {
    const cx<double> rho_new{s[0], s[1]};
    if (!isfinite(s[0]) || !isfinite(s[1])) {
      st->done = kNan;
      return;
    }
    if (init) {
      st->rho = rho_new;
      st->beta = cx<double>{0.0, 0.0};
      return;
    }
    const cx<double> rho = st->rho;
    if (cabs2(rho) == 0.0) {
      st->reason = 3;
      st->done = kBreakdown;
      return;
    }
    st->beta = cdiv_d(rho_new, rho);
    st->rho = rho_new;
  }
};

// p = r + beta p, q = w + beta q, q^T q.
template <class T>
__global__ void __launch_bounds__(256)
    cocr_pq_kernel(int64_t n, const T* r, const T* w, T* p, T* q, CgState* st, double* part) {
  __shared__ double lds[2 * 4];
  if (*(volatile int*)&st->done != kRunning) return;
  const cx<T> be = to_t<T>(st->beta);
  double acc[2] = {0.0, 0.0};
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const cx<T> pv = ldc(r, e) + be * ldc(p, e);
    const cx<T> qv = ldc(w, e) + be * ldc(q, e);
    stc(p, e, pv);
    stc(q, e, qv);
    const double qr = qv.re, qi = qv.im;
    acc[0] += qr * qr - qi * qi;
    acc[1] += 2.0 * qr * qi;
  }
  block_partial<2>(acc, part, lds);
}

struct CocrAlphaFinish {
  CgState* st;
  __device__ bool skip() const { return *(volatile int*)&st->done != kRunning; }
  __device__ void operator()(const double* s) const {
    const cx<double> qq{s[0], s[1]};
    if (!isfinite(s[0]) || !isfinite(s[1])) {
      st->done = kNan;
      return;
    }
    if (cabs2(qq) == 0.0) {
      st->reason = 2;
      st->done = kBreakdown;
      return;
    }
    st->alpha = cdiv_d(st->rho, qq);
  }
};

// x += alpha p, r -= alpha q, ||r||^2.
template <class T>
__global__ void __launch_bounds__(256)
    cocr_xr_kernel(int64_t n, T* x, T* r, const T* p, const T* q, CgState* st, double* part) {
  __shared__ double lds[4];
  if (*(volatile int*)&st->done != kRunning) return;
  const cx<T> al = to_t<T>(st->alpha);
  double acc[1] = {0.0};
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    stc(x, e, ldc(x, e) + al * ldc(p, e));
    const cx<T> rv = ldc(r, e) - al * ldc(q, e);
    stc(r, e, rv);
    acc[0] += cabs2_d(rv);
  }
  block_partial<1>(acc, part, lds);
}

struct CocrResFinish {
  CgState* st;
  __device__ bool skip() const { return *(volatile int*)&st->done != kRunning; }
  __device__ void operator()(const double* s) const {
    const double rr = s[0];
    st->iter += 1;
    if (st->hist && st->iter <= st->hist_len) st->hist[st->iter - 1] = sqrt(rr) * st->hscale;
    if (!isfinite(rr)) {
      st->done = kNan;
      return;
    }
    st->rr = rr;
    if (rr <= st->tol2) {
      st->done = kConverged;
      return;
    }
    if (st->iter >= st->max_iter) st->done = kMaxIter;
  }
};

// ===========================================================================
// TFQMR on A x = r0 from x = 0 (Freund's algorithm in the half-step form:
// half-steps m = 0, 1, 2, ...; an iteration is an even and an odd half-step
// and costs two operator applications).  Conjugated inner products with the
// shadow vector rh; tau, theta real; alpha, beta, eta, rho complex.
// ===========================================================================
struct TqState {
  cx<double> rho, alpha, beta, eta;
  double tau, theta;
  double tol2;    // stop when tau^2 (m + 1) <= tol2 (the QMR residual bound)
  double hscale;  // history value = tau sqrt(m + 1) * hscale
  double rr;      // tau^2 (m + 1) at the last completed iteration
  int iter, max_iter, done, hist_len;
  double* hist;
  int m, reason;  // half-steps done; breakdown test
};

// sigma = <rh, v> (conjugated).
template <class T>
__global__ void __launch_bounds__(256)
    tq_dot_kernel(int64_t n, const T* rh, const T* v, TqState* st, double* part) {
  __shared__ double lds[2 * 4];
  if (*(volatile int*)&st->done != kRunning) return;
  double acc[2] = {0.0, 0.0};
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const cx<double> d = cdotc_d(ldc(rh, e), ldc(v, e));
    acc[0] += d.re;
    acc[1] += d.im;
  }
  block_partial<2>(acc, part, lds);
}

struct TqAlphaFinish {
  TqState* st;
  __device__ bool skip() const { return *(volatile int*)&st->done != kRunning; }
  __device__ void operator()(const double* s) const {
    const cx<double> sig{s[0], s[1]};
    if (!isfinite(s[0]) || !isfinite(s[1])) {
      st->done = kNan;
      return;
    }
    if (cabs2(sig) == 0.0) {
      st->reason = 1;
      st->done = kBreakdown;
      return;
    }
    st->alpha = cdiv_d(st->rho, sig);
  }
};

// One half-step's vector work before its norm: with u the current u_m and
// au = A u_m,
//   (even only) u_next = u - alpha v
//   w -= alpha au
//   d = u + (theta^2 / alpha) eta d
// and ||w||^2.
template <class T, bool EVEN>
__global__ void __launch_bounds__(256)
    tq_half_kernel(int64_t n, const T* u, T* u_next, const T* v, T* w, const T* au, T* d,
                   TqState* st, double* part) {
  __shared__ double lds[4];
  if (*(volatile int*)&st->done != kRunning) return;
  const cx<double> al = st->alpha;
  const cx<T> a = to_t<T>(al);
  const cx<T> cd = to_t<T>(cdiv_d(cx<double>{st->theta * st->theta, 0.0}, al) * st->eta);
  double acc[1] = {0.0};
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const cx<T> uv = ldc(u, e);
    if (EVEN) stc(u_next, e, uv - a * ldc(v, e));
    const cx<T> wv = ldc(w, e) - a * ldc(au, e);
    stc(w, e, wv);
    stc(d, e, uv + cd * ldc(d, e));
    acc[0] += cabs2_d(wv);
  }
  block_partial<1>(acc, part, lds);
}

// theta = ||w|| / tau, c = (1 + theta^2)^{-1/2}, tau = tau theta c,
// eta = c^2 alpha; one more half-step.
struct TqStepFinish {
  TqState* st;
  __device__ bool skip() const { return *(volatile int*)&st->done != kRunning; }
  __device__ void operator()(const double* s) const {
    const double ww = s[0];
    if (!isfinite(ww)) {
      st->done = kNan;
      return;
    }
    const double th = sqrt(ww) / st->tau;
    const double c2 = 1.0 / (1.0 + th * th);
    st->theta = th;
    st->tau = st->tau * th * sqrt(c2);
    st->eta = c2 * st->alpha;
    st->m += 1;
  }
};

// x += eta d; on odd half-steps also rho' = <rh, w>.
template <class T, bool ODD>
__global__ void __launch_bounds__(256)
    tq_x_kernel(int64_t n, T* x, const T* d, const T* rh, const T* w, TqState* st, double* part) {
  __shared__ double lds[2 * 4];
  if (*(volatile int*)&st->done != kRunning) return;
  const cx<T> et = to_t<T>(st->eta);
  double acc[2] = {0.0, 0.0};
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    stc(x, e, ldc(x, e) + et * ldc(d, e));
    if (ODD) {
      const cx<double> q = cdotc_d(ldc(rh, e), ldc(w, e));
      acc[0] += q.re;
      acc[1] += q.im;
    }
  }
  if (ODD) block_partial<2>(acc, part, lds);
}

// End of an iteration (after the odd half-step): the stopping tests on the
// residual bound, then beta = rho' / rho.
struct TqRhoFinish {
  TqState* st;
  __device__ bool skip() const { return *(volatile int*)&st->done != kRunning; }
  __device__ void operator()(const double* s) const {
    const cx<double> rho_new{s[0], s[1]};
    st->iter += 1;
    const double bound2 = st->tau * st->tau * (double)(st->m + 1);
    st->rr = bound2;
    if (st->hist && st->iter <= st->hist_len) st->hist[st->iter - 1] = sqrt(bound2) * st->hscale;
    if (!isfinite(s[0]) || !isfinite(s[1]) || !isfinite(bound2)) {
      st->done = kNan;
      return;
    }
    if (bound2 <= st->tol2) {
      st->done = kConverged;
      return;
    }
    if (cabs2(st->rho) == 0.0 || cabs2(rho_new) == 0.0) {
      st->reason = 3;
      st->done = kBreakdown;
      return;
    }
    st->beta = cdiv_d(rho_new, st->rho);
    st->rho = rho_new;
    if (st->iter >= st->max_iter) st->done = kMaxIter;
  }
};

// u_even = w + beta u_odd.
template <class T>
__global__ void __launch_bounds__(256)
    tq_u_kernel(int64_t n, T* u0, const T* w, const T* u1, const TqState* st) {
  if (*(volatile const int*)&st->done != kRunning) return;
  const cx<T> be = to_t<T>(st->beta);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    stc(u0, e, ldc(w, e) + be * ldc(u1, e));
}

// v = A u_even + beta (A u_odd + beta v).
template <class T>
__global__ void __launch_bounds__(256)
    tq_v_kernel(int64_t n, T* v, const T* au0, const T* au1, const TqState* st) {
  if (*(volatile const int*)&st->done != kRunning) return;
  const cx<T> be = to_t<T>(st->beta);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    stc(v, e, ldc(au0, e) + be * (ldc(au1, e) + be * ldc(v, e)));
}

// ===========================================================================
// CGS (Sonneveld 1989) on A x = r0 from x = 0, conjugated inner products with
// the shadow vector rh:
//   rho = <rh, r>; beta = rho / rho_old (0 at the start, with p = q = 0);
//   u = r + beta q; p = u + beta (q + beta p); v = A p;
//   alpha = rho / <rh, v>; q = u - alpha v; w = u + q;
//   x += alpha w; r -= alpha A w.
// Scalars in TqState (rho, alpha, beta, rr, iteration count, stop code).
// ===========================================================================
template <class T>
__global__ void __launch_bounds__(256)
    cgs_up_kernel(int64_t n, const T* r, T* u, T* p, const T* q, const TqState* st) {
  if (*(volatile const int*)&st->done != kRunning) return;
  const cx<T> be = to_t<T>(st->beta);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const cx<T> qv = ldc(q, e);
    const cx<T> uv = ldc(r, e) + be * qv;
    stc(u, e, uv);
    stc(p, e, uv + be * (qv + be * ldc(p, e)));
  }
}

// q = u - alpha v, w = u + q (w overwrites u).
template <class T>
__global__ void __launch_bounds__(256)
    cgs_qw_kernel(int64_t n, T* u, T* q, const T* v, const TqState* st) {
  if (*(volatile const int*)&st->done != kRunning) return;
  const cx<T> al = to_t<T>(st->alpha);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const cx<T> uv = ldc(u, e);
    const cx<T> qv = uv - al * ldc(v, e);
    stc(q, e, qv);
    stc(u, e, uv + qv);
  }
}

// x += alpha w, r -= alpha A w; ||r||^2 and <rh, r>.
template <class T>
__global__ void __launch_bounds__(256)
    cgs_xr_kernel(int64_t n, T* x, T* r, const T* w, const T* aw, const T* rh, TqState* st,
                  double* part) {
  __shared__ double lds[3 * 4];
  if (*(volatile int*)&st->done != kRunning) return;
  const cx<T> al = to_t<T>(st->alpha);
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    stc(x, e, ldc(x, e) + al * ldc(w, e));
    const cx<T> rv = ldc(r, e) - al * ldc(aw, e);
    stc(r, e, rv);
    acc[0] += cabs2_d(rv);
    const cx<double> d = cdotc_d(ldc(rh, e), rv);
    acc[1] += d.re;
    acc[2] += d.im;
  }
  block_partial<3>(acc, part, lds);
}

// End of a CGS iteration: the stopping tests on the recursive residual, then
// beta = rho' / rho for the next one.
struct CgsFinish {
  TqState* st;
  __device__ bool skip() const { return *(volatile int*)&st->done != kRunning; }
  __device__ void operator()(const double* s) const {
    const double rr = s[0];
    const cx<double> rho_new{s[1], s[2]};
    st->iter += 1;
    if (st->hist && st->iter <= st->hist_len) st->hist[st->iter - 1] = sqrt(rr) * st->hscale;
    if (!isfinite(rr) || !isfinite(s[1]) || !isfinite(s[2])) {
      st->done = kNan;
      return;
    }
    st->rr = rr;
    if (rr <= st->tol2) {
      st->done = kConverged;
      return;
    }
    if (cabs2(st->rho) == 0.0 || cabs2(rho_new) == 0.0) {
      st->reason = 3;
      st->done = kBreakdown;
      return;
    }
    st->beta = cdiv_d(rho_new, st->rho);
    st->rho = rho_new;
    if (st->iter >= st->max_iter) st->done = kMaxIter;
  }
};

// OpMatvec with the solver's stop flag: no work once the iteration ended.
template <class T>
struct OpMatvecIf {
  const T* x;
  T* y;
  const int* done;
  struct Raw {
    cx<T> v[3];
  };
  static constexpr int NRED = 0;
  __device__ bool skip() const { return *(volatile const int*)done != kRunning; }
  __device__ void begin() {}
  __device__ void load(int64_t n, Raw& r) const {
#pragma unroll
    for (int k = 0; k < 3; ++k) r.v[k] = ldc(x, 3 * n + k);
  }
  __device__ void zero(Raw& r) const {
#pragma unroll
    for (int k = 0; k < 3; ++k) r.v[k] = {T(0), T(0)};
  }
  __device__ void input(const Raw& r, cx<T> (&xin)[3]) const {
#pragma unroll
    for (int k = 0; k < 3; ++k) xin[k] = r.v[k];
  }
  __device__ void own_input(int64_t, const cx<T> (&)[3]) const {}
  __device__ void consume(int64_t n, const cx<T> (&yv)[3], const cx<T> (&)[3], double*) const {
#pragma unroll
    for (int k = 0; k < 3; ++k) stc(y, 3 * n + k, yv[k]);
  }
  __host__ __device__ double* partials() const { return nullptr; }
  __device__ unsigned* counter() const { return nullptr; }
  __device__ void finalize(const double*) const {}
};

}  // namespace fit

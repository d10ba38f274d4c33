// Krylov building blocks: device solver state, the stencil Op policies that
// fuse vector updates and dot products into the operator launch, and the
// pointwise / multi-vector kernels.
//
// All scalars of the iteration live in device memory and are produced by the
// last block of the reduction that determines them; the host only reads the
// state every few iterations to test for termination.
#pragma once

#include "fit_internal.h"
#include "reduce.h"
#include "stencil.h"

namespace fit {

enum Done { kRunning = 0, kConverged = 1, kBreakdown = 2, kNan = 3, kMaxIter = 4 };

// BiCGStab scalars (complex, conjugated inner products, van der Vorst 1992).
struct BiState {
  cx<double> rho, alpha, omega, beta;
  double rr;      // ||r||^2 of the recursively updated residual
  double rhrh;    // ||r_hat||^2
  double tol2;    // stop when rr <= tol2
  double hscale;  // history value = sqrt(rr) * hscale
  int iter, max_iter, done, hist_len;
  double* hist;
  int reason;  // which test declared a breakdown (1 sigma, 2 t, 3 rho, 4 omega)
  int pad;
};

// COCG scalars: rho = r^T r, alpha = rho / p^T q, beta = rho_new / rho
// (unconjugated bilinear forms; the operator is complex symmetric).
struct CgState {
  cx<double> rho, alpha, beta;
  double rr, tol2, hscale;
  int iter, max_iter, done, hist_len;
  double* hist;
  int reason, pad;
  // deferred solution update of the fused step (OpCocgPX): x still lacks
  // alpha * p[pbuf] when pend is set
  int pend, pbuf;
};

// Mass-preconditioned COCG step 1 with the preconditioner recomputed in the
// operator launch.  In the unscaled operator's staging the diagonal term is
// d = -omega^2 M_eps,c per free edge, so m = 1/M_eps,c = -omega^2 / d costs no
// memory traffic.  Input p = m .* r + beta p_old (stored for owned nodes),
// output q = A p and p^T q.  The owned nodes also apply the previous
// iteration's solution update x += alpha_prev p_old, one step late, which
// saves the streaming update kernel two vector passes; the last update is
// applied by cocg_fixup_kernel.
template <class T>
struct OpCocgPX {
  const T *r, *p_old;
  T *p_new, *q, *x;
  CgState* st;
  double* part;
  T w2;  // omega^2
  cx<T> beta, alpha_prev;
  struct Raw {
    cx<T> r[3], p[3], x[3];
  };
  static constexpr int NRED = 2;
  static constexpr bool kFused = true;
  static constexpr bool kDeepPrefetch = true;
  __device__ bool skip() const { return *(volatile int*)&st->done != kRunning; }
  __device__ void begin() {
    beta = cx<T>{(T)st->beta.re, (T)st->beta.im};
    alpha_prev = cx<T>{(T)st->alpha.re, (T)st->alpha.im};
  }
  __device__ void load(int64_t n, Raw& a) const {
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      a.r[w] = ldc(r, 3 * n + w);
      a.p[w] = ldc(p_old, 3 * n + w);
    }
  }
  __device__ void load_own(int64_t n, Raw& a) const {
#pragma unroll
    for (int w = 0; w < 3; ++w) a.x[w] = ldc(x, 3 * n + w);
  }
  __device__ void zero(Raw& a) const {
#pragma unroll
    for (int w = 0; w < 3; ++w) a.r[w] = a.p[w] = cx<T>{T(0), T(0)};
  }
  template <class NC>
  __device__ void input_coef(const Raw& a, const NC& nc, cx<T> (&xin)[3]) const {
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      const cx<T> d = nc.e[w];
      const bool fr = (nc.mask >> w) & 1u;
      const T a2 = fr ? d.re * d.re + d.im * d.im : T(1);
      const T f = fr ? -w2 / a2 : T(0);
      const cx<T> m{f * d.re, -f * d.im};
      xin[w] = m * a.r[w] + beta * a.p[w];
    }
  }
  __device__ void own_input_raw(int64_t n, const Raw& a, const cx<T> (&pv)[3]) const {
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      stc(p_new, 3 * n + w, pv[w]);
      stc(x, 3 * n + w, a.x[w] + alpha_prev * a.p[w]);
    }
  }
  __device__ void consume(int64_t n, const cx<T> (&y)[3], const cx<T> (&pv)[3], double* acc) const {
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      stc(q, 3 * n + w, y[w]);
      const double pr = pv[w].re, pi = pv[w].im, yr = y[w].re, yi = y[w].im;
      acc[0] += pr * yr - pi * yi;
      acc[1] += pr * yi + pi * yr;
    }
  }
  __host__ __device__ double* partials() const { return part; }
  __device__ void finalize(const double* s) const {
    const cx<double> gam{s[0], s[1]};
    const double g2 = cabs2(gam);
    st->pend = 0;  // this launch applied the pending update
    if (!isfinite(g2)) {
      st->done = kNan;
      return;
    }
    if (g2 == 0.0) {
      st->reason = 1;
      st->done = kBreakdown;
      return;
    }
    const cx<double> rho = st->rho;
    st->alpha = cx<double>{(rho.re * gam.re + rho.im * gam.im) / g2,
                           (rho.im * gam.re - rho.re * gam.im) / g2};
    st->pend = 1;
    st->pbuf = (st->iter & 1) ^ 1;
  }
};

// COCG step 1: p = r + beta p_old on the fly (stored), q = A p, p^T q.
template <class T>
struct OpCocgP {
  const T *r, *p_old;
  T *p_new, *q;
  CgState* st;
  double* part;
  unsigned* cnt;
  cx<T> beta;
  struct Raw {
    cx<T> r[3], p[3];
  };
  static constexpr int NRED = 2;
  __device__ bool skip() const { return *(volatile int*)&st->done != kRunning; }
  __device__ void begin() { beta = cx<T>{(T)st->beta.re, (T)st->beta.im}; }
  __device__ void load(int64_t n, Raw& a) const {
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      a.r[w] = ldc(r, 3 * n + w);
      a.p[w] = ldc(p_old, 3 * n + w);
    }
  }
  __device__ void zero(Raw& a) const {
#pragma unroll
    for (int w = 0; w < 3; ++w) a.r[w] = a.p[w] = cx<T>{T(0), T(0)};
  }
  __device__ void input(const Raw& a, cx<T> (&x)[3]) const {
#pragma unroll
    for (int w = 0; w < 3; ++w) x[w] = a.r[w] + beta * a.p[w];
  }
  __device__ void own_input(int64_t n, const cx<T> (&x)[3]) const {
#pragma unroll
    for (int w = 0; w < 3; ++w) stc(p_new, 3 * n + w, x[w]);
  }
  __device__ void consume(int64_t n, const cx<T> (&y)[3], const cx<T> (&pv)[3], double* acc) const {
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      stc(q, 3 * n + w, y[w]);
      // p^T q (no conjugation)
      const double pr = pv[w].re, pi = pv[w].im, yr = y[w].re, yi = y[w].im;
      acc[0] += pr * yr - pi * yi;
      acc[1] += pr * yi + pi * yr;
    }
  }
  __host__ __device__ double* partials() const { return part; }
  __device__ unsigned* counter() const { return cnt; }
  __device__ void finalize(const double* s) const {
    const cx<double> gam{s[0], s[1]};
    const double g2 = cabs2(gam);
    if (!isfinite(g2)) {
      st->done = kNan;
      return;
    }
    if (g2 == 0.0) {
      st->reason = 1;
      st->done = kBreakdown;
      return;
    }
    const cx<double> rho = st->rho;
    st->alpha = cx<double>{(rho.re * gam.re + rho.im * gam.im) / g2,
                           (rho.im * gam.re - rho.re * gam.im) / g2};
  }
};

// Restarted (flexible) GMRES state: Hessenberg column, Givens rotations and
// the rotated right-hand side, all in complex FP64.
constexpr int kMaxRestart = 64;
struct GmState {
  cx<double> h[(kMaxRestart + 1) * kMaxRestart];  // column-major, ld = m+1
  cx<double> cs[kMaxRestart], sn[kMaxRestart];
  cx<double> g[kMaxRestart + 1];
  cx<double> y[kMaxRestart];
  cx<double> hcol[kMaxRestart + 1];  // result of the last multi-dot
  double vscale;                      // 1 / norm of the vector to normalise next
  double beta;                        // residual norm at the cycle start
  double tol;                         // stop when |g_{j+1}| <= tol
  double hscale;
  int m, j, k, done, iter, max_iter, hist_len, pad;
  double* hist;
};

// Scalar results of one-off reductions (norms of residuals etc.).
struct RedOut {
  double v[4];
  int flag;
  int pad;
};

inline int pw_blocks(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (int)(b < 4096 ? (b < 1 ? 1 : b) : 4096);
}

template <class T>
__device__ __forceinline__ T tcast(double v) {
  return (T)v;
}

// ---------------------------------------------------------------------------
// BiCGStab step 1: p = r + beta (p_old - omega v_old) on the fly,
// v = A p, and <r_hat, v>.  p_old/v_old and p_new/v_new are distinct buffers
// (neighbouring workgroups still read the old values of the halo).
// ---------------------------------------------------------------------------
template <class T>
struct OpBicgP {
  const T *r, *p_old, *v_old, *rh;
  T *p_new, *v_new;
  BiState* st;
  double* part;
  unsigned* cnt;
  cx<T> beta, omega;
  struct Raw {
    cx<T> r[3], p[3], v[3];
  };
  static constexpr int NRED = 2;
  __device__ bool skip() const { return *(volatile int*)&st->done != kRunning; }
  __device__ void begin() {
    beta = cx<T>{(T)st->beta.re, (T)st->beta.im};
    omega = cx<T>{(T)st->omega.re, (T)st->omega.im};
  }
  __device__ void load(int64_t n, Raw& a) const {
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      a.r[w] = ldc(r, 3 * n + w);
      a.p[w] = ldc(p_old, 3 * n + w);
      a.v[w] = ldc(v_old, 3 * n + w);
    }
  }
  __device__ void zero(Raw& a) const {
#pragma unroll
    for (int w = 0; w < 3; ++w) a.r[w] = a.p[w] = a.v[w] = cx<T>{T(0), T(0)};
  }
  __device__ void input(const Raw& a, cx<T> (&x)[3]) const {
#pragma unroll
    for (int w = 0; w < 3; ++w) x[w] = a.r[w] + beta * (a.p[w] - omega * a.v[w]);
  }
  __device__ void own_input(int64_t n, const cx<T> (&x)[3]) const {
#pragma unroll
    for (int w = 0; w < 3; ++w) stc(p_new, 3 * n + w, x[w]);
  }
  __device__ void consume(int64_t n, const cx<T> (&y)[3], const cx<T> (&)[3], double* acc) const {
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      stc(v_new, 3 * n + w, y[w]);
      const cx<T> h = ldc(rh, 3 * n + w);
      const cx<double> d = cdotc_d(h, y[w]);
      acc[0] += (double)d.re;
      acc[1] += (double)d.im;
    }
  }
  __host__ __device__ double* partials() const { return part; }
  __device__ unsigned* counter() const { return cnt; }
  __device__ void finalize(const double* s) const {
    const cx<double> sig{s[0], s[1]};
    const double a2 = cabs2(sig);
    if (!(a2 == a2) || !isfinite(a2)) {
      st->done = kNan;
      return;
    }
    if (a2 == 0.0 || a2 < 1e-300 * st->rhrh * st->rr) {
      st->reason = 1;
      st->done = kBreakdown;
      return;
    }
    // alpha = rho / sigma
    const cx<double> rho = st->rho;
    st->alpha = cx<double>{(rho.re * sig.re + rho.im * sig.im) / a2,
                           (rho.im * sig.re - rho.re * sig.im) / a2};
  }
};

// BiCGStab step 2: s = r - alpha v on the fly (stored), t = A s, <t, s>, <t, t>.
template <class T>
struct OpBicgS {
  const T *r, *v;
  T *s, *t;
  BiState* st;
  double* part;
  unsigned* cnt;
  cx<T> alpha;
  struct Raw {
    cx<T> r[3], v[3];
  };
  static constexpr int NRED = 3;
  __device__ bool skip() const { return *(volatile int*)&st->done != kRunning; }
  __device__ void begin() { alpha = cx<T>{(T)st->alpha.re, (T)st->alpha.im}; }
  __device__ void load(int64_t n, Raw& a) const {
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      a.r[w] = ldc(r, 3 * n + w);
      a.v[w] = ldc(v, 3 * n + w);
    }
  }
  __device__ void zero(Raw& a) const {
#pragma unroll
    for (int w = 0; w < 3; ++w) a.r[w] = a.v[w] = cx<T>{T(0), T(0)};
  }
  __device__ void input(const Raw& a, cx<T> (&x)[3]) const {
#pragma unroll
    for (int w = 0; w < 3; ++w) x[w] = a.r[w] - alpha * a.v[w];
  }
  __device__ void own_input(int64_t n, const cx<T> (&x)[3]) const {
#pragma unroll
    for (int w = 0; w < 3; ++w) stc(s, 3 * n + w, x[w]);
  }
  __device__ void consume(int64_t n, const cx<T> (&y)[3], const cx<T> (&sv)[3], double* acc) const {
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      stc(t, 3 * n + w, y[w]);
      const cx<double> d = cdotc_d(y[w], sv[w]);
      acc[0] += d.re;
      acc[1] += d.im;
      acc[2] += cabs2_d(y[w]);
    }
  }
  __host__ __device__ double* partials() const { return part; }
  __device__ unsigned* counter() const { return cnt; }
  __device__ void finalize(const double* sum) const {
    const double tt = sum[2];
    if (!(tt == tt) || !isfinite(tt) || !isfinite(sum[0]) || !isfinite(sum[1])) {
      st->done = kNan;
      return;
    }
    if (tt == 0.0) {
      st->reason = 2;
      st->done = kBreakdown;
      return;
    }
    st->omega = cx<double>{sum[0] / tt, sum[1] / tt};
  }
};

// y = A x and r = b - y, ||r||^2 (complex128 true residual), optional
// complex64 copy of r scaled by `out_scale`.
template <class T>
struct OpResidual {
  const T *x, *b;
  T* r;
  float* r32;  // optional
  double out_scale;
  RedOut* out;
  double* part;
  unsigned* cnt;
  struct Raw {
    cx<T> v[3];
  };
  static constexpr int NRED = 1;
  static constexpr bool kDeepPrefetch = true;
  __device__ bool skip() const { return false; }
  __device__ void begin() {}
  __device__ void load(int64_t n, Raw& a) const {
#pragma unroll
    for (int w = 0; w < 3; ++w) a.v[w] = ldc(x, 3 * n + w);
  }
  __device__ void zero(Raw& a) const {
#pragma unroll
    for (int w = 0; w < 3; ++w) a.v[w] = cx<T>{T(0), T(0)};
  }
  __device__ void input(const Raw& a, cx<T> (&xi)[3]) const {
#pragma unroll
    for (int w = 0; w < 3; ++w) xi[w] = a.v[w];
  }
  __device__ void own_input(int64_t, const cx<T> (&)[3]) const {}
  __device__ void consume(int64_t n, const cx<T> (&y)[3], const cx<T> (&)[3], double* acc) const {
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      const cx<T> rv = ldc(b, 3 * n + w) - y[w];
      if (r) stc(r, 3 * n + w, rv);
      if (r32) stc(r32, 3 * n + w, cx<float>{(float)(out_scale * rv.re), (float)(out_scale * rv.im)});
      acc[0] += cabs2_d(rv);
    }
  }
  __host__ __device__ double* partials() const { return part; }
  __device__ unsigned* counter() const { return cnt; }
  __device__ void finalize(const double* s) const {
    out->v[0] = s[0];
    out->flag = isfinite(s[0]) ? 0 : 1;
  }
};

// Plain operator application used by GMRES: input v = w * vscale (w the
// unnormalised Arnoldi vector), stored as basis vector V_j; output A v.
template <class T>
struct OpGmresMv {
  const T* w;
  T* vj;      // may be null (FGMRES normalises separately)
  T* y;
  GmState* st;
  T vscale;
  struct Raw {
    cx<T> v[3];
  };
  static constexpr int NRED = 0;
  __device__ bool skip() const { return *(volatile int*)&st->done != kRunning; }
  __device__ void begin() { vscale = vj ? (T)st->vscale : T(1); }
  __device__ void load(int64_t n, Raw& a) const {
#pragma unroll
    for (int k = 0; k < 3; ++k) a.v[k] = ldc(w, 3 * n + k);
  }
  __device__ void zero(Raw& a) const {
#pragma unroll
    for (int k = 0; k < 3; ++k) a.v[k] = cx<T>{T(0), T(0)};
  }
  __device__ void input(const Raw& a, cx<T> (&x)[3]) const {
#pragma unroll
    for (int k = 0; k < 3; ++k) x[k] = vscale * a.v[k];
  }
  __device__ void own_input(int64_t n, const cx<T> (&x)[3]) const {
    if (vj) {
#pragma unroll
      for (int k = 0; k < 3; ++k) stc(vj, 3 * n + k, x[k]);
    }
  }
  __device__ void consume(int64_t n, const cx<T> (&yv)[3], const cx<T> (&)[3], double*) const {
#pragma unroll
    for (int k = 0; k < 3; ++k) stc(y, 3 * n + k, yv[k]);
  }
  __host__ __device__ double* partials() const { return nullptr; }
  __device__ unsigned* counter() const { return nullptr; }
  __device__ void finalize(const double*) const {}
};

template <class T>
struct OpName<OpCocgPX<T>> {
  static const char* get() { return sizeof(T) == 8 ? "pcocg_step1_c128" : "pcocg_step1_c64"; }
};
template <class T>
struct OpName<OpCocgP<T>> {
  static const char* get() { return sizeof(T) == 8 ? "cocg_step1_c128" : "cocg_step1_c64"; }
};
template <class T>
struct OpName<OpBicgP<T>> {
  static const char* get() { return sizeof(T) == 8 ? "bicgstab_step1_c128" : "bicgstab_step1_c64"; }
};
template <class T>
struct OpName<OpBicgS<T>> {
  static const char* get() { return sizeof(T) == 8 ? "bicgstab_step2_c128" : "bicgstab_step2_c64"; }
};
template <class T>
struct OpName<OpResidual<T>> {
  static const char* get() { return "residual_c128"; }
};
template <class T>
struct OpName<OpGmresMv<T>> {
  static const char* get() { return sizeof(T) == 8 ? "gmres_matvec_c128" : "gmres_matvec_c64"; }
};

}  // namespace fit

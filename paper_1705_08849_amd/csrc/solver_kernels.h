// Pointwise and reduction kernels of the Krylov drivers (shared by the
// single-system solver and the batched sweep).
#pragma once

#include <cstdint>

#include "fit_internal.h"
#include "krylov.h"
#include "reduce.h"
#include "stencil.h"

namespace fit {

// ---------------------------------------------------------------------------
// Node-wise transforms that need the per-edge coefficients (mask, scaling).
// ---------------------------------------------------------------------------
enum XformKind { XF_RHS = 0, XF_SCALE = 1, XF_AXPY = 2, XF_SHADOW = 3 };

// SplitMix64 (Steele, Lea & Flood 2014) as a counter-based generator: the
// output for counter c is the mix of seed + (c+1) * gamma.
__device__ __forceinline__ uint64_t splitmix64(uint64_t counter, uint64_t seed) {
  uint64_t z = seed + (counter + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
constexpr uint64_t kShadowSeed = 0x5EED;

// Uniform [-1, 1) from the top 53 bits.
__device__ __forceinline__ double u11(uint64_t h) {
  return 2.0 * ((double)(h >> 11) * 0x1.0p-53) - 1.0;
}

template <class TI, class TO, int KIND>
__global__ void __launch_bounds__(256)
    node_xform_kernel(GridView g, double omega, int sym, int inverse, const TI* in, TO* out,
                      double factor, RedOut* red, double* part, unsigned* cnt, uint64_t seed) {
  __shared__ MatLds<double> mat;
  __shared__ double lds[4];
  fill_mat_mode<double>(mat, g.mats, omega, MODE_MEC);
  __syncthreads();
  double acc[1] = {0.0};
  int bad = 0;
  const cx<double> pc = port_coef_mode<double>(omega, MODE_MEC);
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < g.np;
       n += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(n % g.nx);
    const int j = (int)((n / g.nx) % g.ny);
    const int p = (int)(n / ((int64_t)g.nx * g.ny));
    const ColGeo<double> cg = col_geo<double>(g, i, j);
    const PlaneRec<double> lo = plane_rec(mat, cg, load_cell_ids(g, i, j, p - 1));
    const PlaneRec<double> hi = plane_rec(mat, cg, load_cell_ids(g, i, j, p));
    const ZGeo<double> z = zgeo<double>(g, p);
    const NodeCoef<double> nc = node_coef(cg, lo, hi, z.hzl, z.hzh, z.ivz, p, pc);
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      const int64_t e = 3 * n + w;
      const bool fr = (nc.mask >> w) & 1u;
      const cx<TI> vi = ldc(in, e);
      const cx<double> v{(double)vi.re, (double)vi.im};
      if (KIND == XF_SHADOW) {
        // dense pseudo-random BiCGStab shadow vector on the free edges
        const double re = u11(splitmix64(2ull * (uint64_t)e, seed));
        const double im = u11(splitmix64(2ull * (uint64_t)e + 1ull, seed));
        const cx<double> sv = fr ? cx<double>{re, im} : cx<double>{0.0, 0.0};
        stc(out, e, cx<TO>{(TO)sv.re, (TO)sv.im});
        acc[0] += cabs2(sv);
        (void)v;
      } else if (KIND == XF_RHS) {
        // b = -j omega j
        const cx<double> b = fr ? cx<double>{omega * v.im, -omega * v.re} : cx<double>{0.0, 0.0};
        if (!fr && (v.re != 0.0 || v.im != 0.0)) bad = 1;
        stc(out, e, cx<TO>{(TO)b.re, (TO)b.im});
        acc[0] += cabs2(b);
      } else {
        cx<double> s{1.0, 0.0};
        if (sym && fr) {
          s = crsqrt(nc.e[w]);
          if (inverse) {
            const double a2 = cabs2(s);
            s = cx<double>{s.re / a2, -s.im / a2};
          }
        }
        cx<double> r = fr ? factor * (s * v) : cx<double>{0.0, 0.0};
        if (KIND == XF_AXPY) {
          const cx<TO> o = ldc(out, e);
          r = cx<double>{r.re + (double)o.re, r.im + (double)o.im};
          if (!fr) r = cx<double>{0.0, 0.0};
        }
        stc(out, e, cx<TO>{(TO)r.re, (TO)r.im});
        acc[0] += cabs2(r);
      }
    }
  }
  if (red) {
    if (bad) atomicOr(&red->flag, 1);
    block_partial<1>(acc, part, lds);
  }
  (void)cnt;
}

// Stores grid-wide sums into a RedOut.
template <int N>
struct StoreSums {
  RedOut* out;
  __device__ bool skip() const { return false; }
  __device__ void operator()(const double* s) const {
    for (int q = 0; q < N; ++q) out->v[q] = s[q];
  }
};

// ---------------------------------------------------------------------------
// Element-wise vector kernels.
// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(256) zero_kernel(T* v, int64_t n2) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n2;
       e += (int64_t)gridDim.x * blockDim.x)
    v[e] = T(0);
}

template <class T>
__global__ void __launch_bounds__(256) copy_kernel(const T* a, T* b, int64_t n2) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n2;
       e += (int64_t)gridDim.x * blockDim.x)
    b[e] = a[e];
}

// BiCGStab step 3: x += alpha p + omega s, r = s - omega t, <r_hat, r>, ||r||^2,
// then the next beta and the termination tests.
template <class T>
__global__ void __launch_bounds__(256)
    bicg_update_kernel(T* x, T* r, const T* p, const T* s, const T* t, const T* rh, int64_t n,
                       BiState* st, double* part, unsigned* cnt) {
  __shared__ double lds[3 * 4];
  if (*(volatile int*)&st->done != kRunning) return;
  const cx<T> al{(T)st->alpha.re, (T)st->alpha.im};
  const cx<T> om{(T)st->omega.re, (T)st->omega.im};
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const cx<T> sv = ldc(s, e);
    const cx<T> xv = ldc(x, e) + al * ldc(p, e) + om * sv;
    const cx<T> rv = sv - om * ldc(t, e);
    stc(x, e, xv);
    stc(r, e, rv);
    const cx<double> d = cdotc_d(ldc(rh, e), rv);
    acc[0] += d.re;
    acc[1] += d.im;
    acc[2] += cabs2_d(rv);
  }
  block_partial<3>(acc, part, lds);
  (void)cnt;
}

// Scalar step after the BiCGStab update's reduction: next beta and rho and
// the termination tests.
struct BicgFinish {
  BiState* st;
  __device__ bool skip() const { return *(volatile int*)&st->done != kRunning; }
  __device__ void operator()(const double* sum) const {
    const cx<double> rho_new{sum[0], sum[1]};
    const double rr = sum[2];
    st->iter += 1;
    if (st->hist && st->iter <= st->hist_len) st->hist[st->iter - 1] = sqrt(rr) * st->hscale;
    if (!isfinite(rr) || !isfinite(sum[0]) || !isfinite(sum[1])) {
      st->done = kNan;
      return;
    }
    // beta = (rho_new / rho) * (alpha / omega)
    const cx<double> rho = st->rho, a = st->alpha, w = st->omega;
    const double r2 = cabs2(rho), w2 = cabs2(w);
    st->rr = rr;
    if (rr <= st->tol2) {
      st->done = kConverged;
      st->rho = rho_new;
      return;
    }
    // <r_hat, r> negligible against |r_hat| |r| at the working precision:
    // the shadow space has collapsed (restart)
    if (r2 == 0.0 || w2 == 0.0 || cabs2(rho_new) < 1e-28 * rr * st->rhrh) {
      st->reason = (r2 == 0.0 || w2 == 0.0) ? 4 : 3;
      st->done = kBreakdown;
      return;
    }
    const cx<double> q{(rho_new.re * rho.re + rho_new.im * rho.im) / r2,
                       (rho_new.im * rho.re - rho_new.re * rho.im) / r2};
    const cx<double> aw{(a.re * w.re + a.im * w.im) / w2, (a.im * w.re - a.re * w.im) / w2};
    st->beta = q * aw;
    st->rho = rho_new;
    if (st->iter >= st->max_iter) st->done = kMaxIter;
  }
};

// Multi-dot h_i = <V_i, w>, i < nv: each block keeps its chunk of w in
// registers and walks the basis vectors; partials[i * nblk + blk].
constexpr int kMdPer = 4;  // complex elements per thread
template <class T>
__global__ void __launch_bounds__(256)
    multidot_kernel(const T* V, int64_t ldv, int nv, const T* w, int64_t n, double* part,
                    const GmState* st) {
  __shared__ double lds[2 * 4];
  if (st && *(volatile const int*)&st->done != kRunning) return;
  const int64_t base = (int64_t)blockIdx.x * 256 * kMdPer;
  cx<T> wl[kMdPer];
#pragma unroll
  for (int q = 0; q < kMdPer; ++q) {
    const int64_t e = base + q * 256 + threadIdx.x;
    wl[q] = e < n ? ldc(w, e) : cx<T>{T(0), T(0)};
  }
  for (int i = 0; i < nv; ++i) {
    double acc[2] = {0.0, 0.0};
#pragma unroll
    for (int q = 0; q < kMdPer; ++q) {
      const int64_t e = base + q * 256 + threadIdx.x;
      if (e < n) {
        const cx<double> d = cdotc_d(ldc(V + 2 * ldv * i, e), wl[q]);
        acc[0] += d.re;
        acc[1] += d.im;
      }
    }
    block_reduce<2>(acc, lds);
    if (threadIdx.x == 0) {
      part[2 * ((int64_t)i * gridDim.x + blockIdx.x)] = acc[0];
      part[2 * ((int64_t)i * gridDim.x + blockIdx.x) + 1] = acc[1];
    }
  }
}

// Sum the multi-dot partials: one block per basis vector, fixed order.
static __global__ void __launch_bounds__(256)
    multidot_finish_kernel(const double* part, int nblk, GmState* st, int accumulate) {
  __shared__ double lds[2 * 4];
  if (*(volatile int*)&st->done != kRunning) return;
  const int i = blockIdx.x;
  double acc[2] = {0.0, 0.0};
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
    acc[0] += part[2 * ((int64_t)i * nblk + b)];
    acc[1] += part[2 * ((int64_t)i * nblk + b) + 1];
  }
  block_reduce<2>(acc, lds);
  if (threadIdx.x == 0) {
    st->hcol[i] = cx<double>{acc[0], acc[1]};
    const int ld = st->m + 1;
    cx<double>& h = st->h[(int64_t)st->j * ld + i];
    h = accumulate ? h + st->hcol[i] : st->hcol[i];
  }
}

// w -= sum_i hcol_i V_i; optionally ||w||^2 into `out`.
template <class T>
__global__ void __launch_bounds__(256)
    multi_axpy_kernel(const T* V, int64_t ldv, int nv, T* w, int64_t n, GmState* st,
                      RedOut* out, double* part, unsigned* cnt) {
  __shared__ double lds[4];
  __shared__ cx<double> hc[kMaxRestart + 1];
  if (*(volatile int*)&st->done != kRunning) return;
  for (int i = threadIdx.x; i < nv; i += blockDim.x) hc[i] = st->hcol[i];
  __syncthreads();
  double acc[1] = {0.0};
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    cx<T> v = ldc(w, e);
    for (int i = 0; i < nv; ++i) {
      const cx<T> h{(T)hc[i].re, (T)hc[i].im};
      v = v - h * ldc(V + 2 * ldv * i, e);
    }
    stc(w, e, v);
    acc[0] += cabs2_d(v);
  }
  if (out) block_partial<1>(acc, part, lds);
  (void)cnt;
}

// Completes Arnoldi step j: h_{j+1,j} = ||w||, applies the previous Givens
// rotations to column j, forms the new one, updates g and tests convergence.
static __global__ void gmres_step_kernel(GmState* st, const RedOut* wn) {
  if (threadIdx.x != 0 || st->done != kRunning) return;
  const int m = st->m, ld = m + 1, j = st->j;
  cx<double>* h = st->h + (int64_t)j * ld;
  const double hn = sqrt(wn->v[0]);
  h[j + 1] = cx<double>{hn, 0.0};
  for (int i = 0; i < j; ++i) {
    const cx<double> c = st->cs[i], s = st->sn[i];
    const cx<double> a = h[i], b = h[i + 1];
    // [conj(c) conj(s); -s c] applied to (a, b)
    h[i] = cx<double>{c.re * a.re + c.im * a.im + s.re * b.re + s.im * b.im,
                      c.re * a.im - c.im * a.re + s.re * b.im - s.im * b.re};
    h[i + 1] = cx<double>{-(s.re * a.re - s.im * a.im) + (c.re * b.re - c.im * b.im),
                          -(s.re * a.im + s.im * a.re) + (c.re * b.im + c.im * b.re)};
  }
  const cx<double> a = h[j], b = h[j + 1];
  const double rho = sqrt(cabs2(a) + cabs2(b));
  cx<double> c{1.0, 0.0}, s{0.0, 0.0};
  if (rho > 0.0) {
    c = cx<double>{a.re / rho, a.im / rho};
    s = cx<double>{b.re / rho, b.im / rho};
  }
  st->cs[j] = c;
  st->sn[j] = s;
  h[j] = cx<double>{rho, 0.0};
  h[j + 1] = cx<double>{0.0, 0.0};
  const cx<double> gj = st->g[j];
  st->g[j + 1] = cx<double>{-(s.re * gj.re - s.im * gj.im), -(s.re * gj.im + s.im * gj.re)};
  st->g[j] = cx<double>{c.re * gj.re + c.im * gj.im, c.re * gj.im - c.im * gj.re};
  st->iter += 1;
  const double res = sqrt(cabs2(st->g[j + 1]));
  if (st->hist && st->iter <= st->hist_len) st->hist[st->iter - 1] = res * st->hscale;
  st->k = j + 1;
  st->vscale = hn > 0.0 ? 1.0 / hn : 0.0;
  st->j = j + 1;
  if (!isfinite(res) || !isfinite(hn)) {
    st->done = kNan;
  } else if (res <= st->tol) {
    st->done = kConverged;
  } else if (hn == 0.0) {
    st->done = kConverged;  // lucky breakdown: the Krylov space is invariant
  } else if (st->iter >= st->max_iter) {
    st->done = kMaxIter;
  } else if (st->j >= m) {
    st->done = kBreakdown;  // cycle complete: restart (not a failure)
  }
}

// Back substitution of the k x k upper-triangular least-squares system.
static __global__ void gmres_solve_kernel(GmState* st) {
  if (threadIdx.x != 0) return;
  const int k = st->k, ld = st->m + 1;
  for (int i = k - 1; i >= 0; --i) {
    cx<double> v = st->g[i];
    for (int q = i + 1; q < k; ++q) v = v - st->h[(int64_t)q * ld + i] * st->y[q];
    const cx<double> d = st->h[(int64_t)i * ld + i];
    const double d2 = cabs2(d);
    st->y[i] = d2 > 0 ? cx<double>{(v.re * d.re + v.im * d.im) / d2, (v.im * d.re - v.re * d.im) / d2}
                      : cx<double>{0.0, 0.0};
  }
}

// x += sum_i y_i B_i (B = V for GMRES, Z for FGMRES).
template <class T>
__global__ void __launch_bounds__(256)
    gmres_update_kernel(T* x, const T* B, int64_t ldb, int64_t n, const GmState* st) {
  __shared__ cx<double> yl[kMaxRestart];
  const int k = st->k;
  for (int i = threadIdx.x; i < k; i += blockDim.x) yl[i] = st->y[i];
  __syncthreads();
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    cx<T> v = ldc(x, e);
    for (int i = 0; i < k; ++i) v = v + cx<T>{(T)yl[i].re, (T)yl[i].im} * ldc(B + 2 * ldb * i, e);
    stc(x, e, v);
  }
}

// COCG step 2: x += alpha p, r -= alpha q, r^T r, ||r||^2, next beta and the
// termination tests.
template <class T>
__global__ void __launch_bounds__(256)
    cocg_update_kernel(T* x, T* r, const T* p, const T* q, int64_t n, CgState* st, double* part,
                       unsigned* cnt) {
  __shared__ double lds[3 * 4];
  if (*(volatile int*)&st->done != kRunning) return;
  const cx<T> al{(T)st->alpha.re, (T)st->alpha.im};
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const cx<T> xv = ldc(x, e) + al * ldc(p, e);
    const cx<T> rv = ldc(r, e) - al * ldc(q, e);
    stc(x, e, xv);
    stc(r, e, rv);
    const double rr = rv.re, ri = rv.im;
    acc[0] += rr * rr - ri * ri;
    acc[1] += 2.0 * rr * ri;
    acc[2] += rr * rr + ri * ri;
  }
  block_partial<3>(acc, part, lds);
  (void)cnt;
}

// Scalar step after the COCG update's reduction.
struct CocgFinish {
  CgState* st;
  __device__ bool skip() const { return *(volatile int*)&st->done != kRunning; }
  __device__ void operator()(const double* sum) const {
    const cx<double> rho_new{sum[0], sum[1]};
    const double rr = sum[2];
    st->iter += 1;
    if (st->hist && st->iter <= st->hist_len) st->hist[st->iter - 1] = sqrt(rr) * st->hscale;
    if (!isfinite(rr) || !isfinite(sum[0]) || !isfinite(sum[1])) {
      st->done = kNan;
      return;
    }
    st->rr = rr;
    if (rr <= st->tol2) {
      st->done = kConverged;
      return;
    }
    const cx<double> rho = st->rho;
    const double r2 = cabs2(rho);
    if (r2 == 0.0 || cabs2(rho_new) < 1e-28 * rr * rr) {
      st->reason = 3;  // r^T r vanishes: r is (nearly) a quasi-null vector
      st->done = kBreakdown;
      return;
    }
    st->beta = cx<double>{(rho_new.re * rho.re + rho_new.im * rho.im) / r2,
                          (rho_new.im * rho.re - rho_new.re * rho.im) / r2};
    st->rho = rho_new;
    if (st->iter >= st->max_iter) st->done = kMaxIter;
  }
};

// The diagonal preconditioner of the mass-preconditioned COCG:
// m = 1/M_eps,c per free edge (0 on masked edges) -- the square of the
// symmetric scaling S, from the same per-edge rule as the operator.
template <class T>
__global__ void __launch_bounds__(256)
    mass_inverse_kernel(GridView g, double omega, T* m_out) {
  __shared__ MatLds<double> mat;
  fill_mat_mode<double>(mat, g.mats, omega, MODE_MEC);
  const cx<double> pc = port_coef_mode<double>(omega, MODE_MEC);
  __syncthreads();
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < g.np;
       n += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(n % g.nx);
    const int j = (int)((n / g.nx) % g.ny);
    const int k = (int)(n / ((int64_t)g.nx * g.ny));
    const ColGeo<double> cg = col_geo<double>(g, i, j);
    const PlaneRec<double> lo = plane_rec(mat, cg, load_cell_ids(g, i, j, k - 1));
    const PlaneRec<double> hi = plane_rec(mat, cg, load_cell_ids(g, i, j, k));
    const ZGeo<double> zg = zgeo<double>(g, k);
    const NodeCoef<double> nc = node_coef(cg, lo, hi, zg.hzl, zg.hzh, zg.ivz, k, pc);
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      cx<T> mv{T(0), T(0)};
      if ((nc.mask >> w) & 1u) {
        const cx<double> me = nc.e[w];
        const double m2 = cabs2(me);
        mv = cx<T>{(T)(me.re / m2), (T)(-me.im / m2)};
      }
      stc(m_out, 3 * n + w, mv);
    }
  }
}

// Mass-preconditioned COCG step 2: x += alpha p, r -= alpha q, z = m .* r,
// r^T z and ||r||^2.  COCG preconditioned by S^2 produces the iterates of
// COCG on S A S while the operator itself runs unscaled.  INIT: only
// z = m .* r and the sums.
template <class T, bool INIT>
__device__ __forceinline__ void pcocg_update_body(int64_t n, T* x, T* r, T* z, const T* p,
                                                  const T* q, const T* m, CgState* st,
                                                  double* part, int bid, int nblk) {
  __shared__ double lds[3 * 4];
  const cx<T> al{(T)st->alpha.re, (T)st->alpha.im};
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t e = (int64_t)bid * blockDim.x + threadIdx.x; e < n; e += (int64_t)nblk * blockDim.x) {
    cx<T> rv = ldc(r, e);
    if (!INIT) {
      stc(x, e, ldc(x, e) + al * ldc(p, e));
      rv = rv - al * ldc(q, e);
      stc(r, e, rv);
    }
    const cx<T> zv = ldc(m, e) * rv;
    stc(z, e, zv);
    const double rr = rv.re, ri = rv.im, zr = zv.re, zi = zv.im;
    acc[0] += rr * zr - ri * zi;
    acc[1] += rr * zi + ri * zr;
    acc[2] += rr * rr + ri * ri;
  }
  block_partial_at<3>(acc, part, lds, bid);
}

template <class T, bool INIT>
__global__ void __launch_bounds__(256)
    pcocg_update_kernel(int64_t n, T* x, T* r, T* z, const T* p, const T* q, const T* m,
                        CgState* st, double* part) {
  if (*(volatile int*)&st->done != kRunning) return;
  pcocg_update_body<T, INIT>(n, x, r, z, p, q, m, st, part, blockIdx.x, gridDim.x);
}

// The same step with the preconditioner diagonal recomputed instead of read:
// m = -omega^2 / d_e from the cell ids, the material table and the 1-D
// widths, by the same expression the fused operator kernel uses for
// p = m .* r + beta p (OpCocgPX::input_coef), so both kernels apply the same
// M.  This drops the stored m vector (one of four vector passes) from the
// kernel.  Layout: a thread owns one node column (i, j) and marches up a
// chunk of `zc` planes, reusing the column geometry and the lower plane's
// cell record; consecutive threads are consecutive columns, so every plane's
// loads and stores are contiguous.  Blocks loop over (column block, z-chunk)
// pairs; block b writes partial b.
template <class T, int ZC>
__device__ __forceinline__ void pcocg_rupdate_otf_body(const GridView& g, double omega, T* r, const T* q,
                                                       CgState* st, double* part, int bid, int nblk) {
  __shared__ MatLds<T> mat;
  __shared__ double lds[3 * 4];
  fill_mat_mode<T>(mat, g.mats, omega, MODE_D);
  __syncthreads();
  const cx<T> al{(T)st->alpha.re, (T)st->alpha.im};
  const cx<T> pc = port_coef_mode<T>(omega, MODE_D);
  const T w2 = (T)(omega * omega);
  const int ncol = g.nx * g.ny;
  const int nbxy = (ncol + 255) / 256, nbz = (g.nz + ZC - 1) / ZC;
  double acc[3] = {0.0, 0.0, 0.0};
  // items run from the top z-chunk down: the operator step before this
  // kernel finishes with the top planes (its tiles run bottom to top), so
  // their r and q are still in the last-level cache, and this kernel ends
  // at the bottom planes, where the next operator step starts reading r
  for (int it = bid; it < nbxy * nbz; it += nblk) {
    const int ch = nbxy * nbz - 1 - it;
    const int c = (ch % nbxy) * 256 + (int)threadIdx.x;
    if (c >= ncol) continue;
    const int k0 = (ch / nbxy) * ZC, k1 = min(k0 + ZC, g.nz);
    const int j = c / g.nx, i = c - j * g.nx;
    // every load of the chunk is issued before any is used (planes past the
    // grid re-read the last plane and are not stored)
    cx<T> rv[ZC][3], qv[ZC][3];
    CellIdsRaw ids[ZC + 1];
    ids[0] = load_cell_ids_raw_inrange(g, i, j, k0 - 1);
#pragma unroll
    for (int u = 0; u < ZC; ++u) {
      const int k = min(k0 + u, k1 - 1);
      const int64_t n = (int64_t)k * ncol + c;
      ids[u + 1] = load_cell_ids_raw_inrange(g, i, j, k);
#pragma unroll
      for (int w = 0; w < 3; ++w) {
        rv[u][w] = ldc(r, 3 * n + w);
        qv[u][w] = ldc(q, 3 * n + w);
      }
    }
    const ColGeo<T> cg = col_geo<T>(g, i, j);
    PlaneRec<T> lo = plane_rec(mat, cg, decode_cell_ids(ids[0]));
#pragma unroll
    for (int u = 0; u < ZC; ++u) {
      const int k = k0 + u;
      if (k >= k1) break;
      const PlaneRec<T> hi = plane_rec(mat, cg, decode_cell_ids(ids[u + 1]));
      const ZGeo<T> z = zgeo_raw<T>(g, k);
      const NodeCoef<T> nc = node_coef(cg, lo, hi, z.hzl, z.hzh, z.ivz, k, pc);
      lo = hi;
      const int64_t n = (int64_t)k * ncol + c;
#pragma unroll
      for (int w = 0; w < 3; ++w) {
        const cx<T> d = nc.e[w];
        const bool fr = (nc.mask >> w) & 1u;
        const T a2 = fr ? d.re * d.re + d.im * d.im : T(1);
        const T f = fr ? -w2 / a2 : T(0);
        const cx<T> m{f * d.re, -f * d.im};
        const cx<T> rn = rv[u][w] - al * qv[u][w];
        stc(r, 3 * n + w, rn);
        const cx<T> zv = m * rn;
        const double rr = rn.re, ri = rn.im, zr = zv.re, zi = zv.im;
        acc[0] += rr * zr - ri * zi;
        acc[1] += rr * zi + ri * zr;
        acc[2] += rr * rr + ri * ri;
      }
    }
  }
  block_partial_at<3>(acc, part, lds, bid);
}

template <class T, int ZC>
__global__ void __launch_bounds__(256)
    pcocg_rupdate_otf_kernel(GridView g, double omega, T* r, const T* q, CgState* st, double* part) {
  if (*(volatile int*)&st->done != kRunning) return;
  pcocg_rupdate_otf_body<T, ZC>(g, omega, r, q, st, part, blockIdx.x, gridDim.x);
}

// The same for several systems (possibly on different grids) in one launch:
// item s owns the blocks [block0, block0 + nblk).
template <class T>
struct OtfItem {
  GridView g;
  double omega;
  T* r;
  const T* q;
  CgState* st;
  double* part;
  int block0, nblk;
};

template <class T, int ZC>
__global__ void __launch_bounds__(256)
    pcocg_rupdate_otf_multi_kernel(const OtfItem<T>* __restrict__ items, int nitems) {
  const int b = blockIdx.x;
  int lo = 0, hi = nitems - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].block0 <= b) lo = mid; else hi = mid - 1;
  }
  const OtfItem<T>& it = items[lo];
  if (*(volatile int*)&it.st->done != kRunning) return;
  pcocg_rupdate_otf_body<T, ZC>(it.g, it.omega, it.r, it.q, it.st, it.part, b - it.block0, it.nblk);
}

// Launch shape of pcocg_rupdate_otf_kernel: z-chunk and block count (at
// most max_blocks partials).
struct OtfShape {
  int zc, blocks;
};
constexpr int kOtfZc = 2;
inline OtfShape otf_shape(const GridView& g, int max_blocks) {
  const int zc = kOtfZc;
  const int64_t nbxy = ((int64_t)g.nx * g.ny + 255) / 256, nbz = (g.nz + zc - 1) / zc;
  const int64_t b = nbxy * nbz;
  return OtfShape{zc, (int)(b < max_blocks ? b : max_blocks)};
}

// The solution update still pending after the last fused step.
template <class T>
__global__ void __launch_bounds__(256)
    cocg_fixup_kernel(int64_t n, T* x, const T* p0, const T* p1, CgState* st) {
  if (!*(volatile int*)&st->pend) return;
  const cx<T> al{(T)st->alpha.re, (T)st->alpha.im};
  const T* p = st->pbuf ? p1 : p0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    stc(x, e, ldc(x, e) + al * ldc(p, e));
}

// Initial scalars of the mass-preconditioned COCG: rho = r^T z, ||r||^2.
struct PcocgInitFinish {
  CgState* st;
  __device__ bool skip() const { return false; }
  __device__ void operator()(const double* sum) const {
    st->rho = cx<double>{sum[0], sum[1]};
    st->rr = sum[2];
    st->beta = cx<double>{0.0, 0.0};
    if (!isfinite(sum[0]) || !isfinite(sum[1]) || !isfinite(sum[2])) st->done = kNan;
  }
};

// <a, b> (or the bilinear a^T b), ||a||^2, ||b||^2 -> out->v[0..3].
template <class T, bool BILINEAR = false>
__global__ void __launch_bounds__(256)
    dot_kernel(const T* a, const T* b, int64_t n, RedOut* out, double* part, unsigned* cnt) {
  __shared__ double lds[4 * 4];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const cx<T> av = ldc(a, e), bv = ldc(b, e);
    const cx<double> d = BILINEAR ? cdotc_d(cx<T>{av.re, -av.im}, bv) : cdotc_d(av, bv);
    acc[0] += d.re;
    acc[1] += d.im;
    acc[2] += cabs2_d(av);
    acc[3] += cabs2_d(bv);
  }
  block_partial<4>(acc, part, lds);
  (void)cnt;
  (void)out;
}

// v_j = w * vscale (FGMRES keeps the normalised vector for the preconditioner).
template <class T>
__global__ void __launch_bounds__(256)
    gm_normalize_kernel(const T* w, T* v, int64_t n, const GmState* st) {
  if (*(volatile const int*)&st->done != kRunning) return;
  const T sc = (T)st->vscale;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    stc(v, e, sc * ldc(w, e));
}

// Re-arm the state after a completed cycle so the restart's operator
// application runs.
static __global__ void gm_restart_prep_kernel(GmState* st) {
  if (threadIdx.x == 0) st->done = kRunning;
}

// w = r0 - w, ||w||^2.
template <class T>
__global__ void __launch_bounds__(256)
    sub_norm_kernel(const T* r0, T* w, int64_t n, RedOut* out, double* part, unsigned* cnt) {
  __shared__ double lds[4];
  double acc[1] = {0.0};
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const cx<T> v = ldc(r0, e) - ldc(w, e);
    stc(w, e, v);
    acc[0] += cabs2_d(v);
  }
  block_partial<1>(acc, part, lds);
  (void)cnt;
  (void)out;
}

}  // namespace fit

// The matrix-free FIT operator as one fused gfx950 kernel.
//
// y = C^T M_nu C x + d(omega) .* x            (FIT_SCALE_NONE, eq. (e2) + losses)
// y = S C^T M_nu C S x - omega^2 x            (FIT_SCALE_SYM,  eqs. (e2s)/(e2t))
//
// The paper applies this operator as five nested primitives that reuse two
// buffers (Sec. III, eq. (e2t)).  Here the whole chain runs in registers and
// LDS without any intermediate vector in HBM: per node it forms the three
// primal-facet fluxes b = C x, scales them by the reluctance of the dual edge
// through each facet, and gathers C^T h back onto the node's three edges.
// Every material coefficient, the PEC/wall mask and the optional symmetric
// scaling are recomputed from the 1-byte cell material ids and the 1-D cell
// widths (Sec. II: permittivity averaged over the dual facet, permeability
// along the dual edge); nothing per edge is stored.
//
// Data movement (MI355X design):
//  * A workgroup owns a TX x TY tile of node columns and marches up a chunk of
//    ZC z-planes.  Lanes run along x, so each plane row is one coalesced
//    48-byte-per-lane (c128) / 24-byte (c64) read; the node records of the
//    paper's (x, y, z)-interleaved layout are consumed whole.
//  * One x-plane (tile + 1-node halo ring) lives in LDS; the facets of the
//    current plane live in LDS for the -x/-y neighbours; the own column's
//    facets of the previous plane stay in registers; the next plane is
//    prefetched into registers one step ahead.
//  * Each z-chunk recomputes one plane of facets below it (warm-up), so HBM
//    reads per node are 1 + 1/ZC plus the halo ring, which neighbouring tiles
//    scheduled on the same XCD mostly find in L2 (XCD-aware block order).
//  * Krylov vector updates and reductions are fused through the Op policy:
//    the input may be produced on the fly from several vectors (and written
//    back for owned nodes), and the output may feed fused dot products.
#pragma once

#include "fit_internal.h"
#include "profile.h"
#include "reduce.h"

namespace fit {

enum CoefMode { MODE_D = 0, MODE_MEC = 1, MODE_EPS = 2, MODE_SIGMA = 3 };

template <class T>
__device__ __forceinline__ void fill_mat_mode(MatLds<T>& m, const MatEntry* mats, double omega,
                                              int mode) {
  for (int id = threadIdx.x; id < 256; id += blockDim.x) {
    MatEntry e = mats[id];
    double cre = 0.0, cim = 0.0;
    if (mode == MODE_D) {
      cre = -omega * omega * e.eps;
      cim = omega * omega * e.eps_tand + omega * e.sigma;
    } else if (mode == MODE_MEC) {
      cre = e.eps;
      cim = omega > 0.0 ? -(e.eps_tand + e.sigma / omega) : 0.0;
    } else if (mode == MODE_EPS) {
      cre = e.eps;
      cim = -e.eps_tand;
    } else {
      cre = e.sigma;
    }
    m.coef[id] = cx<T>{(T)cre, (T)cim};
    m.imu[id] = (T)e.inv_mu;
    m.flg[id] = e.flags;
  }
}

template <class T>
__host__ __device__ __forceinline__ cx<T> port_coef_mode(double omega, int mode) {
  if (mode == MODE_D) return cx<T>{T(0), (T)omega};
  if (mode == MODE_MEC) return cx<T>{T(0), omega > 0.0 ? (T)(-1.0 / omega) : T(0)};
  if (mode == MODE_SIGMA) return cx<T>{T(1), T(0)};
  return cx<T>{T(0), T(0)};
}

// Map the hardware workgroup id (dispatched round-robin over the 8 XCDs)
// to a logical tile so that consecutive logical tiles -- neighbours in y,
// which share halo rows -- run on the same XCD and its L2.
__device__ __forceinline__ int xcd_remap(int bid, int nblk) {
  constexpr int kXcd = 8;
  const int xcd = bid % kXcd, idx = bid / kXcd;
  const int q = nblk / kXcd, r = nblk % kXcd;
  return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

struct StencilLaunch {
  int nbx, nby, nbz, zc;
  double omega;
  int xcd_aware;
};

template <class T>
struct C3 {
  cx<T> c[3];
};

// Per-plane geometry of z-plane p (uniform over the workgroup).
template <class T>
struct ZGeo {
  T hzl, hzh, ivz;
};
template <class T>
__device__ __forceinline__ ZGeo<T> zgeo(const GridView& g, int p) {
  const GeoArrays<T>& a = g.geo<T>();
  ZGeo<T> z;
  if (p >= 0 && p < g.nz) {
    z.hzl = a.hhz[p];
    z.hzh = a.hhz[p + 1];
    z.ivz = a.ivz[p];
  } else {
    z.hzl = z.hzh = z.ivz = T(0);
  }
  return z;
}

// Result of staging one node: the masked input, the staged (scaled) input,
// the diagonal or scaling coefficients and the facet reluctances.
template <class T>
struct Staged {
  cx<T> xr[3];  // masked input value
  cx<T> xs[3];  // value that enters the curl: xr (NONE) or s .* xr (SYM)
  cx<T> cf[3];  // d (NONE) or s (SYM); 0 on masked edges
  T nu[3];
  uint32_t mask;
};

// A halo node only feeds the curl: its staged value and facet reluctances.
template <class T>
struct HaloStaged {
  cx<T> xs[3];
  T nu[3];
};

template <class T, int MODE>
__device__ __forceinline__ void stage_halo(HaloStaged<T>& st, const cx<T> (&xin)[3],
                                           const NodeCoef<T>& nc) {
#pragma unroll
  for (int w = 0; w < 3; ++w) {
    const bool fr = (nc.mask >> w) & 1u;
    cx<T> xv = fr ? xin[w] : cx<T>{T(0), T(0)};
    if (MODE == MODE_MEC) xv = fr ? crsqrt(nc.e[w]) * xv : xv;
    st.xs[w] = xv;
    st.nu[w] = nc.nu[w];
  }
}

template <class T, int MODE>
__device__ __forceinline__ void stage_node(Staged<T>& st, const cx<T> (&xin)[3],
                                           const NodeCoef<T>& nc) {
#pragma unroll
  for (int w = 0; w < 3; ++w) {
    const bool fr = (nc.mask >> w) & 1u;
    cx<T> xv = fr ? xin[w] : cx<T>{T(0), T(0)};
    st.xr[w] = xv;
    if (MODE == MODE_MEC) {
      cx<T> s = fr ? crsqrt(nc.e[w]) : cx<T>{T(0), T(0)};
      st.cf[w] = s;
      st.xs[w] = s * xv;
    } else {
      st.cf[w] = fr ? nc.e[w] : cx<T>{T(0), T(0)};
      st.xs[w] = xv;
    }
    st.nu[w] = nc.nu[w];
  }
  st.mask = nc.mask;
}

// ---------------------------------------------------------------------------
// The kernel.  Op policy interface:
//   struct Raw;                                     per-node prefetched data
//   static constexpr int NRED;                      doubles reduced over the grid
//   bool skip() const;                              early exit (solver done)
//   void begin();                                   read device scalars
//   void load(int64_t node, Raw&) const;            global loads of one node
//   void zero(Raw&) const;
//   void input(const Raw&, cx<T> (&xin)[3]) const;  operator input at the node
//   void own_input(int64_t node, const cx<T> (&xin)[3]) const;   (owned nodes)
//   void consume(int64_t node, const cx<T> (&y)[3], const cx<T> (&xr)[3],
//                double* acc) const;                output at owned nodes
//   void finalize(const double* sums) const;        thread 0 of the last block
// ---------------------------------------------------------------------------
template <class T, int TX, int TY, int MODE, class Op>
__global__ void __launch_bounds__(TX* TY)
    stencil_kernel(GridView g, StencilLaunch L, Op op) {
  constexpr int NT = TX * TY;
  constexpr int NH = 2 * TX + 2 * TY + 2;
  static_assert(NH <= NT, "one halo node per thread");
  static_assert(NT % 64 == 0, "whole wavefronts");
  constexpr bool SYM = (MODE == MODE_MEC);
  constexpr int NR = Op::NRED > 0 ? Op::NRED : 1;

  if (op.skip()) return;
  op.begin();

  __shared__ MatLds<T> mat;
  __shared__ cx<T> X[3][TY + 2][TX + 2];
  __shared__ cx<T> H[3][TY + 1][TX + 1];
  __shared__ double red_lds[NR * (NT / 64)];

  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;
  const int nblk = gridDim.x;
  const int lb = L.xcd_aware ? xcd_remap(blockIdx.x, nblk) : (int)blockIdx.x;
  const int bx = lb % L.nbx;
  const int rest = lb / L.nbx;
  const int by = rest % L.nby;
  const int bz = rest / L.nby;
  const int i0 = bx * TX, j0 = by * TY;
  const int kb = bz * L.zc;
  const int ke = min(kb + L.zc, g.nz);
  const int ks = kb > 0 ? kb - 1 : 0;

  fill_mat_mode<T>(mat, g.mats, L.omega, MODE);
  const cx<T> pcoef = port_coef_mode<T>(L.omega, MODE);
  const T w2 = (T)(L.omega * L.omega);

  // ---- slot 0: the owned node column --------------------------------------
  const int i_0 = i0 + tx, j_0 = j0 + ty;
  const bool in0 = (i_0 < g.nx) && (j_0 < g.ny);
  const ColGeo<T> cg0 = col_geo<T>(g, i_0, j_0);
  const int64_t col0 = (int64_t)j_0 * g.nx + i_0;

  // ---- slot 1: one node of the halo ring (none for some threads) ---------
  int hx1 = -1, hy1 = -1;
  if (tid < NH) {
    int h = tid;
    if (h < TX) {
      hx1 = h + 1; hy1 = 0;                // row below the tile
    } else if ((h -= TX) < TY) {
      hx1 = 0; hy1 = h + 1;                // column left of the tile
    } else if ((h -= TY) < TX) {
      hx1 = h + 1; hy1 = TY + 1;           // row above
    } else if ((h -= TX) < TY) {
      hx1 = TX + 1; hy1 = h + 1;           // column right
    } else if ((h -= TY) == 0) {
      hx1 = TX + 1; hy1 = 0;               // corner (+x, -y)
    } else {
      hx1 = 0; hy1 = TY + 1;               // corner (-x, +y)
    }
  }
  const bool has1 = hx1 >= 0;
  const int i_1 = i0 + hx1 - 1, j_1 = j0 + hy1 - 1;
  const bool in1 = has1 && i_1 >= 0 && j_1 >= 0 && i_1 < g.nx && j_1 < g.ny;
  const ColGeo<T> cg1 = col_geo<T>(g, max(i_1, 0), max(j_1, 0));
  const int64_t col1 = (int64_t)max(j_1, 0) * g.nx + max(i_1, 0);

  auto cell_ids = [&](bool inb, int i, int j, int p) -> uint32_t {
    return inb ? load_cell_ids(g, i, j, p) : 0xFFFFFFFFu;
  };
  auto node_of = [&](int64_t col, int p) -> int64_t { return col + (int64_t)p * g.nx * g.ny; };

  __syncthreads();  // material table ready

  // plane records of plane ks-1 (the "lo" plane of the first staged plane)
  PlaneRec<T> lo0 = plane_rec(mat, cg0, cell_ids(in0, i_0, j_0, ks - 1));
  PlaneRec<T> lo1 = plane_rec(mat, cg1, cell_ids(in1, i_1, j_1, ks - 1));

  Staged<T> s0c, s0n;
  HaloStaged<T> s1c, s1n;
  typename Op::Raw raw0, raw1;
  uint32_t ids0, ids1;

  auto fetch = [&](int q) {
    const bool ok = q < g.nz && q <= ke;
    if (in0 && ok) op.load(node_of(col0, q), raw0); else op.zero(raw0);
    if (in1 && ok) op.load(node_of(col1, q), raw1); else op.zero(raw1);
    ids0 = cell_ids(in0 && q < g.nz, i_0, j_0, q);
    ids1 = cell_ids(in1 && q < g.nz, i_1, j_1, q);
  };
  auto process = [&](int q, Staged<T>& d0, HaloStaged<T>& d1) {
    const ZGeo<T> z = zgeo<T>(g, q);
    PlaneRec<T> hi0 = plane_rec(mat, cg0, ids0);
    NodeCoef<T> nc0 = node_coef(cg0, lo0, hi0, z.hzl, z.hzh, z.ivz, q, pcoef);
    lo0 = hi0;
    cx<T> xin[3];
    op.input(raw0, xin);
    stage_node<T, MODE>(d0, xin, nc0);
    if (in0 && q >= kb && q < ke) op.own_input(node_of(col0, q), d0.xr);
    if (has1) {
      PlaneRec<T> hi1 = plane_rec(mat, cg1, ids1);
      NodeCoef<T> nc1 = node_coef(cg1, lo1, hi1, z.hzl, z.hzh, z.ivz, q, pcoef);
      lo1 = hi1;
      op.input(raw1, xin);
      stage_halo<T, MODE>(d1, xin, nc1);
    }
  };
  auto put_x = [&](const Staged<T>& d0, const HaloStaged<T>& d1) {
#pragma unroll
    for (int w = 0; w < 3; ++w) X[w][ty + 1][tx + 1] = d0.xs[w];
    if (has1) {
#pragma unroll
      for (int w = 0; w < 3; ++w) X[w][hy1][hx1] = d1.xs[w];
    }
  };

  // ---- prologue: stage planes ks and ks+1, prefetch ks+2 -----------------
  fetch(ks);
  process(ks, s0c, s1c);
  fetch(ks + 1);
  process(ks + 1, s0n, s1n);
  put_x(s0c, s1c);
  fetch(ks + 2);
  __syncthreads();

  double acc[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) acc[q] = 0.0;
  cx<T> hpx = {T(0), T(0)}, hpy = {T(0), T(0)};  // own facets of the plane below

  for (int k = ks; k < ke; ++k) {
    // ---- C: facets of plane k ---------------------------------------------
    cx<T> hx, hy, hz;
    {
      const cx<T> xz_jp = X[2][ty + 2][tx + 1], xx_jp = X[0][ty + 2][tx + 1];
      const cx<T> xz_ip = X[2][ty + 1][tx + 2], xy_ip = X[1][ty + 1][tx + 2];
      hx = s0c.nu[0] * (xz_jp - s0c.xs[2] - s0n.xs[1] + s0c.xs[1]);
      hy = s0c.nu[1] * (s0n.xs[0] - s0c.xs[0] - xz_ip + s0c.xs[2]);
      hz = s0c.nu[2] * (xy_ip - s0c.xs[1] - xx_jp + s0c.xs[0]);
      H[0][ty + 1][tx + 1] = hx;
      H[1][ty + 1][tx + 1] = hy;
      H[2][ty + 1][tx + 1] = hz;
    }
    if (tid < TX) {
      // facets (x, z) of node (i0+tid, j0-1): needed by the tile's first row
      const cx<T> hxh = s1c.nu[0] * (X[2][1][tx + 1] - s1c.xs[2] - s1n.xs[1] + s1c.xs[1]);
      const cx<T> hzh = s1c.nu[2] * (X[1][0][tx + 2] - s1c.xs[1] - X[0][1][tx + 1] + s1c.xs[0]);
      H[0][0][tx + 1] = hxh;
      H[2][0][tx + 1] = hzh;
    } else if (tid < TX + TY) {
      // facets (y, z) of node (i0-1, j0+t): needed by the tile's first column
      const int t = tid - TX;
      const cx<T> hyh = s1c.nu[1] * (s1n.xs[0] - s1c.xs[0] - X[2][t + 1][1] + s1c.xs[2]);
      const cx<T> hzh = s1c.nu[2] * (X[1][t + 1][1] - s1c.xs[1] - X[0][t + 2][0] + s1c.xs[0]);
      H[1][t + 1][0] = hyh;
      H[2][t + 1][0] = hzh;
    }
    __syncthreads();

    // ---- E: gather C^T h onto the owned node's edges ----------------------
    if (k >= kb) {
      cx<T> y[3];
      y[0] = hpy - hy + hz - H[2][ty][tx + 1];
      y[1] = H[2][ty + 1][tx] - hz + hx - hpx;
      y[2] = H[0][ty][tx + 1] - hx + hy - H[1][ty + 1][tx];
#pragma unroll
      for (int w = 0; w < 3; ++w) {
        cx<T> v;
        if (SYM) {
          v = s0c.cf[w] * y[w] - w2 * s0c.xr[w];
        } else {
          v = y[w] + s0c.cf[w] * s0c.xr[w];
        }
        y[w] = ((s0c.mask >> w) & 1u) ? v : cx<T>{T(0), T(0)};
      }
      if (in0) op.consume(node_of(col0, k), y, s0c.xr, acc);
    }
    hpx = hx;
    hpy = hy;

    // ---- advance: plane k+1 into LDS, stage k+2, prefetch k+3 -------------
    put_x(s0n, s1n);
    s0c = s0n;
    s1c = s1n;
    process(k + 2, s0n, s1n);
    fetch(k + 3);
    __syncthreads();
  }

  if (Op::NRED > 0) block_partial<NR>(acc, op.partials(), red_lds);
}

// Finish functor: hands the grid-wide sums of an Op's reductions to its
// finalize step (one thread), unless the Op skipped.
template <class Op>
struct OpFinish {
  Op op;
  __device__ bool skip() const { return op.skip(); }
  __device__ void operator()(const double* s) const { op.finalize(s); }
};

// Launch geometry for a grid and tile shape.
struct TileShape {
  int tx, ty, zc;
};

inline StencilLaunch make_launch(const GridView& g, TileShape t, double omega, bool xcd = true) {
  StencilLaunch L;
  L.nbx = (g.nx + t.tx - 1) / t.tx;
  L.nby = (g.ny + t.ty - 1) / t.ty;
  L.zc = t.zc;
  L.nbz = (g.nz + t.zc - 1) / t.zc;
  L.omega = omega;
  L.xcd_aware = xcd ? 1 : 0;
  return L;
}

inline int launch_blocks(const StencilLaunch& L) { return L.nbx * L.nby * L.nbz; }

// Tile shapes compiled into the library.  Every shape keeps a whole number of
// 64-lane wavefronts and room for one halo node per thread.
inline bool tile_supported(TileShape t) {
  return t.zc >= 1 && ((t.tx == 64 && (t.ty == 4 || t.ty == 8)) || (t.tx == 32 && t.ty == 8));
}

// Kernel-family name of an Op for the launch profiler.
template <class Op>
struct OpName {
  static const char* get() { return "stencil"; }
};

template <class T, int MODE, class Op>
fit_status launch_stencil(const GridView& g, TileShape t, double omega, const Op& op,
                          hipStream_t s) {
  if (!tile_supported(t)) {
    set_error("unsupported stencil tile shape");
    return FIT_E_INVALID;
  }
  const StencilLaunch L = make_launch(g, t, omega);
  const dim3 grid((unsigned)launch_blocks(L));
  const int tok = prof_begin(s);
  if (t.tx == 64 && t.ty == 4)
    hipLaunchKernelGGL((stencil_kernel<T, 64, 4, MODE, Op>), grid, dim3(256), 0, s, g, L, op);
  else if (t.tx == 64 && t.ty == 8)
    hipLaunchKernelGGL((stencil_kernel<T, 64, 8, MODE, Op>), grid, dim3(512), 0, s, g, L, op);
  else
    hipLaunchKernelGGL((stencil_kernel<T, 32, 8, MODE, Op>), grid, dim3(256), 0, s, g, L, op);
  FIT_HIP(hipGetLastError());
  prof_end(tok, s, OpName<Op>::get());
  if constexpr (Op::NRED > 0) {
    FIT_HIP(launch_finish<Op::NRED>(op.partials(), (int)grid.x, OpFinish<Op>{op}, s));
  }
  return FIT_OK;
}

// ---------------------------------------------------------------------------
// Plain operator application: y = A x.
// ---------------------------------------------------------------------------
template <class T>
struct OpMatvec {
  const T* x;
  T* y;
  struct Raw {
    cx<T> v[3];
  };
  static constexpr int NRED = 0;
  __device__ bool skip() const { return false; }
  __device__ void begin() {}
  __device__ void load(int64_t n, Raw& r) const {
#pragma unroll
    for (int w = 0; w < 3; ++w) r.v[w] = ldc(x, 3 * n + w);
  }
  __device__ void zero(Raw& r) const {
#pragma unroll
    for (int w = 0; w < 3; ++w) r.v[w] = {T(0), T(0)};
  }
  __device__ void input(const Raw& r, cx<T> (&xin)[3]) const {
#pragma unroll
    for (int w = 0; w < 3; ++w) xin[w] = r.v[w];
  }
  __device__ void own_input(int64_t, const cx<T> (&)[3]) const {}
  __device__ void consume(int64_t n, const cx<T> (&yv)[3], const cx<T> (&)[3], double*) const {
#pragma unroll
    for (int w = 0; w < 3; ++w) stc(y, 3 * n + w, yv[w]);
  }
  __host__ __device__ double* partials() const { return nullptr; }
  __device__ unsigned* counter() const { return nullptr; }
  __device__ void finalize(const double*) const {}
};
template <class T>
struct OpName<OpMatvec<T>> {
  static const char* get() { return "matvec"; }
};

}  // namespace fit

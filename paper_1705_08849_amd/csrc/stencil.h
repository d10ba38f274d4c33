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
//  * A workgroup of BX x BY threads covers a BX x BY block of node columns:
//    the (BX-2) x (BY-2) columns it outputs plus a one-node halo ring.  It
//    marches up a chunk of ZC z-planes.  Each thread owns exactly one column:
//    it stages that node of every plane (load, mask, material coefficients),
//    the tile and its low ring compute their three facet fluxes, and the
//    tile gathers C^T h onto its edges.  Lanes run along x, so every plane
//    row is one coalesced read of whole (x, y, z)-interleaved node records.
//  * The current x-plane and the current facets live in LDS; the own
//    column's facets of the plane below stay in registers; the next plane is
//    staged in registers one step ahead and its raw data prefetched two.
//  * Each z-chunk recomputes one plane of facets below it (warm-up), so HBM
//    reads per node are (1 + 1/ZC) times the block's halo overhead, which
//    neighbouring tiles mostly find in L2 or the last-level cache.
//    Single-system launches run the tiles in plain order (consecutive tiles
//    round-robin over the XCDs, so the whole device works on one compact
//    band of the grid, which measured faster than giving each XCD its own
//    contiguous range); so do the multi-system launches of a sweep, while
//    the batched operator (one grid, several vectors) uses the XCD-aware
//    order below.
//  * Krylov vector updates and reductions are fused through the Op policy:
//    the input may be produced on the fly from several vectors (and written
//    back for owned nodes), and the output may feed fused dot products.
#pragma once

#include <type_traits>

#include "fit_internal.h"
#include "profile.h"
#include "reduce.h"

namespace fit {

// MODE_D: unscaled operator (staged diagonal d); MODE_MEC: symmetric scaling
// (staged s = M_eps,c^{-1/2}); MODE_FACT: the same scaled operator evaluated
// in the factorized order of eq. (e2tt), calA^T (calA x) - omega^2 x with
// calA = M_mu^{-1/2} C M_eps,c^{-1/2} (each facet flux is scaled by
// sqrt(M_nu) on the way out of the curl and again on the way back).
enum CoefMode { MODE_D = 0, MODE_MEC = 1, MODE_EPS = 2, MODE_SIGMA = 3, MODE_FACT = 4 };

template <class T>
__device__ __forceinline__ void fill_mat_mode(MatLds<T>& m, const MatEntry* mats, double omega,
                                              int mode) {
  for (int id = threadIdx.x; id < 256; id += blockDim.x) {
    MatEntry e = mats[id];
    double cre = 0.0, cim = 0.0;
    if (mode == MODE_D) {
      cre = -omega * omega * e.eps;
      cim = omega * omega * e.eps_tand + omega * e.sigma;
    } else if (mode == MODE_MEC || mode == MODE_FACT) {
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
  if (mode == MODE_MEC || mode == MODE_FACT)
    return cx<T>{T(0), omega > 0.0 ? (T)(-1.0 / omega) : T(0)};
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

// Largest z-chunk a block marches (its planes' z-geometry sits in LDS).
constexpr int kMaxZChunk = 128;

struct StencilLaunch {
  int nbx, nby, nbz, zc;
  double omega;
  int xcd_aware;
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

// The same values for an in-range plane 0 <= p < nz, loaded without a branch.
template <class T>
__device__ __forceinline__ ZGeo<T> zgeo_raw(const GridView& g, int p) {
  const GeoArrays<T>& a = g.geo<T>();
  return ZGeo<T>{a.hhz[p], a.hhz[p + 1], a.ivz[p]};
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

template <class T, int MODE>
__device__ __forceinline__ void stage_node(Staged<T>& st, const cx<T> (&xin)[3],
                                           const NodeCoef<T>& nc) {
#pragma unroll
  for (int w = 0; w < 3; ++w) {
    const bool fr = (nc.mask >> w) & 1u;
    cx<T> xv = fr ? xin[w] : cx<T>{T(0), T(0)};
    st.xr[w] = xv;
    if (MODE == MODE_MEC || MODE == MODE_FACT) {
      cx<T> s = fr ? crsqrt(nc.e[w]) : cx<T>{T(0), T(0)};
      st.cf[w] = s;
      st.xs[w] = s * xv;
    } else {
      st.cf[w] = fr ? nc.e[w] : cx<T>{T(0), T(0)};
      st.xs[w] = xv;
    }
    // MODE_FACT stages M_mu^{-1/2}: each facet flux is scaled by it twice
    st.nu[w] = MODE == MODE_FACT ? sqrt(nc.nu[w]) : nc.nu[w];
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
//   double* partials() const;                       block partial sums
//   void finalize(const double* sums) const;        scalar step (finish kernel)
// ---------------------------------------------------------------------------
// Ops that set kFused = true receive the node's coefficients when forming
// their input (input_coef), prefetch extra data for owned nodes (load_own)
// and see their raw data when storing owned inputs (own_input_raw).
template <class Op, class = void>
struct OpFused {
  static constexpr bool value = false;
};
template <class Op>
struct OpFused<Op, std::void_t<decltype(Op::kFused)>> {
  static constexpr bool value = Op::kFused;
};
// Ops that set kDeepPrefetch = true have each plane's loads issued two plane
// steps before the step that consumes them instead of one: both prefetch
// buffers stay live, which costs about 30 VGPRs (still two waves per SIMD in
// complex128) and keeps two planes of loads in flight per wave.
template <class Op, class = void>
struct OpDeep {
  static constexpr bool value = false;
};
template <class Op>
struct OpDeep<Op, std::void_t<decltype(Op::kDeepPrefetch)>> {
  static constexpr bool value = Op::kDeepPrefetch;
};

// Body of one workgroup: logical tile lb of the launch L on grid g.  Its
// reduction partials go to op.partials() at index lb.
template <class T, int BX, int BY, int MODE, class Op>
__device__ __forceinline__ void stencil_body(const GridView& g, const StencilLaunch& L, Op& op,
                                             int lb) {
  constexpr int TX = BX - 2, TY = BY - 2;
  constexpr int NT = BX * BY;
  static_assert(NT % 64 == 0, "whole wavefronts");
  constexpr bool SYM = (MODE == MODE_MEC || MODE == MODE_FACT);
  constexpr bool FACT = (MODE == MODE_FACT);
  constexpr int NR = Op::NRED > 0 ? Op::NRED : 1;
  // Complex128 only (in complex64 the extra registers cost a wave per SIMD,
  // which measured slower), and the fused ops keep the shallow pipeline in
  // the scaled modes, where the deep one would spill.
  constexpr bool DEEP =
      OpDeep<Op>::value && sizeof(T) == 8 && !(SYM && OpFused<Op>::value);

  op.begin();

  __shared__ MatLds<T> mat;
  // staged planes and facets, double-buffered by plane parity so that one
  // barrier per plane separates every write from its readers
  __shared__ cx<T> X[2][3][BY][BX];
  __shared__ cx<T> H[2][3][BY - 1][BX - 1];
  __shared__ double red_lds[NR * (NT / 64)];

  const int tid = threadIdx.x;
  const int tx = tid % BX, ty = tid / BX;
  const int bx = lb % L.nbx;
  const int rest = lb / L.nbx;
  const int by = rest % L.nby;
  const int bz = rest / L.nby;
  const int kb = bz * L.zc;
  const int ke = min(kb + L.zc, g.nz);
  const int ks = kb > 0 ? kb - 1 : 0;

  // this thread's node column
  const int i = bx * TX - 1 + tx, j = by * TY - 1 + ty;
  const bool inb = i >= 0 && j >= 0 && i < g.nx && j < g.ny;
  const bool facets = tx <= TX && ty <= TY;               // tile + low halo ring
  const bool owner = tx >= 1 && tx <= TX && ty >= 1 && ty <= TY && inb;  // outputs
  const int ic = max(i, 0), jc = max(j, 0);
  // loads use the nearest in-grid column (results of out-of-grid columns are
  // discarded), so the prefetch needs no branch
  const int il = min(ic, g.nx - 1), jl = min(jc, g.ny - 1);
  const int64_t col = (int64_t)jl * g.nx + il;
  const int64_t plane = (int64_t)g.nx * g.ny;

  fill_mat_mode<T>(mat, g.mats, L.omega, MODE);
  // z-geometry of the planes this block stages, uniform over the block: held
  // in LDS instead of being loaded by every thread at every plane
  __shared__ T zgeo_lds[3][kMaxZChunk + 3];
  const int qmax = min(ke, g.nz - 1);
  for (int e = tid; e <= qmax - ks; e += NT) {
    const ZGeo<T> z = zgeo_raw<T>(g, ks + e);
    zgeo_lds[0][e] = z.hzl;
    zgeo_lds[1][e] = z.hzh;
    zgeo_lds[2][e] = z.ivz;
  }
  const cx<T> pcoef = port_coef_mode<T>(L.omega, MODE);
  const T w2 = (T)(L.omega * L.omega);
  const ColGeo<T> cg = col_geo<T>(g, ic, jc);
  __syncthreads();  // material table and z-geometry ready

  PlaneRec<T> lo = plane_rec(mat, cg, inb ? load_cell_ids(g, i, j, ks - 1) : 0xFFFFFFFFu);

  // Prefetch pipeline.  fetch(q) loads plane q's vector data and cell ids
  // into one of two buffers; process(q) consumes that buffer one step later
  // (two steps with DEEP).  The buffers alternate (the loop below is unrolled
  // by two), so every load lands in registers that stay put until it is
  // consumed: no register copy -- and hence no wait on the vector memory
  // counter, which would also drain the prefetch behind it -- happens in
  // between.
  struct Pending {
    typename Op::Raw raw;
    CellIdsRaw ids;
  };
  Pending pa, pb;
  Staged<T> sn;  // the next plane (staged one step ahead)
  // the current plane: coefficients and reluctances (its staged values are in LDS)
  cx<T> cur_cf[3], cur_xr[3];
  T cur_nu[3];
  uint32_t cur_mask = 0;

  // Loads are unconditional, from a plane clamped into [0, min(ke, nz-1)];
  // process() applies the validity of the plane it stages.
  auto fetch = [&](int q, Pending& f) {
    const int qc = min(q, qmax);
    op.load(col + (int64_t)qc * plane, f.raw);
    if constexpr (OpFused<Op>::value) {
      if (owner) op.load_own(col + (int64_t)qc * plane, f.raw);
    }
    f.ids = load_cell_ids_raw_inrange(g, il, jl, qc);
  };
  auto process = [&](int q, Pending& f) {
    // planes above the chunk's last needed plane (or the grid) stage as ghosts
    const bool pin = q <= qmax;
    if (!(inb && pin)) op.zero(f.raw);
    const ZGeo<T> z = pin ? ZGeo<T>{zgeo_lds[0][q - ks], zgeo_lds[1][q - ks], zgeo_lds[2][q - ks]}
                          : ZGeo<T>{T(0), T(0), T(0)};
    const PlaneRec<T> hi = plane_rec(mat, cg, (inb && pin) ? decode_cell_ids(f.ids) : 0xFFFFFFFFu);
    const NodeCoef<T> nc = node_coef(cg, lo, hi, z.hzl, z.hzh, z.ivz, q, pcoef);
    lo = hi;
    cx<T> xin[3];
    if constexpr (OpFused<Op>::value) {
      op.input_coef(f.raw, nc, xin);
    } else {
      op.input(f.raw, xin);
    }
    stage_node<T, MODE>(sn, xin, nc);
    if (owner && q >= kb && q < ke) {
      if constexpr (OpFused<Op>::value) {
        op.own_input_raw(col + (int64_t)q * plane, f.raw, sn.xr);
      } else {
        op.own_input(col + (int64_t)q * plane, sn.xr);
      }
    }
  };
  // the staged plane becomes the current one: its values into LDS buffer b,
  // its coefficients into registers
  auto stage_lds = [&](int b) {
#pragma unroll
    for (int w = 0; w < 3; ++w) X[b][w][ty][tx] = sn.xs[w];
  };
  auto advance_regs = [&]() {
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      cur_cf[w] = sn.cf[w];
      cur_nu[w] = sn.nu[w];
      if (SYM) cur_xr[w] = sn.xr[w];
    }
    cur_mask = sn.mask;
  };

  // ---- prologue: stage planes ks and ks+1, prefetch ks+2 (and ks+3) -------
  fetch(ks, pa);
  process(ks, pa);
  stage_lds(0);
  advance_regs();
  fetch(ks + 1, pb);
  process(ks + 1, pb);
  fetch(ks + 2, pa);
  if constexpr (DEEP) fetch(ks + 3, pb);
  __syncthreads();

  double acc[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) acc[q] = 0.0;
  cx<T> hpx = {T(0), T(0)}, hpy = {T(0), T(0)};  // own facets of the plane below

  // One plane step (plane k in LDS buffer b): facets of plane k, plane k+1
  // into buffer b^1, one barrier, gather onto plane k's edges, then stage
  // plane k+2 from `use` and prefetch plane k+3 into `next` (DEEP: plane k+4
  // into `use`, while `next` still holds plane k+3 in flight).  Buffer b's
  // facets are rewritten two steps later, after the next barrier, which
  // every reader of them has passed; buffer b^1's values were last read
  // before the previous barrier.
  auto step = [&](int k, int b, Pending& use, Pending& next) {
    // ---- C: facets of plane k (tile + low halo ring) ----------------------
    cx<T> xo[3];
    cx<T> hx = {T(0), T(0)}, hy = {T(0), T(0)}, hz = {T(0), T(0)};
#pragma unroll
    for (int w = 0; w < 3; ++w) xo[w] = X[b][w][ty][tx];
    if (facets) {
      const cx<T> xz_jp = X[b][2][ty + 1][tx], xx_jp = X[b][0][ty + 1][tx];
      const cx<T> xz_ip = X[b][2][ty][tx + 1], xy_ip = X[b][1][ty][tx + 1];
      hx = cur_nu[0] * (xz_jp - xo[2] - sn.xs[1] + xo[1]);
      hy = cur_nu[1] * (sn.xs[0] - xo[0] - xz_ip + xo[2]);
      hz = cur_nu[2] * (xy_ip - xo[1] - xx_jp + xo[0]);
      if (FACT) {
        // t = calA x on the facet, then M_mu^{-1/2} t enters calA^T
        hx = cur_nu[0] * hx;
        hy = cur_nu[1] * hy;
        hz = cur_nu[2] * hz;
      }
      H[b][0][ty][tx] = hx;
      H[b][1][ty][tx] = hy;
      H[b][2][ty][tx] = hz;
    }
    stage_lds(b ^ 1);
    __syncthreads();

    // ---- E: gather C^T h onto the owned node's edges ----------------------
    if (owner && k >= kb) {
      cx<T> y[3];
      y[0] = hpy - hy + hz - H[b][2][ty - 1][tx];
      y[1] = H[b][2][ty][tx - 1] - hz + hx - hpx;
      y[2] = H[b][0][ty - 1][tx] - hx + hy - H[b][1][ty][tx - 1];
      const cx<T>* xr = SYM ? cur_xr : xo;
#pragma unroll
      for (int w = 0; w < 3; ++w) {
        cx<T> v;
        if (SYM) {
          v = cur_cf[w] * y[w] - w2 * xr[w];
        } else {
          v = y[w] + cur_cf[w] * xr[w];
        }
        y[w] = ((cur_mask >> w) & 1u) ? v : cx<T>{T(0), T(0)};
      }
      cx<T> xrv[3] = {xr[0], xr[1], xr[2]};
      op.consume(col + (int64_t)k * plane, y, xrv, acc);
    }
    hpx = hx;
    hpy = hy;

    // ---- advance: plane k+1 becomes current, stage k+2, prefetch k+3 ------
    advance_regs();
    process(k + 2, use);
    if constexpr (DEEP) {
      fetch(k + 4, use);
    } else {
      fetch(k + 3, next);
    }
  };

  int k = ks;
  for (; k + 1 < ke; k += 2) {
    step(k, 0, pa, pb);
    step(k + 1, 1, pb, pa);
  }
  if (k < ke) step(k, 0, pa, pb);

  if (Op::NRED > 0) block_partial_at<NR>(acc, op.partials(), red_lds, lb);
}

template <class T, int BX, int BY, int MODE, class Op>
__global__ void __launch_bounds__(BX* BY)
    stencil_kernel(GridView g, StencilLaunch L, Op op) {
  if (op.skip()) return;
  const int lb = L.xcd_aware ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
  stencil_body<T, BX, BY, MODE, Op>(g, L, op, lb);
}

// Several operator applications in one launch (systems of a sweep, possibly
// on different grids): item s owns the logical blocks [block0, block0+nblk),
// found from the workgroup id by binary search.
template <class Op>
struct MultiItem {
  GridView g;
  StencilLaunch L;
  Op op;
  int block0, nblk;
};

template <class T, int BX, int BY, int MODE, class Op>
__global__ void __launch_bounds__(BX* BY)
    stencil_multi_kernel(const MultiItem<Op>* __restrict__ items, int nitems) {
  const int gb = (int)blockIdx.x;  // plain order, as for single-system launches
  int lo = 0, hi = nitems - 1;
  while (lo < hi) {  // last item whose block0 <= gb
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].block0 <= gb) lo = mid; else hi = mid - 1;
  }
  Op op = items[lo].op;
  if (op.skip()) return;
  const GridView g = items[lo].g;
  const StencilLaunch L = items[lo].L;
  stencil_body<T, BX, BY, MODE, Op>(g, L, op, gb - items[lo].block0);
}

// Finish functor: hands the grid-wide sums of an Op's reductions to its
// finalize step (one thread), unless the Op skipped.
template <class Op>
struct OpFinish {
  Op op;
  __device__ bool skip() const { return op.skip(); }
  __device__ void operator()(const double* s) const { op.finalize(s); }
};

// Launch geometry: block dims (tx, ty) in node columns including the halo
// ring, so each block outputs (tx-2) x (ty-2) columns; zc planes per chunk.
struct TileShape {
  int tx, ty, zc;
};

inline StencilLaunch make_launch(const GridView& g, TileShape t, double omega, bool xcd = false) {
  StencilLaunch L;
  L.nbx = (g.nx + t.tx - 3) / (t.tx - 2);
  L.nby = (g.ny + t.ty - 3) / (t.ty - 2);
  L.zc = t.zc;
  L.nbz = (g.nz + t.zc - 1) / t.zc;
  L.omega = omega;
  L.xcd_aware = xcd ? 1 : 0;
  return L;
}

inline int launch_blocks(const StencilLaunch& L) { return L.nbx * L.nby * L.nbz; }

// Block shapes compiled into the library (whole wavefronts each).
inline bool tile_supported(TileShape t) {
  return t.zc >= 1 && t.zc <= kMaxZChunk && ((t.tx == 64 && t.ty == 8) || (t.tx == 48 && t.ty == 8) ||
                       (t.tx == 32 && t.ty == 8) || (t.tx == 32 && t.ty == 16));
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
  if (t.tx == 64)
    hipLaunchKernelGGL((stencil_kernel<T, 64, 8, MODE, Op>), grid, dim3(512), 0, s, g, L, op);
  else if (t.tx == 48)
    hipLaunchKernelGGL((stencil_kernel<T, 48, 8, MODE, Op>), grid, dim3(384), 0, s, g, L, op);
  else if (t.ty == 8)
    hipLaunchKernelGGL((stencil_kernel<T, 32, 8, MODE, Op>), grid, dim3(256), 0, s, g, L, op);
  else
    hipLaunchKernelGGL((stencil_kernel<T, 32, 16, MODE, Op>), grid, dim3(512), 0, s, g, L, op);
  FIT_HIP(hipGetLastError());
  prof_end(tok, s, OpName<Op>::get());
  if constexpr (Op::NRED > 0) {
    FIT_HIP(launch_finish<Op::NRED>(op.partials(), (int)grid.x, OpFinish<Op>{op}, s));
  }
  return FIT_OK;
}

// One launch over several systems' tiles (items on the device, `nblocks`
// logical blocks in total); every item uses the block shape (tx, ty).
template <class T, int MODE, class Op>
fit_status launch_stencil_multi(const MultiItem<Op>* items, int nitems, int nblocks, TileShape t,
                                hipStream_t s, const char* prof_name) {
  if (!tile_supported(t) || nitems < 1 || nblocks < 1) {
    set_error("unsupported batched stencil launch");
    return FIT_E_INVALID;
  }
  const dim3 grid((unsigned)nblocks);
  const int tok = prof_begin(s);
  if (t.tx == 64)
    hipLaunchKernelGGL((stencil_multi_kernel<T, 64, 8, MODE, Op>), grid, dim3(512), 0, s, items, nitems);
  else if (t.tx == 48)
    hipLaunchKernelGGL((stencil_multi_kernel<T, 48, 8, MODE, Op>), grid, dim3(384), 0, s, items, nitems);
  else if (t.ty == 8)
    hipLaunchKernelGGL((stencil_multi_kernel<T, 32, 8, MODE, Op>), grid, dim3(256), 0, s, items, nitems);
  else
    hipLaunchKernelGGL((stencil_multi_kernel<T, 32, 16, MODE, Op>), grid, dim3(512), 0, s, items, nitems);
  FIT_HIP(hipGetLastError());
  prof_end(tok, s, prof_name);
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
  static constexpr bool kDeepPrefetch = true;
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

// Several right-hand sides / frequencies on one grid in one launch:
// y_b = A(omega_b) x_b for b < n (n <= kMax); gridDim.y = n.
template <class T>
struct BatchVecs {
  static constexpr int kMax = 16;
  const T* x[kMax];
  T* y[kMax];
  double omega[kMax];
};

template <class T, int BX, int BY, int MODE>
__global__ void __launch_bounds__(BX* BY)
    stencil_batch_kernel(GridView g, StencilLaunch L, BatchVecs<T> a) {
  const int nb = (int)(gridDim.x * gridDim.y);
  const int lin = xcd_remap((int)(blockIdx.x + blockIdx.y * gridDim.x), nb);
  const int b = lin / (int)gridDim.x, lb = lin % (int)gridDim.x;
  OpMatvec<T> op{a.x[b], a.y[b]};
  StencilLaunch Lb = L;
  Lb.omega = a.omega[b];
  stencil_body<T, BX, BY, MODE, OpMatvec<T>>(g, Lb, op, lb);
}

template <class T, int MODE>
fit_status launch_stencil_batch(const GridView& g, TileShape t, const BatchVecs<T>& a, int n,
                                hipStream_t s) {
  if (!tile_supported(t) || n < 1 || n > BatchVecs<T>::kMax) {
    set_error("unsupported batched operator launch");
    return FIT_E_INVALID;
  }
  const StencilLaunch L = make_launch(g, t, a.omega[0]);
  const dim3 grid((unsigned)launch_blocks(L), (unsigned)n);
  const int tok = prof_begin(s);
  if (t.tx == 64)
    hipLaunchKernelGGL((stencil_batch_kernel<T, 64, 8, MODE>), grid, dim3(512), 0, s, g, L, a);
  else if (t.tx == 48)
    hipLaunchKernelGGL((stencil_batch_kernel<T, 48, 8, MODE>), grid, dim3(384), 0, s, g, L, a);
  else if (t.ty == 8)
    hipLaunchKernelGGL((stencil_batch_kernel<T, 32, 8, MODE>), grid, dim3(256), 0, s, g, L, a);
  else
    hipLaunchKernelGGL((stencil_batch_kernel<T, 32, 16, MODE>), grid, dim3(512), 0, s, g, L, a);
  FIT_HIP(hipGetLastError());
  prof_end(tok, s, sizeof(T) == 8 ? "matvec_batched_c128" : "matvec_batched_c64");
  return FIT_OK;
}

}  // namespace fit

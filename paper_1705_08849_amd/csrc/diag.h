// Per-edge diagonals that the operator kernel never needs to store, for the
// diagonal preconditioners of COCG and the material export.
//
// The curl-curl diagonal K_ee = sum over the four primal facets f that
// contain edge e of M_nu,f (every entry of C is +-1, so C_fe^2 = 1).  It is
// the paper's diagonal preconditioner for the factorized form (Sec. III,
// eq. (Precond)): with calA = M_mu^{-1/2} C M_eps^{-1/2} the squared column
// norms are P_ee = K_ee / M_eps,e, and COCG on S A S preconditioned by
// 1/P is COCG on A preconditioned by S (1/P) S = 1/K_ee.
#pragma once

#include "fit_internal.h"
#include "stencil.h"

namespace fit {

// What edge_diag_kernel writes per edge.
enum EdgeDiagKind {
  ED_CURLCURL = 0,  // K_ee on every index (ghost and masked ones included), real
  ED_MASS = 1,      // 1 / M_eps,c = -omega^2 / d_e (the symmetric scaling squared)
  ED_PAPER = 2,     // 1 / K_ee, eq. (Precond) in the unscaled variables
  ED_JACOBI = 3     // 1 / (K_ee + d_e), d_e = -omega^2 M_eps + j omega M_sigma
};

// Coefficients of node (i, j, p), 0 <= i < nx, 0 <= j < ny, 0 <= p < nz.
__device__ __forceinline__ NodeCoef<double> node_coef_at(const GridView& g,
                                                         const MatLds<double>& mat, int i, int j,
                                                         int p, cx<double> pc) {
  const ColGeo<double> cg = col_geo<double>(g, i, j);
  const PlaneRec<double> lo = plane_rec(mat, cg, load_cell_ids(g, i, j, p - 1));
  const PlaneRec<double> hi = plane_rec(mat, cg, load_cell_ids(g, i, j, p));
  const ZGeo<double> z = zgeo<double>(g, p);
  return node_coef(cg, lo, hi, z.hzl, z.hzh, z.ivz, p, pc);
}

// One thread per node: the three edges' diagonal of the requested kind.
// Masked edges get 0 for the preconditioner kinds.
template <class TO>
__global__ void __launch_bounds__(256)
    edge_diag_kernel(GridView g, double omega, int kind, TO* out) {
  __shared__ MatLds<double> mat;
  const int mode = kind == ED_MASS ? MODE_MEC : MODE_D;
  fill_mat_mode<double>(mat, g.mats, omega, mode);
  const cx<double> pc = port_coef_mode<double>(omega, mode);
  __syncthreads();
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < g.np;
       n += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(n % g.nx);
    const int j = (int)((n / g.nx) % g.ny);
    const int k = (int)(n / ((int64_t)g.nx * g.ny));
    const NodeCoef<double> nc = node_coef_at(g, mat, i, j, k, pc);
    // reluctances of the facets owned by the three lower neighbours (0 where
    // the neighbour lies outside the grid: those facets do not exist)
    double nu_im[3] = {0.0, 0.0, 0.0}, nu_jm[3] = {0.0, 0.0, 0.0}, nu_km[3] = {0.0, 0.0, 0.0};
    if (i > 0) {
      const NodeCoef<double> a = node_coef_at(g, mat, i - 1, j, k, pc);
      nu_im[1] = a.nu[1];
      nu_im[2] = a.nu[2];
    }
    if (j > 0) {
      const NodeCoef<double> b = node_coef_at(g, mat, i, j - 1, k, pc);
      nu_jm[0] = b.nu[0];
      nu_jm[2] = b.nu[2];
    }
    if (k > 0) {
      const NodeCoef<double> c = node_coef_at(g, mat, i, j, k - 1, pc);
      nu_km[0] = c.nu[0];
      nu_km[1] = c.nu[1];
    }
    // x-edge: y-facets at k, k-1 and z-facets at j, j-1; cyclically for y, z
    const double kd[3] = {nc.nu[1] + nu_km[1] + nc.nu[2] + nu_jm[2],
                          nc.nu[0] + nu_km[0] + nc.nu[2] + nu_im[2],
                          nc.nu[0] + nu_jm[0] + nc.nu[1] + nu_im[1]};
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      cx<double> v{0.0, 0.0};
      if (kind == ED_CURLCURL) {
        v = cx<double>{kd[w], 0.0};
      } else if ((nc.mask >> w) & 1u) {
        cx<double> den{kd[w], 0.0};
        if (kind == ED_MASS) den = nc.e[w];
        if (kind == ED_JACOBI) den = cx<double>{kd[w] + nc.e[w].re, nc.e[w].im};
        const double a2 = cabs2(den);
        v = cx<double>{den.re / a2, -den.im / a2};
      }
      stc(out, 3 * n + w, cx<TO>{(TO)v.re, (TO)v.im});
    }
  }
}

}  // namespace fit

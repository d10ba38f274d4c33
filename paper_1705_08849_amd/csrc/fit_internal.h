// Internal declarations of the FIT library: device-side grid view, complex
// helpers, the per-edge material rules and the error plumbing.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "fit.h"

namespace fit {

// ---------------------------------------------------------------------------
// Physical constants (SI).  mu0 is the classical 4 pi 1e-7 H/m.
// ---------------------------------------------------------------------------
constexpr double kPi = 3.14159265358979323846;
constexpr double kMu0 = 4.0e-7 * kPi;
constexpr double kC0 = 299792458.0;
constexpr double kEps0 = 1.0 / (kMu0 * kC0 * kC0);

// Material ids 254/255 are reserved for the ghost cells that pad the grid by
// one cell on every side.  A ghost cell carries no material (all coefficients
// zero); beyond an electric wall it is flagged PEC so that the wall's
// tangential edges are masked by the same rule as edges touching PEC cells.
constexpr int kGhost = 255;
constexpr int kGhostPec = 254;
constexpr int kMaxMat = 254;
constexpr uint32_t kFlagPec = 1u;
constexpr uint32_t kFlagGhost = 2u;

// Base material table entry (omega independent), one per id 0..255.
struct MatEntry {
  double eps;       // eps0 * eps_r
  double eps_tand;  // eps0 * eps_r * tan(delta)
  double sigma;     // S/m
  double inv_mu;    // 1 / (mu0 mu_r)
  uint32_t flags;   // kFlagPec | kFlagGhost
  uint32_t pad;
};

struct PortDev {
  int32_t k0, k1;
  double g;  // conductance per edge, (k1-k0)/z0
};

// Geometry arrays in precision T.
//   hh*: half cell widths on the padded cell axis, hh[a+1] = h[a]/2 for
//        a in [-1, nc], with hh[0] = hh[nc+1] = 0 (ghost cells), length nc+2;
//        node i sees the half cells hh[i] (cell i-1) and hh[i+1] (cell i).
//   iv*: inverse edge lengths, iv[i] = 1/h[i] for i < nc, iv[nc] = 0, length nc+1.
template <class T>
struct GeoArrays {
  const T* hhx;
  const T* hhy;
  const T* hhz;
  const T* ivx;
  const T* ivy;
  const T* ivz;
};

// Device view of a grid, passed by value to kernels.
struct GridView {
  int ncx, ncy, ncz;
  int nx, ny, nz;  // nodes per axis
  int64_t np;      // nodes
  const uint8_t* cell;  // padded (ncz+2)(ncy+2)(ncx+2), cell (a,b,c) at ((c+1)(ncy+2)+(b+1))(ncx+2)+(a+1)
  const MatEntry* mats; // 256 entries
  const int8_t* port_col;  // nx*ny, port index or -1
  const PortDev* ports;
  int nports;
  GeoArrays<double> gd;
  GeoArrays<float> gf;

  template <class T>
  __host__ __device__ const GeoArrays<T>& geo() const;

  __host__ __device__ int64_t cell_index(int a, int b, int c) const {
    return ((int64_t)(c + 1) * (ncy + 2) + (b + 1)) * (int64_t)(ncx + 2) + (a + 1);
  }
};
template <>
__host__ __device__ inline const GeoArrays<double>& GridView::geo<double>() const { return gd; }
template <>
__host__ __device__ inline const GeoArrays<float>& GridView::geo<float>() const { return gf; }

// ---------------------------------------------------------------------------
// Complex arithmetic on plain (re, im) pairs.
// ---------------------------------------------------------------------------
template <class T>
struct cx {
  T re, im;
};

template <class T>
__host__ __device__ __forceinline__ cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <class T>
__host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <class T>
__host__ __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class T>
__host__ __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
template <class T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a) { return {-a.re, -a.im}; }
// conj(a) * b
template <class T>
__host__ __device__ __forceinline__ cx<T> cdotc(cx<T> a, cx<T> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <class T>
__host__ __device__ __forceinline__ T cabs2(cx<T> a) { return a.re * a.re + a.im * a.im; }

// Products feeding reductions are formed in double: complex64 iterates can
// exceed the float range once squared (the scaled operator carries omega^2).
template <class T>
__host__ __device__ __forceinline__ cx<double> cdotc_d(cx<T> a, cx<T> b) {
  const double ar = a.re, ai = a.im, br = b.re, bi = b.im;
  return {ar * br + ai * bi, ar * bi - ai * br};
}
template <class T>
__host__ __device__ __forceinline__ double cabs2_d(cx<T> a) {
  const double r = a.re, i = a.im;
  return r * r + i * i;
}

// 1/sqrt(z), principal branch (Re sqrt(z) >= 0).
// Uses t = sqrt((|z| + |Re z|)/2), which involves no cancellation; the other
// component follows from Im z = 2 u v.  Undefined for z = 0.
template <class T>
__device__ __forceinline__ cx<T> crsqrt(cx<T> z) {
  const T r = sqrt(z.re * z.re + z.im * z.im);
  const T t = sqrt(T(0.5) * (r + fabs(z.re)));
  T u, v;
  if (z.re >= T(0)) {
    u = t;
    v = z.im / (T(2) * t);
  } else {
    u = fabs(z.im) / (T(2) * t);
    v = copysign(t, z.im);
  }
  const T inv = T(1) / (u * u + v * v);
  return {u * inv, -v * inv};
}

template <class T>
struct vec2;
template <>
struct vec2<double> {
  using type = double2;
};
template <>
struct vec2<float> {
  using type = float2;
};

// Load / store one complex element of an interleaved vector.
template <class T>
__device__ __forceinline__ cx<T> ldc(const T* base, int64_t idx) {
  auto v = reinterpret_cast<const typename vec2<T>::type*>(base)[idx];
  return {v.x, v.y};
}
template <class T>
__device__ __forceinline__ void stc(T* base, int64_t idx, cx<T> a) {
  typename vec2<T>::type v;
  v.x = a.re;
  v.y = a.im;
  reinterpret_cast<typename vec2<T>::type*>(base)[idx] = v;
}

// ---------------------------------------------------------------------------
// Per-edge material rule, shared by the stencil and the pointwise kernels.
//
// For node (i, j, p) the 8 cells (i-1..i, j-1..j, p-1..p) determine the
// three edges owned by the node.  A "plane record" holds, for one plane of
// 2x2 cells around the node column, the partial sums a node needs from it:
//   px = hy_lo*c(i,j-1) + hy_hi*c(i,j)     (x-edge: cells (i, j-1..j))
//   py = hx_lo*c(i-1,j) + hx_hi*c(i,j)     (y-edge: cells (i-1..i, j))
//   pz = full 2x2 weighted sum               (z-edge: cells (i-1..i, j-1..j))
// where c is the per-unit-area complex coefficient of the cell material
// (its permittivity-like term for the current omega), together with the
// reluctance data of the facets and the PEC/ghost flags.
// ---------------------------------------------------------------------------
template <class T>
struct PlaneRec {
  cx<T> px, py, pz;
  T imu01, imu10, imu11;  // 1/mu of cells (i-1,j), (i,j-1), (i,j)
  uint32_t pec_x, pec_y, pec_z, gh_x, gh_y, gh_z;
};

// Column constants of a node column (i, j).
template <class T>
struct ColGeo {
  T hxl, hxh, hyl, hyh;  // half widths of cells i-1, i and j-1, j
  T ivx, ivy;            // 1/dx[i], 1/dy[j]
  int pk0, pk1;          // port z-range on this column (empty if none)
  T pg;                  // port conductance per edge
};

template <class T>
__device__ __forceinline__ ColGeo<T> col_geo(const GridView& g, int i, int j) {
  const GeoArrays<T>& a = g.geo<T>();
  ColGeo<T> c;
  int ic = min(i, g.ncx), jc = min(j, g.ncy);  // clamp ragged columns (all-ghost anyway)
  c.hxl = a.hhx[ic];
  c.hxh = a.hhx[ic + 1];
  c.hyl = a.hhy[jc];
  c.hyh = a.hhy[jc + 1];
  c.ivx = a.ivx[ic];
  c.ivy = a.ivy[jc];
  c.pk0 = 0;
  c.pk1 = 0;
  c.pg = T(0);
  if (i < g.nx && j < g.ny && g.nports > 0) {
    int pidx = g.port_col[(int64_t)j * g.nx + i];
    if (pidx >= 0) {
      c.pk0 = g.ports[pidx].k0;
      c.pk1 = g.ports[pidx].k1;
      c.pg = (T)g.ports[pidx].g;
    }
  }
  return c;
}

// Ids of the 2x2 cells (i-1..i, j-1..j) in plane p, packed c00|c10<<8|c01<<16|c11<<24.
// The same four ids as two undecoded 16-bit halves (x-pairs at y-1 and y),
// so a prefetch can be issued now and decoded a pipeline step later without
// an early wait on the load.
struct CellIdsRaw {
  uint32_t lo, hi;
};
__device__ __forceinline__ CellIdsRaw load_cell_ids_raw(const GridView& g, int i, int j, int p) {
  CellIdsRaw r{0xFFFFu, 0xFFFFu};
  if (i < 0 || j < 0 || i >= g.nx || j >= g.ny || p > g.ncz || p < -1) return r;
  const uint8_t* base = g.cell + g.cell_index(i - 1, j - 1, p);
  r.lo = (uint32_t)base[0] | ((uint32_t)base[1] << 8);
  r.hi = (uint32_t)base[g.ncx + 2] | ((uint32_t)base[g.ncx + 3] << 8);
  return r;
}
// For 0 <= i < nx, 0 <= j < ny, -1 <= p <= ncz only (no range test, no branch).
__device__ __forceinline__ CellIdsRaw load_cell_ids_raw_inrange(const GridView& g, int i, int j, int p) {
  const uint8_t* base = g.cell + g.cell_index(i - 1, j - 1, p);
  CellIdsRaw r;
  r.lo = (uint32_t)base[0] | ((uint32_t)base[1] << 8);
  r.hi = (uint32_t)base[g.ncx + 2] | ((uint32_t)base[g.ncx + 3] << 8);
  return r;
}
__device__ __forceinline__ uint32_t decode_cell_ids(const CellIdsRaw& r) { return r.lo | (r.hi << 16); }

__device__ __forceinline__ uint32_t load_cell_ids(const GridView& g, int i, int j, int p) {
  if (i < 0 || j < 0 || i >= g.nx || j >= g.ny || p > g.ncz || p < -1)
    return 0xFFFFFFFFu;  // outside the padded grid: all ghost
  const uint8_t* base = g.cell + g.cell_index(i - 1, j - 1, p);
  uint32_t c00 = base[0], c10 = base[1];
  uint32_t c01 = base[g.ncx + 2], c11 = base[g.ncx + 3];
  return c00 | (c10 << 8) | (c01 << 16) | (c11 << 24);
}

// Material table for one omega and coefficient mode, resident in LDS.
template <class T>
struct MatLds {
  cx<T> coef[256];
  T imu[256];
  uint32_t flg[256];
};

template <class T>
__device__ __forceinline__ PlaneRec<T> plane_rec(const MatLds<T>& m, const ColGeo<T>& c,
                                                 uint32_t ids) {
  uint32_t i00 = ids & 255u, i10 = (ids >> 8) & 255u, i01 = (ids >> 16) & 255u, i11 = ids >> 24;
  cx<T> c00 = m.coef[i00], c10 = m.coef[i10], c01 = m.coef[i01], c11 = m.coef[i11];
  uint32_t f00 = m.flg[i00], f10 = m.flg[i10], f01 = m.flg[i01], f11 = m.flg[i11];
  PlaneRec<T> r;
  r.px = c.hyl * c10 + c.hyh * c11;
  r.py = c.hxl * c01 + c.hxh * c11;
  r.pz = c.hxl * (c.hyl * c00 + c.hyh * c01) + c.hxh * (c.hyl * c10 + c.hyh * c11);
  r.imu01 = m.imu[i01];
  r.imu10 = m.imu[i10];
  r.imu11 = m.imu[i11];
  r.pec_x = (f10 | f11) & kFlagPec;
  r.pec_y = (f01 | f11) & kFlagPec;
  r.pec_z = (f00 | f10 | f01 | f11) & kFlagPec;
  r.gh_x = (f10 & f11) & kFlagGhost;
  r.gh_y = (f01 & f11) & kFlagGhost;
  r.gh_z = (f00 & f10 & f01 & f11) & kFlagGhost;
  return r;
}

// Everything the operator needs about the three edges and three facets owned
// by node (i, j, p), from the plane records of planes p-1 (lo) and p (hi).
template <class T>
struct NodeCoef {
  cx<T> e[3];     // dual-facet integrated coefficient / edge length (+ port term)
  T nu[3];        // reluctance of facets (w, i, j, p)
  uint32_t mask;  // bit w set: edge w is free
};

template <class T>
__device__ __forceinline__ NodeCoef<T> node_coef(const ColGeo<T>& c, const PlaneRec<T>& lo,
                                                 const PlaneRec<T>& hi, T hzl, T hzh, T ivz,
                                                 int p, cx<T> port_coef) {
  NodeCoef<T> n;
  n.e[0] = c.ivx * (hzl * lo.px + hzh * hi.px);
  n.e[1] = c.ivy * (hzl * lo.py + hzh * hi.py);
  n.e[2] = ivz * hi.pz;
  if (p >= c.pk0 && p < c.pk1) n.e[2] = n.e[2] + c.pg * port_coef;
  n.nu[0] = (c.hxl * hi.imu01 + c.hxh * hi.imu11) * c.ivy * ivz;
  n.nu[1] = (c.hyl * hi.imu10 + c.hyh * hi.imu11) * ivz * c.ivx;
  n.nu[2] = (hzl * lo.imu11 + hzh * hi.imu11) * c.ivx * c.ivy;
  uint32_t mx = (lo.pec_x | hi.pec_x) | (lo.gh_x & hi.gh_x);
  uint32_t my = (lo.pec_y | hi.pec_y) | (lo.gh_y & hi.gh_y);
  uint32_t mz = hi.pec_z | hi.gh_z;
  n.mask = (mx ? 0u : 1u) | (my ? 0u : 2u) | (mz ? 0u : 4u);
  return n;
}

// ---------------------------------------------------------------------------
// Host-side grid object.
// ---------------------------------------------------------------------------
struct Workspace {
  void* ptr = nullptr;
  size_t bytes = 0;
};

}  // namespace fit

struct fit_grid {
  int device;
  fit::GridView view;
  int64_t ne;
  double min_h;  // smallest spacing (for diagnostics)
  // device allocations
  uint8_t* d_cell = nullptr;
  fit::MatEntry* d_mats = nullptr;
  int8_t* d_port_col = nullptr;
  fit::PortDev* d_ports = nullptr;
  void* d_geo = nullptr;  // all spacing arrays
  // host copies
  std::string name;
  int nports;
  std::vector<fit_port>* host_ports;
  std::vector<fit::MatEntry>* host_mats;
  // per-grid workspace arena (grown on demand; freed by destroy)
  fit::Workspace ws;
  fit::Workspace red;  // reduction partials + counters + solver state
  void* pinned = nullptr;  // pinned host mirror of the solver state
  // edge mask (1 = free edge), computed on first use by the learned
  // preconditioner and kept until destroy
  uint8_t* d_mask = nullptr;
  std::mutex mask_mu;
};

namespace fit {
// thread-local error message
void set_error(const std::string& msg);
fit_status hip_fail(hipError_t e, const char* what);
#define FIT_HIP(call)                                        \
  do {                                                       \
    hipError_t _e = (call);                                  \
    if (_e != hipSuccess) return fit::hip_fail(_e, #call);   \
  } while (0)

fit_status ensure_ws(Workspace& w, size_t bytes, int device);
}  // namespace fit

// Grid creation, validation, device upload, and the pointwise debug exports
// (edge mask, material diagonals).
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "diag.h"
#include "fit_internal.h"
#include "stencil.h"

namespace fit {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

fit_status hip_fail(hipError_t e, const char* what) {
  set_error(std::string("HIP error in ") + what + ": " + hipGetErrorString(e));
  return FIT_E_DEVICE;
}

fit_status ensure_ws(Workspace& w, size_t bytes, int device) {
  if (w.bytes >= bytes) return FIT_OK;
  if (w.ptr) {
    hipError_t e = hipFree(w.ptr);
    w.ptr = nullptr;
    w.bytes = 0;
    if (e != hipSuccess) return hip_fail(e, "hipFree(workspace)");
  }
  (void)device;
  hipError_t e = hipMalloc(&w.ptr, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_error("device allocation of " + std::to_string(bytes) + " bytes failed");
    return FIT_E_NOMEM;
  }
  w.bytes = bytes;
  return FIT_OK;
}

// Restores the calling thread's current device on scope exit.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

// ---------------------------------------------------------------------------
// Pointwise per-node export of the per-edge material rule.  One thread per
// node; uses exactly the same plane-record / node-coefficient functions as
// the stencil.
// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(256)
    node_coef_kernel(GridView g, double omega, int mode, uint8_t* mask_out, double* diag_out,
                     int facet_kind) {
  __shared__ MatLds<T> mat;
  fill_mat_mode<T>(mat, g.mats, omega, mode);
  __syncthreads();
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= g.np) return;
  const int i = (int)(n % g.nx);
  const int j = (int)((n / g.nx) % g.ny);
  const int p = (int)(n / ((int64_t)g.nx * g.ny));
  const ColGeo<T> cg = col_geo<T>(g, i, j);
  const PlaneRec<T> lo = plane_rec(mat, cg, load_cell_ids(g, i, j, p - 1));
  const PlaneRec<T> hi = plane_rec(mat, cg, load_cell_ids(g, i, j, p));
  const ZGeo<T> z = zgeo<T>(g, p);
  const NodeCoef<T> nc = node_coef(cg, lo, hi, z.hzl, z.hzh, z.ivz, p,
                                   port_coef_mode<T>(omega, mode));
  if (mask_out) {
#pragma unroll
    for (int w = 0; w < 3; ++w) mask_out[3 * n + w] = (nc.mask >> w) & 1u;
  }
  if (diag_out) {
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      double re, im;
      if (facet_kind) {
        re = (double)nc.nu[w];
        im = 0.0;
      } else {
        re = (double)nc.e[w].re;
        im = (double)nc.e[w].im;
      }
      diag_out[2 * (3 * n + w)] = re;
      diag_out[2 * (3 * n + w) + 1] = im;
    }
  }
}

}  // namespace fit

using namespace fit;

extern "C" const char* fit_last_error(void) { return g_err.c_str(); }
extern "C" const char* fit_version(void) { return "fit-mi355x 0.1.0"; }

static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

extern "C" fit_status fit_grid_create(const fit_grid_desc* d, int device, fit_grid** out) {
  if (!out) {
    set_error("fit_grid_create: out is NULL");
    return FIT_E_INVALID;
  }
  *out = nullptr;
  if (!d) {
    set_error("fit_grid_create: desc is NULL");
    return FIT_E_INVALID;
  }
  if (d->ncx < 1 || d->ncy < 1 || d->ncz < 1) {
    set_error("fit_grid_create: ncx, ncy, ncz must be >= 1");
    return FIT_E_INVALID;
  }
  const int64_t nx = d->ncx + 1, ny = d->ncy + 1, nz = d->ncz + 1;
  const int64_t np = nx * ny * nz;
  if (np > (int64_t(1) << 36) || nx > (1 << 20) || ny > (1 << 20) || nz > (1 << 20)) {
    set_error("fit_grid_create: grid too large");
    return FIT_E_INVALID;
  }
  if (d->nmat < 1 || d->nmat > kMaxMat) {
    set_error("fit_grid_create: nmat must be in 1..254");
    return FIT_E_INVALID;
  }
  if (!d->dx || !d->dy || !d->dz || !d->cell_mat || !d->mats) {
    set_error("fit_grid_create: NULL array in descriptor");
    return FIT_E_INVALID;
  }
  if (d->nports < 0 || d->nports > 64 || (d->nports > 0 && !d->ports)) {
    set_error("fit_grid_create: nports must be in 0..64 with a port array");
    return FIT_E_INVALID;
  }
  if (d->pec_walls > 0x3Fu) {
    set_error("fit_grid_create: pec_walls has bits above 0x3F");
    return FIT_E_INVALID;
  }
  double min_h = 1e300;
  for (int a = 0; a < d->ncx; ++a)
    if (!finite_pos(d->dx[a])) { set_error("fit_grid_create: dx must be finite and > 0"); return FIT_E_INVALID; } else min_h = std::min(min_h, d->dx[a]);
  for (int a = 0; a < d->ncy; ++a)
    if (!finite_pos(d->dy[a])) { set_error("fit_grid_create: dy must be finite and > 0"); return FIT_E_INVALID; } else min_h = std::min(min_h, d->dy[a]);
  for (int a = 0; a < d->ncz; ++a)
    if (!finite_pos(d->dz[a])) { set_error("fit_grid_create: dz must be finite and > 0"); return FIT_E_INVALID; } else min_h = std::min(min_h, d->dz[a]);
  for (int m = 0; m < d->nmat; ++m) {
    const fit_material& mt = d->mats[m];
    if (!finite_pos(mt.eps_r) || !finite_pos(mt.mu_r) || !std::isfinite(mt.sigma) || mt.sigma < 0 ||
        !std::isfinite(mt.tan_delta) || mt.tan_delta < 0) {
      set_error("fit_grid_create: material " + std::to_string(m) +
                " needs eps_r, mu_r > 0 and sigma, tan_delta >= 0, all finite");
      return FIT_E_INVALID;
    }
  }
  const int64_t ncell = (int64_t)d->ncx * d->ncy * d->ncz;
  for (int64_t c = 0; c < ncell; ++c) {
    if (d->cell_mat[c] >= d->nmat) {
      set_error("fit_grid_create: cell material id out of range at cell " + std::to_string(c));
      return FIT_E_INVALID;
    }
  }
  std::vector<int8_t> port_col((size_t)(nx * ny), (int8_t)-1);
  std::vector<PortDev> ports_dev((size_t)std::max(d->nports, 1));
  for (int p = 0; p < d->nports; ++p) {
    const fit_port& pt = d->ports[p];
    if (pt.i < 0 || pt.i >= nx || pt.j < 0 || pt.j >= ny || pt.k0 < 0 || pt.k1 <= pt.k0 ||
        pt.k1 > d->ncz || !finite_pos(pt.z0)) {
      set_error("fit_grid_create: port " + std::to_string(p) +
                " must satisfy 0<=i<Nx, 0<=j<Ny, 0<=k0<k1<=ncz, z0>0");
      return FIT_E_INVALID;
    }
    int8_t& pc = port_col[(size_t)(pt.j * nx + pt.i)];
    if (pc >= 0) {
      set_error("fit_grid_create: two ports on column (" + std::to_string(pt.i) + "," +
                std::to_string(pt.j) + ")");
      return FIT_E_INVALID;
    }
    pc = (int8_t)p;
    ports_dev[p].k0 = pt.k0;
    ports_dev[p].k1 = pt.k1;
    ports_dev[p].g = (double)(pt.k1 - pt.k0) / pt.z0;
  }

  // Padded cell ids: ghost cells beyond an electric wall are PEC ghosts.
  const int pcx = d->ncx + 2, pcy = d->ncy + 2, pcz = d->ncz + 2;
  std::vector<uint8_t> cells((size_t)pcx * pcy * pcz);
  const uint32_t w = d->pec_walls;
  for (int c = -1; c <= d->ncz; ++c)
    for (int b = -1; b <= d->ncy; ++b)
      for (int a = -1; a <= d->ncx; ++a) {
        uint8_t id;
        if (a >= 0 && a < d->ncx && b >= 0 && b < d->ncy && c >= 0 && c < d->ncz) {
          id = d->cell_mat[(size_t)a + (size_t)d->ncx * ((size_t)b + (size_t)d->ncy * c)];
        } else {
          bool pec = (a < 0 && (w & 1u)) || (a >= d->ncx && (w & 2u)) || (b < 0 && (w & 4u)) ||
                     (b >= d->ncy && (w & 8u)) || (c < 0 && (w & 16u)) || (c >= d->ncz && (w & 32u));
          id = pec ? kGhostPec : kGhost;
        }
        cells[((size_t)(c + 1) * pcy + (b + 1)) * pcx + (a + 1)] = id;
      }

  std::vector<MatEntry> mats(256);
  std::memset(mats.data(), 0, sizeof(MatEntry) * 256);
  for (int m = 0; m < d->nmat; ++m) {
    const fit_material& mt = d->mats[m];
    mats[m].eps = kEps0 * mt.eps_r;
    mats[m].eps_tand = kEps0 * mt.eps_r * mt.tan_delta;
    mats[m].sigma = mt.sigma;
    mats[m].inv_mu = 1.0 / (kMu0 * mt.mu_r);
    mats[m].flags = mt.is_pec ? kFlagPec : 0u;
  }
  mats[kGhost].flags = kFlagGhost;
  mats[kGhostPec].flags = kFlagGhost | kFlagPec;

  // Geometry arrays, double then float, each axis: hh (nc+2), iv (nc+1).
  auto axis = [](const double* h, int nc, std::vector<double>& hh, std::vector<double>& iv) {
    hh.assign((size_t)nc + 2, 0.0);
    iv.assign((size_t)nc + 1, 0.0);
    for (int a = 0; a < nc; ++a) {
      hh[(size_t)a + 1] = 0.5 * h[a];
      iv[(size_t)a] = 1.0 / h[a];
    }
  };
  std::vector<double> hhx, ivx, hhy, ivy, hhz, ivz;
  axis(d->dx, d->ncx, hhx, ivx);
  axis(d->dy, d->ncy, hhy, ivy);
  axis(d->dz, d->ncz, hhz, ivz);
  const std::vector<double>* arrs[6] = {&hhx, &hhy, &hhz, &ivx, &ivy, &ivz};
  size_t ndbl = 0;
  for (auto* a : arrs) ndbl += a->size();
  std::vector<double> geo_d;
  std::vector<float> geo_f;
  geo_d.reserve(ndbl);
  for (auto* a : arrs) geo_d.insert(geo_d.end(), a->begin(), a->end());
  geo_f.resize(ndbl);
  for (size_t q = 0; q < ndbl; ++q) geo_f[q] = (float)geo_d[q];

  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    set_error("fit_grid_create: device " + std::to_string(device) + " not available");
    return FIT_E_DEVICE;
  }
  DeviceGuard guard(device);

  fit_grid* g = new fit_grid();
  g->device = device;
  g->ne = 3 * np;
  g->min_h = min_h;
  g->nports = d->nports;
  g->host_ports = new std::vector<fit_port>(d->ports, d->ports + d->nports);
  g->host_mats = new std::vector<MatEntry>(mats);

  auto fail = [&](fit_status st) {
    fit_grid_destroy(g);
    return st;
  };
  auto alloc = [&](void** p, size_t bytes) -> fit_status {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      set_error("fit_grid_create: device allocation failed");
      return FIT_E_NOMEM;
    }
    return FIT_OK;
  };
  fit_status st;
  if ((st = alloc((void**)&g->d_cell, cells.size())) != FIT_OK) return fail(st);
  if ((st = alloc((void**)&g->d_mats, sizeof(MatEntry) * 256)) != FIT_OK) return fail(st);
  if ((st = alloc((void**)&g->d_port_col, port_col.size())) != FIT_OK) return fail(st);
  if ((st = alloc((void**)&g->d_ports, sizeof(PortDev) * ports_dev.size())) != FIT_OK) return fail(st);
  if ((st = alloc(&g->d_geo, ndbl * (sizeof(double) + sizeof(float)))) != FIT_OK) return fail(st);
  hipError_t e;
  if ((e = hipMemcpy(g->d_cell, cells.data(), cells.size(), hipMemcpyHostToDevice)) != hipSuccess)
    return fail(hip_fail(e, "hipMemcpy(cells)"));
  if ((e = hipMemcpy(g->d_mats, mats.data(), sizeof(MatEntry) * 256, hipMemcpyHostToDevice)) != hipSuccess)
    return fail(hip_fail(e, "hipMemcpy(mats)"));
  if ((e = hipMemcpy(g->d_port_col, port_col.data(), port_col.size(), hipMemcpyHostToDevice)) != hipSuccess)
    return fail(hip_fail(e, "hipMemcpy(port_col)"));
  if ((e = hipMemcpy(g->d_ports, ports_dev.data(), sizeof(PortDev) * ports_dev.size(),
                     hipMemcpyHostToDevice)) != hipSuccess)
    return fail(hip_fail(e, "hipMemcpy(ports)"));
  double* gd = (double*)g->d_geo;
  float* gf = (float*)(gd + ndbl);
  if ((e = hipMemcpy(gd, geo_d.data(), ndbl * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess)
    return fail(hip_fail(e, "hipMemcpy(geo)"));
  if ((e = hipMemcpy(gf, geo_f.data(), ndbl * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess)
    return fail(hip_fail(e, "hipMemcpy(geo f32)"));

  GridView& v = g->view;
  v.ncx = d->ncx;
  v.ncy = d->ncy;
  v.ncz = d->ncz;
  v.nx = (int)nx;
  v.ny = (int)ny;
  v.nz = (int)nz;
  v.np = np;
  v.cell = g->d_cell;
  v.mats = g->d_mats;
  v.port_col = g->d_port_col;
  v.ports = g->d_ports;
  v.nports = d->nports;
  size_t off = 0;
  const double* dp[6];
  const float* fp[6];
  for (int q = 0; q < 6; ++q) {
    dp[q] = gd + off;
    fp[q] = gf + off;
    off += arrs[q]->size();
  }
  v.gd = GeoArrays<double>{dp[0], dp[1], dp[2], dp[3], dp[4], dp[5]};
  v.gf = GeoArrays<float>{fp[0], fp[1], fp[2], fp[3], fp[4], fp[5]};
  *out = g;
  return FIT_OK;
}

extern "C" void fit_grid_destroy(fit_grid* g) {
  if (!g) return;
  DeviceGuard guard(g->device);
  if (g->d_cell) (void)hipFree(g->d_cell);
  if (g->d_mats) (void)hipFree(g->d_mats);
  if (g->d_port_col) (void)hipFree(g->d_port_col);
  if (g->d_ports) (void)hipFree(g->d_ports);
  if (g->d_geo) (void)hipFree(g->d_geo);
  if (g->ws.ptr) (void)hipFree(g->ws.ptr);
  if (g->red.ptr) (void)hipFree(g->red.ptr);
  if (g->pinned) (void)hipHostFree(g->pinned);
  if (g->d_mask) (void)hipFree(g->d_mask);
  delete g->host_ports;
  delete g->host_mats;
  delete g;
}

extern "C" int64_t fit_num_edges(const fit_grid* g) { return g ? g->ne : -1; }

static fit_status launch_node_coef(const fit_grid* g, double omega, int mode, uint8_t* mask,
                                   double* diag, int facet, void* stream) {
  DeviceGuard guard(g->device);
  const int64_t nb = (g->view.np + 255) / 256;
  hipLaunchKernelGGL(node_coef_kernel<double>, dim3((unsigned)nb), dim3(256), 0,
                     (hipStream_t)stream, g->view, omega, mode, mask, diag, facet);
  FIT_HIP(hipGetLastError());
  return FIT_OK;
}

extern "C" fit_status fit_edge_mask(const fit_grid* g, uint8_t* mask_dev, void* stream) {
  if (!g || !mask_dev) {
    set_error("fit_edge_mask: NULL argument");
    return FIT_E_INVALID;
  }
  return launch_node_coef(g, 0.0, MODE_EPS, mask_dev, nullptr, 0, stream);
}

extern "C" fit_status fit_material_diag(const fit_grid* g, int kind, double* out_dev, void* stream) {
  if (!g || !out_dev || kind < 0 || kind > 3) {
    set_error("fit_material_diag: NULL argument or kind not in 0..3");
    return FIT_E_INVALID;
  }
  if (kind == 3) {
    DeviceGuard guard(g->device);
    const int64_t nb = (g->view.np + 255) / 256;
    hipLaunchKernelGGL(edge_diag_kernel<double>, dim3((unsigned)nb), dim3(256), 0,
                       (hipStream_t)stream, g->view, 0.0, (int)ED_CURLCURL, out_dev);
    FIT_HIP(hipGetLastError());
    return FIT_OK;
  }
  const int mode = kind == 1 ? MODE_SIGMA : MODE_EPS;
  return launch_node_coef(g, 0.0, mode, nullptr, out_dev, kind == 2 ? 1 : 0, stream);
}

// Port network parameters from port solves (host code).
//
// A lumped port is a current source of 1 A in parallel with its internal
// impedance z0 (the port model of Sec. IV, read as a Norton source; the port
// edges carry the conductance).  Driving port q with every port so loaded
// gives the loaded impedance column Zl[:, q] = -u[:, q] (u = the port
// voltages, sums of edge voltages from the ground end up).  With the loads
// taken off, the network's own admittance is Zl^-1 - I / z0, so
//   Z = (Zl^-1 - I / z0)^-1,
// and the scattering matrix for reference impedance z0,
//   S = (Z - z0 I)(Z + z0 I)^-1,
// simplifies to S = 2 Zl / z0 - I, which is how it is computed here.
#include <cmath>
#include <complex>
#include <vector>

#include "fit.h"
#include "fit_internal.h"

namespace {

using cd = std::complex<double>;

// In-place inverse of the n x n row-major matrix a by Gauss-Jordan
// elimination with partial pivoting.  False if a pivot is zero relative to
// the matrix norm (singular to working precision).
bool invert(std::vector<cd>& a, int n) {
  double norm = 0.0;
  for (const cd& v : a) norm = std::max(norm, std::abs(v));
  if (!(norm > 0.0) || !std::isfinite(norm)) return false;
  std::vector<cd> inv((size_t)n * n, cd(0.0, 0.0));
  for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::abs(a[(size_t)r * n + col]) > std::abs(a[(size_t)piv * n + col])) piv = r;
    if (std::abs(a[(size_t)piv * n + col]) <= 1e-14 * norm) return false;
    if (piv != col)
      for (int k = 0; k < n; ++k) {
        std::swap(a[(size_t)piv * n + k], a[(size_t)col * n + k]);
        std::swap(inv[(size_t)piv * n + k], inv[(size_t)col * n + k]);
      }
    const cd d = 1.0 / a[(size_t)col * n + col];
    for (int k = 0; k < n; ++k) {
      a[(size_t)col * n + k] *= d;
      inv[(size_t)col * n + k] *= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      const cd f = a[(size_t)r * n + col];
      if (f == cd(0.0, 0.0)) continue;
      for (int k = 0; k < n; ++k) {
        a[(size_t)r * n + k] -= f * a[(size_t)col * n + k];
        inv[(size_t)r * n + k] -= f * inv[(size_t)col * n + k];
      }
    }
  }
  a.swap(inv);
  return true;
}

}  // namespace

extern "C" fit_status fit_port_network(int nports, double z0, const double* zl, double* z_out,
                                       double* s_out) {
  if (nports < 1 || nports > 64 || !(z0 > 0.0) || !std::isfinite(z0) || !zl) {
    fit::set_error("fit_port_network: bad argument (1 <= nports <= 64, z0 > 0, zl not NULL)");
    return FIT_E_INVALID;
  }
  const int n = nports;
  const size_t nn = (size_t)n * n;
  std::vector<cd> a(nn);
  for (size_t k = 0; k < nn; ++k) {
    a[k] = cd(zl[2 * k], zl[2 * k + 1]);
    if (!std::isfinite(a[k].real()) || !std::isfinite(a[k].imag())) {
      fit::set_error("fit_port_network: non-finite loaded impedance");
      return FIT_E_INVALID;
    }
  }
  std::vector<cd> z;
  if (z_out) {
    z = a;
    if (!invert(z, n)) {
      fit::set_error("fit_port_network: loaded impedance matrix is singular");
      return FIT_E_INVALID;
    }
    for (int i = 0; i < n; ++i) z[(size_t)i * n + i] -= 1.0 / z0;
    if (!invert(z, n)) {
      fit::set_error("fit_port_network: the unloaded network has no impedance matrix (singular admittance)");
      return FIT_E_INVALID;
    }
  }
  // every check passed: write the outputs
  if (z_out)
    for (size_t k = 0; k < nn; ++k) {
      z_out[2 * k] = z[k].real();
      z_out[2 * k + 1] = z[k].imag();
    }
  if (s_out)
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < n; ++k) {
        const cd s = 2.0 * a[(size_t)i * n + k] / z0 - (i == k ? 1.0 : 0.0);
        s_out[2 * ((size_t)i * n + k)] = s.real();
        s_out[2 * ((size_t)i * n + k) + 1] = s.imag();
      }
  return FIT_OK;
}

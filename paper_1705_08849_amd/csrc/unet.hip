// The learned right preconditioner: a 3-level 3D U-Net over the node grid,
// z = s * U(v / s) with s = rms(v) over the free edges, applied inside the
// flexible GMRES of the paper's solver comparison (Sec. IV).  FGMRES stores
// the preconditioned directions, so any nonlinear map is admissible there.
//
// Network (c = base channels; ReLU after every layer but the head):
//   enc1a, enc1b  3x3x3 conv, 12 -> c -> c                (full resolution)
//   down1         2x2x2 stride-2 conv, c -> 2c
//   enc2a, enc2b  3x3x3 conv, 2c                           (1/2)
//   down2         2x2x2 stride-2 conv, 2c -> 4c
//   bot_a, bot_b  3x3x3 conv, 4c                           (1/4)
//   up2           2x2x2 stride-2 transposed conv, 4c -> 2c; concat [up2, enc2b]
//   dec2a, dec2b  3x3x3 conv, 4c -> 2c -> 2c
//   up1           transposed conv, 2c -> c; concat [up1, enc1b]
//   dec1a, dec1b  3x3x3 conv, 2c -> c -> c
//   head          1x1x1 conv, c -> 6 = (Re, Im) of the node's x, y, z edges
// Input channels: Re/Im of the three edge values of v/s, eps_r/12 and
// (log10(sigma + 1e-3) + 3)/11 of the cell the node owns, log10(f/GHz)/1.6,
// and log10(h/100 um) of that cell's three widths (the local mesh scale).
// Storage: bf16 activations and weights, fp32 accumulation, biases, master
// weights, gradients and head output.  Every convolution is one BF16 MFMA
// implicit GEMM (unet_gemm.h), forward and backward.
//
// Training (fit_precond_train): residual -> error pairs r = A(omega) e with
// smooth random errors e (seeded noise smoothed a random number of times),
// cropped; loss = mean over free edges of |U(r/s_r) - e/s_e|^2; Adam.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "fit_internal.h"
#include "precond.h"
#include "reduce.h"
#include "solver_ctx.h"
#include "stencil.h"
#include "tuning.h"
#include "unet_gemm.h"

using namespace fit;

namespace {

enum LKind { L_CONV3 = 0, L_DOWN2 = 1, L_UP2 = 2, L_PW = 3 };

constexpr int kNIn = 12, kNOut = 6;
constexpr int kNLayers = 15;
constexpr uint64_t kMagic = 0x3154454E55544946ull;  // "FITUNET1"

__host__ __device__ inline int pad8(int c) { return (c + 7) / 8 * 8; }
int64_t pad32(int64_t v) { return (v + 31) / 32 * 32; }

struct Spec {
  const char* name;
  int kind, taps, cin, cout;
};

std::vector<Spec> specs(int c) {
  auto S = [](const char* n, int k, int ci, int co) {
    const int taps = k == L_CONV3 ? 27 : (k == L_PW ? 1 : 8);
    return Spec{n, k, taps, ci, co};
  };
  return {S("enc1a", L_CONV3, kNIn, c),       S("enc1b", L_CONV3, c, c),
          S("down1", L_DOWN2, c, 2 * c),      S("enc2a", L_CONV3, 2 * c, 2 * c),
          S("enc2b", L_CONV3, 2 * c, 2 * c),  S("down2", L_DOWN2, 2 * c, 4 * c),
          S("bot_a", L_CONV3, 4 * c, 4 * c),  S("bot_b", L_CONV3, 4 * c, 4 * c),
          S("up2", L_UP2, 4 * c, 2 * c),      S("dec2a", L_CONV3, 4 * c, 2 * c),
          S("dec2b", L_CONV3, 2 * c, 2 * c),  S("up1", L_UP2, 2 * c, c),
          S("dec1a", L_CONV3, 2 * c, c),      S("dec1b", L_CONV3, c, c),
          S("head", L_PW, c, kNOut)};
}

// GEMM shapes of a layer: forward and backward-data B matrices.
struct LayerMats {
  int64_t kf, nf;  // forward K (padded channels) and N
  int64_t kb, nb;  // backward-data K and N
};
LayerMats mats_of(const Spec& s) {
  const int ci = pad8(s.cin), co = pad8(s.cout);
  switch (s.kind) {
    case L_CONV3: return {27LL * ci, s.cout, 27LL * co, s.cin};
    case L_DOWN2: return {8LL * ci, s.cout, (int64_t)co, 8LL * s.cin};
    case L_UP2: return {(int64_t)ci, 8LL * s.cout, 8LL * co, s.cin};
    default: return {(int64_t)ci, s.cout, (int64_t)co, s.cin};
  }
}

int ntile(int64_t n) { return n <= 16 ? 16 : (n <= 32 ? 32 : 64); }
// Most K splits of a weight-gradient GEMM (its fp32 partials are splits x M x N).
constexpr int64_t kMaxSplits = 64;
int64_t rows_pad(int64_t n) { const int t = ntile(n); return (n + t - 1) / t * t; }

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// Canonical fp32 weights w[tap][ci][co] -> the forward and backward-data B
// matrices in bf16 (positions never written stay zero).
__global__ void wtransform_kernel(const float* w, int kind, int taps, int cin, int cout, bf16* bf,
                                  int64_t ldf, bf16* bb, int64_t ldb) {
  const int cip = pad8(cin), cop = pad8(cout);
  const int64_t total = (int64_t)taps * cin * cout;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int co = (int)(q % cout), ci = (int)((q / cout) % cin), t = (int)(q / ((int64_t)cout * cin));
    const bf16 v = (bf16)w[q];
    switch (kind) {
      case L_CONV3:
        bf[co * ldf + (int64_t)t * cip + ci] = v;
        bb[ci * ldb + (int64_t)(26 - t) * cop + co] = v;
        break;
      case L_DOWN2:
        bf[co * ldf + (int64_t)t * cip + ci] = v;
        bb[((int64_t)t * cin + ci) * ldb + co] = v;
        break;
      case L_UP2:
        bf[((int64_t)t * cout + co) * ldf + ci] = v;
        bb[ci * ldb + (int64_t)t * cop + co] = v;
        break;
      default:
        bf[co * ldf + ci] = v;
        bb[ci * ldb + co] = v;
        break;
    }
  }
}

// dpre[v][c] = gout[v][c] where out[v][c] > 0 (ReLU'), bf16; channels in
// [cout, cop) are zero.  relu == 0: plain copy (the head).
__global__ void relu_bwd_kernel(const float* g, int64_t g_ld, const bf16* out, int64_t o_ld, int relu,
                                int64_t nv, int cout, int cop, bf16* dpre) {
  const int64_t total = nv * cop;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(q % cop);
    const int64_t v = q / cop;
    float d = 0.f;
    if (c < cout) {
      d = g[v * g_ld + c];
      if (relu && !((float)out[v * o_ld + c] > 0.f)) d = 0.f;
    }
    dpre[q] = (bf16)d;
  }
}

// xt[k][v] = the layer input at voxel v + offset(tap(k)), channel ci(k)
// (k = tap * cip + ci), zero outside the tensor and for v >= nv: the
// transposed im2col of the weight-gradient GEMM.  A workgroup owns one tap
// and 256 voxels: it reads their channels (up to 64 at a time) with 16-byte
// loads from the channels-last input, transposes them through LDS, and
// writes its tap's rows with 16-byte stores (8 consecutive voxels per lane).
constexpr int kIm2colMaxC = 64;
__global__ void __launch_bounds__(256)
    im2colT_kernel(const bf16* a, int64_t a_ld, int cip, int kind, int ix, int iy, int iz, int ox, int oy,
                   int64_t nv, bf16* xt, int64_t ld) {
  __shared__ bf16 tr[kIm2colMaxC][256 + 8];  // +8: rows start on different banks
  const int tap = (int)blockIdx.y;
  const int64_t v0 = (int64_t)blockIdx.x * 256;
  int dx = 0, dy = 0, dz = 0;
  if (kind == L_CONV3) {
    dx = tap % 3 - 1;
    dy = (tap / 3) % 3 - 1;
    dz = tap / 9 - 1;
  } else if (kind == L_DOWN2) {
    dx = tap & 1;
    dy = (tap >> 1) & 1;
    dz = tap >> 2;
  }
  // 1. this thread's voxel: gather its cip channels
  {
    const int64_t v = v0 + threadIdx.x;
    int64_t src = -1;
    if (v < nv) {
      if (kind == L_PW) {
        src = v;
      } else {
        const uint32_t uv = (uint32_t)v, t = uv / (uint32_t)ox, mx = uv - t * (uint32_t)ox;
        const uint32_t mz = t / (uint32_t)oy, my = t - mz * (uint32_t)oy;
        const int x = (kind == L_CONV3 ? (int)mx : 2 * (int)mx) + dx;
        const int y = (kind == L_CONV3 ? (int)my : 2 * (int)my) + dy;
        const int z = (kind == L_CONV3 ? (int)mz : 2 * (int)mz) + dz;
        if (x >= 0 && y >= 0 && z >= 0 && x < ix && y < iy && z < iz) src = ((int64_t)z * iy + y) * ix + x;
      }
    }
    // channels in groups of kIm2colMaxC: gather a group, transpose, write
    const int j = threadIdx.x & 31;  // voxel group of 8 inside the tile
    const int64_t vg = v0 + 8 * j;
    for (int cb = 0; cb < cip; cb += kIm2colMaxC) {
      const int cw = cip - cb < kIm2colMaxC ? cip - cb : kIm2colMaxC;
      for (int c8 = 0; c8 < cw / 8; ++c8) {
        bf16x8 val;
        if (src >= 0) {
          val = *reinterpret_cast<const bf16x8*>(a + src * a_ld + cb + 8 * c8);
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) val[e] = (bf16)0.f;
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) tr[8 * c8 + e][threadIdx.x] = val[e];
      }
      __syncthreads();
      // 2. rows tap * cip + cb + ci, 8 voxels per lane
      if (vg < ld) {
        for (int ci = threadIdx.x >> 5; ci < cw; ci += 8) {
          bf16x8 out;
#pragma unroll
          for (int e = 0; e < 8; ++e) out[e] = tr[ci][8 * j + e];
          *reinterpret_cast<bf16x8*>(xt + ((int64_t)tap * cip + cb + ci) * ld + vg) = out;
        }
      }
      __syncthreads();
    }
  }
}

// dT[n][v] = dpre[v][n] for n < cop (rows up to nrows zero), zero padding v >= nv.
// up: dT[t*cout + c][u] = dpre[child(u, t)][c] (u over the coarse grid ox*oy*oz).
__global__ void dgradT_kernel(const bf16* dpre, int cop, int cout, int up, int ox, int oy, int64_t nv,
                              int nrows, bf16* dt, int64_t ld) {
  const int64_t total = (int64_t)nrows * ld;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = q % ld;
    const int n = (int)(q / ld);
    bf16 val = (bf16)0.f;
    if (v < nv) {
      if (!up) {
        if (n < cop) val = dpre[v * cop + n];
      } else if (n < 8 * cout) {
        const int t = n / cout, c = n % cout;
        const int ux = (int)(v % ox), uy = (int)((v / ox) % oy), uz = (int)(v / ((int64_t)ox * oy));
        const int64_t child = ((int64_t)(2 * uz + (t >> 2)) * (2 * oy) + (2 * uy + ((t >> 1) & 1))) *
                                  (2 * ox) + (2 * ux + (t & 1));
        val = dpre[child * cop + c];
      }
    }
    dt[q] = val;
  }
}

// Sum the split-K partials into the canonical gradient.  A block of 256
// threads owns 64 consecutive outputs; its four wavefronts sum interleaved
// quarters of the splits (lanes read consecutive columns) and the quarters
// are added in a fixed order, so the result does not depend on timing.
__global__ void __launch_bounds__(256) reduce_dw_kernel(const float* part, int splits, int64_t M, int64_t N,
                                                        int kind, int taps, int cin, int cout, float scale,
                                                        float* gw) {
  __shared__ float quarter[4][64];
  const int cip = pad8(cin);
  const int64_t total = (int64_t)taps * cin * cout;
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t q = (int64_t)blockIdx.x * 64 + lane;
  float s = 0.f;
  if (q < total) {
    const int co = (int)(q % cout), ci = (int)((q / cout) % cin), t = (int)(q / ((int64_t)cout * cin));
    int64_t row, col;
    if (kind == L_UP2) {
      row = ci;
      col = (int64_t)t * cout + co;
    } else {
      row = (int64_t)t * cip + ci;
      col = co;
    }
    for (int sp = g; sp < splits; sp += 4) s += part[((int64_t)sp * M + row) * N + col];
  }
  quarter[g][lane] = s;
  __syncthreads();
  if (g == 0 && q < total)
    gw[q] += scale * (((quarter[0][lane] + quarter[1][lane]) + quarter[2][lane]) + quarter[3][lane]);
}

__global__ void __launch_bounds__(1024) bias_grad_kernel(const bf16* dt, int64_t ld, int cout, int up,
                                                         float scale, float* gb) {
  // one block per output channel; 16-byte loads (rows are padded to a
  // multiple of 32 elements, so ld / 8 vectors cover a row exactly)
  __shared__ double lds[1024 / 64];
  const int c = blockIdx.x;
  double acc[1] = {0.0};
  const int reps = up ? 8 : 1;
  for (int t = 0; t < reps; ++t) {
    const bf16x8* row = reinterpret_cast<const bf16x8*>(dt + ((int64_t)t * cout + c) * ld);
    for (int64_t v = threadIdx.x; v < ld / 8; v += blockDim.x) {
      const bf16x8 x = row[v];
      float f = 0.f;
#pragma unroll
      for (int e = 0; e < 8; ++e) f += (float)x[e];
      acc[0] += (double)f;
    }
  }
  block_reduce<1>(acc, lds);
  if (threadIdx.x == 0) gb[c] += scale * (float)acc[0];
}

// Adam with bias correction; weight decay added to the gradient.
__global__ void adam_kernel(float* w, const float* g, float* m, float* v, int64_t n, float lr,
                            float b1, float b2, float eps, float wd, float c1, float c2) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (int64_t)gridDim.x * blockDim.x) {
    const float gq = g[q] + wd * w[q];
    const float mq = b1 * m[q] + (1.f - b1) * gq;
    const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    w[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
  }
}

__global__ void fill_f32_kernel(float* p, int64_t n, float v) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (int64_t)gridDim.x * blockDim.x)
    p[q] = v;
}

// Sums of |v|^2 over free edges and their count inside the node box
// [o, o + ext) (the whole grid for a full box).  Results -> out[0..1].
template <class T>
__global__ void __launch_bounds__(256)
    box_norm_kernel(GridView g, const T* v, const uint8_t* mask, int ox0, int oy0, int oz0, int ex, int ey,
                    int ez, double* part) {
  __shared__ double lds[2 * 4];
  double acc[2] = {0.0, 0.0};
  const int64_t nb = (int64_t)ex * ey * ez;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nb;
       q += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t qq = (uint32_t)q, t = qq / (uint32_t)ex, bx = qq - t * (uint32_t)ex;
    const uint32_t bz = t / (uint32_t)ey, by = t - bz * (uint32_t)ey;
    const int i = ox0 + (int)bx, j = oy0 + (int)by, k = oz0 + (int)bz;
    if (i >= g.nx || j >= g.ny || k >= g.nz) continue;
    const int64_t n = ((int64_t)k * g.ny + j) * g.nx + i;
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      const cx<T> a = ldc(v, 3 * n + w);
      const bool fr = mask[3 * n + w] != 0;
      acc[0] += fr ? cabs2_d(a) : 0.0;
      acc[1] += fr ? 1.0 : 0.0;
    }
  }
  block_partial<2>(acc, part, lds);
}

// Grid sums -> out[0..N).
struct StoreSumsPtr {
  double* out;
  __device__ bool skip() const { return false; }
  __device__ void operator()(const double* s) const {
    out[0] = s[0];
    out[1] = s[1];
  }
};

// Adds the pair's loss (sum of squares / free count) to *loss.
struct LossFinish {
  double* loss;
  const double* counts;
  __device__ bool skip() const { return false; }
  __device__ void operator()(const double* s) const {
    *loss += s[0] / (counts[1] > 0.0 ? counts[1] : 1.0);
  }
};

// s = sqrt(sum / count) -> scal[slot] (0 when nothing is free).
struct RmsFinish {
  double* scal;
  int slot;
  __device__ bool skip() const { return false; }
  __device__ void operator()(const double* s) const {
    scal[slot] = s[1] > 0.0 ? sqrt(s[0] / s[1]) : 0.0;
  }
};

// Input features of the box (size X x Y x Z voxels, all multiples of 4) at
// node offset o: channels 0..5 = Re/Im of v/s (s = scal[slot]), 6 eps_r/12,
// 7 (log10(sigma + 1e-3) + 3)/11, 8 log10(f/GHz)/1.6, 9..11 log10(h/100 um)
// of the owned cell's x, y, z widths, 12..15 zero; voxels outside the grid
// are zero.
template <class T>
__global__ void features_kernel(GridView g, const T* v, const uint8_t* mask, const double* scal, int slot,
                                double omega, int ox0, int oy0, int oz0, int X, int Y, int Z, bf16* x0) {
  const int64_t nv = (int64_t)X * Y * Z;
  const double s = scal[slot];
  const double inv = s > 0.0 ? 1.0 / s : 0.0;
  const float lw = (float)(log10(omega / (2.0 * kPi) / 1e9) / 1.6);
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nv;
       q += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t qq = (uint32_t)q, t = qq / (uint32_t)X, bx = qq - t * (uint32_t)X;
    const uint32_t bz = t / (uint32_t)Y, by = t - bz * (uint32_t)Y;
    const int i = ox0 + (int)bx, j = oy0 + (int)by, k = oz0 + (int)bz;
    float f[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) f[c] = 0.f;
    if (i < g.nx && j < g.ny && k < g.nz) {
      const int64_t n = ((int64_t)k * g.ny + j) * g.nx + i;
#pragma unroll
      for (int w = 0; w < 3; ++w) {
        const cx<T> a = ldc(v, 3 * n + w);
        const bool fr = mask[3 * n + w] != 0;
        f[2 * w] = fr ? (float)((double)a.re * inv) : 0.f;
        f[2 * w + 1] = fr ? (float)((double)a.im * inv) : 0.f;
      }
      const int a = min(i, g.ncx - 1), b = min(j, g.ncy - 1), c = min(k, g.ncz - 1);
      const MatEntry& me = g.mats[g.cell[g.cell_index(a, b, c)]];
      f[6] = (float)(me.eps / kEps0 / 12.0);
      f[7] = (float)((log10(me.sigma + 1e-3) + 3.0) / 11.0);
      f[8] = lw;
      const GeoArrays<double>& ga = g.geo<double>();
      f[9] = (float)(-log10(ga.ivx[a] * 1e-4));
      f[10] = (float)(-log10(ga.ivy[b] * 1e-4));
      f[11] = (float)(-log10(ga.ivz[c] * 1e-4));
    }
    bf16x8 lo, hi;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      lo[c] = (bf16)f[c];
      hi[c] = (bf16)f[8 + c];
    }
    reinterpret_cast<bf16x8*>(x0)[2 * q] = lo;
    reinterpret_cast<bf16x8*>(x0)[2 * q + 1] = hi;
  }
}

// z = s * (y0 + j y1, y2 + j y3, y4 + j y5) on free edges, 0 elsewhere.
template <class T>
__global__ void output_kernel(GridView g, const float* y, const uint8_t* mask, const double* scal, int slot,
                              int X, int Y, T* z) {
  const double s = scal[slot];
  const uint32_t nx = (uint32_t)g.nx, ny = (uint32_t)g.ny;
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < g.np;
       n += (int64_t)gridDim.x * blockDim.x) {
    // 32-bit index arithmetic (a grid has fewer than 2^31 nodes); every load
    // is issued before any is used
    const uint32_t nn = (uint32_t)n, t = nn / nx, i = nn - t * nx, k = t / ny, j = t - k * ny;
    const int64_t vx = ((int64_t)k * Y + j) * X + i;
    const float4 y03 = *reinterpret_cast<const float4*>(y + vx * 8);
    const float2 y45 = *reinterpret_cast<const float2*>(y + vx * 8 + 4);
    const uint8_t m0 = mask[3 * n], m1 = mask[3 * n + 1], m2 = mask[3 * n + 2];
    const cx<T> o0{(T)(s * y03.x), (T)(s * y03.y)}, o1{(T)(s * y03.z), (T)(s * y03.w)},
        o2{(T)(s * y45.x), (T)(s * y45.y)};
    const cx<T> zero{T(0), T(0)};
    stc(z, 3 * n, m0 ? o0 : zero);
    stc(z, 3 * n + 1, m1 ? o1 : zero);
    stc(z, 3 * n + 2, m2 ? o2 : zero);
  }
}

// Loss on the box: target e/s_e on free edges; d = y - t; loss partials of
// sum(d^2) and the free count; dy = 2 d / n_free (n_free from the norm pass,
// scal[cnt_slot]) as bf16 [v][8].
__global__ void __launch_bounds__(256)
    loss_kernel(GridView g, const double* e, const uint8_t* mask, const double* scal, int se_slot,
                const double* counts, int ox0, int oy0, int oz0, int X, int Y, int Z, const float* y,
                bf16* dy, double* part) {
  __shared__ double lds[4];
  double acc[1] = {0.0};
  const int64_t nv = (int64_t)X * Y * Z;
  const double se = scal[se_slot];
  const double ise = se > 0.0 ? 1.0 / se : 0.0;
  const double nf = counts[1] > 0.0 ? counts[1] : 1.0;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nv;
       q += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t qq = (uint32_t)q, t = qq / (uint32_t)X, bx = qq - t * (uint32_t)X;
    const uint32_t bz = t / (uint32_t)Y, by = t - bz * (uint32_t)Y;
    const int i = ox0 + (int)bx, j = oy0 + (int)by, k = oz0 + (int)bz;
    float d[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (i < g.nx && j < g.ny && k < g.nz) {
      const int64_t n = ((int64_t)k * g.ny + j) * g.nx + i;
#pragma unroll
      for (int w = 0; w < 3; ++w) {
        if (!mask[3 * n + w]) continue;
        const cx<double> t = ldc(e, 3 * n + w);
        const double dr = (double)y[q * 8 + 2 * w] - t.re * ise;
        const double di = (double)y[q * 8 + 2 * w + 1] - t.im * ise;
        acc[0] += dr * dr + di * di;
        d[2 * w] = (float)(2.0 * dr / nf);
        d[2 * w + 1] = (float)(2.0 * di / nf);
      }
    }
    bf16x8 o;
#pragma unroll
    for (int c = 0; c < 8; ++c) o[c] = (bf16)d[c];
    reinterpret_cast<bf16x8*>(dy)[q] = o;
  }
  block_partial<1>(acc, part, lds);
}

// Seeded complex noise on the free edges (SplitMix64 counters), in [-1, 1).
__device__ __forceinline__ uint64_t mix64(uint64_t c, uint64_t seed) {
  uint64_t z = seed + (c + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__global__ void noise_kernel(int64_t ne, const uint8_t* mask, uint64_t seed, double* e) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < ne;
       q += (int64_t)gridDim.x * blockDim.x) {
    const double re = 2.0 * ((double)(mix64(2 * q, seed) >> 11) * 0x1.0p-53) - 1.0;
    const double im = 2.0 * ((double)(mix64(2 * q + 1, seed) >> 11) * 0x1.0p-53) - 1.0;
    stc(e, q, mask[q] ? cx<double>{re, im} : cx<double>{0.0, 0.0});
  }
}

// One smoothing pass: each edge value becomes the mean of itself and the
// same component at the six neighbouring nodes (free edges only).
__global__ void smooth_kernel(GridView g, const uint8_t* mask, const double* in, double* out) {
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < g.np;
       n += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t nn = (uint32_t)n, t = nn / (uint32_t)g.nx, k32 = t / (uint32_t)g.ny;
    const int i = (int)(nn - t * (uint32_t)g.nx), j = (int)(t - k32 * (uint32_t)g.ny), k = (int)k32;
    const int64_t sx = 1, sy = g.nx, sz = (int64_t)g.nx * g.ny;
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      const int64_t e = 3 * n + w;
      cx<double> acc = ldc(in, e);
      int cnt = 1;
      if (i > 0) { acc = acc + ldc(in, e - 3 * sx); ++cnt; }
      if (i + 1 < g.nx) { acc = acc + ldc(in, e + 3 * sx); ++cnt; }
      if (j > 0) { acc = acc + ldc(in, e - 3 * sy); ++cnt; }
      if (j + 1 < g.ny) { acc = acc + ldc(in, e + 3 * sy); ++cnt; }
      if (k > 0) { acc = acc + ldc(in, e - 3 * sz); ++cnt; }
      if (k + 1 < g.nz) { acc = acc + ldc(in, e + 3 * sz); ++cnt; }
      const double f = mask[e] ? 1.0 / cnt : 0.0;
      stc(out, e, cx<double>{acc.re * f, acc.im * f});
    }
  }
}

int nblk(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(4096, (n + 255) / 256)); }

// ---------------------------------------------------------------------------
// Network state
// ---------------------------------------------------------------------------
struct DevLayer {
  Spec s;
  LayerMats mm;
  int64_t w_off, b_off;
  bf16* bf = nullptr;  // [rows_pad(nf)][ldf]
  int64_t ldf = 0;
  bf16* bb = nullptr;  // [rows_pad(nb)][ldb]
  int64_t ldb = 0;
};

// Activation (and, for training, gradient) buffers for an X x Y x Z box.
struct Acts {
  int X = 0, Y = 0, Z = 0;
  bool grads = false;
  std::vector<void*> allocs;
  bf16 *x0, *a1, *cat1, *p1, *a2, *cat2, *p2, *a3, *b3, *d2a, *d2b, *d1a, *d1b;
  float* y;
  // training
  float *g_cat1, *g_d1a, *g_d1b, *g_a1, *g_cat2, *g_d2a, *g_d2b, *g_a2, *g_p1, *g_a3, *g_b3, *g_p2;
  bf16 *dy, *dpre, *xt, *dt;
  float* part;
  int64_t xt_bytes = 0, dt_bytes = 0, part_bytes = 0;
  ~Acts() {
    for (void* p : allocs) (void)hipFree(p);
  }
};

}  // namespace

struct fit_precond {
  int device = 0;
  int c = 16;
  int64_t nparams = 0;
  std::vector<DevLayer> layers;
  float *P = nullptr, *G = nullptr, *Mo = nullptr, *Vo = nullptr;  // params, grads, Adam moments
  bf16* wbuf = nullptr;  // all B matrices
  double* scal = nullptr;  // device scalars: [0] s of v / s_r, [1] s_e, [2..3] sums, [4..] partials
  double* part = nullptr;  // reduction partials
  double* counts = nullptr;  // [0] sum, [1] free count of the last box norm
  int adam_t = 0;
  std::unique_ptr<Acts> acts;  // cached for the last box size
  fit_status init(int dev, int c_);
  fit_status upload_weights(hipStream_t s);
  ~fit_precond();
};

namespace {

template <class T>
T* dalloc(Acts& a, int64_t n, fit_status* st) {
  void* p = nullptr;
  if (*st != FIT_OK) return nullptr;
  if (hipMalloc(&p, std::max<int64_t>(n, 1) * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    set_error("preconditioner: device allocation failed");
    *st = FIT_E_NOMEM;
    return nullptr;
  }
  a.allocs.push_back(p);
  return (T*)p;
}

fit_status make_acts(fit_precond* p, int X, int Y, int Z, bool grads, std::unique_ptr<Acts>& out) {
  if (out && out->X == X && out->Y == Y && out->Z == Z && (out->grads || !grads)) return FIT_OK;
  out.reset();
  std::unique_ptr<Acts> a(new Acts());
  a->X = X;
  a->Y = Y;
  a->Z = Z;
  a->grads = grads;
  const int c = p->c;
  const int64_t V1 = (int64_t)X * Y * Z, V2 = V1 / 8, V3 = V1 / 64;
  fit_status st = FIT_OK;
  a->x0 = dalloc<bf16>(*a, V1 * 16, &st);
  a->a1 = dalloc<bf16>(*a, V1 * c, &st);
  a->cat1 = dalloc<bf16>(*a, V1 * 2 * c, &st);
  a->p1 = dalloc<bf16>(*a, V2 * 2 * c, &st);
  a->a2 = dalloc<bf16>(*a, V2 * 2 * c, &st);
  a->cat2 = dalloc<bf16>(*a, V2 * 4 * c, &st);
  a->p2 = dalloc<bf16>(*a, V3 * 4 * c, &st);
  a->a3 = dalloc<bf16>(*a, V3 * 4 * c, &st);
  a->b3 = dalloc<bf16>(*a, V3 * 4 * c, &st);
  a->d2a = dalloc<bf16>(*a, V2 * 2 * c, &st);
  a->d2b = dalloc<bf16>(*a, V2 * 2 * c, &st);
  a->d1a = dalloc<bf16>(*a, V1 * c, &st);
  a->d1b = dalloc<bf16>(*a, V1 * c, &st);
  a->y = dalloc<float>(*a, V1 * 8, &st);
  if (grads) {
    a->g_cat1 = dalloc<float>(*a, V1 * 2 * c, &st);
    a->g_d1a = dalloc<float>(*a, V1 * c, &st);
    a->g_d1b = dalloc<float>(*a, V1 * c, &st);
    a->g_a1 = dalloc<float>(*a, V1 * c, &st);
    a->g_cat2 = dalloc<float>(*a, V2 * 4 * c, &st);
    a->g_d2a = dalloc<float>(*a, V2 * 2 * c, &st);
    a->g_d2b = dalloc<float>(*a, V2 * 2 * c, &st);
    a->g_a2 = dalloc<float>(*a, V2 * 2 * c, &st);
    a->g_p1 = dalloc<float>(*a, V2 * 2 * c, &st);
    a->g_a3 = dalloc<float>(*a, V3 * 4 * c, &st);
    a->g_b3 = dalloc<float>(*a, V3 * 4 * c, &st);
    a->g_p2 = dalloc<float>(*a, V3 * 4 * c, &st);
    a->dy = dalloc<bf16>(*a, V1 * 8, &st);
    a->dpre = dalloc<bf16>(*a, V1 * std::max(c, 8), &st);
    // weight-gradient scratch: XT [rows][ld] and dT [rows][ld] over the largest layer
    static const int in_level[kNLayers] = {1, 1, 1, 2, 2, 2, 3, 3, 3, 2, 2, 2, 1, 1, 1};
    static const int out_level[kNLayers] = {1, 1, 2, 2, 2, 3, 3, 3, 2, 2, 2, 1, 1, 1, 1};
    const int64_t Vs[4] = {0, V1, V2, V3};
    int64_t xt = 0, dt = 0, pt = 0;
    for (size_t li = 0; li < p->layers.size(); ++li) {
      const DevLayer& L = p->layers[li];
      const Spec& s = L.s;
      const bool up = s.kind == L_UP2;
      const int64_t nv = up ? Vs[in_level[li]] : Vs[out_level[li]];
      const int64_t ld = pad32(nv);
      const int64_t m = up ? pad8(s.cin) : L.mm.kf;
      const int64_t ncols = up ? 8LL * s.cout : s.cout;
      const int64_t nrows = std::max<int64_t>(rows_pad(ncols), pad8(s.cout));
      xt = std::max(xt, m * ld);
      dt = std::max(dt, nrows * ld);
      pt = std::max(pt, kMaxSplits * m * ncols);
    }
    a->xt = dalloc<bf16>(*a, xt, &st);
    a->dt = dalloc<bf16>(*a, dt, &st);
    a->part = dalloc<float>(*a, pt, &st);
    a->xt_bytes = xt;
    a->dt_bytes = dt;
    a->part_bytes = pt;
  }
  if (st != FIT_OK) return st;
  // the concat buffers' and x0's unused channels must read as zero
  FIT_HIP(hipMemset(a->x0, 0, V1 * 16 * sizeof(bf16)));
  out = std::move(a);
  return FIT_OK;
}

struct Box {
  int X, Y, Z;
};

// One GEMM launch.
fit_status gemm(const GemmArgs& g, int64_t n_cols, hipStream_t s, int splits = 1) {
  const int nt = ntile(n_cols);
  GemmArgs a = g;
  const int64_t kpad = pad32(a.K);
  if (splits < 1) splits = 1;
  a.k_chunk = pad32((kpad + splits - 1) / splits);
  // 3x3x3 convolutions with 8, 16, 32 or 64 input channels take the
  // LDS-staged kernel
  const bool lds_cin = a.cin == 8 || a.cin == 16 || a.cin == 32 || a.cin == 64;
  // bf16 outputs whose 8-channel groups are 16-byte aligned take the kernels'
  // packed-store instantiation
  const bool pk = a.out == O_BF16 && (a.o_ld & 7) == 0 && (!a.up || (a.up_c & 7) == 0) &&
                  (reinterpret_cast<uintptr_t>(a.o16) & 15) == 0;
  if (a.gather == G_CONV3 && splits == 1 && lds_cin && a.K == 27LL * a.cin && a.ox == a.ix && a.oy == a.iy &&
      a.M == (int64_t)a.ix * a.iy * a.iz && !a.up) {
    const int64_t nb = (int64_t)((a.ix + kBrX - 1) / kBrX) * ((a.iy + kBrY - 1) / kBrY) * ((a.iz + kBrZ - 1) / kBrZ);
    // small coarse levels: narrower column tiles give more workgroups (the B
    // rows stay padded to the wider tile, a multiple of the narrower one)
    int ntc = nt;
    while (ntc > 16 && nb * ((n_cols + ntc - 1) / ntc) < 1024) ntc /= 2;
    const dim3 grid((unsigned)nb, (unsigned)((n_cols + ntc - 1) / ntc), 1);
    const int tok = prof_begin(s);
#define CONV(NT, CI)                                                                   \
  if (ntc == NT && a.cin == CI) {                                                      \
    if (pk)                                                                            \
      hipLaunchKernelGGL((conv3_lds_kernel<NT, CI, true>), grid, dim3(256), 0, s, a);  \
    else                                                                               \
      hipLaunchKernelGGL((conv3_lds_kernel<NT, CI, false>), grid, dim3(256), 0, s, a); \
  }
    CONV(16, 8) CONV(16, 16) CONV(16, 32) CONV(16, 64) CONV(32, 8) CONV(32, 16) CONV(32, 32) CONV(32, 64)
    CONV(64, 8) CONV(64, 16) CONV(64, 32) CONV(64, 64)
#undef CONV
    FIT_HIP(hipGetLastError());
    prof_end(tok, s, "unet_conv3_lds_bf16");
    return FIT_OK;
  }
  const dim3 grid((unsigned)((a.M + 127) / 128), (unsigned)((n_cols + nt - 1) / nt), (unsigned)splits);
  const int tok = prof_begin(s);
#define IGEMM(NT)                                                                  \
  if (nt == NT) {                                                                  \
    if (pk)                                                                        \
      hipLaunchKernelGGL((igemm_kernel<NT, true>), grid, dim3(256), 0, s, a);      \
    else                                                                           \
      hipLaunchKernelGGL((igemm_kernel<NT, false>), grid, dim3(256), 0, s, a);     \
  }
  IGEMM(16) IGEMM(32) IGEMM(64)
#undef IGEMM
  FIT_HIP(hipGetLastError());
  prof_end(tok, s, "unet_igemm_bf16");
  return FIT_OK;
}

// Forward pass of layer L: in (bf16, ld, dims of the input tensor) -> out.
fit_status layer_fwd(const fit_precond* p, const DevLayer& L, const bf16* in, int64_t in_ld, Box bi,
                     bf16* o16, float* o32, int64_t o_ld, hipStream_t s) {
  const Spec& sp = L.s;
  GemmArgs g{};
  g.a = in;
  g.a_ld = in_ld;
  g.cin = pad8(sp.cin);
  g.b = L.bf;
  g.ldb = L.ldf;
  g.bias = p->P + L.b_off;
  g.relu = sp.kind == L_PW ? 0 : 1;
  g.o16 = o16;
  g.o32 = o32;
  g.o_ld = o_ld;
  g.out = o16 ? O_BF16 : O_F32;
  g.ix = bi.X;
  g.iy = bi.Y;
  g.iz = bi.Z;
  g.K = L.mm.kf;
  g.N = (int)L.mm.nf;
  switch (sp.kind) {
    case L_CONV3:
      g.gather = G_CONV3;
      g.M = (int64_t)bi.X * bi.Y * bi.Z;
      g.ox = bi.X;
      g.oy = bi.Y;
      break;
    case L_DOWN2:
      g.gather = G_DOWN2;
      g.M = (int64_t)bi.X * bi.Y * bi.Z / 8;
      g.ox = bi.X / 2;
      g.oy = bi.Y / 2;
      break;
    case L_UP2:
      g.gather = G_PW;
      g.M = (int64_t)bi.X * bi.Y * bi.Z;
      g.ox = bi.X;
      g.oy = bi.Y;
      g.up = 1;
      g.up_c = sp.cout;
      g.up_x = 2 * bi.X;
      g.up_y = 2 * bi.Y;
      break;
    default:
      g.gather = G_PW;
      g.M = (int64_t)bi.X * bi.Y * bi.Z;
      g.ox = bi.X;
      g.oy = bi.Y;
      break;
  }
  return gemm(g, L.mm.nf, s);
}

fit_status forward(fit_precond* p, Acts& a, hipStream_t s) {
  const int c = p->c;
  const Box b1{a.X, a.Y, a.Z}, b2{a.X / 2, a.Y / 2, a.Z / 2}, b3{a.X / 4, a.Y / 4, a.Z / 4};
  const auto& Ls = p->layers;
  fit_status st;
#define FWD(i, in, ld, box, o16, o32, old)                                              \
  if ((st = layer_fwd(p, Ls[i], in, ld, box, o16, o32, old, s)) != FIT_OK) return st;
  FWD(0, a.x0, 16, b1, a.a1, nullptr, c);
  FWD(1, a.a1, c, b1, a.cat1 + c, nullptr, 2 * c);
  FWD(2, a.cat1 + c, 2 * c, b1, a.p1, nullptr, 2 * c);
  FWD(3, a.p1, 2 * c, b2, a.a2, nullptr, 2 * c);
  FWD(4, a.a2, 2 * c, b2, a.cat2 + 2 * c, nullptr, 4 * c);
  FWD(5, a.cat2 + 2 * c, 4 * c, b2, a.p2, nullptr, 4 * c);
  FWD(6, a.p2, 4 * c, b3, a.a3, nullptr, 4 * c);
  FWD(7, a.a3, 4 * c, b3, a.b3, nullptr, 4 * c);
  FWD(8, a.b3, 4 * c, b3, a.cat2, nullptr, 4 * c);
  FWD(9, a.cat2, 4 * c, b2, a.d2a, nullptr, 2 * c);
  FWD(10, a.d2a, 2 * c, b2, a.d2b, nullptr, 2 * c);
  FWD(11, a.d2b, 2 * c, b2, a.cat1, nullptr, 2 * c);
  FWD(12, a.cat1, 2 * c, b1, a.d1a, nullptr, c);
  FWD(13, a.d1a, c, b1, a.d1b, nullptr, c);
  FWD(14, a.d1b, c, b1, nullptr, a.y, 8);
#undef FWD
  return FIT_OK;
}

// Backward of layer L.  in: the layer input (bf16, ld) on box bi; out: its
// bf16 output (ld o_ld) for the ReLU mask (nullptr for the head, whose
// gradient dpre is given); gout: fp32 gradient of the output; gin: fp32
// gradient of the input to accumulate into (nullptr: not needed).
fit_status layer_bwd(fit_precond* p, Acts& a, const DevLayer& L, const bf16* in, int64_t in_ld, Box bi,
                     const bf16* out, int64_t o_ld, const float* gout, int64_t g_ld, const bf16* dpre_given,
                     float* gin, int64_t gin_ld, float scale, hipStream_t s) {
  const Spec& sp = L.s;
  const int cip = pad8(sp.cin), cop = pad8(sp.cout);
  // output box
  Box bo = bi;
  if (sp.kind == L_DOWN2) bo = Box{bi.X / 2, bi.Y / 2, bi.Z / 2};
  if (sp.kind == L_UP2) bo = Box{bi.X * 2, bi.Y * 2, bi.Z * 2};
  const int64_t nvo = (int64_t)bo.X * bo.Y * bo.Z, nvi = (int64_t)bi.X * bi.Y * bi.Z;
  // 1. dpre (bf16, [nvo][cop])
  const bf16* dpre = dpre_given;
  if (!dpre) {
    hipLaunchKernelGGL(relu_bwd_kernel, dim3(nblk(nvo * cop)), dim3(256), 0, s, gout, g_ld, out, o_ld, 1,
                       nvo, sp.cout, cop, a.dpre);
    FIT_HIP(hipGetLastError());
    dpre = a.dpre;
  }
  // 2. weight gradient: XT (rows = forward K) x dT (rows = output channels)
  const bool up = sp.kind == L_UP2;
  const int64_t nv_w = up ? nvi : nvo;  // reduction length (coarse side for up2)
  const int64_t ld = pad32(nv_w);
  const int64_t M = up ? cip : L.mm.kf;
  const int64_t ncols = up ? 8LL * sp.cout : sp.cout;
  const int nrows = (int)rows_pad(ncols);
  if (M * ld > a.xt_bytes || (int64_t)std::max<int64_t>(nrows, cop) * ld > a.dt_bytes) {
    set_error("preconditioner: weight-gradient scratch too small");
    return FIT_E_DEVICE;
  }
  const int gk = up ? L_PW : sp.kind;
  hipLaunchKernelGGL(im2colT_kernel, dim3((unsigned)((ld + 255) / 256), (unsigned)(M / cip)), dim3(256), 0, s,
                     in, in_ld, cip, gk, bi.X, bi.Y, bi.Z, up ? bi.X : bo.X, up ? bi.Y : bo.Y, nv_w, a.xt, ld);
  FIT_HIP(hipGetLastError());
  hipLaunchKernelGGL(dgradT_kernel, dim3(nblk((int64_t)std::max(nrows, cop) * ld)), dim3(256), 0, s, dpre,
                     cop, sp.cout, up ? 1 : 0, bi.X, bi.Y, nv_w, std::max(nrows, cop), a.dt, ld);
  FIT_HIP(hipGetLastError());
  // split K (the voxels) so that the launch has about 1,024 workgroups, each
  // summing at least 256 voxels; the split count depends on the shapes only,
  // so the summation order is fixed
  const int64_t tiles = ((M + 127) / 128) * ((ncols + ntile(ncols) - 1) / ntile(ncols));
  int splits = (int)std::min<int64_t>(std::min<int64_t>(kMaxSplits, std::max<int64_t>(1, ld / 256)),
                                      std::max<int64_t>(1, (1024 + tiles - 1) / tiles));
  while (splits > 1 && (int64_t)splits * M * ncols > a.part_bytes) --splits;
  {
    GemmArgs g{};
    g.a = a.xt;
    g.a_ld = ld;
    g.cin = 8;
    g.gather = G_PW;
    g.M = M;
    g.K = ld;
    g.b = a.dt;
    g.ldb = ld;
    g.N = (int)ncols;
    g.out = O_PART;
    g.o32 = a.part;
    fit_status st = gemm(g, ncols, s, splits);
    if (st != FIT_OK) return st;
  }
  const int64_t nw = (int64_t)sp.taps * sp.cin * sp.cout;
  hipLaunchKernelGGL(reduce_dw_kernel, dim3((unsigned)((nw + 63) / 64)), dim3(256), 0, s, a.part, splits, M,
                     ncols, sp.kind, sp.taps, sp.cin, sp.cout, scale, p->G + L.w_off);
  FIT_HIP(hipGetLastError());
  hipLaunchKernelGGL(bias_grad_kernel, dim3(sp.cout), dim3(1024), 0, s, a.dt, ld, sp.cout, up ? 1 : 0, scale,
                     p->G + L.b_off);
  FIT_HIP(hipGetLastError());
  // 3. input gradient
  if (!gin) return FIT_OK;
  GemmArgs g{};
  g.a = dpre;
  g.a_ld = cop;
  g.cin = cop;
  g.b = L.bb;
  g.ldb = L.ldb;
  g.K = L.mm.kb;
  g.N = (int)L.mm.nb;
  g.out = O_F32ACC;
  g.o32 = gin;
  g.o_ld = gin_ld;
  switch (sp.kind) {
    case L_CONV3:  // conv3 with flipped taps over the output gradient
      g.gather = G_CONV3;
      g.ix = bo.X;
      g.iy = bo.Y;
      g.iz = bo.Z;
      g.M = nvi;
      g.ox = bi.X;
      g.oy = bi.Y;
      break;
    case L_DOWN2:  // transposed form: each coarse voxel scatters to its children
      g.gather = G_PW;
      g.M = nvo;
      g.ox = bo.X;
      g.oy = bo.Y;
      g.up = 1;
      g.up_c = sp.cin;
      g.up_x = bi.X;
      g.up_y = bi.Y;
      break;
    case L_UP2:  // strided form: each coarse voxel gathers its children
      g.gather = G_DOWN2;
      g.ix = bo.X;
      g.iy = bo.Y;
      g.iz = bo.Z;
      g.M = nvi;
      g.ox = bi.X;
      g.oy = bi.Y;
      break;
    default:
      g.gather = G_PW;
      g.M = nvi;
      g.ox = bi.X;
      g.oy = bi.Y;
      break;
  }
  return gemm(g, L.mm.nb, s);
}

fit_status zero_f32(float* p, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(fill_f32_kernel, dim3(nblk(n)), dim3(256), 0, s, p, n, 0.f);
  FIT_HIP(hipGetLastError());
  return FIT_OK;
}

// Backward pass from a.dy; gradients accumulate into p->G scaled by `scale`.
fit_status backward(fit_precond* p, Acts& a, float scale, hipStream_t s) {
  const int c = p->c;
  const Box b1{a.X, a.Y, a.Z}, b2{a.X / 2, a.Y / 2, a.Z / 2}, b3{a.X / 4, a.Y / 4, a.Z / 4};
  const int64_t V1 = (int64_t)a.X * a.Y * a.Z, V2 = V1 / 8, V3 = V1 / 64;
  fit_status st;
  struct Z {
    float* p;
    int64_t n;
  } zs[] = {{a.g_cat1, V1 * 2 * c}, {a.g_d1a, V1 * c}, {a.g_d1b, V1 * c}, {a.g_a1, V1 * c},
            {a.g_cat2, V2 * 4 * c}, {a.g_d2a, V2 * 2 * c}, {a.g_d2b, V2 * 2 * c}, {a.g_a2, V2 * 2 * c},
            {a.g_p1, V2 * 2 * c},   {a.g_a3, V3 * 4 * c},  {a.g_b3, V3 * 4 * c},  {a.g_p2, V3 * 4 * c}};
  for (auto& z : zs)
    if ((st = zero_f32(z.p, z.n, s)) != FIT_OK) return st;
  const auto& Ls = p->layers;
#define BWD(i, in, in_ld, box, out, o_ld, gout, g_ld, dgiven, gin, gin_ld)                          \
  if ((st = layer_bwd(p, a, Ls[i], in, in_ld, box, out, o_ld, gout, g_ld, dgiven, gin, gin_ld, scale, s)) != \
      FIT_OK)                                                                                       \
    return st;
  BWD(14, a.d1b, c, b1, nullptr, 0, nullptr, 0, a.dy, a.g_d1b, c);
  BWD(13, a.d1a, c, b1, a.d1b, c, a.g_d1b, c, nullptr, a.g_d1a, c);
  BWD(12, a.cat1, 2 * c, b1, a.d1a, c, a.g_d1a, c, nullptr, a.g_cat1, 2 * c);
  BWD(11, a.d2b, 2 * c, b2, a.cat1, 2 * c, a.g_cat1, 2 * c, nullptr, a.g_d2b, 2 * c);
  BWD(10, a.d2a, 2 * c, b2, a.d2b, 2 * c, a.g_d2b, 2 * c, nullptr, a.g_d2a, 2 * c);
  BWD(9, a.cat2, 4 * c, b2, a.d2a, 2 * c, a.g_d2a, 2 * c, nullptr, a.g_cat2, 4 * c);
  BWD(8, a.b3, 4 * c, b3, a.cat2, 4 * c, a.g_cat2, 4 * c, nullptr, a.g_b3, 4 * c);
  BWD(7, a.a3, 4 * c, b3, a.b3, 4 * c, a.g_b3, 4 * c, nullptr, a.g_a3, 4 * c);
  BWD(6, a.p2, 4 * c, b3, a.a3, 4 * c, a.g_a3, 4 * c, nullptr, a.g_p2, 4 * c);
  BWD(5, a.cat2 + 2 * c, 4 * c, b2, a.p2, 4 * c, a.g_p2, 4 * c, nullptr, a.g_cat2 + 2 * c, 4 * c);
  BWD(4, a.a2, 2 * c, b2, a.cat2 + 2 * c, 4 * c, a.g_cat2 + 2 * c, 4 * c, nullptr, a.g_a2, 2 * c);
  BWD(3, a.p1, 2 * c, b2, a.a2, 2 * c, a.g_a2, 2 * c, nullptr, a.g_p1, 2 * c);
  BWD(2, a.cat1 + c, 2 * c, b1, a.p1, 2 * c, a.g_p1, 2 * c, nullptr, a.g_cat1 + c, 2 * c);
  BWD(1, a.a1, c, b1, a.cat1 + c, 2 * c, a.g_cat1 + c, 2 * c, nullptr, a.g_a1, c);
  BWD(0, a.x0, 16, b1, a.a1, c, a.g_a1, c, nullptr, nullptr, 0);
#undef BWD
  return FIT_OK;
}

// The grid's edge mask, computed on the first request and cached in the grid
// (which owns it); ready for use on any stream when this returns.
fit_status edge_mask_of(const fit_grid* g, uint8_t** out, hipStream_t s) {
  fit_grid* gm = const_cast<fit_grid*>(g);  // the cache is not part of the grid's value
  std::lock_guard<std::mutex> lk(gm->mask_mu);
  if (!gm->d_mask) {
    void* m = nullptr;
    FIT_HIP(hipMalloc(&m, (size_t)g->ne));
    fit_status st = fit_edge_mask(g, (uint8_t*)m, s);
    if (st == FIT_OK) {
      const hipError_t e = hipStreamSynchronize(s);
      if (e != hipSuccess) st = hip_fail(e, "edge mask");
    }
    if (st != FIT_OK) {
      (void)hipFree(m);
      return st;
    }
    gm->d_mask = (uint8_t*)m;
  }
  *out = gm->d_mask;
  return FIT_OK;
}

// rms over free edges of v in the node box -> p->scal[slot]; sums -> p->counts.
template <class T>
fit_status box_rms(fit_precond* p, const fit_grid* g, const T* v, const uint8_t* mask, int o[3], int ext[3],
                   int slot, hipStream_t s) {
  const int64_t nb = (int64_t)ext[0] * ext[1] * ext[2];
  const int nbk = nblk(nb);
  hipLaunchKernelGGL(box_norm_kernel<T>, dim3(nbk), dim3(256), 0, s, g->view, v, mask, o[0], o[1], o[2],
                     ext[0], ext[1], ext[2], p->part);
  FIT_HIP(hipGetLastError());
  FIT_HIP(launch_finish<2>(p->part, nbk, RmsFinish{p->scal, slot}, s));
  FIT_HIP(launch_finish<2>(p->part, nbk, StoreSumsPtr{p->counts}, s));
  return FIT_OK;
}

int round4(int n) { return (n + 3) / 4 * 4; }

}  // namespace

// ---------------------------------------------------------------------------
// fit_precond members
// ---------------------------------------------------------------------------
fit_status fit_precond::init(int dev, int c_) {
  device = dev;
  c = c_;
  const std::vector<Spec> sp = specs(c);
  int64_t off = 0, wb = 0;
  for (const Spec& s : sp) {
    DevLayer L;
    L.s = s;
    L.mm = mats_of(s);
    L.w_off = off;
    off += (int64_t)s.taps * s.cin * s.cout;
    L.b_off = off;
    off += s.cout;
    L.ldf = pad32(L.mm.kf);
    L.ldb = pad32(L.mm.kb);
    wb += rows_pad(L.mm.nf) * L.ldf + rows_pad(L.mm.nb) * L.ldb;
    layers.push_back(L);
  }
  nparams = off;
  const size_t fb = sizeof(float) * (size_t)nparams;
  FIT_HIP(hipMalloc(&P, fb));
  FIT_HIP(hipMalloc(&G, fb));
  FIT_HIP(hipMalloc(&Mo, fb));
  FIT_HIP(hipMalloc(&Vo, fb));
  FIT_HIP(hipMemset(G, 0, fb));
  FIT_HIP(hipMemset(Mo, 0, fb));
  FIT_HIP(hipMemset(Vo, 0, fb));
  FIT_HIP(hipMalloc(&wbuf, sizeof(bf16) * (size_t)wb));
  FIT_HIP(hipMemset(wbuf, 0, sizeof(bf16) * (size_t)wb));
  bf16* q = wbuf;
  for (DevLayer& L : layers) {
    L.bf = q;
    q += rows_pad(L.mm.nf) * L.ldf;
    L.bb = q;
    q += rows_pad(L.mm.nb) * L.ldb;
  }
  FIT_HIP(hipMalloc(&scal, sizeof(double) * 8));
  FIT_HIP(hipMemset(scal, 0, sizeof(double) * 8));
  FIT_HIP(hipMalloc(&counts, sizeof(double) * 4));
  FIT_HIP(hipMalloc(&part, sizeof(double) * 4 * 4096));
  return FIT_OK;
}

fit_status fit_precond::upload_weights(hipStream_t s) {
  for (DevLayer& L : layers) {
    const Spec& sp = L.s;
    const int64_t n = (int64_t)sp.taps * sp.cin * sp.cout;
    hipLaunchKernelGGL(wtransform_kernel, dim3(nblk(n)), dim3(256), 0, s, P + L.w_off, sp.kind, sp.taps, sp.cin,
                       sp.cout, L.bf, L.ldf, L.bb, L.ldb);
    FIT_HIP(hipGetLastError());
  }
  return FIT_OK;
}

fit_precond::~fit_precond() {
  acts.reset();
  for (void* q : {(void*)P, (void*)G, (void*)Mo, (void*)Vo, (void*)wbuf, (void*)scal, (void*)counts, (void*)part})
    if (q) (void)hipFree(q);
}

namespace {

fit_status create(int c, int device, uint64_t seed, const float* init, fit_precond** out) {
  if (c < 8 || c > 32 || c % 8) {
    set_error("preconditioner: base_channels must be 8, 16, 24 or 32");
    return FIT_E_INVALID;
  }
  std::unique_ptr<fit_precond> p(new fit_precond());
  DeviceScope dev(device);
  fit_status st = p->init(device, c);
  if (st != FIT_OK) return st;
  std::vector<float> h((size_t)p->nparams);
  if (init) {
    std::memcpy(h.data(), init, sizeof(float) * h.size());
  } else {
    // He-uniform weights, zero biases, from a SplitMix64 stream
    uint64_t ctr = 0;
    for (const DevLayer& L : p->layers) {
      const Spec& s = L.s;
      const double lim = std::sqrt(6.0 / (s.taps * s.cin));
      const int64_t nw = (int64_t)s.taps * s.cin * s.cout;
      for (int64_t q = 0; q < nw; ++q) {
        uint64_t z = seed + (++ctr) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        h[L.w_off + q] = (float)(lim * (2.0 * ((double)(z >> 11) * 0x1.0p-53) - 1.0));
      }
      for (int q = 0; q < s.cout; ++q) h[L.b_off + q] = 0.f;
    }
  }
  FIT_HIP(hipMemcpy(p->P, h.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice));
  if ((st = p->upload_weights(nullptr)) != FIT_OK) return st;
  FIT_HIP(hipDeviceSynchronize());
  *out = p.release();
  return FIT_OK;
}

// Forward on the whole grid of g (padded to multiples of 4): z = s U(v/s).
template <class T>
fit_status apply_grid(fit_precond* p, const fit_grid* g, double omega, const T* v, T* z, const uint8_t* mask,
                      hipStream_t s) {
  const int X = round4(g->view.nx), Y = round4(g->view.ny), Z = round4(g->view.nz);
  fit_status st = make_acts(p, X, Y, Z, false, p->acts);
  if (st != FIT_OK) return st;
  Acts& a = *p->acts;
  int o[3] = {0, 0, 0}, ext[3] = {g->view.nx, g->view.ny, g->view.nz};
  if ((st = box_rms<T>(p, g, v, mask, o, ext, 0, s)) != FIT_OK) return st;
  const int64_t V1 = (int64_t)X * Y * Z;
  hipLaunchKernelGGL(features_kernel<T>, dim3(nblk(V1)), dim3(256), 0, s, g->view, v, mask, p->scal, 0, omega,
                     0, 0, 0, X, Y, Z, a.x0);
  FIT_HIP(hipGetLastError());
  if ((st = forward(p, a, s)) != FIT_OK) return st;
  hipLaunchKernelGGL(output_kernel<T>, dim3(nblk(g->view.np)), dim3(256), 0, s, g->view, a.y, mask, p->scal, 0,
                     X, Y, z);
  FIT_HIP(hipGetLastError());
  return FIT_OK;
}

// Loss and gradient (accumulated into p->G with `scale`) of one pair on the
// node box [o, o + ext) (ext multiples of 4).  The loss sum is left in
// p->part[0] (via *loss_dev).
fit_status pair_step(fit_precond* p, const fit_grid* g, double omega, const double* r, const double* e,
                     const uint8_t* mask, int o[3], int ext[3], float scale, double* loss_dev, hipStream_t s) {
  fit_status st = make_acts(p, ext[0], ext[1], ext[2], true, p->acts);
  if (st != FIT_OK) return st;
  Acts& a = *p->acts;
  if ((st = box_rms<double>(p, g, e, mask, o, ext, 1, s)) != FIT_OK) return st;  // s_e, counts
  if ((st = box_rms<double>(p, g, r, mask, o, ext, 0, s)) != FIT_OK) return st;  // s_r
  const int64_t V1 = (int64_t)ext[0] * ext[1] * ext[2];
  hipLaunchKernelGGL(features_kernel<double>, dim3(nblk(V1)), dim3(256), 0, s, g->view, r, mask, p->scal, 0,
                     omega, o[0], o[1], o[2], ext[0], ext[1], ext[2], a.x0);
  FIT_HIP(hipGetLastError());
  if ((st = forward(p, a, s)) != FIT_OK) return st;
  const int nbk = nblk(V1);
  hipLaunchKernelGGL(loss_kernel, dim3(nbk), dim3(256), 0, s, g->view, e, mask, p->scal, 1, p->counts, o[0],
                     o[1], o[2], ext[0], ext[1], ext[2], a.y, a.dy, p->part);
  FIT_HIP(hipGetLastError());
  FIT_HIP(launch_finish<1>(p->part, nbk, LossFinish{loss_dev, p->counts}, s));
  return backward(p, a, scale, s);
}

}  // namespace

// ---------------------------------------------------------------------------
// FGMRES adapter: z = M(v) on the solver's stream.  The network is trained on
// the unscaled system, so with the symmetric scaling (the solver works on
// S A S) it is applied as S^-1 U(S^-1 v).
// ---------------------------------------------------------------------------
namespace {
struct UNetApply : PrecondApply {
  fit_precond* p = nullptr;
  const fit_grid* g = nullptr;
  double omega = 0.0;
  uint8_t* mask = nullptr;
  void* tmp[2] = {nullptr, nullptr};
  ~UNetApply() override {
    (void)hipFree(tmp[0]);
    (void)hipFree(tmp[1]);
  }
  template <class T>
  fit_status run(Ctx& c, const T* v, T* z) {
    if (!c.sym) return apply_grid<T>(p, g, omega, v, z, mask, c.s);
    T* a = (T*)tmp[0];
    T* b = (T*)tmp[1];
    fit_status st = xform<T, T, XF_SCALE>(c, true, true, v, a, 1.0, false);
    if (st == FIT_OK) st = apply_grid<T>(p, g, omega, a, b, mask, c.s);
    if (st == FIT_OK) st = xform<T, T, XF_SCALE>(c, true, true, b, z, 1.0, false);
    return st;
  }
  fit_status apply(Ctx& c, const void* v, void* z, bool f32) override {
    DeviceScope dev(p->device);
    return f32 ? run<float>(c, (const float*)v, (float*)z) : run<double>(c, (const double*)v, (double*)z);
  }
};
}  // namespace

namespace fit {
PrecondApply* precond_apply_of(fit_precond* p, const fit_grid* g, double omega) {
  if (!p || !g || p->device != g->device) return nullptr;
  DeviceScope dev(g->device);
  std::unique_ptr<UNetApply> a(new UNetApply());
  a->p = p;
  a->g = g;
  a->omega = omega;
  if (edge_mask_of(g, &a->mask, nullptr) != FIT_OK) return nullptr;
  for (auto& t : a->tmp)
    if (hipMalloc(&t, (size_t)g->ne * 16) != hipSuccess) return nullptr;
  if (hipDeviceSynchronize() != hipSuccess) return nullptr;
  return a.release();
}
}  // namespace fit

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" fit_status fit_precond_create(const fit_precond_cfg* cfg, int device, fit_precond** out) {
  if (!out) {
    set_error("fit_precond_create: NULL out");
    return FIT_E_INVALID;
  }
  *out = nullptr;
  const int c = cfg && cfg->base_channels ? cfg->base_channels : 16;
  const uint64_t seed = cfg ? (uint64_t)(uint32_t)cfg->seed : 0;
  return create(c, device, seed, nullptr, out);
}

extern "C" void fit_precond_destroy(fit_precond* p) {
  if (!p) return;
  DeviceScope dev(p->device);
  (void)hipDeviceSynchronize();
  delete p;
}

extern "C" fit_status fit_precond_save(const fit_precond* p, void* blob, size_t* n) {
  if (!p || !n) {
    set_error("fit_precond_save: NULL argument");
    return FIT_E_INVALID;
  }
  const size_t need = 24 + sizeof(float) * (size_t)p->nparams;
  if (!blob) {
    *n = need;
    return FIT_OK;
  }
  if (*n < need) {
    set_error("fit_precond_save: blob too small");
    *n = need;
    return FIT_E_INVALID;
  }
  DeviceScope dev(p->device);
  char* b = (char*)blob;
  const uint64_t magic = kMagic;
  const int32_t c = p->c, zero = 0;
  const int64_t np = p->nparams;
  std::memcpy(b, &magic, 8);
  std::memcpy(b + 8, &c, 4);
  std::memcpy(b + 12, &zero, 4);
  std::memcpy(b + 16, &np, 8);
  FIT_HIP(hipDeviceSynchronize());
  FIT_HIP(hipMemcpy(b + 24, p->P, sizeof(float) * (size_t)np, hipMemcpyDeviceToHost));
  *n = need;
  return FIT_OK;
}

extern "C" fit_status fit_precond_load(const void* blob, size_t n, int device, fit_precond** out) {
  if (!blob || !out || n < 24) {
    set_error("fit_precond_load: NULL argument or short blob");
    return FIT_E_INVALID;
  }
  *out = nullptr;
  const char* b = (const char*)blob;
  uint64_t magic;
  int32_t c;
  int64_t np;
  std::memcpy(&magic, b, 8);
  std::memcpy(&c, b + 8, 4);
  std::memcpy(&np, b + 16, 8);
  if (magic != kMagic || c < 8 || c > 32 || c % 8) {
    set_error("fit_precond_load: not a preconditioner blob");
    return FIT_E_INVALID;
  }
  int64_t want = 0;
  for (const Spec& s : specs(c)) want += (int64_t)s.taps * s.cin * s.cout + s.cout;
  if (np != want || n < 24 + sizeof(float) * (size_t)np) {
    set_error("fit_precond_load: parameter count does not match the network");
    return FIT_E_INVALID;
  }
  return create(c, device, 0, (const float*)(b + 24), out);
}

extern "C" fit_status fit_precond_apply(fit_precond* p, const fit_grid* g, double omega, const void* v_dev,
                                        void* z_dev, void* stream) {
  if (!p || !g || !v_dev || !z_dev || !(omega > 0.0) || !std::isfinite(omega)) {
    set_error("fit_precond_apply: NULL argument or omega <= 0");
    return FIT_E_INVALID;
  }
  if (p->device != g->device) {
    set_error("fit_precond_apply: preconditioner and grid live on different devices");
    return FIT_E_INVALID;
  }
  DeviceScope dev(g->device);
  hipStream_t s = (hipStream_t)stream;
  uint8_t* mask = nullptr;
  fit_status st = edge_mask_of(g, &mask, s);
  if (st != FIT_OK) return st;
  st = apply_grid<double>(p, g, omega, (const double*)v_dev, (double*)z_dev, mask, s);
  hipError_t e = hipStreamSynchronize(s);
  if (st == FIT_OK && e != hipSuccess) st = hip_fail(e, "fit_precond_apply");
  return st;
}

extern "C" fit_status fit_precond_loss_grad(fit_precond* p, const fit_grid* g, double omega, const void* r_dev,
                                            const void* e_dev, double* loss, float* grad_host, void* stream) {
  if (!p || !g || !r_dev || !e_dev || !(omega > 0.0) || !std::isfinite(omega)) {
    set_error("fit_precond_loss_grad: NULL argument or omega <= 0");
    return FIT_E_INVALID;
  }
  if (p->device != g->device) {
    set_error("fit_precond_loss_grad: preconditioner and grid live on different devices");
    return FIT_E_INVALID;
  }
  DeviceScope dev(g->device);
  hipStream_t s = (hipStream_t)stream;
  uint8_t* mask = nullptr;
  fit_status st = edge_mask_of(g, &mask, s);
  if (st != FIT_OK) return st;
  double* loss_dev = p->scal + 4;
  int o[3] = {0, 0, 0}, ext[3] = {round4(g->view.nx), round4(g->view.ny), round4(g->view.nz)};
  if (st == FIT_OK) st = zero_f32(p->G, p->nparams, s);
  if (st == FIT_OK && hipMemsetAsync(loss_dev, 0, sizeof(double), s) != hipSuccess) st = FIT_E_DEVICE;
  if (st == FIT_OK)
    st = pair_step(p, g, omega, (const double*)r_dev, (const double*)e_dev, mask, o, ext, 1.0f, loss_dev, s);
  hipError_t e = hipStreamSynchronize(s);
  if (st == FIT_OK && e != hipSuccess) st = hip_fail(e, "fit_precond_loss_grad");
  if (st == FIT_OK && loss && hipMemcpy(loss, loss_dev, sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
    st = FIT_E_DEVICE;
  if (st == FIT_OK && grad_host &&
      hipMemcpy(grad_host, p->G, sizeof(float) * (size_t)p->nparams, hipMemcpyDeviceToHost) != hipSuccess)
    st = FIT_E_DEVICE;
  return st;
}

namespace {
struct Rng {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  int below(int n) { return (int)(next() % (uint64_t)n); }
};
}  // namespace

// Loss history of the last training run (mean loss per optimiser step).
static thread_local std::vector<double> g_last_history;

extern "C" fit_status fit_precond_train(fit_grid* const* train, int ntrain, const double* omegas, int nomega,
                                        const fit_precond_cfg* cfg, fit_precond** out) {
  if (!train || ntrain < 1 || !omegas || nomega < 1 || !out) {
    set_error("fit_precond_train: NULL argument or empty training set");
    return FIT_E_INVALID;
  }
  *out = nullptr;
  for (int i = 0; i < ntrain; ++i)
    if (!train[i] || train[i]->device != train[0]->device) {
      set_error("fit_precond_train: NULL grid or grids on different devices");
      return FIT_E_INVALID;
    }
  for (int f = 0; f < nomega; ++f)
    if (!(omegas[f] > 0.0) || !std::isfinite(omegas[f])) {
      set_error("fit_precond_train: omegas must be finite and > 0");
      return FIT_E_INVALID;
    }
  fit_precond_cfg c{};
  if (cfg) c = *cfg;
  if (c.base_channels <= 0) c.base_channels = 16;
  if (c.steps <= 0) c.steps = 2000;
  if (c.batch <= 0) c.batch = 4;
  if (c.crop <= 0) c.crop = 32;
  if (c.lr <= 0.0) c.lr = 1e-3;
  if (c.crop % 4) {
    set_error("fit_precond_train: crop must be a multiple of 4");
    return FIT_E_INVALID;
  }
  const int device = train[0]->device;
  DeviceScope dev(device);
  hipStream_t s = (hipStream_t)c.stream;
  fit_precond* p = nullptr;
  fit_status st = create(c.base_channels, device, (uint64_t)(uint32_t)c.seed, nullptr, &p);
  if (st != FIT_OK) return st;
  std::unique_ptr<fit_precond, void (*)(fit_precond*)> guard(p, fit_precond_destroy);
  // per-grid masks and the error / residual work vectors
  std::vector<uint8_t*> masks(ntrain, nullptr);
  int64_t ne_max = 0;
  for (int i = 0; i < ntrain; ++i) ne_max = std::max(ne_max, train[i]->ne);
  double *e = nullptr, *e2 = nullptr, *r = nullptr, *hist = nullptr;
  auto cleanup = [&]() {
    (void)hipFree(e);
    (void)hipFree(e2);
    (void)hipFree(r);
    (void)hipFree(hist);
  };
  for (int i = 0; i < ntrain && st == FIT_OK; ++i) st = edge_mask_of(train[i], &masks[i], s);
  if (st == FIT_OK && (hipMalloc(&e, ne_max * 16) != hipSuccess || hipMalloc(&e2, ne_max * 16) != hipSuccess ||
                       hipMalloc(&r, ne_max * 16) != hipSuccess ||
                       hipMalloc(&hist, sizeof(double) * c.steps) != hipSuccess)) {
    set_error("fit_precond_train: out of device memory");
    st = FIT_E_NOMEM;
  }
  if (st == FIT_OK && hipMemsetAsync(hist, 0, sizeof(double) * c.steps, s) != hipSuccess) st = FIT_E_DEVICE;
  Rng rng{(uint64_t)(uint32_t)c.seed * 0x2545F4914F6CDD1Dull + 17};
  const int passes_of[4] = {2, 4, 8, 16};
  const float b1 = 0.9f, b2 = 0.999f;
  for (int step = 0; step < c.steps && st == FIT_OK; ++step) {
    if ((st = zero_f32(p->G, p->nparams, s)) != FIT_OK) break;
    for (int b = 0; b < c.batch && st == FIT_OK; ++b) {
      const int gi = rng.below(ntrain);
      const fit_grid* g = train[gi];
      const double omega = omegas[rng.below(nomega)];
      const int passes = passes_of[rng.below(4)];
      const int dims[3] = {g->view.nx, g->view.ny, g->view.nz};
      int o[3], ext[3];
      for (int d = 0; d < 3; ++d) {
        ext[d] = std::max(4, std::min(c.crop, dims[d] / 4 * 4));
        o[d] = dims[d] > ext[d] ? rng.below(dims[d] - ext[d] + 1) : 0;
      }
      hipLaunchKernelGGL(noise_kernel, dim3(nblk(g->ne)), dim3(256), 0, s, g->ne, masks[gi], rng.next(), e);
      double *src = e, *dst = e2;
      for (int k = 0; k < passes; ++k) {
        hipLaunchKernelGGL(smooth_kernel, dim3(nblk(g->view.np)), dim3(256), 0, s, g->view, masks[gi], src, dst);
        std::swap(src, dst);
      }
      if (hipGetLastError() != hipSuccess) {
        st = FIT_E_DEVICE;
        break;
      }
      OpMatvec<double> mv{src, r};
      if ((st = launch_stencil<double, MODE_D>(g->view, tile_for(g, FIT_C128), omega, mv, s)) != FIT_OK) break;
      st = pair_step(p, g, omega, r, src, masks[gi], o, ext, 1.0f / c.batch, hist + step, s);
    }
    if (st != FIT_OK) break;
    ++p->adam_t;
    const float c1 = 1.f - std::pow(b1, (float)p->adam_t), c2 = 1.f - std::pow(b2, (float)p->adam_t);
    hipLaunchKernelGGL(adam_kernel, dim3(nblk(p->nparams)), dim3(256), 0, s, p->P, p->G, p->Mo, p->Vo,
                       p->nparams, (float)c.lr, b1, b2, 1e-8f, (float)c.weight_decay, c1, c2);
    if (hipGetLastError() != hipSuccess) {
      st = FIT_E_DEVICE;
      break;
    }
    st = p->upload_weights(s);
  }
  if (st == FIT_OK) {
    g_last_history.assign(c.steps, 0.0);
    if (hipStreamSynchronize(s) != hipSuccess ||
        hipMemcpy(g_last_history.data(), hist, sizeof(double) * c.steps, hipMemcpyDeviceToHost) != hipSuccess)
      st = FIT_E_DEVICE;
    for (double& v : g_last_history) v /= c.batch;
  }
  (void)hipStreamSynchronize(s);
  cleanup();
  if (st != FIT_OK) return st;
  *out = guard.release();
  return FIT_OK;
}

extern "C" fit_status fit_precond_train_history(double* out, int max, int* n) {
  if (n) *n = (int)g_last_history.size();
  if (out)
    for (int i = 0; i < std::min<int>(max, (int)g_last_history.size()); ++i) out[i] = g_last_history[i];
  return FIT_OK;
}

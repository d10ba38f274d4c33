// BF16 MFMA implicit GEMM for the learned preconditioner's 3D convolutions.
//
// Every layer of the U-Net, forward and backward, is one GEMM
//     out[m][n] = sum_k A(m, k) * B[n][k]
// whose A operand is gathered on the fly from a channels-last bf16 tensor
// (no im2col buffer in the forward and backward-data passes):
//   G_CONV3  m = output voxel, k = tap*cin + ci, A = in[voxel + offset(tap)][ci]
//            (3x3x3 taps, zero outside the tensor)
//   G_DOWN2  m = output voxel, k = tap*cin + ci, A = in[2*voxel + offset(tap)][ci]
//            (2x2x2 taps, stride 2)
//   G_PW     m = row, k = ci, A = in[m][ci] (1x1x1, or any row-major matrix)
// B is a bf16 matrix with rows padded to the N tile and K padded to 32 with
// zeros.  The epilogue adds the bias, applies ReLU, rounds to bf16, and can
// scatter the 8 children of a transposed 2x2x2 convolution, accumulate into
// fp32 gradients, or write split-K partial sums.
//
// Tiling for CDNA4: a 256-thread workgroup computes 64 rows x NT columns; each
// wavefront owns 16 rows and NT/16 accumulators of the 16x16x32 bf16 MFMA.
// Each lane loads its 8 consecutive K values of A (one 16-byte load, since
// channel counts are multiples of 8) and of B, so no LDS staging is needed:
// the 27-fold reuse of an input voxel across taps is served by L1/L2.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fit {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

enum GatherKind { G_CONV3 = 0, G_DOWN2 = 1, G_PW = 2 };
enum OutKind { O_BF16 = 0, O_F32 = 1, O_F32ACC = 2, O_PART = 3 };

struct GemmArgs {
  // A operand
  const bf16* a;  // tensor base (channel offset already applied)
  int64_t a_ld;   // elements between consecutive voxels (rows for G_PW)
  int cin;        // channels per tap (multiple of 8)
  int gather;     // GatherKind
  int ix, iy, iz; // A tensor spatial dims (G_CONV3 / G_DOWN2)
  int64_t M;      // rows
  int ox, oy;     // row -> (x, y, z) decoding dims (G_CONV3 / G_DOWN2 / up scatter)
  int64_t K;      // true K
  // B operand: [npad][ldb] bf16, K padded with zeros to a multiple of 32
  const bf16* b;
  int64_t ldb;
  int N;          // true N
  // epilogue
  const float* bias;  // per output channel, or nullptr
  int relu;
  int out;            // OutKind
  int up;             // nonzero: column n = t*up_c + c of row u goes to child t of u
  int up_c;           // channels per child
  int up_x, up_y;     // child tensor dims (2 ox, 2 oy)
  bf16* o16;          // O_BF16 destination (channel offset applied)
  float* o32;         // O_F32 / O_F32ACC / O_PART destination
  int64_t o_ld;       // elements between voxels of the destination
  int64_t k_chunk;    // K per split (multiple of 32); gridDim.z splits
};

template <int NT>
__global__ void __launch_bounds__(256) igemm_kernel(GemmArgs p) {
  constexpr int NS = NT / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t m_tile = (int64_t)blockIdx.x * 64 + wave * 16;
  const int n0 = blockIdx.y * NT;
  const int64_t kb = (int64_t)blockIdx.z * p.k_chunk;
  const int64_t ke0 = kb + p.k_chunk;
  const int64_t kpad = (p.K + 31) / 32 * 32;
  const int64_t ke = ke0 < kpad ? ke0 : kpad;

  // this lane's A row and its decoded coordinates
  const int64_t m = m_tile + (lane & 15);
  const bool mv = m < p.M;
  int mx = 0, my = 0, mz = 0;
  if (p.gather != G_PW && mv) {
    mx = (int)(m % p.ox);
    my = (int)((m / p.ox) % p.oy);
    mz = (int)(m / ((int64_t)p.ox * p.oy));
  }
  const int kq = 8 * (lane >> 4);

  floatx4 acc[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) acc[s] = floatx4{0.f, 0.f, 0.f, 0.f};

  for (int64_t kk = kb; kk < ke; kk += 32) {
    const int64_t k = kk + kq;
    bf16x8 av;
#pragma unroll
    for (int e = 0; e < 8; ++e) av[e] = (bf16)0.0f;
    if (mv && k < p.K) {
      const bf16* src = nullptr;
      if (p.gather == G_PW) {
        src = p.a + m * p.a_ld + k;
      } else {
        const int tap = (int)(k / p.cin), ci = (int)(k % p.cin);
        int x, y, z;
        if (p.gather == G_CONV3) {
          x = mx + tap % 3 - 1;
          y = my + (tap / 3) % 3 - 1;
          z = mz + tap / 9 - 1;
        } else {
          x = 2 * mx + (tap & 1);
          y = 2 * my + ((tap >> 1) & 1);
          z = 2 * mz + (tap >> 2);
        }
        if (x >= 0 && y >= 0 && z >= 0 && x < p.ix && y < p.iy && z < p.iz)
          src = p.a + (((int64_t)z * p.iy + y) * p.ix + x) * p.a_ld + ci;
      }
      if (src) av = *reinterpret_cast<const bf16x8*>(src);
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int n = n0 + s * 16 + (lane & 15);
      const bf16x8 bv = *reinterpret_cast<const bf16x8*>(p.b + (int64_t)n * p.ldb + k);
      acc[s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[s], 0, 0, 0);
    }
  }

  // epilogue: lane holds rows m_tile + 4*(lane/16) + r, column n0 + 16 s + lane%16
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int n = n0 + s * 16 + (lane & 15);
    if (n >= p.N) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = m_tile + 4 * (lane >> 4) + r;
      if (row >= p.M) continue;
      float v = acc[s][r];
      if (p.out == O_PART) {
        p.o32[((int64_t)blockIdx.z * p.M + row) * p.N + n] = v;
        continue;
      }
      int64_t vox = row;
      int ch = n;
      if (p.up) {
        const int t = n / p.up_c;
        ch = n % p.up_c;
        const int ux = (int)(row % p.ox), uy = (int)((row / p.ox) % p.oy),
                  uz = (int)(row / ((int64_t)p.ox * p.oy));
        const int cx = 2 * ux + (t & 1), cy = 2 * uy + ((t >> 1) & 1), cz = 2 * uz + (t >> 2);
        vox = ((int64_t)cz * p.up_y + cy) * p.up_x + cx;
      }
      if (p.bias) v += p.bias[ch];
      if (p.relu) v = v > 0.f ? v : 0.f;
      const int64_t dst = vox * p.o_ld + ch;
      if (p.out == O_BF16)
        p.o16[dst] = (bf16)v;
      else if (p.out == O_F32)
        p.o32[dst] = v;
      else
        p.o32[dst] += v;
    }
  }
}

}  // namespace fit

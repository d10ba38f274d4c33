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
// Tiling for CDNA4 (general kernel, igemm_kernel): a 256-thread workgroup
// computes 128 rows x NT columns; each wavefront owns two 16-row subtiles and
// 2 x NT/16 accumulators of the 16x16x32 bf16 MFMA, so each B fragment feeds
// two MFMAs.  Each lane loads its 8 consecutive K values of A (one 16-byte
// load, since channel counts are multiples of 8) and of B straight from
// global memory.  The gather walks K with a per-lane (tap, channel) cursor; a
// tap's element offset is one add, and the row's bounds are three bit tests.
// 3x3x3 convolutions with 8, 16, 32 or 64 input channels, the bulk of the work,
// use conv3_lds_kernel instead, which stages its input brick in LDS.
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

// Epilogue.  An output element (row, n) goes to o16/o32[row_off + col.off]:
// the row part and the column part are computed once per row and once per
// column of a lane's accumulators, in 32-bit index arithmetic (M < 2^31).
struct EpiCol {
  int64_t off;  // column part of the destination offset
  float bias;
  bool ok;      // n < N
};

__device__ __forceinline__ EpiCol epi_col(const GemmArgs& p, int n) {
  EpiCol c;
  c.ok = n < p.N;
  const int nn = c.ok ? n : 0;
  if (p.out == O_PART) {
    c.off = nn;
    c.bias = 0.f;
    return c;
  }
  int ch = nn;
  int64_t child = 0;
  if (p.up) {  // column n = tt * up_c + ch goes to child tt of the row's voxel
    const int tt = nn / p.up_c;
    ch = nn - tt * p.up_c;
    child = ((int64_t)(tt >> 2) * p.up_y + ((tt >> 1) & 1)) * p.up_x + (tt & 1);
  }
  c.off = child * p.o_ld + ch;
  c.bias = p.bias ? p.bias[ch] : 0.f;
  return c;
}

__device__ __forceinline__ int64_t epi_row(const GemmArgs& p, int64_t row) {
  if (p.out == O_PART) return ((int64_t)blockIdx.z * p.M + row) * p.N;
  if (!p.up) return row * p.o_ld;
  const uint32_t r = (uint32_t)row, ox = (uint32_t)p.ox, oy = (uint32_t)p.oy;
  const uint32_t t = r / ox, ux = r - t * ox, uz = t / oy, uy = t - uz * oy;
  return (((int64_t)(2 * uz) * p.up_y + 2 * uy) * p.up_x + 2 * ux) * p.o_ld;
}

__device__ __forceinline__ void epi_put(const GemmArgs& p, int64_t roff, const EpiCol& c, float v) {
  const int64_t dst = roff + c.off;
  if (p.out == O_PART) {
    p.o32[dst] = v;
    return;
  }
  v += c.bias;
  if (p.relu) v = v > 0.f ? v : 0.f;
  if (p.out == O_BF16)
    p.o16[dst] = (bf16)v;
  else if (p.out == O_F32)
    p.o32[dst] = v;
  else
    p.o32[dst] += v;
}

// Per-lane gather cursor over K: the current tap, the channel offset inside
// the tap, and the tap's element offset (uniform over the lanes that share
// the K position; the bounds test is per row).
struct KCursor {
  int tap, ci;
};

// Orders LDS stores of one wavefront before loads by other lanes of the same
// wavefront (a compiler barrier plus wavefront-scope release/acquire fences).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// PK: the launch writes bf16 outputs and may take the packed (LDS-staged,
// 16-byte) store; a separate instantiation, so that the K loop of every other
// launch compiles exactly as without it.
template <int NT, bool PK>
__global__ void __launch_bounds__(256) igemm_kernel(GemmArgs p) {
  constexpr int NS = NT / 16;  // N subtiles per wave
  constexpr int MS = 2;        // 16-row M subtiles per wave
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t m_tile = (int64_t)blockIdx.x * (64 * MS) + wave * (16 * MS);
  const int n0 = blockIdx.y * NT;
  const int64_t kb = (int64_t)blockIdx.z * p.k_chunk;
  const int64_t ke0 = kb + p.k_chunk;
  const int64_t kpad = (p.K + 31) / 32 * 32;
  const int64_t ke = ke0 < kpad ? ke0 : kpad;
  const int kq = 8 * (lane >> 4);
  const bool pw = p.gather == G_PW, conv3 = p.gather == G_CONV3;

  // rows of this lane: base element of its first tap and per-axis validity
  const bf16* base[MS];
  uint32_t okx[MS], oky[MS], okz[MS];  // bit j: offset j-1 (conv3) or j (down2) in range
  bool mv[MS];
#pragma unroll
  for (int s = 0; s < MS; ++s) {
    const int64_t m = m_tile + 16 * s + (lane & 15);
    mv[s] = m < p.M;
    const int64_t mm = mv[s] ? m : 0;
    okx[s] = oky[s] = okz[s] = 7u;
    if (pw) {
      base[s] = p.a + mm * p.a_ld;
    } else {
      const int mx = (int)(mm % p.ox), my = (int)((mm / p.ox) % p.oy), mz = (int)(mm / ((int64_t)p.ox * p.oy));
      if (conv3) {
        base[s] = p.a + (((int64_t)mz * p.iy + my) * p.ix + mx) * p.a_ld;
        okx[s] = (mx > 0 ? 1u : 0u) | 2u | (mx + 1 < p.ix ? 4u : 0u);
        oky[s] = (my > 0 ? 1u : 0u) | 2u | (my + 1 < p.iy ? 4u : 0u);
        okz[s] = (mz > 0 ? 1u : 0u) | 2u | (mz + 1 < p.iz ? 4u : 0u);
      } else {
        base[s] = p.a + (((int64_t)(2 * mz) * p.iy + 2 * my) * p.ix + 2 * mx) * p.a_ld;
      }
    }
  }
  // K cursor of this lane
  KCursor cur{0, 0};
  if (!pw) {
    const int64_t k0 = kb + kq;
    cur.tap = (int)(k0 / p.cin);
    cur.ci = (int)(k0 % p.cin);
  }
  const int64_t sx = p.a_ld, sy = (int64_t)p.ix * p.a_ld, sz = (int64_t)p.iy * p.ix * p.a_ld;

  floatx4 acc[MS][NS];
#pragma unroll
  for (int s = 0; s < MS; ++s)
#pragma unroll
    for (int t = 0; t < NS; ++t) acc[s][t] = floatx4{0.f, 0.f, 0.f, 0.f};

  for (int64_t kk = kb; kk < ke; kk += 32) {
    const int64_t k = kk + kq;
    const bool kv = k < p.K;
    // element offset of this lane's tap and the per-row validity bit
    int64_t off;
    int jx = 1, jy = 1, jz = 1;
    if (pw) {
      off = k;
    } else if (conv3) {
      const int dz = cur.tap / 9, r9 = cur.tap - 9 * dz, dy = r9 / 3, dx = r9 - 3 * dy;
      jx = dx;
      jy = dy;
      jz = dz;
      off = (dz - 1) * sz + (dy - 1) * sy + (dx - 1) * sx + cur.ci;
    } else {
      const int dx = cur.tap & 1, dy = (cur.tap >> 1) & 1, dz = cur.tap >> 2;
      off = dz * sz + dy * sy + dx * sx + cur.ci;
    }
    bf16x8 av[MS];
#pragma unroll
    for (int s = 0; s < MS; ++s) {
      bool ok = mv[s] && kv;
      if (conv3) ok = ok && ((okx[s] >> jx) & (oky[s] >> jy) & (okz[s] >> jz) & 1u);
      if (ok) {
        av[s] = *reinterpret_cast<const bf16x8*>(base[s] + off);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) av[s][e] = (bf16)0.0f;
      }
    }
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      const int n = n0 + t * 16 + (lane & 15);
      const bf16x8 bv = *reinterpret_cast<const bf16x8*>(p.b + (int64_t)n * p.ldb + k);
#pragma unroll
      for (int s = 0; s < MS; ++s)
        acc[s][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[s], bv, acc[s][t], 0, 0, 0);
    }
    if (!pw) {  // advance the cursor by 32 K positions
      cur.ci += 32;
      while (cur.ci >= p.cin) {
        cur.ci -= p.cin;
        ++cur.tap;
      }
    }
  }

  // epilogue: lane holds rows m_tile + 16 s + 4*(lane/16) + r, column n0 + 16 t + lane%16
  EpiCol col[NS];
#pragma unroll
  for (int t = 0; t < NS; ++t) col[t] = epi_col(p, n0 + t * 16 + (lane & 15));
  // bf16 outputs of a full column tile (also the children of a transposed
  // convolution, 8 channels of one child at a time) go through this
  // wavefront's LDS rows and leave as 16-byte stores
  constexpr int kRow = NT + 8;  // halfwords per staged row (16-byte aligned rows)
  if constexpr (PK) {
    __shared__ bf16 stage[4 * 16 * MS * kRow];
    const bool packed = p.out == O_BF16 && n0 + NT <= p.N && (p.o_ld & 7) == 0 &&
                        (!p.up || (p.up_c & 7) == 0) && ((reinterpret_cast<uintptr_t>(p.o16) & 15) == 0);
    if (packed) {  // uniform over the block; each wavefront uses only its own rows
      bf16* stg = stage + wave * 16 * MS * kRow;
#pragma unroll
      for (int s = 0; s < MS; ++s)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int t = 0; t < NS; ++t) {
            float v = acc[s][t][r] + col[t].bias;
            if (p.relu) v = v > 0.f ? v : 0.f;
            stg[(16 * s + 4 * (lane >> 4) + r) * kRow + t * 16 + (lane & 15)] = (bf16)v;
          }
      wave_sync();
      for (int q = lane; q < 16 * MS * (NT / 8); q += 64) {
        const int rloc = q / (NT / 8), c8 = q % (NT / 8);
        const int64_t row = m_tile + rloc;
        if (row >= p.M) continue;
        const EpiCol c = epi_col(p, n0 + 8 * c8);  // 8 channels of one column group (one child)
        const bf16x8 v = *reinterpret_cast<const bf16x8*>(stg + rloc * kRow + 8 * c8);
        *reinterpret_cast<bf16x8*>(p.o16 + epi_row(p, row) + c.off) = v;
      }
      return;
    }
  }
#pragma unroll
  for (int s = 0; s < MS; ++s) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = m_tile + 16 * s + 4 * (lane >> 4) + r;
      if (row >= p.M) continue;
      const int64_t roff = epi_row(p, row);
#pragma unroll
      for (int t = 0; t < NS; ++t)
        if (col[t].ok) epi_put(p, roff, col[t], acc[s][t][r]);
    }
  }
}

// 3x3x3 convolution (G_CONV3, output dims = input dims, CIN in {8, 16, 32,
// 64} input channels) with the input staged in LDS.  A workgroup outputs an
// 8 x 8 x 4 brick of voxels (256 rows); it first copies the brick's input
// with its one-voxel halo (10 x 10 x 6 voxels, zeros outside the tensor) into
// LDS, then reads every tap's A fragment from LDS instead of refetching it
// through L1/L2 27 times.  Each wavefront owns 64 rows (one z-slice of the
// brick, four 16-row subtiles), so a B fragment feeds four MFMAs; B is read
// through a ring of registers several K steps ahead.
//
// LDS layout: voxel h of the halo brick holds C8 = CIN/8 16-byte chunks;
// chunk c is stored at slot c ^ ((h / (8 / C8)) & (C8 - 1)), so the eight
// lanes of an octet (same chunk, eight consecutive voxels) read eight
// different 16-byte slots.  Measured on gfx950 (SQ_LDS_BANK_CONFLICT, 16-byte
// reads): 16 lanes that read one aligned 256-byte block, in any order, take
// no extra cycle; 16 lanes spread over two blocks take extra cycles even when
// their banks differ.  A subtile's rows are two x-rows of 8 voxels and each
// tap shifts them by dx, so no single-copy layout keeps every tap inside one
// block; this one costs four extra LDS cycles per read.  (A chunk-planar
// layout padded to 16-voxel x-groups, conflict-free for dx = 0 only, was
// measured slower: more LDS per workgroup, more conflicts in total.)
// LDS: 600 * CIN * 2 bytes (9.6 / 19.2 / 38.4 / 76.8 KB).
constexpr int kBrX = 8, kBrY = 8, kBrZ = 4;
constexpr int kHaX = kBrX + 2, kHaY = kBrY + 2, kHaZ = kBrZ + 2;
constexpr int kHalo = kHaX * kHaY * kHaZ;

template <int C8>
__device__ __forceinline__ int conv_slot(unsigned h, unsigned c) {
  constexpr unsigned per_line = 8 / C8 > 0 ? 8 / C8 : 1;
  return (int)(h * C8 + (c ^ ((h / per_line) & (C8 - 1))));
}

template <int NT, int CIN, bool PK>
__global__ void __launch_bounds__(256) conv3_lds_kernel(GemmArgs p) {
  constexpr int NS = NT / 16;
  constexpr int MS = 4;
  constexpr int C8 = CIN / 8;
  constexpr int TOT = kHalo * C8;            // 16-byte chunks to stage
  constexpr int NIT = (TOT + 255) / 256;     // chunks per thread
  constexpr int NB = (NIT + 7) / 8;          // batches of at most 8 loads in flight
  constexpr int BATCH = (NIT + NB - 1) / NB;
  __shared__ bf16x8 tile[TOT];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nbx = (p.ix + kBrX - 1) / kBrX, nby = (p.iy + kBrY - 1) / kBrY;
  const int b = blockIdx.x;
  const int bx0 = (b % nbx) * kBrX, by0 = ((b / nbx) % nby) * kBrY, bz0 = (b / (nbx * nby)) * kBrZ;
  // B fragments: a ring of D slots filled ahead of use; the first loads are
  // issued before the halo staging so that their latency overlaps it
  constexpr int K = 27 * CIN;
  constexpr int NFULL = K / 32;
  constexpr bool PART = (K % 32) != 0;
  constexpr int NSTEP = NFULL + (PART ? 1 : 0);
  constexpr int LAST = (NSTEP - 1) * 32;
  constexpr int DW = NS >= 4 ? 2 : 4;  // ring depth (wide tiles already have NS loads per step)
  constexpr int D = NSTEP < DW ? NSTEP : DW;
  const int n0 = blockIdx.y * NT;
  const int kq = 8 * (lane >> 4);
  const bf16* brow[NS];
#pragma unroll
  for (int t = 0; t < NS; ++t) brow[t] = p.b + (int64_t)(n0 + t * 16 + (lane & 15)) * p.ldb + kq;
  auto load_b = [&](bf16x8(&dst)[NS], int kk) {
    const int kc = kk < LAST ? kk : LAST;
#pragma unroll
    for (int t = 0; t < NS; ++t) dst[t] = *reinterpret_cast<const bf16x8*>(brow[t] + kc);
  };
  bf16x8 bq[D][NS];
#pragma unroll
  for (int i = 0; i < D; ++i) load_b(bq[i], i * 32);

  // stage the halo brick: every load is issued from a clamped (in-range)
  // address before any is written to LDS; voxels outside the tensor are
  // replaced by zeros
  for (int q0 = 0; q0 < NB * BATCH * 256; q0 += BATCH * 256) {
    bf16x8 v[BATCH];
    bool in[BATCH];
#pragma unroll
    for (int u = 0; u < BATCH; ++u) {
      const int q = q0 + u * 256 + (int)threadIdx.x;
      const int qq = q < TOT ? q : TOT - 1;
      const int cc = qq % C8, h = qq / C8;
      const int hx = h % kHaX, hy = (h / kHaX) % kHaY, hz = h / (kHaX * kHaY);
      const int x = bx0 + hx - 1, y = by0 + hy - 1, z = bz0 + hz - 1;
      in[u] = x >= 0 && y >= 0 && z >= 0 && x < p.ix && y < p.iy && z < p.iz;
      const int xc = x < 0 ? 0 : (x < p.ix ? x : p.ix - 1);
      const int yc = y < 0 ? 0 : (y < p.iy ? y : p.iy - 1);
      const int zc = z < 0 ? 0 : (z < p.iz ? z : p.iz - 1);
      v[u] = *reinterpret_cast<const bf16x8*>(p.a + (((int64_t)zc * p.iy + yc) * p.ix + xc) * p.a_ld + 8 * cc);
    }
    // threads past the end rewrite chunk TOT - 1 with the value its owner
    // writes, which keeps the stores unconditional
#pragma unroll
    for (int u = 0; u < BATCH; ++u) {
      const int q = q0 + u * 256 + (int)threadIdx.x;
      const int qq = q < TOT ? q : TOT - 1;
      bf16x8 w = v[u];
      if (!in[u]) {
#pragma unroll
        for (int e = 0; e < 8; ++e) w[e] = (bf16)0.0f;
      }
      tile[conv_slot<C8>(qq / C8, qq % C8)] = w;
    }
  }
  __syncthreads();

  // halo voxel of tap (-1, -1, -1) for each row of this lane
  unsigned hbase[MS];
#pragma unroll
  for (int s = 0; s < MS; ++s) {
    const int rl = wave * 64 + 16 * s + (lane & 15);
    const int lx = rl % kBrX, ly = (rl / kBrX) % kBrY, lz = rl / (kBrX * kBrY);
    hbase[s] = (unsigned)((lz * kHaY + ly) * kHaX + lx);
  }
  floatx4 acc[MS][NS];
#pragma unroll
  for (int s = 0; s < MS; ++s)
#pragma unroll
    for (int t = 0; t < NS; ++t) acc[s][t] = floatx4{0.f, 0.f, 0.f, 0.f};

  // K = 27 * CIN runs in NFULL full steps of 32 and, for CIN = 8 or 16, a
  // final partial step whose lanes past K read a valid tap and are zeroed.
  auto step = [&](int kk, const bf16x8(&bc)[NS], bool partial) {
    int kc = kk + kq;
    bool kv = true;
    if (partial) {
      kv = kc < K;
      kc = kv ? kc : K - 8;
    }
    const unsigned tap = (unsigned)kc / CIN, ci = (unsigned)kc % CIN;
    const unsigned dz = tap / 9, r9 = tap - 9 * dz, dy = r9 / 3, dx = r9 - 3 * dy;
    const unsigned hoff = (dz * kHaY + dy) * kHaX + dx;
    bf16x8 av[MS];
#pragma unroll
    for (int s = 0; s < MS; ++s) {
      av[s] = tile[conv_slot<C8>(hbase[s] + hoff, ci >> 3)];
      if (partial && !kv) {
#pragma unroll
        for (int e = 0; e < 8; ++e) av[s][e] = (bf16)0.0f;
      }
    }
#pragma unroll
    for (int t = 0; t < NS; ++t)
#pragma unroll
      for (int s = 0; s < MS; ++s)
        acc[s][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[s], bc[t], acc[s][t], 0, 0, 0);
  };
  // groups of D steps; slot i of the ring serves steps i, i + D, ...; a
  // slot is refilled right after its step, D - 1 steps before it is needed
  int st = 0;
  for (; st + D <= NSTEP; st += D) {
#pragma unroll
    for (int i = 0; i < D; ++i) {
      step((st + i) * 32, bq[i], PART && st + i == NSTEP - 1);
      load_b(bq[i], (st + i + D) * 32);
    }
  }
#pragma unroll
  for (int i = 0; i < NSTEP % D; ++i) step((st + i) * 32, bq[i], PART && st + i == NSTEP - 1);
  // epilogue: the rows of the brick that lie inside the tensor
  EpiCol col[NS];
#pragma unroll
  for (int t = 0; t < NS; ++t) col[t] = epi_col(p, n0 + t * 16 + (lane & 15));
  // bf16 outputs of a full column tile go through LDS (the halo tile is free
  // once every wavefront has left its K loop) and leave as 16-byte stores of
  // 8 channels instead of 2-byte stores
  constexpr int kRow = NT + 8;  // halfwords per staged row (16-byte aligned rows)
  if constexpr (PK && 4 * 64 * kRow * 2 <= (int)sizeof(tile)) {
    const bool packed = p.out == O_BF16 && !p.up && n0 + NT <= p.N && (p.o_ld & 7) == 0 &&
                        ((reinterpret_cast<uintptr_t>(p.o16) & 15) == 0);
    if (packed) {  // uniform over the block
      __syncthreads();
      bf16* stg = reinterpret_cast<bf16*>(tile) + wave * 64 * kRow;
#pragma unroll
      for (int s = 0; s < MS; ++s)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int t = 0; t < NS; ++t) {
            float v = acc[s][t][r] + col[t].bias;
            if (p.relu) v = v > 0.f ? v : 0.f;
            stg[(16 * s + 4 * (lane >> 4) + r) * kRow + t * 16 + (lane & 15)] = (bf16)v;
          }
      // each wavefront reads back only its own rows: no block barrier needed
      wave_sync();
      for (int q = lane; q < 64 * (NT / 8); q += 64) {
        const int row = q / (NT / 8), c8 = q % (NT / 8);
        const int rl = wave * 64 + row;
        const int x = bx0 + rl % kBrX, y = by0 + (rl / kBrX) % kBrY, z = bz0 + rl / (kBrX * kBrY);
        if (x >= p.ix || y >= p.iy || z >= p.iz) continue;
        const bf16x8 v = *reinterpret_cast<const bf16x8*>(stg + row * kRow + 8 * c8);
        *reinterpret_cast<bf16x8*>(p.o16 + (((int64_t)z * p.iy + y) * p.ix + x) * p.o_ld + n0 + 8 * c8) = v;
      }
      return;
    }
  }
#pragma unroll
  for (int s = 0; s < MS; ++s) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int rl = wave * 64 + 16 * s + 4 * (lane >> 4) + r;
      const int x = bx0 + rl % kBrX, y = by0 + (rl / kBrX) % kBrY, z = bz0 + rl / (kBrX * kBrY);
      if (x >= p.ix || y >= p.iy || z >= p.iz) continue;
      const int64_t roff = epi_row(p, ((int64_t)z * p.iy + y) * p.ix + x);
#pragma unroll
      for (int t = 0; t < NS; ++t)
        if (col[t].ok) epi_put(p, roff, col[t], acc[s][t][r]);
    }
  }
}
}  // namespace fit

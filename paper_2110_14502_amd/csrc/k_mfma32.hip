// FP32 matrix-core contraction kernel (fused permute + complex GEMM).
#include "kernels_dev.h"

namespace rqc {

// ---------------------------------------------------------------------------
// MFMA contraction (FP32 matrix cores, v_mfma_f32_32x32x2_f32): 128 rows x
// 64 complex columns per workgroup, 16 complex k per LDS chunk, double
// buffered; 4 waves in a 2x2 grid, each 64 rows x 64 real columns.  The
// operand offsets come from LDS tables built once per workgroup; the output
// tile is staged through LDS in two halves of 64 rows (inside the operand
// buffers) and stored in C's address order.  49.7 KB of LDS: three
// workgroups per CU.
// ---------------------------------------------------------------------------
template <int SA, int SB, int SC>
__global__ __launch_bounds__(256, 3) void k_mfma32(StepDesc d) {
  __shared__ float lds[kMainFloats + 16];
  float* Abuf = lds;                                          // [2][kTK][2][kAPlane]
  float2* Bbuf = reinterpret_cast<float2*>(lds + 2 * kABuf);  // [2][kTK][kBStride]
  float* red = lds + kMainFloats;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  // XCD-aware block order: consecutive logical tiles share the row tile of A
  // and land on the same XCD (blocks are dealt round-robin to the 8 XCDs).
  uint64_t bid = blockIdx.x;
  const uint64_t nblk = gridDim.x;
  if ((nblk & 7) == 0) bid = (bid & 7) * (nblk >> 3) + (bid >> 3);
  const uint64_t no = bid % (uint64_t)d.n_col_tiles;
  const uint64_t ro = bid / (uint64_t)d.n_col_tiles;

  // Per-thread element offsets of the A (2048) and B (1024) chunk tiles.
  int64_t gA[8];
  int lA[8];
  int64_t gB[4];
  int lB[4];
  {
    TileTab* ta = reinterpret_cast<TileTab*>(lds);
    TileTab* tb = ta + 1;
    build_tab(d.tA, 1, 0, kAStride, *ta);
    build_tab(d.tB, 0, 1, kBStride, *tb);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      gA[j] = ta->g[lane] + ta->g[64 + wave + 4 * j];
      lA[j] = ta->c[lane] + ta->c[64 + wave + 4 * j];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      gB[j] = tb->g[lane] + tb->g[64 + wave + 4 * j];
      lB[j] = tb->c[lane] + tb->c[64 + wave + 4 * j];
    }
  }
  // The C tile bit that carries row bit 6 (which half of the tile).
  int hb = 0;
  for (int b = 0; b < d.tC.nbits; ++b)
    if (d.tC.role[b] == 0 && d.tC.cbit[b] == 6) hb = b;
  const int64_t g_half = int64_t(1) << d.tC.gpos[hb];

  // Lane roles inside the real-expanded operands.
  const int lrow = lane & 31;          // row inside a 32-row block
  const int cpart = lane >> 5;         // A_r column parity: 0 re, 1 im
  const int dpart = lane & 1;          // C_r column parity
  const int ncol = (lane & 31) >> 1;   // complex column inside a 16-col block
  const bool bswap = cpart != dpart;
  const float bsign = (cpart == 1 && dpart == 0) ? -1.f : 1.f;

  const int n_kc = 1 << d.n_ko;
  for (int copy = blockIdx.y; copy < d.copies; copy += gridDim.y) {
    const int js = copy % d.gs_c, jb = copy / d.gs_c;
    int64_t oA, oB, oC;
    outer_offsets(d, ro, no, js, jb, oA, oB, oC);
    floatx16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    float2 ra[8], rb[4];
    {
      int64_t kA, kB;
      k_offsets(d, 0, kA, kB);
#pragma unroll
      for (int j = 0; j < 8; ++j) ra[j] = load_c<SA>(d.A, oA + kA + gA[j]);
#pragma unroll
      for (int j = 0; j < 4; ++j) rb[j] = load_c<SB>(d.B, oB + kB + gB[j]);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      Abuf[lA[j]] = ra[j].x;
      Abuf[lA[j] + kAPlane] = ra[j].y;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) Bbuf[lB[j]] = rb[j];
    __syncthreads();

    for (int kc = 0; kc < n_kc; ++kc) {
      const int cur = kc & 1;
      const bool more = kc + 1 < n_kc;
      if (more) {
        int64_t kA, kB;
        k_offsets(d, kc + 1, kA, kB);
#pragma unroll
        for (int j = 0; j < 8; ++j) ra[j] = load_c<SA>(d.A, oA + kA + gA[j]);
#pragma unroll
        for (int j = 0; j < 4; ++j) rb[j] = load_c<SB>(d.B, oB + kB + gB[j]);
      }
      const float* As = Abuf + cur * kABuf + cpart * kAPlane + wm * 64 + lrow;
      const float2* Bs = Bbuf + cur * kBBuf + wn * 32 + ncol;
      // Operands of step k+1 are read from LDS while the MFMAs of step k run.
      float a0 = As[0], a1 = As[32];
      float2 b0 = Bs[0], b1 = Bs[16];
#pragma unroll
      for (int k = 0; k < kTK; ++k) {
        float a0n = 0.f, a1n = 0.f;
        float2 b0n = make_float2(0.f, 0.f), b1n = make_float2(0.f, 0.f);
        if (k + 1 < kTK) {
          a0n = As[(k + 1) * kAStride];
          a1n = As[(k + 1) * kAStride + 32];
          b0n = Bs[(k + 1) * kBStride];
          b1n = Bs[(k + 1) * kBStride + 16];
        }
        const float v0 = bsign * (bswap ? b0.y : b0.x);
        const float v1 = bsign * (bswap ? b1.y : b1.x);
        acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, v0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, v1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, v0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, v1, acc[1][1], 0, 0, 0);
        a0 = a0n;
        a1 = a1n;
        b0 = b0n;
        b1 = b1n;
      }
      if (more) {
        float* An = Abuf + (cur ^ 1) * kABuf;
        float2* Bn = Bbuf + (cur ^ 1) * kBBuf;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          An[lA[j]] = ra[j].x;
          An[lA[j] + kAPlane] = ra[j].y;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) Bn[lB[j]] = rb[j];
      }
      __syncthreads();
    }

    // Epilogue: two halves of 64 rows staged in the operand buffers.
    float* Cs = lds;
    TileTab* tcs = reinterpret_cast<TileTab*>(lds + kCHalf);
    build_tab_skip(d.tC, hb, kCStride, 2, *tcs);
    const Scale sc = compute_scale(d, js, jb);
    float lmax = 0.f;
    int bad = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (wm == h) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              const int row = i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
              const int col = wn * 64 + j * 32 + (lane & 31);
              Cs[row * kCStride + col] = acc[i][j][r];
            }
      }
      __syncthreads();
      const int64_t gl = tcs->g[lane] + (h ? g_half : 0);
      const int32_t cl = tcs->c[lane];
#pragma unroll 4
      for (int j = 0; j < 16; ++j) {
        const int hi = 64 + wave + 4 * j;
        const int c = cl + tcs->c[hi];
        const int64_t at = oC + gl + tcs->g[hi];
        store_out<SC>(d, at, make_float2(Cs[c], Cs[c + 1]), sc, lmax, bad);
      }
      __syncthreads();
    }
    finish_scale<256>(d, js, jb, lmax, bad, red, ro == 0 && no == 0, sc);
    __syncthreads();
  }
}

#define RQC_MFMA_CASE(a, b, c)                                                         \
  if (sa == a && sb == b && sc == c) {                                                 \
    hipLaunchKernelGGL((k_mfma32<a, b, c>), grid, dim3(256), 0, s, d);                \
    return hipGetLastError();                                                          \
  }

hipError_t launch_mfma32_kernel(const StepDesc& d, int sa, int sb, int sc, dim3 grid,
                                hipStream_t s) {
  if (d.rt != 7 || d.nt != 6 || d.kt != 4) return hipErrorInvalidValue;
  RQC_MFMA_CASE(ST_C64, ST_C64, ST_C64)
  RQC_MFMA_CASE(ST_C64, ST_C64, ST_F16)
  RQC_MFMA_CASE(ST_C64, ST_C64, ST_BF16)
  RQC_MFMA_CASE(ST_F16, ST_C64, ST_F16)
  RQC_MFMA_CASE(ST_F16, ST_C64, ST_C64)
  RQC_MFMA_CASE(ST_BF16, ST_C64, ST_BF16)
  RQC_MFMA_CASE(ST_BF16, ST_C64, ST_C64)
  RQC_MFMA_CASE(ST_C64, ST_F16, ST_F16)
  RQC_MFMA_CASE(ST_C64, ST_F16, ST_C64)
  RQC_MFMA_CASE(ST_C64, ST_BF16, ST_BF16)
  RQC_MFMA_CASE(ST_C64, ST_BF16, ST_C64)
  RQC_MFMA_CASE(ST_F16, ST_F16, ST_F16)
  RQC_MFMA_CASE(ST_F16, ST_F16, ST_C64)
  RQC_MFMA_CASE(ST_BF16, ST_BF16, ST_BF16)
  RQC_MFMA_CASE(ST_BF16, ST_BF16, ST_C64)
  return hipErrorInvalidValue;
}
#undef RQC_MFMA_CASE

}  // namespace rqc

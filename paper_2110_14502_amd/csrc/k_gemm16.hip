// FP16 / BF16 matrix-core GEMM for long sums (two-phase reduced-precision
// contraction, Sections 5.4 and 5.5).
#include "kernels_dev.h"

namespace rqc {

// ---------------------------------------------------------------------------
// When a step sums over many indices its arithmetic outweighs its operand
// traffic by orders of magnitude, and the 16-bit matrix cores (16 times the
// FP32 rate) are limited by how fast operands reach them, not by HBM.  Such
// a step runs in two phases: each operand is permuted into a plain
// [row][k] matrix of packed 16-bit (re, im) words, the summed indices
// lowest and in the same order in A and in B (k_permute with conversion);
// then this kernel multiplies the two matrices and writes C in its own
// layout through per-row and per-column offset tables.  The extra traffic
// (read 8 B, write 4 B per operand element) is small against 8 MNK flops.
//
// Tile: 256 rows x 128 complex columns (the real output 256 x 256), 32
// complex k per LDS chunk, 8 waves as 2 (rows) x 4 (columns), each wave 128
// rows x 32 complex columns = 4 x 2 blocks of v_mfma_f32_32x32x16_{f16,bf16}
// (FP32 accumulation).  Operands sit in LDS as packed words, k contiguous,
// rows padded to 36 words: a lane's 8 real k of A_r are one 16-byte read;
// B_r is formed per lane from four packed values of its column by a sign
// flip (output column parity 0: (re, -im)) or a half swap (parity 1:
// (im, re)).  Two LDS buffers and two register sets: while one chunk is
// multiplied the next two are in flight; one barrier per chunk.  111 KB of
// LDS, one workgroup of 512 threads per CU.  When the output has too few
// tiles to fill the GPU, the sum is split 2^ksplit ways: each split writes
// FP32 partials to a plain buffer and a second kernel adds them in split
// order.
//
// Workgroup order: blocks are dealt round-robin to the 8 XCDs, so block b is
// remapped to a contiguous range of tiles per XCD; inside a copy, tiles are
// walked in groups of 8 row tiles, row tiles fastest, so the workgroups of
// an XCD that run together share 8 row panels of A and a few column panels
// of B in that XCD's L2.
// ---------------------------------------------------------------------------
typedef _Float16 g16_halfx8 __attribute__((ext_vector_type(8)));
typedef __bf16 g16_bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int g16_u32x4 __attribute__((ext_vector_type(4)));

constexpr int kG16Row = kGemm16K + 4;         // words per LDS row (16-byte aligned)
constexpr int kG16ABuf = kGemm16M * kG16Row;  // words per A buffer
constexpr int kG16BBuf = kGemm16N * kG16Row;  // words per B buffer

template <int LP>
__device__ __forceinline__ floatx16 g16_mfma(g16_u32x4 a, g16_u32x4 b, floatx16 c);
template <>
__device__ __forceinline__ floatx16 g16_mfma<ST_F16>(g16_u32x4 a, g16_u32x4 b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(g16_halfx8, a),
                                                __builtin_bit_cast(g16_halfx8, b), c, 0, 0, 0);
}
template <>
__device__ __forceinline__ floatx16 g16_mfma<ST_BF16>(g16_u32x4 a, g16_u32x4 b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(g16_bf16x8, a),
                                                 __builtin_bit_cast(g16_bf16x8, b), c, 0, 0, 0);
}

// B_r words of a lane from four packed complex values of its column:
// (re, -im) for output column parity 0, (im, re) for parity 1, as a rotation
// by `rot` (0 or 16 bits) and an xor with `flip`, both fixed per lane (no
// select on the loaded words, which the compiler turns into branches).
__device__ __forceinline__ g16_u32x4 g16_expand_b(g16_u32x4 w, uint32_t rot, uint32_t flip) {
  g16_u32x4 o;
#pragma unroll
  for (int i = 0; i < 4; ++i) o[i] = __builtin_amdgcn_alignbit(w[i], w[i], rot) ^ flip;
  return o;
}

// Vector v of a chunk (row v >> 3, words 4 (v & 7) .. + 3 of the chunk).
__device__ __forceinline__ uint4 g16_ld(const uint32_t* base, int64_t K, int kc, int v) {
  return *reinterpret_cast<const uint4*>(base + (int64_t)(v >> 3) * K + kc * kGemm16K + (v & 7) * 4);
}
__device__ __forceinline__ void g16_st(uint32_t* buf, int v, uint4 x) {
  *reinterpret_cast<uint4*>(buf + (v >> 3) * kG16Row + (v & 7) * 4) = x;
}

template <int LP>
__global__ __launch_bounds__(512, 1) void k_gemm16(Gemm16Desc d) {
  __shared__ __attribute__((aligned(16))) uint32_t lw[2 * kG16ABuf + 2 * kG16BBuf];
  __shared__ int64_t roff[kGemm16M];
  __shared__ int64_t coff[kGemm16N];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 2, wc = wave & 3;

  // Work item of this workgroup: (copy, K split, row tile, column tile);
  // row tiles 2^(m-8), column tiles 2^(n-7), splits 2^ksplit.
  const uint64_t T = gridDim.x;
  uint64_t L = blockIdx.x;
  if ((T & 7) == 0) L = (L & 7) * (T >> 3) + (L >> 3);
  const int rbits = d.m - 8, cbits = d.n - 7;
  const uint64_t l = L & ((uint64_t(1) << (rbits + cbits)) - 1);
  const uint64_t ks = (L >> (rbits + cbits)) & ((uint64_t(1) << d.ksplit) - 1);
  const uint64_t copy = L >> (rbits + cbits + d.ksplit);
  const int gr = rbits < 3 ? rbits : 3;
  const uint64_t grp = l >> (gr + cbits);
  const uint64_t in = l & ((uint64_t(1) << (gr + cbits)) - 1);
  const uint64_t rt = (grp << gr) | (in & ((uint64_t(1) << gr) - 1));
  const uint64_t ct = in >> gr;

  // Output offsets of the tile's rows and columns (complex elements): C's
  // layout, or the plain [row][column] partial buffer of this split.
  if (tid < kGemm16M) {
    const uint64_t r = (rt << 8) | (uint64_t)tid;
    int64_t o = 0;
    if (d.ksplit)
      o = (int64_t)r << d.n;
    else
      for (int b = 0; b < d.m; ++b)
        if ((r >> b) & 1) o += int64_t(1) << d.crow[b];
    roff[tid] = o;
  } else if (tid < kGemm16M + kGemm16N) {
    const uint64_t c = (ct << 7) | (uint64_t)(tid - kGemm16M);
    int64_t o = 0;
    if (d.ksplit)
      o = (int64_t)c;
    else
      for (int b = 0; b < d.n; ++b)
        if ((c >> b) & 1) o += int64_t(1) << d.ccol[b];
    coff[tid - kGemm16M] = o;
  }

  const int64_t K = int64_t(1) << d.k;  // complex k = words per operand row
  const int n_kc = 1 << (d.k - 5 - d.ksplit);  // chunks of this split
  const int kc0 = (int)ks * n_kc;
  const uint32_t* Ab = d.A + (int64_t)copy * d.sA + (int64_t)(rt << 8) * K;
  const uint32_t* Bb = d.B + (int64_t)copy * d.sB + (int64_t)(ct << 7) * K;
  uint32_t* Abuf = lw;
  uint32_t* Bbuf = lw + 2 * kG16ABuf;

  // Chunk kc: A rows 0..255 and B columns 0..127, words 32 kc .. 32 kc + 31
  // (8 vectors of 4 words per row).  Vector v = tid + 512 j: row v >> 3,
  // part v & 7 (eight consecutive threads read one row's 128 bytes).  Two
  // chunks are in flight in two register sets X and Y (named registers: an
  // array captured by a lambda would be promoted to LDS) while a third is
  // multiplied from LDS.
  uint4 xa0, xa1, xa2, xa3, xb0, xb1, ya0, ya1, ya2, ya3, yb0, yb1;
#define G16_LOAD(S, kc)                              \
  S##a0 = g16_ld(Ab, K, kc0 + (kc), tid);            \
  S##a1 = g16_ld(Ab, K, kc0 + (kc), tid + 512);      \
  S##a2 = g16_ld(Ab, K, kc0 + (kc), tid + 1024);     \
  S##a3 = g16_ld(Ab, K, kc0 + (kc), tid + 1536);     \
  S##b0 = g16_ld(Bb, K, kc0 + (kc), tid);            \
  S##b1 = g16_ld(Bb, K, kc0 + (kc), tid + 512);
#define G16_STASH(S, buf)                              \
  g16_st(Abuf + (buf) * kG16ABuf, tid, S##a0);         \
  g16_st(Abuf + (buf) * kG16ABuf, tid + 512, S##a1);   \
  g16_st(Abuf + (buf) * kG16ABuf, tid + 1024, S##a2);  \
  g16_st(Abuf + (buf) * kG16ABuf, tid + 1536, S##a3);  \
  g16_st(Bbuf + (buf) * kG16BBuf, tid, S##b0);         \
  g16_st(Bbuf + (buf) * kG16BBuf, tid + 512, S##b1);

  G16_LOAD(x, 0)
  if (n_kc > 1) {
    G16_LOAD(y, 1)
  }
  G16_STASH(x, 0)
  if (n_kc > 2) {
    G16_LOAD(x, 2)
  }
  __syncthreads();

  const int lrow = lane & 31;
  const int kq = (lane >> 5) * 4;      // first complex k of the lane's 8 real k
  const int ncol = (lane & 31) >> 1;   // complex column inside a 32-column real block
  // C_r column parity 1 takes (im, re), parity 0 (re, -im).
  const uint32_t brot = (lane & 1) ? 16u : 0u, bflip = (lane & 1) ? 0u : 0x80000000u;

  floatx16 acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  auto multiply = [&](int cb) {
    const uint32_t* As = Abuf + cb * kG16ABuf + (wr * 128 + lrow) * kG16Row + kq;
    const uint32_t* Bs = Bbuf + cb * kG16BBuf + (wc * 32 + ncol) * kG16Row + kq;
    // The fragments of step kk + 1 are read from LDS before the products of
    // step kk are issued.
    g16_u32x4 a0[4], b0[2], a1[4], b1[2];
#define G16_FRAGS(A, B, kk)                                                                 \
  _Pragma("unroll") for (int i = 0; i < 4; ++i)                                            \
      A[i] = *reinterpret_cast<const g16_u32x4*>(As + i * 32 * kG16Row + (kk) * 8);       \
  _Pragma("unroll") for (int j = 0; j < 2; ++j)                                            \
      B[j] = *reinterpret_cast<const g16_u32x4*>(Bs + j * 16 * kG16Row + (kk) * 8);
#define G16_PRODUCTS(A, B)                                                                  \
  {                                                                                         \
    g16_u32x4 be[2];                                                                        \
    _Pragma("unroll") for (int j = 0; j < 2; ++j) be[j] = g16_expand_b(B[j], brot, bflip); \
    _Pragma("unroll") for (int i = 0; i < 4; ++i)                                          \
        _Pragma("unroll") for (int j = 0; j < 2; ++j) acc[i][j] =                          \
            g16_mfma<LP>(A[i], be[j], acc[i][j]);                                           \
  }
    G16_FRAGS(a0, b0, 0)
    G16_FRAGS(a1, b1, 1)
    __builtin_amdgcn_sched_barrier(0);
    G16_PRODUCTS(a0, b0)
    __builtin_amdgcn_sched_barrier(0);
    G16_FRAGS(a0, b0, 2)
    __builtin_amdgcn_sched_barrier(0);
    G16_PRODUCTS(a1, b1)
    __builtin_amdgcn_sched_barrier(0);
    G16_FRAGS(a1, b1, 3)
    __builtin_amdgcn_sched_barrier(0);
    G16_PRODUCTS(a0, b0)
    __builtin_amdgcn_sched_barrier(0);
    G16_PRODUCTS(a1, b1)
#undef G16_FRAGS
#undef G16_PRODUCTS
  };

  // Chunk i sits in LDS buffer i & 1; chunk i + 1 in set Y (i even) or X
  // (i odd), chunk i + 2 in the other set.  After chunk i is multiplied,
  // chunk i + 1 goes to the other buffer and its set takes chunk i + 3.
  for (int i = 0; i < n_kc; i += 2) {
    multiply(0);
    if (i + 1 < n_kc) {
      G16_STASH(y, 1)
      if (i + 3 < n_kc) {
        G16_LOAD(y, i + 3)
      }
    }
    __syncthreads();
    if (i + 1 < n_kc) {
      multiply(1);
      if (i + 2 < n_kc) {
        G16_STASH(x, 0)
        if (i + 4 < n_kc) {
          G16_LOAD(x, i + 4)
        }
      }
      __syncthreads();
    }
  }

  // Output: accumulator element r of block (i, j) is real row
  // 8 (r >> 2) + 4 (lane >> 5) + (r & 3) of the block and real column
  // lane & 31, i.e. complex column (lane & 31) >> 1, part lane & 1.
  float* Cf = d.ksplit ? reinterpret_cast<float*>(d.P) +
                             2 * ((int64_t)(copy << d.ksplit | ks) << (d.m + d.n))
                       : reinterpret_cast<float*>(d.C) + 2 * ((int64_t)copy * d.sC);
  const int part = lane & 1;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t co = coff[wc * 32 + j * 16 + ncol];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = wr * 128 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        __builtin_nontemporal_store(acc[i][j][r], Cf + 2 * (roff[row] + co) + part);
      }
    }
#undef G16_LOAD
#undef G16_STASH
}

// Split-K partials summed in split order (the result does not depend on
// timing) and written to C in its layout: one thread per output element.
__global__ __launch_bounds__(256) void k_gemm16_reduce(Gemm16Desc d) {
  const uint64_t per = uint64_t(1) << (d.m + d.n);
  const uint64_t total = per * (uint64_t)d.copies;
  const int S = 1 << d.ksplit;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t copy = e >> (d.m + d.n), rc = e & (per - 1);
    const uint64_t r = rc >> d.n, c = rc & ((uint64_t(1) << d.n) - 1);
    const float2* p = d.P + ((copy << d.ksplit) << (d.m + d.n)) + rc;
    float2 v = p[0];
    for (int s = 1; s < S; ++s) {
      const float2 w = p[(uint64_t)s << (d.m + d.n)];
      v.x += w.x;
      v.y += w.y;
    }
    int64_t o = (int64_t)copy * d.sC;
    for (int b = 0; b < d.m; ++b)
      if ((r >> b) & 1) o += int64_t(1) << d.crow[b];
    for (int b = 0; b < d.n; ++b)
      if ((c >> b) & 1) o += int64_t(1) << d.ccol[b];
    reinterpret_cast<float2*>(d.C)[o] = v;
  }
}

hipError_t launch_gemm16(const Gemm16Desc& d, int lp_kind, hipStream_t s) {
  if (d.m < 8 || d.n < 7 || d.k < 5 || d.m > 40 || d.n > 40 || d.copies < 1)
    return hipErrorInvalidValue;
  if (d.ksplit < 0 || d.k - 5 - d.ksplit < 0 || (d.ksplit && !d.P)) return hipErrorInvalidValue;
  const uint64_t tiles = (uint64_t)d.copies << (d.m - 8 + d.n - 7 + d.ksplit);
  if (tiles > 0x7fffffffull) return hipErrorInvalidValue;
  if (lp_kind == ST_F16)
    hipLaunchKernelGGL(k_gemm16<ST_F16>, dim3((unsigned)tiles), dim3(512), 0, s, d);
  else if (lp_kind == ST_BF16)
    hipLaunchKernelGGL(k_gemm16<ST_BF16>, dim3((unsigned)tiles), dim3(512), 0, s, d);
  else
    return hipErrorInvalidValue;
  if (d.ksplit) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const uint64_t total = (uint64_t)d.copies << (d.m + d.n);
    const uint64_t blocks = (total + 255) / 256;
    hipLaunchKernelGGL(k_gemm16_reduce, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256),
                       0, s, d);
  }
  return hipGetLastError();
}

}  // namespace rqc

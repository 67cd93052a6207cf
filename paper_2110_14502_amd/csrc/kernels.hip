// HIP kernels for gfx950 (CDNA4): fused permute + complex GEMM contraction
// steps (Section 5.4), slice / bitstring instantiation of the leaves
// (Section 5.1), and the FP64 cross-slice reduction (Section 6.4).
//
// Complex arithmetic on the real matrix cores: an interleaved complex
// A[m][k] is read as the real matrix A_r[m][2k+c] (c = 0 re, 1 im); the
// complex B[k][n] is expanded per lane into the real 2x2 block
//   B_r[2k+0][2n+0] = Br   B_r[2k+0][2n+1] = Bi
//   B_r[2k+1][2n+0] = -Bi  B_r[2k+1][2n+1] = Br
// so that A_r * B_r is exactly the interleaved complex C[m][2n+d].  The real
// flops executed equal 8 per complex multiply-add, the algorithmic count.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace rqc {

typedef _Float16 h2 __attribute__((ext_vector_type(2)));
typedef __bf16 b2 __attribute__((ext_vector_type(2)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------------------
// Storage helpers
// ---------------------------------------------------------------------------
template <int S>
__device__ __forceinline__ float2 load_c(const void* p, int64_t i);
template <>
__device__ __forceinline__ float2 load_c<ST_C64>(const void* p, int64_t i) {
  return reinterpret_cast<const float2*>(p)[i];
}
template <>
__device__ __forceinline__ float2 load_c<ST_F16>(const void* p, int64_t i) {
  h2 v = reinterpret_cast<const h2*>(p)[i];
  return make_float2((float)v.x, (float)v.y);
}
template <>
__device__ __forceinline__ float2 load_c<ST_BF16>(const void* p, int64_t i) {
  b2 v = reinterpret_cast<const b2*>(p)[i];
  return make_float2((float)v.x, (float)v.y);
}

template <int S>
__device__ __forceinline__ void store_c(void* p, int64_t i, float2 v);
template <>
__device__ __forceinline__ void store_c<ST_C64>(void* p, int64_t i, float2 v) {
  reinterpret_cast<float2*>(p)[i] = v;
}
template <>
__device__ __forceinline__ void store_c<ST_F16>(void* p, int64_t i, float2 v) {
  h2 o;
  o.x = (_Float16)v.x;
  o.y = (_Float16)v.y;
  reinterpret_cast<h2*>(p)[i] = o;
}
template <>
__device__ __forceinline__ void store_c<ST_BF16>(void* p, int64_t i, float2 v) {
  b2 o;
  o.x = (__bf16)v.x;
  o.y = (__bf16)v.y;
  reinterpret_cast<b2*>(p)[i] = o;
}

// Smallest E with x <= 2^E, for x > 0.
__device__ __forceinline__ int ceil_log2(float x) {
  int e;
  float m = frexpf(x, &e);
  return m == 0.5f ? e - 1 : e;
}

__device__ __forceinline__ void decode(const TileMap& t, uint32_t e, int lo, int hi, int64_t& g,
                                       int& r, int& cc, int& k) {
  for (int b = lo; b < hi; ++b) {
    if ((e >> (b - lo)) & 1) {
      g += int64_t(1) << t.gpos[b];
      const int v = 1 << t.cbit[b];
      if (t.role[b] == 0) r += v;
      else if (t.role[b] == 1) cc += v;
      else k += v;
    }
  }
}

// Per-copy scale bookkeeping shared by both kernels' epilogues.
struct Scale {
  int shift;  // C_stored = acc * 2^-shift
  int expC;
};
__device__ __forceinline__ Scale compute_scale(const StepDesc& d, int js, int jb) {
  Scale s{0, 0};
  if (!d.track) return s;
  const int eA = d.expA ? d.expA[js * d.eA_s + jb * d.eA_b] : 0;
  const int eB = d.expB ? d.expB[js * d.eB_s + jb * d.eB_b] : 0;
  int t = 0;
  if (d.lp_out) {
    const float mA = d.maxA ? d.maxA[js * d.eA_s + jb * d.eA_b] : d.maxA_const;
    const float mB = d.maxB ? d.maxB[js * d.eB_s + jb * d.eB_b] : d.maxB_const;
    // |C_re|,|C_im| <= sum_k |A||B| <= 2^k * (sqrt2 mA)(sqrt2 mB): store so
    // that this bound maps to 2^15, inside the binary16 range.
    if (mA > 0.f && mB > 0.f && mA <= 3.0e38f && mB <= 3.0e38f)
      t = d.k_total + 1 + ceil_log2(mA) + ceil_log2(mB) - 15 - d.bias;
  }
  s.shift = t;
  s.expC = eA + eB + t;
  return s;
}

__device__ __forceinline__ float wave_max(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

template <int BLOCK>
__device__ __forceinline__ void finish_scale(const StepDesc& d, int js, int jb, float local_max,
                                             int bad, float* red, bool write_exp, const Scale& sc) {
  if (!d.track) return;
  float m = wave_max(local_max);
  int anybad = __any(bad);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    red[w] = m;
    reinterpret_cast<int*>(red)[BLOCK / 64 + w] = anybad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float bm = 0.f;
    int bb = 0;
    for (int i = 0; i < BLOCK / 64; ++i) {
      bm = fmaxf(bm, red[i]);
      bb |= reinterpret_cast<int*>(red)[BLOCK / 64 + i];
    }
    const int ci = js * d.eC_s + jb * d.eC_b;
    if (d.maxC) atomicMax(reinterpret_cast<unsigned int*>(d.maxC) + ci, __float_as_uint(bm));
    if (write_exp && d.expC) d.expC[ci] = sc.expC;
    if (bb && d.flag) {
      if (d.dep_s_c) d.flag[js] = 1;
      else
        for (int i = 0; i < d.flag_n; ++i) d.flag[i] = 1;  // shared by every slice
    }
  }
}

__device__ __forceinline__ void outer_offsets(const StepDesc& d, uint64_t ro, uint64_t no, int js,
                                              int jb, int64_t& oA, int64_t& oB, int64_t& oC) {
  oA = js * d.sA_s + jb * d.sA_b;
  oB = js * d.sB_s + jb * d.sB_b;
  oC = js * d.sC_s + jb * d.sC_b;
  for (int i = 0; i < d.n_ro; ++i)
    if ((ro >> i) & 1) {
      oA += int64_t(1) << d.ro_A[i];
      oC += int64_t(1) << d.ro_C[i];
    }
  for (int i = 0; i < d.n_no; ++i)
    if ((no >> i) & 1) {
      oB += int64_t(1) << d.no_B[i];
      oC += int64_t(1) << d.no_C[i];
    }
}

__device__ __forceinline__ void k_offsets(const StepDesc& d, uint32_t kc, int64_t& kA, int64_t& kB) {
  kA = 0;
  kB = 0;
  for (int i = 0; i < d.n_ko; ++i)
    if ((kc >> i) & 1) {
      kA += int64_t(1) << d.ko_A[i];
      kB += int64_t(1) << d.ko_B[i];
    }
}

// ---------------------------------------------------------------------------
// Offset tables of a tile: element e (bits in increasing address order) sits
// at global offset g_lo[e & 63] + g_hi[e >> 6] and at LDS coordinate
// c_lo[e & 63] + c_hi[e >> 6], where the coordinate of a tile bit is its
// weight inside the LDS array (row bits scaled by the row stride).  Built
// once per workgroup into LDS, so the per-element cost is two lookups.
// ---------------------------------------------------------------------------
struct TileTab {
  int64_t g[128];  // [0, 64) low six bits, [64, 128) the high bits
  int32_t c[128];
};

__device__ __forceinline__ void build_tab(const TileMap& t, int row_stride, int col_stride,
                                          int k_stride, TileTab& tab) {
  for (int i = threadIdx.x; i < 128; i += blockDim.x) {
    const int hi = i >= 64;
    const int v = hi ? i - 64 : i;
    const int b0 = hi ? 6 : 0;
    const int b1 = hi ? t.nbits : (t.nbits < 6 ? t.nbits : 6);
    int64_t g = 0;
    int32_t c = 0;
    for (int b = b0; b < b1; ++b) {
      if ((v >> (b - b0)) & 1) {
        g += int64_t(1) << t.gpos[b];
        const int w = 1 << t.cbit[b];
        c += t.role[b] == 0 ? w * row_stride : (t.role[b] == 1 ? w * col_stride : w * k_stride);
      }
    }
    tab.g[i] = g;
    tab.c[i] = c;
  }
}

// Epilogue shared by the SIMT kernels: scale, convert, store, track.
template <int SC>
__device__ __forceinline__ void store_out(const StepDesc& d, int64_t at, float2 v, const Scale& sc,
                                          float& lmax, int& bad) {
  if (sc.shift) {
    v.x = ldexpf(v.x, -sc.shift);
    v.y = ldexpf(v.y, -sc.shift);
  }
  store_c<SC>(d.C, at, v);
  if (d.track) {
    float2 w = v;
    if (SC != ST_C64) w = load_c<SC>(d.C, at);
    const float m = fmaxf(fabsf(w.x), fabsf(w.y));
    if (!(m <= 3.4e38f)) bad = 1;
    else lmax = fmaxf(lmax, m);
  }
}

// ---------------------------------------------------------------------------
// Row-streaming contraction for plan steps (the memory-bound "stem" steps of
// Section 5.4's imbalanced case): A is a row-major [M][K] matrix whose K
// summed bits are its lowest address bits, B is [N][K] with the same K order
// and small enough for LDS.  Each thread streams whole rows of A (K
// contiguous values, vector loads), multiplies them by B read as LDS
// broadcasts, and parks the row's N outputs in LDS; the tile is then written
// out in C's own address order through the offset tables.
// ---------------------------------------------------------------------------
constexpr int kRowsMaxB = 2048;  // N*K
constexpr int kRowsMaxC = 2048;  // R*N
// C tile with a padded row stride ldc = N + 1 (N >= 2) or 1 (N == 1):
// R * ldc <= R*N + R <= 2048 + 1024.
constexpr int kRowsCs = kRowsMaxC + kRowsMaxC / 2;
// Rows each thread keeps in flight (all loads issued before any use).
__host__ __device__ constexpr int rows_per_thread(int kb) { return kb <= 3 ? 8 : (kb == 4 ? 4 : 2); }

// One contiguous row of K complex values with 16-byte loads where the row
// is long enough (rows start at multiples of K elements, so they are aligned).
template <int S, int K>
__device__ __forceinline__ void load_row(const void* p, int64_t base, float2* a) {
  if (S == ST_C64) {
    const float2* q = reinterpret_cast<const float2*>(p) + base;
    if (K >= 2) {
#pragma unroll
      for (int k = 0; k < K; k += 2) {
        const float4 v = *reinterpret_cast<const float4*>(q + k);
        a[k] = make_float2(v.x, v.y);
        a[k + 1] = make_float2(v.z, v.w);
      }
    } else {
      a[0] = q[0];
    }
  } else {
    const uint32_t* q = reinterpret_cast<const uint32_t*>(p) + base;
    uint32_t w[K];
    if (K >= 4) {
#pragma unroll
      for (int k = 0; k < K; k += 4) {
        const uint4 v = *reinterpret_cast<const uint4*>(q + k);
        w[k] = v.x;
        w[k + 1] = v.y;
        w[k + 2] = v.z;
        w[k + 3] = v.w;
      }
    } else if (K == 2) {
      const uint2 v = *reinterpret_cast<const uint2*>(q);
      w[0] = v.x;
      w[1] = v.y;
    } else {
      w[0] = q[0];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (S == ST_F16) {
        const h2 h = __builtin_bit_cast(h2, w[k]);
        a[k] = make_float2((float)h.x, (float)h.y);
      } else {
        const b2 h = __builtin_bit_cast(b2, w[k]);
        a[k] = make_float2((float)h.x, (float)h.y);
      }
    }
  }
}

template <int KB, int SA>
__global__ __launch_bounds__(256) void k_rows(StepDesc d) {
  constexpr int K = 1 << KB;
  constexpr int RP = rows_per_thread(KB);
  extern __shared__ float2 rows_lds[];
  __shared__ TileTab tc;
  __shared__ int64_t bofs[64];
  __shared__ float red[16];
  const int tid = threadIdx.x;
  const int N = 1 << d.nt, R = 1 << d.rt, NC = 1 << d.ncb;
  const int ldc = NC == 1 ? 1 : NC + 1;
  float2* Bs = rows_lds;          // [N][K], columns in C's bit order
  float2* Cs = rows_lds + N * K;  // [R][ldc], one chunk of NC columns
  build_tab(d.tC, ldc, 1, 0, tc);
  // Offset in B of column n (its bits scattered to B's column positions).
  for (int n = tid; n < N; n += 256) {
    int64_t g = 0;
    for (int b = 0; b < d.tB.nbits; ++b)
      if ((n >> b) & 1) g += int64_t(1) << d.tB.gpos[b];
    bofs[n] = g;
  }
  const uint64_t ro = blockIdx.x;
  const int nC = R * NC;
  for (int copy = blockIdx.y; copy < d.copies; copy += gridDim.y) {
    const int js = copy % d.gs_c, jb = copy / d.gs_c;
    int64_t oA, oB, oC;
    outer_offsets(d, ro, 0, js, jb, oA, oB, oC);
    // Issue this thread's row loads first: they are the HBM stream.
    float2 a[RP][K];
#pragma unroll
    for (int rp = 0; rp < RP; ++rp) {
      const int r = tid + 256 * rp;
      if (r < R) load_row<SA, K>(d.A, oA + (int64_t)r * K, a[rp]);
    }
    __syncthreads();
    for (int i = tid; i < N * K; i += 256) {
      const int64_t at = oB + bofs[i / K] + (i % K);
      float2 v;
      if (d.sb_store == ST_F16) v = load_c<ST_F16>(d.B, at);
      else if (d.sb_store == ST_BF16) v = load_c<ST_BF16>(d.B, at);
      else v = load_c<ST_C64>(d.B, at);
      Bs[i] = v;
    }
    const Scale sc = compute_scale(d, js, jb);
    float lmax = 0.f;
    int bad = 0;
    const int64_t glo = tc.g[tid & 63];
    const int32_t clo = tc.c[tid & 63];
    for (int ch = 0; ch < N; ch += NC) {
      __syncthreads();
      // Each B value read from LDS (a broadcast) serves all of the thread's
      // rows.
      for (int nn = 0; nn < NC; ++nn) {
        const float2* b = Bs + (ch + nn) * K;
        float sx[RP], sy[RP];
#pragma unroll
        for (int rp = 0; rp < RP; ++rp) sx[rp] = sy[rp] = 0.f;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const float2 bv = b[k];
#pragma unroll
          for (int rp = 0; rp < RP; ++rp) {
            sx[rp] = fmaf(a[rp][k].x, bv.x, sx[rp]);
            sx[rp] = fmaf(-a[rp][k].y, bv.y, sx[rp]);
            sy[rp] = fmaf(a[rp][k].x, bv.y, sy[rp]);
            sy[rp] = fmaf(a[rp][k].y, bv.x, sy[rp]);
          }
        }
#pragma unroll
        for (int rp = 0; rp < RP; ++rp) {
          const int r = tid + 256 * rp;
          if (r < R) Cs[r * ldc + nn] = make_float2(sx[rp], sy[rp]);
        }
      }
      __syncthreads();
      int64_t gch = 0;
      for (int j = 0; j < d.nt - d.ncb; ++j)
        if (((ch >> d.ncb) >> j) & 1) gch += int64_t(1) << d.nh_C[j];
      for (int e = tid; e < nC; e += 256) {
        const int hi = 64 + (e >> 6);
        const float2 v = Cs[clo + tc.c[hi]];
        const int64_t at = oC + gch + glo + tc.g[hi];
        if (d.sc_store == ST_F16) store_out<ST_F16>(d, at, v, sc, lmax, bad);
        else if (d.sc_store == ST_BF16) store_out<ST_BF16>(d, at, v, sc, lmax, bad);
        else store_out<ST_C64>(d, at, v, sc, lmax, bad);
      }
    }
    finish_scale<256>(d, js, jb, lmax, bad, red, ro == 0, sc);
  }
}

// ---------------------------------------------------------------------------
// Generic SIMT contraction (any layouts, any sizes): tiles of R rows x N
// columns, K in chunks; loads follow each operand's address order through
// the offset tables; optional split-K into partial buffers.
// ---------------------------------------------------------------------------
constexpr int kSimtBlock = 256;
constexpr int kSimtMaxC = 8;  // C tile <= 2048 elements

template <int SA, int SB, int SC>
__global__ __launch_bounds__(kSimtBlock) void k_simt(StepDesc d) {
  extern __shared__ float2 smem2[];
  __shared__ TileTab ta, tb, tcc;
  __shared__ float red[16];
  const int R = 1 << d.rt, N = 1 << d.nt, K = 1 << d.kt;
  const int ldA = K + 1, ldB = N + 1;
  float2* As = smem2;
  float2* Bs = As + R * ldA;
  const int tid = threadIdx.x, lane = tid & 63;
  build_tab(d.tA, ldA, 0, 1, ta);
  build_tab(d.tB, 0, 1, ldB, tb);
  build_tab(d.tC, 4096, 1, 0, tcc);  // coordinate = row * 4096 + col
  const uint64_t tiles = (uint64_t)d.n_row_tiles * (uint64_t)d.n_col_tiles;
  const uint64_t split = blockIdx.x / tiles;
  const uint64_t tile = blockIdx.x % tiles;
  const uint64_t ro = tile % (uint64_t)d.n_row_tiles;
  const uint64_t no = tile / (uint64_t)d.n_row_tiles;
  const int nC = R * N;
  const int nA = R * K, nB = K * N;
  const int n_kc_all = 1 << d.n_ko;
  const int n_kc = n_kc_all >> d.ksplit;
  const int kc0 = (int)split * n_kc;
  __syncthreads();
  // Owned C elements, C address order: global offset and (row, col).
  int64_t cg[kSimtMaxC];
  int crow[kSimtMaxC], ccol[kSimtMaxC];
  const int64_t glo = tcc.g[lane];
  const int32_t clo = tcc.c[lane];
#pragma unroll
  for (int i = 0; i < kSimtMaxC; ++i) {
    const int e = tid + i * kSimtBlock;
    const int hi = 64 + (e >> 6);
    const int ee = e < nC ? hi : 64;
    cg[i] = glo + tcc.g[ee];
    const int c = clo + tcc.c[ee];
    crow[i] = c >> 12;
    ccol[i] = c & 4095;
  }
  const int64_t gAlo = ta.g[lane], gBlo = tb.g[lane];
  const int32_t cAlo = ta.c[lane], cBlo = tb.c[lane];
  for (int copy = blockIdx.y; copy < d.copies; copy += gridDim.y) {
    const int js = copy % d.gs_c, jb = copy / d.gs_c;
    int64_t oA, oB, oC;
    outer_offsets(d, ro, no, js, jb, oA, oB, oC);
    float2 acc[kSimtMaxC];
#pragma unroll
    for (int i = 0; i < kSimtMaxC; ++i) acc[i] = make_float2(0.f, 0.f);
    for (int kc = kc0; kc < kc0 + n_kc; ++kc) {
      int64_t kA, kB;
      k_offsets(d, kc, kA, kB);
      for (int e = tid; e < nA; e += kSimtBlock) {
        const int hi = 64 + (e >> 6);
        As[cAlo + ta.c[hi]] = load_c<SA>(d.A, oA + kA + gAlo + ta.g[hi]);
      }
      for (int e = tid; e < nB; e += kSimtBlock) {
        const int hi = 64 + (e >> 6);
        Bs[cBlo + tb.c[hi]] = load_c<SB>(d.B, oB + kB + gBlo + tb.g[hi]);
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < kSimtMaxC; ++i) {
        if (tid + i * kSimtBlock < nC) {
          const float2* ar = As + crow[i] * ldA;
          const float2* bc = Bs + ccol[i];
          float sx = acc[i].x, sy = acc[i].y;
          for (int k = 0; k < K; ++k) {
            const float2 a = ar[k], b = bc[k * ldB];
            sx = fmaf(a.x, b.x, sx);
            sx = fmaf(-a.y, b.y, sx);
            sy = fmaf(a.x, b.y, sy);
            sy = fmaf(a.y, b.x, sy);
          }
          acc[i] = make_float2(sx, sy);
        }
      }
      __syncthreads();
    }
    if (d.ksplit) {
      // Partial sums: plain complex64, reduced by k_splitk_reduce.
      float2* P = d.P + (int64_t)split * d.p_stride;
#pragma unroll
      for (int i = 0; i < kSimtMaxC; ++i)
        if (tid + i * kSimtBlock < nC) P[oC + cg[i]] = acc[i];
      continue;
    }
    const Scale sc = compute_scale(d, js, jb);
    float lmax = 0.f;
    int bad = 0;
#pragma unroll
    for (int i = 0; i < kSimtMaxC; ++i)
      if (tid + i * kSimtBlock < nC) store_out<SC>(d, oC + cg[i], acc[i], sc, lmax, bad);
    finish_scale<kSimtBlock>(d, js, jb, lmax, bad, red, ro == 0 && no == 0, sc);
  }
}

// Split-K reduction: C = sum over splits of the partial buffers, in split
// order, then the usual scale / store / tracking epilogue.  One workgroup
// per (row tile, column tile) of C and copy, elements in C address order.
template <int SC>
__global__ __launch_bounds__(256) void k_splitk_reduce(StepDesc d) {
  __shared__ TileTab tcc;
  __shared__ float red[16];
  const int tid = threadIdx.x;
  build_tab(d.tC, 0, 0, 0, tcc);
  const uint64_t ro = blockIdx.x % (uint64_t)d.n_row_tiles;
  const uint64_t no = blockIdx.x / (uint64_t)d.n_row_tiles;
  const int nC = 1 << (d.rt + d.nt);
  const int ns = 1 << d.ksplit;
  __syncthreads();
  for (int copy = blockIdx.y; copy < d.copies; copy += gridDim.y) {
    const int js = copy % d.gs_c, jb = copy / d.gs_c;
    int64_t oA, oB, oC;
    outer_offsets(d, ro, no, js, jb, oA, oB, oC);
    const Scale sc = compute_scale(d, js, jb);
    float lmax = 0.f;
    int bad = 0;
    for (int e = tid; e < nC; e += 256) {
      const int64_t at = oC + tcc.g[e & 63] + tcc.g[64 + (e >> 6)];
      float sx = 0.f, sy = 0.f;
      for (int s = 0; s < ns; ++s) {
        const float2 v = d.P[(int64_t)s * d.p_stride + at];
        sx += v.x;
        sy += v.y;
      }
      store_out<SC>(d, at, make_float2(sx, sy), sc, lmax, bad);
    }
    finish_scale<256>(d, js, jb, lmax, bad, red, ro == 0 && no == 0, sc);
  }
}

// ---------------------------------------------------------------------------
// MFMA contraction (FP32 matrix cores, v_mfma_f32_32x32x2_f32): 128 rows x
// 64 complex columns per workgroup, 16 complex k per LDS chunk, double
// buffered; 4 waves in a 2x2 grid, each 64 rows x 64 real columns.  The
// operand offsets come from LDS tables built once per workgroup; the output
// tile is staged through LDS in two halves of 64 rows (inside the operand
// buffers) and stored in C's address order.  49.7 KB of LDS: three
// workgroups per CU.
// ---------------------------------------------------------------------------
constexpr int kTM = 128, kTN = 64, kTK = 16;
constexpr int kAPlane = kTM + 1;          // floats per (k, re/im) plane
constexpr int kAStride = 2 * kAPlane;     // floats per k
constexpr int kABuf = kTK * kAStride;     // floats per buffer
constexpr int kBStride = kTN + 1;         // float2 per k
constexpr int kBBuf = kTK * kBStride;     // float2 per buffer
constexpr int kMainFloats = 2 * kABuf + 4 * kBBuf;
constexpr int kCStride = 2 * kTN + 4;     // floats per staged C row
constexpr int kCHalf = 64 * kCStride;     // floats of one staged half
constexpr int kTabFloats = (int)(sizeof(TileTab) / sizeof(float));
static_assert(kCHalf + kTabFloats <= kMainFloats, "C staging must fit the operand buffers");
static_assert(2 * kTabFloats <= kMainFloats, "operand tables must fit the operand buffers");

// Table over the tile bits of `t` except bit `skip` (lo: first six, hi: rest).
__device__ __forceinline__ void build_tab_skip(const TileMap& t, int skip, int row_stride,
                                               int col_stride, TileTab& tab) {
  int pos[kMaxTile];
  int nb = 0;
  for (int b = 0; b < t.nbits; ++b)
    if (b != skip) pos[nb++] = b;
  for (int i = threadIdx.x; i < 128; i += blockDim.x) {
    const int hi = i >= 64;
    const int v = hi ? i - 64 : i;
    const int b0 = hi ? 6 : 0;
    const int b1 = hi ? nb : (nb < 6 ? nb : 6);
    int64_t g = 0;
    int32_t c = 0;
    for (int j = b0; j < b1; ++j) {
      if ((v >> (j - b0)) & 1) {
        const int b = pos[j];
        g += int64_t(1) << t.gpos[b];
        const int w = 1 << t.cbit[b];
        c += t.role[b] == 0 ? w * row_stride : w * col_stride;
      }
    }
    tab.g[i] = g;
    tab.c[i] = c;
  }
}

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

// ---------------------------------------------------------------------------
// Reduced-precision MFMA contraction (FP16 / BF16 matrix cores,
// v_mfma_f32_32x32x16_{f16,bf16}, FP32 accumulation).  Same tiling as the
// FP32 kernel (128 rows x 64 complex columns, 4 waves 2x2) with 32 complex
// k per LDS chunk.  Operands live in LDS as packed complex words (re in the
// low half, im in the high half), k contiguous: a lane's 8 consecutive real
// k of A_r are one 16-byte read; for B_r the lane reads 4 complex values of
// its column and forms (re, -im) by a sign flip (column parity 0) or
// (im, re) by swapping the halves (parity 1).  An operand stored in
// complex64 is converted with a per-copy power-of-two pre-scale that maps
// its max-abs to 2^14; the output exponent undoes it.
// ---------------------------------------------------------------------------
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kLTK = 32;                 // complex k per chunk
constexpr int kLRow = kLTK + 4;          // words per LDS row (16-byte aligned)
constexpr int kLABuf = kTM * kLRow;      // words per A buffer
constexpr int kLBBuf = kTN * kLRow;      // words per B buffer
constexpr int kLMainWords = 2 * kLABuf + 2 * kLBBuf;
static_assert(kCHalf + kTabFloats <= kLMainWords, "C staging must fit the operand buffers");

template <int LP>
__device__ __forceinline__ uint32_t pack_lp(float2 v);
template <>
__device__ __forceinline__ uint32_t pack_lp<ST_F16>(float2 v) {
  h2 o;
  o.x = (_Float16)v.x;
  o.y = (_Float16)v.y;
  return __builtin_bit_cast(uint32_t, o);
}
template <>
__device__ __forceinline__ uint32_t pack_lp<ST_BF16>(float2 v) {
  b2 o;
  o.x = (__bf16)v.x;
  o.y = (__bf16)v.y;
  return __builtin_bit_cast(uint32_t, o);
}

// Load one operand element as a packed low-precision complex word.
template <int LP, int S>
__device__ __forceinline__ uint32_t load_lp(const void* p, int64_t i, int pre) {
  if (S == LP) return reinterpret_cast<const uint32_t*>(p)[i];
  float2 v = load_c<S>(p, i);
  if (pre) {
    v.x = ldexpf(v.x, pre);
    v.y = ldexpf(v.y, pre);
  }
  return pack_lp<LP>(v);
}

template <int LP>
__device__ __forceinline__ floatx16 mfma16(u32x4 a, u32x4 b, floatx16 c);
template <>
__device__ __forceinline__ floatx16 mfma16<ST_F16>(u32x4 a, u32x4 b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(halfx8, a),
                                                __builtin_bit_cast(halfx8, b), c, 0, 0, 0);
}
template <>
__device__ __forceinline__ floatx16 mfma16<ST_BF16>(u32x4 a, u32x4 b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                 __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// B_r words of a lane from four packed complex values of its column.
__device__ __forceinline__ u32x4 expand_b(u32x4 w, bool swap_halves) {
  u32x4 o;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    o[i] = swap_halves ? ((w[i] >> 16) | (w[i] << 16)) : (w[i] ^ 0x80000000u);
  return o;
}

template <int LP, int SA, int SB, int SC>
__global__ __launch_bounds__(256, 2) void k_mfma16(StepDesc d) {
  __shared__ __attribute__((aligned(16))) uint32_t lw[kLMainWords + 16];
  uint32_t* Abuf = lw;                  // [2][kTM][kLRow]
  uint32_t* Bbuf = lw + 2 * kLABuf;     // [2][kTN][kLRow]
  float* lds = reinterpret_cast<float*>(lw);
  float* red = lds + kLMainWords;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  uint64_t bid = blockIdx.x;
  const uint64_t nblk = gridDim.x;
  if ((nblk & 7) == 0) bid = (bid & 7) * (nblk >> 3) + (bid >> 3);
  const uint64_t no = bid % (uint64_t)d.n_col_tiles;
  const uint64_t ro = bid / (uint64_t)d.n_col_tiles;

  // A chunk tile: 128 rows x 32 k (4096 elements, 16 per thread); B chunk
  // tile: 32 k x 64 columns (2048, 8 per thread).
  int64_t gA[16];
  int lA[16];
  int64_t gB[8];
  int lB[8];
  {
    TileTab* ta = reinterpret_cast<TileTab*>(lds);
    TileTab* tb = ta + 1;
    build_tab(d.tA, kLRow, 0, 1, *ta);
    build_tab(d.tB, 0, kLRow, 1, *tb);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      gA[j] = ta->g[lane] + ta->g[64 + wave + 4 * j];
      lA[j] = ta->c[lane] + ta->c[64 + wave + 4 * j];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      gB[j] = tb->g[lane] + tb->g[64 + wave + 4 * j];
      lB[j] = tb->c[lane] + tb->c[64 + wave + 4 * j];
    }
  }
  int hb = 0;
  for (int b = 0; b < d.tC.nbits; ++b)
    if (d.tC.role[b] == 0 && d.tC.cbit[b] == 6) hb = b;
  const int64_t g_half = int64_t(1) << d.tC.gpos[hb];

  const int lrow = lane & 31;
  const int kq = (lane >> 5) * 4;      // first complex k of the lane's 8 real k
  const int ncol = (lane & 31) >> 1;
  const bool bswap = (lane & 1) != 0;  // C_r column parity 1: (im, re)

  const int n_kc = 1 << d.n_ko;
  for (int copy = blockIdx.y; copy < d.copies; copy += gridDim.y) {
    const int js = copy % d.gs_c, jb = copy / d.gs_c;
    int64_t oA, oB, oC;
    outer_offsets(d, ro, no, js, jb, oA, oB, oC);
    // Pre-scales of complex64 operands and the output scale.
    const float mA = d.maxA ? d.maxA[js * d.eA_s + jb * d.eA_b] : d.maxA_const;
    const float mB = d.maxB ? d.maxB[js * d.eB_s + jb * d.eB_b] : d.maxB_const;
    const int EA = mA > 0.f ? ceil_log2(mA) : 0, EB = mB > 0.f ? ceil_log2(mB) : 0;
    const int pA = (SA == LP || mA <= 0.f) ? 0 : 14 - EA;
    const int pB = (SB == LP || mB <= 0.f) ? 0 : 14 - EB;
    // A complex64 output keeps the operands' own scale (the pre-scales are
    // undone); a 16-bit output is scaled to the bound 2^15.
    Scale sc{pA + pB, 0};
    {
      const int eA = (d.track && d.expA) ? d.expA[js * d.eA_s + jb * d.eA_b] : 0;
      const int eB = (d.track && d.expB) ? d.expB[js * d.eB_s + jb * d.eB_b] : 0;
      sc.expC = eA + eB;
      if (d.track && d.lp_out && mA > 0.f && mB > 0.f && mA <= 3.0e38f && mB <= 3.0e38f) {
        const int t = d.k_total + 1 + (EA + pA) + (EB + pB) - 15 - d.bias;
        sc.shift = t;
        sc.expC = eA - pA + eB - pB + t;
      }
    }
    floatx16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    uint32_t ra[16], rb[8];
    {
      int64_t kA, kB;
      k_offsets(d, 0, kA, kB);
#pragma unroll
      for (int j = 0; j < 16; ++j) ra[j] = load_lp<LP, SA>(d.A, oA + kA + gA[j], pA);
#pragma unroll
      for (int j = 0; j < 8; ++j) rb[j] = load_lp<LP, SB>(d.B, oB + kB + gB[j], pB);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 16; ++j) Abuf[lA[j]] = ra[j];
#pragma unroll
    for (int j = 0; j < 8; ++j) Bbuf[lB[j]] = rb[j];
    __syncthreads();

    for (int kc = 0; kc < n_kc; ++kc) {
      const int cur = kc & 1;
      const bool more = kc + 1 < n_kc;
      if (more) {
        int64_t kA, kB;
        k_offsets(d, kc + 1, kA, kB);
#pragma unroll
        for (int j = 0; j < 16; ++j) ra[j] = load_lp<LP, SA>(d.A, oA + kA + gA[j], pA);
#pragma unroll
        for (int j = 0; j < 8; ++j) rb[j] = load_lp<LP, SB>(d.B, oB + kB + gB[j], pB);
      }
      const uint32_t* As = Abuf + cur * kLABuf + (wm * 64 + lrow) * kLRow + kq;
      const uint32_t* Bs = Bbuf + cur * kLBBuf + (wn * 32 + ncol) * kLRow + kq;
#pragma unroll
      for (int kk = 0; kk < kLTK / 8; ++kk) {
        const u32x4 a0 = *reinterpret_cast<const u32x4*>(As + kk * 8);
        const u32x4 a1 = *reinterpret_cast<const u32x4*>(As + 32 * kLRow + kk * 8);
        const u32x4 b0 = expand_b(*reinterpret_cast<const u32x4*>(Bs + kk * 8), bswap);
        const u32x4 b1 = expand_b(*reinterpret_cast<const u32x4*>(Bs + 16 * kLRow + kk * 8), bswap);
        acc[0][0] = mfma16<LP>(a0, b0, acc[0][0]);
        acc[0][1] = mfma16<LP>(a0, b1, acc[0][1]);
        acc[1][0] = mfma16<LP>(a1, b0, acc[1][0]);
        acc[1][1] = mfma16<LP>(a1, b1, acc[1][1]);
      }
      if (more) {
        uint32_t* An = Abuf + (cur ^ 1) * kLABuf;
        uint32_t* Bn = Bbuf + (cur ^ 1) * kLBBuf;
#pragma unroll
        for (int j = 0; j < 16; ++j) An[lA[j]] = ra[j];
#pragma unroll
        for (int j = 0; j < 8; ++j) Bn[lB[j]] = rb[j];
      }
      __syncthreads();
    }

    float* Cs = lds;
    TileTab* tcs = reinterpret_cast<TileTab*>(lds + kCHalf);
    build_tab_skip(d.tC, hb, kCStride, 2, *tcs);
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

template <int LP>
static hipError_t launch_mfma16(const StepDesc& d, int sa, int sb, int sc, dim3 grid,
                                hipStream_t s) {
  constexpr int C = ST_C64;
#define RQC_LP_CASE(a, b, c)                                                        \
  if (sa == a && sb == b && sc == c) {                                              \
    hipLaunchKernelGGL((k_mfma16<LP, a, b, c>), grid, dim3(256), 0, s, d);         \
    return hipGetLastError();                                                       \
  }
  RQC_LP_CASE(LP, LP, LP)
  RQC_LP_CASE(LP, LP, C)
  RQC_LP_CASE(LP, C, LP)
  RQC_LP_CASE(LP, C, C)
  RQC_LP_CASE(C, LP, LP)
  RQC_LP_CASE(C, LP, C)
  RQC_LP_CASE(C, C, LP)
  RQC_LP_CASE(C, C, C)
#undef RQC_LP_CASE
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Launch dispatch over storage types
// ---------------------------------------------------------------------------
#define RQC_SIMT_CASE(a, b, c)                                                         \
  if (sa == a && sb == b && sc == c) {                                                 \
    hipLaunchKernelGGL((k_simt<a, b, c>), grid, dim3(kSimtBlock), lds, s, d);         \
    e = hipGetLastError();                                                             \
    goto reduce;                                                                       \
  }
#define RQC_MFMA_CASE(a, b, c)                                                         \
  if (sa == a && sb == b && sc == c) {                                                 \
    hipLaunchKernelGGL((k_mfma32<a, b, c>), grid, dim3(256), 0, s, d);                \
    return hipGetLastError();                                                          \
  }

template <int KB>
static hipError_t launch_rows(const StepDesc& d, int sa, dim3 grid, hipStream_t s) {
  const int N = 1 << d.nt, R = 1 << d.rt, NC = 1 << d.ncb;
  const int ldc = NC == 1 ? 1 : NC + 1;
  if (R > 256 * rows_per_thread(KB) || N > 64 || d.ncb > d.nt || N * (1 << KB) > kRowsMaxB ||
      R * ldc > kRowsCs || d.rt + d.ncb > 11)
    return hipErrorInvalidValue;
  const size_t lds = sizeof(float2) * ((size_t)N * (1 << KB) + (size_t)R * ldc);
  if (sa == ST_F16) hipLaunchKernelGGL((k_rows<KB, ST_F16>), grid, dim3(256), lds, s, d);
  else if (sa == ST_BF16) hipLaunchKernelGGL((k_rows<KB, ST_BF16>), grid, dim3(256), lds, s, d);
  else hipLaunchKernelGGL((k_rows<KB, ST_C64>), grid, dim3(256), lds, s, d);
  return hipGetLastError();
}

hipError_t launch_step(const StepDesc& d0, int kernel, int sa, int sb, int sc, int lp_kind,
                       hipStream_t s) {
  StepDesc d = d0;
  d.sb_store = sb;
  d.sc_store = sc;
  const uint64_t tiles = (uint64_t)d.n_row_tiles * (uint64_t)d.n_col_tiles;
  const unsigned gy = (unsigned)(d.copies < 65535 ? d.copies : 65535);
  dim3 grid((unsigned)tiles, gy);
  hipError_t e = hipSuccess;
  if (kernel == KERN_MFMA16) {
    if (d.rt != 7 || d.nt != 6 || d.kt != 5) return hipErrorInvalidValue;
    if (lp_kind == ST_F16) return launch_mfma16<ST_F16>(d, sa, sb, sc, grid, s);
    if (lp_kind == ST_BF16) return launch_mfma16<ST_BF16>(d, sa, sb, sc, grid, s);
    return hipErrorInvalidValue;
  }
  if (kernel == KERN_MFMA) {
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
  if (kernel == KERN_ROWS) {
    switch (d.kt) {
      case 0: return launch_rows<0>(d, sa, grid, s);
      case 1: return launch_rows<1>(d, sa, grid, s);
      case 2: return launch_rows<2>(d, sa, grid, s);
      case 3: return launch_rows<3>(d, sa, grid, s);
      case 4: return launch_rows<4>(d, sa, grid, s);
      case 5: return launch_rows<5>(d, sa, grid, s);
    }
    return hipErrorInvalidValue;
  }
  {
    grid.x = (unsigned)(tiles << d.ksplit);
    const size_t lds = sizeof(float2) * ((size_t)(1 << d.rt) * ((1 << d.kt) + 1) +
                                         (size_t)(1 << d.kt) * ((1 << d.nt) + 1));
    RQC_SIMT_CASE(ST_C64, ST_C64, ST_C64)
    RQC_SIMT_CASE(ST_C64, ST_C64, ST_F16)
    RQC_SIMT_CASE(ST_C64, ST_C64, ST_BF16)
    RQC_SIMT_CASE(ST_F16, ST_C64, ST_F16)
    RQC_SIMT_CASE(ST_F16, ST_C64, ST_C64)
    RQC_SIMT_CASE(ST_BF16, ST_C64, ST_BF16)
    RQC_SIMT_CASE(ST_BF16, ST_C64, ST_C64)
    RQC_SIMT_CASE(ST_C64, ST_F16, ST_F16)
    RQC_SIMT_CASE(ST_C64, ST_F16, ST_C64)
    RQC_SIMT_CASE(ST_C64, ST_BF16, ST_BF16)
    RQC_SIMT_CASE(ST_C64, ST_BF16, ST_C64)
    RQC_SIMT_CASE(ST_F16, ST_F16, ST_F16)
    RQC_SIMT_CASE(ST_F16, ST_F16, ST_C64)
    RQC_SIMT_CASE(ST_BF16, ST_BF16, ST_BF16)
    RQC_SIMT_CASE(ST_BF16, ST_BF16, ST_C64)
    return hipErrorInvalidValue;
  }
reduce:
  if (e != hipSuccess || d.ksplit == 0) return e;
  grid.x = (unsigned)tiles;
  if (sc == ST_F16) hipLaunchKernelGGL(k_splitk_reduce<ST_F16>, grid, dim3(256), 0, s, d);
  else if (sc == ST_BF16) hipLaunchKernelGGL(k_splitk_reduce<ST_BF16>, grid, dim3(256), 0, s, d);
  else hipLaunchKernelGGL(k_splitk_reduce<ST_C64>, grid, dim3(256), 0, s, d);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Leaf instantiation: fix sliced wires to the bits of the slice id and closed
// selectors to the requested bits (Section 5.1), producing one copy per
// (slice, bitstring) of the group that the leaf depends on.
// ---------------------------------------------------------------------------
__global__ void k_leaves(const LeafJob* jobs, const float2* store, float2* dst,
                         const uint64_t* slice_ids, const uint8_t* closed, int n_closed, int gs,
                         int gb) {
  const LeafJob& J = jobs[blockIdx.x];
  const int ne = 1 << J.rank;
  const int cs = J.dep_s ? gs : 1;
  const int cb = J.dep_b ? gb : 1;
  const int total = ne * cs * cb;
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int e = t % ne;
    const int cp = t / ne;
    const int js = cp % cs, jb = cp / cs;
    int64_t src = J.src;
    for (int i = 0; i < J.rank; ++i)
      if ((e >> i) & 1) src += int64_t(1) << J.pos[i];
    for (int s = 0; s < J.nsel; ++s) {
      int v;
      if (J.sel_src[s] >= 0) v = (int)((slice_ids[js] >> J.sel_src[s]) & 1ull);
      else v = closed[(int64_t)jb * n_closed + (-J.sel_src[s] - 1)] & 1;
      if (v) src += int64_t(1) << J.sel_pos[s];
    }
    dst[J.dst + (int64_t)js * J.out_s + (int64_t)jb * J.out_b + e] = store[src];
  }
}

hipError_t launch_leaves(const LeafJob* jobs_dev, int n_jobs, const void* leaf_store,
                         void* dst_base, const uint64_t* slice_ids, const uint8_t* closed_bits,
                         int n_closed, int gs, int gb, int max_rank, hipStream_t s) {
  if (n_jobs <= 0) return hipSuccess;
  (void)max_rank;
  hipLaunchKernelGGL(k_leaves, dim3(n_jobs), dim3(256), 0, s, jobs_dev,
                     reinterpret_cast<const float2*>(leaf_store), reinterpret_cast<float2*>(dst_base),
                     slice_ids, closed_bits, n_closed, gs, gb);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Cross-slice sum in FP64, fixed order (slice 0, 1, ... of the group; groups
// in call order), skipping slices flagged for an FP32 re-run.
// ---------------------------------------------------------------------------
template <int S>
__global__ void k_slice_sum(const void* root, const int32_t* rexp, int64_t rs, int64_t rb,
                            int32_t res, int32_t reb, int n_elems, int gs, int gb, int dep_s,
                            int dep_b, const int32_t* flags, double* out, double* per_slice,
                            int64_t ps_row0, int64_t n_batch_total, int64_t b0, int first) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)n_elems * gb) return;
  const int e = (int)(t % n_elems);
  const int jb = (int)(t / n_elems);
  const int jbs = dep_b ? jb : 0;
  double sr = 0.0, si = 0.0;
  for (int js = 0; js < gs; ++js) {
    const int jss = dep_s ? js : 0;
    double vr = 0.0, vi = 0.0;
    if (!(flags && flags[js])) {
      const float2 v = load_c<S>(root, jss * rs + jbs * rb + e);
      const int ex = rexp ? rexp[jss * res + jbs * reb] : 0;
      vr = ldexp((double)v.x, ex);
      vi = ldexp((double)v.y, ex);
    }
    sr += vr;
    si += vi;
    if (per_slice && !(flags && flags[js])) {
      const int64_t o = (((ps_row0 + js) * n_batch_total + (b0 + jb)) * n_elems + e) * 2;
      per_slice[o] = vr;
      per_slice[o + 1] = vi;
    }
  }
  const int64_t o = ((b0 + jb) * (int64_t)n_elems + e) * 2;
  if (first) {
    out[o] = sr;
    out[o + 1] = si;
  } else {
    out[o] += sr;
    out[o + 1] += si;
  }
}

hipError_t launch_slice_sum(const void* root, int root_store, const int32_t* root_exp,
                            int64_t root_s, int64_t root_b, int32_t re_s, int32_t re_b, int dep_s,
                            int dep_b, int n_elems, int gs, int gb, const int32_t* flags,
                            double* out, double* per_slice, int64_t ps_row0,
                            int64_t n_batch_total, int64_t b0, int first, hipStream_t s) {
  const int64_t n = (int64_t)n_elems * gb;
  const dim3 grid((unsigned)((n + 255) / 256));
  if (root_store == ST_C64)
    hipLaunchKernelGGL(k_slice_sum<ST_C64>, grid, dim3(256), 0, s, root, root_exp, root_s, root_b,
                       re_s, re_b, n_elems, gs, gb, dep_s, dep_b, flags, out, per_slice, ps_row0,
                       n_batch_total, b0, first);
  else if (root_store == ST_F16)
    hipLaunchKernelGGL(k_slice_sum<ST_F16>, grid, dim3(256), 0, s, root, root_exp, root_s, root_b,
                       re_s, re_b, n_elems, gs, gb, dep_s, dep_b, flags, out, per_slice, ps_row0,
                       n_batch_total, b0, first);
  else
    hipLaunchKernelGGL(k_slice_sum<ST_BF16>, grid, dim3(256), 0, s, root, root_exp, root_s, root_b,
                       re_s, re_b, n_elems, gs, gb, dep_s, dep_b, flags, out, per_slice, ps_row0,
                       n_batch_total, b0, first);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Small utility kernels (fills instead of memsets so that graphs replay them)
// ---------------------------------------------------------------------------
__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_f64(double* p, double v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_add_f64(double* d, const double* s, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    d[i] += s[i];
}

static dim3 fill_grid(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return dim3((unsigned)b);
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, fill_grid(n), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}
hipError_t launch_fill_f64(double* p, double v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f64, fill_grid(n), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}
hipError_t launch_add_f64(double* dst, const double* src, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_add_f64, fill_grid(n), dim3(256), 0, s, dst, src, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Stand-alone bit permutation (the separate-permutation baseline): tiles of
// 2^5 x 2^5 elements staged through LDS so that both the reads (low input
// bits) and the writes (low output bits) are contiguous.
// ---------------------------------------------------------------------------
struct PermDesc {
  int32_t rank;
  int8_t src_of_out[48];  // input bit feeding output bit i
};

__global__ __launch_bounds__(256) void k_permute(const float2* in, float2* out, PermDesc p,
                                                 int lo_in, int lo_out, uint32_t lo_in_mask,
                                                 uint32_t lo_out_mask) {
  // Tile = the lowest `lo_in` input bits  U  the lowest `lo_out` output bits.
  __shared__ float2 tile[1024 + 32];
  (void)lo_in_mask;
  (void)lo_out_mask;
  const int r = p.rank;
  int out_of_in[48];
  for (int i = 0; i < r; ++i) out_of_in[p.src_of_out[i]] = i;
  // Tile bits, as output bit indices: the low output bits plus the output
  // bits fed by the low input bits.
  uint64_t tmask = 0;
  for (int i = 0; i < lo_out && i < r; ++i) tmask |= 1ull << i;
  for (int i = 0; i < lo_in && i < r; ++i) tmask |= 1ull << out_of_in[i];
  int tb[20], nt = 0;
  for (int i = 0; i < r; ++i)
    if ((tmask >> i) & 1) tb[nt++] = i;
  int ob[48], no = 0;
  for (int i = 0; i < r; ++i)
    if (!((tmask >> i) & 1)) ob[no++] = i;
  // Block base in output index space.
  uint64_t base_out = 0;
  for (int i = 0; i < no; ++i)
    if ((blockIdx.x >> i) & 1) base_out |= 1ull << ob[i];
  const int nte = 1 << nt;
  // Read phase: element t of the tile in input order (input bits ascending).
  int tin[20], nti = 0;
  {
    // tile bits sorted by their input bit
    int tmp_in[20];
    for (int i = 0; i < nt; ++i) tmp_in[i] = p.src_of_out[tb[i]];
    // selection sort by input bit
    for (int i = 0; i < nt; ++i) {
      int best = i;
      for (int j = i + 1; j < nt; ++j)
        if (tmp_in[j] < tmp_in[best]) best = j;
      int x = tmp_in[i]; tmp_in[i] = tmp_in[best]; tmp_in[best] = x;
    }
    for (int i = 0; i < nt; ++i) tin[nti++] = tmp_in[i];
  }
  uint64_t base_in = 0;
  for (int i = 0; i < r; ++i)
    if ((base_out >> i) & 1) base_in |= 1ull << p.src_of_out[i];
  for (int t = threadIdx.x; t < nte; t += blockDim.x) {
    uint64_t a = base_in;
    int slot = 0;
    for (int i = 0; i < nti; ++i)
      if ((t >> i) & 1) {
        a |= 1ull << tin[i];
        // slot index: position of the output bit inside tb[]
        const int ob_i = out_of_in[tin[i]];
        for (int j = 0; j < nt; ++j)
          if (tb[j] == ob_i) slot |= 1 << j;
      }
    tile[slot + (slot >> 5)] = in[a];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nte; t += blockDim.x) {
    uint64_t a = base_out;
    for (int j = 0; j < nt; ++j)
      if ((t >> j) & 1) a |= 1ull << tb[j];
    out[a] = tile[t + (t >> 5)];
  }
}

hipError_t launch_permute(const void* in, void* out, int rank, const int8_t* src_pos_of_out_bit,
                          hipStream_t s) {
  PermDesc p;
  p.rank = rank;
  for (int i = 0; i < rank; ++i) p.src_of_out[i] = src_pos_of_out_bit[i];
  // Up to 10 tile bits: 5 lowest input bits and 5 lowest output bits.
  int lo_in = rank < 5 ? rank : 5, lo_out = rank < 5 ? rank : 5;
  // Count tile bits (overlap shrinks the tile).
  uint64_t tmask = 0;
  int out_of_in[48];
  for (int i = 0; i < rank; ++i) out_of_in[(int)p.src_of_out[i]] = i;
  for (int i = 0; i < lo_out; ++i) tmask |= 1ull << i;
  for (int i = 0; i < lo_in; ++i) tmask |= 1ull << out_of_in[i];
  const int nt = __builtin_popcountll(tmask);
  const uint64_t blocks = 1ull << (rank - nt);
  hipLaunchKernelGGL(k_permute, dim3((unsigned)blocks), dim3(256), 0, s,
                     reinterpret_cast<const float2*>(in), reinterpret_cast<float2*>(out), p, lo_in,
                     lo_out, 0u, 0u);
  return hipGetLastError();
}

}  // namespace rqc

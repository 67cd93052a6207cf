// Generic table-driven SIMT contraction kernel and its split-K reduction.
#include <type_traits>

#include "kernels_dev.h"

namespace rqc {

// ---------------------------------------------------------------------------
// Generic SIMT contraction (any layouts, any sizes): tiles of R rows x N
// columns, K in chunks; loads follow each operand's address order through
// the offset tables; optional split-K into partial buffers.
// ---------------------------------------------------------------------------
constexpr int kSimtBlock = 256;
constexpr int kSimtMaxC = 8;  // C tile <= 2048 elements

// Loads elements tid + 256 i (i < 16, below n) of an operand tile, whose
// offsets come from the table, into the LDS tile at the table coordinates,
// in rounds of kSimtBatch loads that are all issued before any is written.
constexpr int kSimtBatch = 8;
template <int S>
__device__ __forceinline__ void simt_stage(const void* src, int64_t base, const TileTab& t,
                                           int c_lo, int n, int tid, float2* dst) {
  typedef typename std::conditional<S == ST_C64, uint2, uint32_t>::type Raw;
#pragma unroll
  for (int r = 0; r < 16; r += kSimtBatch) {
    if (tid + r * kSimtBlock >= n) break;
    Raw v[kSimtBatch];
    int at[kSimtBatch];
#pragma unroll
    for (int i = 0; i < kSimtBatch; ++i) {
      const int e = tid + (r + i) * kSimtBlock;
      if (e < n) {
        const int hi = 64 + (e >> 6);
        at[i] = c_lo + t.c[hi];
        v[i] = reinterpret_cast<const Raw*>(src)[base + t.g[hi]];
      }
    }
#pragma unroll
    for (int i = 0; i < kSimtBatch; ++i) {
      if (tid + (r + i) * kSimtBlock < n) {
        if constexpr (S == ST_C64) {
          dst[at[i]] = make_float2(__uint_as_float(v[i].x), __uint_as_float(v[i].y));
        } else if constexpr (S == ST_F16) {
          const h2 h = __builtin_bit_cast(h2, v[i]);
          dst[at[i]] = make_float2((float)h.x, (float)h.y);
        } else {
          const b2 h = __builtin_bit_cast(b2, v[i]);
          dst[at[i]] = make_float2((float)h.x, (float)h.y);
        }
      }
    }
  }
}

template <int SA, int SB, int SC>
__global__ __launch_bounds__(kSimtBlock) void k_simt(StepDesc d) {
  extern __shared__ float2 smem2[];
  __shared__ TileTab ta, tb, tcc;
  __shared__ float red[16];
  __shared__ float2 qsum[kSimtBlock];  // quarter sums of a tiny tile
  const int R = 1 << d.rt, N = 1 << d.nt, K = 1 << d.kt;
  const int ldA = K + 1, ldB = N + 1;
  float2* As = smem2;
  float2* Bs = As + R * ldA;
  const int tid = threadIdx.x, lane = tid & 63;
  __shared__ TileMap maps[3];
  __shared__ OuterTab ot;
  stage_maps(d, maps);
  build_outer(d, ot);
  __syncthreads();
  build_tab(maps[0], ldA, 0, 1, ta);
  build_tab(maps[1], 0, 1, ldB, tb);
  build_tab(maps[2], 4096, 1, 0, tcc);  // coordinate = row * 4096 + col
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
  // Tiny tiles (at most 64 outputs, as in the long sums of the last steps):
  // the four waves take one quarter of each K chunk each, so that every
  // thread multiplies, and the quarters are added in order at the end.
  const bool quarters = nC <= 64 && K >= 4;
  const int qk = K >> 2, q = tid >> 6;
  // Blocked form of the tiny tiles: 4 x 4 output blocks per thread, the
  // sum split over 256 / blocks parts; a thread reads 8 LDS values per 16
  // products instead of 2 per 1 (the tile loop is bound by LDS reads).  The
  // parts are added in part order at the end through the operand buffers.
  const int nbr = R >> 2, nbc = N >> 2, nblk = nbr * nbc;
  const bool blocked = quarters && (R & 3) == 0 && (N & 3) == 0 && nblk > 0 &&
                       K >= kSimtBlock / nblk && R * ldA + K * ldB >= 16 * kSimtBlock;
  const int parts = blocked ? kSimtBlock / nblk : 1;
  const int kpart = blocked ? K / parts : 0;
  const int blk = tid % (blocked ? nblk : 1), part = tid / (blocked ? nblk : 1);
  const int br0 = (blk / (nbc > 0 ? nbc : 1)) * 4, bc0 = (blk % (nbc > 0 ? nbc : 1)) * 4;
  int qrow = 0, qcol = 0;
  int64_t qg = 0;
  if (quarters) {
    const int c = clo + tcc.c[64];
    qrow = c >> 12;
    qcol = c & 4095;
    qg = glo + tcc.g[64];
  }
  for (int copy = blockIdx.y; copy < d.copies; copy += gridDim.y) {
    const int js = copy % d.gs_c, jb = copy / d.gs_c;
    int64_t oA, oB, oC;
    outer_offsets(d, ot, ro, no, js, jb, oA, oB, oC);
    float2 acc[kSimtMaxC];
#pragma unroll
    for (int i = 0; i < kSimtMaxC; ++i) acc[i] = make_float2(0.f, 0.f);
    float bx[4][4], by[4][4];  // blocked form: the thread's 4 x 4 outputs
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) bx[i][j] = by[i][j] = 0.f;
    for (int kc = kc0; kc < kc0 + n_kc; ++kc) {
      int64_t kA, kB;
      k_offsets(d, ot, kc, kA, kB);
      // Up to 16 elements of each operand per thread (tiles hold at most
      // 4096): all loads of an operand are issued, as raw stored words,
      // before any is converted and written.
      simt_stage<SA>(d.A, oA + kA + gAlo, ta, cAlo, nA, tid, As);
      simt_stage<SB>(d.B, oB + kB + gBlo, tb, cBlo, nB, tid, Bs);
      __syncthreads();
      if (blocked) {
        const float2* ar = As + br0 * ldA + part * kpart;
        const float2* bc = Bs + bc0 + part * kpart * ldB;
        for (int k = 0; k < kpart; ++k) {
          float2 a[4], b[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) a[i] = ar[i * ldA + k];
#pragma unroll
          for (int j = 0; j < 4; ++j) b[j] = bc[k * ldB + j];
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              bx[i][j] = fmaf(a[i].x, b[j].x, bx[i][j]);
              bx[i][j] = fmaf(-a[i].y, b[j].y, bx[i][j]);
              by[i][j] = fmaf(a[i].x, b[j].y, by[i][j]);
              by[i][j] = fmaf(a[i].y, b[j].x, by[i][j]);
            }
        }
        __syncthreads();
        continue;
      }
      if (quarters) {
        if (lane < nC) {
          const float2* ar = As + qrow * ldA + q * qk;
          const float2* bc = Bs + qcol + q * qk * ldB;
          float sx = acc[0].x, sy = acc[0].y;
          for (int k = 0; k < qk; ++k) {
            const float2 a = ar[k], b = bc[k * ldB];
            sx = fmaf(a.x, b.x, sx);
            sx = fmaf(-a.y, b.y, sx);
            sy = fmaf(a.x, b.y, sy);
            sy = fmaf(a.y, b.x, sy);
          }
          acc[0] = make_float2(sx, sy);
        }
        __syncthreads();
        continue;
      }
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
    if (blocked) {
      // Partials of thread (part, block) at [part][block][16] in the operand
      // buffers (free after the last chunk); output (qrow, qcol) of lane
      // `lane` of wave 0 = their sum over the parts, in part order.
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          smem2[(part * nblk + blk) * 16 + i * 4 + j] = make_float2(bx[i][j], by[i][j]);
      __syncthreads();
      if (q == 0 && lane < nC) {
        const int ob = (qrow >> 2) * nbc + (qcol >> 2), os = (qrow & 3) * 4 + (qcol & 3);
        float sx = 0.f, sy = 0.f;
        for (int pp = 0; pp < parts; ++pp) {
          const float2 v = smem2[(pp * nblk + ob) * 16 + os];
          sx += v.x;
          sy += v.y;
        }
        acc[0] = make_float2(sx, sy);
      }
      __syncthreads();
    } else if (quarters) {
      // Output lane of wave 0 = sum of the four quarters, in wave order.
      qsum[tid] = acc[0];
      __syncthreads();
      if (q == 0 && lane < nC) {
        float sx = 0.f, sy = 0.f;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          sx += qsum[w * 64 + lane].x;
          sy += qsum[w * 64 + lane].y;
        }
        acc[0] = make_float2(sx, sy);
      }
      __syncthreads();
    }
    if (quarters) {
      if (d.ksplit) {
        if (q == 0 && lane < nC) d.P[(int64_t)split * d.p_stride + oC + qg] = acc[0];
        continue;
      }
      const Scale sc = compute_scale(d, js, jb);
      float lmax = 0.f;
      int bad = 0;
      if (q == 0 && lane < nC) store_out<SC>(d, oC + qg, acc[0], sc, lmax, bad);
      finish_scale<kSimtBlock>(d, js, jb, lmax, bad, red, ro == 0 && no == 0, sc);
      continue;
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
  __shared__ TileMap maps[3];
  stage_maps(d, maps);
  __syncthreads();
  build_tab(maps[2], 0, 0, 0, tcc);
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
// Streaming dot products for tiny outputs with long contiguous sums (the last
// steps of an amplitude contraction: up to 8 x 8 outputs, 2^18 summed terms):
// the summed indices are the lowest address bits of A and B, in the same
// order, so every row of A and every column of B is a contiguous run of K
// complex values.  Each thread reads two consecutive complex64 values (four
// packed 16-bit pairs) of every row and column per 16-byte load (consecutive
// lanes, consecutive values) straight into registers and keeps all 2^LOGN
// outputs in registers, accumulating in FP32; no LDS staging.  Workgroup `split` of a copy sums its K range; the 64 lanes of a
// wave are combined by recursive halving (each exchange step halves the
// outputs a lane holds, so lane l ends with output l), the four waves in wave
// order, and the partial goes to the split-K buffer, summed by
// k_splitk_reduce in split order: the result does not depend on scheduling.
// ---------------------------------------------------------------------------
template <int S>
__device__ __forceinline__ float2 word_c(uint32_t w) {
  if constexpr (S == ST_F16) {
    const h2 h = __builtin_bit_cast(h2, w);
    return make_float2((float)h.x, (float)h.y);
  } else {
    const b2 h = __builtin_bit_cast(b2, w);
    return make_float2((float)h.x, (float)h.y);
  }
}

template <int RT, int NT, int S>
__global__ __launch_bounds__(kSimtBlock) void k_dot(StepDesc d) {
  constexpr int M = 1 << RT, N = 1 << NT, LOGN = RT + NT, NOUT = M * N;
  constexpr int G = S == ST_C64 ? 2 : 4;  // complex values per 16-byte load
  constexpr int EB = S == ST_C64 ? 8 : 4;  // bytes per complex value
  __shared__ int64_t coff[NOUT];
  __shared__ float2 wsum[kSimtBlock / 64][NOUT];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < NOUT; i += kSimtBlock) {
    int64_t c = 0;  // C offset of output i = r * N + n
    for (int x = 0; x < d.tC.nbits; ++x) {
      const int v = d.tC.role[x] == 0 ? i / N : i % N;
      if ((v >> d.tC.cbit[x]) & 1) c += int64_t(1) << d.tC.gpos[x];
    }
    coff[i] = c;
  }
  // Offsets of the rows of A and the columns of B (the same in every
  // thread, so the compiler keeps them in scalar registers).
  int64_t arow[M], bcol[N];
#pragma unroll
  for (int i = 0; i < M; ++i) {
    arow[i] = 0;
    for (int x = 0; x < d.tA.nbits; ++x)
      if (d.tA.role[x] == 0 && ((i >> d.tA.cbit[x]) & 1)) arow[i] += int64_t(1) << d.tA.gpos[x];
  }
#pragma unroll
  for (int j = 0; j < N; ++j) {
    bcol[j] = 0;
    for (int x = 0; x < d.tB.nbits; ++x)
      if (d.tB.role[x] == 1 && ((j >> d.tB.cbit[x]) & 1)) bcol[j] += int64_t(1) << d.tB.gpos[x];
  }
  __syncthreads();
  const int64_t Ks = int64_t(1) << (d.k_total - d.ksplit);
  const int64_t k0 = (int64_t)blockIdx.x * Ks;
  typedef float f4v __attribute__((ext_vector_type(4)));
  typedef unsigned int u4v __attribute__((ext_vector_type(4)));
  for (int copy = blockIdx.y; copy < d.copies; copy += gridDim.y) {
    const int js = copy % d.gs_c, jb = copy / d.gs_c;
    const int64_t oA = js * d.sA_s + jb * d.sA_b, oB = js * d.sB_s + jb * d.sB_b;
    const int64_t oC = js * d.sC_s + jb * d.sC_b;
    // Row i of A from summed index k0 on, in 16-byte groups of G values.
    const u4v* pa[M];
    const u4v* pb[N];
#pragma unroll
    for (int i = 0; i < M; ++i)
      pa[i] = reinterpret_cast<const u4v*>(static_cast<const char*>(d.A) + EB * (oA + arow[i] + k0));
#pragma unroll
    for (int j = 0; j < N; ++j)
      pb[j] = reinterpret_cast<const u4v*>(static_cast<const char*>(d.B) + EB * (oB + bcol[j] + k0));
    float ax[NOUT], ay[NOUT];
#pragma unroll
    for (int o = 0; o < NOUT; ++o) ax[o] = ay[o] = 0.f;
    const int ngroup = (int)(Ks / G);
    for (int p = tid; p < ngroup; p += kSimtBlock) {
      u4v a[M], b[N];
#pragma unroll
      for (int i = 0; i < M; ++i) a[i] = pa[i][p];
#pragma unroll
      for (int j = 0; j < N; ++j) b[j] = pb[j][p];
      if constexpr (S == ST_C64) {
#pragma unroll
        for (int o = 0; o < NOUT; ++o) {
          const f4v x = __builtin_bit_cast(f4v, a[o / N]);
          const f4v y = __builtin_bit_cast(f4v, b[o % N]);
          ax[o] += x[0] * y[0] - x[1] * y[1] + x[2] * y[2] - x[3] * y[3];
          ay[o] += x[0] * y[1] + x[1] * y[0] + x[2] * y[3] + x[3] * y[2];
        }
      } else {
        float2 bf[N][4];
#pragma unroll
        for (int j = 0; j < N; ++j)
#pragma unroll
          for (int q = 0; q < 4; ++q) bf[j][q] = word_c<S>(b[j][q]);
#pragma unroll
        for (int i = 0; i < M; ++i) {
          float2 af[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) af[q] = word_c<S>(a[i][q]);
#pragma unroll
          for (int j = 0; j < N; ++j) {
            const int o = i * N + j;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              ax[o] += af[q].x * bf[j][q].x - af[q].y * bf[j][q].y;
              ay[o] += af[q].x * bf[j][q].y + af[q].y * bf[j][q].x;
            }
          }
        }
      }
    }
    // Recursive halving over the wave: at offset s a lane keeps the lower
    // or upper half of its outputs ((lane & s) set: upper) and adds the
    // partner's copy of that half.
    // The step counter t is the unrolled induction variable, so every count
    // and index below is a compile-time constant (a run-time index would put
    // the output arrays in scratch memory).
#pragma unroll
    for (int t = 0; t < 6; ++t) {
      const int s = 32 >> t;
      const int c = NOUT >> t;  // outputs a lane holds before this step
      if (c > 1) {
        const int h = c >> 1;
        const bool up = (lane & s) != 0;
#pragma unroll
        for (int o = 0; o < NOUT / 2; ++o) {
          if (o < h) {
            const float sx = up ? ax[o] : ax[o + h], sy = up ? ay[o] : ay[o + h];
            const float kx = up ? ax[o + h] : ax[o], ky = up ? ay[o + h] : ay[o];
            ax[o] = kx + __shfl_xor(sx, s, 64);
            ay[o] = ky + __shfl_xor(sy, s, 64);
          }
        }
      } else {
        ax[0] += __shfl_xor(ax[0], s, 64);
        ay[0] += __shfl_xor(ay[0], s, 64);
      }
    }
    // Lane l holds output l >> (6 - LOGN).
    if ((lane & ((64 >> LOGN) - 1)) == 0) wsum[wave][lane >> (6 - LOGN)] = make_float2(ax[0], ay[0]);
    __syncthreads();
    if (tid < NOUT) {
      float sx = 0.f, sy = 0.f;
#pragma unroll
      for (int w = 0; w < kSimtBlock / 64; ++w) {
        sx += wsum[w][tid].x;
        sy += wsum[w][tid].y;
      }
      d.P[(int64_t)blockIdx.x * d.p_stride + oC + coff[tid]] = make_float2(sx, sy);
    }
    __syncthreads();
  }
}

// Whether a step fits k_dot: one output tile of at most 8 x 8 elements,
// split K, operands in one storage type (complex64, or both FP16 or both
// BF16) whose summed indices are the lowest address bits of both, in the
// same order, and at least 64 summed values per split.
static bool dot_fits(const StepDesc& d, int sa, int sb, uint64_t tiles) {
  if (tiles != 1 || d.ksplit == 0 || sa != sb) return false;
  if (d.rt > 3 || d.nt > 3 || d.k_total - d.ksplit < 6 || d.n_ro != 0 || d.n_no != 0) return false;
  for (const TileMap* t : {&d.tA, &d.tB})
    for (int x = 0; x < t->nbits; ++x)
      if (t->role[x] == 2 && t->gpos[x] != t->cbit[x]) return false;
  for (int i = 0; i < d.n_ko; ++i)
    if (d.ko_A[i] != d.kt + i || d.ko_B[i] != d.kt + i) return false;
  return true;
}

template <int RT, int S>
static void launch_dot_rt(const StepDesc& d, dim3 grid, hipStream_t s) {
  switch (d.nt) {
    case 0: hipLaunchKernelGGL((k_dot<RT, 0, S>), grid, dim3(kSimtBlock), 0, s, d); break;
    case 1: hipLaunchKernelGGL((k_dot<RT, 1, S>), grid, dim3(kSimtBlock), 0, s, d); break;
    case 2: hipLaunchKernelGGL((k_dot<RT, 2, S>), grid, dim3(kSimtBlock), 0, s, d); break;
    default: hipLaunchKernelGGL((k_dot<RT, 3, S>), grid, dim3(kSimtBlock), 0, s, d); break;
  }
}

template <int S>
static void launch_dot_s(const StepDesc& d, dim3 grid, hipStream_t s) {
  switch (d.rt) {
    case 0: launch_dot_rt<0, S>(d, grid, s); break;
    case 1: launch_dot_rt<1, S>(d, grid, s); break;
    case 2: launch_dot_rt<2, S>(d, grid, s); break;
    default: launch_dot_rt<3, S>(d, grid, s); break;
  }
}

static void launch_dot(const StepDesc& d, int sa, dim3 grid, hipStream_t s) {
  if (sa == ST_F16) launch_dot_s<ST_F16>(d, grid, s);
  else if (sa == ST_BF16) launch_dot_s<ST_BF16>(d, grid, s);
  else launch_dot_s<ST_C64>(d, grid, s);
}

#define RQC_SIMT_CASE(a, b, c)                                                         \
  if (sa == a && sb == b && sc == c) {                                                 \
    hipLaunchKernelGGL((k_simt<a, b, c>), grid, dim3(kSimtBlock), lds, s, d);         \
    e = hipGetLastError();                                                             \
    goto reduce;                                                                       \
  }

hipError_t launch_simt_kernel(const StepDesc& d, int sa, int sb, int sc, uint64_t tiles,
                              hipStream_t s) {
  // Operand tiles of at most 4096 elements (16 per thread) and C tiles of
  // at most 2048 (kSimtMaxC per thread).
  if (d.rt + d.kt > 12 || d.kt + d.nt > 12 || d.rt + d.nt > 11) return hipErrorInvalidValue;
  const unsigned gy = (unsigned)(d.copies < 65535 ? d.copies : 65535);
  dim3 grid((unsigned)(tiles << d.ksplit), gy);
  hipError_t e = hipSuccess;
  if (dot_fits(d, sa, sb, tiles)) {
    launch_dot(d, sa, grid, s);
    e = hipGetLastError();
    goto reduce;
  }
  {
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
#undef RQC_SIMT_CASE

}  // namespace rqc

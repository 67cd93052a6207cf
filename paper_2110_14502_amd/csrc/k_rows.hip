// Row-streaming contraction kernel (HBM-bound steps with a small B).
#include "kernels_dev.h"

namespace rqc {

// ---------------------------------------------------------------------------
// Row-streaming contraction for plan steps (the memory-bound "stem" steps of
// Section 5.4's imbalanced case): A is a row-major [M][K] matrix whose K
// summed bits are its lowest address bits, B is [N][K] with the same K order
// and small.  The products run on the FP32 matrix cores
// (v_mfma_f32_16x16x4_f32, 16 rows x 8 complex columns per tile) so that the
// vector units only move data.
//
// A row of K complex values is 2K contiguous floats.  Lane l of a wave owns
// row (l mod 16) of a 16-row block and the l/16-th quarter of that row, read
// as one vector load; MFMA j takes float j of every lane's quarter, i.e. the
// real summation indices are dealt out quarter by quarter, and the lane's B
// operand holds the matching entries of the real 2x2 expansion of B
//   B_r[2k][2n] = Br  B_r[2k][2n+1] = Bi  B_r[2k+1][2n] = -Bi  B_r[2k+1][2n+1] = Br.
// The sum is over the same indices, in another order.  Each wave handles 64
// rows (four 16-row blocks), a workgroup 256; output columns go 8 at a time
// through an LDS tile written out in C's own address order.
//
// When A is stored in FP16 / BF16 and a K chunk holds 16 or 32 complex
// values, the products run on the 16-bit matrix cores instead
// (v_mfma_f32_16x16x32_{f16,bf16}, FP32 accumulation): each MFMA takes 8
// consecutive real k of a lane's quarter, which are the raw stored words,
// and B is staged once per copy as packed 16-bit words (pre-scaled by a
// power of two when it is stored in complex64, as in the 16-bit GEMM).
// ---------------------------------------------------------------------------
constexpr int kRowsMaxB = 4096;  // N*K
constexpr int kRowsRows = 256;   // rows per workgroup
constexpr int kRowsLdc = 17;     // floats per staged row: 16 real columns + 1
constexpr uint64_t kRowsGrid = 256 * 16;  // persistent workgroups (16 per CU)

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4r __attribute__((ext_vector_type(4)));
typedef _Float16 halfx8r __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8r __attribute__((ext_vector_type(8)));

template <int S>
__device__ __forceinline__ floatx4 mfma_lp16(u32x4r a, u32x4r b, floatx4 c) {
  if constexpr (S == ST_F16)
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(halfx8r, a),
                                                  __builtin_bit_cast(halfx8r, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8r, a),
                                                   __builtin_bit_cast(bf16x8r, b), c, 0, 0, 0);
}

template <int S>
__device__ __forceinline__ uint32_t pack_word(float2 v) {
  if constexpr (S == ST_F16) {
    h2 o;
    o.x = (_Float16)v.x;
    o.y = (_Float16)v.y;
    return __builtin_bit_cast(uint32_t, o);
  } else {
    b2 o;
    o.x = (__bf16)v.x;
    o.y = (__bf16)v.y;
    return __builtin_bit_cast(uint32_t, o);
  }
}

// Raw words of this lane's quarter of a row of K complex values: floats
// [g*NJ, g*NJ + NJ) (NJ = 2K/4), or for K <= 2 the complex value holding
// float g.  Kept raw while in flight and converted only when multiplied, so
// that a prefetch does not wait for its data.  Rows start at multiples of K
// elements, so vector loads are aligned.
template <int S, int K, int NJ>
struct RawRow {
  static constexpr int W = S == ST_C64 ? (K <= 2 ? 2 : NJ) : (K <= 2 ? 1 : NJ / 2);
  uint32_t w[W];
};

template <int S, int K, int NJ>
__device__ __forceinline__ void load_raw(const void* p, int64_t row, int g, RawRow<S, K, NJ>& r) {
  if (K <= 2) {
    const int64_t at = row + (K == 2 ? (g >> 1) : 0);
    if (K == 1 && g >= 2) {
#pragma unroll
      for (int i = 0; i < RawRow<S, K, NJ>::W; ++i) r.w[i] = 0u;
      return;
    }
    if (S == ST_C64) {
      const uint2 v = reinterpret_cast<const uint2*>(p)[at];
      r.w[0] = v.x;
      r.w[RawRow<S, K, NJ>::W - 1] = v.y;
    } else {
      r.w[0] = reinterpret_cast<const uint32_t*>(p)[at];
    }
    return;
  }
  constexpr int W = RawRow<S, K, NJ>::W;
  const uint32_t* q = reinterpret_cast<const uint32_t*>(p) + (S == ST_C64 ? 2 * row : row) + g * W;
  if (W == 1) {
    r.w[0] = q[0];
  } else if (W == 2) {
    const uint2 v = *reinterpret_cast<const uint2*>(q);
    r.w[0] = v.x;
    r.w[1] = v.y;
  } else {
#pragma unroll
    for (int i = 0; i < W; i += 4) {
      const uint4 v = *reinterpret_cast<const uint4*>(q + i);
      r.w[i] = v.x;
      r.w[i + 1] = v.y;
      r.w[i + 2] = v.z;
      r.w[i + 3] = v.w;
    }
  }
}

template <int S>
__device__ __forceinline__ float2 unpack_word(uint32_t w) {
  if (S == ST_F16) {
    const h2 h = __builtin_bit_cast(h2, w);
    return make_float2((float)h.x, (float)h.y);
  }
  const b2 h = __builtin_bit_cast(b2, w);
  return make_float2((float)h.x, (float)h.y);
}

template <int S, int K, int NJ>
__device__ __forceinline__ void unpack_raw(const RawRow<S, K, NJ>& r, int g, float (&out)[NJ]) {
  if (K <= 2) {
    if (S == ST_C64) {
      // A select between the two words by value: written as (g & 1) ? w[1] :
      // w[0] it is turned into an indexed load, which puts the rows in
      // scratch memory.
      const uint32_t m = 0u - (uint32_t)(g & 1);
      out[0] = __uint_as_float(r.w[0] ^ ((r.w[0] ^ r.w[1]) & m));
    } else {
      const float2 c = unpack_word<S>(r.w[0]);
      out[0] = (g & 1) ? c.y : c.x;
    }
    return;
  }
  if (S == ST_C64) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) out[j] = __uint_as_float(r.w[j]);
  } else {
#pragma unroll
    for (int i = 0; i < NJ / 2; ++i) {
      const float2 c = unpack_word<S>(r.w[i]);
      out[2 * i] = c.x;
      out[2 * i + 1] = c.y;
    }
  }
}

// This lane's raw quarters of its four rows of a 256-row tile, K chunk kc.
// Rows past the tile's R read row R-1 instead (their products are never
// staged): with no load under a per-lane condition the prefetch's wait
// counts stay exact, so multiplying a chunk does not wait for the next one.
template <int SA, int K, int NJ>
__device__ __forceinline__ void load_tile_rows(const StepDesc& d, int64_t oA, int KT, int kc,
                                               int R, int wave, int lc, int g,
                                               RawRow<SA, K, NJ> (&dst)[4]) {
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    const int r0 = wave * 64 + rb * 16 + lc;
    const int r = r0 < R ? r0 : R - 1;
    load_raw<SA, K, NJ>(d.A, oA + (int64_t)r * KT + kc * K, g, dst[rb]);
  }
}

// Persistent: each workgroup walks a contiguous range of tiles (256 rows of
// one copy each, copies one after the other).  The offset tables are built
// once; B, its scale
// and the running max-abs change only with the copy; the rows of the next
// tile (or K chunk) are loaded while the current one is multiplied and
// written.  KB: bits of one K chunk (the whole sum when k <= 4); NCH: chunks
// of 8 complex output columns, whose accumulators stay in registers.  Wider
// outputs (up to 128 columns, sums of at most 16) are walked in groups of
// NCH chunks with the tile's rows held in registers, so that an
// output-heavy step streams its output at the same register cost.
template <int KB, int NCH, int SA, bool ALLOW16>
__global__ __launch_bounds__(256) void k_rows(StepDesc d) {
  constexpr int K = 1 << KB;
  constexpr int NJ = K >= 2 ? (2 * K) / 4 : 1;  // real k per lane quarter (FP32 MFMAs per chunk)
  constexpr bool LPM = ALLOW16 && SA != ST_C64 && KB >= 4;  // 16-bit matrix cores
  extern __shared__ __attribute__((aligned(16))) float2 rows_lds[];  // 16-byte B reads
  __shared__ TileTab tc;
  __shared__ int64_t bofs[128];  // B offset of output column n (N <= 128)
  __shared__ int64_t stepA[kMaxOuter], stepC[kMaxOuter];
  __shared__ int64_t gch_tab[16];  // C offset of column chunk h
  __shared__ float red[16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, lc = lane & 15;
  const int N = 1 << d.nt, R = 1 << d.rt, NC = 1 << d.ncb;
  const int KT = 1 << d.kt, nkc = 1 << (d.kt - KB);
  const int nch_all = N / NC;                          // column chunks of NC columns
  const int ncg = nch_all > NCH ? nch_all / NCH : 1;   // groups of NCH (nkc == 1 when > 1)
  // Row tile ro -> ro + 1 sets the lowest zero bit b of ro and clears the
  // bits below it: the offsets move by stepA[b] / stepC[b].
  for (int b = tid; b < d.n_ro; b += 256) {
    int64_t sa = int64_t(1) << d.ro_A[b], sc = int64_t(1) << d.ro_C[b];
    for (int j = 0; j < b; ++j) {
      sa -= int64_t(1) << d.ro_A[j];
      sc -= int64_t(1) << d.ro_C[j];
    }
    stepA[b] = sa;
    stepC[b] = sc;
  }
  if (tid < nch_all) {
    int64_t g = 0;
    for (int j = 0; j < d.nt - d.ncb; ++j)
      if ((tid >> j) & 1) g += int64_t(1) << d.nh_C[j];
    gch_tab[tid] = g;
  }
  float2* Bs = rows_lds;                                    // [N][KT], columns in C's bit order
  float* Cs = reinterpret_cast<float*>(rows_lds + N * KT);  // [R][kRowsLdc]
  build_tab(d.tC, kRowsLdc, 2, 0, tc);  // coordinates in floats
  for (int n = tid; n < N; n += 256) {
    int64_t o = 0;
    for (int b = 0; b < d.tB.nbits; ++b)
      if ((n >> b) & 1) o += int64_t(1) << d.tB.gpos[b];
    bofs[n] = o;
  }
  const uint64_t n_rt = (uint64_t)d.n_row_tiles;  // 2^n_ro
  const uint64_t rmask = n_rt - 1;
  const int rsh = d.n_ro;
  const uint64_t n_tiles = n_rt * (uint64_t)d.copies;
  const int nC = R * NC;
  const uint64_t per = (n_tiles + gridDim.x - 1) / gridDim.x;
  uint64_t t = (uint64_t)blockIdx.x * per;
  const uint64_t t_end = t + per < n_tiles ? t + per : n_tiles;
  RawRow<SA, K, NJ> a[4], an[4];
  if (t < t_end) {
    const int copy = (int)(t >> rsh);
    int64_t oA, oB, oC;
    outer_offsets(d, t & rmask, 0, copy % d.gs_c, copy / d.gs_c, oA, oB, oC);
    load_tile_rows<SA, K, NJ>(d, oA, KT, 0, R, wave, lc, g, a);
  }
  // Wait for the first tile's rows here (s_waitcnt vmcnt(0)): entering the
  // tile loop with those loads pending, the compiler's wait counting merges
  // them with the loop's own prefetch and waits for the prefetch too, in
  // every chunk.
  __builtin_amdgcn_s_waitcnt(0x0F70);
  int cur = -1, cjs = 0, cjb = 0;
  bool wexp = false;
  Scale sc{0, 0};
  float lmax = 0.f;
  int bad = 0;
  __syncthreads();  // tables ready
  const int64_t glo = tc.g[lane];
  const int32_t clo = tc.c[lane];
  // Vector stores: this thread's four consecutive low elements (the same
  // for every group it stores).
  const int lo4 = (tid & 15) << 2;
  const int64_t glo4 = tc.g[lo4];
  int32_t clo4[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) clo4[i] = tc.c[lo4 + i];
  int64_t oA = 0, oB = 0, oC = 0;
  for (; t < t_end; ++t) {
    const uint64_t ro = t & rmask;
    const int copy = (int)(t >> rsh);
    const int js = copy % d.gs_c, jb = copy / d.gs_c;
    if (copy != cur || ro == 0) {
      outer_offsets(d, ro, 0, js, jb, oA, oB, oC);
    } else {
      const int b = __builtin_ctzll(~(ro - 1));
      oA += stepA[b];
      oC += stepC[b];
    }
    if (copy != cur) {
      if (cur >= 0) finish_scale<256>(d, cjs, cjb, lmax, bad, red, wexp, sc);
      lmax = 0.f;
      bad = 0;
      wexp = false;
      __syncthreads();
      // 16-bit path: B complex64 is pre-scaled so that its max-abs is below
      // 2^15; the accumulator then carries 2^pB, which the output shift
      // removes (the stored exponent is unchanged).
      int pB = 0;
      if (LPM && d.sb_store == ST_C64) {
        const float mB = max_abs_of(d.maxB, js * d.eB_s + jb * d.eB_b, d.maxB_const);
        if (mB > 0.f && mB <= 3.0e38f) pB = 14 - ceil_log2(mB);
      }
      for (int i = tid; i < N * KT; i += 256) {
        const int64_t at = oB + bofs[i >> d.kt] + (i & (KT - 1));
        float2 v;
        if (d.sb_store == ST_F16) v = load_c<ST_F16>(d.B, at);
        else if (d.sb_store == ST_BF16) v = load_c<ST_BF16>(d.B, at);
        else v = load_c<ST_C64>(d.B, at);
        if (LPM) {
          if (pB) {
            v.x = ldexpf(v.x, pB);
            v.y = ldexpf(v.y, pB);
          }
          reinterpret_cast<uint32_t*>(Bs)[i] = pack_word<LPM ? SA : ST_F16>(v);
        } else {
          Bs[i] = v;
        }
      }
      sc = compute_scale(d, js, jb);
      sc.shift += pB;
      cur = copy;
      cjs = js;
      cjb = jb;
      __syncthreads();
    }
    wexp = wexp || ro == 0;
    for (int cg = 0; cg < ncg; ++cg) {
      const bool last_cg = cg + 1 == ncg;
      floatx4 acc[4][NCH];
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int h = 0; h < NCH; ++h) acc[rb][h] = floatx4{0.f, 0.f, 0.f, 0.f};
      for (int kc = 0; kc < nkc; ++kc) {
        // Prefetch the next K chunk, or the first chunk of the next tile; the
        // registers are handed over only after this chunk (or, for the next
        // tile, at its end), so the loads stay in flight meanwhile.
        if (kc + 1 < nkc) {
          load_tile_rows<SA, K, NJ>(d, oA, KT, kc + 1, R, wave, lc, g, an);
        } else if (last_cg && t + 1 < t_end) {
          const uint64_t tn = t + 1;
          int64_t pA;
          if ((tn & rmask) != 0) {
            pA = oA + stepA[__builtin_ctzll(~ro)];
          } else {
            const int cn = (int)(tn >> rsh);
            int64_t pB, pC;
            outer_offsets(d, 0, 0, cn % d.gs_c, cn / d.gs_c, pA, pB, pC);
          }
          load_tile_rows<SA, K, NJ>(d, pA, KT, 0, R, wave, lc, g, an);
        }
        if constexpr (LPM) {
          // MFMA j takes real k g*NJ + 8j .. +7 of every lane quarter: the raw
          // words 4j .. 4j+3 of A, and four packed complex values of B
          // expanded to (Br, -Bi) (column parity 0) or (Bi, Br) (parity 1).
          // Lanes past the chunk's columns read column NC-1 (their results are
          // never stored), so that no read is conditional; the expansion is a
          // rotation by 0 / 16 bits and an xor with a per-lane sign mask (a
          // select between the two forms of a loaded word would be compiled
          // into a branch per word).
          const uint32_t* Bw = reinterpret_cast<const uint32_t*>(Bs);
          const int ncl = (lc >> 1) < NC ? (lc >> 1) : NC - 1;
          const uint32_t brot = (lc & 1) ? 16u : 0u, bflip = (lc & 1) ? 0u : 0x80000000u;
#pragma unroll
          for (int h = 0; h < NCH; ++h) {
            const int n = (cg * NCH + h) * NC + ncl;
#pragma unroll
            for (int j = 0; j < NJ / 8; ++j) {
              u32x4r bw =
                *reinterpret_cast<const u32x4r*>(Bw + n * KT + kc * K + g * (NJ / 2) + 4 * j);
#pragma unroll
              for (int i = 0; i < 4; ++i)
                bw[i] = __builtin_amdgcn_alignbit(bw[i], bw[i], brot) ^ bflip;
#pragma unroll
              for (int rb = 0; rb < 4; ++rb) {
                const u32x4r aw = {a[rb].w[4 * j], a[rb].w[4 * j + 1], a[rb].w[4 * j + 2],
                                   a[rb].w[4 * j + 3]};
                acc[rb][h] = mfma_lp16<LPM ? SA : ST_F16>(aw, bw, acc[rb][h]);
              }
            }
          }
        } else {
          float af[4][NJ];
    #pragma unroll
          for (int rb = 0; rb < 4; ++rb) unpack_raw<SA, K, NJ>(a[rb], g, af[rb]);
          // B operand: real column lc of column chunk h (complex column
          // h*NC + lc/2, part lc&1), real summation index of MFMA j.
          // Unconditional reads (clamped column and summation index: the
          // lanes they serve either hold zero rows of A, K = 1, or columns
          // that are never stored), so that no LDS read sits in a branch.
          // Chunk h + 1's values are read before chunk h's products are
          // issued and used after them (scheduling barriers keep both there;
          // left to itself the scheduler reads them just before their use
          // and waits).
          const int ncl = (lc >> 1) < NC ? (lc >> 1) : NC - 1, q = lc & 1;
          float2 bv[NJ];
    #pragma unroll
          for (int j = 0; j < NJ; ++j) {
            const int rk = K >= 2 ? g * NJ + j : g;
            const int kk = (rk >> 1) < K ? (rk >> 1) : K - 1;
            bv[j] = Bs[((cg * NCH) * NC + ncl) * KT + kc * K + kk];
          }
    #pragma unroll
          for (int h = 0; h < NCH; ++h) {
            float bop[NJ];
    #pragma unroll
            for (int j = 0; j < NJ; ++j) {
              const int rk = K >= 2 ? g * NJ + j : g;
              const float2 b = bv[j];
              bop[j] = (rk & 1) == 0 ? (q == 0 ? b.x : b.y) : (q == 0 ? -b.y : b.x);
            }
            if (h + 1 < NCH) {
    #pragma unroll
              for (int j = 0; j < NJ; ++j) {
                const int rk = K >= 2 ? g * NJ + j : g;
                const int kk = (rk >> 1) < K ? (rk >> 1) : K - 1;
                bv[j] = Bs[((cg * NCH + h + 1) * NC + ncl) * KT + kc * K + kk];
              }
            }
            __builtin_amdgcn_sched_barrier(0);
    #pragma unroll
            for (int rb = 0; rb < 4; ++rb)
    #pragma unroll
              for (int j = 0; j < NJ; ++j)
                acc[rb][h] =
                    __builtin_amdgcn_mfma_f32_16x16x4f32(af[rb][j], bop[j], acc[rb][h], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
          }
        }
        if (kc + 1 < nkc) {
#pragma unroll
          for (int rb = 0; rb < 4; ++rb) a[rb] = an[rb];
        }
      }
#pragma unroll
      for (int h = 0; h < NCH; ++h) {
        __syncthreads();
        // Lane holds rows 4g..4g+3 of each 16-row block at real column lc.
        if (lc < 2 * NC) {
#pragma unroll
          for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int r = wave * 64 + rb * 16 + 4 * g + i;
              if (r < R) Cs[r * kRowsLdc + lc] = acc[rb][h][i];
            }
        }
        __syncthreads();
        // The next tile's rows (loaded during this tile) are waited for here,
        // before this tile's stores are issued: the vector memory counter
        // completes in issue order, so the compiler's wait for them at the
        // hand-over below would also wait for the stores to finish.
        if (h == 0 && last_cg) __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
        const int64_t gch = gch_tab[cg * NCH + h];
        // At most 2048 staged elements (256 rows x 8 columns): eight per
        // thread, or two groups of four.  Table and staging reads are issued
        // together before the stores so that their latencies overlap.
        if (d.vec_c) {
          int64_t g[2];
          int32_t cc[2];
          float2 x[2][4];
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const int v = tid + 256 * u;
            const int hi = 64 + (v < (nC >> 2) ? (v >> 4) : 0);
            g[u] = tc.g[hi];
            cc[u] = tc.c[hi];
          }
#pragma unroll
          for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int c = clo4[i] + cc[u];
              x[u][i] = make_float2(Cs[c], Cs[c + 1]);
            }
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            if (tid + 256 * u >= (nC >> 2)) break;
            const int64_t at = oC + gch + glo4 + g[u];
            if (d.sc_store == ST_F16) store_out4<ST_F16>(d, at, x[u], sc, lmax, bad);
            else if (d.sc_store == ST_BF16) store_out4<ST_BF16>(d, at, x[u], sc, lmax, bad);
            else store_out4<ST_C64>(d, at, x[u], sc, lmax, bad);
          }
        } else {
          int64_t g[8];
          int32_t cc[8];
          float2 x[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int e = tid + 256 * u;
            const int hi = 64 + (e < nC ? (e >> 6) : 0);
            g[u] = tc.g[hi];
            cc[u] = clo + tc.c[hi];
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) x[u] = make_float2(Cs[cc[u]], Cs[cc[u] + 1]);
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            if (tid + 256 * u >= nC) break;
            const int64_t at = oC + gch + glo + g[u];
            if (d.sc_store == ST_F16) store_out<ST_F16>(d, at, x[u], sc, lmax, bad);
            else if (d.sc_store == ST_BF16) store_out<ST_BF16>(d, at, x[u], sc, lmax, bad);
            else store_out<ST_C64>(d, at, x[u], sc, lmax, bad);
          }
        }
      }
    }
    // The next tile's rows become current.
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) a[rb] = an[rb];
  }
  if (cur >= 0) finish_scale<256>(d, cjs, cjb, lmax, bad, red, wexp, sc);
}

// A 16-bit stored A with sums of 16 or more goes to the 16-bit matrix cores
// unless the step asks for FP32 arithmetic (kVarFP32Math).
template <int KB, int NCH>
static hipError_t launch_rows_n(const StepDesc& d, int sa, dim3 grid, size_t lds, hipStream_t s) {
  const bool fp32 = (d.variant & kVarFP32Math) != 0;
  if constexpr (KB == 5) {
    // 32-value chunks: 16-bit stored A on the 16-bit matrix cores only.
    if (sa == ST_F16 && !fp32) hipLaunchKernelGGL((k_rows<KB, NCH, ST_F16, true>), grid, dim3(256), lds, s, d);
    else if (sa == ST_BF16 && !fp32) hipLaunchKernelGGL((k_rows<KB, NCH, ST_BF16, true>), grid, dim3(256), lds, s, d);
    else return hipErrorInvalidValue;
  } else {
    if (sa == ST_F16 && fp32) hipLaunchKernelGGL((k_rows<KB, NCH, ST_F16, false>), grid, dim3(256), lds, s, d);
    else if (sa == ST_F16) hipLaunchKernelGGL((k_rows<KB, NCH, ST_F16, true>), grid, dim3(256), lds, s, d);
    else if (sa == ST_BF16 && fp32) hipLaunchKernelGGL((k_rows<KB, NCH, ST_BF16, false>), grid, dim3(256), lds, s, d);
    else if (sa == ST_BF16) hipLaunchKernelGGL((k_rows<KB, NCH, ST_BF16, true>), grid, dim3(256), lds, s, d);
    else hipLaunchKernelGGL((k_rows<KB, NCH, ST_C64, true>), grid, dim3(256), lds, s, d);
  }
  return hipGetLastError();
}

template <int KB>
static hipError_t launch_rows(const StepDesc& d, int sa, dim3 grid, hipStream_t s) {
  const int N = 1 << d.nt, R = 1 << d.rt, NC = 1 << d.ncb, KT = 1 << d.kt;
  const int nch = N / NC;
  // More than four chunks: groups of four, for a single K chunk only.
  if (R > kRowsRows || NC > 8 || N * KT > kRowsMaxB || d.ncb > d.nt || d.kt < KB ||
      (d.kt > KB && NC != N && nch > 4) || nch > 16 || (nch > 4 && d.kt != KB))
    return hipErrorInvalidValue;
  const size_t lds = sizeof(float2) * (size_t)N * KT + sizeof(float) * (size_t)R * kRowsLdc;
  // Persistent grid: enough workgroups to fill every CU several times over.
  const uint64_t n_tiles = (uint64_t)d.n_row_tiles * (uint64_t)d.copies;
  grid = dim3((unsigned)std::min<uint64_t>(n_tiles, kRowsGrid), 1);
  switch (nch) {
    case 1: return launch_rows_n<KB, 1>(d, sa, grid, lds, s);
    case 2: return launch_rows_n<KB, 2>(d, sa, grid, lds, s);
    case 4:
    case 8:
    case 16: return launch_rows_n<KB, 4>(d, sa, grid, lds, s);
  }
  return hipErrorInvalidValue;
}

// K chunks: the whole sum for k <= 4, chunks of 16 complex values beyond
// (a 32-value complex64 chunk would hold twice the rows' registers and halve
// the number of resident waves).  A 16-bit stored A on the 16-bit matrix
// cores takes 32-value chunks: the same registers, and a chunk of each row
// is one whole 128-byte line (16-value chunks read each line in two halves,
// at different times, and fetched up to 1.7 times the bytes).
hipError_t launch_rows_kernel(const StepDesc& d, int sa, dim3 grid, hipStream_t s) {
  if (d.kt >= 5 && sa != ST_C64 && !(d.variant & kVarFP32Math)) return launch_rows<5>(d, sa, grid, s);
  switch (d.kt) {
    case 0: return launch_rows<0>(d, sa, grid, s);
    case 1: return launch_rows<1>(d, sa, grid, s);
    case 2: return launch_rows<2>(d, sa, grid, s);
    case 3: return launch_rows<3>(d, sa, grid, s);
    case 4: return launch_rows<4>(d, sa, grid, s);
    case 5:
    case 6:
    case 7:
    case 8:
    case 9:
    case 10:
    case 11:
    case 12: return launch_rows<4>(d, sa, grid, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace rqc

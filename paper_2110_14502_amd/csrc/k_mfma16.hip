// FP16 / BF16 matrix-core contraction kernel (reduced precision).
#include <type_traits>

#include "kernels_dev.h"

namespace rqc {

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
static_assert(kCHalf <= kLMainWords, "C staging must fit the operand buffers");
constexpr unsigned kMfma16Grid = 256 * 2;  // persistent workgroups (two per CU)

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

// B_r words of a lane from four packed complex values of its column:
// (re, -im) for output column parity 0, (im, re) for parity 1.  Branch-free:
// a rotation by `rot` (0 or 16 bits) and an xor with `flip` (the sign bit of
// the high half, or 0), both fixed per lane.  (A select between the two
// forms of an LDS-loaded word is compiled into a branch per word, each with
// a wait for the LDS read.)
struct BExpand {
  uint32_t rot, flip;
};
__device__ __forceinline__ BExpand b_expand_of(bool swap_halves) {
  return BExpand{swap_halves ? 16u : 0u, swap_halves ? 0u : 0x80000000u};
}
__device__ __forceinline__ u32x4 expand_b(u32x4 w, BExpand e) {
  u32x4 o;
#pragma unroll
  for (int i = 0; i < 4; ++i) o[i] = __builtin_amdgcn_alignbit(w[i], w[i], e.rot) ^ e.flip;
  return o;
}

// Pre-scales of complex64 operands (to 2^14) and the output scale of a copy:
// the accumulator holds the product times 2^(pA+pB); the output shift maps
// the bound to the storage target (as in compute_scale).
struct CopyScale {
  int pA, pB;
  Scale sc;
};
template <int LP, int SA, int SB>
__device__ __forceinline__ CopyScale lp_copy_scale(const StepDesc& d, int js, int jb) {
  const float mA = max_abs_of(d.maxA, js * d.eA_s + jb * d.eA_b, d.maxA_const);
  const float mB = max_abs_of(d.maxB, js * d.eB_s + jb * d.eB_b, d.maxB_const);
  const int EA = mA > 0.f ? ceil_log2(mA) : 0, EB = mB > 0.f ? ceil_log2(mB) : 0;
  CopyScale r;
  r.pA = (SA == LP || mA <= 0.f) ? 0 : 14 - EA;
  r.pB = (SB == LP || mB <= 0.f) ? 0 : 14 - EB;
  r.sc = Scale{r.pA + r.pB, 0};
  const int eA = (d.track && d.expA) ? d.expA[js * d.eA_s + jb * d.eA_b] : 0;
  const int eB = (d.track && d.expB) ? d.expB[js * d.eB_s + jb * d.eB_b] : 0;
  r.sc.expC = eA + eB;
  if (d.track && mA > 0.f && mB > 0.f && mA <= 3.0e38f && mB <= 3.0e38f) {
    const int t = d.k_total + 1 + (EA + r.pA) + (EB + r.pB) - target_log2(d);
    r.sc.shift = t;
    r.sc.expC = eA - r.pA + eB - r.pB + t;
  }
  return r;
}

// VEC: the two lowest tile bits of A and of B are their two lowest address
// bits (summed indices, as the planner lays out every step), so four
// consecutive tile elements are 16 contiguous bytes: one vector load and
// one 16-byte LDS write per four elements.
template <int LP, int SA, int SB, int SC, bool VEC, int KT>
__device__ __forceinline__ void mfma16_body(const StepDesc& d, uint64_t n_items, uint32_t* lw,
                                            TileTab& tcs, OuterTab& ot) {
  uint32_t* Abuf = lw;                  // [2][kTM][kLRow]
  uint32_t* Bbuf = lw + 2 * kLABuf;     // [2][kTN][kLRow]
  float* lds = reinterpret_cast<float*>(lw);
  float* red = lds + kLMainWords;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  // A chunk tile: 128 rows x 2^KT k (KT = 5: 4096 elements, 16 per thread or
  // 4 vectors of 4); B chunk tile: 2^KT k x 64 columns (KT = 5: 2048, 8 or 2
  // vectors).  KT = 4 fills half of each LDS row.
  constexpr int NA = VEC ? (1 << (KT - 3)) : (1 << (KT - 1));
  constexpr int NB = VEC ? (1 << (KT - 4)) : (1 << (KT - 2));
  int64_t gA[NA];
  int lA[NA];
  int64_t gB[NB];
  int lB[NB];
  {
    TileTab* ta = reinterpret_cast<TileTab*>(lds);
    TileTab* tb = ta + 1;
    build_tab(d.tA, kLRow, 0, 1, *ta);
    build_tab(d.tB, 0, kLRow, 1, *tb);
    build_outer(d, ot);
    __syncthreads();
    if (VEC) {
      // Vector v = tid + 256 j covers elements 4v .. 4v+3.
      const int lo = (tid & 15) << 2, hi0 = 64 + (tid >> 4);
#pragma unroll
      for (int j = 0; j < NA; ++j) {
        gA[j] = ta->g[lo] + ta->g[hi0 + 16 * j];
        lA[j] = ta->c[lo] + ta->c[hi0 + 16 * j];
      }
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        gB[j] = tb->g[lo] + tb->g[hi0 + 16 * j];
        lB[j] = tb->c[lo] + tb->c[hi0 + 16 * j];
      }
    } else {
#pragma unroll
      for (int j = 0; j < NA; ++j) {
        gA[j] = ta->g[lane] + ta->g[64 + wave + 4 * j];
        lA[j] = ta->c[lane] + ta->c[64 + wave + 4 * j];
      }
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        gB[j] = tb->g[lane] + tb->g[64 + wave + 4 * j];
        lB[j] = tb->c[lane] + tb->c[64 + wave + 4 * j];
      }
    }
  }
  int hb = 0;
  for (int b = 0; b < d.tC.nbits; ++b)
    if (d.tC.role[b] == 0 && d.tC.cbit[b] == 6) hb = b;
  const int64_t g_half = int64_t(1) << d.tC.gpos[hb];
  build_tab_skip(d.tC, hb, kCStride, 2, tcs);
  __syncthreads();  // operand tables copied out; the buffers are free
  const int64_t g_lane = tcs.g[lane];
  const int c_lane = tcs.c[lane];
  // Vector stores when C's two lowest address bits are the two lowest
  // C-order bits of the staged half.
  const bool vec_c = d.tC.nbits > 2 && hb > 1 && d.tC.gpos[0] == 0 && d.tC.gpos[1] == 1;
  const int64_t g_lo4 = tcs.g[(tid & 15) << 2];
  int c_lo4[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) c_lo4[i] = tcs.c[((tid & 15) << 2) + i];

  const int lrow = lane & 31;
  const int kq = (lane >> 5) * 4;      // first complex k of the lane's 8 real k
  const int ncol = (lane & 31) >> 1;
  const BExpand bswap = b_expand_of((lane & 1) != 0);  // C_r column parity 1: (im, re)

  auto copy_scale = [&](int js, int jb) { return lp_copy_scale<LP, SA, SB>(d, js, jb); };

  // A chunk in flight is kept raw in registers: 16-bit stored operands as
  // their packed words, complex64 operands as their float pairs.  The
  // conversion to packed 16-bit words (with the copy's power-of-two
  // pre-scale) happens only when the chunk is written to LDS, so issuing the
  // next chunk's loads never waits for their data.  (The scalar-load path of
  // other layouts converts at load time: its raw chunk would not fit the
  // register budget.)
  constexpr int EA = (VEC && SA != LP) ? 2 : 1, EB = (VEC && SB != LP) ? 2 : 1;  // words per element
  constexpr int WA = (VEC ? 4 * NA : NA) * EA, WB = (VEC ? 4 * NB : NB) * EB;
  uint32_t ra[WA], rb[WB];
  auto load_chunk = [&](int64_t oA, int64_t oB, int kc, int pA, int pB) {
    int64_t kA, kB;
    k_offsets(d, ot, kc, kA, kB);
    const uint32_t* pa = reinterpret_cast<const uint32_t*>(d.A);
    const uint32_t* pb = reinterpret_cast<const uint32_t*>(d.B);
    if (VEC) {
#pragma unroll
      for (int j = 0; j < NA; ++j)
#pragma unroll
        for (int h = 0; h < EA; ++h) {
          const uint4 v = *reinterpret_cast<const uint4*>(pa + EA * (oA + kA + gA[j]) + 4 * h);
          ra[(4 * j + 0) * EA + 4 * h + 0] = v.x;
          ra[(4 * j + 0) * EA + 4 * h + 1] = v.y;
          ra[(4 * j + 0) * EA + 4 * h + 2] = v.z;
          ra[(4 * j + 0) * EA + 4 * h + 3] = v.w;
        }
#pragma unroll
      for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int h = 0; h < EB; ++h) {
          const uint4 v = *reinterpret_cast<const uint4*>(pb + EB * (oB + kB + gB[j]) + 4 * h);
          rb[(4 * j + 0) * EB + 4 * h + 0] = v.x;
          rb[(4 * j + 0) * EB + 4 * h + 1] = v.y;
          rb[(4 * j + 0) * EB + 4 * h + 2] = v.z;
          rb[(4 * j + 0) * EB + 4 * h + 3] = v.w;
        }
    } else {
      auto one = [&](const void* p, int64_t i, bool lp, int pre) -> uint32_t {
        if (lp) return reinterpret_cast<const uint32_t*>(p)[i];
        float2 v = reinterpret_cast<const float2*>(p)[i];
        if (pre) {
          v.x = ldexpf(v.x, pre);
          v.y = ldexpf(v.y, pre);
        }
        return pack_lp<LP>(v);
      };
#pragma unroll
      for (int j = 0; j < NA; ++j) ra[j] = one(d.A, oA + kA + gA[j], SA == LP, pA);
#pragma unroll
      for (int j = 0; j < NB; ++j) rb[j] = one(d.B, oB + kB + gB[j], SB == LP, pB);
    }
  };
  // Packed word of raw element i of a register array (E words per element).
  auto word = [&](const uint32_t* r, int E, int i, int pre) -> uint32_t {
    if (E == 1) return r[i];
    float2 v = make_float2(__uint_as_float(r[2 * i]), __uint_as_float(r[2 * i + 1]));
    if (pre) {
      v.x = ldexpf(v.x, pre);
      v.y = ldexpf(v.y, pre);
    }
    return pack_lp<LP>(v);
  };
  auto store_chunk = [&](int buf, int pA, int pB) {
    uint32_t* An = Abuf + buf * kLABuf;
    uint32_t* Bn = Bbuf + buf * kLBBuf;
    if (VEC) {
#pragma unroll
      for (int j = 0; j < NA; ++j)
        *reinterpret_cast<uint4*>(An + lA[j]) =
            make_uint4(word(ra, EA, 4 * j, pA), word(ra, EA, 4 * j + 1, pA),
                       word(ra, EA, 4 * j + 2, pA), word(ra, EA, 4 * j + 3, pA));
#pragma unroll
      for (int j = 0; j < NB; ++j)
        *reinterpret_cast<uint4*>(Bn + lB[j]) =
            make_uint4(word(rb, EB, 4 * j, pB), word(rb, EB, 4 * j + 1, pB),
                       word(rb, EB, 4 * j + 2, pB), word(rb, EB, 4 * j + 3, pB));
    } else {
#pragma unroll
      for (int j = 0; j < NA; ++j) An[lA[j]] = word(ra, EA, j, pA);
#pragma unroll
      for (int j = 0; j < NB; ++j) Bn[lB[j]] = word(rb, EB, j, pB);
    }
  };

  // Persistent walk over (copy, tile) items as in the FP32 kernel: tile
  // counts are powers of two, column tiles fastest.
  const int n_kc = 1 << d.n_ko;
  const int tbits = d.n_ro + d.n_no;
  const uint64_t tmask = (uint64_t(1) << tbits) - 1, cmask = (uint64_t(1) << d.n_no) - 1;
  // Step i of the walk covers items i*G .. i*G + G - 1, dealt so that the
  // workgroups of one XCD (blocks go round-robin to the 8 XCDs) take
  // consecutive items: they share rows of A in that XCD's L2.
  const uint64_t G = gridDim.x;
  uint64_t t = (G & 7) == 0 ? (blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3) : blockIdx.x;
  int cur = -1, cjs = 0, cjb = 0;
  bool wexp = false;
  // A copy's scales are read when its first tile is prefetched (before those
  // loads are issued), not at the top of the tile, where the wait for them
  // would also wait for the previous tile's output stores.
  CopyScale cs{0, 0, Scale{0, 0}}, ncs{0, 0, Scale{0, 0}};
  float lmax = 0.f;
  int bad = 0;
  if (t < n_items) {
    const int copy = (int)(t >> tbits);
    const uint64_t bid = t & tmask;
    const int js = copy % d.gs_c, jb = copy / d.gs_c;
    int64_t oA, oB, oC;
    outer_offsets(d, ot, bid >> d.n_no, bid & cmask, js, jb, oA, oB, oC);
    ncs = copy_scale(js, jb);
    load_chunk(oA, oB, 0, ncs.pA, ncs.pB);
    store_chunk(0, ncs.pA, ncs.pB);
  }
  __syncthreads();
  for (; t < n_items; t += G) {
    const int copy = (int)(t >> tbits);
    const uint64_t bid = t & tmask;
    const int js = copy % d.gs_c, jb = copy / d.gs_c;
    if (copy != cur) {
      if (cur >= 0) finish_scale<256>(d, cjs, cjb, lmax, bad, red, wexp, cs.sc);
      cs = ncs;
      lmax = 0.f;
      bad = 0;
      wexp = false;
      cur = copy;
      cjs = js;
      cjb = jb;
    }
    wexp = wexp || bid == 0;
    int64_t oA, oB, oC;
    outer_offsets(d, ot, bid >> d.n_no, bid & cmask, js, jb, oA, oB, oC);
    const bool next_tile = t + G < n_items;

    floatx16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    for (int kc = 0; kc < n_kc; ++kc) {
      const int cb = kc & 1;
      const bool more = kc + 1 < n_kc;
      // Next chunk of this tile, or the first chunk of the next tile (kept
      // in registers until this tile's output has left the LDS).
      if (more) {
        load_chunk(oA, oB, kc + 1, cs.pA, cs.pB);
      } else if (next_tile) {
        const int cn = (int)((t + G) >> tbits);
        const uint64_t bn = (t + G) & tmask;
        const int jsn = cn % d.gs_c, jbn = cn / d.gs_c;
        int64_t pA, pB, pC;
        outer_offsets(d, ot, bn >> d.n_no, bn & cmask, jsn, jbn, pA, pB, pC);
        if (cn != copy) ncs = copy_scale(jsn, jbn);
        load_chunk(pA, pB, 0, ncs.pA, ncs.pB);
      }
      const uint32_t* As = Abuf + cb * kLABuf + (wm * 64 + lrow) * kLRow + kq;
      const uint32_t* Bs = Bbuf + cb * kLBBuf + (wn * 32 + ncol) * kLRow + kq;
#pragma unroll
      for (int kk = 0; kk < (1 << KT) / 8; ++kk) {
        const u32x4 a0 = *reinterpret_cast<const u32x4*>(As + kk * 8);
        const u32x4 a1 = *reinterpret_cast<const u32x4*>(As + 32 * kLRow + kk * 8);
        const u32x4 b0 = expand_b(*reinterpret_cast<const u32x4*>(Bs + kk * 8), bswap);
        const u32x4 b1 = expand_b(*reinterpret_cast<const u32x4*>(Bs + 16 * kLRow + kk * 8), bswap);
        acc[0][0] = mfma16<LP>(a0, b0, acc[0][0]);
        acc[0][1] = mfma16<LP>(a0, b1, acc[0][1]);
        acc[1][0] = mfma16<LP>(a1, b0, acc[1][0]);
        acc[1][1] = mfma16<LP>(a1, b1, acc[1][1]);
      }
      if (more) store_chunk(cb ^ 1, cs.pA, cs.pB);
      __syncthreads();
    }

    float* Cs = lds;
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
      if (vec_c)
        store_half4<SC>(d, Cs, tcs, oC + g_lo4 + (h ? g_half : 0), c_lo4, tid, cs.sc, lmax, bad);
      else
        store_half<SC, VEC ? 8 : 4>(d, Cs, tcs, oC + g_lane + (h ? g_half : 0), c_lane, wave, cs.sc, lmax, bad);
      __syncthreads();
    }
    if (next_tile) {
      store_chunk(0, ncs.pA, ncs.pB);
      __syncthreads();
    }
  }
  if (cur >= 0) finish_scale<256>(d, cjs, cjb, lmax, bad, red, wexp, cs.sc);
}

template <int LP, int SA, int SB, int SC, bool VEC, int KT>
__global__ __launch_bounds__(256, 2) void k_mfma16(StepDesc d, uint64_t n_items) {
  __shared__ __attribute__((aligned(16))) uint32_t lw[kLMainWords + 16];
  __shared__ TileTab tcs;
  __shared__ OuterTab ot;
  mfma16_body<LP, SA, SB, SC, VEC, KT>(d, n_items, lw, tcs, ot);
}


// ---------------------------------------------------------------------------
// Streaming form for memory-bound steps whose whole sum fits one LDS tile of
// B (sums of 32..128 complex terms, A stored in 16 bits, the planner's
// layout): each workgroup walks a contiguous range of (copy, column tile,
// row tile) items, row tiles fastest, so the 64-column tile of B over the
// whole sum is loaded into LDS once per (copy, column tile) and stays there;
// only A streams, two 32-term chunks in flight (raw 16-bit words in
// registers) while the current one is multiplied, across tile boundaries.
// 34 KB (B resident) + 37 KB (A double buffer, the output staging inside
// it) of LDS: two workgroups per CU.
// ---------------------------------------------------------------------------
constexpr int kStreamMaxK = 128;                   // complex terms of the sum
constexpr int kBResWords = kTN * (kStreamMaxK + 4);  // resident B tile
constexpr int kStreamAWords = 2 * kLABuf;            // A double buffer
static_assert(kCHalf <= kStreamAWords, "C staging must fit the A buffers");

template <int LP, int SB, int SC>
__device__ __forceinline__ void mfma16_stream_body(const StepDesc& d, uint64_t n_items,
                                                   uint32_t* lw, uint32_t* bres, TileTab& tcs,
                                                   OuterTab& ot) {
  constexpr int SA = LP;
  constexpr int NA = 4;  // vectors of 4 elements per thread and A chunk (128 x 32)
  constexpr int NB = 2;  // per B chunk (32 x 64)
  constexpr int EB = SB == LP ? 1 : 2;
  uint32_t* Abuf = lw;  // [2][kTM][kLRow]
  float* lds = reinterpret_cast<float*>(lw);
  float* red = lds + kStreamAWords;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int KT = 1 << d.k_total;          // whole sum, <= kStreamMaxK
  const int bRow = KT + 4;                // words per resident B column
  int64_t gA[NA], gB[NB];
  int lA[NA], lB[NB];
  {
    TileTab* ta = reinterpret_cast<TileTab*>(lds);
    TileTab* tb = ta + 1;
    build_tab(d.tA, kLRow, 0, 1, *ta);
    build_tab(d.tB, 0, bRow, 1, *tb);
    build_outer(d, ot);
    __syncthreads();
    const int lo = (tid & 15) << 2, hi0 = 64 + (tid >> 4);
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      gA[j] = ta->g[lo] + ta->g[hi0 + 16 * j];
      lA[j] = ta->c[lo] + ta->c[hi0 + 16 * j];
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      gB[j] = tb->g[lo] + tb->g[hi0 + 16 * j];
      lB[j] = tb->c[lo] + tb->c[hi0 + 16 * j];
    }
  }
  int hb = 0;
  for (int b = 0; b < d.tC.nbits; ++b)
    if (d.tC.role[b] == 0 && d.tC.cbit[b] == 6) hb = b;
  const int64_t g_half = int64_t(1) << d.tC.gpos[hb];
  build_tab_skip(d.tC, hb, kCStride, 2, tcs);
  __syncthreads();
  const bool vec_c = d.tC.nbits > 2 && hb > 1 && d.tC.gpos[0] == 0 && d.tC.gpos[1] == 1;
  const int64_t g_lane = tcs.g[lane];
  const int c_lane = tcs.c[lane];
  const int64_t g_lo4 = tcs.g[(tid & 15) << 2];
  int c_lo4[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) c_lo4[i] = tcs.c[((tid & 15) << 2) + i];
  const int lrow = lane & 31;
  const int kq = (lane >> 5) * 4;
  const int ncol = (lane & 31) >> 1;
  const BExpand bswap = b_expand_of((lane & 1) != 0);

  // Items: copy, then column tile, then row tile (fastest); contiguous
  // ranges per workgroup.  Chunk q of the range: item t0 + (q >> n_ko),
  // K chunk q & (n_kc - 1).
  const int n_ko = d.n_ko, n_kc = 1 << n_ko;
  const int tbits = d.n_ro + d.n_no;
  const uint64_t tmask = (uint64_t(1) << tbits) - 1, rmask = (uint64_t(1) << d.n_ro) - 1;
  // Workgroup w takes the w-th contiguous range; w is dealt so that
  // consecutive ranges run on the same XCD (blocks go round-robin to the 8
  // XCDs): the ranges of one copy's column tiles then stream the same rows of
  // A at the same time and share them in that XCD's L2.
  const uint64_t G = gridDim.x;
  const uint64_t w = (G & 7) == 0 ? (blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3) : blockIdx.x;
  const uint64_t per = (n_items + G - 1) / G;
  const uint64_t t0 = w * per;
  const uint64_t t1 = t0 + per < n_items ? t0 + per : n_items;
  if (t0 >= t1) return;
  const uint64_t n_q = (t1 - t0) << n_ko;
  auto item_offsets = [&](uint64_t t, int64_t& oA, int64_t& oB, int64_t& oC) {
    const int copy = (int)(t >> tbits);
    const uint64_t bid = t & tmask;
    outer_offsets(d, ot, bid & rmask, bid >> d.n_ro, copy % d.gs_c, copy / d.gs_c, oA, oB, oC);
  };
  uint32_t ra[2][4 * NA];
  auto load_a = [&](uint64_t q, uint32_t (&r)[4 * NA]) {
    int64_t oA, oB, oC, kA, kB;
    item_offsets(t0 + (q >> n_ko), oA, oB, oC);
    k_offsets(d, ot, (uint32_t)(q & (n_kc - 1)), kA, kB);
    const uint32_t* pa = reinterpret_cast<const uint32_t*>(d.A);
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const uint4 v = *reinterpret_cast<const uint4*>(pa + oA + kA + gA[j]);
      r[4 * j] = v.x, r[4 * j + 1] = v.y, r[4 * j + 2] = v.z, r[4 * j + 3] = v.w;
    }
  };
  auto store_a = [&](int buf, const uint32_t (&r)[4 * NA]) {
    uint32_t* An = Abuf + buf * kLABuf;
#pragma unroll
    for (int j = 0; j < NA; ++j)
      *reinterpret_cast<uint4*>(An + lA[j]) = make_uint4(r[4 * j], r[4 * j + 1], r[4 * j + 2], r[4 * j + 3]);
  };
  // The resident B tile of an item's (copy, column tile), all K chunks.
  auto load_b = [&](uint64_t t, int pB) {
    int64_t oA, oB, oC;
    item_offsets(t, oA, oB, oC);
    const uint32_t* pb = reinterpret_cast<const uint32_t*>(d.B);
    for (int kc = 0; kc < n_kc; ++kc) {
      int64_t kA, kB;
      k_offsets(d, ot, (uint32_t)kc, kA, kB);
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        uint32_t w[4];
        const int64_t at = oB + kB + gB[j];
        if (EB == 1) {
          const uint4 v = *reinterpret_cast<const uint4*>(pb + at);
          w[0] = v.x, w[1] = v.y, w[2] = v.z, w[3] = v.w;
        } else {
          const float4 x = *reinterpret_cast<const float4*>(pb + 2 * at);
          const float4 y = *reinterpret_cast<const float4*>(pb + 2 * at + 4);
          const float2 v[4] = {make_float2(x.x, x.y), make_float2(x.z, x.w),
                               make_float2(y.x, y.y), make_float2(y.z, y.w)};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            float2 u = v[e];
            if (pB) {
              u.x = ldexpf(u.x, pB);
              u.y = ldexpf(u.y, pB);
            }
            w[e] = pack_lp<LP>(u);
          }
        }
        *reinterpret_cast<uint4*>(bres + lB[j] + kc * 32) = make_uint4(w[0], w[1], w[2], w[3]);
      }
    }
  };

  int cur = -1, cjs = 0, cjb = 0;
  int64_t bkey = -1;  // resident B: copy * n_col_tiles + column tile
  bool wexp = false;
  CopyScale cs{0, 0, Scale{0, 0}};
  float lmax = 0.f;
  int bad = 0;
  // Chunks 0 and 1 in flight; chunk 0 to LDS buffer 0.  Chunk q uses
  // register set and LDS buffer q & 1; the loop handles chunks in pairs so
  // that the register set of each is known at compile time (a register
  // array indexed at run time would serialise the loads in flight).
  load_a(0, ra[0]);
  if (n_q > 1) load_a(1, ra[1]);
  store_a(0, ra[0]);
  floatx16 acc[2][2];
  auto chunk = [&](auto P, uint64_t q) {
    constexpr int p = decltype(P)::value;
    const int kc = (int)(q & (n_kc - 1));
    const uint64_t t = t0 + (q >> n_ko);
    if (kc == 0) {
      const int copy = (int)(t >> tbits);
      const uint64_t bid = t & tmask;
      const int js = copy % d.gs_c, jb = copy / d.gs_c;
      if (copy != cur) {
        if (cur >= 0) finish_scale<256>(d, cjs, cjb, lmax, bad, red, wexp, cs.sc);
        cs = lp_copy_scale<LP, SA, SB>(d, js, jb);
        lmax = 0.f;
        bad = 0;
        wexp = false;
        cur = copy;
        cjs = js;
        cjb = jb;
      }
      wexp = wexp || bid == 0;
      const int64_t key = (int64_t)copy * d.n_col_tiles + (int64_t)(bid >> d.n_ro);
      if (key != bkey) {
        __syncthreads();  // every wave is done with the previous B tile
        load_b(t, cs.pB);
        bkey = key;
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
    }
    // Chunk q + 2 into the register set chunk q came from.
    if (q + 2 < n_q) load_a(q + 2, ra[p]);
    __syncthreads();  // chunk q (and a new B tile) visible in LDS
    const uint32_t* As = Abuf + p * kLABuf + (wm * 64 + lrow) * kLRow + kq;
    const uint32_t* Bs = bres + (wn * 32 + ncol) * bRow + kc * 32 + kq;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const u32x4 a0 = *reinterpret_cast<const u32x4*>(As + kk * 8);
      const u32x4 a1 = *reinterpret_cast<const u32x4*>(As + 32 * kLRow + kk * 8);
      const u32x4 b0 = expand_b(*reinterpret_cast<const u32x4*>(Bs + kk * 8), bswap);
      const u32x4 b1 = expand_b(*reinterpret_cast<const u32x4*>(Bs + 16 * bRow + kk * 8), bswap);
      acc[0][0] = mfma16<LP>(a0, b0, acc[0][0]);
      acc[0][1] = mfma16<LP>(a0, b1, acc[0][1]);
      acc[1][0] = mfma16<LP>(a1, b0, acc[1][0]);
      acc[1][1] = mfma16<LP>(a1, b1, acc[1][1]);
    }
    const bool last = kc == n_kc - 1;
    if (!last && q + 1 < n_q) store_a(p ^ 1, ra[p ^ 1]);
    if (last) {
      int64_t oA, oB, oC;
      item_offsets(t, oA, oB, oC);
      float* Cs = lds;
      __syncthreads();  // every wave is done reading the A buffers
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
        if (vec_c)
          store_half4<SC>(d, Cs, tcs, oC + g_lo4 + (h ? g_half : 0), c_lo4, tid, cs.sc, lmax, bad);
        else
          store_half<SC, 8>(d, Cs, tcs, oC + g_lane + (h ? g_half : 0), c_lane, wave, cs.sc, lmax, bad);
        __syncthreads();
      }
      if (q + 1 < n_q) store_a(p ^ 1, ra[p ^ 1]);
    }
  };
  for (uint64_t q = 0; q < n_q; q += 2) {
    chunk(std::integral_constant<int, 0>{}, q);
    if (q + 1 < n_q) chunk(std::integral_constant<int, 1>{}, q + 1);
  }
  if (cur >= 0) finish_scale<256>(d, cjs, cjb, lmax, bad, red, wexp, cs.sc);
}

template <int LP, int SB, int SC>
__global__ __launch_bounds__(256, 2) void k_mfma16_stream(StepDesc d, uint64_t n_items) {
  __shared__ __attribute__((aligned(16))) uint32_t lw[kStreamAWords + 16];
  __shared__ __attribute__((aligned(16))) uint32_t bres[kBResWords];
  __shared__ TileTab tcs;
  __shared__ OuterTab ot;
  mfma16_stream_body<LP, SB, SC>(d, n_items, lw, bres, tcs, ot);
}

// The streaming form applies to the planner's vector layout with sums of
// 32..128 terms and a 16-bit stored A.
inline bool mfma16_stream_ok(const StepDesc& d, int sa, int lp) {
  return sa == lp && d.kt == 5 && d.k_total <= 7 && lp_vec_layout(d);
}

template <int LP>
static hipError_t launch_mfma16(const StepDesc& d, int sa, int sb, int sc, dim3 grid,
                                hipStream_t s) {
  constexpr int C = ST_C64;
  const uint64_t n_items = (uint64_t)grid.x * (uint64_t)d.copies;
  grid = dim3((unsigned)(n_items < kMfma16Grid ? n_items : kMfma16Grid), 1);
  const bool vec = lp_vec_layout(d);
  if (d.kt == 4 && !vec) return hipErrorInvalidValue;  // the planner's layouts only
  if ((d.variant & kVarStream) && mfma16_stream_ok(d, sa, LP)) {
    if (sb == LP && sc == LP)
      hipLaunchKernelGGL((k_mfma16_stream<LP, LP, LP>), grid, dim3(256), 0, s, d, n_items);
    else if (sb == LP)
      hipLaunchKernelGGL((k_mfma16_stream<LP, LP, ST_C64>), grid, dim3(256), 0, s, d, n_items);
    else if (sc == LP)
      hipLaunchKernelGGL((k_mfma16_stream<LP, ST_C64, LP>), grid, dim3(256), 0, s, d, n_items);
    else
      hipLaunchKernelGGL((k_mfma16_stream<LP, ST_C64, ST_C64>), grid, dim3(256), 0, s, d, n_items);
    return hipGetLastError();
  }
#define RQC_LP_CASE(a, b, c)                                                        \
  if (sa == a && sb == b && sc == c) {                                              \
    if (d.kt == 4)                                                                  \
      hipLaunchKernelGGL((k_mfma16<LP, a, b, c, true, 4>), grid, dim3(256), 0, s, d, n_items); \
    else if (vec)                                                                   \
      hipLaunchKernelGGL((k_mfma16<LP, a, b, c, true, 5>), grid, dim3(256), 0, s, d, n_items); \
    else                                                                            \
      hipLaunchKernelGGL((k_mfma16<LP, a, b, c, false, 5>), grid, dim3(256), 0, s, d, n_items); \
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
hipError_t launch_mfma16_kernel(const StepDesc& d, int sa, int sb, int sc, int lp_kind, dim3 grid,
                                hipStream_t s) {
  if (d.rt != 7 || d.nt != 6 || (d.kt != 5 && d.kt != 4)) return hipErrorInvalidValue;
  if (lp_kind == ST_F16) return launch_mfma16<ST_F16>(d, sa, sb, sc, grid, s);
  if (lp_kind == ST_BF16) return launch_mfma16<ST_BF16>(d, sa, sb, sc, grid, s);
  return hipErrorInvalidValue;
}

}  // namespace rqc

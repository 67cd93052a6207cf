// Device-side helpers shared by the contraction kernels: storage types,
// per-copy power-of-two scaling, offset tables and tile constants.
//
// Complex arithmetic on the real matrix cores: an interleaved complex
// A[m][k] is read as the real matrix A_r[m][2k+c] (c = 0 re, 1 im); the
// complex B[k][n] is expanded per lane into the real 2x2 block
//   B_r[2k+0][2n+0] = Br   B_r[2k+0][2n+1] = Bi
//   B_r[2k+1][2n+0] = -Bi  B_r[2k+1][2n+1] = Br
// so that A_r * B_r is exactly the interleaved complex C[m][2n+d].  The real
// flops executed equal 8 per complex multiply-add, the algorithmic count.
#pragma once

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

// Step outputs are written with nontemporal stores: they are read back by a
// later step, mostly after far more data than the caches hold has passed.
template <int S>
__device__ __forceinline__ void store_c(void* p, int64_t i, float2 v);
template <>
__device__ __forceinline__ void store_c<ST_C64>(void* p, int64_t i, float2 v) {
  typedef float f2v __attribute__((ext_vector_type(2)));
  f2v w = {v.x, v.y};
  __builtin_nontemporal_store(w, reinterpret_cast<f2v*>(p) + i);
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

// The value a store of type S keeps (identity for complex64).
template <int S>
__device__ __forceinline__ float2 round_c(float2 v) {
  if (S == ST_F16) return make_float2((float)(_Float16)v.x, (float)(_Float16)v.y);
  if (S == ST_BF16) return make_float2((float)(__bf16)v.x, (float)(__bf16)v.y);
  return v;
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

// Per-copy scale bookkeeping shared by the kernels' epilogues.  Every
// stored tensor copy carries a power-of-two exponent: value = stored * 2^exp.
// The output shift t is chosen from the rigorous bound
//   |C_re|, |C_im| <= 2^k * (sqrt2 mA)(sqrt2 mB) <= 2^(k+1+E(mA)+E(mB))
// so that the bound lands on 2^15 for 16-bit storage (inside the binary16
// range) and on 2^0 for complex64.  The complex64 normalisation keeps
// heavily sliced networks, whose slice values are far below 2^-126, inside
// the FP32 range; a power-of-two shift changes no rounding.
constexpr int kC64Target = 0;
struct Scale {
  int shift;  // C_stored = acc * 2^-shift
  int expC;
};
__device__ __forceinline__ int target_log2(const StepDesc& d) {
  return d.lp_out ? 15 + d.bias : kC64Target;
}
// An operand's max-abs value: the array entry, or the step's constant when
// there is no array.  The load stays a global-memory load: written as
// `p ? p[i] : c` the compiler may select between the two addresses and load
// through a generic pointer, and a pending generic (FLAT) load makes every
// later wait of the wave wait for all of its memory operations.
typedef __attribute__((address_space(1))) const float global_float;
__device__ __forceinline__ float max_abs_of(const float* p, int64_t i, float c) {
  if (!p) return c;
  return ((global_float*)p)[i];
}

// The operands' exponents and max-abs values of copy (js, jb): read by
// load_scale, turned into the copy's Scale by scale_of.  Kept apart so that a
// kernel can issue the reads early and use them later.
struct ScaleIn {
  int eA, eB;
  float mA, mB;
};

__device__ __forceinline__ ScaleIn load_scale(const StepDesc& d, int js, int jb) {
  ScaleIn r{0, 0, 0.f, 0.f};
  if (!d.track) return r;
  r.eA = d.expA ? d.expA[js * d.eA_s + jb * d.eA_b] : 0;
  r.eB = d.expB ? d.expB[js * d.eB_s + jb * d.eB_b] : 0;
  r.mA = max_abs_of(d.maxA, js * d.eA_s + jb * d.eA_b, d.maxA_const);
  r.mB = max_abs_of(d.maxB, js * d.eB_s + jb * d.eB_b, d.maxB_const);
  return r;
}

__device__ __forceinline__ Scale scale_of(const StepDesc& d, const ScaleIn& r) {
  Scale s{0, 0};
  if (!d.track) return s;
  int t = 0;
  if (r.mA > 0.f && r.mB > 0.f && r.mA <= 3.0e38f && r.mB <= 3.0e38f)
    t = d.k_total + 1 + ceil_log2(r.mA) + ceil_log2(r.mB) - target_log2(d);
  s.shift = t;
  s.expC = r.eA + r.eB + t;
  return s;
}

__device__ __forceinline__ Scale compute_scale(const StepDesc& d, int js, int jb) {
  return scale_of(d, load_scale(d, js, jb));
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

// Outer-bit weights of a step, copied into LDS once per workgroup.  The
// descriptor's bit positions are bytes in the kernel-argument segment: a loop
// over them reads them with vector loads, and each such load waits for every
// load and store the wave has in flight (the counter is in order), which
// would stall the prefetches and output stores of a tile loop.
struct OuterTab {
  int64_t rA[kMaxOuter], rC[kMaxOuter];  // row tile bit i
  int64_t nB[kMaxOuter], nC[kMaxOuter];  // column tile bit i
  int64_t kA[kMaxOuter], kB[kMaxOuter];  // K chunk bit i
};

__device__ __forceinline__ void build_outer(const StepDesc& d, OuterTab& o) {
  for (int i = threadIdx.x; i < kMaxOuter; i += blockDim.x) {
    // All six bytes are read before any is used (one round trip).
    const int ra = d.ro_A[i], rc = d.ro_C[i], nb = d.no_B[i], nc = d.no_C[i];
    const int ka = d.ko_A[i], kb = d.ko_B[i];
    o.rA[i] = i < d.n_ro ? int64_t(1) << ra : 0;
    o.rC[i] = i < d.n_ro ? int64_t(1) << rc : 0;
    o.nB[i] = i < d.n_no ? int64_t(1) << nb : 0;
    o.nC[i] = i < d.n_no ? int64_t(1) << nc : 0;
    o.kA[i] = i < d.n_ko ? int64_t(1) << ka : 0;
    o.kB[i] = i < d.n_ko ? int64_t(1) << kb : 0;
  }
}

__device__ __forceinline__ void outer_offsets(const StepDesc& d, const OuterTab& o, uint64_t ro,
                                              uint64_t no, int js, int jb, int64_t& oA,
                                              int64_t& oB, int64_t& oC) {
  oA = js * d.sA_s + jb * d.sA_b;
  oB = js * d.sB_s + jb * d.sB_b;
  oC = js * d.sC_s + jb * d.sC_b;
  for (int i = 0; i < d.n_ro; ++i)
    if ((ro >> i) & 1) {
      oA += o.rA[i];
      oC += o.rC[i];
    }
  for (int i = 0; i < d.n_no; ++i)
    if ((no >> i) & 1) {
      oB += o.nB[i];
      oC += o.nC[i];
    }
}

__device__ __forceinline__ void k_offsets(const StepDesc& d, const OuterTab& o, uint32_t kc,
                                          int64_t& kA, int64_t& kB) {
  kA = 0;
  kB = 0;
  for (int i = 0; i < d.n_ko; ++i)
    if ((kc >> i) & 1) {
      kA += o.kA[i];
      kB += o.kB[i];
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
    const float2 w = round_c<SC>(v);
    const float m = fmaxf(fabsf(w.x), fabsf(w.y));
    if (!(m <= 3.4e38f)) bad = 1;
    else lmax = fmaxf(lmax, m);
  }
}

// Four consecutive output elements (C addresses at, at+1, at+2, at+3; at a
// multiple of 4) in one 16-byte (16-bit storage) or two 16-byte stores.
template <int SC>
__device__ __forceinline__ void store_out4(const StepDesc& d, int64_t at, float2 (&v)[4],
                                           const Scale& sc, float& lmax, int& bad) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (sc.shift) {
      v[i].x = ldexpf(v[i].x, -sc.shift);
      v[i].y = ldexpf(v[i].y, -sc.shift);
    }
  }
  if (SC == ST_C64) {
    typedef float f4v __attribute__((ext_vector_type(4)));
    f4v* q = reinterpret_cast<f4v*>(reinterpret_cast<float2*>(d.C) + at);
    f4v w0 = {v[0].x, v[0].y, v[1].x, v[1].y}, w1 = {v[2].x, v[2].y, v[3].x, v[3].y};
    // Plain stores: across a wave each of the two instructions writes every
    // other 16 bytes, and with the nontemporal hint such half-covered lines
    // were measured to drain at ~2 TB/s against ~5 TB/s without it.
    q[0] = w0;
    q[1] = w1;
  } else {
    uint32_t w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (SC == ST_F16) {
        h2 o;
        o.x = (_Float16)v[i].x;
        o.y = (_Float16)v[i].y;
        w[i] = __builtin_bit_cast(uint32_t, o);
      } else {
        b2 o;
        o.x = (__bf16)v[i].x;
        o.y = (__bf16)v[i].y;
        w[i] = __builtin_bit_cast(uint32_t, o);
      }
    }
    *reinterpret_cast<uint4*>(reinterpret_cast<uint32_t*>(d.C) + at) = make_uint4(w[0], w[1], w[2], w[3]);
  }
  if (d.track) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float2 r = round_c<SC>(v[i]);
      const float m = fmaxf(fabsf(r.x), fabsf(r.y));
      if (!(m <= 3.4e38f)) bad = 1;
      else lmax = fmaxf(lmax, m);
    }
  }
}

// ---------------------------------------------------------------------------
// Tile constants of the MFMA kernels and the C staging table builder.
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

// Copies the descriptor's three tile maps into LDS (threads 0..38 one word
// each, one round trip); the caller synchronises before use.  Tables built
// straight from the kernel-argument block read its byte fields under per-lane
// indices, one global byte load and one wait at a time: several memory round
// trips before a workgroup's first load, which kernels with one tile per
// workgroup pay in every workgroup.
__device__ __forceinline__ void stage_maps(const StepDesc& d, TileMap (&m)[3]) {
  static_assert(sizeof(TileMap) % 4 == 0, "tile map copied as words");
  constexpr int W = (int)(sizeof(TileMap) / 4);
  const int t = threadIdx.x;
  if (t < 3 * W) {
    const TileMap* src = t < W ? &d.tA : (t < 2 * W ? &d.tB : &d.tC);
    reinterpret_cast<int*>(&m[t / W])[t % W] = reinterpret_cast<const int*>(src)[t % W];
  }
}

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


// Stores one staged half (64 rows) of a 128 x 64 output tile: thread
// (wave, lane) writes C-order elements lane + 64 (wave + 4 j), j < 16.  The
// table and staging reads go out in groups of G so that their latencies
// overlap instead of adding up per element.  `base` is the tile's C offset
// plus this lane's low-bit offset, `cl` the lane's staging coordinate.
template <int SC, int G>
__device__ __forceinline__ void store_half(const StepDesc& d, const float* Cs, const TileTab& tcs,
                                           int64_t base, int cl, int wave, const Scale& sc,
                                           float& lmax, int& bad) {
#pragma unroll
  for (int j0 = 0; j0 < 16; j0 += G) {
    int32_t c[G];
    int64_t g[G];
    float2 v[G];
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const int hi = 64 + wave + 4 * (j0 + j);
      c[j] = cl + tcs.c[hi];
      g[j] = tcs.g[hi];
    }
#pragma unroll
    for (int j = 0; j < G; ++j) v[j] = make_float2(Cs[c[j]], Cs[c[j] + 1]);
#pragma unroll
    for (int j = 0; j < G; ++j) store_out<SC>(d, base + g[j], v[j], sc, lmax, bad);
  }
}

// Vector variant of store_half for tiles whose two lowest C-order bits are
// C's two lowest address bits (and not the half bit): thread t writes the
// groups of four consecutive elements 4 (t + 256 j), j < 4, with one
// 16-byte store (16-bit storage) or two (complex64) per group.  `lo4` are
// the thread's low-bit offset and the staging coordinates of its four.
template <int SC>
__device__ __forceinline__ void store_half4(const StepDesc& d, const float* Cs, const TileTab& tcs,
                                            int64_t base, const int (&lo4)[4], int tid,
                                            const Scale& sc, float& lmax, int& bad) {
  int64_t g[4];
  int c[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int hi = 64 + (tid >> 4) + 16 * j;
    g[j] = tcs.g[hi];
    c[j] = tcs.c[hi];
  }
  float2 x[4][4];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int i = 0; i < 4; ++i) x[j][i] = make_float2(Cs[lo4[i] + c[j]], Cs[lo4[i] + c[j] + 1]);
#pragma unroll
  for (int j = 0; j < 4; ++j) store_out4<SC>(d, base + g[j], x[j], sc, lmax, bad);
}

// Per-kernel launchers (one translation unit each).
hipError_t launch_rows_kernel(const StepDesc& d, int sa, dim3 grid, hipStream_t s);
hipError_t launch_simt_kernel(const StepDesc& d, int sa, int sb, int sc, uint64_t tiles,
                              hipStream_t s);
hipError_t launch_mfma32_kernel(const StepDesc& d, int sa, int sb, int sc, dim3 grid,
                                hipStream_t s);
hipError_t launch_mfma16_kernel(const StepDesc& d, int sa, int sb, int sc, int lp_kind, dim3 grid,
                                hipStream_t s);

}  // namespace rqc

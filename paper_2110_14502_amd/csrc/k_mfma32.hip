// FP32 matrix-core contraction kernel (fused permute + complex GEMM).
#include "kernels_dev.h"

namespace rqc {

// ---------------------------------------------------------------------------
// MFMA contraction (FP32 matrix cores, v_mfma_f32_32x32x2_f32): 128 rows x
// 64 complex columns per tile, 16 complex k per LDS chunk, double buffered;
// 4 waves in a 2x2 grid, each 64 rows x 64 real columns.  The operand
// offsets come from LDS tables built once per workgroup; the output tile is
// staged through LDS in two halves of 64 rows (inside the operand buffers)
// and stored in C's address order.
//
// Persistent: the (copy, tile) items, column tiles fastest, are walked in
// steps of one item per workgroup, the workgroups of an XCD taking
// consecutive items, so that the tiles in flight on an XCD share rows of A.
// A workgroup loads the first chunk of its next tile while its current
// tile's last chunk is multiplied, and writes it to LDS before the current
// tile's output stores go out, so that those stores drain during the next
// tile's products; the scale and the running max-abs are flushed when the
// copy changes.  62 KB of LDS; two workgroups per CU.
// ---------------------------------------------------------------------------
constexpr unsigned kMfmaGrid = 256 * 2;

// ---------------------------------------------------------------------------
// Arithmetic of one 16-k chunk for one wave (64 rows x 32 complex columns of
// the tile), in two forms:
//
// 4M: the real 2x2 expansion of B (kernels_dev.h): A_r (64 x 32 real k) times
//     B_r (32 real k x 64 real columns) on four 32x32 accumulators; 8 real
//     flops executed per complex multiply-add.
// 3M: three real products per complex product (Gauss):
//         P1 = Ar Br,  P2 = Ai Bi,  P3 = (Ar + Ai)(Br + Bi),
//         Re C = P1 - P2,  Im C = P3 - P1 - P2,
//     on six 32x32 accumulators (two row blocks x three products); each
//     MFMA takes two complex k (one per half wave), so a chunk is 48 MFMAs
//     instead of 64: 6 real flops executed per complex multiply-add, with
//     half the LDS reads.  The sums Ar + Ai and Br + Bi are formed in
//     registers from the same LDS planes.
// ---------------------------------------------------------------------------
template <bool M3>
struct Acc32 {
  floatx16 v[M3 ? 6 : 4];
};

template <bool M3>
__device__ __forceinline__ void acc_zero(Acc32<M3>& acc) {
#pragma unroll
  for (int i = 0; i < (M3 ? 6 : 4); ++i)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc.v[i][r] = 0.f;
}

// Abuf_cb / Bbuf_cb: the chunk's LDS buffers ([k][re|im][row] floats and
// [k][col] complex values).
template <bool M3>
__device__ __forceinline__ void chunk_mfma(const float* Abuf_cb, const float2* Bbuf_cb, int lane,
                                           int wm, int wn, Acc32<M3>& acc) {
  if constexpr (!M3) {
    const int lrow = lane & 31;
    const int cpart = lane >> 5;         // A_r column parity: 0 re, 1 im
    const int dpart = lane & 1;          // C_r column parity
    const int ncol = (lane & 31) >> 1;   // complex column inside a 16-col block
    const bool bswap = cpart != dpart;
    const float bsign = (cpart == 1 && dpart == 0) ? -1.f : 1.f;
    const float* As = Abuf_cb + cpart * kAPlane + wm * 64 + lrow;
    const float2* Bs = Bbuf_cb + wn * 32 + ncol;
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
      acc.v[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, v0, acc.v[0], 0, 0, 0);
      acc.v[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, v1, acc.v[1], 0, 0, 0);
      acc.v[2] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, v0, acc.v[2], 0, 0, 0);
      acc.v[3] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, v1, acc.v[3], 0, 0, 0);
      a0 = a0n;
      a1 = a1n;
      b0 = b0n;
      b1 = b1n;
    }
  } else {
    // Lane half h takes complex k = 2 kk + h; rows / columns lane & 31.
    const int h = lane >> 5, l = lane & 31;
    const float* As = Abuf_cb + h * kAStride + wm * 64 + l;
    const float2* Bs = Bbuf_cb + h * kBStride + wn * 32 + l;
    float ar0 = As[0], ai0 = As[kAPlane], ar1 = As[32], ai1 = As[kAPlane + 32];
    float2 b = Bs[0];
#pragma unroll
    for (int kk = 0; kk < kTK / 2; ++kk) {
      float nr0 = 0.f, ni0 = 0.f, nr1 = 0.f, ni1 = 0.f;
      float2 nb = make_float2(0.f, 0.f);
      if (kk + 1 < kTK / 2) {
        const int o = 2 * (kk + 1) * kAStride;
        nr0 = As[o];
        ni0 = As[o + kAPlane];
        nr1 = As[o + 32];
        ni1 = As[o + kAPlane + 32];
        nb = Bs[2 * (kk + 1) * kBStride];
      }
      // Keep the next step's LDS reads ahead of this step's products (left
      // to itself the scheduler sinks them below the products and waits for
      // them right away).
      __builtin_amdgcn_sched_barrier(0);
      const float bs = b.x + b.y, as0 = ar0 + ai0, as1 = ar1 + ai1;
      acc.v[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar0, b.x, acc.v[0], 0, 0, 0);
      acc.v[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai0, b.y, acc.v[1], 0, 0, 0);
      acc.v[2] = __builtin_amdgcn_mfma_f32_32x32x2f32(as0, bs, acc.v[2], 0, 0, 0);
      acc.v[3] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar1, b.x, acc.v[3], 0, 0, 0);
      acc.v[4] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai1, b.y, acc.v[4], 0, 0, 0);
      acc.v[5] = __builtin_amdgcn_mfma_f32_32x32x2f32(as1, bs, acc.v[5], 0, 0, 0);
      ar0 = nr0;
      ai0 = ni0;
      ar1 = nr1;
      ai1 = ni1;
      b = nb;
    }
  }
}

// Writes this wave's 64 x 32 complex accumulators into the staged half Cs
// ([row][real column] floats, kCStride per row).
template <bool M3>
__device__ __forceinline__ void stage_acc(float* Cs, const Acc32<M3>& acc, int lane, int wn) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      if constexpr (!M3) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int col = wn * 64 + j * 32 + (lane & 31);
          Cs[row * kCStride + col] = acc.v[2 * i + j][r];
        }
      } else {
        const float p1 = acc.v[3 * i][r], p2 = acc.v[3 * i + 1][r], p3 = acc.v[3 * i + 2][r];
        const int col = 2 * (wn * 32 + (lane & 31));
        *reinterpret_cast<float2*>(Cs + row * kCStride + col) = make_float2(p1 - p2, p3 - p1 - p2);
      }
    }
}

// LDS of the persistent kernel: buffer b holds A's chunk at b * kPersPair
// and B's right after it; the output staging area starts at buffer 1 and
// runs past it, so that buffer 0 can take the next tile's first chunk while
// the current tile's output is staged.
constexpr int kPersPair = kABuf + 2 * kBBuf;
constexpr int kPersFloats = kPersPair + kCHalf;
static_assert(kPersFloats >= 2 * kPersPair && kPersPair % 4 == 0, "persistent LDS layout");

template <int SA, int SB, int SC, bool M3>
__global__ __launch_bounds__(256, 2) void k_mfma32(StepDesc d, uint64_t n_items) {
  __shared__ float lds[kPersFloats + 16];
  __shared__ TileTab tcs;
  __shared__ OuterTab ot;
  float* Abuf = lds;                                      // [2][kTK][2][kAPlane], pair stride
  float2* Bbuf = reinterpret_cast<float2*>(lds + kABuf);  // [2][kTK][kBStride], pair stride
  float* red = lds + kPersFloats;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  // Per-thread element offsets of the A (2048) and B (1024) chunk tiles.
  int64_t gA[8];
  int lA[8];
  int64_t gB[4];
  int lB[4];
  // The C tile bit that carries row bit 6 (which half of the tile).
  int hb = 0;
  for (int b = 0; b < d.tC.nbits; ++b)
    if (d.tC.role[b] == 0 && d.tC.cbit[b] == 6) hb = b;
  {
    TileTab* ta = reinterpret_cast<TileTab*>(lds);
    TileTab* tb = ta + 1;
    build_tab(d.tA, 1, 0, kAStride, *ta);
    build_tab(d.tB, 0, 1, kBStride, *tb);
    build_tab_skip(d.tC, hb, kCStride, 2, tcs);
    build_outer(d, ot);
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
    __syncthreads();
  }
  const int64_t g_half = int64_t(1) << d.tC.gpos[hb];
  const int64_t g_lane = tcs.g[lane];
  const int c_lane = tcs.c[lane];
  // Vector stores when C's two lowest address bits are the two lowest
  // C-order bits of the staged half.
  const bool vec_c = d.tC.nbits > 2 && hb > 1 && d.tC.gpos[0] == 0 && d.tC.gpos[1] == 1;
  const int64_t g_lo4 = tcs.g[(tid & 15) << 2];
  int c_lo4[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) c_lo4[i] = tcs.c[((tid & 15) << 2) + i];

  const int n_kc = 1 << d.n_ko;
  // Tile counts are powers of two: item t is copy t >> tb, row tile
  // (t & tmask) >> n_no, column tile t & cmask.
  const int tb = d.n_ro + d.n_no;
  const uint64_t tmask = (uint64_t(1) << tb) - 1, cmask = (uint64_t(1) << d.n_no) - 1;
  // Step i of the walk covers items i*G .. i*G + G - 1, dealt so that the
  // workgroups of one XCD (blocks go round-robin to the 8 XCDs) take
  // consecutive items: they share rows of A in that XCD's L2.
  const uint64_t G = gridDim.x;
  uint64_t t = (G & 7) == 0 ? (blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3) : blockIdx.x;

  auto item_offsets = [&](uint64_t it, int64_t& oA, int64_t& oB, int64_t& oC) {
    const int copy = (int)(it >> tb);
    const uint64_t bid = it & tmask;
    outer_offsets(d, ot, bid >> d.n_no, bid & cmask, copy % d.gs_c, copy / d.gs_c, oA, oB, oC);
  };
  float2 ra[8], rb[4];
  auto load_chunk = [&](int64_t oA, int64_t oB, int kc) {
    int64_t kA, kB;
    k_offsets(d, ot, kc, kA, kB);
#pragma unroll
    for (int j = 0; j < 8; ++j) ra[j] = load_c<SA>(d.A, oA + kA + gA[j]);
#pragma unroll
    for (int j = 0; j < 4; ++j) rb[j] = load_c<SB>(d.B, oB + kB + gB[j]);
  };
  auto store_chunk = [&](int buf) {
    float* An = Abuf + buf * kPersPair;
    float2* Bn = Bbuf + buf * (kPersPair / 2);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      An[lA[j]] = ra[j].x;
      An[lA[j] + kAPlane] = ra[j].y;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) Bn[lB[j]] = rb[j];
  };

  // The scale of a copy is read when its first tile is prefetched (before
  // those loads are issued), not at the top of the tile, where the wait for
  // it would also wait for the previous tile's output stores.
  Scale sc{0, 0}, nsc{0, 0};
  if (t < n_items) {
    int64_t oA, oB, oC;
    const int copy = (int)(t >> tb);
    nsc = compute_scale(d, copy % d.gs_c, copy / d.gs_c);
    item_offsets(t, oA, oB, oC);
    load_chunk(oA, oB, 0);
    store_chunk(0);
  }
  __syncthreads();
  int cur = -1;
  int cjs = 0, cjb = 0;
  bool wexp = false;
  float lmax = 0.f;
  int bad = 0;
  for (; t < n_items; t += G) {
    const int copy = (int)(t >> tb);
    const uint64_t bid = t & tmask;
    const int js = copy % d.gs_c, jb = copy / d.gs_c;
    if (copy != cur) {
      if (cur >= 0) finish_scale<256>(d, cjs, cjb, lmax, bad, red, wexp, sc);
      sc = nsc;
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

    Acc32<M3> acc;
    acc_zero(acc);

    // Every chunk but the last: the next chunk is loaded while this one is
    // multiplied.  The products run at raised wave priority, so that the
    // other workgroup's epilogue on this CU does not hold back their issue.
    for (int kc = 0; kc + 1 < n_kc; ++kc) {
      const int cb = kc & 1;
      load_chunk(oA, oB, kc + 1);
      __builtin_amdgcn_s_setprio(1);
      chunk_mfma<M3>(Abuf + cb * kPersPair, Bbuf + cb * (kPersPair / 2), lane, wm, wn, acc);
      __builtin_amdgcn_s_setprio(0);
      store_chunk(cb ^ 1);
      __syncthreads();
    }
    // The last chunk: meanwhile the next tile's first chunk is loaded, and
    // the scale inputs of its copy before it (unconditionally: loads and
    // uses under one condition keep the compiler's wait counts exact).
    ScaleIn nin{0, 0, 0.f, 0.f};
    if (next_tile) {
      const int cn = (int)((t + G) >> tb);
      nin = load_scale(d, cn % d.gs_c, cn / d.gs_c);
      int64_t pA, pB, pC;
      item_offsets(t + G, pA, pB, pC);
      load_chunk(pA, pB, 0);
    }
    {
      const int cb = (n_kc - 1) & 1;
      __builtin_amdgcn_s_setprio(1);
      chunk_mfma<M3>(Abuf + cb * kPersPair, Bbuf + cb * (kPersPair / 2), lane, wm, wn, acc);
      __builtin_amdgcn_s_setprio(0);
    }
    __syncthreads();
    // The next tile's first chunk goes to buffer 0 (free since the barrier
    // above) before this tile's output stores are issued: the vector memory
    // counter completes in issue order, so a wait for these loads placed
    // after the stores would also wait for the stores to finish.
    if (next_tile) {
      store_chunk(0);
      nsc = scale_of(d, nin);
    }

    // Epilogue: two halves of 64 rows staged from buffer 1 on; the first
    // barrier also publishes buffer 0.
    float* Cs = lds + kPersPair;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (wm == h) stage_acc<M3>(Cs, acc, lane, wn);
      __syncthreads();
      if (vec_c)
        store_half4<SC>(d, Cs, tcs, oC + g_lo4 + (h ? g_half : 0), c_lo4, tid, sc, lmax, bad);
      else
        store_half<SC, 8>(d, Cs, tcs, oC + g_lane + (h ? g_half : 0), c_lane, wave, sc, lmax, bad);
      __syncthreads();
    }
  }
  if (cur >= 0) finish_scale<256>(d, cjs, cjb, lmax, bad, red, wexp, sc);
}

// ---------------------------------------------------------------------------
// Long sums (K >= 256): one tile per workgroup, three workgroups per CU.  The
// per-tile overheads the persistent walk hides are small against hundreds of
// chunks, and the third resident wave per SIMD keeps the matrix cores busier
// in the chunk loop.  Same tiling and arithmetic; the output table is built in
// the operand buffers after the last chunk.  51.8 KB of LDS.
// ---------------------------------------------------------------------------
template <int SA, int SB, int SC, bool M3>
__global__ __launch_bounds__(256, M3 ? 2 : 3) void k_mfma32_tiles(StepDesc d) {
  __shared__ float lds[kMainFloats + 16];
  __shared__ OuterTab ot;
  __shared__ TileMap maps[3];  // A, B, C
  float* Abuf = lds;
  float2* Bbuf = reinterpret_cast<float2*>(lds + 2 * kABuf);
  float* red = lds + kMainFloats;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  // XCD-aware block order: consecutive logical tiles share the row tile of A
  // and land on the same XCD (blocks are dealt round-robin to the 8 XCDs).
  uint64_t bid = blockIdx.x;
  const uint64_t nblk = gridDim.x;
  if ((nblk & 7) == 0) bid = (bid & 7) * (nblk >> 3) + (bid >> 3);
  const uint64_t cmask = (uint64_t(1) << d.n_no) - 1;
  const uint64_t no = bid & cmask, ro = bid >> d.n_no;

  int64_t gA[8];
  int lA[8];
  int64_t gB[4];
  int lB[4];
  {
    TileTab* ta = reinterpret_cast<TileTab*>(lds);
    TileTab* tb = ta + 1;
    stage_maps(d, maps);
    build_outer(d, ot);
    __syncthreads();
    build_tab(maps[0], 1, 0, kAStride, *ta);
    build_tab(maps[1], 0, 1, kBStride, *tb);
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
  int hb = 0;
  for (int b = 0; b < maps[2].nbits; ++b)
    if (maps[2].role[b] == 0 && maps[2].cbit[b] == 6) hb = b;
  const int64_t g_half = int64_t(1) << maps[2].gpos[hb];

  const int n_kc = 1 << d.n_ko;
  float2 ra[8], rb[4];
  for (int copy = blockIdx.y; copy < d.copies; copy += gridDim.y) {
    const int js = copy % d.gs_c, jb = copy / d.gs_c;
    int64_t oA, oB, oC;
    outer_offsets(d, ot, ro, no, js, jb, oA, oB, oC);
    auto load_chunk = [&](int kc) {
      int64_t kA, kB;
      k_offsets(d, ot, kc, kA, kB);
#pragma unroll
      for (int j = 0; j < 8; ++j) ra[j] = load_c<SA>(d.A, oA + kA + gA[j]);
#pragma unroll
      for (int j = 0; j < 4; ++j) rb[j] = load_c<SB>(d.B, oB + kB + gB[j]);
    };
    auto store_chunk = [&](int buf) {
      float* An = Abuf + buf * kABuf;
      float2* Bn = Bbuf + buf * kBBuf;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        An[lA[j]] = ra[j].x;
        An[lA[j] + kAPlane] = ra[j].y;
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) Bn[lB[j]] = rb[j];
    };
    Acc32<M3> acc;
    acc_zero(acc);
    // The copy's scale inputs are read before the first chunk, whose wait
    // covers them; they are used only in the epilogue.
    ScaleIn sin = load_scale(d, js, jb);
    load_chunk(0);
    __syncthreads();  // the tables (or the previous copy's output) are done with
    store_chunk(0);
    __syncthreads();
    for (int kc = 0; kc < n_kc; ++kc) {
      const int cb = kc & 1;
      const bool more = kc + 1 < n_kc;
      if (more) load_chunk(kc + 1);
      __builtin_amdgcn_s_setprio(1);
      chunk_mfma<M3>(Abuf + cb * kABuf, Bbuf + cb * kBBuf, lane, wm, wn, acc);
      __builtin_amdgcn_s_setprio(0);
      if (more) store_chunk(cb ^ 1);
      __syncthreads();
    }

    // Epilogue: the C table and two halves of 64 rows in the operand buffers.
    float* Cs = lds;
    TileTab* tcs = reinterpret_cast<TileTab*>(lds + kCHalf);
    build_tab_skip(maps[2], hb, kCStride, 2, *tcs);
    asm volatile("" : "+v"(sin.eA), "+v"(sin.eB), "+v"(sin.mA), "+v"(sin.mB));
    const Scale sc = scale_of(d, sin);
    float lmax = 0.f;
    int bad = 0;
    __syncthreads();
    const int64_t g_lane = tcs->g[lane];
    const int c_lane = tcs->c[lane];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (wm == h) stage_acc<M3>(Cs, acc, lane, wn);
      __syncthreads();
      const int64_t gl = g_lane + (h ? g_half : 0);
#pragma unroll 4
      for (int j = 0; j < 16; ++j) {
        const int hi = 64 + wave + 4 * j;
        const int c = c_lane + tcs->c[hi];
        store_out<SC>(d, oC + gl + tcs->g[hi], make_float2(Cs[c], Cs[c + 1]), sc, lmax, bad);
      }
      __syncthreads();
    }
    finish_scale<256>(d, js, jb, lmax, bad, red, ro == 0 && no == 0, sc);
  }
}

#define RQC_MFMA_CASE(a, b, c)                                                          \
  if (sa == a && sb == b && sc == c) {                                                  \
    if (tiles_kernel && m3)                                                             \
      hipLaunchKernelGGL((k_mfma32_tiles<a, b, c, true>), grid, dim3(256), 0, s, d);   \
    else if (tiles_kernel)                                                              \
      hipLaunchKernelGGL((k_mfma32_tiles<a, b, c, false>), grid, dim3(256), 0, s, d);  \
    else if (m3)                                                                        \
      hipLaunchKernelGGL((k_mfma32<a, b, c, true>), grid, dim3(256), 0, s, d, n_items); \
    else                                                                                \
      hipLaunchKernelGGL((k_mfma32<a, b, c, false>), grid, dim3(256), 0, s, d, n_items); \
    return hipGetLastError();                                                           \
  }

hipError_t launch_mfma32_kernel(const StepDesc& d, int sa, int sb, int sc, dim3 grid,
                                hipStream_t s) {
  if (d.rt != 7 || d.nt != 6 || d.kt != 4) return hipErrorInvalidValue;
  const uint64_t n_items = (uint64_t)grid.x * (uint64_t)d.copies;
  // Sums of 256 or more complex terms: one tile per workgroup (grid = tiles
  // x copies as given); shorter sums: the persistent walk.
  const bool tiles_kernel = d.variant & kVarTiles ? true : (d.variant & kVarPersistent ? false : d.n_ko >= 4);
  const bool m3 = (d.variant & kVar4M) == 0;
  if (!tiles_kernel) grid = dim3((unsigned)(n_items < kMfmaGrid ? n_items : kMfmaGrid), 1);
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

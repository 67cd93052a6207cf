// Row-streaming contraction kernel (HBM-bound steps with a small B).
#include "kernels_dev.h"

namespace rqc {

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

hipError_t launch_rows_kernel(const StepDesc& d, int sa, dim3 grid, hipStream_t s) {
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

}  // namespace rqc

// Step dispatch and the small kernels of the path: slice / bitstring
// instantiation of the leaves (Section 5.1), the FP64 cross-slice reduction
// (Section 6.4), fills, and the unfused permute used as a baseline.
#include "kernels_dev.h"

namespace rqc {

hipError_t launch_step(const StepDesc& d0, int kernel, int sa, int sb, int sc, int lp_kind,
                       hipStream_t s) {
  StepDesc d = d0;
  d.sb_store = sb;
  d.sc_store = sc;
  const uint64_t tiles = (uint64_t)d.n_row_tiles * (uint64_t)d.n_col_tiles;
  const unsigned gy = (unsigned)(d.copies < 65535 ? d.copies : 65535);
  const dim3 grid((unsigned)tiles, gy);
  switch (kernel) {
    case KERN_MFMA16: return launch_mfma16_kernel(d, sa, sb, sc, lp_kind, grid, s);
    case KERN_MFMA: return launch_mfma32_kernel(d, sa, sb, sc, grid, s);
    case KERN_ROWS: return launch_rows_kernel(d, sa, grid, s);
    case KERN_SIMT: return launch_simt_kernel(d, sa, sb, sc, tiles, s);
  }
  return hipErrorInvalidValue;
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
// Bit permutation (the separate-permutation baseline, and the packing phase
// of the two-phase 16-bit contraction, which also converts to packed 16-bit
// words): tiles of 2^5 x 2^5 elements staged through LDS so that both the
// reads (low input bits) and the writes (low output bits) are contiguous.
// ---------------------------------------------------------------------------
struct PermDesc {
  int32_t rank;
  int8_t src_of_out[48];  // input bit feeding output bit i
};

template <int OUT>
__device__ __forceinline__ void put_elem(void* out, uint64_t i, float2 v);
template <>
__device__ __forceinline__ void put_elem<ST_C64>(void* out, uint64_t i, float2 v) {
  reinterpret_cast<float2*>(out)[i] = v;
}
template <>
__device__ __forceinline__ void put_elem<ST_F16>(void* out, uint64_t i, float2 v) {
  h2 o;
  o.x = (_Float16)v.x;
  o.y = (_Float16)v.y;
  reinterpret_cast<h2*>(out)[i] = o;
}
template <>
__device__ __forceinline__ void put_elem<ST_BF16>(void* out, uint64_t i, float2 v) {
  b2 o;
  o.x = (__bf16)v.x;
  o.y = (__bf16)v.y;
  reinterpret_cast<b2*>(out)[i] = o;
}

// Four consecutive output elements from one aligned group (the output's two
// lowest bits are the tile's): one 16-byte store of packed 16-bit words, or
// two of complex64.
template <int OUT>
__device__ __forceinline__ void put_elem4(void* out, uint64_t i, float2 a, float2 b, float2 c,
                                          float2 e) {
  if constexpr (OUT == ST_C64) {
    float4* o = reinterpret_cast<float4*>(reinterpret_cast<float2*>(out) + i);
    o[0] = make_float4(a.x, a.y, b.x, b.y);
    o[1] = make_float4(c.x, c.y, e.x, e.y);
  } else {
    uint32_t w[4];
    const float2 v[4] = {a, b, c, e};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if constexpr (OUT == ST_F16) {
        h2 x;
        x.x = (_Float16)v[j].x;
        x.y = (_Float16)v[j].y;
        w[j] = __builtin_bit_cast(uint32_t, x);
      } else {
        b2 x;
        x.x = (__bf16)v[j].x;
        x.y = (__bf16)v[j].y;
        w[j] = __builtin_bit_cast(uint32_t, x);
      }
    }
    *reinterpret_cast<uint4*>(reinterpret_cast<uint32_t*>(out) + i) = make_uint4(w[0], w[1], w[2], w[3]);
  }
}

template <int OUT>
__global__ __launch_bounds__(256) void k_permute(const float2* in, void* out, PermDesc p,
                                                 int lo_in, int lo_out, uint64_t n_blocks,
                                                 int vec) {
  // Tile = the lowest `lo_in` input bits  U  the lowest `lo_out` output bits.
  // The tile's element offsets (relative to the tile base) and LDS slots are
  // tabulated once per workgroup; workgroups stride over the tiles (a grid
  // has at most 2^32 work-items), each tile base a sum over its set bits.
  __shared__ float2 tile[1024 + 32];
  __shared__ int64_t toff_in[1024];   // input offset of tile element t (input order)
  __shared__ int16_t tslot[1024];     // its slot in output order
  __shared__ int64_t toff_out[1024];  // output offset of tile element t (output order)
  __shared__ int64_t bin[48], bout[48];  // input / output offset of outer bit i
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
  int no = 0;
  for (int i = 0; i < r; ++i)
    if (!((tmask >> i) & 1)) {
      if ((int)threadIdx.x == no) {
        bout[no] = int64_t(1) << i;
        bin[no] = int64_t(1) << p.src_of_out[i];
      }
      ++no;
    }
  const int nte = 1 << nt;
  // Tile bits sorted by their input bit: element t of the read phase.
  int tin[20];
  for (int i = 0; i < nt; ++i) tin[i] = p.src_of_out[tb[i]];
  for (int i = 0; i < nt; ++i) {
    int best = i;
    for (int j = i + 1; j < nt; ++j)
      if (tin[j] < tin[best]) best = j;
    const int x = tin[i];
    tin[i] = tin[best];
    tin[best] = x;
  }
  // Slot bit of read-order bit i: the position of its output bit in tb.
  int sbit[20];
  for (int i = 0; i < nt; ++i) {
    const int ob_i = out_of_in[tin[i]];
    sbit[i] = 0;
    for (int j = 0; j < nt; ++j)
      if (tb[j] == ob_i) sbit[i] = j;
  }
  for (int t = threadIdx.x; t < nte; t += blockDim.x) {
    int64_t a = 0;
    int slot = 0;
    for (int i = 0; i < nt; ++i)
      if ((t >> i) & 1) {
        a |= int64_t(1) << tin[i];
        slot |= 1 << sbit[i];
      }
    toff_in[t] = a;
    tslot[t] = (int16_t)slot;
    int64_t o = 0;
    for (int j = 0; j < nt; ++j)
      if ((t >> j) & 1) o |= int64_t(1) << tb[j];
    toff_out[t] = o;
  }
  __syncthreads();
  for (uint64_t blk = blockIdx.x; blk < n_blocks; blk += gridDim.x) {
    int64_t base_in = 0, base_out = 0;
    for (uint64_t b = blk; b; b &= b - 1) {
      const int i = __builtin_ctzll(b);
      base_in += bin[i];
      base_out += bout[i];
    }
    if (vec) {
      // Full tile, 16-byte aligned operands, tile bits 0 and 1 being input
      // bits 0, 1 and output bits 0, 1: thread u moves elements 4u .. 4u+3,
      // contiguous on both sides.
      const int t = 4 * (int)threadIdx.x;
      const float4* src = reinterpret_cast<const float4*>(in + base_in + toff_in[t]);
      const float4 v0 = src[0], v1 = src[1];
      const float2 e[4] = {make_float2(v0.x, v0.y), make_float2(v0.z, v0.w),
                           make_float2(v1.x, v1.y), make_float2(v1.z, v1.w)};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int sl = tslot[t + j];
        tile[sl + (sl >> 5)] = e[j];
      }
      __syncthreads();
      const int c = t + (t >> 5);
      put_elem4<OUT>(out, base_out + toff_out[t], tile[c], tile[c + 1], tile[c + 2], tile[c + 3]);
      __syncthreads();
      continue;
    }
    for (int t = threadIdx.x; t < nte; t += blockDim.x) {
      const int sl = tslot[t];
      tile[sl + (sl >> 5)] = in[base_in + toff_in[t]];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nte; t += blockDim.x)
      put_elem<OUT>(out, base_out + toff_out[t], tile[t + (t >> 5)]);
    __syncthreads();
  }
}

hipError_t launch_permute(const void* in, void* out, int rank, const int8_t* src_pos_of_out_bit,
                          hipStream_t s, int out_store) {
  PermDesc p;
  p.rank = rank;
  for (int i = 0; i < rank; ++i) p.src_of_out[i] = src_pos_of_out_bit[i];
  // Tile = the lo_in lowest input bits and the lo_out lowest output bits,
  // at most 10 bits (1024 elements): both grown alternately while the union
  // fits, so a permutation that keeps its low bits still gets full tiles.
  int out_of_in[48];
  for (int i = 0; i < rank; ++i) out_of_in[(int)p.src_of_out[i]] = i;
  auto tile_bits = [&](int li, int lo) {
    uint64_t m = 0;
    for (int i = 0; i < lo; ++i) m |= 1ull << i;
    for (int i = 0; i < li; ++i) m |= 1ull << out_of_in[i];
    return __builtin_popcountll(m);
  };
  int lo_in = 0, lo_out = 0;
  for (bool grew = true; grew;) {
    grew = false;
    if (lo_out < rank && tile_bits(lo_in, lo_out + 1) <= 10) ++lo_out, grew = true;
    if (lo_in < rank && tile_bits(lo_in + 1, lo_out) <= 10) ++lo_in, grew = true;
  }
  const int nt = tile_bits(lo_in, lo_out);
  const uint64_t blocks = 1ull << (rank - nt);
  // Eight workgroups per CU, each walking many tiles (its tables are built
  // once).
  const uint64_t grid = blocks < 2048 ? blocks : 2048;
  const float2* src = reinterpret_cast<const float2*>(in);
  // Vector form: full 1024-element tiles (the kernel runs 256 threads of four
  // elements), the two lowest input and output bits inside the tile, both
  // buffers 16-byte aligned.
  const int vec = nt == 10 && lo_in >= 2 && lo_out >= 2 &&
                  (reinterpret_cast<uintptr_t>(in) & 15) == 0 &&
                  (reinterpret_cast<uintptr_t>(out) & 15) == 0;
  if (out_store == ST_F16)
    hipLaunchKernelGGL(k_permute<ST_F16>, dim3((unsigned)grid), dim3(256), 0, s, src, out, p, lo_in,
                       lo_out, blocks, vec);
  else if (out_store == ST_BF16)
    hipLaunchKernelGGL(k_permute<ST_BF16>, dim3((unsigned)grid), dim3(256), 0, s, src, out, p,
                       lo_in, lo_out, blocks, vec);
  else
    hipLaunchKernelGGL(k_permute<ST_C64>, dim3((unsigned)grid), dim3(256), 0, s, src, out, p,
                       lo_in, lo_out, blocks, vec);
  return hipGetLastError();
}

}  // namespace rqc

namespace rqc {

// ---------------------------------------------------------------------------
// Statistics of an amplitude batch in FP64 (one workgroup, fixed summation
// order, so the result does not depend on timing): sum |a|^2, sum |a|^4, and
// the linear cross-entropy values derived from them; optionally the mean
// |a|^2 over sampled entries of the batch (bounds-checked: an index outside
// the batch makes that result NaN).
// ---------------------------------------------------------------------------
constexpr int kStatThreads = 1024;

__global__ __launch_bounds__(kStatThreads) void k_batch_stats(const double* amps, uint64_t n,
                                                               double dim, const uint64_t* samples,
                                                               uint64_t n_samples, double* out) {
  __shared__ double r1[kStatThreads], r2[kStatThreads], r3[kStatThreads];
  __shared__ int bad_any[kStatThreads];
  const int t = threadIdx.x;
  double s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int bad = 0;
  for (uint64_t i = t; i < n; i += kStatThreads) {
    const double re = amps[2 * i], im = amps[2 * i + 1];
    const double p = re * re + im * im;
    s1 += p;
    s2 += p * p;
  }
  for (uint64_t j = t; j < n_samples; j += kStatThreads) {
    const uint64_t i = samples[j];
    if (i >= n) {
      bad = 1;
      continue;
    }
    const double re = amps[2 * i], im = amps[2 * i + 1];
    s3 += re * re + im * im;
  }
  r1[t] = s1;
  r2[t] = s2;
  r3[t] = s3;
  bad_any[t] = bad;
  __syncthreads();
  for (int w = kStatThreads / 2; w > 0; w >>= 1) {
    if (t < w) {
      r1[t] += r1[t + w];
      r2[t] += r2[t + w];
      r3[t] += r3[t + w];
      bad_any[t] |= bad_any[t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    const double sum_p = r1[0], sum_p2 = r2[0];
    out[0] = sum_p;
    out[1] = sum_p2;
    out[2] = n ? dim * sum_p / (double)n - 1.0 : 0.0;  // all entries taken as samples
    out[3] = sum_p > 0.0 ? dim * sum_p2 / sum_p - 1.0 : 0.0;  // entries drawn with p = |a|^2
    out[4] = n_samples == 0 ? 0.0
             : (bad_any[0] ? __builtin_nan("") : dim * r3[0] / (double)n_samples - 1.0);
  }
}

hipError_t launch_batch_stats(const double* amps, uint64_t n, int n_qubits, const uint64_t* samples,
                              uint64_t n_samples, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_stats, dim3(1), dim3(kStatThreads), 0, s, amps, n,
                     ldexp(1.0, n_qubits), samples, n_samples, out);
  return hipGetLastError();
}

}  // namespace rqc

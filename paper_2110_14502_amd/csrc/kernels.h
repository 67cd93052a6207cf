// Device-side descriptors shared by the kernels and the executor.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace rqc {

// Storage type codes of an operand.
enum Store : int { ST_C64 = 0, ST_F16 = 1, ST_BF16 = 2 };

constexpr int kMaxTile = 16;   // tile bits per operand
constexpr int kMaxOuter = 44;  // outer bits per role

// Where each tile bit of one operand lives: its address bit in global
// memory and its coordinate bit in the LDS tile.  Tile bits are listed in
// increasing global address order so that consecutive lanes touch
// consecutive (or nearly consecutive) addresses.
struct TileMap {
  int32_t nbits;
  int8_t gpos[kMaxTile];  // address bit in the operand
  int8_t role[kMaxTile];  // 0 row (M), 1 col (N), 2 summed (K)
  int8_t cbit[kMaxTile];  // bit inside that role's tile index
};

// One pairwise contraction C[m,n] = sum_k A[m,k] B[k,n] with every index of
// dimension 2 and arbitrary bit layouts (the permutation is folded into the
// tile loads and the store, Section 5.4).  `copies` independent problems run
// side by side (slices x bitstrings of a group); copy j splits into
// js = j % gs_c and jb = j / gs_c.
struct StepDesc {
  const void* A;
  const void* B;
  void* C;
  // Per-copy power-of-two exponents and max-abs (reduced precision).
  const int32_t* expA;
  const int32_t* expB;
  int32_t* expC;
  const float* maxA;
  const float* maxB;
  float* maxC;
  int32_t* flag;  // per slice (js) non-finite flag, may be null
  float maxA_const, maxB_const;
  int64_t sA_s, sA_b, sB_s, sB_b, sC_s, sC_b;  // copy strides, elements
  int32_t eA_s, eA_b, eB_s, eB_b, eC_s, eC_b;  // copy strides, scale arrays
  int32_t gs_c, copies;
  int32_t rt, nt, kt;        // tile bits per role
  int32_t n_ro, n_no, n_ko;  // outer bits per role
  int32_t k_total;           // all summed bits
  int32_t track;             // 1: exponents / max-abs / flags maintained
  int32_t lp_out;            // 1: C stored in 16 bits (scaled)
  int32_t bias;              // test hook: subtracted from the storage shift
  int32_t dep_s_c;           // C varies with the slice (flag index js)
  int32_t flag_n;            // slices of the group flagged when it does not
  int32_t n_row_tiles, n_col_tiles;
  // Split-K: 2^ksplit blocks share one output tile, each summing a slice of
  // the K range into its own partial buffer P + split * p_stride (complex64,
  // laid out like C); a reduction kernel then forms C in fixed order.
  int32_t ksplit;
  float2* P;
  int64_t p_stride;
  int32_t sb_store, sc_store;  // storage codes of B and C (runtime copies)
  // Row kernel: output columns staged 2^ncb at a time; the remaining column
  // bits (their C positions in nh_C) select the chunk.
  int32_t ncb;
  int32_t vec_c;      // 1: tile bits 0 and 1 are C's address bits 0 and 1 (4-element stores)
  int32_t variant;    // kernel variant bits (kVar*), chosen per step by the tuner; 0 = default
  int8_t nh_C[16];
  int8_t ro_A[kMaxOuter], ro_C[kMaxOuter];
  int8_t no_B[kMaxOuter], no_C[kMaxOuter];
  int8_t ko_A[kMaxOuter], ko_B[kMaxOuter];
  TileMap tA, tB, tC;
};

// Leaf instantiation (slice and bitstring binding).
struct LeafJob {
  int64_t src;        // element offset of the base tensor in the leaf store
  int64_t dst;        // element offset of copy 0 in the destination
  int32_t rank;       // bits of the instantiated tensor
  int32_t nsel;       // selector bits
  int8_t pos[8];      // base address bit of output bit i (LSB first)
  int8_t sel_pos[8];  // base address bit of selector s
  int16_t sel_src[8]; // >= 0: slice bit index; < 0: -(closed column) - 1
  int32_t dep_s, dep_b;  // which copy dimensions the leaf varies along
  int32_t dst_store;  // Store code of the destination
  int32_t out_s, out_b;  // copy strides of the destination (elements)
};

// Kernel variant bits of a step (StepDesc::variant).  FP32 matrix-core
// kernel: the complex products as four real products on the real expansion
// of B (kVar4M) or as three (the default); one tile per workgroup
// (kVarTiles) or the persistent walk (kVarPersistent); neither: per-tile for
// sums of 256 or more.
// Any kernel: kVarFP32Math keeps the arithmetic in FP32 on 16-bit stored
// operands (the row kernel would otherwise use the 16-bit matrix cores).
// 16-bit matrix-core kernel: kVarStream streams A past a resident B tile
// (sums of 32..128 terms, A stored in 16 bits).
// kVarSwap: the operands are exchanged (the kernel's A is the step's B), so
// that a step with a 128-column output takes one row tile of the kernel and
// its large operand is read once instead of once per column tile.  The
// descriptor is built from (B, A) and the executor binds B's data as A.
constexpr int32_t kVar4M = 1, kVarTiles = 2, kVarPersistent = 4, kVarFP32Math = 8,
                  kVarStream = 16, kVarSwap = 32;

// Kernel kinds of a step.
// KERN_MFMA16: FP16/BF16 matrix cores, 32 complex k per chunk (reduced
// precision only).
enum Kernel : int { KERN_SIMT = 0, KERN_MFMA = 1, KERN_ROWS = 2, KERN_MFMA16 = 3 };

// Launchers (kernels.hip).  All return hipError_t of the launch.
// The 16-bit matrix-core kernel's vector path: the two lowest tile bits of A
// and of B are their two lowest address bits and summed indices 0 and 1.
inline bool lp_vec_layout(const StepDesc& d) {
  return d.tA.nbits >= 2 && d.tB.nbits >= 2 && d.tA.gpos[0] == 0 && d.tA.gpos[1] == 1 &&
         d.tB.gpos[0] == 0 && d.tB.gpos[1] == 1 && d.tA.role[0] == 2 && d.tA.role[1] == 2 &&
         d.tB.role[0] == 2 && d.tB.role[1] == 2 && d.tA.cbit[0] == 0 && d.tA.cbit[1] == 1 &&
         d.tB.cbit[0] == 0 && d.tB.cbit[1] == 1;
}

hipError_t launch_step(const StepDesc& d, int kernel, int sa, int sb, int sc, int lp_kind,
                       hipStream_t s);
hipError_t launch_leaves(const LeafJob* jobs_dev, int n_jobs, const void* leaf_store,
                         void* dst_base, const uint64_t* slice_ids, const uint8_t* closed_bits,
                         int n_closed, int gs, int gb, int max_rank, hipStream_t s);
hipError_t launch_slice_sum(const void* root, int root_store, const int32_t* root_exp,
                            int64_t root_s, int64_t root_b, int32_t re_s, int32_t re_b,
                            int dep_s, int dep_b, int n_elems, int gs, int gb,
                            const int32_t* flags, double* out, double* per_slice,
                            int64_t ps_row0, int64_t n_batch_total, int64_t b0, int first,
                            hipStream_t s);
// FP64 statistics of an amplitude batch: out[0] = sum |a|^2, out[1] = sum
// |a|^4, out[2..4] the linear cross-entropy values (see rqc_batch_xeb).
hipError_t launch_batch_stats(const double* amps, uint64_t n, int n_qubits, const uint64_t* samples,
                              uint64_t n_samples, double* out, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_f64(double* p, double v, int64_t n, hipStream_t s);
hipError_t launch_add_f64(double* dst, const double* src, int64_t n, hipStream_t s);
// Bit permutation out (bit i fed by input bit src_pos_of_out_bit[i]) of a
// complex64 tensor; out_store ST_F16 / ST_BF16 writes packed 16-bit (re, im)
// words (round to nearest, no scaling).
hipError_t launch_permute(const void* in, void* out, int rank, const int8_t* src_pos_of_out_bit,
                          hipStream_t s, int out_store = ST_C64);

// 16-bit matrix-core GEMM of the two-phase long-sum contraction
// (k_gemm16.hip): A [copy][2^m rows][2^k] and B [copy][2^n columns][2^k]
// packed 16-bit (re, im) words, summed index lowest and in the same order in
// both; C (complex64) element (row r, column c) of copy j at
// j * sC + sum_b bit_b(r) 2^crow[b] + sum_b bit_b(c) 2^ccol[b].
constexpr int kGemm16M = 256, kGemm16N = 128, kGemm16K = 32;  // tile rows, complex columns, chunk k
struct Gemm16Desc {
  const uint32_t* A;
  const uint32_t* B;
  void* C;
  int64_t sA, sB, sC;  // copy strides: words of A and B (0 = shared), complex elements of C
  int32_t m, n, k;     // bits: rows (>= 8), columns (>= 7), summed (>= 5)
  int32_t copies;
  int32_t ksplit;      // the sum split 2^ksplit ways (partials in P, then reduced)
  float2* P;           // partials [copy][split][row][column], when ksplit > 0
  int8_t crow[40];
  int8_t ccol[40];
};
hipError_t launch_gemm16(const Gemm16Desc& d, int lp_kind, hipStream_t s);
hipError_t launch_cgemm(int64_t M, int64_t N, int64_t K, const void* A, const void* B, void* C,
                        hipStream_t s);

}  // namespace rqc

/*
 * rqc.h -- C ABI of the sliced tensor-network amplitude engine for random
 * quantum circuits on one AMD MI355X (gfx950).
 *
 * The method (paper: "Closing the 'Quantum Supremacy' Gap", SC'21):
 *   - a circuit becomes a tensor network, one tensor per gate (Section 3.2,
 *     tensor approach);
 *   - a contraction path is searched (Section 5.2) and a set of wires is
 *     sliced: each slice fixes those wires to one assignment of values and
 *     the independent slice results are summed (Section 5.1);
 *   - every contraction step is an index permutation followed by a complex
 *     matrix multiply (Section 5.4), here fused into one GPU kernel;
 *   - a batch of "open" qubits yields 2^n_open amplitudes per contraction
 *     (Section 5.1, last paragraph);
 *   - reduced precision with adaptive scaling (Section 5.5);
 *   - a final reduction of the slice results (Section 6.4).
 *
 * Conventions
 *   - Complex numbers are stored interleaved (re, im).
 *   - Bit strings: qubit q of an n-qubit state is bit (n-1-q) of the state
 *     index.  An amplitude batch has 2^n_open entries; bit i of the entry
 *     index is the value of open_qubits[i] (the first open qubit is the
 *     least significant bit).  Closed bits are given in increasing qubit
 *     order of the closed qubits.
 *   - A canonical wire (q, s), s >= 1, is the wire of qubit q leaving the
 *     s-th two-qubit gate that acts on q.  Slice id bit j is the value of the
 *     j-th sliced wire in plan order.
 *   - Device pointers come from the caller (for example torch tensors); the
 *     library never frees caller memory.  Handles belong to the library
 *     until their destroy call.  A plan is not thread-safe; a server is.
 *   - Every function returns RQC_OK (0) or a negative rqc_status; no C++
 *     exception crosses this boundary.  rqc_last_error() gives a message for
 *     the last failure on the calling thread.  Errors of asynchronous device
 *     work surface at the next call that synchronises (for example
 *     rqc_contract_status).
 */
#ifndef RQC_H
#define RQC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rqc_status;
#define RQC_OK            0
#define RQC_EINVAL       -1  /* invalid argument */
#define RQC_ENOMEM       -2  /* host allocation failed */
#define RQC_EHBM         -3  /* device memory given (or budget) too small */
#define RQC_EDEVICE      -4  /* HIP runtime error */
#define RQC_EUNSUPPORTED -5  /* valid request the library does not support */
#define RQC_ENUMERIC     -6  /* non-finite values persisted after FP32 rerun */

/* Gate kinds.  Matrices are M[out][in]; two-qubit basis index 2*b(q0)+b(q1).
 * FSIM(theta, phi) = [[1,0,0,0],[0,c,-is,0],[0,-is,c,0],[0,0,0,e^{-i phi}]]
 * with c = cos(theta), s = sin(theta) (the fSim gate of Section 5.2);
 * SQRT_G satisfies SQRT_G^2 = -i G for G in {X, Y, W=(X+Y)/sqrt(2)}. */
enum {
  RQC_GATE_H = 0,
  RQC_GATE_SQRT_X = 1,
  RQC_GATE_SQRT_Y = 2,
  RQC_GATE_SQRT_W = 3,
  RQC_GATE_FSIM = 4,
  RQC_GATE_U1 = 5,  /* explicit 2x2 matrix in u[0..7] (re, im row-major) */
  RQC_GATE_U2 = 6   /* explicit 4x4 matrix in u[0..31] */
};

typedef struct rqc_gate {
  int32_t kind;
  int32_t q0;
  int32_t q1;   /* -1 for single-qubit gates */
  int32_t reserved;
  double theta;
  double phi;
  double u[32];
} rqc_gate;

/* Arithmetic of the contraction steps.  F32: complex64 storage, FP32 MFMA.
 * F16 / BF16: large intermediates stored as complex half / bfloat16 with a
 * per-slice power-of-two exponent (adaptive scaling, Section 5.5), FP32
 * accumulation; small tensors stay complex64.  The cross-slice sum is FP64
 * in every mode. */
enum { RQC_F32 = 0, RQC_F16 = 1, RQC_BF16 = 2 };

typedef struct rqc_circuit rqc_circuit;
typedef struct rqc_network rqc_network;
typedef struct rqc_plan rqc_plan;
typedef struct rqc_server rqc_server;
typedef void* rqc_stream; /* a hipStream_t; NULL is the default stream */

/* ---- circuit and network (Section 3.2, tensor approach) ---------------- */

/* Copy n_gates gates applied in array order to |0...0> of n_qubits qubits.
 * EINVAL for a qubit index out of range, q0 == q1, or an unknown kind. */
rqc_status rqc_circuit_create(int32_t n_qubits, const rqc_gate* gates,
                              size_t n_gates, rqc_circuit** out);
void rqc_circuit_destroy(rqc_circuit* c);

/* Tensor network of <b|U|0> with the listed qubits left open.  Single-qubit
 * gates and the input |0> are absorbed forward into the next two-qubit gate
 * of their qubit; each qubit's final single-qubit gates and its output
 * (projection onto the closed bit, or the open index) into its last
 * two-qubit gate.  The circuit may be destroyed afterwards. */
rqc_status rqc_network_create(const rqc_circuit* c, const int32_t* open_qubits,
                              int32_t n_open, rqc_network** out);
void rqc_network_destroy(rqc_network* n);

/* ---- plan: contraction path and slicing (Sections 5.1-5.2) ------------- */

typedef struct rqc_plan_opts {
  int32_t max_log2_elems; /* bound on any per-slice intermediate, log2 of
                             elements; 0 = no bound */
  int32_t n_sliced;       /* -1: as few wires as the bound needs; else exact */
  int32_t path_trials;    /* randomized path searches; 0 = default (256) */
  int32_t reconf_rounds;  /* subtree re-optimisation sweeps; -1 = default */
  uint64_t seed;
  int32_t n_forced;       /* wires that must be sliced, first in slice order */
  const int32_t* forced_wires; /* n_forced (qubit, segment) pairs */
  int32_t lp_min_log2;    /* RQC_F16 stores intermediates of at least
                             2^lp_min_log2 elements per slice in 16 bits;
                             0 = default (14) */
  int32_t bf16_min_log2;  /* the same for RQC_BF16, whose 8-bit significand
                             rounds more per stored stage; 0 = default (24) */
  /* Slice share (Section 5.1: slices are independent sub-tasks, so a device
   * can own a contiguous range of them).  0: every sliced wire is enumerated
   * by the slice ids of rqc_contract (at most 62 wires).  L > 0: only the
   * first L sliced wires (slice bits 0..L-1, L <= 62) are enumerated; sliced
   * wire L+i is fixed to share_bits[i] (0 for i >= n_share_bits), so the
   * plan computes the 2^L slices whose high slice bits are share_bits.  Every
   * subtree that carries only fixed wires is contracted once at bind.  With
   * a share the full slicing may have more than 62 wires.  share_bits is
   * read during rqc_plan_create only. */
  int32_t n_local_sliced;
  int32_t n_share_bits;
  const uint8_t* share_bits;
  int32_t restarts;       /* independent searches with seeds derived from
                             `seed`; the plan with the lowest estimated time
                             is kept; 0 = 1 */
  int32_t precision_policy; /* which intermediates use 16-bit storage and
                               arithmetic in RQC_F16 / RQC_BF16 calls, see
                               RQC_POLICY_*; 0 = RQC_POLICY_SIZE */
  uint64_t hbm_budget_bytes; /* 0: unbounded.  Otherwise the plan's resident
                                bytes plus the workspace of one slice and one
                                bitstring in FP32 must fit, else EHBM */
} rqc_plan_opts;

/* Precision policies (Section 5.5: the parts of the network near the slice
 * cuts are the most sensitive to reduced precision).
 *   SIZE: an intermediate is stored (and multiplied) in 16 bits when it has
 *         at least 2^lp_min_log2 (FP16) / 2^bf16_min_log2 (BF16) elements
 *         per slice;
 *   CALIBRATED: as SIZE, then rqc_plan_calibrate measures each step's
 *         sensitivity on one slice and keeps the most sensitive steps in
 *         complex64 until the estimated error meets the requested bound;
 *   STORAGE: 16-bit storage by the size rule, every product in FP32 on the
 *         converted values (half storage, FP32 arithmetic: halves the bytes
 *         of memory-bound steps at FP32 rounding of the arithmetic). */
enum { RQC_POLICY_SIZE = 0, RQC_POLICY_CALIBRATED = 1, RQC_POLICY_STORAGE = 2 };

void rqc_plan_opts_default(rqc_plan_opts* o);

/* Search a path, slice it and lay out every step.  Host only. */
rqc_status rqc_plan_create(const rqc_network* n, const rqc_plan_opts* opts,
                           rqc_plan** out);
void rqc_plan_destroy(rqc_plan* p);

typedef struct rqc_plan_info_s {
  int32_t n_qubits, n_open, n_closed, n_sliced;
  uint64_t n_slices;
  int32_t n_leaves, n_steps;       /* steps = pairwise contractions */
  int32_t n_invariant_steps;       /* steps shared by all slices and bitstrings */
  int32_t max_log2_elems;          /* largest per-slice intermediate */
  double flops_per_slice;          /* steps that depend on the sliced wires, per slice
                                      and bitstring; 8 real flops per complex
                                      multiply-add */
  double flops_invariant;          /* once per plan (slice-invariant subtrees) */
  double bytes_per_slice;          /* complex64 bytes read+written per slice */
  double log2_total_flops;         /* all slices, one bitstring */
  double flops_per_bitstring;      /* steps that depend on the closed bits but on
                                      no sliced wire: once per bitstring, shared
                                      by all slices */
} rqc_plan_info_t;

rqc_status rqc_plan_info(const rqc_plan* p, rqc_plan_info_t* out);

/* Per-step shape: m, n, k are the numbers of row, column and summed index
 * bits of C[m,n] = A[m,k] B[k,n]; kernel 0 = generic SIMT, 1 = FP32 MFMA,
 * 2 = row streaming, 3 = 16-bit MFMA. */
typedef struct rqc_step_info {
  int32_t m, n, k;
  int32_t kernel;         /* kernel of the step in RQC_F32 calls */
  int32_t kernel_lp;      /* kernel of the step in RQC_F16 / RQC_BF16 calls */
  int32_t depends_on_slice, depends_on_bits;
  int32_t lp_output;      /* output stored in 16 bits in RQC_F16 calls */
  int32_t lp_output_bf16; /* output stored in 16 bits in RQC_BF16 calls */
  int32_t reserved;
  double flops;           /* 8 * 2^(m+n+k) */
  double bytes_c64;       /* 8 * (|A| + |B| + |C|) */
} rqc_step_info;

rqc_status rqc_plan_get_step(const rqc_plan* p, int32_t i, rqc_step_info* out);

/* JSON description: sliced canonical wires (slice-bit order), open and
 * closed qubits, the contraction tree and every step's layouts.  Writes at
 * most cap bytes (NUL-terminated when it fits); *needed gets the full size
 * including the NUL. */
rqc_status rqc_plan_export_json(const rqc_plan* p, char* buf, size_t cap,
                                size_t* needed);

/* ---- device residency and contraction ---------------------------------- */

/* Device bytes the plan keeps resident: leaf tensors and slice-invariant
 * intermediates for all three precisions. */
rqc_status rqc_plan_resident_bytes(const rqc_plan* p, size_t* bytes);

/* Upload leaves into caller memory (dev_ptr, 256-byte aligned, at least
 * rqc_plan_resident_bytes) and compute the slice-invariant subtrees on
 * `stream` (the call waits for them).  The memory must stay valid until the
 * plan is destroyed or re-bound. */
rqc_status rqc_plan_bind_memory(rqc_plan* p, void* dev_ptr, size_t bytes,
                                rqc_stream stream);

/* Workspace for a contraction of n_ids slices and n_batch bitstrings:
 * *min_bytes runs one slice and one bitstring at a time, *pref_bytes runs
 * everything in one group.  More workspace lets more slices run together. */
rqc_status rqc_contract_workspace(const rqc_plan* p, uint64_t n_ids,
                                  uint64_t n_batch, int32_t prec,
                                  size_t* min_bytes, size_t* pref_bytes);

/* Amplitudes of n_batch bitstrings, summed over the given slices
 * (Section 5.1: slices are independent sub-tasks; Section 6.4: the final
 * reduction, here in FP64 in a fixed order).
 *   slice_ids   host array of n_ids slice ids (NULL with n_ids = 0: all);
 *   closed_bits host array n_batch x n_closed (0/1 bytes);
 *   workspace   device memory, 256-byte aligned, ws_bytes >= min_bytes;
 *   out         device, n_batch x 2^n_open x 2 doubles (overwritten);
 *   per_slice   device or NULL: n_ids x n_batch x 2^n_open x 2 doubles
 *               holding each slice's own contribution.
 * All work is enqueued on `stream` as one graph launch (cached per shape);
 * the call returns before it finishes.  Slices whose reduced-precision run
 * produced a non-finite value are re-run in FP32 when rqc_contract_status
 * is called. */
rqc_status rqc_contract(rqc_plan* p, const uint64_t* slice_ids, uint64_t n_ids,
                        const uint8_t* closed_bits, uint64_t n_batch,
                        int32_t prec, void* workspace, size_t ws_bytes,
                        double* out, double* per_slice, rqc_stream stream);

typedef struct rqc_run_report {
  uint64_t n_slices;       /* slices summed */
  uint64_t fp32_reruns;    /* slices re-run in FP32 (filter of Section 5.5) */
  int32_t slices_per_group, bits_per_group;
  int32_t graph_reused;    /* 1 when the cached graph was launched again */
  int32_t reserved;
  double flops;            /* algorithmic flops of the call */
} rqc_run_report;

/* Synchronise `stream`, re-run flagged slices in FP32 (synchronously) and
 * report.  A slice is flagged per group of bitstrings; its FP32 result is
 * added for exactly the bitstrings whose sum skipped it.  ENUMERIC if
 * non-finite values remain after the re-run (or appear in an FP32 call). */
rqc_status rqc_contract_status(rqc_plan* p, rqc_stream stream,
                               rqc_run_report* out);

/* ---- one pairwise contraction (Section 5.4) ----------------------------- */

/* C = sum over shared labels of A * B for tensors with every dimension 2.
 * labels_x lists operand x's index labels from the most significant address
 * bit to the least significant one (numpy C order of shape (2,)*rank).  A
 * label in A and B but not in C is summed; labels_c must be exactly the
 * other labels.  A, B, C are device complex64 arrays (float2); batch_count
 * independent problems lie at strides (elements) stride_a, stride_b,
 * stride_c (0 = shared).  Ranks up to 40.  kernel: -1 auto, 0 generic SIMT,
 * 1 MFMA (needs m >= 7, n >= 6, k >= 4), 2 row streaming (needs the summed
 * labels to be the lowest bits of A and of B in the same order, k <= 5,
 * n <= 6); an unmet condition falls back to the generic kernel.  prec
 * RQC_F16 / RQC_BF16 runs dense shapes (m >= 7, n >= 6, k >= 5) on the
 * 16-bit matrix cores (operands rounded to 16 bits, FP32 accumulation,
 * complex64 in and out); other shapes and RQC_F32 use FP32 arithmetic. */
rqc_status rqc_pair_contract(const int32_t* labels_a, int32_t rank_a,
                             const int32_t* labels_b, int32_t rank_b,
                             const int32_t* labels_c, int32_t rank_c,
                             const void* A, const void* B, void* C,
                             int32_t batch_count, int64_t stride_a,
                             int64_t stride_b, int64_t stride_c,
                             int32_t kernel, int32_t prec, rqc_stream stream);

/* Device workspace that rqc_pair_contract_ws needs for this call, in bytes
 * (*bytes = 0: the call runs without one, exactly as rqc_pair_contract).
 * Nonzero only for automatic kernel choice (kernel -1) in RQC_F16 /
 * RQC_BF16 when the sum has at least 2^8 terms and m >= 8, n >= 7 (at least
 * one 256 x 128 output tile): then the call takes the two-phase long-sum
 * form of Sections 5.4 and 5.5 (each operand permuted into a plain
 * [free][summed] matrix of packed 16-bit values, then a 16-bit matrix-core
 * GEMM that writes C in its own layout); the workspace holds the two packed
 * operands, 4 bytes per element per distinct operand copy (a copy stride of
 * 0 shares one copy), and, when the output has fewer than 1024 tiles of
 * 256 x 128, FP32 partial outputs of a split sum (8 bytes per output
 * element per split, summed afterwards in split order).  Also nonzero for
 * RQC_F32 calls that run on the generic kernel (kernel -1 or 0) with output
 * tiles too few to fill the GPU and a long sum: the sum is split over
 * workgroups (as for plan steps) and the workspace holds the complex64
 * partial outputs, 8 bytes per output element per copy per split, added
 * afterwards in split order.  Arguments as in rqc_pair_contract; EINVAL on
 * bad labels or ranks. */
rqc_status rqc_pair_workspace_bytes(const int32_t* labels_a, int32_t rank_a,
                                    const int32_t* labels_b, int32_t rank_b,
                                    const int32_t* labels_c, int32_t rank_c,
                                    int32_t batch_count, int64_t stride_a,
                                    int64_t stride_b, int32_t kernel, int32_t prec,
                                    uint64_t* bytes);

/* rqc_pair_contract with a caller-owned device workspace of ws_bytes
 * (256-byte aligned, at least rqc_pair_workspace_bytes; its contents are
 * overwritten).  Operands are rounded to 16 bits without scaling (values
 * must lie in the 16-bit range) and products accumulate in FP32; C is
 * complex64.  With a batch, stride_c must be at least one output.  A split
 * FP32 sum on the generic kernel needs a batch's outputs back to back
 * (stride_c = 2^rank_c); with another stride the call runs unsplit.  Calls
 * that need no workspace behave exactly as rqc_pair_contract. */
rqc_status rqc_pair_contract_ws(const int32_t* labels_a, int32_t rank_a,
                                const int32_t* labels_b, int32_t rank_b,
                                const int32_t* labels_c, int32_t rank_c,
                                const void* A, const void* B, void* C,
                                int32_t batch_count, int64_t stride_a,
                                int64_t stride_b, int64_t stride_c,
                                int32_t kernel, int32_t prec, void* workspace,
                                uint64_t ws_bytes, rqc_stream stream);

/* Bit permutation of a complex64 tensor: out (labels_out) = in (labels_in).
 * The separate-permutation baseline of Section 5.4. */
rqc_status rqc_permute(const int32_t* labels_in, const int32_t* labels_out,
                       int32_t rank, const void* in, void* out,
                       rqc_stream stream);

/* Plain row-major complex64 GEMM C[M,N] = A[M,K] B[K,N] on MFMA, used with
 * rqc_permute as the unfused baseline. */
rqc_status rqc_cgemm(int64_t M, int64_t N, int64_t K, const void* A,
                     const void* B, void* C, rqc_stream stream);

/* rqc_contract for callers that cannot allocate device memory (code under a
 * HIP graph capture of their own, tight serving loops, harnesses that forbid
 * allocation).  Same arguments and results as rqc_contract without the
 * workspace: the call's workspace lives in a static device array of
 * rqc_contract_noalloc_scratch_bytes() bytes (256 MiB) that each GPU the
 * library runs on holds until the process ends; its address is looked up
 * once per device.  The kernels are launched directly on `stream` (no graph
 * is captured or cached).  EHBM, before anything is launched, when even one
 * slice and one bitstring at a time do not fit the scratch.  Every call on a
 * GPU shares that GPU's array, which keeps the last call's contents: calls
 * that overlap on one GPU (other streams or threads, including the FP32
 * re-run inside rqc_contract_status) race and must be serialised by the
 * caller.  Complete each call with rqc_contract_status before the next. */
rqc_status rqc_contract_noalloc(rqc_plan* p, const uint64_t* slice_ids,
                                uint64_t n_ids, const uint8_t* closed_bits,
                                uint64_t n_batch, int32_t prec, double* out,
                                double* per_slice, rqc_stream stream);
uint64_t rqc_contract_noalloc_scratch_bytes(void);

/* ---- large correlated batches: linear cross-entropy ------------------- */

/* Statistics of an amplitude batch of an n_qubits circuit, in FP64 on the
 * device (Appendix A: a bunch of 2^21 correlated amplitudes, fixing some
 * qubits and exhausting the others, scored by the linear cross-entropy
 * benchmark).  amps: device, n_amps x {re, im} doubles (the output of
 * rqc_contract); samples: device array of n_samples entry indices or NULL.
 * Writes 5 doubles to the device array out:
 *   out[0] = sum |a|^2 over the batch; out[1] = sum |a|^4;
 *   out[2] = 2^n_qubits * mean |a|^2 - 1  (every entry taken as a sample);
 *   out[3] = 2^n_qubits * sum |a|^4 / sum |a|^2 - 1  (the expected linear
 *            cross-entropy of entries drawn with probability |a|^2 / sum,
 *            i.e. ideal sampling within the batch);
 *   out[4] = 2^n_qubits * mean over samples of |a|^2 - 1 (0 without
 *            samples; NaN if a sample index is >= n_amps).
 * Enqueued on `stream`; one workgroup, fixed summation order. */
rqc_status rqc_batch_xeb(const double* amps, uint64_t n_amps, int32_t n_qubits,
                         const uint64_t* samples, uint64_t n_samples,
                         double* out, rqc_stream stream);

/* ---- serving: continuous batching of amplitude requests ---------------- */

typedef struct rqc_server_opts {
  void* device_pool;          /* caller-owned device memory the server
                                 sub-allocates (256-byte aligned) */
  uint64_t hbm_budget_bytes;  /* size of device_pool: plans, workspaces and
                                 outputs of admitted requests must fit */
  int32_t max_inflight;       /* contraction calls on the device at once */
  int32_t n_streams;          /* HIP streams used (default priority) */
  int32_t max_batch;          /* requests of one plan merged into one call */
  int32_t device;             /* HIP device ordinal */
} rqc_server_opts;

typedef struct rqc_request {
  int32_t n_qubits;
  int32_t n_open;
  const rqc_gate* gates;      /* copied at submit */
  uint64_t n_gates;
  const int32_t* open_qubits; /* copied */
  const uint8_t* closed_bits; /* one bitstring, n_qubits - n_open bytes */
  int32_t prec;
  int32_t max_log2_elems;     /* plan bound, 0 = default (26) */
  uint64_t plan_key;          /* requests with equal nonzero keys share a plan */
  uint64_t seed;
} rqc_request;

typedef struct rqc_result {
  uint64_t ticket;
  rqc_status status;
  int32_t n_open;
  double* amplitudes;         /* 2^n_open x 2 doubles, owned by the server
                                 until rqc_server_release(ticket) */
  double t_submit, t_start, t_done; /* seconds on the server clock */
  uint64_t fp32_reruns;
} rqc_result;

rqc_status rqc_server_create(const rqc_server_opts* o, rqc_server** out);
/* Queue a request; never blocks on the device.  Requests are admitted in
 * arrival order as device memory and in-flight slots free up; requests that
 * share a plan (equal nonzero plan_key, or identical circuit, open qubits
 * and precision) and are waiting together run as one batched contraction.
 * A request whose plan alone cannot fit the budget finishes with EHBM. */
rqc_status rqc_server_submit(rqc_server* s, const rqc_request* r,
                             uint64_t* ticket);
/* Collect finished results (up to cap). */
rqc_status rqc_server_poll(rqc_server* s, rqc_result* out, size_t cap,
                           size_t* n);
rqc_status rqc_server_release(rqc_server* s, uint64_t ticket);
/* Block until every submitted request has finished. */
rqc_status rqc_server_drain(rqc_server* s);
typedef struct rqc_server_stats {
  uint64_t submitted, completed, rejected;
  uint64_t plans_built, plans_reused;
  uint64_t peak_bytes, max_inflight_seen;
} rqc_server_stats;
rqc_status rqc_server_get_stats(rqc_server* s, rqc_server_stats* out);
void rqc_server_destroy(rqc_server* s);

/* ---- execution tuning ---------------------------------------------------- */

/* Per-step kernel tuning (Section 5.4 designs a kernel per contraction case;
 * here the choice per step is measured).  For every step of the plan with
 * more than one valid (kernel, variant) pair -- the FP32 matrix-core kernel
 * with three or four real products per complex product, per-tile or
 * persistent, and either kernel with the operands exchanged where B has
 * the fewer free indices and at least seven; the row-streaming kernel where
 * its conditions hold -- each
 * pair is timed with HIP events on `stream` for the group of slices and
 * bitstrings that a call of n_ids slices (0 = all) and n_batch bitstrings
 * in precision `prec` gets in this workspace, and the fastest is kept for
 * that precision.  The workspace (256-byte aligned, at least the call's
 * minimum) is overwritten; the call synchronises `stream`.  cache_path
 * (optional, NULL or ""): a text file of "signature kernel variant" lines
 * (signature: the step's shape and layouts up to renaming of labels, its
 * operand storage and the group size), read first and rewritten after;
 * steps found in it are not timed.  Results do not depend on the choices
 * beyond FP32 rounding. */
typedef struct rqc_tune_report {
  int32_t steps;        /* steps with more than one candidate */
  int32_t timed;        /* of which timed on the device */
  int32_t cached;       /* of which taken from the cache file */
  int32_t changed;      /* steps whose choice differs from the previous one */
  double ms_default;    /* timed steps: summed time of the previous choices */
  double ms_tuned;      /* timed steps: summed time of the chosen ones */
} rqc_tune_report;

rqc_status rqc_plan_autotune(rqc_plan* p, int32_t prec, uint64_t n_ids,
                             uint64_t n_batch, void* workspace, size_t ws_bytes,
                             const char* cache_path, rqc_stream stream,
                             rqc_tune_report* out);

/* Precision pre-analysis for RQC_F16 / RQC_BF16 calls (Section 5.5: the
 * parts of the network near the slice cuts are the most sensitive).  Slice
 * `slice_id` with closed bits `closed_bits` (host, n_closed bytes) is
 * contracted in FP32, then once per candidate step (one whose output the size
 * rule stores in 16 bits, or whose kernel uses the 16-bit matrix cores) with
 * only that step in reduced precision; its error against the FP32 result,
 * max |a - a32| / max(RMS(a32), err_floor), is its sensitivity.  Steps are
 * then put in reduced precision from the least sensitive on while the root
 * sum of squares of their errors stays <= target_err; the others store
 * complex64 and multiply in FP32 in calls of precision `prec`.  The whole
 * assignment is checked on the same slice (dropping the most sensitive kept
 * step while the measured error is above the target).  err_floor is for
 * slices whose value cancels far below their natural size (for example
 * 2^-(n+S)/2 for S sliced wires); 0 measures against the slice's own RMS.
 * The workspace must hold one slice and one bitstring in FP32 plus
 * 16 x 2^n_open bytes; it is overwritten, and `stream` is synchronised. */
typedef struct rqc_calib_report {
  int32_t candidates;   /* steps whose precision was chosen */
  int32_t reduced;      /* of which left in reduced precision */
  double estimated_err; /* root sum of squares of the kept steps' errors */
  double measured_err;  /* error of the final assignment on the slice */
  double min_step_err, max_step_err;
} rqc_calib_report;

rqc_status rqc_plan_calibrate(rqc_plan* p, int32_t prec, uint64_t slice_id,
                              const uint8_t* closed_bits, double target_err,
                              double err_floor, void* workspace,
                              size_t ws_bytes, rqc_stream stream,
                              rqc_calib_report* out);

/* Upper bounds on the slices and bitstrings contracted side by side in one
 * group (one batched launch per step); 0 = no bound beyond the workspace.
 * Smaller groups keep a group's intermediates within the GPU's last-level
 * cache between steps; larger groups give each launch more work.  Takes
 * effect at the next rqc_contract; results do not depend on it. */
rqc_status rqc_plan_set_group_limit(rqc_plan* p, int32_t max_slices, int32_t max_bits);

/* ---- misc --------------------------------------------------------------- */

const char* rqc_last_error(void);
const char* rqc_version(void);

/* ======================================================================
 * Test and measurement hooks.  Not part of the amplitude path: they exist
 * so that tests can force rare conditions from the host and so that the
 * benchmark can time kernels on their own stream.
 * ====================================================================== */

/* Timing probe.  kernel 0 (SIMT), 1 (FP32 or 16-bit MFMA), 2 (rows),
 * 3 (16-bit MFMA only) or 4 (every step launch): later rqc_contract calls of
 * this plan launch their kernels directly on the caller's stream instead of
 * replaying a graph, and every probed launch is bracketed by a pair of HIP
 * events recorded on that stream; -1 turns the probe off and restores graph
 * launches. */
rqc_status rqc_plan_set_timing(rqc_plan* p, int32_t kernel);

typedef struct rqc_timing {
  uint64_t launches;    /* probed launches in the last reported call */
  double total_ms;      /* their summed event-measured duration */
  double flops;         /* their summed algorithmic flops (8 per complex MAC) */
  double bytes;         /* their summed algorithmic bytes: each operand read
                           once and the output written once, per copy */
} rqc_timing;

/* Valid after rqc_contract_status of the call. */
rqc_status rqc_plan_get_timing(const rqc_plan* p, rqc_timing* out);

/* One probed launch of the last reported call (i < launches). */
typedef struct rqc_launch_timing {
  int32_t step;         /* plan step index (rqc_plan_get_step) */
  int32_t kernel;       /* 0 SIMT, 1 FP32 MFMA, 2 rows, 3 16-bit MFMA */
  int32_t m, n, k;      /* bits of C[m,n] = A[m,k] B[k,n] */
  int32_t copies;       /* independent problems of the launch */
  int32_t store_a, store_b, store_c; /* 0 complex64, 1 FP16, 2 BF16 pairs */
  int32_t variant;      /* kernel variant bits (as in rqc_pair_contract_stored) */
  double ms, flops, bytes;
} rqc_launch_timing;

rqc_status rqc_plan_get_launch_timing(const rqc_plan* p, uint64_t i,
                                      rqc_launch_timing* out);

/* Failure path of Section 5.5: adds `bias` to every reduced-precision
 * storage exponent shift of the launches for bitstring groups that start at
 * bitstring index first_bitstring or later (positive values force overflow
 * to inf, which flags those (slice, bitstring group) pairs for an FP32
 * re-run).  The kernels themselves run normally. */
rqc_status rqc_plan_set_scale_bias(rqc_plan* p, int32_t bias,
                                   uint64_t first_bitstring);

/* One pairwise contraction with explicit operand storage (0 complex64,
 * 1 FP16, 2 BF16: packed (re, im) 16-bit pairs, 4 bytes per element) and
 * explicit kernel: 0 generic SIMT, 1 FP32 MFMA, 2 row streaming, 3 16-bit
 * MFMA (mma_prec RQC_F16 or RQC_BF16).  With kernels 0 and 1 the arithmetic
 * is FP32 on the converted operands (16-bit storage, FP32 compute); kernel 2
 * uses the 16-bit matrix cores when A is stored in 16 bits and the summed
 * labels fill chunks of 16 or more complex values, FP32 otherwise.  Labels,
 * batching and strides as in rqc_pair_contract; no scaling is applied (the
 * caller keeps values inside the 16-bit range).  variant: kernel variant
 * bits (0 = default; FP32 matrix cores: 1 = four real products per complex
 * product instead of three, 2 = one tile per workgroup, 4 = persistent
 * walk; any kernel: 8 = FP32 arithmetic on 16-bit stored operands; 16-bit
 * matrix cores: 16 = stream A past a resident tile of B, for sums of 32 to
 * 128 terms with A stored in 16 bits; FP32 and 16-bit matrix cores: 32 =
 * the operands exchanged inside the kernel, B taking the tile rows and A the
 * columns, same result).  EINVAL when the kernel's shape or layout
 * conditions are not met (no fallback). */
rqc_status rqc_pair_contract_stored(const int32_t* labels_a, int32_t rank_a,
                                    const int32_t* labels_b, int32_t rank_b,
                                    const int32_t* labels_c, int32_t rank_c,
                                    const void* A, const void* B, void* C,
                                    int32_t store_a, int32_t store_b,
                                    int32_t store_c, int32_t batch_count,
                                    int64_t stride_a, int64_t stride_b,
                                    int64_t stride_c, int32_t kernel,
                                    int32_t mma_prec, int32_t variant,
                                    rqc_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* RQC_H */

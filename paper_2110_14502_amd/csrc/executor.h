// Executor: residency, per-group memory layout, step descriptors, graph
// capture of a whole contraction call.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <tuple>

#include "core.h"
#include "kernels.h"

namespace rqc {

// Where a tensor of the contraction tree lives during a call.
struct Placement {
  bool resident = false;     // invariant: in the plan's resident memory
  int64_t off = 0;           // bytes from the region base
  int store = ST_C64;
  int64_t s_stride = 0, b_stride = 0;  // copy strides, elements
  int64_t e_off = -1;        // bytes of the exponent array (-1: none)
  int64_t m_off = -1;        // bytes of the max array (-1: none)
  int32_t es = 0, eb = 0;    // copy strides of the scale arrays
  float max_const = 0.f;     // leaves: bound on |re|, |im|
  bool dep_s = false, dep_b = false;
};

// Memory layout of one (precision, slices per group, bits per group).
struct GroupLayout {
  int prec = RQC_F32, gs = 1, gb = 1;
  std::vector<Placement> place;  // per tree node
  int64_t arena_bytes = 0;       // variable tensors
  int64_t scale_bytes = 0;       // exponent / max arrays
  std::vector<LeafJob> jobs;     // variable leaves
  int max_leaf_rank = 0;
  std::vector<int> ksplit;       // per step: split-K bits (generic kernel)
  std::vector<int64_t> p_off;    // per step: partial buffer in the arena
};

struct GraphKey {
  int prec, gs, gb;
  uint64_t n_ids, n_batch;
  const void* ws;
  const void* out;
  const void* per_slice;
  bool operator<(const GraphKey& o) const {
    return std::tie(prec, gs, gb, n_ids, n_batch, ws, out, per_slice) <
           std::tie(o.prec, o.gs, o.gb, o.n_ids, o.n_batch, o.ws, o.out, o.per_slice);
  }
};

struct PendingRun {
  bool active = false;
  int prec = RQC_F32;
  uint64_t n_ids = 0, n_batch = 0;
  std::vector<uint64_t> ids;
  std::vector<uint8_t> bits;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  double* out = nullptr;
  double* per_slice = nullptr;
  int gs = 1, gb = 1;
  int graph_reused = 0;
  double flops = 0;
};

// Workspace of one call.  Flags: one int32 per (bitstring group, slice), set
// when a reduced-precision copy of that slice in that group of bitstrings
// held a non-finite value (the slice sum then skipped it).
struct WsLayout {
  int64_t ids_off, bits_off, flags_off, jobs_off, tmp_off, scale_off, arena_off, total;
  int64_t n_bgroups;
};

// A captured call and the event recorded after its last launch (an exec is
// destroyed only once that event has completed).
struct GraphEntry {
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;
  uint64_t last_use = 0;
};

// One probed launch of the timing hook.
struct LaunchRecord {
  int step, kernel, m, n, k, copies, sa, sb, sc, variant;
  double flops, bytes;
};

}  // namespace rqc

struct rqc_plan {
  rqc::PlanData pd;
  // Resident memory.
  char* res = nullptr;
  size_t res_bytes = 0;
  bool bound = false;
  std::vector<int64_t> leaf_store_off;  // per leaf, element offset (c64)
  int64_t leaf_store_elems = 0;
  std::vector<float> leaf_max;          // per leaf
  std::vector<int64_t> inv_off;         // per node: bytes in resident, -1
  int64_t inv_max_off = 0;              // bytes: float per node
  int64_t inv_exp_off = 0;              // bytes: int32 exponent per node
  int64_t inv_bytes = 0;
  int scale_bias = 0;
  uint64_t scale_bias_from = 0;         // first bitstring whose groups get the bias
  // Per-step descriptor templates (layout only) and default kernels.
  std::vector<rqc::StepDesc> tmpl, tmpl_lp;  // FP32 and reduced precision
  std::vector<int> kern, kern_lp;
  // Per precision mode (RQC_F32, RQC_F16, RQC_BF16) and step: whether the
  // step runs in reduced precision (16-bit storage of its output by the size
  // rule, 16-bit matrix cores; modes 1 and 2 only), the tuner's choice of
  // kernel and variant (-1: none), and the descriptor and kernel launched.
  std::vector<char> lp_on[3];
  std::vector<int> tuned_kern[3], tuned_var[3];
  std::vector<rqc::StepDesc> sel_desc[3];
  std::vector<int> sel_kern[3];
  // Timing probe: events around launches of one kernel kind (or of all).
  int timing_kernel = -1;
  int group_limit_s = 0, group_limit_b = 0;  // 0: bounded by the workspace only
  std::vector<hipEvent_t> tev;          // pairs (start, stop)
  std::vector<rqc::LaunchRecord> trec;  // per probed launch
  std::vector<double> tms;              // per probed launch, after the report
  rqc_timing last_timing{};
  // Caches.
  std::map<std::tuple<int, int, int>, rqc::GroupLayout> layouts;
  std::map<rqc::GraphKey, rqc::GraphEntry> graphs;
  uint64_t graph_clock = 0;
  hipStream_t capture_stream = nullptr;
  rqc::PendingRun pending;
  ~rqc_plan();
};

namespace rqc {

size_t resident_bytes(rqc_plan* p);
void bind_plan(rqc_plan* p, void* dev, size_t bytes, hipStream_t s);
const GroupLayout& group_layout(rqc_plan* p, int prec, int gs, int gb);
WsLayout ws_layout(rqc_plan* p, const GroupLayout& L, uint64_t n_ids, uint64_t n_batch);
// Enqueue a contraction call on `s` (one graph launch); `run` keeps what the
// report needs.
// direct: launch on `s` without capturing or caching a graph.
void contract(rqc_plan* p, const uint64_t* ids, uint64_t n_ids, const uint8_t* bits,
              uint64_t n_batch, int prec, void* ws, size_t ws_bytes, double* out,
              double* per_slice, hipStream_t s, PendingRun& run, bool direct = false);
// Group sizes (slices, bitstrings) for a call within ws_bytes; EHBM if one
// slice and one bitstring do not fit.
void choose_group(rqc_plan* p, int prec, uint64_t n_ids, uint64_t n_batch, size_t ws_bytes,
                  int& gs, int& gb);
bool fits(rqc_plan* p, int prec, int gs, int gb, uint64_t n_ids, uint64_t n_batch,
          size_t ws_bytes);

// Every launch of one call (ids, bits and leaf jobs already in the
// workspace), in order on `s`.
void record_call(rqc_plan* p, const GroupLayout& L, const WsLayout& W, uint64_t n_ids,
                 uint64_t n_batch, char* ws, double* out, double* per_slice, int64_t ps_row0,
                 hipStream_t s);

// Descriptor of step i for one group (gsc slices x gbc bitstrings) with its
// operands, strides and scale arrays bound, and its launch.
StepDesc bind_step(rqc_plan* p, const GroupLayout& L, const WsLayout& W, char* ws, size_t i,
                   int gsc, int gbc, int32_t* gflags, int bias);
hipError_t launch_bound_step(const rqc_plan* p, const GroupLayout& L, size_t i, const StepDesc& d,
                             int kern, hipStream_t s);

// Per-step kernel tuning and the precision pre-analysis (tune.cpp).
void autotune(rqc_plan* p, int prec, uint64_t n_ids, uint64_t n_batch, void* ws, size_t ws_bytes,
              const char* cache_path, hipStream_t s, rqc_tune_report* rep);
void calibrate(rqc_plan* p, int prec, uint64_t slice_id, const uint8_t* bits, double target,
               double err_floor, void* ws, size_t ws_bytes, hipStream_t s, rqc_calib_report* rep);

// Synchronise `s`, re-run flagged slices in FP32, fill the report.
// sync = false: the caller knows the call's work has completed (for example
// from an event recorded after it) and `s` is not synchronised; it is only
// used for an FP32 re-run.
void report(rqc_plan* p, PendingRun& run, hipStream_t s, rqc_run_report* r, bool sync = true);

// Build the descriptor of one pairwise contraction given operand labels
// (MSB first).  `kernel` is the requested kind (-1: choose) and returns the
// kind actually used (MFMA and row-streaming need their shape conditions).
StepDesc make_pair_desc(const std::vector<int>& la, const std::vector<int>& lb,
                        const std::vector<int>& lc, int& kernel);

// The descriptor of step `st` for kernel `kernel` (updated as by
// make_pair_desc) and variant bits `variant`: built from (B, A) when the
// variant exchanges the operands (kVarSwap).
StepDesc step_desc(const Step& st, int& kernel, int variant);

// Exchanges the bound A and B operands of a descriptor (pointers, copy
// strides and scale arrays); the tile geometry is left as it is.
void swap_operands(StepDesc& d);

void hip_check(hipError_t e, const char* what);

// Destroy every cached graph exec of the plan, each after its last launch
// has completed.
void clear_graphs(rqc_plan* p);

// Rebuild the launched descriptor and kernel of every step and mode from the
// defaults, the precision policy, the per-step reduced-precision switches and
// the tuner's choices; drops cached layouts and graphs.
void select_steps(rqc_plan* p);

// Whether step i stores its output in 16 bits in mode `prec`.
bool step_lp_store(const rqc_plan* p, int prec, size_t i);

// Timing probe kinds: a kernel kind, or every step launch.
constexpr int kTimeAll = 4;
// Cached graph execs per plan.
constexpr size_t kMaxGraphs = 32;

}  // namespace rqc

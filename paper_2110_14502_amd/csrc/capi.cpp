// C ABI (include/rqc.h).  Every entry point catches C++ exceptions and turns
// them into rqc_status codes with a thread-local message.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "executor.h"

struct rqc_circuit {
  rqc::Circuit c;
};
struct rqc_network {
  rqc::Network n;
};

namespace rqc {
static thread_local std::string g_err;
void set_error(const std::string& m) { g_err = m; }
}  // namespace rqc

#define RQC_TRY try {
#define RQC_CATCH                                              \
  }                                                            \
  catch (const rqc::Error& e) {                                \
    rqc::set_error(e.msg);                                     \
    return e.code;                                             \
  }                                                            \
  catch (const std::bad_alloc&) {                              \
    rqc::set_error("host allocation failed");                  \
    return RQC_ENOMEM;                                         \
  }                                                            \
  catch (const std::exception& e) {                            \
    rqc::set_error(e.what());                                  \
    return RQC_EINVAL;                                         \
  }

extern "C" {

const char* rqc_last_error(void) { return rqc::g_err.c_str(); }
const char* rqc_version(void) { return "rqc 0.1 gfx950"; }

rqc_status rqc_circuit_create(int32_t n_qubits, const rqc_gate* gates, size_t n_gates,
                              rqc_circuit** out) {
  RQC_TRY
  if (!out) throw rqc::Error{RQC_EINVAL, "out is NULL"};
  *out = nullptr;
  if (n_qubits <= 0 || n_qubits > 4096) throw rqc::Error{RQC_EINVAL, "n_qubits out of range"};
  if (n_gates && !gates) throw rqc::Error{RQC_EINVAL, "gates is NULL"};
  auto* c = new rqc_circuit;
  c->c.n = n_qubits;
  for (size_t i = 0; i < n_gates; ++i) {
    const rqc_gate& g = gates[i];
    rqc::Gate h;
    h.kind = g.kind;
    h.q0 = g.q0;
    h.q1 = g.q1;
    h.theta = g.theta;
    h.phi = g.phi;
    const bool two = g.kind == RQC_GATE_FSIM || g.kind == RQC_GATE_U2;
    if (g.kind < RQC_GATE_H || g.kind > RQC_GATE_U2) {
      delete c;
      throw rqc::Error{RQC_EINVAL, "unknown gate kind at index " + std::to_string(i)};
    }
    if (g.q0 < 0 || g.q0 >= n_qubits || (two && (g.q1 < 0 || g.q1 >= n_qubits || g.q1 == g.q0))) {
      delete c;
      throw rqc::Error{RQC_EINVAL, "bad qubit index at gate " + std::to_string(i)};
    }
    if (!two) h.q1 = -1;
    if (g.kind == RQC_GATE_U1)
      for (int j = 0; j < 4; ++j) h.u.emplace_back(g.u[2 * j], g.u[2 * j + 1]);
    if (g.kind == RQC_GATE_U2)
      for (int j = 0; j < 16; ++j) h.u.emplace_back(g.u[2 * j], g.u[2 * j + 1]);
    c->c.gates.push_back(std::move(h));
  }
  *out = c;
  return RQC_OK;
  RQC_CATCH
}

void rqc_circuit_destroy(rqc_circuit* c) { delete c; }

rqc_status rqc_network_create(const rqc_circuit* c, const int32_t* open_qubits, int32_t n_open,
                              rqc_network** out) {
  RQC_TRY
  if (!c || !out) throw rqc::Error{RQC_EINVAL, "NULL argument"};
  *out = nullptr;
  if (n_open < 0 || n_open > 24 || (n_open && !open_qubits))
    throw rqc::Error{RQC_EINVAL, "n_open must be in [0, 24]"};
  std::vector<int> open(open_qubits, open_qubits + n_open);
  auto* n = new rqc_network;
  try {
    n->n = rqc::build_network(c->c, open);
  } catch (...) {
    delete n;
    throw;
  }
  *out = n;
  return RQC_OK;
  RQC_CATCH
}

void rqc_network_destroy(rqc_network* n) { delete n; }

void rqc_plan_opts_default(rqc_plan_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->max_log2_elems = 0;
  o->n_sliced = -1;
  o->path_trials = 256;
  o->reconf_rounds = -1;
  o->seed = 0;
  o->lp_min_log2 = 14;
  o->bf16_min_log2 = 24;
}

rqc_status rqc_plan_create(const rqc_network* n, const rqc_plan_opts* opts, rqc_plan** out) {
  RQC_TRY
  if (!n || !out) throw rqc::Error{RQC_EINVAL, "NULL argument"};
  *out = nullptr;
  rqc_plan_opts o;
  rqc_plan_opts_default(&o);
  if (opts) o = *opts;
  if (o.max_log2_elems < 0 || o.max_log2_elems > 40) throw rqc::Error{RQC_EINVAL, "max_log2_elems out of range"};
  if (o.n_sliced < -1) throw rqc::Error{RQC_EINVAL, "n_sliced < -1"};
  if (o.n_forced < 0 || (o.n_forced && !o.forced_wires)) throw rqc::Error{RQC_EINVAL, "forced wires"};
  if (o.n_local_sliced < 0 || o.n_local_sliced > 62) throw rqc::Error{RQC_EINVAL, "n_local_sliced out of range"};
  if (o.n_share_bits < 0 || (o.n_share_bits && !o.share_bits)) throw rqc::Error{RQC_EINVAL, "share bits"};
  auto* p = new rqc_plan;
  try {
    p->pd.net = n->n;
    rqc::PlanOpts& po = p->pd.opts;
    po.max_log2 = o.max_log2_elems;
    po.n_sliced = o.n_sliced;
    po.trials = o.path_trials > 0 ? o.path_trials : 256;
    po.reconf_rounds = o.reconf_rounds < 0 ? 4 : o.reconf_rounds;
    po.seed = o.seed;
    for (int i = 0; i < o.n_forced; ++i) po.forced.push_back({o.forced_wires[2 * i], o.forced_wires[2 * i + 1]});
    po.lp_min_log2 = o.lp_min_log2 > 0 ? o.lp_min_log2 : 14;
    po.bf16_min_log2 = o.bf16_min_log2 > 0 ? o.bf16_min_log2 : 24;
    po.n_local = o.n_local_sliced;
    if (o.restarts < 0 || o.restarts > 1024) throw rqc::Error{RQC_EINVAL, "restarts out of range"};
    po.restarts = o.restarts > 0 ? o.restarts : 1;
    po.share_bits.assign(o.share_bits, o.share_bits + o.n_share_bits);
    for (auto& b : po.share_bits)
      if (b > 1) throw rqc::Error{RQC_EINVAL, "share bits must be 0 or 1"};
    if (o.precision_policy != RQC_POLICY_SIZE && o.precision_policy != RQC_POLICY_CALIBRATED &&
        o.precision_policy != RQC_POLICY_STORAGE)
      throw rqc::Error{RQC_EINVAL, "unknown precision policy"};
    po.precision_policy = o.precision_policy;
    rqc::make_plan(p->pd);
    const size_t res = rqc::resident_bytes(p);
    if (o.hbm_budget_bytes) {
      const rqc::GroupLayout& L1 = rqc::group_layout(p, RQC_F32, 1, 1);
      const size_t need = res + (size_t)rqc::ws_layout(p, L1, 1, 1).total;
      if (need > o.hbm_budget_bytes)
        throw rqc::Error{RQC_EHBM, "plan needs " + std::to_string(need) +
                                       " device bytes for one slice, above the budget"};
    }
  } catch (...) {
    delete p;
    throw;
  }
  *out = p;
  return RQC_OK;
  RQC_CATCH
}

void rqc_plan_destroy(rqc_plan* p) { delete p; }

rqc_status rqc_plan_info(const rqc_plan* p, rqc_plan_info_t* out) {
  RQC_TRY
  if (!p || !out) throw rqc::Error{RQC_EINVAL, "NULL argument"};
  const rqc::PlanData& pd = p->pd;
  std::memset(out, 0, sizeof *out);
  out->n_qubits = pd.net.n_qubits;
  out->n_open = (int)pd.net.open.size();
  out->n_closed = (int)pd.net.closed.size();
  out->n_sliced = (int)pd.sliced.size();
  out->n_slices = uint64_t(1) << pd.sliced.size();
  out->n_leaves = pd.tree.n_leaves;
  out->n_steps = (int)pd.steps.size();
  for (auto& st : pd.steps) out->n_invariant_steps += st.invariant ? 1 : 0;
  out->max_log2_elems = pd.max_log2;
  out->flops_per_slice = pd.flops_per_slice;
  out->flops_invariant = pd.flops_invariant;
  out->bytes_per_slice = pd.bytes_per_slice;
  out->flops_per_bitstring = pd.flops_per_bitstring;
  out->log2_total_flops = std::log2(pd.flops_per_slice * (double)out->n_slices +
                                    pd.flops_per_bitstring + pd.flops_invariant + 1e-300);
  return RQC_OK;
  RQC_CATCH
}

rqc_status rqc_plan_get_step(const rqc_plan* p, int32_t i, rqc_step_info* out) {
  RQC_TRY
  if (!p || !out) throw rqc::Error{RQC_EINVAL, "NULL argument"};
  if (i < 0 || i >= (int)p->pd.steps.size()) throw rqc::Error{RQC_EINVAL, "step index out of range"};
  const rqc::Step& st = p->pd.steps[i];
  std::memset(out, 0, sizeof *out);
  out->m = st.m;
  out->n = st.n;
  out->k = st.k;
  out->kernel = p->sel_kern[RQC_F32][i];
  out->kernel_lp = p->sel_kern[RQC_F16][i];
  out->depends_on_slice = st.dep_s;
  out->depends_on_bits = st.dep_b;
  out->lp_output = rqc::step_lp_store(p, RQC_F16, (size_t)i);
  out->lp_output_bf16 = rqc::step_lp_store(p, RQC_BF16, (size_t)i);
  out->flops = 8.0 * std::ldexp(1.0, st.m + st.n + st.k);
  out->bytes_c64 = 8.0 * (std::ldexp(1.0, st.m + st.k) + std::ldexp(1.0, st.n + st.k) + std::ldexp(1.0, st.m + st.n));
  return RQC_OK;
  RQC_CATCH
}

rqc_status rqc_plan_export_json(const rqc_plan* p, char* buf, size_t cap, size_t* needed) {
  RQC_TRY
  if (!p) throw rqc::Error{RQC_EINVAL, "NULL plan"};
  const std::string s = rqc::plan_json(p->pd);
  if (needed) *needed = s.size() + 1;
  if (buf && cap) {
    const size_t n = std::min(cap - 1, s.size());
    std::memcpy(buf, s.data(), n);
    buf[n] = 0;
    if (cap < s.size() + 1) throw rqc::Error{RQC_EINVAL, "buffer too small"};
  }
  return RQC_OK;
  RQC_CATCH
}

rqc_status rqc_plan_resident_bytes(const rqc_plan* p, size_t* bytes) {
  RQC_TRY
  if (!p || !bytes) throw rqc::Error{RQC_EINVAL, "NULL argument"};
  *bytes = (size_t)p->inv_bytes;
  return RQC_OK;
  RQC_CATCH
}

rqc_status rqc_plan_bind_memory(rqc_plan* p, void* dev_ptr, size_t bytes, rqc_stream stream) {
  RQC_TRY
  if (!p || !dev_ptr) throw rqc::Error{RQC_EINVAL, "NULL argument"};
  rqc::bind_plan(p, dev_ptr, bytes, static_cast<hipStream_t>(stream));
  return RQC_OK;
  RQC_CATCH
}

rqc_status rqc_contract_workspace(const rqc_plan* pc, uint64_t n_ids, uint64_t n_batch, int32_t prec,
                                  size_t* min_bytes, size_t* pref_bytes) {
  RQC_TRY
  if (!pc) throw rqc::Error{RQC_EINVAL, "NULL plan"};
  rqc_plan* p = const_cast<rqc_plan*>(pc);
  if (prec != RQC_F32 && prec != RQC_F16 && prec != RQC_BF16) throw rqc::Error{RQC_EINVAL, "bad precision"};
  if (n_ids == 0) n_ids = uint64_t(1) << p->pd.sliced.size();
  if (n_batch == 0) throw rqc::Error{RQC_EINVAL, "n_batch must be positive"};
  const rqc::GroupLayout& L1 = rqc::group_layout(p, prec, 1, 1);
  if (min_bytes) *min_bytes = (size_t)rqc::ws_layout(p, L1, n_ids, n_batch).total;
  if (pref_bytes) {
    const int gs = (int)std::min<uint64_t>(n_ids, 4096), gb = (int)std::min<uint64_t>(n_batch, 4096);
    const rqc::GroupLayout& L = rqc::group_layout(p, prec, gs, gb);
    *pref_bytes = (size_t)rqc::ws_layout(p, L, n_ids, n_batch).total;
  }
  return RQC_OK;
  RQC_CATCH
}

rqc_status rqc_contract(rqc_plan* p, const uint64_t* slice_ids, uint64_t n_ids,
                        const uint8_t* closed_bits, uint64_t n_batch, int32_t prec, void* workspace,
                        size_t ws_bytes, double* out, double* per_slice, rqc_stream stream) {
  RQC_TRY
  if (!p) throw rqc::Error{RQC_EINVAL, "NULL plan"};
  rqc::contract(p, slice_ids, n_ids, closed_bits, n_batch, prec, workspace, ws_bytes, out, per_slice,
                static_cast<hipStream_t>(stream), p->pending);
  return RQC_OK;
  RQC_CATCH
}

rqc_status rqc_contract_status(rqc_plan* p, rqc_stream stream, rqc_run_report* out) {
  RQC_TRY
  if (!p || !out) throw rqc::Error{RQC_EINVAL, "NULL argument"};
  rqc::report(p, p->pending, static_cast<hipStream_t>(stream), out);
  return RQC_OK;
  RQC_CATCH
}

rqc_status rqc_plan_set_scale_bias(rqc_plan* p, int32_t bias, uint64_t first_bitstring) {
  RQC_TRY
  if (!p) throw rqc::Error{RQC_EINVAL, "NULL plan"};
  if (bias < -64 || bias > 64) throw rqc::Error{RQC_EINVAL, "bias out of range"};
  p->scale_bias = bias;
  p->scale_bias_from = first_bitstring;
  rqc::clear_graphs(p);
  return RQC_OK;
  RQC_CATCH
}

rqc_status rqc_plan_set_group_limit(rqc_plan* p, int32_t max_slices, int32_t max_bits) {
  RQC_TRY
  if (!p) throw rqc::Error{RQC_EINVAL, "NULL plan"};
  if (max_slices < 0 || max_bits < 0) throw rqc::Error{RQC_EINVAL, "negative group limit"};
  p->group_limit_s = max_slices;
  p->group_limit_b = max_bits;
  return RQC_OK;
  RQC_CATCH
}

rqc_status rqc_plan_autotune(rqc_plan* p, int32_t prec, uint64_t n_ids, uint64_t n_batch,
                             void* workspace, size_t ws_bytes, const char* cache_path,
                             rqc_stream stream, rqc_tune_report* out) {
  RQC_TRY
  if (!p || !out) throw rqc::Error{RQC_EINVAL, "NULL argument"};
  rqc::autotune(p, prec, n_ids, n_batch, workspace, ws_bytes, cache_path,
                static_cast<hipStream_t>(stream), out);
  return RQC_OK;
  RQC_CATCH
}

rqc_status rqc_plan_calibrate(rqc_plan* p, int32_t prec, uint64_t slice_id,
                              const uint8_t* closed_bits, double target_err, double err_floor,
                              void* workspace, size_t ws_bytes, rqc_stream stream,
                              rqc_calib_report* out) {
  RQC_TRY
  if (!p || !out) throw rqc::Error{RQC_EINVAL, "NULL argument"};
  rqc::calibrate(p, prec, slice_id, closed_bits, target_err, err_floor, workspace, ws_bytes,
                 static_cast<hipStream_t>(stream), out);
  return RQC_OK;
  RQC_CATCH
}

rqc_status rqc_plan_set_timing(rqc_plan* p, int32_t kernel) {
  RQC_TRY
  if (!p) throw rqc::Error{RQC_EINVAL, "NULL plan"};
  if (kernel < -1 || kernel > rqc::kTimeAll)
    throw rqc::Error{RQC_EINVAL, "kernel must be -1, 0, 1, 2, 3 or 4"};
  p->timing_kernel = kernel;
  rqc::clear_graphs(p);
  return RQC_OK;
  RQC_CATCH
}

rqc_status rqc_plan_get_timing(const rqc_plan* p, rqc_timing* out) {
  RQC_TRY
  if (!p || !out) throw rqc::Error{RQC_EINVAL, "NULL argument"};
  *out = p->last_timing;
  return RQC_OK;
  RQC_CATCH
}

rqc_status rqc_plan_get_launch_timing(const rqc_plan* p, uint64_t i, rqc_launch_timing* out) {
  RQC_TRY
  if (!p || !out) throw rqc::Error{RQC_EINVAL, "NULL argument"};
  if (i >= p->tms.size() || i >= p->trec.size()) throw rqc::Error{RQC_EINVAL, "launch index out of range"};
  const rqc::LaunchRecord& r = p->trec[i];
  std::memset(out, 0, sizeof *out);
  out->step = r.step;
  out->kernel = r.kernel;
  out->m = r.m;
  out->n = r.n;
  out->k = r.k;
  out->copies = r.copies;
  out->store_a = r.sa;
  out->store_b = r.sb;
  out->store_c = r.sc;
  out->variant = r.variant;
  out->ms = p->tms[i];
  out->flops = r.flops;
  out->bytes = r.bytes;
  return RQC_OK;
  RQC_CATCH
}

// ---- single pairwise contraction, permutation, GEMM ---------------------

rqc_status rqc_pair_contract(const int32_t* labels_a, int32_t rank_a, const int32_t* labels_b,
                             int32_t rank_b, const int32_t* labels_c, int32_t rank_c, const void* A,
                             const void* B, void* C, int32_t batch_count, int64_t stride_a,
                             int64_t stride_b, int64_t stride_c, int32_t kernel, int32_t prec,
                             rqc_stream stream) {
  RQC_TRY
  if (!A || !B || !C) throw rqc::Error{RQC_EINVAL, "NULL device pointer"};
  if (rank_a < 0 || rank_b < 0 || rank_c < 0 || rank_a > 40 || rank_b > 40 || rank_c > 40)
    throw rqc::Error{RQC_EINVAL, "rank out of range"};
  if ((rank_a && !labels_a) || (rank_b && !labels_b) || (rank_c && !labels_c))
    throw rqc::Error{RQC_EINVAL, "NULL labels"};
  if (batch_count < 1 || batch_count > 65535) throw rqc::Error{RQC_EINVAL, "batch_count out of range"};
  if (kernel < -1 || kernel > 2) throw rqc::Error{RQC_EINVAL, "kernel must be -1, 0, 1 or 2"};
  if (prec != RQC_F32 && prec != RQC_F16 && prec != RQC_BF16) throw rqc::Error{RQC_EINVAL, "bad precision"};
  std::vector<int> la(labels_a, labels_a + rank_a), lb(labels_b, labels_b + rank_b),
      lc(labels_c, labels_c + rank_c);
  for (auto* l : {&la, &lb}) {
    std::vector<int> s(*l);
    std::sort(s.begin(), s.end());
    if (std::adjacent_find(s.begin(), s.end()) != s.end()) throw rqc::Error{RQC_EINVAL, "repeated label"};
  }
  int kern = kernel;
  if (prec != RQC_F32 && (kernel == -1 || kernel == rqc::KERN_MFMA)) kern = rqc::KERN_MFMA16;
  rqc::StepDesc d = rqc::make_pair_desc(la, lb, lc, kern);
  d.A = A;
  d.B = B;
  d.C = C;
  d.sA_s = stride_a;
  d.sB_s = stride_b;
  d.sC_s = stride_c;
  d.gs_c = batch_count;
  d.copies = batch_count;
  const int lp_kind = prec == RQC_F16 ? rqc::ST_F16 : (prec == RQC_BF16 ? rqc::ST_BF16 : 0);
  rqc::hip_check(rqc::launch_step(d, kern, rqc::ST_C64, rqc::ST_C64, rqc::ST_C64, lp_kind,
                                  static_cast<hipStream_t>(stream)),
                 "pair contract");
  return RQC_OK;
  RQC_CATCH
}

}  // extern "C"

namespace {

// Two-phase long-sum form of a 16-bit contraction (permute + convert each
// operand, then k_gemm16): taken by automatic kernel choice in FP16 / BF16
// when the sum has at least 2^kGemm16MinK terms and the output at least one
// 256 x 128 tile.  m < 0: the call does not take it.
constexpr int kGemm16MinK = 8;
struct Gemm16Shape {
  int m = -1, n = 0, k = 0, ksplit = 0;
  std::vector<int> Mf, Nf, K;  // A's free labels, B's free labels, summed labels (A's order)
  uint64_t bytes_a = 0, bytes_b = 0, bytes_p = 0, copies_a = 1, copies_b = 1;
  uint64_t total() const { return bytes_a + bytes_b + bytes_p; }
};

Gemm16Shape gemm16_shape(const std::vector<int>& la, const std::vector<int>& lb,
                         const std::vector<int>& lc, int32_t batch, int64_t stride_a,
                         int64_t stride_b, int32_t kernel, int32_t prec) {
  Gemm16Shape g;
  if ((prec != RQC_F16 && prec != RQC_BF16) || kernel != -1) return g;
  for (int x : la) (std::find(lb.begin(), lb.end(), x) != lb.end() ? g.K : g.Mf).push_back(x);
  for (int x : lb)
    if (std::find(la.begin(), la.end(), x) == la.end()) g.Nf.push_back(x);
  // Rows and columns of the packed operands in C's order (the lowest row
  // and column bits are C's lowest address bits among them), so that the
  // GEMM's output tiles write runs of C that are as long as possible.
  auto c_order = [&](std::vector<int>& v) {
    std::stable_sort(v.begin(), v.end(), [&](int x, int y) {
      return std::find(lc.begin(), lc.end(), x) < std::find(lc.begin(), lc.end(), y);
    });
  };
  c_order(g.Mf);
  c_order(g.Nf);
  if ((int)g.K.size() < kGemm16MinK || g.Mf.size() < 8 || g.Nf.size() < 7) return g;
  g.m = (int)g.Mf.size();
  g.n = (int)g.Nf.size();
  g.k = (int)g.K.size();
  g.copies_a = stride_a ? (uint64_t)batch : 1;
  g.copies_b = stride_b ? (uint64_t)batch : 1;
  g.bytes_a = ((g.copies_a << (g.m + g.k)) * 4 + 255) & ~uint64_t(255);
  g.bytes_b = ((g.copies_b << (g.n + g.k)) * 4 + 255) & ~uint64_t(255);
  // Split the sum while the output tiles cannot fill the GPU (1024 work
  // items: four per CU), keeping at least 16 chunks of 32 terms per split.
  const uint64_t tiles = (uint64_t)batch << (g.m - 8 + g.n - 7);
  while ((tiles << g.ksplit) < 1024 && g.k - 5 - g.ksplit > 4) ++g.ksplit;
  if (g.ksplit) g.bytes_p = (((uint64_t)batch << g.ksplit) << (g.m + g.n)) * 8;
  return g;
}

// Split sum of an FP32 call on the generic kernel whose output tiles cannot
// fill the GPU (as the planner's layouts split plan steps): 2^ks workgroups
// per output tile, each summing a contiguous range of the summed indices into
// its own partial buffer (complex64, batch copies of C back to back), added
// in split order afterwards.  ks = 0: no split.
struct SimtSplit {
  int ks = 0;
  uint64_t bytes = 0;
};

SimtSplit simt_split(const std::vector<int>& la, const std::vector<int>& lb,
                     const std::vector<int>& lc, int32_t batch, int32_t kernel, int32_t prec) {
  SimtSplit sp;
  if (prec != RQC_F32) return sp;
  int kern = kernel;
  const rqc::StepDesc d = rqc::make_pair_desc(la, lb, lc, kern);
  if (kern != rqc::KERN_SIMT || d.n_ko < 2) return sp;
  const int64_t work = (int64_t)d.n_row_tiles * d.n_col_tiles * batch;
  int ks = 0;
  while (ks < d.n_ko && ((work << ks) < 4096 || d.n_ko - ks > 12)) ++ks;
  const int64_t cbytes = ((int64_t)batch << lc.size()) * 8;
  while (ks > 0 && (cbytes << ks) > (int64_t(1) << 30)) --ks;
  sp.ks = ks;
  sp.bytes = ks ? (uint64_t)(((cbytes << ks) + 255) & ~int64_t(255)) : 0;
  return sp;
}

// Output bit i of the permutation of `in` into `out` order: its input bit.
std::vector<int8_t> perm_sources(const std::vector<int>& in, const std::vector<int>& out) {
  const int r = (int)in.size();
  std::vector<int8_t> src(r);
  for (int i = 0; i < r; ++i) {
    const int pos = (int)(std::find(in.begin(), in.end(), out[r - 1 - i]) - in.begin());
    src[i] = (int8_t)(r - 1 - pos);
  }
  return src;
}

// Labels of a pairwise call, validated (ranks, NULLs, repeats, batch).
void pair_labels(const int32_t* labels_a, int32_t rank_a, const int32_t* labels_b, int32_t rank_b,
                 const int32_t* labels_c, int32_t rank_c, int32_t batch_count, std::vector<int>& la,
                 std::vector<int>& lb, std::vector<int>& lc) {
  if (rank_a < 0 || rank_b < 0 || rank_c < 0 || rank_a > 40 || rank_b > 40 || rank_c > 40)
    throw rqc::Error{RQC_EINVAL, "rank out of range"};
  if ((rank_a && !labels_a) || (rank_b && !labels_b) || (rank_c && !labels_c))
    throw rqc::Error{RQC_EINVAL, "NULL labels"};
  if (batch_count < 1 || batch_count > 65535) throw rqc::Error{RQC_EINVAL, "batch_count out of range"};
  la.assign(labels_a, labels_a + rank_a);
  lb.assign(labels_b, labels_b + rank_b);
  lc.assign(labels_c, labels_c + rank_c);
  for (auto* l : {&la, &lb, &lc}) {
    std::vector<int> v(*l);
    std::sort(v.begin(), v.end());
    if (std::adjacent_find(v.begin(), v.end()) != v.end()) throw rqc::Error{RQC_EINVAL, "repeated label"};
  }
}

}  // namespace

extern "C" {

rqc_status rqc_pair_workspace_bytes(const int32_t* labels_a, int32_t rank_a,
                                    const int32_t* labels_b, int32_t rank_b,
                                    const int32_t* labels_c, int32_t rank_c, int32_t batch_count,
                                    int64_t stride_a, int64_t stride_b, int32_t kernel,
                                    int32_t prec, uint64_t* bytes) {
  RQC_TRY
  if (!bytes) throw rqc::Error{RQC_EINVAL, "NULL argument"};
  std::vector<int> la, lb, lc;
  pair_labels(labels_a, rank_a, labels_b, rank_b, labels_c, rank_c, batch_count, la, lb, lc);
  const Gemm16Shape g = gemm16_shape(la, lb, lc, batch_count, stride_a, stride_b, kernel, prec);
  *bytes = g.m >= 0 ? g.total() : simt_split(la, lb, lc, batch_count, kernel, prec).bytes;
  return RQC_OK;
  RQC_CATCH
}

rqc_status rqc_pair_contract_ws(const int32_t* labels_a, int32_t rank_a, const int32_t* labels_b,
                                int32_t rank_b, const int32_t* labels_c, int32_t rank_c,
                                const void* A, const void* B, void* C, int32_t batch_count,
                                int64_t stride_a, int64_t stride_b, int64_t stride_c,
                                int32_t kernel, int32_t prec, void* workspace,
                                uint64_t ws_bytes, rqc_stream stream) {
  RQC_TRY
  std::vector<int> la, lb, lc;
  pair_labels(labels_a, rank_a, labels_b, rank_b, labels_c, rank_c, batch_count, la, lb, lc);
  const Gemm16Shape g = gemm16_shape(la, lb, lc, batch_count, stride_a, stride_b, kernel, prec);
  if (g.m < 0) {
    const SimtSplit sp = simt_split(la, lb, lc, batch_count, kernel, prec);
    if (sp.ks == 0 || (batch_count > 1 && stride_c != ((int64_t)1 << rank_c)))
      return rqc_pair_contract(labels_a, rank_a, labels_b, rank_b, labels_c, rank_c, A, B, C,
                               batch_count, stride_a, stride_b, stride_c, kernel, prec, stream);
    if (!A || !B || !C) throw rqc::Error{RQC_EINVAL, "NULL device pointer"};
    if (!workspace || ws_bytes < sp.bytes)
      throw rqc::Error{RQC_EINVAL, "workspace smaller than rqc_pair_workspace_bytes"};
    if ((uintptr_t)workspace % 256) throw rqc::Error{RQC_EINVAL, "workspace not 256-byte aligned"};
    int kern = kernel;
    rqc::StepDesc d = rqc::make_pair_desc(la, lb, lc, kern);
    d.A = A;
    d.B = B;
    d.C = C;
    d.sA_s = stride_a;
    d.sB_s = stride_b;
    d.sC_s = stride_c;
    d.gs_c = batch_count;
    d.copies = batch_count;
    d.ksplit = sp.ks;
    d.P = static_cast<float2*>(workspace);
    d.p_stride = (int64_t)batch_count << rank_c;
    rqc::hip_check(rqc::launch_step(d, kern, rqc::ST_C64, rqc::ST_C64, rqc::ST_C64, 0,
                                    static_cast<hipStream_t>(stream)),
                   "pair contract (split sum)");
    return RQC_OK;
  }
  if (!A || !B || !C) throw rqc::Error{RQC_EINVAL, "NULL device pointer"};
  if (!workspace || ws_bytes < g.total())
    throw rqc::Error{RQC_EINVAL, "workspace smaller than rqc_pair_workspace_bytes"};
  if ((uintptr_t)workspace % 256) throw rqc::Error{RQC_EINVAL, "workspace not 256-byte aligned"};
  // The labels of C must be exactly the free labels of A and B.
  {
    std::vector<int> f(g.Mf);
    f.insert(f.end(), g.Nf.begin(), g.Nf.end());
    std::vector<int> c(lc);
    std::sort(f.begin(), f.end());
    std::sort(c.begin(), c.end());
    if (f != c) throw rqc::Error{RQC_EINVAL, "labels_c must be the labels of A and B that are not summed"};
  }
  if (batch_count > 1 && stride_c < ((int64_t)1 << (g.m + g.n)))
    throw rqc::Error{RQC_EINVAL, "stride_c smaller than one output"};
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const int lp = prec == RQC_F16 ? rqc::ST_F16 : rqc::ST_BF16;
  uint8_t* wa = static_cast<uint8_t*>(workspace);
  uint8_t* wb = wa + g.bytes_a;
  std::vector<int> oa(g.Mf), ob(g.Nf);
  oa.insert(oa.end(), g.K.begin(), g.K.end());
  ob.insert(ob.end(), g.K.begin(), g.K.end());
  const std::vector<int8_t> srca = perm_sources(la, oa), srcb = perm_sources(lb, ob);
  const uint64_t ea = uint64_t(1) << (g.m + g.k), eb = uint64_t(1) << (g.n + g.k);
  for (uint64_t j = 0; j < g.copies_a; ++j)
    rqc::hip_check(rqc::launch_permute(static_cast<const float2*>(A) + j * stride_a, wa + j * ea * 4,
                                       rank_a, srca.data(), s, lp),
                   "pack A");
  for (uint64_t j = 0; j < g.copies_b; ++j)
    rqc::hip_check(rqc::launch_permute(static_cast<const float2*>(B) + j * stride_b, wb + j * eb * 4,
                                       rank_b, srcb.data(), s, lp),
                   "pack B");
  rqc::Gemm16Desc d{};
  d.A = reinterpret_cast<const uint32_t*>(wa);
  d.B = reinterpret_cast<const uint32_t*>(wb);
  d.C = C;
  d.sA = g.copies_a > 1 ? (int64_t)ea : 0;
  d.sB = g.copies_b > 1 ? (int64_t)eb : 0;
  d.sC = stride_c;
  d.m = g.m;
  d.n = g.n;
  d.k = g.k;
  d.copies = batch_count;
  d.ksplit = g.ksplit;
  d.P = g.ksplit ? reinterpret_cast<float2*>(wb + g.bytes_b) : nullptr;
  auto c_bit = [&](int label) {
    return (int8_t)(rank_c - 1 - (std::find(lc.begin(), lc.end(), label) - lc.begin()));
  };
  for (int b = 0; b < g.m; ++b) d.crow[b] = c_bit(g.Mf[g.m - 1 - b]);
  for (int b = 0; b < g.n; ++b) d.ccol[b] = c_bit(g.Nf[g.n - 1 - b]);
  rqc::hip_check(rqc::launch_gemm16(d, lp, s), "16-bit GEMM");
  return RQC_OK;
  RQC_CATCH
}

rqc_status rqc_pair_contract_stored(const int32_t* labels_a, int32_t rank_a,
                                    const int32_t* labels_b, int32_t rank_b,
                                    const int32_t* labels_c, int32_t rank_c, const void* A,
                                    const void* B, void* C, int32_t store_a, int32_t store_b,
                                    int32_t store_c, int32_t batch_count, int64_t stride_a,
                                    int64_t stride_b, int64_t stride_c, int32_t kernel,
                                    int32_t mma_prec, int32_t variant, rqc_stream stream) {
  RQC_TRY
  if (!A || !B || !C) throw rqc::Error{RQC_EINVAL, "NULL device pointer"};
  if (rank_a < 0 || rank_b < 0 || rank_c < 0 || rank_a > 40 || rank_b > 40 || rank_c > 40)
    throw rqc::Error{RQC_EINVAL, "rank out of range"};
  if ((rank_a && !labels_a) || (rank_b && !labels_b) || (rank_c && !labels_c))
    throw rqc::Error{RQC_EINVAL, "NULL labels"};
  if (batch_count < 1 || batch_count > 65535) throw rqc::Error{RQC_EINVAL, "batch_count out of range"};
  for (int32_t st : {store_a, store_b, store_c})
    if (st < rqc::ST_C64 || st > rqc::ST_BF16) throw rqc::Error{RQC_EINVAL, "storage code out of range"};
  if (kernel < rqc::KERN_SIMT || kernel > rqc::KERN_MFMA16) throw rqc::Error{RQC_EINVAL, "kernel must be 0..3"};
  if (kernel == rqc::KERN_MFMA16 && mma_prec != RQC_F16 && mma_prec != RQC_BF16)
    throw rqc::Error{RQC_EINVAL, "the 16-bit MFMA kernel needs mma_prec RQC_F16 or RQC_BF16"};
  // One 16-bit type per call (the kernels are built for one LP type mixed
  // with complex64).
  int lp = 0;
  for (int32_t st : {store_a, store_b, store_c})
    if (st != rqc::ST_C64) {
      if (lp && st != lp) throw rqc::Error{RQC_EINVAL, "FP16 and BF16 storage in one call"};
      lp = st;
    }
  if (kernel == rqc::KERN_MFMA16 && lp && lp != (mma_prec == RQC_F16 ? rqc::ST_F16 : rqc::ST_BF16))
    throw rqc::Error{RQC_EINVAL, "16-bit storage type differs from mma_prec"};
  std::vector<int> la(labels_a, labels_a + rank_a), lb(labels_b, labels_b + rank_b),
      lc(labels_c, labels_c + rank_c);
  for (auto* l : {&la, &lb}) {
    std::vector<int> v(*l);
    std::sort(v.begin(), v.end());
    if (std::adjacent_find(v.begin(), v.end()) != v.end()) throw rqc::Error{RQC_EINVAL, "repeated label"};
  }
  if (variant < 0 || variant > 63) throw rqc::Error{RQC_EINVAL, "variant out of range"};
  const bool swap = (variant & rqc::kVarSwap) != 0;
  if (swap && kernel != rqc::KERN_MFMA && kernel != rqc::KERN_MFMA16)
    throw rqc::Error{RQC_EINVAL, "exchanged operands need a matrix-core kernel"};
  int kern = kernel;
  rqc::StepDesc d = swap ? rqc::make_pair_desc(lb, la, lc, kern) : rqc::make_pair_desc(la, lb, lc, kern);
  if (kern != kernel) throw rqc::Error{RQC_EINVAL, "shape or layout not supported by the requested kernel"};
  d.A = A;
  d.B = B;
  d.C = C;
  d.sA_s = stride_a;
  d.sB_s = stride_b;
  d.sC_s = stride_c;
  d.gs_c = batch_count;
  d.copies = batch_count;
  d.variant = variant;
  if (swap) rqc::swap_operands(d);
  const int lp_kind = kernel == rqc::KERN_MFMA16 ? (mma_prec == RQC_F16 ? rqc::ST_F16 : rqc::ST_BF16) : 0;
  rqc::hip_check(rqc::launch_step(d, kern, swap ? store_b : store_a, swap ? store_a : store_b, store_c,
                                  lp_kind, static_cast<hipStream_t>(stream)),
                 "pair contract (stored)");
  return RQC_OK;
  RQC_CATCH
}

rqc_status rqc_batch_xeb(const double* amps, uint64_t n_amps, int32_t n_qubits,
                         const uint64_t* samples, uint64_t n_samples, double* out,
                         rqc_stream stream) {
  RQC_TRY
  if (!amps || !out) throw rqc::Error{RQC_EINVAL, "NULL device pointer"};
  if (n_samples && !samples) throw rqc::Error{RQC_EINVAL, "samples is NULL"};
  if (n_qubits < 1 || n_qubits > 1000) throw rqc::Error{RQC_EINVAL, "n_qubits out of range"};
  rqc::hip_check(rqc::launch_batch_stats(amps, n_amps, n_qubits, samples, n_samples, out,
                                         static_cast<hipStream_t>(stream)),
                 "batch statistics");
  return RQC_OK;
  RQC_CATCH
}

rqc_status rqc_permute(const int32_t* labels_in, const int32_t* labels_out, int32_t rank,
                       const void* in, void* out, rqc_stream stream) {
  RQC_TRY
  if (!in || !out || rank < 0 || rank > 40 || (rank && (!labels_in || !labels_out)))
    throw rqc::Error{RQC_EINVAL, "bad argument"};
  if (in == out) throw rqc::Error{RQC_EINVAL, "in-place permutation not supported"};
  std::vector<int8_t> src(rank > 0 ? rank : 1);
  std::vector<int> li(labels_in, labels_in + rank);
  for (int i = 0; i < rank; ++i) {
    const int x = labels_out[rank - 1 - i];  // output bit i
    auto it = std::find(li.begin(), li.end(), x);
    if (it == li.end()) throw rqc::Error{RQC_EINVAL, "labels_out is not a permutation of labels_in"};
    src[i] = (int8_t)(rank - 1 - (it - li.begin()));
  }
  {
    std::vector<int8_t> s(src.begin(), src.begin() + rank);
    std::sort(s.begin(), s.end());
    if (std::adjacent_find(s.begin(), s.end()) != s.end()) throw rqc::Error{RQC_EINVAL, "repeated label"};
  }
  if (rank == 0) {
    rqc::hip_check(hipMemcpyAsync(out, in, 8, hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)), "copy");
    return RQC_OK;
  }
  rqc::hip_check(rqc::launch_permute(in, out, rank, src.data(), static_cast<hipStream_t>(stream)), "permute");
  return RQC_OK;
  RQC_CATCH
}

rqc_status rqc_cgemm(int64_t M, int64_t N, int64_t K, const void* A, const void* B, void* C,
                     rqc_stream stream) {
  RQC_TRY
  auto lg = [](int64_t x) {
    if (x <= 0 || (x & (x - 1))) throw rqc::Error{RQC_EUNSUPPORTED, "dimensions must be powers of two"};
    int l = 0;
    while ((int64_t(1) << l) < x) ++l;
    return l;
  };
  const int m = lg(M), n = lg(N), k = lg(K);
  if (!A || !B || !C) throw rqc::Error{RQC_EINVAL, "NULL device pointer"};
  std::vector<int> la, lb, lc;
  for (int i = 0; i < m; ++i) la.push_back(i);
  for (int i = 0; i < k; ++i) la.push_back(100 + i);
  for (int i = 0; i < k; ++i) lb.push_back(100 + i);
  for (int i = 0; i < n; ++i) lb.push_back(200 + i);
  for (int i = 0; i < m; ++i) lc.push_back(i);
  for (int i = 0; i < n; ++i) lc.push_back(200 + i);
  int use = -1;
  rqc::StepDesc d = rqc::make_pair_desc(la, lb, lc, use);
  d.A = A;
  d.B = B;
  d.C = C;
  rqc::hip_check(rqc::launch_step(d, use, rqc::ST_C64, rqc::ST_C64, rqc::ST_C64, 0,
                                  static_cast<hipStream_t>(stream)),
                 "cgemm");
  return RQC_OK;
  RQC_CATCH
}

}  // extern "C"

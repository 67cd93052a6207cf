// Per-step kernel tuning and the precision pre-analysis.
//
// Tuning (Section 5.4 designs a kernel per contraction case; here the choice
// is measured): every step with more than one valid (kernel, variant) pair is
// timed on the device for the call shape the workspace allows, and the
// fastest pair is kept per step and precision mode.  Choices can be cached
// in a text file keyed by a canonical signature of the step.
//
// Pre-analysis (Section 5.5: the parts of the network near the slice cuts
// are the most precision-sensitive): one slice is contracted in FP32, then
// once per candidate step with only that step in reduced precision; the
// least sensitive steps are taken into reduced precision while the error
// estimate stays within the target.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>

#include "executor.h"

namespace rqc {

namespace {

int pos_of(const std::vector<int>& l, int x) {
  for (size_t i = 0; i < l.size(); ++i)
    if (l[i] == x) return (int)i;
  return -1;
}

// Canonical description of a step's shape: labels renamed in order of first
// appearance in C, then A; storage and sharing of the operands; group size.
std::string signature(const rqc_plan* p, const GroupLayout& L, size_t i) {
  const Step& st = p->pd.steps[i];
  std::vector<int> names;
  auto id = [&](int x) {
    int k = pos_of(names, x);
    if (k < 0) {
      names.push_back(x);
      k = (int)names.size() - 1;
    }
    return k;
  };
  std::ostringstream o;
  o << "p" << L.prec << "_g" << L.gs << "x" << L.gb << "_C";
  for (int x : st.lc) o << "." << id(x);
  o << "_A";
  for (int x : st.la) o << "." << id(x);
  o << "_B";
  for (int x : st.lb) o << "." << id(x);
  const Placement &A = L.place[st.a], &B = L.place[st.b], &C = L.place[st.node];
  o << "_s" << A.store << B.store << C.store << "_d" << A.dep_s << A.dep_b << B.dep_s << B.dep_b
    << C.dep_s << C.dep_b << "_v" << (p->sel_desc[L.prec][i].variant & kVarFP32Math);
  return o.str();
}

// Valid (kernel, variant) pairs of step i in mode m; the first is the
// current choice.
std::vector<std::pair<int, int>> candidates(rqc_plan* p, int m, size_t i) {
  const Step& st = p->pd.steps[i];
  const int cur = p->sel_kern[m][i];
  const int base_var = p->sel_desc[m][i].variant & kVarFP32Math;
  std::vector<std::pair<int, int>> c{{cur, p->sel_desc[m][i].variant}};
  auto valid = [&](int k, int v = 0) {
    int kk = k;
    step_desc(st, kk, v);
    return kk == k;
  };
  auto add = [&](int k, int v) {
    v |= base_var;
    for (auto& x : c)
      if (x.first == k && x.second == v) return;
    c.push_back({k, v});
  };
  const bool fp32_mma = cur == KERN_MFMA || (cur == KERN_ROWS && valid(KERN_MFMA));
  if (fp32_mma && valid(KERN_MFMA))
    for (int v : {kVarTiles, kVarTiles | kVar4M, kVarPersistent, kVarPersistent | kVar4M})
      add(KERN_MFMA, v);
  // Exchanged operands: a 128- or 256-column output becomes one or two row
  // tiles, so the large operand is read once or twice instead of two or
  // four times (the small one stays in L2).
  if (fp32_mma && st.n >= 7 && st.m > st.n && valid(KERN_MFMA, kVarSwap))
    for (int v : {kVarTiles, kVarPersistent}) add(KERN_MFMA, v | kVarSwap);
  if (cur == KERN_MFMA16 && st.k >= 5 && st.k <= 7) add(KERN_MFMA16, kVarStream);
  // The same exchange on the 16-bit matrix cores: a 128-column output is
  // written in whole 128-column rows (one row tile) instead of half rows.
  if (cur == KERN_MFMA16 && st.n >= 7 && st.m > st.n && valid(KERN_MFMA16, kVarSwap))
    add(KERN_MFMA16, kVarSwap);
  // Reduced precision: a row-kernel step that the 16-bit matrix-core kernel
  // can also take.
  if (m != RQC_F32 && cur == KERN_ROWS && !base_var && valid(KERN_MFMA16)) add(KERN_MFMA16, 0);
  if ((cur == KERN_MFMA || cur == KERN_MFMA16) && valid(KERN_ROWS)) add(KERN_ROWS, 0);
  if (c.size() == 1) c.clear();
  return c;
}

void copy_call_inputs(rqc_plan* p, const GroupLayout& L, const WsLayout& W, char* ws,
                      const std::vector<uint64_t>& ids, const std::vector<uint8_t>& bits,
                      hipStream_t s) {
  hip_check(hipMemcpyAsync(ws + W.ids_off, ids.data(), 8 * ids.size(), hipMemcpyHostToDevice, s), "ids");
  hip_check(hipMemcpyAsync(ws + W.bits_off, bits.data(), bits.size(), hipMemcpyHostToDevice, s), "bits");
  if (!L.jobs.empty())
    hip_check(hipMemcpyAsync(ws + W.jobs_off, L.jobs.data(), sizeof(LeafJob) * L.jobs.size(),
                             hipMemcpyHostToDevice, s),
              "jobs");
}

struct Events {
  hipEvent_t a = nullptr, b = nullptr;
  Events() {
    hip_check(hipEventCreate(&a), "event");
    hip_check(hipEventCreate(&b), "event");
  }
  ~Events() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

}  // namespace

void autotune(rqc_plan* p, int prec, uint64_t n_ids, uint64_t n_batch, void* ws_v, size_t ws_bytes,
              const char* cache_path, hipStream_t s, rqc_tune_report* rep) {
  std::memset(rep, 0, sizeof *rep);
  PlanData& pd = p->pd;
  if (!p->bound) throw Error{RQC_EINVAL, "plan is not bound to device memory"};
  if (prec != RQC_F32 && prec != RQC_F16 && prec != RQC_BF16) throw Error{RQC_EINVAL, "bad precision"};
  if (!ws_v || (reinterpret_cast<uintptr_t>(ws_v) & 255) != 0)
    throw Error{RQC_EINVAL, "workspace NULL or not 256-byte aligned"};
  const uint64_t n_slices = uint64_t(1) << pd.sliced.size();
  if (n_ids == 0 || n_ids > n_slices) n_ids = n_slices;
  if (n_batch == 0) throw Error{RQC_EINVAL, "n_batch must be positive"};
  int gs, gb;
  choose_group(p, prec, n_ids, n_batch, ws_bytes, gs, gb);
  // Cached choices.
  std::map<std::string, std::pair<int, int>> cache;
  if (cache_path && *cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      if (line.empty() || line[0] == '#') continue;
      std::istringstream is(line);
      std::string sig;
      int k = -1, v = 0;
      if (is >> sig >> k >> v) cache[sig] = {k, v};
    }
  }
  const GroupLayout L = group_layout(p, prec, gs, gb);  // copy: select_steps drops the cache
  const WsLayout W = ws_layout(p, L, (uint64_t)gs, (uint64_t)gb);
  char* ws = static_cast<char*>(ws_v);
  // One call on the first group fills the workspace with this plan's data
  // (the timed launches then read realistic operands and scales).
  std::vector<uint64_t> ids(gs);
  for (int i = 0; i < gs; ++i) ids[i] = (uint64_t)i;
  std::vector<uint8_t> bits((size_t)gb * std::max<size_t>(1, pd.net.closed.size()), 0);
  copy_call_inputs(p, L, W, ws, ids, bits, s);
  double* out = reinterpret_cast<double*>(ws + W.tmp_off);
  record_call(p, L, W, (uint64_t)gs, (uint64_t)gb, ws, out, nullptr, 0, s);
  hip_check(hipStreamSynchronize(s), "tuning warm-up");
  int32_t* flags = reinterpret_cast<int32_t*>(ws + W.flags_off);
  Events ev;
  std::vector<std::pair<std::string, std::pair<int, int>>> learned;
  for (size_t i = 0; i < pd.steps.size(); ++i) {
    if (pd.steps[i].invariant) continue;
    const auto cand = candidates(p, prec, i);
    if (cand.empty()) continue;
    rep->steps++;
    const std::string sig = signature(p, L, i);
    std::pair<int, int> best = cand[0];
    auto hit = cache.find(sig);
    const StepDesc keep_d = p->sel_desc[prec][i];
    const int keep_k = p->sel_kern[prec][i];
    if (hit != cache.end()) {
      best = hit->second;
      rep->cached++;
    } else {
      double best_ms = 1e30;
      for (size_t c = 0; c < cand.size(); ++c) {
        int k = cand[c].first;
        StepDesc d0 = step_desc(pd.steps[i], k, cand[c].second);
        if (k != cand[c].first) continue;
        d0.variant = cand[c].second;
        p->sel_desc[prec][i] = d0;
        p->sel_kern[prec][i] = k;
        const StepDesc d = bind_step(p, L, W, ws, i, gs, gb, flags, 0);
        hip_check(launch_bound_step(p, L, i, d, k, s), "tuning launch");
        hip_check(hipEventRecord(ev.a, s), "event");
        constexpr int kReps = 3;
        for (int r = 0; r < kReps; ++r) hip_check(launch_bound_step(p, L, i, d, k, s), "tuning launch");
        hip_check(hipEventRecord(ev.b, s), "event");
        hip_check(hipEventSynchronize(ev.b), "event sync");
        float ms = 0.f;
        hip_check(hipEventElapsedTime(&ms, ev.a, ev.b), "event time");
        const double t = ms / kReps;
        if (c == 0) rep->ms_default += t;
        if (t < best_ms) {
          best_ms = t;
          best = cand[c];
        }
      }
      rep->ms_tuned += best_ms;
      rep->timed++;
      learned.push_back({sig, best});
    }
    p->sel_desc[prec][i] = keep_d;
    p->sel_kern[prec][i] = keep_k;
    if (best != cand[0]) rep->changed++;
    p->tuned_kern[prec][i] = best.first;
    p->tuned_var[prec][i] = best.second & ~kVarFP32Math;
  }
  hip_check(hipStreamSynchronize(s), "tuning");
  select_steps(p);
  if (cache_path && *cache_path && !learned.empty()) {
    for (auto& kv : learned) cache[kv.first] = kv.second;
    std::ofstream o(cache_path, std::ios::trunc);
    if (!o) throw Error{RQC_EINVAL, std::string("cannot write tuning cache ") + cache_path};
    o << "# rqc per-step kernel choices: signature kernel variant\n";
    for (auto& kv : cache) o << kv.first << " " << kv.second.first << " " << kv.second.second << "\n";
  }
}

void calibrate(rqc_plan* p, int prec, uint64_t slice_id, const uint8_t* bits_in, double target,
               double err_floor, void* ws_v, size_t ws_bytes, hipStream_t s, rqc_calib_report* rep) {
  std::memset(rep, 0, sizeof *rep);
  PlanData& pd = p->pd;
  if (!p->bound) throw Error{RQC_EINVAL, "plan is not bound to device memory"};
  if (prec != RQC_F16 && prec != RQC_BF16) throw Error{RQC_EINVAL, "calibration needs RQC_F16 or RQC_BF16"};
  if (!(target > 0.0) || !(err_floor >= 0.0)) throw Error{RQC_EINVAL, "target must be positive"};
  if (slice_id >= (uint64_t(1) << pd.sliced.size())) throw Error{RQC_EINVAL, "slice id out of range"};
  if (!pd.net.closed.empty() && !bits_in) throw Error{RQC_EINVAL, "closed_bits is NULL"};
  if (!ws_v || (reinterpret_cast<uintptr_t>(ws_v) & 255) != 0)
    throw Error{RQC_EINVAL, "workspace NULL or not 256-byte aligned"};
  const size_t ne = size_t(1) << pd.net.open.size();
  const size_t out_bytes = (16 * ne + 255) & ~size_t(255);
  if (ws_bytes < out_bytes + 256) throw Error{RQC_EHBM, "workspace too small for calibration"};
  const size_t main_bytes = (ws_bytes - out_bytes) & ~size_t(255);
  char* ws = static_cast<char*>(ws_v);
  double* out = reinterpret_cast<double*>(ws + main_bytes);
  std::vector<uint8_t> bits(bits_in, bits_in + pd.net.closed.size());
  std::vector<std::complex<double>> host(ne);
  auto run = [&](int mode) {
    PendingRun r;
    contract(p, &slice_id, 1, bits.data(), 1, mode, ws, main_bytes, out, nullptr, s, r, true);
    rqc_run_report rr;
    report(p, r, s, &rr);
    std::vector<double> h(2 * ne);
    hip_check(hipMemcpy(h.data(), out, 16 * ne, hipMemcpyDeviceToHost), "calibration result");
    for (size_t e = 0; e < ne; ++e) host[e] = {h[2 * e], h[2 * e + 1]};
    return host;
  };
  const std::vector<char> keep = p->lp_on[prec];
  try {
    const std::vector<std::complex<double>> ref = run(RQC_F32);
    double rms = 0.0;
    for (auto& v : ref) rms += std::norm(v);
    rms = std::sqrt(rms / (double)ne);
    const double unit = std::max(rms, err_floor);
    if (!(unit > 0.0)) throw Error{RQC_ENUMERIC, "the calibration slice is zero"};
    auto err_of = [&](const std::vector<std::complex<double>>& a) {
      double e = 0.0;
      for (size_t i = 0; i < ne; ++i) e = std::max(e, std::abs(a[i] - ref[i]));
      return e / unit;
    };
    // Candidates: steps whose output the size rule stores in 16 bits, or
    // whose kernel differs in reduced precision (16-bit matrix cores).
    std::vector<std::pair<double, size_t>> sens;
    for (size_t i = 0; i < pd.steps.size(); ++i) {
      const Step& st = pd.steps[i];
      if (st.invariant) continue;
      const bool store16 = prec == RQC_BF16 ? st.lp_bf16 : st.lp;
      if (!store16 && p->kern_lp[i] == p->kern[i]) continue;
      std::vector<char> one(pd.steps.size(), 0);
      one[i] = 1;
      p->lp_on[prec] = one;
      select_steps(p);
      sens.push_back({err_of(run(prec)), i});
    }
    rep->candidates = (int32_t)sens.size();
    std::sort(sens.begin(), sens.end());
    std::vector<char> mask(pd.steps.size(), 0);
    std::vector<std::pair<double, size_t>> kept;
    double est2 = 0.0;
    for (auto& e : sens) {
      if (std::sqrt(est2 + e.first * e.first) <= target) {
        est2 += e.first * e.first;
        mask[e.second] = 1;
        kept.push_back(e);
      }
    }
    if (!sens.empty()) {
      rep->min_step_err = sens.front().first;
      rep->max_step_err = sens.back().first;
    }
    // Check the assignment as a whole; drop the most sensitive kept step
    // while the measured error is above the target.
    double measured = 0.0;
    while (true) {
      p->lp_on[prec] = mask;
      select_steps(p);
      measured = kept.empty() ? 0.0 : err_of(run(prec));
      if (measured <= target || kept.empty()) break;
      mask[kept.back().second] = 0;
      est2 -= kept.back().first * kept.back().first;
      kept.pop_back();
    }
    rep->reduced = (int32_t)kept.size();
    rep->estimated_err = std::sqrt(std::max(0.0, est2));
    rep->measured_err = measured;
  } catch (...) {
    p->lp_on[prec] = keep;
    select_steps(p);
    throw;
  }
}

}  // namespace rqc

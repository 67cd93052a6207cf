// Executor: turns a plan into device work.
//
// Slices (Section 5.1) and bitstrings are the batch dimension of every step:
// a group of gs slices x gb bitstrings runs each contraction step as one
// batched launch, tensors that do not depend on the slice (or on the
// bitstring) are shared through zero copy strides, and tensors that depend
// on neither are computed once when the plan is bound and stay resident.
// A whole contraction call -- all groups, all steps, the FP64 slice sum --
// is captured once into a HIP graph and replayed with one launch.
#include "executor.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <list>

namespace rqc {

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Error{RQC_EDEVICE, std::string(what) + ": " + hipGetErrorString(e)};
}

static int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }
static int elsize(int store) { return store == ST_C64 ? 8 : 4; }

static int pos_in(const std::vector<int>& l, int x) {
  for (size_t i = 0; i < l.size(); ++i)
    if (l[i] == x) return (int)(l.size() - 1 - i);
  return -1;
}

// ---------------------------------------------------------------------------
// Tile selection for one step (the permutation folded into the tiles)
// ---------------------------------------------------------------------------
StepDesc step_desc(const Step& st, int& kernel, int variant) {
  return variant & kVarSwap ? make_pair_desc(st.lb, st.la, st.lc, kernel)
                            : make_pair_desc(st.la, st.lb, st.lc, kernel);
}

void swap_operands(StepDesc& d) {
  std::swap(d.A, d.B);
  std::swap(d.expA, d.expB);
  std::swap(d.maxA, d.maxB);
  std::swap(d.maxA_const, d.maxB_const);
  std::swap(d.sA_s, d.sB_s);
  std::swap(d.sA_b, d.sB_b);
  std::swap(d.eA_s, d.eB_s);
  std::swap(d.eA_b, d.eB_b);
}

StepDesc make_pair_desc(const std::vector<int>& la, const std::vector<int>& lb,
                        const std::vector<int>& lc, int& kernel) {
  StepDesc d;
  std::memset(&d, 0, sizeof d);
  std::vector<int> M, N, K;
  for (int x : la) {
    const bool inb = pos_in(lb, x) >= 0, inc = pos_in(lc, x) >= 0;
    if (inb && inc) throw Error{RQC_EUNSUPPORTED, "index shared by A, B and C"};
    if (inb) K.push_back(x);
    else if (inc) M.push_back(x);
    else throw Error{RQC_EINVAL, "label of A in neither B nor C"};
  }
  for (int x : lb)
    if (pos_in(la, x) < 0) {
      if (pos_in(lc, x) < 0) throw Error{RQC_EINVAL, "label of B in neither A nor C"};
      N.push_back(x);
    }
  if (M.size() + N.size() != lc.size()) throw Error{RQC_EINVAL, "labels of C do not match"};
  {
    std::vector<int> s(lc);
    std::sort(s.begin(), s.end());
    if (std::adjacent_find(s.begin(), s.end()) != s.end()) throw Error{RQC_EINVAL, "repeated label"};
  }
  const int m = (int)M.size(), n = (int)N.size(), k = (int)K.size();
  if (m + k > 40 || n + k > 40 || m + n > 40) throw Error{RQC_EUNSUPPORTED, "rank above 40"};
  auto pa = [&](int x) { return pos_in(la, x); };
  auto pb = [&](int x) { return pos_in(lb, x); };
  auto pc = [&](int x) { return pos_in(lc, x); };
  // Row-streaming kernel: K is the lowest k address bits of both A and B, in
  // the same order; B small (N K <= 4096, staged whole in LDS).  Outputs of
  // 64 or 128 columns only with sums of at most 16 (one K chunk, the columns
  // walked in groups).
  bool rows_ok = k <= 12 && (n <= 5 || (n <= 7 && k <= 4)) && (int64_t(1) << (n + k)) <= 4096;
  for (int p = 0; p < k && rows_ok; ++p) {
    const int xa = la[la.size() - 1 - p];
    rows_ok = pos_in(lb, xa) == p;
  }
  const bool mfma_ok = m >= 7 && n >= 6 && k >= 4;
  const bool mfma16_ok = m >= 7 && n >= 6 && k >= 4;
  // Short sums (k <= 4) are memory-bound: row streaming beats one MFMA chunk.
  if (kernel < 0)
    kernel = (mfma_ok && !(rows_ok && k <= 4)) ? KERN_MFMA : (rows_ok ? KERN_ROWS : KERN_SIMT);
  if (kernel == KERN_MFMA16 && !mfma16_ok) kernel = mfma_ok ? KERN_MFMA : KERN_SIMT;
  if (kernel == KERN_MFMA && !mfma_ok) kernel = KERN_SIMT;
  if (kernel == KERN_ROWS && !rows_ok) kernel = KERN_SIMT;
  int rt, nt, kt;
  if (kernel == KERN_MFMA) {
    rt = 7;
    nt = 6;
    kt = 4;
  } else if (kernel == KERN_MFMA16) {
    rt = 7;
    nt = 6;
    kt = k >= 5 ? 5 : 4;  // sums of 16 fill half of the kernel's 32-term chunk
  } else if (kernel == KERN_ROWS) {
    kt = k;
    nt = n;
    // 256 rows per workgroup; output columns staged 8 at a time (all of
    // them for N <= 8, so that the staged tile covers C's lowest address
    // bits and the stores coalesce).
    d.ncb = std::min(n, 3);
    rt = std::min(m, 8);
    if ((int64_t(1) << (n + k)) > 4096) throw Error{RQC_EINVAL, "internal: row kernel B too large"};
  } else if (m + n <= 8) {
    // Tiny output, long sum: deep K tiles (split-K spreads them over blocks).
    rt = m;
    nt = n;
    kt = std::min(k, 12 - std::max(m, n));
    while (kt > 0 && (((int64_t(1) << rt) * ((int64_t(1) << kt) + 1) +
                       (int64_t(1) << kt) * ((int64_t(1) << nt) + 1)) * 8) > 56 * 1024)
      --kt;
  } else {
    kt = std::min(k, 4);
    nt = std::min(n, 4);
    rt = std::min(m, std::min(11 - nt, 12 - kt));
    // Generic kernel: <= 8 owned C elements per thread, tables of <= 12 bits.
    if (rt + nt > 11 || rt + kt > 12 || kt + nt > 12)
      throw Error{RQC_EINVAL, "internal: generic tile too large"};
  }
  auto by = [](std::vector<int> v, auto key) {
    std::stable_sort(v.begin(), v.end(), [&](int x, int y) { return key(x) < key(y); });
    return v;
  };
  std::vector<int> Ms, Ns, Ks;
  if (kernel == KERN_ROWS) {
    // Rows: the lowest M bits of A (just above K); columns in C's order so
    // that a chunk of output columns is (nearly) contiguous in C.
    Ms = by(M, pa);
    Ns = by(N, pc);
    Ks = by(K, pa);
  } else {
    Ms = by(M, [&](int x) { return std::min(pa(x), pc(x)); });
    Ns = by(N, [&](int x) { return std::min(pb(x), pc(x)); });
    Ks = by(K, [&](int x) { return std::min(pa(x), pb(x)); });
  }
  std::vector<int> Rt(Ms.begin(), Ms.begin() + rt), Ro(Ms.begin() + rt, Ms.end());
  std::vector<int> Nt(Ns.begin(), Ns.begin() + nt), No(Ns.begin() + nt, Ns.end());
  std::vector<int> Kt(Ks.begin(), Ks.begin() + kt), Ko(Ks.begin() + kt, Ks.end());
  Ro = by(Ro, pc);
  No = by(No, pc);
  Ko = by(Ko, pa);
  // One workgroup of 256 work-items per output tile, and a launch holds fewer
  // than 2^32 work-items along x.
  if ((int)(Ro.size() + No.size()) > 23)
    throw Error{RQC_EUNSUPPORTED, "step output has more than 2^23 tiles"};

  auto tile = [&](TileMap& t, const std::vector<std::pair<int, int>>& bits, auto posf) {
    // bits: (label, role); cbit = index inside the role's tile list
    std::vector<std::tuple<int, int, int>> v;  // (gpos, role, cbit)
    for (auto& br : bits) {
      const int x = br.first, role = br.second;
      const std::vector<int>& lst = role == 0 ? Rt : (role == 1 ? Nt : Kt);
      const int cb = (int)(std::find(lst.begin(), lst.end(), x) - lst.begin());
      v.emplace_back(posf(x), role, cb);
    }
    std::sort(v.begin(), v.end());
    t.nbits = (int)v.size();
    for (size_t i = 0; i < v.size(); ++i) {
      t.gpos[i] = (int8_t)std::get<0>(v[i]);
      t.role[i] = (int8_t)std::get<1>(v[i]);
      t.cbit[i] = (int8_t)std::get<2>(v[i]);
    }
  };
  std::vector<std::pair<int, int>> ba, bb, bc;
  for (int x : Rt) ba.push_back({x, 0}), bc.push_back({x, 0});
  for (int x : Kt) ba.push_back({x, 2}), bb.push_back({x, 2});
  for (int x : Nt) bb.push_back({x, 1}), bc.push_back({x, 1});
  if (kernel != KERN_ROWS) {
    tile(d.tA, ba, pa);
    tile(d.tB, bb, pb);
    tile(d.tC, bc, pc);
  } else {
    // tB: column bit j (in C order) -> its B position; tC: rows and the
    // chunk's low column bits; nh_C: C positions of the chunk-selecting bits.
    d.tB.nbits = n;
    for (int j = 0; j < n; ++j) {
      d.tB.gpos[j] = (int8_t)pb(Nt[j]);
      d.tB.role[j] = 1;
      d.tB.cbit[j] = (int8_t)j;
    }
    std::vector<std::pair<int, int>> bcr;
    for (int x : Rt) bcr.push_back({x, 0});
    for (int j = 0; j < d.ncb; ++j) bcr.push_back({Nt[j], 1});
    tile(d.tC, bcr, pc);
    for (int j = d.ncb; j < n; ++j) d.nh_C[j - d.ncb] = (int8_t)pc(Nt[j]);
    // Vector stores need C's two lowest address bits to be the tile's
    // lowest bits, and whole groups of four per thread.
    d.vec_c = (d.tC.nbits >= 2 && d.tC.gpos[0] == 0 && d.tC.gpos[1] == 1 &&
               d.tC.nbits >= 8) ? 1 : 0;
  }
  d.rt = rt;
  d.nt = nt;
  d.kt = kt;
  d.n_ro = (int)Ro.size();
  d.n_no = (int)No.size();
  d.n_ko = (int)Ko.size();
  for (size_t i = 0; i < Ro.size(); ++i) d.ro_A[i] = (int8_t)pa(Ro[i]), d.ro_C[i] = (int8_t)pc(Ro[i]);
  for (size_t i = 0; i < No.size(); ++i) d.no_B[i] = (int8_t)pb(No[i]), d.no_C[i] = (int8_t)pc(No[i]);
  for (size_t i = 0; i < Ko.size(); ++i) d.ko_A[i] = (int8_t)pa(Ko[i]), d.ko_B[i] = (int8_t)pb(Ko[i]);
  d.k_total = k;
  d.n_row_tiles = 1 << d.n_ro;
  d.n_col_tiles = 1 << d.n_no;
  d.gs_c = 1;
  d.copies = 1;
  d.flag_n = 1;
  // The 16-term chunk of the 16-bit kernel exists for the vector layout only.
  if (kernel == KERN_MFMA16 && kt == 4 && !lp_vec_layout(d)) {
    kernel = KERN_MFMA;
    return make_pair_desc(la, lb, lc, kernel);
  }
  return d;
}

// ---------------------------------------------------------------------------
// Residency
// ---------------------------------------------------------------------------
static std::vector<cd> permute_leaf(const Leaf& L, const std::vector<int>& layout) {
  const int r = (int)layout.size(), rf = (int)L.labels.size();
  if (r != rf) throw Error{RQC_EINVAL, "internal: leaf layout rank"};
  std::vector<cd> out(size_t(1) << r);
  std::vector<int> src_pos(r);
  for (int i = 0; i < r; ++i) src_pos[i] = pos_in(L.labels, layout[r - 1 - i]);
  for (size_t e = 0; e < out.size(); ++e) {
    size_t a = 0;
    for (int i = 0; i < r; ++i)
      if ((e >> i) & 1) a |= size_t(1) << src_pos[i];
    out[e] = L.data[a];
  }
  return out;
}

size_t resident_bytes(rqc_plan* p) {
  PlanData& pd = p->pd;
  const int nn = (int)pd.tree.left.size();
  const int nl = pd.tree.n_leaves;
  p->leaf_store_off.assign(nl, 0);
  p->leaf_max.assign(nl, 0.f);
  int64_t elems = 0;
  for (int i = 0; i < nl; ++i) {
    p->leaf_store_off[i] = elems;
    elems += (int64_t)pd.net.leaves[i].data.size();
    float mx = 0.f;
    for (const cd& v : pd.net.leaves[i].data)
      mx = std::max(mx, (float)std::max(std::abs(v.real()), std::abs(v.imag())));
    p->leaf_max[i] = mx;
  }
  p->leaf_store_elems = elems;
  int64_t off = align256(elems * 8);
  p->inv_off.assign(nn, -1);
  for (int v = 0; v < nn; ++v) {
    if (pd.dep_s[v] || pd.dep_b[v]) continue;
    if (v >= nl && pd.step_of_node[v] < 0) continue;  // unused node id
    p->inv_off[v] = off;
    off = align256(off + (int64_t(8) << pd.node_labels[v].size()));
  }
  p->inv_max_off = off;
  off = align256(off + 4 * (int64_t)nn);
  p->inv_exp_off = off;
  off = align256(off + 4 * (int64_t)nn);
  p->inv_bytes = off;
  p->tmpl.clear();
  p->kern.clear();
  p->tmpl_lp.clear();
  p->kern_lp.clear();
  for (const Step& st : pd.steps) {
    int k = -1;
    p->tmpl.push_back(make_pair_desc(st.la, st.lb, st.lc, k));
    p->kern.push_back(k);
    // Reduced precision: dense steps go to the FP16/BF16 MFMA (sums of 16
    // only with the vector layout; make_pair_desc falls back otherwise).
    int k2 = k == KERN_MFMA ? KERN_MFMA16 : k;
    p->tmpl_lp.push_back(make_pair_desc(st.la, st.lb, st.lc, k2));
    p->kern_lp.push_back(k2);
  }
  for (int m = 0; m < 3; ++m) {
    p->lp_on[m].assign(pd.steps.size(), m == RQC_F32 ? 0 : 1);
    p->tuned_kern[m].assign(pd.steps.size(), -1);
    p->tuned_var[m].assign(pd.steps.size(), 0);
  }
  select_steps(p);
  return (size_t)off;
}

bool step_lp_store(const rqc_plan* p, int prec, size_t i) {
  if (prec == RQC_F32 || !p->lp_on[prec][i]) return false;
  const Step& st = p->pd.steps[i];
  return prec == RQC_BF16 ? st.lp_bf16 : st.lp;
}

void select_steps(rqc_plan* p) {
  const PlanData& pd = p->pd;
  const bool storage_only = pd.opts.precision_policy == RQC_POLICY_STORAGE;
  for (int m = 0; m < 3; ++m) {
    p->sel_desc[m].resize(pd.steps.size());
    p->sel_kern[m].resize(pd.steps.size());
    for (size_t i = 0; i < pd.steps.size(); ++i) {
      const Step& st = pd.steps[i];
      // Reduced-precision arithmetic: the step's LP kernel, unless the
      // policy keeps all arithmetic in FP32 or the step was taken out of
      // reduced precision.
      const bool lp_math = m != RQC_F32 && p->lp_on[m][i] && !storage_only;
      int k = lp_math ? p->kern_lp[i] : p->kern[i];
      StepDesc d = lp_math ? p->tmpl_lp[i] : p->tmpl[i];
      int var = p->tuned_var[m][i];
      if (p->tuned_kern[m][i] >= 0) {
        int kt = p->tuned_kern[m][i];
        StepDesc dt = step_desc(st, kt, var);
        if (kt == p->tuned_kern[m][i]) {
          k = kt;
          d = dt;
        } else {
          var &= ~kVarSwap;
        }
      } else {
        var &= ~kVarSwap;
      }
      d.variant = var;
      if (m != RQC_F32 && !lp_math) d.variant |= kVarFP32Math;
      p->sel_desc[m][i] = d;
      p->sel_kern[m][i] = k;
    }
  }
  p->layouts.clear();
  clear_graphs(p);
}

void bind_plan(rqc_plan* p, void* dev, size_t bytes, hipStream_t s) {
  const size_t need = resident_bytes(p);
  if (bytes < need) throw Error{RQC_EHBM, "resident memory too small: need " + std::to_string(need)};
  if ((reinterpret_cast<uintptr_t>(dev) & 255) != 0) throw Error{RQC_EINVAL, "resident memory not 256-byte aligned"};
  PlanData& pd = p->pd;
  const int nl = pd.tree.n_leaves;
  const int nn = (int)pd.tree.left.size();
  char* base = static_cast<char*>(dev);
  // Leaf store (natural label order, selectors included).
  std::vector<float> host(2 * p->leaf_store_elems);
  for (int i = 0; i < nl; ++i)
    for (size_t e = 0; e < pd.net.leaves[i].data.size(); ++e) {
      host[2 * (p->leaf_store_off[i] + e)] = (float)pd.net.leaves[i].data[e].real();
      host[2 * (p->leaf_store_off[i] + e) + 1] = (float)pd.net.leaves[i].data[e].imag();
    }
  hip_check(hipMemcpyAsync(base, host.data(), host.size() * 4, hipMemcpyHostToDevice, s), "upload leaves");
  // Invariant leaves in their layout order; maxima.
  std::vector<float> maxes(nn, 0.f);
  std::vector<std::vector<float>> keep;
  for (int i = 0; i < nl; ++i) {
    maxes[i] = p->leaf_max[i];
    if (p->inv_off[i] < 0) continue;
    std::vector<cd> v = permute_leaf(pd.net.leaves[i], pd.layout[i]);
    keep.emplace_back(2 * v.size());
    for (size_t e = 0; e < v.size(); ++e) {
      keep.back()[2 * e] = (float)v[e].real();
      keep.back()[2 * e + 1] = (float)v[e].imag();
    }
    hip_check(hipMemcpyAsync(base + p->inv_off[i], keep.back().data(), keep.back().size() * 4,
                             hipMemcpyHostToDevice, s),
              "upload invariant leaf");
  }
  hip_check(hipMemcpyAsync(base + p->inv_max_off, maxes.data(), 4 * nn, hipMemcpyHostToDevice, s),
            "upload maxima");
  const std::vector<int32_t> zeros(nn, 0);
  hip_check(hipMemcpyAsync(base + p->inv_exp_off, zeros.data(), 4 * nn, hipMemcpyHostToDevice, s),
            "upload exponents");
  // Slice-invariant subtrees: contracted once, kept resident.
  for (const Step& st : pd.steps) {
    if (!st.invariant) continue;
    const size_t si = &st - &pd.steps[0];
    const int kern = p->sel_kern[RQC_F32][si];
    StepDesc d = p->sel_desc[RQC_F32][si];
    d.A = base + p->inv_off[st.a];
    d.B = base + p->inv_off[st.b];
    d.C = base + p->inv_off[st.node];
    float* mx = reinterpret_cast<float*>(base + p->inv_max_off);
    int32_t* ex = reinterpret_cast<int32_t*>(base + p->inv_exp_off);
    d.maxA = mx + st.a;
    d.maxB = mx + st.b;
    d.maxC = mx + st.node;
    d.expA = ex + st.a;
    d.expB = ex + st.b;
    d.expC = ex + st.node;
    d.track = 1;
    d.lp_out = 0;
    d.copies = 1;
    d.gs_c = 1;
    if (d.variant & kVarSwap) swap_operands(d);
    hip_check(launch_step(d, kern, ST_C64, ST_C64, ST_C64, 0, s), "invariant step");
  }
  hip_check(hipStreamSynchronize(s), "bind");
  p->res = base;
  p->res_bytes = bytes;
  p->bound = true;
  clear_graphs(p);
}

void clear_graphs(rqc_plan* p) {
  for (auto& kv : p->graphs) {
    if (kv.second.done) {
      (void)hipEventSynchronize(kv.second.done);
      (void)hipEventDestroy(kv.second.done);
    }
    (void)hipGraphExecDestroy(kv.second.exec);
  }
  p->graphs.clear();
}

// ---------------------------------------------------------------------------
// Group memory layout
// ---------------------------------------------------------------------------
static GroupLayout compute_layout(rqc_plan* p, int prec, int gs, int gb) {
  PlanData& pd = p->pd;
  const int nn = (int)pd.tree.left.size();
  const int nl = pd.tree.n_leaves;
  GroupLayout L;
  L.prec = prec;
  L.gs = gs;
  L.gb = gb;
  L.place.assign(nn, Placement());
  // Exponents and maxima are kept in every precision (complex64 outputs are
  // normalised too); 16-bit storage only in reduced precision.
  const bool track = true;
  const bool lp_mode = prec != RQC_F32;
  const int lp_store = prec == RQC_F16 ? ST_F16 : ST_BF16;
  std::vector<int64_t> bytes(nn, 0);
  for (int v = 0; v < nn; ++v) {
    Placement& P = L.place[v];
    P.dep_s = pd.dep_s[v];
    P.dep_b = pd.dep_b[v];
    if (v >= nl && pd.step_of_node[v] < 0) continue;
    const int64_t E = int64_t(1) << pd.node_labels[v].size();
    if (v < nl) P.max_const = p->leaf_max[v];
    if (!P.dep_s && !P.dep_b) {
      P.resident = true;
      P.off = p->inv_off[v];
      P.store = ST_C64;
      if (v >= nl) P.m_off = p->inv_max_off + 4 * v;
      P.e_off = p->inv_exp_off + 4 * v;
      continue;
    }
    const int cs = P.dep_s ? gs : 1, cb = P.dep_b ? gb : 1;
    const bool lp16 = v >= nl && step_lp_store(p, prec, (size_t)pd.step_of_node[v]);
    P.store = (lp_mode && lp16) ? lp_store : ST_C64;
    P.s_stride = P.dep_s ? E : 0;
    P.b_stride = P.dep_b ? E * cs : 0;
    bytes[v] = align256(E * cs * cb * elsize(P.store));
    if (track && v >= nl) {
      P.es = P.dep_s ? 1 : 0;
      P.eb = P.dep_b ? cs : 0;
      P.e_off = L.scale_bytes;
      L.scale_bytes = align256(L.scale_bytes + 4 * cs * cb);
      P.m_off = L.scale_bytes;
      L.scale_bytes = align256(L.scale_bytes + 4 * cs * cb);
    }
  }
  // First-fit arena over the execution order.
  std::list<std::pair<int64_t, int64_t>> used;  // (offset, size) sorted
  int64_t peak = 0;
  auto alloc = [&](int64_t sz) {
    int64_t at = 0;
    auto it = used.begin();
    for (; it != used.end(); ++it) {
      if (it->first - at >= sz) break;
      at = std::max(at, it->first + it->second);
    }
    used.insert(it, {at, sz});
    peak = std::max(peak, at + sz);
    return at;
  };
  auto release = [&](int64_t at) {
    for (auto it = used.begin(); it != used.end(); ++it)
      if (it->first == at) {
        used.erase(it);
        return;
      }
  };
  for (int v = 0; v < nl; ++v)
    if (!L.place[v].resident) L.place[v].off = alloc(bytes[v]);
  L.ksplit.assign(pd.steps.size(), 0);
  L.p_off.assign(pd.steps.size(), -1);
  for (size_t i = 0; i < pd.steps.size(); ++i) {
    const Step& st = pd.steps[i];
    if (st.invariant) continue;
    L.place[st.node].off = alloc(bytes[st.node]);
    // Split-K for generic steps whose output tiles cannot fill the GPU.
    const StepDesc& t = p->sel_desc[prec][i];
    if (p->sel_kern[prec][i] == KERN_SIMT && t.n_ko >= 2) {
      const Placement& C = L.place[st.node];
      const int64_t copies = (int64_t)(C.dep_s ? gs : 1) * (C.dep_b ? gb : 1);
      const int64_t work = (int64_t)t.n_row_tiles * t.n_col_tiles * copies;
      // Enough workgroups to fill the GPU, and no more than 2^12 summed
      // chunks left per workgroup.
      int ks = 0;
      while (ks < t.n_ko && ((work << ks) < 4096 || t.n_ko - ks > 12)) ++ks;
      const int64_t cbytes = (int64_t(8) << pd.node_labels[st.node].size()) *
                             (C.dep_s ? gs : 1) * (C.dep_b ? gb : 1);
      while (ks > 0 && (cbytes << ks) > (int64_t(1) << 30)) --ks;
      if (ks > 0) {
        L.ksplit[i] = ks;
        L.p_off[i] = alloc(align256(cbytes << ks));
        release(L.p_off[i]);
      }
    }
    for (int x : {st.a, st.b})
      if (!L.place[x].resident) release(L.place[x].off);
  }
  L.arena_bytes = align256(peak);
  // Leaf jobs.
  std::vector<char> sliced(pd.net.labels.size(), 0);
  std::vector<int> slice_bit(pd.net.labels.size(), -1);
  for (size_t j = 0; j < pd.sliced.size(); ++j) {
    sliced[pd.sliced[j]] = 1;
    slice_bit[pd.sliced[j]] = (int)j;
  }
  for (int v = 0; v < nl; ++v) {
    const Placement& P = L.place[v];
    if (P.resident) continue;
    const Leaf& leaf = pd.net.leaves[v];
    LeafJob J;
    std::memset(&J, 0, sizeof J);
    J.src = p->leaf_store_off[v];
    J.dst = P.off / 8;
    const std::vector<int>& lay = pd.layout[v];
    J.rank = (int)lay.size();
    for (int i = 0; i < J.rank; ++i) J.pos[i] = (int8_t)pos_in(leaf.labels, lay[J.rank - 1 - i]);
    J.nsel = 0;
    for (int x : leaf.labels) {
      const bool closed = pd.net.labels[x].kind == CLOSED;
      if (!closed && !sliced[x]) continue;
      J.sel_pos[J.nsel] = (int8_t)pos_in(leaf.labels, x);
      J.sel_src[J.nsel] = closed ? (int16_t)(-pd.net.closed_col[x] - 1) : (int16_t)slice_bit[x];
      J.nsel++;
    }
    J.dep_s = P.dep_s;
    J.dep_b = P.dep_b;
    J.dst_store = ST_C64;
    J.out_s = (int32_t)P.s_stride;
    J.out_b = (int32_t)P.b_stride;
    L.max_leaf_rank = std::max(L.max_leaf_rank, J.rank);
    L.jobs.push_back(J);
  }
  return L;
}

const GroupLayout& group_layout(rqc_plan* p, int prec, int gs, int gb) {
  auto key = std::make_tuple(prec, gs, gb);
  auto it = p->layouts.find(key);
  if (it != p->layouts.end()) return it->second;
  if (p->layouts.size() > 64) p->layouts.clear();
  return p->layouts.emplace(key, compute_layout(p, prec, gs, gb)).first->second;
}

WsLayout ws_layout(rqc_plan* p, const GroupLayout& L, uint64_t n_ids, uint64_t n_batch) {
  const PlanData& pd = p->pd;
  WsLayout w;
  int64_t o = 0;
  w.ids_off = o;
  o = align256(o + 8 * (int64_t)n_ids);
  w.bits_off = o;
  o = align256(o + (int64_t)n_batch * (int64_t)std::max<size_t>(1, pd.net.closed.size()));
  w.n_bgroups = ((int64_t)n_batch + L.gb - 1) / L.gb;
  w.flags_off = o;
  o = align256(o + 4 * (int64_t)n_ids * w.n_bgroups);
  w.jobs_off = o;
  o = align256(o + (int64_t)sizeof(LeafJob) * (int64_t)std::max<size_t>(1, L.jobs.size()));
  w.tmp_off = o;
  o = align256(o + 16 * (int64_t)n_batch * (int64_t(1) << pd.net.open.size()));
  w.scale_off = o;
  o = align256(o + L.scale_bytes);
  w.arena_off = o;
  o = align256(o + L.arena_bytes);
  w.total = o;
  return w;
}

// ---------------------------------------------------------------------------
// Recording one call (captured into a graph, or run directly for re-runs)
// ---------------------------------------------------------------------------
// Descriptor of step i for one group (gsc slices x gbc bitstrings, slice
// flags at `gflags`) with its operands, strides and scale arrays bound.
StepDesc bind_step(rqc_plan* p, const GroupLayout& L, const WsLayout& W, char* ws, size_t i,
                   int gsc, int gbc, int32_t* gflags, int bias) {
  const PlanData& pd = p->pd;
  char* arena = ws + W.arena_off;
  char* scale = ws + W.scale_off;
  auto ptr = [&](const Placement& P) -> char* { return P.resident ? p->res + P.off : arena + P.off; };
  auto eptr = [&](const Placement& P) -> int32_t* {
    if (P.e_off < 0) return nullptr;
    return reinterpret_cast<int32_t*>(P.resident ? p->res + P.e_off : scale + P.e_off);
  };
  auto mptr = [&](const Placement& P) -> float* {
    if (P.m_off < 0) return nullptr;
    return reinterpret_cast<float*>(P.resident ? p->res + P.m_off : scale + P.m_off);
  };
  const Step& st = pd.steps[i];
  StepDesc d = p->sel_desc[L.prec][i];
  const Placement &A = L.place[st.a], &B = L.place[st.b], &C = L.place[st.node];
  d.A = ptr(A);
  d.B = ptr(B);
  d.C = ptr(C);
  d.sA_s = A.s_stride, d.sA_b = A.b_stride;
  d.sB_s = B.s_stride, d.sB_b = B.b_stride;
  d.sC_s = C.s_stride, d.sC_b = C.b_stride;
  d.gs_c = C.dep_s ? gsc : 1;
  d.copies = d.gs_c * (C.dep_b ? gbc : 1);
  // Exponents and maxima are kept in every precision.
  d.track = 1;
  d.expA = eptr(A), d.expB = eptr(B), d.expC = eptr(C);
  d.maxA = mptr(A), d.maxB = mptr(B), d.maxC = mptr(C);
  d.maxA_const = A.max_const, d.maxB_const = B.max_const;
  d.eA_s = A.es, d.eA_b = A.eb, d.eB_s = B.es, d.eB_b = B.eb, d.eC_s = C.es, d.eC_b = C.eb;
  d.lp_out = C.store != ST_C64;
  d.bias = bias;
  d.flag = gflags;
  d.dep_s_c = C.dep_s;
  d.flag_n = gsc;
  if (d.variant & kVarSwap) swap_operands(d);
  if (L.ksplit[i]) {
    d.ksplit = L.ksplit[i];
    d.P = reinterpret_cast<float2*>(arena + L.p_off[i]);
    d.p_stride = (int64_t(1) << pd.node_labels[st.node].size()) * (C.dep_s ? L.gs : 1) *
                 (C.dep_b ? L.gb : 1);
  }
  return d;
}

hipError_t launch_bound_step(const rqc_plan* p, const GroupLayout& L, size_t i, const StepDesc& d,
                             int kern, hipStream_t s) {
  const Step& st = p->pd.steps[i];
  const int lp_kind = L.prec == RQC_F16 ? ST_F16 : (L.prec == RQC_BF16 ? ST_BF16 : 0);
  const bool swap = (d.variant & kVarSwap) != 0;
  const int sa = L.place[swap ? st.b : st.a].store, sb = L.place[swap ? st.a : st.b].store;
  return launch_step(d, kern, sa, sb, L.place[st.node].store, lp_kind, s);
}

void record_call(rqc_plan* p, const GroupLayout& L, const WsLayout& W, uint64_t n_ids,
                 uint64_t n_batch, char* ws, double* out, double* per_slice, int64_t ps_row0,
                 hipStream_t s) {
  PlanData& pd = p->pd;
  const bool track = true;                  // exponents in every precision
  const bool lp_mode = L.prec != RQC_F32;   // slice flags drive FP32 re-runs
  char* arena = ws + W.arena_off;
  char* scale = ws + W.scale_off;
  int32_t* flags = reinterpret_cast<int32_t*>(ws + W.flags_off);
  const uint64_t* ids = reinterpret_cast<const uint64_t*>(ws + W.ids_off);
  const uint8_t* bits = reinterpret_cast<const uint8_t*>(ws + W.bits_off);
  const LeafJob* jobs = reinterpret_cast<const LeafJob*>(ws + W.jobs_off);
  const int n_closed = (int)pd.net.closed.size();
  const int n_elems = 1 << pd.net.open.size();
  auto ptr = [&](const Placement& P) -> char* { return P.resident ? p->res + P.off : arena + P.off; };
  auto eptr = [&](const Placement& P) -> int32_t* {
    if (P.e_off < 0) return nullptr;
    return reinterpret_cast<int32_t*>(P.resident ? p->res + P.e_off : scale + P.e_off);
  };
  hip_check(launch_fill_i32(flags, 0, (int64_t)n_ids * W.n_bgroups, s), "clear flags");
  size_t probe = 0;
  p->trec.clear();
  for (uint64_t b0 = 0; b0 < n_batch; b0 += L.gb) {
    const int gbc = (int)std::min<uint64_t>(L.gb, n_batch - b0);
    // This bitstring group's row of flags: one per slice.
    int32_t* gflags = flags + (int64_t)(b0 / L.gb) * (int64_t)n_ids;
    const int bias = b0 >= p->scale_bias_from ? p->scale_bias : 0;
    for (uint64_t g0 = 0; g0 < n_ids; g0 += L.gs) {
      const int gsc = (int)std::min<uint64_t>(L.gs, n_ids - g0);
      if (track && L.scale_bytes > 0)
        hip_check(launch_fill_i32(reinterpret_cast<int32_t*>(scale), 0, L.scale_bytes / 4, s),
                  "clear scales");
      hip_check(launch_leaves(jobs, (int)L.jobs.size(), p->res, arena, ids + g0,
                              bits + b0 * (uint64_t)std::max(1, n_closed), n_closed, gsc, gbc,
                              L.max_leaf_rank, s),
                "leaves");
      for (size_t i = 0; i < pd.steps.size(); ++i) {
        const Step& st = pd.steps[i];
        if (st.invariant) continue;
        StepDesc d = bind_step(p, L, W, ws, i, gsc, gbc, gflags + g0, bias);
        const Placement &A = L.place[st.a], &B = L.place[st.b], &C = L.place[st.node];
        const int kern = p->sel_kern[L.prec][i];
        const bool timed = p->timing_kernel == kTimeAll || kern == p->timing_kernel ||
                           (kern == KERN_MFMA16 && p->timing_kernel == KERN_MFMA);
        if (timed) {
          if (p->tev.size() < 2 * (probe + 1)) {
            // Timing only: no system-scope fence, so that the recorded
            // interval does not include writing back the caches.
            hipEvent_t a, b;
            hip_check(hipEventCreateWithFlags(&a, hipEventDisableSystemFence), "event");
            hip_check(hipEventCreateWithFlags(&b, hipEventDisableSystemFence), "event");
            p->tev.push_back(a);
            p->tev.push_back(b);
          }
          hip_check(hipEventRecord(p->tev[2 * probe], s), "event record");
        }
        hip_check(launch_bound_step(p, L, i, d, kern, s), "step");
        if (timed) {
          hip_check(hipEventRecord(p->tev[2 * probe + 1], s), "event record");
          ++probe;
          const double cp = (double)d.copies;
          const int ca = (A.dep_s ? (C.dep_s ? gsc : 1) : 1) * (A.dep_b ? (C.dep_b ? gbc : 1) : 1);
          const int cb = (B.dep_s ? (C.dep_s ? gsc : 1) : 1) * (B.dep_b ? (C.dep_b ? gbc : 1) : 1);
          LaunchRecord lr;
          lr.step = (int)i;
          lr.kernel = kern;
          lr.m = st.m, lr.n = st.n, lr.k = st.k;
          lr.copies = d.copies;
          lr.sa = A.store, lr.sb = B.store, lr.sc = C.store;
          lr.variant = d.variant;
          lr.flops = 8.0 * std::ldexp(1.0, st.m + st.n + st.k) * cp;
          lr.bytes = elsize(A.store) * std::ldexp(1.0, st.m + st.k) * ca +
                     elsize(B.store) * std::ldexp(1.0, st.n + st.k) * cb +
                     elsize(C.store) * std::ldexp(1.0, st.m + st.n) * cp;
          p->trec.push_back(lr);
        }
      }
      const int root = pd.tree.root;
      const Placement& R = L.place[root];
      hip_check(launch_slice_sum(ptr(R), R.store, eptr(R), R.s_stride, R.b_stride, R.es, R.eb,
                                 R.dep_s, R.dep_b, n_elems, gsc, gbc, lp_mode ? gflags + g0 : nullptr,
                                 out, per_slice, ps_row0 + (int64_t)g0, (int64_t)n_batch,
                                 (int64_t)b0, g0 == 0 ? 1 : 0, s),
                "slice sum");
    }
  }
}

bool fits(rqc_plan* p, int prec, int gs, int gb, uint64_t n_ids, uint64_t n_batch,
          size_t ws_bytes) {
  GroupLayout L = compute_layout(p, prec, gs, gb);
  return (size_t)ws_layout(p, L, n_ids, n_batch).total <= ws_bytes;
}

void choose_group(rqc_plan* p, int prec, uint64_t n_ids, uint64_t n_batch, size_t ws_bytes,
                  int& gs, int& gb) {
  int max_gs = (int)std::min<uint64_t>(n_ids, 4096);
  int max_gb = (int)std::min<uint64_t>(n_batch, 4096);
  if (p->group_limit_s > 0) max_gs = std::min(max_gs, p->group_limit_s);
  if (p->group_limit_b > 0) max_gb = std::min(max_gb, p->group_limit_b);
  // Copies per launch are bounded by the grid's y dimension.
  gb = max_gb;
  while (gb > 1 && !fits(p, prec, 1, gb, n_ids, n_batch, ws_bytes)) gb = (gb + 1) / 2;
  if (!fits(p, prec, 1, gb, n_ids, n_batch, ws_bytes)) {
    GroupLayout L = compute_layout(p, prec, 1, 1);
    throw Error{RQC_EHBM, "workspace too small: need at least " +
                              std::to_string(ws_layout(p, L, n_ids, n_batch).total) + " bytes"};
  }
  int lo = 1, hi = max_gs;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if ((int64_t)mid * gb <= 65535 && fits(p, prec, mid, gb, n_ids, n_batch, ws_bytes)) lo = mid;
    else hi = mid - 1;
  }
  gs = lo;
}

void contract(rqc_plan* p, const uint64_t* ids_in, uint64_t n_ids, const uint8_t* bits,
              uint64_t n_batch, int prec, void* ws_v, size_t ws_bytes, double* out,
              double* per_slice, hipStream_t s, PendingRun& r, bool direct) {
  PlanData& pd = p->pd;
  if (!p->bound) throw Error{RQC_EINVAL, "plan is not bound to device memory"};
  if (prec != RQC_F32 && prec != RQC_F16 && prec != RQC_BF16) throw Error{RQC_EINVAL, "bad precision"};
  if (!out || !ws_v) throw Error{RQC_EINVAL, "null device pointer"};
  if ((reinterpret_cast<uintptr_t>(ws_v) & 255) != 0) throw Error{RQC_EINVAL, "workspace not 256-byte aligned"};
  if (n_batch == 0) throw Error{RQC_EINVAL, "n_batch must be positive"};
  const uint64_t n_slices = uint64_t(1) << pd.sliced.size();
  std::vector<uint64_t> ids;
  if (!ids_in) {
    if (n_ids != 0 && n_ids != n_slices) throw Error{RQC_EINVAL, "slice_ids is NULL but n_ids is not 0"};
    n_ids = n_slices;
    ids.resize(n_ids);
    for (uint64_t i = 0; i < n_ids; ++i) ids[i] = i;
  } else {
    if (n_ids == 0) throw Error{RQC_EINVAL, "n_ids is 0"};
    ids.assign(ids_in, ids_in + n_ids);
    for (uint64_t v : ids)
      if (v >= n_slices) throw Error{RQC_EINVAL, "slice id out of range"};
  }
  const size_t n_closed = pd.net.closed.size();
  std::vector<uint8_t> b(n_batch * std::max<size_t>(1, n_closed), 0);
  if (n_closed > 0) {
    if (!bits) throw Error{RQC_EINVAL, "closed_bits is NULL"};
    for (size_t i = 0; i < n_batch * n_closed; ++i) {
      if (bits[i] > 1) throw Error{RQC_EINVAL, "closed bits must be 0 or 1"};
      b[i] = bits[i];
    }
  }
  int gs, gb;
  choose_group(p, prec, n_ids, n_batch, ws_bytes, gs, gb);
  const GroupLayout& L = group_layout(p, prec, gs, gb);
  const WsLayout W = ws_layout(p, L, n_ids, n_batch);
  char* ws = static_cast<char*>(ws_v);
  hip_check(hipMemcpyAsync(ws + W.ids_off, ids.data(), 8 * n_ids, hipMemcpyHostToDevice, s), "ids");
  hip_check(hipMemcpyAsync(ws + W.bits_off, b.data(), b.size(), hipMemcpyHostToDevice, s), "bits");
  if (!L.jobs.empty())
    hip_check(hipMemcpyAsync(ws + W.jobs_off, L.jobs.data(), sizeof(LeafJob) * L.jobs.size(),
                             hipMemcpyHostToDevice, s),
              "jobs");
  GraphKey key{prec, gs, gb, n_ids, n_batch, ws_v, out, per_slice};
  auto it = p->graphs.find(key);
  int reused = 0;
  if (p->timing_kernel >= 0 || direct) {
    // Timing probe, or a caller that wants no graph objects: direct launches
    // on `s` (each probed launch bracketed by events recorded on `s`).
    record_call(p, L, W, n_ids, n_batch, ws, out, per_slice, 0, s);
  } else if (it != p->graphs.end()) {
    hip_check(hipGraphLaunch(it->second.exec, s), "graph launch");
    hip_check(hipEventRecord(it->second.done, s), "graph event");
    it->second.last_use = ++p->graph_clock;
    reused = 1;
  } else {
    if (!p->capture_stream)
      hip_check(hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking), "capture stream");
    hip_check(hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal), "begin capture");
    try {
      record_call(p, L, W, n_ids, n_batch, ws, out, per_slice, 0, p->capture_stream);
    } catch (...) {
      hipGraph_t g;
      (void)hipStreamEndCapture(p->capture_stream, &g);
      throw;
    }
    hipGraph_t g;
    hip_check(hipStreamEndCapture(p->capture_stream, &g), "end capture");
    GraphEntry ge;
    hipError_t e = hipGraphInstantiate(&ge.exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    hip_check(e, "graph instantiate");
    e = hipEventCreateWithFlags(&ge.done, hipEventDisableTiming);
    if (e != hipSuccess) {
      (void)hipGraphExecDestroy(ge.exec);
      hip_check(e, "graph event");
    }
    // Bounded cache: the least recently launched exec goes, once its last
    // launch (possibly still running on another stream) has completed.
    while (p->graphs.size() >= kMaxGraphs) {
      auto victim = p->graphs.begin();
      for (auto jt = p->graphs.begin(); jt != p->graphs.end(); ++jt)
        if (jt->second.last_use < victim->second.last_use) victim = jt;
      (void)hipEventSynchronize(victim->second.done);
      (void)hipEventDestroy(victim->second.done);
      (void)hipGraphExecDestroy(victim->second.exec);
      p->graphs.erase(victim);
    }
    ge.last_use = ++p->graph_clock;
    GraphEntry& slot = p->graphs[key];
    slot = ge;
    hip_check(hipGraphLaunch(slot.exec, s), "graph launch");
    hip_check(hipEventRecord(slot.done, s), "graph event");
  }
  r.active = true;
  r.prec = prec;
  r.n_ids = n_ids;
  r.n_batch = n_batch;
  r.ids = ids;
  r.bits = b;
  r.ws = ws;
  r.ws_bytes = ws_bytes;
  r.out = out;
  r.per_slice = per_slice;
  r.gs = gs;
  r.gb = gb;
  r.graph_reused = reused;
  r.flops = (pd.flops_per_slice * (double)n_ids + pd.flops_per_bitstring) * (double)n_batch;
}

void report(rqc_plan* p, PendingRun& r, hipStream_t s, rqc_run_report* rep, bool sync) {
  std::memset(rep, 0, sizeof *rep);
  if (sync) hip_check(hipStreamSynchronize(s), "synchronize");
  if (!r.active) return;
  p->last_timing = rqc_timing{};
  p->tms.clear();
  for (size_t i = 0; i < p->trec.size() && p->timing_kernel >= 0; ++i) {
    float ms = 0.f;
    hip_check(hipEventElapsedTime(&ms, p->tev[2 * i], p->tev[2 * i + 1]), "event time");
    p->tms.push_back(ms);
    p->last_timing.launches++;
    p->last_timing.total_ms += ms;
    p->last_timing.flops += p->trec[i].flops;
    p->last_timing.bytes += p->trec[i].bytes;
  }
  rep->n_slices = r.n_ids;
  rep->slices_per_group = r.gs;
  rep->bits_per_group = r.gb;
  rep->graph_reused = r.graph_reused;
  rep->flops = r.flops;
  const GroupLayout& L0 = group_layout(p, r.prec, r.gs, r.gb);
  const WsLayout W0 = ws_layout(p, L0, r.n_ids, r.n_batch);
  const int64_t nbg = W0.n_bgroups;
  std::vector<int32_t> flags((size_t)(r.n_ids * nbg));
  hip_check(hipMemcpy(flags.data(), r.ws + W0.flags_off, 4 * flags.size(), hipMemcpyDeviceToHost),
            "flags");
  // A slice is re-run when any of its bitstring groups was flagged; its FP32
  // result is then added for exactly those groups, whose slice sums skipped it.
  std::vector<uint64_t> redo;
  for (uint64_t i = 0; i < r.n_ids; ++i)
    for (int64_t g = 0; g < nbg; ++g)
      if (flags[(size_t)(g * (int64_t)r.n_ids + (int64_t)i)]) {
        redo.push_back(i);
        break;
      }
  r.active = false;
  if (redo.empty()) return;
  // With normalised complex64 storage a non-finite FP32 value can only come
  // from non-finite inputs.
  if (r.prec == RQC_F32) throw Error{RQC_ENUMERIC, "non-finite values in the FP32 contraction"};
  // Filter of Section 5.5, re-read: a slice whose reduced-precision result is
  // not finite is contracted again in FP32 instead of being discarded.
  int gb = (int)std::min<uint64_t>(r.n_batch, 4096);
  while (gb > 1 && !fits(p, RQC_F32, 1, gb, 1, r.n_batch, r.ws_bytes)) gb = (gb + 1) / 2;
  if (!fits(p, RQC_F32, 1, gb, 1, r.n_batch, r.ws_bytes))
    throw Error{RQC_EHBM, "workspace too small for the FP32 re-run"};
  const GroupLayout& L = group_layout(p, RQC_F32, 1, gb);
  const WsLayout W = ws_layout(p, L, 1, r.n_batch);
  const int64_t ne2 = int64_t(2) << p->pd.net.open.size();  // doubles per bitstring
  const std::vector<LaunchRecord> keep_rec = p->trec;  // the probed call's records
  double* tmp = reinterpret_cast<double*>(r.ws + W.tmp_off);
  std::vector<int32_t> f32_flags((size_t)W.n_bgroups);
  for (uint64_t idx : redo) {
    const uint64_t id = r.ids[idx];
    hip_check(hipMemcpyAsync(r.ws + W.ids_off, &id, 8, hipMemcpyHostToDevice, s), "ids");
    hip_check(hipMemcpyAsync(r.ws + W.bits_off, r.bits.data(), r.bits.size(), hipMemcpyHostToDevice, s), "bits");
    if (!L.jobs.empty())
      hip_check(hipMemcpyAsync(r.ws + W.jobs_off, L.jobs.data(), sizeof(LeafJob) * L.jobs.size(),
                               hipMemcpyHostToDevice, s),
                "jobs");
    record_call(p, L, W, 1, r.n_batch, r.ws, tmp, nullptr, 0, s);
    for (int64_t g = 0; g < nbg; ++g) {
      if (!flags[(size_t)(g * (int64_t)r.n_ids + (int64_t)idx)]) continue;
      const int64_t b0 = g * r.gb;
      const int64_t nb = std::min<int64_t>(r.gb, (int64_t)r.n_batch - b0);
      hip_check(launch_add_f64(r.out + b0 * ne2, tmp + b0 * ne2, nb * ne2, s), "add re-run");
      if (r.per_slice)
        hip_check(hipMemcpyAsync(r.per_slice + ((int64_t)idx * (int64_t)r.n_batch + b0) * ne2,
                                 tmp + b0 * ne2, 8 * nb * ne2, hipMemcpyDeviceToDevice, s),
                  "per-slice re-run");
    }
    hip_check(hipStreamSynchronize(s), "re-run");
    hip_check(hipMemcpy(f32_flags.data(), r.ws + W.flags_off, 4 * f32_flags.size(),
                        hipMemcpyDeviceToHost),
              "re-run flags");
    for (int32_t f : f32_flags)
      if (f) {
        p->trec = keep_rec;
        throw Error{RQC_ENUMERIC, "non-finite values persisted after the FP32 re-run of slice " +
                                      std::to_string(id)};
      }
    rep->fp32_reruns++;
  }
  p->trec = keep_rec;
}

}  // namespace rqc

rqc_plan::~rqc_plan() {
  rqc::clear_graphs(this);
  for (auto e : tev) (void)hipEventDestroy(e);
  if (capture_stream) (void)hipStreamDestroy(capture_stream);
}

// Contraction-path search and slicing (Sections 5.1 and 5.2).
//
// The paper searches paths with a hyper-optimiser whose loss weighs both the
// contraction cost and the compute density of the steps (Section 5.2), and
// slices wires so that each sub-task fits a node's memory while the total
// cost grows little (Section 5.1).  This planner is written from scratch:
//   1. many randomized greedy trees (score size(C) - alpha*(size(A)+size(B))
//      with Gumbel noise, alpha and temperature sampled per trial);
//   2. per trial, greedy slicing: repeatedly slice the wire that keeps the
//      total (all-slice) cost lowest, preferring wires that shrink the
//      largest intermediate while it exceeds the bound;
//   3. subtree re-optimisation of the 32 best trees: small subtrees are
//      re-solved exactly by dynamic programming over subsets, and the best
//      re-optimised tree wins;
//   4. execution order, slice/bit dependence, and per-step layouts chosen
//      top-down so that each operand's summed labels are its lowest address
//      bits (contiguous K runs) and its free labels keep the order of the
//      step output.
#include <algorithm>
#include <bitset>
#include <cmath>
#include <cstring>
#include <functional>
#include <numeric>
#include <queue>
#include <random>
#include <set>
#include <sstream>
#include <thread>
#include <unordered_map>

#include "core.h"

namespace rqc {

using LSet = std::vector<int>;  // sorted labels

static LSet symdiff(const LSet& a, const LSet& b) {
  LSet out;
  out.reserve(a.size() + b.size());
  std::set_symmetric_difference(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(out));
  return out;
}
static int union_size(const LSet& a, const LSet& b) {
  size_t i = 0, j = 0;
  int common = 0;
  while (i < a.size() && j < b.size()) {
    if (a[i] < b[j]) ++i;
    else if (b[j] < a[i]) ++j;
    else { ++common; ++i; ++j; }
  }
  return (int)(a.size() + b.size()) - common;
}
static LSet remove_labels(const LSet& a, const std::vector<char>& drop) {
  LSet out;
  for (int x : a)
    if (!drop[x]) out.push_back(x);
  return out;
}

// ---------------------------------------------------------------------------
// Randomized greedy
// ---------------------------------------------------------------------------
static Tree greedy_tree(const std::vector<LSet>& leaf_sets, int n_labels, double alpha, double temp,
                        std::mt19937_64& rng) {
  const int nl = (int)leaf_sets.size();
  Tree t;
  t.n_leaves = nl;
  t.left.assign(nl, -1);
  t.right.assign(nl, -1);
  std::vector<LSet> sets(leaf_sets);
  std::vector<char> alive(nl, 1);
  std::vector<std::array<int, 2>> owners(n_labels, {-1, -1});
  for (int i = 0; i < nl; ++i)
    for (int x : sets[i]) {
      auto& o = owners[x];
      if (o[0] < 0) o[0] = i;
      else o[1] = i;
    }
  std::uniform_real_distribution<double> U(1e-12, 1.0);
  struct Cand {
    double s;
    int a, b;
    bool operator<(const Cand& o) const {
      if (s != o.s) return s > o.s;  // min-heap
      if (a != o.a) return a > o.a;
      return b > o.b;
    }
  };
  std::priority_queue<Cand> heap;
  auto score = [&](int a, int b) {
    const int ua = union_size(sets[a], sets[b]);
    const int shared = (int)(sets[a].size() + sets[b].size()) - ua;
    const int rc = ua - shared;
    double v = std::ldexp(1.0, rc) - alpha * (std::ldexp(1.0, (int)sets[a].size()) +
                                              std::ldexp(1.0, (int)sets[b].size()));
    double s = v >= 0 ? std::log2(1.0 + v) : -std::log2(1.0 - v);
    if (temp > 0) s -= temp * (-std::log(-std::log(U(rng))));
    return s;
  };
  auto push_pair = [&](int a, int b) {
    if (a == b || a < 0 || b < 0) return;
    if (a > b) std::swap(a, b);
    heap.push({score(a, b), a, b});
  };
  for (int x = 0; x < n_labels; ++x)
    if (owners[x][0] >= 0 && owners[x][1] >= 0) push_pair(owners[x][0], owners[x][1]);
  int live = nl;
  while (!heap.empty()) {
    Cand c = heap.top();
    heap.pop();
    if (!alive[c.a] || !alive[c.b]) continue;
    const int id = (int)sets.size();
    sets.push_back(symdiff(sets[c.a], sets[c.b]));
    alive.push_back(1);
    alive[c.a] = alive[c.b] = 0;
    t.left.push_back(c.a);
    t.right.push_back(c.b);
    --live;
    for (int x : sets[id]) {
      auto& o = owners[x];
      for (int k = 0; k < 2; ++k)
        if (o[k] == c.a || o[k] == c.b) o[k] = id;
    }
    for (int x : sets[id]) {
      auto& o = owners[x];
      const int other = o[0] == id ? o[1] : o[0];
      if (other >= 0 && alive[other]) push_pair(id, other);
    }
  }
  // Disconnected components: outer products, smallest first.
  std::vector<int> rest;
  for (int i = 0; i < (int)sets.size(); ++i)
    if (alive[i]) rest.push_back(i);
  while (rest.size() > 1) {
    std::sort(rest.begin(), rest.end(), [&](int a, int b) {
      return sets[a].size() != sets[b].size() ? sets[a].size() > sets[b].size() : a > b;
    });
    const int a = rest.back();
    rest.pop_back();
    const int b = rest.back();
    rest.pop_back();
    const int id = (int)sets.size();
    sets.push_back(symdiff(sets[a], sets[b]));
    t.left.push_back(a);
    t.right.push_back(b);
    rest.push_back(id);
  }
  t.root = rest.empty() ? -1 : rest[0];
  return t;
}

// Label sets of every node of `t` given leaf sets (contracted labels only).
static std::vector<LSet> node_sets(const Tree& t, const std::vector<LSet>& leaf_sets) {
  std::vector<LSet> s(t.left.size());
  for (int i = 0; i < t.n_leaves; ++i) s[i] = leaf_sets[i];
  // Internal nodes are created after their children in greedy order, but
  // reconfiguration may break that; evaluate recursively.
  std::vector<char> done(t.left.size(), 0);
  for (int i = 0; i < t.n_leaves; ++i) done[i] = 1;
  std::function<void(int)> ev = [&](int v) {
    if (done[v]) return;
    ev(t.left[v]);
    ev(t.right[v]);
    s[v] = symdiff(s[t.left[v]], s[t.right[v]]);
    done[v] = 1;
  };
  if (t.root >= 0) ev(t.root);
  return s;
}

// Time-like cost of one pairwise step, in complex multiply-adds: the larger
// of its multiply-adds and its mandatory traffic (each operand read once,
// the output written once) weighted by the GPU's balance of matrix-core
// rate to HBM rate, about 20 multiply-adds per complex64 element moved.
// Trees with similar flop counts differ by several times in traffic, and
// sliced plans are mostly traffic-bound, so the search ranks by this.
constexpr double kMacsPerElement = 20.0;
static double step_cost(int un, int sa, int sb, int sc) {
  const double macs = std::ldexp(1.0, un);
  const double elems = std::ldexp(1.0, sa) + std::ldexp(1.0, sb) + std::ldexp(1.0, sc);
  return std::max(macs, kMacsPerElement * elems);
}

static CostModel tree_cost(const Tree& t, const std::vector<LSet>& s) {
  CostModel c;
  for (int v = t.n_leaves; v < (int)t.left.size(); ++v) {
    if (t.left[v] < 0) continue;
    const LSet& a = s[t.left[v]];
    const LSet& b = s[t.right[v]];
    const int un = union_size(a, b);
    c.flops += std::ldexp(1.0, un);
    c.cost += step_cost(un, (int)a.size(), (int)b.size(), (int)s[v].size());
    c.width = std::max(c.width, (int)s[v].size());
  }
  for (int i = 0; i < t.n_leaves; ++i) c.width = std::max(c.width, (int)s[i].size());
  return c;
}

// ---------------------------------------------------------------------------
// Slicing (Section 5.1)
// ---------------------------------------------------------------------------
struct SliceResult {
  std::vector<int> sliced;
  CostModel per_slice;
};

static SliceResult slice_tree(const Tree& t, const std::vector<LSet>& leaf_sets, int n_labels,
                              const std::vector<char>& sliceable, const std::vector<int>& forced,
                              int bound, int n_target) {
  SliceResult r;
  std::vector<char> drop(n_labels, 0);
  for (int x : forced) {
    drop[x] = 1;
    r.sliced.push_back(x);
  }
  auto cur_leaf = [&]() {
    std::vector<LSet> ls(leaf_sets.size());
    for (size_t i = 0; i < ls.size(); ++i) ls[i] = remove_labels(leaf_sets[i], drop);
    return ls;
  };
  std::vector<LSet> s = node_sets(t, cur_leaf());
  CostModel c = tree_cost(t, s);
  const int nn = (int)t.left.size();
  while (true) {
    // An exact wire count (n_target >= 0) is never exceeded; the caller
    // checks the bound afterwards.
    const bool need_width = n_target < 0 && bound > 0 && c.width > bound;
    const bool need_count = n_target >= 0 && (int)r.sliced.size() < n_target;
    if (!need_width && !need_count) break;
    // savings[x]: per-slice cost removed if x is sliced.
    std::vector<double> save(n_labels, 0.0);
    std::vector<int> cnt_max(n_labels, 0);
    int n_max = 0;
    for (int v = 0; v < nn; ++v) {
      if ((int)s[v].size() == c.width) {
        ++n_max;
        for (int x : s[v]) cnt_max[x]++;
      }
      if (v < t.n_leaves || t.left[v] < 0) continue;
      const LSet& a = s[t.left[v]];
      const LSet& b = s[t.right[v]];
      const LSet& cc = s[v];
      const int un = union_size(a, b), sa = (int)a.size(), sb = (int)b.size(), sc = (int)cc.size();
      const double now = step_cost(un, sa, sb, sc);
      auto gain = [&](int x) {
        const int xa = std::binary_search(a.begin(), a.end(), x) ? 1 : 0;
        const int xb = std::binary_search(b.begin(), b.end(), x) ? 1 : 0;
        const int xc = std::binary_search(cc.begin(), cc.end(), x) ? 1 : 0;
        return now - step_cost(un - 1, sa - xa, sb - xb, sc - xc);
      };
      for (int x : a) save[x] += gain(x);
      for (int x : b)
        if (!std::binary_search(a.begin(), a.end(), x)) save[x] += gain(x);
    }
    int best = -1;
    double best_cost = 0;
    bool best_w = false;
    for (int x = 0; x < n_labels; ++x) {
      if (!sliceable[x] || drop[x] || save[x] <= 0) continue;
      const bool reduces = cnt_max[x] == n_max;
      const double total = (c.cost - save[x]) * 2.0;  // relative: x2 slices
      bool better;
      if (best < 0) better = true;
      else if (need_width && reduces != best_w) better = reduces;
      else better = total < best_cost;
      if (better) {
        best = x;
        best_cost = total;
        best_w = reduces;
      }
    }
    if (best < 0) break;
    drop[best] = 1;
    r.sliced.push_back(best);
    s = node_sets(t, cur_leaf());
    c = tree_cost(t, s);
  }
  r.per_slice = c;
  return r;
}

// ---------------------------------------------------------------------------
// Subtree re-optimisation by exact dynamic programming over subsets
// ---------------------------------------------------------------------------
static bool reconf_node(Tree& t, std::vector<LSet>& s, int v, int kmax, int width_bound) {
  if (v < t.n_leaves) return false;
  std::vector<int> front = {v};
  std::vector<int> internal;
  while ((int)front.size() < kmax) {
    int pick = -1;
    for (int i = 0; i < (int)front.size(); ++i) {
      const int f = front[i];
      if (f < t.n_leaves) continue;
      if (pick < 0 || s[f].size() > s[front[pick]].size()) pick = i;
    }
    if (pick < 0) break;
    const int f = front[pick];
    internal.push_back(f);
    front.erase(front.begin() + pick);
    front.push_back(t.left[f]);
    front.push_back(t.right[f]);
  }
  const int m = (int)front.size();
  if (m < 3) return false;
  // Local label universe.
  std::unordered_map<int, int> loc;
  for (int f : front)
    for (int x : s[f])
      if (!loc.count(x)) loc[x] = (int)loc.size();
  if (loc.size() > 512) return false;
  using BS = std::bitset<512>;
  std::vector<BS> fb(m);
  for (int i = 0; i < m; ++i)
    for (int x : s[front[i]]) fb[i].set(loc[x]);
  const int full = (1 << m) - 1;
  std::vector<BS> L(full + 1);
  std::vector<int> Lsz(full + 1, 0);
  for (int S = 1; S <= full; ++S) {
    const int low = __builtin_ctz(S);
    L[S] = L[S & (S - 1)] ^ fb[low];
    Lsz[S] = (int)L[S].count();
  }
  const double INF = 1e300;
  std::vector<double> best(full + 1, INF);
  std::vector<int> split(full + 1, 0);
  for (int i = 0; i < m; ++i) best[1 << i] = 0;
  for (int S = 1; S <= full; ++S) {
    if ((S & (S - 1)) == 0) continue;
    if (width_bound > 0 && Lsz[S] > width_bound && S != full) continue;
    double bc = INF;
    int bs = 0;
    for (int sub = (S - 1) & S; sub; sub = (sub - 1) & S) {
      const int o = S ^ sub;
      if (sub > o) continue;
      if (best[sub] >= INF || best[o] >= INF) continue;
      const int un = (int)(L[sub] | L[o]).count();
      const double c = best[sub] + best[o] + step_cost(un, Lsz[sub], Lsz[o], Lsz[S]);
      if (c < bc) {
        bc = c;
        bs = sub;
      }
    }
    best[S] = bc;
    split[S] = bs;
  }
  double old = 0;
  for (int f : internal)
    old += step_cost(union_size(s[t.left[f]], s[t.right[f]]), (int)s[t.left[f]].size(),
                     (int)s[t.right[f]].size(), (int)s[f].size());
  if (!(best[full] < old * (1 - 1e-12))) return false;
  // Rebuild with the old internal ids (v stays the subtree root).
  std::vector<int> pool(internal.begin(), internal.end());
  std::sort(pool.begin(), pool.end());
  pool.erase(std::find(pool.begin(), pool.end(), v));
  std::function<int(int, bool)> mk = [&](int S, bool top) -> int {
    if ((S & (S - 1)) == 0) return front[__builtin_ctz(S)];
    const int a = mk(split[S], false);
    const int b = mk(S ^ split[S], false);
    int id;
    if (top) id = v;
    else {
      id = pool.back();
      pool.pop_back();
    }
    t.left[id] = a;
    t.right[id] = b;
    s[id] = symdiff(s[a], s[b]);
    return id;
  };
  mk(full, true);
  return true;
}

static void reconfigure(Tree& t, std::vector<LSet>& s, int rounds, int kmax, int width_bound,
                        std::mt19937_64& rng) {
  for (int r = 0; r < rounds; ++r) {
    std::vector<int> order;
    for (int v = t.n_leaves; v < (int)t.left.size(); ++v) order.push_back(v);
    // Most expensive nodes first, then a shuffle of the rest.
    std::shuffle(order.begin(), order.end(), rng);
    int improved = 0;
    for (int v : order) improved += reconf_node(t, s, v, kmax, width_bound) ? 1 : 0;
    if (!improved) break;
  }
}

// ---------------------------------------------------------------------------
// Steps, dependence and layouts
// ---------------------------------------------------------------------------
int choose_kernel(int m, int n, int k) {
  // MFMA only where the step is a real dense contraction: at least one full
  // 32x32 real tile per wave in both free dimensions and several summed bits.
  if (m >= 6 && n >= 5 && k >= 3) return 1;
  return 0;
}

static void build_steps(PlanData& p) {
  const Tree& t = p.tree;
  const int nn = (int)t.left.size();
  auto& s = p.node_labels;
  p.dep_s.assign(nn, 0);
  p.dep_b.assign(nn, 0);
  std::vector<char> sl(p.net.labels.size(), 0);
  for (int x : p.sliced) sl[x] = 1;
  for (int i = 0; i < t.n_leaves; ++i) {
    for (int x : p.net.leaves[i].labels) {
      if (sl[x]) p.dep_s[i] = 1;
      if (p.net.labels[x].kind == CLOSED) p.dep_b[i] = 1;
    }
  }
  // Post-order: larger child first (its big intermediate is freed earlier).
  std::vector<int> order;
  std::function<void(int)> dfs = [&](int v) {
    if (v < t.n_leaves) return;
    int a = t.left[v], b = t.right[v];
    if (s[b].size() > s[a].size()) std::swap(a, b);
    dfs(a);
    dfs(b);
    p.dep_s[v] = p.dep_s[a] | p.dep_s[b];
    p.dep_b[v] = p.dep_b[a] | p.dep_b[b];
    order.push_back(v);
  };
  dfs(t.root);

  // Layouts top-down.  Root: open qubits, open[0] least significant.
  p.layout.assign(nn, {});
  if (t.root >= 0) {
    for (int i = (int)p.net.open_label.size() - 1; i >= 0; --i) p.layout[t.root].push_back(p.net.open_label[i]);
    if (t.root < t.n_leaves) p.layout[t.root] = p.layout[t.root];
  }
  for (int idx = (int)order.size() - 1; idx >= 0; --idx) {
    const int v = order[idx];
    const LSet& sc = s[v];
    const std::vector<int>& lc = p.layout[v];
    for (int child : {t.left[v], t.right[v]}) {
      const int other = child == t.left[v] ? t.right[v] : t.left[v];
      const LSet& sx = s[child];
      std::vector<int> free_part, summed;
      for (int x : lc)
        if (std::binary_search(sx.begin(), sx.end(), x)) free_part.push_back(x);
      for (int x : sx)
        if (!std::binary_search(sc.begin(), sc.end(), x)) summed.push_back(x);
      (void)other;
      // Summed labels lowest, in ascending label order for both operands.
      std::vector<int> lay = free_part;
      for (int i = (int)summed.size() - 1; i >= 0; --i) lay.push_back(summed[i]);
      p.layout[child] = lay;
    }
  }

  p.steps.clear();
  p.step_of_node.assign(nn, -1);
  p.flops_invariant = 0;
  p.flops_per_slice = 0;
  p.bytes_per_slice = 0;
  p.flops_per_bitstring = 0;
  p.bytes_per_bitstring = 0;
  p.max_log2 = 0;
  for (int i = 0; i < t.n_leaves; ++i) p.max_log2 = std::max(p.max_log2, (int)s[i].size());
  for (int v : order) {
    Step st;
    st.node = v;
    int a = t.left[v], b = t.right[v];
    if (s[b].size() > s[a].size()) std::swap(a, b);
    st.a = a;
    st.b = b;
    st.la = p.layout[a];
    st.lb = p.layout[b];
    st.lc = p.layout[v];
    const int ua = union_size(s[a], s[b]);
    st.k = (int)(s[a].size() + s[b].size()) - ua;
    st.m = (int)s[a].size() - st.k;
    st.n = (int)s[b].size() - st.k;
    st.kernel = choose_kernel(st.m, st.n, st.k);
    st.dep_s = p.dep_s[v];
    st.dep_b = p.dep_b[v];
    st.invariant = !st.dep_s && !st.dep_b;
    st.lp = !st.invariant && (int)s[v].size() >= p.opts.lp_min_log2;
    st.lp_bf16 = !st.invariant && (int)s[v].size() >= p.opts.bf16_min_log2;
    const double fl = 8.0 * std::ldexp(1.0, st.m + st.n + st.k);
    const double by = 8.0 * (std::ldexp(1.0, (int)s[a].size()) + std::ldexp(1.0, (int)s[b].size()) +
                             std::ldexp(1.0, (int)s[v].size()));
    if (st.invariant) {
      p.flops_invariant += fl;
    } else if (st.dep_s) {
      p.flops_per_slice += fl;
      p.bytes_per_slice += by;
    } else {
      p.flops_per_bitstring += fl;
      p.bytes_per_bitstring += by;
    }
    p.max_log2 = std::max(p.max_log2, (int)s[v].size());
    p.step_of_node[v] = (int)p.steps.size();
    p.steps.push_back(std::move(st));
  }
}

// Fixes `label` of a leaf to `value`: keeps the half of the data with that
// address bit and drops the label.
static void project_leaf(Leaf& leaf, int label, int value) {
  const auto it = std::find(leaf.labels.begin(), leaf.labels.end(), label);
  if (it == leaf.labels.end()) return;
  const int rank = (int)leaf.labels.size();
  const int bit = rank - 1 - (int)(it - leaf.labels.begin());  // address bit, LSB = 0
  std::vector<cd> out(leaf.data.size() / 2);
  for (size_t e = 0; e < out.size(); ++e) {
    const size_t lo = e & ((size_t(1) << bit) - 1);
    const size_t hi = (e >> bit) << (bit + 1);
    out[e] = leaf.data[hi | (size_t(value) << bit) | lo];
  }
  leaf.labels.erase(it);
  leaf.data = std::move(out);
}

// Wires that carry a single value: a leaf whose slab at one value of a wire
// is zero (relative to the leaf's largest entry) forces the other value, as
// when the input |0> and the first single-qubit gates of a qubit leave it in
// a basis state that the next two-qubit gate, a phased swap for
// fSim(pi/2, phi), passes on.  Fixing such a wire to the forced value drops
// only zero terms, so it is projected out of every leaf (repeatedly, since a
// projection can expose more).  Wires in `keep` stay.  Returns the pruned
// wires with their values.
static std::vector<std::pair<int, int>> prune_constant_wires(Network& net,
                                                             const std::vector<char>& keep) {
  std::vector<std::pair<int, int>> pruned;
  bool changed = true;
  while (changed) {
    changed = false;
    for (Leaf& leaf : net.leaves) {
      double mx = 0;
      for (const cd& v : leaf.data) mx = std::max(mx, std::abs(v));
      if (mx == 0) continue;
      const int rank = (int)leaf.labels.size();
      for (int pos = 0; pos < rank; ++pos) {
        const int x = leaf.labels[pos];
        if (net.labels[x].kind != WIRE || keep[x]) continue;
        const int bit = rank - 1 - pos;
        double slab[2] = {0, 0};
        for (size_t e = 0; e < leaf.data.size(); ++e)
          slab[(e >> bit) & 1] = std::max(slab[(e >> bit) & 1], std::abs(leaf.data[e]));
        int forced = -1;
        if (slab[0] <= 1e-13 * mx && slab[1] > 1e-13 * mx) forced = 1;
        if (slab[1] <= 1e-13 * mx && slab[0] > 1e-13 * mx) forced = 0;
        if (forced < 0) continue;
        for (Leaf& other : net.leaves) project_leaf(other, x, forced);
        net.wire_label.erase({net.labels[x].q, net.labels[x].seg});
        pruned.push_back({x, forced});
        changed = true;
        break;  // this leaf's labels changed
      }
    }
  }
  return pruned;
}

static void make_plan_once(PlanData& p) {
  Network& net = p.net;
  const int nlab = (int)net.labels.size();
  const int nl = (int)net.leaves.size();
  if (nl == 0) throw Error{RQC_EINVAL, "empty network"};
  std::vector<LSet> leaf_sets(nl);
  for (int i = 0; i < nl; ++i) {
    for (int x : net.leaves[i].labels)
      if (net.labels[x].kind != CLOSED) leaf_sets[i].push_back(x);
    std::sort(leaf_sets[i].begin(), leaf_sets[i].end());
  }
  std::vector<char> sliceable(nlab, 0);
  for (auto& kv : net.wire_label) sliceable[kv.second] = 1;
  std::vector<int> forced;
  for (auto& w : p.opts.forced) {
    auto it = net.wire_label.find(w);
    if (it == net.wire_label.end()) throw Error{RQC_EINVAL, "forced sliced wire does not exist"};
    if (std::find(forced.begin(), forced.end(), it->second) != forced.end())
      throw Error{RQC_EINVAL, "forced sliced wire listed twice"};
    forced.push_back(it->second);
  }
  if (p.opts.n_sliced >= 0 && p.opts.n_sliced < (int)forced.size())
    throw Error{RQC_EINVAL, "n_sliced smaller than the forced wires"};
  {
    std::vector<char> keep(nlab, 0);
    for (int x : forced) keep[x] = 1;
    p.pruned = prune_constant_wires(net, keep);
    for (int i = 0; i < nl; ++i) {
      leaf_sets[i].clear();
      for (int x : net.leaves[i].labels)
        if (net.labels[x].kind != CLOSED) leaf_sets[i].push_back(x);
      std::sort(leaf_sets[i].begin(), leaf_sets[i].end());
    }
    std::fill(sliceable.begin(), sliceable.end(), 0);
    for (auto& kv : net.wire_label) sliceable[kv.second] = 1;
  }
  if (p.opts.n_sliced > 62 && p.opts.n_local == 0)
    throw Error{RQC_EUNSUPPORTED, "more than 62 sliced wires need a slice share (n_local_sliced)"};
  if (p.opts.n_sliced > 4096) throw Error{RQC_EUNSUPPORTED, "more than 4096 sliced wires"};

  const double temps[] = {0.0, 0.02, 0.1, 0.3, 0.6, 1.0};
  const int trials = std::max(1, p.opts.trials);
  struct Candidate {
    double score = 1e308;  // log2(per-slice multiply-adds) + sliced wires + width penalty
    Tree tree;
    std::vector<LSet> sets;
    std::vector<int> sliced;
  };
  auto width_penalty = [&](int width) {
    return p.opts.max_log2 > 0 ? 4.0 * std::max(0, width - p.opts.max_log2) : 0.0;
  };
  auto sliced_leaves = [&](const std::vector<int>& sl) {
    std::vector<char> drop(nlab, 0);
    for (int x : sl) drop[x] = 1;
    std::vector<LSet> out(nl);
    for (int i = 0; i < nl; ++i) out[i] = remove_labels(leaf_sets[i], drop);
    return out;
  };
  // One search: n_trials randomized greedy trees, each sliced (the given
  // wires first, then greedily up to n_target or the width bound); the best
  // 32 are re-optimised on their sliced networks.  With `on_sliced` the
  // greedy trees are built on the network with the given wires removed.
  // Trial t draws from its own generator seeded by (seed, salt, t), so the
  // result does not depend on how trials are spread over threads.
  auto search = [&](const std::vector<int>& given, int n_target, uint64_t salt, int n_trials,
                    bool on_sliced) {
    std::vector<Candidate> res(n_trials);
    const std::vector<LSet> base = on_sliced ? sliced_leaves(given) : leaf_sets;
    auto run_trial = [&](int tr) {
      std::mt19937_64 rng(p.opts.seed * 0x9E3779B97F4A7C15ull + 0x51ED27ull * (uint64_t)tr + 12345 +
                          salt * 0xD1B54A32D192ED03ull);
      std::uniform_real_distribution<double> ua(0.0, 1.6);
      const double alpha = tr == 0 ? 1.0 : ua(rng);
      const double temp = tr == 0 ? 0.0 : temps[rng() % 6];
      Tree t = greedy_tree(base, nlab, alpha, temp, rng);
      SliceResult sr = slice_tree(t, leaf_sets, nlab, sliceable, given, p.opts.max_log2, n_target);
      res[tr].score = std::log2(sr.per_slice.cost) + (double)sr.sliced.size() +
                      width_penalty(sr.per_slice.width);
      res[tr].tree = std::move(t);
      res[tr].sliced = std::move(sr.sliced);
    };
    {
      std::vector<std::thread> pool;
      for (int w = 0; w < std::min(8, n_trials); ++w)
        pool.emplace_back([&, w] {
          for (int tr = w; tr < n_trials; tr += 8) run_trial(tr);
        });
      for (auto& th : pool) th.join();
    }
    std::vector<int> order(n_trials);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return res[x].score < res[y].score; });
    const int n_refine = std::min(n_trials, 32);
    auto refine = [&](int r) {
      Candidate& c = res[order[r]];
      const std::vector<LSet> sl = sliced_leaves(c.sliced);
      std::vector<LSet> ss = node_sets(c.tree, sl);
      const int w0 = tree_cost(c.tree, ss).width;
      const int wb = p.opts.max_log2 > 0 ? std::max(p.opts.max_log2, w0) : w0;
      if (p.opts.reconf_rounds > 0) {
        std::mt19937_64 rng(p.opts.seed * 0x2545F4914F6CDD1Dull + (uint64_t)r + 777 + salt * 0x9E37ull);
        reconfigure(c.tree, ss, p.opts.reconf_rounds, 8, wb, rng);
        ss = node_sets(c.tree, sl);
      }
      const CostModel cm = tree_cost(c.tree, ss);
      c.score = std::log2(cm.cost) + (double)c.sliced.size() + width_penalty(cm.width);
      c.sets = std::move(ss);
    };
    {
      std::vector<std::thread> pool;
      for (int w = 0; w < std::min(8, n_refine); ++w)
        pool.emplace_back([&, w] {
          for (int r = w; r < n_refine; r += 8) refine(r);
        });
      for (auto& th : pool) th.join();
    }
    int best = order[0];
    for (int r = 1; r < n_refine; ++r)
      if (res[order[r]].score < res[best].score) best = order[r];
    return std::move(res[best]);
  };

  Candidate best = search(forced, p.opts.n_sliced, 0, trials, false);
  // Improvement rounds, choosing path and slicing together: the first
  // search slices trees built for the whole network, so trees built
  // again with the chosen wires fixed -- greedily on the whole network and
  // on the sliced one -- are often far cheaper per slice.  With automatic
  // slicing, wires whose removal keeps every intermediate within the bound
  // are then un-sliced (the total cost never grows: a slice at most doubles).
  const int n_user = (int)forced.size();
  auto research = [&](int round) {
    const int t2 = std::max(8, std::min(512, trials / 2));
    bool improved = false;
    for (bool on_sliced : {false, true}) {
      Candidate c = search(best.sliced, (int)best.sliced.size(), 2 * round + on_sliced, t2, on_sliced);
      if (c.score < best.score - 1e-9) {
        best = std::move(c);
        improved = true;
      }
    }
    return improved;
  };
  auto unslice = [&]() {
    bool any = false;
    while ((int)best.sliced.size() > n_user) {
      int pick = -1;
      double pick_flops = 0;
      for (int j = n_user; j < (int)best.sliced.size(); ++j) {
        std::vector<int> sl = best.sliced;
        sl.erase(sl.begin() + j);
        const CostModel cm = tree_cost(best.tree, node_sets(best.tree, sliced_leaves(sl)));
        if (cm.width > p.opts.max_log2) continue;
        if (pick < 0 || cm.cost < pick_flops) {
          pick = j;
          pick_flops = cm.cost;
        }
      }
      if (pick < 0) break;
      best.sliced.erase(best.sliced.begin() + pick);
      any = true;
    }
    if (any) {
      best.sets = node_sets(best.tree, sliced_leaves(best.sliced));
      const CostModel cm = tree_cost(best.tree, best.sets);
      best.score = std::log2(cm.cost) + (double)best.sliced.size() + width_penalty(cm.width);
    }
    return any;
  };
  const bool auto_slicing = p.opts.n_sliced < 0 && p.opts.max_log2 > 0;
  bool again = !best.sliced.empty();
  for (int round = 1; round <= 6 && again; ++round) {
    const bool improved = research(round);
    const bool unsliced = auto_slicing && unslice();
    again = improved || unsliced;
    if (round == 6 && unsliced) research(7);
  }
  if (p.opts.max_log2 > 0 && tree_cost(best.tree, best.sets).width > p.opts.max_log2)
    throw Error{RQC_EUNSUPPORTED, "no tree found within the width bound with the requested sliced wires"};
  Tree best_tree = std::move(best.tree);
  std::vector<LSet> s = std::move(best.sets);
  SliceResult best_sl;
  best_sl.sliced = best.sliced;

  if (best_sl.sliced.size() > 62 && p.opts.n_local == 0)
    throw Error{RQC_EUNSUPPORTED,
                "the width bound needs more than 62 sliced wires: use a slice share (n_local_sliced)"};
  if (p.opts.n_local > (int)best_sl.sliced.size())
    throw Error{RQC_EINVAL, "n_local_sliced exceeds the number of sliced wires"};
  p.tree = std::move(best_tree);
  p.sliced = best_sl.sliced;
  p.fixed.clear();
  if (p.opts.n_local > 0) {
    // Wires beyond the share's enumerated ones take the share's bits and
    // are projected out of the leaves now.
    for (size_t j = p.opts.n_local; j < p.sliced.size(); ++j) {
      const size_t i = j - p.opts.n_local;
      const int v = i < p.opts.share_bits.size() ? (int)p.opts.share_bits[i] : 0;
      p.fixed.push_back({p.sliced[j], v});
    }
    p.sliced.resize(p.opts.n_local);
    for (Leaf& leaf : net.leaves)
      for (const auto& fv : p.fixed) project_leaf(leaf, fv.first, fv.second);
  }
  p.node_labels = s;
  p.cost = tree_cost(p.tree, s);
  p.score = std::log2(p.cost.cost) + (double)(p.sliced.size() + p.fixed.size());
  build_steps(p);
}

void make_plan(PlanData& p) {
  const int restarts = std::max(1, p.opts.restarts);
  if (restarts == 1) {
    make_plan_once(p);
    return;
  }
  // Independent searches; each starts from the unplanned network.
  const PlanData start = p;
  bool have = false;
  for (int r = 0; r < restarts; ++r) {
    PlanData q = start;
    q.opts.seed = start.opts.seed + 0x9E3779B97F4A7C15ull * (uint64_t)r;
    try {
      make_plan_once(q);
    } catch (const Error&) {
      if (r + 1 == restarts && !have) throw;
      continue;
    }
    if (!have || q.score < p.score) {
      p = std::move(q);
      have = true;
    }
  }
}

// ---------------------------------------------------------------------------
// JSON export
// ---------------------------------------------------------------------------
static void json_list(std::ostringstream& o, const std::vector<int>& v) {
  o << '[';
  for (size_t i = 0; i < v.size(); ++i) o << (i ? "," : "") << v[i];
  o << ']';
}

std::string plan_json(const PlanData& p) {
  std::ostringstream o;
  o.precision(17);
  const Network& net = p.net;
  o << "{\"n_qubits\":" << net.n_qubits << ",\"open\":";
  json_list(o, net.open);
  o << ",\"closed\":";
  json_list(o, net.closed);
  o << ",\"sliced_wires\":[";
  for (size_t j = 0; j < p.sliced.size(); ++j) {
    const Label& L = net.labels[p.sliced[j]];
    o << (j ? "," : "") << '[' << L.q << ',' << L.seg << ']';
  }
  o << "],\"fixed_wires\":[";
  for (size_t j = 0; j < p.fixed.size(); ++j) {
    const Label& L = net.labels[p.fixed[j].first];
    o << (j ? "," : "") << '[' << L.q << ',' << L.seg << ',' << p.fixed[j].second << ']';
  }
  o << "],\"pruned_wires\":[";
  for (size_t j = 0; j < p.pruned.size(); ++j) {
    const Label& L = net.labels[p.pruned[j].first];
    o << (j ? "," : "") << '[' << L.q << ',' << L.seg << ',' << p.pruned[j].second << ']';
  }
  o << "],\"labels\":[";
  for (size_t i = 0; i < net.labels.size(); ++i) {
    const Label& L = net.labels[i];
    o << (i ? "," : "") << '[' << L.kind << ',' << L.q << ',' << L.seg << ']';
  }
  o << "],\"leaves\":[";
  for (size_t i = 0; i < net.leaves.size(); ++i) {
    o << (i ? "," : "");
    json_list(o, net.leaves[i].labels);
  }
  o << "],\"root\":" << p.tree.root << ",\"steps\":[";
  for (size_t i = 0; i < p.steps.size(); ++i) {
    const Step& st = p.steps[i];
    o << (i ? "," : "") << "{\"node\":" << st.node << ",\"a\":" << st.a << ",\"b\":" << st.b
      << ",\"m\":" << st.m << ",\"n\":" << st.n << ",\"k\":" << st.k
      << ",\"dep_s\":" << (int)st.dep_s << ",\"dep_b\":" << (int)st.dep_b << ",\"lp\":" << (int)st.lp
      << ",\"la\":";
    json_list(o, st.la);
    o << ",\"lb\":";
    json_list(o, st.lb);
    o << ",\"lc\":";
    json_list(o, st.lc);
    o << '}';
  }
  o << "],\"flops_per_slice\":" << p.flops_per_slice
    << ",\"flops_per_bitstring\":" << p.flops_per_bitstring << ",\"flops_invariant\":" << p.flops_invariant
    << ",\"max_log2\":" << p.max_log2 << '}';
  return o.str();
}

}  // namespace rqc

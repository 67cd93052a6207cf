// Circuit -> tensor network (Section 3.2, tensor approach: a two-qubit gate
// is a rank-4 tensor; the network is contracted pairwise until one tensor
// is left).  Single-qubit gates, the |0> inputs and the output projections
// are absorbed into the two-qubit gate tensors so that every leaf is one
// two-qubit gate with rank <= 4.
#include <algorithm>
#include <cmath>
#include <stdexcept>

#include "core.h"

namespace rqc {

static const double kS = 0.70710678118654752440;

std::vector<cd> gate_matrix(const Gate& g) {
  const cd I(0, 1);
  switch (g.kind) {
    case RQC_GATE_H:
      return {kS, kS, kS, -kS};
    case RQC_GATE_SQRT_X:  // (sqrt X)^2 = -i X
      return {kS, -I * kS, -I * kS, kS};
    case RQC_GATE_SQRT_Y:  // (sqrt Y)^2 = -i Y
      return {kS, -kS, kS, kS};
    case RQC_GATE_SQRT_W: {  // W = (X + Y)/sqrt 2, (sqrt W)^2 = -i W
      const cd sqrt_i = std::polar(1.0, M_PI / 4);
      const cd sqrt_mi = std::polar(1.0, -M_PI / 4);
      return {kS, -sqrt_i * kS, sqrt_mi * kS, kS};
    }
    case RQC_GATE_FSIM: {
      const double c = std::cos(g.theta), s = std::sin(g.theta);
      std::vector<cd> m(16, 0.0);
      m[0] = 1.0;
      m[5] = c;
      m[6] = -I * s;
      m[9] = -I * s;
      m[10] = c;
      m[15] = std::polar(1.0, -g.phi);
      return m;
    }
    case RQC_GATE_U1:
    case RQC_GATE_U2:
      return g.u;
  }
  throw Error{RQC_EINVAL, "unknown gate kind"};
}

static std::vector<cd> matmul2(const std::vector<cd>& a, const std::vector<cd>& b) {
  return {a[0] * b[0] + a[1] * b[2], a[0] * b[1] + a[1] * b[3],
          a[2] * b[0] + a[3] * b[2], a[2] * b[1] + a[3] * b[3]};
}

// Replace label `w` (at some position of leaf L) by label `x` through the
// 2x2 map cap[x][w].
static void absorb_cap(Leaf& L, int w, int x, const std::vector<cd>& cap) {
  const int r = (int)L.labels.size();
  int pos = -1;
  for (int i = 0; i < r; ++i)
    if (L.labels[i] == w) pos = i;
  if (pos < 0) throw Error{RQC_EINVAL, "internal: wire not found in leaf"};
  const int bit = r - 1 - pos;
  std::vector<cd> out(L.data.size(), 0.0);
  for (size_t e = 0; e < L.data.size(); ++e) {
    const int xv = (int)((e >> bit) & 1);
    const size_t base = e & ~(size_t(1) << bit);
    for (int wv = 0; wv < 2; ++wv)
      out[e] += cap[xv * 2 + wv] * L.data[base | (size_t(wv) << bit)];
  }
  L.data.swap(out);
  L.labels[pos] = x;
}

Network build_network(const Circuit& c, const std::vector<int>& open) {
  Network net;
  const int n = c.n;
  net.n_qubits = n;
  net.open = open;
  std::vector<char> is_open(n, 0);
  for (int q : open) {
    if (q < 0 || q >= n) throw Error{RQC_EINVAL, "open qubit out of range"};
    if (is_open[q]) throw Error{RQC_EINVAL, "open qubit listed twice"};
    is_open[q] = 1;
  }
  for (int q = 0; q < n; ++q)
    if (!is_open[q]) net.closed.push_back(q);

  const std::vector<cd> ident = {1.0, 0.0, 0.0, 1.0};
  std::vector<std::vector<cd>> pend(n, ident);
  std::vector<int> cur(n, -1), seg(n, 0), owner(n, -1);

  auto new_label = [&](int kind, int q, int s) {
    net.labels.push_back({kind, q, s});
    return (int)net.labels.size() - 1;
  };

  for (const Gate& g : c.gates) {
    std::vector<cd> m = gate_matrix(g);
    if (g.q1 < 0) {
      pend[g.q0] = matmul2(m, pend[g.q0]);
      continue;
    }
    const int q0 = g.q0, q1 = g.q1;
    // T[o0 o1][i0 i1] = sum G[o0 o1][j0 j1] P0[j0][i0] P1[j1][i1]
    std::vector<cd> t(16, 0.0);
    for (int o = 0; o < 4; ++o)
      for (int i0 = 0; i0 < 2; ++i0)
        for (int i1 = 0; i1 < 2; ++i1) {
          cd s = 0;
          for (int j0 = 0; j0 < 2; ++j0)
            for (int j1 = 0; j1 < 2; ++j1)
              s += m[o * 4 + j0 * 2 + j1] * pend[q0][j0 * 2 + i0] * pend[q1][j1 * 2 + i1];
          t[o * 4 + i0 * 2 + i1] = s;
        }
    Leaf L;
    const int o0 = new_label(WIRE, q0, seg[q0] + 1);
    const int o1 = new_label(WIRE, q1, seg[q1] + 1);
    L.labels = {o0, o1};
    const bool in0 = cur[q0] >= 0, in1 = cur[q1] >= 0;
    if (in0) L.labels.push_back(cur[q0]);
    if (in1) L.labels.push_back(cur[q1]);
    // Inputs of a qubit's first two-qubit gate are fixed to |0>.
    for (int o = 0; o < 4; ++o)
      for (int i0 = 0; i0 < 2; ++i0)
        for (int i1 = 0; i1 < 2; ++i1) {
          if ((!in0 && i0) || (!in1 && i1)) continue;
          L.data.push_back(t[o * 4 + i0 * 2 + i1]);
        }
    net.leaves.push_back(std::move(L));
    const int id = (int)net.leaves.size() - 1;
    for (int q : {q0, q1}) {
      seg[q] += 1;
      pend[q] = ident;
      owner[q] = id;
    }
    cur[q0] = o0;
    cur[q1] = o1;
    net.wire_label[{q0, seg[q0]}] = o0;
    net.wire_label[{q1, seg[q1]}] = o1;
  }

  net.open_label.assign(open.size(), -1);
  std::vector<int> qlabel(n, -1);
  for (int q = 0; q < n; ++q) qlabel[q] = new_label(is_open[q] ? OPEN : CLOSED, q, 0);
  for (size_t i = 0; i < open.size(); ++i) net.open_label[i] = qlabel[open[i]];
  net.closed_col.assign(net.labels.size(), -1);
  for (size_t ci = 0; ci < net.closed.size(); ++ci) net.closed_col[qlabel[net.closed[ci]]] = (int)ci;

  for (int q = 0; q < n; ++q) {
    const std::vector<cd>& P = pend[q];  // cap[x][w] = P[x][w]
    if (owner[q] < 0) {
      // No two-qubit gate on q: an isolated factor P|0> over its output.
      Leaf L;
      L.labels = {qlabel[q]};
      L.data = {P[0], P[2]};
      net.leaves.push_back(std::move(L));
    } else {
      absorb_cap(net.leaves[owner[q]], cur[q], qlabel[q], P);
      // The final wire segment disappears: it is internal to the leaf now.
      net.wire_label.erase({q, seg[q]});
    }
  }
  return net;
}

}  // namespace rqc

// Internal host-side data structures of the amplitude engine.
#pragma once

#include <complex>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "rqc.h"

namespace rqc {

using cd = std::complex<double>;

// Thread-local error message behind rqc_last_error().
void set_error(const std::string& msg);

struct Error {
  rqc_status code;
  std::string msg;
};

// ---------------------------------------------------------------------------
// Circuit
// ---------------------------------------------------------------------------
struct Gate {
  int kind = 0, q0 = 0, q1 = -1;
  double theta = 0, phi = 0;
  std::vector<cd> u;  // explicit matrix for U1/U2
};

struct Circuit {
  int n = 0;
  std::vector<Gate> gates;
};

// Gate matrix M[out][in] (2x2 or 4x4, row-major) from its definition.
std::vector<cd> gate_matrix(const Gate& g);

// ---------------------------------------------------------------------------
// Tensor network (Section 3.2): one tensor per two-qubit gate after the
// single-qubit gates, the |0> inputs and the output projections have been
// absorbed.  Index labels have a kind:
//   WIRE   canonical wire (q, s): leaves the s-th two-qubit gate on q;
//   OPEN   free output index of an open qubit;
//   CLOSED selector of a closed qubit: bound to the requested bit before
//          contraction, never contracted.
// ---------------------------------------------------------------------------
enum LabelKind { WIRE = 0, OPEN = 1, CLOSED = 2 };

struct Label {
  int kind;
  int q;
  int seg;  // WIRE only
};

struct Leaf {
  std::vector<int> labels;  // most significant address bit first
  std::vector<cd> data;     // 2^rank values, C order over `labels`
};

struct Network {
  int n_qubits = 0;
  std::vector<int> open;          // batch order: open[0] is the LSB
  std::vector<int> closed;        // ascending qubit order
  std::vector<Label> labels;
  std::vector<Leaf> leaves;
  std::map<std::pair<int, int>, int> wire_label;  // (q, s) -> label
  std::vector<int> open_label;    // label of open[i]
  std::vector<int> closed_col;    // per label: column in closed bits or -1
};

Network build_network(const Circuit& c, const std::vector<int>& open);

// ---------------------------------------------------------------------------
// Planning (Sections 5.1-5.2): a binary contraction tree over the leaves,
// a set of sliced wires and, per step, operand layouts.
// ---------------------------------------------------------------------------
struct PlanOpts {
  int max_log2 = 0;
  int n_sliced = -1;
  int trials = 256;
  int reconf_rounds = 4;
  uint64_t seed = 0;
  std::vector<std::pair<int, int>> forced;
  int lp_min_log2 = 14;
  int bf16_min_log2 = 24;
  int n_local = 0;            // 0: all sliced wires enumerated by slice ids
  std::vector<uint8_t> share_bits;  // values of the fixed sliced wires
  int restarts = 1;                 // independent searches, best kept
  int precision_policy = 0;         // RQC_POLICY_*
};

struct Tree {
  // Nodes 0..n_leaves-1 are leaves; internal nodes follow.
  std::vector<int> left, right;
  int root = -1;
  int n_leaves = 0;
};

// Labels of each node of the contraction network restricted to what is
// contracted: CLOSED selectors and sliced wires removed.
struct CostModel {
  double flops = 0;   // complex multiply-adds summed over steps
  double cost = 0;    // time-like cost (multiply-adds or weighted traffic per step)
  int width = 0;      // largest intermediate, log2 elements
};

// One pairwise contraction of the plan in execution order.
struct Step {
  int node;            // tree node produced
  int a, b;            // tree nodes consumed (a = larger operand)
  // Layouts (most significant label first) of A, B, C.
  std::vector<int> la, lb, lc;
  int m = 0, n = 0, k = 0;
  int kernel = 0;      // 0 SIMT, 1 MFMA
  bool dep_s = false, dep_b = false;  // output depends on slice / bits
  bool invariant = false;
  bool lp = false;     // output stored in 16 bits in FP16 mode
  bool lp_bf16 = false;  // output stored in 16 bits in BF16 mode
};

struct PlanData {
  Network net;
  PlanOpts opts;
  Tree tree;
  std::vector<int> sliced;              // enumerated sliced wire labels, slice-bit order
  std::vector<std::pair<int, int>> fixed;  // sliced wires fixed by the share: (label, value)
  std::vector<std::vector<int>> node_labels;  // contracted labels per node
  std::vector<int> node_layout_dummy;
  std::vector<std::vector<int>> layout; // per node: chosen layout
  std::vector<char> dep_s, dep_b;       // per node
  std::vector<Step> steps;              // execution order
  std::vector<int> step_of_node;        // node -> step index or -1
  CostModel cost;                       // per slice
  double flops_invariant = 0;
  double flops_per_slice = 0;      // steps that depend on the sliced wires
  double bytes_per_slice = 0;
  double flops_per_bitstring = 0;  // steps on the closed bits only: shared by all slices
  double bytes_per_bitstring = 0;
  int max_log2 = 0;
  std::vector<std::pair<int, int>> pruned;  // single-valued wires projected out: (label, value)
  double score = 0;                     // search objective of the chosen plan
};

// Builds everything in PlanData from the network and options.
void make_plan(PlanData& p);
std::string plan_json(const PlanData& p);

// Kernel selection and tiling for one step given operand layouts.
int choose_kernel(int m, int n, int k);

}  // namespace rqc

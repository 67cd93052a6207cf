// Host-only driver of the circuit -> network -> plan code (network.cpp,
// planner.cpp) for a build with AddressSanitizer and UndefinedBehavior-
// Sanitizer.  Reads circuits from a text file written by the test:
//   circuit <n_qubits> <n_gates> <n_open> <open qubits...>
//   <kind> <q0> <q1> <theta> <phi>           (one line per gate)
// and plans each one under several option sets (automatic and exact
// slicing, forced wires, slice shares, restarts), printing one summary line
// per plan.  Any sanitizer report makes the process fail.
#include <cstdio>
#include <fstream>
#include <iostream>
#include <string>

#include "core.h"

namespace rqc {
void set_error(const std::string&) {}
}  // namespace rqc

int main(int argc, char** argv) {
  if (argc < 2) {
    std::fprintf(stderr, "usage: plan_driver circuits.txt\n");
    return 2;
  }
  std::ifstream in(argv[1]);
  std::string tag;
  int n_plans = 0, n_rejected = 0;
  while (in >> tag) {
    if (tag != "circuit") return 3;
    rqc::Circuit c;
    size_t n_gates = 0;
    int n_open = 0;
    in >> c.n >> n_gates >> n_open;
    std::vector<int> open(n_open);
    for (int& q : open) in >> q;
    for (size_t i = 0; i < n_gates; ++i) {
      rqc::Gate g;
      in >> g.kind >> g.q0 >> g.q1 >> g.theta >> g.phi;
      c.gates.push_back(g);
    }
    try {
      const rqc::Network net = rqc::build_network(c, open);
      struct Opt {
        int max_log2, n_sliced, n_local, restarts;
        bool forced;
      };
      const Opt opts[] = {{0, -1, 0, 1, false}, {12, -1, 0, 1, false}, {0, 4, 0, 2, false},
                          {10, -1, 0, 1, true}, {10, -1, 2, 1, false}};
      std::vector<std::pair<int, int>> first_wires;
      for (const Opt& o : opts) {
        try {
          rqc::PlanData pd;
          pd.net = net;
          pd.opts.max_log2 = o.max_log2;
          pd.opts.n_sliced = o.n_sliced;
          pd.opts.trials = 16;
          pd.opts.reconf_rounds = 2;
          pd.opts.seed = 7;
          pd.opts.n_local = o.n_local;
          pd.opts.restarts = o.restarts;
          if (o.forced) pd.opts.forced = first_wires;
          rqc::make_plan(pd);
          if (first_wires.empty())
            for (int lab : pd.sliced) {
              const rqc::Label& L = pd.net.labels[lab];
              first_wires.push_back({L.q, L.seg});
            }
          const std::string js = rqc::plan_json(pd);
          std::printf("plan n=%d steps=%zu sliced=%zu fixed=%zu width=%d json=%zu\n", c.n,
                      pd.steps.size(), pd.sliced.size(), pd.fixed.size(), pd.max_log2, js.size());
          ++n_plans;
        } catch (const rqc::Error& e) {
          // Option sets a small circuit cannot satisfy are refused.
          std::printf("rejected %d %s\n", e.code, e.msg.c_str());
          ++n_rejected;
        }
      }
    } catch (const rqc::Error& e) {
      std::printf("error %d %s\n", e.code, e.msg.c_str());
      return 5;
    }
  }
  std::printf("plans %d rejected %d\n", n_plans, n_rejected);
  return n_plans > 0 ? 0 : 4;
}

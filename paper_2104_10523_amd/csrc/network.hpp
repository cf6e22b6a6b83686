// Circuit -> tensor network and the path planner (host side).
#pragma once

#include <functional>
#include <map>
#include <vector>

#include "common.hpp"
#include "gates.hpp"

namespace tn {

// One network tensor: axes labelled by integers, every extent 2 (qubit legs).
struct NetTensor {
  std::vector<int> labels;   // axis order, row-major data
  std::vector<cd> data;      // 2^rank entries
};

struct Network {
  int n_qubits = 0;
  int n_labels = 0;
  std::vector<NetTensor> tensors;
  std::vector<int> out_label;  // per qubit
};

// Folds |0> inputs and one-qubit gates into two-qubit gate tensors; see tn.h.
Network build_network(const tn_circuit& c);

// Cost model evaluated in IEEE double arithmetic (mirrors tn.h).
struct Step {
  int i, j;                    // SSA ids of the operands
  std::vector<int> a, b, c;    // sorted label sets after slicing
};

struct PathStats {
  double flops = 0;            // per slice
  double peak = 0;             // live + |C| + |A| + |B| (elements)
  int peak_step = -1;
  double n_slices = 1;
  double total_flops = 0;
  std::vector<Step> steps;
};

using LabelSets = std::vector<std::vector<int>>;  // sorted labels per leaf

struct PathProblem {
  LabelSets leaves;            // labels after removing projected outputs
  std::vector<double> ext;     // extent per label
  std::vector<char> open;      // per label: 1 = open output
};

// Live tensors of a path search: label sets by SSA id, label reference
// counts, and the candidate pairs of the next step.
struct PathState {
  const PathProblem& pr;
  std::vector<std::vector<int>> sets;   // sorted labels; cleared when consumed
  std::vector<char> alive;
  std::vector<int> count;
  int n_alive = 0;
  PathState(const PathProblem& p, const std::vector<int>& sliced);
  std::vector<int> result(int i, int j) const;
  int merge(int i, int j);
  std::vector<std::pair<int, int>> candidates() const;
};

// One candidate pair (i < j) with the sizes the path searches rank it by:
// |A|, |B|, |C| (the result), |A u B| (flops / 8) and the shared label count.
struct Cand {
  int i, j;
  double sa, sb, sc, su;
  int shared;
};

// The candidate pairs of a PathState kept current across merges, in the
// order and with the values PathState::candidates() + result() give.  A
// merge (i, j) -> k changes the result of no pair that avoids i, j and k: a
// label whose count drops is still held by k, so every other pair keeps it.
// Hence only pairs with i or j are dropped and pairs (x, k) added.
class CandidateSet {
 public:
  explicit CandidateSet(const PathState& st);
  // st.merge(i, j) plus the candidate update; returns the new SSA id.
  int merge(PathState& st, int i, int j);
  const std::vector<Cand>& list() const { return c_; }

 private:
  Cand make(const PathState& st, int i, int j) const;
  void all_pairs(const PathState& st);
  std::vector<std::vector<int>> by_label_;   // live tensors per label, ascending
  std::vector<Cand> c_;
  bool all_pairs_ = false;                   // no live pair shares a label
};

double size_of_labels(const std::vector<int>& s, const std::vector<double>& ext);
std::vector<int> union_of(const std::vector<int>& a, const std::vector<int>& b);
// Path problem of a network: projected output labels removed, open ones kept.
PathProblem make_problem(const Network& net, const std::vector<char>& open_q);

std::vector<std::pair<int, int>> greedy_path(const PathProblem& pr, uint64_t* rng_state,
                                             double temperature);
// With budget_bytes > 0 the kRerank best candidates by unsliced (flops,
// peak) are sliced to the budget and the lowest (total flops, peak) wins.
constexpr int kRerank = 16;
std::vector<std::pair<int, int>> random_greedy_path(const PathProblem& pr, uint64_t seed,
                                                    int trials, double temperature,
                                                    double budget_bytes = 0.0);
PathStats path_stats(const PathProblem& pr, const std::vector<std::pair<int, int>>& path,
                     const std::vector<int>& sliced);
// One recursive-bisection contraction tree (parameters and seed leaves drawn
// from the SplitMix64 stream `rng`), and the best of greedy + `trials` such
// trees by sliced (total flops, peak).
std::vector<std::pair<int, int>> partition_path(const PathProblem& pr, uint64_t* rng);
// Subtree reconfiguration of a complete path: every internal node's subtree
// frontier (at most kReconf tensors) is reordered optimally by flops.
std::vector<std::pair<int, int>> reconfigure_path(const PathProblem& pr,
                                                  const std::vector<std::pair<int, int>>& path);
// The same with another additive step cost of (A, B, result) label sets.
using StepCost = std::function<double(const std::vector<int>&, const std::vector<int>&, const std::vector<int>&)>;
std::vector<std::pair<int, int>> reconfigure_path(const PathProblem& pr, const std::vector<std::pair<int, int>>& path,
                                                  const StepCost& step_cost);
// Modelled seconds of one pairwise step of a slice (sliced labels at extent
// 1 in pr): max(flops / F, bytes / B) + launch, the faster of FP32 and split
// FP16x3 where the GEMM is large enough (M, N, K >= 128), whose operands
// take a max-abs and a packing pass (24 bytes per entry) first.
double step_seconds(const PathProblem& pr, const std::vector<int>& a, const std::vector<int>& b,
                    const std::vector<int>& c);
// Subtree reconfiguration by step_seconds on the sliced problem (passes
// until the summed step time stops falling); the caller re-slices.
std::vector<std::pair<int, int>> reconfigure_for_time(const PathProblem& pr,
                                                      const std::vector<std::pair<int, int>>& path,
                                                      const std::vector<int>& sliced);
// The `keep` best partition-search candidates by (total flops, peak, index),
// best first (at least one: greedy when the budget rejects everything).
std::vector<std::vector<std::pair<int, int>>> partition_candidates(const PathProblem& pr, uint64_t seed,
                                                                  int trials, double budget_bytes, int keep);
std::vector<std::pair<int, int>> partition_search(const PathProblem& pr, uint64_t seed, int trials,
                                                  double budget_bytes);
std::vector<int> slice_path(const PathProblem& pr, const std::vector<std::pair<int, int>>& path,
                            double budget_bytes);
// body(i) for i in [0, n) on up to 16 host threads; rethrows the first error.
void run_parallel(int n, const std::function<void(int)>& body);
uint64_t splitmix64_next(uint64_t* state);
double splitmix64_uniform(uint64_t* state);

}  // namespace tn

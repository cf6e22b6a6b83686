// Circuit -> tensor network (Sec. 3.1, Fig. 1) and the pairwise path planner
// (Sec. 3.1: Flop-minimising contraction order, index slicing).
//
// Network: qubits are rank-1 tensors, one-qubit gates rank-2 and two-qubit
// gates rank-4.  Small gate tensors are folded into the two-qubit gates
// (Sec. 3.1.1): a wire's |0> input and the one-qubit gates before a two-qubit
// gate go into that gate's input side, trailing one-qubit gates into the last
// gate's output leg; a wire without two-qubit gates is one rank-1 tensor.
// Tensors: two-qubit gates in circuit order, then lone wires in qubit order.
// Labels are handed out as legs are created (a's output, then b's).
#include <algorithm>
#include <numeric>
#include <functional>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <exception>
#include <limits>
#include <mutex>
#include <thread>

#include "network.hpp"

namespace tn {

Network build_network(const tn_circuit& c) {
  TN_REQUIRE(c.n_qubits >= 1 && c.n_qubits <= 4096, TN_ERR_ARG, "n_qubits out of range");
  TN_REQUIRE(c.n_ops >= 0 && (c.n_ops == 0 || c.ops != nullptr), TN_ERR_ARG, "bad op list");
  const int n = c.n_qubits;
  Network net;
  net.n_qubits = n;
  std::vector<Mat> pend(n, Mat::identity(2));
  std::vector<int> wire(n, -1);
  std::vector<std::pair<int, int>> owner(n, {-1, -1});
  int nxt = 0;
  for (int64_t k = 0; k < c.n_ops; ++k) {
    const tn_op& op = c.ops[k];
    TN_REQUIRE(!gate_is_channel(op.gate), TN_ERR_GATE,
               "channel op in a noiseless network (use tn_run_trajectories)");
    const int ar = gate_arity(op.gate);
    TN_REQUIRE(op.q0 >= 0 && op.q0 < n, TN_ERR_GATE, "qubit index out of range");
    if (ar == 1) {
      pend[op.q0] = matmul(gate_unitary(op), pend[op.q0]);
      continue;
    }
    const int a = op.q0, b = op.q1;
    TN_REQUIRE(b >= 0 && b < n && a != b, TN_ERR_GATE, "bad second qubit");
    Mat U = matmul(gate_unitary(op), kron(pend[a], pend[b]));
    pend[a] = Mat::identity(2);
    pend[b] = Mat::identity(2);
    // U row = (oa, ob), col = (ia, ib); tensor axes [oa, ob, (ia), (ib)]
    const bool keep_a = wire[a] >= 0, keep_b = wire[b] >= 0;
    NetTensor t;
    t.labels = {nxt, nxt + 1};
    if (keep_a) t.labels.push_back(wire[a]);
    if (keep_b) t.labels.push_back(wire[b]);
    nxt += 2;
    const int ra = keep_a ? 2 : 1, rb = keep_b ? 2 : 1;
    t.data.assign(size_t(4) * ra * rb, cd(0, 0));
    for (int oa = 0; oa < 2; ++oa)
      for (int ob = 0; ob < 2; ++ob)
        for (int ia = 0; ia < ra; ++ia)
          for (int ib = 0; ib < rb; ++ib)
            t.data[((size_t(oa) * 2 + ob) * ra + ia) * rb + ib] = U(oa * 2 + ob, ia * 2 + ib);
    const int tid = int(net.tensors.size());
    net.tensors.push_back(std::move(t));
    wire[a] = nxt - 2;
    wire[b] = nxt - 1;
    owner[a] = {tid, 0};
    owner[b] = {tid, 1};
  }
  for (int q = 0; q < n; ++q) {
    if (owner[q].first < 0 || is_identity(pend[q])) continue;
    NetTensor& t = net.tensors[owner[q].first];
    const int ax = owner[q].second, rank = int(t.labels.size());
    const size_t stride = size_t(1) << (rank - 1 - ax);
    for (size_t i = 0; i < t.data.size(); ++i) {
      if (i & stride) continue;
      const cd x0 = t.data[i], x1 = t.data[i | stride];
      t.data[i] = pend[q](0, 0) * x0 + pend[q](0, 1) * x1;
      t.data[i | stride] = pend[q](1, 0) * x0 + pend[q](1, 1) * x1;
    }
  }
  for (int q = 0; q < n; ++q) {
    if (owner[q].first >= 0) continue;
    NetTensor t;
    t.labels = {nxt};
    t.data = {pend[q](0, 0), pend[q](1, 0)};
    net.tensors.push_back(std::move(t));
    wire[q] = nxt++;
  }
  net.out_label = wire;
  net.n_labels = nxt;
  return net;
}

// ---------------------------------------------------------------- planner

uint64_t splitmix64_next(uint64_t* s) {
  *s += 0x9E3779B97F4A7C15ull;
  uint64_t z = *s;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double splitmix64_uniform(uint64_t* s) {
  return double(splitmix64_next(s) >> 11) * (1.0 / 9007199254740992.0);
}

using Set = std::vector<int>;  // sorted labels

std::vector<int> union_of(const Set& a, const Set& b) {
  Set r;
  r.reserve(a.size() + b.size());
  std::set_union(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(r));
  return r;
}

double size_of_labels(const Set& s, const std::vector<double>& ext) {
  double v = 1.0;
  for (int l : s) v = v * ext[l];
  return v;
}

namespace {
inline Set set_union(const Set& a, const Set& b) { return union_of(a, b); }
inline double size_of(const Set& s, const std::vector<double>& ext) { return size_of_labels(s, ext); }
using State = PathState;
}  // namespace

PathState::PathState(const PathProblem& p, const std::vector<int>& sliced) : pr(p), count(p.ext.size(), 0) {
  std::vector<char> cut(p.ext.size(), 0);
  for (int l : sliced) cut[l] = 1;
  for (const Set& s : p.leaves) {
    Set t;
    for (int l : s)
      if (!cut[l]) t.push_back(l);
    for (int l : t) count[l]++;
    sets.push_back(std::move(t));
    alive.push_back(1);
    n_alive++;
  }
}

Set PathState::result(int i, int j) const {
  const Set &a = sets[i], &b = sets[j];
  Set u = set_union(a, b), c;
  for (int l : u) {
    const int in_a = std::binary_search(a.begin(), a.end(), l);
    const int in_b = std::binary_search(b.begin(), b.end(), l);
    if (pr.open[l] || count[l] - in_a - in_b > 0) c.push_back(l);
  }
  return c;
}

int PathState::merge(int i, int j) {
  Set c = result(i, j);
  for (int l : sets[i]) count[l]--;
  for (int l : sets[j]) count[l]--;
  for (int l : c) count[l]++;
  sets[i].clear();
  sets[j].clear();
  alive[i] = alive[j] = 0;
  sets.push_back(std::move(c));
  alive.push_back(1);
  n_alive--;
  return int(sets.size()) - 1;
}

std::vector<std::pair<int, int>> PathState::candidates() const {
  std::vector<std::vector<int>> by_label(pr.ext.size());
  for (size_t i = 0; i < sets.size(); ++i)
    if (alive[i])
      for (int l : sets[i]) by_label[l].push_back(int(i));
  std::vector<std::pair<int, int>> pairs;
  for (const auto& ids : by_label)
    for (size_t x = 0; x < ids.size(); ++x)
      for (size_t y = x + 1; y < ids.size(); ++y) pairs.push_back({ids[x], ids[y]});
  if (pairs.empty()) {
    std::vector<int> ids;
    for (size_t i = 0; i < sets.size(); ++i)
      if (alive[i]) ids.push_back(int(i));
    for (size_t x = 0; x < ids.size(); ++x)
      for (size_t y = x + 1; y < ids.size(); ++y) pairs.push_back({ids[x], ids[y]});
  }
  std::sort(pairs.begin(), pairs.end());
  pairs.erase(std::unique(pairs.begin(), pairs.end()), pairs.end());
  return pairs;
}

PathProblem make_problem(const Network& net, const std::vector<char>& open_q) {
  PathProblem pr;
  pr.ext.assign(net.n_labels, 2.0);
  pr.open.assign(net.n_labels, 0);
  std::vector<char> proj(net.n_labels, 0);
  for (int q = 0; q < net.n_qubits; ++q) {
    if (open_q[q]) pr.open[net.out_label[q]] = 1;
    else proj[net.out_label[q]] = 1;
  }
  for (const auto& t : net.tensors) {
    std::vector<int> s;
    for (int l : t.labels)
      if (!proj[l]) s.push_back(l);
    std::sort(s.begin(), s.end());
    pr.leaves.push_back(s);
  }
  return pr;
}

CandidateSet::CandidateSet(const PathState& st) : by_label_(st.pr.ext.size()) {
  for (size_t i = 0; i < st.sets.size(); ++i)
    if (st.alive[i])
      for (int l : st.sets[i]) by_label_[l].push_back(int(i));
  std::vector<std::pair<int, int>> pairs;
  for (const auto& ids : by_label_)
    for (size_t x = 0; x < ids.size(); ++x)
      for (size_t y = x + 1; y < ids.size(); ++y) pairs.push_back({ids[x], ids[y]});
  std::sort(pairs.begin(), pairs.end());
  pairs.erase(std::unique(pairs.begin(), pairs.end()), pairs.end());
  for (auto [i, j] : pairs) c_.push_back(make(st, i, j));
  if (c_.empty() && st.n_alive > 1) all_pairs(st);
}

Cand CandidateSet::make(const PathState& st, int i, int j) const {
  const Set &a = st.sets[i], &b = st.sets[j];
  const auto& ext = st.pr.ext;
  int shared = 0;
  for (int l : a)
    if (std::binary_search(b.begin(), b.end(), l)) ++shared;
  return {i, j, size_of(a, ext), size_of(b, ext), size_of(st.result(i, j), ext), size_of(set_union(a, b), ext),
          shared};
}

void CandidateSet::all_pairs(const PathState& st) {
  all_pairs_ = true;
  c_.clear();
  std::vector<int> ids;
  for (size_t i = 0; i < st.sets.size(); ++i)
    if (st.alive[i]) ids.push_back(int(i));
  for (size_t x = 0; x < ids.size(); ++x)
    for (size_t y = x + 1; y < ids.size(); ++y) c_.push_back(make(st, ids[x], ids[y]));
}

int CandidateSet::merge(PathState& st, int i, int j) {
  for (int t : {i, j})
    for (int l : st.sets[t]) {
      auto& v = by_label_[l];
      v.erase(std::lower_bound(v.begin(), v.end(), t));
    }
  const int k = st.merge(i, j);
  for (int l : st.sets[k]) by_label_[l].push_back(k);
  // partners of k, ascending
  std::vector<int> xs;
  if (all_pairs_) {
    for (int x = 0; x < k; ++x)
      if (st.alive[x]) xs.push_back(x);
  } else {
    for (int l : st.sets[k])
      for (int x : by_label_[l])
        if (x != k) xs.push_back(x);
    std::sort(xs.begin(), xs.end());
    xs.erase(std::unique(xs.begin(), xs.end()), xs.end());
  }
  // (x, k) sorts after every (x, y < k) and before every (x' > x, .)
  std::vector<Cand> next;
  next.reserve(c_.size() + xs.size());
  size_t q = 0;
  for (const Cand& e : c_) {
    if (e.i == i || e.j == i || e.i == j || e.j == j) continue;
    while (q < xs.size() && xs[q] < e.i) next.push_back(make(st, xs[q++], k));
    next.push_back(e);
  }
  while (q < xs.size()) next.push_back(make(st, xs[q++], k));
  c_.swap(next);
  if (c_.empty() && !all_pairs_ && st.n_alive > 1) all_pairs(st);
  return k;
}

std::vector<std::pair<int, int>> greedy_path(const PathProblem& pr, uint64_t* rng,
                                             double temperature) {
  State st(pr, {});
  CandidateSet cs(st);
  std::vector<std::pair<int, int>> path;
  std::vector<double> sig, w;
  while (st.n_alive > 1) {
    const auto& cands = cs.list();
    const size_t nc = cands.size();
    auto d_of = [&](size_t k) { return cands[k].sc - cands[k].sa - cands[k].sb; };
    size_t pick = 0;
    if (rng == nullptr) {
      double dp = d_of(0), fp = 8.0 * cands[0].su;
      for (size_t k = 1; k < nc; ++k) {
        const double dk = d_of(k), fk = 8.0 * cands[k].su;
        if (dk < dp || (dk == dp && fk < fp)) {   // ties keep the lower pair (ascending order)
          pick = k;
          dp = dk;
          fp = fk;
        }
      }
    } else {
      sig.resize(nc);
      w.resize(nc);
      double smin = std::numeric_limits<double>::infinity();
      for (size_t k = 0; k < nc; ++k) {
        const double d = d_of(k);
        sig[k] = std::copysign(std::log2(1.0 + std::fabs(d)), d);
        smin = std::min(smin, sig[k]);
      }
      double tot = 0.0;
      for (size_t k = 0; k < nc; ++k) {
        w[k] = std::exp(-(sig[k] - smin) / temperature);
        tot += w[k];
      }
      const double u = splitmix64_uniform(rng) * tot;
      double acc = 0.0;
      pick = nc - 1;
      for (size_t k = 0; k < nc; ++k) {
        acc += w[k];
        if (acc >= u) { pick = k; break; }
      }
    }
    const std::pair<int, int> step{cands[pick].i, cands[pick].j};
    cs.merge(st, step.first, step.second);
    path.push_back(step);
  }
  return path;
}

PathStats path_stats(const PathProblem& pr, const std::vector<std::pair<int, int>>& path,
                     const std::vector<int>& sliced) {
  State st(pr, sliced);
  const int n_leaves = int(pr.leaves.size());
  TN_REQUIRE(int(path.size()) == std::max(n_leaves - 1, 0), TN_ERR_ARG,
             "path must have n_tensors - 1 steps");
  PathStats ps;
  double live = 0.0;
  for (const Set& s : st.sets) live += size_of(s, pr.ext);
  for (size_t t = 0; t < path.size(); ++t) {
    const int i = path[t].first, j = path[t].second;
    TN_REQUIRE(i >= 0 && j >= 0 && i != j && i < int(st.sets.size()) && j < int(st.sets.size()) &&
                   st.alive[i] && st.alive[j],
               TN_ERR_ARG, "path step uses a consumed or unknown tensor");
    Step s;
    s.i = i;
    s.j = j;
    s.a = st.sets[i];
    s.b = st.sets[j];
    s.c = st.result(i, j);
    const double sa = size_of(s.a, pr.ext), sb = size_of(s.b, pr.ext), sc = size_of(s.c, pr.ext);
    const double p = live + sc + sa + sb;
    if (p > ps.peak) {
      ps.peak = p;
      ps.peak_step = int(t);
    }
    ps.flops += 8.0 * size_of(set_union(s.a, s.b), pr.ext);
    st.merge(i, j);
    live = live - sa - sb + sc;
    ps.steps.push_back(std::move(s));
  }
  if (path.empty()) ps.peak = live;
  Set sl(sliced.begin(), sliced.end());
  std::sort(sl.begin(), sl.end());
  ps.n_slices = 1.0;
  for (int l : sl) ps.n_slices *= pr.ext[l];
  ps.total_flops = ps.flops * ps.n_slices;
  return ps;
}

namespace {
int path_threads(int work) {
  int nt = int(std::max(1u, std::thread::hardware_concurrency()));
  if (const char* e = std::getenv("OMP_NUM_THREADS")) nt = std::min(nt, std::max(1, std::atoi(e)));
  return std::max(1, std::min({nt, 16, work}));
}

// Runs body(i) for i in [0, n) on host threads; the first exception wins.
template <class F>
void parallel_for(int n, F&& body) {
  std::atomic<int> next{0};
  std::exception_ptr err;
  std::mutex err_mu;
  auto worker = [&]() {
    for (int i; (i = next.fetch_add(1)) < n;) {
      try {
        body(i);
      } catch (...) {
        std::lock_guard<std::mutex> lk(err_mu);
        if (!err) err = std::current_exception();
      }
    }
  };
  const int nt = path_threads(n);
  std::vector<std::thread> pool;
  for (int t = 1; t < nt; ++t) pool.emplace_back(worker);
  worker();
  for (auto& th : pool) th.join();
  if (err) std::rethrow_exception(err);
}
}  // namespace

void run_parallel(int n, const std::function<void(int)>& body) { parallel_for(n, body); }

std::vector<std::pair<int, int>> random_greedy_path(const PathProblem& pr, uint64_t seed,
                                                    int trials, double temperature, double budget_bytes) {
  // Trial r draws from its own stream (seed + r * golden ratio), so the
  // trials run on host threads in any order.  Candidates are the plain
  // greedy path (rank -1) and the trials, ordered by unsliced (flops, peak,
  // rank); without a budget the first wins, exactly as a sequential scan
  // would pick.
  trials = std::max(trials, 0);
  std::vector<std::vector<std::pair<int, int>>> paths(trials + 1);
  std::vector<double> fl(trials + 1), pk(trials + 1);
  paths[0] = greedy_path(pr, nullptr, temperature);
  {
    const PathStats s = path_stats(pr, paths[0], {});
    fl[0] = s.flops;
    pk[0] = s.peak;
  }
  parallel_for(trials, [&](int r) {
    uint64_t g = seed + uint64_t(r) * 0x9E3779B97F4A7C15ull;
    uint64_t st = splitmix64_next(&g);
    paths[r + 1] = greedy_path(pr, &st, temperature);
    const PathStats s = path_stats(pr, paths[r + 1], {});
    fl[r + 1] = s.flops;
    pk[r + 1] = s.peak;
  });
  std::vector<int> order(trials + 1);
  for (int i = 0; i <= trials; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return fl[a] < fl[b] || (fl[a] == fl[b] && pk[a] < pk[b]);
  });
  if (budget_bytes <= 0) return std::move(paths[order[0]]);
  // re-rank the best few by what slicing to the budget leaves
  const int nr = std::min(kRerank, trials + 1);
  std::vector<double> tf(nr, 0.0), tp(nr, 0.0);
  std::vector<char> ok(nr, 0);
  parallel_for(nr, [&](int i) {
    try {
      const auto& path = paths[order[i]];
      const PathStats s = path_stats(pr, path, slice_path(pr, path, budget_bytes));
      tf[i] = s.total_flops;
      tp[i] = s.peak;
      ok[i] = 1;
    } catch (const Error& e) {
      if (e.code != TN_ERR_BUDGET) throw;
    }
  });
  int win = -1;
  for (int i = 0; i < nr; ++i)
    if (ok[i] && (win < 0 || tf[i] < tf[win] || (tf[i] == tf[win] && tp[i] < tp[win]))) win = i;
  return std::move(paths[order[win < 0 ? 0 : win]]);
}

// ------------------------------------------- recursive-bisection search

namespace {

// Leaf graph: one adjacency entry per label shared by exactly two leaves
// (open labels excluded), both directions, in ascending label order.
struct LeafGraph {
  std::vector<std::vector<int>> adj;
  std::vector<std::vector<int>> holders;   // per label
};

LeafGraph leaf_graph(const PathProblem& pr) {
  LeafGraph g;
  const int n = int(pr.leaves.size());
  g.adj.assign(n, {});
  g.holders.assign(pr.ext.size(), {});
  for (int i = 0; i < n; ++i)
    for (int l : pr.leaves[i]) g.holders[l].push_back(i);
  for (size_t l = 0; l < g.holders.size(); ++l) {
    const auto& h = g.holders[l];
    if (h.size() == 2 && !pr.open[l]) {
      g.adj[h[0]].push_back(h[1]);
      g.adj[h[1]].push_back(h[0]);
    }
  }
  return g;
}

constexpr int kRestarts = 8;

struct Bisector {
  const PathProblem& pr;
  const LeafGraph& g;
  double eps;
  int cutoff;
  uint64_t* rng;
  std::vector<int> side;      // -1 outside the current node set
  std::vector<int> aux;       // links into part 0 / gains
  std::vector<char> locked;
  std::vector<std::pair<int, int>> pairs;
  int next_id;

  Bisector(const PathProblem& p, const LeafGraph& gr, double e, int c, uint64_t* r)
      : pr(p), g(gr), eps(e), cutoff(c), rng(r), side(p.leaves.size(), -1), aux(p.leaves.size(), 0),
        locked(p.leaves.size(), 0), next_id(int(p.leaves.size())) {}

  // Splits `nodes` in two: the lowest cut of kRestarts bisections (each
  // from its own seed leaf; the first on ties).
  void bisect(const std::vector<int>& nodes, std::vector<int>& p0, std::vector<int>& p1) {
    int best = -1;
    std::vector<int> a, b;
    for (int r = 0; r < kRestarts; ++r) {
      const int c = bisect_once(nodes, a, b);
      if (best < 0 || c < best) {
        best = c;
        p0 = a;
        p1 = b;
      }
    }
  }

  // One bisection of `nodes` (ascending): part 0 grown from a random seed
  // leaf by most links into it (ties: smallest id) to half the set, then
  // Fiduccia-Mattheyses passes: move the unlocked leaf of largest cut gain
  // (ties: smallest id) that keeps both parts within [lo, hi], keep the
  // best prefix of moves, stop when a pass no longer lowers the cut.
  // Returns the final cut.
  int bisect_once(const std::vector<int>& nodes, std::vector<int>& p0, std::vector<int>& p1) {
    const int n = int(nodes.size());
    for (int v : nodes) {
      side[v] = 1;
      aux[v] = 0;
    }
    const int seed = nodes[splitmix64_next(rng) % uint64_t(n)];
    auto add0 = [&](int v) {
      side[v] = 0;
      for (int u : g.adj[v])
        if (side[u] >= 0) ++aux[u];
    };
    add0(seed);
    for (int na = 1; na < n / 2; ++na) {
      int pick = -1;
      for (int v : nodes)
        if (side[v] == 1 && aux[v] > 0 && (pick < 0 || aux[v] > aux[pick])) pick = v;
      if (pick < 0)
        for (int v : nodes)
          if (side[v] == 1) { pick = v; break; }
      add0(pick);
    }
    const int lo = std::max(1, int(std::floor((1.0 - eps) * n / 2.0))), hi = n - lo;
    auto cut_of = [&]() {
      int c = 0;
      for (int v : nodes)
        for (int u : g.adj[v])
          if (side[u] >= 0 && side[u] != side[v]) ++c;
      return c / 2;
    };
    int cut = cut_of();
    for (int pass = 0; pass < 6; ++pass) {
      int sizes[2] = {0, 0};
      for (int v : nodes) {
        ++sizes[side[v]];
        locked[v] = 0;
        int gn = 0;
        for (int u : g.adj[v])
          if (side[u] >= 0) gn += side[u] != side[v] ? 1 : -1;
        aux[v] = gn;
      }
      int cur = cut, best_c = cut, best_k = 0;
      std::vector<int> moved;
      for (int k = 0; k < n; ++k) {
        int pick = -1;
        for (int v : nodes) {
          if (locked[v] || sizes[side[v]] - 1 < lo || sizes[1 - side[v]] + 1 > hi) continue;
          if (pick < 0 || aux[v] > aux[pick]) pick = v;
        }
        if (pick < 0) break;
        const int s0 = side[pick];
        side[pick] = 1 - s0;
        --sizes[s0];
        ++sizes[1 - s0];
        cur -= aux[pick];
        aux[pick] = -aux[pick];
        locked[pick] = 1;
        moved.push_back(pick);
        for (int u : g.adj[pick])
          if (side[u] >= 0) aux[u] += side[u] == s0 ? 2 : -2;
        if (cur < best_c) {
          best_c = cur;
          best_k = k + 1;
        }
      }
      for (int k = int(moved.size()) - 1; k >= best_k; --k) side[moved[k]] = 1 - side[moved[k]];
      if (best_c >= cut) break;
      cut = best_c;
    }
    p0.clear();
    p1.clear();
    for (int v : nodes) (side[v] == 0 ? p0 : p1).push_back(v);
    for (int v : nodes) side[v] = -1;
    return cut;
  }

  // Contraction tree of `nodes`: the two halves' results contracted last;
  // sets of at most `cutoff` leaves ordered by greedy, keeping the labels
  // they share with the rest of the network.  Returns the result's SSA id.
  int build(const std::vector<int>& nodes) {
    if (nodes.size() == 1) return nodes[0];
    if (int(nodes.size()) <= cutoff) {
      PathProblem sub;
      sub.ext = pr.ext;
      sub.open = pr.open;
      for (int v : nodes) side[v] = 0;
      for (int v : nodes)
        for (int l : pr.leaves[v])
          for (int h : g.holders[l])
            if (side[h] < 0) sub.open[l] = 1;
      for (int v : nodes) side[v] = -1;
      for (int v : nodes) sub.leaves.push_back(pr.leaves[v]);
      const auto gp = greedy_path(sub, nullptr, 1.0);
      std::vector<int> ids(nodes);
      for (const auto& st : gp) {
        pairs.push_back({ids[st.first], ids[st.second]});
        ids.push_back(next_id++);
      }
      return ids.back();
    }
    std::vector<int> p0, p1;
    bisect(nodes, p0, p1);
    const int a = build(p0);
    const int b = build(p1);
    pairs.push_back({a, b});
    return next_id++;
  }
};

}  // namespace

std::vector<std::pair<int, int>> partition_path(const PathProblem& pr, uint64_t* rng) {
  static const int kCutoffs[5] = {2, 4, 8, 16, 32};
  const double eps = 0.05 + 0.85 * splitmix64_uniform(rng);
  const int cutoff = kCutoffs[splitmix64_next(rng) % 5];
  const int n = int(pr.leaves.size());
  if (n <= 1) return {};
  const LeafGraph g = leaf_graph(pr);
  Bisector b(pr, g, eps, cutoff, rng);
  std::vector<int> all(n);
  for (int i = 0; i < n; ++i) all[i] = i;
  b.build(all);
  return std::move(b.pairs);
}

// Subtree reconfiguration: for every internal node (in creation order) the
// frontier of its subtree is grown to at most kReconf tensors by expanding
// the largest internal frontier node (ties: smallest id); the cheapest order
// of that frontier (exact search over subsets, flops 8*size(A u B) per step,
// kept labels = the node's result) replaces the subtree when it is cheaper.
// The cost of a step is its flops, or any StepCost of (A, B, result).
constexpr int kReconf = 8;
constexpr int kReconfPasses = 8;   // passes until one no longer lowers the flops

std::vector<std::pair<int, int>> reconfigure_path(const PathProblem& pr,
                                                  const std::vector<std::pair<int, int>>& path) {
  return reconfigure_path(pr, path, [&pr](const std::vector<int>& a, const std::vector<int>& b,
                                          const std::vector<int>&) {
    return 8.0 * size_of(set_union(a, b), pr.ext);
  });
}

std::vector<std::pair<int, int>> reconfigure_path(const PathProblem& pr, const std::vector<std::pair<int, int>>& path,
                                                  const StepCost& step_cost) {
  const int n = int(pr.leaves.size());
  const int total = n + int(path.size());
  std::vector<int> ca(total, -1), cb(total, -1);
  for (size_t t = 0; t < path.size(); ++t) {
    ca[n + t] = path[t].first;
    cb[n + t] = path[t].second;
  }
  // result label sets bottom-up (labels leaving the subtree, or open)
  std::vector<int> holders_n(pr.ext.size(), 0);
  for (const auto& L : pr.leaves)
    for (int l : L) ++holders_n[l];
  std::vector<std::vector<int>> sets(total);
  // label counts inside each subtree as sorted (label, count) vectors
  std::vector<std::vector<std::pair<int, int>>> cnt(total);
  for (int i = 0; i < n; ++i) {
    for (int l : pr.leaves[i]) cnt[i].push_back({l, 1});
    sets[i] = pr.leaves[i];
  }
  auto merge_cnt = [](const std::vector<std::pair<int, int>>& x, const std::vector<std::pair<int, int>>& y) {
    std::vector<std::pair<int, int>> r;
    size_t i = 0, j = 0;
    while (i < x.size() || j < y.size()) {
      if (j == y.size() || (i < x.size() && x[i].first < y[j].first)) r.push_back(x[i++]);
      else if (i == x.size() || y[j].first < x[i].first) r.push_back(y[j++]);
      else { r.push_back({x[i].first, x[i].second + y[j].second}); ++i; ++j; }
    }
    return r;
  };
  for (int v = n; v < total; ++v) {
    cnt[v] = merge_cnt(cnt[ca[v]], cnt[cb[v]]);
    std::vector<int> r;
    for (const auto& [l, c] : cnt[v])
      if (pr.open[l] || c < holders_n[l]) r.push_back(l);
    sets[v] = std::move(r);
  }
  std::vector<double> cost(total, 0.0);
  for (int v = n; v < total; ++v) cost[v] = step_cost(sets[ca[v]], sets[cb[v]], sets[v]);
  for (int v = n; v < total; ++v) {
    // frontier of v
    std::vector<int> F = {ca[v], cb[v]};
    std::vector<int> region = {v};
    while (int(F.size()) < kReconf) {
      int pick = -1;
      for (size_t k = 0; k < F.size(); ++k) {
        const int u = F[k];
        if (u < n) continue;
        if (pick < 0 || size_of(sets[u], pr.ext) > size_of(sets[F[pick]], pr.ext) ||
            (size_of(sets[u], pr.ext) == size_of(sets[F[pick]], pr.ext) && u < F[pick]))
          pick = int(k);
      }
      if (pick < 0) break;
      const int u = F[pick];
      region.push_back(u);
      F.erase(F.begin() + pick);
      F.push_back(ca[u]);
      F.push_back(cb[u]);
    }
    if (F.size() < 3) continue;
    double cur = 0.0;
    for (int u : region) cur += cost[u];
    // exact search over subsets of the frontier
    const int m = int(F.size());
    const int full = (1 << m) - 1;
    // labels of each subset's result: labels in the subset's union that are in sets[v]
    // or held by another frontier member
    std::vector<std::vector<int>> rs(full + 1);
    std::vector<double> best(full + 1, 0.0);
    std::vector<int> split(full + 1, 0);
    for (int S = 1; S <= full; ++S) {
      std::vector<int> u;
      for (int k = 0; k < m; ++k)
        if (S >> k & 1) u = set_union(u, sets[F[k]]);
      if ((S & (S - 1)) == 0) {
        rs[S] = sets[F[__builtin_ctz(S)]];
        continue;
      }
      std::vector<int> outside;
      for (int k = 0; k < m; ++k)
        if (!(S >> k & 1)) outside = set_union(outside, sets[F[k]]);
      std::vector<int> r;
      for (int l : u)
        if (std::binary_search(sets[v].begin(), sets[v].end(), l) ||
            std::binary_search(outside.begin(), outside.end(), l))
          r.push_back(l);
      rs[S] = std::move(r);
    }
    for (int S = 1; S <= full; ++S) {
      if ((S & (S - 1)) == 0) continue;
      const int low = S & -S;
      double bv = -1.0;
      int bs = 0;
      for (int A = (S - 1) & S; A > 0; A = (A - 1) & S) {
        if (!(A & low)) continue;
        const int B = S ^ A;
        const double c = best[A] + best[B] + step_cost(rs[A], rs[B], rs[S]);
        if (bv < 0 || c < bv) { bv = c; bs = A; }
      }
      best[S] = bv;
      split[S] = bs;
    }
    if (!(best[full] < cur)) continue;
    // rebuild the region: reuse the region's node ids for the new internal nodes
    std::vector<int> ids(region);   // v stays the root
    std::sort(ids.begin() + 1, ids.end());
    int next = 1;
    std::function<int(int)> make = [&](int S) -> int {
      if ((S & (S - 1)) == 0) return F[__builtin_ctz(S)];
      const int A = split[S], B = S ^ A;
      const int x = make(A), y = make(B);
      const int node = S == full ? v : ids[next++];
      ca[node] = x;
      cb[node] = y;
      sets[node] = rs[S];
      cost[node] = step_cost(sets[x], sets[y], sets[node]);
      return node;
    };
    make(full);
  }
  // emit SSA pairs in a post-order of the new tree
  std::vector<std::pair<int, int>> out;
  std::vector<int> ssa(total, -1);
  for (int i = 0; i < n; ++i) ssa[i] = i;
  int nid = n;
  std::function<int(int)> emit = [&](int u) -> int {
    if (u < n) return u;
    const int x = emit(ca[u]), y = emit(cb[u]);
    out.push_back({x, y});
    return nid++;
  };
  emit(total - 1);
  return out;
}

double step_seconds(const PathProblem& pr, const std::vector<int>& a, const std::vector<int>& b,
                    const std::vector<int>& c) {
  constexpr double kSplit = 350e12, kFp32 = 120e12, kHbm = 4.0e12, kLaunch = 5e-6;
  std::vector<int> inter, batch, summed;
  std::set_intersection(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(inter));
  for (int l : inter) (std::binary_search(c.begin(), c.end(), l) ? batch : summed).push_back(l);
  const double sa = size_of(a, pr.ext), sb = size_of(b, pr.ext), sc = size_of(c, pr.ext);
  const double fl = 8.0 * size_of(set_union(a, b), pr.ext);
  const double k = size_of(summed, pr.ext), bt = size_of(batch, pr.ext);
  const double m = sa / (k * bt), nn = sb / (k * bt);
  const double mem = 8.0 * (sa + sb + sc) / kHbm;
  double t = std::max(fl / kFp32, mem);
  if (m >= 128 && nn >= 128 && k >= 128) t = std::min(t, std::max(fl / kSplit, mem) + 24.0 * (sa + sb) / kHbm);
  return t + kLaunch;
}

std::vector<std::pair<int, int>> reconfigure_for_time(const PathProblem& pr,
                                                      const std::vector<std::pair<int, int>>& path,
                                                      const std::vector<int>& sliced) {
  PathProblem ps = pr;
  for (int l : sliced) ps.ext[l] = 1.0;
  const StepCost cost = [&ps](const std::vector<int>& a, const std::vector<int>& b, const std::vector<int>& c) {
    return step_seconds(ps, a, b, c);
  };
  auto total = [&](const std::vector<std::pair<int, int>>& p) {
    double t = 0;
    for (const Step& s : path_stats(ps, p, {}).steps) t += step_seconds(ps, s.a, s.b, s.c);
    return t;
  };
  auto cur = path;
  double tc = total(cur);
  for (int pass = 0; pass < kReconfPasses; ++pass) {
    auto nxt = reconfigure_path(ps, cur, cost);
    const double tn = total(nxt);
    if (!(tn < tc)) break;
    cur = std::move(nxt);
    tc = tn;
  }
  return cur;
}

std::vector<std::vector<std::pair<int, int>>> partition_candidates(const PathProblem& pr, uint64_t seed,
                                                                  int trials, double budget_bytes, int keep) {
  // Candidates: the plain greedy path (index 0) and `trials` bisection trees
  // (trial r seeded like the randomised greedy).  Each is sliced to the
  // budget (if any); the `keep` lowest by (total flops, peak, index) are
  // returned in that order (the first is the search's winner).
  trials = std::max(trials, 0);
  std::vector<std::vector<std::pair<int, int>>> paths(trials + 1);
  std::vector<double> tf(trials + 1, 0.0), tp(trials + 1, 0.0);
  std::vector<char> ok(trials + 1, 0);
  auto score = [&](int i) {
    try {
      const PathStats s = path_stats(pr, paths[i], slice_path(pr, paths[i], budget_bytes));
      tf[i] = s.total_flops;
      tp[i] = s.peak;
      ok[i] = 1;
    } catch (const Error& e) {
      if (e.code != TN_ERR_BUDGET) throw;
    }
  };
  paths[0] = greedy_path(pr, nullptr, 1.0);
  score(0);
  parallel_for(trials, [&](int r) {
    uint64_t gs = seed + uint64_t(r) * 0x9E3779B97F4A7C15ull;
    uint64_t st = splitmix64_next(&gs);
    {
      auto cur = partition_path(pr, &st);
      double fl = path_stats(pr, cur, {}).flops;
      for (int pass = 0; pass < kReconfPasses; ++pass) {
        auto nxt = reconfigure_path(pr, cur);
        const double f2 = path_stats(pr, nxt, {}).flops;
        cur = std::move(nxt);
        if (!(f2 < fl)) break;
        fl = f2;
      }
      paths[r + 1] = std::move(cur);
    }
    score(r + 1);
  });
  // order by (total flops, peak, index); candidates the budget rejects go last
  std::vector<int> order(trials + 1);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    if (ok[a] != ok[b]) return ok[a] > ok[b];
    if (tf[a] != tf[b]) return tf[a] < tf[b];
    return tp[a] < tp[b];
  });
  std::vector<std::vector<std::pair<int, int>>> out;
  for (int k = 0; k < std::max(1, keep) && k <= trials; ++k) {
    if (!ok[order[k]] && k > 0) break;
    out.push_back(std::move(paths[order[k]]));
  }
  return out;
}

std::vector<std::pair<int, int>> partition_search(const PathProblem& pr, uint64_t seed, int trials,
                                                  double budget_bytes) {
  return std::move(partition_candidates(pr, seed, trials, budget_bytes, 1)[0]);
}

std::vector<int> slice_path(const PathProblem& pr, const std::vector<std::pair<int, int>>& path,
                            double budget_bytes) {
  std::vector<int> sliced;
  if (budget_bytes <= 0) return sliced;
  PathStats cur = path_stats(pr, path, sliced);
  while (8.0 * cur.peak > budget_bytes) {
    TN_REQUIRE(cur.peak_step >= 0, TN_ERR_BUDGET, "memory budget smaller than the leaves");
    const Step& s = cur.steps[cur.peak_step];
    Set u = set_union(set_union(s.a, s.b), s.c);
    bool found = false;
    double bpk = 0, bfl = 0;
    int bl = -1;
    PathStats bst;
    for (int l : u) {
      if (pr.open[l] || std::find(sliced.begin(), sliced.end(), l) != sliced.end()) continue;
      auto trial = sliced;
      trial.push_back(l);
      PathStats ts = path_stats(pr, path, trial);
      if (!found || ts.peak < bpk || (ts.peak == bpk && (ts.total_flops < bfl ||
                                                        (ts.total_flops == bfl && l < bl)))) {
        found = true;
        bpk = ts.peak;
        bfl = ts.total_flops;
        bl = l;
        bst = std::move(ts);
      }
    }
    TN_REQUIRE(found, TN_ERR_BUDGET, "memory budget cannot be met by slicing");
    sliced.push_back(bl);
    cur = std::move(bst);
  }
  return sliced;
}

}  // namespace tn

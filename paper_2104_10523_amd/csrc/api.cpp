// C ABI of the library (declared in include/tn.h).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <set>

#include "common.hpp"
#include "kernels.hpp"
#include "network.hpp"
#include "plan.hpp"

namespace tn {

static thread_local std::string g_last_error;
void set_last_error(const std::string& msg) { g_last_error = msg; }

namespace {

struct Workspace {
  void* ptr = nullptr;
  size_t bytes = 0;
};
std::mutex g_mu;
std::map<int, Workspace> g_ws;        // per device
std::map<int, float2*> g_one;         // per device: constant 1+0i

int current_device() {
  int d = 0;
  TN_HIP(hipGetDevice(&d));
  return d;
}

Workspace get_ws() {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_ws[current_device()];
}

float2* device_one() {
  const int d = current_device();
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_one.find(d);
  if (it != g_one.end()) return it->second;
  float2* p = nullptr;
  TN_HIP(hipMalloc(&p, 256));
  // 1 + 0i as complex64 at byte 0 and as complex128 at byte 16
  unsigned char host[32] = {};
  const float2 one = make_float2(1.f, 0.f);
  const double2 one64 = make_double2(1.0, 0.0);
  std::memcpy(host, &one, sizeof(one));
  std::memcpy(host + 16, &one64, sizeof(one64));
  TN_HIP(hipMemcpy(p, host, sizeof(host), hipMemcpyHostToDevice));
  g_one[d] = p;
  return p;
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace
}  // namespace tn

using namespace tn;

#include "handles.hpp"

namespace {

std::vector<char> read_open(const Network& net, const int8_t* mask) {
  std::vector<char> o(net.n_qubits, 0);
  if (mask)
    for (int q = 0; q < net.n_qubits; ++q) o[q] = mask[q] ? 1 : 0;
  return o;
}

void fill_cost(const PathStats& ps, const std::vector<int>& sliced, int algo, tn_path_cost* c) {
  std::memset(c, 0, sizeof(*c));
  c->flops_per_slice = ps.flops;
  c->total_flops = ps.total_flops;
  c->peak_elems = ps.peak;
  c->n_slices = ps.n_slices;
  c->n_steps = int(ps.steps.size());
  c->n_sliced = int(sliced.size());
  c->algo_used = algo;
}

tn_path* finish_path(const Network& net, const tn_path_opts* o,
                     std::vector<std::pair<int, int>> pairs, int algo, tn_path_cost* cost) {
  const auto open_q = read_open(net, o ? o->open_mask : nullptr);
  const PathProblem pr = make_problem(net, open_q);
  const double budget = o ? o->mem_budget_bytes : 0.0;
  std::vector<int> sliced = slice_path(pr, pairs, budget);
  const PathStats ps = path_stats(pr, pairs, sliced);
  auto* p = new tn_path();
  p->pairs = std::move(pairs);
  p->sliced = std::move(sliced);
  p->open_q = open_q;
  fill_cost(ps, p->sliced, algo, &p->cost);
  if (cost) *cost = p->cost;
  return p;
}

std::shared_ptr<AmpPlan> get_plan(tn_network* n, tn_path* p, int precision) {
  std::lock_guard<std::mutex> lk(p->mu);
  auto it = p->plans.find(precision);
  if (it != p->plans.end()) return it->second;
  auto plan = std::make_shared<AmpPlan>(compile_amplitudes(n->net, p->pairs, p->sliced, p->open_q, precision));
  p->plans[precision] = plan;
  return plan;
}

struct WsLayout {
  size_t ctl = 0, bits = 0, descs = 0, leaves = 0, work = 0, flag = 0, total = 0;
};

WsLayout ws_layout(const AmpPlan& P, int64_t n_bs) {
  WsLayout L;
  size_t o = 0;
  L.ctl = o; o += 256;
  L.flag = o; o += 256;
  L.bits = o; o += align256(size_t(n_bs) * size_t(P.n_qubits));
  L.descs = o; o += align256(P.leaves.size() * sizeof(LeafDesc));
  L.leaves = o; o += align256(size_t(P.leaf_elems) * (P.precision == TN_PREC_FP64 ? sizeof(double2) : sizeof(float2)));
  L.work = o; o += align256(size_t(P.work_elems) * sizeof(float2));
  L.total = o;
  return L;
}

float2* upload_leaves(tn_network* n) {
  const int d = current_device();
  std::lock_guard<std::mutex> lk(n->mu);
  auto it = n->dev_full.find(d);
  if (it != n->dev_full.end()) return it->second;
  std::vector<float2> host;
  for (const auto& t : n->net.tensors)
    for (const cd& v : t.data) host.push_back(make_float2(float(v.real()), float(v.imag())));
  if (host.empty()) host.push_back(make_float2(0.f, 0.f));
  float2* dptr = nullptr;
  TN_HIP(hipMalloc(&dptr, host.size() * sizeof(float2)));
  TN_HIP(hipMemcpy(dptr, host.data(), host.size() * sizeof(float2), hipMemcpyHostToDevice));
  n->dev_full[d] = dptr;
  return dptr;
}

double2* upload_leaves64(tn_network* n) {
  const int d = current_device();
  std::lock_guard<std::mutex> lk(n->mu);
  auto it = n->dev_full64.find(d);
  if (it != n->dev_full64.end()) return it->second;
  std::vector<double2> host;
  for (const auto& t : n->net.tensors)
    for (const cd& v : t.data) host.push_back(make_double2(v.real(), v.imag()));
  if (host.empty()) host.push_back(make_double2(0.0, 0.0));
  double2* dptr = nullptr;
  TN_HIP(hipMalloc(&dptr, host.size() * sizeof(double2)));
  TN_HIP(hipMemcpy(dptr, host.data(), host.size() * sizeof(double2), hipMemcpyHostToDevice));
  n->dev_full64[d] = dptr;
  return dptr;
}

// Expands user labels into one-bit labels (extent 2^e -> e bits, most
// significant first); label id * 64 + bit.
std::vector<int> bit_labels(const tn_tensor* T, const int32_t* modes, std::map<int32_t, int>& ids,
                            std::map<int32_t, int64_t>& ext) {
  TN_REQUIRE(T->rank >= 0 && T->rank <= 64, TN_ERR_ARG, "rank out of range");
  TN_REQUIRE(T->rank == 0 || (modes && T->extents), TN_ERR_ARG, "null modes or extents");
  TN_REQUIRE(T->dtype == TN_C64 || T->dtype == TN_C128, TN_ERR_ARG, "bad dtype");
  std::set<int32_t> seen;
  std::vector<int> out;
  for (int i = 0; i < T->rank; ++i) {
    const int32_t m = modes[i];
    TN_REQUIRE(seen.insert(m).second, TN_ERR_MODES, "repeated label in one tensor");
    const int64_t e = T->extents[i];
    TN_REQUIRE(e >= 1, TN_ERR_ARG, "extent < 1");
    auto it = ext.find(m);
    if (it != ext.end()) TN_REQUIRE(it->second == e, TN_ERR_EXTENT, "label extents differ");
    ext[m] = e;
    TN_REQUIRE((e & (e - 1)) == 0, TN_ERR_UNSUPPORTED, "extents must be powers of two");
    if (!ids.count(m)) {
      const int id = int(ids.size());
      ids[m] = id;
    }
    int bits = 0;
    while ((int64_t(1) << bits) < e) ++bits;
    for (int b = bits - 1; b >= 0; --b) out.push_back(ids[m] * 64 + b);
  }
  TN_REQUIRE(out.size() <= 62, TN_ERR_UNSUPPORTED, "tensor has more than 2^62 elements");
  return out;
}

}  // namespace

namespace tn {

PairPlan compile_contract_pair(const tn_tensor* A, const int32_t* modesA, const tn_tensor* B,
                               const int32_t* modesB, const tn_tensor* C, const int32_t* modesC,
                               int32_t precision) {
  TN_REQUIRE(A && B && C, TN_ERR_ARG, "null tensor");
  TN_REQUIRE(precision >= TN_PREC_FP32 && precision <= TN_PREC_FP64, TN_ERR_ARG, "bad precision");
  std::map<int32_t, int> ids;
  std::map<int32_t, int64_t> ext;
  TRef X, Y;
  X.buf = BUF_EXT_A;
  Y.buf = BUF_EXT_B;
  X.labels = bit_labels(A, modesA, ids, ext);
  Y.labels = bit_labels(B, modesB, ids, ext);
  std::map<int32_t, int64_t> ext_in = ext;
  std::map<int32_t, int> ids_in = ids;
  // output labels must come from the inputs, with the same extents
  for (int i = 0; i < C->rank; ++i)
    TN_REQUIRE(modesC && ids_in.count(modesC[i]), TN_ERR_MODES, "output label not in A or B");
  std::vector<int> want = bit_labels(C, modesC, ids, ext);
  TN_REQUIRE(ids.size() == ids_in.size(), TN_ERR_MODES, "output label not in A or B");
  for (auto& kv : ext_in) TN_REQUIRE(ext[kv.first] == kv.second, TN_ERR_EXTENT, "label extents differ");
  TN_REQUIRE(A->data && B->data && C->data, TN_ERR_ARG, "null data pointer");
  TN_REQUIRE(A->dtype == B->dtype && B->dtype == C->dtype, TN_ERR_ARG, "tensors of different dtypes");
  TN_REQUIRE((A->dtype == TN_C128) == (precision == TN_PREC_FP64), TN_ERR_ARG,
             "complex128 tensors go with TN_PREC_FP64 and only they do");
  Arena arena;
  PairPlan pp;
  std::vector<int64_t> scratch;
  compile_pair(X, Y, want, &want, BUF_EXT_C, 0, arena, precision, pp.ops, &scratch);
  pp.scratch_bytes = size_t(arena.high_water()) * sizeof(float2);
  return pp;
}

void run_contract_pair(const PairPlan& pp, const tn_tensor* A, const tn_tensor* B, tn_tensor* C, void* scratch,
                       float2* one, hipStream_t stream) {
  float2* bufs[6] = {nullptr, static_cast<float2*>(scratch), static_cast<float2*>(A->data),
                     static_cast<float2*>(B->data), static_cast<float2*>(C->data), one};
  run_ops(pp.ops, bufs, stream);
}

}  // namespace tn

extern "C" {

const char* tn_last_error(void) { return g_last_error.c_str(); }
const char* tn_version(void) { return "tn-mi355x 0.1 gfx950"; }

tn_status tn_build_network(const tn_circuit* c, tn_network** out) {
  return guarded([&] {
    TN_REQUIRE(c && out, TN_ERR_ARG, "null argument");
    auto n = std::make_unique<tn_network>();
    n->net = build_network(*c);
    *out = n.release();
  });
}

tn_status tn_network_destroy(tn_network* n) {
  return guarded([&] { delete n; });
}

tn_status tn_network_get_info(const tn_network* n, tn_network_info* info) {
  return guarded([&] {
    TN_REQUIRE(n && info, TN_ERR_ARG, "null argument");
    info->n_qubits = n->net.n_qubits;
    info->n_tensors = int32_t(n->net.tensors.size());
    info->n_labels = n->net.n_labels;
  });
}

tn_status tn_network_get_tensor(const tn_network* n, int32_t i, int32_t* rank, int32_t* labels,
                                double* data) {
  return guarded([&] {
    TN_REQUIRE(n && rank, TN_ERR_ARG, "null argument");
    TN_REQUIRE(i >= 0 && i < int(n->net.tensors.size()), TN_ERR_ARG, "tensor index out of range");
    const auto& t = n->net.tensors[i];
    *rank = int32_t(t.labels.size());
    if (labels)
      for (size_t k = 0; k < t.labels.size(); ++k) labels[k] = t.labels[k];
    if (data)
      for (size_t k = 0; k < t.data.size(); ++k) {
        data[2 * k] = t.data[k].real();
        data[2 * k + 1] = t.data[k].imag();
      }
  });
}

tn_status tn_network_output_labels(const tn_network* n, int32_t* labels) {
  return guarded([&] {
    TN_REQUIRE(n && labels, TN_ERR_ARG, "null argument");
    for (int q = 0; q < n->net.n_qubits; ++q) labels[q] = n->net.out_label[q];
  });
}

tn_status tn_find_path(const tn_network* n, const tn_path_opts* o, tn_path** out, tn_path_cost* cost) {
  return guarded([&] {
    TN_REQUIRE(n && out, TN_ERR_ARG, "null argument");
    const int algo = o ? o->algo : TN_PATH_GREEDY;
    TN_REQUIRE(algo == TN_PATH_GREEDY || algo == TN_PATH_RANDOM_GREEDY || algo == TN_PATH_LEARNED ||
                   algo == TN_PATH_PARTITION,
               TN_ERR_ARG, "unknown path algorithm");
    const auto open_q = read_open(n->net, o ? o->open_mask : nullptr);
    const PathProblem pr = make_problem(n->net, open_q);
    std::vector<std::pair<int, int>> pairs;
    if (algo == TN_PATH_GREEDY) {
      pairs = greedy_path(pr, nullptr, 1.0);
    } else if (algo == TN_PATH_RANDOM_GREEDY) {
      TN_REQUIRE(o->trials >= 0 && o->temperature > 0, TN_ERR_ARG, "bad random-greedy options");
      pairs = random_greedy_path(pr, o->seed, o->trials, o->temperature, o->mem_budget_bytes);
    } else if (algo == TN_PATH_PARTITION) {
      TN_REQUIRE(o->trials >= 0, TN_ERR_ARG, "bad partition options");
      TN_REQUIRE(o->rank == TN_RANK_FLOPS || o->rank == TN_RANK_TIME, TN_ERR_ARG, "bad rank");
      if (o->rank == TN_RANK_FLOPS) {
        pairs = partition_search(pr, o->seed, o->trials, o->mem_budget_bytes);
      } else {
        TN_REQUIRE(o->rank_precision >= TN_PREC_FP32 && o->rank_precision <= TN_PREC_FP64, TN_ERR_ARG,
                   "bad rank precision");
        auto cands = partition_candidates(pr, o->seed, o->trials, o->mem_budget_bytes, 16);
        // modelled seconds of all slices of each candidate (infinite when
        // the budget rejects it), candidates evaluated on host threads
        std::vector<double> tc(cands.size(), std::numeric_limits<double>::infinity());
        auto modelled = [&](const std::vector<std::pair<int, int>>& p) {
          const std::vector<int> sl = slice_path(pr, p, o->mem_budget_bytes);
          const PathStats ps = path_stats(pr, p, sl);
          return ps.n_slices * modelled_job_seconds(compile_amplitudes(n->net, p, sl, open_q, o->rank_precision));
        };
        run_parallel(int(cands.size()), [&](int c) {
          try {
            tc[c] = modelled(cands[c]);
          } catch (const Error& e) {
            if (e.code != TN_ERR_BUDGET) throw;
            return;
          }
          // the same tree reconfigured for modelled step time at its slice
          // sizes (then re-sliced), kept when the whole plan models faster
          auto alt = reconfigure_for_time(pr, cands[c], slice_path(pr, cands[c], o->mem_budget_bytes));
          if (alt == cands[c]) return;
          try {
            const double t2 = modelled(alt);
            if (t2 < tc[c]) {
              cands[c] = std::move(alt);
              tc[c] = t2;
            }
          } catch (const Error& e) {
            if (e.code != TN_ERR_BUDGET) throw;
          }
        });
        int best = -1;
        for (size_t c = 0; c < cands.size(); ++c)
          if (tc[c] < std::numeric_limits<double>::infinity() && (best < 0 || tc[c] < tc[best])) best = int(c);
        pairs = std::move(cands[best < 0 ? 0 : best]);
      }
    } else {
      TN_REQUIRE(o->model != nullptr, TN_ERR_STATE, "learned path needs a model");
      int used = TN_PATH_GREEDY;
      pairs = learned_path_with_fallback(o->model, pr, o->rescore_every, &used);
      *out = finish_path(n->net, o, std::move(pairs), used, cost);
      return;
    }
    *out = finish_path(n->net, o, std::move(pairs), algo, cost);
  });
}

tn_status tn_path_from_pairs(const tn_network* n, const tn_path_opts* o, const int32_t* pairs,
                             int32_t n_steps, tn_path** out, tn_path_cost* cost) {
  return guarded([&] {
    TN_REQUIRE(n && out && (pairs || n_steps == 0) && n_steps >= 0, TN_ERR_ARG, "null argument");
    std::vector<std::pair<int, int>> pv;
    for (int t = 0; t < n_steps; ++t) pv.push_back({pairs[2 * t], pairs[2 * t + 1]});
    *out = finish_path(n->net, o, std::move(pv), -1, cost);
  });
}

tn_status tn_path_get(const tn_path* p, int32_t* pairs, int32_t* sliced_labels) {
  return guarded([&] {
    TN_REQUIRE(p, TN_ERR_ARG, "null path");
    if (pairs)
      for (size_t t = 0; t < p->pairs.size(); ++t) {
        pairs[2 * t] = p->pairs[t].first;
        pairs[2 * t + 1] = p->pairs[t].second;
      }
    if (sliced_labels)
      for (size_t k = 0; k < p->sliced.size(); ++k) sliced_labels[k] = p->sliced[k];
  });
}

tn_status tn_path_destroy(tn_path* p) {
  return guarded([&] { delete p; });
}

tn_status tn_set_workspace(void* device_ptr, size_t bytes) {
  return guarded([&] {
    TN_REQUIRE(bytes == 0 || device_ptr != nullptr, TN_ERR_ARG, "null workspace");
    const int d = current_device();
    std::lock_guard<std::mutex> lk(g_mu);
    g_ws[d] = Workspace{bytes ? device_ptr : nullptr, bytes};
  });
}

tn_status tn_contract_pair(const tn_tensor* A, const int32_t* modesA, const tn_tensor* B,
                           const int32_t* modesB, tn_tensor* C, const int32_t* modesC,
                           int32_t precision, void* stream) {
  return guarded([&] {
    const PairPlan pp = compile_contract_pair(A, modesA, B, modesB, C, modesC, precision);
    const Workspace ws = get_ws();
    TN_REQUIRE(pp.scratch_bytes == 0 || (ws.ptr && ws.bytes >= pp.scratch_bytes), TN_ERR_WORKSPACE,
               "workspace too small: need " + std::to_string(pp.scratch_bytes) + " bytes");
    run_contract_pair(pp, A, B, C, ws.ptr, device_one(), static_cast<hipStream_t>(stream));
  });
}

tn_status tn_amplitudes_workspace(const tn_network* n, const tn_path* p, int64_t n_bs,
                                  int32_t precision, size_t* bytes) {
  return guarded([&] {
    TN_REQUIRE(n && p && bytes && n_bs >= 1, TN_ERR_ARG, "bad argument");
    TN_REQUIRE(precision >= TN_PREC_FP32 && precision <= TN_PREC_FP64, TN_ERR_ARG, "bad precision");
    auto plan = get_plan(const_cast<tn_network*>(n), const_cast<tn_path*>(p), precision);
    *bytes = ws_layout(*plan, n_bs).total;
  });
}

tn_status tn_amplitudes(const tn_network* n_, const tn_path* p_, const int8_t* bits, int64_t n_bs,
                        const tn_exec_opts* opts, void* out, tn_report* rep, void* stream) {
  return guarded([&] {
    auto* n = const_cast<tn_network*>(n_);
    auto* p = const_cast<tn_path*>(p_);
    TN_REQUIRE(n && p && bits && out && n_bs >= 1, TN_ERR_ARG, "bad argument");
    tn_exec_opts o{TN_PREC_FP32, 0, 0, -1, 0, 0, nullptr};
    if (opts) o = *opts;
    TN_REQUIRE(o.precision >= TN_PREC_FP32 && o.precision <= TN_PREC_FP64, TN_ERR_ARG, "bad precision");
    const int nq = n->net.n_qubits;
    TN_REQUIRE(int(p->open_q.size()) == nq, TN_ERR_ARG, "path belongs to another network");
    for (int64_t b = 0; b < n_bs; ++b)
      for (int q = 0; q < nq; ++q) {
        const int v = bits[b * nq + q];
        TN_REQUIRE(v == 0 || v == 1 || v == -1, TN_ERR_BITS, "bit values must be 0, 1 or -1");
        TN_REQUIRE((v == -1) == (p->open_q[q] != 0), TN_ERR_BITS,
                   "bit-string open set differs from the path's open set");
      }
    const double ns = p->cost.n_slices;
    int64_t sbeg = o.slice_begin, scount = o.slice_count;
    TN_REQUIRE(sbeg >= 0 && double(sbeg) < ns, TN_ERR_ARG, "slice_begin out of range");
    if (scount < 0) scount = int64_t(ns) - sbeg;
    TN_REQUIRE(scount >= 1 && double(sbeg + scount) <= ns, TN_ERR_ARG, "slice range out of range");
    auto plan = get_plan(n, p, o.precision);
    const AmpPlan& P = *plan;
    const WsLayout L = ws_layout(P, n_bs);
    const Workspace ws = get_ws();
    TN_REQUIRE(ws.ptr && ws.bytes >= L.total, TN_ERR_WORKSPACE,
               "workspace too small: need " + std::to_string(L.total) + " bytes");
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* base = static_cast<char*>(ws.ptr);
    const bool f64 = P.precision == TN_PREC_FP64;
    float2* full = f64 ? nullptr : upload_leaves(n);
    double2* full64 = f64 ? upload_leaves64(n) : nullptr;
    int64_t ctl[3] = {0, sbeg, scount};
    TN_HIP(hipMemcpyAsync(base + L.ctl, ctl, sizeof(ctl), hipMemcpyHostToDevice, s));
    TN_HIP(hipMemsetAsync(base + L.flag, 0, 4, s));
    TN_HIP(hipMemcpyAsync(base + L.bits, bits, size_t(n_bs) * nq, hipMemcpyHostToDevice, s));
    if (!P.leaves.empty())
      TN_HIP(hipMemcpyAsync(base + L.descs, P.leaves.data(), P.leaves.size() * sizeof(LeafDesc),
                            hipMemcpyHostToDevice, s));
    TN_HIP(hipStreamSynchronize(s));  // host staging buffers are released below
    int64_t* dctl = reinterpret_cast<int64_t*>(base + L.ctl);
    float2* bufs[6] = {reinterpret_cast<float2*>(base + L.leaves), reinterpret_cast<float2*>(base + L.work),
                       nullptr, nullptr, nullptr, device_one()};
    const int64_t jobs = n_bs * scount;
    auto one_job = [&]() {
      const LeafDesc* descs = reinterpret_cast<const LeafDesc*>(base + L.descs);
      const int8_t* dbits = reinterpret_cast<const int8_t*>(base + L.bits);
      if (f64)
        launch_gather_leaves(full64, reinterpret_cast<double2*>(bufs[BUF_LEAF]), descs, int(P.leaves.size()),
                             P.max_leaf_bits, dbits, nq, dctl, s);
      else
        launch_gather_leaves(full, bufs[BUF_LEAF], descs, int(P.leaves.size()), P.max_leaf_bits, dbits, nq,
                             dctl, s);
      run_ops(P.ops, bufs, s);
      if (f64)
        launch_accumulate(reinterpret_cast<const double2*>(bufs[P.final_buf] + P.final_off),
                          static_cast<double2*>(out), P.final_bits, P.final_pos, dctl, o.accumulate, s);
      else
        launch_accumulate(bufs[P.final_buf] + P.final_off, static_cast<double2*>(out), P.final_bits,
                          P.final_pos, dctl, o.accumulate, s);
    };
    const bool profile = o.op_seconds != nullptr;
    if (profile) {
      o.sync = 1;
      o.use_graph = 0;
      for (size_t k = 0; k < P.ops.size(); ++k) o.op_seconds[k] = 0.0;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (o.sync) {
      TN_HIP(hipEventCreate(&e0));
      TN_HIP(hipEventCreate(&e1));
      TN_HIP(hipEventRecord(e0, s));
    }
    if (o.use_graph) {
      // capture on a library-owned stream (the legacy default stream cannot
      // be captured), ordered after the caller's stream by an event
      hipStream_t cs = nullptr;
      hipEvent_t dep = nullptr;
      hipGraph_t g = nullptr;
      hipGraphExec_t ge = nullptr;
      TN_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
      auto cleanup = [&]() {
        if (ge) (void)hipGraphExecDestroy(ge);
        if (g) (void)hipGraphDestroy(g);
        if (dep) (void)hipEventDestroy(dep);
        (void)hipStreamDestroy(cs);
      };
      try {
        TN_HIP(hipEventCreateWithFlags(&dep, hipEventDisableTiming));
        TN_HIP(hipEventRecord(dep, s));
        TN_HIP(hipStreamWaitEvent(cs, dep, 0));
        TN_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        hipStream_t keep = s;
        s = cs;
        try {
          launch_advance_job(dctl, s);
          one_job();
        } catch (...) {
          s = keep;
          hipGraph_t dummy = nullptr;
          (void)hipStreamEndCapture(cs, &dummy);
          if (dummy) (void)hipGraphDestroy(dummy);
          throw;
        }
        s = keep;
        TN_HIP(hipStreamEndCapture(cs, &g));
        TN_HIP(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
        launch_set_job(dctl, -1, s);
        for (int64_t j = 0; j < jobs; ++j) TN_HIP(hipGraphLaunch(ge, s));
        TN_HIP(hipStreamSynchronize(s));
      } catch (...) {
        cleanup();
        throw;
      }
      cleanup();
    } else if (profile) {
      std::vector<hipEvent_t> ev(P.ops.size() + 1);
      for (auto& e : ev) TN_HIP(hipEventCreate(&e));
      for (int64_t j = 0; j < jobs; ++j) {
        launch_set_job(dctl, j, s);
        launch_gather_leaves(full, bufs[BUF_LEAF], reinterpret_cast<const LeafDesc*>(base + L.descs),
                             int(P.leaves.size()), P.max_leaf_bits,
                             reinterpret_cast<const int8_t*>(base + L.bits), nq, dctl, s);
        TN_HIP(hipEventRecord(ev[0], s));
        for (size_t k = 0; k < P.ops.size(); ++k) {
          run_ops(std::vector<PlanOp>(P.ops.begin() + k, P.ops.begin() + k + 1), bufs, s);
          TN_HIP(hipEventRecord(ev[k + 1], s));
        }
        launch_accumulate(bufs[P.final_buf] + P.final_off, static_cast<double2*>(out), P.final_bits,
                          P.final_pos, dctl, o.accumulate, s);
        TN_HIP(hipEventSynchronize(ev.back()));
        for (size_t k = 0; k < P.ops.size(); ++k) {
          float t = 0.f;
          TN_HIP(hipEventElapsedTime(&t, ev[k], ev[k + 1]));
          o.op_seconds[k] += t * 1e-3;
        }
      }
      for (auto& e : ev) (void)hipEventDestroy(e);
    } else {
      for (int64_t j = 0; j < jobs; ++j) {
        launch_set_job(dctl, j, s);
        one_job();
      }
    }
    const int64_t n_out = n_bs * (int64_t(1) << P.n_open);
    launch_nonfinite(static_cast<const double2*>(out), n_out, reinterpret_cast<int*>(base + L.flag), s);
    float ms = 0.f;
    int flag = 0;
    if (o.sync) {
      TN_HIP(hipEventRecord(e1, s));
      TN_HIP(hipEventSynchronize(e1));
      TN_HIP(hipEventElapsedTime(&ms, e0, e1));
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      TN_HIP(hipMemcpy(&flag, base + L.flag, 4, hipMemcpyDeviceToHost));
    }
    if (rep) {
      std::memset(rep, 0, sizeof(*rep));
      rep->seconds = ms * 1e-3;
      rep->flops = P.flops_per_job * double(jobs);
      rep->bytes = P.bytes_per_job * double(jobs);
      rep->slices_run = double(jobs);
      rep->kernels = double(P.ops.size() + 2);
      rep->precision = o.precision;
      rep->nonfinite = flag;
      rep->err_bound = P.err_bound;
    }
  });
}

tn_status tn_amplitudes_autotune(const tn_network* n_, const tn_path* p_, int32_t precision, int32_t reps,
                                 void* stream) {
  return guarded([&] {
    auto* n = const_cast<tn_network*>(n_);
    auto* p = const_cast<tn_path*>(p_);
    TN_REQUIRE(n && p && reps >= 1, TN_ERR_ARG, "bad argument");
    TN_REQUIRE(precision >= TN_PREC_FP32 && precision <= TN_PREC_FP64, TN_ERR_ARG, "bad precision");
    auto plan = get_plan(n, p, precision);
    const WsLayout L = ws_layout(*plan, 1);
    const Workspace ws = get_ws();
    TN_REQUIRE(ws.ptr && ws.bytes >= L.total, TN_ERR_WORKSPACE,
               "workspace too small: need " + std::to_string(L.total) + " bytes");
    char* base = static_cast<char*>(ws.ptr);
    float2* bufs[6] = {reinterpret_cast<float2*>(base + L.leaves), reinterpret_cast<float2*>(base + L.work),
                       nullptr, nullptr, nullptr, device_one()};
    std::lock_guard<std::mutex> lk(p->mu);
    autotune_ops(plan->ops, bufs, reps, static_cast<hipStream_t>(stream));
  });
}

tn_status tn_amplitudes_plan_info(const tn_network* n, const tn_path* p, int32_t precision,
                                  tn_plan_info* info) {
  return guarded([&] {
    TN_REQUIRE(n && p && info, TN_ERR_ARG, "null argument");
    TN_REQUIRE(precision >= TN_PREC_FP32 && precision <= TN_PREC_FP64, TN_ERR_ARG, "bad precision");
    auto plan = get_plan(const_cast<tn_network*>(n), const_cast<tn_path*>(p), precision);
    std::memset(info, 0, sizeof(*info));
    info->n_ops = int32_t(plan->ops.size());
    for (const PlanOp& op : plan->ops) {
      info->n_by_kind[op.kind]++;
      info->flops_by_kind[op.kind] += op.flops;
      info->bytes_by_kind[op.kind] += op.bytes;
    }
    info->workspace_bytes = double(ws_layout(*plan, 1).total);
    info->err_bound = plan->err_bound;
  });
}

tn_status tn_amplitudes_plan_ops(const tn_network* n, const tn_path* p, int32_t precision,
                                 int32_t* kind, double* flops, double* bytes, int64_t* shape) {
  return guarded([&] {
    TN_REQUIRE(n && p, TN_ERR_ARG, "null argument");
    TN_REQUIRE(precision >= TN_PREC_FP32 && precision <= TN_PREC_FP64, TN_ERR_ARG, "bad precision");
    auto plan = get_plan(const_cast<tn_network*>(n), const_cast<tn_path*>(p), precision);
    for (size_t k = 0; k < plan->ops.size(); ++k) {
      const PlanOp& op = plan->ops[k];
      if (kind) kind[k] = op.kind;
      if (flops) flops[k] = op.flops;
      if (bytes) bytes[k] = op.bytes;
      if (shape) {
        int64_t* r = shape + 8 * k;
        r[0] = r[1] = r[2] = r[3] = 1;
        r[4] = -1;
        r[5] = 0;
        r[6] = op.kind == OP_GEMM ? 0 : 1;
        r[7] = 0;
        if (op.kind == OP_GEMM) {
          r[0] = op.gm.M; r[1] = op.gm.N; r[2] = op.gm.K; r[3] = op.gm.batch;
          r[4] = op.f64 ? -1 : gemm_tile_of(op.gm);
          r[5] = op.gm.packed;
          r[6] = op.f64 ? 1 : gemm_dispatches(op.gm);
        } else if (op.kind == OP_APPLY) {
          r[0] = int64_t(1) << (op.ap.a_bits - op.ap.nk);
          r[1] = int64_t(1) << op.ap.nn;
          r[2] = int64_t(1) << op.ap.nk;
          r[3] = apply_variant(op.ap, nullptr, nullptr);
        } else if (op.kind == OP_DOT) {
          r[0] = op.dot_m; r[1] = op.dot_n; r[2] = op.dot_k; r[3] = op.dot_batch;
          r[5] = op.skinny;
        } else {
          r[0] = int64_t(1) << op.pm.nb;
          r[1] = op.pm.np;
          r[2] = op.pm.f16;
          r[3] = permute_variant(op.pm);
        }
      }
    }
  });
}

// MPS and trajectories are defined in their own translation units.

}  // extern "C"

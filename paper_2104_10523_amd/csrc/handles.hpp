// Opaque handle types of the C ABI, shared by the translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "network.hpp"
#include "plan.hpp"

struct tn_network {
  tn::Network net;
  std::mutex mu;
  std::map<int, float2*> dev_full;     // per device: all leaves, complex64
  std::map<int, double2*> dev_full64;  // per device: all leaves, complex128 (FP64 plans)
  ~tn_network() {
    auto release = [](int dev, void* p) {
      int cur = 0;
      if (hipGetDevice(&cur) == hipSuccess && hipSetDevice(dev) == hipSuccess) {
        (void)hipFree(p);
        (void)hipSetDevice(cur);
      }
    };
    for (auto& kv : dev_full) release(kv.first, kv.second);
    for (auto& kv : dev_full64) release(kv.first, kv.second);
  }
};

struct tn_path {
  std::vector<std::pair<int, int>> pairs;
  std::vector<int> sliced;
  std::vector<char> open_q;
  tn_path_cost cost;
  std::mutex mu;
  std::map<int, std::shared_ptr<tn::AmpPlan>> plans;  // by precision
};


namespace tn {
// Learned path with greedy fallback (defined with the scorer).
// rescore_every: merges taken per scoring (<= 1: one).
std::vector<std::pair<int, int>> learned_path_with_fallback(const tn_model* m, const PathProblem& pr,
                                                            int rescore_every, int* algo_used);
}  // namespace tn

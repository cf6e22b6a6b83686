// Allocation-free variant of tn_contract_pair for callers that cannot
// allocate device memory (code under stream capture, serving loops): the
// contraction's scratch (permuted operands, split-precision planes and
// their scale slots, split-K partials) lives in a file-scope device array
// of fixed size instead of the caller's workspace.
#include <map>
#include <mutex>

#include "common.hpp"
#include "plan.hpp"

namespace tn {
namespace {
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
}  // namespace
}  // namespace tn

// One copy per device, held until the process ends.  Host code must never
// pass these names to a kernel or a copy: they are host-side stand-ins; the
// device addresses come from hipGetSymbolAddress below.
static __device__ __align__(256) unsigned char scratch[tn::kNoAllocScratchBytes];
// 1 + 0i as complex64 at byte 0 and as complex128 at byte 16 (IEEE bits,
// little-endian words)
static __device__ __align__(256) unsigned int scratch_one[8] = {0x3f800000u, 0u, 0u, 0u, 0u, 0x3ff00000u, 0u, 0u};

namespace tn {
namespace {

struct ScratchPtrs {
  void* scratch = nullptr;
  float2* one = nullptr;
};
std::mutex g_scratch_mu;
std::map<int, ScratchPtrs> g_scratch;   // per device

// Device addresses of this device's copies, looked up once per device (with
// that device current).
ScratchPtrs scratch_ptrs() {
  int d = 0;
  TN_HIP(hipGetDevice(&d));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch.find(d);
  if (it != g_scratch.end()) return it->second;
  ScratchPtrs p;
  void* one = nullptr;
  TN_HIP(hipGetSymbolAddress(&p.scratch, HIP_SYMBOL(scratch)));
  TN_HIP(hipGetSymbolAddress(&one, HIP_SYMBOL(scratch_one)));
  TN_REQUIRE(p.scratch != nullptr && one != nullptr, TN_ERR_DEVICE, "no device address for the scratch array");
  p.one = static_cast<float2*>(one);
  g_scratch[d] = p;
  return p;
}

}  // namespace
}  // namespace tn

using namespace tn;

extern "C" {

tn_status tn_contract_pair_noalloc(const tn_tensor* A, const int32_t* modesA, const tn_tensor* B,
                                   const int32_t* modesB, tn_tensor* C, const int32_t* modesC,
                                   int32_t precision, void* stream) {
  return guarded([&] {
    const PairPlan pp = compile_contract_pair(A, modesA, B, modesB, C, modesC, precision);
    TN_REQUIRE(pp.scratch_bytes <= kNoAllocScratchBytes, TN_ERR_WORKSPACE,
               "tn_contract_pair_noalloc: this contraction needs " + std::to_string(pp.scratch_bytes) +
                   " bytes of scratch, above the fixed " + std::to_string(kNoAllocScratchBytes) +
                   " (use tn_contract_pair with a workspace)");
    const ScratchPtrs sp = scratch_ptrs();
    run_contract_pair(pp, A, B, C, sp.scratch, sp.one, static_cast<hipStream_t>(stream));
  });
}

}  // extern "C"

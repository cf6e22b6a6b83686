// Plan compiler and executor: SSA path -> kernel sequence for one job
// (one bit-string x one slice), replayed over all jobs.
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <vector>

#include "kernels.hpp"
#include "network.hpp"

namespace tn {

enum Buf : int { BUF_LEAF = 0, BUF_WORK = 1, BUF_EXT_A = 2, BUF_EXT_B = 3, BUF_EXT_C = 4, BUF_ONE = 5 };

struct TRef {
  int buf = BUF_WORK;
  int64_t off = 0;            // element offset in the buffer
  std::vector<int> labels;    // layout, outermost first; every label is one bit
  int64_t smax = -1;          // split-FP16 planes: BUF_WORK offset of the max slot
  // result of a split-precision GEMM or of an apply: a max slot reserved
  // with it (released with it) and the index of that op, so that an fp16
  // packing of this tensor can take its max from the op instead of a pass
  // of its own
  int64_t cslot = -1;
  int producer = -1;
};

enum OpKind : int { OP_APPLY = 0, OP_PERMUTE = 1, OP_GEMM = 2, OP_DOT = 3 };

struct PlanOp {
  OpKind kind;
  int a_buf = 0, b_buf = 0, c_buf = 0;
  int64_t a_off = 0, b_off = 0, c_off = 0;
  int64_t work_off = -1;      // split-K / dot scratch (elements of float2)
  int64_t work_elems = 0;     // size of that scratch
  int64_t smax = -1;          // PERMUTE to fp16 planes: its max slot (BUF_WORK offset)
  int64_t smax_a = -1, smax_b = -1;   // GEMM on fp16 planes: the operands' slots
  int64_t cmax = -1;          // GEMM / APPLY: slot for the largest |re|, |im| of its result
  ApplySmallDesc ap;
  PermuteDesc pm;
  GemmDesc gm;
  int64_t dot_k = 0, dot_batch = 0;
  int64_t dot_m = 1, dot_n = 1;   // DOT over all (m, n) row pairs of [b][m][k] x [b][n][k]
  int f64 = 0;                     // complex128 operands (TN_PREC_FP64 plans)
  int skinny = 0;                  // DOT as the skinny long-K GEMM (batch 1), layouts below
  int dot_ta = 0, dot_tb = 1;      // skinny: transA / transB as for GEMMs
  double flops = 0, bytes = 0;
};

// Arena allocator over element offsets (first fit, 256-byte aligned).
class Arena {
 public:
  int64_t alloc(int64_t elems);
  void release(int64_t off);
  int64_t high_water() const { return high_; }

 private:
  std::vector<std::pair<int64_t, int64_t>> used_;  // (off, len), sorted
  int64_t high_ = 0;
};

// Emits the ops of one pairwise contraction.  X and Y are the operands,
// `keep` the labels of the result (any order); if `want` is non-empty the
// result must land in that layout at (want_buf, want_off).  Returns the
// result reference.  Scratch and the result come from `arena` (unless
// `want` is given); precision applies to MFMA GEMMs.
TRef compile_pair(const TRef& X, const TRef& Y, const std::vector<int>& keep,
                  const std::vector<int>* want, int want_buf, int64_t want_off, Arena& arena,
                  int precision, std::vector<PlanOp>& ops, std::vector<int64_t>* scratch);

void run_ops(const std::vector<PlanOp>& ops, float2* const bufs[6], hipStream_t s);

// Autotune cache: fastest tile id per GEMM shape and fastest kernel per
// apply descriptor (process-wide; -1 when not tuned).
int tuned_apply(const ApplySmallDesc& d);
int tuned_tile(const GemmDesc& g);
void remember_tile(const GemmDesc& g, int tile);
// Times every candidate tile of every GEMM op, and every candidate kernel
// of every apply op, on the given buffers and stores the fastest in the op
// (and the cache).  Synchronises `s`.
void autotune_ops(std::vector<PlanOp>& ops, float2* const bufs[6], int reps, hipStream_t s);

struct AmpPlan {
  int n_qubits = 0;
  int n_open = 0;
  std::vector<int> open_qubits;
  std::vector<int> sliced;        // labels, slot 0 = most significant slice bit
  double n_slices = 1;
  std::vector<LeafDesc> leaves;
  int max_leaf_bits = 0;
  int64_t leaf_elems = 0;
  int64_t work_elems = 0;
  std::vector<PlanOp> ops;
  int final_buf = BUF_LEAF;
  int64_t final_off = 0;
  int final_bits = 0;
  int8_t final_pos[kMaxBits];
  double flops_per_job = 0, bytes_per_job = 0;
  int precision = 0;
  double err_bound = 0;
  int gemm_ops = 0;
};

// One pairwise contraction of caller-owned tensors (tn_contract_pair):
// its kernel sequence and the scratch bytes that sequence needs.
struct PairPlan {
  std::vector<PlanOp> ops;
  size_t scratch_bytes = 0;
};
// Validates labels, extents and dtypes (TN_ERR_MODES / _EXTENT / _ARG /
// _UNSUPPORTED) and compiles the contraction; host only.
PairPlan compile_contract_pair(const tn_tensor* A, const int32_t* modesA, const tn_tensor* B,
                               const int32_t* modesB, const tn_tensor* C, const int32_t* modesC,
                               int32_t precision);
// Launches the compiled sequence on `stream`; `scratch` holds at least
// scratch_bytes (256-byte aligned), `one` a device complex 1 + 0i.
void run_contract_pair(const PairPlan& pp, const tn_tensor* A, const tn_tensor* B, tn_tensor* C, void* scratch,
                       float2* one, hipStream_t stream);

struct PathData;  // defined in api
AmpPlan compile_amplitudes(const Network& net, const std::vector<std::pair<int, int>>& path,
                           const std::vector<int>& sliced, const std::vector<char>& open_q,
                           int precision);

// Modelled seconds of one job of the plan: the sum over its kernels of
// max(flops / F, bytes / B) plus a launch latency, F = 350e12 for
// split-precision GEMMs and 120e12 otherwise, B = 4.0e12 B/s.
double modelled_job_seconds(const AmpPlan& P);

}  // namespace tn

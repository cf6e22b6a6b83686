// Launch interface of the gfx950 kernels.  Every tensor is complex64
// (float2), row-major, with power-of-two extents viewed as bits: bit 0 is the
// fastest-varying index bit.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace tn {

constexpr int kMaxBits = 64;

// Bit permutation out[o] = in[gather(o)]: output bit j takes input bit src[j];
// src[j] == -1 broadcasts (stride 0).  `nb` output bits; `nb_in` input bits.
// np = 2 or 3 additionally splits every entry into np bfloat16 parts and
// writes np planes of packed (re | im << 16) words, plane p at out + p * 2^nb.
// f16 = 1 (np = 2): the parts are fp16 parts of the entry times 2^s, with s
// set from the largest |re|, |im| of the input, whose float bits the call
// first writes to *smax (a 4-byte device slot; null otherwise).
struct PermuteDesc {
  int nb = 0;
  int nb_in = 0;
  int np = 0;
  int f16 = 0;
  int maxabs = 0;          // 1: only the max-abs pre-pass of an fp16 operand (into smax)
  int8_t src[kMaxBits];
};
void launch_permute(const float2* in, void* out, const PermuteDesc& d, uint32_t* smax, hipStream_t s);
// Which kernel launch_permute runs on 16-byte aligned buffers: 0 device
// copy, 1 permute_simple_kernel, 2 permute_tiled_kernel (6..11 bits),
// 3 maxabs_kernel (pre-pass), 4 permute_pipe_kernel (>= 12 bits).
int permute_variant(const PermuteDesc& d);

// C[m * 2^nn + n] = sum_k A[expand(m) + kscat(k)] * B[bscat(k, n)]
//   A: `a_bits` bits; K bits of A at positions kpos (ascending), others are M.
//   B: small (<= 2^12 entries); its K bits at bk[] and N bits at bn[] (bit
//      positions in B's index; -1 = stride 0, i.e. B broadcast along a bit);
//   A's "dangling" bits (summed out) are K bits with bk = -1.
// Row-major output [M bits of A in A's order][N bits in bn order].
struct ApplySmallDesc {
  int a_bits = 0;
  int nk = 0;              // number of K bits (<= 6)
  int nn = 0;              // number of N bits (<= 4; 5 or 6 on the matrix cores only)
  int nb_b = 0;            // bits of B
  int8_t kpos[8];          // in A, ascending
  int8_t bk[8];            // K bit i of B (bit i of k <-> kpos[i])
  int8_t bn[8];            // N bit i of B
  int8_t b_extra[12];      // B bits summed out (dangling in B), -1 padded
  int n_b_extra = 0;
  int variant = -1;        // kernel (see apply_variant); -1: the default rule
};
// cmax (optional): a 4-byte device slot that receives the largest |re|, |im|
// of C as float bits (for the fp16 packing of C by a later GEMM), computed
// as the matrix-core apply stores C or else by a pass over C.
void launch_apply_small(const float2* A, const float2* B, float2* C, const ApplySmallDesc& d,
                        hipStream_t s, uint32_t* cmax = nullptr);
// Whether launch_apply_small runs apply_tile_kernel (A and C may be NULL:
// then alignment is assumed, as for the plan's buffers).
bool apply_tiled_ok(const ApplySmallDesc& d, const void* A, const void* C);
// Kernel launch_apply_small picks: 0 one thread per row, 1 LDS-tiled, 2 matrix cores (NN = 16, 32
// or 64; at least 64 rows; the only kernel for nn = 5, 6).
// d.variant = 0 or 2 asks for that kernel where it applies (the autotuner's
// choice); -1 takes the default: 1 where it applies, else 2 where it applies, else 0.
int apply_variant(const ApplySmallDesc& d, const void* A, const void* C);
// Kernels the autotuner may time for an apply (at least one).
std::vector<int> apply_variant_candidates(const ApplySmallDesc& d);

// Complex GEMM C[b][m][n] = sum_k A[b](m,k) * B[b](k,n), contiguous operands.
// transA = 0: A[b][m][k]; 1: A[b][k][m].  transB = 0: B[b][k][n]; 1: B[b][n][k].
// packed = 1: A and B are bf16 planes from launch_permute (np = 2 for
// BF16X3, 3 for BF16X6; fp16 planes for F16X3, whose operand max slots
// smax_a / smax_b give the scales to undo) in the layouts [b][M][K] and
// [b][N][K] (k fastest); plane_a / plane_b are the plane strides in words;
// K must be a multiple of 4.
struct GemmDesc {
  int64_t M = 1, N = 1, K = 1, batch = 1;
  int transA = 0, transB = 0;
  int precision = 0;       // TN_PREC_FP32 / BF16X3 / BF16X6 / F16X3
  int packed = 0;
  int64_t plane_a = 0, plane_b = 0;
  int tile = -1;           // block tile id (-1: shape heuristic)
  int order = -1;          // packed block order: 0 grouped, 1 XCD regions, 2 row-major (-1: heuristic)
};
// Workspace needed for split-K partials (bytes); 0 when no split is used.
size_t gemm_workspace_bytes(const GemmDesc& g);
// Tile ids valid for this GEMM (the autotuner's candidates), and the id a
// launch uses (the heuristic when g.tile < 0).
std::vector<int> gemm_tile_candidates(const GemmDesc& g);
int gemm_tile_of(const GemmDesc& g);
// Launches of the GEMM kernel itself one launch_gemm makes (K chunks of the
// accumulator chains; a split-K reduction is not counted).
int64_t gemm_dispatches(const GemmDesc& g);
// cmax (optional): a 4-byte device slot that receives the largest |re|, |im|
// of C as float bits (for the fp16 packing of C by a later GEMM), computed in
// the direct-to-LDS kernel's final flush or else by a pass over C.
void launch_gemm(const float2* A, const float2* B, float2* C, const GemmDesc& g, void* work,
                 const uint32_t* smax_a, const uint32_t* smax_b, hipStream_t s, uint32_t* cmax = nullptr);

// Gather every leaf of one job into the leaf arena: fixed labels take their
// value from the job's bit-string (kind 0) or slice index (kind 1).
struct LeafFixed {
  int8_t pos;      // bit position in the full (unprojected) leaf
  int8_t kind;     // 0: bit-string entry, 1: slice bit
  int16_t which;   // qubit index, or slice bit number (0 = LSB of slice id)
};
struct LeafDesc {
  int64_t src_off;
  int64_t dst_off;
  int32_t out_bits;
  int32_t n_fixed;
  int8_t in_pos[8];          // full-leaf bit position of output bit j
  LeafFixed fixed[8];
};
// ctl: device int64 [0] = job index, [1] = slice_begin, [2] = slice_count.
void launch_gather_leaves(const float2* full, float2* arena, const LeafDesc* descs, int n_leaves,
                          int max_out, const int8_t* bits, int n_qubits, const int64_t* ctl,
                          hipStream_t s);
void launch_gather_leaves(const double2* full, double2* arena, const LeafDesc* descs, int n_leaves,
                          int max_out, const int8_t* bits, int n_qubits, const int64_t* ctl,
                          hipStream_t s);
void launch_set_job(int64_t* ctl, int64_t job, hipStream_t s);
void launch_advance_job(int64_t* ctl, hipStream_t s);

// out[b][i] (complex128) (+)= R[gather(i)]; b = job / slice_count.
void launch_accumulate(const float2* R, double2* out, int nbits, const int8_t* pos_of_bit,
                       const int64_t* ctl, int accumulate_first, hipStream_t s);
void launch_accumulate(const double2* R, double2* out, int nbits, const int8_t* pos_of_bit,
                       const int64_t* ctl, int accumulate_first, hipStream_t s);

// Dot products (M = N = 1) with split-K; result written as complex64.
size_t dot_workspace_bytes(int64_t K, int64_t batch);
// Long-K GEMM with few outputs (M, N powers of two <= 16, 1 < M N <= 64,
// batch 1): A and B read once, FP32 per-thread sums, FP64 block sums.
// transA = 0: A[m][k], 1: A[k][m]; transB = 0: B[k][n], 1: B[n][k].
bool skinny_supported(int64_t m, int64_t n);
size_t skinny_workspace_bytes(int64_t K, int64_t m, int64_t n);
void launch_skinny(const float2* A, const float2* B, float2* C, int64_t K, int64_t m, int64_t n, int transA,
                   int transB, void* work, hipStream_t s);
// C[b][m][n] = sum_k A[b][m][k] B[b][n][k] (complex, FP64 accumulation);
// m = n = 1 is the plain batched dot.
void launch_dot(const float2* A, const float2* B, float2* C, int64_t K, int64_t batch, int64_t m,
                int64_t n, void* work, hipStream_t s);

// Sets *flag to 1 if any entry of x is non-finite.
void launch_nonfinite(const double2* x, int64_t n, int* flag, hipStream_t s);

// Complex128 (validation precision TN_PREC_FP64) counterparts, same
// addressing as the complex64 launches (kernels64.hip).
void launch_apply64(const double2* A, const double2* B, double2* C, const ApplySmallDesc& d, hipStream_t s);
void launch_permute64(const double2* in, double2* out, const PermuteDesc& d, hipStream_t s);
// work: split-K partials (gemm64_workspace_bytes(g) bytes); NULL = no split.
size_t gemm64_workspace_bytes(const GemmDesc& g);
void launch_gemm64(const double2* A, const double2* B, double2* C, const GemmDesc& g, void* work, hipStream_t s);
size_t dot64_workspace_bytes(int64_t K, int64_t outs);
void launch_dot64(const double2* A, const double2* B, double2* C, int64_t K, int64_t batch, int64_t m, int64_t n,
                  int transA, int transB, void* work, hipStream_t s);

}  // namespace tn

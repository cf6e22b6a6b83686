/*
 * tn.h -- C ABI of the MI355X tensor-network circuit simulator.
 *
 * The library contracts the complex tensor network that a quantum circuit
 * defines (gate tensors, Kraus-channel tensors, MPS site tensors) along a
 * precomputed pairwise path over independent index slices, on one gfx950
 * GPU.  Everything that crosses this boundary is a plain pointer or size.
 *
 * Conventions shared by every call
 *   - Status: every call returns tn_status; TN_OK (0) on success, a negative
 *     code otherwise.  tn_last_error() returns a thread-local message for the
 *     last failing call on the calling thread.  No C++ exception crosses the
 *     ABI.  Errors of asynchronous device work surface at the next call that
 *     synchronises, as TN_ERR_DEVICE.
 *   - Complex numbers: interleaved (re, im).  complex64 = two floats,
 *     complex128 = two doubles.
 *   - Bit order: qubit 0 is the most significant bit of a flat amplitude
 *     index.  Two-qubit matrices act on |a b> where a is the op's first qubit
 *     (the more significant bit); row = output, column = input.
 *   - Streams: `stream` is a hipStream_t passed as void* (NULL = the legacy
 *     default stream).  Device work is enqueued on it; calls do not
 *     synchronise the stream unless stated.
 *   - Ownership: handles (tn_network, tn_path, tn_mps, tn_model) are created
 *     and destroyed by the library.  Device buffers passed in are owned by the
 *     caller and are never freed by the library.
 */
#ifndef TN_H_
#define TN_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tn_status;

enum {
  TN_OK = 0,
  TN_ERR_ARG = -1,         /* null pointer, negative size, bad enum value     */
  TN_ERR_MODES = -2,       /* repeated label in one tensor, label not found   */
  TN_ERR_EXTENT = -3,      /* the same label has different extents            */
  TN_ERR_BITS = -4,        /* bit-string length/values/open set inconsistent  */
  TN_ERR_BUDGET = -5,      /* no slicing meets the memory budget              */
  TN_ERR_WORKSPACE = -6,   /* workspace missing or smaller than the plan needs*/
  TN_ERR_DEVICE = -7,      /* a HIP runtime call or a kernel launch failed    */
  TN_ERR_GATE = -8,        /* unknown gate, bad qubit index, channel where a  */
                           /* unitary is required, non-unitary gate matrix    */
  TN_ERR_SITE = -9,        /* MPS site out of range                           */
  TN_ERR_UNSUPPORTED = -10,/* valid request the library does not implement    */
  TN_ERR_NOMEM = -11,      /* host or device allocation failed                */
  TN_ERR_STATE = -12       /* handle used in a state that does not allow it   */
};

/* Thread-local message for the last failing call ("" if none). */
const char* tn_last_error(void);
/* Library version string, e.g. "tn-mi355x 0.1 gfx950". */
const char* tn_version(void);

/* ---------------------------------------------------------------------- */
/* Circuits (Sec. 3.1: qubits, one- and two-qubit gates; Sec. 3.3, Eq. 3:  */
/* Kraus channels)                                                         */
/* ---------------------------------------------------------------------- */

/* Gate / channel identifiers.  The library builds each matrix itself from
 * the id and params: sqrt_x, sqrt_y, sqrt_w are R_P(pi/2) =
 * cos(pi/4) I - i sin(pi/4) P for P = X, Y, (X+Y)/sqrt2; FSIM(theta, phi)
 * has cos(theta) on |01>,|10> diagonal, -i sin(theta) between them and
 * exp(-i phi) on |11>; CPHASE(phi) puts exp(i phi) on |11>; RZ(phi) =
 * diag(exp(-i phi/2), exp(i phi/2)); CX has q0 as control.
 * CUSTOM1 / CUSTOM2 take `matrix` (2x2 / 4x4 complex128, row-major).
 * Channels: DEPOL1(p) Kraus {sqrt(1-p) I, sqrt(p/3) X, Y, Z};
 * DEPOL2(p) {sqrt(1-p) II, sqrt(p/15) PQ for the 15 non-identity Pauli pairs,
 * P over I,X,Y,Z on q0 the outer loop}; AMP_DAMP(g) {[[1,0],[0,sqrt(1-g)]],
 * [[0,sqrt(g)],[0,0]]}.  Branch k of a channel is chosen when a uniform u
 * falls in [P_0+..+P_{k-1}, P_0+..+P_k). */
enum {
  TN_GATE_SQRT_X = 1, TN_GATE_SQRT_Y, TN_GATE_SQRT_W, TN_GATE_H, TN_GATE_X,
  TN_GATE_Y, TN_GATE_Z, TN_GATE_S, TN_GATE_T, TN_GATE_RZ,
  TN_GATE_CZ = 20, TN_GATE_CX, TN_GATE_FSIM, TN_GATE_CPHASE, TN_GATE_SWAP,
  TN_GATE_CUSTOM1 = 40, TN_GATE_CUSTOM2,
  TN_CHAN_DEPOL1 = 60, TN_CHAN_DEPOL2, TN_CHAN_AMP_DAMP
};

typedef struct {
  int32_t gate;          /* TN_GATE_* or TN_CHAN_*                          */
  int32_t q0;            /* first qubit                                     */
  int32_t q1;            /* second qubit, -1 for one-qubit ops              */
  double param[2];       /* angles (radians) or channel rates               */
  const double* matrix;  /* CUSTOM1/2 only: 2x2 or 4x4 complex128, read once */
} tn_op;

typedef struct {
  int32_t n_qubits;      /* 1 .. 4096                                       */
  int64_t n_ops;
  const tn_op* ops;      /* host memory, copied by the callee               */
} tn_circuit;

/* ---------------------------------------------------------------------- */
/* Network (Sec. 3.1, Fig. 1; small gates absorbed, Sec. 3.1.1)           */
/* ---------------------------------------------------------------------- */

typedef struct tn_network tn_network;

/* Build the tensor network of a noiseless circuit.  The |0> inputs and all
 * one-qubit gates are folded into neighbouring two-qubit gate tensors (a
 * wire without two-qubit gates becomes one rank-1 tensor); output legs stay
 * open until tn_amplitudes projects them.  Host only (no device work).
 * Errors: TN_ERR_ARG (null, n_qubits out of range), TN_ERR_GATE (unknown
 * id, bad qubit, q0 == q1, channel op). */
tn_status tn_build_network(const tn_circuit* c, tn_network** out);
tn_status tn_network_destroy(tn_network* n);

typedef struct {
  int32_t n_qubits;
  int32_t n_tensors;
  int32_t n_labels;      /* labels are 0 .. n_labels-1                      */
} tn_network_info;
tn_status tn_network_get_info(const tn_network* n, tn_network_info* info);
/* Tensor i: rank, labels (axis order) and complex128 data (row-major,
 * 2^rank entries).  labels / data may be NULL to query the rank only. */
tn_status tn_network_get_tensor(const tn_network* n, int32_t i, int32_t* rank,
                                int32_t* labels, double* data);
/* Output label of every qubit (n_qubits entries). */
tn_status tn_network_output_labels(const tn_network* n, int32_t* labels);

/* ---------------------------------------------------------------------- */
/* Contraction path and slicing (Sec. 3.1: Flop-minimising order, slicing) */
/* ---------------------------------------------------------------------- */

typedef struct tn_path tn_path;
typedef struct tn_model tn_model;

enum { TN_PATH_GREEDY = 0, TN_PATH_RANDOM_GREEDY = 1, TN_PATH_LEARNED = 2, TN_PATH_PARTITION = 3 };

typedef struct {
  int32_t algo;               /* TN_PATH_*                                  */
  int32_t trials;             /* random greedy: number of trials (>= 0)     */
  uint64_t seed;              /* random greedy: SplitMix64 seed             */
  double temperature;         /* random greedy: > 0, log2 units             */
  double mem_budget_bytes;    /* slice until 8*peak <= budget; <= 0: never  */
  const int8_t* open_mask;    /* n_qubits entries, 1 = output leg stays     */
                              /* open; NULL = every leg projected           */
  const tn_model* model;      /* TN_PATH_LEARNED: trained scorer; the path  */
                              /* takes the highest-scoring candidate each   */
                              /* step and falls back to greedy when greedy  */
                              /* is cheaper (flops, then peak)              */
  int32_t rank;               /* TN_PATH_PARTITION: TN_RANK_FLOPS (default) */
                              /* or TN_RANK_TIME (see tn_find_path)         */
  int32_t rank_precision;     /* TN_RANK_TIME: TN_PREC_* of the modelled    */
                              /* amplitude plan                             */
  int32_t rescore_every;      /* TN_PATH_LEARNED: merges per scoring (<= 1: */
                              /* re-score after every merge); each scoring  */
                              /* takes its best-scored pairs that share no  */
                              /* tensor, best first                         */
} tn_path_opts;

enum { TN_RANK_FLOPS = 0, TN_RANK_TIME = 1 };

typedef struct {
  double flops_per_slice;     /* 8 * sum over steps of prod(extents A u B)  */
  double total_flops;         /* flops_per_slice * n_slices                 */
  double peak_elems;          /* max over steps: live + |C| + |A| + |B|     */
  double n_slices;
  int32_t n_steps;
  int32_t n_sliced;
  int32_t algo_used;          /* LEARNED falls back to GREEDY when cheaper  */
  int32_t reserved;
} tn_path_cost;

/* Search a pairwise order (SSA pairs: leaves 0..n-1, step t creates id
 * n+t), then slice.  Cost model and heuristics: a greedy step picks the
 * connected pair minimising (|C|-|A|-|B|, flops, i, j); the randomised
 * version samples exp(-(sigma - sigma_min)/T), sigma = sign(d)log2(1+|d|),
 * from SplitMix64 (trial r seeded with seed + r * 0x9E3779B97F4A7C15, trials
 * on up to 16 host threads) and keeps the best of greedy + `trials` by
 * (flops, peak); with a budget, the 16 best by (flops, peak) are sliced and
 * the lowest (total flops, peak) is kept.  Slicing adds, while 8*peak >
 * budget, the label of the peak step that minimises (peak, total flops,
 * label).
 * PARTITION (Sec. 3.1 names graph partitioning plus heuristics): trial r
 * (stream seeded as above) draws an imbalance eps = 0.05 + 0.85 u and a
 * cutoff from {2, 4, 8, 16, 32}, then bisects the leaf graph (edges = labels
 * shared by two leaves) recursively: part 0 grows from a random seed leaf by
 * most links into it (ties: smallest id) to half the set, and
 * Fiduccia-Mattheyses passes move the unlocked leaf of largest cut gain
 * (ties: smallest id) within part sizes [max(1, floor((1-eps)n/2)),
 * n - that], keeping the best prefix, until a pass stops lowering the cut;
 * each split keeps the lowest cut of 8 such bisections (first on ties);
 * sets of at most `cutoff` leaves are ordered by greedy, the two halves are
 * contracted last.  Each tree is then reconfigured: for every internal node
 * (creation order) the frontier of its subtree grows to at most 8 tensors by
 * expanding the internal frontier node of largest result size (ties:
 * smallest id), and the flop-optimal order of that frontier (exact search
 * over subsets) replaces the subtree when strictly cheaper; passes repeat
 * (at most 8) until one no longer lowers the tree's flops.  The plain
 * greedy path and the trials are each sliced to the budget and the lowest
 * (total flops, peak, index) wins.  With rank = TN_RANK_TIME the 16 lowest
 * by that key are compiled into amplitude plans (all legs projected unless
 * open_mask says otherwise, precision rank_precision) and the one of least
 * modelled time wins (earlier on ties): n_slices x the sum over kernels of
 * max(flops / F, bytes / 4.0e12 B/s) + 5 us per launch, F = 350e12 flop/s
 * for split-precision GEMMs and 120e12 for the rest (sustained rates of
 * these kernels on MI355X); the contraction is memory-bound on this GPU, so
 * the flop count alone misranks trees.  Host only.
 * Errors: TN_ERR_ARG, TN_ERR_BUDGET, TN_ERR_STATE (LEARNED without model). */
tn_status tn_find_path(const tn_network* n, const tn_path_opts* o,
                       tn_path** out, tn_path_cost* cost);
/* Use a caller-given SSA path (2*n_steps ints) and slice it per o. */
tn_status tn_path_from_pairs(const tn_network* n, const tn_path_opts* o,
                             const int32_t* pairs, int32_t n_steps,
                             tn_path** out, tn_path_cost* cost);
/* Copy out the pairs (2*n_steps) and sliced labels (n_sliced); either may be
 * NULL. */
tn_status tn_path_get(const tn_path* p, int32_t* pairs, int32_t* sliced_labels);
tn_status tn_path_destroy(tn_path* p);

/* ---------------------------------------------------------------------- */
/* Learned contraction-order scorer (path quality vs search time, Sec. 4.3)*/
/* ---------------------------------------------------------------------- */

/* A message-passing network over the candidate pairwise contractions of a
 * path-search state (nodes; two candidates are neighbours when they share a
 * tensor).  16 features per candidate (log sizes of A, B, C and A u B,
 * shared labels, the greedy score and its offset from the best, live-tensor
 * and candidate counts, tensor degrees, outer-product flag, constant 1).
 *   h0 = relu(X W0 + b0); h_l = relu(h Ws_l + mean_nbrs(h) Wn_l + b_l),
 *   l = 1..L; score = relu(h_L Wh + bh) . wo + bo.
 * Parameters, in this order, row-major: W0 (16 x H), b0 (H), then per layer
 * Ws (H x H), Wn (H x H), b (H), then Wh (H x H), bh (H), wo (H), bo (1).
 * Trained by imitation of teacher paths: loss = logsumexp(scores) -
 * score[teacher choice] per state; Adam.  Forward, backward and Adam run in
 * hand-written FP32 kernels on the GPU. */

/* H in 1..256, L in 0..8.  Parameters start at zero: set them with
 * tn_model_set_params.  Errors: TN_ERR_ARG, TN_ERR_NOMEM, TN_ERR_DEVICE. */
tn_status tn_model_create(int32_t hidden, int32_t layers, tn_model** out);
tn_status tn_model_destroy(tn_model* m);
tn_status tn_model_n_params(const tn_model* m, int64_t* n);
/* Host FP64 arrays of n_params values (converted to / from FP32). */
tn_status tn_model_set_params(tn_model* m, const double* theta);
tn_status tn_model_get_params(const tn_model* m, double* theta);

/* Features and line-graph neighbours of the state reached after applying the
 * first n_prefix steps of `pairs` to network n (open legs per open_mask,
 * NULL = all projected).  Outputs (any may be NULL): *n_cands; cand
 * (2 * n_cands ints, SSA ids); X (n_cands x 16 doubles); nbr_ptr
 * (n_cands + 1); nbr_idx (nbr_ptr[n_cands] ints, ascending per node).
 * Call with NULL arrays first to learn n_cands and the neighbour count
 * (*n_nbr).  Host only. */
tn_status tn_model_state_features(const tn_network* n, const int8_t* open_mask,
                                  const int32_t* pairs, int32_t n_prefix,
                                  int32_t* n_cands, int32_t* n_nbr,
                                  int32_t* cand, double* X, int32_t* nbr_ptr,
                                  int32_t* nbr_idx);

/* Loss and gradient (n_params doubles) of one state on the GPU: features X
 * (n_cands x 16 doubles, host), CSR neighbours, teacher choice `label`.
 * Synchronises. */
tn_status tn_model_loss_grad(tn_model* m, int32_t n_cands, const double* X,
                             const int32_t* nbr_ptr, const int32_t* nbr_idx,
                             int32_t label, double* loss, double* grad,
                             double* scores, void* stream);

/* Append every `stride`-th state of the teacher path `pairs` (n_steps, a
 * path for network n) to the model's training set.  Host only. */
tn_status tn_model_add_teacher(tn_model* m, const tn_network* n,
                               const int8_t* open_mask, const int32_t* pairs,
                               int32_t n_steps, int32_t stride);
/* Adam (beta 0.9 / 0.999, eps 1e-8) over the training set: `epochs` passes
 * in SplitMix64-shuffled mini-batches of `batch` states.  *loss_first and
 * *loss_last (may be NULL) receive the mean loss of the first and last
 * epoch.  Synchronises.  Errors: TN_ERR_STATE (empty training set). */
tn_status tn_model_train(tn_model* m, int32_t epochs, int32_t batch,
                         double lr, uint64_t seed, double* loss_first,
                         double* loss_last, void* stream);

/* ---------------------------------------------------------------------- */
/* Pairwise contraction (Sec. 3.1; Table 2 is dominated by it)            */
/* ---------------------------------------------------------------------- */

enum { TN_C64 = 0, TN_C128 = 1 };

/* Arithmetic of the complex GEMMs.  FP32: FP32 MFMA.  BF16X3: each operand
 * split as hi + lo bfloat16, products hi*hi + hi*lo + lo*hi, FP32
 * accumulation (about 2^-17 relative per GEMM).  BF16X6: three-way bfloat16
 * split, six products (about FP32 accuracy).  F16X3: each operand scaled by
 * a power of two chosen from its largest entry (so it spans [2^14, 2^15)),
 * split as hi + lo fp16, three products, FP32 accumulation, scales undone
 * exactly (about 2^-21 relative per GEMM at the speed of BF16X3).  AUTO: the
 * library picks per contraction: F16X3 when K >= 64, M >= 1024 and N >= 64,
 * FP32 elsewhere.  At every precision, a contraction longer than 2^20 runs on
 * the FP32 kernel (split-K chains of at most 4096, partials summed in FP64),
 * and one with at most 16 outputs per batch entry and K >= 2^16 as FP64
 * dot products.  FP64 is the validation precision: every tensor is
 * complex128 (leaves from the FP64 gate matrices, FP64 multiply-adds
 * throughout, twice the workspace), so other precisions' results can be
 * compared with it on the device; tn_contract_pair takes it for TN_C128
 * tensors (and only those). */
enum { TN_PREC_FP32 = 0, TN_PREC_BF16X3 = 1, TN_PREC_BF16X6 = 2,
       TN_PREC_AUTO = 3, TN_PREC_F16X3 = 4, TN_PREC_FP64 = 5 };

typedef struct {
  void* data;                 /* device pointer, row-major, caller-owned    */
  int32_t rank;               /* 0 .. 64                                    */
  int32_t dtype;              /* TN_C64, or TN_C128 with TN_PREC_FP64       */
  const int64_t* extents;     /* host array of `rank` extents (>= 1)        */
} tn_tensor;

/* Caller-owned device scratch for tn_contract_pair and tn_amplitudes.  The
 * pointer must stay valid until replaced; calls that overlap on one device
 * share it.  bytes == 0 clears it. */
tn_status tn_set_workspace(void* device_ptr, size_t bytes);

/* C[modesC] = sum over the other labels of A[modesA] * B[modesB] (einsum
 * semantics): a label in A and B but not C is summed; in one input and C it
 * is free; in A, B and C it is a batch label; in one input only and not in C
 * it is summed out of that input.  modes are host arrays of `rank` ints.
 * Asynchronous on `stream`.  Uses up to |A|+|B|+|C| complex64 of workspace
 * when operands must be permuted.
 * Errors: TN_ERR_ARG, TN_ERR_MODES (repeat, or C label not in A or B),
 * TN_ERR_EXTENT, TN_ERR_UNSUPPORTED (C128), TN_ERR_WORKSPACE,
 * TN_ERR_DEVICE. */
tn_status tn_contract_pair(const tn_tensor* A, const int32_t* modesA,
                           const tn_tensor* B, const int32_t* modesB,
                           tn_tensor* C, const int32_t* modesC,
                           int32_t precision, void* stream);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * contraction, same arguments, kernels and results as tn_contract_pair, but
 * its scratch (permuted operands, split-precision planes and scale slots,
 * split-K partials) comes from a fixed 64 MiB device array inside the
 * library instead of tn_set_workspace.  The call allocates nothing: no
 * hipMalloc or hipFree, on the first call on a device included (each GPU
 * holds its own copy of the array from the library's load until the
 * process ends).  Every call on one GPU shares that array and leaves its
 * contents behind, so calls that overlap on one device (different streams
 * or threads, without ordering between them) race; calls ordered on one
 * stream are safe.
 * Errors: as tn_contract_pair, plus TN_ERR_WORKSPACE when the contraction
 * needs more than 64 MiB of scratch. */
tn_status tn_contract_pair_noalloc(const tn_tensor* A, const int32_t* modesA,
                                   const tn_tensor* B, const int32_t* modesB,
                                   tn_tensor* C, const int32_t* modesC,
                                   int32_t precision, void* stream);

/* ---------------------------------------------------------------------- */
/* Amplitudes (Eq. 1; batches, Sec. 3.1; marginal slices, Sec. 4.4)       */
/* ---------------------------------------------------------------------- */

typedef struct {
  double seconds;             /* device time of the run (HIP events)        */
  double flops;               /* algorithmic flops executed                 */
  double bytes;               /* algorithmic HBM bytes of the kernels       */
  double slices_run;          /* bit-string x slice jobs executed           */
  double kernels;             /* kernel launches per job                    */
  int32_t precision;          /* precision used (AUTO resolved)             */
  int32_t nonfinite;          /* 1 if an output entry is NaN or Inf         */
  double err_bound;           /* a-priori relative error estimate           */
} tn_report;

typedef struct {
  int32_t precision;          /* TN_PREC_*                                  */
  int32_t use_graph;          /* 1: capture one job as a hipGraph (on a     */
                              /* library-owned stream) and replay it per    */
                              /* job on `stream`                            */
  int64_t slice_begin;        /* first slice of the range to run            */
  int64_t slice_count;        /* number of slices; -1 = all                 */
  int32_t accumulate;         /* 1: add into `out`; 0: overwrite            */
  int32_t sync;               /* 1: wait for the stream before returning    */
                              /* (fills seconds / nonfinite)                */
  double* op_seconds;         /* NULL, or host array of tn_plan_info.n_ops: */
                              /* per-op device time summed over jobs (HIP   */
                              /* events around every op; implies sync, no   */
                              /* graph)                                     */
} tn_exec_opts;

/* Amplitudes <x|U|0..0> for n_bs bit-strings (host int8 array n_bs x
 * n_qubits, values 0, 1 or -1 = open).  Every bit-string must have the open
 * set the path was built for (TN_ERR_BITS otherwise).  `out` is a device
 * array of n_bs x 2^(#open) complex128: open qubits ascending, the first one
 * the most significant bit.  The result is the sum over the path's slices
 * (or over [slice_begin, slice_begin+slice_count)) of the per-slice
 * complex64 contraction, accumulated in FP64.  opts may be NULL (FP32, all
 * slices, overwrite, no sync).  rep may be NULL.
 * Errors: TN_ERR_ARG, TN_ERR_BITS, TN_ERR_WORKSPACE, TN_ERR_DEVICE. */
tn_status tn_amplitudes(const tn_network* n, const tn_path* p,
                        const int8_t* bits, int64_t n_bs,
                        const tn_exec_opts* opts, void* out, tn_report* rep,
                        void* stream);

/* Summary of the kernel sequence of one job (one bit-string, one slice). */
enum { TN_OP_APPLY = 0, TN_OP_PERMUTE = 1, TN_OP_GEMM = 2, TN_OP_DOT = 3 };
typedef struct {
  int32_t n_ops;              /* ops per job (plus gather and accumulate)   */
  int32_t n_by_kind[4];       /* indexed by TN_OP_*                         */
  double flops_by_kind[4];    /* algorithmic flops per job                  */
  double bytes_by_kind[4];    /* algorithmic HBM bytes per job              */
  double workspace_bytes;     /* tn_amplitudes_workspace for n_bs = 1       */
  double err_bound;           /* a-priori relative error estimate           */
} tn_plan_info;
tn_status tn_amplitudes_plan_info(const tn_network* n, const tn_path* p,
                                  int32_t precision, tn_plan_info* info);
/* Per-op detail (arrays of n_ops, any may be NULL): kind (TN_OP_*),
 * algorithmic flops and bytes, and `shape`, 8 int64 per op: m, n, k, batch,
 * block-tile id, packed flag, GEMM kernel launches (K-chunked accumulation:
 * ceil(k / 4096) unless split-K is used), 0 — for GEMMs; other kinds give
 * 1, 1, 1, 1, -1, 0, 1, 0 except APPLY: rows, 2^#N, 2^#K and the kernel
 * (0 apply_small_kernel, 1 the LDS-tiled apply_tile_kernel, 2 the matrix-core
 * apply16_mfma_kernel for 2^#N = 16) in the first four,
 * DOT: m, n, k, batch, and in the sixth 1 for the skinny long-K kernel
 * (batch 1, both operands read once) or 0 for one dot per (m, n), PERMUTE: output entries, planes
 * (0 = complex64, 2 or 3 split planes), fp16 flag and the kernel (0 device
 * copy, 1 permute_simple_kernel, 2 permute_tiled_kernel, 3 the max-abs
 * pre-pass of an fp16 operand, 4 permute_pipe_kernel) in the first four. */
tn_status tn_amplitudes_plan_ops(const tn_network* n, const tn_path* p,
                                 int32_t precision, int32_t* kind,
                                 double* flops, double* bytes, int64_t* shape);

/* Autotuner: time every candidate block-tile shape of every GEMM of this
 * path's plan (reps launches each, on the plan's own workspace buffers, whose
 * contents are overwritten), keep the fastest per GEMM for later
 * tn_amplitudes calls, and remember it for GEMMs of the same shape in plans
 * compiled afterwards (process-wide).  Needs the workspace of
 * tn_amplitudes_workspace (n_bs = 1).  Synchronises the stream. */
tn_status tn_amplitudes_autotune(const tn_network* n, const tn_path* p,
                                 int32_t precision, int32_t reps, void* stream);

/* Workspace bytes tn_amplitudes needs for this path, n_bs bit-strings and
 * precision (job control words, bit-strings, gathered leaves, intermediates
 * and permute / split-K scratch of one job).  Host only. */
tn_status tn_amplitudes_workspace(const tn_network* n, const tn_path* p,
                                  int64_t n_bs, int32_t precision,
                                  size_t* bytes);

/* ---------------------------------------------------------------------- */
/* Expectation values of Pauli strings (Sec. 3.1, operator expectation    */
/* values: Eq. 2, Table 1)                                                */
/* ---------------------------------------------------------------------- */

/* A Pauli string is an int8 array of n_qubits entries TN_PAULI_*. */
enum { TN_PAULI_I = 0, TN_PAULI_X = 1, TN_PAULI_Y = 2, TN_PAULI_Z = 3 };

/* Conjugate (double-depth) network of <Psi|P|Psi> = <0|C^dagger P C|0>,
 * Psi = C|0..0>.  A gate that contracts with its own conjugate (every gate
 * outside the backward light cone of P's support) is dropped with it before
 * the network is built; `kept_ops` (may be NULL) receives the number of
 * gates of C that remain.  The network is the one of the circuit C_L, P,
 * C_L^dagger (adjoints as CUSTOM gates), with the same folding and labels as
 * tn_build_network: find a path with no open qubits, and tn_amplitudes with
 * the all-zero bit-string returns <P> (real up to rounding).  Host only.
 * Errors: TN_ERR_ARG (null, sizes, Pauli entries outside 0..3), TN_ERR_GATE
 * (channel op, unknown id, bad qubit). */
tn_status tn_build_expectation_network(const tn_circuit* c, const int8_t* pauli,
                                       tn_network** out, int64_t* kept_ops);

/* Density-matrix network of Tr(rho P) (Sec. 3.3, Eq. 3): rho is the state
 * of the circuit c, which may hold channels (TN_CHAN_*), started in
 * |0..0><0..0|.  Every qubit carries a ket and a bra label; every op in P's
 * backward light cone becomes its superoperator sum_j A_j (x) conj(A_j) (a
 * unitary U: U (x) conj(U)) on the (ket, bra) legs, one-qubit ops folded
 * into the next two-qubit tensor of their qubit; ops outside the cone are
 * trace-preserving and drop out.  Each live qubit starts as a rank-2
 * |0><0| tensor and is closed by the rank-2 tensor P_q^T on its (ket, bra)
 * legs.  The network has no open legs (n_qubits 0): find a path and call
 * tn_amplitudes with one empty bit-string (n_bs = 1, zero entries); the one
 * output entry is Tr(rho P).  `kept_ops` (may be NULL) receives the number
 * of ops of c that remain.  Host only.  Errors: TN_ERR_ARG (null, sizes,
 * Pauli entries), TN_ERR_GATE (unknown id, bad qubit, bad channel rate). */
tn_status tn_build_density_network(const tn_circuit* c, const int8_t* pauli,
                                   tn_network** out, int64_t* kept_ops);

/* Samples from a marginal wave-function slice (Sec. 4.4; Table 1's
 * sampling from partial state vectors): psi is a device array of n complex128
 * amplitudes (e.g. one tn_amplitudes output row with open qubits), uniforms
 * m host values in [0, 1).  out[s] (host) receives the first index k with
 * C(k) > u_s * C(n-1), C the inclusive cumulative sum of |psi|^2 (FP64,
 * summed chunk by chunk of 4096 entries, chunks in index order), i.e. a
 * draw with probability |psi_k|^2 / sum |psi|^2; total (host, may be NULL)
 * receives sum |psi|^2.  Allocates a small device scratch and synchronises
 * the stream.  Errors: TN_ERR_ARG (null, sizes, a uniform outside [0, 1),
 * all amplitudes zero), TN_ERR_UNSUPPORTED, TN_ERR_DEVICE. */
tn_status tn_sample_amplitudes(const void* psi, int64_t n, const double* uniforms,
                               int64_t m, int64_t* out, double* total, void* stream);

/* <P> by wave-function slicing: `psi` is the device output of tn_amplitudes
 * for the n_slices bit-strings `bits` (host, n_slices x n_qubits, 0 / 1 for
 * projected qubits, -1 for the open qubits, the same open set in every row),
 * i.e. n_slices x 2^#open complex128.  Returns in out[0], out[1] (host) the
 * real and imaginary parts of sum_s <psi_s|P|psi_s>, accumulated in FP64 on
 * the device in a fixed order.  X and Y factors of P must act on open
 * qubits; a Z factor on a projected qubit contributes the slice's sign.  At
 * most 30 open qubits.  Allocates a small device scratch and synchronises
 * the stream.  Errors: TN_ERR_ARG (null, sizes, Pauli entries, X/Y on a
 * projected qubit), TN_ERR_BITS (values, open sets differ), TN_ERR_UNSUPPORTED,
 * TN_ERR_DEVICE. */
tn_status tn_pauli_expectation(const void* psi, const int8_t* bits, int64_t n_slices,
                               int32_t n_qubits, const int8_t* pauli, double* out,
                               void* stream);

/* ---------------------------------------------------------------------- */
/* Matrix product states (Sec. 3.2)                                       */
/* ---------------------------------------------------------------------- */

typedef struct tn_mps tn_mps;

/* |0...0> on n_sites qubits with bond dimensions up to chi_max (1..1024).
 * The site tensors live in library-owned device memory.
 * Errors: TN_ERR_ARG, TN_ERR_NOMEM, TN_ERR_DEVICE. */
tn_status tn_mps_create(int32_t n_sites, int32_t chi_max, void* stream,
                        tn_mps** out);
tn_status tn_mps_destroy(tn_mps* m);
/* One-qubit gate (2x2 complex128 row-major, host) absorbed into the site. */
tn_status tn_mps_apply_gate1(tn_mps* m, int32_t site, const double* gate,
                             void* stream);
/* Two-qubit gate (4x4 complex128, host) on sites (site, site+1), with the
 * more significant bit on `site`: move the orthogonality centre to `site`
 * (FP64 QR), contract both sites with the gate, FP64 SVD of the
 * (2 chi_l) x (2 chi_r) matrix, keep at most chi_max singular values with
 * s/s_max > cutoff, renormalise the kept values to unit norm, write back.
 * *discarded (may be NULL) receives the discarded weight sum s_dropped^2 /
 * sum s^2.  Synchronises the stream.
 * Errors: TN_ERR_SITE, TN_ERR_ARG (chi_max < 1, cutoff < 0), TN_ERR_DEVICE. */
tn_status tn_mps_apply_gate(tn_mps* m, int32_t site, const double* gate,
                            int32_t chi_max, double cutoff,
                            double* discarded, void* stream);
/* Bond dimensions (n_sites - 1 ints, host). */
tn_status tn_mps_bond_dims(const tn_mps* m, int32_t* dims);
/* Singular values of bond `bond` (between sites bond and bond+1) from the
 * last two-qubit gate on that bond (Sec. 3.2: the kept values of its SVD
 * after truncation and renormalisation to unit norm, descending; {1} before
 * any gate).  *count receives their number; `values` (host, may be NULL to
 * query the count) must hold `capacity` >= count doubles.  Gates on other
 * bonds after that one do not update it.  Host only.
 * Errors: TN_ERR_ARG, TN_ERR_SITE. */
tn_status tn_mps_bond_spectrum(const tn_mps* m, int32_t bond, double* values,
                               int32_t capacity, int32_t* count);
/* <Z_i> for every site (host array of n_sites doubles).  Synchronises. */
tn_status tn_mps_expect_z(tn_mps* m, double* out, void* stream);
/* Amplitudes of n_bs 0/1 bit-strings (host int8 n_bs x n_sites) into host
 * complex128 `out`.  Synchronises. */
tn_status tn_mps_amplitudes(tn_mps* m, const int8_t* bits, int64_t n_bs,
                            double* out, void* stream);

/* ---------------------------------------------------------------------- */
/* Locally-purified MPS (Sec. 3.4, the locally-purified MPS figure and the */
/* Kraus-contraction figure)                                               */
/* ---------------------------------------------------------------------- */

/* rho = Tr_K |X><X|: X is an MPS whose site tensors T[l, s, k, r] carry a
 * Kraus leg k (dimension K_i <= k_max) beside the physical leg s and the
 * virtual bonds (<= d_max); the Kraus leg is traced between X and its
 * conjugate.  Sites are complex64 in library-owned device memory; SVDs and
 * QRs run in FP64 (one-sided Jacobi, Householder), the merged pair on the
 * complex MFMA GEMM. */
typedef struct tn_pmps tn_pmps;

/* |0..0><0..0| on n_sites qubits (every K = 1).  d_max 1..256, k_max
 * 1..64, and the factorisation workspace (16 d_max^2 (2 k_max)^2 complex128
 * for a merged pair under a 16-operator channel) at most 16 GiB.
 * Errors: TN_ERR_ARG, TN_ERR_UNSUPPORTED, TN_ERR_NOMEM, TN_ERR_DEVICE. */
tn_status tn_pmps_create(int32_t n_sites, int32_t d_max, int32_t k_max,
                         void* stream, tn_pmps** out);
tn_status tn_pmps_destroy(tn_pmps* p);
/* One-qubit gate (2x2 complex128 row-major, host) on the physical leg. */
tn_status tn_pmps_apply_gate1(tn_pmps* p, int32_t site, const double* gate,
                              void* stream);
/* Two-qubit gate (4x4 complex128, host; `site` the more significant bit)
 * on (site, site+1), as tn_mps_apply_gate: the centre moves onto the pair,
 * the merged pair is split by an SVD of the (l, s, k) x (s, k, r) matrix,
 * at most d_max values with s / s_max > cutoff kept and renormalised; only
 * the virtual bond changes.  *discarded (may be NULL): dropped weight.
 * Synchronises.  Errors: TN_ERR_SITE, TN_ERR_ARG, TN_ERR_UNSUPPORTED,
 * TN_ERR_DEVICE. */
tn_status tn_pmps_apply_gate(tn_pmps* p, int32_t site, const double* gate,
                             double cutoff, double* discarded, void* stream);
/* Channel of n_kraus (1..16) operators on n_qubits (1 or 2) qubits starting
 * at `site` (host, complex128 row-major, 2x2 or 4x4 each, sum A^dagger A =
 * 1): each operator is contracted with the physical leg(s), its index
 * joining the (first) site's Kraus leg, which is then compressed at the
 * orthogonality centre by an SVD along it (T <- U S; at most k_max values
 * with s / s_max > cutoff, renormalised).  A two-qubit channel acts on the
 * merged pair, split as a gate with S on the first site.  *discarded_bond /
 * *discarded_kraus (may be NULL): dropped weights.  Synchronises.
 * Errors: TN_ERR_SITE, TN_ERR_ARG, TN_ERR_UNSUPPORTED, TN_ERR_DEVICE. */
tn_status tn_pmps_apply_channel(tn_pmps* p, int32_t site, int32_t n_qubits,
                                const double* kraus, int32_t n_kraus,
                                double cutoff, double* discarded_bond,
                                double* discarded_kraus, void* stream);
/* Bond dimensions (n_sites - 1) and Kraus dimensions (n_sites); either may
 * be NULL.  Host only. */
tn_status tn_pmps_dims(const tn_pmps* p, int32_t* bond_dims, int32_t* kraus_dims);
/* <Z_i> = Tr(rho Z_i) for every site (host, n_sites doubles).  Moves the
 * centre; synchronises. */
tn_status tn_pmps_expect_z(tn_pmps* p, double* out, void* stream);
/* Site tensor as complex128 (l, 2, K, r) row-major into host `data` (may
 * be NULL to query), its four dimensions into dims.  Synchronises. */
tn_status tn_pmps_get_site(tn_pmps* p, int32_t site, double* data, int32_t* dims,
                           void* stream);

/* ---------------------------------------------------------------------- */
/* Stochastic Kraus trajectories (Sec. 3.3, Eq. 3, sampled)               */
/* ---------------------------------------------------------------------- */

/* Run traj_per_circ trajectories of every circuit (noisy ops included) as
 * one batch.  For channel event e of trajectory t the branch is chosen by
 * uniforms[t * ld_uniforms + e] against p_k = |A_k psi|^2 (FP64), then the
 * state is renormalised.  Trajectory t = c * traj_per_circ + j runs circuit
 * c.  z_out (host, n_circ*traj_per_circ x n_qubits doubles) receives <Z_q>
 * of each final state.  All circuits must have the same n_qubits (<= 30).
 * Synchronises.  Errors: TN_ERR_ARG, TN_ERR_GATE, TN_ERR_NOMEM,
 * TN_ERR_DEVICE. */
tn_status tn_run_trajectories(const tn_circuit* const* circs, int32_t n_circ,
                              int32_t traj_per_circ, const double* uniforms,
                              int64_t ld_uniforms, double* z_out,
                              tn_report* rep, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* TN_H_ */

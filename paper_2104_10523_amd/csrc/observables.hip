// Expectation values of Pauli strings (Sec. 3.1, operator expectation values:
// Eq. 2 and the two methods of Table 1).
//
// Conjugate (double-depth) network: <Psi|P|Psi> = <0|C^dagger P C|0>.  A gate
// of C whose output never reaches the support of P meets its own conjugate
// in C^dagger with nothing in between, and the pair contracts to the
// identity; walking C backwards from P's support keeps exactly the gates in
// P's backward light cone.  The kept gates, the Pauli factors as one-qubit
// gates and the adjoints of the kept gates in reverse order form an ordinary
// circuit, so its network, path search, slicing and amplitude kernels are
// the ones of a single amplitude (all-zero bit-string).
//
// Density-matrix network (Sec. 3.3, Eq. 3): Tr(rho P) for a noisy circuit,
// every op as its superoperator on (ket, bra) legs, closed by P; a closed
// network with no output legs, contracted on the same engine.
//
// Sampling from a marginal slice (Sec. 4.4 slices as sampling input):
// bit-strings drawn with probability |psi_x|^2 / sum |psi|^2 by inverting
// the cumulative distribution (FP64) at caller-given uniforms.
//
// Wave-function slicing: the amplitudes of every projection of the closed
// qubits (tn_amplitudes with the open set left open) are reduced on the
// device as sum_s sum_x conj(psi_s[x]) (P psi_s)[x] in FP64.  X and Y
// factors must sit on open qubits (they would couple different slices); a
// Z factor on a projected qubit is a sign per slice.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <vector>

#include "common.hpp"
#include "gates.hpp"
#include "handles.hpp"
#include "network.hpp"

namespace tn {
namespace {

constexpr int kRedBlocks = 512;

// One block-partial of sum_x w_s (-1)^{popc(x & zmask)} conj(psi[s][x]) psi[s][x ^ flip]
// over a grid-stride range of the flattened (s, x) index; FP64 throughout.
__global__ __launch_bounds__(256) void pauli_partial_kernel(const double2* __restrict__ psi, int64_t n_slices,
                                                            int n_open, uint32_t flip, uint32_t zmask,
                                                            const double* __restrict__ w,
                                                            double2* __restrict__ part) {
  __shared__ double red[2][4];
  const int64_t dim = int64_t(1) << n_open;
  const int64_t total = n_slices * dim;
  double re = 0, im = 0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t s = i >> n_open;
    const uint32_t x = uint32_t(i & (dim - 1));
    const double2 a = psi[i];
    const double2 b = psi[(s << n_open) + (x ^ flip)];
    const double sg = (__popc(x & zmask) & 1) ? -w[s] : w[s];
    re += sg * (a.x * b.x + a.y * b.y);   // conj(a) b
    im += sg * (a.x * b.y - a.y * b.x);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    re += __shfl_xor(re, o);
    im += __shfl_xor(im, o);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = re;
    red[1][threadIdx.x >> 6] = im;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    part[blockIdx.x] = make_double2(red[0][0] + red[0][1] + red[0][2] + red[0][3],
                                    red[1][0] + red[1][1] + red[1][2] + red[1][3]);
}

// Sum of the block partials in a fixed order (one wave).
__global__ void pauli_final_kernel(const double2* __restrict__ part, int n, double2* __restrict__ out) {
  double re = 0, im = 0;
  for (int i = threadIdx.x; i < n; i += 64) {
    re += part[i].x;
    im += part[i].y;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    re += __shfl_xor(re, o);
    im += __shfl_xor(im, o);
  }
  if (threadIdx.x == 0) *out = make_double2(re, im);
}

constexpr int kSampleChunk = 4096;   // amplitudes per block of the sampler

// Sum of |psi|^2 over each chunk of kSampleChunk entries (FP64).
__global__ __launch_bounds__(256) void chunk_prob_kernel(const double2* __restrict__ psi, int64_t n,
                                                         double* __restrict__ chunk) {
  __shared__ double red[4];
  const int64_t base = int64_t(blockIdx.x) * kSampleChunk;
  double acc = 0;
  for (int i = threadIdx.x; i < kSampleChunk; i += 256) {
    const int64_t k = base + i;
    if (k < n) acc += psi[k].x * psi[k].x + psi[k].y * psi[k].y;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) chunk[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// In-place inclusive prefix sum of the chunk sums, in index order (one thread).
__global__ void chunk_scan_kernel(double* __restrict__ chunk, int64_t nc) {
  double acc = 0;
  for (int64_t i = 0; i < nc; ++i) {
    acc += chunk[i];
    chunk[i] = acc;
  }
}

// Sample s: the first index k with (prefix of chunks before k's chunk) +
// (|psi|^2 summed over k's chunk up to k) > u_s * total.
__global__ void sample_kernel(const double2* __restrict__ psi, int64_t n, const double* __restrict__ cum,
                              int64_t nc, const double* __restrict__ u, int64_t m,
                              int64_t* __restrict__ out) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= m) return;
  const double target = u[s] * cum[nc - 1];
  int64_t lo = 0, hi = nc - 1;           // first chunk whose inclusive sum exceeds target
  while (lo < hi) {
    const int64_t mid = (lo + hi) / 2;
    if (cum[mid] > target) hi = mid;
    else lo = mid + 1;
  }
  double acc = lo > 0 ? cum[lo - 1] : 0.0;
  const int64_t b0 = lo * kSampleChunk, b1 = min(n, b0 + kSampleChunk);
  int64_t pick = b1 - 1;
  for (int64_t k = b0; k < b1; ++k) {
    acc += psi[k].x * psi[k].x + psi[k].y * psi[k].y;
    if (acc > target) { pick = k; break; }
  }
  out[s] = pick;
}

}  // namespace

// Ops of C in P's backward light cone, in circuit order.  Channels are
// accepted when `channels` is set (trace-preserving maps outside the cone
// drop out of a trace as unitaries do).
std::vector<tn_op> light_cone_ops(const tn_circuit& c, const int8_t* pauli, bool channels = false) {
  std::vector<char> live(c.n_qubits, 0);
  for (int q = 0; q < c.n_qubits; ++q) {
    TN_REQUIRE(pauli[q] >= TN_PAULI_I && pauli[q] <= TN_PAULI_Z, TN_ERR_ARG, "Pauli entries must be 0..3");
    live[q] = pauli[q] != TN_PAULI_I;
  }
  std::vector<char> keep(c.n_ops, 0);
  for (int64_t k = c.n_ops - 1; k >= 0; --k) {
    const tn_op& op = c.ops[k];
    TN_REQUIRE(channels || !gate_is_channel(op.gate), TN_ERR_GATE,
               "conjugate-network expectation values take unitary gates only");
    const int ar = gate_arity(op.gate);
    TN_REQUIRE(op.q0 >= 0 && op.q0 < c.n_qubits && (ar == 1 || (op.q1 >= 0 && op.q1 < c.n_qubits && op.q1 != op.q0)),
               TN_ERR_GATE, "bad qubit index");
    const bool hit = live[op.q0] || (ar == 2 && live[op.q1]);
    if (!hit) continue;
    keep[k] = 1;
    live[op.q0] = 1;
    if (ar == 2) live[op.q1] = 1;
  }
  std::vector<tn_op> out;
  for (int64_t k = 0; k < c.n_ops; ++k)
    if (keep[k]) out.push_back(c.ops[k]);
  return out;
}

// Superoperator of a one- or two-qubit op on interleaved (ket, bra) indices:
// one qubit: S[(k, b)][(k', b')] = sum_j A_j[k][k'] conj(A_j[b][b']);
// two qubits (a, c): row and column index (k_a, b_a, k_c, b_c).
Mat superop(const tn_op& op) {
  std::vector<Mat> ks;
  if (gate_is_channel(op.gate)) ks = channel_kraus(op);
  else ks.push_back(gate_unitary(op));
  const int d = ks[0].dim;            // 2 or 4
  Mat S(d * d);
  for (const Mat& A : ks)
    for (int ko = 0; ko < d; ++ko)
      for (int bo = 0; bo < d; ++bo)
        for (int ki = 0; ki < d; ++ki)
          for (int bi = 0; bi < d; ++bi) {
            const cd v = A(ko, ki) * std::conj(A(bo, bi));
            int r, c;
            if (d == 2) {
              r = ko * 2 + bo;
              c = ki * 2 + bi;
            } else {   // (k_a k_c), (b_a b_c) -> (k_a b_a k_c b_c)
              r = ((ko >> 1) << 3) | ((bo >> 1) << 2) | ((ko & 1) << 1) | (bo & 1);
              c = ((ki >> 1) << 3) | ((bi >> 1) << 2) | ((ki & 1) << 1) | (bi & 1);
            }
            S(r, c) += v;
          }
  return S;
}

// Density-matrix network of Tr(rho P), rho = Phi_m ... Phi_1(|0><0|)
// (Sec. 3.3, Eq. 3): each qubit carries a ket and a bra label; every op of
// P's backward light cone becomes its superoperator, one-qubit ops folded
// into the next two-qubit tensor of their qubit (rank 8 over (k, b) of both
// qubits, outputs first); each live qubit starts as a rank-2 |0><0| tensor
// and is closed by a rank-2 tensor C[k][b] = P_q[b][k] (with any pending
// one-qubit ops folded in).  No open legs: n_qubits of the network is 0.
Network build_density_network(const tn_circuit& c, const int8_t* pauli, int64_t* kept_ops) {
  const std::vector<tn_op> cone = light_cone_ops(c, pauli, true);
  const int n = c.n_qubits;
  std::vector<char> live(n, 0);
  for (int q = 0; q < n; ++q) live[q] = pauli[q] != TN_PAULI_I;
  for (const tn_op& op : cone) {
    live[op.q0] = 1;
    if (gate_arity(op.gate) == 2) live[op.q1] = 1;
  }
  Network net;
  net.n_qubits = 0;
  std::vector<Mat> pend(n, Mat::identity(4));
  std::vector<int> wk(n, -1), wb(n, -1);
  int nxt = 0;
  bool any = false;
  for (int q = 0; q < n; ++q) {
    if (!live[q]) continue;
    any = true;
    NetTensor t;                       // |0><0| on (k, b)
    t.labels = {nxt, nxt + 1};
    t.data = {cd(1, 0), cd(0, 0), cd(0, 0), cd(0, 0)};
    wk[q] = nxt;
    wb[q] = nxt + 1;
    nxt += 2;
    net.tensors.push_back(std::move(t));
  }
  for (const tn_op& op : cone) {
    const Mat S = superop(op);
    if (gate_arity(op.gate) == 1) {
      pend[op.q0] = matmul(S, pend[op.q0]);
      continue;
    }
    const int a = op.q0, b = op.q1;
    const Mat T = matmul(S, kron(pend[a], pend[b]));
    pend[a] = Mat::identity(4);
    pend[b] = Mat::identity(4);
    NetTensor t;
    t.labels = {nxt, nxt + 1, nxt + 2, nxt + 3, wk[a], wb[a], wk[b], wb[b]};
    t.data.assign(256, cd(0, 0));
    for (int r = 0; r < 16; ++r)
      for (int col = 0; col < 16; ++col) t.data[size_t(r) * 16 + col] = T(r, col);
    wk[a] = nxt;
    wb[a] = nxt + 1;
    wk[b] = nxt + 2;
    wb[b] = nxt + 3;
    nxt += 4;
    net.tensors.push_back(std::move(t));
  }
  static const cd PM[4][4] = {{1, 0, 0, 1}, {0, 1, 1, 0}, {0, cd(0, -1), cd(0, 1), 0}, {1, 0, 0, -1}};
  for (int q = 0; q < n; ++q) {
    if (!live[q]) continue;
    // closing row vector over (k, b): P[b][k], then the pending ops
    const cd* P = PM[int(pauli[q])];
    NetTensor t;
    t.labels = {wk[q], wb[q]};
    t.data.assign(4, cd(0, 0));
    for (int i = 0; i < 4; ++i) {
      cd acc(0, 0);
      for (int o = 0; o < 4; ++o) {
        const int ko = o >> 1, bo = o & 1;
        acc += P[bo * 2 + ko] * pend[q](o, i);
      }
      t.data[i] = acc;
    }
    net.tensors.push_back(std::move(t));
  }
  if (!any) {                          // Tr(rho) of nothing: one traced |0><0|
    NetTensor t0, t1;
    t0.labels = t1.labels = {0, 1};
    t0.data = {cd(1, 0), cd(0, 0), cd(0, 0), cd(0, 0)};
    t1.data = {cd(1, 0), cd(0, 0), cd(0, 0), cd(1, 0)};
    net.tensors.push_back(std::move(t0));
    net.tensors.push_back(std::move(t1));
    nxt = 2;
  }
  net.n_labels = nxt;
  if (kept_ops) *kept_ops = int64_t(cone.size());
  return net;
}

}  // namespace tn

using namespace tn;

extern "C" {

tn_status tn_build_expectation_network(const tn_circuit* c, const int8_t* pauli, tn_network** out,
                                       int64_t* kept_ops) {
  return guarded([&] {
    TN_REQUIRE(c && pauli && out, TN_ERR_ARG, "null argument");
    TN_REQUIRE(c->n_qubits >= 1 && c->n_qubits <= 4096, TN_ERR_ARG, "n_qubits must be 1..4096");
    TN_REQUIRE(c->n_ops >= 0 && (c->n_ops == 0 || c->ops), TN_ERR_ARG, "bad op array");
    const std::vector<tn_op> cone = light_cone_ops(*c, pauli);
    // C_L, then P, then C_L^dagger (each kept gate's adjoint, reverse order)
    std::vector<tn_op> ops(cone);
    for (int q = 0; q < c->n_qubits; ++q) {
      if (pauli[q] == TN_PAULI_I) continue;
      tn_op p;
      std::memset(&p, 0, sizeof(p));
      p.gate = pauli[q] == TN_PAULI_X ? TN_GATE_X : pauli[q] == TN_PAULI_Y ? TN_GATE_Y : TN_GATE_Z;
      p.q0 = q;
      p.q1 = -1;
      ops.push_back(p);
    }
    std::vector<std::vector<double>> mats;   // adjoint matrices, alive until the build
    mats.reserve(cone.size());
    for (auto it = cone.rbegin(); it != cone.rend(); ++it) {
      const Mat U = gate_unitary(*it);
      std::vector<double> m(size_t(2) * U.dim * U.dim);
      for (int r = 0; r < U.dim; ++r)
        for (int k = 0; k < U.dim; ++k) {
          const cd a = std::conj(U(k, r));
          m[2 * (size_t(r) * U.dim + k)] = a.real();
          m[2 * (size_t(r) * U.dim + k) + 1] = a.imag();
        }
      mats.push_back(std::move(m));
      tn_op a;
      std::memset(&a, 0, sizeof(a));
      a.gate = U.dim == 2 ? TN_GATE_CUSTOM1 : TN_GATE_CUSTOM2;
      a.q0 = it->q0;
      a.q1 = U.dim == 2 ? -1 : it->q1;
      a.matrix = mats.back().data();
      ops.push_back(a);
    }
    tn_circuit dd;
    dd.n_qubits = c->n_qubits;
    dd.n_ops = int64_t(ops.size());
    dd.ops = ops.data();
    auto n = std::make_unique<tn_network>();
    n->net = build_network(dd);
    if (kept_ops) *kept_ops = int64_t(cone.size());
    *out = n.release();
  });
}

tn_status tn_build_density_network(const tn_circuit* c, const int8_t* pauli, tn_network** out,
                                   int64_t* kept_ops) {
  return guarded([&] {
    TN_REQUIRE(c && pauli && out, TN_ERR_ARG, "null argument");
    TN_REQUIRE(c->n_qubits >= 1 && c->n_qubits <= 4096, TN_ERR_ARG, "n_qubits must be 1..4096");
    TN_REQUIRE(c->n_ops >= 0 && (c->n_ops == 0 || c->ops), TN_ERR_ARG, "bad op array");
    auto n = std::make_unique<tn_network>();
    n->net = build_density_network(*c, pauli, kept_ops);
    *out = n.release();
  });
}

tn_status tn_sample_amplitudes(const void* psi, int64_t n, const double* uniforms, int64_t m, int64_t* out,
                               double* total, void* stream) {
  return guarded([&] {
    TN_REQUIRE(psi && uniforms && out && n >= 1 && m >= 0, TN_ERR_ARG, "bad argument");
    for (int64_t s = 0; s < m; ++s)
      TN_REQUIRE(uniforms[s] >= 0.0 && uniforms[s] < 1.0, TN_ERR_ARG, "uniforms must lie in [0, 1)");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t nc = (n + kSampleChunk - 1) / kSampleChunk;
    TN_REQUIRE(nc <= (int64_t(1) << 31) - 1, TN_ERR_UNSUPPORTED, "too many amplitudes");
    double *cum = nullptr, *du = nullptr;
    int64_t* dout = nullptr;
    auto cleanup = [&]() {
      for (void* p : {(void*)cum, (void*)du, (void*)dout})
        if (p) (void)hipFree(p);
    };
    try {
      TN_HIP(hipMalloc(&cum, size_t(nc) * sizeof(double)));
      TN_HIP(hipMalloc(&du, size_t(std::max<int64_t>(m, 1)) * sizeof(double)));
      TN_HIP(hipMalloc(&dout, size_t(std::max<int64_t>(m, 1)) * sizeof(int64_t)));
      chunk_prob_kernel<<<unsigned(nc), 256, 0, st>>>(static_cast<const double2*>(psi), n, cum);
      TN_HIP(hipGetLastError());
      chunk_scan_kernel<<<1, 1, 0, st>>>(cum, nc);
      TN_HIP(hipGetLastError());
      if (m > 0) {
        TN_HIP(hipMemcpyAsync(du, uniforms, size_t(m) * sizeof(double), hipMemcpyHostToDevice, st));
        sample_kernel<<<unsigned((m + 255) / 256), 256, 0, st>>>(static_cast<const double2*>(psi), n, cum, nc,
                                                                  du, m, dout);
        TN_HIP(hipGetLastError());
        TN_HIP(hipMemcpyAsync(out, dout, size_t(m) * sizeof(int64_t), hipMemcpyDeviceToHost, st));
      }
      double tot = 0;
      TN_HIP(hipMemcpyAsync(&tot, cum + nc - 1, sizeof(double), hipMemcpyDeviceToHost, st));
      TN_HIP(hipStreamSynchronize(st));
      TN_REQUIRE(tot > 0, TN_ERR_ARG, "all amplitudes are zero");
      if (total) *total = tot;
    } catch (...) {
      cleanup();
      throw;
    }
    cleanup();
  });
}

tn_status tn_pauli_expectation(const void* psi, const int8_t* bits, int64_t n_slices, int32_t n_qubits,
                               const int8_t* pauli, double* out, void* stream) {
  return guarded([&] {
    TN_REQUIRE(psi && bits && pauli && out, TN_ERR_ARG, "null argument");
    TN_REQUIRE(n_slices >= 1 && n_qubits >= 1 && n_qubits <= 4096, TN_ERR_ARG, "bad sizes");
    // open set from the first bit-string; every slice must share it
    std::vector<int> open;
    for (int q = 0; q < n_qubits; ++q) {
      TN_REQUIRE(bits[q] >= -1 && bits[q] <= 1, TN_ERR_BITS, "bit values must be 0, 1 or -1");
      if (bits[q] < 0) open.push_back(q);
    }
    const int n_open = int(open.size());
    TN_REQUIRE(n_open <= 30, TN_ERR_UNSUPPORTED, "at most 30 open qubits");
    uint32_t flip = 0, zmask = 0;
    int n_y = 0;
    for (int j = 0; j < n_open; ++j) {
      const int q = open[j];
      const uint32_t b = uint32_t(1) << (n_open - 1 - j);   // first open qubit = most significant bit
      TN_REQUIRE(pauli[q] >= TN_PAULI_I && pauli[q] <= TN_PAULI_Z, TN_ERR_ARG, "Pauli entries must be 0..3");
      if (pauli[q] == TN_PAULI_X || pauli[q] == TN_PAULI_Y) flip |= b;
      if (pauli[q] == TN_PAULI_Y || pauli[q] == TN_PAULI_Z) zmask |= b;
      if (pauli[q] == TN_PAULI_Y) ++n_y;
    }
    // per-slice weight: Z factors on projected qubits
    std::vector<double> w(n_slices, 1.0);
    for (int64_t s = 0; s < n_slices; ++s)
      for (int q = 0; q < n_qubits; ++q) {
        const int8_t b = bits[s * n_qubits + q];
        TN_REQUIRE(b >= -1 && b <= 1, TN_ERR_BITS, "bit values must be 0, 1 or -1");
        TN_REQUIRE((b < 0) == (bits[q] < 0), TN_ERR_BITS, "every slice needs the same open set");
        if (b < 0) continue;
        TN_REQUIRE(pauli[q] >= TN_PAULI_I && pauli[q] <= TN_PAULI_Z, TN_ERR_ARG, "Pauli entries must be 0..3");
        TN_REQUIRE(pauli[q] != TN_PAULI_X && pauli[q] != TN_PAULI_Y, TN_ERR_ARG,
                   "X and Y factors must act on open qubits");
        if (pauli[q] == TN_PAULI_Z && b == 1) w[s] = -w[s];
      }
    hipStream_t st = static_cast<hipStream_t>(stream);
    double* dw = nullptr;
    double2* part = nullptr;
    double2* res = nullptr;
    auto cleanup = [&]() {
      for (void* p : {(void*)dw, (void*)part, (void*)res})
        if (p) (void)hipFree(p);
    };
    try {
      TN_HIP(hipMalloc(&dw, size_t(n_slices) * sizeof(double)));
      TN_HIP(hipMalloc(&part, kRedBlocks * sizeof(double2)));
      TN_HIP(hipMalloc(&res, sizeof(double2)));
      TN_HIP(hipMemcpyAsync(dw, w.data(), size_t(n_slices) * sizeof(double), hipMemcpyHostToDevice, st));
      const int64_t total = n_slices << n_open;
      const int blocks = int(std::min<int64_t>(kRedBlocks, (total + 255) / 256));
      pauli_partial_kernel<<<blocks, 256, 0, st>>>(static_cast<const double2*>(psi), n_slices, n_open, flip, zmask,
                                                   dw, part);
      TN_HIP(hipGetLastError());
      pauli_final_kernel<<<1, 64, 0, st>>>(part, blocks, res);
      TN_HIP(hipGetLastError());
      double2 r;
      TN_HIP(hipMemcpyAsync(&r, res, sizeof(double2), hipMemcpyDeviceToHost, st));
      TN_HIP(hipStreamSynchronize(st));
      // (-i)^{n_y}: each Y contributes -i on top of its flip and sign
      double re = r.x, im = r.y;
      for (int k = 0; k < (n_y & 3); ++k) {
        const double t = re;
        re = im;
        im = -t;
      }
      out[0] = re;
      out[1] = im;
    } catch (...) {
      cleanup();
      throw;
    }
    cleanup();
  });
}

}  // extern "C"

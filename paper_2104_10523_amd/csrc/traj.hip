// Stochastic Kraus trajectories (Sec. 3.3, Eq. 3 in sampled form), batched:
// all trajectories of all circuits advance together, one pass per gate.
//
// A trajectory's ops are grouped as [gate, channels on its qubits...].
// Depolarising channels are mixtures of Paulis with state-independent
// weights, so their branch is drawn on the host from the shared uniform and
// folded into the gate matrix.  Amplitude damping has state-dependent branch
// probabilities: the pass that applies a gate also accumulates (FP64) the
// joint marginal of the gate's qubits; the next pass first reduces those
// partials, draws the damping branches from the uniforms, and applies the
// chosen Kraus operators (renormalised), then its own gate, to amplitudes
// held in registers in groups of 16 (four local index bits).  Trajectories
// are sorted by length so the active ones form a prefix (uneven depths).
// The final pass applies the last damping; a last kernel accumulates <Z_q>.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "common.hpp"
#include "gates.hpp"

namespace tn {
namespace {

constexpr int kBlocksPerTraj = 64;
constexpr int kMaxQubits = 30;

struct GroupDesc {
  int nq;               // 0 (no gate), 1 or 2
  int q[2];
  float2 G[16];         // 2^nq x 2^nq, row-major, depolarising Paulis folded in
  int n_damp;           // damping events after the gate (0..2), in order
  int damp_lq[2];       // local qubit of the gate (0 = q[0], 1 = q[1])
  float gamma[2];
  double u[2];
};

__device__ __forceinline__ float2 cmulf(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__global__ void init_state_kernel(float2* __restrict__ psi, int64_t dim) {
  const int64_t t = blockIdx.y;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < dim; i += int64_t(gridDim.x) * blockDim.x)
    psi[t * dim + i] = make_float2(i == 0 ? 1.f : 0.f, 0.f);
}

__device__ __forceinline__ float2 cfma(float2 a, float2 b, float2 acc) {
  return make_float2(acc.x + a.x * b.x - a.y * b.y, acc.y + a.x * b.y + a.y * b.x);
}

// The 2 x 2 operator A (row-major) on local bit B of the 16 register values.
template <int B>
__device__ __forceinline__ void apply_bit(float2 (&v)[16], const float2 (&A)[4]) {
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    if (i & (1 << B)) continue;
    const int j = i | (1 << B);
    const float2 x = v[i], y = v[j];
    v[i] = cfma(A[1], y, cmulf(A[0], x));
    v[j] = cfma(A[3], y, cmulf(A[2], x));
  }
}

typedef float f2v __attribute__((ext_vector_type(2)));

struct PassOps {
  float2 g4[16];        // gate x damping on local bits 0-1, scaled by the renormalisation
  float2 A2[4], A3[4];  // damping Kraus operators on local bits 2 and 3 (identity if none)
  int nq;               // gate arity (marginal index: i & 3, i & 1 or 0)
};

// The pass over this block's groups: 16 amplitudes per thread (addresses
// base | bits of e); the state is read and written once per pass, so the
// accesses are non-temporal.
__device__ __forceinline__ void run_groups(float2* st, int64_t groups, int nblk, const int (&sorted)[4],
                                           const int64_t (&bit)[4], const PassOps* os, double (&m4)[4]) {
  float2 g4[16], A2[4], A3[4];
#pragma unroll
  for (int i = 0; i < 16; ++i) g4[i] = os->g4[i];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    A2[i] = os->A2[i];
    A3[i] = os->A3[i];
  }
  const int nq = os->nq;
  for (int64_t gidx = int64_t(blockIdx.x) * 256 + threadIdx.x; gidx < groups; gidx += int64_t(nblk) * 256) {
    int64_t base = gidx;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int p = sorted[a];
      base = ((base >> p) << (p + 1)) | (base & ((int64_t(1) << p) - 1));
    }
    int64_t addr[16];
#pragma unroll
    for (int e = 0; e < 16; ++e)
      addr[e] = base | ((e & 1) ? bit[0] : 0) | ((e & 2) ? bit[1] : 0) | ((e & 4) ? bit[2] : 0) |
                ((e & 8) ? bit[3] : 0);
    float2 v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const f2v x = __builtin_nontemporal_load(reinterpret_cast<const f2v*>(st + addr[e]));
      v[e] = make_float2(x.x, x.y);
    }
    apply_bit<2>(v, A2);   // identity unless a damped qubit sits there
    apply_bit<3>(v, A3);
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const float2 x0 = v[4 * h], x1 = v[4 * h + 1], x2 = v[4 * h + 2], x3 = v[4 * h + 3];
#pragma unroll
      for (int r = 0; r < 4; ++r)
        v[4 * h + r] = cfma(g4[4 * r + 3], x3, cfma(g4[4 * r + 2], x2, cfma(g4[4 * r + 1], x1, cmulf(g4[4 * r], x0))));
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const f2v x = {v[i].x, v[i].y};
      __builtin_nontemporal_store(x, reinterpret_cast<f2v*>(st + addr[i]));
      const double pr = double(v[i].x) * v[i].x + double(v[i].y) * v[i].y;
      if (nq == 2) m4[i & 3] += pr;
      else if (nq == 1) m4[i & 1] += pr;
      else m4[0] += pr;
    }
  }
}

// One pass.  blockIdx.y = trajectory slot (sorted, active prefix);
// blockIdx.x = block within the trajectory (nblk of them; the previous pass
// used nblk_prev).  Each thread holds 16 amplitudes that differ in four
// index bits: the current gate's qubits sit on local bits 0 (second qubit)
// and 1 (first qubit), the previous gate's qubits follow, then the highest
// unused index bits, so consecutive lanes touch consecutive amplitudes.  The
// chosen damping Kraus operators of the previous group act first: those on
// local bits 2-3 as 2 x 2 operators, those on bits 0-1 folded into the gate's
// 4 x 4 operator (scaled by the renormalisation), which acts last.
__global__ __launch_bounds__(256) void traj_pass_kernel(float2* __restrict__ psi, int n,
                                                        const GroupDesc* __restrict__ desc, int max_len,
                                                        const int* __restrict__ len, int pass, int nblk,
                                                        int nblk_prev, const double* __restrict__ part_prev,
                                                        double* __restrict__ part_cur) {
  __shared__ PassOps ops_s;
  __shared__ int upos[4];
  __shared__ double redp[4][4];
  const int t = blockIdx.y;
  const int L = len[t];
  const int64_t dim = int64_t(1) << n;
  const GroupDesc* cur = pass < L ? desc + int64_t(t) * max_len + pass : nullptr;
  const GroupDesc* prev = pass > 0 ? desc + int64_t(t) * max_len + pass - 1 : nullptr;
  const int tid = threadIdx.x;
  const bool damp = prev && prev->n_damp > 0;
  if (damp) {
    // joint marginal of the previous gate's qubits: the previous pass's
    // per-block partials, reduced in a fixed order
    const double* pp = part_prev + int64_t(t) * nblk_prev * 4;
    double acc = 0;
    for (int x = tid; x < nblk_prev * 4; x += 256) acc += pp[x];
#pragma unroll
    for (int o = 32; o >= 4; o >>= 1) acc += __shfl_xor(acc, o);
    if ((tid & 63) < 4) redp[tid >> 6][tid & 3] = acc;
  }
  __syncthreads();
  if (tid == 0) {
    int k = 0;
    auto add = [&](int bp) {
      for (int i = 0; i < k; ++i)
        if (upos[i] == bp) return;
      upos[k++] = bp;
    };
    if (cur && cur->nq == 2) { add(n - 1 - cur->q[1]); add(n - 1 - cur->q[0]); }
    if (cur && cur->nq == 1) add(n - 1 - cur->q[0]);
    if (damp)
      for (int i = 0; i < prev->nq; ++i) add(n - 1 - prev->q[i]);
    for (int bp = n - 1; k < 4 && bp >= 0; --bp) add(bp);
    PassOps& o = ops_s;
    o.nq = cur ? cur->nq : 0;
    float2 Dl[2][4];     // damping on local bits 0 and 1 (identity if none)
    for (int i = 0; i < 4; ++i) {
      const float2 id = make_float2(i == 0 || i == 3 ? 1.f : 0.f, 0.f);
      o.A2[i] = o.A3[i] = Dl[0][i] = Dl[1][i] = id;
    }
    double dscale = 1.0;
    if (damp) {
      // damping decisions of the previous group from its marginals; P is
      // indexed by (first qubit's bit) x 2 + second's
      double P[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) P[j] = redp[0][j] + redp[1][j] + redp[2][j] + redp[3][j];
      const int pn = prev->nq;
      for (int e = 0; e < prev->n_damp; ++e) {
        const int lq = prev->damp_lq[e];
        const int bit = pn == 2 ? (lq == 0 ? 1 : 0) : 0;
        const double g = prev->gamma[e];
        double T = 0, P1 = 0;
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          T += P[x];
          if ((x >> bit) & 1) P1 += P[x];
        }
        const double p0 = T > 0 ? (T - g * P1) / T : 1.0;
        const int kb = prev->u[e] < p0 ? 0 : 1;
        float2 A[4];
        if (kb == 0) {   // A0 = diag(1, sqrt(1 - g))
          A[0] = make_float2(1.f, 0.f);
          A[1] = A[2] = make_float2(0.f, 0.f);
          A[3] = make_float2(float(sqrt(1.0 - g)), 0.f);
#pragma unroll
          for (int x = 0; x < 4; ++x)
            if ((x >> bit) & 1) P[x] *= (1.0 - g);
        } else {         // A1 = sqrt(g) |0><1|
          A[0] = A[2] = A[3] = make_float2(0.f, 0.f);
          A[1] = make_float2(float(sqrt(g)), 0.f);
          double Q[4];
#pragma unroll
          for (int x = 0; x < 4; ++x) {
            double up = 0;   // P[x with the damped bit set]
#pragma unroll
            for (int y = 0; y < 4; ++y)
              if (y == (x | (1 << bit))) up = P[y];
            Q[x] = ((x >> bit) & 1) ? 0.0 : g * up;
          }
#pragma unroll
          for (int x = 0; x < 4; ++x) P[x] = Q[x];
        }
        const int bp = n - 1 - prev->q[lq];
        int loc = 0;
        for (int i = 0; i < 4; ++i)
          if (upos[i] == bp) loc = i;
        float2* dst = loc == 0 ? Dl[0] : loc == 1 ? Dl[1] : loc == 2 ? o.A2 : o.A3;
        for (int i = 0; i < 4; ++i) dst[i] = A[i];
      }
      double N2 = 0;
#pragma unroll
      for (int x = 0; x < 4; ++x) N2 += P[x];
      dscale = N2 > 0 ? 1.0 / sqrt(N2) : 1.0;
    }
    // the gate on local bits 0-1 (rows: first qubit's bit x 2 + second's),
    // times the damping on those bits (applied first), times the scale
    float2 Gm[16], Dm[16];
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c < 4; ++c) {
        float2 g = make_float2(0.f, 0.f);
        if (!cur || cur->nq == 0) {
          if (r == c) g = make_float2(1.f, 0.f);
        } else if (cur->nq == 1) {
          if ((r >> 1) == (c >> 1)) g = cur->G[(r & 1) * 2 + (c & 1)];
        } else {
          g = cur->G[r * 4 + c];
        }
        Gm[r * 4 + c] = g;
        // local bit 1 is the high bit of the 4 x 4 index
        Dm[r * 4 + c] = cmulf(Dl[1][(r >> 1) * 2 + (c >> 1)], Dl[0][(r & 1) * 2 + (c & 1)]);
      }
    const float ds = float(dscale);
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c < 4; ++c) {
        float2 acc = make_float2(0.f, 0.f);
        for (int k = 0; k < 4; ++k) acc = cfma(Gm[r * 4 + k], Dm[k * 4 + c], acc);
        o.g4[r * 4 + c] = make_float2(acc.x * ds, acc.y * ds);
      }
  }
  __syncthreads();
  int sorted[4] = {upos[0], upos[1], upos[2], upos[3]};
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = a + 1; b < 4; ++b)
      if (sorted[b] < sorted[a]) { const int x = sorted[a]; sorted[a] = sorted[b]; sorted[b] = x; }
  const int64_t bit[4] = {int64_t(1) << upos[0], int64_t(1) << upos[1], int64_t(1) << upos[2],
                          int64_t(1) << upos[3]};
  float2* st = psi + int64_t(t) * dim;
  double m4[4] = {0, 0, 0, 0};
  run_groups(st, dim >> 4, nblk, sorted, bit, &ops_s, m4);
  // block reductions in a fixed order (deterministic)
  __shared__ double redm[4][4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double x = m4[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    if ((tid & 63) == 0) redm[tid >> 6][k] = x;
  }
  __syncthreads();
  if (tid < 4)
    part_cur[(int64_t(t) * nblk + blockIdx.x) * 4 + tid] = redm[0][tid] + redm[1][tid] + redm[2][tid] + redm[3][tid];
}

// Per-block sums of |psi_x|^2 and of |psi_x|^2 x_q for every qubit q.
__global__ __launch_bounds__(256) void z_partial_kernel(const float2* __restrict__ psi, int n,
                                                        double* __restrict__ zpart) {
  __shared__ double red[256];
  const int t = blockIdx.y;
  const int64_t dim = int64_t(1) << n;
  const float2* st = psi + int64_t(t) * dim;
  double zs[kMaxQubits + 1];
#pragma unroll
  for (int q = 0; q <= kMaxQubits; ++q) zs[q] = 0;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < dim; i += int64_t(kBlocksPerTraj) * 256) {
    const float2 a = st[i];
    const double pr = double(a.x) * a.x + double(a.y) * a.y;
    zs[kMaxQubits] += pr;
#pragma unroll
    for (int q = 0; q < kMaxQubits; ++q)
      if (q < n && ((i >> (n - 1 - q)) & 1)) zs[q] += pr;
  }
#pragma unroll
  for (int k = 0; k <= kMaxQubits; ++k) {
    if (k < n || k == kMaxQubits) {
      red[threadIdx.x] = zs[k];
      __syncthreads();
      for (int w2 = 128; w2 > 0; w2 >>= 1) {
        if (threadIdx.x < w2) red[threadIdx.x] += red[threadIdx.x + w2];
        __syncthreads();
      }
      if (threadIdx.x == 0) {
        const int slot = k == kMaxQubits ? n : k;
        zpart[(int64_t(t) * kBlocksPerTraj + blockIdx.x) * (n + 1) + slot] = red[0];
      }
      __syncthreads();
    }
  }
}

__global__ void z_final_kernel(const double* __restrict__ zpart, int n, int n_traj, double* __restrict__ z) {
  const int t = blockIdx.x;
  for (int q = threadIdx.x; q < n; q += blockDim.x) {
    double s1 = 0, tot = 0;
    for (int b = 0; b < kBlocksPerTraj; ++b) {
      s1 += zpart[(int64_t(t) * kBlocksPerTraj + b) * (n + 1) + q];
      tot += zpart[(int64_t(t) * kBlocksPerTraj + b) * (n + 1) + n];
    }
    z[int64_t(t) * n + q] = tot > 0 ? (tot - 2 * s1) / tot : 0.0;
  }
}

// Host: compile one trajectory's op list into gate groups.
std::vector<GroupDesc> compile_traj(const tn_circuit& c, const double* u, int64_t n_u) {
  std::vector<GroupDesc> gs;
  int64_t e = 0;
  auto take_u = [&]() {
    TN_REQUIRE(e < n_u, TN_ERR_ARG, "fewer uniforms than channel events");
    return u[e++];
  };
  auto new_group = [&](int nq, int q0, int q1, const Mat& U) {
    GroupDesc g;
    std::memset(&g, 0, sizeof(g));
    g.nq = nq;
    g.q[0] = q0;
    g.q[1] = q1;
    for (int i = 0; i < U.dim * U.dim; ++i) g.G[i] = make_float2(float(U.a[i].real()), float(U.a[i].imag()));
    gs.push_back(g);
  };
  std::vector<Mat> gate_mats;  // FP64 copy of the current group's gate
  Mat curU;
  for (int64_t k = 0; k < c.n_ops; ++k) {
    const tn_op& op = c.ops[k];
    const int ar = gate_arity(op.gate);
    TN_REQUIRE(op.q0 >= 0 && op.q0 < c.n_qubits && (ar == 1 || (op.q1 >= 0 && op.q1 < c.n_qubits && op.q1 != op.q0)),
               TN_ERR_GATE, "bad qubit index");
    if (!gate_is_channel(op.gate)) {
      curU = gate_unitary(op);
      new_group(ar, op.q0, ar == 2 ? op.q1 : -1, curU);
      continue;
    }
    GroupDesc* g = gs.empty() ? nullptr : &gs.back();
    auto on_group = [&](int q) -> int {
      if (!g) return -1;
      for (int i = 0; i < g->nq; ++i)
        if (g->q[i] == q) return i;
      return -1;
    };
    if (op.gate == TN_CHAN_DEPOL1 || op.gate == TN_CHAN_DEPOL2) {
      // state-independent branch weights: draw on the host, fold the Pauli
      const auto ks = channel_kraus(op);
      const double p = op.param[0];
      const int nk = int(ks.size());
      std::vector<double> w(nk);
      for (int i = 0; i < nk; ++i) w[i] = i == 0 ? 1 - p : (op.gate == TN_CHAN_DEPOL1 ? p / 3 : p / 15);
      const double uu = take_u();
      double acc = 0;
      int kb = nk - 1;
      for (int i = 0; i < nk; ++i) {
        acc += w[i];
        if (uu < acc) { kb = i; break; }
      }
      Mat P = ks[kb];
      const double sw = std::sqrt(w[kb]);
      for (auto& x : P.a) x /= sw;
      const bool same = g && g->n_damp == 0 &&
                        ((ar == 1 && g->nq == 1 && g->q[0] == op.q0) ||
                         (ar == 2 && g->nq == 2 && g->q[0] == op.q0 && g->q[1] == op.q1));
      if (same) {
        curU = matmul(P, curU);
        for (int i = 0; i < curU.dim * curU.dim; ++i)
          g->G[i] = make_float2(float(curU.a[i].real()), float(curU.a[i].imag()));
      } else {
        curU = P;
        new_group(ar, op.q0, ar == 2 ? op.q1 : -1, P);
      }
      continue;
    }
    // amplitude damping on one qubit
    int lq = on_group(op.q0);
    bool repeat = false;
    if (g && lq >= 0)
      for (int i = 0; i < g->n_damp; ++i)
        if (g->damp_lq[i] == lq) repeat = true;
    if (!g || lq < 0 || repeat || g->n_damp >= 2) {
      curU = Mat::identity(2);
      new_group(1, op.q0, -1, curU);
      g = &gs.back();
      lq = 0;
    }
    TN_REQUIRE(op.param[0] >= 0 && op.param[0] <= 1, TN_ERR_GATE, "damping rate outside [0,1]");
    g->damp_lq[g->n_damp] = lq;
    g->gamma[g->n_damp] = float(op.param[0]);
    g->u[g->n_damp] = take_u();
    g->n_damp++;
  }
  return gs;
}

}  // namespace
}  // namespace tn

using namespace tn;

extern "C" tn_status tn_run_trajectories(const tn_circuit* const* circs, int32_t n_circ, int32_t traj_per_circ,
                                         const double* uniforms, int64_t ld_uniforms, double* z_out,
                                         tn_report* rep, void* stream) {
  return guarded([&] {
    TN_REQUIRE(circs && uniforms && z_out && n_circ >= 1 && traj_per_circ >= 1 && ld_uniforms >= 1,
               TN_ERR_ARG, "bad argument");
    const int n = circs[0]->n_qubits;
    TN_REQUIRE(n >= 4 && n <= kMaxQubits, TN_ERR_ARG, "trajectories need 4..30 qubits");
    for (int c = 0; c < n_circ; ++c)
      TN_REQUIRE(circs[c] && circs[c]->n_qubits == n, TN_ERR_ARG, "all circuits need the same qubit count");
    const int64_t n_traj = int64_t(n_circ) * traj_per_circ;
    std::vector<std::vector<GroupDesc>> groups(n_traj);
    int max_len = 1;
    for (int64_t t = 0; t < n_traj; ++t) {
      groups[t] = compile_traj(*circs[t / traj_per_circ], uniforms + t * ld_uniforms, ld_uniforms);
      max_len = std::max<int>(max_len, int(groups[t].size()));
    }
    // longest first: the active trajectories of every pass form a prefix
    std::vector<int64_t> order(n_traj);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t a, int64_t b) { return groups[a].size() > groups[b].size(); });
    std::vector<GroupDesc> descs(size_t(n_traj) * max_len);
    std::vector<int> lens(n_traj);
    for (int64_t s = 0; s < n_traj; ++s) {
      const auto& g = groups[order[s]];
      lens[s] = int(g.size());
      std::copy(g.begin(), g.end(), descs.begin() + s * max_len);
    }
    const int64_t dim = int64_t(1) << n;
    hipStream_t s = static_cast<hipStream_t>(stream);
    float2* psi = nullptr;
    GroupDesc* ddesc = nullptr;
    int* dlen = nullptr;
    double *part = nullptr, *zpart = nullptr, *dz = nullptr;
    auto cleanup = [&]() {
      for (void* p : {(void*)psi, (void*)ddesc, (void*)dlen, (void*)part, (void*)zpart, (void*)dz})
        if (p) (void)hipFree(p);
    };
    try {
      TN_REQUIRE(hipMalloc(&psi, size_t(n_traj) * dim * sizeof(float2)) == hipSuccess, TN_ERR_NOMEM,
                 "cannot allocate the trajectory states");
      TN_HIP(hipMalloc(&ddesc, descs.size() * sizeof(GroupDesc)));
      TN_HIP(hipMalloc(&dlen, n_traj * sizeof(int)));
      // blocks per trajectory: at least 4096 blocks per pass while each
      // thread keeps at least one group (fewer trajectories -> more blocks)
      const int64_t max_blk = std::max<int64_t>(1, std::min<int64_t>(1024, (dim / 16 + 255) / 256));
      auto blocks_for = [&](int64_t active) {
        return int(std::min<int64_t>(max_blk, std::max<int64_t>(64, (4096 + active - 1) / active)));
      };
      TN_HIP(hipMalloc(&part, size_t(2) * n_traj * max_blk * 4 * sizeof(double)));
      TN_HIP(hipMalloc(&zpart, size_t(n_traj) * kBlocksPerTraj * (n + 1) * sizeof(double)));
      TN_HIP(hipMalloc(&dz, size_t(n_traj) * n * sizeof(double)));
      TN_HIP(hipMemcpyAsync(ddesc, descs.data(), descs.size() * sizeof(GroupDesc), hipMemcpyHostToDevice, s));
      TN_HIP(hipMemcpyAsync(dlen, lens.data(), n_traj * sizeof(int), hipMemcpyHostToDevice, s));
      hipEvent_t e0, e1;
      TN_HIP(hipEventCreate(&e0));
      TN_HIP(hipEventCreate(&e1));
      TN_HIP(hipEventRecord(e0, s));
      TN_REQUIRE(n_traj <= 65535, TN_ERR_UNSUPPORTED, "at most 65535 trajectories per call");
      init_state_kernel<<<dim3(unsigned(std::min<int64_t>((dim + 255) / 256, 1024)), unsigned(n_traj)), 256, 0, s>>>(psi, dim);
      TN_HIP(hipGetLastError());
      double bytes = 0;
      int nblk_prev = 1;
      for (int p = 0; p <= max_len; ++p) {
        int64_t active = 0;
        while (active < n_traj && lens[active] >= p) ++active;
        if (active == 0) break;
        const int nblk = blocks_for(active);
        const double* pp = part + size_t((p + 1) & 1) * n_traj * max_blk * 4;
        double* pc = part + size_t(p & 1) * n_traj * max_blk * 4;
        traj_pass_kernel<<<dim3(unsigned(nblk), unsigned(active)), 256, 0, s>>>(psi, n, ddesc, max_len, dlen, p,
                                                                                 nblk, nblk_prev, pp, pc);
        TN_HIP(hipGetLastError());
        bytes += double(active) * dim * 16.0;
        nblk_prev = nblk;
      }
      z_partial_kernel<<<dim3(kBlocksPerTraj, unsigned(n_traj)), 256, 0, s>>>(psi, n, zpart);
      TN_HIP(hipGetLastError());
      bytes += double(n_traj) * dim * 8.0;
      z_final_kernel<<<unsigned(n_traj), 64, 0, s>>>(zpart, n, int(n_traj), dz);
      TN_HIP(hipGetLastError());
      TN_HIP(hipEventRecord(e1, s));
      std::vector<double> z(size_t(n_traj) * n);
      TN_HIP(hipMemcpyAsync(z.data(), dz, z.size() * sizeof(double), hipMemcpyDeviceToHost, s));
      TN_HIP(hipStreamSynchronize(s));
      float ms = 0;
      TN_HIP(hipEventElapsedTime(&ms, e0, e1));
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      for (int64_t sl = 0; sl < n_traj; ++sl)
        for (int q = 0; q < n; ++q) z_out[order[sl] * n + q] = z[sl * n + q];
      if (rep) {
        std::memset(rep, 0, sizeof(*rep));
        rep->seconds = ms * 1e-3;
        rep->bytes = bytes;
        rep->flops = bytes / 16.0 * 4 * 8;    // 4x4 gate operator per 4 amplitudes
        rep->slices_run = double(n_traj);
        rep->kernels = double(max_len + 2);
      }
    } catch (...) {
      cleanup();
      throw;
    }
    cleanup();
  });
}

// Matrix product states (Sec. 3.2): one-qubit gates absorbed into sites;
// two-qubit gates by merge -> SVD -> truncate -> update.
//
// Site tensors are complex64 (chi_l, 2, chi_r) in library-owned device
// memory.  The two-site tensor theta is formed by the complex MFMA GEMM; the
// gate is mixed in while theta is converted to FP64; the SVD is one-sided
// Jacobi in FP64 (parallel column-pair rounds, one workgroup per pair, a
// whole sweep replayed as a hipGraph until no rotation exceeds the
// tolerance); the orthogonality centre is moved by FP64 Householder QR.
// Truncation keeps s / s_max > cutoff, at most chi_max values, renormalised
// to unit norm; S is absorbed toward the side the centre came from.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <numeric>
#include <vector>

#include "common.hpp"
#include "gates.hpp"
#include "kernels.hpp"
#include "linalg64.hpp"

namespace tn {
namespace {

struct Mat4 {
  double2 g[16];
};
struct Mat2 {
  double2 g[4];
};

__global__ void gate1_kernel(float2* __restrict__ A, int chil, int chir, Mat2 G) {
  const int64_t n = int64_t(chil) * chir;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t l = i / chir, r = i % chir;
    const float2 a0 = A[(l * 2 + 0) * chir + r], a1 = A[(l * 2 + 1) * chir + r];
    const double2 x0 = make_double2(a0.x, a0.y), x1 = make_double2(a1.x, a1.y);
    const double2 y0 = cadd(cmul(G.g[0], x0), cmul(G.g[1], x1));
    const double2 y1 = cadd(cmul(G.g[2], x0), cmul(G.g[3], x1));
    A[(l * 2 + 0) * chir + r] = make_float2(float(y0.x), float(y0.y));
    A[(l * 2 + 1) * chir + r] = make_float2(float(y1.x), float(y1.y));
  }
}

// theta[(l,s1),(s2,r)] (complex64, from the GEMM) -> gate-mixed FP64 matrix
// M[(l,t1),(t2,r)], stored column-major as W: if !trans, W column j = M[:, j]
// (mm = 2 chil rows); else W column j = conj(M[j, :]) (mm = 2 chir rows).
__global__ void mix_kernel(const float2* __restrict__ theta, double2* __restrict__ W, int chil, int chir,
                           Mat4 G, int trans) {
  const int64_t rows = 2 * int64_t(chil), cols = 2 * int64_t(chir);
  const int64_t n = rows * cols;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t row = i / cols, col = i % cols;
    const int64_t l = row >> 1, t1 = row & 1, t2 = col / chir, r = col % chir;
    double2 acc = make_double2(0, 0);
    for (int s1 = 0; s1 < 2; ++s1)
      for (int s2 = 0; s2 < 2; ++s2) {
        const float2 th = theta[(l * 2 + s1) * cols + s2 * chir + r];
        acc = cadd(acc, cmul(G.g[(t1 * 2 + t2) * 4 + s1 * 2 + s2], make_double2(th.x, th.y)));
      }
    if (!trans) W[col * rows + row] = acc;
    else W[row * cols + col] = make_double2(acc.x, -acc.y);
  }
}

// New sites from the factorisation.  U column k (m = 2 chil entries) and Vh
// row k (2 chir entries) for kept index order[k]:
//   !trans: U[:,k] = W[:,j] / s_j,   Vh[k,:] = conj(V[:, j])^T
//    trans: U[:,k] = V[:, j],         Vh[k,:] = conj(W[:, j])^T / s_j
// right: A_i = U, A_{i+1} = S Vh; left: A_i = U S, A_{i+1} = Vh (S scaled).
__global__ void write_sites_kernel(const double2* __restrict__ W, const double2* __restrict__ V,
                                   const double* __restrict__ S, const int* __restrict__ order, int keep,
                                   double scale, int chil, int chir, int mm, int nn, int trans, int right,
                                   float2* __restrict__ Ai, float2* __restrict__ Aj) {
  const int64_t nu = int64_t(2) * chil * keep, nv = int64_t(keep) * 2 * chir;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nu + nv; i += int64_t(gridDim.x) * blockDim.x) {
    if (i < nu) {
      const int64_t row = i / keep, k = i % keep;   // A_i[(l,s), k]
      const int j = order[k];
      const double sj = S[j];
      double2 u;
      if (!trans) {
        const double2 w = W[int64_t(j) * mm + row];
        u = sj > 0 ? make_double2(w.x / sj, w.y / sj) : make_double2(0, 0);
      } else {
        u = V[int64_t(j) * nn + row];
      }
      if (!right) u = make_double2(u.x * sj * scale, u.y * sj * scale);
      Ai[row * keep + k] = make_float2(float(u.x), float(u.y));
    } else {
      const int64_t t = i - nu;
      const int64_t k = t / (2 * chir), col = t % (2 * chir);   // A_{i+1}[k, (s,r)]
      const int j = order[k];
      const double sj = S[j];
      double2 v;
      if (!trans) {
        const double2 x = V[int64_t(j) * nn + col];
        v = make_double2(x.x, -x.y);
      } else {
        const double2 w = W[int64_t(j) * mm + col];
        v = sj > 0 ? make_double2(w.x / sj, -w.y / sj) : make_double2(0, 0);
      }
      if (right) v = make_double2(v.x * sj * scale, v.y * sj * scale);
      Aj[k * 2 * chir + col] = make_float2(float(v.x), float(v.y));
    }
  }
}

// ---------------------------------------------------------------- QR

// X (m x n, column-major, FP64) from a site: !adj: X[(l,s), r] = A[l,s,r]
// (m = 2 chil, n = chir); adj: X = (A as chil x 2chir)^dagger (m = 2 chir,
// n = chil).  Columns are contiguous so a wave streams one column.
__global__ void site_to_x_kernel(const float2* __restrict__ A, double2* __restrict__ X, int chil, int chir,
                                 int adj) {
  const int64_t n = int64_t(chil) * 2 * chir;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const float2 a = A[i];
    if (!adj) {
      const int64_t row = i / chir, col = i % chir;          // row = (l, s)
      X[col * (2 * chil) + row] = make_double2(a.x, a.y);
    } else {
      const int64_t l = i / (2 * chir), c = i % (2 * chir);  // X[c, l] = conj A[l, c]
      X[l * (2 * chir) + c] = make_double2(a.x, -a.y);
    }
  }
}

// <Z> of the centre site: sum |A[l,s,r]|^2 (1 - 2s) / sum |A|^2.
__global__ __launch_bounds__(256) void site_z_kernel(const float2* __restrict__ A, int chil, int chir, double* out) {
  __shared__ double red[8];
  double z = 0, nn = 0;
  const int64_t n = int64_t(chil) * 2 * chir;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const float2 a = A[i];
    const double p = double(a.x) * a.x + double(a.y) * a.y;
    const int s = int((i / chir) & 1);
    z += s ? -p : p;
    nn += p;
  }
  z = block_sum(z, red);
  __syncthreads();
  nn = block_sum(nn, red);
  if (threadIdx.x == 0) *out = nn > 0 ? z / nn : 0.0;
}

// Amplitudes: one workgroup per bit-string, v <- v A_i[:, b_i, :] in FP64.
__global__ __launch_bounds__(256) void mps_amp_kernel(const float2* const* __restrict__ sites,
                                                     const int* __restrict__ chi, int n_sites,
                                                     const int8_t* __restrict__ bits, double2* __restrict__ out,
                                                     int cmax) {
  extern __shared__ double2 vbuf[];
  double2* v = vbuf;
  double2* w = vbuf + cmax;
  const int8_t* b = bits + int64_t(blockIdx.x) * n_sites;
  if (threadIdx.x == 0) v[0] = make_double2(1, 0);
  __syncthreads();
  int cl = 1;
  for (int i = 0; i < n_sites; ++i) {
    const int cr = i + 1 < n_sites ? chi[i] : 1;
    const float2* A = sites[i];
    const int s = b[i];
    for (int r = threadIdx.x; r < cr; r += blockDim.x) {
      double2 acc = make_double2(0, 0);
      for (int l = 0; l < cl; ++l) {
        const float2 a = A[(int64_t(l) * 2 + s) * cr + r];
        acc = cadd(acc, cmul(v[l], make_double2(a.x, a.y)));
      }
      w[r] = acc;
    }
    __syncthreads();
    for (int r = threadIdx.x; r < cr; r += blockDim.x) v[r] = w[r];
    __syncthreads();
    cl = cr;
  }
  if (threadIdx.x == 0) out[blockIdx.x] = v[0];
}

int grid_for(int64_t n) { return int(std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096))); }

}  // namespace
}  // namespace tn

using namespace tn;

struct tn_mps {
  int n = 0, cmax = 0, center = 0, dev = 0;
  std::vector<int> chi;            // bond i between sites i and i+1
  std::vector<std::vector<double>> spec;   // bond i: kept, renormalised values of its last SVD
  std::vector<float2*> site;       // capacity cmax * 2 * cmax each
  float2* theta = nullptr;         // (2 cmax) x (2 cmax) complex64
  float2* tmp = nullptr;           // site-sized scratch
  double2 *W = nullptr, *V = nullptr, *X = nullptr, *Q = nullptr, *R = nullptr, *tau = nullptr;
  double* S = nullptr;
  double* zbuf = nullptr;
  int* flag = nullptr;
  int* order = nullptr;
  void* gemm_work = nullptr;
  size_t gemm_work_bytes = 0;
  std::map<std::pair<int, int>, hipGraphExec_t> sweeps;   // (mm, nn) -> one Jacobi sweep
  std::map<std::pair<int, int>, hipGraphExec_t> qrs;      // (rows, cols) -> Householder QR
  hipStream_t gstream = nullptr;

  int chil(int i) const { return i == 0 ? 1 : chi[i - 1]; }
  int chir(int i) const { return i == n - 1 ? 1 : chi[i]; }

  ~tn_mps() {
    for (auto& kv : sweeps) (void)hipGraphExecDestroy(kv.second);
    for (auto& kv : qrs) (void)hipGraphExecDestroy(kv.second);
    for (float2* p : site) (void)hipFree(p);
    for (void* p : {(void*)theta, (void*)tmp, (void*)W, (void*)V, (void*)X, (void*)Q, (void*)R, (void*)tau,
                    (void*)S, (void*)zbuf, (void*)flag, (void*)order, gemm_work})
      if (p) (void)hipFree(p);
    if (gstream) (void)hipStreamDestroy(gstream);
  }
};

namespace {

// Householder QR of X (rows x cols, column-major) into R (k x cols, row-major)
// and Q (rows x k, column-major), k = min(rows, cols): per step j one
// reflector kernel and one trailing update (a wave per column), then Q from
// the reflectors in reverse order.  Captured once per shape as a hipGraph
// (the buffers are the MPS's own) and replayed on `s`.
void run_qr(tn_mps* m, int rows, int cols, hipStream_t s) {
  const auto key = std::make_pair(rows, cols);
  auto it = m->qrs.find(key);
  if (it == m->qrs.end()) {
    if (!m->gstream) TN_HIP(hipStreamCreateWithFlags(&m->gstream, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    TN_HIP(hipStreamBeginCapture(m->gstream, hipStreamCaptureModeThreadLocal));
    record_blocked_qr(m->X, m->R, m->Q, m->tau, rows, cols, m->gstream, 4096);
    const hipError_t e = hipStreamEndCapture(m->gstream, &g);
    TN_REQUIRE(e == hipSuccess, TN_ERR_DEVICE, "graph capture of the QR failed");
    TN_HIP(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
    (void)hipGraphDestroy(g);
    it = m->qrs.emplace(key, ge).first;
  }
  TN_HIP(hipGraphLaunch(it->second, s));   // stream-ordered with the caller's work
}

void move_right(tn_mps* m, int c, hipStream_t s) {
  const int cl = m->chil(c), cr = m->chir(c);
  const int rows = 2 * cl, cols = cr, k = std::min(rows, cols);
  site_to_x_kernel<<<grid_for(int64_t(cl) * 2 * cr), 256, 0, s>>>(m->site[c], m->X, cl, cr, 0);
  run_qr(m, rows, cols, s);
  q_to_site_kernel<<<grid_for(int64_t(rows) * k), 256, 0, s>>>(m->Q, m->site[c], rows, k, 0);
  // next site: (cr, 2, cr2) -> (k, 2, cr2)
  const int cr2 = m->chir(c + 1);
  const int64_t other = int64_t(2) * cr2;
  apply_r_kernel<<<grid_for(int64_t(k) * other), 256, 0, s>>>(m->R, k, cr, m->site[c + 1], m->tmp, other, 1);
  TN_HIP(hipMemcpyAsync(m->site[c + 1], m->tmp, size_t(k) * other * sizeof(float2), hipMemcpyDeviceToDevice, s));
  TN_HIP(hipGetLastError());
  m->chi[c] = k;
  m->center = c + 1;
}

void move_left(tn_mps* m, int c, hipStream_t s) {
  const int cl = m->chil(c), cr = m->chir(c);
  const int rows = 2 * cr, cols = cl, k = std::min(rows, cols);   // X = A^dagger
  site_to_x_kernel<<<grid_for(int64_t(cl) * 2 * cr), 256, 0, s>>>(m->site[c], m->X, cl, cr, 1);
  run_qr(m, rows, cols, s);
  // A_c = Q^dagger : (k, 2 cr)
  q_to_site_kernel<<<grid_for(int64_t(rows) * k), 256, 0, s>>>(m->Q, m->site[c], rows, k, 1);
  // previous site (cl2, 2, cl) -> (cl2, 2, k): B R^dagger
  const int cl2 = m->chil(c - 1);
  const int64_t rowsb = int64_t(cl2) * 2;
  apply_r_kernel<<<grid_for(rowsb * k), 256, 0, s>>>(m->R, k, cl, m->site[c - 1], m->tmp, rowsb, 0);
  TN_HIP(hipMemcpyAsync(m->site[c - 1], m->tmp, size_t(rowsb) * k * sizeof(float2), hipMemcpyDeviceToDevice, s));
  TN_HIP(hipGetLastError());
  m->chi[c - 1] = k;
  m->center = c - 1;
}

void move_center(tn_mps* m, int target, hipStream_t s) {
  while (m->center < target) move_right(m, m->center, s);
  while (m->center > target) move_left(m, m->center, s);
}

// One Jacobi sweep (npad - 1 rounds) on (mm, nn), captured once.
hipGraphExec_t sweep_graph(tn_mps* m, int mm, int nn) {
  auto key = std::make_pair(mm, nn);
  auto it = m->sweeps.find(key);
  if (it != m->sweeps.end()) return it->second;
  const int npad = nn + (nn & 1);
  // rotations below this relative size are rounding noise of the m-term dot products
  const double tol = 2.3e-16 * double(std::max(mm, 8));
  if (!m->gstream) TN_HIP(hipStreamCreateWithFlags(&m->gstream, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  TN_HIP(hipStreamBeginCapture(m->gstream, hipStreamCaptureModeThreadLocal));
  flag_reset_kernel<<<1, 1, 0, m->gstream>>>(m->flag);
  for (int r = 0; r < npad - 1; ++r)
    jacobi_round_kernel<<<npad / 2, 256, 0, m->gstream>>>(m->W, m->V, mm, nn, npad, r, tol, m->flag);
  const hipError_t e = hipStreamEndCapture(m->gstream, &g);
  TN_REQUIRE(e == hipSuccess, TN_ERR_DEVICE, "graph capture of the Jacobi sweep failed");
  TN_HIP(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
  (void)hipGraphDestroy(g);
  m->sweeps[key] = ge;
  return ge;
}

void read_mat(const double* gate, int d, double2* out) {
  for (int i = 0; i < d * d; ++i) out[i] = make_double2(gate[2 * i], gate[2 * i + 1]);
}

}  // namespace

extern "C" {

tn_status tn_mps_create(int32_t n_sites, int32_t chi_max, void* stream, tn_mps** out) {
  return guarded([&] {
    TN_REQUIRE(out && n_sites >= 2 && n_sites <= 4096, TN_ERR_ARG, "n_sites must be 2..4096");
    TN_REQUIRE(chi_max >= 1 && chi_max <= 1024, TN_ERR_ARG, "chi_max must be 1..1024");
    auto m = std::make_unique<tn_mps>();
    m->n = n_sites;
    m->cmax = chi_max;
    TN_HIP(hipGetDevice(&m->dev));
    m->chi.assign(n_sites - 1, 1);
    m->spec.assign(n_sites - 1, std::vector<double>(1, 1.0));
    const size_t cap = size_t(chi_max) * 2 * chi_max;
    const size_t big = size_t(2 * chi_max) * size_t(2 * chi_max);
    for (int i = 0; i < n_sites; ++i) {
      float2* p = nullptr;
      TN_HIP(hipMalloc(&p, cap * sizeof(float2)));
      m->site.push_back(p);
      const float2 init[2] = {make_float2(1.f, 0.f), make_float2(0.f, 0.f)};
      TN_HIP(hipMemcpy(p, init, sizeof(init), hipMemcpyHostToDevice));
    }
    TN_HIP(hipMalloc(&m->theta, big * sizeof(float2)));
    TN_HIP(hipMalloc(&m->tmp, cap * sizeof(float2)));
    TN_HIP(hipMalloc(&m->W, big * sizeof(double2)));
    TN_HIP(hipMalloc(&m->V, big * sizeof(double2)));
    TN_HIP(hipMalloc(&m->X, cap * sizeof(double2)));
    TN_HIP(hipMalloc(&m->Q, cap * sizeof(double2)));
    TN_HIP(hipMalloc(&m->R, cap * sizeof(double2)));
    TN_HIP(hipMalloc(&m->tau, size_t(2 * chi_max) * sizeof(double2)));
    TN_HIP(hipMalloc(&m->S, size_t(2 * chi_max) * sizeof(double)));
    TN_HIP(hipMalloc(&m->zbuf, size_t(n_sites) * sizeof(double)));
    TN_HIP(hipMalloc(&m->flag, 256));
    TN_HIP(hipMalloc(&m->order, size_t(2 * chi_max) * sizeof(int)));
    m->gemm_work_bytes = size_t(64) << 20;
    TN_HIP(hipMalloc(&m->gemm_work, m->gemm_work_bytes));
    m->center = 0;
    *out = m.release();
  });
}

tn_status tn_mps_destroy(tn_mps* m) {
  return guarded([&] { delete m; });
}

tn_status tn_mps_bond_dims(const tn_mps* m, int32_t* dims) {
  return guarded([&] {
    TN_REQUIRE(m && dims, TN_ERR_ARG, "null argument");
    for (int i = 0; i < m->n - 1; ++i) dims[i] = m->chi[i];
  });
}

tn_status tn_mps_bond_spectrum(const tn_mps* m, int32_t bond, double* values, int32_t capacity,
                                int32_t* count) {
  return guarded([&] {
    TN_REQUIRE(m && count, TN_ERR_ARG, "null argument");
    TN_REQUIRE(bond >= 0 && bond < m->n - 1, TN_ERR_SITE, "bond out of range");
    const auto& v = m->spec[bond];
    *count = int32_t(v.size());
    TN_REQUIRE(values == nullptr || capacity >= int32_t(v.size()), TN_ERR_ARG, "capacity below the bond dimension");
    if (values) std::copy(v.begin(), v.end(), values);
  });
}

tn_status tn_mps_apply_gate1(tn_mps* m, int32_t site, const double* gate, void* stream) {
  return guarded([&] {
    TN_REQUIRE(m && gate, TN_ERR_ARG, "null argument");
    TN_REQUIRE(site >= 0 && site < m->n, TN_ERR_SITE, "site out of range");
    Mat2 G;
    read_mat(gate, 2, G.g);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int cl = m->chil(site), cr = m->chir(site);
    gate1_kernel<<<grid_for(int64_t(cl) * cr), 256, 0, s>>>(m->site[site], cl, cr, G);
    TN_HIP(hipGetLastError());
  });
}

tn_status tn_mps_apply_gate(tn_mps* m, int32_t site, const double* gate, int32_t chi_max, double cutoff,
                            double* discarded, void* stream) {
  return guarded([&] {
    TN_REQUIRE(m && gate, TN_ERR_ARG, "null argument");
    TN_REQUIRE(site >= 0 && site + 1 < m->n, TN_ERR_SITE, "site out of range (needs site + 1 < n)");
    TN_REQUIRE(chi_max >= 1 && cutoff >= 0, TN_ERR_ARG, "chi_max must be >= 1 and cutoff >= 0");
    chi_max = std::min(chi_max, m->cmax);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool right = m->center <= site;
    move_center(m, right ? site : site + 1, s);
    const int cl = m->chil(site), cm = m->chi[site], cr = m->chir(site + 1);
    // theta = A_i (2cl x cm) . A_{i+1} (cm x 2cr) on the complex MFMA GEMM
    GemmDesc g;
    g.M = 2 * cl;
    g.N = 2 * cr;
    g.K = cm;
    g.precision = TN_PREC_FP32;
    TN_REQUIRE(gemm_workspace_bytes(g) <= m->gemm_work_bytes, TN_ERR_WORKSPACE, "MPS GEMM scratch too small");
    launch_gemm(m->site[site], m->site[site + 1], m->theta, g, m->gemm_work, nullptr, nullptr, s);
    Mat4 G;
    read_mat(gate, 4, G.g);
    const int rows = 2 * cl, cols = 2 * cr;
    const int trans = cols > rows ? 1 : 0;
    const int mm = trans ? cols : rows, nn = trans ? rows : cols;
    mix_kernel<<<grid_for(int64_t(rows) * cols), 256, 0, s>>>(m->theta, m->W, cl, cr, G, trans);
    eye_kernel<<<grid_for(int64_t(nn) * nn), 256, 0, s>>>(m->V, nn, m->flag);
    TN_HIP(hipGetLastError());
    // Jacobi sweeps until no pair needed a rotation (at most 60 sweeps)
    hipGraphExec_t ge = sweep_graph(m, mm, nn);
    hipEvent_t ev = nullptr;
    TN_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    TN_HIP(hipEventRecord(ev, s));
    TN_HIP(hipStreamWaitEvent(m->gstream, ev, 0));
    int sweeps = 0, flag = 1;
    while (flag && sweeps < 60) {
      TN_HIP(hipGraphLaunch(ge, m->gstream));
      TN_HIP(hipMemcpyAsync(&flag, m->flag, sizeof(int), hipMemcpyDeviceToHost, m->gstream));
      TN_HIP(hipStreamSynchronize(m->gstream));
      ++sweeps;
    }
    colnorm_kernel<<<nn, 256, 0, m->gstream>>>(m->W, mm, m->S);
    std::vector<double> S(nn);
    TN_HIP(hipMemcpyAsync(S.data(), m->S, nn * sizeof(double), hipMemcpyDeviceToHost, m->gstream));
    TN_HIP(hipStreamSynchronize(m->gstream));
    // truncation on the host: descending order, ties by index
    std::vector<int> order(nn);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return S[a] > S[b]; });
    const double smax = S[order[0]];
    int keep = 0;
    for (int k = 0; k < nn; ++k)
      if (smax > 0 && S[order[k]] > cutoff * smax) ++keep;
    keep = std::max(1, std::min(keep, chi_max));
    double total = 0, kept = 0;
    for (int k = 0; k < nn; ++k) {
      total += S[order[k]] * S[order[k]];
      if (k < keep) kept += S[order[k]] * S[order[k]];
    }
    if (discarded) *discarded = total > 0 ? (total - kept) / total : 0.0;
    const double scale = kept > 0 ? 1.0 / std::sqrt(kept) : 1.0;
    TN_HIP(hipMemcpyAsync(m->order, order.data(), keep * sizeof(int), hipMemcpyHostToDevice, m->gstream));
    const int64_t tot = int64_t(2) * cl * keep + int64_t(keep) * 2 * cr;
    write_sites_kernel<<<grid_for(tot), 256, 0, m->gstream>>>(m->W, m->V, m->S, m->order, keep, scale, cl, cr,
                                                              mm, nn, trans, right ? 1 : 0, m->site[site],
                                                              m->site[site + 1]);
    TN_HIP(hipGetLastError());
    TN_HIP(hipEventRecord(ev, m->gstream));
    TN_HIP(hipStreamWaitEvent(s, ev, 0));
    TN_HIP(hipStreamSynchronize(s));
    (void)hipEventDestroy(ev);
    m->chi[site] = keep;
    m->spec[site].resize(keep);
    for (int k = 0; k < keep; ++k) m->spec[site][k] = S[order[k]] * scale;
    m->center = right ? site + 1 : site;
  });
}

tn_status tn_mps_expect_z(tn_mps* m, double* out, void* stream) {
  return guarded([&] {
    TN_REQUIRE(m && out, TN_ERR_ARG, "null argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    move_center(m, 0, s);
    for (int i = 0; i < m->n; ++i) {
      if (i > 0) move_right(m, i - 1, s);
      site_z_kernel<<<1, 256, 0, s>>>(m->site[i], m->chil(i), m->chir(i), m->zbuf + i);
    }
    TN_HIP(hipGetLastError());
    TN_HIP(hipMemcpyAsync(out, m->zbuf, m->n * sizeof(double), hipMemcpyDeviceToHost, s));
    TN_HIP(hipStreamSynchronize(s));
  });
}

tn_status tn_mps_amplitudes(tn_mps* m, const int8_t* bits, int64_t n_bs, double* out, void* stream) {
  return guarded([&] {
    TN_REQUIRE(m && bits && out && n_bs >= 1, TN_ERR_ARG, "bad argument");
    for (int64_t i = 0; i < n_bs * m->n; ++i)
      TN_REQUIRE(bits[i] == 0 || bits[i] == 1, TN_ERR_BITS, "MPS amplitudes need 0/1 bits");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t nb = size_t(n_bs) * m->n;
    int8_t* dbits = nullptr;
    double2* dout = nullptr;
    float2** dsites = nullptr;
    int* dchi = nullptr;
    TN_HIP(hipMalloc(&dbits, nb));
    TN_HIP(hipMalloc(&dout, n_bs * sizeof(double2)));
    TN_HIP(hipMalloc(&dsites, m->n * sizeof(float2*)));
    TN_HIP(hipMalloc(&dchi, std::max(1, m->n - 1) * sizeof(int)));
    TN_HIP(hipMemcpyAsync(dbits, bits, nb, hipMemcpyHostToDevice, s));
    TN_HIP(hipMemcpyAsync(dsites, m->site.data(), m->n * sizeof(float2*), hipMemcpyHostToDevice, s));
    TN_HIP(hipMemcpyAsync(dchi, m->chi.data(), (m->n - 1) * sizeof(int), hipMemcpyHostToDevice, s));
    mps_amp_kernel<<<unsigned(n_bs), 256, 2 * m->cmax * sizeof(double2), s>>>(dsites, dchi, m->n, dbits, dout,
                                                                              m->cmax);
    TN_HIP(hipGetLastError());
    TN_HIP(hipMemcpyAsync(out, dout, n_bs * sizeof(double2), hipMemcpyDeviceToHost, s));
    TN_HIP(hipStreamSynchronize(s));
    (void)hipFree(dbits);
    (void)hipFree(dout);
    (void)hipFree(dsites);
    (void)hipFree(dchi);
  });
}

}  // extern "C"

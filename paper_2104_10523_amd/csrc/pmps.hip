// Locally-purified matrix product state (Sec. 3.4): rho = Tr_K |X><X| with
// site tensors T_i[l, s, k, r] -- virtual bonds l, r (at most d_max), the
// physical leg s and a Kraus leg k (at most k_max) summed between X and its
// conjugate.  Stored complex64 as (l, s * K + k, r): the physical bit is the
// major part of the combined leg of dimension d = 2 K.
//
//  * gates act on the physical leg as in the MPS of Sec. 3.2: one-qubit
//    gates are absorbed into the site; a two-qubit gate merges the pair on
//    the complex MFMA GEMM, mixes the gate in while converting to FP64, and
//    splits by the FP64 one-sided Jacobi SVD (only the virtual bond changes);
//  * a channel {A_a} is contracted with the physical leg, multiplying the
//    Kraus dimension by the number of operators, and the Kraus leg is then
//    compressed by an SVD along it at the orthogonality centre: with the
//    site as W[(l, s, r), (k, a)], Jacobi rotations orthogonalise the
//    columns and the kept columns (largest norms, at most k_max, s / s_max >
//    cutoff, rescaled to unit norm) are the new site (T <- U S; the right
//    factor drops out because the Kraus leg is traced);
//  * a two-qubit channel acts on the merged pair; its Kraus index joins the
//    first site's Kraus leg before the split, and that leg is compressed
//    after it;
//  * the orthogonality centre moves by FP64 Householder QR over the combined
//    (s, k) leg.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <numeric>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "linalg64.hpp"

namespace tn {
namespace {

struct PMat2 {
  double2 g[4];
};

// One-qubit gate on the physical leg of T (chil, 2K, chir).
__global__ void pmps_gate1_kernel(float2* __restrict__ T, int chil, int K, int chir, PMat2 G) {
  const int64_t n = int64_t(chil) * K * chir;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t l = i / (int64_t(K) * chir), k = (i / chir) % K, r = i % chir;
    const int64_t i0 = ((l * 2 + 0) * K + k) * chir + r, i1 = ((l * 2 + 1) * K + k) * chir + r;
    const double2 x0 = make_double2(T[i0].x, T[i0].y), x1 = make_double2(T[i1].x, T[i1].y);
    const double2 y0 = cadd(cmul(G.g[0], x0), cmul(G.g[1], x1));
    const double2 y1 = cadd(cmul(G.g[2], x0), cmul(G.g[3], x1));
    T[i0] = make_float2(float(y0.x), float(y0.y));
    T[i1] = make_float2(float(y1.x), float(y1.y));
  }
}

// Site (chil, d, chir) -> FP64 column-major X: !adj X[(l, c), r] (rows d chil);
// adj X = (T as chil x (d chir))^dagger (rows d chir).
__global__ void pmps_site_to_x_kernel(const float2* __restrict__ T, double2* __restrict__ X, int chil, int d,
                                      int chir, int adj) {
  const int64_t n = int64_t(chil) * d * chir;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const float2 a = T[i];
    if (!adj) {
      const int64_t row = i / chir, col = i % chir;
      X[col * (int64_t(d) * chil) + row] = make_double2(a.x, a.y);
    } else {
      const int64_t l = i / (int64_t(d) * chir), c = i % (int64_t(d) * chir);
      X[l * (int64_t(d) * chir) + c] = make_double2(a.x, -a.y);
    }
  }
}

// theta[(l, s1, k1), (s2, k2, r)] (complex64) mixed with nA two-qubit
// operators G_a (row-major 4 x 4, (t1 t2) x (s1 s2)) into the FP64 matrix
// M[(l, t1, k1 * nA + a), (t2, k2, r)], stored column-major in W (!trans)
// or as its conjugate transpose (trans).
__global__ void pmps_mix_kernel(const float2* __restrict__ theta, double2* __restrict__ W,
                                const double2* __restrict__ G, int nA, int chil, int K1, int K2, int chir,
                                int trans) {
  const int64_t rows = int64_t(chil) * 2 * K1 * nA, cols = int64_t(2) * K2 * chir;
  const int64_t tcols = cols;                       // theta has the same columns
  const int64_t n = rows * cols;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t row = i / cols, col = i % cols;
    const int64_t l = row / (2 * K1 * nA), t1 = (row / (K1 * nA)) % 2, ka = row % (int64_t(K1) * nA);
    const int64_t k1 = ka / nA, a = ka % nA;
    const int64_t t2 = col / (int64_t(K2) * chir), rest = col % (int64_t(K2) * chir);
    const double2* g = G + a * 16;
    double2 acc = make_double2(0, 0);
    for (int s1 = 0; s1 < 2; ++s1)
      for (int s2 = 0; s2 < 2; ++s2) {
        const float2 th = theta[((l * 2 + s1) * K1 + k1) * tcols + s2 * K2 * chir + rest];
        acc = cadd(acc, cmul(g[(t1 * 2 + t2) * 4 + s1 * 2 + s2], make_double2(th.x, th.y)));
      }
    if (!trans) W[col * rows + row] = acc;
    else W[row * cols + col] = make_double2(acc.x, -acc.y);
  }
}

// New pair from the factorisation (rows_u = rows of A_i, cols_v = columns of
// A_{i+1}); as the MPS's: !trans U = W / s, Vh = V^dagger; trans U = V,
// Vh = W^dagger / s; right: A_i = U, A_{i+1} = S Vh; left: A_i = U S.
__global__ void pmps_write_pair_kernel(const double2* __restrict__ W, const double2* __restrict__ V,
                                       const double* __restrict__ S, const int* __restrict__ order, int keep,
                                       double scale, int64_t rows_u, int64_t cols_v, int mm, int nn, int trans,
                                       int right, float2* __restrict__ Ai, float2* __restrict__ Aj) {
  const int64_t nu = rows_u * keep, nv = int64_t(keep) * cols_v;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nu + nv; i += int64_t(gridDim.x) * blockDim.x) {
    if (i < nu) {
      const int64_t row = i / keep, k = i % keep;
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
      const int64_t k = t / cols_v, col = t % cols_v;
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
      Aj[k * cols_v + col] = make_float2(float(v.x), float(v.y));
    }
  }
}

// Kraus contraction into W: column (k, a) (index k nA + a), rows (l, s, r):
// W = sum_s' A_a[s, s'] T[l, (s', k), r]; A: nA row-major 2 x 2 operators.
__global__ void pmps_kraus_to_w_kernel(const float2* __restrict__ T, double2* __restrict__ W,
                                       const double2* __restrict__ A, int nA, int chil, int K, int chir) {
  const int64_t rows = int64_t(chil) * 2 * chir, cols = int64_t(K) * nA;
  const int64_t n = rows * cols;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t col = i / rows, row = i % rows;
    const int64_t k = col / nA, a = col % nA;
    const int64_t l = row / (2 * chir), s = (row / chir) % 2, r = row % chir;
    const double2* g = A + a * 4;
    double2 acc = make_double2(0, 0);
    for (int sp = 0; sp < 2; ++sp) {
      const float2 x = T[((l * 2 + sp) * K + k) * chir + r];
      acc = cadd(acc, cmul(g[s * 2 + sp], make_double2(x.x, x.y)));
    }
    W[col * rows + row] = acc;
  }
}

// Kept Kraus columns back into the site: T[l, (s, k'), r] = W[order[k']] * scale.
__global__ void pmps_w_to_site_kernel(const double2* __restrict__ W, const int* __restrict__ order, int keep,
                                      double scale, int chil, int chir, float2* __restrict__ T) {
  const int64_t rows = int64_t(chil) * 2 * chir, n = rows * keep;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t l = i / (int64_t(2) * keep * chir), s = (i / (int64_t(keep) * chir)) % 2;
    const int64_t k = (i / chir) % keep, r = i % chir;
    const double2 w = W[int64_t(order[k]) * rows + (l * 2 + s) * chir + r];
    T[i] = make_float2(float(w.x * scale), float(w.y * scale));
  }
}

// <Z> of the centre site (chil, 2K, chir): sum |T|^2 (1 - 2s) / sum |T|^2.
__global__ __launch_bounds__(256) void pmps_site_z_kernel(const float2* __restrict__ T, int chil, int K, int chir,
                                                          double* out) {
  __shared__ double red[8];
  double z = 0, nrm = 0;
  const int64_t n = int64_t(chil) * 2 * K * chir;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const float2 a = T[i];
    const double p = double(a.x) * a.x + double(a.y) * a.y;
    const int s = int(((i / chir) % (2 * K)) / K);
    z += s ? -p : p;
    nrm += p;
  }
  z = block_sum(z, red);
  __syncthreads();
  nrm = block_sum(nrm, red);
  if (threadIdx.x == 0) *out = nrm > 0 ? z / nrm : 0.0;
}

int grid_n(int64_t n) { return int(std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096))); }

constexpr int kMaxKraus = 16;

}  // namespace
}  // namespace tn

using namespace tn;

namespace {

// ------------------------------------------------ rank-revealing pre-pass
//
// Pivoted Householder QR of W (mm x nn, column-major, mm >= nn, in place),
// stopped at the numerical rank r: step j takes the column with the largest
// remaining norm (rows j..) as pivot, and stops once that norm is below
// 1e-13 of the largest column norm (the level of the factorisation's own
// rounding).  After step j the column's rows > j hold the reflector, rd[j] =
// R[j][j], and rows j of the later columns hold R[j][c]; perm[j] is the
// input column now at j.  ctl[0] = r once found, ctl[1] = 1 then (later
// steps do nothing).

__global__ __launch_bounds__(256) void qrp_init_kernel(const double2* __restrict__ W, int mm, double* pn, int* perm,
                                                       int* ctl) {
  __shared__ double red[8];
  const double2* w = W + int64_t(blockIdx.x) * mm;
  double a = 0;
  for (int i = threadIdx.x; i < mm; i += blockDim.x) a += w[i].x * w[i].x + w[i].y * w[i].y;
  a = block_sum(a, red);
  if (threadIdx.x == 0) {
    pn[blockIdx.x] = a;
    perm[blockIdx.x] = blockIdx.x;
    if (blockIdx.x == 0) ctl[0] = ctl[1] = 0;
  }
}

__global__ __launch_bounds__(256) void qrp_pivot_kernel(double2* __restrict__ W, int mm, int nn, int j, double* pn,
                                                        int* perm, int* ctl, double* thr2) {
  if (ctl[1]) return;   // rank already found (uniform)
  __shared__ double bv[256];
  __shared__ int bi[256];
  const int t = threadIdx.x;
  double best = -1.0;
  int bc = nn;
  for (int c = j + t; c < nn; c += 256)
    if (pn[c] > best) {   // ascending c: ties keep the lowest index
      best = pn[c];
      bc = c;
    }
  bv[t] = best;
  bi[t] = bc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o && (bv[t + o] > bv[t] || (bv[t + o] == bv[t] && bi[t + o] < bi[t]))) {
      bv[t] = bv[t + o];
      bi[t] = bi[t + o];
    }
    __syncthreads();
  }
  const int p = bi[0];
  const double v = bv[0];
  if (j == 0 && t == 0) *thr2 = 1e-26 * v;          // (1e-13 of the largest column norm)^2
  const double lim = j == 0 ? 1e-26 * v : *thr2;
  if (!(v > lim)) {                                   // numerical rank reached (uniform)
    if (t == 0) {
      ctl[0] = j;
      ctl[1] = 1;
    }
    return;
  }
  if (p != j) {
    for (int i = t; i < mm; i += 256) {
      const double2 a = W[int64_t(j) * mm + i];
      W[int64_t(j) * mm + i] = W[int64_t(p) * mm + i];
      W[int64_t(p) * mm + i] = a;
    }
    if (t == 0) {
      const double x = pn[j];
      pn[j] = pn[p];
      pn[p] = x;
      const int q = perm[j];
      perm[j] = perm[p];
      perm[p] = q;
    }
  }
}

// Reflector of column j (rows j..): v = x - beta e_j, beta = -e^{i arg x_j} |x|,
// rd[j] = beta, tau[j] = 2 / |v|^2.
__global__ __launch_bounds__(256) void qrp_reflect_kernel(double2* __restrict__ W, int mm, int j, double2* rd,
                                                          double2* tau, const int* ctl) {
  if (ctl[1]) return;
  __shared__ double red[8];
  double2* x = W + int64_t(j) * mm;
  double ss = 0;
  for (int i = j + threadIdx.x; i < mm; i += blockDim.x) ss += x[i].x * x[i].x + x[i].y * x[i].y;
  ss = block_sum(ss, red);
  if (threadIdx.x == 0) {
    const double2 alpha = x[j];
    const double an = sqrt(alpha.x * alpha.x + alpha.y * alpha.y);
    const double nrm = sqrt(ss);
    const double2 ph = an > 0 ? make_double2(alpha.x / an, alpha.y / an) : make_double2(1, 0);
    const double2 beta = make_double2(-ph.x * nrm, -ph.y * nrm);
    const double2 v0 = make_double2(alpha.x - beta.x, alpha.y - beta.y);
    const double vn2 = ss - an * an + v0.x * v0.x + v0.y * v0.y;
    x[j] = v0;
    rd[j] = beta;
    tau[j] = make_double2(vn2 > 0 ? 2.0 / vn2 : 0.0, 0.0);
  }
}

// Applies reflector j to columns j+1 .. nn-1 (one wave per column, rows j..)
// and leaves each column's remaining norm (rows j+1..) in pn.
__global__ __launch_bounds__(256) void qrp_apply_kernel(double2* __restrict__ W, int mm, int nn, int j,
                                                        const double2* __restrict__ tau, double* pn, const int* ctl) {
  if (ctl[1]) return;
  const int c = j + 1 + blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (c >= nn) return;
  const double t2 = tau[j].x;
  const double2* v = W + int64_t(j) * mm;
  double2* y = W + int64_t(c) * mm;
  double dr = 0, di = 0;
  for (int i = j + lane; i < mm; i += 64) {
    const double2 a = v[i], b = y[i];
    dr += a.x * b.x + a.y * b.y;
    di += a.x * b.y - a.y * b.x;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    dr += __shfl_xor(dr, o);
    di += __shfl_xor(di, o);
  }
  const double2 f = make_double2(t2 * dr, t2 * di);
  double rest = 0;
  for (int i = j + lane; i < mm; i += 64) {
    const double2 fv = cmul(v[i], f);
    double2 b = y[i];
    b.x -= fv.x;
    b.y -= fv.y;
    y[i] = b;
    if (i > j) rest += b.x * b.x + b.y * b.y;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) rest += __shfl_xor(rest, o);
  if (lane == 0) pn[c] = rest;
}

// X = R_r^dagger (nn x r, column-major): X[c, k] = conj(R[k][c]), zero below R's diagonal.
__global__ void qrp_form_x_kernel(const double2* __restrict__ W, int mm, int nn, int r, const double2* __restrict__ rd,
                                  double2* __restrict__ X) {
  const int64_t n = int64_t(nn) * r;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x) {
    const int k = int(e / nn), c = int(e % nn);
    double2 v = make_double2(0, 0);
    if (c > k) v = W[int64_t(c) * mm + k];
    else if (c == k) v = rd[k];
    X[e] = make_double2(v.x, -v.y);
  }
}

// Right singular vectors: V[perm[c], k] = X[c, k] / S[k] (nn x r, column-major).
__global__ void qrp_right_kernel(const double2* __restrict__ X, const double* __restrict__ S,
                                 const int* __restrict__ perm, int nn, int r, double2* __restrict__ V) {
  const int64_t n = int64_t(nn) * r;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x) {
    const int k = int(e / nn), c = int(e % nn);
    const double sk = S[k];
    const double2 x = X[e];
    V[int64_t(k) * nn + perm[c]] = sk > 0 ? make_double2(x.x / sk, x.y / sk) : make_double2(0, 0);
  }
}

}  // namespace

struct tn_pmps {
  int n = 0, dmax = 0, kmax = 0, center = 0;
  std::vector<int> chi;             // bond i between sites i and i+1
  std::vector<int> K;               // Kraus dimension per site
  std::vector<float2*> site;        // capacity dmax * 2 kmax * dmax
  float2* theta = nullptr;
  float2* tmp = nullptr;
  float2* wide = nullptr;           // a first site whose Kraus leg a two-qubit channel has widened
  double2 *W = nullptr, *V = nullptr, *X = nullptr, *Q = nullptr, *R = nullptr, *tau = nullptr, *G = nullptr;
  double* S = nullptr;
  // rank-revealing pre-pass of the SVD: copy of the input, R^dagger, pivots,
  // partial column norms, R's diagonal, reflector scales, control words
  double2 *Wo = nullptr, *XR = nullptr, *rd = nullptr, *qtau = nullptr;
  double* pn = nullptr;
  int *perm = nullptr, *ctl = nullptr;
  double* qthr = nullptr;
  double* zbuf = nullptr;
  int* flag = nullptr;
  int* order = nullptr;
  void* gemm_work = nullptr;
  size_t gemm_work_bytes = 0, w_elems = 0, v_elems = 0, s_elems = 0;
  std::map<std::pair<int, int>, hipGraphExec_t> sweeps;
  std::map<std::pair<int, int>, hipGraphExec_t> sweeps_xr;   // Jacobi sweeps on XR
  std::map<std::pair<int, int>, hipGraphExec_t> qrs;
  hipStream_t gstream = nullptr;

  int chil(int i) const { return i == 0 ? 1 : chi[i - 1]; }
  int chir(int i) const { return i == n - 1 ? 1 : chi[i]; }
  int d(int i) const { return 2 * K[i]; }

  ~tn_pmps() {
    for (auto& kv : sweeps) (void)hipGraphExecDestroy(kv.second);
    for (auto& kv : sweeps_xr) (void)hipGraphExecDestroy(kv.second);
    for (auto& kv : qrs) (void)hipGraphExecDestroy(kv.second);
    for (float2* p : site) (void)hipFree(p);
    for (void* p : {(void*)theta, (void*)tmp, (void*)wide, (void*)W, (void*)V, (void*)X, (void*)Q, (void*)R, (void*)tau,
                    (void*)G, (void*)S, (void*)zbuf, (void*)flag, (void*)order, gemm_work, (void*)Wo, (void*)XR,
                    (void*)rd, (void*)qtau, (void*)pn, (void*)perm, (void*)ctl, (void*)qthr})
      if (p) (void)hipFree(p);
    if (gstream) (void)hipStreamDestroy(gstream);
  }
};

namespace {

void ensure_gstream(tn_pmps* m) {
  if (!m->gstream) TN_HIP(hipStreamCreateWithFlags(&m->gstream, hipStreamNonBlocking));
}

// Householder QR of X (rows x cols) into R and Q, captured once per shape.
void pmps_qr(tn_pmps* m, int rows, int cols, hipStream_t s) {
  const auto key = std::make_pair(rows, cols);
  auto it = m->qrs.find(key);
  if (it == m->qrs.end()) {
    ensure_gstream(m);
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
  TN_HIP(hipGraphLaunch(it->second, s));
}

void pmps_move_right(tn_pmps* m, int c, hipStream_t s) {
  const int cl = m->chil(c), cr = m->chir(c), d = m->d(c);
  const int rows = d * cl, cols = cr, k = std::min(rows, cols);
  pmps_site_to_x_kernel<<<grid_n(int64_t(cl) * d * cr), 256, 0, s>>>(m->site[c], m->X, cl, d, cr, 0);
  pmps_qr(m, rows, cols, s);
  q_to_site_kernel<<<grid_n(int64_t(rows) * k), 256, 0, s>>>(m->Q, m->site[c], rows, k, 0);
  const int64_t other = int64_t(m->d(c + 1)) * m->chir(c + 1);
  apply_r_kernel<<<grid_n(int64_t(k) * other), 256, 0, s>>>(m->R, k, cr, m->site[c + 1], m->tmp, other, 1);
  TN_HIP(hipMemcpyAsync(m->site[c + 1], m->tmp, size_t(k) * other * sizeof(float2), hipMemcpyDeviceToDevice, s));
  TN_HIP(hipGetLastError());
  m->chi[c] = k;
  m->center = c + 1;
}

void pmps_move_left(tn_pmps* m, int c, hipStream_t s) {
  const int cl = m->chil(c), cr = m->chir(c), d = m->d(c);
  const int rows = d * cr, cols = cl, k = std::min(rows, cols);
  pmps_site_to_x_kernel<<<grid_n(int64_t(cl) * d * cr), 256, 0, s>>>(m->site[c], m->X, cl, d, cr, 1);
  pmps_qr(m, rows, cols, s);
  q_to_site_kernel<<<grid_n(int64_t(rows) * k), 256, 0, s>>>(m->Q, m->site[c], rows, k, 1);
  const int64_t rowsb = int64_t(m->chil(c - 1)) * m->d(c - 1);
  apply_r_kernel<<<grid_n(rowsb * k), 256, 0, s>>>(m->R, k, cl, m->site[c - 1], m->tmp, rowsb, 0);
  TN_HIP(hipMemcpyAsync(m->site[c - 1], m->tmp, size_t(rowsb) * k * sizeof(float2), hipMemcpyDeviceToDevice, s));
  TN_HIP(hipGetLastError());
  m->chi[c - 1] = k;
  m->center = c - 1;
}

void pmps_move_center(tn_pmps* m, int target, hipStream_t s) {
  while (m->center < target) pmps_move_right(m, m->center, s);
  while (m->center > target) pmps_move_left(m, m->center, s);
}

// One-sided Jacobi sweeps on A (mm x nn) and V (nn x nn, set to I by the
// caller), the sweep captured once per shape into `graphs`, until no pair
// rotates (at most 60).  On the library stream.
void jacobi_until_converged(tn_pmps* m, double2* A, double2* V, int mm, int nn,
                            std::map<std::pair<int, int>, hipGraphExec_t>& graphs) {
  if (nn < 2) return;
  const auto key = std::make_pair(mm, nn);
  auto it = graphs.find(key);
  if (it == graphs.end()) {
    const int npad = nn + (nn & 1);
    const double tol = 2.3e-16 * double(std::max(mm, 8));
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    TN_HIP(hipStreamBeginCapture(m->gstream, hipStreamCaptureModeThreadLocal));
    flag_reset_kernel<<<1, 1, 0, m->gstream>>>(m->flag);
    for (int r = 0; r < npad - 1; ++r)
      jacobi_round_kernel<<<npad / 2, 256, 0, m->gstream>>>(A, V, mm, nn, npad, r, tol, m->flag);
    const hipError_t e = hipStreamEndCapture(m->gstream, &g);
    TN_REQUIRE(e == hipSuccess, TN_ERR_DEVICE, "graph capture of the Jacobi sweep failed");
    TN_HIP(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
    (void)hipGraphDestroy(g);
    it = graphs.emplace(key, ge).first;
  }
  int sweeps = 0, flag = 1;
  while (flag && sweeps < 60) {
    TN_HIP(hipGraphLaunch(it->second, m->gstream));
    TN_HIP(hipMemcpyAsync(&flag, m->flag, sizeof(int), hipMemcpyDeviceToHost, m->gstream));
    TN_HIP(hipStreamSynchronize(m->gstream));
    ++sweeps;
  }
}

// SVD of W (mm x nn, column-major): on return W (mm x r) holds
// U S, V (nn x r) the right singular vectors (W_in = U S V^dagger), and the
// r singular values come back on the host (and in m->S).  Narrow or wide
// matrices (nn <= 32 or nn > mm): one-sided Jacobi on W itself (r = nn).
// Tall ones with more columns first
// reveal their numerical rank by a pivoted QR, W P = Q R, then run the
// one-sided Jacobi on X = R_r^dagger (nn x r, rows of R past the rank
// dropped): the columns of X are close to orthogonal, so few sweeps do
// (the preconditioning of Drmac and Veselic), and a sweep has r - 1 rounds
// instead of nn - 1.  With X V' = U' S: V = P U' and U S = W_in V.
// Runs on the library stream after `s`.
std::vector<double> pmps_svd(tn_pmps* m, int mm, int nn, hipStream_t s) {
  TN_REQUIRE(size_t(mm) * nn <= m->w_elems && size_t(nn) * nn <= m->v_elems && size_t(nn) <= m->s_elems,
             TN_ERR_UNSUPPORTED, "PMPS factorisation larger than its buffers");
  ensure_gstream(m);
  hipEvent_t ev = nullptr;
  TN_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  TN_HIP(hipEventRecord(ev, s));
  TN_HIP(hipStreamWaitEvent(m->gstream, ev, 0));
  (void)hipEventDestroy(ev);
  hipStream_t g = m->gstream;
  int r = nn;
  bool pre = nn > 32 && mm >= nn;
  if (pre) {
    TN_HIP(hipMemcpyAsync(m->Wo, m->W, size_t(mm) * nn * sizeof(double2), hipMemcpyDeviceToDevice, g));
    qrp_init_kernel<<<nn, 256, 0, g>>>(m->W, mm, m->pn, m->perm, m->ctl);
    TN_HIP(hipGetLastError());
    for (int j0 = 0; j0 < nn; j0 += 16) {
      for (int j = j0; j < std::min(nn, j0 + 16); ++j) {
        qrp_pivot_kernel<<<1, 256, 0, g>>>(m->W, mm, nn, j, m->pn, m->perm, m->ctl, m->qthr);
        qrp_reflect_kernel<<<1, 256, 0, g>>>(m->W, mm, j, m->rd, m->qtau, m->ctl);
        if (j + 1 < nn)
          qrp_apply_kernel<<<(nn - j - 1 + 3) / 4, 256, 0, g>>>(m->W, mm, nn, j, m->qtau, m->pn, m->ctl);
      }
      TN_HIP(hipGetLastError());
      int c[2] = {0, 0};
      TN_HIP(hipMemcpyAsync(c, m->ctl, sizeof(c), hipMemcpyDeviceToHost, g));
      TN_HIP(hipStreamSynchronize(g));
      if (c[1]) {
        r = c[0];
        break;
      }
    }
    if (r == 0) {   // a zero matrix: the plain path on the saved input
      TN_HIP(hipMemcpyAsync(m->W, m->Wo, size_t(mm) * nn * sizeof(double2), hipMemcpyDeviceToDevice, g));
      pre = false;
      r = nn;
    }
  }
  std::vector<double> S(r);
  if (!pre) {
    eye_kernel<<<grid_n(int64_t(nn) * nn), 256, 0, g>>>(m->V, nn, m->flag);
    TN_HIP(hipGetLastError());
    jacobi_until_converged(m, m->W, m->V, mm, nn, m->sweeps);
    colnorm_kernel<<<nn, 256, 0, g>>>(m->W, mm, m->S);
  } else {
    qrp_form_x_kernel<<<grid_n(int64_t(nn) * r), 256, 0, g>>>(m->W, mm, nn, r, m->rd, m->XR);
    eye_kernel<<<grid_n(int64_t(r) * r), 256, 0, g>>>(m->V, r, m->flag);
    TN_HIP(hipGetLastError());
    jacobi_until_converged(m, m->XR, m->V, nn, r, m->sweeps_xr);
    colnorm_kernel<<<r, 256, 0, g>>>(m->XR, nn, m->S);
    qrp_right_kernel<<<grid_n(int64_t(nn) * r), 256, 0, g>>>(m->XR, m->S, m->perm, nn, r, m->V);
    TN_HIP(hipGetLastError());
    // U S = W_in V: row-major (r x nn) times (nn x mm) -> (r x mm), i.e. column-major mm x r
    GemmDesc gd;
    gd.M = r;
    gd.N = mm;
    gd.K = nn;
    launch_gemm64(m->V, m->Wo, m->W, gd, nullptr, g);
  }
  TN_HIP(hipGetLastError());
  TN_HIP(hipMemcpyAsync(S.data(), m->S, r * sizeof(double), hipMemcpyDeviceToHost, g));
  TN_HIP(hipStreamSynchronize(g));
  return S;
}

// Descending order (ties by index), kept count (at most cap, s / s_max >
// cutoff, at least one), discarded weight, 1 / sqrt(kept weight).
struct Trunc {
  std::vector<int> order;
  int keep = 1;
  double discarded = 0, scale = 1;
};
Trunc truncate(const std::vector<double>& S, int cap, double cutoff) {
  Trunc t;
  const int nn = int(S.size());
  t.order.resize(nn);
  std::iota(t.order.begin(), t.order.end(), 0);
  std::stable_sort(t.order.begin(), t.order.end(), [&](int a, int b) { return S[a] > S[b]; });
  const double smax = S[t.order[0]];
  int keep = 0;
  for (int k = 0; k < nn; ++k)
    if (smax > 0 && S[t.order[k]] > cutoff * smax) ++keep;
  t.keep = std::max(1, std::min(keep, cap));
  double total = 0, kept = 0;
  for (int k = 0; k < nn; ++k) {
    total += S[t.order[k]] * S[t.order[k]];
    if (k < t.keep) kept += S[t.order[k]] * S[t.order[k]];
  }
  t.discarded = total > 0 ? (total - kept) / total : 0.0;
  t.scale = kept > 0 ? 1.0 / std::sqrt(kept) : 1.0;
  return t;
}

// Merged pair with nA operators mixed in (gate: nA = 1) and split; the
// operators' index joins site's Kraus leg (K_site *= nA).  right: S goes to
// the right site (centre ends on site + 1), else to the left one.  With
// nA > 1 the first site (Kraus leg K nA) is written to m->wide, to be
// compressed into its slot by pmps_kraus.
double pmps_merge_split(tn_pmps* m, int site, const std::vector<double2>& ops, int nA, bool right, double cutoff,
                        hipStream_t s) {
  const int cl = m->chil(site), cm = m->chi[site], cr = m->chir(site + 1);
  const int K1 = m->K[site], K2 = m->K[site + 1];
  GemmDesc g;
  g.M = int64_t(cl) * 2 * K1;
  g.N = int64_t(2) * K2 * cr;
  g.K = cm;
  g.precision = TN_PREC_FP32;
  TN_REQUIRE(gemm_workspace_bytes(g) <= m->gemm_work_bytes, TN_ERR_WORKSPACE, "PMPS GEMM scratch too small");
  launch_gemm(m->site[site], m->site[site + 1], m->theta, g, m->gemm_work, nullptr, nullptr, s);
  TN_HIP(hipMemcpyAsync(m->G, ops.data(), ops.size() * sizeof(double2), hipMemcpyHostToDevice, s));
  const int64_t rows = int64_t(cl) * 2 * K1 * nA, cols = int64_t(2) * K2 * cr;
  const int trans = cols > rows ? 1 : 0;
  const int mm = int(trans ? cols : rows), nn = int(trans ? rows : cols);
  pmps_mix_kernel<<<grid_n(rows * cols), 256, 0, s>>>(m->theta, m->W, m->G, nA, cl, K1, K2, cr, trans);
  TN_HIP(hipGetLastError());
  const std::vector<double> S = pmps_svd(m, mm, nn, s);
  const Trunc t = truncate(S, m->dmax, cutoff);
  TN_HIP(hipMemcpyAsync(m->order, t.order.data(), t.keep * sizeof(int), hipMemcpyHostToDevice, m->gstream));
  pmps_write_pair_kernel<<<grid_n(rows * t.keep + int64_t(t.keep) * cols), 256, 0, m->gstream>>>(
      m->W, m->V, m->S, m->order, t.keep, t.scale, rows, cols, mm, nn, trans, right ? 1 : 0,
      nA > 1 ? m->wide : m->site[site], m->site[site + 1]);
  TN_HIP(hipGetLastError());
  hipEvent_t ev = nullptr;
  TN_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  TN_HIP(hipEventRecord(ev, m->gstream));
  TN_HIP(hipStreamWaitEvent(s, ev, 0));
  TN_HIP(hipStreamSynchronize(s));
  (void)hipEventDestroy(ev);
  m->chi[site] = t.keep;
  m->K[site] = K1 * nA;
  m->center = right ? site + 1 : site;
  return t.discarded;
}

// Channel {A_a} (nA one-qubit operators) on the centre site, read from
// `src` (its slot, or m->wide), then the Kraus leg compressed to at most
// k_max into the site's slot.  nA = 1 with the identity only compresses.
double pmps_kraus(tn_pmps* m, int site, const float2* src, const std::vector<double2>& ops, int nA, double cutoff,
                  hipStream_t s) {
  TN_REQUIRE(m->center == site, TN_ERR_ARG, "internal: Kraus leg compressed away from the centre");
  const int cl = m->chil(site), cr = m->chir(site), K = m->K[site];
  TN_HIP(hipMemcpyAsync(m->G, ops.data(), ops.size() * sizeof(double2), hipMemcpyHostToDevice, s));
  const int mm = 2 * cl * cr, nn = K * nA;
  pmps_kraus_to_w_kernel<<<grid_n(int64_t(mm) * nn), 256, 0, s>>>(src, m->W, m->G, nA, cl, K, cr);
  TN_HIP(hipGetLastError());
  const std::vector<double> S = pmps_svd(m, mm, nn, s);
  const Trunc t = truncate(S, m->kmax, cutoff);
  TN_HIP(hipMemcpyAsync(m->order, t.order.data(), t.keep * sizeof(int), hipMemcpyHostToDevice, m->gstream));
  pmps_w_to_site_kernel<<<grid_n(int64_t(mm) * t.keep), 256, 0, m->gstream>>>(m->W, m->order, t.keep, t.scale, cl,
                                                                              cr, m->site[site]);
  TN_HIP(hipGetLastError());
  hipEvent_t ev = nullptr;
  TN_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  TN_HIP(hipEventRecord(ev, m->gstream));
  TN_HIP(hipStreamWaitEvent(s, ev, 0));
  TN_HIP(hipStreamSynchronize(s));
  (void)hipEventDestroy(ev);
  m->K[site] = t.keep;
  return t.discarded;
}

std::vector<double2> read_ops(const double* re_im, int count) {
  std::vector<double2> v(count);
  for (int i = 0; i < count; ++i) v[i] = make_double2(re_im[2 * i], re_im[2 * i + 1]);
  return v;
}

}  // namespace

extern "C" {

tn_status tn_pmps_create(int32_t n_sites, int32_t d_max, int32_t k_max, void* stream, tn_pmps** out) {
  return guarded([&] {
    (void)stream;
    TN_REQUIRE(out && n_sites >= 2 && n_sites <= 4096, TN_ERR_ARG, "n_sites must be 2..4096");
    TN_REQUIRE(d_max >= 1 && d_max <= 256 && k_max >= 1 && k_max <= 64, TN_ERR_ARG,
               "d_max must be 1..256 and k_max 1..64");
    auto m = std::make_unique<tn_pmps>();
    m->n = n_sites;
    m->dmax = d_max;
    m->kmax = k_max;
    m->chi.assign(n_sites - 1, 1);
    m->K.assign(n_sites, 1);
    const size_t cap = size_t(d_max) * 2 * k_max * d_max;        // one site
    // merged pair: rows (l, s, k1 * nA) <= d_max 2 k_max 16, columns (s, k2, r) <= 2 k_max d_max
    const size_t rows = size_t(d_max) * 2 * k_max * kMaxKraus, cols = size_t(2) * k_max * d_max;
    const size_t kraus_rows = size_t(2) * d_max * d_max, kraus_cols = size_t(k_max) * kMaxKraus;
    m->w_elems = std::max(rows * cols, kraus_rows * kraus_cols);
    TN_REQUIRE(m->w_elems * sizeof(double2) <= (size_t(16) << 30), TN_ERR_UNSUPPORTED,
               "d_max and k_max need more than 16 GiB of factorisation workspace");
    const size_t nn_max = std::max({std::min(rows, cols), kraus_cols});
    m->v_elems = nn_max * nn_max;
    m->s_elems = nn_max;
    for (int i = 0; i < n_sites; ++i) {
      float2* p = nullptr;
      TN_HIP(hipMalloc(&p, cap * sizeof(float2)));
      m->site.push_back(p);
      const float2 init[2] = {make_float2(1.f, 0.f), make_float2(0.f, 0.f)};
      TN_HIP(hipMemcpy(p, init, sizeof(init), hipMemcpyHostToDevice));
    }
    TN_HIP(hipMalloc(&m->theta, size_t(d_max) * 2 * k_max * cols * sizeof(float2)));
    TN_HIP(hipMalloc(&m->tmp, cap * sizeof(float2)));
    TN_HIP(hipMalloc(&m->wide, cap * kMaxKraus * sizeof(float2)));
    TN_HIP(hipMalloc(&m->W, m->w_elems * sizeof(double2)));
    TN_HIP(hipMalloc(&m->V, m->v_elems * sizeof(double2)));
    TN_HIP(hipMalloc(&m->X, cap * sizeof(double2)));
    TN_HIP(hipMalloc(&m->Q, cap * sizeof(double2)));
    TN_HIP(hipMalloc(&m->R, cap * sizeof(double2)));
    TN_HIP(hipMalloc(&m->tau, size_t(2) * k_max * d_max * sizeof(double2)));
    TN_HIP(hipMalloc(&m->G, size_t(kMaxKraus) * 16 * sizeof(double2)));
    TN_HIP(hipMalloc(&m->S, m->s_elems * sizeof(double)));
    TN_HIP(hipMalloc(&m->zbuf, size_t(n_sites) * sizeof(double)));
    TN_HIP(hipMalloc(&m->flag, 256));
    TN_HIP(hipMalloc(&m->order, m->s_elems * sizeof(int)));
    TN_HIP(hipMalloc(&m->Wo, m->w_elems * sizeof(double2)));
    TN_HIP(hipMalloc(&m->XR, m->v_elems * sizeof(double2)));
    TN_HIP(hipMalloc(&m->rd, m->s_elems * sizeof(double2)));
    TN_HIP(hipMalloc(&m->qtau, m->s_elems * sizeof(double2)));
    TN_HIP(hipMalloc(&m->pn, m->s_elems * sizeof(double)));
    TN_HIP(hipMalloc(&m->perm, m->s_elems * sizeof(int)));
    TN_HIP(hipMalloc(&m->ctl, 256));
    TN_HIP(hipMalloc(&m->qthr, 256));
    m->gemm_work_bytes = size_t(64) << 20;
    TN_HIP(hipMalloc(&m->gemm_work, m->gemm_work_bytes));
    *out = m.release();
  });
}

tn_status tn_pmps_destroy(tn_pmps* m) {
  return guarded([&] { delete m; });
}

tn_status tn_pmps_apply_gate1(tn_pmps* m, int32_t site, const double* gate, void* stream) {
  return guarded([&] {
    TN_REQUIRE(m && gate, TN_ERR_ARG, "null argument");
    TN_REQUIRE(site >= 0 && site < m->n, TN_ERR_SITE, "site out of range");
    PMat2 G;
    for (int i = 0; i < 4; ++i) G.g[i] = make_double2(gate[2 * i], gate[2 * i + 1]);
    hipStream_t s = static_cast<hipStream_t>(stream);
    pmps_gate1_kernel<<<grid_n(int64_t(m->chil(site)) * m->K[site] * m->chir(site)), 256, 0, s>>>(
        m->site[site], m->chil(site), m->K[site], m->chir(site), G);
    TN_HIP(hipGetLastError());
  });
}

tn_status tn_pmps_apply_gate(tn_pmps* m, int32_t site, const double* gate, double cutoff, double* discarded,
                             void* stream) {
  return guarded([&] {
    TN_REQUIRE(m && gate, TN_ERR_ARG, "null argument");
    TN_REQUIRE(site >= 0 && site + 1 < m->n, TN_ERR_SITE, "site out of range (needs site + 1 < n)");
    TN_REQUIRE(cutoff >= 0, TN_ERR_ARG, "cutoff must be >= 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool right = m->center <= site;
    pmps_move_center(m, right ? site : site + 1, s);
    const double d = pmps_merge_split(m, site, read_ops(gate, 16), 1, right, cutoff, s);
    if (discarded) *discarded = d;
  });
}

tn_status tn_pmps_apply_channel(tn_pmps* m, int32_t site, int32_t n_qubits, const double* kraus, int32_t n_kraus,
                                double cutoff, double* discarded_bond, double* discarded_kraus, void* stream) {
  return guarded([&] {
    TN_REQUIRE(m && kraus, TN_ERR_ARG, "null argument");
    TN_REQUIRE(n_qubits == 1 || n_qubits == 2, TN_ERR_ARG, "channels act on 1 or 2 qubits");
    TN_REQUIRE(n_kraus >= 1 && n_kraus <= kMaxKraus, TN_ERR_ARG, "1..16 Kraus operators");
    TN_REQUIRE(site >= 0 && site + n_qubits - 1 < m->n, TN_ERR_SITE, "site out of range");
    TN_REQUIRE(cutoff >= 0, TN_ERR_ARG, "cutoff must be >= 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    double db = 0, dk = 0;
    if (n_qubits == 1) {
      pmps_move_center(m, site, s);
      dk = pmps_kraus(m, site, m->site[site], read_ops(kraus, 4 * n_kraus), n_kraus, cutoff, s);
    } else {
      const bool right = m->center <= site;
      pmps_move_center(m, right ? site : site + 1, s);
      // split with S on the first site (the centre ends there), then compress
      // its Kraus leg, which the operators' index has just joined
      db = pmps_merge_split(m, site, read_ops(kraus, 16 * n_kraus), n_kraus, false, cutoff, s);
      const double2 id[4] = {make_double2(1, 0), make_double2(0, 0), make_double2(0, 0), make_double2(1, 0)};
      dk = pmps_kraus(m, site, m->wide, std::vector<double2>(id, id + 4), 1, cutoff, s);
    }
    if (discarded_bond) *discarded_bond = db;
    if (discarded_kraus) *discarded_kraus = dk;
  });
}

tn_status tn_pmps_dims(const tn_pmps* m, int32_t* bond_dims, int32_t* kraus_dims) {
  return guarded([&] {
    TN_REQUIRE(m, TN_ERR_ARG, "null argument");
    if (bond_dims)
      for (int i = 0; i < m->n - 1; ++i) bond_dims[i] = m->chi[i];
    if (kraus_dims)
      for (int i = 0; i < m->n; ++i) kraus_dims[i] = m->K[i];
  });
}

tn_status tn_pmps_expect_z(tn_pmps* m, double* out, void* stream) {
  return guarded([&] {
    TN_REQUIRE(m && out, TN_ERR_ARG, "null argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    pmps_move_center(m, 0, s);
    for (int i = 0; i < m->n; ++i) {
      if (i > 0) pmps_move_right(m, i - 1, s);
      pmps_site_z_kernel<<<1, 256, 0, s>>>(m->site[i], m->chil(i), m->K[i], m->chir(i), m->zbuf + i);
    }
    TN_HIP(hipGetLastError());
    TN_HIP(hipMemcpyAsync(out, m->zbuf, m->n * sizeof(double), hipMemcpyDeviceToHost, s));
    TN_HIP(hipStreamSynchronize(s));
  });
}

tn_status tn_pmps_get_site(tn_pmps* m, int32_t site, double* data, int32_t* dims, void* stream) {
  return guarded([&] {
    TN_REQUIRE(m && dims, TN_ERR_ARG, "null argument");
    TN_REQUIRE(site >= 0 && site < m->n, TN_ERR_SITE, "site out of range");
    dims[0] = m->chil(site);
    dims[1] = 2;
    dims[2] = m->K[site];
    dims[3] = m->chir(site);
    if (!data) return;
    const size_t n = size_t(dims[0]) * 2 * dims[2] * dims[3];
    std::vector<float2> host(n);
    hipStream_t s = static_cast<hipStream_t>(stream);
    TN_HIP(hipMemcpyAsync(host.data(), m->site[site], n * sizeof(float2), hipMemcpyDeviceToHost, s));
    TN_HIP(hipStreamSynchronize(s));
    for (size_t i = 0; i < n; ++i) {
      data[2 * i] = host[i].x;
      data[2 * i + 1] = host[i].y;
    }
  });
}

}  // extern "C"

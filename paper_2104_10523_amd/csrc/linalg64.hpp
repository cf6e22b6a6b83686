// FP64 linear-algebra kernels shared by the MPS (Sec. 3.2) and the
// locally-purified MPS (Sec. 3.4): complex helpers, one-sided Jacobi SVD
// rounds, column norms, Householder QR steps.  Each including translation
// unit gets its own internal copy.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tn {
namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

__global__ void eye_kernel(double2* __restrict__ V, int nn, int* flag) {
  const int64_t n = int64_t(nn) * nn;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    V[i] = make_double2((i / nn) == (i % nn) ? 1.0 : 0.0, 0.0);
  if (blockIdx.x == 0 && threadIdx.x == 0) *flag = 0;
}

__global__ void flag_reset_kernel(int* flag) { *flag = 0; }

__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double t = 0;
  const int nw = blockDim.x >> 6;
  for (int k = 0; k < nw; ++k) t += red[k];
  return t;
}

// One round of the parallel (circle-method) ordering: block k rotates the
// column pair (p, q) of W (mm x nn, column-major) and of V (nn x nn).  Each
// thread keeps up to kJRowsPerThread rows of both pairs in registers, so the
// V columns are fetched together with W, and the four sums share one
// two-barrier reduction; larger matrices stream the rest from memory.
constexpr int kJRowsPerThread = 2;

__device__ __forceinline__ void rotate(double2& a, double2& b, double c, double2 sp, double2 sm) {
  const double2 sb = cmul(sm, b), sa = cmul(sp, a);
  a = make_double2(c * a.x - sb.x, c * a.y - sb.y);
  b = make_double2(sa.x + c * b.x, sa.y + c * b.y);
}

__global__ __launch_bounds__(256) void jacobi_round_kernel(double2* __restrict__ W, double2* __restrict__ V,
                                                           int mm, int nn, int npad, int round, double tol,
                                                           int* flag) {
  __shared__ double red[4][4];
  const int k = blockIdx.x, tid = threadIdx.x;
  auto idx = [&](int i) { return i == 0 ? 0 : ((i - 1 + round) % (npad - 1)) + 1; };
  int p = idx(k), q = idx(npad - 1 - k);
  if (p > q) { const int t = p; p = q; q = t; }
  if (q >= nn) return;  // pair with the padding column
  double2* wp = W + int64_t(p) * mm;
  double2* wq = W + int64_t(q) * mm;
  double2* vp = V + int64_t(p) * nn;
  double2* vq = V + int64_t(q) * nn;
  double2 ra[kJRowsPerThread], rb[kJRowsPerThread], va[kJRowsPerThread], vb[kJRowsPerThread];
#pragma unroll
  for (int u = 0; u < kJRowsPerThread; ++u) {
    const int i = tid + 256 * u;
    ra[u] = i < mm ? wp[i] : make_double2(0, 0);
    rb[u] = i < mm ? wq[i] : make_double2(0, 0);
    va[u] = i < nn ? vp[i] : make_double2(0, 0);
    vb[u] = i < nn ? vq[i] : make_double2(0, 0);
  }
  double al = 0, be = 0, gr = 0, gi = 0;
  auto accum = [&](double2 a, double2 b) {
    al += a.x * a.x + a.y * a.y;
    be += b.x * b.x + b.y * b.y;
    gr += a.x * b.x + a.y * b.y;
    gi += a.x * b.y - a.y * b.x;
  };
#pragma unroll
  for (int u = 0; u < kJRowsPerThread; ++u) accum(ra[u], rb[u]);
  for (int i = tid + 256 * kJRowsPerThread; i < mm; i += 256) accum(wp[i], wq[i]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    al += __shfl_xor(al, o);
    be += __shfl_xor(be, o);
    gr += __shfl_xor(gr, o);
    gi += __shfl_xor(gi, o);
  }
  const int w = tid >> 6;
  if ((tid & 63) == 0) {
    red[0][w] = al;
    red[1][w] = be;
    red[2][w] = gr;
    red[3][w] = gi;
  }
  __syncthreads();
  al = red[0][0] + red[0][1] + red[0][2] + red[0][3];
  be = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  gr = red[2][0] + red[2][1] + red[2][2] + red[2][3];
  gi = red[3][0] + red[3][1] + red[3][2] + red[3][3];
  const double g = sqrt(gr * gr + gi * gi);
  if (!(g > tol * sqrt(al * be)) || g == 0.0) return;
  if (tid == 0) *flag = 1;
  const double zeta = (be - al) / (2.0 * g);
  const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
  const double2 e = make_double2(gr / g, gi / g);               // e^{i phi}
  const double2 sp = make_double2(s * e.x, s * e.y);             // s e^{i phi}
  const double2 sm = make_double2(s * e.x, -s * e.y);            // s e^{-i phi}
#pragma unroll
  for (int u = 0; u < kJRowsPerThread; ++u) {
    const int i = tid + 256 * u;
    if (i < mm) {
      rotate(ra[u], rb[u], c, sp, sm);
      wp[i] = ra[u];
      wq[i] = rb[u];
    }
    if (i < nn) {
      rotate(va[u], vb[u], c, sp, sm);
      vp[i] = va[u];
      vq[i] = vb[u];
    }
  }
  for (int i = tid + 256 * kJRowsPerThread; i < mm; i += 256) {
    double2 a = wp[i], b = wq[i];
    rotate(a, b, c, sp, sm);
    wp[i] = a;
    wq[i] = b;
  }
  for (int i = tid + 256 * kJRowsPerThread; i < nn; i += 256) {
    double2 a = vp[i], b = vq[i];
    rotate(a, b, c, sp, sm);
    vp[i] = a;
    vq[i] = b;
  }
}

__global__ __launch_bounds__(256) void colnorm_kernel(const double2* __restrict__ W, int mm, double* S) {
  __shared__ double red[8];
  const double2* w = W + int64_t(blockIdx.x) * mm;
  double a = 0;
  for (int i = threadIdx.x; i < mm; i += blockDim.x) a += w[i].x * w[i].x + w[i].y * w[i].y;
  a = block_sum(a, red);
  if (threadIdx.x == 0) S[blockIdx.x] = sqrt(a);
}

__global__ void zero_kernel(double2* __restrict__ p, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    p[i] = make_double2(0, 0);
}

// Panel step of the blocked Householder QR of X (m x n, column-major, in
// place): for j = j0 .. j1-1 in order, the reflector of column j, v = x -
// beta e_j with beta = -e^{i arg x_j} |x| (rows j..), stored over the
// column, R[j][j] = beta (R: k x n row-major), tau[j] = 2 / |v|^2; then its
// application to the panel's later columns (recording R[j][c]); one
// workgroup.
__global__ __launch_bounds__(256) void hh_panel_kernel(double2* __restrict__ X, int m, int n, int j0, int j1,
                                                       double2* __restrict__ R, double2* __restrict__ tau) {
  __shared__ double red[8];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int j = j0; j < j1; ++j) {
    double2* x = X + int64_t(j) * m;
    double ss = 0;
    for (int i = j + threadIdx.x; i < m; i += blockDim.x) ss += x[i].x * x[i].x + x[i].y * x[i].y;
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
      R[int64_t(j) * n + j] = beta;
      tau[j] = make_double2(vn2 > 0 ? 2.0 / vn2 : 0.0, 0.0);
    }
    __syncthreads();   // v_j and tau_j written
    const double t2 = tau[j].x;
    for (int c = j + 1 + wave; c < j1; c += int(blockDim.x >> 6)) {
      double2* y = X + int64_t(c) * m;
      double dr = 0, di = 0;
      for (int i = j + lane; i < m; i += 64) {
        const double2 a = x[i], b = y[i];
        dr += a.x * b.x + a.y * b.y;
        di += a.x * b.y - a.y * b.x;
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        dr += __shfl_xor(dr, o);
        di += __shfl_xor(di, o);
      }
      const double2 f = make_double2(t2 * dr, t2 * di);
      for (int i = j + lane; i < m; i += 64) {
        const double2 fv = cmul(x[i], f);
        double2 b = y[i];
        b.x -= fv.x;
        b.y -= fv.y;
        y[i] = b;
        if (i == j) R[int64_t(j) * n + c] = b;
      }
    }
    __syncthreads();   // the panel's columns updated before the next reflector
  }
}

// Reflectors j0 .. j1-1 (in V, as left by hh_panel_kernel) applied to
// columns c0 .. c1-1 of Y, one wave per column: in order (reverse = 0,
// recording R[j][c] when R is given) or in reverse order (reverse = 1, for
// accumulating Q).
__global__ __launch_bounds__(256) void hh_apply_block_kernel(const double2* __restrict__ V, int m, int j0, int j1,
                                                             int reverse, const double2* __restrict__ tau,
                                                             double2* __restrict__ Y, int c0, int c1,
                                                             double2* __restrict__ R, int n) {
  const int c = c0 + blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (c >= c1) return;
  double2* y = Y + int64_t(c) * m;
  for (int t = 0; t < j1 - j0; ++t) {
    const int j = reverse ? j1 - 1 - t : j0 + t;
    const double t2 = tau[j].x;
    const double2* v = V + int64_t(j) * m;
    double dr = 0, di = 0;
    for (int i = j + lane; i < m; i += 64) {
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
    for (int i = j + lane; i < m; i += 64) {
      const double2 fv = cmul(v[i], f);
      double2 b = y[i];
      b.x -= fv.x;
      b.y -= fv.y;
      y[i] = b;
      if (R && i == j) R[int64_t(j) * n + c] = b;
    }
  }
}

// Q (m x k, column-major) = [I; 0], before the reflectors are applied.
__global__ void q_init_kernel(double2* __restrict__ Q, int m, int k) {
  const int64_t n = int64_t(m) * k;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    Q[i] = make_double2((i % m) == (i / m) ? 1.0 : 0.0, 0.0);
}

// Columns per panel of the blocked QR.
constexpr int kQrPanel = 8;

// Records the blocked Householder QR of X (rows x cols, column-major, in
// place) on s: R (k x cols row-major, k = min(rows, cols)) and Q (rows x k,
// column-major) = H_0 ... H_{k-1} [I; 0].  3 k / kQrPanel launches.
inline void record_blocked_qr(double2* X, double2* R, double2* Q, double2* tau, int rows, int cols, hipStream_t s,
                              int grid_cap) {
  const int k = rows < cols ? rows : cols;
  auto grid = [&](int64_t n) { return int(n / 256 + 1 < grid_cap ? n / 256 + 1 : grid_cap); };
  zero_kernel<<<grid(int64_t(k) * cols), 256, 0, s>>>(R, int64_t(k) * cols);
  for (int j0 = 0; j0 < k; j0 += kQrPanel) {
    const int j1 = j0 + kQrPanel < k ? j0 + kQrPanel : k;
    hh_panel_kernel<<<1, 256, 0, s>>>(X, rows, cols, j0, j1, R, tau);
    if (j1 < cols)
      hh_apply_block_kernel<<<(cols - j1 + 3) / 4, 256, 0, s>>>(X, rows, j0, j1, 0, tau, X, j1, cols, R, cols);
  }
  q_init_kernel<<<grid(int64_t(rows) * k), 256, 0, s>>>(Q, rows, k);
  for (int j1 = k; j1 > 0; j1 -= kQrPanel) {
    const int j0 = j1 - kQrPanel > 0 ? j1 - kQrPanel : 0;
    hh_apply_block_kernel<<<(k - j0 + 3) / 4, 256, 0, s>>>(X, rows, j0, j1, 1, tau, Q, j0, k, nullptr, 0);
  }
}



// Write Q (m x k, column-major) back as the site: !adj: A[(l,s), k] = Q;
// adj: A = Q^dagger (k x 2chir) -> A[k, (s,r)].
__global__ void q_to_site_kernel(const double2* __restrict__ Q, float2* __restrict__ A, int m, int k, int adj) {
  const int64_t n = int64_t(m) * k;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t r = i / k, c = i % k;
    const double2 q = Q[c * m + r];
    if (!adj) A[i] = make_float2(float(q.x), float(q.y));
    else A[c * m + r] = make_float2(float(q.x), float(-q.y));
  }
}

// Neighbour update.  right: B'[k, (s,r)] = sum_c R[k, c] B[c, (s,r)]
// (B rows = chir_old); left: B'[(l,s), k] = sum_c B[(l,s), c] conj(R[k, c]).
__global__ void apply_r_kernel(const double2* __restrict__ R, int k, int nr, const float2* __restrict__ B,
                               float2* __restrict__ Bout, int64_t other, int right) {
  const int64_t n = int64_t(k) * other;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    double2 acc = make_double2(0, 0);
    if (right) {
      const int64_t kk = i / other, col = i % other;
      for (int c = 0; c < nr; ++c) {
        const float2 b = B[int64_t(c) * other + col];
        acc = cadd(acc, cmul(R[kk * nr + c], make_double2(b.x, b.y)));
      }
      Bout[kk * other + col] = make_float2(float(acc.x), float(acc.y));
    } else {
      const int64_t row = i / k, kk = i % k;
      for (int c = 0; c < nr; ++c) {
        const float2 b = B[row * nr + c];
        acc = cadd(acc, cmulc(R[kk * nr + c], make_double2(b.x, b.y)));
      }
      Bout[row * k + kk] = make_float2(float(acc.x), float(acc.y));
    }
  }
}

}  // namespace
}  // namespace tn

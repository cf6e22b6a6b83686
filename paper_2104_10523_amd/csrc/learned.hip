// Learned contraction-order scorer: a message-passing network over the
// candidate pairwise contractions of a path-search state, trained by
// imitation of teacher paths (randomised greedy), with hand-written FP32
// forward, backward and Adam kernels.  The path it proposes is kept only when
// the exact cost model rates it no worse than greedy.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "common.hpp"
#include "handles.hpp"
#include "network.hpp"

namespace tn {
namespace {

constexpr int kF = 16;

struct StateFeat {
  std::vector<std::pair<int, int>> cand;
  std::vector<double> X;     // nc x kF
  std::vector<int> ptr, idx; // CSR line-graph neighbours, ascending
};

// Features of every candidate of a state (see include/tn.h for the list),
// from the candidate sizes the CandidateSet keeps current.
StateFeat featurize(const PathState& st, const CandidateSet& cs, int n_leaves) {
  StateFeat f;
  const auto& cl = cs.list();
  const int nc = int(cl.size());
  f.cand.resize(nc);
  std::vector<int> deg(st.sets.size(), 0);
  struct Row {
    double a, b, c, u, sig;
  };
  std::vector<Row> rows(nc);
  double smin = INFINITY, umin = INFINITY;
  for (int k = 0; k < nc; ++k) {
    const Cand& q = cl[k];
    f.cand[k] = {q.i, q.j};
    deg[q.i]++;
    deg[q.j]++;
    const double d = q.sc - q.sa - q.sb;
    const double sig = std::copysign(std::log2(1.0 + std::fabs(d)), d);
    rows[k] = {std::log2(q.sa), std::log2(q.sb), std::log2(q.sc), std::log2(q.su), sig};
    smin = std::min(smin, sig);
    umin = std::min(umin, rows[k].u);
  }
  f.X.assign(size_t(nc) * kF, 0.0);
  for (int k = 0; k < nc; ++k) {
    const Row& r = rows[k];
    const auto [i, j] = f.cand[k];
    double* x = &f.X[size_t(k) * kF];
    x[0] = r.a / 32;
    x[1] = r.b / 32;
    x[2] = r.c / 32;
    x[3] = r.u / 32;
    x[4] = (r.a + r.b - r.u) / 8;
    x[5] = (r.c - std::max(r.a, r.b)) / 8;
    x[6] = r.sig / 32;
    x[7] = (r.sig - smin) / 8;
    x[8] = r.sig == smin ? 1.0 : 0.0;
    x[9] = double(st.n_alive) / double(n_leaves);
    x[10] = std::log2(1.0 + nc) / 16;
    x[11] = (r.u - umin) / 8;
    x[12] = double(deg[i]) / 16;
    x[13] = double(deg[j]) / 16;
    x[14] = cl[k].shared == 0 ? 1.0 : 0.0;
    x[15] = 1.0;
  }
  std::vector<std::vector<int>> by_t(st.sets.size());
  for (int k = 0; k < nc; ++k) {
    by_t[f.cand[k].first].push_back(k);
    by_t[f.cand[k].second].push_back(k);
  }
  f.ptr.assign(nc + 1, 0);
  for (int k = 0; k < nc; ++k) {
    std::vector<int> nb = union_of(by_t[f.cand[k].first], by_t[f.cand[k].second]);
    for (int v : nb)
      if (v != k) f.idx.push_back(v);
    f.ptr[k + 1] = int(f.idx.size());
  }
  return f;
}

// ------------------------------------------------------------------ kernels

using floatx16 = __attribute__((__vector_size__(16 * sizeof(float)))) float;

// C[M,N] = op(A) op(B) (+ C) (+ bias[n]) (relu); op(A)[m][k] = transA ?
// A[k*lda+m] : A[m*lda+k]; op(B)[k][n] = transB ? B[n*ldb+k] : B[k*ldb+n].
// FP32 matrix cores: a 64 x 64 tile per block of four waves, each wave one
// 32 x 32 accumulator of v_mfma_f32_32x32x2f32 (lane l feeds A row l % 32
// and B column l % 32 at k offset l / 32; accumulator register r holds row
// 8 (r / 4) + 4 (l / 32) + r % 4 of column l % 32).  K is staged through
// LDS 16 at a time.  With gridDim.z > 1 block z covers k in [z kchunk,
// (z + 1) kchunk) and stores its partial tile at C + z M ldc (no bias or
// relu then); splitk_reduce_kernel sums the partials in a fixed order, so
// results do not depend on block scheduling.
__global__ __launch_bounds__(256) void sgemm_mfma_kernel(const float* __restrict__ A, const float* __restrict__ B,
                                                         float* __restrict__ C, int M, int N, int K, int lda, int ldb,
                                                         int ldc, int transA, int transB, int accumulate,
                                                         const float* __restrict__ bias, int relu, int kchunk) {
  __shared__ float As[64][17];   // [m][k]: a wave's 32 rows fall on distinct banks
  __shared__ float Bs[16][65];   // [k][n]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 31, lh = lane >> 5;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
  floatx16 acc = {};
  for (int k0 = kb; k0 < ke; k0 += 16) {
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      // the index fastest in memory runs fastest over threads
      int mm = transA ? (e & 63) : (e >> 4), kk = transA ? (e >> 6) : (e & 15);
      int m = m0 + mm, k = k0 + kk;
      As[mm][kk] = (m < M && k < ke) ? (transA ? A[int64_t(k) * lda + m] : A[int64_t(m) * lda + k]) : 0.f;
      const int nn = transB ? (e >> 4) : (e & 63);
      kk = transB ? (e & 15) : (e >> 6);
      const int n = n0 + nn;
      k = k0 + kk;
      Bs[kk][nn] = (n < N && k < ke) ? (transB ? B[int64_t(n) * ldb + k] : B[int64_t(k) * ldb + n]) : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; kk += 2)
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(As[wm + li][kk + lh], Bs[kk + lh][wn + li], acc, 0, 0, 0);
    __syncthreads();
  }
  const int n = n0 + wn + li;
  if (n >= N) return;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int m = m0 + wm + 8 * (r >> 2) + 4 * lh + (r & 3);
    if (m >= M) continue;
    float* c = C + (int64_t(blockIdx.z) * M + m) * ldc + n;
    if (gridDim.z > 1) {
      *c = acc[r];
    } else {
      float v = acc[r];
      if (accumulate) v += *c;
      if (bias) v += bias[n];
      if (relu) v = fmaxf(v, 0.f);
      *c = v;
    }
  }
}

// C[m][n] = (accumulate ? C[m][n] : 0) + sum over z = 0 .. Z-1, in order, of
// part[z][m][n] (part dense, M x N per z).
__global__ void splitk_reduce_kernel(const float* __restrict__ part, int Z, int M, int N, float* __restrict__ C,
                                     int ldc, int accumulate) {
  const int64_t n = int64_t(M) * N;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x) {
    float s = 0.f;
    for (int z = 0; z < Z; ++z) s += part[int64_t(z) * n + e];
    float* c = C + (e / N) * ldc + e % N;
    *c = accumulate ? *c + s : s;
  }
}

__global__ void zero_rows_kernel(float* __restrict__ C, int M, int N, int ldc) {
  const int64_t n = int64_t(M) * N;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x)
    C[(e / N) * ldc + e % N] = 0.f;
}

// forward (transpose = 0): out[i] = mean_{j in nbr(i)} h[j];
// adjoint (transpose = 1): out[j] = sum_{i in nbr(j)} h[i] / deg(i)
// (the neighbour relation is symmetric).
__global__ void agg_kernel(const float* __restrict__ h, const int* __restrict__ ptr, const int* __restrict__ idx,
                           float* __restrict__ out, int N, int H, int transpose) {
  const int64_t n = int64_t(N) * H;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x) {
    const int i = int(e / H), c = int(e % H);
    const int b = ptr[i], t = ptr[i + 1];
    float s = 0.f;
    if (!transpose) {
      for (int q = b; q < t; ++q) s += h[int64_t(idx[q]) * H + c];
      if (t > b) s /= float(t - b);
    } else {
      for (int q = b; q < t; ++q) {
        const int j = idx[q];
        s += h[int64_t(j) * H + c] / float(ptr[j + 1] - ptr[j]);
      }
    }
    out[e] = s;
  }
}

__global__ void mask_kernel(float* __restrict__ g, const float* __restrict__ h, int64_t n) {
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x)
    if (!(h[e] > 0.f)) g[e] = 0.f;
}

// part[b][c] = sum_i G[i][c] over the rows [b R, (b + 1) R) of block b.
__global__ void colsum_kernel(const float* __restrict__ G, float* __restrict__ part, int N, int H, int R) {
  const int i0 = blockIdx.x * R, i1 = min(N, i0 + R);
  for (int c = threadIdx.x; c < H; c += blockDim.x) {
    float s = 0.f;
    for (int i = i0; i < i1; ++i) s += G[int64_t(i) * H + c];
    part[int64_t(blockIdx.x) * H + c] = s;
  }
}

// Softmax cross-entropy per segment; ds = (softmax - onehot) * scale.
__global__ void ce_kernel(const float* __restrict__ s, const int* __restrict__ seg, const int* __restrict__ label,
                          int S, float scale, float* __restrict__ ds, float* __restrict__ loss) {
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < S; q += gridDim.x * blockDim.x) {
    const int b = seg[q], t = seg[q + 1];
    float mx = -INFINITY;
    for (int i = b; i < t; ++i) mx = fmaxf(mx, s[i]);
    double z = 0;
    for (int i = b; i < t; ++i) z += exp(double(s[i] - mx));
    for (int i = b; i < t; ++i) {
      const double p = exp(double(s[i] - mx)) / z;
      ds[i] = float((p - (i - b == label[q] ? 1.0 : 0.0)) * scale);
    }
    loss[q] = float(double(mx) + log(z) - double(s[b + label[q]]));
  }
}

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t n, float lr, float bc1, float bc2) {
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x) {
    const float gg = g[e];
    const float mm = 0.9f * m[e] + 0.1f * gg;
    const float vv = 0.999f * v[e] + 0.001f * gg * gg;
    m[e] = mm;
    v[e] = vv;
    p[e] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + 1e-8f);
  }
}

int blocks_for(int64_t n) { return int(std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096))); }

}  // namespace
}  // namespace tn

using namespace tn;

struct tn_model {
  int H = 0, L = 0;
  int64_t np = 0;
  int dev = 0;
  float *P = nullptr, *G = nullptr, *Mo = nullptr, *Vo = nullptr;
  float* part = nullptr;   // split-K and column-sum partials (kPartFloats)
  int64_t adam_t = 0;
  // activations (grown on demand)
  int cap_nodes = 0, cap_nbr = 0, cap_seg = 0;
  float *X = nullptr, *work = nullptr, *s = nullptr, *ds = nullptr, *loss = nullptr;
  int *ptr = nullptr, *idx = nullptr, *seg = nullptr, *lab = nullptr;
  // training set (host)
  struct Sample {
    std::vector<float> X;
    std::vector<int> ptr, idx;
    int label;
  };
  std::vector<Sample> data;

  // parameter offsets
  int64_t off_W0() const { return 0; }
  int64_t off_b0() const { return int64_t(kF) * H; }
  int64_t off_layer(int l) const { return off_b0() + H + int64_t(l) * (2 * H * H + H); }
  int64_t off_Wh() const { return off_layer(L); }
  int64_t off_bh() const { return off_Wh() + int64_t(H) * H; }
  int64_t off_wo() const { return off_bh() + H; }
  int64_t off_bo() const { return off_wo() + H; }

  // per-node activation buffers inside `work`: h_0..h_L, m_0..m_{L-1}, hh, t1, t2
  float* hbuf(int l) { return work + int64_t(l) * cap_nodes * H; }
  float* mbuf(int l) { return work + int64_t(L + 1 + l) * cap_nodes * H; }
  float* hh() { return work + int64_t(2 * L + 1) * cap_nodes * H; }
  float* t1() { return work + int64_t(2 * L + 2) * cap_nodes * H; }
  float* t2() { return work + int64_t(2 * L + 3) * cap_nodes * H; }

  void reserve(int nodes, int nbr, int segs) {
    if (nodes > cap_nodes) {
      (void)hipFree(X);
      (void)hipFree(work);
      (void)hipFree(s);
      (void)hipFree(ds);
      cap_nodes = std::max(nodes, 1024);
      TN_HIP(hipMalloc(&X, size_t(cap_nodes) * kF * sizeof(float)));
      TN_HIP(hipMalloc(&work, size_t(2 * L + 4) * cap_nodes * H * sizeof(float)));
      TN_HIP(hipMalloc(&s, size_t(cap_nodes) * sizeof(float)));
      TN_HIP(hipMalloc(&ds, size_t(cap_nodes) * sizeof(float)));
      (void)hipFree(ptr);
      TN_HIP(hipMalloc(&ptr, size_t(cap_nodes + 1) * sizeof(int)));
    }
    if (nbr > cap_nbr) {
      (void)hipFree(idx);
      cap_nbr = std::max(nbr, 4096);
      TN_HIP(hipMalloc(&idx, size_t(cap_nbr) * sizeof(int)));
    }
    if (segs > cap_seg) {
      (void)hipFree(seg);
      (void)hipFree(lab);
      (void)hipFree(loss);
      cap_seg = std::max(segs, 64);
      TN_HIP(hipMalloc(&seg, size_t(cap_seg + 1) * sizeof(int)));
      TN_HIP(hipMalloc(&lab, size_t(cap_seg) * sizeof(int)));
      TN_HIP(hipMalloc(&loss, size_t(cap_seg) * sizeof(float)));
    }
  }

  ~tn_model() {
    for (void* p : {(void*)P, (void*)G, (void*)Mo, (void*)Vo, (void*)part, (void*)X, (void*)work, (void*)s, (void*)ds,
                    (void*)loss, (void*)ptr, (void*)idx, (void*)seg, (void*)lab})
      if (p) (void)hipFree(p);
  }
};

namespace {

// Split-K partials and column-sum partials: ksplit <= 512 / tiles bounds a
// GEMM's partials by 512 tiles of 64 x 64; column sums take <= 1024 x 256.
constexpr int64_t kPartFloats = int64_t(512) * 64 * 64;

void gemm(float* part, const float* A, const float* B, float* C, int M, int N, int K, int lda, int ldb, int ldc,
          int tA, int tB, int acc, const float* bias, int relu, hipStream_t s) {
  const int tiles = ((M + 63) / 64) * ((N + 63) / 64);
  int ksplit = 1, kchunk = std::max(K, 1);
  // long-K products with few output tiles (weight gradients: K = nodes)
  // split K over blocks so that the chip fills
  if (!bias && !relu && tiles < 256 && K > 2048) {
    ksplit = std::min((K + 1023) / 1024, std::max(1, 512 / tiles));
    kchunk = ((K + ksplit - 1) / ksplit + 15) / 16 * 16;
    ksplit = (K + kchunk - 1) / kchunk;
  }
  dim3 grid((N + 63) / 64, (M + 63) / 64, ksplit);
  if (ksplit > 1) {
    TN_REQUIRE(int64_t(M) * N * ksplit <= kPartFloats, TN_ERR_ARG, "split-K partials exceed their buffer");
    sgemm_mfma_kernel<<<grid, 256, 0, s>>>(A, B, part, M, N, K, lda, ldb, N, tA, tB, 0, nullptr, 0, kchunk);
    TN_HIP(hipGetLastError());
    splitk_reduce_kernel<<<blocks_for(int64_t(M) * N), 256, 0, s>>>(part, ksplit, M, N, C, ldc, acc);
  } else {
    sgemm_mfma_kernel<<<grid, 256, 0, s>>>(A, B, C, M, N, K, lda, ldb, ldc, tA, tB, acc, bias, relu, kchunk);
  }
  TN_HIP(hipGetLastError());
}

// out[0..H) = column sums of G[N][H]
void colsum(float* part, const float* G, float* out, int N, int H, hipStream_t s) {
  if (N <= 0) {
    zero_rows_kernel<<<1, 256, 0, s>>>(out, 1, H, H);
    return;
  }
  const int nb = std::max(1, std::min((N + 63) / 64, 1024));
  const int R = (N + nb - 1) / nb;
  const int blocks = (N + R - 1) / R;
  TN_REQUIRE(int64_t(blocks) * H <= kPartFloats, TN_ERR_ARG, "column-sum partials exceed their buffer");
  colsum_kernel<<<blocks, std::min(256, std::max(64, (H + 63) / 64 * 64)), 0, s>>>(G, part, N, H, R);
  splitk_reduce_kernel<<<blocks_for(H), 256, 0, s>>>(part, blocks, 1, H, out, H, 0);
}

// Forward over `nodes` nodes already uploaded (X, ptr, idx); scores into m->s.
void forward(tn_model* m, int nodes, hipStream_t st) {
  const int H = m->H;
  const float* P = m->P;
  gemm(m->part, m->X, P + m->off_W0(), m->hbuf(0), nodes, H, kF, kF, H, H, 0, 0, 0, P + m->off_b0(), 1, st);
  for (int l = 0; l < m->L; ++l) {
    const int64_t o = m->off_layer(l);
    agg_kernel<<<blocks_for(int64_t(nodes) * H), 256, 0, st>>>(m->hbuf(l), m->ptr, m->idx, m->mbuf(l), nodes, H, 0);
    gemm(m->part, m->hbuf(l), P + o, m->hbuf(l + 1), nodes, H, H, H, H, H, 0, 0, 0, nullptr, 0, st);
    gemm(m->part, m->mbuf(l), P + o + int64_t(H) * H, m->hbuf(l + 1), nodes, H, H, H, H, H, 0, 0, 1,
         P + o + 2 * int64_t(H) * H, 1, st);
  }
  gemm(m->part, m->hbuf(m->L), P + m->off_Wh(), m->hh(), nodes, H, H, H, H, H, 0, 0, 0, P + m->off_bh(), 1, st);
  gemm(m->part, m->hh(), P + m->off_wo(), m->s, nodes, 1, H, H, 1, 1, 0, 0, 0, P + m->off_bo(), 0, st);
}

// Backward from m->ds; gradients into m->G (overwritten).
void backward(tn_model* m, int nodes, hipStream_t st) {
  const int H = m->H;
  const float* P = m->P;
  float* G = m->G;
  // head
  gemm(m->part, m->hh(), m->ds, G + m->off_wo(), H, 1, nodes, H, 1, 1, 1, 0, 0, nullptr, 0, st);
  colsum(m->part, m->ds, G + m->off_bo(), nodes, 1, st);
  gemm(m->part, m->ds, P + m->off_wo(), m->t1(), nodes, H, 1, 1, H, H, 0, 0, 0, nullptr, 0, st);   // dhh
  mask_kernel<<<blocks_for(int64_t(nodes) * H), 256, 0, st>>>(m->t1(), m->hh(), int64_t(nodes) * H);
  gemm(m->part, m->hbuf(m->L), m->t1(), G + m->off_Wh(), H, H, nodes, H, H, H, 1, 0, 0, nullptr, 0, st);
  colsum(m->part, m->t1(), G + m->off_bh(), nodes, H, st);
  gemm(m->part, m->t1(), P + m->off_Wh(), m->t2(), nodes, H, H, H, H, H, 0, 1, 0, nullptr, 0, st);   // dh_L
  for (int l = m->L - 1; l >= 0; --l) {
    const int64_t o = m->off_layer(l);
    // dz = dh_{l+1} masked, kept in t2
    mask_kernel<<<blocks_for(int64_t(nodes) * H), 256, 0, st>>>(m->t2(), m->hbuf(l + 1), int64_t(nodes) * H);
    gemm(m->part, m->hbuf(l), m->t2(), G + o, H, H, nodes, H, H, H, 1, 0, 0, nullptr, 0, st);
    gemm(m->part, m->mbuf(l), m->t2(), G + o + int64_t(H) * H, H, H, nodes, H, H, H, 1, 0, 0, nullptr, 0, st);
    colsum(m->part, m->t2(), G + o + 2 * int64_t(H) * H, nodes, H, st);
    // dh_l = dz Ws^T + agg^T(dz Wn^T): t1 = dz Wn^T, then mbuf(l) <- agg^T(t1)
    gemm(m->part, m->t2(), P + o + int64_t(H) * H, m->t1(), nodes, H, H, H, H, H, 0, 1, 0, nullptr, 0, st);
    agg_kernel<<<blocks_for(int64_t(nodes) * H), 256, 0, st>>>(m->t1(), m->ptr, m->idx, m->mbuf(l), nodes, H, 1);
    gemm(m->part, m->t2(), P + o, m->mbuf(l), nodes, H, H, H, H, H, 0, 1, 1, nullptr, 0, st);
    TN_HIP(hipMemcpyAsync(m->t2(), m->mbuf(l), size_t(nodes) * H * sizeof(float), hipMemcpyDeviceToDevice, st));
  }
  mask_kernel<<<blocks_for(int64_t(nodes) * H), 256, 0, st>>>(m->t2(), m->hbuf(0), int64_t(nodes) * H);
  gemm(m->part, m->X, m->t2(), G + m->off_W0(), kF, H, nodes, kF, H, H, 1, 0, 0, nullptr, 0, st);
  colsum(m->part, m->t2(), G + m->off_b0(), nodes, H, st);
  TN_HIP(hipGetLastError());
}

void upload_batch(tn_model* m, const std::vector<const tn_model::Sample*>& batch, int* nodes_out, hipStream_t st) {
  int nodes = 0, nbr = 0;
  for (auto* b : batch) {
    nodes += int(b->ptr.size()) - 1;
    nbr += int(b->idx.size());
  }
  m->reserve(nodes, nbr, int(batch.size()));
  // concatenate: node ids and neighbour offsets of each state are shifted
  std::vector<float> X;
  std::vector<int> ptr{0}, idx, seg{0}, lab;
  X.reserve(size_t(nodes) * kF);
  int base = 0, run = 0;
  for (auto* b : batch) {
    const int nc = int(b->ptr.size()) - 1;
    X.insert(X.end(), b->X.begin(), b->X.end());
    for (int k = 0; k < nc; ++k) ptr.push_back(run + b->ptr[k + 1]);
    for (int q : b->idx) idx.push_back(q + base);
    run += b->ptr[nc];
    base += nc;
    seg.push_back(base);
    lab.push_back(b->label);
  }
  TN_HIP(hipMemcpyAsync(m->X, X.data(), X.size() * sizeof(float), hipMemcpyHostToDevice, st));
  TN_HIP(hipMemcpyAsync(m->ptr, ptr.data(), ptr.size() * sizeof(int), hipMemcpyHostToDevice, st));
  if (!idx.empty()) TN_HIP(hipMemcpyAsync(m->idx, idx.data(), idx.size() * sizeof(int), hipMemcpyHostToDevice, st));
  TN_HIP(hipMemcpyAsync(m->seg, seg.data(), seg.size() * sizeof(int), hipMemcpyHostToDevice, st));
  TN_HIP(hipMemcpyAsync(m->lab, lab.data(), lab.size() * sizeof(int), hipMemcpyHostToDevice, st));
  TN_HIP(hipStreamSynchronize(st));   // host staging vectors go out of scope
  *nodes_out = nodes;
}

tn_model::Sample make_sample(const StateFeat& f, int label) {
  tn_model::Sample s;
  s.X.assign(f.X.begin(), f.X.end());
  s.ptr = f.ptr;
  s.idx = f.idx;
  s.label = label;
  return s;
}

}  // namespace

namespace tn {

std::vector<std::pair<int, int>> learned_path_with_fallback(const tn_model* mc, const PathProblem& pr,
                                                            int rescore_every, int* algo_used) {
  const int r = std::max(1, rescore_every);
  tn_model* m = const_cast<tn_model*>(mc);
  hipStream_t st = nullptr;
  TN_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  std::vector<std::pair<int, int>> path;
  try {
    PathState state(pr, {});
    CandidateSet cs(state);
    const int n_leaves = int(pr.leaves.size());
    while (state.n_alive > 1) {
      const StateFeat f = featurize(state, cs, n_leaves);
      const int nc = int(f.cand.size());
      tn_model::Sample smp = make_sample(f, 0);
      int nodes = 0;
      upload_batch(m, {&smp}, &nodes, st);
      forward(m, nodes, st);
      std::vector<float> sc(nc);
      TN_HIP(hipMemcpyAsync(sc.data(), m->s, nc * sizeof(float), hipMemcpyDeviceToHost, st));
      TN_HIP(hipStreamSynchronize(st));
      // Up to r merges per scoring, best score first, no tensor in two of
      // them: a merge changes no other candidate whose tensors it avoids.
      std::vector<int> order(nc);
      for (int k = 0; k < nc; ++k) order[k] = k;
      std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return sc[a] > sc[b]; });
      std::vector<int> used;
      for (int k : order) {
        if (int(used.size()) >= 2 * r) break;
        const auto pq = f.cand[k];
        if (std::find(used.begin(), used.end(), pq.first) != used.end() ||
            std::find(used.begin(), used.end(), pq.second) != used.end())
          continue;
        used.push_back(pq.first);
        used.push_back(pq.second);
        path.push_back(pq);
        cs.merge(state, pq.first, pq.second);
      }
    }
  } catch (...) {
    (void)hipStreamDestroy(st);
    throw;
  }
  (void)hipStreamDestroy(st);
  auto greedy = greedy_path(pr, nullptr, 1.0);
  const PathStats sl = path_stats(pr, path, {}), sg = path_stats(pr, greedy, {});
  if (sl.flops < sg.flops || (sl.flops == sg.flops && sl.peak <= sg.peak)) {
    *algo_used = TN_PATH_LEARNED;
    return path;
  }
  *algo_used = TN_PATH_GREEDY;
  return greedy;
}

}  // namespace tn

extern "C" {

tn_status tn_model_create(int32_t hidden, int32_t layers, tn_model** out) {
  return guarded([&] {
    TN_REQUIRE(out && hidden >= 1 && hidden <= 256 && layers >= 0 && layers <= 8, TN_ERR_ARG,
               "hidden must be 1..256 and layers 0..8");
    auto m = std::make_unique<tn_model>();
    m->H = hidden;
    m->L = layers;
    m->np = m->off_bo() + 1;
    TN_HIP(hipGetDevice(&m->dev));
    for (float** p : {&m->P, &m->G, &m->Mo, &m->Vo}) {
      TN_HIP(hipMalloc(p, size_t(m->np) * sizeof(float)));
      TN_HIP(hipMemset(*p, 0, size_t(m->np) * sizeof(float)));
    }
    TN_HIP(hipMalloc(&m->part, size_t(kPartFloats) * sizeof(float)));
    *out = m.release();
  });
}

tn_status tn_model_destroy(tn_model* m) {
  return guarded([&] { delete m; });
}

tn_status tn_model_n_params(const tn_model* m, int64_t* n) {
  return guarded([&] {
    TN_REQUIRE(m && n, TN_ERR_ARG, "null argument");
    *n = m->np;
  });
}

tn_status tn_model_set_params(tn_model* m, const double* theta) {
  return guarded([&] {
    TN_REQUIRE(m && theta, TN_ERR_ARG, "null argument");
    std::vector<float> h(theta, theta + m->np);
    TN_HIP(hipMemcpy(m->P, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice));
    TN_HIP(hipMemset(m->Mo, 0, size_t(m->np) * sizeof(float)));
    TN_HIP(hipMemset(m->Vo, 0, size_t(m->np) * sizeof(float)));
    m->adam_t = 0;
  });
}

tn_status tn_model_get_params(const tn_model* m, double* theta) {
  return guarded([&] {
    TN_REQUIRE(m && theta, TN_ERR_ARG, "null argument");
    std::vector<float> h(m->np);
    TN_HIP(hipMemcpy(h.data(), m->P, h.size() * sizeof(float), hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < m->np; ++i) theta[i] = h[i];
  });
}

tn_status tn_model_state_features(const tn_network* n, const int8_t* open_mask, const int32_t* pairs,
                                  int32_t n_prefix, int32_t* n_cands, int32_t* n_nbr, int32_t* cand, double* X,
                                  int32_t* nbr_ptr, int32_t* nbr_idx) {
  return guarded([&] {
    TN_REQUIRE(n && (pairs || n_prefix == 0) && n_prefix >= 0, TN_ERR_ARG, "bad argument");
    std::vector<char> open_q(n->net.n_qubits, 0);
    if (open_mask)
      for (int q = 0; q < n->net.n_qubits; ++q) open_q[q] = open_mask[q] ? 1 : 0;
    const PathProblem pr = make_problem(n->net, open_q);
    PathState st(pr, {});
    for (int t = 0; t < n_prefix; ++t) {
      const int i = pairs[2 * t], j = pairs[2 * t + 1];
      TN_REQUIRE(i >= 0 && j >= 0 && i < int(st.sets.size()) && j < int(st.sets.size()) && i != j &&
                     st.alive[i] && st.alive[j],
                 TN_ERR_ARG, "prefix step uses a consumed or unknown tensor");
      st.merge(i, j);
    }
    TN_REQUIRE(st.n_alive > 1, TN_ERR_STATE, "no candidates left after the prefix");
    const StateFeat f = featurize(st, CandidateSet(st), int(pr.leaves.size()));
    const int nc = int(f.cand.size());
    if (n_cands) *n_cands = nc;
    if (n_nbr) *n_nbr = int(f.idx.size());
    if (cand)
      for (int k = 0; k < nc; ++k) {
        cand[2 * k] = f.cand[k].first;
        cand[2 * k + 1] = f.cand[k].second;
      }
    if (X) std::copy(f.X.begin(), f.X.end(), X);
    if (nbr_ptr) std::copy(f.ptr.begin(), f.ptr.end(), nbr_ptr);
    if (nbr_idx) std::copy(f.idx.begin(), f.idx.end(), nbr_idx);
  });
}

tn_status tn_model_loss_grad(tn_model* m, int32_t n_cands, const double* X, const int32_t* nbr_ptr,
                             const int32_t* nbr_idx, int32_t label, double* loss, double* grad, double* scores,
                             void* stream) {
  return guarded([&] {
    TN_REQUIRE(m && X && nbr_ptr && n_cands >= 1 && label >= 0 && label < n_cands, TN_ERR_ARG, "bad argument");
    TN_REQUIRE(nbr_ptr[0] == 0 && (nbr_ptr[n_cands] == 0 || nbr_idx), TN_ERR_ARG, "bad neighbour lists");
    for (int i = 0; i < n_cands; ++i) TN_REQUIRE(nbr_ptr[i + 1] >= nbr_ptr[i], TN_ERR_ARG, "bad neighbour lists");
    for (int q = 0; q < nbr_ptr[n_cands]; ++q)
      TN_REQUIRE(nbr_idx[q] >= 0 && nbr_idx[q] < n_cands, TN_ERR_ARG, "neighbour index out of range");
    hipStream_t st = static_cast<hipStream_t>(stream);
    tn_model::Sample smp;
    smp.X.assign(X, X + size_t(n_cands) * kF);
    smp.ptr.assign(nbr_ptr, nbr_ptr + n_cands + 1);
    smp.idx.assign(nbr_idx, nbr_idx + nbr_ptr[n_cands]);
    smp.label = label;
    int nodes = 0;
    upload_batch(m, {&smp}, &nodes, st);
    forward(m, nodes, st);
    ce_kernel<<<1, 64, 0, st>>>(m->s, m->seg, m->lab, 1, 1.0f, m->ds, m->loss);
    backward(m, nodes, st);
    float l = 0;
    TN_HIP(hipMemcpyAsync(&l, m->loss, sizeof(float), hipMemcpyDeviceToHost, st));
    std::vector<float> g(m->np), sc(n_cands);
    TN_HIP(hipMemcpyAsync(g.data(), m->G, g.size() * sizeof(float), hipMemcpyDeviceToHost, st));
    TN_HIP(hipMemcpyAsync(sc.data(), m->s, sc.size() * sizeof(float), hipMemcpyDeviceToHost, st));
    TN_HIP(hipStreamSynchronize(st));
    if (loss) *loss = l;
    if (grad)
      for (int64_t i = 0; i < m->np; ++i) grad[i] = g[i];
    if (scores)
      for (int i = 0; i < n_cands; ++i) scores[i] = sc[i];
  });
}

tn_status tn_model_add_teacher(tn_model* m, const tn_network* n, const int8_t* open_mask, const int32_t* pairs,
                               int32_t n_steps, int32_t stride) {
  return guarded([&] {
    TN_REQUIRE(m && n && pairs && n_steps >= 1 && stride >= 1, TN_ERR_ARG, "bad argument");
    std::vector<char> open_q(n->net.n_qubits, 0);
    if (open_mask)
      for (int q = 0; q < n->net.n_qubits; ++q) open_q[q] = open_mask[q] ? 1 : 0;
    const PathProblem pr = make_problem(n->net, open_q);
    PathState st(pr, {});
    CandidateSet cs(st);
    for (int t = 0; t < n_steps; ++t) {
      const std::pair<int, int> step{pairs[2 * t], pairs[2 * t + 1]};
      if (t % stride == 0 && st.n_alive > 2) {
        const StateFeat f = featurize(st, cs, int(pr.leaves.size()));
        const auto it = std::find(f.cand.begin(), f.cand.end(), step);
        TN_REQUIRE(it != f.cand.end(), TN_ERR_ARG, "teacher step is not a candidate");
        m->data.push_back(make_sample(f, int(it - f.cand.begin())));
      }
      TN_REQUIRE(step.first >= 0 && step.second >= 0 && step.first < int(st.sets.size()) &&
                     step.second < int(st.sets.size()) && st.alive[step.first] && st.alive[step.second],
                 TN_ERR_ARG, "teacher path uses a consumed or unknown tensor");
      cs.merge(st, step.first, step.second);
    }
  });
}

tn_status tn_model_train(tn_model* m, int32_t epochs, int32_t batch, double lr, uint64_t seed, double* loss_first,
                         double* loss_last, void* stream) {
  return guarded([&] {
    TN_REQUIRE(m && epochs >= 1 && batch >= 1 && lr > 0, TN_ERR_ARG, "bad argument");
    TN_REQUIRE(!m->data.empty(), TN_ERR_STATE, "empty training set (tn_model_add_teacher first)");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int ns = int(m->data.size());
    std::vector<int> order(ns);
    std::iota(order.begin(), order.end(), 0);
    uint64_t rng = seed;
    std::vector<float> lossv;
    for (int ep = 0; ep < epochs; ++ep) {
      for (int i = ns - 1; i > 0; --i) {   // Fisher-Yates with SplitMix64
        const int j = int(splitmix64_next(&rng) % uint64_t(i + 1));
        std::swap(order[i], order[j]);
      }
      double tot = 0;
      for (int b0 = 0; b0 < ns; b0 += batch) {
        std::vector<const tn_model::Sample*> bt;
        for (int k = b0; k < std::min(ns, b0 + batch); ++k) bt.push_back(&m->data[order[k]]);
        int nodes = 0;
        upload_batch(m, bt, &nodes, st);
        forward(m, nodes, st);
        const int S = int(bt.size());
        ce_kernel<<<blocks_for(S), 256, 0, st>>>(m->s, m->seg, m->lab, S, 1.0f / float(S), m->ds, m->loss);
        backward(m, nodes, st);
        m->adam_t++;
        const float bc1 = 1.f - std::pow(0.9f, float(m->adam_t)), bc2 = 1.f - std::pow(0.999f, float(m->adam_t));
        adam_kernel<<<blocks_for(m->np), 256, 0, st>>>(m->P, m->G, m->Mo, m->Vo, m->np, float(lr), bc1, bc2);
        TN_HIP(hipGetLastError());
        lossv.resize(S);
        TN_HIP(hipMemcpyAsync(lossv.data(), m->loss, S * sizeof(float), hipMemcpyDeviceToHost, st));
        TN_HIP(hipStreamSynchronize(st));
        for (float v : lossv) tot += v;
      }
      const double mean = tot / ns;
      if (ep == 0 && loss_first) *loss_first = mean;
      if (loss_last) *loss_last = mean;
    }
  });
}

}  // extern "C"

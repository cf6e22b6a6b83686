// Complex128 (FP64) kernels of the contraction path: the validation
// precision TN_PREC_FP64 runs a job's whole plan with these, so the error of
// the complex64 / split-precision runs can be measured against it on the
// device (reading the paper's TF32 remark in Table 2 as a measured error).
// They mirror the complex64 kernels' addressing; throughput is secondary:
//
//  * apply64      : small-operand contraction by bit addresses (one row per
//                   thread, FP64 multiply-adds);
//  * permute64    : LDS-tiled bit permutation, 64 x 64 entries per tile
//                   (6 input + 6 output bits, as the complex64 tiles);
//  * gemm64       : 64 x 64 complex block tile, 8-wide K steps in LDS,
//                   4 x 4 outputs per thread, FP64 FMA (either operand
//                   layout, batched);
//  * skinny64/dot : long-K contractions with few outputs, FP64 throughout.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

namespace tn {
namespace {

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

__device__ __forceinline__ void zmac(double2& acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}

// ------------------------------------------------------------------ apply

struct Apply64Args {
  int nk, nn, n_b_extra;
  int64_t n_rows;
  int8_t kpos[8];
  int8_t bk[8];
  int8_t bn[8];
  int8_t b_extra[12];
};

template <int NN>
__global__ __launch_bounds__(256) void apply64_kernel(const double2* __restrict__ A, const double2* __restrict__ B,
                                                      double2* __restrict__ C, Apply64Args P) {
  __shared__ double2 sB[64 * NN];
  __shared__ int64_t s_koff[64];
  const int KK = 1 << P.nk;
  const int t = threadIdx.x;
  for (int idx = t; idx < KK * NN; idx += 256) {
    const int k = idx / NN, n = idx % NN;
    int64_t off = 0;
    for (int i = 0; i < P.nk; ++i)
      if (P.bk[i] >= 0 && ((k >> i) & 1)) off |= int64_t(1) << P.bk[i];
    for (int i = 0; i < P.nn; ++i)
      if ((n >> i) & 1) off |= int64_t(1) << P.bn[i];
    double2 v = make_double2(0.0, 0.0);
    for (int e = 0; e < (1 << P.n_b_extra); ++e) {
      int64_t o2 = off;
      for (int i = 0; i < P.n_b_extra; ++i)
        if ((e >> i) & 1) o2 |= int64_t(1) << P.b_extra[i];
      v.x += B[o2].x;
      v.y += B[o2].y;
    }
    sB[idx] = v;
  }
  if (t < KK) {
    int64_t off = 0;
    for (int i = 0; i < P.nk; ++i)
      if ((t >> i) & 1) off |= int64_t(1) << P.kpos[i];
    s_koff[t] = off;
  }
  __syncthreads();
  for (int64_t m = int64_t(blockIdx.x) * 256 + t; m < P.n_rows; m += int64_t(gridDim.x) * 256) {
    int64_t base = m;
    for (int i = 0; i < P.nk; ++i) {
      const int p = P.kpos[i];
      base = ((base >> p) << (p + 1)) | (base & ((int64_t(1) << p) - 1));
    }
    double2 acc[NN];
#pragma unroll
    for (int n = 0; n < NN; ++n) acc[n] = make_double2(0.0, 0.0);
    for (int k = 0; k < KK; ++k) {
      const double2 a = A[base + s_koff[k]];
#pragma unroll
      for (int n = 0; n < NN; ++n) zmac(acc[n], a, sB[k * NN + n]);
    }
#pragma unroll
    for (int n = 0; n < NN; ++n) C[m * NN + n] = acc[n];
  }
}

// ---------------------------------------------------------------- permute

struct Perm64Bits {
  int8_t src[kMaxBits];   // output bit j <- input bit src[j] (-1: fixed 0)
};

// Gather form for small tensors and non-permutations: out[o] = in[src(o)].
__global__ __launch_bounds__(256) void permute64_simple_kernel(const double2* __restrict__ in,
                                                               double2* __restrict__ out, int nb,
                                                               Perm64Bits P, int64_t n) {
  for (int64_t o = int64_t(blockIdx.x) * 256 + threadIdx.x; o < n; o += int64_t(gridDim.x) * 256) {
    int64_t off = 0;
    for (int j = 0; j < nb; ++j)
      if (P.src[j] >= 0 && ((o >> j) & 1)) off |= int64_t(1) << P.src[j];
    out[o] = in[off];
  }
}

// Tiled form: a tile is the 6 lowest input bits x the input bits of the 6
// lowest output bits; reads and writes move 64 consecutive entries.
struct Perm64Tile {
  int rb;
  int64_t n_tiles;
  int8_t tin[12];      // tile bit -> input bit (0..5 the lowest input bits)
  int8_t tout[12];     // tile bit -> output bit
  int8_t r_in[64];
  int8_t r_out[64];
};

__global__ __launch_bounds__(256) void permute64_tiled_kernel(const double2* __restrict__ in,
                                                              double2* __restrict__ out, Perm64Tile P) {
  __shared__ double2 tile[64 * 65];
  __shared__ int64_t s_in[2][64], s_out[2][64];
  __shared__ int s_rd[2][64];
  const int t = threadIdx.x;
  if (t < 64) {
    // load side: e = (hi << 6) | lo with lo over input bits 0..5 (tile bits
    // 0..5) and hi over tile bits 6..11; store side: f = (fhi << 6) | flo over
    // output bits 0..5 (their tile bits) and the remaining tile bits
    int64_t a = 0, b = 0, c = 0, d = 0;
    int ra = 0, rb = 0;
    for (int i = 0; i < 6; ++i) {
      if (!((t >> i) & 1)) continue;
      a |= int64_t(1) << P.tin[i];
      b |= int64_t(1) << P.tin[6 + i];
    }
    s_in[0][t] = a;
    s_in[1][t] = b;
    // tile bits in output order: the output-bit slots 0..5 come first
    int lo_bits[6] = {0, 0, 0, 0, 0, 0}, hi_bits[6] = {0, 0, 0, 0, 0, 0}, nh = 0;
    for (int tb = 0; tb < 12; ++tb)
      if (P.tout[tb] < 6) lo_bits[P.tout[tb]] = tb;
    for (int tb = 0; tb < 12; ++tb)
      if (P.tout[tb] >= 6) hi_bits[nh++] = tb;
    for (int i = 0; i < 6; ++i) {
      if (!((t >> i) & 1)) continue;
      c |= int64_t(1) << P.tout[lo_bits[i]];
      d |= int64_t(1) << P.tout[hi_bits[i]];
      ra |= 1 << lo_bits[i];
      rb |= 1 << hi_bits[i];
    }
    s_out[0][t] = c;
    s_out[1][t] = d;
    s_rd[0][t] = ra;
    s_rd[1][t] = rb;
  }
  __syncthreads();
  for (int64_t tau = blockIdx.x; tau < P.n_tiles; tau += gridDim.x) {
    int64_t ib = 0, ob = 0;
    for (int k = 0; k < P.rb; ++k)
      if ((tau >> k) & 1) {
        ib |= int64_t(1) << P.r_in[k];
        ob |= int64_t(1) << P.r_out[k];
      }
    for (int e = t; e < 4096; e += 256) {
      const int lo = e & 63, hi = e >> 6;
      tile[hi * 65 + lo] = in[ib + s_in[0][lo] + s_in[1][hi]];
    }
    __syncthreads();
    for (int f = t; f < 4096; f += 256) {
      const int lo = f & 63, hi = f >> 6;
      const int e = s_rd[0][lo] | s_rd[1][hi];
      out[ob + s_out[0][lo] + s_out[1][hi]] = tile[(e >> 6) * 65 + (e & 63)];
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------- GEMM

struct Gemm64Args {
  int64_t M, N, K;
  int transA, transB;
  int64_t kchunk;   // K range of one blockIdx.y (K when not split)
};

// C[b][m][n] = sum_k A(m, k) B(k, n); transA = 0: A[b][m][k], 1: A[b][k][m];
// transB = 0: B[b][k][n], 1: B[b][n][k].  Block y sums k in [y kchunk,
// (y + 1) kchunk) and writes C + y batch M N (split-K partials when
// gridDim.y > 1, summed by gemm64_reduce_kernel).
__global__ __launch_bounds__(256) void gemm64_kernel(const double2* __restrict__ A, const double2* __restrict__ B,
                                                     double2* __restrict__ C, Gemm64Args P) {
  __shared__ double2 As[8][64 + 1];
  __shared__ double2 Bs[8][64 + 1];
  const int64_t tiles_n = cdiv(P.N, 64);
  const int64_t m0 = int64_t(blockIdx.x / tiles_n) * 64, n0 = int64_t(blockIdx.x % tiles_n) * 64;
  const int64_t b = blockIdx.z;
  const double2* Ab = A + b * P.M * P.K;
  const double2* Bb = B + b * P.K * P.N;
  double2* Cb = C + (int64_t(blockIdx.y) * gridDim.z + b) * P.M * P.N;
  const int64_t kb = int64_t(blockIdx.y) * P.kchunk, ke = min(P.K, kb + P.kchunk);
  const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
  double2 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = make_double2(0.0, 0.0);
  for (int64_t k0 = kb; k0 < ke; k0 += 8) {
    for (int e = t; e < 512; e += 256) {
      // A tile: 64 rows x 8 k; B tile: 8 k x 64 columns
      int kk, mm;
      if (P.transA) { kk = e >> 6; mm = e & 63; } else { mm = e >> 3; kk = e & 7; }
      const int64_t gm = m0 + mm, gk = k0 + kk;
      double2 v = make_double2(0.0, 0.0);
      if (gm < P.M && gk < ke) v = P.transA ? Ab[gk * P.M + gm] : Ab[gm * P.K + gk];
      As[kk][mm] = v;
      int kb, nn;
      if (P.transB) { nn = e >> 3; kb = e & 7; } else { kb = e >> 6; nn = e & 63; }
      const int64_t gn = n0 + nn, gkb = k0 + kb;
      double2 w = make_double2(0.0, 0.0);
      if (gn < P.N && gkb < ke) w = P.transB ? Bb[gn * P.K + gkb] : Bb[gkb * P.N + gn];
      Bs[kb][nn] = w;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      double2 a[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = Bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) zmac(acc[i][j], a[i], bv[j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t gm = m0 + ty + 16 * i, gn = n0 + tx + 16 * j;
      if (gm < P.M && gn < P.N) Cb[gm * P.N + gn] = acc[i][j];
    }
}

// C[e] = sum over y = 0 .. Z-1, in order, of part[y][e], e < n.
__global__ void gemm64_reduce_kernel(const double2* __restrict__ part, int Z, int64_t n, double2* __restrict__ C) {
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x) {
    double2 acc = make_double2(0.0, 0.0);
    for (int y = 0; y < Z; ++y) {
      const double2 v = part[int64_t(y) * n + e];
      acc.x += v.x;
      acc.y += v.y;
    }
    C[e] = acc;
  }
}

// ------------------------------------------------------ long-K, few outputs

// C[b][o] = sum_k A(b, m, k) B(b, k, n) for o = (m, n): each block sums a
// K range for every output of one batch entry (strides as for the skinny
// complex64 kernel), FP64 partials per block, then a final FP64 sum.
constexpr int kDot64Blocks = 512;

__global__ __launch_bounds__(256) void dot64_partial_kernel(const double2* __restrict__ A,
                                                            const double2* __restrict__ B,
                                                            double2* __restrict__ part, int64_t K, int m,
                                                            int n, int64_t sam, int64_t sak, int64_t sbk,
                                                            int64_t sbn, int64_t sa_b, int64_t sb_b) {
  __shared__ double2 red[4];
  const int64_t o = blockIdx.y;                       // (batch, m, n)
  const int64_t bi = o / (int64_t(m) * n), mi = (o / n) % m, ni = o % n;
  const double2* a = A + bi * sa_b + mi * sam;
  const double2* bb = B + bi * sb_b + ni * sbn;
  double2 acc = make_double2(0.0, 0.0);
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < K; k += int64_t(gridDim.x) * 256)
    zmac(acc, a[k * sak], bb[k * sbk]);
  for (int s = 32; s > 0; s >>= 1) {
    acc.x += __shfl_xor(acc.x, s);
    acc.y += __shfl_xor(acc.y, s);
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double2 v = make_double2(red[0].x + red[1].x + red[2].x + red[3].x, red[0].y + red[1].y + red[2].y + red[3].y);
    part[o * gridDim.x + blockIdx.x] = v;
  }
}

__global__ void dot64_final_kernel(const double2* __restrict__ part, double2* __restrict__ C, int nparts,
                                   int64_t outs) {
  const int64_t o = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (o >= outs) return;
  double sr = 0.0, si = 0.0;
  for (int p = 0; p < nparts; ++p) {
    sr += part[o * nparts + p].x;
    si += part[o * nparts + p].y;
  }
  C[o] = make_double2(sr, si);
}

int dot64_parts(int64_t K) { return int(std::max<int64_t>(1, std::min<int64_t>(kDot64Blocks, cdiv(K, 4096)))); }

}  // namespace

void launch_apply64(const double2* A, const double2* B, double2* C, const ApplySmallDesc& d, hipStream_t s) {
  TN_REQUIRE(d.nk >= 0 && d.nk <= 6 && d.nn >= 0 && d.nn <= 4 && d.n_b_extra <= 12, TN_ERR_UNSUPPORTED,
             "apply shape out of range");
  Apply64Args P;
  std::memset(&P, 0, sizeof(P));
  P.nk = d.nk;
  P.nn = d.nn;
  P.n_b_extra = d.n_b_extra;
  P.n_rows = int64_t(1) << (d.a_bits - d.nk);
  for (int i = 0; i < 8; ++i) {
    P.kpos[i] = d.kpos[i];
    P.bk[i] = d.bk[i];
    P.bn[i] = d.bn[i];
  }
  for (int i = 0; i < 12; ++i) P.b_extra[i] = d.b_extra[i];
  const dim3 g(unsigned(std::max<int64_t>(1, std::min<int64_t>(cdiv(P.n_rows, 256), 8192)))), b(256);
  switch (1 << d.nn) {
    case 1: apply64_kernel<1><<<g, b, 0, s>>>(A, B, C, P); break;
    case 2: apply64_kernel<2><<<g, b, 0, s>>>(A, B, C, P); break;
    case 4: apply64_kernel<4><<<g, b, 0, s>>>(A, B, C, P); break;
    case 8: apply64_kernel<8><<<g, b, 0, s>>>(A, B, C, P); break;
    default: apply64_kernel<16><<<g, b, 0, s>>>(A, B, C, P); break;
  }
  TN_HIP(hipGetLastError());
}

void launch_permute64(const double2* in, double2* out, const PermuteDesc& d, hipStream_t s) {
  const int nb = d.nb;
  TN_REQUIRE(nb >= 0 && nb <= 62 && d.np == 0 && !d.f16 && !d.maxabs, TN_ERR_ARG, "internal: FP64 permute");
  const int64_t n = int64_t(1) << nb;
  bool is_perm = d.nb_in == nb;
  std::vector<int> inv(std::max(nb, 1), -1);
  for (int j = 0; j < nb && is_perm; ++j) {
    if (d.src[j] < 0 || d.src[j] >= nb || inv[d.src[j]] >= 0) {
      is_perm = false;
      break;
    }
    inv[d.src[j]] = j;
  }
  if (!is_perm || nb < 12) {
    Perm64Bits P;
    std::memset(&P, 0, sizeof(P));
    for (int j = 0; j < kMaxBits; ++j) P.src[j] = j < nb ? d.src[j] : -1;
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(cdiv(n, 256), 8192));
    permute64_simple_kernel<<<dim3(unsigned(blocks)), 256, 0, s>>>(in, out, nb, P, n);
    TN_HIP(hipGetLastError());
    return;
  }
  // tile bits: input bits 0..5, then the sources of output bits 0..5 (or,
  // where those already are input bits 0..5, the next lowest input bits)
  std::vector<char> inT(nb, 0);
  std::vector<int> tin;
  for (int i = 0; i < 6; ++i) {
    inT[i] = 1;
    tin.push_back(i);
  }
  for (int j = 0; j < 6; ++j)
    if (!inT[d.src[j]]) {
      inT[d.src[j]] = 1;
      tin.push_back(d.src[j]);
    }
  for (int i = 0; i < nb && int(tin.size()) < 12; ++i)
    if (!inT[i]) {
      inT[i] = 1;
      tin.push_back(i);
    }
  Perm64Tile P;
  std::memset(&P, 0, sizeof(P));
  for (int tb = 0; tb < 12; ++tb) {
    P.tin[tb] = int8_t(tin[tb]);
    P.tout[tb] = int8_t(inv[tin[tb]]);
  }
  int rb = 0;
  for (int i = 0; i < nb; ++i)
    if (!inT[i]) {
      P.r_in[rb] = int8_t(i);
      P.r_out[rb] = int8_t(inv[i]);
      ++rb;
    }
  P.rb = rb;
  P.n_tiles = int64_t(1) << rb;
  const int64_t blocks = std::min<int64_t>(P.n_tiles, 256 * 16);
  permute64_tiled_kernel<<<dim3(unsigned(blocks)), 256, 0, s>>>(in, out, P);
  TN_HIP(hipGetLastError());
}

// Split-K for GEMMs of few tiles and long K: about 1024 blocks, each K
// range at least 4096 long and a multiple of 8.
static int64_t gemm64_kchunk(const GemmDesc& g) {
  const int64_t blocks = cdiv(g.M, 64) * cdiv(g.N, 64) * g.batch;
  if (blocks >= 256 || g.K < 8192) return g.K;
  const int64_t ks = std::max<int64_t>(1, std::min<int64_t>(cdiv(1024, blocks), g.K / 4096));
  return cdiv(cdiv(g.K, ks), 8) * 8;
}

size_t gemm64_workspace_bytes(const GemmDesc& g) {
  const int64_t kc = gemm64_kchunk(g);
  return kc >= g.K ? 0 : size_t(cdiv(g.K, kc)) * size_t(g.batch * g.M * g.N) * sizeof(double2);
}

void launch_gemm64(const double2* A, const double2* B, double2* C, const GemmDesc& g, void* work, hipStream_t s) {
  TN_REQUIRE(g.M >= 1 && g.N >= 1 && g.K >= 1 && g.batch >= 1 && g.batch <= 65535, TN_ERR_ARG, "bad GEMM shape");
  const int64_t tiles = cdiv(g.M, 64) * cdiv(g.N, 64);
  TN_REQUIRE(tiles < (int64_t(1) << 31), TN_ERR_UNSUPPORTED, "GEMM grid too large");
  const int64_t kc = work ? gemm64_kchunk(g) : g.K;
  const int64_t ks = cdiv(g.K, kc);
  Gemm64Args P{g.M, g.N, g.K, g.transA, g.transB, kc};
  double2* out = ks > 1 ? static_cast<double2*>(work) : C;
  gemm64_kernel<<<dim3(unsigned(tiles), unsigned(ks), unsigned(g.batch)), 256, 0, s>>>(A, B, out, P);
  TN_HIP(hipGetLastError());
  if (ks > 1) {
    const int64_t n = g.batch * g.M * g.N;
    gemm64_reduce_kernel<<<dim3(unsigned(std::min<int64_t>(cdiv(n, 256), 4096))), 256, 0, s>>>(out, int(ks), n, C);
    TN_HIP(hipGetLastError());
  }
}

size_t dot64_workspace_bytes(int64_t K, int64_t outs) {
  return size_t(dot64_parts(K)) * size_t(outs) * sizeof(double2);
}

void launch_dot64(const double2* A, const double2* B, double2* C, int64_t K, int64_t batch, int64_t m, int64_t n,
                  int transA, int transB, void* work, hipStream_t s) {
  TN_REQUIRE(work != nullptr, TN_ERR_WORKSPACE, "dot needs workspace");
  const int64_t outs = batch * m * n;
  TN_REQUIRE(m >= 1 && n >= 1 && outs <= 65535, TN_ERR_UNSUPPORTED, "dot batch too large");
  // layouts as the GEMM operands: transA = 0: A[b][m][k], 1: A[b][k][m];
  // transB = 0: B[b][k][n], 1: B[b][n][k]
  const int64_t sam = transA ? 1 : K, sak = transA ? m : 1;
  const int64_t sbk = transB ? 1 : n, sbn = transB ? K : 1;
  const int parts = dot64_parts(K);
  dot64_partial_kernel<<<dim3(unsigned(parts), unsigned(outs)), 256, 0, s>>>(
      A, B, static_cast<double2*>(work), K, int(m), int(n), sam, sak, sbk, sbn, m * K, K * n);
  TN_HIP(hipGetLastError());
  dot64_final_kernel<<<dim3(unsigned(cdiv(outs, 256))), 256, 0, s>>>(static_cast<double2*>(work), C, parts, outs);
  TN_HIP(hipGetLastError());
}

}  // namespace tn

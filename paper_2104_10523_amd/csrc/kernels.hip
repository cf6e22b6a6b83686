// gfx950 kernels of the contraction hot path.
//
//  * permute_tiled   : bit permutation of a complex64 tensor through an LDS
//                      tile; 32-element (256 B) runs on both the read and the
//                      write side.
//  * apply_small     : contraction of a large tensor with a small one
//                      (<= 64 x 16 matrix) addressed by bit positions, so the
//                      large operand is read once, in place, without a
//                      separate permutation pass.
//  * gemm_mfma       : complex GEMM on MFMA.  The complex product is a real
//                      GEMM of the interleaved A (M x 2K) with the 2x2 real
//                      block form of B ([[br, bi], [-bi, br]], 2K x 2N); the
//                      product is C in interleaved form.  FP32 uses
//                      v_mfma_f32_32x32x2_f32; BF16X3 / BF16X6 split each
//                      operand into bfloat16 parts in LDS and use
//                      v_mfma_f32_32x32x16_bf16 with FP32 accumulation.
//  * dot             : full contractions (M = N = 1) with split-K, FP64 sums.
//  * gather / accumulate / job control: per-job leaf projection and FP64
//                      accumulation of slice results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "../../include/tn.h"
#include "common.hpp"
#include "kernels.hpp"

namespace tn {

static inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

static int grid_cap() { return 256 * 16; }

// ------------------------------------------------------- bfloat16 helpers

// Round-to-nearest-even float -> bfloat16 bits (finite inputs).
__device__ __forceinline__ uint32_t bf16_bits(float x) {
  const uint32_t u = __float_as_uint(x);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float bf16_to_float(uint32_t h) { return __uint_as_float(h << 16); }

// Split a complex value into NP bfloat16 parts, each packed (re | im << 16):
// part p holds the rounding of what parts 0..p-1 left over.
template <int NP>
__device__ __forceinline__ void split_c(float2 v, uint32_t* w) {
  float r = v.x, i = v.y;
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const uint32_t hr = bf16_bits(r), hi = bf16_bits(i);
    w[p] = hr | (hi << 16);
    r -= bf16_to_float(hr);
    i -= bf16_to_float(hi);
  }
}

// Split-FP16 operands: the value times a power of two (chosen per operand
// from its largest magnitude, so that it lands in [2^14, 2^15)) split into a
// round-to-nearest fp16 part and the fp16 rounding of the remainder.
constexpr int kF16 = 4;   // plane mode: two planes of packed fp16 words
__device__ __forceinline__ uint32_t f16_bits(float x) {
  return uint32_t(__builtin_bit_cast(unsigned short, static_cast<_Float16>(x)));
}
__device__ __forceinline__ float f16_to_float(uint32_t h) {
  return static_cast<float>(__builtin_bit_cast(_Float16, static_cast<unsigned short>(h)));
}
__device__ __forceinline__ void split_c_f16(float2 v, float scale, uint32_t* w) {
  float r = v.x * scale, i = v.y * scale;
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const uint32_t hr = f16_bits(r), hi = f16_bits(i);
    w[p] = hr | (hi << 16);
    r -= f16_to_float(hr);
    i -= f16_to_float(hi);
  }
}
// Exponent s of the operand scale 2^s from the bits of its largest |re|, |im|
// (0 for an all-zero or non-finite operand).
__device__ __forceinline__ int f16_scale_exp(uint32_t max_bits) {
  const float m = __uint_as_float(max_bits);
  if (!(m > 0.f) || !isfinite(m)) return 0;
  return min(100, max(-100, 14 - ilogbf(m)));
}

// NP = 0 writes complex64; NP = 2 / 3 writes NP planes of packed bf16 words,
// NP = kF16 two planes of packed fp16 words of the scaled value (plane p at
// out + p * plane).
template <int NP>
__device__ __forceinline__ void put(void* out, int64_t plane, int64_t idx, float2 v, float scale) {
  if constexpr (NP == 0) {
    static_cast<float2*>(out)[idx] = v;
  } else if constexpr (NP == kF16) {
    uint32_t w[2];
    split_c_f16(v, scale, w);
    static_cast<uint32_t*>(out)[idx] = w[0];
    static_cast<uint32_t*>(out)[plane + idx] = w[1];
  } else {
    uint32_t w[NP];
    split_c<NP>(v, w);
#pragma unroll
    for (int p = 0; p < NP; ++p) static_cast<uint32_t*>(out)[p * plane + idx] = w[p];
  }
}

__device__ __forceinline__ float operand_scale(const uint32_t* smax) {
  return smax ? ldexpf(1.f, f16_scale_exp(*smax)) : 1.f;
}

// ------------------------------------------------------------------ permute

constexpr int kPermBits = 12;                 // tile = 6 input + 6 output bits
constexpr int kPermTile = 1 << kPermBits;

struct PermArgs {
  int tb, rb;
  int64_t n_tiles;
  int64_t plane;
  int8_t tpos[kPermBits];
  int8_t opos[kPermBits];
  int8_t map[kPermBits];
  int8_t r_in[kMaxBits];
  int8_t r_out[kMaxBits];
};

template <int NP>
__global__ __launch_bounds__(256) void permute_tiled_kernel(const float2* __restrict__ in,
                                                            void* __restrict__ out, PermArgs P,
                                                            const uint32_t* __restrict__ smax) {
  const float scale = NP == kF16 ? operand_scale(smax) : 1.f;
  __shared__ int64_t s_in_lo[64], s_in_hi[64], s_out_lo[64], s_out_hi[64];
  __shared__ int s_l_lo[64], s_l_hi[64];
  __shared__ float2 tile[kPermTile + kPermTile / 64];
  const int t = threadIdx.x;
  if (t < 64) {
    int64_t il = 0, ih = 0, ol = 0, oh = 0;
    int ll = 0, lh = 0;
    for (int i = 0; i < 6; ++i) {
      if (!((t >> i) & 1)) continue;
      if (i < P.tb) {
        il |= int64_t(1) << P.tpos[i];
        ol |= int64_t(1) << P.opos[i];
        ll |= 1 << P.map[i];
      }
      if (i + 6 < P.tb) {
        ih |= int64_t(1) << P.tpos[i + 6];
        oh |= int64_t(1) << P.opos[i + 6];
        lh |= 1 << P.map[i + 6];
      }
    }
    s_in_lo[t] = il; s_in_hi[t] = ih;
    s_out_lo[t] = ol; s_out_hi[t] = oh;
    s_l_lo[t] = ll; s_l_hi[t] = lh;
  }
  __syncthreads();
  const int tsize = 1 << P.tb;
  for (int64_t tau = blockIdx.x; tau < P.n_tiles; tau += gridDim.x) {
    int64_t ib = 0, ob = 0;
    for (int k = 0; k < P.rb; ++k) {
      if ((tau >> k) & 1) {
        ib |= int64_t(1) << P.r_in[k];
        ob |= int64_t(1) << P.r_out[k];
      }
    }
    for (int e = t; e < tsize; e += 256)
      tile[e + (e >> 6)] = in[ib + s_in_lo[e & 63] + s_in_hi[e >> 6]];
    __syncthreads();
    for (int f = t; f < tsize; f += 256) {
      const int e = s_l_lo[f & 63] | s_l_hi[f >> 6];
      put<NP>(out, P.plane, ob + s_out_lo[f & 63] + s_out_hi[f >> 6], tile[e + (e >> 6)], scale);
    }
    __syncthreads();
  }
}

// Pipelined variant for tensors of >= 2^12 entries with 16-byte aligned
// buffers (the tile then has all 12 bits, input bits 0..5 and output bits
// 0..5 among them).  Each thread moves 16 entries per tile: it loads them as
// 8 x 16-byte pairs (input bit 0 inside a pair) and stores 4 x 4 consecutive
// outputs (output bits 0 and 1 inside a group) with 16-byte stores, 32-byte
// for complex64.  The loads of the next tile are issued before the current
// tile leaves LDS, so a block keeps 32 KB of reads in flight while it writes.
// Every per-thread offset inside a tile is the same for all tiles and is
// computed once.  LDS rows of 64 entries are padded by one float2 (an odd
// stride of 130 dwords): reads that walk down a column then hit distinct
// banks.  An even pad (16-byte aligned rows) measured 3.3-3.5 TB/s against
// 4.8-5.1 TB/s for this layout on 2^30-entry permutations; the price is two
// 8-byte LDS writes per 16-byte load.
constexpr int kPipePad = 1;   // float2 of padding per 64-entry LDS row
__device__ __forceinline__ int pipe_pos(int e) { return e + kPipePad * (e >> 6); }

template <int NP>
__global__ __launch_bounds__(256) void permute_pipe_kernel(const float2* __restrict__ in,
                                                           void* __restrict__ out, PermArgs P,
                                                           const uint32_t* __restrict__ smax) {
  const float scale = NP == kF16 ? operand_scale(smax) : 1.f;
  __shared__ int64_t s_in_lo[64], s_in_hi[64], s_out_lo[64], s_out_hi[64];
  __shared__ int s_l_lo[64], s_l_hi[64];
  __shared__ __align__(16) float2 tile[kPermTile + kPipePad * (kPermTile / 64)];
  const int t = threadIdx.x;
  if (t < 64) {
    int64_t il = 0, ih = 0, ol = 0, oh = 0;
    int ll = 0, lh = 0;
    for (int i = 0; i < 6; ++i) {
      if (!((t >> i) & 1)) continue;
      il |= int64_t(1) << P.tpos[i];
      ol |= int64_t(1) << P.opos[i];
      ll |= 1 << P.map[i];
      ih |= int64_t(1) << P.tpos[i + 6];
      oh |= int64_t(1) << P.opos[i + 6];
      lh |= 1 << P.map[i + 6];
    }
    s_in_lo[t] = il; s_in_hi[t] = ih;
    s_out_lo[t] = ol; s_out_hi[t] = oh;
    s_l_lo[t] = ll; s_l_hi[t] = lh;
  }
  __syncthreads();
  int64_t ld_off[8], st_off[4];
  int ld_pos[8], rd_pos[16];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int e = 2 * (t + 256 * i);
    ld_off[i] = s_in_lo[e & 63] + s_in_hi[e >> 6];
    ld_pos[i] = pipe_pos(e);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int f0 = 4 * (t + 256 * j);
    st_off[j] = s_out_lo[f0 & 63] + s_out_hi[f0 >> 6];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int f = f0 + q;
      rd_pos[4 * j + q] = pipe_pos(s_l_lo[f & 63] | s_l_hi[f >> 6]);
    }
  }
  int64_t tau = blockIdx.x;
  if (tau >= P.n_tiles) return;
  auto deposit = [&](int64_t x, const int8_t* pos) {
    int64_t r = 0;
    for (int k = 0; k < P.rb; ++k)
      if ((x >> k) & 1) r |= int64_t(1) << pos[k];
    return r;
  };
  float4 v[8];
  {
    const int64_t ib = deposit(tau, P.r_in);
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = *reinterpret_cast<const float4*>(in + ib + ld_off[i]);
  }
  while (true) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      tile[ld_pos[i]] = make_float2(v[i].x, v[i].y);
      tile[ld_pos[i] + 1] = make_float2(v[i].z, v[i].w);
    }
    __syncthreads();
    const int64_t ob = deposit(tau, P.r_out);
    const int64_t nxt = tau + gridDim.x;
    if (nxt < P.n_tiles) {
      const int64_t ib = deposit(nxt, P.r_in);
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = *reinterpret_cast<const float4*>(in + ib + ld_off[i]);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float2 x[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) x[q] = tile[rd_pos[4 * j + q]];
      const int64_t o = ob + st_off[j];
      if constexpr (NP == 0) {
        float4* dst = reinterpret_cast<float4*>(static_cast<float2*>(out) + o);
        dst[0] = make_float4(x[0].x, x[0].y, x[1].x, x[1].y);
        dst[1] = make_float4(x[2].x, x[2].y, x[3].x, x[3].y);
      } else if constexpr (NP == kF16) {
        uint32_t w[4][2];
#pragma unroll
        for (int q = 0; q < 4; ++q) split_c_f16(x[q], scale, w[q]);
        uint32_t* dst = static_cast<uint32_t*>(out) + o;
#pragma unroll
        for (int p = 0; p < 2; ++p)
          *reinterpret_cast<uint4*>(dst + p * P.plane) = make_uint4(w[0][p], w[1][p], w[2][p], w[3][p]);
      } else {
        uint32_t w[4][NP];
#pragma unroll
        for (int q = 0; q < 4; ++q) split_c<NP>(x[q], w[q]);
        uint32_t* dst = static_cast<uint32_t*>(out) + o;
#pragma unroll
        for (int p = 0; p < NP; ++p)
          *reinterpret_cast<uint4*>(dst + p * P.plane) = make_uint4(w[0][p], w[1][p], w[2][p], w[3][p]);
      }
    }
    __syncthreads();
    if (nxt >= P.n_tiles) break;
    tau = nxt;
  }
}

struct PermSimpleArgs {
  int nb;
  int identity;
  int64_t plane;
  int8_t src[kMaxBits];
};

template <int NP>
__global__ __launch_bounds__(256) void permute_simple_kernel(const float2* __restrict__ in,
                                                             void* __restrict__ out,
                                                             PermSimpleArgs P, int64_t n,
                                                             const uint32_t* __restrict__ smax) {
  const float scale = NP == kF16 ? operand_scale(smax) : 1.f;
  for (int64_t o = int64_t(blockIdx.x) * 256 + threadIdx.x; o < n; o += int64_t(gridDim.x) * 256) {
    int64_t off = o;
    if (!P.identity) {
      off = 0;
      for (int j = 0; j < P.nb; ++j)
        if (P.src[j] >= 0 && ((o >> j) & 1)) off |= int64_t(1) << P.src[j];
    }
    put<NP>(out, P.plane, o, in[off], scale);
  }
}

// The pipelined permute handles full 12-bit tiles on 16-byte aligned buffers.
static bool pipe_ok(const PermuteDesc& d, const void* in, const void* out) {
  return d.nb >= kPermBits && (reinterpret_cast<uintptr_t>(in) & 15) == 0 &&
         (reinterpret_cast<uintptr_t>(out) & 15) == 0;
}

template <int NP>
static void launch_permute_np(const float2* in, void* out, const PermuteDesc& d, const uint32_t* smax,
                              hipStream_t s) {
  const int nb = d.nb;
  const int64_t n = int64_t(1) << nb;
  bool is_perm = d.nb_in == nb;
  bool ident = true;
  std::vector<int> inv(std::max(nb, 1), -1);
  for (int j = 0; j < nb && is_perm; ++j) {
    if (d.src[j] < 0 || d.src[j] >= nb || inv[d.src[j]] >= 0) {
      is_perm = false;
      break;
    }
    inv[d.src[j]] = j;
    if (d.src[j] != j) ident = false;
  }
  if (is_perm && ident && NP == 0) {
    TN_HIP(hipMemcpyAsync(out, in, size_t(n) * sizeof(float2), hipMemcpyDeviceToDevice, s));
    return;
  }
  if (!is_perm || ident || nb < 6) {
    PermSimpleArgs P;
    std::memset(&P, 0, sizeof(P));
    P.nb = nb;
    P.identity = is_perm && ident;
    P.plane = n;
    for (int j = 0; j < kMaxBits; ++j) P.src[j] = j < nb ? d.src[j] : -1;
    const int64_t blocks = std::min<int64_t>(ceil_div(n, 256), grid_cap() * 2);
    permute_simple_kernel<NP><<<dim3(unsigned(blocks)), dim3(256), 0, s>>>(in, out, P, n, smax);
    TN_HIP(hipGetLastError());
    return;
  }
  // tile bits: the 6 lowest input bits and the input bits of the 6 lowest
  // output bits, padded with the next lowest input bits up to 12.
  std::vector<char> inT(nb, 0);
  const int a = std::min(kPermBits / 2, nb);
  for (int i = 0; i < a; ++i) inT[i] = 1;
  for (int j = 0; j < a; ++j) inT[d.src[j]] = 1;
  int cnt = 0;
  for (int i = 0; i < nb; ++i) cnt += inT[i];
  const int want = std::min(kPermBits, nb);
  for (int i = 0; i < nb && cnt < want; ++i)
    if (!inT[i]) { inT[i] = 1; ++cnt; }
  PermArgs P;
  std::memset(&P, 0, sizeof(P));
  P.tb = cnt;
  P.plane = n;
  std::vector<int> tpos, opos;
  for (int i = 0; i < nb; ++i)
    if (inT[i]) tpos.push_back(i);
  for (int j = 0; j < nb; ++j)
    if (inT[d.src[j]]) opos.push_back(j);
  for (int p = 0; p < cnt; ++p) {
    P.tpos[p] = int8_t(tpos[p]);
    P.opos[p] = int8_t(opos[p]);
    const int src = d.src[opos[p]];
    P.map[p] = int8_t(std::find(tpos.begin(), tpos.end(), src) - tpos.begin());
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
  const int64_t blocks = std::min<int64_t>(P.n_tiles, 256 * 32);
  if (pipe_ok(d, in, out)) {
    TN_REQUIRE(P.tb == kPermBits && P.tpos[0] == 0 && P.opos[0] == 0 && P.opos[1] == 1, TN_ERR_ARG,
               "internal: pipelined permute needs a full tile holding bits 0 and 1");
    permute_pipe_kernel<NP><<<dim3(unsigned(blocks)), dim3(256), 0, s>>>(in, out, P, smax);
  } else {
    permute_tiled_kernel<NP><<<dim3(unsigned(blocks)), dim3(256), 0, s>>>(in, out, P, smax);
  }
  TN_HIP(hipGetLastError());
}

__global__ void scale_clear_kernel(uint32_t* slot) { *slot = 0u; }

// Largest |re|, |im| of n complex values, as float bits (order-preserving for
// non-negative floats) combined into *slot with an atomic max.
__global__ __launch_bounds__(256) void maxabs_kernel(const float2* __restrict__ in, int64_t n,
                                                     uint32_t* __restrict__ slot) {
  float m = 0.f;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const float2 v = in[i];
    m = fmaxf(m, fmaxf(fabsf(v.x), fabsf(v.y)));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  __shared__ float part[4];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0)
    atomicMax(slot, __float_as_uint(fmaxf(fmaxf(part[0], part[1]), fmaxf(part[2], part[3]))));
}

int permute_variant(const PermuteDesc& d) {
  if (d.maxabs) return 3;
  const int nb = d.nb;
  bool is_perm = d.nb_in == nb, ident = true;
  std::vector<char> seen(std::max(nb, 1), 0);
  for (int j = 0; j < nb && is_perm; ++j) {
    if (d.src[j] < 0 || d.src[j] >= nb || seen[d.src[j]]) {
      is_perm = false;
      break;
    }
    seen[d.src[j]] = 1;
    if (d.src[j] != j) ident = false;
  }
  const int np = d.f16 ? kF16 : d.np;
  if (is_perm && ident && np == 0) return 0;
  if (!is_perm || ident || nb < 6) return 1;
  return nb >= kPermBits ? 4 : 2;   // plan buffers are 256-byte aligned
}

void launch_permute(const float2* in, void* out, const PermuteDesc& d, uint32_t* smax, hipStream_t s) {
  TN_REQUIRE(d.nb >= 0 && d.nb <= 62, TN_ERR_UNSUPPORTED, "tensor too large to permute");
  if (d.maxabs) {
    TN_REQUIRE(smax != nullptr, TN_ERR_ARG, "internal: the max-abs pre-pass needs a scale slot");
    const int64_t n_in = int64_t(1) << d.nb_in;
    scale_clear_kernel<<<1, 1, 0, s>>>(smax);
    const int64_t blocks = std::min<int64_t>(ceil_div(n_in, 256), grid_cap());
    maxabs_kernel<<<dim3(unsigned(blocks)), dim3(256), 0, s>>>(in, n_in, smax);
    TN_HIP(hipGetLastError());
    return;
  }
  if (d.f16) {
    TN_REQUIRE(d.np == 2 && smax != nullptr, TN_ERR_ARG, "internal: fp16 planes need a scale slot");
    launch_permute_np<kF16>(in, out, d, smax, s);
    return;
  }
  switch (d.np) {
    case 0: launch_permute_np<0>(in, out, d, nullptr, s); break;
    case 2: launch_permute_np<2>(in, out, d, nullptr, s); break;
    case 3: launch_permute_np<3>(in, out, d, nullptr, s); break;
    default: throw Error(TN_ERR_ARG, "internal: bad plane count");
  }
}

// -------------------------------------------------------------- apply_small

struct ApplyArgs {
  int nk, nn, n_b_extra;
  int64_t n_rows;
  int8_t kpos[8];
  int8_t bk[8];
  int8_t bn[8];
  int8_t b_extra[12];
  uint32_t* cmax;         // matrix-core apply: largest |re|, |im| of C (atomic max), or null
};

__device__ __forceinline__ void cmac(float2& acc, float2 a, float2 b) {
  acc.x = fmaf(a.x, b.x, acc.x);
  acc.x = fmaf(-a.y, b.y, acc.x);
  acc.y = fmaf(a.x, b.y, acc.y);
  acc.y = fmaf(a.y, b.x, acc.y);
}

// One thread per output row, reading its K values of A in place.  (Staging
// the block's outputs in LDS for 16-byte stores measured slower for NN = 16,
// 2.9 against 3.3 TB/s: the extra LDS lowers occupancy to 3 waves per SIMD.)
template <int NN>
__global__ __launch_bounds__(256) void apply_small_kernel(const float2* __restrict__ A,
                                                          const float2* __restrict__ B,
                                                          float2* __restrict__ C, ApplyArgs P) {
  __shared__ float2 sB[64 * NN];
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
    float2 v = make_float2(0.f, 0.f);
    for (int e = 0; e < (1 << P.n_b_extra); ++e) {
      int64_t o2 = off;
      for (int i = 0; i < P.n_b_extra; ++i)
        if ((e >> i) & 1) o2 |= int64_t(1) << P.b_extra[i];
      const float2 b = B[o2];
      v.x += b.x;
      v.y += b.y;
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
    float2 acc[NN];
#pragma unroll
    for (int n = 0; n < NN; ++n) acc[n] = make_float2(0.f, 0.f);
    for (int k = 0; k < KK; ++k) {
      const float2 a = A[base + s_koff[k]];
#pragma unroll
      for (int n = 0; n < NN; ++n) cmac(acc[n], a, sB[k * NN + n]);
    }
#pragma unroll
    for (int n = 0; n < NN; ++n) C[m * NN + n] = acc[n];
  }
}

// Variant for the case where the lowest bits of A are K bits (so a thread's
// row is strided and its direct reads would touch a new 128-byte line per
// lane) and the 256 rows of a block span one contiguous run of A (every K
// bit below bit 8 + nk): the block reads that run with coalesced 16-byte
// loads into LDS (rows of 64 entries padded by one float2), every thread
// then takes its row's K values from LDS, and the results leave through the
// same buffer as contiguous 16-byte stores.  Needs KK <= 16, NN <= 16, full
// 256-row blocks and 16-byte aligned A and C.
template <int NN>
__global__ __launch_bounds__(256) void apply_tile_kernel(const float2* __restrict__ A,
                                                         const float2* __restrict__ B,
                                                         float2* __restrict__ C, ApplyArgs P) {
  __shared__ float2 sB[16 * NN];
  __shared__ int64_t s_koff[16];
  __shared__ float2 tile[4096 + 64];
  const int KK = 1 << P.nk;
  const int t = threadIdx.x;
  for (int idx = t; idx < KK * NN; idx += 256) {
    const int k = idx / NN, n = idx % NN;
    int64_t off = 0;
    for (int i = 0; i < P.nk; ++i)
      if (P.bk[i] >= 0 && ((k >> i) & 1)) off |= int64_t(1) << P.bk[i];
    for (int i = 0; i < P.nn; ++i)
      if ((n >> i) & 1) off |= int64_t(1) << P.bn[i];
    float2 v = make_float2(0.f, 0.f);
    for (int e = 0; e < (1 << P.n_b_extra); ++e) {
      int64_t o2 = off;
      for (int i = 0; i < P.n_b_extra; ++i)
        if ((e >> i) & 1) o2 |= int64_t(1) << P.b_extra[i];
      const float2 b = B[o2];
      v.x += b.x;
      v.y += b.y;
    }
    sB[idx] = v;
  }
  if (t < KK) {
    int64_t off = 0;
    for (int i = 0; i < P.nk; ++i)
      if ((t >> i) & 1) off |= int64_t(1) << P.kpos[i];
    s_koff[t] = off;
  }
  auto expand = [&](int64_t m) {
    for (int i = 0; i < P.nk; ++i) {
      const int p = P.kpos[i];
      m = ((m >> p) << (p + 1)) | (m & ((int64_t(1) << p) - 1));
    }
    return m;
  };
  auto pos = [](int x) { return x + (x >> 6); };
  const int lb = int(expand(t));          // this row's offset inside the block's run
  const int run = 256 * KK;               // entries of A per block
  __syncthreads();
  for (int64_t m0 = int64_t(blockIdx.x) * 256; m0 < P.n_rows; m0 += int64_t(gridDim.x) * 256) {
    const float4* src = reinterpret_cast<const float4*>(A + expand(m0));
    for (int g = t; g < run / 2; g += 256) {
      const float4 v = src[g];
      tile[pos(2 * g)] = make_float2(v.x, v.y);
      tile[pos(2 * g + 1)] = make_float2(v.z, v.w);
    }
    __syncthreads();
    float2 acc[NN];
#pragma unroll
    for (int n = 0; n < NN; ++n) acc[n] = make_float2(0.f, 0.f);
    for (int k = 0; k < KK; ++k) {
      const float2 a = tile[pos(lb + int(s_koff[k]))];
#pragma unroll
      for (int n = 0; n < NN; ++n) cmac(acc[n], a, sB[k * NN + n]);
    }
    __syncthreads();
#pragma unroll
    for (int n = 0; n < NN; ++n) tile[pos(t * NN + n)] = acc[n];
    __syncthreads();
    float4* dst = reinterpret_cast<float4*>(C + m0 * NN);
    for (int g = t; g < 128 * NN; g += 256) {
      const float2 x0 = tile[pos(2 * g)], x1 = tile[pos(2 * g + 1)];
      dst[g] = make_float4(x0.x, x0.y, x1.x, x1.y);
    }
    __syncthreads();
  }
}

typedef float floatx16 __attribute__((ext_vector_type(16)));

// NN = 16 NG (NG = 1, 2, 4: 4 to 6 N bits) on the FP32 matrix cores, each
// group of 16 outputs one MFMA column block.  A wave takes 2 x 32 rows at a time:
// every K value is one v_mfma_f32_32x32x2f32 per 32 rows in the real 2 x 2
// block form of the complex product (the MFMA's two k slots carry re a and
// im a; its 32 columns are the 16 outputs' re and im parts, B entered as
// [[re b, im b], [-im b, re b]]), so a row costs KK MFMA issues instead of
// 64 KK VALU FMAs.  Lane l loads only its own float of row l % 32's entry
// (re for l < 32, im above), so a load instruction covers 32 rows' entries
// once; accumulator register r holds row 8 (r / 4) + 4 (l / 32) + r % 4, so
// each store instruction writes two contiguous 128-byte row segments.  A's
// K values are loaded CH at a time ahead of their MFMAs; every (32-row
// group, column block) pair keeps its own accumulator chain.  Needs n_rows
// a multiple of 64.
template <int KK, int NG>
__global__ __launch_bounds__(256) void apply16_mfma_kernel(const float2* __restrict__ A,
                                                           const float2* __restrict__ B,
                                                           float2* __restrict__ C, ApplyArgs P) {
  constexpr int CH = KK < 8 ? KK : 8;
  constexpr int NN = 16 * NG;
  __shared__ float2 sB[KK * NN];
  __shared__ int64_t s_koff[KK];
  const int t = threadIdx.x;
  for (int idx = t; idx < KK * NN; idx += 256) {
    const int k = idx / NN, n = idx % NN;
    int64_t off = 0;
    for (int i = 0; i < P.nk; ++i)
      if (P.bk[i] >= 0 && ((k >> i) & 1)) off |= int64_t(1) << P.bk[i];
    for (int i = 0; i < P.nn; ++i)
      if ((n >> i) & 1) off |= int64_t(1) << P.bn[i];
    float2 v = make_float2(0.f, 0.f);
    for (int e = 0; e < (1 << P.n_b_extra); ++e) {
      int64_t o2 = off;
      for (int i = 0; i < P.n_b_extra; ++i)
        if ((e >> i) & 1) o2 |= int64_t(1) << P.b_extra[i];
      const float2 b = B[o2];
      v.x += b.x;
      v.y += b.y;
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
  const int lane = t & 63, wave = t >> 6;
  const int li = lane & 31, lh = lane >> 5;
  const int bn = li >> 1, bt = li & 1;
  const bool pick_re = lh == bt;
  const float sgn = (lh == 1 && bt == 0) ? -1.f : 1.f;
  const float* Af = reinterpret_cast<const float*>(A) + lh;
  float* Cf = reinterpret_cast<float*>(C);
  auto expand = [&](int64_t m) {
    for (int i = 0; i < P.nk; ++i) {
      const int p = P.kpos[i];
      m = ((m >> p) << (p + 1)) | (m & ((int64_t(1) << p) - 1));
    }
    return m;
  };
  const int64_t groups = P.n_rows >> 6;
  float mx = 0.f;   // largest magnitude this lane stores (NG = 1)
  for (int64_t g = int64_t(blockIdx.x) * 4 + wave; g < groups; g += int64_t(gridDim.x) * 4) {
    const int64_t b0 = 2 * expand(g * 64 + li), b1 = 2 * expand(g * 64 + 32 + li);
    floatx16 acc0[NG], acc1[NG];
#pragma unroll
    for (int c = 0; c < NG; ++c) {
      acc0[c] = floatx16{};
      acc1[c] = floatx16{};
    }
    auto mfma_chunk = [&](const float* a0, const float* a1, int k0) {
#pragma unroll
      for (int j = 0; j < CH; ++j) {
#pragma unroll
        for (int c = 0; c < NG; ++c) {
          const float2 b = sB[(k0 + j) * NN + c * 16 + bn];
          const float bv = sgn * (pick_re ? b.x : b.y);
          acc0[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0[j], bv, acc0[c], 0, 0, 0);
          acc1[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1[j], bv, acc1[c], 0, 0, 0);
        }
      }
    };
    if constexpr (NG == 1) {
      // memory-bound: K values CH at a time, a small register footprint
      // keeps more waves resident to cover the load latency
#pragma unroll 1
      for (int k0 = 0; k0 < KK; k0 += CH) {
        float a0[CH], a1[CH];
#pragma unroll
        for (int j = 0; j < CH; ++j) {
          const int64_t o = 2 * s_koff[k0 + j];
          a0[j] = Af[b0 + o];
          a1[j] = Af[b1 + o];
        }
        mfma_chunk(a0, a1, k0);
      }
    } else {
      // MFMA-bound: the next chunk's loads are issued before this chunk's
      // MFMAs so that their latency overlaps the matrix work
      float a0[CH], a1[CH];
#pragma unroll
      for (int j = 0; j < CH; ++j) {
        const int64_t o = 2 * s_koff[j];
        a0[j] = Af[b0 + o];
        a1[j] = Af[b1 + o];
      }
#pragma unroll 1
      for (int k0 = 0; k0 < KK; k0 += CH) {
        float n0[CH], n1[CH];
        if (k0 + CH < KK) {
#pragma unroll
          for (int j = 0; j < CH; ++j) {
            const int64_t o = 2 * s_koff[k0 + CH + j];
            n0[j] = Af[b0 + o];
            n1[j] = Af[b1 + o];
          }
        }
        mfma_chunk(a0, a1, k0);
        if (k0 + CH < KK) {
#pragma unroll
          for (int j = 0; j < CH; ++j) {
            a0[j] = n0[j];
            a1[j] = n1[j];
          }
        }
      }
    }
#pragma unroll
    for (int c = 0; c < NG; ++c)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t row = g * 64 + 8 * (r >> 2) + 4 * lh + (r & 3);
        Cf[(row * NN + c * 16 + bn) * 2 + bt] = acc0[c][r];
        Cf[((row + 32) * NN + c * 16 + bn) * 2 + bt] = acc1[c][r];
        if constexpr (NG == 1) mx = fmaxf(mx, fmaxf(fabsf(acc0[c][r]), fabsf(acc1[c][r])));
      }
  }
  // (one column block only: tracking the max costs the wider variants
  // registers and resident waves, so their callers take a separate pass)
  if constexpr (NG == 1) if (P.cmax) {
    // the largest |re|, |im| of C for the fp16 packing of a later GEMM
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    if (lane == 0) atomicMax(P.cmax, __float_as_uint(mx));
  }
}

// The LDS-tiled apply: lowest A bit is a K bit, every K bit below 8 + nk
// (a block's 256 rows are one run of A), KK <= 16, full blocks, and 16-byte
// aligned A and C (the plan's buffers are).
bool apply_tiled_ok(const ApplySmallDesc& d, const void* A, const void* C) {
  if (d.nk < 1 || d.nk > 4 || d.kpos[0] != 0 || d.a_bits - d.nk < 8) return false;
  for (int i = 0; i < d.nk; ++i)
    if (d.kpos[i] >= 8 + d.nk) return false;
  if (A && (reinterpret_cast<uintptr_t>(A) & 15)) return false;
  if (C && (reinterpret_cast<uintptr_t>(C) & 15)) return false;
  return true;
}

namespace {
bool apply_mfma_ok(const ApplySmallDesc& d) { return d.nn >= 4 && d.nn <= 6 && d.a_bits - d.nk >= 6; }
}  // namespace

int apply_variant(const ApplySmallDesc& d, const void* A, const void* C) {
  if (d.nn > 4) return 2;   // 32 or 64 outputs per row: matrix cores only
  if (d.variant == 2 && apply_mfma_ok(d)) return 2;
  const bool tiled = apply_tiled_ok(d, A, C);
  if (d.variant == 0) return tiled ? 1 : 0;
  if (tiled) return 1;
  return apply_mfma_ok(d) ? 2 : 0;
}

std::vector<int> apply_variant_candidates(const ApplySmallDesc& d) {
  if (d.nn > 4) return {2};
  std::vector<int> v{0};
  if (apply_mfma_ok(d)) v.push_back(2);
  return v;
}

namespace {
template <int NG>
void launch_apply_mfma(const float2* A, const float2* B, float2* C, const ApplyArgs& P, int nk, dim3 g, dim3 b,
                       hipStream_t s) {
  switch (1 << nk) {
    case 1: apply16_mfma_kernel<1, NG><<<g, b, 0, s>>>(A, B, C, P); break;
    case 2: apply16_mfma_kernel<2, NG><<<g, b, 0, s>>>(A, B, C, P); break;
    case 4: apply16_mfma_kernel<4, NG><<<g, b, 0, s>>>(A, B, C, P); break;
    case 8: apply16_mfma_kernel<8, NG><<<g, b, 0, s>>>(A, B, C, P); break;
    case 16: apply16_mfma_kernel<16, NG><<<g, b, 0, s>>>(A, B, C, P); break;
    case 32: apply16_mfma_kernel<32, NG><<<g, b, 0, s>>>(A, B, C, P); break;
    default: apply16_mfma_kernel<64, NG><<<g, b, 0, s>>>(A, B, C, P); break;
  }
}
}  // namespace

namespace {
// apply_tile_kernel (variant 1) or apply_small_kernel (variant 0)
void apply_scalar_kernels(const float2* A, const float2* B, float2* C, const ApplyArgs& P, const ApplySmallDesc& d,
                          int variant, hipStream_t s);
}  // namespace

void launch_apply_small(const float2* A, const float2* B, float2* C, const ApplySmallDesc& d,
                        hipStream_t s, uint32_t* cmax) {
  TN_REQUIRE(d.nk >= 0 && d.nk <= 6 && d.nn >= 0 && d.n_b_extra <= 12 && (d.nn <= 4 || apply_mfma_ok(d)),
             TN_ERR_UNSUPPORTED, "apply_small shape out of range");
  ApplyArgs P;
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
  const int variant = apply_variant(d, A, C);
  if (cmax) scale_clear_kernel<<<1, 1, 0, s>>>(cmax);
  if (variant == 2) {
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(ceil_div(P.n_rows, 256), grid_cap() * 2));
    const dim3 g = dim3(unsigned(blocks)), b = dim3(256);
    if (d.nn == 4) {
      P.cmax = cmax;   // computed as the kernel stores C
      cmax = nullptr;
      launch_apply_mfma<1>(A, B, C, P, d.nk, g, b, s);
    } else if (d.nn == 5) {
      launch_apply_mfma<2>(A, B, C, P, d.nk, g, b, s);
    } else {
      launch_apply_mfma<4>(A, B, C, P, d.nk, g, b, s);
    }
    TN_HIP(hipGetLastError());
  } else {
    apply_scalar_kernels(A, B, C, P, d, variant, s);
  }
  if (cmax) {
    // not computed by the kernel: a pass over the finished C
    const int64_t n = P.n_rows << d.nn;
    maxabs_kernel<<<dim3(unsigned(std::min<int64_t>(ceil_div(n, 256), grid_cap()))), dim3(256), 0, s>>>(C, n, cmax);
    TN_HIP(hipGetLastError());
  }
}

namespace {
void apply_scalar_kernels(const float2* A, const float2* B, float2* C, const ApplyArgs& P, const ApplySmallDesc& d,
                          int variant, hipStream_t s) {
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(ceil_div(P.n_rows, 256), grid_cap() * 2));
  const dim3 g = dim3(unsigned(blocks)), b = dim3(256);
  if (variant == 1) {
    switch (1 << d.nn) {
      case 1: apply_tile_kernel<1><<<g, b, 0, s>>>(A, B, C, P); break;
      case 2: apply_tile_kernel<2><<<g, b, 0, s>>>(A, B, C, P); break;
      case 4: apply_tile_kernel<4><<<g, b, 0, s>>>(A, B, C, P); break;
      case 8: apply_tile_kernel<8><<<g, b, 0, s>>>(A, B, C, P); break;
      default: apply_tile_kernel<16><<<g, b, 0, s>>>(A, B, C, P); break;
    }
    TN_HIP(hipGetLastError());
    return;
  }
  switch (1 << d.nn) {
    case 1: apply_small_kernel<1><<<g, b, 0, s>>>(A, B, C, P); break;
    case 2: apply_small_kernel<2><<<g, b, 0, s>>>(A, B, C, P); break;
    case 4: apply_small_kernel<4><<<g, b, 0, s>>>(A, B, C, P); break;
    case 8: apply_small_kernel<8><<<g, b, 0, s>>>(A, B, C, P); break;
    default: apply_small_kernel<16><<<g, b, 0, s>>>(A, B, C, P); break;
  }
  TN_HIP(hipGetLastError());
}
}  // namespace

// -------------------------------------------------------------- MFMA GEMM

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

struct GemmArgs {
  int64_t M, N, K;
  int64_t kchunk;       // K range per split
  int ksplit;
  int transA, transB;
  int tiles_m, tiles_n;
  int64_t kbase;        // first k of this launch (K-chunked launches)
  int beta;             // 1: add into C (later K chunks); 0: overwrite
};

// Block tile BM x BN complex outputs, BK complex per K step; 4 waves laid out
// WGM x WGN; each wave owns (BM/WGM) x (BN/WGN) = TM x TN MFMA tiles of
// 32 rows x 16 complex columns.
template <int BM, int BN, int BK, int WGM, int WGN, int PREC>
__global__ __launch_bounds__(256) void gemm_mfma_kernel(const float2* __restrict__ A,
                                                        const float2* __restrict__ B,
                                                        float2* __restrict__ C, GemmArgs P) {
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int TM = WM / 32, TN = WN / 16;
  static_assert(TM >= 1 && TN >= 1, "wave tile too small");
  constexpr int NP = PREC == TN_PREC_FP32 ? 0 : (PREC == TN_PREC_BF16X3 ? 2 : 3);
  // LDS: FP32 keeps float2; split modes keep NP packed bf16 planes.
  constexpr int LDK = NP == 0 ? BK + 1 : BK + 4;          // row stride (elements)
  constexpr int ELEM = NP == 0 ? 2 : NP;                   // 32-bit words per complex
  __shared__ __attribute__((aligned(16))) uint32_t lds[(BM + BN) * LDK * ELEM];
  uint32_t* As = lds;
  uint32_t* Bs = lds + BM * LDK * ELEM;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave / WGN) * WM, wn0 = (wave % WGN) * WN;

  // XCD-aware tile order: consecutive logical tiles land on one XCD.
  const int nblk = gridDim.x;
  int pid = blockIdx.x;
  if ((nblk & 7) == 0) pid = (pid & 7) * (nblk >> 3) + (pid >> 3);
  constexpr int GROUP = 8;
  const int group_size = GROUP * P.tiles_n;
  const int g = pid / group_size;
  const int first_m = g * GROUP;
  const int gm = min(P.tiles_m - first_m, GROUP);
  const int tm_idx = first_m + (pid % group_size) % gm;
  const int tn_idx = (pid % group_size) / gm;
  const int64_t m0 = int64_t(tm_idx) * BM, n0 = int64_t(tn_idx) * BN;

  const int zb = blockIdx.z;
  const int ks = zb % P.ksplit;
  const int64_t bidx = zb / P.ksplit;
  const int64_t kbeg = P.kbase + int64_t(ks) * P.kchunk;
  const int64_t kend = min(P.K, kbeg + P.kchunk);
  const float2* Ab = A + bidx * P.M * P.K;
  const float2* Bb = B + bidx * P.K * P.N;

  floatx16 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  constexpr int A_PER = (BM * BK + 255) / 256, B_PER = (BN * BK + 255) / 256;
  float2 ra[A_PER], rb[B_PER];

  auto load_tiles = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < A_PER; ++i) {
      const int idx = tid + 256 * i;
      int r, c;
      if (P.transA == 0) { r = idx / BK; c = idx % BK; } else { c = idx / BM; r = idx % BM; }
      const int64_t m = m0 + r, k = k0 + c;
      float2 v = make_float2(0.f, 0.f);
      if (idx < BM * BK && m < P.M && k < kend) v = P.transA == 0 ? Ab[m * P.K + k] : Ab[k * P.M + m];
      ra[i] = v;
    }
#pragma unroll
    for (int i = 0; i < B_PER; ++i) {
      const int idx = tid + 256 * i;
      int r, c;  // r = n, c = k
      if (P.transB == 1) { r = idx / BK; c = idx % BK; } else { c = idx / BN; r = idx % BN; }
      const int64_t n = n0 + r, k = k0 + c;
      float2 v = make_float2(0.f, 0.f);
      if (idx < BN * BK && n < P.N && k < kend) v = P.transB == 1 ? Bb[n * P.K + k] : Bb[k * P.N + n];
      rb[i] = v;
    }
  };
  auto store_tiles = [&]() {
#pragma unroll
    for (int i = 0; i < A_PER; ++i) {
      const int idx = tid + 256 * i;
      if (idx >= BM * BK) break;
      int r, c;
      if (P.transA == 0) { r = idx / BK; c = idx % BK; } else { c = idx / BM; r = idx % BM; }
      if constexpr (NP == 0) {
        As[(r * LDK + c) * 2] = __float_as_uint(ra[i].x);
        As[(r * LDK + c) * 2 + 1] = __float_as_uint(ra[i].y);
      } else {
        uint32_t w[NP];
        split_c<NP>(ra[i], w);
#pragma unroll
        for (int p = 0; p < NP; ++p) As[(p * BM + r) * LDK + c] = w[p];
      }
    }
#pragma unroll
    for (int i = 0; i < B_PER; ++i) {
      const int idx = tid + 256 * i;
      if (idx >= BN * BK) break;
      int r, c;
      if (P.transB == 1) { r = idx / BK; c = idx % BK; } else { c = idx / BN; r = idx % BN; }
      if constexpr (NP == 0) {
        Bs[(r * LDK + c) * 2] = __float_as_uint(rb[i].x);
        Bs[(r * LDK + c) * 2 + 1] = __float_as_uint(rb[i].y);
      } else {
        uint32_t w[NP];
        split_c<NP>(rb[i], w);
#pragma unroll
        for (int p = 0; p < NP; ++p) Bs[(p * BN + r) * LDK + c] = w[p];
      }
    }
  };

  const int li = lane & 31, lh = lane >> 5;
  const int bn_local = li >> 1, bt = li & 1;
  // B entry of the real 2x2 block form, branch-free per lane: FP32 lanes
  // pick re b (lh == bt) or im b and negate for (lh, bt) = (1, 0); packed
  // words rotate (odd lanes: (im, re)) and flip the sign of im (even lanes)
  const uint32_t sel_re = lh == bt ? 0xffffffffu : 0u, neg = (lh == 1 && bt == 0) ? 0x80000000u : 0u;
  const uint32_t brot = bt ? 16u : 0u, bxor = bt ? 0u : 0x80000000u;

  if (kbeg < kend) load_tiles(kbeg);
  for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
    __syncthreads();
    store_tiles();
    __syncthreads();
    if (k0 + BK < kend) load_tiles(k0 + BK);
    if constexpr (NP == 0) {
#pragma unroll
      for (int kk = 0; kk < BK; ++kk) {
        float av[TM], bv[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i)
          av[i] = __uint_as_float(As[((wm0 + i * 32 + li) * LDK + kk) * 2 + lh]);
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const int row = (wn0 + j * 16 + bn_local) * LDK + kk;
          const uint32_t br = Bs[row * 2], bi = Bs[row * 2 + 1];
          bv[j] = __uint_as_float(((br & sel_re) | (bi & ~sel_re)) ^ neg);
        }
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i], bv[j], acc[i][j], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 8) {
        u32x4 av[NP][TM], bv[NP][TN];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
#pragma unroll
          for (int i = 0; i < TM; ++i)
            av[p][i] = *reinterpret_cast<const u32x4*>(&As[(p * BM + wm0 + i * 32 + li) * LDK + kk + 4 * lh]);
#pragma unroll
          for (int j = 0; j < TN; ++j) {
            u32x4 w = *reinterpret_cast<const u32x4*>(&Bs[(p * BN + wn0 + j * 16 + bn_local) * LDK + kk + 4 * lh]);
#pragma unroll
            for (int q = 0; q < 4; ++q) w[q] = __builtin_amdgcn_alignbit(w[q], w[q], brot) ^ bxor;
            bv[p][j] = w;
          }
        }
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) {
            // smallest products first: the FP32 accumulator sees them before
            // the leading term is added
#pragma unroll
            for (int s = NP - 1; s >= 1; --s)
#pragma unroll
              for (int pa = 0; pa <= s; ++pa) {
                const int pb = s - pa;
                if (pb >= NP) continue;
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                    __builtin_bit_cast(bf16x8, av[pa][i]), __builtin_bit_cast(bf16x8, bv[pb][j]),
                    acc[i][j], 0, 0, 0);
              }
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                __builtin_bit_cast(bf16x8, av[0][i]), __builtin_bit_cast(bf16x8, bv[0][j]), acc[i][j],
                0, 0, 0);
          }
      }
    }
  }

  float* Cf = reinterpret_cast<float*>(C + (int64_t(ks) * gridDim.z / P.ksplit + bidx) * P.M * P.N);
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t m = m0 + wm0 + i * 32 + 8 * (r >> 2) + 4 * lh + (r & 3);
        const int64_t n = n0 + wn0 + j * 16 + bn_local;
        if (m < P.M && n < P.N) {
          float* c = Cf + (m * P.N + n) * 2 + bt;
          *c = P.beta ? *c + acc[i][j][r] : acc[i][j][r];
        }
      }
}

// Packed-plane complex GEMM for the split precisions.  Operands arrive as NP
// bf16 planes (from the permute/split pass) with k fastest, so a K tile is
// copied global -> registers -> LDS with 16-byte accesses and no conversion.
// LDS holds two stages (one barrier per K tile, bank-conflict-free XOR
// layout).  Each wave owns TM x TN MFMA tiles of 32 rows x
// 16 complex columns; a K step of 8 complex values is one
// v_mfma_f32_32x32x16_bf16 per product pair.
//
// Global loads are raw buffer loads on a descriptor per operand panel: rows
// past M (N) and k past the chunk end fall outside the descriptor's range and
// read as zero in hardware, so the K loop has no divergent branches.
struct PackedArgs {
  int64_t M, N, K;
  int64_t kchunk;
  int ksplit;
  int tiles_m, tiles_n;
  int order;                   // block order (see packed_tile_of)
  int64_t plane_a, plane_b;
  const uint32_t* smax_a;      // split-FP16: operand max bits (scale 2^s); else null
  const uint32_t* smax_b;
  int64_t kbase;               // first k of this launch (K-chunked launches)
  int beta;                    // 1: add into C (later K chunks); 0: overwrite
  int flush_tiles;             // direct-to-LDS kernel: add the accumulators into C
                               // every flush_tiles K tiles (0: only at the end)
  uint32_t* cmax;              // direct-to-LDS kernel, ksplit 1: largest |re|, |im| of
                               // the final C as float bits, combined with an atomic max
};

// Block -> output tile.  Workgroups are dispatched round-robin over the 8
// XCDs (block b runs on XCD b % 8).  Order 1 (XCD regions): the blocks of
// one XCD walk 4 x 8-tile regions (the 32 tiles its CUs hold at once share 4
// A and 8 B panels in that XCD's L2), and the 8 XCDs take 8 neighbouring
// regions (2 region rows x 4 region columns) so that the last-level cache
// sees the panels they share.  Order 0: each XCD takes a contiguous range of
// a grouped (8 tile rows) order.  Order 2: row-major in block order.
__device__ inline void packed_tile_of(int b, int nblk, const PackedArgs& P, int& tm, int& tn) {
  if (P.order == 2) {
    tm = b / P.tiles_n;
    tn = b % P.tiles_n;
    return;
  }
  if (P.order == 1) {
    const int x = b & 7, j = b >> 3;
    const int g = (j >> 5) * 8 + x, w = j & 31;
    const int RN = P.tiles_n >> 3;
    const int rm = (g / (2 * RN)) * 2 + (g & 1);
    const int rn = (g >> 1) % RN;
    tm = rm * 4 + (w & 3);
    tn = rn * 8 + (w >> 2);
    return;
  }
  int pid = b;
  if ((nblk & 7) == 0) pid = (pid & 7) * (nblk >> 3) + (pid >> 3);
  constexpr int GROUP = 8;
  const int group_size = GROUP * P.tiles_n;
  const int first_m = (pid / group_size) * GROUP;
  const int gm = min(P.tiles_m - first_m, GROUP);
  tm = first_m + (pid % group_size) % gm;
  tn = (pid % group_size) / gm;
}

__device__ inline __amdgpu_buffer_rsrc_t panel_rsrc(const uint32_t* base, uint32_t bytes) {
  // gfx9 raw buffer: stride 0, num_records in bytes, default dst_sel/format
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t*>(base), 0, int(bytes), 0x00020000);
}

// LDS tile rows of BK words (16-byte chunks, no padding); chunk c of row r
// is stored at position c ^ f(r).  With f as below, the 16-byte accesses of
// any 8 (32 banks) or 16 (64 banks) consecutive lanes hit distinct banks
// both for the copy-in pattern (KQ lanes per row, consecutive rows) and for
// the MFMA fragment reads (one chunk of 32 consecutive rows).
template <int BK>
__device__ __forceinline__ int lds_word(int r, int c) {
  static_assert(BK == 16 || BK == 32, "swizzle defined for 4 or 8 chunks per row");
  const int f = BK == 16 ? (((r >> 1) ^ (r >> 3)) & 3) : ((r ^ (r >> 3)) & 7);
  return r * BK + 4 * (c ^ f);
}

// Fragments of one K step (8 complex values) of a wave's TM x TN MFMA tiles
// from an LDS stage: every plane's A rows and B columns, raw words.
template <int BM, int BN, int BK, int NP, int TM, int TN>
__device__ __forceinline__ void packed_load_frags(const uint32_t* As, const uint32_t* Bs, int kk, u32x4 (&av)[NP][TM],
                                                  u32x4 (&bv)[NP][TN], int wm0, int wn0, int li, int lh,
                                                  int bn_local) {
#pragma unroll
  for (int p = 0; p < NP; ++p) {
#pragma unroll
    for (int i = 0; i < TM; ++i)
      av[p][i] = *reinterpret_cast<const u32x4*>(As + lds_word<BK>(p * BM + wm0 + i * 32 + li, kk / 4 + lh));
#pragma unroll
    for (int j = 0; j < TN; ++j)
      bv[p][j] = *reinterpret_cast<const u32x4*>(Bs + lds_word<BK>(p * BN + wn0 + j * 16 + bn_local, kk / 4 + lh));
  }
}

// The B block-form swizzle and one v_mfma_f32_32x32x16_bf16 (or _f16) per
// product pair (pa, pb), pa + pb < NP, smallest first, and MFMA tile; the
// tile loops are innermost so consecutive MFMAs use independent accumulators.
template <int NP, int TM, int TN, bool F16>
__device__ __forceinline__ void packed_mma(const u32x4 (&av)[NP][TM], u32x4 (&bv)[NP][TN], floatx16 (&acc)[TM][TN],
                                           uint32_t brot, uint32_t bxor) {
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) bv[p][j][q] = __builtin_amdgcn_alignbit(bv[p][j][q], bv[p][j][q], brot) ^ bxor;
#pragma unroll
  for (int s2 = NP - 1; s2 >= 0; --s2)
#pragma unroll
    for (int pa = 0; pa <= s2; ++pa) {
      const int pb = s2 - pa;
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          if constexpr (F16)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, av[pa][i]),
                                                               __builtin_bit_cast(f16x8, bv[pb][j]), acc[i][j], 0,
                                                               0, 0);
          else
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av[pa][i]),
                                                                __builtin_bit_cast(bf16x8, bv[pb][j]), acc[i][j],
                                                                0, 0, 0);
        }
    }
}

// One K tile of the packed GEMM from an LDS stage, K step by K step.
template <int BM, int BN, int BK, int NP, int TM, int TN, bool F16>
__device__ __forceinline__ void packed_multiply(const uint32_t* As, const uint32_t* Bs, floatx16 (&acc)[TM][TN],
                                                int wm0, int wn0, int li, int lh, int bn_local, uint32_t brot,
                                                uint32_t bxor) {
#pragma unroll
  for (int kk = 0; kk < BK; kk += 8) {
    u32x4 av[NP][TM], bv[NP][TN];
    packed_load_frags<BM, BN, BK, NP, TM, TN>(As, Bs, kk, av, bv, wm0, wn0, li, lh, bn_local);
    packed_mma<NP, TM, TN, F16>(av, bv, acc, brot, bxor);
  }
}

// Writes a wave's TM x TN accumulator tiles (32 rows x 16 complex columns
// each, rows from mw, complex columns from nw) to C (row-major M x N
// complex), times 2^shift, added to what C holds when `beta`; entries
// outside M x N are skipped.
template <int TM, int TN, bool F16>
__device__ __forceinline__ void packed_store_c(float* Cf, const floatx16 (&acc)[TM][TN], int64_t mw, int64_t nw,
                                               int lh, int bn_local, int bt, int64_t M, int64_t N, int shift,
                                               int beta) {
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t m = mw + i * 32 + 8 * (r >> 2) + 4 * lh + (r & 3);
        const int64_t n = nw + j * 16 + bn_local;
        if (m < M && n < N) {
          const float v = F16 ? ldexpf(acc[i][j][r], shift) : acc[i][j][r];
          float* c = Cf + (m * N + n) * 2 + bt;
          *c = beta ? *c + v : v;
        }
      }
}

// Adds (beta) or writes a wave's accumulator tiles into an exactly tiled C
// through a buffer descriptor on the wave's 64 x 64 complex block: one
// per-lane byte offset, and per element a uniform (scalar) row offset, so the
// flush needs almost no address registers.  `row_bytes` = 8 N.  Returns the
// largest magnitude among the floats this lane stored.
template <int TM, int TN, bool F16>
__device__ __forceinline__ float packed_flush_exact(__amdgpu_buffer_rsrc_t cb, const floatx16 (&acc)[TM][TN],
                                                    uint32_t lane_off, uint32_t row_bytes, int shift, int beta) {
  float mx = 0.f;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const uint32_t soff = uint32_t(i * 32 + 8 * (r >> 2) + (r & 3)) * row_bytes + uint32_t(j * 16 * 8);
        float v = F16 ? ldexpf(acc[i][j][r], shift) : acc[i][j][r];
        if (beta) v += __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(cb, lane_off, soff, 0));
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), cb, lane_off, soff, 0);
        mx = fmaxf(mx, fabsf(v));
      }
  return mx;
}

// Undoes the two operand scales of a split-FP16 GEMM.
__device__ __forceinline__ int packed_shift(const PackedArgs& P) {
  return P.smax_a ? -(f16_scale_exp(*P.smax_a) + f16_scale_exp(*P.smax_b)) : 0;
}

template <int BM, int BN, int BK, int WGM, int WGN, int NP, bool F16>
__global__ __launch_bounds__(WGM * WGN * 64) void gemm_packed_kernel(const uint32_t* __restrict__ Ap,
                                                          const uint32_t* __restrict__ Bp,
                                                          float2* __restrict__ C, PackedArgs P) {
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int TM = WM / 32, TN = WN / 16;
  static_assert(TM >= 1 && TN >= 1 && BK % 8 == 0, "bad tile");
  constexpr int A_WORDS = NP * BM * BK, B_WORDS = NP * BN * BK;
  constexpr int STAGE = A_WORDS + B_WORDS;
  extern __shared__ __attribute__((aligned(16))) uint32_t smem[];
  constexpr int KQ = BK / 4;                        // uint4 per row per plane
  constexpr int AQ = BM * KQ, BQ = BN * KQ;         // uint4 per plane
  constexpr int NT = WGM * WGN * 64;
  constexpr int A_PP = (AQ + NT - 1) / NT, B_PP = (BQ + NT - 1) / NT;  // per thread per plane
  constexpr uint32_t OOB = 0x80000000u;             // beyond every panel's range

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave / WGN) * WM, wn0 = (wave % WGN) * WN;

  int tm_idx, tn_idx;
  packed_tile_of(blockIdx.x, gridDim.x, P, tm_idx, tn_idx);
  const int64_t m0 = int64_t(tm_idx) * BM, n0 = int64_t(tn_idx) * BN;

  const int zb = blockIdx.z;
  const int ks = zb % P.ksplit;
  const int64_t bidx = zb / P.ksplit;
  const int64_t kbeg = P.kbase + int64_t(ks) * P.kchunk;
  const int64_t kend = min(P.K, kbeg + P.kchunk);
  const int klen = int(kend - kbeg);
  const int64_t rows_a = min<int64_t>(BM, P.M - m0), rows_b = min<int64_t>(BN, P.N - n0);

  // one descriptor per plane; its range ends after element (last row, kend)
  __amdgpu_buffer_rsrc_t src_a[NP], src_b[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    src_a[p] = panel_rsrc(Ap + bidx * P.M * P.K + p * P.plane_a + m0 * P.K + kbeg,
                          uint32_t(((rows_a - 1) * P.K + klen) * 4));
    src_b[p] = panel_rsrc(Bp + bidx * P.N * P.K + p * P.plane_b + n0 * P.K + kbeg,
                          uint32_t(((rows_b - 1) * P.K + klen) * 4));
  }
  // thread chunk i of a plane: row q / KQ, word column 4 (q % KQ), q = tid + NT i;
  // byte offset of that chunk at the start of the K chunk
  uint32_t off_a[A_PP], off_b[B_PP];
  int col_a[A_PP], col_b[B_PP];
#pragma unroll
  for (int i = 0; i < A_PP; ++i) {
    const int q = min(tid + NT * i, AQ - 1);
    off_a[i] = uint32_t((int64_t(q / KQ) * P.K + 4 * (q % KQ)) * 4);
    col_a[i] = 4 * (q % KQ);
  }
#pragma unroll
  for (int i = 0; i < B_PP; ++i) {
    const int q = min(tid + NT * i, BQ - 1);
    off_b[i] = uint32_t((int64_t(q / KQ) * P.K + 4 * (q % KQ)) * 4);
    col_b[i] = 4 * (q % KQ);
  }

  floatx16 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  using ASet = u32x4[NP][A_PP];
  using BSet = u32x4[NP][B_PP];
  u32x4 ra0[NP][A_PP], rb0[NP][B_PP];
  auto load = [&](int kl, ASet& ra, BSet& rb) {  // kl: word offset of the tile in the K chunk
    const uint32_t dk = uint32_t(kl) * 4;
#pragma unroll
    for (int i = 0; i < A_PP; ++i) {
      const uint32_t off = kl + col_a[i] < klen ? off_a[i] + dk : OOB;
#pragma unroll
      for (int p = 0; p < NP; ++p) ra[p][i] = __builtin_amdgcn_raw_buffer_load_b128(src_a[p], off, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < B_PP; ++i) {
      const uint32_t off = kl + col_b[i] < klen ? off_b[i] + dk : OOB;
#pragma unroll
      for (int p = 0; p < NP; ++p) rb[p][i] = __builtin_amdgcn_raw_buffer_load_b128(src_b[p], off, 0, 0);
    }
  };
  auto store = [&](int buf, const ASet& ra, const BSet& rb) {
    uint32_t* As = smem + buf * STAGE;
    uint32_t* Bs = As + A_WORDS;
#pragma unroll
    for (int i = 0; i < A_PP; ++i) {
      const int q = tid + NT * i;
      if (AQ % NT != 0 && q >= AQ) break;
#pragma unroll
      for (int p = 0; p < NP; ++p)
        *reinterpret_cast<u32x4*>(As + lds_word<BK>(p * BM + q / KQ, q % KQ)) = ra[p][i];
    }
#pragma unroll
    for (int i = 0; i < B_PP; ++i) {
      const int q = tid + NT * i;
      if (BQ % NT != 0 && q >= BQ) break;
#pragma unroll
      for (int p = 0; p < NP; ++p)
        *reinterpret_cast<u32x4*>(Bs + lds_word<BK>(p * BN + q / KQ, q % KQ)) = rb[p][i];
    }
  };

  const int li = lane & 31, lh = lane >> 5;
  const int bn_local = li >> 1, bt = li & 1;
  // B column of the real block form: even lanes (real part of C) take
  // (re b, -im b), odd lanes (imaginary part) take (im b, re b); as one
  // branch-free rotate-and-xor per word
  const uint32_t brot = bt ? 16u : 0u, bxor = bt ? 0u : 0x80000000u;

  auto multiply = [&](int buf) {
    const uint32_t* As = smem + buf * STAGE;
    packed_multiply<BM, BN, BK, NP, TM, TN, F16>(As, As + A_WORDS, acc, wm0, wn0, li, lh, bn_local, brot, bxor);
  };

  // K tile t (word offset kl = t BK) is multiplied from stage t % 2 while
  // tile t + 1 is loaded into registers; it goes to the other stage after
  int buf = 0;
  if (klen > 0) {
    load(0, ra0, rb0);
    store(0, ra0, rb0);
  }
  __syncthreads();
  for (int kl = 0; kl < klen; kl += BK) {
    const bool more = kl + BK < klen;
    if (more) load(kl + BK, ra0, rb0);
    multiply(buf);
    if (more) store(buf ^ 1, ra0, rb0);
    __syncthreads();
    buf ^= 1;
  }

  packed_store_c<TM, TN, F16>(reinterpret_cast<float*>(C + (int64_t(ks) * (gridDim.z / P.ksplit) + bidx) * P.M * P.N),
                              acc, m0 + wm0, n0 + wn0, lh, bn_local, bt, P.M, P.N, packed_shift(P), P.beta);
}

// Direct-to-LDS variant for exactly tiled GEMMs (M % BM == N % BN == 0 and
// every K chunk a whole number of BK tiles).  Each wave copies 64 x 16-byte
// chunks per instruction with buffer_load ... lds straight into the swizzled
// LDS layout (lane l lands at byte 16 l of its 1 KB block, so it fetches the
// logical chunk that the XOR layout stores there).  No staging registers are
// needed, so LDS holds three stages and the copy of K tile t + 2 is issued
// while tile t is multiplied: a load has two tiles of MFMA work to land.
// Synchronisation per tile: wait until this wave's copies of tile t are done
// (the ones of tile t + 1 may still be in flight), then one barrier, which
// also frees the stage tile t - 1 occupied.
template <int BM, int BN, int BK, int WGM, int WGN, int NP, bool F16>
__global__ __launch_bounds__(WGM * WGN * 64) void gemm_packed_dma_kernel(const uint32_t* __restrict__ Ap,
                                                              const uint32_t* __restrict__ Bp,
                                                              float2* __restrict__ C, PackedArgs P) {
#if defined(__HIP_DEVICE_COMPILE__)  // device-only builtins; the host pass needs only the stub
  constexpr int NW = WGM * WGN;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int TM = WM / 32, TN = WN / 16;
  constexpr int KQ = BK / 4;                         // 16-byte chunks per row
  constexpr int RPL = 64 / KQ;                       // rows covered by one wave-wide copy
  constexpr int AB = BM / RPL, BB = BN / RPL;        // row blocks per plane
  static_assert(AB % NW == 0 && BB % NW == 0, "row blocks must split evenly over the waves");
  constexpr int A_PW = NP * AB / NW, B_PW = NP * BB / NW;   // copies per wave per K tile
  constexpr int PER_TILE = A_PW + B_PW;
  static_assert(2 * PER_TILE <= 15, "vmcnt immediate");
  constexpr int A_WORDS = NP * BM * BK, B_WORDS = NP * BN * BK;
  constexpr int STAGE = A_WORDS + B_WORDS;
  extern __shared__ __attribute__((aligned(16))) uint32_t smem[];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm0 = (wave / WGN) * WM, wn0 = (wave % WGN) * WN;

  int tm_idx, tn_idx;
  packed_tile_of(blockIdx.x, gridDim.x, P, tm_idx, tn_idx);
  const int64_t m0 = int64_t(tm_idx) * BM, n0 = int64_t(tn_idx) * BN;
  const int zb = blockIdx.z;
  const int ks = zb % P.ksplit;
  const int64_t bidx = zb / P.ksplit;
  const int64_t kbeg = P.kbase + int64_t(ks) * P.kchunk;
  const int klen = int(min(P.K, kbeg + P.kchunk) - kbeg);
  const int ntiles = klen / BK;

  __amdgpu_buffer_rsrc_t src_a[NP], src_b[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    src_a[p] = panel_rsrc(Ap + bidx * P.M * P.K + p * P.plane_a + m0 * P.K + kbeg,
                          uint32_t(((BM - 1) * P.K + klen) * 4));
    src_b[p] = panel_rsrc(Bp + bidx * P.N * P.K + p * P.plane_b + n0 * P.K + kbeg,
                          uint32_t(((BN - 1) * P.K + klen) * 4));
  }
  // copy i of this wave: row block (NW i + wave) of the planes laid out one
  // after another; lane l takes row l / KQ of the block and the logical chunk
  // stored at physical position l % KQ
  uint32_t voff_a[A_PW], voff_b[B_PW];
#pragma unroll
  for (int i = 0; i < A_PW; ++i) {
    const int blk = (NW * i) % AB + wave;
    const int p = (NW * i) / AB;
    const int r = blk * RPL + lane / KQ;
    const int c = (lane % KQ) ^ ((lds_word<BK>(p * BM + r, 0) >> 2) & (KQ - 1));
    voff_a[i] = uint32_t((int64_t(r) * P.K + 4 * c) * 4);
  }
#pragma unroll
  for (int i = 0; i < B_PW; ++i) {
    const int blk = (NW * i) % BB + wave;
    const int p = (NW * i) / BB;
    const int r = blk * RPL + lane / KQ;
    const int c = (lane % KQ) ^ ((lds_word<BK>(p * BN + r, 0) >> 2) & (KQ - 1));
    voff_b[i] = uint32_t((int64_t(r) * P.K + 4 * c) * 4);
  }
  auto issue = [&](int t, int stage) {
    uint32_t* base = smem + stage * STAGE;
    const uint32_t dk = uint32_t(t * BK) * 4;
#pragma unroll
    for (int i = 0; i < A_PW; ++i) {
      const int p = (NW * i) / AB;
      uint32_t* dst = base + (p * BM + ((NW * i) % AB + wave) * RPL) * BK;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(src_a[p], (__attribute__((address_space(3))) void*)dst, 16,
                                               voff_a[i] + dk, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < B_PW; ++i) {
      const int p = (NW * i) / BB;
      uint32_t* dst = base + A_WORDS + (p * BN + ((NW * i) % BB + wave) * RPL) * BK;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(src_b[p], (__attribute__((address_space(3))) void*)dst, 16,
                                               voff_b[i] + dk, 0, 0, 0);
    }
  };

  floatx16 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  const int li = lane & 31, lh = lane >> 5;
  const int bn_local = li >> 1, bt = li & 1;
  const uint32_t brot = bt ? 16u : 0u, bxor = bt ? 0u : 0x80000000u;

  // the barrier is an s_barrier between compiler memory fences (no wait on
  // the copies still in flight); the vmcnt waits are explicit
  auto barrier = [&]() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  };
  // Per tile t (stage t % 3, fragments of its two K steps in registers F0 and
  // F1): read F1, multiply F0; then wait for tile t + 1 and pass the barrier
  // while those MFMAs run (every wave is done reading stage t % 3, so the copy
  // of tile t + 3 goes there), read the next tile's F0, multiply F1.
  static_assert(BK == 16, "two K steps per tile");
  // C block of this wave (exact tiles: every element in range)
  float2* Cw = C + (int64_t(ks) * (gridDim.z / P.ksplit) + bidx) * P.M * P.N + (m0 + wm0) * P.N + (n0 + wn0);
  const uint32_t row_bytes = uint32_t(P.N * 8);
  const __amdgpu_buffer_rsrc_t cb = __builtin_amdgcn_make_buffer_rsrc(
      Cw, 0, int(uint32_t(WM - 1) * row_bytes + uint32_t(WN * 8)), 0x00020000);
  const uint32_t lane_off = uint32_t(4 * (lane >> 5)) * row_bytes + uint32_t(((lane & 31) >> 1) * 8 + (lane & 1) * 4);
  const int shift = packed_shift(P);
  int beta = P.beta;
  u32x4 a0[NP][TM], b0[NP][TN], a1[NP][TM], b1[NP][TN];
  for (int t = 0; t < 3 && t < ntiles; ++t) issue(t, t);
  if (ntiles > 0) {
    if (ntiles > 2) __builtin_amdgcn_s_waitcnt(0x0F70 | (2 * PER_TILE));
    else if (ntiles > 1) __builtin_amdgcn_s_waitcnt(0x0F70 | PER_TILE);
    else __builtin_amdgcn_s_waitcnt(0x0F70);
    barrier();
    packed_load_frags<BM, BN, BK, NP, TM, TN>(smem, smem + A_WORDS, 0, a0, b0, wm0, wn0, li, lh, bn_local);
  }
  int stage = 0;
  for (int t = 0; t < ntiles; ++t) {
    const uint32_t* As = smem + stage * STAGE;
    packed_load_frags<BM, BN, BK, NP, TM, TN>(As, As + A_WORDS, 8, a1, b1, wm0, wn0, li, lh, bn_local);
    __builtin_amdgcn_sched_barrier(0);
    packed_mma<NP, TM, TN, F16>(a0, b0, acc, brot, bxor);
    __builtin_amdgcn_sched_barrier(0);
    if (t + 1 < ntiles) {
      // this wave's reads of stage t % 3 are complete and tile t + 1 landed
      // (tile t + 2's copies may still be in flight)
      if (t + 2 < ntiles) __builtin_amdgcn_s_waitcnt(0x0070 | PER_TILE);   // vmcnt(PER_TILE), lgkmcnt(0)
      else __builtin_amdgcn_s_waitcnt(0x0070);                             // vmcnt(0), lgkmcnt(0)
      barrier();
      if (t + 3 < ntiles) issue(t + 3, stage);
      const int next = stage == 2 ? 0 : stage + 1;
      const uint32_t* An = smem + next * STAGE;
      packed_load_frags<BM, BN, BK, NP, TM, TN>(An, An + A_WORDS, 0, a0, b0, wm0, wn0, li, lh, bn_local);
      stage = next;
    }
    __builtin_amdgcn_sched_barrier(0);
    packed_mma<NP, TM, TN, F16>(a1, b1, acc, brot, bxor);
    __builtin_amdgcn_sched_barrier(0);
    if (P.flush_tiles > 0 && (t + 1) % P.flush_tiles == 0 && t + 1 < ntiles) {
      // cut the FP32 accumulator chain: add this K chunk's sums into C
      packed_flush_exact<TM, TN, F16>(cb, acc, lane_off, row_bytes, shift, beta);
      beta = 1;
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
          for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
    }
  }

  const float mx = packed_flush_exact<TM, TN, F16>(cb, acc, lane_off, row_bytes, shift, beta);
  if (P.cmax) {
    // the largest |re|, |im| of C for the fp16 packing of a later GEMM: a
    // wave reduction, the block's waves through LDS, one atomic per block
    __shared__ float wave_max[NW];
    float m = mx;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    if (lane == 0) wave_max[wave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      float b = wave_max[0];
#pragma unroll
      for (int w = 1; w < NW; ++w) b = fmaxf(b, wave_max[w]);
      atomicMax(P.cmax, __float_as_uint(b));
    }
  }
#endif
}

__global__ __launch_bounds__(256) void reduce_splitk_kernel(const float2* __restrict__ part,
                                                            float2* __restrict__ C, int ksplit,
                                                            int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    double sx = 0.0, sy = 0.0;     // FP64: up to 32768 partials per entry
    for (int k = 0; k < ksplit; ++k) {
      const float2 v = part[int64_t(k) * n + i];
      sx += v.x;
      sy += v.y;
    }
    C[i] = make_float2(float(sx), float(sy));
  }
}

// ---------------------------------------------------------- tile shapes
//
// Candidate block tiles (rows x complex columns); GemmDesc::tile picks one
// (-1: the shape heuristic below), the autotuner times the candidates.
namespace {
struct TileShape {
  int bm, bn;
};
constexpr TileShape kUnpackedTiles[4] = {{256, 16}, {128, 32}, {128, 64}, {64, 64}};
constexpr TileShape kPackedTiles[6] = {{256, 16}, {128, 32}, {128, 64}, {256, 128}, {128, 128}, {256, 128}};

constexpr int64_t kAccChunk = 4096;   // complex k per FP32 accumulator chain (all MFMA GEMMs)

// Tile 5 (direct-to-LDS copies) needs whole tiles in M, N and K.
bool dma_exact(const GemmDesc& g) {
  // the C flush addresses a wave's 64-row block with 32-bit byte offsets
  return g.packed && (g.precision == TN_PREC_BF16X3 || g.precision == TN_PREC_F16X3) && g.M % 256 == 0 &&
         g.N % 128 == 0 && g.K % 16 == 0 && 64 * 8 * g.N < (int64_t(1) << 31);
}

int default_tile(const GemmDesc& g) {
  if (g.N <= 16) return 0;
  if (g.N <= 32) return 1;
  if (!g.packed && g.M <= 64 && g.N <= 64) return 3;   // one 64 x 64 tile
  if (g.packed && (g.precision == TN_PREC_BF16X3 || g.precision == TN_PREC_F16X3) && g.N >= 128 && g.M >= 256 &&
      g.M * g.N >= (int64_t(1) << 22))
    return dma_exact(g) ? 5 : 3;
  return 2;
}

int tile_of(const GemmDesc& g) { return g.tile >= 0 ? g.tile : default_tile(g); }

// K step (complex values) of a tile.
int tile_bk(const GemmDesc& g, int id) {
  if (!g.packed) return g.precision == TN_PREC_FP32 ? 8 : 16;
  if (g.precision == TN_PREC_BF16X6) return 16;
  return (id == 3 || id == 4 || id == 5) ? 16 : 32;
}

int choose_ksplit(const GemmDesc& g, int id, int64_t* kchunk) {
  const TileShape t = g.packed ? kPackedTiles[id] : kUnpackedTiles[id];
  const int bk = tile_bk(g, id);
  const int64_t tiles = ceil_div(g.M, t.bm) * ceil_div(g.N, t.bn) * g.batch;
  const int64_t ksteps = ceil_div(g.K, bk);
  const int64_t minsteps = g.packed ? 8 : 16;
  int ks = 1;
  while (tiles * ks < 1024 && ksteps / (ks * 2) >= minsteps && ks < 256) ks *= 2;
  // once split, keep every block's FP32 chain within kAccChunk complex k
  // (few-tile GEMMs with very long K), up to 32768 splits per launch
  if (ks > 1)
    while (ceil_div(ksteps, ks) * bk > kAccChunk && ksteps / (ks * 2) >= minsteps &&
           g.batch * ks * 2 <= 32768)
      ks *= 2;
  *kchunk = ceil_div(ksteps, ks) * bk;
  return int(ceil_div(g.K, *kchunk));
}
}  // namespace

int gemm_tile_of(const GemmDesc& g) { return tile_of(g); }

int64_t gemm_dispatches(const GemmDesc& g) {
  int64_t kchunk = 0;
  const int id = tile_of(g);
  const int ksplit = choose_ksplit(g, id, &kchunk);
  return ksplit == 1 && !(g.packed && id == 5) ? ceil_div(g.K, kAccChunk) : 1;
}

std::vector<int> gemm_tile_candidates(const GemmDesc& g) {
  if (!g.packed) return {0, 1, 2, 3};
  if (g.precision == TN_PREC_BF16X6) return {0, 1, 2, 4};
  if (dma_exact(g)) return {0, 1, 2, 3, 4, 5};
  return {0, 1, 2, 3, 4};
}

size_t gemm_workspace_bytes(const GemmDesc& g) {
  int64_t kchunk;
  const int ks = choose_ksplit(g, tile_of(g), &kchunk);
  return ks > 1 ? size_t(ks) * size_t(g.batch * g.M * g.N) * sizeof(float2) : 0;
}

template <int BM, int BN, int BK, int WGM, int WGN, int PREC>
static void launch_gemm_cfg(const float2* A, const float2* B, float2* C, const GemmArgs& P,
                            int64_t batch, hipStream_t s) {
  dim3 grid(unsigned(P.tiles_m * P.tiles_n), 1, unsigned(batch * P.ksplit));
  gemm_mfma_kernel<BM, BN, BK, WGM, WGN, PREC><<<grid, 256, 0, s>>>(A, B, C, P);
}

template <int PREC, int BK>
static void launch_gemm_prec(const float2* A, const float2* B, float2* C, const GemmArgs& P,
                             int64_t batch, int id, hipStream_t s) {
  switch (id) {
    case 0: launch_gemm_cfg<256, 16, BK, 4, 1, PREC>(A, B, C, P, batch, s); break;
    case 1: launch_gemm_cfg<128, 32, BK, 4, 1, PREC>(A, B, C, P, batch, s); break;
    case 3: launch_gemm_cfg<64, 64, BK, 2, 2, PREC>(A, B, C, P, batch, s); break;
    default: launch_gemm_cfg<128, 64, BK, 2, 2, PREC>(A, B, C, P, batch, s); break;
  }
}

template <int BM, int BN, int BK, int WGM, int WGN, int NP, bool F16>
static void launch_packed_cfg(const uint32_t* A, const uint32_t* B, float2* C, const PackedArgs& P,
                              int64_t batch, hipStream_t s) {
  constexpr size_t lds = size_t(2) * NP * (BM + BN) * BK * sizeof(uint32_t);
  static_assert(lds <= 160 * 1024, "LDS tile exceeds the 160 KB of a CU");
  static bool attr_set = false;
  if (!attr_set) {
    TN_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm_packed_kernel<BM, BN, BK, WGM, WGN, NP, F16>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
    attr_set = true;
  }
  dim3 grid(unsigned(P.tiles_m * P.tiles_n), 1, unsigned(batch * P.ksplit));
  gemm_packed_kernel<BM, BN, BK, WGM, WGN, NP, F16><<<grid, WGM * WGN * 64, lds, s>>>(A, B, C, P);
}

template <int BM, int BN, int BK, int WGM, int WGN, int NP, bool F16>
static void launch_packed_dma(const uint32_t* A, const uint32_t* B, float2* C, const PackedArgs& P,
                              int64_t batch, hipStream_t s) {
  constexpr size_t lds = size_t(3) * NP * (BM + BN) * BK * sizeof(uint32_t);
  static_assert(lds <= 160 * 1024, "LDS stages exceed the 160 KB of a CU");
  static bool attr_set = false;
  if (!attr_set) {
    TN_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm_packed_dma_kernel<BM, BN, BK, WGM, WGN, NP, F16>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
    attr_set = true;
  }
  dim3 grid(unsigned(P.tiles_m * P.tiles_n), 1, unsigned(batch * P.ksplit));
  gemm_packed_dma_kernel<BM, BN, BK, WGM, WGN, NP, F16><<<grid, WGM * WGN * 64, lds, s>>>(A, B, C, P);
}

template <int NP, int BK, bool F16>
static void launch_packed_np(const uint32_t* A, const uint32_t* B, float2* C, const PackedArgs& P,
                             int64_t batch, int id, hipStream_t s) {
  switch (id) {
    case 0: launch_packed_cfg<256, 16, BK, 4, 1, NP, F16>(A, B, C, P, batch, s); break;
    case 1: launch_packed_cfg<128, 32, BK, 4, 1, NP, F16>(A, B, C, P, batch, s); break;
    case 3:
      if constexpr (NP == 2) { launch_packed_cfg<256, 128, 16, 4, 2, 2, F16>(A, B, C, P, batch, s); break; }
      [[fallthrough]];
    case 4: launch_packed_cfg<128, 128, 16, 2, 2, NP, F16>(A, B, C, P, batch, s); break;
    case 5:
      if constexpr (NP == 2) { launch_packed_dma<256, 128, 16, 4, 2, 2, F16>(A, B, C, P, batch, s); break; }
      launch_packed_cfg<128, 128, 16, 2, 2, NP, F16>(A, B, C, P, batch, s);
      break;
    default: launch_packed_cfg<128, 64, BK, 2, 2, NP, F16>(A, B, C, P, batch, s); break;
  }
}

void launch_gemm(const float2* A, const float2* B, float2* C, const GemmDesc& g, void* work,
                 const uint32_t* smax_a, const uint32_t* smax_b, hipStream_t s, uint32_t* cmax) {
  TN_REQUIRE(g.M >= 1 && g.N >= 1 && g.K >= 1 && g.batch >= 1, TN_ERR_ARG, "bad GEMM shape");
  TN_REQUIRE(!g.packed || g.K % 4 == 0, TN_ERR_ARG, "internal: packed GEMM needs K % 4 == 0");
  const int id = tile_of(g);
  const auto cands = gemm_tile_candidates(g);
  TN_REQUIRE(std::find(cands.begin(), cands.end(), id) != cands.end(), TN_ERR_ARG, "internal: bad tile id");
  const TileShape t = g.packed ? kPackedTiles[id] : kUnpackedTiles[id];
  int64_t kchunk = 0;
  const int ksplit = choose_ksplit(g, id, &kchunk);
  const int tiles_m = int(ceil_div(g.M, t.bm)), tiles_n = int(ceil_div(g.N, t.bn));
  TN_REQUIRE(int64_t(tiles_m) * tiles_n < (int64_t(1) << 31) && g.batch * ksplit <= 65535,
             TN_ERR_UNSUPPORTED, "GEMM grid too large");
  float2* out = C;
  if (ksplit > 1) {
    TN_REQUIRE(work != nullptr, TN_ERR_WORKSPACE, "split-K GEMM needs workspace");
    out = static_cast<float2*>(work);
  }
  if (g.packed) {
    PackedArgs P;
    P.M = g.M;
    P.N = g.N;
    P.K = g.K;
    P.plane_a = g.plane_a;
    P.plane_b = g.plane_b;
    P.smax_a = nullptr;
    P.smax_b = nullptr;
    P.kbase = 0;
    P.beta = 0;
    P.flush_tiles = 0;
    P.cmax = nullptr;
    P.ksplit = ksplit;
    P.kchunk = kchunk;
    P.tiles_m = tiles_m;
    P.tiles_n = tiles_n;
    const bool regions_fit = tiles_m % 8 == 0 && tiles_n % 8 == 0 && (int64_t(tiles_m) * tiles_n) % 256 == 0;
    P.order = g.order == 2 ? 2 : (g.order == 0 || !regions_fit) ? 0 : 1;
    // buffer offsets are 32-bit: a (BM x K) panel of one plane must stay below 2 GiB
    TN_REQUIRE(int64_t(t.bm > t.bn ? t.bm : t.bn) * g.K * 4 < (int64_t(1) << 31), TN_ERR_UNSUPPORTED,
               "packed GEMM: K too long for one panel");
    const uint32_t* Ap = reinterpret_cast<const uint32_t*>(A);
    const uint32_t* Bp = reinterpret_cast<const uint32_t*>(B);
    if (g.precision == TN_PREC_F16X3) {
      TN_REQUIRE(smax_a && smax_b, TN_ERR_ARG, "internal: split-FP16 GEMM needs operand scales");
      P.smax_a = smax_a;
      P.smax_b = smax_b;
    }
    // Long contractions cut their FP32 accumulator chains every kAccChunk
    // complex k, adding each chunk's sums into C in K order: inside the
    // direct-to-LDS kernel (tile 5), else as one launch per K chunk.
    const int64_t nchunks = ksplit == 1 && id != 5 ? ceil_div(g.K, kAccChunk) : 1;
    if (id == 5) P.flush_tiles = int(kAccChunk / 16);
    if (cmax && id == 5 && ksplit == 1) {
      scale_clear_kernel<<<1, 1, 0, s>>>(cmax);
      P.cmax = cmax;
      cmax = nullptr;   // computed in the kernel's final flush
    }
    for (int64_t c = 0; c < nchunks; ++c) {
      if (nchunks > 1) {
        P.kbase = c * kAccChunk;
        P.kchunk = kAccChunk;
        P.beta = c > 0 ? 1 : 0;
      }
      if (g.precision == TN_PREC_BF16X6) launch_packed_np<3, 16, false>(Ap, Bp, out, P, g.batch, id, s);
      else if (g.precision == TN_PREC_F16X3) launch_packed_np<2, 32, true>(Ap, Bp, out, P, g.batch, id, s);
      else launch_packed_np<2, 32, false>(Ap, Bp, out, P, g.batch, id, s);
    }
  } else {
    const int prec = g.precision == TN_PREC_BF16X3 || g.precision == TN_PREC_BF16X6 ? g.precision
                                                                                     : TN_PREC_FP32;
    GemmArgs P;
    P.M = g.M;
    P.N = g.N;
    P.K = g.K;
    P.transA = g.transA;
    P.transB = g.transB;
    P.ksplit = ksplit;
    P.kchunk = kchunk;
    P.tiles_m = tiles_m;
    P.tiles_n = tiles_n;
    P.kbase = 0;
    P.beta = 0;
    const int64_t nchunks = ksplit == 1 ? ceil_div(g.K, kAccChunk) : 1;   // as for the packed GEMMs
    for (int64_t c = 0; c < nchunks; ++c) {
      if (nchunks > 1) {
        P.kbase = c * kAccChunk;
        P.kchunk = kAccChunk;
        P.beta = c > 0 ? 1 : 0;
      }
      switch (prec) {
        case TN_PREC_FP32: launch_gemm_prec<TN_PREC_FP32, 8>(A, B, out, P, g.batch, id, s); break;
        case TN_PREC_BF16X3: launch_gemm_prec<TN_PREC_BF16X3, 16>(A, B, out, P, g.batch, id, s); break;
        default: launch_gemm_prec<TN_PREC_BF16X6, 16>(A, B, out, P, g.batch, id, s); break;
      }
    }
  }
  TN_HIP(hipGetLastError());
  if (ksplit > 1) {
    const int64_t n = g.batch * g.M * g.N;
    const int64_t blocks = std::min<int64_t>(ceil_div(n, 256), grid_cap());
    reduce_splitk_kernel<<<dim3(unsigned(blocks)), 256, 0, s>>>(out, C, ksplit, n);
    TN_HIP(hipGetLastError());
  }
  if (cmax) {
    // not fused into this kernel: a pass over the finished C
    const int64_t n = g.batch * g.M * g.N;
    scale_clear_kernel<<<1, 1, 0, s>>>(cmax);
    maxabs_kernel<<<dim3(unsigned(std::min<int64_t>(ceil_div(n, 256), grid_cap()))), dim3(256), 0, s>>>(C, n, cmax);
    TN_HIP(hipGetLastError());
  }
}

// --------------------------------------------------------------------- dot

__global__ __launch_bounds__(256) void dot_partial_kernel(const float2* __restrict__ A,
                                                          const float2* __restrict__ B,
                                                          double2* __restrict__ part, int64_t K,
                                                          int64_t m, int64_t n) {
  __shared__ double2 red[256];
  const int64_t b = blockIdx.y;                 // output (batch, row of A, row of B)
  const int64_t bi = b / (m * n), mi = (b / n) % m, ni = b % n;
  const float2* a = A + (bi * m + mi) * K;
  const float2* bb = B + (bi * n + ni) * K;
  double sr = 0.0, si = 0.0;
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < K; k += int64_t(gridDim.x) * 256) {
    const float2 x = a[k], y = bb[k];
    sr += double(x.x) * double(y.x) - double(x.y) * double(y.y);
    si += double(x.x) * double(y.y) + double(x.y) * double(y.x);
  }
  red[threadIdx.x] = make_double2(sr, si);
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      red[threadIdx.x].x += red[threadIdx.x + w].x;
      red[threadIdx.x].y += red[threadIdx.x + w].y;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[b * gridDim.x + blockIdx.x] = red[0];
}

__global__ void dot_final_kernel(const double2* __restrict__ part, float2* __restrict__ C, int nparts,
                                 int64_t batch) {
  const int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  double sr = 0.0, si = 0.0;
  for (int p = 0; p < nparts; ++p) {
    sr += part[b * nparts + p].x;
    si += part[b * nparts + p].y;
  }
  C[b] = make_float2(float(sr), float(si));
}

static int dot_parts(int64_t K) { return int(std::max<int64_t>(1, std::min<int64_t>(1024, ceil_div(K, 4096)))); }

size_t dot_workspace_bytes(int64_t K, int64_t batch) {
  return size_t(dot_parts(K)) * size_t(batch) * sizeof(double2);
}

void launch_dot(const float2* A, const float2* B, float2* C, int64_t K, int64_t batch, int64_t m,
                int64_t n, void* work, hipStream_t s) {
  TN_REQUIRE(work != nullptr, TN_ERR_WORKSPACE, "dot needs workspace");
  TN_REQUIRE(m >= 1 && n >= 1, TN_ERR_ARG, "dot row counts must be positive");
  const int64_t outs = batch * m * n;
  TN_REQUIRE(outs <= 65535, TN_ERR_UNSUPPORTED, "dot batch too large");
  const int parts = dot_parts(K);
  dot_partial_kernel<<<dim3(parts, unsigned(outs)), 256, 0, s>>>(A, B, static_cast<double2*>(work), K, m, n);
  TN_HIP(hipGetLastError());
  dot_final_kernel<<<dim3(unsigned(ceil_div(outs, 256))), 256, 0, s>>>(static_cast<double2*>(work), C,
                                                                      parts, outs);
  TN_HIP(hipGetLastError());
}

// ------------------------------------------------------ skinny long-K GEMM

// C[m][n] = sum_k A(m, k) B(k, n) for M, N <= 16 (M N <= 64) over a long K:
// every thread accumulates all M x N outputs for its strided share of k in
// FP32 registers, reading A and B once (M + N complex per k), so the pass
// streams at HBM rate where an MFMA tile would mostly idle.  A(m, k) sits
// at A[m * sam + k * sak], B(k, n) at B[k * sbk + n * sbn].  Block sums go
// to `part` in FP64 and skinny_final_kernel adds them in FP64.
constexpr int kSkinnyBlocks = 1024;

template <int MM, int NN>
__global__ __launch_bounds__(256) void skinny_partial_kernel(const float2* __restrict__ A,
                                                             const float2* __restrict__ B,
                                                             double2* __restrict__ part, int64_t K,
                                                             int64_t sam, int64_t sak, int64_t sbk,
                                                             int64_t sbn) {
  float2 acc[MM][NN];
#pragma unroll
  for (int m = 0; m < MM; ++m)
#pragma unroll
    for (int n = 0; n < NN; ++n) acc[m][n] = make_float2(0.f, 0.f);
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < K; k += int64_t(gridDim.x) * 256) {
    float2 a[MM], b[NN];
#pragma unroll
    for (int m = 0; m < MM; ++m) a[m] = A[m * sam + k * sak];
#pragma unroll
    for (int n = 0; n < NN; ++n) b[n] = B[k * sbk + n * sbn];
#pragma unroll
    for (int m = 0; m < MM; ++m)
#pragma unroll
      for (int n = 0; n < NN; ++n) cmac(acc[m][n], a[m], b[n]);
  }
  __shared__ double2 red[4][MM * NN];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int m = 0; m < MM; ++m)
#pragma unroll
    for (int n = 0; n < NN; ++n) {
      double re = acc[m][n].x, im = acc[m][n].y;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        re += __shfl_xor(re, o);
        im += __shfl_xor(im, o);
      }
      if (lane == 0) red[w][m * NN + n] = make_double2(re, im);
    }
  __syncthreads();
  for (int i = threadIdx.x; i < MM * NN; i += 256) {
    const double2 v = make_double2(red[0][i].x + red[1][i].x + red[2][i].x + red[3][i].x,
                                   red[0][i].y + red[1][i].y + red[2][i].y + red[3][i].y);
    part[int64_t(blockIdx.x) * (MM * NN) + i] = v;
  }
}

__global__ void skinny_final_kernel(const double2* __restrict__ part, float2* __restrict__ C, int nparts,
                                    int outs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= outs) return;
  double sr = 0.0, si = 0.0;
  for (int p = 0; p < nparts; ++p) {
    sr += part[int64_t(p) * outs + i].x;
    si += part[int64_t(p) * outs + i].y;
  }
  C[i] = make_float2(float(sr), float(si));
}

static int skinny_blocks(int64_t K) {
  return int(std::max<int64_t>(1, std::min<int64_t>(kSkinnyBlocks, ceil_div(K, 256 * 16))));
}

size_t skinny_workspace_bytes(int64_t K, int64_t m, int64_t n) {
  return size_t(skinny_blocks(K)) * size_t(m * n) * sizeof(double2);
}

bool skinny_supported(int64_t m, int64_t n) {
  auto p2 = [](int64_t x) { return x >= 1 && x <= 16 && (x & (x - 1)) == 0; };
  return p2(m) && p2(n) && m * n <= 64 && m * n > 1;
}

template <int MM, int NN>
static void launch_skinny_mn(const float2* A, const float2* B, double2* part, int64_t K, int64_t sam,
                             int64_t sak, int64_t sbk, int64_t sbn, int blocks, hipStream_t s) {
  skinny_partial_kernel<MM, NN><<<blocks, 256, 0, s>>>(A, B, part, K, sam, sak, sbk, sbn);
}

void launch_skinny(const float2* A, const float2* B, float2* C, int64_t K, int64_t m, int64_t n, int transA,
                   int transB, void* work, hipStream_t s) {
  TN_REQUIRE(work != nullptr, TN_ERR_WORKSPACE, "skinny GEMM needs workspace");
  TN_REQUIRE(skinny_supported(m, n), TN_ERR_ARG, "internal: skinny GEMM shape");
  // transA = 0: A[m][k]; 1: A[k][m].  transB = 0: B[k][n]; 1: B[n][k].
  const int64_t sam = transA ? 1 : K, sak = transA ? m : 1;
  const int64_t sbk = transB ? 1 : n, sbn = transB ? K : 1;
  const int blocks = skinny_blocks(K);
  double2* part = static_cast<double2*>(work);
  const int key = int(m) * 32 + int(n);
  switch (key) {
#define TN_SKINNY(MM, NN) \
  case MM * 32 + NN: launch_skinny_mn<MM, NN>(A, B, part, K, sam, sak, sbk, sbn, blocks, s); break;
    TN_SKINNY(1, 2) TN_SKINNY(2, 1) TN_SKINNY(1, 4) TN_SKINNY(4, 1) TN_SKINNY(2, 2)
    TN_SKINNY(1, 8) TN_SKINNY(8, 1) TN_SKINNY(2, 4) TN_SKINNY(4, 2) TN_SKINNY(1, 16) TN_SKINNY(16, 1)
    TN_SKINNY(2, 8) TN_SKINNY(8, 2) TN_SKINNY(4, 4) TN_SKINNY(2, 16) TN_SKINNY(16, 2) TN_SKINNY(4, 8)
    TN_SKINNY(8, 4) TN_SKINNY(4, 16) TN_SKINNY(16, 4) TN_SKINNY(8, 8)
#undef TN_SKINNY
    default: throw Error(TN_ERR_ARG, "internal: skinny GEMM shape");
  }
  TN_HIP(hipGetLastError());
  const int outs = int(m * n);
  skinny_final_kernel<<<dim3(unsigned(ceil_div(outs, 256))), 256, 0, s>>>(part, C, blocks, outs);
  TN_HIP(hipGetLastError());
}

// ----------------------------------------------------- jobs, leaves, output

__global__ void set_job_kernel(int64_t* ctl, int64_t job) { ctl[0] = job; }
__global__ void advance_job_kernel(int64_t* ctl) { ctl[0] += 1; }

void launch_set_job(int64_t* ctl, int64_t job, hipStream_t s) {
  set_job_kernel<<<1, 1, 0, s>>>(ctl, job);
  TN_HIP(hipGetLastError());
}
void launch_advance_job(int64_t* ctl, hipStream_t s) {
  advance_job_kernel<<<1, 1, 0, s>>>(ctl);
  TN_HIP(hipGetLastError());
}

template <typename T>
__global__ __launch_bounds__(256) void gather_leaves_kernel(const T* __restrict__ full,
                                                            T* __restrict__ arena,
                                                            const LeafDesc* __restrict__ descs,
                                                            const int8_t* __restrict__ bits,
                                                            int n_qubits,
                                                            const int64_t* __restrict__ ctl) {
  const LeafDesc& d = descs[blockIdx.x];
  const int64_t job = ctl[0], sbeg = ctl[1], scount = ctl[2];
  const int64_t bs = job / scount;
  const int64_t slice = sbeg + job % scount;
  int64_t fixed_off = 0;
  for (int f = 0; f < d.n_fixed; ++f) {
    const LeafFixed& x = d.fixed[f];
    const int v = x.kind == 0 ? int(bits[bs * n_qubits + x.which]) : int((slice >> x.which) & 1);
    if (v) fixed_off |= int64_t(1) << x.pos;
  }
  const int n = 1 << d.out_bits;
  for (int o = threadIdx.x; o < n; o += blockDim.x) {
    int64_t off = fixed_off;
    for (int j = 0; j < d.out_bits; ++j)
      if ((o >> j) & 1) off |= int64_t(1) << d.in_pos[j];
    arena[d.dst_off + o] = full[d.src_off + off];
  }
}

template <typename T>
static void gather_leaves(const T* full, T* arena, const LeafDesc* descs, int n_leaves, int max_out,
                          const int8_t* bits, int n_qubits, const int64_t* ctl, hipStream_t s) {
  if (n_leaves == 0) return;
  const int threads = std::min(256, std::max(64, 1 << max_out));
  gather_leaves_kernel<T><<<dim3(n_leaves), dim3(threads), 0, s>>>(full, arena, descs, bits, n_qubits, ctl);
  TN_HIP(hipGetLastError());
}

void launch_gather_leaves(const float2* full, float2* arena, const LeafDesc* descs, int n_leaves,
                          int max_out, const int8_t* bits, int n_qubits, const int64_t* ctl,
                          hipStream_t s) {
  gather_leaves(full, arena, descs, n_leaves, max_out, bits, n_qubits, ctl, s);
}

void launch_gather_leaves(const double2* full, double2* arena, const LeafDesc* descs, int n_leaves,
                          int max_out, const int8_t* bits, int n_qubits, const int64_t* ctl,
                          hipStream_t s) {
  gather_leaves(full, arena, descs, n_leaves, max_out, bits, n_qubits, ctl, s);
}

struct AccArgs {
  int nbits;
  int accumulate;
  int8_t pos[kMaxBits];
};

template <typename T>
__global__ __launch_bounds__(256) void accumulate_kernel(const T* __restrict__ R,
                                                         double2* __restrict__ out, AccArgs P,
                                                         const int64_t* __restrict__ ctl) {
  const int64_t job = ctl[0], scount = ctl[2];
  const int64_t bs = job / scount;
  const bool add = P.accumulate || (job % scount) != 0;
  const int64_t n = int64_t(1) << P.nbits;
  double2* o = out + bs * n;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    int64_t src = 0;
    for (int j = 0; j < P.nbits; ++j)
      if ((i >> j) & 1) src |= int64_t(1) << P.pos[j];
    const T v = R[src];
    double2 r = make_double2(double(v.x), double(v.y));
    if (add) {
      r.x += o[i].x;
      r.y += o[i].y;
    }
    o[i] = r;
  }
}

template <typename T>
static void accumulate(const T* R, double2* out, int nbits, const int8_t* pos_of_bit, const int64_t* ctl,
                       int accumulate, hipStream_t s) {
  AccArgs P;
  std::memset(&P, 0, sizeof(P));
  P.nbits = nbits;
  P.accumulate = accumulate;
  for (int j = 0; j < nbits; ++j) P.pos[j] = pos_of_bit[j];
  const int64_t n = int64_t(1) << nbits;
  const int64_t blocks = std::min<int64_t>(ceil_div(n, 256), grid_cap());
  accumulate_kernel<T><<<dim3(unsigned(blocks)), 256, 0, s>>>(R, out, P, ctl);
  TN_HIP(hipGetLastError());
}

void launch_accumulate(const float2* R, double2* out, int nbits, const int8_t* pos_of_bit,
                       const int64_t* ctl, int acc, hipStream_t s) {
  accumulate(R, out, nbits, pos_of_bit, ctl, acc, s);
}

void launch_accumulate(const double2* R, double2* out, int nbits, const int8_t* pos_of_bit,
                       const int64_t* ctl, int acc, hipStream_t s) {
  accumulate(R, out, nbits, pos_of_bit, ctl, acc, s);
}

__global__ void nonfinite_kernel(const double2* __restrict__ x, int64_t n, int* flag) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
    if (!isfinite(x[i].x) || !isfinite(x[i].y)) *flag = 1;
}

void launch_nonfinite(const double2* x, int64_t n, int* flag, hipStream_t s) {
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 256), 1024));
  nonfinite_kernel<<<dim3(unsigned(blocks)), 256, 0, s>>>(x, n, flag);
  TN_HIP(hipGetLastError());
}

}  // namespace tn

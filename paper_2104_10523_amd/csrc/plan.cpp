// Plan compiler: a pairwise contraction becomes one of
//   apply  - large operand read in place by bit positions, small operand
//            (<= 2^12 entries) staged in LDS;
//   gemm   - operands brought into [batch][M][K] / [batch][K][N] (or the
//            transposed forms) by bit permutations only when their layout is
//            not already grouped that way, then a complex MFMA GEMM;
//   dot    - full contraction of two operands.
// Results of the GEMM are laid out [batch][M][N], so the next step often
// finds its operand grouped already.  Workspace is carved from one arena by
// liveness (first fit).
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <tuple>

namespace tn {

// ------------------------------------------------------------------ arena

int64_t Arena::alloc(int64_t elems) {
  const int64_t len = ((std::max<int64_t>(elems, 1) + 31) / 32) * 32;
  int64_t cur = 0;
  size_t pos = 0;
  for (; pos < used_.size(); ++pos) {
    if (used_[pos].first - cur >= len) break;
    cur = used_[pos].first + used_[pos].second;
  }
  used_.insert(used_.begin() + pos, {cur, len});
  high_ = std::max(high_, cur + len);
  return cur;
}

void Arena::release(int64_t off) {
  for (size_t i = 0; i < used_.size(); ++i)
    if (used_[i].first == off) {
      used_.erase(used_.begin() + i);
      return;
    }
  throw Error(TN_ERR_ARG, "internal: arena release of unknown block");
}

// ------------------------------------------------------------ pair compile

namespace {

// complex128 plans (TN_PREC_FP64): tensors take two float2 slots per entry
thread_local int g_esz = 1;

int pos_of(const std::vector<int>& layout, int label) {
  const auto it = std::find(layout.begin(), layout.end(), label);
  if (it == layout.end()) return -1;
  return int(layout.size()) - 1 - int(it - layout.begin());
}

std::vector<int> filter(const std::vector<int>& v, const std::set<int>& s, bool in) {
  std::vector<int> r;
  for (int l : v)
    if ((s.count(l) > 0) == in) r.push_back(l);
  return r;
}

std::vector<int> cat(std::initializer_list<std::vector<int>> parts) {
  std::vector<int> r;
  for (const auto& p : parts) r.insert(r.end(), p.begin(), p.end());
  return r;
}

// relative order of `sub` labels as they appear in `layout`
std::vector<int> order_in(const std::vector<int>& layout, const std::set<int>& sub) {
  std::vector<int> r;
  for (int l : layout)
    if (sub.count(l)) r.push_back(l);
  return r;
}

double p2(size_t bits) { return std::ldexp(1.0, int(bits)); }

// np > 0: the output is np planes of packed bfloat16 parts (for the split
// GEMMs) instead of complex64.
TRef emit_permute(const TRef& in, const std::vector<int>& target, Arena& arena,
                  std::vector<PlanOp>& ops, std::vector<int64_t>* scratch, int out_buf = -1,
                  int64_t out_off = 0, int np = 0, bool f16 = false) {
  PlanOp op;
  op.kind = OP_PERMUTE;
  op.pm.nb = int(target.size());
  op.pm.nb_in = int(in.labels.size());
  op.pm.np = np;
  op.pm.f16 = f16 ? 1 : 0;
  TN_REQUIRE(op.pm.nb <= kMaxBits && op.pm.nb_in <= kMaxBits, TN_ERR_UNSUPPORTED, "rank > 64");
  for (int j = 0; j < op.pm.nb; ++j)
    op.pm.src[j] = int8_t(pos_of(in.labels, target[op.pm.nb - 1 - j]));
  TRef out;
  out.labels = target;
  if (out_buf >= 0) {
    out.buf = out_buf;
    out.off = out_off;
  } else {
    out.buf = BUF_WORK;
    const int64_t elems = int64_t(1) << op.pm.nb;
    out.off = arena.alloc(np ? (elems * np + 1) / 2 : elems * g_esz);
    scratch->push_back(out.off);
  }
  if (f16 && in.cslot >= 0 && in.producer >= 0 && in.producer < int(ops.size()) &&
      (ops[in.producer].kind == OP_GEMM || ops[in.producer].kind == OP_APPLY) &&
      ops[in.producer].c_buf == in.buf && ops[in.producer].c_off == in.off) {
    // the GEMM or apply that produced the input reports its largest |re|,
    // |im| into the slot reserved with its result
    ops[in.producer].cmax = in.cslot;
    op.smax = in.cslot;
    out.smax = op.smax;
  } else if (f16) {
    op.smax = arena.alloc(1);
    scratch->push_back(op.smax);
    out.smax = op.smax;
    // the operand's largest |re|, |im| first (its own pass over the input)
    PlanOp pre = op;
    pre.pm.maxabs = 1;
    pre.a_buf = in.buf;
    pre.a_off = in.off;
    pre.c_buf = out.buf;
    pre.c_off = out.off;
    pre.bytes = 8.0 * p2(op.pm.nb_in);
    ops.push_back(pre);
  }
  op.a_buf = in.buf;
  op.a_off = in.off;
  op.c_buf = out.buf;
  op.c_off = out.off;
  op.bytes = 8.0 * p2(op.pm.nb_in) + (np ? 4.0 * np : 8.0) * p2(op.pm.nb);
  ops.push_back(op);
  return out;
}

// Sum out `dang` labels of X (apply against the constant 1).
TRef emit_sum_out(const TRef& X, const std::vector<int>& dang, Arena& arena,
                  std::vector<PlanOp>& ops, std::vector<int64_t>* scratch) {
  TN_REQUIRE(dang.size() <= 6, TN_ERR_UNSUPPORTED, "too many summed-out labels");
  PlanOp op;
  op.kind = OP_APPLY;
  std::memset(&op.ap, 0, sizeof(op.ap));
  std::memset(op.ap.b_extra, -1, sizeof(op.ap.b_extra));
  op.ap.variant = -1;
  op.ap.a_bits = int(X.labels.size());
  std::vector<int> kp;
  for (int l : dang) kp.push_back(pos_of(X.labels, l));
  std::sort(kp.begin(), kp.end());
  op.ap.nk = int(kp.size());
  for (int i = 0; i < 8; ++i) {
    op.ap.kpos[i] = i < op.ap.nk ? int8_t(kp[i]) : 0;
    op.ap.bk[i] = -1;
    op.ap.bn[i] = 0;
  }
  op.ap.nn = 0;
  op.ap.nb_b = 0;
  TRef out;
  out.labels = filter(X.labels, std::set<int>(dang.begin(), dang.end()), false);
  out.buf = BUF_WORK;
  out.off = arena.alloc((int64_t(1) << out.labels.size()) * g_esz);
  scratch->push_back(out.off);
  op.a_buf = X.buf;
  op.a_off = X.off;
  op.b_buf = BUF_ONE;
  op.b_off = 0;
  op.c_buf = out.buf;
  op.c_off = out.off;
  op.flops = 8.0 * p2(X.labels.size());
  op.bytes = 8.0 * (p2(X.labels.size()) + p2(out.labels.size()));
  ops.push_back(op);
  return out;
}

// AUTO: among the precisions whose a-priori error for this GEMM stays
// within kAutoErr (u sqrt(1 + log2 K): scaled split-FP16x3 and FP32 always,
// split-BF16x3 never), the one of least modelled time: max(flops / F,
// GEMM bytes / B) plus the operand passes it needs -- for FP32 a permute
// (16 bytes per entry) of an operand whose labels are not grouped for the
// GEMM, for the split form the max-abs pass and the packing permute of both
// operands (8 + 16 bytes per entry).  F and B as in the time ranking of
// paths (350e12 split, 120e12 FP32, 4.0e12 B/s).
constexpr double kAutoErr = 2e-6;
int auto_precision(int64_t Bn, int64_t M, int64_t N, int64_t K, bool permA, bool permB, bool packable) {
  constexpr double kSplit = 350e12, kFp32 = 120e12, kHbm = 4.0e12;
  const double b = double(Bn), fl = 8.0 * b * M * N * K;
  const double ab = b * M * K, bb = b * K * N, cb = b * M * N;
  const double gemm_bytes = 8.0 * (ab + bb + cb);
  const double t32 = std::max(fl / kFp32, gemm_bytes / kHbm) + 16.0 * ((permA ? ab : 0) + (permB ? bb : 0)) / kHbm;
  if (!packable) return TN_PREC_FP32;
  const double e16 = std::ldexp(1.0, -21) * std::sqrt(1.0 + std::log2(double(K)));
  if (e16 > kAutoErr) return TN_PREC_FP32;
  const double t16 = std::max(fl / kSplit, gemm_bytes / kHbm) + 24.0 * (ab + bb) / kHbm;
  return t16 < t32 ? TN_PREC_F16X3 : TN_PREC_FP32;
}

}  // namespace

namespace {
TRef compile_pair_impl(const TRef& X0, const TRef& Y0, const std::vector<int>& keep_v,
                       const std::vector<int>* want, int want_buf, int64_t want_off, Arena& arena,
                       int precision, std::vector<PlanOp>& ops, std::vector<int64_t>* scratch) {
  const std::set<int> keep(keep_v.begin(), keep_v.end());
  TRef X = X0, Y = Y0;
  {
    std::set<int> sx(X.labels.begin(), X.labels.end()), sy(Y.labels.begin(), Y.labels.end());
    for (int l : keep) TN_REQUIRE(sx.count(l) || sy.count(l), TN_ERR_MODES, "result label not in an operand");
  }
  auto dangling = [&](const TRef& T, const TRef& O) {
    std::set<int> so(O.labels.begin(), O.labels.end());
    std::vector<int> d;
    for (int l : T.labels)
      if (!so.count(l) && !keep.count(l)) d.push_back(l);
    return d;
  };
  const auto dx = dangling(X, Y), dy = dangling(Y, X);
  const bool x_big = X.labels.size() >= Y.labels.size();
  TRef& big = x_big ? X : Y;
  TRef& small = x_big ? Y : X;
  const std::set<int> sbig(big.labels.begin(), big.labels.end()), ssmall(small.labels.begin(), small.labels.end());
  std::vector<int> K, batch, Nsm;
  for (int l : big.labels)
    if (ssmall.count(l)) (keep.count(l) ? batch : K).push_back(l);
  for (int l : small.labels)
    if (!sbig.count(l) && keep.count(l)) Nsm.push_back(l);
  const auto& dbig = x_big ? dx : dy;
  const auto& dsmall = x_big ? dy : dx;

  // ------------------------------------------------------------ apply path
  // up to 16 outputs per row on every kernel; 32 or 64 (5 or 6 N bits) on
  // the matrix-core apply, which reads the large operand in place where a
  // GEMM would first regroup it, at complex64 precisions and >= 64 rows
  const size_t n_max =
      precision != TN_PREC_FP64 && big.labels.size() >= K.size() + dbig.size() + 6 ? 6 : 4;
  if (batch.empty() && small.labels.size() <= 12 && K.size() + dbig.size() <= 6 && Nsm.size() <= n_max &&
      dsmall.size() <= 12) {
    const std::set<int> kset(K.begin(), K.end()), dbset(dbig.begin(), dbig.end());
    std::vector<int> Mbig;
    for (int l : big.labels)
      if (!kset.count(l) && !dbset.count(l)) Mbig.push_back(l);
    std::vector<int> Norder = Nsm;
    bool direct = false;
    if (want) {
      if (want->size() == Mbig.size() + Nsm.size() &&
          std::equal(Mbig.begin(), Mbig.end(), want->begin())) {
        std::vector<int> wn(want->begin() + Mbig.size(), want->end());
        std::vector<int> a = wn, b = Nsm;
        std::sort(a.begin(), a.end());
        std::sort(b.begin(), b.end());
        if (a == b) {
          Norder = wn;
          direct = true;
        }
      }
    }
    PlanOp op;
    op.kind = OP_APPLY;
    std::memset(&op.ap, 0, sizeof(op.ap));
    std::memset(op.ap.b_extra, -1, sizeof(op.ap.b_extra));
    op.ap.a_bits = int(big.labels.size());
    std::vector<std::pair<int, int>> kp;  // (pos in big, label or -1)
    for (int l : K) kp.push_back({pos_of(big.labels, l), l});
    for (int l : dbig) kp.push_back({pos_of(big.labels, l), -1});
    std::sort(kp.begin(), kp.end());
    op.ap.nk = int(kp.size());
    for (int i = 0; i < op.ap.nk; ++i) {
      op.ap.kpos[i] = int8_t(kp[i].first);
      op.ap.bk[i] = kp[i].second < 0 ? int8_t(-1) : int8_t(pos_of(small.labels, kp[i].second));
    }
    op.ap.nn = int(Norder.size());
    for (int i = 0; i < op.ap.nn; ++i) op.ap.bn[i] = int8_t(pos_of(small.labels, Norder[op.ap.nn - 1 - i]));
    op.ap.n_b_extra = int(dsmall.size());
    for (size_t i = 0; i < dsmall.size(); ++i) op.ap.b_extra[i] = int8_t(pos_of(small.labels, dsmall[i]));
    op.ap.nb_b = int(small.labels.size());
    op.ap.variant = tuned_apply(op.ap);
    TRef out;
    out.labels = cat({Mbig, Norder});
    if (want && direct) {
      out.buf = want_buf;
      out.off = want_off;
    } else {
      out.buf = BUF_WORK;
      out.off = arena.alloc((int64_t(1) << out.labels.size()) * g_esz);
      if (want) scratch->push_back(out.off);
    }
    op.a_buf = big.buf;
    op.a_off = big.off;
    op.b_buf = small.buf;
    op.b_off = small.off;
    op.c_buf = out.buf;
    op.c_off = out.off;
    const double rows = p2(big.labels.size() - kp.size());
    op.flops = 8.0 * rows * p2(kp.size()) * p2(Norder.size());
    op.bytes = 8.0 * (p2(big.labels.size()) + rows * p2(Norder.size()) + p2(small.labels.size()));
    ops.push_back(op);
    if (want && !direct) return emit_permute(out, *want, arena, ops, scratch, want_buf, want_off);
    if (g_esz == 1 && out.buf == BUF_WORK) {
      out.cslot = arena.alloc(1);
      out.producer = int(ops.size()) - 1;
    }
    return out;
  }

  // ------------------------------------------------------------ gemm path
  if (!dx.empty()) X = emit_sum_out(X, dx, arena, ops, scratch);
  if (!dy.empty()) Y = emit_sum_out(Y, dy, arena, ops, scratch);
  const std::set<int> sx(X.labels.begin(), X.labels.end()), sy(Y.labels.begin(), Y.labels.end());
  std::set<int> bset, kset;
  for (int l : X.labels)
    if (sy.count(l)) (keep.count(l) ? bset : kset).insert(l);
  std::set<int> mx, ny;
  for (int l : X.labels)
    if (!sy.count(l)) mx.insert(l);
  for (int l : Y.labels)
    if (!sx.count(l)) ny.insert(l);

  // roles: A carries M, B carries N.  Try to match a requested layout.
  bool a_is_x = mx.size() >= ny.size();
  std::vector<int> b_o, m_o, n_o;
  bool direct = false;
  auto try_role = [&](bool ax) {
    const std::set<int>& ms = ax ? mx : ny;
    const std::set<int>& ns = ax ? ny : mx;
    const size_t nb = bset.size(), nm = ms.size(), nn = ns.size();
    if (want->size() != nb + nm + nn) return false;
    for (size_t i = 0; i < nb; ++i)
      if (!bset.count((*want)[i])) return false;
    for (size_t i = nb; i < nb + nm; ++i)
      if (!ms.count((*want)[i])) return false;
    for (size_t i = nb + nm; i < want->size(); ++i)
      if (!ns.count((*want)[i])) return false;
    a_is_x = ax;
    b_o.assign(want->begin(), want->begin() + nb);
    m_o.assign(want->begin() + nb, want->begin() + nb + nm);
    n_o.assign(want->begin() + nb + nm, want->end());
    return true;
  };
  if (want) direct = try_role(a_is_x) || try_role(!a_is_x);
  TRef& A = a_is_x ? X : Y;
  TRef& B = a_is_x ? Y : X;
  const bool a_larger = A.labels.size() >= B.labels.size();
  if (!direct) {
    b_o = order_in(a_larger ? A.labels : B.labels, bset);
    m_o = order_in(A.labels, a_is_x ? mx : ny);
    n_o = order_in(B.labels, a_is_x ? ny : mx);
  }
  const std::vector<int> k_o = order_in(a_larger ? A.labels : B.labels, kset);
  const int64_t Mn = int64_t(1) << m_o.size(), Nn = int64_t(1) << n_o.size(),
                Kn = int64_t(1) << k_o.size(), Bn = int64_t(1) << b_o.size();

  auto lowest = [](const TRef& T) { return T.labels.empty() ? -1 : T.labels.back(); };
  int transA = 0, transB = 0;
  TRef Ap = A, Bp = B;
  // packed planes are addressed with 32-bit panel offsets: a 256-row panel
  // of one plane (4 bytes per entry) must stay below 2 GiB, so K <= 2^20;
  // longer contractions run on the FP32 kernel at every precision
  const bool long_k = Kn > (int64_t(1) << 20);
  // a few outputs over a long contraction: one FP64-accumulated dot product
  // per (m, n) pair of k-contiguous rows (an MFMA tile would mostly idle)
  // batch 1: the skinny kernel reads A and B once for all (m, n)
  const bool skinny = Bn == 1 && Kn >= (int64_t(1) << 16) && skinny_supported(Mn, Nn);
  const bool dot_mn = skinny || (!(Mn == 1 && Nn == 1) && Mn * Nn <= 16 && Kn >= (int64_t(1) << 16) &&
                                 Bn * Mn * Nn <= 4096);
  const bool packable = Kn % 4 == 0 && !long_k && !dot_mn && !(Mn == 1 && Nn == 1);
  int prec = precision;
  if (prec == TN_PREC_AUTO) {
    // would the FP32 GEMM have to permute an operand first?
    const auto ga0 = cat({b_o, m_o, k_o}), ga1 = cat({b_o, k_o, m_o});
    const auto gb0 = cat({b_o, k_o, n_o}), gb1 = cat({b_o, n_o, k_o});
    const bool permA = !(A.labels == ga0 || A.labels == ga1), permB = !(B.labels == gb0 || B.labels == gb1);
    prec = auto_precision(Bn, Mn, Nn, Kn, permA, permB, packable);
  }
  if (long_k && prec != TN_PREC_FP64) prec = TN_PREC_FP32;
  // split-FP16 exists only on packed planes; elsewhere such GEMMs run FP32
  if (prec == TN_PREC_F16X3 && !packable) prec = TN_PREC_FP32;
  const bool packed = (prec == TN_PREC_BF16X3 || prec == TN_PREC_BF16X6 || prec == TN_PREC_F16X3) && packable;
  const int np = prec == TN_PREC_BF16X6 ? 3 : 2;
  const bool f16 = prec == TN_PREC_F16X3;
  if (packed) {
    Ap = emit_permute(A, cat({b_o, m_o, k_o}), arena, ops, scratch, -1, 0, np, f16);
    Bp = emit_permute(B, cat({b_o, n_o, k_o}), arena, ops, scratch, -1, 0, np, f16);
    transA = 0;
    transB = 1;
  } else if (Mn == 1 && Nn == 1) {
    const auto fa = cat({b_o, k_o});
    if (A.labels != fa) Ap = emit_permute(A, fa, arena, ops, scratch);
    if (B.labels != fa) Bp = emit_permute(B, fa, arena, ops, scratch);
  } else if (skinny) {
    // either layout of each operand, as found (no permute when it already is one)
    const auto fa0 = cat({m_o, k_o}), fa1 = cat({k_o, m_o});
    if (A.labels == fa0) transA = 0;
    else if (A.labels == fa1) transA = 1;
    else {
      transA = kset.count(lowest(A)) ? 0 : 1;
      Ap = emit_permute(A, transA ? fa1 : fa0, arena, ops, scratch);
    }
    const auto fb0 = cat({k_o, n_o}), fb1 = cat({n_o, k_o});
    if (B.labels == fb0) transB = 0;
    else if (B.labels == fb1) transB = 1;
    else {
      transB = kset.count(lowest(B)) ? 1 : 0;
      Bp = emit_permute(B, transB ? fb1 : fb0, arena, ops, scratch);
    }
  } else if (dot_mn) {
    const auto fa = cat({b_o, m_o, k_o}), fb = cat({b_o, n_o, k_o});
    if (A.labels != fa) Ap = emit_permute(A, fa, arena, ops, scratch);
    if (B.labels != fb) Bp = emit_permute(B, fb, arena, ops, scratch);
  } else {
    const auto fa0 = cat({b_o, m_o, k_o}), fa1 = cat({b_o, k_o, m_o});
    if (A.labels == fa0) transA = 0;
    else if (A.labels == fa1) transA = 1;
    else {
      transA = kset.count(lowest(A)) ? 0 : 1;
      Ap = emit_permute(A, transA ? fa1 : fa0, arena, ops, scratch);
    }
    const auto fb0 = cat({b_o, k_o, n_o}), fb1 = cat({b_o, n_o, k_o});
    if (B.labels == fb0) transB = 0;
    else if (B.labels == fb1) transB = 1;
    else {
      transB = kset.count(lowest(B)) ? 1 : 0;
      Bp = emit_permute(B, transB ? fb1 : fb0, arena, ops, scratch);
    }
  }
  TRef out;
  out.labels = cat({b_o, m_o, n_o});
  if (want && direct) {
    out.buf = want_buf;
    out.off = want_off;
  } else {
    out.buf = BUF_WORK;
    out.off = arena.alloc(Bn * Mn * Nn * g_esz);
    if (want) scratch->push_back(out.off);
  }
  PlanOp op;
  op.a_buf = Ap.buf;
  op.a_off = Ap.off;
  op.b_buf = Bp.buf;
  op.b_off = Bp.off;
  op.c_buf = out.buf;
  op.c_off = out.off;
  if ((Mn == 1 && Nn == 1) || dot_mn) {
    op.kind = OP_DOT;
    op.dot_k = Kn;
    op.dot_batch = Bn;
    op.dot_m = Mn;
    op.dot_n = Nn;
    op.skinny = skinny ? 1 : 0;
    // operand layouts: chosen freely on the skinny branch, else [b][m][k] x [b][n][k]
    op.dot_ta = skinny ? transA : 0;
    op.dot_tb = skinny ? transB : 1;
    const size_t wbytes = prec == TN_PREC_FP64 ? dot64_workspace_bytes(Kn, Bn * Mn * Nn)
                          : skinny             ? skinny_workspace_bytes(Kn, Mn, Nn)
                                               : dot_workspace_bytes(Kn, Bn * Mn * Nn);
    op.work_elems = int64_t((wbytes + 7) / 8);
    op.work_off = arena.alloc(op.work_elems);
    scratch->push_back(op.work_off);
  } else {
    op.kind = OP_GEMM;
    op.gm.M = Mn;
    op.gm.N = Nn;
    op.gm.K = Kn;
    op.gm.batch = Bn;
    op.gm.transA = transA;
    op.gm.transB = transB;
    op.gm.precision = prec;
    op.gm.packed = packed ? 1 : 0;
    op.gm.plane_a = Bn * Mn * Kn;
    op.gm.plane_b = Bn * Nn * Kn;
    op.smax_a = Ap.smax;
    op.smax_b = Bp.smax;
    op.gm.tile = tuned_tile(op.gm);
    // room for the split-K partials of any candidate tile, so the
    // autotuner may pick any of them later
    size_t wb = 0;
    if (prec == TN_PREC_FP64) {
      wb = gemm64_workspace_bytes(op.gm);
    } else {
      for (int c : gemm_tile_candidates(op.gm)) {
        GemmDesc gc = op.gm;
        gc.tile = c;
        wb = std::max(wb, gemm_workspace_bytes(gc));
      }
    }
    if (wb > 0) {
      op.work_elems = int64_t((wb + 7) / 8);
      op.work_off = arena.alloc(op.work_elems);
      scratch->push_back(op.work_off);
    }
  }
  op.flops = 8.0 * double(Bn) * double(Mn) * double(Nn) * double(Kn);
  op.bytes = 8.0 * double(Bn) * (double(Mn) * Kn + double(Kn) * Nn + double(Mn) * Nn);
  ops.push_back(op);
  if (want && !direct) return emit_permute(out, *want, arena, ops, scratch, want_buf, want_off);
  if (op.kind == OP_GEMM && packed && out.buf == BUF_WORK) {
    out.cslot = arena.alloc(1);
    out.producer = int(ops.size()) - 1;
  }
  return out;
}

}  // namespace

TRef compile_pair(const TRef& X0, const TRef& Y0, const std::vector<int>& keep_v,
                  const std::vector<int>* want, int want_buf, int64_t want_off, Arena& arena,
                  int precision, std::vector<PlanOp>& ops, std::vector<int64_t>* scratch) {
  const bool f64 = precision == TN_PREC_FP64;
  const size_t first = ops.size();
  const int saved = g_esz;
  g_esz = f64 ? 2 : 1;
  TRef r;
  try {
    r = compile_pair_impl(X0, Y0, keep_v, want, want_buf, want_off, arena, precision, ops, scratch);
  } catch (...) {
    g_esz = saved;
    throw;
  }
  g_esz = saved;
  if (f64)
    for (size_t k = first; k < ops.size(); ++k) {
      ops[k].f64 = 1;
      ops[k].bytes *= 2.0;      // 16-byte entries
    }
  return r;
}

namespace {
uint32_t* slot(float2* const bufs[6], int64_t off) {
  return off >= 0 ? reinterpret_cast<uint32_t*>(bufs[BUF_WORK] + off) : nullptr;
}
}  // namespace

namespace {
void run_op64(const PlanOp& op, float2* const bufs[6], hipStream_t s) {
  auto d2 = [&](int buf, int64_t off) {
    // the constant one buffer holds 1+0i as complex64 at byte 0 and as
    // complex128 at byte 16
    if (buf == BUF_ONE) return reinterpret_cast<double2*>(reinterpret_cast<char*>(bufs[BUF_ONE]) + 16);
    return reinterpret_cast<double2*>(bufs[buf] + off);
  };
  const double2* a = d2(op.a_buf, op.a_off);
  const double2* b = d2(op.b_buf, op.b_off);
  double2* c = d2(op.c_buf, op.c_off);
  void* w = op.work_off >= 0 ? static_cast<void*>(bufs[BUF_WORK] + op.work_off) : nullptr;
  switch (op.kind) {
    case OP_APPLY: launch_apply64(a, b, c, op.ap, s); break;
    case OP_PERMUTE: launch_permute64(a, c, op.pm, s); break;
    case OP_GEMM: launch_gemm64(a, b, c, op.gm, w, s); break;
    case OP_DOT:
      launch_dot64(a, b, c, op.dot_k, op.dot_batch, op.dot_m, op.dot_n, op.dot_ta, op.dot_tb, w, s);
      break;
  }
}
}  // namespace

void run_ops(const std::vector<PlanOp>& ops, float2* const bufs[6], hipStream_t s) {
  for (const PlanOp& op : ops) {
    if (op.f64) {
      run_op64(op, bufs, s);
      continue;
    }
    const float2* a = bufs[op.a_buf] + op.a_off;
    const float2* b = bufs[op.b_buf] + op.b_off;
    float2* c = bufs[op.c_buf] + op.c_off;
    void* w = op.work_off >= 0 ? static_cast<void*>(bufs[BUF_WORK] + op.work_off) : nullptr;
    switch (op.kind) {
      case OP_APPLY: launch_apply_small(a, b, c, op.ap, s, slot(bufs, op.cmax)); break;
      case OP_PERMUTE: launch_permute(a, c, op.pm, slot(bufs, op.smax), s); break;
      case OP_GEMM:
        launch_gemm(a, b, c, op.gm, w, slot(bufs, op.smax_a), slot(bufs, op.smax_b), s, slot(bufs, op.cmax));
        break;
      case OP_DOT:
        if (op.skinny) launch_skinny(a, b, c, op.dot_k, op.dot_m, op.dot_n, op.dot_ta, op.dot_tb, w, s);
        else launch_dot(a, b, c, op.dot_k, op.dot_batch, op.dot_m, op.dot_n, w, s);
        break;
    }
  }
}

// ------------------------------------------------------------- autotune

namespace {
using TileKey = std::tuple<int64_t, int64_t, int64_t, int64_t, int, int, int, int>;
std::mutex g_tile_mu;
std::map<TileKey, int> g_tiles;
TileKey key_of(const GemmDesc& g) {
  return TileKey{g.M, g.N, g.K, g.batch, g.precision, g.packed, g.transA, g.transB};
}
}  // namespace

int tuned_tile(const GemmDesc& g) {
  std::lock_guard<std::mutex> lk(g_tile_mu);
  auto it = g_tiles.find(key_of(g));
  return it == g_tiles.end() ? -1 : it->second;
}

void remember_tile(const GemmDesc& g, int tile) {
  std::lock_guard<std::mutex> lk(g_tile_mu);
  g_tiles[key_of(g)] = tile;
}

namespace {
// an apply's identity for the cache: its descriptor without the variant
std::vector<int> apply_key(const ApplySmallDesc& d) {
  std::vector<int> k{d.a_bits, d.nk, d.nn, d.nb_b, d.n_b_extra};
  for (int i = 0; i < 8; ++i) k.insert(k.end(), {d.kpos[i], d.bk[i], d.bn[i]});
  for (int i = 0; i < 12; ++i) k.push_back(d.b_extra[i]);
  return k;
}
std::map<std::vector<int>, int> g_applies;
}  // namespace

int tuned_apply(const ApplySmallDesc& d) {
  std::lock_guard<std::mutex> lk(g_tile_mu);
  auto it = g_applies.find(apply_key(d));
  return it == g_applies.end() ? -1 : it->second;
}

// Times the apply kernels that fit op (on its first 2^24 or so rows: every
// address stays inside the real operands) and keeps the fastest.
void autotune_apply(PlanOp& op, float2* const bufs[6], int reps, hipEvent_t e0, hipEvent_t e1, hipStream_t s) {
  const std::vector<int> cands = apply_variant_candidates(op.ap);
  if (cands.size() < 2) return;
  const float2* a = bufs[op.a_buf] + op.a_off;
  const float2* b = bufs[op.b_buf] + op.b_off;
  float2* c = bufs[op.c_buf] + op.c_off;
  ApplySmallDesc d = op.ap;
  const int kmax = d.nk > 0 ? d.kpos[d.nk - 1] + 1 : 0;
  d.a_bits = std::max({kmax, d.nk + 6, std::min(d.a_bits, d.nk + 24)});
  float best_ms = 0;
  int best = -1;
  for (int v : cands) {
    d.variant = v;
    launch_apply_small(a, b, c, d, s);  // warm
    TN_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) launch_apply_small(a, b, c, d, s);
    TN_HIP(hipEventRecord(e1, s));
    TN_HIP(hipEventSynchronize(e1));
    float ms = 0;
    TN_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (best < 0 || ms < best_ms) {
      best = v;
      best_ms = ms;
    }
  }
  op.ap.variant = best;
  std::lock_guard<std::mutex> lk(g_tile_mu);
  g_applies[apply_key(op.ap)] = best;
}

void autotune_ops(std::vector<PlanOp>& ops, float2* const bufs[6], int reps, hipStream_t s) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  TN_HIP(hipEventCreate(&e0));
  TN_HIP(hipEventCreate(&e1));
  std::map<TileKey, int> done;
  std::map<std::vector<int>, int> done_apply;
  try {
    for (PlanOp& op : ops) {
      if (op.kind == OP_APPLY && !op.f64) {
        const auto key = apply_key(op.ap);
        auto it = done_apply.find(key);
        if (it != done_apply.end()) {
          op.ap.variant = it->second;
        } else {
          autotune_apply(op, bufs, reps, e0, e1, s);
          done_apply[key] = op.ap.variant;
        }
        continue;
      }
      if (op.kind != OP_GEMM || op.f64) continue;
      auto it = done.find(key_of(op.gm));
      if (it != done.end()) {
        op.gm.tile = it->second;
        continue;
      }
      const float2* a = bufs[op.a_buf] + op.a_off;
      const float2* b = bufs[op.b_buf] + op.b_off;
      float2* c = bufs[op.c_buf] + op.c_off;
      void* w = op.work_off >= 0 ? static_cast<void*>(bufs[BUF_WORK] + op.work_off) : nullptr;
      float best_ms = 0, def_ms = 0;
      int best = -1;
      GemmDesc gdef = op.gm;
      gdef.tile = -1;
      const int def_tile = gemm_tile_of(gdef);
      for (int cand : gemm_tile_candidates(op.gm)) {
        GemmDesc g = op.gm;
        g.tile = cand;
        // time a K-truncated proxy: the tile ranking hardly depends on K once
        // the launch fills the chip, and every address of the proxy stays
        // inside the op's real operands.  GEMMs of few output tiles split a
        // long K over blocks; their proxy keeps a sixteenth of K (at least
        // 512, a multiple of 64) so that it splits, and fills the chip, alike.
        const int64_t out_tiles = ((g.M + 63) / 64) * ((g.N + 63) / 64) * g.batch;
        g.K = std::min<int64_t>(g.K, out_tiles < 256 ? std::max<int64_t>(512, (g.K / 16) & ~int64_t(63)) : 512);
        if (gemm_workspace_bytes(g) > size_t(op.work_elems) * sizeof(float2)) continue;
        const uint32_t* sa = slot(bufs, op.smax_a);
        const uint32_t* sb = slot(bufs, op.smax_b);
        launch_gemm(a, b, c, g, w, sa, sb, s);  // warm
        TN_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < reps; ++r) launch_gemm(a, b, c, g, w, sa, sb, s);
        TN_HIP(hipEventRecord(e1, s));
        TN_HIP(hipEventSynchronize(e1));
        float ms = 0;
        TN_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (cand == def_tile) def_ms = ms;
        if (best < 0 || ms < best_ms) {
          best = cand;
          best_ms = ms;
        }
      }
      // two timed launches are noisy: the shape heuristic's tile stays
      // unless another is at least 5% faster
      if (best >= 0 && def_ms > 0 && best_ms > 0.95f * def_ms) best = def_tile;
      if (best >= 0) {
        op.gm.tile = best;
        done[key_of(op.gm)] = best;
        remember_tile(op.gm, best);
      }
    }
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

// ------------------------------------------------------ amplitude planning

AmpPlan compile_amplitudes(const Network& net, const std::vector<std::pair<int, int>>& path,
                           const std::vector<int>& sliced, const std::vector<char>& open_q,
                           int precision) {
  AmpPlan P;
  P.n_qubits = net.n_qubits;
  P.precision = precision;
  P.sliced = sliced;
  const int n_sl = int(sliced.size());
  TN_REQUIRE(n_sl <= 62, TN_ERR_UNSUPPORTED, "too many sliced labels");
  P.n_slices = std::ldexp(1.0, n_sl);
  // fixed labels: projected outputs and sliced labels
  std::vector<int> fixed_kind(net.n_labels, -1), fixed_which(net.n_labels, 0);
  std::vector<char> open_label(net.n_labels, 0);
  for (int q = 0; q < net.n_qubits; ++q) {
    const int l = net.out_label[q];
    if (open_q[q]) {
      open_label[l] = 1;
      P.open_qubits.push_back(q);
    } else {
      fixed_kind[l] = 0;
      fixed_which[l] = q;
    }
  }
  for (int s = 0; s < n_sl; ++s) {
    TN_REQUIRE(!open_label[sliced[s]], TN_ERR_ARG, "an open label cannot be sliced");
    fixed_kind[sliced[s]] = 1;
    fixed_which[sliced[s]] = n_sl - 1 - s;
  }
  P.n_open = int(P.open_qubits.size());
  TN_REQUIRE(P.n_open <= 40, TN_ERR_UNSUPPORTED, "more than 40 open qubits");

  const int nt = int(net.tensors.size());
  std::vector<TRef> refs(nt);
  int64_t src_off = 0;
  for (int i = 0; i < nt; ++i) {
    const auto& L = net.tensors[i].labels;
    const int r = int(L.size());
    LeafDesc d;
    std::memset(&d, 0, sizeof(d));
    d.src_off = src_off;
    src_off += int64_t(1) << r;
    std::vector<int> red;
    for (int l : L)
      if (fixed_kind[l] < 0) red.push_back(l);
    d.out_bits = int(red.size());
    TN_REQUIRE(r <= 8, TN_ERR_UNSUPPORTED, "leaf rank > 8");
    for (int j = 0; j < d.out_bits; ++j) {
      const int lab = red[d.out_bits - 1 - j];
      d.in_pos[j] = int8_t(r - 1 - int(std::find(L.begin(), L.end(), lab) - L.begin()));
    }
    for (int a = 0; a < r; ++a) {
      const int l = L[a];
      if (fixed_kind[l] < 0) continue;
      LeafFixed& f = d.fixed[d.n_fixed++];
      f.pos = int8_t(r - 1 - a);
      f.kind = int8_t(fixed_kind[l]);
      f.which = int16_t(fixed_which[l]);
    }
    d.dst_off = P.leaf_elems;
    P.leaf_elems += ((int64_t(1) << d.out_bits) + 7) / 8 * 8;
    P.max_leaf_bits = std::max(P.max_leaf_bits, d.out_bits);
    P.leaves.push_back(d);
    refs[i].buf = BUF_LEAF;
    refs[i].off = d.dst_off * (precision == TN_PREC_FP64 ? 2 : 1);   // float2 slots
    refs[i].labels = red;
  }

  // per-step result label sets from the cost model (same reading as the path)
  PathProblem pr;
  pr.ext.assign(net.n_labels, 2.0);
  pr.open.assign(net.n_labels, 0);
  for (int l = 0; l < net.n_labels; ++l) pr.open[l] = open_label[l];
  for (int i = 0; i < nt; ++i) {
    std::vector<int> s;
    for (int l : net.tensors[i].labels)
      if (fixed_kind[l] != 0) s.push_back(l);
    std::sort(s.begin(), s.end());
    pr.leaves.push_back(s);
  }
  const PathStats ps = path_stats(pr, path, sliced);

  Arena arena;
  double err2 = 0;
  for (size_t t = 0; t < path.size(); ++t) {
    const auto [i, j] = path[t];
    std::vector<int64_t> scratch;
    const size_t first = P.ops.size();
    TRef r = compile_pair(refs[i], refs[j], ps.steps[t].c, nullptr, 0, 0, arena, precision, P.ops,
                          &scratch);
    for (size_t k = first; k < P.ops.size(); ++k) {
      const PlanOp& op = P.ops[k];
      P.flops_per_job += op.flops;
      P.bytes_per_job += op.bytes;
      if (op.f64) {
        // complex128 throughout: unit roundoff 2^-53 per operation chain
        if (op.kind == OP_GEMM) P.gemm_ops++;
        const double K = op.kind == OP_GEMM ? double(op.gm.K) : 1.0;
        err2 += std::ldexp(1.0, -106) * (1.0 + K);
      } else if (op.kind == OP_GEMM) {
        P.gemm_ops++;
        const double u = op.gm.precision == TN_PREC_BF16X3   ? std::ldexp(1.0, -17)
                         : op.gm.precision == TN_PREC_F16X3 ? std::ldexp(1.0, -21)
                                                            : std::ldexp(1.0, -24);
        // FP32 roundings along one accumulator chain, cut every 4096
        // complex k (then one add per chunk): split kernels round once per
        // product per 8 complex k, the FP32 MFMA once per complex k
        const double K = double(op.gm.K);
        const double nprod = op.gm.precision == TN_PREC_BF16X6 ? 6.0 : 3.0;
        const double per_chunk = op.gm.packed ? std::min(K, 4096.0) / 8.0 * nprod : std::min(K, 4096.0);
        const double chain = per_chunk + std::ceil(K / 4096.0);
        err2 += u * u * (1.0 + std::log2(K)) + std::ldexp(1.0, -48) * chain;
      } else if (op.kind != OP_PERMUTE) {
        err2 += std::ldexp(1.0, -48);
      }
    }
    for (int64_t off : scratch) arena.release(off);
    for (const TRef* t : {&refs[i], &refs[j]}) {
      if (t->buf == BUF_WORK) arena.release(t->off);
      if (t->cslot >= 0) arena.release(t->cslot);
    }
    refs.push_back(r);
  }
  P.err_bound = std::sqrt(err2);
  const TRef& fin = refs.back();
  P.final_buf = fin.buf;
  P.final_off = fin.off;
  P.final_bits = P.n_open;
  TN_REQUIRE(int(fin.labels.size()) == P.n_open, TN_ERR_ARG,
             "internal: final tensor does not carry exactly the open legs");
  std::memset(P.final_pos, 0, sizeof(P.final_pos));
  for (int j = 0; j < P.n_open; ++j) {
    const int q = P.open_qubits[P.n_open - 1 - j];
    const int p = pos_of(fin.labels, net.out_label[q]);
    TN_REQUIRE(p >= 0, TN_ERR_ARG, "internal: open leg missing from the result");
    P.final_pos[j] = int8_t(p);
  }
  P.work_elems = arena.high_water();
  return P;
}

double modelled_job_seconds(const AmpPlan& P) {
  constexpr double kSplitGemm = 350e12, kOther = 120e12, kHbm = 4.0e12, kLaunch = 5e-6;
  double t = 0;
  for (const PlanOp& op : P.ops) {
    const double f = op.kind == OP_GEMM && op.gm.packed ? kSplitGemm : kOther;
    t += std::max(op.flops / f, op.bytes / kHbm) + kLaunch;
  }
  return t;
}

}  // namespace tn

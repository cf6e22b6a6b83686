// Gate and channel matrices.  Definitions: the gate-set conventions stated in
// tn.h (sqrt-rotations R_P(pi/2), fSim, controlled phase) and the Kraus sets
// of the depolarising and amplitude-damping channels (Sec. 3.3, Eq. 3, whose
// completeness sum_k A_k^+ A_k = 1 each set satisfies).
#include "gates.hpp"

#include <cmath>

namespace tn {

Mat Mat::identity(int d) {
  Mat m(d);
  for (int i = 0; i < d; ++i) m(i, i) = 1.0;
  return m;
}

Mat matmul(const Mat& x, const Mat& y) {
  Mat r(x.dim);
  for (int i = 0; i < x.dim; ++i)
    for (int k = 0; k < x.dim; ++k) {
      cd v = x(i, k);
      if (v == cd(0, 0)) continue;
      for (int j = 0; j < x.dim; ++j) r(i, j) += v * y(k, j);
    }
  return r;
}

Mat kron(const Mat& x, const Mat& y) {
  Mat r(x.dim * y.dim);
  for (int i = 0; i < x.dim; ++i)
    for (int j = 0; j < x.dim; ++j)
      for (int k = 0; k < y.dim; ++k)
        for (int l = 0; l < y.dim; ++l) r(i * y.dim + k, j * y.dim + l) = x(i, j) * y(k, l);
  return r;
}

bool is_identity(const Mat& m) {
  for (int i = 0; i < m.dim; ++i)
    for (int j = 0; j < m.dim; ++j)
      if (m(i, j) != (i == j ? cd(1, 0) : cd(0, 0))) return false;
  return true;
}

bool is_unitary(const Mat& m, double tol) {
  for (int i = 0; i < m.dim; ++i)
    for (int j = 0; j < m.dim; ++j) {
      cd s(0, 0);
      for (int k = 0; k < m.dim; ++k) s += std::conj(m(k, i)) * m(k, j);
      if (std::abs(s - (i == j ? cd(1, 0) : cd(0, 0))) > tol) return false;
    }
  return true;
}

static Mat pauli(int k) {
  Mat m(2);
  switch (k) {
    case 0: m(0, 0) = 1; m(1, 1) = 1; break;
    case 1: m(0, 1) = 1; m(1, 0) = 1; break;
    case 2: m(0, 1) = cd(0, -1); m(1, 0) = cd(0, 1); break;
    default: m(0, 0) = 1; m(1, 1) = -1; break;
  }
  return m;
}

// cos(theta/2) I - i sin(theta/2) P
static Mat rotation(const Mat& P, double theta) {
  Mat r(2);
  const double c = std::cos(theta / 2), s = std::sin(theta / 2);
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) r(i, j) = (i == j ? c : 0.0) + cd(0, -s) * P(i, j);
  return r;
}

bool gate_is_channel(int g) {
  return g == TN_CHAN_DEPOL1 || g == TN_CHAN_DEPOL2 || g == TN_CHAN_AMP_DAMP;
}

int gate_arity(int g) {
  switch (g) {
    case TN_GATE_SQRT_X: case TN_GATE_SQRT_Y: case TN_GATE_SQRT_W: case TN_GATE_H:
    case TN_GATE_X: case TN_GATE_Y: case TN_GATE_Z: case TN_GATE_S: case TN_GATE_T:
    case TN_GATE_RZ: case TN_GATE_CUSTOM1: case TN_CHAN_DEPOL1: case TN_CHAN_AMP_DAMP:
      return 1;
    case TN_GATE_CZ: case TN_GATE_CX: case TN_GATE_FSIM: case TN_GATE_CPHASE:
    case TN_GATE_SWAP: case TN_GATE_CUSTOM2: case TN_CHAN_DEPOL2:
      return 2;
    default:
      throw Error(TN_ERR_GATE, "unknown gate id " + std::to_string(g));
  }
}

Mat gate_unitary(const tn_op& op) {
  const double PI = 3.14159265358979323846;
  switch (op.gate) {
    case TN_GATE_SQRT_X: return rotation(pauli(1), PI / 2);
    case TN_GATE_SQRT_Y: return rotation(pauli(2), PI / 2);
    case TN_GATE_SQRT_W: {
      Mat W(2);
      const double r = 1.0 / std::sqrt(2.0);
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) W(i, j) = r * (pauli(1)(i, j) + pauli(2)(i, j));
      return rotation(W, PI / 2);
    }
    case TN_GATE_H: {
      Mat m(2);
      const double r = 1.0 / std::sqrt(2.0);
      m(0, 0) = r; m(0, 1) = r; m(1, 0) = r; m(1, 1) = -r;
      return m;
    }
    case TN_GATE_X: return pauli(1);
    case TN_GATE_Y: return pauli(2);
    case TN_GATE_Z: return pauli(3);
    case TN_GATE_S: { Mat m(2); m(0, 0) = 1; m(1, 1) = cd(0, 1); return m; }
    case TN_GATE_T: { Mat m(2); m(0, 0) = 1; m(1, 1) = std::polar(1.0, PI / 4); return m; }
    case TN_GATE_RZ: {
      Mat m(2);
      m(0, 0) = std::polar(1.0, -op.param[0] / 2);
      m(1, 1) = std::polar(1.0, op.param[0] / 2);
      return m;
    }
    case TN_GATE_CZ: { Mat m = Mat::identity(4); m(3, 3) = -1; return m; }
    case TN_GATE_CX: {
      Mat m(4);
      m(0, 0) = 1; m(1, 1) = 1; m(2, 3) = 1; m(3, 2) = 1;
      return m;
    }
    case TN_GATE_SWAP: {
      Mat m(4);
      m(0, 0) = 1; m(1, 2) = 1; m(2, 1) = 1; m(3, 3) = 1;
      return m;
    }
    case TN_GATE_CPHASE: { Mat m = Mat::identity(4); m(3, 3) = std::polar(1.0, op.param[0]); return m; }
    case TN_GATE_FSIM: {
      Mat m(4);
      const double c = std::cos(op.param[0]), s = std::sin(op.param[0]);
      m(0, 0) = 1;
      m(1, 1) = c; m(2, 2) = c;
      m(1, 2) = cd(0, -s); m(2, 1) = cd(0, -s);
      m(3, 3) = std::polar(1.0, -op.param[1]);
      return m;
    }
    case TN_GATE_CUSTOM1:
    case TN_GATE_CUSTOM2: {
      const int d = op.gate == TN_GATE_CUSTOM1 ? 2 : 4;
      TN_REQUIRE(op.matrix != nullptr, TN_ERR_ARG, "custom gate without matrix");
      Mat m(d);
      for (int i = 0; i < d * d; ++i) m.a[i] = cd(op.matrix[2 * i], op.matrix[2 * i + 1]);
      TN_REQUIRE(is_unitary(m, 1e-9), TN_ERR_GATE, "custom gate matrix is not unitary");
      return m;
    }
    default:
      throw Error(TN_ERR_GATE, "not a unitary gate id " + std::to_string(op.gate));
  }
}

std::vector<Mat> channel_kraus(const tn_op& op) {
  std::vector<Mat> ks;
  if (op.gate == TN_CHAN_DEPOL1) {
    const double p = op.param[0];
    TN_REQUIRE(p >= 0 && p <= 1, TN_ERR_GATE, "depolarising rate outside [0,1]");
    for (int k = 0; k < 4; ++k) {
      Mat m = pauli(k);
      const double w = std::sqrt(k == 0 ? 1 - p : p / 3);
      for (auto& v : m.a) v *= w;
      ks.push_back(m);
    }
  } else if (op.gate == TN_CHAN_DEPOL2) {
    const double p = op.param[0];
    TN_REQUIRE(p >= 0 && p <= 1, TN_ERR_GATE, "depolarising rate outside [0,1]");
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        Mat m = kron(pauli(a), pauli(b));
        const double w = std::sqrt((a == 0 && b == 0) ? 1 - p : p / 15);
        for (auto& v : m.a) v *= w;
        ks.push_back(m);
      }
  } else if (op.gate == TN_CHAN_AMP_DAMP) {
    const double g = op.param[0];
    TN_REQUIRE(g >= 0 && g <= 1, TN_ERR_GATE, "damping rate outside [0,1]");
    Mat a0(2), a1(2);
    a0(0, 0) = 1; a0(1, 1) = std::sqrt(1 - g);
    a1(0, 1) = std::sqrt(g);
    ks.push_back(a0);
    ks.push_back(a1);
  } else {
    throw Error(TN_ERR_GATE, "not a channel id " + std::to_string(op.gate));
  }
  return ks;
}

}  // namespace tn

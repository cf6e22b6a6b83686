// Gate and Kraus matrices built from identifiers (library side).
#pragma once

#include <vector>

#include "common.hpp"

namespace tn {

// Dense complex matrix, row-major, dim x dim.
struct Mat {
  int dim = 0;
  std::vector<cd> a;
  Mat() = default;
  explicit Mat(int d) : dim(d), a(size_t(d) * d, cd(0, 0)) {}
  cd& operator()(int r, int c) { return a[size_t(r) * dim + c]; }
  const cd& operator()(int r, int c) const { return a[size_t(r) * dim + c]; }
  static Mat identity(int d);
};

Mat matmul(const Mat& x, const Mat& y);
Mat kron(const Mat& x, const Mat& y);
bool is_identity(const Mat& m);
bool is_unitary(const Mat& m, double tol);

bool gate_is_channel(int gate);
int gate_arity(int gate);  // 1 or 2; throws TN_ERR_GATE for unknown ids
// Unitary of a gate op; throws TN_ERR_GATE for channels / unknown ids.
Mat gate_unitary(const tn_op& op);
// Kraus operators of a channel op, in branch order.
std::vector<Mat> channel_kraus(const tn_op& op);

}  // namespace tn

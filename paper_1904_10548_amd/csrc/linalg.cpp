// Small dense FP64 linear algebra on the host for the offline factor step:
// products, a Householder QR of E' (basis of ker E and the minimum-norm
// particular input), and Cholesky factorisation/solves.
#include <cmath>

#include "internal.h"

namespace tapg {

Mat Mat::eye(int n) {
  Mat I(n, n);
  for (int i = 0; i < n; ++i) I(i, i) = 1.0;
  return I;
}

Mat Mat::from(const double* p, int rows, int cols) {
  Mat M(rows, cols);
  for (size_t i = 0; i < M.a.size(); ++i) M.a[i] = p[i];
  return M;
}

Mat matmul(const Mat& A, const Mat& B) {
  Mat C(A.r, B.c);
  for (int i = 0; i < A.r; ++i) {
    double* ci = &C.a[(size_t)i * C.c];
    for (int k = 0; k < A.c; ++k) {
      const double aik = A(i, k);
      if (aik == 0.0) continue;
      const double* bk = &B.a[(size_t)k * B.c];
      for (int j = 0; j < B.c; ++j) ci[j] += aik * bk[j];
    }
  }
  return C;
}

Mat transpose(const Mat& A) {
  Mat T(A.c, A.r);
  for (int i = 0; i < A.r; ++i)
    for (int j = 0; j < A.c; ++j) T(j, i) = A(i, j);
  return T;
}

Mat add(const Mat& A, const Mat& B, double beta) {
  Mat C = A;
  for (size_t i = 0; i < C.a.size(); ++i) C.a[i] += beta * B.a[i];
  return C;
}

bool null_space_and_particular(const Mat& E, const Mat& Ed, Mat& Z, Mat& Pd) {
  const int ns = E.r, nu = E.c, nd = Ed.c;
  Mat M = transpose(E);  // nu x ns, reduced to R in place
  std::vector<std::vector<double>> vs;
  double scale = 0.0;
  for (double v : E.a) scale = std::fmax(scale, std::fabs(v));
  for (int j = 0; j < ns; ++j) {
    double nrm = 0.0;
    for (int i = j; i < nu; ++i) nrm += M(i, j) * M(i, j);
    nrm = std::sqrt(nrm);
    if (!(nrm > 1e-12 * std::fmax(scale, 1e-300))) return false;
    const double alpha = M(j, j) > 0 ? -nrm : nrm;
    std::vector<double> v(nu - j);
    for (int i = j; i < nu; ++i) v[i - j] = M(i, j);
    v[0] -= alpha;
    double vn = 0.0;
    for (double t : v) vn += t * t;
    vn = std::sqrt(vn);
    for (double& t : v) t /= vn;
    for (int c = j; c < ns; ++c) {
      double d = 0.0;
      for (int i = j; i < nu; ++i) d += v[i - j] * M(i, c);
      for (int i = j; i < nu; ++i) M(i, c) -= 2.0 * d * v[i - j];
    }
    vs.push_back(std::move(v));
  }
  // Q = H_0 ... H_{ns-1}, applied to the identity from the last reflection.
  Mat Q = Mat::eye(nu);
  for (int j = ns - 1; j >= 0; --j) {
    const std::vector<double>& v = vs[j];
    for (int c = 0; c < nu; ++c) {
      double d = 0.0;
      for (int i = j; i < nu; ++i) d += v[i - j] * Q(i, c);
      for (int i = j; i < nu; ++i) Q(i, c) -= 2.0 * d * v[i - j];
    }
  }
  const int m = nu - ns;
  Z = Mat(nu, m);
  for (int i = 0; i < nu; ++i)
    for (int k = 0; k < m; ++k) Z(i, k) = Q(i, ns + k);
  // E = R' Q1'; minimum-norm solution of E u = b is Q1 R'^{-1} b.
  Mat Y(ns, nd);
  for (int c = 0; c < nd; ++c) {
    for (int i = 0; i < ns; ++i) {  // R' is lower triangular: (R')_{ik} = R_{ki}
      double s = Ed(i, c);
      for (int k = 0; k < i; ++k) s -= M(k, i) * Y(k, c);
      Y(i, c) = s / M(i, i);
    }
  }
  Pd = Mat(nu, nd);
  for (int i = 0; i < nu; ++i)
    for (int c = 0; c < nd; ++c) {
      double s = 0.0;
      for (int k = 0; k < ns; ++k) s += Q(i, k) * Y(k, c);
      Pd(i, c) = -s;
    }
  return true;
}

bool cholesky(Mat& M) {
  const int n = M.r;
  for (int j = 0; j < n; ++j) {
    double d = M(j, j);
    for (int k = 0; k < j; ++k) d -= M(j, k) * M(j, k);
    if (!(d > 0.0)) return false;
    d = std::sqrt(d);
    M(j, j) = d;
    for (int i = j + 1; i < n; ++i) {
      double s = M(i, j);
      for (int k = 0; k < j; ++k) s -= M(i, k) * M(j, k);
      M(i, j) = s / d;
    }
    for (int i = 0; i < j; ++i) M(i, j) = 0.0;
  }
  return true;
}

void chol_solve(const Mat& L, Mat& B) {
  const int n = L.r;
  for (int c = 0; c < B.c; ++c) {
    for (int i = 0; i < n; ++i) {
      double s = B(i, c);
      for (int k = 0; k < i; ++k) s -= L(i, k) * B(k, c);
      B(i, c) = s / L(i, i);
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = B(i, c);
      for (int k = i + 1; k < n; ++k) s -= L(k, i) * B(k, c);
      B(i, c) = s / L(i, i);
    }
  }
}

}  // namespace tapg

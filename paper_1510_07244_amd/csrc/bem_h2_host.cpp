// Host-side pieces of the Green cross approximation (Sec. 2.3-2.4): Green
// boxes and quadrature points, and adaptive cross approximation with full
// pivoting (the adaptive part that stays on the CPU).
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "bem_internal.h"

namespace {

using cplx = std::complex<double>;

// LU factorisation with partial pivoting and inverse of a k x k matrix
// (column-major), in place into inv.  Returns false if singular.
template <class T>
bool invert(int k, std::vector<T> &a, std::vector<T> &inv) {
  std::vector<int> perm(k);
  for (int i = 0; i < k; ++i) perm[i] = i;
  for (int c = 0; c < k; ++c) {
    int p = c;
    for (int r = c + 1; r < k; ++r)
      if (std::abs(a[r + (size_t)k * c]) > std::abs(a[p + (size_t)k * c])) p = r;
    if (std::abs(a[p + (size_t)k * c]) == 0.0) return false;
    if (p != c) {
      for (int j = 0; j < k; ++j) std::swap(a[c + (size_t)k * j], a[p + (size_t)k * j]);
      std::swap(perm[c], perm[p]);
    }
    for (int r = c + 1; r < k; ++r) {
      const T f = a[r + (size_t)k * c] / a[c + (size_t)k * c];
      a[r + (size_t)k * c] = f;
      for (int j = c + 1; j < k; ++j) a[r + (size_t)k * j] -= f * a[c + (size_t)k * j];
    }
  }
  // solve L U x = e_perm for every unit vector
  inv.assign((size_t)k * k, T(0));
  std::vector<T> x(k);
  for (int col = 0; col < k; ++col) {
    for (int i = 0; i < k; ++i) x[i] = perm[i] == col ? T(1) : T(0);
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < i; ++j) x[i] -= a[i + (size_t)k * j] * x[j];
    for (int i = k - 1; i >= 0; --i) {
      for (int j = i + 1; j < k; ++j) x[i] -= a[i + (size_t)k * j] * x[j];
      x[i] /= a[i + (size_t)k * i];
    }
    for (int i = 0; i < k; ++i) inv[i + (size_t)k * col] = x[i];
  }
  return true;
}

// ACA with full pivoting on an n x m matrix: repeatedly pick the entry of
// largest modulus of the residual (ties: smallest row, then column), stop
// when it is at most eps times the first pivot or max_rank is reached, and
// subtract the rank-one cross through it.
template <class T>
int aca_one(int n, int m, const T *A, double eps, int max_rank, int32_t *prow, int32_t *pcol,
            T *pinv) {
  std::vector<T> R(A, A + (size_t)n * m);
  double first = -1.0;
  int k = 0;
  const int kmax = std::min(max_rank, std::min(n, m));
  while (k < kmax) {
    int bi = 0, bj = 0;
    double best = -1.0;
    for (int j = 0; j < m; ++j)
      for (int i = 0; i < n; ++i) {
        const double v = std::abs(R[i + (size_t)n * j]);
        if (v > best || (v == best && (i < bi || (i == bi && j < bj)))) {
          // column-major scan: the strict > keeps the smallest column for a
          // row; the explicit tie rule makes the order independent of it
          best = v;
          bi = i;
          bj = j;
        }
      }
    if (first < 0) first = best;
    if (!(best > eps * first) || best == 0.0) break;
    const T p = R[bi + (size_t)n * bj];
    std::vector<T> col(n), row(m);
    for (int i = 0; i < n; ++i) col[i] = R[i + (size_t)n * bj];
    for (int j = 0; j < m; ++j) row[j] = R[bi + (size_t)n * j] / p;
    for (int j = 0; j < m; ++j)
      for (int i = 0; i < n; ++i) R[i + (size_t)n * j] -= col[i] * row[j];
    prow[k] = bi;
    pcol[k] = bj;
    ++k;
  }
  // inverse of the pivot block A[rows, cols]
  std::vector<T> blk((size_t)k * k), inv;
  for (int c = 0; c < k; ++c)
    for (int r = 0; r < k; ++r) blk[r + (size_t)k * c] = A[prow[r] + (size_t)n * pcol[c]];
  if (k > 0 && !invert(k, blk, inv)) return -1;
  for (size_t t = 0; t < (size_t)k * k; ++t) pinv[t] = inv[t];
  return k;
}

}  // namespace

extern "C" {

int bem_green_points(int32_t ncl, const double *cl_box, int32_t qg, double *z, double *zn,
                     double *zw, double *delta) {
  if (ncl < 0 || qg < 1 || qg > BEM_MAX_ORDER || (ncl > 0 && (!cl_box || !z || !zn || !zw || !delta)))
    return BEM_EINVAL;
  std::vector<double> gx(qg), gw(qg);
  bem::gauss_legendre01(qg, gx.data(), gw.data());
  const int m = 6 * qg * qg;
  for (int32_t c = 0; c < ncl; ++c) {
    const double *b = cl_box + 6 * (size_t)c;
    double lo[3], hi[3], d2 = 0;
    for (int k = 0; k < 3; ++k) d2 += (b[3 + k] - b[k]) * (b[3 + k] - b[k]);
    const double dt = std::sqrt(d2);
    for (int k = 0; k < 3; ++k) lo[k] = b[k] - dt / 2.0, hi[k] = b[3 + k] + dt / 2.0;
    delta[c] = dt;
    int p = 0;
    for (int axis = 0; axis < 3; ++axis) {
      const int u = axis == 0 ? 1 : 0, w = axis == 2 ? 1 : 2;
      const double area = (hi[u] - lo[u]) * (hi[w] - lo[w]);
      for (int side = 0; side < 2; ++side)
        for (int a = 0; a < qg; ++a)
          for (int bb = 0; bb < qg; ++bb, ++p) {
            double *pz = z + 3 * ((size_t)c * m + p), *pn = zn + 3 * ((size_t)c * m + p);
            pz[axis] = side ? hi[axis] : lo[axis];
            pz[u] = lo[u] + gx[a] * (hi[u] - lo[u]);
            pz[w] = lo[w] + gx[bb] * (hi[w] - lo[w]);
            pn[0] = pn[1] = pn[2] = 0.0;
            pn[axis] = side ? 1.0 : -1.0;
            zw[(size_t)c * m + p] = gw[a] * gw[bb] * area;
          }
    }
  }
  return BEM_OK;
}

int bem_aca(int32_t nmat, const int64_t *a_off, const int32_t *nrows, int32_t ncols,
            int32_t is_complex, const double *A, double eps, int32_t max_rank, int32_t *rank,
            int32_t *piv_rows, int32_t *piv_cols, double *pinv) {
  if (nmat < 0 || ncols < 0 || max_rank < 1 || !(eps >= 0) ||
      (nmat > 0 && (!a_off || !nrows || !A || !rank || !piv_rows || !piv_cols || !pinv)))
    return BEM_EINVAL;
  for (int32_t t = 0; t < nmat; ++t)
    if (nrows[t] < 0 || a_off[t] < 0) return BEM_EINVAL;
  int status = BEM_OK;
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t t = 0; t < nmat; ++t) {
    const size_t kk = (size_t)max_rank * max_rank;
    int k;
    if (is_complex) {
      k = aca_one<cplx>(nrows[t], ncols, reinterpret_cast<const cplx *>(A) + a_off[t], eps,
                        max_rank, piv_rows + (size_t)t * max_rank,
                        piv_cols + (size_t)t * max_rank,
                        reinterpret_cast<cplx *>(pinv) + t * kk);
    } else {
      k = aca_one<double>(nrows[t], ncols, A + a_off[t], eps, max_rank,
                          piv_rows + (size_t)t * max_rank, piv_cols + (size_t)t * max_rank,
                          pinv + t * kk);
    }
    if (k < 0) {
#pragma omp critical
      status = BEM_ENONFINITE;
      k = 0;
    }
    rank[t] = k;
  }
  return status;
}

}  // extern "C"

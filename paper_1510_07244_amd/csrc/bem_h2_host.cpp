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
// subtract the rank-one cross through it.  Moduli are compared squared; the
// subtraction of a cross and the search for the next pivot share one pass
// over the residual (a column's maximum by a vectorisable reduction, its
// first row only when it can win).
inline double mag2(double v) { return v * v; }
inline double mag2(const cplx &v) { return v.real() * v.real() + v.imag() * v.imag(); }
// c[i] -= col[i] * r over a column of n doubles (complex: n / 2 entries,
// products written out), returning the largest squared modulus of the
// updated column.  Four lanes at a time in vector registers (the maximum of
// non-negative squares does not depend on the order it is taken in).
typedef double d4 __attribute__((ext_vector_type(4)));
inline d4 load4(const double *p) {
  d4 v;
  __builtin_memcpy(&v, p, sizeof(v));
  return v;
}
inline void store4(double *p, d4 v) { __builtin_memcpy(p, &v, sizeof(v)); }
inline double hmax(d4 v) { return std::max(std::max(v[0], v[1]), std::max(v[2], v[3])); }

inline double sub_cross(double *__restrict__ c, const double *__restrict__ col, double r, int n) {
  d4 m4 = {0, 0, 0, 0};
  int i = 0;
  for (; i + 4 <= n; i += 4) {
    const d4 v = load4(c + i) - load4(col + i) * r;
    store4(c + i, v);
    m4 = __builtin_elementwise_max(m4, v * v);
  }
  double cm = hmax(m4);
  for (; i < n; ++i) {
    const double v = c[i] - col[i] * r;
    c[i] = v;
    cm = std::max(cm, v * v);
  }
  return cm;
}
inline double sub_cross(cplx *c, const cplx *col, cplx r, int n) {
  double *__restrict__ cd = reinterpret_cast<double *>(c);
  const double *__restrict__ kd = reinterpret_cast<const double *>(col);
  const double rr = r.real(), ri = r.imag();
  // interleaved (re, im) pairs: (a + ib)(rr + i ri) = (a rr - b ri) + i (a ri + b rr)
  const d4 sr = {rr, rr, rr, rr}, si = {-ri, ri, -ri, ri};
  d4 m4 = {0, 0, 0, 0};
  int i = 0;
  for (; i + 2 <= n; i += 2) {
    const d4 k = load4(kd + 2 * i);
    const d4 ks = {k[1], k[0], k[3], k[2]};  // (b, a) pairs
    const d4 v = load4(cd + 2 * i) - (k * sr + ks * si);
    store4(cd + 2 * i, v);
    const d4 q = v * v;
    const d4 qs = {q[1], q[0], q[3], q[2]};
    m4 = __builtin_elementwise_max(m4, q + qs);
  }
  double cm = hmax(m4);
  for (; i < n; ++i) {
    const double a = kd[2 * i], b = kd[2 * i + 1];
    const double x = cd[2 * i] - (a * rr - b * ri), y = cd[2 * i + 1] - (a * ri + b * rr);
    cd[2 * i] = x;
    cd[2 * i + 1] = y;
    cm = std::max(cm, x * x + y * y);
  }
  return cm;
}

// The pivot steps on a residual R (n x m, overwritten) with workspace col
// (n) and row (m); returns the rank and fills prow / pcol.
template <class T>
__attribute__((always_inline)) inline int aca_steps(int n, int m, T *R, T *col, T *row,
                                                    double eps, int kmax, int32_t *prow,
                                                    int32_t *pcol) {
  double first = -1.0, best = -1.0;
  int k = 0, bi = 0, bj = 0;
  // winner of the current scan: larger modulus, then smaller row, then
  // smaller column (columns arrive in increasing order)
  auto offer_column = [&](int j, const T *c, double cm) {  // cm: the column's largest
    if (cm < best || n == 0) return;
    int ci = 0;
    while (ci < n - 1 && mag2(c[ci]) != cm) ++ci;  // bounded: a column of NaN has no match
    if (cm > best || ci < bi) best = cm, bi = ci, bj = j;
  };
  for (int j = 0; j < m; ++j) {
    const T *c = R + (size_t)n * j;
    double cm = 0.0;
    for (int i = 0; i < n; ++i) cm = std::max(cm, mag2(c[i]));
    offer_column(j, c, cm);
  }
  while (k < kmax) {
    if (first < 0) first = best;
    if (!(best > eps * eps * first) || best == 0.0) break;
    const T p = R[bi + (size_t)n * bj];
    for (int i = 0; i < n; ++i) col[i] = R[i + (size_t)n * bj];
    for (int j = 0; j < m; ++j) row[j] = R[bi + (size_t)n * j] / p;
    prow[k] = bi;
    pcol[k] = bj;
    ++k;
    best = -1.0;
    bi = bj = 0;
    for (int j = 0; j < m; ++j) {
      T *c = R + (size_t)n * j;
      offer_column(j, c, sub_cross(c, col, row[j], n));
    }
  }
  return k;
}

// The two entry types, each also built for AVX2 (chosen at load time on
// hosts that have it).  hipcc also runs a device pass over this file, which
// has no function multiversioning: there they are plain functions.
#if defined(__HIP_DEVICE_COMPILE__)
#define BEM_HOST_CLONES
#else
#define BEM_HOST_CLONES __attribute__((target_clones("avx2", "default")))
#endif
BEM_HOST_CLONES int aca_steps_real(int n, int m, double *R, double *col, double *row,
                                   double eps, int kmax, int32_t *prow, int32_t *pcol) {
  return aca_steps<double>(n, m, R, col, row, eps, kmax, prow, pcol);
}
BEM_HOST_CLONES int aca_steps_cplx(int n, int m, cplx *R, cplx *col, cplx *row, double eps,
                                   int kmax, int32_t *prow, int32_t *pcol) {
  return aca_steps<cplx>(n, m, R, col, row, eps, kmax, prow, pcol);
}
inline int aca_steps_t(int n, int m, double *R, double *col, double *row, double eps, int kmax,
                       int32_t *prow, int32_t *pcol) {
  return aca_steps_real(n, m, R, col, row, eps, kmax, prow, pcol);
}
inline int aca_steps_t(int n, int m, cplx *R, cplx *col, cplx *row, double eps, int kmax,
                       int32_t *prow, int32_t *pcol) {
  return aca_steps_cplx(n, m, R, col, row, eps, kmax, prow, pcol);
}

template <class T>
int aca_one(int n, int m, const T *A, double eps, int max_rank, int32_t *prow, int32_t *pcol,
            T *pinv) {
  std::vector<T> R(A, A + (size_t)n * m), col(n), row(m);
  const int kmax = std::min(max_rank, std::min(n, m));
  const int k = aca_steps_t(n, m, R.data(), col.data(), row.data(), eps, kmax, prow, pcol);
  // inverse of the pivot block A[rows, cols]
  if (!pinv) return k;  // pivots only (the inverse is formed on the device)
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
      (nmat > 0 && (!a_off || !nrows || !A || !rank || !piv_rows || !piv_cols)))
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
                        pinv ? reinterpret_cast<cplx *>(pinv) + t * kk : nullptr);
    } else {
      k = aca_one<double>(nrows[t], ncols, A + a_off[t], eps, max_rank,
                          piv_rows + (size_t)t * max_rank, piv_cols + (size_t)t * max_rank,
                          pinv ? pinv + t * kk : nullptr);
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

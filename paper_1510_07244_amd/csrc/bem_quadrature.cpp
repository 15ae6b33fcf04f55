// Host-side quadrature tables of the library: Gauss-Legendre rules, the
// per-triangle regular rules and the Sauter-Schwab region rules.  Built once
// per (rule, order) and uploaded to the device by the context.
#include <array>
#include <cmath>
#include <stdexcept>

#include "bem_internal.h"

namespace bem {

// Gauss-Legendre nodes on [-1,1] are the zeros of the Legendre polynomial
// P_q; each is found by Newton's method from the classical estimate
// cos(pi (4k + 3) / (4q + 2)), with P_q and its derivative evaluated by the
// three-term recurrence (n+1) P_{n+1} = (2n+1) x P_n - n P_{n-1} and
// P_q' = q (x P_q - P_{q-1}) / (x^2 - 1).  Weights 2 / ((1 - x^2) P_q'^2).
static void legendre_and_derivative(int q, double x, double *p, double *dp) {
  double pm1 = 1.0, pq = x;
  for (int n = 1; n < q; ++n) {
    const double pn1 = ((2 * n + 1) * x * pq - n * pm1) / (n + 1);
    pm1 = pq;
    pq = pn1;
  }
  if (q == 0) pq = 1.0, pm1 = 0.0;
  *p = pq;
  *dp = q * (x * pq - pm1) / (x * x - 1.0);
}

void gauss_legendre01(int q, double *x, double *w) {
  if (q < 1) throw std::invalid_argument("gauss order");
  for (int k = 0; k < q; ++k) {
    double z = std::cos(M_PI * (4.0 * k + 3.0) / (4.0 * q + 2.0));
    double p, dp;
    for (int it = 0; it < 200; ++it) {
      legendre_and_derivative(q, z, &p, &dp);
      const double step = p / dp;
      z -= step;
      if (std::fabs(step) <= 1e-17) break;
    }
    legendre_and_derivative(q, z, &p, &dp);
    // z decreases with k: fill from the back so nodes on [0,1] increase
    x[q - 1 - k] = 0.5 * (1.0 + z);
    w[q - 1 - k] = 1.0 / ((1.0 - z * z) * dp * dp);  // = (2 / (...)) / 2
  }
}

TriRule triangle_rule(int rule, int q) {
  TriRule r;
  if (rule == BEM_RULE_TRI7) {
    // Radon's seven-point degree-5 rule: centroid plus two orbits of three
    // points (barycentric (a, a, 1 - 2a)), weights summing to one.
    const double rt = std::sqrt(15.0);
    const double a[2] = {(6.0 - rt) / 21.0, (6.0 + rt) / 21.0};
    const double wo[2] = {(155.0 - rt) / 1200.0, (155.0 + rt) / 1200.0};
    std::vector<std::array<double, 4>> pts;  // l0, l1, l2, weight
    pts.push_back({1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0, 9.0 / 40.0});
    for (int o = 0; o < 2; ++o) {
      const double b = 1.0 - 2.0 * a[o];
      pts.push_back({a[o], a[o], b, wo[o]});
      pts.push_back({a[o], b, a[o], wo[o]});
      pts.push_back({b, a[o], a[o], wo[o]});
    }
    // x = l0 v0 + l1 v1 + l2 v2 = Phi(l1 + l2, l2); int_tau f = (sqrt(g)/2) sum w f
    for (auto &p : pts) {
      r.s.push_back(p[1] + p[2]);
      r.t.push_back(p[2]);
      r.w.push_back(0.5 * p[3]);
    }
    return r;
  }
  if (q < 1 || q > BEM_MAX_ORDER) throw std::invalid_argument("order");
  // Duffy: (s, t) = (x1, x1 x2) on [0,1]^2, Jacobian x1 (Sec. 2.2)
  std::vector<double> gx(q), gw(q);
  gauss_legendre01(q, gx.data(), gw.data());
  for (int a = 0; a < q; ++a)
    for (int b = 0; b < q; ++b) {
      r.s.push_back(gx[a]);
      r.t.push_back(gx[a] * gx[b]);
      r.w.push_back(gw[a] * gw[b] * gx[a]);
    }
  return r;
}

// One point of a Sauter-Schwab region: returns (x^1, x^2, y^1, y^2) and the
// Jacobian of the region map at (xi, h1, h2, h3) in [0,1]^4.  The maps send
// [0,1]^4 onto a piece of {0 <= x2 <= x1 <= 1}^2 such that the pieces of one
// class tile it; the singular set (x^ = y^, resp. the common edge x^2 = y^2
// = 0 with x^1 = y^1, resp. the common vertex 0) is pulled back to xi = 0,
// where the Jacobian's factor xi^3 cancels the kernel's singularity.
static void ss_point(int cls, int reg, double xi, double h1, double h2, double h3,
                     double out[4], double *jac) {
  switch (cls) {
    case CLS_IDENTICAL: {
      double p[4];
      const int piece = reg >> 1;
      if (piece == 0) {
        p[0] = xi;
        p[1] = xi * (1.0 - h1 + h1 * h2);
        p[2] = xi * (1.0 - h1 * h2 * h3);
        p[3] = xi * (1.0 - h1);
      } else if (piece == 1) {
        p[0] = xi;
        p[1] = xi * h1 * (1.0 - h2 + h2 * h3);
        p[2] = xi * (1.0 - h1 * h2);
        p[3] = xi * h1 * (1.0 - h2);
      } else {
        p[0] = xi * (1.0 - h1 * h2 * h3);
        p[1] = xi * h1 * (1.0 - h2 * h3);
        p[2] = xi;
        p[3] = xi * h1 * (1.0 - h2);
      }
      // odd pieces: the mirror image with x^ and y^ exchanged
      const int sw = (reg & 1) ? 2 : 0;
      out[0] = p[sw];
      out[1] = p[sw + 1];
      out[2] = p[2 - sw];
      out[3] = p[3 - sw];
      *jac = xi * xi * xi * h1 * h1 * h2;
      return;
    }
    case CLS_EDGE: {
      const double x3 = xi * xi * xi;
      switch (reg) {
        case 0:
          out[0] = xi;                     out[1] = xi * h1 * h3;
          out[2] = xi * (1.0 - h1 * h2);    out[3] = xi * h1 * (1.0 - h2);
          *jac = x3 * h1 * h1;
          return;
        case 1:
          out[0] = xi;                     out[1] = xi * h1;
          out[2] = xi * (1.0 - h1 * h2 * h3); out[3] = xi * h1 * h2 * (1.0 - h3);
          break;
        case 2:
          out[0] = xi * (1.0 - h1 * h2);    out[1] = xi * h1 * (1.0 - h2);
          out[2] = xi;                     out[3] = xi * h1 * h2 * h3;
          break;
        case 3:
          out[0] = xi * (1.0 - h1 * h2 * h3); out[1] = xi * h1 * h2 * (1.0 - h3);
          out[2] = xi;                     out[3] = xi * h1;
          break;
        default:
          out[0] = xi * (1.0 - h1 * h2 * h3); out[1] = xi * h1 * (1.0 - h2 * h3);
          out[2] = xi;                     out[3] = xi * h1 * h2;
          break;
      }
      *jac = x3 * h1 * h1 * h2;
      return;
    }
    default: {  // CLS_VERTEX
      const double a0 = xi, a1 = xi * h1, b0 = xi * h2, b1 = xi * h2 * h3;
      if (reg == 0) {
        out[0] = a0; out[1] = a1; out[2] = b0; out[3] = b1;
      } else {
        out[0] = b0; out[1] = b1; out[2] = a0; out[3] = a1;
      }
      *jac = xi * xi * xi * h2;
      return;
    }
  }
}

// Every region map above is linear in xi and every Jacobian carries the
// factor xi^3, so a rule point factors into its xi part and its eta part:
//   (x^, y^) = xi * g(eta),   weight = (w_a xi_a^3) * (w_b w_c w_d J(eta) / xi^3).
// The table stores g (the map at xi = 1) and the eta weight for every region
// and (eta1, eta2, eta3) Gauss triple; the xi nodes and weights are separate.
SSRule ss_rule(int cls, int q) {
  if (q < 1 || q > BEM_MAX_ORDER) throw std::invalid_argument("order");
  const int nreg = cls == CLS_IDENTICAL ? 6 : cls == CLS_EDGE ? 5 : cls == CLS_VERTEX ? 2 : 0;
  if (!nreg) throw std::invalid_argument("class");
  std::vector<double> gx(q), gw(q);
  gauss_legendre01(q, gx.data(), gw.data());
  SSRule r;
  for (int reg = 0; reg < nreg; ++reg)
    for (int b = 0; b < q; ++b)
      for (int c = 0; c < q; ++c)
        for (int d = 0; d < q; ++d) {
          double p[4], jac;
          ss_point(cls, reg, 1.0, gx[b], gx[c], gx[d], p, &jac);  // xi = 1: J = eta part
          r.xs.push_back(p[0]);
          r.xt.push_back(p[1]);
          r.ys.push_back(p[2]);
          r.yt.push_back(p[3]);
          r.w.push_back(gw[b] * gw[c] * gw[d] * jac);
        }
  return r;
}

// Identical pairs with a kernel symmetric in x and y (single layers): the odd
// regions are the mirror images (x^ <-> y^) of the even ones on the same
// triangle, so their sums are equal and the even regions with doubled
// weights give the same rule.
SSRule ss_rule_identical_symmetric(int q) {
  const SSRule full = ss_rule(CLS_IDENTICAL, q);
  const size_t per = (size_t)q * q * q;
  SSRule r;
  for (int reg = 0; reg < 6; reg += 2)
    for (size_t k = reg * per; k < (reg + 1) * per; ++k) {
      r.xs.push_back(full.xs[k]);
      r.xt.push_back(full.xt[k]);
      r.ys.push_back(full.ys[k]);
      r.yt.push_back(full.yt[k]);
      r.w.push_back(2.0 * full.w[k]);
    }
  return r;
}

XiRule xi_rule(int q) {
  if (q < 1 || q > BEM_MAX_ORDER) throw std::invalid_argument("order");
  std::vector<double> gx(q), gw(q);
  gauss_legendre01(q, gx.data(), gw.data());
  XiRule r;
  for (int a = 0; a < q; ++a) {
    r.x.push_back(gx[a]);
    r.w3.push_back(gw[a] * gx[a] * gx[a] * gx[a]);
  }
  return r;
}

}  // namespace bem

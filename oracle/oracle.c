/*
 * Plain FP64 CPU oracle for Galerkin boundary-element matrix entries
 * (Boerm & Christophersen, "Approximation of boundary element matrices using
 * GPGPUs and nested cross approximation", arXiv 1510.07244).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant generator
 * with the HIP path.
 *
 * What it computes, for piecewise-constant (indicator) bases on flat
 * triangles tau_i (Sec. 2.1, eq. matrix_entry, and Sec. 4 for the P0 setting):
 *
 *     G_ij = int_{tau_i} int_{tau_j} k(x, y) dy dx
 *
 * with k one of (Sec. 2.1, eq. kernels; Sec. 4 for the normal derivative):
 *     Laplace SLP     1 / (4 pi r)
 *     Laplace DLP     <x - y, n(y)> / (4 pi r^3)
 *     Helmholtz SLP   exp(i kappa r) / (4 pi r)
 *     Helmholtz DLP   exp(i kappa r) (1 - i kappa r) <x - y, n(y)> / (4 pi r^3)
 * where r = |x - y| and n(y) is the outward unit normal of tau_j taken from the
 * mesh's vertex order.  The value is not the exact integral but the quadrature
 * rule of Sec. 2.2: a tensor Gauss rule after the Duffy transformation for
 * disjoint triangles, and the Sauter-Schwab rules for identical, edge- and
 * vertex-adjacent triangles.  The Sauter-Schwab region maps are not printed in
 * the paper (it cites Sauter & Schwab, Boundary Element Methods, Sec. 5.2); the
 * maps used here are the standard ones on the reference triangle
 * {0 <= t <= s <= 1} of Sec. 2.2 and are pinned by the tests (polynomial
 * reproduction, the closed-form self-integral, semi-analytic brute force and
 * the Gauss identity).
 *
 * Everything is written straight from the formulas: no blocking, no fusion,
 * no reordering beyond the order of the sums as written.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

enum { O_LAPLACE = 0, O_HELMHOLTZ = 1 };
enum { O_SLP = 0, O_DLP = 1 };
enum { O_RULE_DUFFY = 0, O_RULE_TRI7 = 1 };
enum { O_IDENTICAL = 3, O_EDGE = 2, O_VERTEX = 1, O_DISJOINT = 0 };

/* ------------------------------------------------------------------------ */
/* 1-D Gauss-Legendre rule on [0,1] (the "one dimensional Gaussian quadrature
 * formula" of Sec. 4, higher quadrature orders).  Nodes are the roots of the
 * Legendre polynomial P_q found by Newton's method from the classical
 * asymptotic guess cos(pi (k - 1/4) / (q + 1/2)); P_q and P_q' come from the
 * three-term recurrence.  Nodes are returned in increasing order.           */
int oracle_gauss01(int q, double *x, double *w)
{
    if (q < 1 || q > 64) return -1;
    for (int k = 1; k <= q; ++k) {
        double z = cos(M_PI * (k - 0.25) / (q + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;               /* P_0, P_1 */
            for (int n = 2; n <= q; ++n) {
                double p2 = ((2.0 * n - 1.0) * z * p1 - (n - 1.0) * p0) / n;
                p0 = p1;
                p1 = p2;
            }
            if (q == 1) { p1 = z; p0 = 1.0; }
            /* p1 = P_q(z), p0 = P_{q-1}(z) */
            dp = q * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        /* recompute the derivative at the converged root for the weight */
        {
            double p0 = 1.0, p1 = z;
            for (int n = 2; n <= q; ++n) {
                double p2 = ((2.0 * n - 1.0) * z * p1 - (n - 1.0) * p0) / n;
                p0 = p1;
                p1 = p2;
            }
            if (q == 1) { p1 = z; p0 = 1.0; }
            dp = q * (z * p1 - p0) / (z * z - 1.0);
        }
        double wk = 2.0 / ((1.0 - z * z) * dp * dp);
        /* z_k decreases with k; map to [0,1] increasing */
        x[k - 1] = 0.5 * (1.0 - z);
        w[k - 1] = 0.5 * wk;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Seven-point degree-5 rule on a triangle (Radon), barycentric coordinates and
 * weights normalised to sum to one.  Used for regular pairs in the dense
 * 512-triangle workload ("7-point Gauss per triangle").                     */
void oracle_tri7(double *bary, double *w)
{
    const double s15 = sqrt(15.0);
    const double a1 = (6.0 - s15) / 21.0, b1 = (9.0 + 2.0 * s15) / 21.0;
    const double a2 = (6.0 + s15) / 21.0, b2 = (9.0 - 2.0 * s15) / 21.0;
    const double w0 = 9.0 / 40.0;
    const double w1 = (155.0 - s15) / 1200.0, w2 = (155.0 + s15) / 1200.0;
    const double pts[7][3] = {
        {1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0},
        {a1, a1, b1}, {a1, b1, a1}, {b1, a1, a1},
        {a2, a2, b2}, {a2, b2, a2}, {b2, a2, a2},
    };
    const double ws[7] = {w0, w1, w1, w1, w2, w2, w2};
    for (int k = 0; k < 7; ++k) {
        for (int c = 0; c < 3; ++c) bary[3 * k + c] = pts[k][c];
        w[k] = ws[k];
    }
}

/* ------------------------------------------------------------------------ */
/* Geometry of a flat triangle (Sec. 2.2): the affine map
 *     Phi(s,t) = v0 + s (v1 - v0) + t (v2 - v1)
 * sends the reference triangle {0 <= t <= s <= 1} onto (v0,v1,v2) with
 * Phi(0,0)=v0, Phi(1,0)=v1, Phi(1,1)=v2; its Gram determinant is constant and
 * sqrt(g) = |(v1 - v0) x (v2 - v1)| = 2 * area.                             */
typedef struct {
    double v0[3], e1[3], e2[3];
} affmap;

static void sub3(const double *a, const double *b, double *c)
{
    c[0] = a[0] - b[0];
    c[1] = a[1] - b[1];
    c[2] = a[2] - b[2];
}

static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double *a, const double *b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

static double norm3(const double *a) { return sqrt(dot3(a, a)); }

static const double *vtx(const double *v, int k) { return v + 3 * (size_t)k; }

static void make_map(const double *v, int a, int b, int c, affmap *m)
{
    memcpy(m->v0, vtx(v, a), sizeof m->v0);
    sub3(vtx(v, b), vtx(v, a), m->e1);
    sub3(vtx(v, c), vtx(v, b), m->e2);
}

static void apply_map(const affmap *m, double s, double t, double *x)
{
    for (int c = 0; c < 3; ++c) x[c] = m->v0[c] + s * m->e1[c] + t * m->e2[c];
}

/* sqrt of the Gram determinant of a triangle given by vertex ids */
static double sqrt_gram(const double *v, const int *t3)
{
    double e1[3], e2[3], n[3];
    sub3(vtx(v, t3[1]), vtx(v, t3[0]), e1);
    sub3(vtx(v, t3[2]), vtx(v, t3[1]), e2);
    cross3(e1, e2, n);
    return norm3(n);
}

/* outward unit normal from the mesh's vertex order (counter-clockwise seen
 * from outside) */
static void unit_normal(const double *v, const int *t3, double *n)
{
    double e1[3], e2[3];
    sub3(vtx(v, t3[1]), vtx(v, t3[0]), e1);
    sub3(vtx(v, t3[2]), vtx(v, t3[0]), e2);
    cross3(e1, e2, n);
    double l = norm3(n);
    n[0] /= l;
    n[1] /= l;
    n[2] /= l;
}

/* ------------------------------------------------------------------------ */
/* Kernel functions (Sec. 2.1, eq. kernels; Sec. 4).  ny is the unit normal
 * at y; it is used by the double-layer kernels only.                        */
static double complex kernel_eval(int kernel, int layer, double kappa,
                                  const double *x, const double *y,
                                  const double *ny)
{
    double d[3];
    sub3(x, y, d);
    double r = norm3(d);
    if (kernel == O_LAPLACE) {
        if (layer == O_SLP) return 1.0 / (4.0 * M_PI * r);
        return dot3(d, ny) / (4.0 * M_PI * r * r * r);
    }
    double complex e = cexp(I * kappa * r);
    if (layer == O_SLP) return e / (4.0 * M_PI * r);
    return e * (1.0 - I * kappa * r) * dot3(d, ny) / (4.0 * M_PI * r * r * r);
}

/* ------------------------------------------------------------------------ */
/* Number of vertex indices two triangles have in common: 3 identical,
 * 2 common edge, 1 common vertex, 0 disjoint (Sec. 2.2, four cases).      */
int oracle_shared_vertices(const int32_t *tri, int i, int j)
{
    int c = 0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            if (tri[3 * (size_t)i + a] == tri[3 * (size_t)j + b]) ++c;
    return c;
}

/* ------------------------------------------------------------------------ */
/* Sauter-Schwab region maps (x^, y^) = R(xi, eta1, eta2, eta3) from [0,1]^4
 * into pairs of points of the reference triangle {0 <= x2 <= x1 <= 1}, with
 * their Jacobians.  Returns the number of regions for the case.
 *   identical: 6 regions, J = xi^3 eta1^2 eta2
 *   edge:      5 regions, J = xi^3 eta1^2 (region 1), xi^3 eta1^2 eta2 (2-5);
 *              the common edge is Phi(s, 0) of both triangles
 *   vertex:    2 regions, J = xi^3 eta2; the common vertex is Phi(0,0) of both */
int oracle_ss_nregions(int cs)
{
    return cs == O_IDENTICAL ? 6 : cs == O_EDGE ? 5 : cs == O_VERTEX ? 2 : 0;
}

static void ss_map(int cs, int reg, double xi, double e1, double e2, double e3,
                   double *xh, double *yh, double *jac)
{
    if (cs == O_IDENTICAL) {
        *jac = xi * xi * xi * e1 * e1 * e2;
        double a1, a2, b1, b2;
        switch (reg / 2) {
        case 0:
            a1 = xi;                     a2 = xi * (1.0 - e1 + e1 * e2);
            b1 = xi * (1.0 - e1 * e2 * e3); b2 = xi * (1.0 - e1);
            break;
        case 1:
            a1 = xi;                     a2 = xi * e1 * (1.0 - e2 + e2 * e3);
            b1 = xi * (1.0 - e1 * e2);    b2 = xi * e1 * (1.0 - e2);
            break;
        default:
            a1 = xi * (1.0 - e1 * e2 * e3); a2 = xi * e1 * (1.0 - e2 * e3);
            b1 = xi;                     b2 = xi * e1 * (1.0 - e2);
            break;
        }
        if (reg % 2 == 0) {
            xh[0] = a1; xh[1] = a2; yh[0] = b1; yh[1] = b2;
        } else { /* the same region with the roles of x^ and y^ exchanged */
            xh[0] = b1; xh[1] = b2; yh[0] = a1; yh[1] = a2;
        }
        return;
    }
    if (cs == O_EDGE) {
        switch (reg) {
        case 0:
            *jac = xi * xi * xi * e1 * e1;
            xh[0] = xi;                       xh[1] = xi * e1 * e3;
            yh[0] = xi * (1.0 - e1 * e2);      yh[1] = xi * e1 * (1.0 - e2);
            break;
        case 1:
            *jac = xi * xi * xi * e1 * e1 * e2;
            xh[0] = xi;                       xh[1] = xi * e1;
            yh[0] = xi * (1.0 - e1 * e2 * e3); yh[1] = xi * e1 * e2 * (1.0 - e3);
            break;
        case 2:
            *jac = xi * xi * xi * e1 * e1 * e2;
            xh[0] = xi * (1.0 - e1 * e2);      xh[1] = xi * e1 * (1.0 - e2);
            yh[0] = xi;                       yh[1] = xi * e1 * e2 * e3;
            break;
        case 3:
            *jac = xi * xi * xi * e1 * e1 * e2;
            xh[0] = xi * (1.0 - e1 * e2 * e3); xh[1] = xi * e1 * e2 * (1.0 - e3);
            yh[0] = xi;                       yh[1] = xi * e1;
            break;
        default:
            *jac = xi * xi * xi * e1 * e1 * e2;
            xh[0] = xi * (1.0 - e1 * e2 * e3); xh[1] = xi * e1 * (1.0 - e2 * e3);
            yh[0] = xi;                       yh[1] = xi * e1 * e2;
            break;
        }
        return;
    }
    /* common vertex */
    *jac = xi * xi * xi * e2;
    double a1 = xi, a2 = xi * e1, b1 = xi * e2, b2 = xi * e2 * e3;
    if (reg == 0) {
        xh[0] = a1; xh[1] = a2; yh[0] = b1; yh[1] = b2;
    } else {
        xh[0] = b1; xh[1] = b2; yh[0] = a1; yh[1] = a2;
    }
}

/* All points of a Sauter-Schwab rule of order q in reference coordinates:
 * pts[4*p + (0..3)] = (x^1, x^2, y^1, y^2), w[p] = Gauss weight * Jacobian.
 * Point p enumerates region, then xi, eta1, eta2, eta3 (last fastest).
 * Returns the number of points, or -1.                                      */
long oracle_ss_rule(int cs, int q, double *pts, double *w)
{
    double gx[64], gw[64];
    if (oracle_gauss01(q, gx, gw)) return -1;
    int nreg = oracle_ss_nregions(cs);
    if (nreg == 0) return -1;
    long p = 0;
    for (int reg = 0; reg < nreg; ++reg)
        for (int a = 0; a < q; ++a)
            for (int b = 0; b < q; ++b)
                for (int c = 0; c < q; ++c)
                    for (int d = 0; d < q; ++d) {
                        double jac;
                        ss_map(cs, reg, gx[a], gx[b], gx[c], gx[d], pts + 4 * p,
                               pts + 4 * p + 2, &jac);
                        w[p] = gw[a] * gw[b] * gw[c] * gw[d] * jac;
                        ++p;
                    }
    return p;
}

/* ------------------------------------------------------------------------ */
/* Relabelling of a singular pair so that the common vertices come first
 * (the convention the region maps above assume):
 *   identical: both in mesh order;
 *   edge:      common vertices {a, b} with a < b (global index); each
 *              triangle becomes (a, b, its third vertex), so the common edge
 *              is Phi(s, 0) of both;
 *   vertex:    common vertex a becomes v0 of both; the other two follow in
 *              the mesh's cyclic order after a.
 * The DLP normal is always taken from the original mesh order.             */
static void relabel(const int32_t *ti, const int32_t *tj, int cs, int *oi, int *oj)
{
    if (cs == O_IDENTICAL) {
        for (int k = 0; k < 3; ++k) { oi[k] = ti[k]; oj[k] = tj[k]; }
        return;
    }
    if (cs == O_EDGE) {
        int common[2], nc = 0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                if (ti[a] == tj[b]) common[nc++] = ti[a];
        int lo = common[0] < common[1] ? common[0] : common[1];
        int hi = common[0] < common[1] ? common[1] : common[0];
        int ci = -1, cj = -1;
        for (int k = 0; k < 3; ++k) {
            if (ti[k] != lo && ti[k] != hi) ci = ti[k];
            if (tj[k] != lo && tj[k] != hi) cj = tj[k];
        }
        oi[0] = lo; oi[1] = hi; oi[2] = ci;
        oj[0] = lo; oj[1] = hi; oj[2] = cj;
        return;
    }
    /* vertex */
    int ka = -1, kb = -1;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            if (ti[a] == tj[b]) { ka = a; kb = b; }
    for (int k = 0; k < 3; ++k) {
        oi[k] = ti[(ka + k) % 3];
        oj[k] = tj[(kb + k) % 3];
    }
}

/* ------------------------------------------------------------------------ */
typedef struct {
    int kernel, layer, rule, q_reg, q_sing;
    double kappa;
} oop;

/* Regular pair by the Duffy transformation T(s,t) = (s, s t) on both
 * triangles and a tensor Gauss rule on [0,1]^4 (Sec. 2.2):
 *   sqrt(g_i g_j) sum_{a,b,c,d} w_a w_b w_c w_d xi1 xi3
 *                 k(Phi_i(xi1, xi1 xi2), Phi_j(xi3, xi3 xi4))               */
static double complex entry_duffy(const double *v, const int32_t *ti,
                                  const int32_t *tj, const oop *p)
{
    double gx[64], gw[64];
    oracle_gauss01(p->q_reg, gx, gw);
    affmap mi, mj;
    make_map(v, ti[0], ti[1], ti[2], &mi);
    make_map(v, tj[0], tj[1], tj[2], &mj);
    double ny[3];
    unit_normal(v, tj, ny);
    const int q = p->q_reg;
    double complex sum = 0.0;
    for (int a = 0; a < q; ++a)
        for (int b = 0; b < q; ++b)
            for (int c = 0; c < q; ++c)
                for (int d = 0; d < q; ++d) {
                    double x[3], y[3];
                    apply_map(&mi, gx[a], gx[a] * gx[b], x);
                    apply_map(&mj, gx[c], gx[c] * gx[d], y);
                    double wt = gw[a] * gw[b] * gw[c] * gw[d] * gx[a] * gx[c];
                    sum += wt * kernel_eval(p->kernel, p->layer, p->kappa, x, y, ny);
                }
    return sqrt_gram(v, ti) * sqrt_gram(v, tj) * sum;
}

/* Regular pair by the 7-point rule on each triangle:
 *   area_i area_j sum_{a,b} w_a w_b k(x_a, y_b)                             */
static double complex entry_tri7(const double *v, const int32_t *ti,
                                 const int32_t *tj, const oop *p)
{
    double bary[21], w7[7];
    oracle_tri7(bary, w7);
    double ny[3];
    unit_normal(v, tj, ny);
    double complex sum = 0.0;
    for (int a = 0; a < 7; ++a)
        for (int b = 0; b < 7; ++b) {
            double x[3], y[3];
            for (int c = 0; c < 3; ++c) {
                x[c] = bary[3 * a + 0] * vtx(v, ti[0])[c] + bary[3 * a + 1] * vtx(v, ti[1])[c] +
                       bary[3 * a + 2] * vtx(v, ti[2])[c];
                y[c] = bary[3 * b + 0] * vtx(v, tj[0])[c] + bary[3 * b + 1] * vtx(v, tj[1])[c] +
                       bary[3 * b + 2] * vtx(v, tj[2])[c];
            }
            sum += w7[a] * w7[b] * kernel_eval(p->kernel, p->layer, p->kappa, x, y, ny);
        }
    double area_i = 0.5 * sqrt_gram(v, ti), area_j = 0.5 * sqrt_gram(v, tj);
    return area_i * area_j * sum;
}

/* Singular pair by the Sauter-Schwab rule of the case:
 *   sqrt(g_i g_j) sum_regions sum_{[0,1]^4 Gauss} W J k(Phi_i(x^), Phi_j(y^)) */
static double complex entry_ss(const double *v, const int32_t *ti,
                               const int32_t *tj, int cs, const oop *p)
{
    double gx[64], gw[64];
    oracle_gauss01(p->q_sing, gx, gw);
    int li[3], lj[3];
    relabel(ti, tj, cs, li, lj);
    affmap mi, mj;
    make_map(v, li[0], li[1], li[2], &mi);
    make_map(v, lj[0], lj[1], lj[2], &mj);
    double ny[3];
    unit_normal(v, tj, ny); /* original orientation */
    const int q = p->q_sing;
    double complex sum = 0.0;
    for (int reg = 0; reg < oracle_ss_nregions(cs); ++reg)
        for (int a = 0; a < q; ++a)
            for (int b = 0; b < q; ++b)
                for (int c = 0; c < q; ++c)
                    for (int d = 0; d < q; ++d) {
                        double xh[2], yh[2], jac, x[3], y[3];
                        ss_map(cs, reg, gx[a], gx[b], gx[c], gx[d], xh, yh, &jac);
                        apply_map(&mi, xh[0], xh[1], x);
                        apply_map(&mj, yh[0], yh[1], y);
                        double wt = gw[a] * gw[b] * gw[c] * gw[d] * jac;
                        sum += wt * kernel_eval(p->kernel, p->layer, p->kappa, x, y, ny);
                    }
    return sqrt_gram(v, ti) * sqrt_gram(v, tj) * sum;
}

static double complex entry(const double *v, const int32_t *tri, int i, int j,
                            const oop *p)
{
    const int32_t *ti = tri + 3 * (size_t)i, *tj = tri + 3 * (size_t)j;
    int cs = oracle_shared_vertices(tri, i, j);
    if (cs == O_DISJOINT)
        return p->rule == O_RULE_TRI7 ? entry_tri7(v, ti, tj, p) : entry_duffy(v, ti, tj, p);
    return entry_ss(v, ti, tj, cs, p);
}

/* Entries G(rows[k], cols[k]) for k < n; out[2k], out[2k+1] = Re, Im.
 * kernel: 0 Laplace, 1 Helmholtz; layer: 0 SLP, 1 DLP; rule: 0 Duffy tensor
 * Gauss of order q_reg, 1 seven-point rule; q_sing: Sauter-Schwab order.
 * Returns 0, or -1 on invalid arguments.  OpenMP over entries.             */
int oracle_entries(const double *v, int nv, const int32_t *tri, int nt,
                   int kernel, int layer, double kappa, int rule, int q_reg, int q_sing,
                   long n, const int32_t *rows, const int32_t *cols, double *out)
{
    if (kernel < 0 || kernel > 1 || layer < 0 || layer > 1) return -1;
    if (q_reg < 1 || q_reg > 64 || q_sing < 1 || q_sing > 64) return -1;
    for (long k = 0; k < 3L * nt; ++k)
        if (tri[k] < 0 || tri[k] >= nv) return -1;
    for (long k = 0; k < n; ++k)
        if (rows[k] < 0 || rows[k] >= nt || cols[k] < 0 || cols[k] >= nt) return -1;
    oop p = {kernel, layer, rule, q_reg, q_sing, kappa};
#pragma omp parallel for schedule(dynamic, 16)
    for (long k = 0; k < n; ++k) {
        double complex g = entry(v, tri, rows[k], cols[k], &p);
        out[2 * k] = creal(g);
        out[2 * k + 1] = cimag(g);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Piecewise-linear bases (Sec. 2.2, eq. reference_integral: the transformed
 * basis functions are low-order polynomials).  For a pair of triangles the
 * 3 x 3 local matrix
 *     L_kl = int_{tau_i} int_{tau_j} lambda_k(x) k(x, y) mu_l(y) dy dx,
 * with lambda_k, mu_l the nodal (barycentric) functions of the vertices of
 * tau_i and tau_j in mesh order, by the same rules as the piecewise-constant
 * entries: on the reference triangle Phi(s, t) = v0 + s (v1 - v0) +
 * t (v2 - v1) the barycentric coordinates of (v0, v1, v2) are
 * (1 - s, s - t, t); for a singular pair they are taken in the relabelled
 * order and assigned back to the mesh-order vertices.                       */
static void bary_of(double s, double t, double *b)
{
    b[0] = 1.0 - s;
    b[1] = s - t;
    b[2] = t;
}

/* local position in t3 of vertex id w */
static int local_of(const int32_t *t3, int w)
{
    return t3[0] == w ? 0 : (t3[1] == w ? 1 : 2);
}

static void p1_duffy(const double *v, const int32_t *ti, const int32_t *tj, const oop *p,
                     double complex L[9])
{
    double gx[64], gw[64];
    oracle_gauss01(p->q_reg, gx, gw);
    affmap mi, mj;
    make_map(v, ti[0], ti[1], ti[2], &mi);
    make_map(v, tj[0], tj[1], tj[2], &mj);
    double ny[3];
    unit_normal(v, tj, ny);
    const int q = p->q_reg;
    for (int e = 0; e < 9; ++e) L[e] = 0.0;
    for (int a = 0; a < q; ++a)
        for (int b = 0; b < q; ++b)
            for (int c = 0; c < q; ++c)
                for (int d = 0; d < q; ++d) {
                    double x[3], y[3], bx[3], by[3];
                    apply_map(&mi, gx[a], gx[a] * gx[b], x);
                    apply_map(&mj, gx[c], gx[c] * gx[d], y);
                    bary_of(gx[a], gx[a] * gx[b], bx);
                    bary_of(gx[c], gx[c] * gx[d], by);
                    double wt = gw[a] * gw[b] * gw[c] * gw[d] * gx[a] * gx[c];
                    double complex kv = wt * kernel_eval(p->kernel, p->layer, p->kappa, x, y, ny);
                    for (int k = 0; k < 3; ++k)
                        for (int l = 0; l < 3; ++l) L[3 * k + l] += bx[k] * kv * by[l];
                }
    double sg = sqrt_gram(v, ti) * sqrt_gram(v, tj);
    for (int e = 0; e < 9; ++e) L[e] *= sg;
}

static void p1_ss(const double *v, const int32_t *ti, const int32_t *tj, int cs, const oop *p,
                  double complex L[9])
{
    double gx[64], gw[64];
    oracle_gauss01(p->q_sing, gx, gw);
    int li[3], lj[3];
    relabel(ti, tj, cs, li, lj);
    affmap mi, mj;
    make_map(v, li[0], li[1], li[2], &mi);
    make_map(v, lj[0], lj[1], lj[2], &mj);
    double ny[3];
    unit_normal(v, tj, ny); /* original orientation */
    int pi[3], pj[3]; /* mesh-order position of relabelled vertex k */
    for (int k = 0; k < 3; ++k) {
        pi[k] = local_of(ti, li[k]);
        pj[k] = local_of(tj, lj[k]);
    }
    const int q = p->q_sing;
    for (int e = 0; e < 9; ++e) L[e] = 0.0;
    for (int reg = 0; reg < oracle_ss_nregions(cs); ++reg)
        for (int a = 0; a < q; ++a)
            for (int b = 0; b < q; ++b)
                for (int c = 0; c < q; ++c)
                    for (int d = 0; d < q; ++d) {
                        double xh[2], yh[2], jac, x[3], y[3], bx[3], by[3];
                        ss_map(cs, reg, gx[a], gx[b], gx[c], gx[d], xh, yh, &jac);
                        apply_map(&mi, xh[0], xh[1], x);
                        apply_map(&mj, yh[0], yh[1], y);
                        bary_of(xh[0], xh[1], bx);
                        bary_of(yh[0], yh[1], by);
                        double wt = gw[a] * gw[b] * gw[c] * gw[d] * jac;
                        double complex kv =
                            wt * kernel_eval(p->kernel, p->layer, p->kappa, x, y, ny);
                        for (int k = 0; k < 3; ++k)
                            for (int l = 0; l < 3; ++l)
                                L[3 * pi[k] + pj[l]] += bx[k] * kv * by[l];
                    }
    double sg = sqrt_gram(v, ti) * sqrt_gram(v, tj);
    for (int e = 0; e < 9; ++e) L[e] *= sg;
}

/* Local matrices of the pairs (rows[k], cols[k]): out[18 k + 2 (3 a + b)],
 * out[.. + 1] = Re, Im of L_ab (a: vertex of the row triangle, b: of the
 * column triangle, mesh order).  Duffy rule of order q_reg for disjoint
 * pairs (the seven-point rule is not offered), Sauter-Schwab of order q_sing
 * otherwise.  OpenMP over pairs.                                           */
int oracle_p1_pairs(const double *v, int nv, const int32_t *tri, int nt, int kernel, int layer,
                    double kappa, int q_reg, int q_sing, long n, const int32_t *rows,
                    const int32_t *cols, double *out)
{
    if (kernel < 0 || kernel > 1 || layer < 0 || layer > 1) return -1;
    if (q_reg < 1 || q_reg > 64 || q_sing < 1 || q_sing > 64) return -1;
    for (long k = 0; k < 3L * nt; ++k)
        if (tri[k] < 0 || tri[k] >= nv) return -1;
    for (long k = 0; k < n; ++k)
        if (rows[k] < 0 || rows[k] >= nt || cols[k] < 0 || cols[k] >= nt) return -1;
    oop p = {kernel, layer, O_RULE_DUFFY, q_reg, q_sing, kappa};
#pragma omp parallel for schedule(dynamic, 16)
    for (long k = 0; k < n; ++k) {
        const int32_t *ti = tri + 3 * (size_t)rows[k], *tj = tri + 3 * (size_t)cols[k];
        int cs = oracle_shared_vertices(tri, rows[k], cols[k]);
        double complex L[9];
        if (cs == O_DISJOINT) p1_duffy(v, ti, tj, &p, L);
        else p1_ss(v, ti, tj, cs, &p, L);
        for (int e = 0; e < 9; ++e) {
            out[18 * k + 2 * e] = creal(L[e]);
            out[18 * k + 2 * e + 1] = cimag(L[e]);
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Green quadrature matrices of Sec. 2.3 (eq. green_matrix).  For triangle
 * tau_i and Green quadrature point z_nu (weight w_nu, outward unit normal
 * n_nu of the box omega_t) two columns nu and m + nu:
 *   side 0 (row basis, SLP and DLP):
 *     a+ = sqrt(w) int_{tau_i} g(x, z) dx
 *     a- = sqrt(w) delta int_{tau_i} d/dn(z) g(x, z) dx
 *   side 1 (column basis of the DLP, kernel d/dn(y) g(x, y)):
 *     c+ = sqrt(w) int_{tau_j} d/dn(y) g(y, z) dy
 *     c- = sqrt(w) delta int_{tau_j} d/dn(y) d/dn(z) g(y, z) dy
 * The triangle integrals use the Duffy transformation and a q x q Gauss rule:
 *   int_tau f = sqrt(g) sum_{a,b} w_a w_b xi_a f(Phi(xi_a, xi_a xi_b)).
 * Output out[(row) + nrows * col] column-major, complex interleaved.       */
/* value of the four Green integrands at one point (x, nx) against (z, nz) */
static void green_values(int kernel, double kappa, const double *x, const double *nx,
                         const double *z, const double *nz,
                         double complex *g, double complex *dgz,
                         double complex *dgx, double complex *dgxz)
{
    double d[3];
    sub3(x, z, d); /* d = x - z */
    double r = norm3(d);
    double complex e = kernel == O_LAPLACE ? 1.0 : cexp(I * kappa * r);
    double kr = kernel == O_LAPLACE ? 0.0 : kappa * r;
    double fr = 4.0 * M_PI;
    /* g(x,z) = e / (4 pi r) */
    *g = e / (fr * r);
    /* d/dn(z) g(x,z) = e (1 - i k r) <x - z, n_z> / (4 pi r^3) */
    *dgz = e * (1.0 - I * kr) * dot3(d, nz) / (fr * r * r * r);
    /* d/dn(x) g(x,z) = e (1 - i k r) <z - x, n_x> / (4 pi r^3) */
    *dgx = -e * (1.0 - I * kr) * dot3(d, nx) / (fr * r * r * r);
    /* d/dn(x) d/dn(z) g(x,z)
     *   = e [ (1 - i k r) <n_x, n_z> / r^3
     *         + (k^2 r^2 - 3 + 3 i k r) <x - z, n_x><x - z, n_z> / r^5 ] / 4 pi  */
    *dgxz = e * ((1.0 - I * kr) * dot3(nx, nz) / (r * r * r) +
                 (kr * kr - 3.0 + 3.0 * I * kr) * dot3(d, nx) * dot3(d, nz) /
                     (r * r * r * r * r)) / fr;
}

int oracle_green_matrix(const double *v, int nv, const int32_t *tri, int nt,
                        int kernel, double kappa, int side, int q,
                        int nrows, const int32_t *rows,
                        int m, const double *z, const double *zn, const double *zw,
                        double delta, double *out)
{
    if (q < 1 || q > 64 || side < 0 || side > 1) return -1;
    for (int k = 0; k < nrows; ++k)
        if (rows[k] < 0 || rows[k] >= nt) return -1;
    for (long k = 0; k < 3L * nt; ++k)
        if (tri[k] < 0 || tri[k] >= nv) return -1;
    double gx[64], gw[64];
    oracle_gauss01(q, gx, gw);
#pragma omp parallel for schedule(dynamic, 4)
    for (int k = 0; k < nrows; ++k) {
        const int32_t *t3 = tri + 3 * (size_t)rows[k];
        affmap mp;
        make_map(v, t3[0], t3[1], t3[2], &mp);
        double nx[3];
        unit_normal(v, t3, nx);
        double sg = sqrt_gram(v, t3);
        for (int nu = 0; nu < m; ++nu) {
            double complex sp = 0.0, sm = 0.0;
            for (int a = 0; a < q; ++a)
                for (int b = 0; b < q; ++b) {
                    double x[3];
                    apply_map(&mp, gx[a], gx[a] * gx[b], x);
                    double wt = gw[a] * gw[b] * gx[a];
                    double complex g, dgz, dgx, dgxz;
                    green_values(kernel, kappa, x, nx, z + 3 * nu, zn + 3 * nu, &g, &dgz,
                                 &dgx, &dgxz);
                    if (side == 0) {
                        sp += wt * g;
                        sm += wt * dgz;
                    } else {
                        sp += wt * dgx;
                        sm += wt * dgxz;
                    }
                }
            double sw = sqrt(zw[nu]);
            double complex ap = sw * sg * sp, am = sw * delta * sg * sm;
            size_t ip = (size_t)k + (size_t)nrows * nu;
            size_t im = (size_t)k + (size_t)nrows * (m + nu);
            out[2 * ip] = creal(ap);
            out[2 * ip + 1] = cimag(ap);
            out[2 * im] = creal(am);
            out[2 * im + 1] = cimag(am);
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Algebraic interpolation of Sec. 2.3 (the cluster basis of the Green cross
 * approximation): with a cluster's Green matrix A (n rows, acols columns),
 * pivot rows t~ and pivot columns tau chosen by cross approximation (k of
 * each), the basis is
 *     V = A[:, tau] A[t~, tau]^{-1},
 * so that the rows t~ of V form the identity (R_t V = I) and V interpolates
 * every column of A that lies in the span of the pivot columns.
 * Matrices are column-major and complex interleaved (re, im).             */

/* Inverse of the k x k matrix M by Gauss-Jordan elimination with partial
 * pivoting (largest modulus in the column).  P receives M^{-1}.  Returns 0,
 * or -1 when a pivot is exactly zero.                                      */
int oracle_inverse(int k, const double *M, double *P)
{
    if (k < 1) return -1;
    size_t kk = (size_t)k * k;
    double complex *a = malloc(kk * sizeof *a), *b = malloc(kk * sizeof *b);
    if (!a || !b) { free(a); free(b); return -1; }
    for (size_t e = 0; e < kk; ++e) {
        a[e] = M[2 * e] + I * M[2 * e + 1];
        b[e] = 0.0;
    }
    for (int e = 0; e < k; ++e) b[e + (size_t)k * e] = 1.0;
    int rc = 0;
    for (int c = 0; c < k && !rc; ++c) {
        int p = c;
        for (int r = c + 1; r < k; ++r)
            if (cabs(a[r + (size_t)k * c]) > cabs(a[p + (size_t)k * c])) p = r;
        if (a[p + (size_t)k * c] == 0.0) { rc = -1; break; }
        if (p != c)
            for (int j = 0; j < k; ++j) {
                double complex t = a[c + (size_t)k * j];
                a[c + (size_t)k * j] = a[p + (size_t)k * j];
                a[p + (size_t)k * j] = t;
                t = b[c + (size_t)k * j];
                b[c + (size_t)k * j] = b[p + (size_t)k * j];
                b[p + (size_t)k * j] = t;
            }
        double complex d = a[c + (size_t)k * c];
        for (int j = 0; j < k; ++j) {
            a[c + (size_t)k * j] /= d;
            b[c + (size_t)k * j] /= d;
        }
        for (int r = 0; r < k; ++r) {
            if (r == c) continue;
            double complex f = a[r + (size_t)k * c];
            if (f == 0.0) continue;
            for (int j = 0; j < k; ++j) {
                a[r + (size_t)k * j] -= f * a[c + (size_t)k * j];
                b[r + (size_t)k * j] -= f * b[c + (size_t)k * j];
            }
        }
    }
    if (!rc)
        for (size_t e = 0; e < kk; ++e) {
            P[2 * e] = creal(b[e]);
            P[2 * e + 1] = cimag(b[e]);
        }
    free(a);
    free(b);
    return rc;
}

/* V = A[:, tau] P for a given k x k matrix P (n x k result): the basis
 * contraction, one sum per entry over the k pivot columns.                 */
int oracle_contract(int n, int acols, const double *A, int k, const int32_t *tau,
                    const double *P, double *V)
{
    if (n < 0 || k < 1) return -1;
    for (int c = 0; c < k; ++c)
        if (tau[c] < 0 || tau[c] >= acols) return -1;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < k; ++j) {
            double complex s = 0.0;
            for (int l = 0; l < k; ++l) {
                size_t ia = (size_t)i + (size_t)n * tau[l];
                size_t ip = (size_t)l + (size_t)k * j;
                s += (A[2 * ia] + I * A[2 * ia + 1]) * (P[2 * ip] + I * P[2 * ip + 1]);
            }
            size_t iv = (size_t)i + (size_t)n * j;
            V[2 * iv] = creal(s);
            V[2 * iv + 1] = cimag(s);
        }
    return 0;
}

/* The interpolation basis from the pivots alone: P = A[t~, tau]^{-1} by
 * oracle_inverse, then V = A[:, tau] P by oracle_contract.  P (k x k) may be
 * NULL.                                                                    */
int oracle_interp_basis(int n, int acols, const double *A, int k, const int32_t *prow,
                        const int32_t *tau, double *V, double *P)
{
    if (n < 1 || k < 1 || k > n || k > acols) return -1;
    for (int c = 0; c < k; ++c)
        if (prow[c] < 0 || prow[c] >= n || tau[c] < 0 || tau[c] >= acols) return -1;
    size_t kk = (size_t)k * k;
    double *M = malloc(2 * kk * sizeof *M), *Pi = malloc(2 * kk * sizeof *Pi);
    if (!M || !Pi) { free(M); free(Pi); return -1; }
    for (int c = 0; c < k; ++c)
        for (int r = 0; r < k; ++r) {
            size_t ia = (size_t)prow[r] + (size_t)n * tau[c];
            size_t im = (size_t)r + (size_t)k * c;
            M[2 * im] = A[2 * ia];
            M[2 * im + 1] = A[2 * ia + 1];
        }
    int rc = oracle_inverse(k, M, Pi);
    if (!rc) rc = oracle_contract(n, acols, A, k, tau, Pi, V);
    if (!rc && P) memcpy(P, Pi, 2 * kk * sizeof *P);
    free(M);
    free(Pi);
    return rc;
}

/* Number of OpenMP threads the oracle's parallel loops use. */
#ifdef _OPENMP
#include <omp.h>
#endif
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the following parallel loops (n >= 1). */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

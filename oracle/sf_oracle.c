/*
 * sf_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct FP64 CPU implementation of what the
 * sum-factorised assembly path computes, written directly from the
 * definitions in Homolya, Kirby & Ham, "Exposing and exploiting structure:
 * optimal code generation for high-order finite element methods":
 *
 *   - the element matrix is the plain quadrature sum of the pulled-back
 *     bilinear form (Sec. 1.1, eq. laplace_prefiat / eq. laplace_quadrature),
 *     evaluated point by point with full 3-D tables Psi_i(xi_q) and
 *     grad Psi_i(xi_q) and NO factorisation of any kind;
 *   - the operator action is the linear form a(psi_i, u) of Sec. 1.1
 *     (matrix-free action), evaluated by first summing the trial field at
 *     every quadrature point over all basis functions (eq. coeff_eval) and
 *     then testing it against every basis function (eq. form_eval), again
 *     with no factorisation: O(N_f * N_q) per cell;
 *   - tensor-product quadrature and elements (Sec. 1.2, eq. tpps,
 *     eq. limits_tpe), GL / GLL node sets (Sec. 2.5), enriched elements with
 *     concatenated bases (Sec. 2.6, eq. enriched_basis) and the H(div) /
 *     H(curl) Q^- members built from P_k and dP_{k-1} interval factors
 *     (Sec. 2.7, eq. rtcf_impl).
 *
 * Only tests/, the smoke check and the benchmark's CPU-baseline leg may load
 * this library.  It shares no code, header, table or constant with the GPU
 * library: quadrature nodes come from Newton iteration on the Legendre
 * three-term recurrence in long double, Lagrange polynomials from the product
 * formula.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math, no
 * FMA contraction), see oracle/build_oracle.py.
 *
 * Conventions (readings of the paper, stated once):
 *   - reference cell [0,1]^3; 1-D rules mapped from [-1,1] (weights sum to 1);
 *   - a cell's 8 vertices are stored at index 4*v0+2*v1+v2 for the reference
 *     vertex (v0,v1,v2) in {0,1}^3; the map x(xi) is trilinear (the vector-Q1
 *     coordinate field of Sec. 3.1);
 *   - within a block, basis functions are numbered row-major over the
 *     per-axis indices, last axis fastest (the flattening used for the
 *     RTCF_2 example in Sec. 3.5); blocks are concatenated in order;
 *   - H(div) (NCF) blocks: block c is P_k on axis c (GLL_{k+1} nodes) times
 *     dP_{k-1} (GL_k nodes) on the other axes, value +phi e_c;
 *     H(curl) (NCE) blocks: dP_{k-1} on axis c, P_k elsewhere, value +phi e_c;
 *   - vector Q_p (VQ): three blocks, block c the scalar Q_p element with
 *     value +phi e_c and no Piola map (Sec. 2.3), i.e. local DOF (c, i) at
 *     c (p+1)^3 + i;
 *   - contravariant Piola  Psi = J Psi^ / det J,  div Psi = div^ Psi^ / det J;
 *     covariant Piola      Psi = J^{-T} Psi^,    curl Psi = J curl^ Psi^ / det J;
 *   - row i = test function, column j = trial function; y = A u.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_Q 0
#define ORC_DQ 1
#define ORC_NCF 2
/* ORC_QGLL (4): Q_p on GLL nodes integrated with the GLL rule of p+1 points, so that
 * nodes and quadrature points coincide (the collocated, under-integrated spectral
 * element variant of Sec. 2.5); the same element as ORC_Q with another rule. */
#define ORC_QGLL 4
#define ORC_VQ 5
#define ORC_NCE 3

#define ORC_MASS 0
#define ORC_LAPLACE 1
#define ORC_HDIV 2
#define ORC_HCURL 3

#define ORC_MAXN 40

/* ------------------------------------------------------------------------ */
/* 1-D quadrature on [0,1] (Sec. 2.5: Gauss-Legendre and Gauss-Lobatto).    */
/* ------------------------------------------------------------------------ */

/* Legendre P_m(x) and P_{m-1}(x) by the three-term recurrence
 * (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}. */
static void legendre_pair(int m, long double x, long double *pm, long double *pm1)
{
    long double p0 = 1.0L, p1 = x;
    if (m == 0) { *pm = 1.0L; *pm1 = 0.0L; return; }
    for (int k = 1; k < m; ++k) {
        long double p2 = ((2.0L * k + 1.0L) * x * p1 - (long double)k * p0) / (k + 1.0L);
        p0 = p1;
        p1 = p2;
    }
    *pm = p1;
    *pm1 = p0;
}

/* m-point Gauss-Legendre rule on [0,1]: nodes are the roots of P_m, found by
 * Newton iteration from the Chebyshev-like initial guess; weights
 * 2 / ((1 - x^2) P_m'(x)^2) on [-1,1], halved on [0,1]. */
int orc_gauss_legendre(int m, double *x, double *w)
{
    if (m < 1 || m > ORC_MAXN) return -1;
    for (int i = 0; i < m; ++i) {
        long double t = cosl(3.14159265358979323846264338327950288L * (i + 0.75L) / (m + 0.5L));
        long double dp = 1.0L;
        for (int it = 0; it < 100; ++it) {
            long double pm, pm1;
            legendre_pair(m, t, &pm, &pm1);
            dp = (long double)m * (t * pm - pm1) / (t * t - 1.0L);
            long double dt = pm / dp;
            t -= dt;
            if (fabsl(dt) < 1e-30L) break;
        }
        {
            long double pm, pm1;
            legendre_pair(m, t, &pm, &pm1);
            dp = (long double)m * (t * pm - pm1) / (t * t - 1.0L);
        }
        /* root i of the cosine guess is in decreasing order; store ascending */
        x[m - 1 - i] = (double)((1.0L + t) * 0.5L);
        w[m - 1 - i] = (double)(1.0L / ((1.0L - t * t) * dp * dp));
    }
    if (m == 1) { x[0] = 0.5; w[0] = 1.0; }
    return 0;
}

/* m-point Gauss-Lobatto-Legendre rule on [0,1] (m >= 2): the end points and
 * the roots of P'_{m-1}; weights 2 / (m (m-1) P_{m-1}(x)^2) on [-1,1]. */
int orc_gauss_lobatto(int m, double *x, double *w)
{
    if (m < 2 || m > ORC_MAXN) return -1;
    int n = m - 1; /* polynomial degree whose derivative vanishes inside */
    for (int i = 0; i < m; ++i) {
        long double t;
        if (i == 0) t = -1.0L;
        else if (i == m - 1) t = 1.0L;
        else {
            t = -cosl(3.14159265358979323846264338327950288L * i / (long double)n);
            for (int it = 0; it < 100; ++it) {
                long double pn, pn1;
                legendre_pair(n, t, &pn, &pn1);
                /* (1-t^2) P_n' = n (P_{n-1} - t P_n);
                 * (1-t^2) P_n'' = 2 t P_n' - n (n+1) P_n */
                long double d1 = (long double)n * (pn1 - t * pn) / (1.0L - t * t);
                long double d2 = (2.0L * t * d1 - (long double)n * (n + 1.0L) * pn) / (1.0L - t * t);
                long double dt = d1 / d2;
                t -= dt;
                if (fabsl(dt) < 1e-30L) break;
            }
        }
        long double pn, pn1;
        legendre_pair(n, t, &pn, &pn1);
        x[i] = (double)((1.0L + t) * 0.5L);
        w[i] = (double)(1.0L / ((long double)m * (long double)n * pn * pn));
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Lagrange polynomials by the product formula.                             */
/* ------------------------------------------------------------------------ */

double orc_lagrange(const double *nodes, int n, int i, double x)
{
    double v = 1.0;
    for (int j = 0; j < n; ++j)
        if (j != i) v *= (x - nodes[j]) / (nodes[i] - nodes[j]);
    return v;
}

double orc_lagrange_deriv(const double *nodes, int n, int i, double x)
{
    double s = 0.0;
    for (int k = 0; k < n; ++k) {
        if (k == i) continue;
        double term = 1.0 / (nodes[i] - nodes[k]);
        for (int j = 0; j < n; ++j)
            if (j != i && j != k) term *= (x - nodes[j]) / (nodes[i] - nodes[j]);
        s += term;
    }
    return s;
}

/* ------------------------------------------------------------------------ */
/* Elements: tensor-product blocks of interval factors (Secs. 2.4, 2.6, 2.7)*/
/* ------------------------------------------------------------------------ */

typedef struct {
    int n[3];                 /* functions per axis                */
    double nodes[3][ORC_MAXN];/* interval nodes per axis           */
    int comp;                 /* vector component (-1 for scalar)  */
    int offset;               /* first flat index of the block     */
} orc_block;

typedef struct {
    int family, degree, nblocks, ndof, vector;
    orc_block b[3];
} orc_element;

static void set_axis(orc_block *bl, int a, int npts, int lobatto)
{
    double w[ORC_MAXN];
    bl->n[a] = npts;
    if (lobatto) orc_gauss_lobatto(npts, bl->nodes[a], w);
    else orc_gauss_legendre(npts, bl->nodes[a], w);
}

static int make_element(int family, int degree, orc_element *e)
{
    memset(e, 0, sizeof(*e));
    e->family = family;
    e->degree = degree;
    if (family == ORC_Q || family == ORC_DQ || family == ORC_QGLL) {
        if (degree < 1 || degree + 1 > ORC_MAXN) return -1;
        e->nblocks = 1;
        e->vector = 0;
        for (int a = 0; a < 3; ++a) set_axis(&e->b[0], a, degree + 1, family != ORC_DQ);
        e->b[0].comp = -1;
        e->b[0].offset = 0;
        e->ndof = (degree + 1) * (degree + 1) * (degree + 1);
        return 0;
    }
    if (family == ORC_VQ) { /* vector Q_p: the scalar basis times the unit vectors (Sec. 2.3) */
        if (degree < 1 || degree + 1 > ORC_MAXN) return -1;
        int n = degree + 1;
        e->nblocks = 3;
        e->vector = 1;
        for (int c = 0; c < 3; ++c) {
            for (int a = 0; a < 3; ++a) set_axis(&e->b[c], a, n, 1);
            e->b[c].comp = c;
            e->b[c].offset = c * n * n * n;
        }
        e->ndof = 3 * n * n * n;
        return 0;
    }
    if (family == ORC_NCF || family == ORC_NCE) {
        int k = degree;
        if (k < 1 || k + 1 > ORC_MAXN) return -1;
        e->nblocks = 3;
        e->vector = 1;
        int off = 0;
        for (int c = 0; c < 3; ++c) {
            for (int a = 0; a < 3; ++a) {
                int pk_axis = (family == ORC_NCF) ? (a == c) : (a != c);
                if (pk_axis) set_axis(&e->b[c], a, k + 1, 1); /* P_k on GLL_{k+1} */
                else set_axis(&e->b[c], a, k, 0);             /* dP_{k-1} on GL_k */
            }
            e->b[c].comp = c;
            e->b[c].offset = off;
            off += e->b[c].n[0] * e->b[c].n[1] * e->b[c].n[2];
        }
        e->ndof = off;
        return 0;
    }
    return -1;
}

int orc_element_ndof(int family, int degree)
{
    orc_element e;
    if (make_element(family, degree, &e)) return -1;
    return e.ndof;
}

/* Reference values at point xi.  For every basis function i:
 *   val[i*3 + c]    vector value (scalar families: val[i*3] only),
 *   grad[i*9 + 3*c + b] = d(val_c)/d xi_b.                                 */
static void tabulate_point(const orc_element *e, const double xi[3], double *val, double *grad)
{
    for (int bI = 0; bI < e->nblocks; ++bI) {
        const orc_block *bl = &e->b[bI];
        double l[3][ORC_MAXN], dl[3][ORC_MAXN];
        for (int a = 0; a < 3; ++a)
            for (int i = 0; i < bl->n[a]; ++i) {
                l[a][i] = orc_lagrange(bl->nodes[a], bl->n[a], i, xi[a]);
                dl[a][i] = orc_lagrange_deriv(bl->nodes[a], bl->n[a], i, xi[a]);
            }
        int c = bl->comp < 0 ? 0 : bl->comp;
        for (int i0 = 0; i0 < bl->n[0]; ++i0)
            for (int i1 = 0; i1 < bl->n[1]; ++i1)
                for (int i2 = 0; i2 < bl->n[2]; ++i2) {
                    int I = bl->offset + (i0 * bl->n[1] + i1) * bl->n[2] + i2;
                    double phi = l[0][i0] * l[1][i1] * l[2][i2];
                    double g[3] = {dl[0][i0] * l[1][i1] * l[2][i2],
                                   l[0][i0] * dl[1][i1] * l[2][i2],
                                   l[0][i0] * l[1][i1] * dl[2][i2]};
                    for (int cc = 0; cc < 3; ++cc) {
                        val[I * 3 + cc] = (cc == c) ? phi : 0.0;
                        for (int b = 0; b < 3; ++b) grad[I * 9 + 3 * cc + b] = (cc == c) ? g[b] : 0.0;
                    }
                }
    }
}

/* exported for tests: reference tabulation at one point */
int orc_tabulate(int family, int degree, const double *xi, double *val, double *grad)
{
    orc_element e;
    if (make_element(family, degree, &e)) return -1;
    tabulate_point(&e, xi, val, grad);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Geometry: trilinear (vector-Q1) coordinate map, Sec. 1.1 and Sec. 3.1.   */
/* ------------------------------------------------------------------------ */

static void jacobian(const double *X /*[8][3]*/, const double xi[3], double J[3][3])
{
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) J[a][b] = 0.0;
    for (int v0 = 0; v0 < 2; ++v0)
        for (int v1 = 0; v1 < 2; ++v1)
            for (int v2 = 0; v2 < 2; ++v2) {
                int v = 4 * v0 + 2 * v1 + v2;
                double f0 = v0 ? xi[0] : 1.0 - xi[0];
                double f1 = v1 ? xi[1] : 1.0 - xi[1];
                double f2 = v2 ? xi[2] : 1.0 - xi[2];
                double d0 = v0 ? 1.0 : -1.0, d1 = v1 ? 1.0 : -1.0, d2 = v2 ? 1.0 : -1.0;
                double dphi[3] = {d0 * f1 * f2, f0 * d1 * f2, f0 * f1 * d2};
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) J[a][b] += X[v * 3 + a] * dphi[b];
            }
}

static double det3(double J[3][3])
{
    return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
         - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
         + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

/* G = J^{-1} by cofactors */
static void inverse3(double J[3][3], double det, double G[3][3])
{
    G[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    G[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    G[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    G[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    G[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    G[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    G[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    G[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    G[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
}

int orc_jacobian(const double *X, const double *xi, double *Jout)
{
    double J[3][3];
    jacobian(X, xi, J);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) Jout[3 * a + b] = J[a][b];
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Physical basis data at one quadrature point.                             */
/*                                                                          */
/* For every basis function i we form the pushed-forward quantities:        */
/*   scalar families: f[i] = (Psi_i, grad Psi_i) with grad = G^T grad^;     */
/*   NCF:  f[i] = (J Psi^ / det, div^ Psi^ / det);                          */
/*   NCE:  f[i] = (G^T Psi^, J curl^ Psi^ / det).                           */
/*   VQ:   f[i] = (Psi^, grad Psi^ G) (no Piola map: the vector element's   */
/*         values are the scalar basis times fixed unit vectors).           */
/* 4 slots for scalar / divergence data, 6 for curl data, 12 for VQ.        */
/* ------------------------------------------------------------------------ */

#define ORC_SLOTS 12

static void push_forward(const orc_element *e, const double *val, const double *grad,
                         double J[3][3], double G[3][3], double det, double *f)
{
    for (int i = 0; i < e->ndof; ++i) {
        const double *v = val + 3 * i;
        const double *g = grad + 9 * i; /* g[3*c+b] = d v_c / d xi_b */
        double *o = f + ORC_SLOTS * i;
        for (int s = 0; s < ORC_SLOTS; ++s) o[s] = 0.0;
        if (!e->vector) {
            o[0] = v[0];
            for (int a = 0; a < 3; ++a) {
                double s = 0.0;
                for (int b = 0; b < 3; ++b) s += G[b][a] * g[b]; /* (G^T grad^)_a */
                o[1 + a] = s;
            }
        } else if (e->family == ORC_VQ) {
            for (int c = 0; c < 3; ++c) {
                o[c] = v[c];
                for (int a = 0; a < 3; ++a) {
                    double s = 0.0;
                    for (int b = 0; b < 3; ++b) s += g[3 * c + b] * G[b][a]; /* d v_c / d x_a */
                    o[3 + 3 * c + a] = s;
                }
            }
        } else if (e->family == ORC_NCF) {
            for (int a = 0; a < 3; ++a) {
                double s = 0.0;
                for (int c = 0; c < 3; ++c) s += J[a][c] * v[c];
                o[a] = s / det;
            }
            o[3] = (g[0] + g[4] + g[8]) / det; /* div^ = sum_c d v_c / d xi_c */
        } else { /* NCE */
            for (int a = 0; a < 3; ++a) {
                double s = 0.0;
                for (int c = 0; c < 3; ++c) s += G[c][a] * v[c];
                o[a] = s;
            }
            /* curl^ v = (d2 v1 ... ) with (curl v)_a = eps_abc d_b v_c */
            double cr[3];
            cr[0] = g[3 * 2 + 1] - g[3 * 1 + 2];
            cr[1] = g[3 * 0 + 2] - g[3 * 2 + 0];
            cr[2] = g[3 * 1 + 0] - g[3 * 0 + 1];
            for (int a = 0; a < 3; ++a) {
                double s = 0.0;
                for (int c = 0; c < 3; ++c) s += J[a][c] * cr[c];
                o[3 + a] = s / det;
            }
        }
    }
}

/* The integrand of each form as a symmetric bilinear function of the
 * pushed-forward data of the test (ft) and trial (fs) functions. */
static double integrand(int family, int form, double alpha, double beta, const double *ft, const double *fs)
{
    if (family == ORC_Q || family == ORC_DQ || family == ORC_QGLL) {
        if (form == ORC_MASS) return ft[0] * fs[0];
        return ft[1] * fs[1] + ft[2] * fs[2] + ft[3] * fs[3]; /* LAPLACE */
    }
    if (family == ORC_VQ) {
        double m = 0.0;
        if (form == ORC_MASS)
            for (int s = 0; s < 3; ++s) m += ft[s] * fs[s]; /* u . v */
        else
            for (int s = 3; s < 12; ++s) m += ft[s] * fs[s]; /* grad u : grad v */
        return m;
    }
    double m = ft[0] * fs[0] + ft[1] * fs[1] + ft[2] * fs[2];
    if (form == ORC_MASS) return m;
    if (family == ORC_NCF) return alpha * m + beta * ft[3] * fs[3];          /* HDIV  */
    return alpha * m + beta * (ft[3] * fs[3] + ft[4] * fs[4] + ft[5] * fs[5]); /* HCURL */
}

static int form_valid(int family, int form)
{
    if (family == ORC_Q || family == ORC_DQ || family == ORC_QGLL || family == ORC_VQ)
        return form == ORC_MASS || form == ORC_LAPLACE;
    if (family == ORC_NCF) return form == ORC_MASS || form == ORC_HDIV;
    if (family == ORC_NCE) return form == ORC_MASS || form == ORC_HCURL;
    return 0;
}

typedef struct {
    orc_element e;
    int nq1, nq;
    double xq[ORC_MAXN], wq[ORC_MAXN];
    double *val, *grad; /* reference tables at every point: [nq][ndof*3], [nq][ndof*9] */
} orc_setup;

static int setup(int family, int degree, int form, int nq1, orc_setup *s)
{
    if (make_element(family, degree, &s->e)) return -1;
    if (!form_valid(family, form)) return -2;
    if (nq1 <= 0) nq1 = (family == ORC_Q || family == ORC_DQ) ? degree + 1 : degree + 1;
    if (nq1 > ORC_MAXN) return -3;
    s->nq1 = nq1;
    s->nq = nq1 * nq1 * nq1;
    if (family == ORC_QGLL) {
        if (nq1 < 2) return -3;
        orc_gauss_lobatto(nq1, s->xq, s->wq);
    } else {
        orc_gauss_legendre(nq1, s->xq, s->wq);
    }
    int nd = s->e.ndof;
    s->val = (double *)malloc(sizeof(double) * (size_t)s->nq * nd * 3);
    s->grad = (double *)malloc(sizeof(double) * (size_t)s->nq * nd * 9);
    if (!s->val || !s->grad) return -4;
    for (int q0 = 0; q0 < nq1; ++q0)
        for (int q1 = 0; q1 < nq1; ++q1)
            for (int q2 = 0; q2 < nq1; ++q2) {
                int q = (q0 * nq1 + q1) * nq1 + q2;
                double xi[3] = {s->xq[q0], s->xq[q1], s->xq[q2]};
                tabulate_point(&s->e, xi, s->val + (size_t)q * nd * 3, s->grad + (size_t)q * nd * 9);
            }
    return 0;
}

static void teardown(orc_setup *s)
{
    free(s->val);
    free(s->grad);
}

/* quadrature point q = (q0 q1 q2), q2 fastest, weight w_q0 w_q1 w_q2 (eq. tpps) */
static void point(const orc_setup *s, int q, double xi[3], double *w)
{
    int q2 = q % s->nq1, q1 = (q / s->nq1) % s->nq1, q0 = q / (s->nq1 * s->nq1);
    xi[0] = s->xq[q0];
    xi[1] = s->xq[q1];
    xi[2] = s->xq[q2];
    *w = s->wq[q0] * s->wq[q1] * s->wq[q2];
}

/*
 * Element matrices A[c][i][j] = sum_q w_q kappa_q |det J_q| F(Psi_i, Psi_j)(xi_q)
 * with F the pushed-forward integrand above (row i = test, column j = trial).
 * kappa may be NULL (kappa = 1).  Returns 0, or <0 on bad arguments, or
 * 1 + (index of the first cell with det J <= 0) when geometry degenerates
 * (that cell is still computed with |det J|).
 */
int orc_element_matrix(int family, int degree, int form, int nq1, double alpha, double beta,
                       long ncells, const double *vertices, const double *kappa, double *A)
{
    orc_setup s;
    int rc = setup(family, degree, form, nq1, &s);
    if (rc) return rc;
    const int nd = s.e.ndof, nq = s.nq;
    long bad = -1;
#pragma omp parallel
    {
        double *f = (double *)malloc(sizeof(double) * (size_t)nq * nd * ORC_SLOTS);
        double *sc = (double *)malloc(sizeof(double) * (size_t)nq);
#pragma omp for schedule(dynamic, 1)
        for (long c = 0; c < ncells; ++c) {
            const double *X = vertices + c * 24;
            for (int q = 0; q < nq; ++q) {
                double xi[3], w, J[3][3], G[3][3];
                point(&s, q, xi, &w);
                jacobian(X, xi, J);
                double det = det3(J);
                if (det <= 0.0) {
#pragma omp critical
                    if (bad < 0 || c < bad) bad = c;
                }
                inverse3(J, det, G);
                push_forward(&s.e, s.val + (size_t)q * nd * 3, s.grad + (size_t)q * nd * 9, J, G, det,
                             f + (size_t)q * nd * ORC_SLOTS);
                sc[q] = w * (kappa ? kappa[c * nq + q] : 1.0) * fabs(det);
            }
            double *Ac = A + (size_t)c * nd * nd;
            for (int i = 0; i < nd; ++i)
                for (int j = 0; j < nd; ++j) {
                    double sum = 0.0;
                    for (int q = 0; q < nq; ++q)
                        sum += sc[q] * integrand(family, form, alpha, beta, f + ((size_t)q * nd + i) * ORC_SLOTS,
                                                 f + ((size_t)q * nd + j) * ORC_SLOTS);
                    Ac[(size_t)i * nd + j] = sum;
                }
        }
        free(f);
        free(sc);
    }
    teardown(&s);
    return bad >= 0 ? (int)(1 + (bad > 2000000000L ? 2000000000L : bad)) : 0;
}

/*
 * Operator action y[c][i] = a(psi_i, u_c) (Sec. 1.1, matrix-free action):
 * the trial field and its pushed-forward derivatives are summed at every
 * quadrature point over all basis functions (eq. coeff_eval), then tested
 * against every basis function (eq. form_eval).  Same return codes.
 */
int orc_action(int family, int degree, int form, int nq1, double alpha, double beta, long ncells,
               const double *vertices, const double *kappa, const double *u, double *y)
{
    orc_setup s;
    int rc = setup(family, degree, form, nq1, &s);
    if (rc) return rc;
    const int nd = s.e.ndof, nq = s.nq;
    long bad = -1;
#pragma omp parallel
    {
        double *f = (double *)malloc(sizeof(double) * (size_t)nq * nd * ORC_SLOTS);
        double *uq = (double *)malloc(sizeof(double) * (size_t)nq * ORC_SLOTS);
        double *sc = (double *)malloc(sizeof(double) * (size_t)nq);
#pragma omp for schedule(dynamic, 16)
        for (long c = 0; c < ncells; ++c) {
            const double *X = vertices + c * 24;
            const double *uc = u + (size_t)c * nd;
            for (int q = 0; q < nq; ++q) {
                double xi[3], w, J[3][3], G[3][3];
                point(&s, q, xi, &w);
                jacobian(X, xi, J);
                double det = det3(J);
                if (det <= 0.0) {
#pragma omp critical
                    if (bad < 0 || c < bad) bad = c;
                }
                inverse3(J, det, G);
                double *fq = f + (size_t)q * nd * ORC_SLOTS;
                push_forward(&s.e, s.val + (size_t)q * nd * 3, s.grad + (size_t)q * nd * 9, J, G, det, fq);
                sc[q] = w * (kappa ? kappa[c * nq + q] : 1.0) * fabs(det);
                /* trial field at the point: sum_j u_j f_j */
                for (int t = 0; t < ORC_SLOTS; ++t) {
                    double sum = 0.0;
                    for (int j = 0; j < nd; ++j) sum += uc[j] * fq[(size_t)j * ORC_SLOTS + t];
                    uq[q * ORC_SLOTS + t] = sum;
                }
            }
            for (int i = 0; i < nd; ++i) {
                double sum = 0.0;
                for (int q = 0; q < nq; ++q)
                    sum += sc[q] * integrand(family, form, alpha, beta, f + ((size_t)q * nd + i) * ORC_SLOTS,
                                             uq + q * ORC_SLOTS);
                y[(size_t)c * nd + i] = sum;
            }
        }
        free(f);
        free(uq);
        free(sc);
    }
    teardown(&s);
    return bad >= 0 ? (int)(1 + (bad > 2000000000L ? 2000000000L : bad)) : 0;
}

/* ------------------------------------------------------------------------ */
/* Saint Venant-Kirchhoff hyperelasticity on the vector Q_p element: the    */
/* hyperelastic model of the paper's evaluation (strain energy, first       */
/* Piola-Kirchhoff stress, residual form, and the bilinear form obtained by */
/* linearising the residual, eq. bilinear_form), on the vector element of   */
/* Sec. 2.3 (scalar basis times unit vectors).                              */
/* ------------------------------------------------------------------------ */

/*
 * Vector element: the scalar basis of `family` (ORC_Q: GLL nodes, GL rule;
 * ORC_QGLL: GLL nodes and GLL rule) times the unit vectors; DOF (component c,
 * node i) has local index c * nd + i and value Psi_i e_c.
 * At a point, with grad u the physical displacement gradient (grad u)_{ca} =
 * d u_c / d x_a:
 *   F = I + grad u,  C = F^T F,  E = (C - I) / 2,
 *   W(E) = lambda/2 tr(E)^2 + mu tr(E E)     (strain energy density),
 *   S = lambda tr(E) I + 2 mu E              (dW/dE),     P = F S.
 * mode 0: out[c] = sum_q w_q |det J_q| W(E_q)                (strain energy)
 * mode 1: out[c][c'*nd + i] = sum_q w |det J| P : grad(Psi_i e_c')
 *         (the residual form with no body force; du unused)
 * mode 2: the same test functions against
 *         dP = dF S + F dS,  dF = grad du,  dE = (dF^T F + F^T dF) / 2,
 *         dS = lambda tr(dE) I + 2 mu dE
 *         (the derivative of mode 1 at u0 in the direction du: the bilinear
 *         form with trial function du and coefficient u0).
 * u0 and du: [ncells][3 nd].  Trilinear geometry per point.  Returns as
 * orc_action.
 */
static void svk_point(double lambda, double mu, const double H[3][3], const double dH[3][3], int mode,
                      double *energy, double P[3][3])
{
    double F[3][3], E[3][3], S[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) F[a][b] = (a == b ? 1.0 : 0.0) + H[a][b];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double c = 0.0;
            for (int k = 0; k < 3; ++k) c += F[k][a] * F[k][b]; /* C = F^T F */
            E[a][b] = 0.5 * (c - (a == b ? 1.0 : 0.0));
        }
    double trE = E[0][0] + E[1][1] + E[2][2];
    double EE = 0.0; /* tr(E E) */
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) EE += E[a][b] * E[b][a];
    *energy = 0.5 * lambda * trE * trE + mu * EE;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) S[a][b] = (a == b ? lambda * trE : 0.0) + 2.0 * mu * E[a][b];
    if (mode != 2) {
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double t = 0.0;
                for (int k = 0; k < 3; ++k) t += F[a][k] * S[k][b];
                P[a][b] = t;
            }
        return;
    }
    double dE[3][3], dS[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double t = 0.0;
            for (int k = 0; k < 3; ++k) t += dH[k][a] * F[k][b] + F[k][a] * dH[k][b];
            dE[a][b] = 0.5 * t;
        }
    double trdE = dE[0][0] + dE[1][1] + dE[2][2];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) dS[a][b] = (a == b ? lambda * trdE : 0.0) + 2.0 * mu * dE[a][b];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double t = 0.0;
            for (int k = 0; k < 3; ++k) t += dH[a][k] * S[k][b] + F[a][k] * dS[k][b];
            P[a][b] = t;
        }
}

/*
 * Tangent modulus of the first Piola-Kirchhoff stress at F (dP = Amod : dF,
 * dP_{ce} = sum_{c'e'} Amod[c][e][c'][e'] dF_{c'e'}), from differentiating
 * P = F S(E(F)) term by term:
 *   Amod = delta_{cc'} S_{e'e} + lambda F_{ce} F_{c'e'}
 *          + mu ((F F^T)_{cc'} delta_{ee'} + F_{ce'} F_{c'e}).
 */
static void svk_tangent(double lambda, double mu, const double H[3][3], double Amod[3][3][3][3])
{
    double F[3][3], E[3][3], S[3][3], FFt[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) F[a][b] = (a == b ? 1.0 : 0.0) + H[a][b];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double c = 0.0, d = 0.0;
            for (int k = 0; k < 3; ++k) {
                c += F[k][a] * F[k][b];
                d += F[a][k] * F[b][k];
            }
            E[a][b] = 0.5 * (c - (a == b ? 1.0 : 0.0));
            FFt[a][b] = d;
        }
    double trE = E[0][0] + E[1][1] + E[2][2];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) S[a][b] = (a == b ? lambda * trE : 0.0) + 2.0 * mu * E[a][b];
    for (int c = 0; c < 3; ++c)
        for (int e = 0; e < 3; ++e)
            for (int cc = 0; cc < 3; ++cc)
                for (int ee = 0; ee < 3; ++ee)
                    Amod[c][e][cc][ee] = (c == cc ? S[ee][e] : 0.0) + lambda * F[c][e] * F[cc][ee] +
                                         mu * (FFt[c][cc] * (e == ee ? 1.0 : 0.0) + F[c][ee] * F[cc][e]);
}

/*
 * Element matrices of the linearised residual at u0 (the bilinear form with
 * trial function du, test function v):
 *   A[c][(c',i)][(c'',j)] = sum_q w |det J| sum_{e,e'} dPsi_i/dx_e Amod[c'][e][c''][e'] dPsi_j/dx_e'
 * [ncells][3 nd][3 nd], row = test.  Returns as orc_action.
 */
int orc_svk_matrix(int family, int degree, int nq1, double lambda, double mu, long ncells,
                   const double *vertices, const double *u0, double *A)
{
    if (family != ORC_Q && family != ORC_QGLL) return -2;
    orc_setup s;
    int rc = setup(family, degree, ORC_LAPLACE, nq1, &s);
    if (rc) return rc;
    const int nd = s.e.ndof, nq = s.nq, NDV = 3 * nd;
    long bad = -1;
#pragma omp parallel
    {
        double *f = (double *)malloc(sizeof(double) * (size_t)nd * ORC_SLOTS);
#pragma omp for schedule(dynamic, 1)
        for (long c = 0; c < ncells; ++c) {
            const double *X = vertices + c * 24;
            const double *uc = u0 + (size_t)c * NDV;
            double *Ac = A + (size_t)c * NDV * NDV;
            for (size_t t = 0; t < (size_t)NDV * NDV; ++t) Ac[t] = 0.0;
            for (int q = 0; q < nq; ++q) {
                double xi[3], w, J[3][3], G[3][3];
                point(&s, q, xi, &w);
                jacobian(X, xi, J);
                double det = det3(J);
                if (det <= 0.0) {
#pragma omp critical
                    if (bad < 0 || c < bad) bad = c;
                }
                inverse3(J, det, G);
                push_forward(&s.e, s.val + (size_t)q * nd * 3, s.grad + (size_t)q * nd * 9, J, G, det, f);
                double H[3][3] = {{0}};
                for (int cc = 0; cc < 3; ++cc)
                    for (int i = 0; i < nd; ++i)
                        for (int a = 0; a < 3; ++a) H[cc][a] += uc[cc * nd + i] * f[i * ORC_SLOTS + 1 + a];
                double Amod[3][3][3][3];
                svk_tangent(lambda, mu, H, Amod);
                double sc = w * fabs(det);
                for (int c1 = 0; c1 < 3; ++c1)
                    for (int c2 = 0; c2 < 3; ++c2)
                        for (int i = 0; i < nd; ++i)
                            for (int j = 0; j < nd; ++j) {
                                double t = 0.0;
                                for (int e = 0; e < 3; ++e)
                                    for (int ee = 0; ee < 3; ++ee)
                                        t += f[i * ORC_SLOTS + 1 + e] * Amod[c1][e][c2][ee] * f[j * ORC_SLOTS + 1 + ee];
                                Ac[(size_t)(c1 * nd + i) * NDV + c2 * nd + j] += sc * t;
                            }
            }
        }
        free(f);
    }
    teardown(&s);
    return bad >= 0 ? (int)(1 + (bad > 2000000000L ? 2000000000L : bad)) : 0;
}

int orc_svk(int family, int degree, int nq1, double lambda, double mu, int mode, long ncells,
            const double *vertices, const double *u0, const double *du, double *out)
{
    if (family != ORC_Q && family != ORC_QGLL) return -2;
    if (mode < 0 || mode > 2 || (mode == 2 && !du)) return -2;
    orc_setup s;
    int rc = setup(family, degree, ORC_LAPLACE, nq1, &s);
    if (rc) return rc;
    const int nd = s.e.ndof, nq = s.nq;
    long bad = -1;
#pragma omp parallel
    {
        double *f = (double *)malloc(sizeof(double) * (size_t)nd * ORC_SLOTS);
#pragma omp for schedule(dynamic, 4)
        for (long c = 0; c < ncells; ++c) {
            const double *X = vertices + c * 24;
            const double *uc = u0 + (size_t)c * 3 * nd;
            const double *dc = du ? du + (size_t)c * 3 * nd : 0;
            double *oc = out + (mode == 0 ? (size_t)c : (size_t)c * 3 * nd);
            if (mode == 0) oc[0] = 0.0;
            else
                for (int i = 0; i < 3 * nd; ++i) oc[i] = 0.0;
            for (int q = 0; q < nq; ++q) {
                double xi[3], w, J[3][3], G[3][3];
                point(&s, q, xi, &w);
                jacobian(X, xi, J);
                double det = det3(J);
                if (det <= 0.0) {
#pragma omp critical
                    if (bad < 0 || c < bad) bad = c;
                }
                inverse3(J, det, G);
                /* physical gradients of the scalar basis: f[i*SLOTS + 1 + a] */
                push_forward(&s.e, s.val + (size_t)q * nd * 3, s.grad + (size_t)q * nd * 9, J, G, det, f);
                double H[3][3] = {{0}}, dH[3][3] = {{0}};
                for (int cc = 0; cc < 3; ++cc)
                    for (int i = 0; i < nd; ++i)
                        for (int a = 0; a < 3; ++a) {
                            H[cc][a] += uc[cc * nd + i] * f[i * ORC_SLOTS + 1 + a];
                            if (dc) dH[cc][a] += dc[cc * nd + i] * f[i * ORC_SLOTS + 1 + a];
                        }
                double energy, P[3][3];
                svk_point(lambda, mu, H, dH, mode, &energy, P);
                double sc = w * fabs(det);
                if (mode == 0) {
                    oc[0] += sc * energy;
                    continue;
                }
                /* P : grad(Psi_i e_cc) = sum_a P[cc][a] d Psi_i / d x_a */
                for (int cc = 0; cc < 3; ++cc)
                    for (int i = 0; i < nd; ++i) {
                        double t = 0.0;
                        for (int a = 0; a < 3; ++a) t += P[cc][a] * f[i * ORC_SLOTS + 1 + a];
                        oc[cc * nd + i] += sc * t;
                    }
            }
        }
        free(f);
    }
    teardown(&s);
    return bad >= 0 ? (int)(1 + (bad > 2000000000L ? 2000000000L : bad)) : 0;
}

/* ------------------------------------------------------------------------ */
/* DOF maps.                                                                */
/* ------------------------------------------------------------------------ */

typedef struct { long a, b, c; } orc_lat;

static int lat_cmp(const void *p, const void *q)
{
    const orc_lat *x = (const orc_lat *)p, *y = (const orc_lat *)q;
    if (x->a != y->a) return x->a < y->a ? -1 : 1;
    if (x->b != y->b) return x->b < y->b ? -1 : 1;
    if (x->c != y->c) return x->c < y->c ? -1 : 1;
    return 0;
}

/*
 * Global C0 Q_p numbering on an nx*ny*nz grid of cells by brute force: every
 * local node of cell (i,j,k) (cell number (i*ny+j)*nz+k) sits on the integer
 * lattice point (i*p+i0, j*p+i1, k*p+i2); the distinct lattice points are
 * sorted lexicographically and numbered in that order.  map[cell][local]
 * receives the number.  Returns the number of distinct points, <0 on error.
 */
long orc_dofmap_q(int nx, int ny, int nz, int p, int *map)
{
    if (nx < 1 || ny < 1 || nz < 1 || p < 1) return -1;
    int n = p + 1, nloc = n * n * n;
    long ncells = (long)nx * ny * nz, tot = ncells * nloc;
    orc_lat *all = (orc_lat *)malloc(sizeof(orc_lat) * (size_t)tot);
    orc_lat *uniq = (orc_lat *)malloc(sizeof(orc_lat) * (size_t)tot);
    if (!all || !uniq) { free(all); free(uniq); return -2; }
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j)
            for (int k = 0; k < nz; ++k) {
                long cell = ((long)i * ny + j) * nz + k;
                for (int i0 = 0; i0 < n; ++i0)
                    for (int i1 = 0; i1 < n; ++i1)
                        for (int i2 = 0; i2 < n; ++i2) {
                            orc_lat L = {(long)i * p + i0, (long)j * p + i1, (long)k * p + i2};
                            all[cell * nloc + (i0 * n + i1) * n + i2] = L;
                        }
            }
    memcpy(uniq, all, sizeof(orc_lat) * (size_t)tot);
    qsort(uniq, (size_t)tot, sizeof(orc_lat), lat_cmp);
    long nu = 0;
    for (long t = 0; t < tot; ++t)
        if (nu == 0 || lat_cmp(&uniq[nu - 1], &uniq[t]) != 0) uniq[nu++] = uniq[t];
    for (long t = 0; t < tot; ++t) {
        orc_lat *hit = (orc_lat *)bsearch(&all[t], uniq, (size_t)nu, sizeof(orc_lat), lat_cmp);
        map[t] = (int)(hit - uniq);
    }
    free(all);
    free(uniq);
    return nu;
}

/*
 * Concatenated numbering of an enriched element's blocks (Sec. 2.6 and the
 * indexed-buffer splitting of Sec. 3.5), any dimension: the blocks' basis
 * functions are enumerated in order, each block's multi-indices in
 * lexicographic order (last index fastest), and numbered consecutively.
 * extents[b*ndim + a]; out receives, for each block in turn, the flat number
 * of each multi-index in enumeration order (so out is simply 0..N-1 in this
 * enumeration); index_of[] gives, for a query (block, multi-index), its
 * number, by walking the enumeration until the query is met.
 */
long orc_concat_index(int ndim, int nblocks, const int *extents, int block, const int *multi)
{
    long counter = 0;
    for (int b = 0; b < nblocks; ++b) {
        int idx[16];
        for (int a = 0; a < ndim; ++a) idx[a] = 0;
        long total = 1;
        for (int a = 0; a < ndim; ++a) total *= extents[b * ndim + a];
        for (long t = 0; t < total; ++t) {
            int match = (b == block);
            for (int a = 0; a < ndim && match; ++a) match = (idx[a] == multi[a]);
            if (match) return counter;
            ++counter;
            /* advance the multi-index, last axis fastest */
            for (int a = ndim - 1; a >= 0; --a) {
                if (++idx[a] < extents[b * ndim + a]) break;
                idx[a] = 0;
            }
        }
    }
    return -1;
}

int orc_num_threads(void)
{
    int n = 1;
#ifdef _OPENMP
#pragma omp parallel
    {
#pragma omp single
        n = omp_get_num_threads();
    }
#endif
    return n;
}

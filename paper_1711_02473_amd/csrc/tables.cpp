// 1-D rules and tabulation matrices (host side, FP64).
//
// Quadrature nodes are the eigenvalues of the Jacobi matrix of the
// orthogonal-polynomial recurrence (Golub & Welsch's characterisation),
// located by Sturm-sequence bisection (Givens' method): Legendre for
// Gauss-Legendre, Jacobi(1,1) for the interior Gauss-Lobatto-Legendre nodes.
// Gauss weights are Christoffel numbers 1 / sum_k phat_k(x)^2 over the
// orthonormal Legendre polynomials; Lobatto weights are the integrals of the
// Lagrange basis, computed with an exact Gauss rule.  Lagrange values and
// derivatives use the barycentric form.  (Sec. 1.2 tabulation matrices,
// Sec. 2.5 GL / GLL node sets.)
#include <cmath>
#include <cstring>
#include <vector>

#include "sf_internal.hpp"

namespace sf {

namespace {

// number of eigenvalues of the symmetric tridiagonal matrix (zero diagonal,
// squared off-diagonal b2[1..m-1]) that are smaller than x
int sturm_count(int m, const double *b2, double x)
{
    int count = 0;
    double q = -x;
    if (q < 0) ++count;
    for (int k = 1; k < m; ++k) {
        if (q == 0.0) q = 1e-300;
        q = -x - b2[k] / q;
        if (q < 0) ++count;
    }
    return count;
}

// all eigenvalues in ascending order by bisection on [-1, 1]
void jacobi_eigs(int m, const double *b2, double *out)
{
    for (int j = 0; j < m; ++j) {
        double lo = -1.0, hi = 1.0;
        for (int it = 0; it < 200; ++it) {
            double mid = 0.5 * (lo + hi);
            if (mid <= lo || mid >= hi) break;
            if (sturm_count(m, b2, mid) > j) hi = mid;
            else lo = mid;
        }
        out[j] = 0.5 * (lo + hi);
    }
}

void gauss_legendre(int m, double *x, double *w)
{
    std::vector<double> b2(m, 0.0), t(m);
    for (int k = 1; k < m; ++k) b2[k] = double(k) * k / (4.0 * k * k - 1.0);
    jacobi_eigs(m, b2.data(), t.data());
    for (int j = 0; j < m; ++j) {
        // Christoffel number with orthonormal Legendre phat_k = sqrt(k+1/2) P_k
        double p0 = 1.0, p1 = t[j], s = 0.5;
        if (m > 1) s += 1.5 * p1 * p1;
        for (int k = 1; k + 1 < m; ++k) {
            double p2 = ((2.0 * k + 1.0) * t[j] * p1 - k * p0) / (k + 1.0);
            p0 = p1;
            p1 = p2;
            s += (k + 1.5) * p2 * p2;
        }
        x[j] = 0.5 * (1.0 + t[j]);
        w[j] = 0.5 / s; // halved: [-1,1] -> [0,1]
    }
}

void gauss_lobatto(int m, double *x, double *w)
{
    x[0] = 0.0;
    x[m - 1] = 1.0;
    int mi = m - 2;
    if (mi > 0) {
        std::vector<double> b2(mi, 0.0), t(mi);
        for (int k = 1; k < mi; ++k) b2[k] = double(k) * (k + 2.0) / ((2.0 * k + 1.0) * (2.0 * k + 3.0));
        jacobi_eigs(mi, b2.data(), t.data());
        for (int j = 0; j < mi; ++j) x[j + 1] = 0.5 * (1.0 + t[j]);
    }
    // weights = integrals of the Lagrange basis on the nodes, by an m-point
    // Gauss rule (exact for degree m-1)
    std::vector<double> gx(m), gw(m), B(size_t(m) * m), D(size_t(m) * m);
    gauss_legendre(m, gx.data(), gw.data());
    lagrange_table(m, x, m, gx.data(), B.data(), D.data());
    for (int i = 0; i < m; ++i) {
        double s = 0.0;
        for (int q = 0; q < m; ++q) s += gw[q] * B[size_t(q) * m + i];
        w[i] = s;
    }
}

} // namespace

int rule_1d(int kind, int m, double *x, double *w)
{
    if (!x || !w || m < 1 || m > kMaxRule) return SF_ERR_ARG;
    if (kind == 0) gauss_legendre(m, x, w);
    else if (kind == 1) {
        if (m < 2) return SF_ERR_ARG;
        gauss_lobatto(m, x, w);
    } else return SF_ERR_ARG;
    return SF_OK;
}

// barycentric Lagrange values and derivatives of the basis on `nodes` at `pts`
int lagrange_table(int nn, const double *nodes, int np, const double *pts, double *B, double *D)
{
    if (nn < 1 || np < 1 || !nodes || !pts || !B || !D) return SF_ERR_ARG;
    std::vector<double> lam(nn);
    for (int j = 0; j < nn; ++j) {
        double p = 1.0;
        for (int k = 0; k < nn; ++k)
            if (k != j) p *= nodes[j] - nodes[k];
        lam[j] = 1.0 / p;
    }
    for (int p = 0; p < np; ++p) {
        const double x = pts[p];
        double *b = B + size_t(p) * nn;
        double *d = D + size_t(p) * nn;
        int hit = -1;
        for (int k = 0; k < nn; ++k)
            if (std::fabs(x - nodes[k]) <= 1e-15) hit = k;
        if (hit >= 0) {
            // x is a node: l_j(x) = delta, derivative from the barycentric
            // differentiation matrix
            double diag = 0.0;
            for (int j = 0; j < nn; ++j) {
                b[j] = (j == hit) ? 1.0 : 0.0;
                if (j != hit) {
                    d[j] = (lam[j] / lam[hit]) / (nodes[hit] - nodes[j]);
                    diag += 1.0 / (nodes[hit] - nodes[j]);
                }
            }
            d[hit] = diag;
            continue;
        }
        double den = 0.0;
        for (int k = 0; k < nn; ++k) den += lam[k] / (x - nodes[k]);
        for (int j = 0; j < nn; ++j) {
            b[j] = (lam[j] / (x - nodes[j])) / den;
            double s = 0.0;
            for (int k = 0; k < nn; ++k)
                if (k != j) s += 1.0 / (x - nodes[k]);
            d[j] = b[j] * s;
        }
    }
    return SF_OK;
}

} // namespace sf

extern "C" int sf_rule_1d(int32_t kind, int32_t m, double *x, double *w) { return sf::rule_1d(kind, m, x, w); }

extern "C" int sf_lagrange_table(int32_t nnodes, const double *nodes, int32_t npts, const double *pts, double *B,
                                 double *D)
{
    return sf::lagrange_table(nnodes, nodes, npts, pts, B, D);
}

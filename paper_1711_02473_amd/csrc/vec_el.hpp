// Shared pieces of the H(div) / H(curl) kernels: block extents of the enriched
// element (Sec. 2.6-2.7) and the per-cell Piola factors.
#pragma once

#include "sf_device.hpp"

namespace sf {

namespace {

// extents of block C (0..2) along axis A for family FAM and degree K
template <int FAM, int K> struct VecEl {
    static constexpr int NQ = K + 1;
    static constexpr int NP = K + 1; // P_k factor
    static constexpr int ND = K;     // dP_{k-1} factor
    static constexpr bool pk(int c, int a) { return FAM == SF_NCF ? a == c : a != c; }
    static constexpr int ext(int c, int a) { return pk(c, a) ? NP : ND; }
    static constexpr int bsize(int c) { return ext(c, 0) * ext(c, 1) * ext(c, 2); }
    static constexpr int off(int c) { return c == 0 ? 0 : (c == 1 ? bsize(0) : bsize(0) + bsize(1)); }
    static constexpr int NF = bsize(0) + bsize(1) + bsize(2);
};

// P0, P1: extents of the two axes other than AX, in increasing axis order
template <int AX, int E0, int E1, int E2> struct Others {
    static constexpr int P0 = (AX == 0) ? E1 : E0;
    static constexpr int P1 = (AX == 2) ? E1 : E2;
};

// geometry per cell: M0 = |J| G G^T, M1 = J^T J / |J| (symmetric, 6 each), 1/|J|
__device__ inline int vec_geometry(const double *X, double M0[6], double M1[6], double &rS)
{
    double J[3][3], det;
    const int f = affine_jacobian(X, J, det);
    laplace_factor(J, det, M0);
    const double S = fabs(det);
    rS = 1.0 / S;
    int t = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int l = k; l < 3; ++l) M1[t++] = (J[0][k] * J[0][l] + J[1][k] * J[1][l] + J[2][k] * J[2][l]) * rS;
    return f;
}

// the same factors at one point of a trilinear cell (J from the eight vertices at
// reference point (x0, x1, x2)); returns det J
__device__ inline double vec_point_geometry(const double *X, double x0, double x1, double x2, double M0[6],
                                            double M1[6], double &rS)
{
    double J[3][3];
    const double det = trilinear_jacobian(X, x0, x1, x2, J);
    const double S = fabs(det);
    rS = S > 0.0 ? 1.0 / S : 0.0;
#pragma unroll
    for (int t = 0; t < 6; ++t) M0[t] = 0.0;
    if (det != 0.0) laplace_factor(J, det, M0);
    int t = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int l = k; l < 3; ++l) M1[t++] = (J[0][k] * J[0][l] + J[1][k] * J[1][l] + J[2][k] * J[2][l]) * rS;
    return det;
}

template <typename T> __device__ __forceinline__ void symmv(const T m[6], T a, T b, T c, T &x, T &y, T &z)
{
    x = m[0] * a + m[1] * b + m[2] * c;
    y = m[1] * a + m[3] * b + m[4] * c;
    z = m[2] * a + m[4] * b + m[5] * c;
}

} // namespace

} // namespace sf

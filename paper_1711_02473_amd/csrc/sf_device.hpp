// Device-side building blocks shared by the gfx950 assembly kernels.
//
// Per-cell tensors live in LDS as [a][b][c] with row strides S1, S2 (S2 odd
// so that pencils along the last axis, whose lanes step by S2, hit distinct
// banks).  A "pencil" is the line of a tensor along one axis; each thread owns
// one pencil per stage, keeps it in registers, applies a 1-D matrix to it and
// writes it back, so that every contraction is a chain of register FMAs whose
// matrix operand is wave-uniform (held in scalar registers).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/sf.h"

namespace sf {

template <int NQ> struct Lds3 {
    static constexpr int S2 = (NQ % 2) ? NQ : NQ + 1;
    static constexpr int S1 = NQ * S2;
    static constexpr int CS = NQ * S1; // one cell's tensor
};

// Read-only table pointer in the constant address space.  Every use site
// takes a fresh copy through an empty asm, so the compiler cannot merge table
// loads of different stages: each stage reloads its 1-D matrix into scalar
// registers (s_load) right before its FMAs instead of keeping every table
// live across the kernel and spilling it into vector-register lanes.
template <typename T> using cptr = const T __attribute__((address_space(4))) *;

__device__ __forceinline__ uint64_t uniform_u64(uint64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(v));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(v >> 32));
    return (uint64_t(hi) << 32) | lo;
}

template <typename T> __device__ __forceinline__ cptr<T> fresh(const T *p)
{
    uint64_t v = uniform_u64(reinterpret_cast<uint64_t>(p));
    asm volatile("" : "+s"(v));
    return (cptr<T>)v;
}

// fused multiply-add in the operands' own precision
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

__device__ __forceinline__ double to_d(double x) { return x; }
__device__ __forceinline__ double to_d(float x) { return static_cast<double>(x); }
template <typename T> __device__ __forceinline__ T conv(double x) { return static_cast<T>(x); }

// Same, but the copy cannot be taken before `dep` is computed: a data
// dependence that orders table loads after earlier arithmetic.
template <typename T, typename D> __device__ __forceinline__ cptr<T> fresh_after(const T *p, const D &dep)
{
    uint64_t v = uniform_u64(reinterpret_cast<uint64_t>(p));
    asm volatile("" : "+s"(v) : "v"(dep));
    return (cptr<T>)v;
}

// One-axis contraction of a register pencil with a row-major NO x NI matrix
// M (device pointer, wave-uniform): out[q] (=|+=) sum_i M[q*NI + i] in[i].
// Rows are processed in chunks of R; the table pointer of chunk k is taken
// after the last output of chunk k-2 exists, so at most two chunks of matrix
// rows are live in scalar registers while their loads overlap the FMAs of
// the previous chunk.
template <int NO, int NI, bool ACC, typename T>
__device__ __forceinline__ void apply_rows(const T *M, const T (&in)[NI], T (&out)[NO])
{
    constexpr int R = (NI >= 6) ? 1 : ((NI >= 4) ? 2 : 4);
#pragma unroll
    for (int q0 = 0; q0 < NO; q0 += R) {
        cptr<T> m = (q0 >= 2 * R) ? fresh_after(M, out[q0 - R - 1]) : fresh(M);
#pragma unroll
        for (int q = q0; q < q0 + R && q < NO; ++q) {
            T acc;
            int i0 = 0;
            if constexpr (ACC) {
                acc = out[q];
            } else {
                acc = m[q * NI] * in[0];
                i0 = 1;
            }
#pragma unroll
            for (int i = i0; i < NI; ++i) acc = fmadd(T(m[q * NI + i]), in[i], acc);
            out[q] = acc;
        }
    }
}

// Coefficient values at E points (offsets off + i * stride), loaded in one
// batch so that their memory latencies overlap; ones when kappa is absent or
// ok is false (padding cells, idle threads).
template <int E, typename T, typename IO>
__device__ __forceinline__ void ld_coeff(const IO *__restrict__ kappa, bool ok, int64_t off, int stride, T (&k)[E])
{
    if (kappa != nullptr && ok) {
#pragma unroll
        for (int i = 0; i < E; ++i) k[i] = T(to_d(kappa[off + int64_t(i) * stride]));
    } else {
#pragma unroll
        for (int i = 0; i < E; ++i) k[i] = T(1);
    }
}

// Even-odd application of a square N x N matrix with M[N-1-q][N-1-i] =
// s M[q][i] (s = +1, or -1 when SKEW): with x_e[i] = x[i] + x[N-1-i] and
// x_o[i] = x[i] - x[N-1-i] (i < h = N/2), rows q < h give E = sum Me x_e
// (+ M[q][h] x[h] for odd N) and O = sum Mo x_o, and y[q] = E + O,
// y[N-1-q] = E - O (SKEW: O - E); for odd N the middle row uses x_e (x_o
// when SKEW).  About (N^2 + N) / 2 + 2N operations instead of N^2.  The packed
// layout of M (host-built) is documented with pack_eo.  ACC adds into y.
template <int N, bool SKEW, bool ACC, typename T>
__device__ __forceinline__ void apply_eo(const T *M, const T (&x)[N], T (&y)[N])
{
    constexpr int h = N / 2, od = N % 2, RW = 2 * h + od;
    static_assert(h >= 1, "N >= 2");
    T xe[h], xo[h];
#pragma unroll
    for (int i = 0; i < h; ++i) {
        xe[i] = x[i] + x[N - 1 - i];
        xo[i] = x[i] - x[N - 1 - i];
    }
#pragma unroll
    for (int q = 0; q < h; ++q) {
        cptr<T> m = (q >= 2) ? fresh_after(M, y[q - 2]) : fresh(M);
        T e = T(m[q * RW]) * xe[0];
#pragma unroll
        for (int i = 1; i < h; ++i) e = fmadd(T(m[q * RW + i]), xe[i], e);
        if constexpr (od) e = fmadd(T(m[q * RW + h]), x[h], e);
        T o = T(m[q * RW + h + od]) * xo[0];
#pragma unroll
        for (int i = 1; i < h; ++i) o = fmadd(T(m[q * RW + h + od + i]), xo[i], o);
        const T lo = e + o, hi = SKEW ? o - e : e - o;
        if constexpr (ACC) {
            y[q] += lo;
            y[N - 1 - q] += hi;
        } else {
            y[q] = lo;
            y[N - 1 - q] = hi;
        }
    }
    if constexpr (od) {
        cptr<T> m = fresh_after(M, y[h - 1]);
        T a;
        if constexpr (SKEW) {
            a = T(m[h * RW]) * xo[0];
#pragma unroll
            for (int i = 1; i < h; ++i) a = fmadd(T(m[h * RW + i]), xo[i], a);
        } else {
            a = T(m[h * RW]) * xe[0];
#pragma unroll
            for (int i = 1; i < h; ++i) a = fmadd(T(m[h * RW + i]), xe[i], a);
            a = fmadd(T(m[h * RW + h]), x[h], a);
        }
        if constexpr (ACC) y[h] += a;
        else y[h] = a;
    }
}

// Even-odd application of a rectangular NO x NI matrix with M[NO-1-q][NI-1-i] =
// s M[q][i] (s = -1 when SKEW), packed as pack_eo_rect builds it: rows q < NO/2
// give E (half-sums against x_e, plus the middle column against x[NI/2] for odd
// NI) and O (half-differences against x_o), y[q] = E + O, y[NO-1-q] = s (E - O);
// the middle row of odd NO uses x_e and the middle entry (x_o when SKEW).  NI = 1
// or NO = 1 are allowed.  About NO NI / 2 + NI + NO operations instead of NO NI.
template <int NO, int NI, bool SKEW, bool ACC, typename T>
__device__ __forceinline__ void apply_eo_rect(const T *M, const T (&x)[NI], T (&y)[NO])
{
    constexpr int hi = NI / 2, oi = NI % 2, ho = NO / 2, oo = NO % 2, RW = 2 * hi + oi;
    T xe[hi > 0 ? hi : 1], xo[hi > 0 ? hi : 1];
#pragma unroll
    for (int i = 0; i < hi; ++i) {
        xe[i] = x[i] + x[NI - 1 - i];
        xo[i] = x[i] - x[NI - 1 - i];
    }
#pragma unroll
    for (int q = 0; q < ho; ++q) {
        cptr<T> m = (q >= 2) ? fresh_after(M, y[q - 2]) : fresh(M);
        T e;
        if constexpr (hi > 0) {
            e = T(m[q * RW]) * xe[0];
#pragma unroll
            for (int i = 1; i < hi; ++i) e = fmadd(T(m[q * RW + i]), xe[i], e);
            if constexpr (oi) e = fmadd(T(m[q * RW + hi]), x[hi], e);
        } else {
            e = T(m[q * RW]) * x[0];
        }
        T lo = e, up = SKEW ? -e : e;
        if constexpr (hi > 0) {
            T o = T(m[q * RW + hi + oi]) * xo[0];
#pragma unroll
            for (int i = 1; i < hi; ++i) o = fmadd(T(m[q * RW + hi + oi + i]), xo[i], o);
            lo = e + o;
            up = SKEW ? o - e : e - o;
        }
        if constexpr (ACC) {
            y[q] += lo;
            y[NO - 1 - q] += up;
        } else {
            y[q] = lo;
            y[NO - 1 - q] = up;
        }
    }
    if constexpr (oo) {
        cptr<T> m = (ho >= 1) ? fresh_after(M, y[ho - 1]) : fresh(M);
        T a = T(0);
        if constexpr (SKEW) {
            if constexpr (hi > 0) {
                a = T(m[ho * RW]) * xo[0];
#pragma unroll
                for (int i = 1; i < hi; ++i) a = fmadd(T(m[ho * RW + i]), xo[i], a);
            }
        } else {
            if constexpr (hi > 0) {
                a = T(m[ho * RW]) * xe[0];
#pragma unroll
                for (int i = 1; i < hi; ++i) a = fmadd(T(m[ho * RW + i]), xe[i], a);
                if constexpr (oi) a = fmadd(T(m[ho * RW + hi]), x[hi], a);
            } else {
                a = T(m[ho * RW]) * x[0];
            }
        }
        if constexpr (ACC) y[ho] += a;
        else y[ho] = a;
    }
}

// This thread's share (slots t = threadIdx.x + k NT < C E) of a group's
// cell-major rows of E entries, loaded in one batch so that the loads
// overlap; `fill` for padding cells, empty slots or a NULL array.
template <int C, int E, int NT, typename T, typename IO>
__device__ __forceinline__ void ld_rows(const IO *__restrict__ src, int64_t cell0, int64_t ncells, T fill,
                                        T (&v)[(C * E + NT - 1) / NT])
{
    constexpr int K = (C * E + NT - 1) / NT;
    if (src == nullptr) {
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = fill;
        return;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int t = threadIdx.x + k * NT;
        const int c = t / E;
        const bool ok = t < C * E && cell0 + c < ncells;
        const IO x = src[ok ? (cell0 + c) * E + (t - c * E) : 0];
        v[k] = ok ? T(to_d(x)) : fill;
    }
}

// out[q] = sum_i M[q][i] in[i] with M row-major NO x NI
template <int NO, int NI, typename T>
__device__ __forceinline__ void mv(const T *M, const T (&in)[NI], T (&out)[NO])
{
    apply_rows<NO, NI, false>(M, in, out);
}
// out[i] = sum_q M[q][i] in[q], given MT = M^T row-major NI x NO
template <int NO, int NI, typename T>
__device__ __forceinline__ void mtv(const T *MT, const T (&in)[NO], T (&out)[NI])
{
    apply_rows<NI, NO, false>(MT, in, out);
}
template <int NO, int NI, typename T>
__device__ __forceinline__ void mtv_acc(const T *MT, const T (&in)[NO], T (&out)[NI])
{
    apply_rows<NI, NO, true>(MT, in, out);
}

// pencil access in an LDS tensor with strides S1, S2 (axis 0, 1, 2)
template <int AX, int E, int S1, int S2, typename T>
__device__ __forceinline__ void ld_pencil(const T *base, int a, int b, T (&r)[E])
{
#pragma unroll
    for (int k = 0; k < E; ++k) {
        if constexpr (AX == 0) r[k] = base[k * S1 + a * S2 + b];
        else if constexpr (AX == 1) r[k] = base[a * S1 + k * S2 + b];
        else r[k] = base[a * S1 + b * S2 + k];
    }
}

template <int AX, int E, int S1, int S2, typename T>
__device__ __forceinline__ void st_pencil(T *base, int a, int b, const T (&r)[E])
{
#pragma unroll
    for (int k = 0; k < E; ++k) {
        if constexpr (AX == 0) base[k * S1 + a * S2 + b] = r[k];
        else if constexpr (AX == 1) base[a * S1 + k * S2 + b] = r[k];
        else base[a * S1 + b * S2 + k] = r[k];
    }
}

// Loop over the C*P0*P1 pencils of a stage: f(cell_in_group, a, b).
template <int C, int P0, int P1, int NT, typename F> __device__ __forceinline__ void pencils(F &&f)
{
    constexpr int NP = P0 * P1;
    for (int t = threadIdx.x; t < C * NP; t += NT) {
        const int c = t / NP;
        const int r = t - c * NP;
        const int a = r / P1;
        const int b = r - a * P1;
        f(c, a, b);
    }
}

// Pencils of one of several independent stages that run side by side (the
// blocks of an enriched element): threads [lo, lo + span) take this stage's
// C*P0*P1 pencils, the other threads skip it.
template <int C, int P0, int P1, typename F> __device__ __forceinline__ void pencils_part(int lo, int span, F &&f)
{
    constexpr int NP = P0 * P1;
    const int t0 = int(threadIdx.x) - lo;
    if (t0 < 0 || t0 >= span) return;
    for (int t = t0; t < C * NP; t += span) {
        const int c = t / NP;
        const int r = t - c * NP;
        const int a = r / P1;
        const int b = r - a * P1;
        f(c, a, b);
    }
}

// Jacobian of the trilinear (vector-Q1) coordinate map at reference point xi:
// x(xi) = sum_v X_v phi_v(xi), phi_v = prod_d (v_d ? xi_d : 1 - xi_d) for the
// vertex v = 4 v0 + 2 v1 + v2 (Sec. 3.1, the coordinate field evaluated at a
// quadrature point); J[a][b] = d x_a / d xi_b.  Returns det J.
__device__ inline double trilinear_jacobian(const double *__restrict__ X, double x0, double x1, double x2,
                                            double J[3][3])
{
    const double f[3][2] = {{1.0 - x0, x0}, {1.0 - x1, x1}, {1.0 - x2, x2}};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) J[a][b] = 0.0;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const int v0 = v >> 2, v1 = (v >> 1) & 1, v2 = v & 1;
        const double s0 = v0 ? 1.0 : -1.0, s1 = v1 ? 1.0 : -1.0, s2 = v2 ? 1.0 : -1.0;
        const double d0 = s0 * f[1][v1] * f[2][v2];
        const double d1 = f[0][v0] * s1 * f[2][v2];
        const double d2 = f[0][v0] * f[1][v1] * s2;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double xa = X[3 * v + a];
            J[a][0] = fma(xa, d0, J[a][0]);
            J[a][1] = fma(xa, d1, J[a][1]);
            J[a][2] = fma(xa, d2, J[a][2]);
        }
    }
    return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

// The same Jacobian along a line of reference points on which only coordinate
// AX varies (the other two fixed at xa < xb's axes order, i.e. xa on the lower
// of the two other axes): the map is linear in each reference coordinate, so
// J(t) = Ja + t Jb, column AX of Jb being zero.  One evaluation per line
// instead of one per point.
template <int AX>
__device__ inline void trilinear_line(const double *__restrict__ X, double xa, double xb, double Ja[3][3],
                                      double Jb[3][3])
{
    constexpr int D1 = AX == 0 ? 1 : 0, D2 = AX == 2 ? 1 : 2; // the fixed axes, D1 < D2
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) Ja[a][b] = Jb[a][b] = 0.0;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const int bit[3] = {v >> 2, (v >> 1) & 1, v & 1};
        const double s1 = bit[D1] ? 1.0 : -1.0, s2 = bit[D2] ? 1.0 : -1.0, sx = bit[AX] ? 1.0 : -1.0;
        const double f1 = bit[D1] ? xa : 1.0 - xa, f2 = bit[D2] ? xb : 1.0 - xb;
        const double ax0 = bit[AX] ? 0.0 : 1.0; // the AX factor is ax0 + sx t
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double xv = X[3 * v + a];
            Ja[a][AX] = fma(xv, sx * f1 * f2, Ja[a][AX]);
            Ja[a][D1] = fma(xv, s1 * f2 * ax0, Ja[a][D1]);
            Jb[a][D1] = fma(xv, s1 * f2 * sx, Jb[a][D1]);
            Ja[a][D2] = fma(xv, s2 * f1 * ax0, Ja[a][D2]);
            Jb[a][D2] = fma(xv, s2 * f1 * sx, Jb[a][D2]);
        }
    }
}

// Affine cell geometry from the 8 vertices (vector-Q1 coordinate field with
// the delta-cancelled scalar Q1 table, Sec. 3.1, evaluated for an affine map):
// J = [x(1,0,0)-x0, x(0,1,0)-x0, x(0,0,1)-x0]; the remaining vertices must be
// the affine images x0 + J v, otherwise SF_FLAG_NONAFFINE is returned.
__device__ inline int affine_jacobian(const double *__restrict__ X, double J[3][3], double &det)
{
    double x0[3], scale = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) x0[a] = X[a];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        J[a][0] = X[4 * 3 + a] - x0[a];
        J[a][1] = X[2 * 3 + a] - x0[a];
        J[a][2] = X[1 * 3 + a] - x0[a];
    }
    int flags = 0;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
#pragma unroll
        for (int a = 0; a < 3; ++a) scale = fmax(scale, fabs(X[3 * v + a]));
    }
    const double tol = 1e-11 * (scale + 1e-300);
#pragma unroll
    for (int v = 3; v < 8; ++v) {
        if (v == 4) continue;
        const double v0 = (v >> 2) & 1, v1 = (v >> 1) & 1, v2 = v & 1;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double pred = x0[a] + J[a][0] * v0 + J[a][1] * v1 + J[a][2] * v2;
            if (fabs(X[3 * v + a] - pred) > tol) flags |= SF_FLAG_NONAFFINE;
        }
    }
    det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
          J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    if (!(det > 0.0)) flags |= SF_FLAG_DETJ;
    return flags;
}

// G = J^{-1} by cofactors
__device__ inline void inverse3(const double J[3][3], double det, double G[3][3])
{
    const double r = 1.0 / det;
    G[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) * r;
    G[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * r;
    G[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * r;
    G[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) * r;
    G[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * r;
    G[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * r;
    G[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) * r;
    G[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * r;
    G[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * r;
}

// Symmetric pointwise factor of the Laplacian (argument factorisation,
// Sec. 3.2): P_kl = |det J| sum_m G_km G_lm, stored as P00 P01 P02 P11 P12 P22.
__device__ inline void laplace_factor(const double J[3][3], double det, double P[6])
{
    double G[3][3];
    inverse3(J, det, G);
    const double S = fabs(det);
    int t = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int l = k; l < 3; ++l) {
            P[t++] = S * (G[k][0] * G[l][0] + G[k][1] * G[l][1] + G[k][2] * G[l][2]);
        }
}

} // namespace sf

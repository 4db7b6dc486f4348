// Device helpers shared by the dense Kronecker mixed-precision actions
// (mixed_kron.hip, mixed_kron2.hip): operand splitting, the MFMA wrappers and the
// FP64 cell factor computed by four lanes per cell.
#pragma once

#include "mixed_body.inc"
#include "sf_device.hpp"
#include "sf_internal.hpp"

namespace sf {
namespace kron {

template <int MODE> struct KronMode {
    static constexpr int NPL = MODE == SF_BF16X3 ? 3 : 1;    // operand terms
    static constexpr int NPROD = MODE == SF_BF16X3 ? 6 : 1;  // products per tile
    static constexpr int PLANE0 = MODE == SF_FP16 ? 3 : 0;   // table plane of the single-term modes
};

// (table term, data term) of product k
__device__ __forceinline__ constexpr int prod_a(int k) { return k == 2 || k == 4 ? 1 : (k == 5 ? 2 : 0); }
__device__ __forceinline__ constexpr int prod_b(int k) { return k == 1 || k == 4 ? 1 : (k == 3 ? 2 : 0); }

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// operand terms of the pair (x0, x1), each term two 16-bit values packed in one dword
// (x0 in the low half): one rounding (BF16 / FP16), or the three-way BF16 split
// hi = bf16(x), mid = bf16(x - hi), lo = bf16(x - hi - mid), all rounded to nearest
template <int MODE> __device__ __forceinline__ void terms2(float x0, float x1, uint32_t (&t)[3])
{
    if constexpr (MODE == SF_FP16) {
        t[0] = __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{x0, x1}, f16x2));
    } else {
        const uint32_t h = __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{x0, x1}, bf16x2));
        t[0] = h;
        if constexpr (MODE == SF_BF16X3) {
            const float r0 = x0 - __builtin_bit_cast(float, h << 16);
            const float r1 = x1 - __builtin_bit_cast(float, h & 0xffff0000u);
            const uint32_t m = __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{r0, r1}, bf16x2));
            t[1] = m;
            const float q0 = r0 - __builtin_bit_cast(float, m << 16);
            const float q1 = r1 - __builtin_bit_cast(float, m & 0xffff0000u);
            t[2] = __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{q0, q1}, bf16x2));
        }
    }
}

template <int MODE> __device__ __forceinline__ f32x4 mfma32(u32x4 a, u32x4 b, f32x4 c)
{
    if constexpr (MODE == SF_FP16)
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0,
                                                      0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                       c, 0, 0, 0);
}

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

template <int MODE> __device__ __forceinline__ f32x4 mfma16(u32x2 a, u32x2 b, f32x4 c)
{
    if constexpr (MODE == SF_FP16)
        return __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(f16x4, a), __builtin_bit_cast(f16x4, b), c, 0, 0,
                                                     0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s16x4, a), __builtin_bit_cast(s16x4, b), c,
                                                         0, 0, 0);
}

// FP64 factor of cell `cl` (Sec. 3.2: |J| G G^T for the Laplacian, |J| for the mass
// form), computed by each of the four lanes col + 16 g of the cell's column: lane group
// g loads vertices 2 g and 2 g + 1 (cell_vertices), the vertices that span the Jacobian
// (0, 1, 2, 4) and the coordinate scale are exchanged by cross-lane permutes, and each
// lane checks its own vertices against the affine map (cell_factor_from).  Same
// arithmetic and flags as affine_jacobian.
__device__ __forceinline__ void cell_vertices(const double *__restrict__ vert, int64_t cl, int g, double (&xa)[3],
                                              double (&xb)[3])
{
    const double *X = vert + cl * 24 + 6 * g;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        xa[a] = X[a];
        xb[a] = X[3 + a];
    }
}

template <int FORM>
__device__ __forceinline__ void cell_factor_from(const double (&xa)[3], const double (&xb)[3], bool live, int col,
                                                 int g, int *__restrict__ err, float P[6])
{
    double sc = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) sc = fmax(sc, fmax(fabs(xa[a]), fabs(xb[a])));
    sc = fmax(sc, __shfl_xor(sc, 16));
    sc = fmax(sc, __shfl_xor(sc, 32));
    double x0[3], J[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        x0[a] = __shfl(xa[a], col);
        J[a][0] = __shfl(xa[a], col + 32) - x0[a]; // vertex 4
        J[a][1] = __shfl(xa[a], col + 16) - x0[a]; // vertex 2
        J[a][2] = __shfl(xb[a], col) - x0[a];      // vertex 1
    }
    const double tol = 1e-11 * (sc + 1e-300);
    int flags = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int v = 2 * g + h;
        const double v0 = (v >> 2) & 1, v1 = (v >> 1) & 1, v2 = v & 1;
        bool off = false;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double pred = x0[a] + J[a][0] * v0 + J[a][1] * v1 + J[a][2] * v2;
            off = off || fabs((h ? xb[a] : xa[a]) - pred) > tol;
        }
        if (v >= 3 && v != 4 && off) flags |= SF_FLAG_NONAFFINE;
    }
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                       J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    if (g == 0 && !(det > 0.0)) flags |= SF_FLAG_DETJ;
    if (flags && live) atomicOr(err, flags);
    if constexpr (FORM == SF_LAPLACE) {
        double Pd[6];
        laplace_factor(J, det, Pd);
#pragma unroll
        for (int e = 0; e < 6; ++e) P[e] = float(Pd[e]);
    } else {
        P[0] = float(fabs(det));
#pragma unroll
        for (int e = 1; e < 6; ++e) P[e] = 0.0f;
    }
}

template <int FORM>
__device__ __forceinline__ void cell_factor(const double *__restrict__ vert, int64_t cl, bool live, int col, int g,
                                            int *__restrict__ err, float P[6])
{
    double xa[3], xb[3];
    cell_vertices(vert, cl, g, xa, xb);
    cell_factor_from<FORM>(xa, xb, live, col, g, err, P);
}

} // namespace kron
} // namespace sf

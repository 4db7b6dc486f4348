// Layout of the dense Kronecker tables of the low-degree mixed-precision action
// (host-built in api.cpp, read by mixed_kron.hip).
//
// For n <= 4 points per axis a cell has nd = n^3 <= 64 DOFs and as many Gauss
// points, so the three one-axis contractions of the interpolation (and of each
// gradient component) collapse into one dense nd x nd matrix applied to the cell:
//   G0 = B (x) B (x) B,  G1 = D (x) B (x) B,  G2 = B (x) D (x) B,  G3 = B (x) B (x) D,
// row (q0, q1, q2) = (q0 n + q1) n + q2 (the Gauss point), column (i0, i1, i2) the
// DOF, the first factor acting on axis 0.  The contractions are the same finite sums
// as the sum-factorised ones (Sec. 3.3 eq. coeff_eval: the tensor-product form of the
// basis at the points); only their grouping differs.
//
// For every matrix and every plane (bf16 hi, mid, lo with v = hi + mid + lo to
// about 24 significand bits, and fp16) two fragment arrays, uint16:
//   forward  [MT][KS][64 lanes][8]: A operand of v_mfma_f32_16x16x32 for rows
//            16 m + (lane % 16) (points) and columns 32 s + 8 (lane / 16) + j (DOFs);
//   backward [NT][MT2][64 lanes][8]: A operand of v_mfma_f32_16x16x32 for the
//            transposed matrix, rows 16 t + (lane % 16) (DOFs), slot j of lane group
//            lane / 16 on point 32 m2 + 16 (j / 4) + 4 (lane / 16) + j % 4, i.e.
//            G[32 m2 + 16 (j/4) + 4 (lane/16) + j%4][16 t + lane%16].  This order of the
//            K index pairs two forward tiles: the forward results (four consecutive
//            points per lane group) of tiles 2 m2 and 2 m2 + 1 are, slot for slot, the
//            B operand of the backward product;
// entries outside nd x nd are zero.  After the 16 arrays: the 3-D weights
// w_q0 w_q1 w_q2 as MT * 16 floats (zero past nd).
#pragma once

namespace sf {

struct KronLayout {
    int n, nd, MT, MT2, KS, NT;
    constexpr KronLayout(int n_)
        : n(n_), nd(n_ * n_ * n_), MT((n_ * n_ * n_ + 15) / 16), MT2((n_ * n_ * n_ + 31) / 32),
          KS((n_ * n_ * n_ + 31) / 32), NT((n_ * n_ * n_ + 15) / 16)
    {
    }
    constexpr int fwd_elems() const { return MT * KS * 64 * 8; }
    constexpr int bwd_elems() const { return NT * MT2 * 64 * 8; }
    constexpr int plane_elems() const { return fwd_elems() + bwd_elems(); }
    // uint16 offset of (matrix, plane) forward / backward fragments
    constexpr int fwd(int mat, int plane) const { return (mat * 4 + plane) * plane_elems(); }
    constexpr int bwd(int mat, int plane) const { return fwd(mat, plane) + fwd_elems(); }
    constexpr int w3() const { return 16 * plane_elems(); } // uint16 offset, 4-byte aligned
    constexpr int total() const { return w3() + 2 * MT * 16; }
};

constexpr int kKronMaxN = 4; // the dense form is built for n <= 4 (p <= 3)

} // namespace sf

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

namespace sf {

// Layout of the split Kronecker tables of the mixed-precision action at 5 <= n <= 9
// points per axis (host-built in api.cpp, read by mixed_kron2.hip).
//
// A cell's interpolation factors as a dense n^2 x n^2 matrix on axes 1 and 2 (the
// plane index i1 n + i2, resp. q1 n + q2) and an n x n matrix on axis 0:
//   plane matrices  P0 = B (x) B,  P1 = D (x) B,  P2 = B (x) D   (first factor on axis 1)
//   axis-0 matrices M0 = B,        M1 = D
// (values and the three reference gradients: (P0, M1), (P1, M0), (P2, M0); the mass
// form (P0, M0)).  The rows of an MFMA tile are (cell slot s, i0), row rs s + i0: three
// cells at n = 5 (rs = 5), two at n = 6..8 (rs = 8), one at n = 9 (rs = 16).  Per plane of every
// matrix (bf16 hi, mid, lo, fp16), uint16:
//   s1f  [NQ][KS][64 lanes][8]  B operand of v_mfma_f32_16x16x32: slot j of lane l is
//        P[16 c + l%16][32 k + 8 (l/16) + j]   (point column c, DOF step k)
//   s1b  [NQ][NQ2][64][8]      A operand of v_mfma_f32_16x16x32 for P^T: slot j of lane
//        l is P[32 m + 16 (j/4) + 4 (l/16) + j%4][16 t + l%16]   (DOF row tile t,
//        point step m: two point tiles, in the order the products deliver them)
//   s2f  [64][4]  A operand of v_mfma_f32_16x16x16: slot j of lane l is
//        Mblk[l%16][4 (l/16) + j]
//   s2b  [64][4]  B operand of v_mfma_f32_16x16x16: slot j of lane l is
//        Mblk[4 (l/16) + j][l%16]
// with Mblk the block-diagonal 16 x 16 matrix holding M once per cell slot (zero
// outside n x n blocks); entries outside the matrices are zero.  After the tables:
// the plane weights w_q1 w_q2 (NQ * 16 floats) and the axis-0 weights per tile row
// (16 floats), zero past the points.
struct Kron2Layout {
    int n, q2, cpt, rs, NQ, KS, NQ2;
    constexpr Kron2Layout(int n_)
        : n(n_), q2(n_ * n_), cpt(n_ == 5 ? 3 : (n_ <= 8 ? 2 : 1)), rs(n_ == 5 ? 5 : (n_ <= 8 ? 8 : 16)),
          NQ((n_ * n_ + 15) / 16),
          KS((n_ * n_ + 31) / 32), NQ2(((n_ * n_ + 15) / 16 + 1) / 2)
    {
    }
    constexpr int s1f_elems() const { return NQ * KS * 512; }
    constexpr int s1b_elems() const { return NQ * NQ2 * 512; }
    constexpr int s1_plane() const { return s1f_elems() + s1b_elems(); }
    // uint16 offsets: plane matrix pm in 0..2, axis-0 matrix am in 0..1, plane pl in 0..3
    constexpr int s1f(int pm, int pl) const { return (pm * 4 + pl) * s1_plane(); }
    constexpr int s1b(int pm, int pl) const { return s1f(pm, pl) + s1f_elems(); }
    constexpr int s2f(int am, int pl) const { return 12 * s1_plane() + (am * 4 + pl) * 512; }
    constexpr int s2b(int am, int pl) const { return s2f(am, pl) + 256; }
    constexpr int w2() const { return 12 * s1_plane() + 8 * 512; } // uint16 offset, 4-byte aligned
    constexpr int w0() const { return w2() + 2 * NQ * 16; }
    constexpr int total() const { return w0() + 2 * 16; }
};

constexpr int kKron2MinN = 5, kKron2MaxN = 9;

} // namespace sf

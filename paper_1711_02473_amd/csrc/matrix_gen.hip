// Element matrices of the scalar families on general cells (affine or
// trilinear hexahedra), FP64 arithmetic, FP64 or FP32 output.
//
// Two kernels:
//
// * matrix_qgen_kernel (Q_p and the vector Q_p element, Gauss-Legendre
//   points): argument factorisation (Sec. 3.2) writes the Laplacian as the
//   nine products a,b in {0,1,2} of eq. poisson_gem, product (a,b) having
//   the derivative table D on axis a of the test function and on axis b of
//   the trial function, B elsewhere, times the per-point factor
//   W_ab(q) = w_q kappa_q |J_q| (G_q G_q^T)_ab (P^{(a,b)}; symmetric, six
//   fields).  Every product is sum-factorised with the same quadrature
//   order q2 -> q1 -> q0 (Alg. 1 on a hexahedron; Sec. 3.6 pass 5):
//     stage 1 (q2, one i2 slice at a time): the products grouped by their
//       axis-2 table pair (BB, BD, DB, DD) and weight field give eight
//       tensors T1[q0][q1][j2] ((0,1) and (1,0) share one: same pair, same
//       symmetric weight);
//     phase A (q1, one i1 at a time): the nine products summed into four
//       tensors T2[q0][j1][j2] grouped by their axis-0 table pair;
//     phase B (q0): the final contraction merged by distributivity (pass 6):
//       A = sum_q0 D[q0][i0] g_D[q0] + B[q0][i0] g_B[q0] with g_D = D[q0][j0]
//       T2_DD + B[q0][j0] T2_DB and g_B = D[q0][j0] T2_BD + B[q0][j0] T2_BB:
//       the same two sweeps as on a box, so the n^7 term keeps its box cost.
//   The mass form is the single product BB BB BB with W = w kappa |J|.
//   Flops per cell (Laplace) about 4n^7 + 20n^6 + 16n^5.
//
// * matrix_coll_kernel (the collocated variants: SF_QGLL, Gauss-Lobatto
//   points on Gauss-Lobatto nodes, and SF_DQ, Gauss points on Gauss nodes):
//   B = I (Sec. 2.5), so delta cancellation removes every B factor.  A
//   derivative of basis function i along axis a at point q is
//   Dh[q_a][i_a] times the deltas of the other two axes, which leaves
//     (a,a):  A_ij = [i_b = j_b, b != a] sum_{q_a} Dh[q_a][i_a] Dh[q_a][j_a] W_aa
//     (a,b), a != b, c the third axis:
//             A_ij = [i_c = j_c] Dh[j_a][i_a] Dh[i_b][j_b] W_ab(q_a = j_a, q_b = i_b, q_c = i_c)
//   and the mass matrix is diagonal, A_ii = w kappa |J| at point i.  The
//   nonzeros cost O(n^5) per cell (the 4(n+1)^5 guide line of the paper's
//   underintegration measurements) instead of the O(n^7) of the general
//   product; the rest of the dense output is written as zeros.
//
// Geometry: TRI = false, affine cells (one Jacobian per cell; vertices that
// are not an affine image raise SF_FLAG_NONAFFINE); TRI = true, general
// trilinear cells, J evaluated at every point from the eight vertices (the
// vector-Q1 coordinate field, Sec. 3.1).  det J <= 0 raises SF_FLAG_DETJ.
#include "sf_device.hpp"
#include "sf_internal.hpp"

namespace sf {

namespace {

// Per-point weights of C cells: W[c][k][q] for the NW fields of the form
// (Laplace: w kappa P_k with P = |J| G G^T stored P00 P01 P02 P11 P12 P22;
// mass: w kappa |J|), q = (q0 NQ + q1) NQ + q2.  sX, sWq: the 1-D points and
// weights; sGeo: C x 7 scratch for the affine per-cell factors.
template <int NQ, int FORM, bool TRI, int C, int NT, typename IO>
__device__ __forceinline__ void point_weights(const int64_t cell0, const int64_t ncells,
                                              const double *__restrict__ vert, const IO *__restrict__ kappa,
                                              const double *sX, const double *sWq, double *sGeo, double *sW,
                                              int *__restrict__ err)
{
    constexpr int NQ3 = NQ * NQ * NQ;
    constexpr int NW = FORM == SF_LAPLACE ? 6 : 1;
    if constexpr (!TRI) {
        if (threadIdx.x < C) {
            const int64_t gc = cell0 + threadIdx.x;
            double P[7] = {0, 0, 0, 0, 0, 0, 0};
            if (gc < ncells) {
                double J[3][3], det;
                const int f = affine_jacobian(vert + gc * 24, J, det);
                if (f) atomicOr(err, f);
                if (FORM == SF_LAPLACE && det != 0.0) laplace_factor(J, det, P);
                P[6] = fabs(det);
            }
#pragma unroll
            for (int k = 0; k < 7; ++k) sGeo[threadIdx.x * 7 + k] = P[k];
        }
        __syncthreads();
    }
    int flags = 0;
    for (int t = threadIdx.x; t < C * NQ3; t += NT) {
        const int c = t / NQ3, q = t - c * NQ3;
        const int q0 = q / (NQ * NQ), q1 = (q / NQ) % NQ, q2 = q % NQ;
        const int64_t gc = cell0 + c;
        double wk = 0.0, P[7] = {0, 0, 0, 0, 0, 0, 0};
        if (gc < ncells) {
            wk = sWq[q0] * sWq[q1] * sWq[q2] * (kappa ? to_d(kappa[gc * NQ3 + q]) : 1.0);
            if constexpr (TRI) {
                double J[3][3];
                const double det = trilinear_jacobian(vert + gc * 24, sX[q0], sX[q1], sX[q2], J);
                if (!(det > 0.0)) flags |= SF_FLAG_DETJ;
                if (FORM == SF_LAPLACE && det != 0.0) laplace_factor(J, det, P);
                P[6] = fabs(det);
            } else {
#pragma unroll
                for (int k = 0; k < 7; ++k) P[k] = sGeo[c * 7 + k];
            }
        }
        if constexpr (FORM == SF_LAPLACE) {
#pragma unroll
            for (int k = 0; k < 6; ++k) sW[(c * NW + k) * NQ3 + q] = wk * P[k];
        } else {
            sW[c * NQ3 + q] = wk * P[6];
        }
    }
    if (flags) atomicOr(err, flags);
}

// clears a buffer with a kernel (not a memset, so that launches can be captured)
template <typename IO> __global__ void gen_clear_kernel(IO *A, int64_t n)
{
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += int64_t(gridDim.x) * blockDim.x)
        A[t] = IO(0);
}

} // namespace

template <int N, int FORM, bool TRI, typename IO, int C, int NT, int R>
__global__ void __launch_bounds__(NT)
    matrix_qgen_kernel(const int64_t ncells, const double *__restrict__ vert, const IO *__restrict__ kappa,
                       IO *__restrict__ A, const double *__restrict__ tab, int *__restrict__ err)
{
    constexpr int N2 = N * N, N3 = N2 * N;
    constexpr bool LAP = FORM == SF_LAPLACE;
    constexpr int NW = LAP ? 6 : 1;  // weight fields
    constexpr int NT1 = LAP ? 8 : 1; // stage-1 tensors per slice
    constexpr int NT2 = LAP ? 4 : 1; // phase-A groups
    constexpr TabLayout TL(N, 0, N);
    __shared__ double sW[C * NW * N3];
    __shared__ double sT1[NT1 * C * N3]; // [k][c][q0][q1][j2] for the current i2
    __shared__ double sT2[NT2 * C * N3]; // [g][c][q0][j1][j2] for the current (i1, i2)
    __shared__ double sB[N2], sD[N2];    // B[q][j], D[q][j]
    __shared__ double sX[N], sWq[N], sGeo[C * 7];

    const int64_t cell0 = int64_t(blockIdx.x) * C;
    for (int t = threadIdx.x; t < N2; t += NT) {
        sB[t] = tab[TL.B0() + t];
        sD[t] = tab[TL.D0() + t];
    }
    if (threadIdx.x < N) {
        sX[threadIdx.x] = tab[TL.XQ() + threadIdx.x];
        sWq[threadIdx.x] = tab[TL.W() + threadIdx.x];
    }
    __syncthreads();
    point_weights<N, FORM, TRI, C, NT, IO>(cell0, ncells, vert, kappa, sX, sWq, sGeo, sW, err);
    __syncthreads();

    for (int i2 = 0; i2 < N; ++i2) {
        // ---- stage 1: T1_k[q0][q1][j2] = sum_q2 X2[q2][i2] Y2[q2][j2] W_k(q0, q1, q2)
        for (int t = threadIdx.x; t < C * N2; t += NT) {
            const int c = t / N2, q01 = t - c * N2;
            const double *w = sW + c * NW * N3 + q01 * N;
            for (int j2 = 0; j2 < N; ++j2) {
                double acc[NT1];
#pragma unroll
                for (int k = 0; k < NT1; ++k) acc[k] = 0.0;
#pragma unroll
                for (int q2 = 0; q2 < N; ++q2) {
                    const double bi = sB[q2 * N + i2], yb = sB[q2 * N + j2];
                    if constexpr (LAP) {
                        const double di = sD[q2 * N + i2], yd = sD[q2 * N + j2];
                        const double bb = bi * yb, bd = bi * yd, db = di * yb, dd = di * yd;
                        const double w00 = w[0 * N3 + q2], w01 = w[1 * N3 + q2], w02 = w[2 * N3 + q2];
                        const double w11 = w[3 * N3 + q2], w12 = w[4 * N3 + q2], w22 = w[5 * N3 + q2];
                        acc[0] = fma(bb, w00, acc[0]); // BB, W00
                        acc[1] = fma(bb, w01, acc[1]); // BB, W01
                        acc[2] = fma(bb, w11, acc[2]); // BB, W11
                        acc[3] = fma(bd, w02, acc[3]); // BD, W02
                        acc[4] = fma(bd, w12, acc[4]); // BD, W12
                        acc[5] = fma(db, w02, acc[5]); // DB, W02
                        acc[6] = fma(db, w12, acc[6]); // DB, W12
                        acc[7] = fma(dd, w22, acc[7]); // DD, W22
                    } else {
                        acc[0] = fma(bi * yb, w[q2], acc[0]);
                    }
                }
#pragma unroll
                for (int k = 0; k < NT1; ++k) sT1[(k * C + c) * N3 + q01 * N + j2] = acc[k];
            }
        }
        __syncthreads();
        for (int i1 = 0; i1 < N; ++i1) {
            // ---- phase A: contract q1, products summed by their axis-0 table pair
            for (int t = threadIdx.x; t < C * N3; t += NT) {
                const int c = t / N3, r = t - c * N3;
                const int q0 = r / N2, j12 = r - q0 * N2, j1 = j12 / N, j2 = j12 - j1 * N;
                const double *t1 = sT1 + c * N3 + q0 * N2 + j2;
                double aDD = 0.0, aDB = 0.0, aBD = 0.0, aBB = 0.0;
#pragma unroll
                for (int q1 = 0; q1 < N; ++q1) {
                    const double bI = sB[q1 * N + i1], yB = sB[q1 * N + j1];
                    const double *tq = t1 + q1 * N;
                    if constexpr (LAP) {
                        const double dI = sD[q1 * N + i1], yD = sD[q1 * N + j1];
                        constexpr int S = C * N3; // stride between the stage-1 tensors
                        const double bb00 = tq[0], bb01 = tq[S], bb11 = tq[2 * S], bd02 = tq[3 * S];
                        const double bd12 = tq[4 * S], db02 = tq[5 * S], db12 = tq[6 * S], dd22 = tq[7 * S];
                        const double BB = bI * yB, BDt = bI * yD, DBt = dI * yB, DDt = dI * yD;
                        aDD = fma(BB, bb00, aDD);                                     // (0,0)
                        aDB = fma(BDt, bb01, fma(BB, bd02, aDB));                     // (0,1) (0,2)
                        aBD = fma(DBt, bb01, fma(BB, db02, aBD));                     // (1,0) (2,0)
                        aBB = fma(DDt, bb11, fma(DBt, bd12, fma(BDt, db12, fma(BB, dd22, aBB)))); // (1,1) (1,2) (2,1) (2,2)
                    } else {
                        aBB = fma(bI * yB, tq[0], aBB);
                    }
                }
                if constexpr (LAP) {
                    sT2[(0 * C + c) * N3 + r] = aDD;
                    sT2[(1 * C + c) * N3 + r] = aDB;
                    sT2[(2 * C + c) * N3 + r] = aBD;
                    sT2[(3 * C + c) * N3 + r] = aBB;
                } else {
                    sT2[c * N3 + r] = aBB;
                }
            }
            __syncthreads();
            // ---- phase B: contract q0 (merged by distributivity), write n rows of n^3 entries
            for (int t = threadIdx.x; t < C * N3; t += NT) {
                const int c = t / N3, j = t - c * N3;
                const int j0 = j / N2, j12 = j - j0 * N2;
                const int64_t gc = cell0 + c;
                double gD[N], gB[N], out[N];
#pragma unroll
                for (int q0 = 0; q0 < N; ++q0) {
                    const double *t2 = sT2 + c * N3 + q0 * N2 + j12;
                    const double yB = sB[q0 * N + j0];
                    if constexpr (LAP) {
                        constexpr int S = C * N3;
                        const double yD = sD[q0 * N + j0];
                        gD[q0] = fma(yD, t2[0], yB * t2[S]);
                        gB[q0] = fma(yD, t2[2 * S], yB * t2[3 * S]);
                    } else {
                        gB[q0] = yB * t2[0];
                    }
                }
#pragma unroll
                for (int i0 = 0; i0 < N; ++i0) {
                    double s = 0.0;
#pragma unroll
                    for (int q0 = 0; q0 < N; ++q0) {
                        if constexpr (LAP) s = fma(sD[q0 * N + i0], gD[q0], s);
                        s = fma(sB[q0 * N + i0], gB[q0], s);
                    }
                    out[i0] = s;
                }
                if (gc < ncells) {
                    constexpr int64_t ND = int64_t(R) * N3;
#pragma unroll
                    for (int rb = 0; rb < R; ++rb) {
                        IO *row = A + gc * ND * ND + int64_t(rb * N3 + i1 * N + i2) * ND + rb * N3 + j;
#pragma unroll
                        for (int i0 = 0; i0 < N; ++i0) row[int64_t(i0) * N2 * ND] = IO(out[i0]);
                    }
                }
            }
            __syncthreads(); // the next phase A overwrites T2 (and, after the last i1, stage 1 T1)
        }
    }
}

template <int N, int FORM, bool TRI, typename IO, int C, int NT>
__global__ void __launch_bounds__(NT)
    matrix_coll_kernel(const int64_t ncells, const double *__restrict__ vert, const IO *__restrict__ kappa,
                       IO *__restrict__ A, const double *__restrict__ tab, int *__restrict__ err)
{
    constexpr int N2 = N * N, N3 = N2 * N;
    constexpr bool LAP = FORM == SF_LAPLACE;
    constexpr int NW = LAP ? 6 : 1;
    constexpr TabLayout TL(N, 0, N);
    __shared__ double sW[C * NW * N3];
    __shared__ double sDh[N2]; // Dh[q][i] = l_i'(x_q) on the collocated points
    __shared__ double sX[N], sWq[N], sGeo[C * 7];

    const int64_t cell0 = int64_t(blockIdx.x) * C;
    for (int t = threadIdx.x; t < N2; t += NT) sDh[t] = tab[TL.Dh() + t];
    if (threadIdx.x < N) {
        sX[threadIdx.x] = tab[TL.XQ() + threadIdx.x];
        sWq[threadIdx.x] = tab[TL.W() + threadIdx.x];
    }
    __syncthreads();
    point_weights<N, FORM, TRI, C, NT, IO>(cell0, ncells, vert, kappa, sX, sWq, sGeo, sW, err);
    __syncthreads();

    // one column j per thread, rows in order: for each row the lanes store consecutive columns
    for (int t = threadIdx.x; t < C * N3; t += NT) {
        const int c = t / N3, j = t - c * N3;
        const int64_t gc = cell0 + c;
        if (gc >= ncells) continue;
        const int j0 = j / N2, j1 = (j / N) % N, j2 = j % N;
        const double *W = sW + c * NW * N3;
        IO *col = A + gc * int64_t(N3) * N3 + j;
        int i = 0;
        for (int i0 = 0; i0 < N; ++i0)
            for (int i1 = 0; i1 < N; ++i1)
                for (int i2 = 0; i2 < N; ++i2, ++i) {
                    double v = 0.0;
                    if constexpr (LAP) {
                        const bool e0 = i0 == j0, e1 = i1 == j1, e2 = i2 == j2;
                        const double *W00 = W, *W01 = W + N3, *W02 = W + 2 * N3;
                        const double *W11 = W + 3 * N3, *W12 = W + 4 * N3, *W22 = W + 5 * N3;
                        if (e1 && e2)
                            for (int q = 0; q < N; ++q)
                                v = fma(sDh[q * N + i0] * sDh[q * N + j0], W00[(q * N + i1) * N + i2], v);
                        if (e0 && e2)
                            for (int q = 0; q < N; ++q)
                                v = fma(sDh[q * N + i1] * sDh[q * N + j1], W11[(i0 * N + q) * N + i2], v);
                        if (e0 && e1)
                            for (int q = 0; q < N; ++q)
                                v = fma(sDh[q * N + i2] * sDh[q * N + j2], W22[(i0 * N + i1) * N + q], v);
                        if (e2) // (0,1) at q = (j0, i1, i2), (1,0) at q = (i0, j1, i2)
                            v += sDh[j0 * N + i0] * sDh[i1 * N + j1] * W01[(j0 * N + i1) * N + i2] +
                                 sDh[j1 * N + i1] * sDh[i0 * N + j0] * W01[(i0 * N + j1) * N + i2];
                        if (e1) // (0,2) at q = (j0, i1, i2), (2,0) at q = (i0, i1, j2)
                            v += sDh[j0 * N + i0] * sDh[i2 * N + j2] * W02[(j0 * N + i1) * N + i2] +
                                 sDh[j2 * N + i2] * sDh[i0 * N + j0] * W02[(i0 * N + i1) * N + j2];
                        if (e0) // (1,2) at q = (i0, j1, i2), (2,1) at q = (i0, i1, j2)
                            v += sDh[j1 * N + i1] * sDh[i2 * N + j2] * W12[(i0 * N + j1) * N + i2] +
                                 sDh[j2 * N + i2] * sDh[i1 * N + j1] * W12[(i0 * N + i1) * N + j2];
                    } else {
                        if (i == j) v = W[j];
                    }
                    col[int64_t(i) * N3] = IO(v);
                }
    }
}

namespace {

template <int N, int FORM, bool TRI, typename IO, int R>
int launch_qgen_one(const LaunchArgs &a)
{
    constexpr int N3 = N * N * N;
    constexpr int NT = 256;
    constexpr int C = (NT / N3) > 0 ? NT / N3 : 1;
    const int64_t groups = (a.ncells + C - 1) / C;
    if (groups > 0x7fffffffLL) return SF_ERR_CAPACITY;
    if (R > 1) {
        const int64_t n = a.ncells * int64_t(R * N3) * (R * N3);
        const int64_t blocks = (n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192;
        hipLaunchKernelGGL(gen_clear_kernel<IO>, dim3(unsigned(blocks)), dim3(256), 0, a.stream,
                           static_cast<IO *>(a.A), n);
    }
    hipLaunchKernelGGL((matrix_qgen_kernel<N, FORM, TRI, IO, C, NT, R>), dim3(unsigned(groups)), dim3(NT), 0,
                       a.stream, a.ncells, a.vert, static_cast<const IO *>(a.kappa), static_cast<IO *>(a.A), a.tab64,
                       a.err);
    return hipGetLastError() == hipSuccess ? SF_OK : SF_ERR_HIP;
}

template <int N, int FORM, bool TRI, typename IO>
int launch_coll_one(const LaunchArgs &a)
{
    constexpr int N3 = N * N * N;
    constexpr int NT = 256;
    constexpr int C = (NT / N3) > 0 ? NT / N3 : 1;
    const int64_t groups = (a.ncells + C - 1) / C;
    if (groups > 0x7fffffffLL) return SF_ERR_CAPACITY;
    hipLaunchKernelGGL((matrix_coll_kernel<N, FORM, TRI, IO, C, NT>), dim3(unsigned(groups)), dim3(NT), 0, a.stream,
                       a.ncells, a.vert, static_cast<const IO *>(a.kappa), static_cast<IO *>(a.A), a.tab64, a.err);
    return hipGetLastError() == hipSuccess ? SF_OK : SF_ERR_HIP;
}

template <int N, bool COLL, bool TRI, typename IO>
int gen_form(const LaunchArgs &a)
{
    if constexpr (COLL) {
        if (a.form == SF_MASS) return launch_coll_one<N, SF_MASS, TRI, IO>(a);
        if (a.form == SF_LAPLACE) return launch_coll_one<N, SF_LAPLACE, TRI, IO>(a);
    } else {
        const bool vec = a.family == SF_VQ;
        if (a.form == SF_MASS)
            return vec ? launch_qgen_one<N, SF_MASS, TRI, IO, 3>(a) : launch_qgen_one<N, SF_MASS, TRI, IO, 1>(a);
        if (a.form == SF_LAPLACE)
            return vec ? launch_qgen_one<N, SF_LAPLACE, TRI, IO, 3>(a) : launch_qgen_one<N, SF_LAPLACE, TRI, IO, 1>(a);
    }
    return SF_ERR_UNSUPPORTED;
}

template <int N, bool COLL>
int gen_n(const LaunchArgs &a)
{
    if (a.precision != SF_FP64) return SF_ERR_UNSUPPORTED;
    if (a.trilinear)
        return a.io == SF_F64 ? gen_form<N, COLL, true, double>(a) : gen_form<N, COLL, true, float>(a);
    return a.io == SF_F64 ? gen_form<N, COLL, false, double>(a) : gen_form<N, COLL, false, float>(a);
}

template <bool COLL>
int gen_dispatch(const LaunchArgs &a)
{
    if (a.nq != a.degree + 1) return SF_ERR_UNSUPPORTED;
    switch (a.degree + 1) {
    case 2: return gen_n<2, COLL>(a);
    case 3: return gen_n<3, COLL>(a);
    case 4: return gen_n<4, COLL>(a);
    case 5: return gen_n<5, COLL>(a);
    case 6: return gen_n<6, COLL>(a);
    case 7: return gen_n<7, COLL>(a);
    case 8: return gen_n<8, COLL>(a);
    case 9: return gen_n<9, COLL>(a);
    default: return SF_ERR_UNSUPPORTED;
    }
}

} // namespace

int launch_matrix_qgen(const LaunchArgs &a)
{
    if (a.family != SF_Q && a.family != SF_VQ) return SF_ERR_UNSUPPORTED;
    return gen_dispatch<false>(a);
}

int launch_matrix_coll(const LaunchArgs &a)
{
    if (a.family != SF_QGLL && a.family != SF_DQ) return SF_ERR_UNSUPPORTED;
    return gen_dispatch<true>(a);
}

} // namespace sf

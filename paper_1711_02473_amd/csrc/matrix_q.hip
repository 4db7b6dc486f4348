// Element matrices for the scalar families (Q_p, dQ_p), mass and Laplace
// forms, on axis-aligned box cells, FP64 arithmetic, FP64 or FP32 output.
//
// Method (Sec. 3.2): after argument factorisation the Laplacian on a box is a
// sum of three products, product a having the derivative table D on axis a
// and the value table B on the other axes, times the per-cell factor
// |J| / h_a^2 (the diagonal of |J| G G^T).  Each product is sum-factorised
// (eq. opt1_product / opt2_product, Alg. 1: for a hexahedron every order of
// the three quadrature indices costs 2n^5 + 2n^6 + 2n^7), with the same order
// q2 -> q1 -> q0 for all products (Sec. 3.6, pass 5) so that the last stage
// can be merged by distributivity (pass 6): products 1 and 2 share the value
// table on axis 0, so the final contraction runs two GEMM-like sweeps
// (D and B on axis 0) instead of three.  The 1-D weight w_q of each axis is
// folded into that axis' stage.
//
// Stage 1 (per cell): T1_s[q0][q1][i2][j2] = sum_q2 w X_s[q2][i2] X_s[q2][j2] kappa[q0][q1][q2]
//   with s = BB (and DD for the Laplacian), kept in LDS.
// Then for every output row block (i1, i2):
//   phase A: T2_r[q0][j1][j2] = sum_q1 (factor) w X[q1][i1] Y[q1][j1] T1_s[q0][q1][i2][j2]
//   phase B: A[(i0,i1,i2), (j0,j1,j2)] = sum_r sum_q0 w X_r[q0][i0] Y_r[q0][j0] T2_r[q0][j1][j2]
// Phase B's lanes run over consecutive columns j, so each of the n rows of the
// block is written as one contiguous n^3-long run (coalesced).
#include "sf_device.hpp"
#include "sf_internal.hpp"

namespace sf {

template <int N, int NQ, int FORM, typename IO, int C, int NT>
__global__ void __launch_bounds__(NT) matrix_q_kernel(const int64_t ncells, const double *__restrict__ vert,
                                                      const IO *__restrict__ kappa, IO *__restrict__ A,
                                                      const double *__restrict__ tab, int *__restrict__ err)
{
    constexpr TabLayout TL(N, 0, NQ);
    constexpr int N2 = N * N, N3 = N2 * N, NQ2 = NQ * NQ, NQ3 = NQ2 * NQ;
    constexpr int NS = (FORM == SF_LAPLACE) ? 2 : 1; // stage-1 types: BB, DD
    constexpr int NR = NS;                            // final-stage types: r=0 (D on axis 0 / mass: B), r=1 (B)
    constexpr int T1SZ = NQ2 * N2;
    constexpr int T2SZ = NQ * N2;
    const double *const BT = tab + TL.B0T(); // B^T [n][nq]: row i = column i of B
    const double *const DT = tab + TL.D0T();

    __shared__ double sT1[NS * C * T1SZ];
    __shared__ double sT2[2 * NR * C * T2SZ];
    __shared__ double sBw[NQ * N], sDw[NQ * N], sW[NQ]; // w_q B[q][j], w_q D[q][j]
    __shared__ double sCoef[C][3];

    const int64_t cell0 = int64_t(blockIdx.x) * C;
    const bool has_kappa = kappa != nullptr;

    for (int t = threadIdx.x; t < NQ * N; t += NT) { // lane-varying reads: plain vector loads
        const double w = tab[TL.W() + t / N];
        sBw[t] = w * tab[TL.B0() + t];
        sDw[t] = w * tab[TL.D0() + t];
    }
    if (threadIdx.x < NQ) sW[threadIdx.x] = tab[TL.W() + threadIdx.x];
    if (threadIdx.x < C) {
        const int64_t gc = cell0 + threadIdx.x;
        double cf[3] = {0, 0, 0};
        if (gc < ncells) {
            double J[3][3], det;
            int f = affine_jacobian(vert + gc * 24, J, det);
            const double off = fabs(J[0][1]) + fabs(J[0][2]) + fabs(J[1][0]) + fabs(J[1][2]) + fabs(J[2][0]) + fabs(J[2][1]);
            const double dia = fabs(J[0][0]) + fabs(J[1][1]) + fabs(J[2][2]);
            if (off > 1e-12 * dia) f |= SF_FLAG_NONBOX;
            if (f) atomicOr(err, f);
            const double S = fabs(det);
            if (FORM == SF_LAPLACE) {
                cf[0] = S / (J[0][0] * J[0][0]);
                cf[1] = S / (J[1][1] * J[1][1]);
                cf[2] = S / (J[2][2] * J[2][2]);
            } else {
                cf[0] = S;
            }
        }
        sCoef[threadIdx.x][0] = cf[0];
        sCoef[threadIdx.x][1] = cf[1];
        sCoef[threadIdx.x][2] = cf[2];
    }
    __syncthreads();

    // ---- stage 1: contract q2 (innermost quadrature index)
    for (int t = threadIdx.x; t < C * NQ2; t += NT) {
        const int c = t / NQ2, q01 = t - c * NQ2;
        const int64_t gc = cell0 + c;
        double kw[NQ];
#pragma unroll
        for (int q2 = 0; q2 < NQ; ++q2)
            kw[q2] = sW[q2] * ((has_kappa && gc < ncells) ? to_d(kappa[gc * NQ3 + q01 * NQ + q2]) : 1.0);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const double *XT = s == 0 ? BT : DT;
            double *dst = sT1 + (s * C + c) * T1SZ + q01 * N2;
#pragma unroll
            for (int j2 = 0; j2 < N; ++j2) {
                double tmp[NQ], col[N];
                cptr<double> xr = fresh(XT + j2 * NQ);
#pragma unroll
                for (int q2 = 0; q2 < NQ; ++q2) tmp[q2] = xr[q2] * kw[q2];
                mv<N, NQ>(XT, tmp, col); // col[i2] = sum_q2 X[q2][i2] tmp[q2]
#pragma unroll
                for (int i2 = 0; i2 < N; ++i2) dst[i2 * N + j2] = col[i2];
            }
        }
    }
    __syncthreads();

    for (int i1 = 0; i1 < N; ++i1) {
        for (int i2 = 0; i2 < N; ++i2) {
            const int buf = (i1 * N + i2) & 1;
            double *T2 = sT2 + buf * NR * C * T2SZ;
            // ---- phase A: contract q1 for this (i1, i2)
            {
                cptr<double> bi = fresh(BT + i1 * NQ); // B[q1][i1]
                cptr<double> di = fresh(DT + i1 * NQ); // D[q1][i1]
                for (int t = threadIdx.x; t < C * NQ * N2; t += NT) {
                    const int c = t / (NQ * N2);
                    const int r = t - c * (NQ * N2);
                    const int q0 = r / N2;
                    const int j12 = r - q0 * N2;
                    const int j1 = j12 / N, j2 = j12 - j1 * N;
                    const double *t1 = sT1 + c * T1SZ + (q0 * NQ) * N2 + i2 * N + j2;
                    if constexpr (FORM == SF_LAPLACE) {
                        const double *t1d = t1 + C * T1SZ;
                        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
                        for (int q1 = 0; q1 < NQ; ++q1) {
                            const double tb = t1[q1 * N2], td = t1d[q1 * N2];
                            const double yb = sBw[q1 * N + j1], yd = sDw[q1 * N + j1];
                            a0 = __builtin_fma(bi[q1], yb * tb, a0);
                            a1 = __builtin_fma(di[q1], yd * tb, a1);
                            a2 = __builtin_fma(bi[q1], yb * td, a2);
                        }
                        T2[(0 * C + c) * T2SZ + r] = sCoef[c][0] * a0;
                        T2[(1 * C + c) * T2SZ + r] = sCoef[c][1] * a1 + sCoef[c][2] * a2;
                    } else {
                        double a0 = 0.0;
#pragma unroll
                        for (int q1 = 0; q1 < NQ; ++q1) a0 = __builtin_fma(bi[q1], sBw[q1 * N + j1] * t1[q1 * N2], a0);
                        T2[c * T2SZ + r] = sCoef[c][0] * a0;
                    }
                }
            }
            __syncthreads();
            // ---- phase B: contract q0, write n rows of n^3 entries
            for (int t = threadIdx.x; t < C * N3; t += NT) {
                const int c = t / N3;
                const int j = t - c * N3;
                const int64_t gc = cell0 + c;
                const int j0 = j / N2, j12 = j - j0 * N2;
                double g0[NQ], g1[NQ], out[N];
#pragma unroll
                for (int q0 = 0; q0 < NQ; ++q0) {
                    const double *t2 = T2 + c * T2SZ + q0 * N2 + j12;
                    if constexpr (FORM == SF_LAPLACE) {
                        g0[q0] = sDw[q0 * N + j0] * t2[0];
                        g1[q0] = sBw[q0 * N + j0] * t2[C * T2SZ];
                    } else {
                        g0[q0] = sBw[q0 * N + j0] * t2[0];
                    }
                }
                if constexpr (FORM == SF_LAPLACE) {
                    mv<N, NQ>(DT, g0, out); // out[i0] = sum_q0 D[q0][i0] g0[q0]
                    apply_rows<N, NQ, true>(BT, g1, out);
                } else {
                    mv<N, NQ>(BT, g0, out);
                }
                if (gc < ncells) { // computed above in uniform control flow, stored only for real cells
                    IO *row = A + gc * int64_t(N3) * N3 + int64_t(i1 * N + i2) * N3 + j;
#pragma unroll
                    for (int i0 = 0; i0 < N; ++i0) row[int64_t(i0) * N2 * N3] = IO(out[i0]);
                }
            }
        }
    }
}

namespace {

template <int N, int FORM, typename IO>
int launch_one(const LaunchArgs &a)
{
    constexpr int N3 = N * N * N;
    constexpr int C = (256 / N3) > 0 ? 256 / N3 : 1;
    constexpr int NT0 = ((C * N3 + 63) / 64) * 64;
    constexpr int NT = NT0 > 1024 ? 1024 : NT0;
    const int64_t groups = (a.ncells + C - 1) / C;
    if (groups > 0x7fffffffLL) return SF_ERR_CAPACITY;
    hipLaunchKernelGGL((matrix_q_kernel<N, N, FORM, IO, C, NT>), dim3(unsigned(groups)), dim3(NT), 0, a.stream,
                       a.ncells, a.vert, static_cast<const IO *>(a.kappa), static_cast<IO *>(a.A), a.tab64, a.err);
    return hipGetLastError() == hipSuccess ? SF_OK : SF_ERR_HIP;
}

template <int N>
int launch_n(const LaunchArgs &a)
{
    if (a.precision != SF_FP64) return SF_ERR_UNSUPPORTED;
    if (a.form == SF_MASS) return a.io == SF_F64 ? launch_one<N, SF_MASS, double>(a) : launch_one<N, SF_MASS, float>(a);
    if (a.form == SF_LAPLACE)
        return a.io == SF_F64 ? launch_one<N, SF_LAPLACE, double>(a) : launch_one<N, SF_LAPLACE, float>(a);
    return SF_ERR_UNSUPPORTED;
}

} // namespace

int launch_matrix_q(const LaunchArgs &a)
{
    if (a.nq != a.degree + 1) return SF_ERR_UNSUPPORTED;
    switch (a.degree + 1) {
    case 2: return launch_n<2>(a);
    case 3: return launch_n<3>(a);
    case 4: return launch_n<4>(a);
    case 5: return launch_n<5>(a);
    case 6: return launch_n<6>(a);
    case 7: return launch_n<7>(a);
    case 8: return launch_n<8>(a);
    case 9: return launch_n<9>(a);
    default: return SF_ERR_UNSUPPORTED;
    }
}

} // namespace sf

// Operator action for the scalar families (Q_p on GLL nodes, dQ_p on GL
// nodes), mass and Laplace forms, FP64 or FP32 contractions, on gfx950.
//
// Method (Sec. 3.3, eq. coeff_eval / eq. form_eval, with the tensor-product
// structure of Sec. 1.2): the trial coefficients u^K are interpolated to the
// tensor Gauss points one axis at a time with the 1-D matrix B (skipped for
// dQ_p with p+1 Gauss points: the table is the identity, Sec. 2.5,
// eq. colocated); the reference gradient at the points is then obtained with
// the collocation derivative matrix Dh of the Gauss-point Lagrange basis,
// one axis at a time; the symmetric pointwise factor w_q kappa_q |J| G G^T
// (argument factorisation, Sec. 3.2) is applied; and the transposed matrices
// Dh^T and B^T bring the result back to the local DOFs.  Interpolating first
// and differentiating in the collocated basis needs 12 one-axis contractions
// per cell (6 B, 6 Dh) instead of the 16 of the direct B/D factorisation;
// both are exact reorderings of the same finite sum.
//
// Mapping: one workgroup owns C consecutive cells; each stage assigns one
// pencil (a line of a per-cell tensor along one axis) to a thread, which
// holds it in registers; tensors live in LDS between stages.  Stages that
// touch HBM use x-axis pencils, whose lanes step through consecutive
// addresses, so u, kappa and y move with coalesced loads and stores.
#include "sf_device.hpp"
#include "sf_internal.hpp"

namespace sf {

template <int N, int NQ, int FORM, bool COLL, typename T, typename IO, int C, int NT>
__global__ void __launch_bounds__(NT) action_q_kernel(const int64_t ncells, const double *__restrict__ vert,
                                                      const IO *__restrict__ kappa, const IO *__restrict__ u,
                                                      IO *__restrict__ y, const T *__restrict__ tab,
                                                      int *__restrict__ err)
{
    using L = Lds3<NQ>;
    constexpr int S1 = L::S1, S2 = L::S2, CS = L::CS;
    constexpr int NBUF = (FORM == SF_LAPLACE) ? 3 : 2;
    constexpr TabLayout TL(N, 0, NQ);
    constexpr int N3 = N * N * N, NQ3 = NQ * NQ * NQ;
    const T *const Bt = tab + TL.B0();   // B [nq][n]
    const T *const BtT = tab + TL.B0T(); // B^T [n][nq]
    const T *const Dh = tab + TL.Dh();
    const T *const DhT = tab + TL.DhT();
    const T *const tW = tab + TL.W();
#define W fresh(tW)

    constexpr bool NEED_LDS = !(COLL && FORM == SF_MASS);
    __shared__ T lds[NEED_LDS ? NBUF * C * CS : 1];
    __shared__ double sP[C][6];

    const int64_t cell0 = int64_t(blockIdx.x) * C;
    const bool has_kappa = kappa != nullptr;

    // ---- geometry: FP64 Jacobian, inverse, determinant, pointwise factor
    if (threadIdx.x < C) {
        const int64_t gc = cell0 + threadIdx.x;
        double P[6] = {0, 0, 0, 0, 0, 0};
        if (gc < ncells) {
            double J[3][3], det;
            const int f = affine_jacobian(vert + gc * 24, J, det);
            if (f) atomicOr(err, f);
            if (FORM == SF_LAPLACE) laplace_factor(J, det, P);
            else P[0] = fabs(det);
        }
#pragma unroll
        for (int t = 0; t < 6; ++t) sP[threadIdx.x][t] = P[t];
    }
    __syncthreads();

    if constexpr (COLL && FORM == SF_MASS) {
        // collocated mass: the operator is diagonal, y = w kappa |J| u
        pencils<C, N, N, NT>([&](int c, int i2, int i3) {
            const int64_t gc = cell0 + c;
            if (gc >= ncells) return;
            const double S = sP[c][0];
            const T w23 = W[i2] * W[i3];
#pragma unroll
            for (int i1 = 0; i1 < N; ++i1) {
                const int64_t o = gc * N3 + (i1 * N + i2) * N + i3;
                T om = T(S) * W[i1] * w23;
                if (has_kappa) om *= T(to_d(kappa[o]));
                y[o] = IO(om * T(to_d(u[o])));
            }
        });
        return;
    } else {
        T *L0 = lds;
        T *L1 = lds + C * CS;
        T *L2 = lds + 2 * C * CS;

        // ---- stage 1 (x): u -> B_x u; kappa staged for the mass form
        pencils<C, N, N, NT>([&](int c, int i2, int i3) {
            const int64_t gc = cell0 + c;
            T in[N];
#pragma unroll
            for (int i1 = 0; i1 < N; ++i1) in[i1] = gc < ncells ? T(to_d(u[gc * N3 + (i1 * N + i2) * N + i3])) : T(0);
            if constexpr (COLL) {
                st_pencil<0, N, S1, S2>(L0 + c * CS, i2, i3, in);
            } else {
                T out[NQ];
                mv<NQ, N>(Bt, in, out);
                st_pencil<0, NQ, S1, S2>(L0 + c * CS, i2, i3, out);
            }
        });
        if constexpr (FORM == SF_MASS) {
            pencils<C, NQ, NQ, NT>([&](int c, int q2, int q3) {
                const int64_t gc = cell0 + c;
                T k[NQ];
#pragma unroll
                for (int q1 = 0; q1 < NQ; ++q1)
                    k[q1] = (has_kappa && gc < ncells) ? T(to_d(kappa[gc * NQ3 + (q1 * NQ + q2) * NQ + q3])) : T(1);
                st_pencil<0, NQ, S1, S2>(L1 + c * CS, q2, q3, k);
            });
        }
        __syncthreads();

        // ---- stage 2 (y): B_y
        if constexpr (!COLL) {
            pencils<C, NQ, N, NT>([&](int c, int q1, int i3) {
                T in[N], out[NQ];
                ld_pencil<1, N, S1, S2>(L0 + c * CS, q1, i3, in);
                mv<NQ, N>(Bt, in, out);
                st_pencil<1, NQ, S1, S2>(L0 + c * CS, q1, i3, out);
            });
            __syncthreads();
        }

        if constexpr (FORM == SF_MASS) {
            // ---- stage 3 (z): B_z, pointwise w kappa |J|, B_z^T
            pencils<C, NQ, NQ, NT>([&](int c, int q1, int q2) {
                T in[N], ut[NQ], k[NQ], t[N];
                ld_pencil<2, N, S1, S2>(L0 + c * CS, q1, q2, in);
                mv<NQ, N>(Bt, in, ut);
                ld_pencil<2, NQ, S1, S2>(L1 + c * CS, q1, q2, k);
                const T w12 = T(sP[c][0]) * W[q1] * W[q2];
#pragma unroll
                for (int q3 = 0; q3 < NQ; ++q3) ut[q3] *= w12 * W[q3] * k[q3];
                mtv<NQ, N>(BtT, ut, t);
                st_pencil<2, N, S1, S2>(L0 + c * CS, q1, q2, t);
            });
            __syncthreads();
        } else {
            // ---- stage 3 (z): B_z u -> u~ at the points; g_z = Dh_z u~
            pencils<C, NQ, NQ, NT>([&](int c, int q1, int q2) {
                T ut[NQ], gz[NQ];
                if constexpr (COLL) {
                    ld_pencil<2, NQ, S1, S2>(L0 + c * CS, q1, q2, ut);
                } else {
                    T in[N];
                    ld_pencil<2, N, S1, S2>(L0 + c * CS, q1, q2, in);
                    mv<NQ, N>(Bt, in, ut);
                    st_pencil<2, NQ, S1, S2>(L0 + c * CS, q1, q2, ut);
                }
                mv<NQ, NQ>(Dh, ut, gz);
                st_pencil<2, NQ, S1, S2>(L1 + c * CS, q1, q2, gz);
            });
            __syncthreads();
            // ---- stage 4 (y): g_y = Dh_y u~
            pencils<C, NQ, NQ, NT>([&](int c, int q1, int q3) {
                T ut[NQ], gy[NQ];
                ld_pencil<1, NQ, S1, S2>(L0 + c * CS, q1, q3, ut);
                mv<NQ, NQ>(Dh, ut, gy);
                st_pencil<1, NQ, S1, S2>(L2 + c * CS, q1, q3, gy);
            });
            __syncthreads();
            // ---- stage 5 (x): g_x, pointwise P = w kappa |J| G G^T, w = Dh_x^T v_x
            pencils<C, NQ, NQ, NT>([&](int c, int q2, int q3) {
                const int64_t gc = cell0 + c;
                T ut[NQ], gx[NQ], gy[NQ], gz[NQ], k[NQ];
                ld_pencil<0, NQ, S1, S2>(L0 + c * CS, q2, q3, ut);
                ld_pencil<0, NQ, S1, S2>(L2 + c * CS, q2, q3, gy);
                ld_pencil<0, NQ, S1, S2>(L1 + c * CS, q2, q3, gz);
#pragma unroll
                for (int q1 = 0; q1 < NQ; ++q1)
                    k[q1] = (has_kappa && gc < ncells) ? T(to_d(kappa[gc * NQ3 + (q1 * NQ + q2) * NQ + q3])) : T(1);
                mv<NQ, NQ>(Dh, ut, gx);
                const T w23 = W[q2] * W[q3];
                const T p00 = T(sP[c][0]), p01 = T(sP[c][1]), p02 = T(sP[c][2]);
                const T p11 = T(sP[c][3]), p12 = T(sP[c][4]), p22 = T(sP[c][5]);
#pragma unroll
                for (int q1 = 0; q1 < NQ; ++q1) {
                    const T om = k[q1] * W[q1] * w23;
                    const T a = gx[q1], b = gy[q1], d = gz[q1];
                    gx[q1] = om * (p00 * a + p01 * b + p02 * d);
                    gy[q1] = om * (p01 * a + p11 * b + p12 * d);
                    gz[q1] = om * (p02 * a + p12 * b + p22 * d);
                }
                mtv<NQ, NQ>(DhT, gx, ut);
                st_pencil<0, NQ, S1, S2>(L0 + c * CS, q2, q3, ut);
                st_pencil<0, NQ, S1, S2>(L2 + c * CS, q2, q3, gy);
                st_pencil<0, NQ, S1, S2>(L1 + c * CS, q2, q3, gz);
            });
            __syncthreads();
            // ---- stage 6 (y): w += Dh_y^T v_y
            pencils<C, NQ, NQ, NT>([&](int c, int q1, int q3) {
                T wv[NQ], vy[NQ];
                ld_pencil<1, NQ, S1, S2>(L0 + c * CS, q1, q3, wv);
                ld_pencil<1, NQ, S1, S2>(L2 + c * CS, q1, q3, vy);
                mtv_acc<NQ, NQ>(DhT, vy, wv);
                st_pencil<1, NQ, S1, S2>(L0 + c * CS, q1, q3, wv);
            });
            __syncthreads();
            // ---- stage 7 (z): w += Dh_z^T v_z, then B_z^T
            pencils<C, NQ, NQ, NT>([&](int c, int q1, int q2) {
                T wv[NQ], vz[NQ];
                ld_pencil<2, NQ, S1, S2>(L0 + c * CS, q1, q2, wv);
                ld_pencil<2, NQ, S1, S2>(L1 + c * CS, q1, q2, vz);
                mtv_acc<NQ, NQ>(DhT, vz, wv);
                if constexpr (COLL) {
                    st_pencil<2, NQ, S1, S2>(L0 + c * CS, q1, q2, wv);
                } else {
                    T t[N];
                    mtv<NQ, N>(BtT, wv, t);
                    st_pencil<2, N, S1, S2>(L0 + c * CS, q1, q2, t);
                }
            });
            __syncthreads();
        }

        // ---- stage 8 (y): B_y^T
        if constexpr (!COLL) {
            pencils<C, NQ, N, NT>([&](int c, int q1, int i3) {
                T in[NQ], out[N];
                ld_pencil<1, NQ, S1, S2>(L0 + c * CS, q1, i3, in);
                mtv<NQ, N>(BtT, in, out);
                st_pencil<1, N, S1, S2>(L0 + c * CS, q1, i3, out);
            });
            __syncthreads();
        }
        // ---- stage 9 (x): B_x^T, store y (coalesced)
        pencils<C, N, N, NT>([&](int c, int i2, int i3) {
            const int64_t gc = cell0 + c;
            if (gc >= ncells) return;
            T in[NQ], out[N];
            ld_pencil<0, NQ, S1, S2>(L0 + c * CS, i2, i3, in);
            if constexpr (COLL) {
#pragma unroll
                for (int i1 = 0; i1 < N; ++i1) out[i1] = in[i1];
            } else {
                mtv<NQ, N>(BtT, in, out);
            }
#pragma unroll
            for (int i1 = 0; i1 < N; ++i1) y[gc * N3 + (i1 * N + i2) * N + i3] = IO(out[i1]);
        });
    }
}

#undef W

namespace {

template <int N, int NQ, int FORM, bool COLL, typename T, typename IO>
int launch_one(const LaunchArgs &a, const T *tab)
{
    constexpr int NT = 256;
    constexpr int C = (NT / (NQ * NQ)) > 0 ? NT / (NQ * NQ) : 1;
    const int64_t groups = (a.ncells + C - 1) / C;
    if (groups > 0x7fffffffLL) return SF_ERR_CAPACITY;
    hipLaunchKernelGGL((action_q_kernel<N, NQ, FORM, COLL, T, IO, C, NT>), dim3(unsigned(groups)), dim3(NT), 0,
                       a.stream, a.ncells, a.vert, static_cast<const IO *>(a.kappa), static_cast<const IO *>(a.u),
                       static_cast<IO *>(a.y), tab, a.err);
    return hipGetLastError() == hipSuccess ? SF_OK : SF_ERR_HIP;
}

template <int N, int FORM, bool COLL>
int launch_prec(const LaunchArgs &a)
{
    if (a.precision == SF_FP64) {
        if (a.io == SF_F64) return launch_one<N, N, FORM, COLL, double, double>(a, a.tab64);
        return launch_one<N, N, FORM, COLL, double, float>(a, a.tab64);
    }
    if (a.precision == SF_FP32) {
        if (a.io == SF_F64) return launch_one<N, N, FORM, COLL, float, double>(a, a.tab32);
        return launch_one<N, N, FORM, COLL, float, float>(a, a.tab32);
    }
    return SF_ERR_UNSUPPORTED;
}

template <int N>
int launch_n(const LaunchArgs &a)
{
    const bool coll = a.family == SF_DQ;
    if (a.form == SF_MASS) return coll ? launch_prec<N, SF_MASS, true>(a) : launch_prec<N, SF_MASS, false>(a);
    if (a.form == SF_LAPLACE) return coll ? launch_prec<N, SF_LAPLACE, true>(a) : launch_prec<N, SF_LAPLACE, false>(a);
    return SF_ERR_UNSUPPORTED;
}

} // namespace

int launch_action_q(const LaunchArgs &a)
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

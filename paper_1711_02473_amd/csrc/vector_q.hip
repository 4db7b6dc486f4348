// Actions on the vector Q_p element (vector element of Sec. 2.3), matrix-free,
// FP64, on gfx950: the vector mass and vector Laplace forms (family SF_VQ,
// pointwise coefficient kappa) and Saint Venant-Kirchhoff hyperelasticity (the
// hyperelastic model of the paper's evaluation: forms SF_SVK, SF_SVK_RESIDUAL).
//
// Vector element: the scalar Q_p basis (GLL nodes) times the unit vectors,
// local DOF (component c, node i) at c * n^3 + i.  Because every vector
// basis function has a single nonzero component (Psi_(i,c) = Psi_i e_c, the
// Kronecker-delta structure of Sec. 2.3), the tested flux separates by
// component: y_(c,i) = sum_q sum_d dPsi_i/dxi_d (q) phi_(c,d)(q), one scalar
// backward contraction chain per component (delta cancellation, Sec. 3.4).
//
// Per point, with grad u = (reference gradient) G, G = J^{-1}:
//   vector mass:     w kappa |det J| u;   vector Laplace: w kappa |det J| grad u G^T;
//   F = I + grad u,  E = (F^T F - I) / 2,  S = lambda tr(E) I + 2 mu E,
//   residual form:   P = F S
//   linearised form: dF = grad du, dE = (dF^T F + F^T dF) / 2,
//                    dS = lambda tr(dE) I + 2 mu dE,  P = dF S + F dS,
// and the reference flux phi = w |det J| P G^T.
//
// Method: sum factorisation with the collocated derivative, as in the scalar
// actions (Sec. 3.3, eq. coeff_eval / eq. form_eval): every field is
// interpolated to the Gauss points with B one axis at a time (skipped for the
// GLL-collocated variant, B = I, Sec. 2.5), differentiated with the
// collocation matrix Dh along each axis, combined pointwise, and brought back
// with Dh^T (summed over the three directions) and B^T.
//
// Mapping: one workgroup owns C cells and keeps every per-cell tensor in LDS
// (3 per interpolated field: the values, overwritten by the axis-0 derivative,
// and the axis-1 and axis-2 derivatives).  The linearised form interpolates
// six fields (u0 and du), the residual three.  Inputs and outputs move
// between HBM and LDS with linear, fully coalesced copies; each contraction
// stage gives a thread one pencil (a line of one tensor along one axis) and
// applies the even-odd form of the 1-D matrix in registers.
#include "sf_device.hpp"
#include "sf_internal.hpp"

namespace sf {

// threads per workgroup: 512 where one cell's eighteen tensors fill most of
// the LDS (one workgroup per CU), so that the CU still holds eight waves
__host__ __device__ constexpr int vq_nt(int n, int form) { return (form == SF_SVK && n >= 8) ? 512 : 256; }

template <int N, int FORM> struct VqShape {
    using L = Lds3<N>;
    static constexpr int NF = FORM == SF_SVK ? 6 : 3;   // interpolated fields
    static constexpr int SPF = FORM == SF_MASS ? 1 : 3; // LDS tensors per field
    static constexpr int NS = SPF * NF;                 // LDS tensors per cell
    static constexpr int GEO = 34;                      // per-cell geometry: vertices (24), G (9), |det J|
    static constexpr int CELL = NS * L::CS + GEO;
    static constexpr int C = (8192 / CELL) > 0 ? 8192 / CELL : 1; // about 64 KB of tensors per group
    static constexpr int NT = vq_nt(N, FORM);
};

// Loop over the C * NF * N * N pencils along one axis of field tensors
// (slot 3 f + SLOT of every cell): f(cell, field, a, b).
template <int N, int C, int NF, int NT, typename Fn> __device__ __forceinline__ void vq_pencils(Fn &&fn)
{
    constexpr int NP = N * N, PER = NF * NP;
    for (int t = threadIdx.x; t < C * PER; t += NT) {
        const int c = t / PER;
        const int r = t - c * PER;
        const int f = r / NP;
        const int p = r - f * NP;
        const int a = p / N;
        fn(c, f, a, p - a * N);
    }
}

// Two independent pencil stages over the same fields (each lambda loads and stores
// along its own axis), run as one loop so that all threads have work.
template <int N, int C, int NF, int NT, typename F1, typename F2>
__device__ __forceinline__ void vq_pencils_2(F1 &&f1, F2 &&f2)
{
    constexpr int NP = N * N, PER = NF * NP, TOT = C * PER;
    for (int t = threadIdx.x; t < 2 * TOT; t += NT) {
        const bool second = t >= TOT;
        const int u = second ? t - TOT : t;
        const int c = u / PER;
        const int r = u - c * PER;
        const int f = r / NP;
        const int p = r - f * NP;
        const int a = p / N;
        if (second) f2(c, f, a, p - a * N);
        else f1(c, f, a, p - a * N);
    }
}

// Pointwise stage: reference gradients gu (u0, or the displacement) and gd
// (du) at one point -> reference flux w |det J| P G^T, returned in gu.
template <bool JAC>
__device__ __forceinline__ void svk_point(double (&gu)[3][3], const double (&gd)[3][3], const double (&G)[3][3],
                                          double wdet, double lambda, double mu)
{
    double F[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            double h = gu[c][0] * G[0][e];
            h = fma(gu[c][1], G[1][e], h);
            h = fma(gu[c][2], G[2][e], h);
            F[c][e] = (c == e ? 1.0 : 0.0) + h;
        }
    double S[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = a; b < 3; ++b) {
            double t = F[0][a] * F[0][b];
            t = fma(F[1][a], F[1][b], t);
            t = fma(F[2][a], F[2][b], t);
            S[a][b] = 0.5 * (t - (a == b ? 1.0 : 0.0)); // E
        }
    const double ltr = lambda * (S[0][0] + S[1][1] + S[2][2]);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = a; b < 3; ++b) {
            S[a][b] = 2.0 * mu * S[a][b] + (a == b ? ltr : 0.0);
            S[b][a] = S[a][b];
        }
    double P[3][3];
    if constexpr (!JAC) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int e = 0; e < 3; ++e) P[c][e] = F[c][0] * S[0][e] + F[c][1] * S[1][e] + F[c][2] * S[2][e];
    } else {
        double dF[3][3];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                double h = gd[c][0] * G[0][e];
                h = fma(gd[c][1], G[1][e], h);
                dF[c][e] = fma(gd[c][2], G[2][e], h);
            }
        double dS[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = a; b < 3; ++b) {
                double t = 0.0;
#pragma unroll
                for (int k = 0; k < 3; ++k) t += dF[k][a] * F[k][b] + F[k][a] * dF[k][b];
                dS[a][b] = 0.5 * t; // dE
            }
        const double ldtr = lambda * (dS[0][0] + dS[1][1] + dS[2][2]);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = a; b < 3; ++b) {
                dS[a][b] = 2.0 * mu * dS[a][b] + (a == b ? ldtr : 0.0);
                dS[b][a] = dS[a][b];
            }
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                double t = 0.0;
#pragma unroll
                for (int k = 0; k < 3; ++k) t += dF[c][k] * S[k][e] + F[c][k] * dS[k][e];
                P[c][e] = t;
            }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int d = 0; d < 3; ++d) gu[c][d] = wdet * (P[c][0] * G[d][0] + P[c][1] * G[d][1] + P[c][2] * G[d][2]);
}

// Vector Laplace pointwise stage: reference gradients gu -> w kappa |det J| (gu G) G^T.
__device__ __forceinline__ void vlap_point(double (&gu)[3][3], const double (&G)[3][3], double s)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double h[3];
#pragma unroll
        for (int e = 0; e < 3; ++e) h[e] = gu[c][0] * G[0][e] + gu[c][1] * G[1][e] + gu[c][2] * G[2][e];
#pragma unroll
        for (int d = 0; d < 3; ++d) gu[c][d] = s * (h[0] * G[d][0] + h[1] * G[d][1] + h[2] * G[d][2]);
    }
}

template <int N, bool COLL, int FORM, bool TRI>
__global__ void __launch_bounds__(vq_nt(N, FORM))
    vq_action_kernel(const int64_t ncells, const double *__restrict__ vert, const double *__restrict__ f0,
                     const double *__restrict__ f1, const double *__restrict__ coef, double *__restrict__ y,
                     const double *__restrict__ tab, const double lambda, const double mu, int *__restrict__ err)
{
    using Sh = VqShape<N, FORM>;
    using L = Lds3<N>;
    constexpr bool JAC = FORM == SF_SVK, GRAD = FORM != SF_MASS;
    constexpr int C = Sh::C, NF = Sh::NF, NS = Sh::NS, SPF = Sh::SPF, NT = Sh::NT, N3 = N * N * N;
    constexpr int S1 = L::S1, S2 = L::S2, CS = L::CS;
    constexpr TabLayout TL(N, 0, N);
    constexpr int N2 = N * N;
    // inputs of one group: the C * NF * N2 axis-0 lines (x-pencils) of the fields, N values
    // each, and C * 24 vertex coordinates
    constexpr int NPEN = C * NF * N2, KP = (NPEN + NT - 1) / NT, KV = (C * 24 + NT - 1) / NT;
    __shared__ double smem[C * Sh::CELL];
    double *geo = smem;              // [C][GEO]: vertices (24), G (9), |det J|
    double *ts = smem + C * Sh::GEO; // [C][NS][CS], field f: slots SPF f (values / d0), SPF f + 1 (d1), + 2 (d2)
    auto tensor = [&](int c, int s) { return ts + (c * NS + s) * CS; };
    const int64_t ngroups = (ncells + C - 1) / C;
    const double *BE = tab + TL.BEO(), *BTE = tab + TL.BTEO();

    // This thread's share of a group's inputs, requested in one unrolled batch: x-pencils
    // (lanes on consecutive pencils read consecutive addresses) and vertex coordinates.
    // Every lane loads (lanes without data read vert[0] and discard it).  Fields f < 3 are
    // component f of f0, f >= 3 component f - 3 of f1 (zero when the array is NULL);
    // padding cells get zero fields and the unit cube.
    double pf[KP][N], pv[KV];
    auto fetch = [&](int64_t g) {
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            const int t = threadIdx.x + k * NT;
            const int c = t / (NF * N2), r = t - c * (NF * N2), f = r / N2;
            const double *base = f < 3 ? f0 : f1;
            const bool ok = t < NPEN && base != nullptr && g * C + c < ncells;
            const double *src = ok ? base + (g * C + c) * (3 * N3) + (f % 3) * N3 + (r - f * N2) : vert;
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const double x = src[ok ? i * N2 : 0];
                pf[k][i] = ok ? x : 0.0;
            }
        }
#pragma unroll
        for (int k = 0; k < KV; ++k) {
            const int t = threadIdx.x + k * NT;
            const int c = t / 24, e = t - c * 24, v = e / 3, ax = e - v * 3;
            const bool ok = t < C * 24 && g * C + c < ncells;
            const double x = vert[ok ? (g * C + c) * 24 + e : 0];
            pv[k] = ok ? x : (((v >> (2 - ax)) & 1) ? 1.0 : 0.0);
        }
    };
    // the x-pencils go to LDS already interpolated along axis 0 (B_0 in registers)
    auto stash = [&]() {
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            const int t = threadIdx.x + k * NT;
            if (t < NPEN) {
                const int c = t / (NF * N2), r = t - c * (NF * N2), f = r / N2, pr = r - f * N2;
                if constexpr (COLL) {
                    st_pencil<0, N, S1, S2>(tensor(c, SPF * f), pr / N, pr % N, pf[k]);
                } else {
                    double o[N];
                    apply_eo<N, false, false>(BE, pf[k], o);
                    st_pencil<0, N, S1, S2>(tensor(c, SPF * f), pr / N, pr % N, o);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < KV; ++k) {
            const int t = threadIdx.x + k * NT;
            if (t < C * 24) geo[(t / 24) * Sh::GEO + t % 24] = pv[k];
        }
    };

    // persistent workgroups: group g + gridDim.x is requested while g is computed
    int64_t g = blockIdx.x;
    if (g < ngroups) fetch(g);
    for (; g < ngroups; g += gridDim.x) {
        const int64_t cell0 = g * C;
        stash();
        if (g + gridDim.x < ngroups) fetch(g + gridDim.x);
        __syncthreads();
        if constexpr (!TRI) { // affine cells: G and |det J| once per cell
            if (threadIdx.x < C) {
                const int c = threadIdx.x;
                double J[3][3], G[3][3], det = 1.0;
                const int fl = affine_jacobian(geo + c * Sh::GEO, J, det);
                if (fl && cell0 + c < ncells) atomicOr(err, fl);
                inverse3(J, det, G);
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) geo[c * Sh::GEO + 24 + 3 * a + b] = G[a][b];
                geo[c * Sh::GEO + 33] = fabs(det);
            }
        }

        // forward: interpolation along axis 1, then along axis 2 fused with the axis-2
        // derivative (written to its own tensor); then the axis-1 derivative and, once
        // every read of the values is done, the axis-0 derivative in place
        const double *DE = tab + TL.DhEO();
        if constexpr (!COLL) {
            vq_pencils<N, C, NF, NT>([&](int c, int f, int a, int b) {
                double x[N], o[N];
                ld_pencil<1, N, S1, S2>(tensor(c, SPF * f), a, b, x);
                apply_eo<N, false, false>(BE, x, o);
                st_pencil<1, N, S1, S2>(tensor(c, SPF * f), a, b, o);
            });
            __syncthreads();
        }
        vq_pencils<N, C, NF, NT>([&](int c, int f, int a, int b) {
            double x[N], o[N];
            ld_pencil<2, N, S1, S2>(tensor(c, SPF * f), a, b, x);
            if constexpr (!COLL) {
                apply_eo<N, false, false>(BE, x, o);
                st_pencil<2, N, S1, S2>(tensor(c, SPF * f), a, b, o);
            } else {
#pragma unroll
                for (int j = 0; j < N; ++j) o[j] = x[j];
            }
            if constexpr (GRAD) {
                apply_eo<N, true, false>(DE, o, x);
                st_pencil<2, N, S1, S2>(tensor(c, 3 * f + 2), a, b, x);
            }
        });
        __syncthreads();
        if constexpr (GRAD) {
            vq_pencils<N, C, NF, NT>([&](int c, int f, int a, int b) {
                double x[N], o[N];
                ld_pencil<1, N, S1, S2>(tensor(c, 3 * f), a, b, x);
                apply_eo<N, true, false>(DE, x, o);
                st_pencil<1, N, S1, S2>(tensor(c, 3 * f + 1), a, b, o);
            });
            __syncthreads();
            vq_pencils<N, C, NF, NT>([&](int c, int f, int a, int b) {
                double x[N], o[N];
                ld_pencil<0, N, S1, S2>(tensor(c, 3 * f), a, b, x);
                apply_eo<N, true, false>(DE, x, o);
                st_pencil<0, N, S1, S2>(tensor(c, 3 * f), a, b, o);
            });
            __syncthreads();
        }

        // pointwise: flux of component c along reference direction d into slot 3c + d
        // (mass: the scaled value of component c in slot c)
        {
            const double *W = tab + TL.W();
            const double *XQ = tab + TL.XQ();
            int bad = 0;
            for (int t = threadIdx.x; t < C * N3; t += NT) {
                const int c = t / N3;
                const int i = t - c * N3;
                const int q0 = i / (N * N), q1 = (i / N) % N, q2 = i % N;
                const int o = q0 * S1 + q1 * S2 + q2;
                double G[3][3], wdet;
                const double w = W[q0] * W[q1] * W[q2];
                if constexpr (TRI) {
                    double J[3][3];
                    const double det = trilinear_jacobian(geo + c * Sh::GEO, XQ[q0], XQ[q1], XQ[q2], J);
                    if (!(det > 0.0) && cell0 + c < ncells) bad = SF_FLAG_DETJ;
                    inverse3(J, det, G);
                    wdet = w * fabs(det);
                } else {
#pragma unroll
                    for (int a = 0; a < 3; ++a)
#pragma unroll
                        for (int b = 0; b < 3; ++b) G[a][b] = geo[c * Sh::GEO + 24 + 3 * a + b];
                    wdet = w * geo[c * Sh::GEO + 33];
                }
                if constexpr (FORM == SF_MASS || FORM == SF_LAPLACE) {
                    if (coef != nullptr && cell0 + c < ncells) wdet *= coef[(cell0 + c) * N3 + i];
                }
                if constexpr (FORM == SF_MASS) {
#pragma unroll
                    for (int k = 0; k < 3; ++k) tensor(c, k)[o] *= wdet;
                } else {
                    double gu[3][3], gd[3][3];
#pragma unroll
                    for (int k = 0; k < 3; ++k)
#pragma unroll
                        for (int d = 0; d < 3; ++d) {
                            gu[k][d] = tensor(c, 3 * k + d)[o];
                            if constexpr (JAC) gd[k][d] = tensor(c, 9 + 3 * k + d)[o];
                            else gd[k][d] = 0.0;
                        }
                    if constexpr (FORM == SF_LAPLACE) vlap_point(gu, G, wdet);
                    else svk_point<JAC>(gu, gd, G, wdet, lambda, mu);
#pragma unroll
                    for (int k = 0; k < 3; ++k)
#pragma unroll
                        for (int d = 0; d < 3; ++d) tensor(c, 3 * k + d)[o] = gu[k][d];
                }
            }
            if (bad) atomicOr(err, bad);
        }
        __syncthreads();

        // back to the DOFs: Dh^T along axes 0 and 1 in place; along axis 2 the three
        // directions summed (and B^T_2 applied on the same pencil); B^T_1; then B^T_0 on
        // x-pencils straight into y (lanes on consecutive pencils, coalesced)
        if constexpr (GRAD) {
            const double *DTE = tab + TL.DhTEO();
            vq_pencils_2<N, C, 3, NT>(
                [&](int c, int k, int a, int b) {
                    double x[N], o[N];
                    ld_pencil<0, N, S1, S2>(tensor(c, 3 * k), a, b, x);
                    apply_eo<N, true, false>(DTE, x, o);
                    st_pencil<0, N, S1, S2>(tensor(c, 3 * k), a, b, o);
                },
                [&](int c, int k, int a, int b) {
                    double x[N], o[N];
                    ld_pencil<1, N, S1, S2>(tensor(c, 3 * k + 1), a, b, x);
                    apply_eo<N, true, false>(DTE, x, o);
                    st_pencil<1, N, S1, S2>(tensor(c, 3 * k + 1), a, b, o);
                });
            __syncthreads();
            vq_pencils<N, C, 3, NT>([&](int c, int k, int a, int b) {
                double x[N], o[N];
                ld_pencil<2, N, S1, S2>(tensor(c, 3 * k + 2), a, b, x);
                ld_pencil<2, N, S1, S2>(tensor(c, 3 * k), a, b, o);
                apply_eo<N, true, true>(DTE, x, o);
                ld_pencil<2, N, S1, S2>(tensor(c, 3 * k + 1), a, b, x);
#pragma unroll
                for (int j = 0; j < N; ++j) o[j] += x[j];
                if constexpr (!COLL) {
                    apply_eo<N, false, false>(BTE, o, x);
                    st_pencil<2, N, S1, S2>(tensor(c, 3 * k), a, b, x);
                } else {
                    st_pencil<2, N, S1, S2>(tensor(c, 3 * k), a, b, o);
                }
            });
            __syncthreads();
        } else if constexpr (!COLL) {
            vq_pencils<N, C, 3, NT>([&](int c, int k, int a, int b) {
                double x[N], o[N];
                ld_pencil<2, N, S1, S2>(tensor(c, SPF * k), a, b, x);
                apply_eo<N, false, false>(BTE, x, o);
                st_pencil<2, N, S1, S2>(tensor(c, SPF * k), a, b, o);
            });
            __syncthreads();
        }
        if constexpr (!COLL) {
            vq_pencils<N, C, 3, NT>([&](int c, int k, int a, int b) {
                double x[N], o[N];
                ld_pencil<1, N, S1, S2>(tensor(c, SPF * k), a, b, x);
                apply_eo<N, false, false>(BTE, x, o);
                st_pencil<1, N, S1, S2>(tensor(c, SPF * k), a, b, o);
            });
            __syncthreads();
        }
        vq_pencils<N, C, 3, NT>([&](int c, int k, int a, int b) {
            if (cell0 + c >= ncells) return;
            double x[N], o[N];
            ld_pencil<0, N, S1, S2>(tensor(c, SPF * k), a, b, x);
            if constexpr (!COLL) {
                apply_eo<N, false, false>(BTE, x, o);
            } else {
#pragma unroll
                for (int j = 0; j < N; ++j) o[j] = x[j];
            }
            double *yo = y + (cell0 + c) * (3 * N3) + k * N3 + a * N + b;
#pragma unroll
            for (int i0 = 0; i0 < N; ++i0) yo[i0 * N2] = o[i0];
        });
        __syncthreads(); // the next group overwrites the tensors
    }
}

namespace {

template <int N, bool COLL, int FORM, bool TRI> int launch_vq4(const LaunchArgs &a)
{
    using Sh = VqShape<N, FORM>;
    static int resident = 0; // workgroups the device holds at once (occupancy x CUs)
    auto kern = vq_action_kernel<N, COLL, FORM, TRI>;
    if (resident <= 0) {
        int per_cu = 0, ncu = 0, dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, Sh::NT, 0) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return SF_ERR_HIP;
        resident = (per_cu > 0 ? per_cu : 1) * (ncu > 0 ? ncu : 1);
    }
    const int64_t groups = (a.ncells + Sh::C - 1) / Sh::C;
    const int grid = int(groups < resident ? groups : resident);
    // SF_SVK: fields u0 (the coefficient) and du; the others: the input vector, with
    // kappa as the pointwise coefficient of the vector mass / Laplace forms
    const double *f0 = FORM == SF_SVK ? static_cast<const double *>(a.kappa) : static_cast<const double *>(a.u);
    const double *f1 = FORM == SF_SVK ? static_cast<const double *>(a.u) : nullptr;
    const double *coef = (FORM == SF_MASS || FORM == SF_LAPLACE) ? static_cast<const double *>(a.kappa) : nullptr;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(Sh::NT), 0, a.stream, a.ncells, a.vert, f0, f1, coef,
                       static_cast<double *>(a.y), a.tab64, a.alpha, a.beta, a.err);
    return hipGetLastError() == hipSuccess ? SF_OK : SF_ERR_HIP;
}

template <int N, int FORM> int launch_vq_geo(const LaunchArgs &a)
{
    if (a.family == SF_QGLL) return a.trilinear ? launch_vq4<N, true, FORM, true>(a) : launch_vq4<N, true, FORM, false>(a);
    return a.trilinear ? launch_vq4<N, false, FORM, true>(a) : launch_vq4<N, false, FORM, false>(a);
}

template <int N> int launch_vq_n(const LaunchArgs &a)
{
    switch (a.form) {
    case SF_SVK: return launch_vq_geo<N, SF_SVK>(a);
    case SF_SVK_RESIDUAL: return launch_vq_geo<N, SF_SVK_RESIDUAL>(a);
    case SF_MASS: return a.trilinear ? launch_vq4<N, false, SF_MASS, true>(a) : launch_vq4<N, false, SF_MASS, false>(a);
    case SF_LAPLACE:
        return a.trilinear ? launch_vq4<N, false, SF_LAPLACE, true>(a) : launch_vq4<N, false, SF_LAPLACE, false>(a);
    default: return SF_ERR_UNSUPPORTED;
    }
}

} // namespace

int launch_action_vq(const LaunchArgs &a)
{
    if (a.nq != a.degree + 1 || a.precision != SF_FP64 || a.io != SF_F64) return SF_ERR_UNSUPPORTED;
    const bool svk = a.form == SF_SVK || a.form == SF_SVK_RESIDUAL;
    if (svk ? (a.family != SF_Q && a.family != SF_QGLL) : (a.family != SF_VQ)) return SF_ERR_UNSUPPORTED;
    switch (a.degree + 1) {
    case 2: return launch_vq_n<2>(a);
    case 3: return launch_vq_n<3>(a);
    case 4: return launch_vq_n<4>(a);
    case 5: return launch_vq_n<5>(a);
    case 6: return launch_vq_n<6>(a);
    case 7: return launch_vq_n<7>(a);
    case 8: return launch_vq_n<8>(a);
    case 9: return launch_vq_n<9>(a);
    default: return SF_ERR_UNSUPPORTED;
    }
}

} // namespace sf

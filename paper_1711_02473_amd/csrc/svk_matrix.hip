// Element matrices of the linearised Saint Venant-Kirchhoff residual on the
// vector Q_p element (the left-hand side of the hyperelastic model in the
// paper's evaluation), FP64, p <= 8, on gfx950.
//
// Argument factorisation (Sec. 3.2): with the tangent modulus Amod of P at
// the linearisation point,
//   A_{(c,i),(c',j)} = sum_q sum_{d,d'} dPsi_i/dxi_d (q) K^{cc'}_{dd'}(q) dPsi_j/dxi_d' (q),
//   K^{cc'}_{dd'} = w |det J| sum_{e,e'} G_{de} Amod_{c e c' e'} G_{d'e'},
//   Amod_{cec'e'} = delta_{cc'} S_{e'e} + lambda F_{ce} F_{c'e'}
//                   + mu ((F F^T)_{cc'} delta_{ee'} + F_{ce'} F_{c'e}),
// so each of the nine component blocks (c, c') is a sum of nine products
// (d, d'), product (d, d') having the derivative table D on axis d for the
// test function and on axis d' for the trial function and the value table B
// elsewhere.  Every product is sum-factorised over q2, then q1, then q0
// (Alg. 1's order for a hexahedron; every order costs the same here), one
// i2-slice of the first stage at a time, and the products are merged by
// distributivity (Sec. 3.6, pass 6) once only the axis-0 tables remain: the
// nine products fall into four groups by their axis-0 pair (B or D for the
// test and trial functions), so the last stage runs four sweeps, not nine.
//
// Mapping: one workgroup per (cell, block), one thread per column of the block
// for p <= 3 (one wave), so that the last stage keeps every lane busy.  The
// cell's u0 is staged in LDS and its reference gradient sum-factorised (eight
// one-axis contractions per component); the block's nine coefficient fields K
// then stay in LDS for the matrix stages.  Rows of the
// block are written as contiguous (p+1)^3-long runs.
#include "sf_device.hpp"
#include "sf_internal.hpp"

namespace sf {

// threads per workgroup: one per column j of a block row, (p+1)^3 rounded up to a
// wave, for p <= 3; 256 for p = 4..5, where the first two stages' extra threads pay more
// than the idle lanes of the last one cost (measured); 512 from p = 6 on, where the
// LDS holds one or two workgroups per CU and more waves hide the write latency
__host__ __device__ constexpr int svk_matrix_nt(int n) { return n <= 4 ? (n * n * n + 63) / 64 * 64 : (n <= 6 ? 256 : 512); }
// phase-A buffers: two (the next phase A overlaps this phase B) while the LDS holds
// 29 n^3 doubles, one (and a barrier) above
__host__ __device__ constexpr int svk_t2_buffers(int n) { return 29 * n * n * n * 8 <= 150 * 1024 ? 2 : 1; }

template <int N, bool TRI>
__global__ void __launch_bounds__(svk_matrix_nt(N))
    svk_matrix_kernel(const int64_t ncells, const double *__restrict__ vert, const double *__restrict__ u0,
                      double *__restrict__ A, const double *__restrict__ tab, const double lambda, const double mu,
                      int *__restrict__ err)
{
    constexpr int NT = svk_matrix_nt(N), N2 = N * N, N3 = N2 * N, ND = 3 * N3;
    constexpr TabLayout TL(N, 0, N);
    constexpr int T1SZ = N * N * N; // one i2-slice of one product: [q0][q1][j2]
    constexpr int T2SZ = N * N * N; // one group: [q0][j1][j2]
    __shared__ double sU[3 * N3];      // u0 by component
    __shared__ double sB[N * N];       // B[q][i]
    __shared__ double sD[N * N];       // D[q][i]
    __shared__ double sW[N], sX[N];    // weights and points
    __shared__ double sGeo[34];        // vertices (24), G (9), |det J|
    __shared__ double sK[9 * N3];      // K_{dd'} at the points, product p = 3 d + d'
    __shared__ double sT1[9 * T1SZ];   // stage 1, one i2-slice per product
    constexpr int NB2 = svk_t2_buffers(N);
    __shared__ double sT2[NB2 * 4 * T2SZ]; // phase A, four groups, one or two buffers

    const int64_t cell = int64_t(blockIdx.x) / 9;
    const int blk = int(blockIdx.x - cell * 9), cr = blk / 3, cc = blk - cr * 3; // block (test cr, trial cc)
    const int tid = threadIdx.x;
    if (cell >= ncells) return; // the grid holds exactly 9 ncells groups: never taken

    for (int t = tid; t < 3 * N3; t += NT) sU[t] = u0 != nullptr ? u0[cell * ND + t] : 0.0;
    for (int t = tid; t < N2; t += NT) {
        sB[t] = tab[TL.B0() + t];
        sD[t] = tab[TL.D0() + t];
    }
    if (tid < N) {
        sW[tid] = tab[TL.W() + tid];
        sX[tid] = tab[TL.XQ() + tid];
    }
    if (tid < 24) sGeo[tid] = vert[cell * 24 + tid];
    __syncthreads();
    if constexpr (!TRI) {
        if (tid == 0) {
            double J[3][3], G[3][3], det = 1.0;
            const int fl = affine_jacobian(sGeo, J, det);
            if (fl && blk == 0) atomicOr(err, fl);
            inverse3(J, det, G);
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) sGeo[24 + 3 * a + b] = G[a][b];
            sGeo[33] = fabs(det);
        }
        __syncthreads();
    }

    // ---- reference gradient of u0 at the points, sum-factorised one axis at a time:
    // axis 2 with B and D (sT1: [c][B|D][i0][i1][q2]); axis 1 (sK: [c][BB|DB|BD][i0][q1][q2],
    // the first letter the axis-1 table); axis 0 into sT1 ([c][d][q]: d0 = D0 BB, d1 = B0 DB,
    // d2 = B0 BD).  The pointwise stage below reads a point's nine values from sT1 and
    // writes the coefficients to sK.
    for (int t = tid; t < 6 * N3; t += NT) {
        const int cs = t / N3, r = t - cs * N3, c = cs >> 1;
        const int i01 = r / N, q2 = r - i01 * N;
        const double *X = (cs & 1) ? sD : sB;
        const double *uc = sU + c * N3 + i01 * N;
        double acc = 0.0;
#pragma unroll
        for (int i2 = 0; i2 < N; ++i2) acc = fma(X[q2 * N + i2], uc[i2], acc);
        sT1[t] = acc;
    }
    __syncthreads();
    for (int t = tid; t < 9 * N3; t += NT) {
        const int ck = t / N3, r = t - ck * N3, c = ck / 3, k = ck - c * 3;
        const int i0 = r / N2, q1 = (r / N) % N, q2 = r % N;
        const double *X = k == 1 ? sD : sB;                                   // axis-1 table
        const double *src = sT1 + (2 * c + (k == 2 ? 1 : 0)) * N3 + i0 * N2 + q2; // B or D on axis 2
        double acc = 0.0;
#pragma unroll
        for (int i1 = 0; i1 < N; ++i1) acc = fma(X[q1 * N + i1], src[i1 * N], acc);
        sK[t] = acc;
    }
    __syncthreads();
    for (int t = tid; t < 9 * N3; t += NT) {
        const int cd = t / N3, q = t - cd * N3, c = cd / 3, d = cd - c * 3;
        const int q0 = q / N2, q12 = q - q0 * N2;
        const double *X = d == 0 ? sD : sB; // axis-0 table
        const double *src = sK + (3 * c + d) * N3 + q12;
        double acc = 0.0;
#pragma unroll
        for (int i0 = 0; i0 < N; ++i0) acc = fma(X[q0 * N + i0], src[i0 * N2], acc);
        sT1[t] = acc;
    }
    __syncthreads();

    // ---- coefficient fields of this block at every point
    for (int q = tid; q < N3; q += NT) {
        const int q0 = q / N2, q1 = (q / N) % N, q2 = q % N;
        double G[3][3], wdet;
        if constexpr (TRI) {
            double J[3][3];
            const double det = trilinear_jacobian(sGeo, sX[q0], sX[q1], sX[q2], J);
            if (!(det > 0.0) && blk == 0) atomicOr(err, SF_FLAG_DETJ);
            inverse3(J, det, G);
            wdet = fabs(det);
        } else {
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) G[a][b] = sGeo[24 + 3 * a + b];
            wdet = sGeo[33];
        }
        wdet *= sW[q0] * sW[q1] * sW[q2];
        double gu[3][3]; // reference gradient of u0 at q
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int d = 0; d < 3; ++d) gu[c][d] = sT1[(3 * c + d) * N3 + q];
        double F[3][3];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int e = 0; e < 3; ++e)
                F[c][e] = (c == e ? 1.0 : 0.0) + gu[c][0] * G[0][e] + gu[c][1] * G[1][e] + gu[c][2] * G[2][e];
        double S[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b)
                S[a][b] = 0.5 * (F[0][a] * F[0][b] + F[1][a] * F[1][b] + F[2][a] * F[2][b] - (a == b ? 1.0 : 0.0));
        const double ltr = lambda * (S[0][0] + S[1][1] + S[2][2]);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) S[a][b] = 2.0 * mu * S[a][b] + (a == b ? ltr : 0.0);
        const double ff = F[cr][0] * F[cc][0] + F[cr][1] * F[cc][1] + F[cr][2] * F[cc][2]; // (F F^T)_{cr cc}
        double Am[3][3]; // Amod_{cr e cc e'}
#pragma unroll
        for (int e = 0; e < 3; ++e)
#pragma unroll
            for (int f = 0; f < 3; ++f)
                Am[e][f] = (cr == cc ? S[f][e] : 0.0) + lambda * F[cr][e] * F[cc][f] +
                           mu * ((e == f ? ff : 0.0) + F[cr][f] * F[cc][e]);
        double GA[3][3]; // G Am
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int f = 0; f < 3; ++f) GA[d][f] = G[d][0] * Am[0][f] + G[d][1] * Am[1][f] + G[d][2] * Am[2][f];
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int dd = 0; dd < 3; ++dd)
                sK[(3 * d + dd) * N3 + q] = wdet * (GA[d][0] * G[dd][0] + GA[d][1] * G[dd][1] + GA[d][2] * G[dd][2]);
    }
    __syncthreads();

    // ---- sum-factorised products, merged by their axis-0 pair in the last stage
    const int64_t rowbase = cell * int64_t(ND) * ND + int64_t(cr * N3) * ND + cc * N3;
    for (int i2 = 0; i2 < N; ++i2) {
        // stage 1: one line per task, product p1 and (q0, q1)
        for (int t = tid; t < 9 * N2; t += NT) {
            const int p1 = t / N2, q01 = t - p1 * N2;
            const int d1 = p1 / 3, dd1 = p1 - d1 * 3;
            const double *X = d1 == 2 ? sD : sB;  // test table on axis 2
            const double *Y = dd1 == 2 ? sD : sB; // trial table on axis 2
            const double *k = sK + p1 * N3 + q01 * N;
            double row[N];
#pragma unroll
            for (int j2 = 0; j2 < N; ++j2) row[j2] = 0.0;
#pragma unroll
            for (int q2 = 0; q2 < N; ++q2) {
                const double xk = X[q2 * N + i2] * k[q2];
#pragma unroll
                for (int j2 = 0; j2 < N; ++j2) row[j2] = fma(xk, Y[q2 * N + j2], row[j2]);
            }
#pragma unroll
            for (int j2 = 0; j2 < N; ++j2) sT1[p1 * T1SZ + q01 * N + j2] = row[j2];
        }
        __syncthreads();
        for (int i1 = 0; i1 < N; ++i1) {
            double *T2 = sT2 + (NB2 == 2 ? ((i2 * N + i1) & 1) : 0) * 4 * T2SZ;
            // phase A: T2_g[q0][j1][j2] = sum over products p of group g of
            //          sum_q1 X1_p[q1][i1] Y1_p[q1][j1] T1_p[q0][q1][j2]
            for (int t = tid; t < 4 * N3; t += NT) {
                const int g = t / N3, r = t - g * N3;
                const int q0 = r / N2, j1 = (r / N) % N, j2 = r % N;
                const int tD = g >> 1, tT = g & 1; // axis-0 test / trial table is D
                double acc = 0.0;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    if ((d == 0) != bool(tD)) continue;
#pragma unroll
                    for (int dd = 0; dd < 3; ++dd) {
                        if ((dd == 0) != bool(tT)) continue;
                        const double *X = d == 1 ? sD : sB;
                        const double *Y = dd == 1 ? sD : sB;
                        const double *t1 = sT1 + (3 * d + dd) * T1SZ + q0 * N2 + j2;
#pragma unroll
                        for (int q1 = 0; q1 < N; ++q1) acc = fma(X[q1 * N + i1] * Y[q1 * N + j1], t1[q1 * N], acc);
                    }
                }
                T2[g * T2SZ + r] = acc;
            }
            __syncthreads();
            // phase B: A[(i0 i1 i2), j] = sum_g sum_q0 X0_g[q0][i0] Y0_g[q0][j0] T2_g[q0][j1 j2]
            for (int j = tid; j < N3; j += NT) {
                const int j0 = j / N2, j12 = j - j0 * N2;
                double out[N];
#pragma unroll
                for (int i0 = 0; i0 < N; ++i0) out[i0] = 0.0;
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const double *X = (g >> 1) ? sD : sB;
                    const double *Y = (g & 1) ? sD : sB;
                    // at n >= 8 a rolled q0 loop: unrolled, the compiler keeps every table
                    // entry of the sweep in registers across the column loop and spills
#pragma unroll(N >= 8 ? 1 : N)
                    for (int q0 = 0; q0 < N; ++q0) {
                        const double yt = Y[q0 * N + j0] * T2[g * T2SZ + q0 * N2 + j12];
#pragma unroll
                        for (int i0 = 0; i0 < N; ++i0) out[i0] = fma(X[q0 * N + i0], yt, out[i0]);
                    }
                }
#pragma unroll
                for (int i0 = 0; i0 < N; ++i0) A[rowbase + int64_t(i0 * N2 + i1 * N + i2) * ND + j] = out[i0];
            }
            // with two buffers the next phase A writes the other one; stage 1 of the next
            // slice is separated from this phase B's T1-free reads by the barrier after
            // phase A; with one buffer the next phase A waits for this phase B
            if constexpr (NB2 == 1) __syncthreads();
        }
        __syncthreads(); // the next stage 1 overwrites T1 read by the last phase A
    }
}

namespace {

template <int N, bool TRI> int launch_svk_matrix_n(const LaunchArgs &a)
{
    const int64_t groups = a.ncells * 9;
    if (groups > 0x7fffffffLL) return SF_ERR_CAPACITY;
    hipLaunchKernelGGL((svk_matrix_kernel<N, TRI>), dim3(unsigned(groups)), dim3(svk_matrix_nt(N)), 0, a.stream,
                       a.ncells, a.vert, static_cast<const double *>(a.kappa), static_cast<double *>(a.A), a.tab64,
                       a.alpha, a.beta, a.err);
    return hipGetLastError() == hipSuccess ? SF_OK : SF_ERR_HIP;
}

} // namespace

int launch_matrix_svk(const LaunchArgs &a)
{
    if (a.form != SF_SVK || a.nq != a.degree + 1 || a.precision != SF_FP64 || a.io != SF_F64) return SF_ERR_UNSUPPORTED;
    if (a.family != SF_Q && a.family != SF_QGLL) return SF_ERR_UNSUPPORTED;
    switch (a.degree + 1) {
    case 2: return a.trilinear ? launch_svk_matrix_n<2, true>(a) : launch_svk_matrix_n<2, false>(a);
    case 3: return a.trilinear ? launch_svk_matrix_n<3, true>(a) : launch_svk_matrix_n<3, false>(a);
    case 4: return a.trilinear ? launch_svk_matrix_n<4, true>(a) : launch_svk_matrix_n<4, false>(a);
    case 5: return a.trilinear ? launch_svk_matrix_n<5, true>(a) : launch_svk_matrix_n<5, false>(a);
    case 6: return a.trilinear ? launch_svk_matrix_n<6, true>(a) : launch_svk_matrix_n<6, false>(a);
    case 7: return a.trilinear ? launch_svk_matrix_n<7, true>(a) : launch_svk_matrix_n<7, false>(a);
    case 8: return a.trilinear ? launch_svk_matrix_n<8, true>(a) : launch_svk_matrix_n<8, false>(a);
    case 9: return a.trilinear ? launch_svk_matrix_n<9, true>(a) : launch_svk_matrix_n<9, false>(a);
    default: return SF_ERR_UNSUPPORTED;
    }
}

} // namespace sf

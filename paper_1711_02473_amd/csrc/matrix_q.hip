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
// For every i2: stage 1 builds the slice
//   T1_s[q0][q1][j2] = sum_q2 w X_s[q2][i2] X_s[q2][j2] kappa[q0][q1][q2]
//   (s = BB, and DD for the Laplacian) in LDS (n times less LDS than the
//   whole T1 tensor at the same flop count); then for every i1:
//   phase A: T2_r[q0][j1][j2] = sum_q1 (factor) w X[q1][i1] Y[q1][j1] T1_s[q0][q1][i2][j2]
//   phase B: A[(i0,i1,i2), (j0,j1,j2)] = sum_r sum_q0 w X_r[q0][i0] Y_r[q0][j0] T2_r[q0][j1][j2]
// Phase B's lanes run over consecutive columns j, so each of the n rows of the
// block is written as one contiguous n^3-long run (coalesced).
#include "sf_device.hpp"
#include "sf_internal.hpp"
#include "mixed_body.inc"
#include "matrix_q_body.inc"

namespace sf {

// Register target of five waves per SIMD (80 VGPRs, no spills): more resident workgroups
// hide the write latency; measured faster for p = 1 and 3, slower for p = 2 (kept at the
// compiler's default there), no effect for p >= 4.
// MODE: SF_FP64, or SF_BF16 / SF_FP16 / SF_BF16X3 for the final (q0) contraction on the
// matrix cores with FP32 accumulation (stage 1 and phase A stay FP64).
template <int N, int NQ, int FORM, typename IO, int C, int NT, int R, int MODE = SF_FP64>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(N == 3 || MODE != SF_FP64 ? 1 : 5, 8)))
    matrix_q_kernel(const int64_t ncells, const double *__restrict__ vert, const IO *__restrict__ kappa,
                    IO *__restrict__ A, const double *__restrict__ tab, int *__restrict__ err)
{
    __shared__ double smem[MatrixQSmem<N, NQ, FORM, C>::doubles];
    matrix_q_body<N, NQ, FORM, IO, C, NT, R, MODE>(int64_t(blockIdx.x) * C, ncells, vert, kappa, A, 0, tab, err,
                                                    smem);
}

// clears the off-diagonal blocks' buffer before the vector element's diagonal
// blocks are assigned (a kernel, not a memset, so that the launch can be captured)
template <typename IO> __global__ void matrix_clear_kernel(IO *A, int64_t n)
{
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += int64_t(gridDim.x) * blockDim.x)
        A[t] = IO(0);
}

namespace {

template <int N, int FORM, typename IO, int R, int MODE = SF_FP64>
int launch_one(const LaunchArgs &a)
{
    constexpr int N3 = N * N * N;
    constexpr int C = (256 / N3) > 0 ? 256 / N3 : 1;
    constexpr int NT0 = ((C * N3 + 63) / 64) * 64;
    constexpr int NT = NT0 > 1024 ? 1024 : NT0;
    const int64_t groups = (a.ncells + C - 1) / C;
    if (groups > 0x7fffffffLL) return SF_ERR_CAPACITY;
    if (R > 1) {
        const int64_t n = a.ncells * int64_t(R * N3) * (R * N3);
        const int64_t blocks = (n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192;
        hipLaunchKernelGGL(matrix_clear_kernel<IO>, dim3(unsigned(blocks)), dim3(256), 0, a.stream,
                           static_cast<IO *>(a.A), n);
    }
    hipLaunchKernelGGL((matrix_q_kernel<N, N, FORM, IO, C, NT, R, MODE>), dim3(unsigned(groups)), dim3(NT), 0, a.stream,
                       a.ncells, a.vert, static_cast<const IO *>(a.kappa), static_cast<IO *>(a.A), a.tab64, a.err);
    return hipGetLastError() == hipSuccess ? SF_OK : SF_ERR_HIP;
}

template <int N, int FORM, typename IO>
int launch_mixed(const LaunchArgs &a)
{
    switch (a.precision) {
    case SF_BF16: return launch_one<N, FORM, IO, 1, SF_BF16>(a);
    case SF_FP16: return launch_one<N, FORM, IO, 1, SF_FP16>(a);
    case SF_BF16X3: return launch_one<N, FORM, IO, 1, SF_BF16X3>(a);
    default: return SF_ERR_UNSUPPORTED;
    }
}

template <int N, int R>
int launch_nr(const LaunchArgs &a)
{
    if (a.precision != SF_FP64) {
        // lower-precision final contraction: scalar Q_p / dQ_p, box cells
        if (R != 1) return SF_ERR_UNSUPPORTED;
        if (a.form == SF_MASS)
            return a.io == SF_F64 ? launch_mixed<N, SF_MASS, double>(a) : launch_mixed<N, SF_MASS, float>(a);
        if (a.form == SF_LAPLACE)
            return a.io == SF_F64 ? launch_mixed<N, SF_LAPLACE, double>(a) : launch_mixed<N, SF_LAPLACE, float>(a);
        return SF_ERR_UNSUPPORTED;
    }
    if (a.form == SF_MASS)
        return a.io == SF_F64 ? launch_one<N, SF_MASS, double, R>(a) : launch_one<N, SF_MASS, float, R>(a);
    if (a.form == SF_LAPLACE)
        return a.io == SF_F64 ? launch_one<N, SF_LAPLACE, double, R>(a) : launch_one<N, SF_LAPLACE, float, R>(a);
    return SF_ERR_UNSUPPORTED;
}

template <int N>
int launch_n(const LaunchArgs &a)
{
    return a.family == SF_VQ ? launch_nr<N, 3>(a) : launch_nr<N, 1>(a);
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

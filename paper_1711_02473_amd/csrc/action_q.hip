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
#include "action_q_body.inc"

namespace sf {


// Trilinear Laplace at p = 6: a register target of three waves per SIMD (the LDS limit;
// 168 VGPRs, a few spilled) measured 10 % faster than the compiler's two; the same at p = 4
// (four waves) and p = 8 spilled too much and was slower.
template <int N, int NQ, int FORM, bool COLL, typename T, typename IO, int C, int NT, bool TRI>
__global__ void __launch_bounds__(NT)
    __attribute__((amdgpu_waves_per_eu(TRI && FORM == SF_LAPLACE && N == 7 ? 3 : 1, 8)))
    action_q_kernel(const int64_t ncells, const double *__restrict__ vert, const IO *__restrict__ kappa,
                    const IO *__restrict__ u, IO *__restrict__ y, const T *__restrict__ tab, int *__restrict__ err)
{
    __shared__ double smem[ActionQSmem<N, NQ, FORM, COLL, T, C>::bytes / 8];
    action_q_body<N, NQ, FORM, COLL, T, IO, C, NT, TRI>(int64_t(blockIdx.x) * C, ncells, vert, kappa, u, y, tab,
                                                        err, smem);
}

namespace {

template <int N, int NQ, int FORM, bool COLL, typename T, typename IO, bool TRI = false>
int launch_one(const LaunchArgs &a, const T *tab)
{
    constexpr int NT = 256;
    constexpr int C = (NT / (NQ * NQ)) > 0 ? NT / (NQ * NQ) : 1;
    const int64_t groups = (a.ncells + C - 1) / C;
    if (groups > 0x7fffffffLL) return SF_ERR_CAPACITY;
    hipLaunchKernelGGL((action_q_kernel<N, NQ, FORM, COLL, T, IO, C, NT, TRI>), dim3(unsigned(groups)), dim3(NT), 0,
                       a.stream, a.ncells, a.vert, static_cast<const IO *>(a.kappa), static_cast<const IO *>(a.u),
                       static_cast<IO *>(a.y), tab, a.err);
    return hipGetLastError() == hipSuccess ? SF_OK : SF_ERR_HIP;
}

template <int N, int FORM, bool COLL>
int launch_prec(const LaunchArgs &a)
{
    if (a.trilinear) { // per-point geometry: FP64 contractions, FP64 storage
        if (a.precision != SF_FP64 || a.io != SF_F64) return SF_ERR_UNSUPPORTED;
        return launch_one<N, N, FORM, COLL, double, double, true>(a, a.tab64);
    }
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
    const bool coll = a.family == SF_DQ || a.family == SF_QGLL; // B = I
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

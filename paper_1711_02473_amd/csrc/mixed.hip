// Mixed-precision operator action for the scalar families (Q_p, dQ_p; mass
// and Laplace) on gfx950: every one-axis contraction runs on the matrix
// cores (v_mfma_f32_16x16x32_{bf16,f16}) with FP32 accumulation, while the
// Jacobian, its inverse and determinant and the pointwise factor
// |J| G G^T are assembled in FP64 (then applied in FP32).
//
// Same algorithm as the FP64 kernel (interpolation to the Gauss points, the
// collocated derivative, transposed contractions; Sec. 3.3 eq. coeff_eval /
// eq. form_eval), with one 16x16x32 MFMA tile per 16 pencils: the 1-D matrix
// (rows = output points, padded to 16) is the A operand, held in registers
// for the whole kernel; 16 pencils of the FP32 LDS tensor, converted on the
// fly, are the B operand; the 16x16 FP32 result gives each lane four output
// points of one pencil.
//
// Modes:
//   BF16, FP16: one MFMA per tile, operands rounded once (about 2^-8 / 2^-11
//               relative per contraction).
//   BF16X3:     operands split into three BF16 terms x = hi + mid + lo; the
//               products hi*hi, mid*hi, lo*hi (first MFMA) and hi*mid,
//               mid*mid, hi*lo (second MFMA) are packed side by side along
//               the K dimension of two MFMAs (K = 32 holds three slots of
//               width n <= 10), which recovers about 24 significand bits.
#include "sf_device.hpp"
#include "sf_internal.hpp"
#include "mixed_body.inc"

namespace sf {

// Register target: four waves per SIMD for the single-term modes; three for BF16X3,
// whose split operands need more registers (at four it spilled to scratch)
template <int N, int NQ, int FORM, bool COLL, int MODE, typename IO, int C, int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(MODE == SF_BF16X3 ? 3 : 4, 8)))
    action_mixed_kernel(const int64_t ncells, const double *__restrict__ vert, const IO *__restrict__ kappa,
                        const IO *__restrict__ u, IO *__restrict__ y, const double *__restrict__ tab64,
                        const uint16_t *__restrict__ mix, int *__restrict__ err)
{
    __shared__ double smem[ActionMixedSmem<N, NQ, FORM, C>::bytes / 8];
    action_mixed_body<N, NQ, FORM, COLL, MODE, IO, C, NT>(int64_t(blockIdx.x) * C, ncells, vert, kappa, u, y, tab64,
                                                          mix, err, smem);
}

namespace {

template <int N, int FORM, bool COLL, int MODE, typename IO>
int launch_one(const LaunchArgs &a)
{
    constexpr int NQ = N;
    constexpr int NBUF = (FORM == SF_LAPLACE) ? 4 : 1;
    constexpr int CS = Lds3<NQ>::CS;
    // as many cells as keep the whole LDS footprint (tensors, per-cell factors, weights)
    // within 40 KiB, so that four workgroups fit in a CU's 160 KiB
    constexpr int C0 = (40 * 1024 - 4 * (NQ + 64) - 8) / (NBUF * CS * 4 + 8 * 6);
    constexpr int C = C0 < 1 ? 1 : (C0 > 64 ? 64 : C0);
    constexpr int NT = 256;
    const int64_t groups = (a.ncells + C - 1) / C;
    if (groups > 0x7fffffffLL) return SF_ERR_CAPACITY;
    hipLaunchKernelGGL((action_mixed_kernel<N, NQ, FORM, COLL, MODE, IO, C, NT>), dim3(unsigned(groups)), dim3(NT),
                       0, a.stream, a.ncells, a.vert, static_cast<const IO *>(a.kappa),
                       static_cast<const IO *>(a.u), static_cast<IO *>(a.y), a.tab64,
                       static_cast<const uint16_t *>(a.tabmix), a.err);
    return hipGetLastError() == hipSuccess ? SF_OK : SF_ERR_HIP;
}

template <int N, int FORM, bool COLL, int MODE>
int launch_io(const LaunchArgs &a)
{
    return a.io == SF_F64 ? launch_one<N, FORM, COLL, MODE, double>(a) : launch_one<N, FORM, COLL, MODE, float>(a);
}

template <int N, int FORM, bool COLL>
int launch_mode(const LaunchArgs &a)
{
    switch (a.precision) {
    case SF_BF16: return launch_io<N, FORM, COLL, SF_BF16>(a);
    case SF_FP16: return launch_io<N, FORM, COLL, SF_FP16>(a);
    case SF_BF16X3: return launch_io<N, FORM, COLL, SF_BF16X3>(a);
    default: return SF_ERR_UNSUPPORTED;
    }
}

template <int N>
int launch_n(const LaunchArgs &a)
{
    const bool coll = a.family == SF_DQ || a.family == SF_QGLL; // B = I
    if (a.form == SF_LAPLACE) return coll ? launch_mode<N, SF_LAPLACE, true>(a) : launch_mode<N, SF_LAPLACE, false>(a);
    if (a.form == SF_MASS) return coll ? launch_mode<N, SF_MASS, true>(a) : launch_mode<N, SF_MASS, false>(a);
    return SF_ERR_UNSUPPORTED;
}

} // namespace

int launch_action_mixed(const LaunchArgs &a)
{
    if (a.family != SF_Q && a.family != SF_DQ && a.family != SF_QGLL) return SF_ERR_UNSUPPORTED;
    if (a.nq != a.degree + 1 || !a.tabmix) return SF_ERR_UNSUPPORTED;
    if (a.variant != 1 && a.tabkron) {
        // the dense Kronecker kernels; tables too large for LDS fall through
        const int rc = a.degree + 1 <= 4 ? launch_action_kron(a) : launch_action_kron2(a);
        if (rc != SF_ERR_UNSUPPORTED) return rc;
    }
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

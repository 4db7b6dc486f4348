// Mixed-precision operator action for the scalar families at n <= 4 points per
// axis (p <= 3): every contraction on the matrix cores, with no LDS tensor.
//
// With nd = n^3 <= 64 DOFs and points per cell, the interpolation of a cell
// (and each reference gradient component) is one dense nd x nd product with the
// Kronecker table G (kron_layout.hpp), and the transposed contraction is the
// product with G^T.  Sixteen cells form the N dimension of the MFMA tiles:
//   forward   g_a[q][c] = sum_i G_a[q][i] u[c][i]          (v_mfma_f32_16x16x32, K = DOFs)
//   pointwise s_a = w_q kappa_q sum_b P_ab g_b              (FP32; P = |J| G G^T in FP64)
//   backward  y[i][c]  = sum_a sum_q G_a[q][i] s_a[q][c]    (v_mfma_f32_16x16x32, K = points)
// The forward result holds, in each lane, four consecutive points of one cell;
// the results of two forward tiles are, slot for slot, the B operand of one
// backward product (the transposed tables take their K index in that order), so
// the values go from one product to the next in registers.  u enters as
// eight consecutive DOFs per lane, y leaves as four consecutive DOFs per lane
// (each cell's block is contiguous in HBM).  Only the table fragments live in LDS,
// loaded once per persistent workgroup; every wave walks its own 16-cell tiles.
// Same finite sums as the sum-factorised contractions (Sec. 3.3 eq. coeff_eval /
// eq. form_eval); the Jacobian, its inverse, determinant and the factor
// |J| G G^T stay FP64 (any affine cell, no box restriction).
//
// Modes: BF16 and FP16 round each operand once; BF16X3 splits both operands into
// three BF16 terms and sums the six products hi*hi, hi*mid, mid*hi, hi*lo,
// mid*mid, lo*hi (about 24 significand bits).
#include <algorithm>

#include "kron_common.hpp"
#include "kron_layout.hpp"
#include "mixed_kron_body.inc"

namespace sf {

using namespace kron;

namespace {

// Waves per workgroup and the register budget: 8 waves and at most 128 VGPRs (four
// waves per SIMD, two or more workgroups per CU), except the three-term split at
// n = 4, whose tables take 144 KiB of LDS (one workgroup per CU): with FP64 storage
// 8 waves of at most 256 VGPRs (two per SIMD) that load the next tile's vertices, u
// and kappa while the current one computes (4 % faster than without; at n <= 3 and
// with FP32 storage the prefetch measured no faster or slower), with FP32 storage
// 12 waves of at most 168 VGPRs (three per SIMD)
#ifndef KRON_PF
#define KRON_PF 1
#endif
template <int N, int MODE, typename IO> struct KronCfg {
    static constexpr bool BIG = MODE == SF_BF16X3 && N == 4;
    static constexpr bool PF = KRON_PF && BIG && sizeof(IO) == 8;
    static constexpr int WAVES = PF ? 8 : BIG ? 12 : 8;
    static constexpr int WPE = PF ? 2 : BIG ? 3 : 4;
};

} // namespace

template <int N, int FORM, int MODE, typename IO, int WAVES>
__global__ void __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(KronCfg<N, MODE, IO>::WPE, 8)))
    action_kron_kernel(const int64_t ncells, const double *__restrict__ vert, const IO *__restrict__ kappa,
                       const IO *__restrict__ u, IO *__restrict__ y, const uint16_t *__restrict__ kron,
                       int *__restrict__ err)
{
    using SM = KronSmem<N, FORM, MODE>;
    constexpr KronLayout K = SM::K;
    constexpr int NPL = SM::NPL;
    __shared__ __align__(16) unsigned char smem[SM::bytes];
    uint16_t *const sF = reinterpret_cast<uint16_t *>(smem);
    uint16_t *const sB = reinterpret_cast<uint16_t *>(smem + SM::off_bwd);
    float *const sW = reinterpret_cast<float *>(smem + SM::off_w);

    // ---- the fragments of the used matrices and planes, once per workgroup
    kron_stage<N, FORM, MODE, 64 * WAVES>(kron, smem);
    __syncthreads();

    const int wave = threadIdx.x >> 6;
    auto ffrag = [&](int a, int p, int i) {
        return reinterpret_cast<const u32x4 *>(sF + (a * NPL + p) * K.fwd_elems())[i];
    };
    auto bfrag = [&](int a, int p, int i) {
        return reinterpret_cast<const u32x4 *>(sB + (a * NPL + p) * K.bwd_elems())[i];
    };
    const int64_t ntiles = (ncells + 15) / 16;
    if constexpr (KronCfg<N, MODE, IO>::PF) {
        kron_tiles_prefetch<N, FORM, MODE, IO>(int64_t(blockIdx.x) * WAVES + wave, int64_t(gridDim.x) * WAVES, ntiles,
                                               ncells, ffrag, bfrag, sW, vert, kappa, u, y, err);
    } else {
        for (int64_t tile = int64_t(blockIdx.x) * WAVES + wave; tile < ntiles; tile += int64_t(gridDim.x) * WAVES)
            kron_tile<N, FORM, MODE, IO>(tile * 16, ncells, ffrag, bfrag, sW, vert, kappa, u, y, err);
    }
}

namespace {

template <int N, int FORM, int MODE, typename IO>
int launch_kron_one(const LaunchArgs &a)
{
    constexpr int WAVES = KronCfg<N, MODE, IO>::WAVES;
    static_assert(KronSmem<N, FORM, MODE>::bytes <= 160 * 1024, "LDS");
    auto kern = action_kron_kernel<N, FORM, MODE, IO, WAVES>;
    static int cache = 0;
    if (cache <= 0) {
        int per_cu = 0, ncu = 0, dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * WAVES, 0) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return SF_ERR_HIP;
        cache = std::max(1, per_cu) * std::max(1, ncu);
    }
    const int64_t ntiles = (a.ncells + 15) / 16;
    const int64_t blocks = std::min<int64_t>(cache, (ntiles + WAVES - 1) / WAVES);
    hipLaunchKernelGGL(kern, dim3(unsigned(blocks)), dim3(64 * WAVES), 0, a.stream, a.ncells, a.vert,
                       static_cast<const IO *>(a.kappa), static_cast<const IO *>(a.u), static_cast<IO *>(a.y),
                       static_cast<const uint16_t *>(a.tabkron), a.err);
    return hipGetLastError() == hipSuccess ? SF_OK : SF_ERR_HIP;
}

template <int N, int FORM, int MODE>
int launch_kron_io(const LaunchArgs &a)
{
    return a.io == SF_F64 ? launch_kron_one<N, FORM, MODE, double>(a) : launch_kron_one<N, FORM, MODE, float>(a);
}

template <int N, int FORM>
int launch_kron_mode(const LaunchArgs &a)
{
    switch (a.precision) {
    case SF_BF16: return launch_kron_io<N, FORM, SF_BF16>(a);
    case SF_FP16: return launch_kron_io<N, FORM, SF_FP16>(a);
    case SF_BF16X3: return launch_kron_io<N, FORM, SF_BF16X3>(a);
    default: return SF_ERR_UNSUPPORTED;
    }
}

template <int N>
int launch_kron_n(const LaunchArgs &a)
{
    if (a.form == SF_LAPLACE) return launch_kron_mode<N, SF_LAPLACE>(a);
    if (a.form == SF_MASS) return launch_kron_mode<N, SF_MASS>(a);
    return SF_ERR_UNSUPPORTED;
}

} // namespace

int launch_action_kron(const LaunchArgs &a)
{
    if (a.nq != a.degree + 1 || !a.tabkron) return SF_ERR_UNSUPPORTED;
    switch (a.degree + 1) {
    case 2: return launch_kron_n<2>(a);
    case 3: return launch_kron_n<3>(a);
    case 4: return launch_kron_n<4>(a);
    default: return SF_ERR_UNSUPPORTED;
    }
}

} // namespace sf

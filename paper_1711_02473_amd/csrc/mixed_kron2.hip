// Mixed-precision operator action for the scalar families at 5 <= n <= 9 points
// per axis (p = 4..8): every contraction on the matrix cores, with no LDS tensor.
//
// The interpolation of a cell splits into a dense n^2 x n^2 matrix P on axes 1
// and 2 (kron_layout.hpp) and an n x n matrix M on axis 0; the rows of an MFMA tile
// are (cell slot, i0): three cells per tile for n = 5, two for n = 6..8, one for n = 9.  Per component
// a (values, or the three reference gradients) and per 16 plane points:
//   stage 1    V[i0][q']  = sum_{i'} u[i0][i'] P_a[q'][i']    (16x16x32, K = plane DOFs)
//   stage 2    g[q0][q']  = sum_{i0} M_a[q0][i0] V[i0][q']    (16x16x16, K = axis-0 DOFs;
//                                                             BF16X3: two products per 16x16x32)
//   pointwise  s_a = w kappa sum_b P_ab g_b                   (FP32; P = |J| G G^T in FP64)
//   stage 2^T  t[q'][i0]  = sum_{q0} s_a[q0][q'] M_a[q0][i0]  (16x16x16, K = axis-0 points)
//   stage 1^T  y[i'][i0] += sum_{q'} P_a[q'][i'] t[q'][i0]    (16x16x32, K = plane points)
// Each product's result is, in its lane layout, the operand the next one takes (the
// D layout of a 16 x 16 tile is the B layout of its rows and the A layout of its
// transpose), so the values stay in registers from the u load to the y store; u
// enters as eight consecutive DOFs per lane and y leaves as four.  Only the table
// fragments live in LDS, loaded once per persistent workgroup.  Same finite sums as
// the one-axis contractions (Sec. 3.3 eq. coeff_eval / eq. form_eval), grouped two
// axes and one; geometry in FP64 for any affine cell.
//
// Modes as in the n <= 4 kernel: BF16 / FP16 single term, BF16X3 six products of
// three-term splits.  BF16X3 at n = 9 would need 324 KiB of tables and is left to
// the sum-factorised kernel.
#include <algorithm>

#include "kron_common.hpp"
#include "kron_layout.hpp"
#include "mixed_kron2_body.inc"

namespace sf {

using namespace kron;

namespace {

// Workgroup shape and register budget.  Except in the three-term split at n = 5 with
// FP32 storage, the next tile's u is loaded while the current one computes, and at
// n = 9 (single term), at n = 5 with FP32 storage (single term) and in the other
// three-term cases the next tile's kappa as well.  Budgets: 168 VGPRs (three waves per SIMD) for the single-term modes at
// n = 5..8 and the three-term split at n = 5 with FP32 storage, 256 (two) for the rest,
// where the prefetched u and kappa cover the load latency that more waves without them
// did not (64^3 cells, FP64 storage: n = 9 single term 1.83 -> 1.25 ms; three-term
// split at n = 5..8 9-22 % faster than at three waves per SIMD without prefetch).
// Twelve waves per workgroup where three per SIMD fit and one workgroup holds the CU,
// and for the three-term split at n = 5 with FP32 storage; the single-term modes
// (HBM-bound) were faster with eight.
#ifndef KRON2_PF
#define KRON2_PF 1
#endif
template <int N, int FORM, int MODE, typename IO> struct K2Cfg {
    static constexpr bool X3 = MODE == SF_BF16X3;
    static constexpr bool XPF = X3 && KRON2_PF && (sizeof(IO) == 8 || N >= 6); // three-term prefetch
    static constexpr bool KPF = (!X3 && KRON2_PF && (N == 9 || (N == 5 && sizeof(IO) == 4))) || XPF;
    static constexpr bool PF = (!X3 && KRON2_PF) || XPF;
    static constexpr bool BIG = K2Smem<N, FORM, MODE>::bytes > 80 * 1024;
    static constexpr int WPE = (N == 9 && PF) || XPF ? 2 : (X3 || PF ? 3 : 4);
    static constexpr int WAVES = WPE == 2 ? 8 : BIG ? (WPE == 3 ? 12 : 16) : (X3 ? 12 : 8);
};

} // namespace

template <int N, int FORM, int MODE, typename IO, int WAVES>
__global__ void __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(K2Cfg<N, FORM, MODE, IO>::WPE, 8)))
    action_kron2_kernel(const int64_t ncells, const double *__restrict__ vert, const IO *__restrict__ kappa,
                        const IO *__restrict__ u, IO *__restrict__ y, const uint16_t *__restrict__ tab,
                        int *__restrict__ err)
{
    constexpr int CPT = Kron2Layout(N).cpt;
    __shared__ __align__(16) unsigned char smem[K2Smem<N, FORM, MODE>::bytes];
    const auto tabs = Kron2LdsTables<N, FORM, MODE>::at(smem);
    // ---- tables into LDS, once per workgroup
    kron2_stage<N, FORM, MODE, 64 * WAVES>(tab, smem);
    __syncthreads();

    const int wave = threadIdx.x >> 6;
    // a batch is the cells of 16 / CPT tiles (16, or 15 with three cells per tile)
    constexpr int BATCH = CPT * (16 / CPT);
    const int64_t nbatch = (ncells + BATCH - 1) / BATCH;
    for (int64_t bt = int64_t(blockIdx.x) * WAVES + wave; bt < nbatch; bt += int64_t(gridDim.x) * WAVES) {
        kron2_batch<N, FORM, MODE, IO, K2Cfg<N, FORM, MODE, IO>::PF, decltype(tabs), K2Cfg<N, FORM, MODE, IO>::KPF>(bt * BATCH, ncells, tabs, vert, kappa, u, y, err);
    }
}

namespace {

template <int N, int FORM, int MODE, typename IO>
int launch_kron2_one(const LaunchArgs &a)
{
    constexpr int WAVES = K2Cfg<N, FORM, MODE, IO>::WAVES;
    static_assert(K2Smem<N, FORM, MODE>::bytes <= 160 * 1024, "LDS");
    auto kern = action_kron2_kernel<N, FORM, MODE, IO, WAVES>;
    static int cache = 0;
    if (cache <= 0) {
        int per_cu = 0, ncu = 0, dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * WAVES, 0) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return SF_ERR_HIP;
        cache = std::max(1, per_cu) * std::max(1, ncu);
    }
    constexpr int BATCH = Kron2Layout(N).cpt * (16 / Kron2Layout(N).cpt);
    const int64_t nbatch = (a.ncells + BATCH - 1) / BATCH;
    const int64_t blocks = std::min<int64_t>(cache, (nbatch + WAVES - 1) / WAVES);
    hipLaunchKernelGGL(kern, dim3(unsigned(blocks)), dim3(64 * WAVES), 0, a.stream, a.ncells, a.vert,
                       static_cast<const IO *>(a.kappa), static_cast<const IO *>(a.u), static_cast<IO *>(a.y),
                       static_cast<const uint16_t *>(a.tabkron), a.err);
    return hipGetLastError() == hipSuccess ? SF_OK : SF_ERR_HIP;
}

template <int N, int FORM, int MODE>
int launch_kron2_io(const LaunchArgs &a)
{
    if constexpr (K2Smem<N, FORM, MODE>::bytes > 160 * 1024) {
        return SF_ERR_UNSUPPORTED; // tables larger than LDS: the sum-factorised kernel
    } else {
        return a.io == SF_F64 ? launch_kron2_one<N, FORM, MODE, double>(a)
                              : launch_kron2_one<N, FORM, MODE, float>(a);
    }
}

template <int N, int FORM>
int launch_kron2_mode(const LaunchArgs &a)
{
    switch (a.precision) {
    case SF_BF16: return launch_kron2_io<N, FORM, SF_BF16>(a);
    case SF_FP16: return launch_kron2_io<N, FORM, SF_FP16>(a);
    case SF_BF16X3: return launch_kron2_io<N, FORM, SF_BF16X3>(a);
    default: return SF_ERR_UNSUPPORTED;
    }
}

template <int N>
int launch_kron2_n(const LaunchArgs &a)
{
    if (a.form == SF_LAPLACE) return launch_kron2_mode<N, SF_LAPLACE>(a);
    if (a.form == SF_MASS) return launch_kron2_mode<N, SF_MASS>(a);
    return SF_ERR_UNSUPPORTED;
}

} // namespace

int launch_action_kron2(const LaunchArgs &a)
{
    if (a.nq != a.degree + 1 || !a.tabkron) return SF_ERR_UNSUPPORTED;
    switch (a.degree + 1) {
    case 5: return launch_kron2_n<5>(a);
    case 6: return launch_kron2_n<6>(a);
    case 7: return launch_kron2_n<7>(a);
    case 8: return launch_kron2_n<8>(a);
    case 9: return launch_kron2_n<9>(a);
    default: return SF_ERR_UNSUPPORTED;
    }
}

} // namespace sf

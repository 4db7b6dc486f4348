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

namespace sf {

using namespace kron;

namespace {

// LDS of one workgroup: the fragments of the matrices the form uses and the 3-D weights
template <int N, int FORM, int MODE> struct KronSmem {
    static constexpr KronLayout K = KronLayout(N);
    static constexpr int NMAT = FORM == SF_LAPLACE ? 3 : 1;
    static constexpr int NPL = KronMode<MODE>::NPL;
    static constexpr int fwd_u16 = NMAT * NPL * K.fwd_elems(), bwd_u16 = NMAT * NPL * K.bwd_elems();
    static constexpr int off_bwd = fwd_u16 * 2, off_w = off_bwd + bwd_u16 * 2;
    static constexpr int bytes = off_w + K.MT * 16 * 4;
};

// Waves per workgroup and the register budget: 8 waves and at most 128 VGPRs (four
// waves per SIMD, two or more workgroups per CU), except the three-term split at
// n = 4, whose tables take 144 KiB of LDS (one workgroup per CU): 12 waves of at most
// 168 VGPRs (three per SIMD)
template <int N, int MODE> struct KronCfg {
    static constexpr bool BIG = MODE == SF_BF16X3 && N == 4;
    static constexpr int WAVES = BIG ? 12 : 8;
    static constexpr int WPE = BIG ? 3 : 4;
};

} // namespace

template <int N, int FORM, int MODE, typename IO, int WAVES>
__global__ void __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(KronCfg<N, MODE>::WPE, 8)))
    action_kron_kernel(const int64_t ncells, const double *__restrict__ vert, const IO *__restrict__ kappa,
                       const IO *__restrict__ u, IO *__restrict__ y, const uint16_t *__restrict__ kron,
                       int *__restrict__ err)
{
    using SM = KronSmem<N, FORM, MODE>;
    constexpr KronLayout K = SM::K;
    constexpr int ND = K.nd, MT = K.MT, MT2 = K.MT2, KS = K.KS, NTL = K.NT;
    constexpr int NMAT = SM::NMAT, NPL = SM::NPL, NPROD = KronMode<MODE>::NPROD;
    constexpr int MAT0 = FORM == SF_LAPLACE ? 1 : 0; // first table matrix the form uses
    __shared__ __align__(16) unsigned char smem[SM::bytes];
    uint16_t *const sF = reinterpret_cast<uint16_t *>(smem);
    uint16_t *const sB = reinterpret_cast<uint16_t *>(smem + SM::off_bwd);
    float *const sW = reinterpret_cast<float *>(smem + SM::off_w);

    // ---- the fragments of the used matrices and planes, once per workgroup: every
    // thread issues all of its 16-byte loads before the first LDS store
    {
        constexpr int FW = K.fwd_elems() / 8, BW = K.bwd_elems() / 8; // 16-byte words per block
        constexpr int NBLK = NMAT * NPL, TOT = NBLK * (FW + BW), R = (TOT + 64 * WAVES - 1) / (64 * WAVES);
        uint4 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            int t = int(threadIdx.x) + r * 64 * WAVES;
            t = t < TOT ? t : TOT - 1;
            const bool fw = t < NBLK * FW;
            const int tt = fw ? t : t - NBLK * FW;
            const int mp = fw ? tt / FW : tt / BW, e = fw ? tt % FW : tt % BW;
            const int mat = MAT0 + mp / NPL, pl = NPL == 1 ? KronMode<MODE>::PLANE0 : mp % NPL;
            v[r] = reinterpret_cast<const uint4 *>(kron + (fw ? K.fwd(mat, pl) : K.bwd(mat, pl)))[e];
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int t = int(threadIdx.x) + r * 64 * WAVES;
            if (t < TOT) reinterpret_cast<uint4 *>(smem)[t] = v[r]; // sF then sB, contiguous
        }
    }
    for (int t = threadIdx.x; t < MT * 16; t += 64 * WAVES) sW[t] = reinterpret_cast<const float *>(kron + K.w3())[t];
    __syncthreads();

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
    const int64_t ntiles = (ncells + 15) / 16;
    for (int64_t tile = int64_t(blockIdx.x) * WAVES + wave; tile < ntiles; tile += int64_t(gridDim.x) * WAVES) {
        {
            const int64_t cell = tile * 16 + col;
            const bool live = cell < ncells;
            // every load of the tile is unconditional, so all are in flight at once:
            // columns past the last cell read the last cell, DOFs and points past nd the
            // last one; those u values are replaced by zero, those kappa values meet a
            // zero weight
            const int64_t cl = live ? cell : ncells - 1;
            // ---- FP64 geometry of the tile's cells (four lanes per cell)
            float P[6];
            cell_factor<FORM>(vert, cl, live, col, g, err, P);
            __builtin_amdgcn_sched_barrier(0);
            // ---- this lane's u fragments: DOFs 32 s + 8 g + j of cell `col`, split into terms
            u32x4 ub[KS][NPL];
#pragma unroll
            for (int s = 0; s < KS; ++s)
#pragma unroll
                for (int j = 0; j < 8; j += 2) {
                    float x[2];
#pragma unroll
                    for (int e = 0; e < 2; ++e) {
                        const int i = 32 * s + 8 * g + j + e;
                        const float v = float(to_d(u[cl * ND + (i < ND ? i : ND - 1)]));
                        x[e] = (live && i < ND) ? v : 0.0f;
                    }
                    uint32_t t[3];
                    terms2<MODE>(x[0], x[1], t);
#pragma unroll
                    for (int p = 0; p < NPL; ++p) ub[s][p][j / 2] = t[p];
                }

            f32x4 yacc[NTL];
#pragma unroll
            for (int t = 0; t < NTL; ++t) yacc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int m2 = 0; m2 < MT2; ++m2) {
                // the results of the forward m-tiles 2 m2 and 2 m2 + 1 form, slot for slot,
                // the B operand of one K = 32 backward product (slots 0-3 and 4-7)
                u32x4 sb[NMAT][NPL];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int m = 2 * m2 + h;
                    if (m >= MT) {
#pragma unroll
                        for (int a = 0; a < NMAT; ++a)
#pragma unroll
                            for (int p = 0; p < NPL; ++p)
#pragma unroll
                                for (int j = 0; j < 2; ++j) sb[a][p][2 * h + j] = 0u;
                        continue;
                    }
                    // ---- forward: this m-tile's points for every matrix of the form
                    f32x4 gacc[NMAT];
#pragma unroll
                    for (int a = 0; a < NMAT; ++a) {
                        gacc[a] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                        for (int s = 0; s < KS; ++s) {
                            u32x4 af[NPL];
#pragma unroll
                            for (int p = 0; p < NPL; ++p)
                                af[p] = reinterpret_cast<const u32x4 *>(
                                    sF + (a * NPL + p) * K.fwd_elems())[(m * KS + s) * 64 + lane];
#pragma unroll
                            for (int q = 0; q < NPROD; ++q)
                                gacc[a] = mfma32<MODE>(af[prod_a(q)], ub[s][prod_b(q)], gacc[a]);
                        }
                    }
                    // ---- pointwise on this lane's four points q = 16 m + 4 g + j of cell `col`
                    float kq[4];
                    if (kappa == nullptr) {
#pragma unroll
                        for (int j = 0; j < 4; ++j) kq[j] = 1.0f;
                    } else if constexpr (ND == 16 * MT) {
                        // every point of the tile exists (n = 4): four consecutive points of
                        // the cell, one vector load
                        const IO *kp = kappa + cl * ND + 16 * m + 4 * g;
#pragma unroll
                        for (int j = 0; j < 4; ++j) kq[j] = float(to_d(kp[j]));
                    } else {
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const int q = 16 * m + 4 * g + j;
                            kq[j] = float(to_d(kappa[cl * ND + (q < ND ? q : ND - 1)]));
                        }
                    }
#pragma unroll
                    for (int j = 0; j < 4; j += 2) {
                        float sv[2][NMAT];
#pragma unroll
                        for (int e = 0; e < 2; ++e) {
                            const int q = 16 * m + 4 * g + j + e;
                            const float om = sW[q] * kq[j + e]; // zero past the last point
                            if constexpr (FORM == SF_LAPLACE) {
                                const float gx = gacc[0][j + e], gy = gacc[1][j + e], gz = gacc[2][j + e];
                                sv[e][0] = om * (P[0] * gx + P[1] * gy + P[2] * gz);
                                sv[e][1] = om * (P[1] * gx + P[3] * gy + P[4] * gz);
                                sv[e][2] = om * (P[2] * gx + P[4] * gy + P[5] * gz);
                            } else {
                                sv[e][0] = om * P[0] * gacc[0][j + e];
                            }
                        }
#pragma unroll
                        for (int a = 0; a < NMAT; ++a) {
                            uint32_t t[3];
                            terms2<MODE>(sv[0][a], sv[1][a], t);
#pragma unroll
                            for (int p = 0; p < NPL; ++p) sb[a][p][2 * h + j / 2] = t[p];
                        }
                    }
                    if constexpr (NPL > 1) __builtin_amdgcn_sched_barrier(0);
                }
                // ---- backward: these 32 points' share of every DOF tile
#pragma unroll
                for (int t = 0; t < NTL; ++t) {
#pragma unroll
                    for (int a = 0; a < NMAT; ++a) {
                        u32x4 bf[NPL];
#pragma unroll
                        for (int p = 0; p < NPL; ++p)
                            bf[p] = reinterpret_cast<const u32x4 *>(
                                sB + (a * NPL + p) * K.bwd_elems())[(t * MT2 + m2) * 64 + lane];
#pragma unroll
                        for (int q = 0; q < NPROD; ++q)
                            yacc[t] = mfma32<MODE>(bf[prod_a(q)], sb[a][prod_b(q)], yacc[t]);
                    }
                }
                __builtin_amdgcn_sched_barrier(0); // one pair's registers at a time
            }
            // ---- y: this lane's four consecutive DOFs 16 t + 4 g + j of cell `col`
            if (live) {
#pragma unroll
                for (int t = 0; t < NTL; ++t)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int i = 16 * t + 4 * g + j;
                        if (i < ND) y[cell * ND + i] = IO(yacc[t][j]);
                    }
            }
        }
    }
}

namespace {

template <int N, int FORM, int MODE, typename IO>
int launch_kron_one(const LaunchArgs &a)
{
    constexpr int WAVES = KronCfg<N, MODE>::WAVES;
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

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

namespace sf {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short s16x8 __attribute__((ext_vector_type(8)));

// Mixed table block (host-built, see api.cpp): for each of the matrices
// B [nq][n], Dh [nq][nq], B^T [n][nq], Dh^T [nq][nq], four 16x16 uint16 planes:
// bf16 hi, bf16 mid, bf16 lo, fp16.
constexpr int kMixPlane = 256;
constexpr int kMixMat = 4 * kMixPlane;
enum { MIX_B = 0, MIX_DH = 1, MIX_BT = 2, MIX_DHT = 3 };

template <int MODE> struct MixMode {
    static constexpr int NM = (MODE == SF_BF16X3) ? 2 : 1;
    static constexpr bool F16 = (MODE == SF_FP16);
};

// term of the A operand (table) / B operand (data) in MFMA m, slot s (BF16X3)
__device__ __forceinline__ int a_term(int m, int s) { return m == 0 ? s : (s == 2 ? 0 : s); }
__device__ __forceinline__ int b_term(int m, int s) { return m == 0 ? 0 : (s == 2 ? 2 : 1); }

struct Frag {
    s16x8 v[2];
};

// A-operand fragment of a table for this lane (row r = lane % 16, k-group g)
template <int MODE, int NO, int NI>
__device__ inline Frag load_frag(const uint16_t *__restrict__ mat)
{
    const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
    Frag f;
#pragma unroll
    for (int m = 0; m < MixMode<MODE>::NM; ++m) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = 8 * g + j;
            uint16_t val = 0;
            if constexpr (MODE == SF_BF16X3) {
                const int s = k / NI, e = k - s * NI;
                if (r < NO && s < 3) val = mat[a_term(m, s) * kMixPlane + r * 16 + e];
            } else {
                const int plane = MixMode<MODE>::F16 ? 3 : 0;
                if (r < NO && k < NI) val = mat[plane * kMixPlane + r * 16 + k];
            }
            f.v[m][j] = short(val);
        }
    }
    return f;
}

__device__ __forceinline__ void split3(float x, __bf16 &hi, __bf16 &mid, __bf16 &lo)
{
    hi = __bf16(x);
    const float r1 = x - float(hi);
    mid = __bf16(r1);
    lo = __bf16(r1 - float(mid));
}

// One contraction stage over all pencils of the workgroup: for every pencil
// (cell, a, b) along axis AX, out[q] (+)= sum_i M[q][i] in[i], q < NO, i < NI,
// read from src and written to dst (FP32 LDS tensors, strides S1, S2, CS).
template <int MODE, int NO, int NI, int AX, int P0, int P1, int C, int NT, int S1, int S2, int CS, bool ACC>
__device__ inline void mfma_stage(const float *src, float *dst, const Frag &A)
{
    constexpr int NPEN = C * P0 * P1;
    constexpr int NTILE = (NPEN + 15) / 16;
    constexpr int ST = AX == 0 ? S1 : (AX == 1 ? S2 : 1);
    const int lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
    for (int tile = threadIdx.x >> 6; tile < NTILE; tile += NT / 64) {
        const int p = tile * 16 + col;
        const bool live = p < NPEN;
        const int pp = live ? p : 0;
        const int c = pp / (P0 * P1), rr = pp - c * (P0 * P1), a = rr / P1, b = rr - a * P1;
        const int base = c * CS + (AX == 0 ? a * S2 + b : (AX == 1 ? a * S1 + b : a * S1 + b * S2));
        s16x8 bop[2];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = 8 * g + j;
            if constexpr (MODE == SF_BF16X3) {
                const int s = k / NI, e = k - s * NI;
                const bool ok = live && s < 3;
                const float x = ok ? src[base + (ok ? e : 0) * ST] : 0.0f;
                __bf16 hi, mid, lo;
                split3(x, hi, mid, lo);
                const __bf16 t1 = (s == 2) ? lo : mid;
                bop[0][j] = __builtin_bit_cast(short, hi);
                bop[1][j] = __builtin_bit_cast(short, t1);
            } else {
                const bool ok = live && k < NI;
                const float x = ok ? src[base + (ok ? k : 0) * ST] : 0.0f;
                if constexpr (MixMode<MODE>::F16) bop[0][j] = __builtin_bit_cast(short, _Float16(x));
                else bop[0][j] = __builtin_bit_cast(short, __bf16(x));
            }
        }
        f32x4 d;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int q = 4 * g + j;
            d[j] = (ACC && live && q < NO) ? dst[base + q * ST] : 0.0f;
        }
#pragma unroll
        for (int m = 0; m < MixMode<MODE>::NM; ++m) {
            if constexpr (MixMode<MODE>::F16)
                d = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, A.v[m]),
                                                           __builtin_bit_cast(f16x8, bop[m]), d, 0, 0, 0);
            else
                d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, A.v[m]),
                                                            __builtin_bit_cast(bf16x8, bop[m]), d, 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int q = 4 * g + j;
            if (live && q < NO) dst[base + q * ST] = d[j];
        }
    }
}

template <int N, int NQ, int FORM, bool COLL, int MODE, typename IO, int C, int NT>
__global__ void __launch_bounds__(NT)
    action_mixed_kernel(const int64_t ncells, const double *__restrict__ vert, const IO *__restrict__ kappa,
                        const IO *__restrict__ u, IO *__restrict__ y, const double *__restrict__ tab64,
                        const uint16_t *__restrict__ mix, int *__restrict__ err)
{
    using L = Lds3<NQ>;
    constexpr int S1 = L::S1, S2 = L::S2, CS = L::CS;
    constexpr int NBUF = (FORM == SF_LAPLACE) ? 4 : 1;
    constexpr int N3 = N * N * N, NQ3 = NQ * NQ * NQ;
    constexpr TabLayout TL(N, 0, NQ);

    __shared__ float lds[NBUF * C * CS];
    __shared__ double sP[C][6];
    __shared__ float sW[NQ];

    const int64_t cell0 = int64_t(blockIdx.x) * C;
    const bool has_kappa = kappa != nullptr;

    if (threadIdx.x < NQ) sW[threadIdx.x] = float(tab64[TL.W() + threadIdx.x]);
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
    // register-resident A fragments of the 1-D matrices
    Frag fB, fBT, fD, fDT;
    if constexpr (!COLL) {
        fB = load_frag<MODE, NQ, N>(mix + MIX_B * kMixMat);
        fBT = load_frag<MODE, N, NQ>(mix + MIX_BT * kMixMat);
    }
    if constexpr (FORM == SF_LAPLACE) {
        fD = load_frag<MODE, NQ, NQ>(mix + MIX_DH * kMixMat);
        fDT = load_frag<MODE, NQ, NQ>(mix + MIX_DHT * kMixMat);
    }
    float *L0 = lds;
    float *L1 = lds + 1 * C * CS;
    float *L2 = lds + 2 * C * CS;
    float *L3 = lds + 3 * C * CS;

    // ---- stage the local coefficients (coalesced), FP32 in LDS
    for (int t = threadIdx.x; t < C * N3; t += NT) {
        const int c = t / N3, r = t - c * N3;
        const int i0 = r / (N * N), i1 = (r / N) % N, i2 = r % N;
        const int64_t gc = cell0 + c;
        L0[c * CS + i0 * S1 + i1 * S2 + i2] = gc < ncells ? float(to_d(u[gc * N3 + r])) : 0.0f;
    }
    __syncthreads();
    // ---- interpolation to the Gauss points: x, y, z
    if constexpr (!COLL) {
        mfma_stage<MODE, NQ, N, 0, N, N, C, NT, S1, S2, CS, false>(L0, L0, fB);
        __syncthreads();
        mfma_stage<MODE, NQ, N, 1, NQ, N, C, NT, S1, S2, CS, false>(L0, L0, fB);
        __syncthreads();
        mfma_stage<MODE, NQ, N, 2, NQ, NQ, C, NT, S1, S2, CS, false>(L0, L0, fB);
        __syncthreads();
    }
    if constexpr (FORM == SF_LAPLACE) {
        // ---- reference gradient with the collocated derivative
        mfma_stage<MODE, NQ, NQ, 0, NQ, NQ, C, NT, S1, S2, CS, false>(L0, L3, fD);
        mfma_stage<MODE, NQ, NQ, 1, NQ, NQ, C, NT, S1, S2, CS, false>(L0, L2, fD);
        mfma_stage<MODE, NQ, NQ, 2, NQ, NQ, C, NT, S1, S2, CS, false>(L0, L1, fD);
        __syncthreads();
        // ---- pointwise: v = w kappa |J| G G^T g (factor assembled in FP64)
        for (int t = threadIdx.x; t < C * NQ3; t += NT) {
            const int c = t / NQ3, r = t - c * NQ3;
            const int q0 = r / (NQ * NQ), q1 = (r / NQ) % NQ, q2 = r % NQ;
            const int64_t gc = cell0 + c;
            const int o = c * CS + q0 * S1 + q1 * S2 + q2;
            float om = sW[q0] * sW[q1] * sW[q2];
            if (has_kappa && gc < ncells) om *= float(to_d(kappa[gc * NQ3 + r]));
            const float gx = L3[o], gy = L2[o], gz = L1[o];
            const float p00 = float(sP[c][0]), p01 = float(sP[c][1]), p02 = float(sP[c][2]);
            const float p11 = float(sP[c][3]), p12 = float(sP[c][4]), p22 = float(sP[c][5]);
            L3[o] = om * (p00 * gx + p01 * gy + p02 * gz);
            L2[o] = om * (p01 * gx + p11 * gy + p12 * gz);
            L1[o] = om * (p02 * gx + p12 * gy + p22 * gz);
        }
        __syncthreads();
        // ---- transposed derivative: w = Dh_x^T v_x + Dh_y^T v_y + Dh_z^T v_z
        mfma_stage<MODE, NQ, NQ, 0, NQ, NQ, C, NT, S1, S2, CS, false>(L3, L0, fDT);
        __syncthreads();
        mfma_stage<MODE, NQ, NQ, 1, NQ, NQ, C, NT, S1, S2, CS, true>(L2, L0, fDT);
        __syncthreads();
        mfma_stage<MODE, NQ, NQ, 2, NQ, NQ, C, NT, S1, S2, CS, true>(L1, L0, fDT);
        __syncthreads();
    } else {
        for (int t = threadIdx.x; t < C * NQ3; t += NT) {
            const int c = t / NQ3, r = t - c * NQ3;
            const int q0 = r / (NQ * NQ), q1 = (r / NQ) % NQ, q2 = r % NQ;
            const int64_t gc = cell0 + c;
            const int o = c * CS + q0 * S1 + q1 * S2 + q2;
            float om = sW[q0] * sW[q1] * sW[q2] * float(sP[c][0]);
            if (has_kappa && gc < ncells) om *= float(to_d(kappa[gc * NQ3 + r]));
            L0[o] *= om;
        }
        __syncthreads();
    }
    // ---- back to the local DOFs: z, y, x
    if constexpr (!COLL) {
        mfma_stage<MODE, N, NQ, 2, NQ, NQ, C, NT, S1, S2, CS, false>(L0, L0, fBT);
        __syncthreads();
        mfma_stage<MODE, N, NQ, 1, NQ, N, C, NT, S1, S2, CS, false>(L0, L0, fBT);
        __syncthreads();
        mfma_stage<MODE, N, NQ, 0, N, N, C, NT, S1, S2, CS, false>(L0, L0, fBT);
        __syncthreads();
    }
    for (int t = threadIdx.x; t < C * N3; t += NT) {
        const int c = t / N3, r = t - c * N3;
        const int i0 = r / (N * N), i1 = (r / N) % N, i2 = r % N;
        const int64_t gc = cell0 + c;
        if (gc < ncells) y[gc * N3 + r] = IO(L0[c * CS + i0 * S1 + i1 * S2 + i2]);
    }
}

namespace {

template <int N, int FORM, bool COLL, int MODE, typename IO>
int launch_one(const LaunchArgs &a)
{
    constexpr int NQ = N;
    constexpr int NBUF = (FORM == SF_LAPLACE) ? 4 : 1;
    constexpr int CS = Lds3<NQ>::CS;
    constexpr int C0 = (40 * 1024) / (NBUF * CS * 4);
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
    const bool coll = a.family == SF_DQ;
    if (a.form == SF_LAPLACE) return coll ? launch_mode<N, SF_LAPLACE, true>(a) : launch_mode<N, SF_LAPLACE, false>(a);
    if (a.form == SF_MASS) return coll ? launch_mode<N, SF_MASS, true>(a) : launch_mode<N, SF_MASS, false>(a);
    return SF_ERR_UNSUPPORTED;
}

} // namespace

int launch_action_mixed(const LaunchArgs &a)
{
    if (a.family != SF_Q && a.family != SF_DQ) return SF_ERR_UNSUPPORTED;
    if (a.nq != a.degree + 1 || !a.tabmix) return SF_ERR_UNSUPPORTED;
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

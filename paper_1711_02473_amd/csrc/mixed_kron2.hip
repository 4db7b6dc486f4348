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

namespace sf {

using namespace kron;

namespace {

// LDS of one workgroup: the plane-matrix fragments (forward, then transposed) of the
// components the form uses, the axis-0 fragments, the plane and axis-0 weights
template <int N, int FORM, int MODE> struct K2Smem {
    static constexpr Kron2Layout K = Kron2Layout(N);
    static constexpr int NMAT = FORM == SF_LAPLACE ? 3 : 1; // plane matrices (one per component)
    static constexpr int NAM = FORM == SF_LAPLACE ? 2 : 1;  // axis-0 matrices B (and D)
    static constexpr int NPL = KronMode<MODE>::NPL;
    static constexpr int s1f_u16 = NMAT * NPL * K.s1f_elems(), s1b_u16 = NMAT * NPL * K.s1b_elems();
    static constexpr int s2_u16 = NAM * NPL * 512;
    static constexpr int off_s1b = 2 * s1f_u16, off_s2 = off_s1b + 2 * s1b_u16, off_w2 = off_s2 + 2 * s2_u16;
    static constexpr int off_w0 = off_w2 + 4 * 16 * K.NQ;
    static constexpr int bytes = off_w0 + 4 * 16;
};

// Workgroup shape: at most 128 VGPRs (single term) or 168 (three-term split), and
// more waves per workgroup where the tables allow only one workgroup per CU
#ifndef KRON2_PF
#define KRON2_PF 1
#endif
template <int N, int FORM, int MODE, typename IO> struct K2Cfg {
    static constexpr bool X3 = MODE == SF_BF16X3;
    // load the next tile's u during the current one (not where the registers run out:
    // the three-term split, FP64 storage at n = 9)
    static constexpr bool PF = !X3 && !(N == 9 && sizeof(IO) == 8) && KRON2_PF;
    static constexpr bool BIG = K2Smem<N, FORM, MODE>::bytes > 80 * 1024;
    static constexpr int WPE = X3 || PF ? 3 : 4; // FP64 storage at n = 9: occupancy over the spill
    static constexpr int WAVES = BIG ? (WPE == 3 ? 12 : 16) : 8;
};

// the axis-0 matrix of component a: D for the axis-0 gradient, B otherwise
template <int FORM> __device__ __forceinline__ constexpr int am_of(int a)
{
    return FORM == SF_LAPLACE && a == 0 ? 1 : 0;
}

} // namespace

template <int N, int FORM, int MODE, typename IO, int WAVES>
__global__ void __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(K2Cfg<N, FORM, MODE, IO>::WPE, 8)))
    action_kron2_kernel(const int64_t ncells, const double *__restrict__ vert, const IO *__restrict__ kappa,
                        const IO *__restrict__ u, IO *__restrict__ y, const uint16_t *__restrict__ tab,
                        int *__restrict__ err)
{
    using SM = K2Smem<N, FORM, MODE>;
    constexpr Kron2Layout K = SM::K;
    constexpr int Q2 = K.q2, N3 = N * Q2, CPT = K.cpt, RS = K.rs, NQ = K.NQ, KS = K.KS, NQ2 = K.NQ2;
    constexpr int NMAT = SM::NMAT, NAM = SM::NAM, NPL = SM::NPL, NPROD = KronMode<MODE>::NPROD;
    constexpr int PL0 = KronMode<MODE>::PLANE0;
    __shared__ __align__(16) unsigned char smem[SM::bytes];
    const uint16_t *const s1f = reinterpret_cast<const uint16_t *>(smem);
    const uint16_t *const s1b = reinterpret_cast<const uint16_t *>(smem + SM::off_s1b);
    const uint16_t *const s2 = reinterpret_cast<const uint16_t *>(smem + SM::off_s2);
    const float *const sW2 = reinterpret_cast<const float *>(smem + SM::off_w2);
    const float *const sW0 = reinterpret_cast<const float *>(smem + SM::off_w0);

    // ---- tables into LDS, once per workgroup; each thread issues all of its loads of
    // a section before its stores.  LDS order: s1f [a][plane], s1b [a][plane],
    // s2 [axis-0 matrix][plane] (s2f then s2b), plane weights, axis-0 weights.
    {
        constexpr int W1F = K.s1f_elems() / 8, W1B = K.s1b_elems() / 8; // 16-byte words per block
        constexpr int T1 = NMAT * NPL * (W1F + W1B), T2 = NAM * NPL * 64, TW = (16 * NQ + 16) / 4;
        constexpr int TOT = T1 + T2 + TW, R = (TOT + 64 * WAVES - 1) / (64 * WAVES);
        uint4 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            int t = int(threadIdx.x) + r * 64 * WAVES;
            t = t < TOT ? t : TOT - 1;
            int src; // uint16 offset of the word in the global block
            if (t < NMAT * NPL * W1F) {
                const int mp = t / W1F, e = t % W1F;
                src = K.s1f(mp / NPL, NPL == 1 ? PL0 : mp % NPL) + 8 * e;
            } else if (t < T1) {
                const int tt = t - NMAT * NPL * W1F, mp = tt / W1B, e = tt % W1B;
                src = K.s1b(mp / NPL, NPL == 1 ? PL0 : mp % NPL) + 8 * e;
            } else if (t < T1 + T2) {
                const int tt = t - T1, mp = tt / 64, e = tt % 64;
                src = K.s2f(mp / NPL, NPL == 1 ? PL0 : mp % NPL) + 8 * e;
            } else {
                src = K.w2() + 8 * (t - T1 - T2); // w2 and w0 are contiguous
            }
            v[r] = *reinterpret_cast<const uint4 *>(tab + src);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int t = int(threadIdx.x) + r * 64 * WAVES;
            if (t < TOT) reinterpret_cast<uint4 *>(smem)[t] = v[r];
        }
    }
    __syncthreads();

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
    // a batch is the cells of 16 / CPT tiles (16, or 15 with three cells per tile)
    constexpr int UPB = 16 / CPT, BATCH = CPT * UPB;
    // with RS = 5 a lane's four result rows 4 g + j may belong to two cells
    constexpr bool ROWP = RS % 4 != 0;
    const int64_t nbatch = (ncells + BATCH - 1) / BATCH;
    for (int64_t bt = int64_t(blockIdx.x) * WAVES + wave; bt < nbatch; bt += int64_t(gridDim.x) * WAVES) {
        // ---- FP64 geometry of the batch's 16 cells, four lanes per cell (cell 16 bt + col)
        float Pm[6];
        {
            const int64_t c = bt * BATCH + col;
            const bool live = col < BATCH && c < ncells;
            cell_factor<FORM>(vert, live ? c : ncells - 1, live, col, g, err, Pm);
        }
        __builtin_amdgcn_sched_barrier(0);
        const int64_t left = ncells - bt * BATCH;
        const int nunit = left >= BATCH ? UPB : int((left + CPT - 1) / CPT);
        // every load is unconditional: rows past the cells, DOFs and points past the cell
        // read inside the last cell; those u values become zero, those kappa values meet
        // a zero weight.  u as the A operand of stage 1: row col = (slot, i0), DOFs
        // 32 ks + 8 g + j.  Single-term modes load the next tile's u while the current
        // one computes (registers the three-term split does not have).
        constexpr bool PF = K2Cfg<N, FORM, MODE, IO>::PF;
        const int uslot = col / RS, ui0 = col % RS;
        auto load_u = [&](int kk, IO (&raw)[KS][8]) {
            const int64_t cell = bt * BATCH + int64_t(CPT) * kk + uslot;
            const IO *ur = u + (cell < ncells ? cell : ncells - 1) * N3 + (ui0 < N ? ui0 : N - 1) * Q2;
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int i = 32 * ks + 8 * g + j;
                    raw[ks][j] = ur[i < Q2 ? i : Q2 - 1];
                }
        };
        IO uraw[KS][8];
        if constexpr (PF) load_u(0, uraw);
#pragma unroll 1
        for (int k = 0; k < nunit; ++k) {
            const int64_t c0 = bt * BATCH + int64_t(CPT) * k; // first cell of the tile
            u32x4 ua[KS][NPL];
            {
                if constexpr (!PF) load_u(k, uraw);
                const bool ok = uslot < CPT && ui0 < N && c0 + uslot < ncells;
#pragma unroll
                for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                    for (int j = 0; j < 8; j += 2) {
                        float x[2];
#pragma unroll
                        for (int e = 0; e < 2; ++e) {
                            const int i = 32 * ks + 8 * g + j + e;
                            x[e] = (ok && i < Q2) ? float(to_d(uraw[ks][j + e])) : 0.0f;
                        }
                        uint32_t t[3];
                        terms2<MODE>(x[0], x[1], t);
#pragma unroll
                        for (int p = 0; p < NPL; ++p) ua[ks][p][j / 2] = t[p];
                    }
            }
            // ---- the factor of the cell of each of this lane's result rows 4 g + j
            // (slot (4 g + j) / RS; one cell for all four unless RS = 5; padding rows past
            // the tile's cells take the last slot's and meet a zero weight)
            // (rows 4 g .. 4 g + 3 span at most two cells: the first row's and the last's)
            float P[ROWP ? 2 : 1][6];
#pragma unroll
            for (int r = 0; r < (ROWP ? 2 : 1); ++r) {
                const int sl = (4 * g + 3 * r) / RS;
#pragma unroll
                for (int e = 0; e < 6; ++e) P[r][e] = __shfl(Pm[e], CPT * k + (sl < CPT ? sl : CPT - 1));
            }
            const IO *kr = kappa;
            // kappa at rows 4 g + j, plane points 16 c + col: in the single-term modes the
            // whole tile's loads up front with FP32 storage (per pair of point tiles with
            // FP64 storage, where the registers run out), then the next tile's u
            constexpr bool KUP = PF && sizeof(IO) == 4;
            auto kload = [&](int c, int j) {
                const int sl = (4 * g + j) / RS, q0 = (4 * g + j) % RS, qp = 16 * c + col;
                const int64_t cell = c0 + sl;
                return kr[(cell < ncells ? cell : ncells - 1) * N3 + (q0 < N ? q0 : N - 1) * Q2 + (qp < Q2 ? qp : Q2 - 1)];
            };
            IO kraw[KUP ? NQ : 1][4];
            if constexpr (PF) {
                if (KUP && kr != nullptr) {
#pragma unroll
                    for (int c = 0; c < NQ; ++c)
#pragma unroll
                        for (int j = 0; j < 4; ++j) kraw[c][j] = kload(c, j);
                }
                if (k + 1 < nunit) load_u(k + 1, uraw);
            }

            f32x4 yacc[NQ];
#pragma unroll
            for (int t = 0; t < NQ; ++t) yacc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int m = 0; m < NQ2; ++m) {
                // B operand of stage 1^T: the stage-2^T results of plane-point tiles
                // 2 m (slots 0-3) and 2 m + 1 (slots 4-7)
                u32x4 tb[NMAT][NPL];
                IO kpair[2][4];
                if constexpr (PF && !KUP) {
                    if (kr != nullptr) {
#pragma unroll
                        for (int h = 0; h < 2; ++h)
#pragma unroll
                            for (int j = 0; j < 4; ++j) kpair[h][j] = kload(2 * m + h < NQ ? 2 * m + h : NQ - 1, j);
                    }
                }
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int c = 2 * m + h;
                    if (c >= NQ) {
#pragma unroll
                        for (int a = 0; a < NMAT; ++a)
#pragma unroll
                            for (int p = 0; p < NPL; ++p) tb[a][p][2 * h] = tb[a][p][2 * h + 1] = 0u;
                        continue;
                    }
                    // ---- stage 1 and stage 2: this tile's 16 plane points, every component
                    f32x4 G[NMAT];
#pragma unroll
                    for (int a = 0; a < NMAT; ++a) {
                        f32x4 V = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                        for (int ks = 0; ks < KS; ++ks) {
                            u32x4 bf[NPL];
#pragma unroll
                            for (int p = 0; p < NPL; ++p)
                                bf[p] = reinterpret_cast<const u32x4 *>(
                                    s1f + (a * NPL + p) * K.s1f_elems())[(c * KS + ks) * 64 + lane];
#pragma unroll
                            for (int q = 0; q < NPROD; ++q) V = mfma32<MODE>(ua[ks][prod_b(q)], bf[prod_a(q)], V);
                        }
                        u32x2 vb[NPL];
                        {
                            uint32_t t0[3], t1[3];
                            terms2<MODE>(V[0], V[1], t0);
                            terms2<MODE>(V[2], V[3], t1);
#pragma unroll
                            for (int p = 0; p < NPL; ++p) vb[p] = u32x2{t0[p], t1[p]};
                        }
                        u32x2 af[NPL];
#pragma unroll
                        for (int p = 0; p < NPL; ++p)
                            af[p] = reinterpret_cast<const u32x2 *>(s2 + (am_of<FORM>(a) * NPL + p) * 512)[lane];
                        G[a] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
                        if constexpr (NPROD == 6) {
                            // two products per K = 32 product: slots 0-3 one term pair,
                            // slots 4-7 the next (the K order is the same on both sides)
#pragma unroll
                            for (int q = 0; q < 6; q += 2)
                                G[a] = mfma32<MODE>(u32x4{af[prod_a(q)][0], af[prod_a(q)][1], af[prod_a(q + 1)][0],
                                                          af[prod_a(q + 1)][1]},
                                                    u32x4{vb[prod_b(q)][0], vb[prod_b(q)][1], vb[prod_b(q + 1)][0],
                                                          vb[prod_b(q + 1)][1]},
                                                    G[a]);
                        } else {
                            G[a] = mfma16<MODE>(af[0], vb[0], G[a]);
                        }
                    }
                    // ---- pointwise on rows 4 g + j (axis-0 point (4 g + j) % RS of the
                    // lane's cell) and plane point 16 c + col
                    const int qp = 16 * c + col;
                    const float w2 = sW2[qp]; // zero past the plane points
                    float sv[NMAT][4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int q0 = (4 * g + j) % RS;
                        float kq = 1.0f;
                        if (kr != nullptr) {
                            if constexpr (KUP) kq = float(to_d(kraw[c][j]));
                            else if constexpr (PF) kq = float(to_d(kpair[h][j]));
                            else kq = float(to_d(kload(c, j)));
                        }
                        const float om = sW0[4 * g + j] * w2 * kq; // zero past the axis-0 points
                        float Pj[6];
#pragma unroll
                        for (int e = 0; e < 6; ++e)
                            Pj[e] = ROWP && (4 * g + j) / RS != (4 * g) / RS ? P[ROWP ? 1 : 0][e] : P[0][e];
                        if constexpr (FORM == SF_LAPLACE) {
                            const float gx = G[0][j], gy = G[1][j], gz = G[2][j];
                            sv[0][j] = om * (Pj[0] * gx + Pj[1] * gy + Pj[2] * gz);
                            sv[1][j] = om * (Pj[1] * gx + Pj[3] * gy + Pj[4] * gz);
                            sv[2][j] = om * (Pj[2] * gx + Pj[4] * gy + Pj[5] * gz);
                        } else {
                            sv[0][j] = om * Pj[0] * G[0][j];
                        }
                    }
                    // ---- stage 2^T: s^T (A operand, the D layout of s) times M
#pragma unroll
                    for (int a = 0; a < NMAT; ++a) {
                        u32x2 sa[NPL];
                        {
                            uint32_t t0[3], t1[3];
                            terms2<MODE>(sv[a][0], sv[a][1], t0);
                            terms2<MODE>(sv[a][2], sv[a][3], t1);
#pragma unroll
                            for (int p = 0; p < NPL; ++p) sa[p] = u32x2{t0[p], t1[p]};
                        }
                        u32x2 bm[NPL];
#pragma unroll
                        for (int p = 0; p < NPL; ++p)
                            bm[p] = reinterpret_cast<const u32x2 *>(s2 + (am_of<FORM>(a) * NPL + p) * 512 + 256)[lane];
                        f32x4 T = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
                        if constexpr (NPROD == 6) {
#pragma unroll
                            for (int q = 0; q < 6; q += 2)
                                T = mfma32<MODE>(u32x4{sa[prod_b(q)][0], sa[prod_b(q)][1], sa[prod_b(q + 1)][0],
                                                       sa[prod_b(q + 1)][1]},
                                                 u32x4{bm[prod_a(q)][0], bm[prod_a(q)][1], bm[prod_a(q + 1)][0],
                                                       bm[prod_a(q + 1)][1]},
                                                 T);
                        } else {
                            T = mfma16<MODE>(sa[0], bm[0], T);
                        }
                        uint32_t t0[3], t1[3];
                        terms2<MODE>(T[0], T[1], t0);
                        terms2<MODE>(T[2], T[3], t1);
#pragma unroll
                        for (int p = 0; p < NPL; ++p) {
                            tb[a][p][2 * h] = t0[p];
                            tb[a][p][2 * h + 1] = t1[p];
                        }
                    }
                    if constexpr (NPL > 1) __builtin_amdgcn_sched_barrier(0);
                }
                __builtin_amdgcn_sched_barrier(0);
                // ---- stage 1^T: these 32 plane points' share of every plane-DOF tile
#pragma unroll
                for (int t = 0; t < NQ; ++t) {
#pragma unroll
                    for (int a = 0; a < NMAT; ++a) {
                        u32x4 af[NPL];
#pragma unroll
                        for (int p = 0; p < NPL; ++p)
                            af[p] = reinterpret_cast<const u32x4 *>(
                                s1b + (a * NPL + p) * K.s1b_elems())[(t * NQ2 + m) * 64 + lane];
#pragma unroll
                        for (int q = 0; q < NPROD; ++q) yacc[t] = mfma32<MODE>(af[prod_a(q)], tb[a][prod_b(q)], yacc[t]);
                    }
                    if (t % 2 == 1) __builtin_amdgcn_sched_barrier(0); // two DOF tiles' fragments at a time
                }
                __builtin_amdgcn_sched_barrier(0); // one pair of point tiles' registers at a time
            }
            // ---- y: column col = (slot, i0), plane DOFs 16 t + 4 g + j (four consecutive)
            {
                const int slot = col / RS, i0 = col % RS;
                const int64_t cell = c0 + slot;
                if (slot < CPT && i0 < N && cell < ncells) {
                    IO *yr = y + cell * N3 + i0 * Q2;
#pragma unroll
                    for (int t = 0; t < NQ; ++t)
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const int i = 16 * t + 4 * g + j;
                            if (i < Q2) yr[i] = IO(yacc[t][j]);
                        }
                }
            }
        }
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

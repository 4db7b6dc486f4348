// Operator action for Q_p / dQ_p (mass, Laplace), FP64 or FP32 contractions:
// the production kernel behind assemble_action.
//
// Same mathematics as action_q_body.inc (interpolate to the Gauss points with
// B, collocated derivative Dh, pointwise factor, transposed contractions;
// Sec. 3.3 eq. coeff_eval / eq. form_eval), organised for occupancy and
// latency on gfx950:
//
// * Axis-aligned box cells only (selected by sf_set_geometry(SF_GEOM_BOX)):
//   |J| G G^T is diagonal, so the Laplacian splits into three independent
//   directional chains Dh_a^T (w kappa P_aa) Dh_a.  Each chain runs inside
//   one pencil orientation - gradient, pointwise factor and transposed
//   gradient in registers - and accumulates into one LDS tensor: two LDS
//   tensors per cell instead of three.  A cell with off-diagonal J raises
//   SF_FLAG_NONBOX (only the diagonal factor is applied to it).
// * Persistent workgroups: each one walks cell groups g, g + G, ... and
//   issues the next group's u, kappa and vertex loads into registers right
//   after the current values are consumed, so HBM latency overlaps compute.
//   u / kappa / y are touched through x-axis pencils (consecutive lanes,
//   consecutive addresses).
#include <algorithm>

#include "sf_device.hpp"
#include "sf_internal.hpp"

namespace sf {

template <int N, int NQ, int FORM, bool COLL, typename T, int C> struct ActionFastSmem {
    static constexpr int NB = (FORM == SF_LAPLACE) ? 2 : 1;
    static constexpr int tensor_bytes = NB * C * Lds3<NQ>::CS * int(sizeof(T));
    static constexpr int bytes = tensor_bytes + 8 * (6 * C + 24 * C) + 16 * C;
};

// PREF: prefetch the next group's inputs into registers (more registers,
// latency overlap) or load them when needed; MINB: workgroups per CU the
// register allocation must allow.
// GLB: u and y are global C0 vectors of an nx x ny x nz cell grid (cell (i,j,k) is
// number (i*ny + j)*nz + k): local DOFs are gathered through the lattice numbering and
// the local results are added into y with FP64 atomics (y cleared beforehand).
template <int N, int NQ, int FORM, bool COLL, typename T, typename IO, int C, int NT, bool PREF, int MINB,
          bool GLB = false>
__global__ void __launch_bounds__(NT, MINB)
    action_q_fast_kernel(const int64_t ncells, const double *__restrict__ vert, const IO *__restrict__ kappa,
                         const IO *__restrict__ u, IO *__restrict__ y, const T *__restrict__ tab,
                         int *__restrict__ err, int *__restrict__ sched, const int gny = 0, const int gnz = 0)
{
    static_assert(N == NQ, "the fast kernel assumes n Gauss points per axis");
    static_assert(!(GLB && COLL), "global vectors are for the continuous family");
    static_assert(C * N * N <= NT, "one pencil per thread and stage");
    using L = Lds3<NQ>;
    constexpr int S1 = L::S1, S2 = L::S2, CS = L::CS;
    constexpr int NB = (FORM == SF_LAPLACE) ? 2 : 1;
    constexpr TabLayout TL(N, 0, NQ);
    constexpr int N2 = N * N, N3 = N2 * N;
    // even-odd packed tables: B, B^T centrosymmetric, Dh, Dh^T skew-centrosymmetric
    const T *const Bt = tab + TL.BEO();
    const T *const BtT = tab + TL.BTEO();
    const T *const Dh = tab + TL.DhEO();
    const T *const DhT = tab + TL.DhTEO();
    const T *const tW = tab + TL.W();

    __shared__ T lds[NB * C * CS];
    __shared__ double sP[C][6];
    __shared__ double sV[C][24];
    // 1-D weights in LDS for the lane-dependent w[q] factors: a vector global load here
    // would add a vector-memory wait to every stage that uses them
    __shared__ T sWq[NQ];
    T *const L0 = lds;
    T *const L1 = lds + (NB - 1) * C * CS;

    const int64_t ngroups = (ncells + C - 1) / C;
    const int tid = threadIdx.x;
    // this thread's x-pencil in the HBM stages (stage 1: u; the x stage: kappa)
    const bool pen = tid < C * N2;
    const int pc = pen ? tid / N2 : 0, pr = tid - pc * N2, pa = pr / N, pb = pr - pa * N;
    // the group's 24 C vertex coordinates, VR per thread (contiguous in HBM)
    constexpr int VR = (24 * C + NT - 1) / NT;

    T ureg[N], kreg[NQ];
    double vreg[VR];
    auto load_v = [&](int64_t g) {
#pragma unroll
        for (int r = 0; r < VR; ++r) {
            const int t = tid + r * NT;
            vreg[r] = (t < 24 * C && g * C + t / 24 < ncells) ? vert[g * C * 24 + t] : 0.0;
        }
    };
    // global lattice numbering (GLB): local (i0, i1, i2) of cell (ci, cj, ck) is lattice point
    // (ci p + i0, cj p + i1, ck p + i2), numbered (a (ny p + 1) + b)(nz p + 1) + c
    constexpr int P = N - 1;
    const int64_t lz = int64_t(gnz) * P + 1, lyz = (int64_t(gny) * P + 1) * lz;
    auto gbase = [&](int64_t gc) {
        const int64_t ci = gc / (int64_t(gny) * gnz), cj = (gc / gnz) % gny, ck = gc % gnz;
        return (ci * P) * lyz + (cj * P + pa) * lz + ck * P + pb;
    };
    auto load_u = [&](int64_t g) {
        const int64_t gc = g * C + pc;
        const bool ok = pen && gc < ncells;
        if constexpr (GLB) {
            const int64_t b0 = ok ? gbase(gc) : 0;
#pragma unroll
            for (int i = 0; i < N; ++i) ureg[i] = ok ? T(to_d(u[b0 + i * lyz])) : T(0);
        } else {
#pragma unroll
            for (int i = 0; i < N; ++i) ureg[i] = ok ? T(to_d(u[gc * N3 + i * N2 + pr])) : T(0);
        }
    };
    auto load_k = [&](int64_t g) {
        const int64_t gc = g * C + pc;
        ld_coeff(kappa, pen && gc < ncells, gc * N3 + pr, N2, kreg);
    };

    // Group schedule: groups are dealt round-robin (round r gives workgroup b group
    // b + r gridDim.x).  For the large cells (n >= 7) only three quarters are dealt; the
    // rest are claimed one at a time, workgroup b from counter b % P of the P = min(8,
    // gridDim.x) counters in sched (one 128-byte line each), counter x handing out
    // groups base + x + P k, so that workgroups that run faster take more of them and
    // all finish within about one group of each other.  Group numbers are fixed two
    // iterations ahead (thread 0, through LDS) so that the prefetch knows the next one.
    // A workgroup stops at its first group >= ngroups: dealt groups below the claimed
    // range are all valid, and a counter's claims only grow, so no claimed group is
    // left behind.  With fewer than two full rounds the schedule is purely round-robin.
    constexpr bool DYN = N >= 7;
    __shared__ int64_t s_claim;
    const int64_t rounds = DYN ? (ngroups * 3 / 4) / gridDim.x : 0;
    const int parts = gridDim.x < 8 ? int(gridDim.x) : 8, part = int(blockIdx.x) % parts;
    int64_t g = blockIdx.x, gn = int64_t(blockIdx.x) + gridDim.x, it = 0;
    if (tid < NQ) sWq[tid] = tW[tid]; // read after the loop's first barrier
    if (PREF && g < ngroups) {
        load_v(g);
        load_u(g);
        if constexpr (FORM == SF_LAPLACE) load_k(g);
    }
    while (g < ngroups) {
        int64_t claim = 0; // the group after gn
        if (tid == 0)
            claim = (rounds < 2 || it + 2 < rounds)
                        ? blockIdx.x + (it + 2) * gridDim.x
                        : rounds * gridDim.x + part + int64_t(parts) * atomicAdd(sched + kSchedLine * part, 1);
        const bool more = PREF && gn < ngroups;
        const int64_t cell0 = g * C;
        if (!PREF) {
            load_v(g);
            load_u(g);
            if constexpr (FORM == SF_LAPLACE) load_k(g);
        }
#pragma unroll
        for (int r = 0; r < VR; ++r) {
            const int t = tid + r * NT;
            if (t < 24 * C) sV[t / 24][t % 24] = vreg[r];
        }
        // The next group's inputs are requested once this group has issued its last
        // global load (vmcnt waits are in order: an earlier prefetch would make every
        // later wait of this group wait for it too).
        auto prefetch_next = [&] {
            if (more) {
                load_v(gn);
                load_u(gn);
                if constexpr (FORM == SF_LAPLACE) load_k(gn);
            }
        };
        __syncthreads(); // vertices staged; the previous group's last LDS reads are done

        // ---- geometry (FP64): J, det, |J| G G^T (or |J|), box test
        if (tid < C) {
            double P[6] = {0, 0, 0, 0, 0, 0};
            if (cell0 + tid < ncells) {
                double J[3][3], det;
                int f = affine_jacobian(sV[tid], J, det);
                if (FORM == SF_LAPLACE) {
                    laplace_factor(J, det, P);
                    const double off = fabs(J[0][1]) + fabs(J[0][2]) + fabs(J[1][0]) + fabs(J[1][2]) +
                                       fabs(J[2][0]) + fabs(J[2][1]);
                    const double dia = fabs(J[0][0]) + fabs(J[1][1]) + fabs(J[2][2]);
                    if (off > 1e-14 * dia) f |= SF_FLAG_NONBOX; // only the diagonal of G G^T is applied
                } else {
                    P[0] = fabs(det);
                }
                if (f) atomicOr(err, f);
            }
#pragma unroll
            for (int t = 0; t < 6; ++t) sP[tid][t] = P[t];
        }

        if constexpr (COLL && FORM == SF_MASS) {
            // collocated mass: diagonal operator, y = w kappa |J| u, no LDS tensors
            __syncthreads();
            if (pen && cell0 + pc < ncells) {
                cptr<T> W = fresh(tW);
                const T s23 = T(sP[pc][0]) * sWq[pa] * sWq[pb];
                const int64_t base = (cell0 + pc) * N3 + pr;
                T k[N];
                ld_coeff(kappa, true, base, N2, k);
#pragma unroll
                for (int i = 0; i < N; ++i) y[base + i * N2] = IO(s23 * W[i] * k[i] * ureg[i]);
            }
            prefetch_next();
        } else {
            // ---- stage 1 (x): u -> B_x u; for the Laplace form kappa is staged in L1
            // (read back along z, then overwritten by the z stage's output)
            if (pen) {
                if constexpr (COLL) {
                    st_pencil<0, N, S1, S2>(L0 + pc * CS, pa, pb, ureg);
                } else {
                    T out[NQ];
                    apply_eo<N, false, false>(Bt, ureg, out);
                    st_pencil<0, NQ, S1, S2>(L0 + pc * CS, pa, pb, out);
                }
                if constexpr (FORM == SF_LAPLACE) st_pencil<0, NQ, S1, S2>(L1 + pc * CS, pa, pb, kreg);
            }
            // kappa along this thread's y-stage pencil (one pencil per thread: C = NT / n^2)
            T ky[NQ];
            if constexpr (FORM == SF_LAPLACE) ld_coeff(kappa, pen && cell0 + pc < ncells, (cell0 + pc) * N3 + pa * N2 + pb, NQ, ky);
            __syncthreads();
            // ---- stage 2 (y): B_y
            if constexpr (!COLL) {
                pencils<C, NQ, N, NT>([&](int c, int q1, int i3) {
                    T in[N], out[NQ];
                    ld_pencil<1, N, S1, S2>(L0 + c * CS, q1, i3, in);
                    apply_eo<N, false, false>(Bt, in, out);
                    st_pencil<1, NQ, S1, S2>(L0 + c * CS, q1, i3, out);
                });
                __syncthreads();
            }

            if constexpr (FORM == SF_MASS) {
                // ---- stage 3 (z): B_z, w kappa |J|, B_z^T
                pencils<C, NQ, NQ, NT>([&](int c, int q1, int q2) {
                    const int64_t gc = cell0 + c;
                    T in[N], ut[NQ], t[N], k[NQ];
                    ld_coeff(kappa, gc < ncells, gc * N3 + (q1 * NQ + q2) * NQ, 1, k);
                    ld_pencil<2, N, S1, S2>(L0 + c * CS, q1, q2, in);
                    apply_eo<N, false, false>(Bt, in, ut);
                    cptr<T> W = fresh(tW);
                    const T w12 = T(sP[c][0]) * sWq[q1] * sWq[q2];
#pragma unroll
                    for (int q3 = 0; q3 < NQ; ++q3) ut[q3] *= w12 * W[q3] * k[q3];
                    apply_eo<N, false, false>(BtT, ut, t);
                    st_pencil<2, N, S1, S2>(L0 + c * CS, q1, q2, t);
                });
                prefetch_next();
                __syncthreads();
            } else {
                // ---- box path.  stage 3 (z): u~ = B_z(.), store u~; w = Dh_z^T (w kappa P_zz Dh_z u~)
                pencils<C, NQ, NQ, NT>([&](int c, int q1, int q2) {
                    T ut[NQ], gz[NQ], k[NQ];
                    ld_pencil<2, NQ, S1, S2>(L1 + c * CS, q1, q2, k);
                    if constexpr (COLL) {
                        ld_pencil<2, NQ, S1, S2>(L0 + c * CS, q1, q2, ut);
                    } else {
                        T in[N];
                        ld_pencil<2, N, S1, S2>(L0 + c * CS, q1, q2, in);
                        apply_eo<N, false, false>(Bt, in, ut);
                        st_pencil<2, NQ, S1, S2>(L0 + c * CS, q1, q2, ut);
                    }
                    apply_eo<N, true, false>(Dh, ut, gz);
                    cptr<T> W = fresh(tW);
                    const T w12 = T(sP[c][5]) * sWq[q1] * sWq[q2];
#pragma unroll
                    for (int q3 = 0; q3 < NQ; ++q3) gz[q3] *= w12 * W[q3] * k[q3];
                    apply_eo<N, true, false>(DhT, gz, ut);
                    st_pencil<2, NQ, S1, S2>(L1 + c * CS, q1, q2, ut);
                });
                __syncthreads();
                // ---- stage 4 (y): w += Dh_y^T (w kappa P_yy Dh_y u~)
                pencils<C, NQ, NQ, NT>([&](int c, int q1, int q3) {
                    const T(&k)[NQ] = ky; // this thread's only pencil
                    T ut[NQ], gy[NQ], wv[NQ];
                    ld_pencil<1, NQ, S1, S2>(L0 + c * CS, q1, q3, ut);
                    apply_eo<N, true, false>(Dh, ut, gy);
                    cptr<T> W = fresh(tW);
                    const T w13 = T(sP[c][3]) * sWq[q1] * sWq[q3];
#pragma unroll
                    for (int q2 = 0; q2 < NQ; ++q2) gy[q2] *= w13 * W[q2] * k[q2];
                    ld_pencil<1, NQ, S1, S2>(L1 + c * CS, q1, q3, wv);
                    apply_eo<N, true, true>(DhT, gy, wv);
                    st_pencil<1, NQ, S1, S2>(L1 + c * CS, q1, q3, wv);
                });
                __syncthreads();
                // ---- stage 5 (x): w += Dh_x^T (w kappa P_xx Dh_x u~); kappa from registers
                if (pen) {
                    T ut[NQ], gx[NQ], wv[NQ];
                    ld_pencil<0, NQ, S1, S2>(L0 + pc * CS, pa, pb, ut);
                    apply_eo<N, true, false>(Dh, ut, gx);
                    cptr<T> W = fresh(tW);
                    const T w23 = T(sP[pc][0]) * sWq[pa] * sWq[pb];
#pragma unroll
                    for (int q1 = 0; q1 < NQ; ++q1) gx[q1] *= w23 * W[q1] * kreg[q1];
                    ld_pencil<0, NQ, S1, S2>(L1 + pc * CS, pa, pb, wv);
                    apply_eo<N, true, true>(DhT, gx, wv);
                    st_pencil<0, NQ, S1, S2>(L1 + pc * CS, pa, pb, wv);
                }
                prefetch_next();
                __syncthreads();
                // ---- backward interpolation, z then y then x; the complete w is in L1
                if constexpr (!COLL) {
                    pencils<C, NQ, NQ, NT>([&](int c, int q1, int q2) {
                        T in[NQ], t[N];
                        ld_pencil<2, NQ, S1, S2>(L1 + c * CS, q1, q2, in);
                        apply_eo<N, false, false>(BtT, in, t);
                        st_pencil<2, N, S1, S2>(L1 + c * CS, q1, q2, t);
                    });
                    __syncthreads();
                }
            }
            T *const LB = (FORM == SF_LAPLACE) ? L1 : L0; // tensor holding the backward data
            if constexpr (!COLL) {
                pencils<C, NQ, N, NT>([&](int c, int q1, int i3) {
                    T in[NQ], out[N];
                    ld_pencil<1, NQ, S1, S2>(LB + c * CS, q1, i3, in);
                    apply_eo<N, false, false>(BtT, in, out);
                    st_pencil<1, N, S1, S2>(LB + c * CS, q1, i3, out);
                });
                __syncthreads();
            }
            // ---- last stage (x): B_x^T, store y (coalesced)
            if (pen && cell0 + pc < ncells) {
                T in[NQ], out[N];
                ld_pencil<0, NQ, S1, S2>(LB + pc * CS, pa, pb, in);
                if constexpr (COLL) {
#pragma unroll
                    for (int i = 0; i < N; ++i) out[i] = in[i];
                } else {
                    apply_eo<N, false, false>(BtT, in, out);
                }
                if constexpr (GLB) {
                    const int64_t b0 = gbase(cell0 + pc);
#pragma unroll
                    for (int i = 0; i < N; ++i) unsafeAtomicAdd(y + b0 + i * lyz, IO(out[i]));
                } else {
                    IO *yo = y + (cell0 + pc) * N3 + pr;
#pragma unroll
                    for (int i = 0; i < N; ++i) yo[i * N2] = IO(out[i]);
                }
            }
        }
        if (tid == 0) s_claim = claim;
        __syncthreads();
        g = gn;
        gn = s_claim;
        ++it;
    }
    // the last workgroup to leave resets the counters for the next launch on this slot
    if (tid == 0 && atomicAdd(sched + kSchedLine * 8, 1) == int(gridDim.x) - 1) {
        for (int x = 0; x < 8; ++x) atomicExch(sched + kSchedLine * x, 0);
        atomicExch(sched + kSchedLine * 8, 0);
    }
}

namespace {

template <typename K> int grid_for(K kernel, int nt, int64_t groups, int *cache)
{
    if (*cache <= 0) {
        int per_cu = 0, ncu = 0, dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, nt, 0) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return -1;
        *cache = std::max(1, per_cu) * std::max(1, ncu);
    }
    return int(std::min<int64_t>(groups, *cache));
}

template <int N, int FORM, bool COLL, typename T, typename IO, bool PREF, int MINB, int NT = 256>
int launch_fast_v(const LaunchArgs &a, const T *tab)
{
    constexpr int C = (NT / (N * N)) > 0 ? NT / (N * N) : 1;
    static int cache = 0;
    const int64_t groups = (a.ncells + C - 1) / C;
    auto kern = action_q_fast_kernel<N, N, FORM, COLL, T, IO, C, NT, PREF, MINB>;
    const int grid = grid_for(kern, NT, groups, &cache);
    if (grid < 0) return SF_ERR_HIP;
    if (!a.sched) return SF_ERR_ARG;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), 0, a.stream, a.ncells, a.vert, static_cast<const IO *>(a.kappa),
                       static_cast<const IO *>(a.u), static_cast<IO *>(a.y), tab, a.err, a.sched, 0, 0);
    return hipGetLastError() == hipSuccess ? SF_OK : SF_ERR_HIP;
}

// tile variants (autotuner search space; 3 is the general kernel, launched elsewhere):
// 256-thread workgroups: 0 = prefetch, >= 3 workgroups/CU; 1 = no prefetch, >= 4;
// 2 = prefetch, >= 2.  128-thread workgroups (fewer cells per group, more groups in
// flight): 4 = prefetch, >= 6 workgroups/CU; 5 = no prefetch, >= 8.
template <int N, int FORM, bool COLL, typename T, typename IO>
int launch_fast(const LaunchArgs &a, const T *tab)
{
    switch (a.variant) {
    case 1: return launch_fast_v<N, FORM, COLL, T, IO, false, 4>(a, tab);
    case 2: return launch_fast_v<N, FORM, COLL, T, IO, true, 2>(a, tab);
    case 4: return launch_fast_v<N, FORM, COLL, T, IO, true, 3, 128>(a, tab);
    case 5: return launch_fast_v<N, FORM, COLL, T, IO, false, 4, 128>(a, tab);
    default: return launch_fast_v<N, FORM, COLL, T, IO, true, 3>(a, tab);
    }
}

template <int N, int FORM, bool COLL>
int fast_prec(const LaunchArgs &a)
{
    if (a.precision == SF_FP64)
        return a.io == SF_F64 ? launch_fast<N, FORM, COLL, double, double>(a, a.tab64)
                              : launch_fast<N, FORM, COLL, double, float>(a, a.tab64);
    if (a.precision == SF_FP32)
        return a.io == SF_F64 ? launch_fast<N, FORM, COLL, float, double>(a, a.tab32)
                              : launch_fast<N, FORM, COLL, float, float>(a, a.tab32);
    return SF_ERR_UNSUPPORTED;
}

template <int N>
int fast_n(const LaunchArgs &a)
{
    const bool coll = a.family == SF_DQ || a.family == SF_QGLL; // B = I
    if (a.form == SF_MASS) return coll ? fast_prec<N, SF_MASS, true>(a) : fast_prec<N, SF_MASS, false>(a);
    if (a.form == SF_LAPLACE) return coll ? fast_prec<N, SF_LAPLACE, true>(a) : fast_prec<N, SF_LAPLACE, false>(a);
    return SF_ERR_UNSUPPORTED;
}

__global__ void fill_zero_kernel(double *y, int64_t n)
{
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += int64_t(gridDim.x) * blockDim.x)
        y[t] = 0.0;
}

template <int N, int FORM>
int launch_global_n(const LaunchArgs &a, int ny, int nz, int64_t nglobal)
{
    constexpr int NT = 256;
    constexpr int C = NT / (N * N) > 0 ? NT / (N * N) : 1;
    static int cache = 0;
    const int64_t groups = (a.ncells + C - 1) / C;
    auto kern = action_q_fast_kernel<N, N, FORM, false, double, double, C, NT, true, 3, true>;
    const int grid = grid_for(kern, NT, groups, &cache);
    if (grid < 0 || !a.sched) return SF_ERR_HIP;
    // clear with a kernel (also inside captured graphs), then accumulate
    hipLaunchKernelGGL(fill_zero_kernel, dim3(unsigned(std::min<int64_t>(4096, (nglobal + 255) / 256))), dim3(256), 0,
                       a.stream, static_cast<double *>(a.y), nglobal);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), 0, a.stream, a.ncells, a.vert, static_cast<const double *>(a.kappa),
                       static_cast<const double *>(a.u), static_cast<double *>(a.y), a.tab64, a.err, a.sched, ny, nz);
    return hipGetLastError() == hipSuccess ? SF_OK : SF_ERR_HIP;
}

template <int N>
int global_form(const LaunchArgs &a, int ny, int nz, int64_t ng)
{
    if (a.form == SF_LAPLACE) return launch_global_n<N, SF_LAPLACE>(a, ny, nz, ng);
    if (a.form == SF_MASS) return launch_global_n<N, SF_MASS>(a, ny, nz, ng);
    return SF_ERR_UNSUPPORTED;
}

} // namespace

int launch_action_q_global(const LaunchArgs &a, int nx, int ny, int nz)
{
    if (a.family != SF_Q || a.nq != a.degree + 1 || a.precision != SF_FP64 || a.io != SF_F64) return SF_ERR_UNSUPPORTED;
    const int p = a.degree;
    const int64_t ng = (int64_t(nx) * p + 1) * (int64_t(ny) * p + 1) * (int64_t(nz) * p + 1);
    switch (p + 1) {
    case 2: return global_form<2>(a, ny, nz, ng);
    case 3: return global_form<3>(a, ny, nz, ng);
    case 4: return global_form<4>(a, ny, nz, ng);
    case 5: return global_form<5>(a, ny, nz, ng);
    case 6: return global_form<6>(a, ny, nz, ng);
    case 7: return global_form<7>(a, ny, nz, ng);
    case 8: return global_form<8>(a, ny, nz, ng);
    case 9: return global_form<9>(a, ny, nz, ng);
    default: return SF_ERR_UNSUPPORTED;
    }
}

int launch_action_q_fast(const LaunchArgs &a)
{
    if (a.nq != a.degree + 1) return SF_ERR_UNSUPPORTED;
    switch (a.degree + 1) {
    case 2: return fast_n<2>(a);
    case 3: return fast_n<3>(a);
    case 4: return fast_n<4>(a);
    case 5: return fast_n<5>(a);
    case 6: return fast_n<6>(a);
    case 7: return fast_n<7>(a);
    case 8: return fast_n<8>(a);
    case 9: return fast_n<9>(a);
    default: return SF_ERR_UNSUPPORTED;
    }
}

} // namespace sf

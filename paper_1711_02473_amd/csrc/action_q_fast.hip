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

#include "action_box_body.inc"
#include "sf_device.hpp"
#include "sf_internal.hpp"

namespace sf {

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
    static_assert(!(GLB && COLL), "global vectors are for the continuous family");
    using SM = BoxSmem<N, NQ, FORM, COLL, T, C>;
    __shared__ __align__(16) unsigned char smem[SM::bytes];
    constexpr TabLayout TL(N, 0, NQ);
    constexpr int VR = BoxVR<C, NT>::VR;
    T *const sWq = reinterpret_cast<T *>(smem + SM::off_W);

    const int64_t ngroups = (ncells + C - 1) / C;
    const int tid = threadIdx.x;
    const BoxPencil<N, C, NT> pp;
    const BoxLattice<N> lat(gny, gnz);
    T ureg[N], kreg[NQ];
    double vreg[VR];
    auto load = [&](int64_t g) {
        box_load<N, NQ, FORM, T, IO, C, NT, GLB>(g * C, ncells, vert, kappa, u, pp, lat, vreg, ureg, kreg);
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
    if (tid < NQ) sWq[tid] = tab[TL.W() + tid]; // read after the group body's first barrier
    if (PREF && g < ngroups) load(g);
    while (g < ngroups) {
        int64_t claim = 0; // the group after gn
        if (tid == 0)
            claim = (rounds < 2 || it + 2 < rounds)
                        ? blockIdx.x + (it + 2) * gridDim.x
                        : rounds * gridDim.x + part + int64_t(parts) * atomicAdd(sched + kSchedLine * part, 1);
        const bool more = PREF && gn < ngroups;
        if (!PREF) load(g);
        box_group<N, NQ, FORM, COLL, T, IO, C, NT, GLB>(g * C, ncells, kappa, y, tab, err, smem, pp, lat, vreg, ureg,
                                                       kreg, [&] {
                                                           if (more) load(gn);
                                                       });
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

// p = 1 (two points per axis): one cell per thread, no LDS.  The cell's 24 vertex
// coordinates, 8 DOFs and 8 coefficients are read as 16-byte vectors into registers
// (each thread a contiguous run; the lines a wave touches are used in full), the
// tensor-product stages run on [2][2][2] register arrays, and the 8 results are
// written the same way.  Same operator as the group kernels: interpolate with B
// (skipped for the collocated families), the diagonal box factor on the gradient
// (Laplace) or w kappa |J| (mass), transposed contractions.
template <int FORM, bool COLL, typename T, typename IO>
__global__ void __launch_bounds__(256)
    action_q_cell2_kernel(const int64_t ncells, const double *__restrict__ vert, const IO *__restrict__ kappa,
                          const IO *__restrict__ u, IO *__restrict__ y, const T *__restrict__ tab,
                          int *__restrict__ err)
{
    constexpr TabLayout TL(2, 0, 2);
    const cptr<T> B = fresh(tab + TL.B0()), Dh = fresh(tab + TL.Dh()), W = fresh(tab + TL.W());
    for (int64_t gc = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; gc < ncells;
         gc += int64_t(gridDim.x) * blockDim.x) {
        double X[24];
        const double2 *xv = reinterpret_cast<const double2 *>(vert + gc * 24);
#pragma unroll
        for (int i = 0; i < 12; ++i) {
            const double2 v = xv[i];
            X[2 * i] = v.x;
            X[2 * i + 1] = v.y;
        }
        T uc[8], kc[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) uc[i] = T(to_d(u[gc * 8 + i]));
#pragma unroll
        for (int i = 0; i < 8; ++i) kc[i] = kappa != nullptr ? T(to_d(kappa[gc * 8 + i])) : T(1);
        double J[3][3], det;
        int f = affine_jacobian(X, J, det);
        double P[3];
        if constexpr (FORM == SF_LAPLACE) {
            double PF[6];
            laplace_factor(J, det, PF);
            P[0] = PF[0];
            P[1] = PF[3];
            P[2] = PF[5];
            const double off = fabs(J[0][1]) + fabs(J[0][2]) + fabs(J[1][0]) + fabs(J[1][2]) + fabs(J[2][0]) +
                               fabs(J[2][1]);
            const double dia = fabs(J[0][0]) + fabs(J[1][1]) + fabs(J[2][2]);
            if (off > 1e-14 * dia) f |= SF_FLAG_NONBOX; // only the diagonal of G G^T is applied
        } else {
            P[0] = P[1] = P[2] = fabs(det);
        }
        if (f) atomicOr(err, f);
        // one-axis application of a 2 x 2 matrix M (row-major [q][i]) or its transpose
        auto ax = [&](const cptr<T> &M, bool tr, int a, const T (&in)[8], T (&out)[8]) {
            const int s = a == 0 ? 4 : (a == 1 ? 2 : 1);
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                if (t & s) continue;
                const T x0 = in[t], x1 = in[t + s];
                const T m00 = T(M[0]), m01 = tr ? T(M[2]) : T(M[1]), m10 = tr ? T(M[1]) : T(M[2]), m11 = T(M[3]);
                out[t] = fmadd(m00, x0, m01 * x1);
                out[t + s] = fmadd(m10, x0, m11 * x1);
            }
        };
        T ut[8], t1[8];
        if constexpr (COLL) {
#pragma unroll
            for (int i = 0; i < 8; ++i) ut[i] = uc[i];
        } else {
            ax(B, false, 0, uc, ut);
            ax(B, false, 1, ut, t1);
            ax(B, false, 2, t1, ut);
        }
        T wv[8];
        // point weights w_q0 w_q1 w_q2 kappa_q
#pragma unroll
        for (int q = 0; q < 8; ++q) kc[q] *= T(W[q >> 2]) * T(W[(q >> 1) & 1]) * T(W[q & 1]);
        if constexpr (FORM == SF_MASS) {
#pragma unroll
            for (int q = 0; q < 8; ++q) wv[q] = T(P[0]) * kc[q] * ut[q];
        } else {
            T g[8], h[8];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                ax(Dh, false, a, ut, g);
#pragma unroll
                for (int q = 0; q < 8; ++q) g[q] *= T(P[a]) * kc[q];
                ax(Dh, true, a, g, h);
#pragma unroll
                for (int q = 0; q < 8; ++q) wv[q] = a == 0 ? h[q] : wv[q] + h[q];
            }
        }
        T yo[8];
        if constexpr (COLL) {
#pragma unroll
            for (int i = 0; i < 8; ++i) yo[i] = wv[i];
        } else {
            ax(B, true, 2, wv, t1);
            ax(B, true, 1, t1, wv);
            ax(B, true, 0, wv, yo);
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) y[gc * 8 + i] = IO(yo[i]);
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
template <int FORM, bool COLL, typename T, typename IO>
int launch_cell2(const LaunchArgs &a, const T *tab)
{
    const int64_t blocks = std::min<int64_t>((a.ncells + 255) / 256, int64_t(1) << 20);
    hipLaunchKernelGGL((action_q_cell2_kernel<FORM, COLL, T, IO>), dim3(unsigned(blocks)), dim3(256), 0, a.stream,
                       a.ncells, a.vert, static_cast<const IO *>(a.kappa), static_cast<const IO *>(a.u),
                       static_cast<IO *>(a.y), tab, a.err);
    return hipGetLastError() == hipSuccess ? SF_OK : SF_ERR_HIP;
}

template <int N, int FORM, bool COLL, typename T, typename IO>
int launch_fast(const LaunchArgs &a, const T *tab)
{
    if (a.variant == 6) {
        if constexpr (N == 2) return launch_cell2<FORM, COLL, T, IO>(a, tab);
        return SF_ERR_UNSUPPORTED;
    }
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

// H(div) NCF_k and H(curl) NCE_k operator action on affine cells, FP64 or FP32
// contractions: the production kernel behind assemble_action for these families.
//
// Same mathematics as the one-group-per-workgroup action in vec.hip (the enriched
// element split into its three tensor-product blocks, Sec. 3.5 eq. rtcf_split_x/y;
// each block sum-factorised with the contraction order of Alg. 1; Piola factors
// once per affine cell), organised for the instruction budget on gfx950, where that
// form is bound by vector-instruction issue (about four vector instructions per
// useful FMA, a third of them index arithmetic):
//
// * Every 1-D contraction uses the even-odd form of its matrix.  The node sets
//   (GLL for the P_k factor, GL for the dP_{k-1} factor) and the Gauss points are
//   symmetric about 1/2, so the value tables are centrosymmetric and the derivative
//   table skew-centrosymmetric, rectangular ones included: about half the FMAs.
// * Persistent workgroups walk the groups g, g + G, g + 2G, ... (G = grid size).
//   The map from a thread's staging slots (flat local DOF index) to the block
//   tensors is computed once per thread, and the next group's DOFs are requested
//   into registers as soon as the current ones are in LDS.
// * The Piola factors, with alpha and beta folded in, are computed for 16 cells at
//   a time (this workgroup's next 16 / C groups), one lane per cell, into LDS.
#include <algorithm>
#include <type_traits>

#include "sf_device.hpp"
#include "sf_internal.hpp"
#include "vec_el.hpp"

namespace sf {

namespace {
constexpr int kVecGeomCells = 16; // cells per batch of Piola factors
enum { VK_BD = 0, VK_P = 1 };     // 1-D factor of a forward contraction: dP_{k-1}, or P_k

// Factors per cell: NCF alpha J^T J / |J| (6 entries) and beta / |J|; NCE alpha |J| G G^T
// and beta J^T J / |J| (6 each).  On box cells only the diagonals: NCF alpha h_c^2 / |J|
// and beta / |J|, NCE alpha |J| / h_c^2 and beta h_c^2 / |J|, double-buffered.
template <int FAM, bool BOX> constexpr int vec_nfac() { return BOX ? (FAM == SF_NCF ? 4 : 6) : (FAM == SF_NCF ? 7 : 12); }

// LDS footprint and register target.  Affine form: as many waves per SIMD as the LDS
// footprint lets 3-wave workgroups reach (160 KiB per CU), between 4 and 6, so that the
// rarely run factor batch (24 vertex coordinates per lane) does not set the allocation
// above what LDS allows.
template <int FAM, int K, typename T, int C, bool BOX> struct VecFastCfg {
    static constexpr int NQ = K + 1, S2 = (NQ % 2) ? NQ : NQ + 1;
    static constexpr int lds = ((FAM == SF_NCF ? 6 : 9) * C * NQ * NQ * S2 +
                                (BOX ? 2 : 1) * (kVecGeomCells / C) * C * vec_nfac<FAM, BOX>()) * int(sizeof(T));
    static constexpr int wg = 163840 / lds, wps = (3 * wg + 3) / 4;
    // the box-cell form holds a pencil's values across the barriers of its fused stages:
    // 128 VGPRs (four waves per SIMD), measured faster than a tighter target that spills
    static constexpr int wpe = BOX ? 4 : (wps < 4 ? 4 : (wps > 6 ? 6 : wps));
};
}

// BOX: axis-aligned box cells (both Piola factors diagonal; a cell with off-diagonal J
// raises SF_FLAG_NONBOX and only the diagonal is applied).  The blocks then couple only
// through the divergence (NCF) or the curl (NCE), so the pointwise stage is fused into
// each block's last forward and first transposed contraction, which run on the same
// pencils: the values stay in registers and only the derivatives the other blocks need
// cross LDS.
template <int FAM, int K, typename T, typename IO, int C, int NT, bool BOX>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(VecFastCfg<FAM, K, T, C, BOX>::wpe, 8)))
    action_vec_fast_kernel(const int64_t ncells, const double *__restrict__ vert, const IO *__restrict__ kappa,
                           const IO *__restrict__ u, IO *__restrict__ y, const T *__restrict__ tab,
                           int *__restrict__ err, const double alpha, const double beta)
{
    using E = VecEl<FAM, K>;
    constexpr int NQ = E::NQ, NP = E::NP, ND = E::ND, NF = E::NF;
    using L = Lds3<NQ>;
    constexpr int S1 = L::S1, S2 = L::S2, CS = L::CS;
    constexpr int NQ3 = NQ * NQ * NQ;
    // tensors per cell: NCF: V0 V1 V2 D0 D1 D2; NCE: V0 V1 V2 and dV_c along its two P axes
    constexpr int NTEN = (FAM == SF_NCF) ? 6 : 9;
    constexpr int NG = vec_nfac<FAM, BOX>();
    constexpr int GB = kVecGeomCells / C; // groups per batch of factors
    static_assert(C >= 1 && GB >= 1 && GB * C <= NT, "one lane per cell of a factor batch");
    static_assert(NT % 3 == 0, "three equal thread ranges");
    constexpr int SPAN = NT / 3;
    constexpr TabLayout TL(NP, ND, NQ);
    const T *const BPe = tab + TL.BEO();    // B of P_k at the points, NQ x NP
    const T *const DPe = tab + TL.D0EO();   // its derivative (skew)
    const T *const BDe = tab + TL.B1EO();   // B of dP_{k-1}, NQ x ND
    const T *const BPTe = tab + TL.BTEO();  // transposes
    const T *const DPTe = tab + TL.D0TEO();
    const T *const BDTe = tab + TL.B1TEO();
    const T *const W3 = tab + TL.W3();      // w_q0 w_q1 w_q2

    __shared__ T lds[NTEN * C * CS];
    __shared__ T sG[BOX ? 2 : 1][GB * C][NG];
    static_assert(int(sizeof(lds) + sizeof(sG)) == VecFastCfg<FAM, K, T, C, BOX>::lds, "LDS footprint");
    auto TEN = [&](int i, int c) { return lds + (i * C + c) * CS; };

    const int tid = threadIdx.x;
    const int64_t ngroups = (ncells + C - 1) / C;
    const int64_t nflat = ncells * NF;

    // Wave w (threads [64 w, 64 w + 64)) owns block w: it stages, contracts and writes
    // back that block alone, so only the pointwise stage, which couples the blocks at
    // each point, needs the workgroup barrier; between its own stages a wave orders its
    // LDS accesses with a wavefront-scope fence.
    static_assert(SPAN == 64, "one wave per block");
    static_assert(E::bsize(0) == E::bsize(1) && E::bsize(1) == E::bsize(2), "equal blocks");
    constexpr int B = E::bsize(0);
    const int w = tid / 64, lane = tid - 64 * w;
    // slot s = lane + 64 k of this block's C B values in a group (cell j = s / B, index r in
    // the block): its place in the tensor and in the group's flat DOF range
    constexpr int KB = (C * B + 63) / 64;
    // packed as goff << 16 | soff (both below 2^16; goff = 0xffff past the end)
    static_assert(NTEN * C * CS < 65536 && C * NF < 65535, "16-bit slot offsets");
    constexpr int kPast = 0xffff;
    int sgo[KB];
    auto soff = [&](int k) { return sgo[k] & 0xffff; };
    auto goff = [&](int k) { return int(unsigned(sgo[k]) >> 16); };
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        const int sl = lane + 64 * k;
        sgo[k] = kPast << 16;
        if (sl < C * B) {
            const int j = sl / B, r = sl - j * B;
            const int e2 = w == 0 ? E::ext(0, 2) : (w == 1 ? E::ext(1, 2) : E::ext(2, 2));
            const int e1 = w == 0 ? E::ext(0, 1) : (w == 1 ? E::ext(1, 1) : E::ext(2, 1));
            const int i2 = r % e2, i1 = (r / e2) % e1, i0 = r / (e2 * e1);
            const int so = (w * C + j) * CS + i0 * S1 + i1 * S2 + i2;
            const int go = j * NF + (w == 0 ? 0 : (w == 1 ? E::off(1) : E::off(2))) + r;
            sgo[k] = (go << 16) | so;
        }
    }
    // number of valid flat offsets of group g (fewer than C NF only for the last group)
    auto valid = [&](int64_t g) {
        const int64_t rem = nflat - g * (C * NF);
        return rem < C * NF ? int(rem) : C * NF;
    };
    T uv[KB];
    auto load = [&](int64_t g) {
        const IO *ug = u + g * (C * NF);
        const int lim = valid(g);
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            const bool ok = goff(k) < lim;
            const IO x = ug[ok ? goff(k) : 0];
            uv[k] = ok ? T(to_d(x)) : T(0);
        }
    };
    auto wave_sync = [] {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };

    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    using I4 = std::integral_constant<int, 4>;
    using I5 = std::integral_constant<int, 5>;
    using I6 = std::integral_constant<int, 6>;
    using I7 = std::integral_constant<int, 7>;
    using I8 = std::integral_constant<int, 8>;
    using INONE = std::integral_constant<int, -1>;
    using INP = std::integral_constant<int, NP>;
    using IND = std::integral_constant<int, ND>;
    using INQ = std::integral_constant<int, NQ>;
    using KBD = std::integral_constant<int, VK_BD>;
    using KP = std::integral_constant<int, VK_P>;

    // forward contraction of tensor TN (extents E0 E1 E2) along AX on thread range RG:
    // in place with B of the factor KIND; for KIND = P with TN2 >= 0 also D into tensor TN2
    auto fwd = [&](auto rg, auto tn, auto ax, auto e0, auto e1, auto e2, auto kind, auto tn2) {
        constexpr int RG = decltype(rg)::value, TN = decltype(tn)::value, AX = decltype(ax)::value;
        constexpr int E0 = decltype(e0)::value, E1 = decltype(e1)::value, E2 = decltype(e2)::value;
        constexpr int KIND = decltype(kind)::value, TN2 = decltype(tn2)::value;
        constexpr int EI = AX == 0 ? E0 : (AX == 1 ? E1 : E2);
        static_assert(EI == (KIND == VK_BD ? ND : NP), "input extent of the 1-D factor");
        using O = Others<AX, E0, E1, E2>;
        pencils_part<C, O::P0, O::P1>(RG * SPAN, SPAN, [&](int c, int a, int b) {
            T in[EI], o1[NQ];
            ld_pencil<AX, EI, S1, S2>(TEN(TN, c), a, b, in);
            if constexpr (KIND == VK_BD) {
                apply_eo_rect<NQ, EI, false, false>(BDe, in, o1);
            } else {
                if constexpr (TN2 >= 0) {
                    T o2[NQ];
                    apply_eo_rect<NQ, EI, true, false>(DPe, in, o2);
                    st_pencil<AX, NQ, S1, S2>(TEN(TN2, c), a, b, o2);
                }
                apply_eo_rect<NQ, EI, false, false>(BPe, in, o1);
            }
            st_pencil<AX, NQ, S1, S2>(TEN(TN, c), a, b, o1);
        });
    };
    // transposed contraction of block CB's tensor along AX (NQ -> ND) with B of dP_{k-1}
    auto bwd_d = [&](auto cb, auto ax, auto e0, auto e1, auto e2) {
        constexpr int CB = decltype(cb)::value, AX = decltype(ax)::value;
        constexpr int E0 = decltype(e0)::value, E1 = decltype(e1)::value, E2 = decltype(e2)::value;
        using O = Others<AX, E0, E1, E2>;
        pencils_part<C, O::P0, O::P1>(CB * SPAN, SPAN, [&](int c, int a, int b) {
            T v[NQ], o[ND];
            ld_pencil<AX, NQ, S1, S2>(TEN(CB, c), a, b, v);
            apply_eo_rect<ND, NQ, false, false>(BDTe, v, o);
            st_pencil<AX, ND, S1, S2>(TEN(CB, c), a, b, o);
        });
    };

    // box cells: this lane's pencil of the fused stages (cell pc, positions pa < pb on the
    // two axes across the pencil), the same for all three blocks and every group
    const int pc = C == 1 ? 0 : lane / (NQ * NQ), pr = lane - pc * NQ * NQ;
    const int pa = pr / NQ, pb = pr - pa * NQ;
    const bool pact = lane < C * NQ * NQ;
    const T wab = (BOX && pact) ? T(tab[TL.W() + pa]) * T(tab[TL.W() + pb]) : T(0);
    // w_q kappa_q at the NQ points of this lane's pencil along AX in cell gc (the point
    // offsets are formed here, not kept across the group loop)
    auto pencil_weights = [&](auto ax, int64_t gc, T(&om)[NQ]) {
        constexpr int AX = decltype(ax)::value, QS = AX == 0 ? NQ * NQ : (AX == 1 ? NQ : 1);
        int a = pa, b = pb;
        asm volatile("" : "+v"(a), "+v"(b));
        const int qb = AX == 0 ? a * NQ + b : (AX == 1 ? a * NQ * NQ + b : (a * NQ + b) * NQ);
        const cptr<T> tw = fresh(tab + TL.W());
        if (kappa != nullptr && gc < ncells) {
            const IO *kc = kappa + gc * NQ3 + qb;
#pragma unroll
            for (int k = 0; k < NQ; ++k) om[k] = T(to_d(kc[k * QS]));
#pragma unroll
            for (int k = 0; k < NQ; ++k) om[k] *= T(tw[k]) * wab;
        } else {
#pragma unroll
            for (int k = 0; k < NQ; ++k) om[k] = T(tw[k]) * wab;
        }
    };

    int64_t g = blockIdx.x;
    if (g < ngroups) load(g);
    for (int it = 0; g < ngroups; ++it, g += gridDim.x) {
        const int64_t cell0 = g * C;
        const int slot = it % GB, buf = BOX ? (it / GB) & 1 : 0;
        if (slot == 0 && tid < GB * C) {
            // factors of cell c of group g + j G, this workgroup's next GB groups
            const int j = tid / C, c = tid - j * C;
            const int64_t gc = (g + int64_t(j) * gridDim.x) * C + c;
            T f[NG];
#pragma unroll
            for (int e = 0; e < NG; ++e) f[e] = T(0);
            if (gc < ncells) {
              if constexpr (BOX) {
                double J[3][3], det;
                int fl = affine_jacobian(vert + gc * 24, J, det);
                const double off = fabs(J[0][1]) + fabs(J[0][2]) + fabs(J[1][0]) + fabs(J[1][2]) +
                                   fabs(J[2][0]) + fabs(J[2][1]);
                const double dia = fabs(J[0][0]) + fabs(J[1][1]) + fabs(J[2][2]);
                if (off > 1e-14 * dia) fl |= SF_FLAG_NONBOX; // only the diagonal factors are applied
                if (fl) atomicOr(err, fl);
                const double S = fabs(det), rS = S > 0.0 ? 1.0 / S : 0.0;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const double h2 = J[a][a] * J[a][a];
                    if constexpr (FAM == SF_NCF) {
                        f[a] = T(alpha * h2 * rS);
                    } else {
                        f[a] = T(h2 > 0.0 ? alpha * S / h2 : 0.0);
                        f[3 + a] = T(beta * h2 * rS);
                    }
                }
                if constexpr (FAM == SF_NCF) f[3] = T(beta * rS);
              } else {
                double M0[6], M1[6], rS;
                const int fl = vec_geometry(vert + gc * 24, M0, M1, rS);
                if (fl) atomicOr(err, fl);
#pragma unroll
                for (int e = 0; e < 6; ++e) {
                    if constexpr (FAM == SF_NCF) {
                        f[e] = T(alpha * M1[e]);
                    } else {
                        f[e] = T(alpha * M0[e]);
                        f[6 + e] = T(beta * M1[e]);
                    }
                }
                if constexpr (FAM == SF_NCF) f[6] = T(beta * rS);
              }
            }
#pragma unroll
            for (int e = 0; e < NG; ++e) sG[buf][tid][e] = f[e];
        }
        // stage this block's DOFs, then request the next group's
#pragma unroll
        for (int k = 0; k < KB; ++k)
            if (goff(k) != kPast) lds[soff(k)] = uv[k];
        if (g + gridDim.x < ngroups) load(g + gridDim.x);
        wave_sync();

        if constexpr (FAM == SF_NCF) {
            // block c: P_k on axis c, dP_{k-1} on the others.  Forward: the two dP axes, then axis c
            fwd(I0{}, I0{}, I1{}, INP{}, IND{}, IND{}, KBD{}, INONE{});
            fwd(I1{}, I1{}, I0{}, IND{}, INP{}, IND{}, KBD{}, INONE{});
            fwd(I2{}, I2{}, I0{}, IND{}, IND{}, INP{}, KBD{}, INONE{});
            wave_sync();
            fwd(I0{}, I0{}, I2{}, INP{}, INQ{}, IND{}, KBD{}, INONE{});
            fwd(I1{}, I1{}, I2{}, INQ{}, INP{}, IND{}, KBD{}, INONE{});
            fwd(I2{}, I2{}, I1{}, INQ{}, IND{}, INP{}, KBD{}, INONE{});
            wave_sync();
            if constexpr (BOX) {
                // axis c: value V_c kept in registers, derivative D_c into tensor 3 + c for
                // the other blocks; then on the same pencils s = beta w kappa (D_0 + D_1 + D_2)
                // / |J|, v = alpha w kappa h_c^2 / |J| V_c, and BP^T v + DP^T s (NQ -> NP)
                __syncthreads(); // the previous group's reads of the D tensors are done
                T Vr[NQ], Dr[NQ];
                auto part1 = [&](auto cb) {
                    constexpr int CB = decltype(cb)::value;
                    if (w != CB || !pact) return;
                    T in[NP];
                    ld_pencil<CB, NP, S1, S2>(TEN(CB, pc), pa, pb, in);
                    apply_eo_rect<NQ, NP, true, false>(DPe, in, Dr);
                    st_pencil<CB, NQ, S1, S2>(TEN(3 + CB, pc), pa, pb, Dr);
                    apply_eo_rect<NQ, NP, false, false>(BPe, in, Vr);
                };
                part1(I0{});
                part1(I1{});
                part1(I2{});
                __syncthreads(); // every block's D is in LDS
                auto part2 = [&](auto cb) {
                    constexpr int CB = decltype(cb)::value;
                    if (w != CB || !pact) return;
                    {
                        T d1[NQ];
                        ld_pencil<CB, NQ, S1, S2>(TEN(3 + (CB + 1) % 3, pc), pa, pb, d1);
#pragma unroll
                        for (int k = 0; k < NQ; ++k) Dr[k] += d1[k];
                    }
                    {
                        T d2[NQ];
                        ld_pencil<CB, NQ, S1, S2>(TEN(3 + (CB + 2) % 3, pc), pa, pb, d2);
#pragma unroll
                        for (int k = 0; k < NQ; ++k) Dr[k] += d2[k];
                    }
                    const T *m = sG[buf][slot * C + pc];
                    const T fm = m[CB], fd = m[3];
                    {
                        T om[NQ];
                        pencil_weights(std::integral_constant<int, CB>{}, cell0 + pc, om);
#pragma unroll
                        for (int k = 0; k < NQ; ++k) {
                            Vr[k] = om[k] * fm * Vr[k];
                            Dr[k] = om[k] * fd * Dr[k];
                        }
                    }
                    T o[NP];
                    apply_eo_rect<NP, NQ, false, false>(BPTe, Vr, o);
                    apply_eo_rect<NP, NQ, true, true>(DPTe, Dr, o);
                    st_pencil<CB, NP, S1, S2>(TEN(CB, pc), pa, pb, o);
                };
                part2(I0{});
                part2(I1{});
                part2(I2{});
                wave_sync();
            } else {
                // axis c: value in place, derivative into tensor 3 + c
                fwd(I0{}, I0{}, I0{}, INP{}, INQ{}, INQ{}, KP{}, I3{});
                fwd(I1{}, I1{}, I1{}, INQ{}, INP{}, INQ{}, KP{}, I4{});
                fwd(I2{}, I2{}, I2{}, INQ{}, INQ{}, INP{}, KP{}, I5{});
                __syncthreads();
                // pointwise: v = alpha w kappa (J^T J / |J|) V, s = beta w kappa div^ V / |J|
                for (int t = tid; t < C * NQ3; t += NT) {
                    const int c = (C == 1) ? 0 : t / NQ3, q = t - c * NQ3;
                    const int o = (NQ % 2) ? q : q + q / NQ; // (q0 S1 + q1 S2 + q2)
                    const int64_t gc = cell0 + c;
                    const T kq = (kappa != nullptr && gc < ncells) ? T(to_d(kappa[gc * NQ3 + q])) : T(1);
                    const T om = W3[q] * kq;
                    const T *m = sG[0][slot * C + c];
                    T *t0 = TEN(0, c) + o, *t1 = TEN(1, c) + o, *t2 = TEN(2, c) + o;
                    T *t3 = TEN(3, c) + o, *t4 = TEN(4, c) + o, *t5 = TEN(5, c) + o;
                    const T a0 = *t0, a1 = *t1, a2 = *t2;
                    const T dv = *t3 + *t4 + *t5;
                    *t0 = om * (m[0] * a0 + m[1] * a1 + m[2] * a2);
                    *t1 = om * (m[1] * a0 + m[3] * a1 + m[4] * a2);
                    *t2 = om * (m[2] * a0 + m[4] * a1 + m[5] * a2);
                    const T sv = om * m[6] * dv; // one copy per block: each wave reads its own
                    *t3 = sv;
                    *t4 = sv;
                    *t5 = sv;
                }
                __syncthreads();
                // axis c: BP^T v + DP^T s (NQ -> NP), in place
                auto bwd_c = [&](auto cb) {
                    constexpr int CB = decltype(cb)::value;
                    pencils_part<C, NQ, NQ>(CB * SPAN, SPAN, [&](int c, int a, int b) {
                        T v[NQ], s[NQ], o[NP];
                        ld_pencil<CB, NQ, S1, S2>(TEN(CB, c), a, b, v);
                        ld_pencil<CB, NQ, S1, S2>(TEN(3 + CB, c), a, b, s);
                        apply_eo_rect<NP, NQ, false, false>(BPTe, v, o);
                        apply_eo_rect<NP, NQ, true, true>(DPTe, s, o);
                        st_pencil<CB, NP, S1, S2>(TEN(CB, c), a, b, o);
                    });
                };
                bwd_c(I0{});
                bwd_c(I1{});
                bwd_c(I2{});
                wave_sync();
            }
            // the dP axes in the reverse order of the forward pass
            bwd_d(I0{}, I2{}, INP{}, INQ{}, INQ{});
            bwd_d(I1{}, I2{}, INQ{}, INP{}, INQ{});
            bwd_d(I2{}, I1{}, INQ{}, INQ{}, INP{});
            wave_sync();
            bwd_d(I0{}, I1{}, INP{}, INQ{}, IND{});
            bwd_d(I1{}, I0{}, INQ{}, INP{}, IND{});
            bwd_d(I2{}, I0{}, INQ{}, IND{}, INP{});
            wave_sync();
        } else {
            // block c: dP_{k-1} on axis c, P_k on the others (o0 < o1).  Tensors: V_c = c,
            // dV_c / d o0 = 3 + c, dV_c / d o1 = 6 + c.  Forward: axis c, then o0, then o1.
            fwd(I0{}, I0{}, I0{}, IND{}, INP{}, INP{}, KBD{}, INONE{});
            fwd(I1{}, I1{}, I1{}, INP{}, IND{}, INP{}, KBD{}, INONE{});
            fwd(I2{}, I2{}, I2{}, INP{}, INP{}, IND{}, KBD{}, INONE{});
            wave_sync();
            fwd(I0{}, I0{}, I1{}, INQ{}, INP{}, INP{}, KP{}, I3{}); // block 0: o0 = 1
            fwd(I1{}, I1{}, I0{}, INP{}, INQ{}, INP{}, KP{}, I4{}); // block 1: o0 = 0
            fwd(I2{}, I2{}, I0{}, INP{}, INP{}, INQ{}, KP{}, I5{}); // block 2: o0 = 0
            wave_sync();
            if constexpr (BOX) {
                // o1: V (B), dV/d o1 (D) and dV/d o0 (B of tensor 3 + c) on the same pencils; the
                // two derivatives go to LDS for the other blocks' curl, V stays in registers
                T Vr[NQ], Or[NP], O0r[NP];
                auto part1 = [&](auto cb) {
                    constexpr int CB = decltype(cb)::value, O1 = CB == 2 ? 1 : 2;
                    if (w != CB || !pact) return;
                    {
                        T in[NP], Xr[NQ];
                        ld_pencil<O1, NP, S1, S2>(TEN(3 + CB, pc), pa, pb, in);
                        apply_eo_rect<NQ, NP, false, false>(BPe, in, Xr);
                        st_pencil<O1, NQ, S1, S2>(TEN(3 + CB, pc), pa, pb, Xr);
                    }
                    T in[NP], Yr[NQ];
                    ld_pencil<O1, NP, S1, S2>(TEN(CB, pc), pa, pb, in);
                    apply_eo_rect<NQ, NP, true, false>(DPe, in, Yr);
                    st_pencil<O1, NQ, S1, S2>(TEN(6 + CB, pc), pa, pb, Yr);
                    apply_eo_rect<NQ, NP, false, false>(BPe, in, Vr);
                };
                part1(I0{});
                part1(I1{});
                part1(I2{});
                __syncthreads(); // every block's derivatives are in LDS
                // c_a = beta w kappa h_a^2 / |J| (curl^ V)_a from the block's own two derivatives
                // (X along o0, Y along o1) and two of the other blocks'; the test-side terms
                // r_o0, r_o1 of block c (r_bc = sum_a eps_abc c_a), then BP^T v + DP^T r_o1
                // and BP^T r_o0 along o1, held until every block has read the derivatives
                auto part2 = [&](auto cb) {
                    constexpr int CB = decltype(cb)::value, O1 = CB == 2 ? 1 : 2;
                    constexpr int TA = CB == 0 ? 4 : (CB == 1 ? 3 : 6), TB = CB == 0 ? 5 : (CB == 1 ? 8 : 7);
                    if (w != CB || !pact) return;
                    const T *m = sG[buf][slot * C + pc];
                    // the block's own derivatives are read back (fewer registers held across
                    // the barrier)
                    T Xr[NQ], Yr[NQ];
                    ld_pencil<O1, NQ, S1, S2>(TEN(3 + CB, pc), pa, pb, Xr);
                    {
                        // r_o0 from the block's X and the other block's fa
                        T fa[NQ];
                        ld_pencil<O1, NQ, S1, S2>(TEN(TA, pc), pa, pb, fa);
#pragma unroll
                        for (int k = 0; k < NQ; ++k) {
                            if constexpr (CB == 0) Xr[k] = m[5] * (Xr[k] - fa[k]);      // -c2: fa = d0 V1, X = d1 V0
                            else if constexpr (CB == 1) Xr[k] = m[5] * (Xr[k] - fa[k]); //  c2: fa = d1 V0, X = d0 V1
                            else Xr[k] = m[4] * (Xr[k] - fa[k]);                        // -c1: fa = d2 V0, X = d0 V2
                        }
                    }
                    ld_pencil<O1, NQ, S1, S2>(TEN(6 + CB, pc), pa, pb, Yr);
                    {
                        // r_o1 from the block's Y and the other block's fb
                        T fb[NQ];
                        ld_pencil<O1, NQ, S1, S2>(TEN(TB, pc), pa, pb, fb);
#pragma unroll
                        for (int k = 0; k < NQ; ++k) {
                            if constexpr (CB == 0) Yr[k] = m[4] * (Yr[k] - fb[k]);      //  c1: fb = d0 V2, Y = d2 V0
                            else if constexpr (CB == 1) Yr[k] = m[3] * (Yr[k] - fb[k]); // -c0: fb = d1 V2, Y = d2 V1
                            else Yr[k] = m[3] * (Yr[k] - fb[k]);                        //  c0: fb = d2 V1, Y = d1 V2
                        }
                    }
                    {
                        T om[NQ];
                        pencil_weights(std::integral_constant<int, O1>{}, cell0 + pc, om);
#pragma unroll
                        for (int k = 0; k < NQ; ++k) {
                            Xr[k] *= om[k];
                            Yr[k] *= om[k];
                            Vr[k] = om[k] * m[CB] * Vr[k];
                        }
                    }
                    apply_eo_rect<NP, NQ, false, false>(BPTe, Xr, O0r);
                    apply_eo_rect<NP, NQ, false, false>(BPTe, Vr, Or);
                    apply_eo_rect<NP, NQ, true, true>(DPTe, Yr, Or);
                };
                part2(I0{});
                part2(I1{});
                part2(I2{});
                __syncthreads(); // the derivative tensors may be overwritten
                auto part3 = [&](auto cb) {
                    constexpr int CB = decltype(cb)::value, O1 = CB == 2 ? 1 : 2;
                    if (w != CB || !pact) return;
                    st_pencil<O1, NP, S1, S2>(TEN(CB, pc), pa, pb, Or);
                    st_pencil<O1, NP, S1, S2>(TEN(3 + CB, pc), pa, pb, O0r);
                };
                part3(I0{});
                part3(I1{});
                part3(I2{});
                wave_sync();
            } else {
                fwd(I0{}, I0{}, I2{}, INQ{}, INQ{}, INP{}, KP{}, I6{}); // block 0: o1 = 2
                fwd(I1{}, I1{}, I2{}, INQ{}, INQ{}, INP{}, KP{}, I7{}); // block 1: o1 = 2
                fwd(I2{}, I2{}, I1{}, INQ{}, INP{}, INQ{}, KP{}, I8{}); // block 2: o1 = 1
                fwd(I0{}, I3{}, I2{}, INQ{}, INQ{}, INP{}, KP{}, INONE{});
                fwd(I1{}, I4{}, I2{}, INQ{}, INQ{}, INP{}, KP{}, INONE{});
                fwd(I2{}, I5{}, I1{}, INQ{}, INP{}, INQ{}, KP{}, INONE{});
                __syncthreads();
                // pointwise: v = alpha w kappa |J| G G^T V, c = beta w kappa (J^T J / |J|) curl^ V,
                // and the curl's test-side terms r_bc = sum_a eps_abc c_a for each block's two derivatives
                for (int t = tid; t < C * NQ3; t += NT) {
                    const int c = (C == 1) ? 0 : t / NQ3, q = t - c * NQ3;
                    const int o = (NQ % 2) ? q : q + q / NQ;
                    const int64_t gc = cell0 + c;
                    const T kq = (kappa != nullptr && gc < ncells) ? T(to_d(kappa[gc * NQ3 + q])) : T(1);
                    const T om = W3[q] * kq;
                    const T *m = sG[0][slot * C + c];
                    T *const p0 = TEN(0, c) + o;
                    const T v0 = p0[0], v1 = p0[C * CS], v2 = p0[2 * C * CS];
                    const T d10 = p0[3 * C * CS], d01 = p0[4 * C * CS], d02 = p0[5 * C * CS];
                    const T d20 = p0[6 * C * CS], d21 = p0[7 * C * CS], d12 = p0[8 * C * CS];
                    const T cr0 = d12 - d21, cr1 = d20 - d02, cr2 = d01 - d10;
                    const T c0 = om * (m[6] * cr0 + m[7] * cr1 + m[8] * cr2);
                    const T c1 = om * (m[7] * cr0 + m[9] * cr1 + m[10] * cr2);
                    const T c2 = om * (m[8] * cr0 + m[10] * cr1 + m[11] * cr2);
                    p0[0] = om * (m[0] * v0 + m[1] * v1 + m[2] * v2);
                    p0[C * CS] = om * (m[1] * v0 + m[3] * v1 + m[4] * v2);
                    p0[2 * C * CS] = om * (m[2] * v0 + m[4] * v1 + m[5] * v2);
                    p0[3 * C * CS] = -c2; // block 0, d1
                    p0[6 * C * CS] = c1;  // block 0, d2
                    p0[4 * C * CS] = c2;  // block 1, d0
                    p0[7 * C * CS] = -c0; // block 1, d2
                    p0[5 * C * CS] = -c1; // block 2, d0
                    p0[8 * C * CS] = c0;  // block 2, d1
                }
                __syncthreads();
                // o1: V <- BP^T V + DP^T r_o1, r_o0 <- BP^T r_o0 (NQ -> NP)
                auto bwd_o1 = [&](auto cb, auto ax) {
                    constexpr int CB = decltype(cb)::value, AX = decltype(ax)::value;
                    pencils_part<C, NQ, NQ>(CB * SPAN, SPAN, [&](int c, int a, int b) {
                        {
                            T r0[NQ], o0[NP];
                            ld_pencil<AX, NQ, S1, S2>(TEN(3 + CB, c), a, b, r0);
                            apply_eo_rect<NP, NQ, false, false>(BPTe, r0, o0);
                            st_pencil<AX, NP, S1, S2>(TEN(3 + CB, c), a, b, o0);
                        }
                        T v[NQ], r1[NQ], o[NP];
                        ld_pencil<AX, NQ, S1, S2>(TEN(CB, c), a, b, v);
                        ld_pencil<AX, NQ, S1, S2>(TEN(6 + CB, c), a, b, r1);
                        apply_eo_rect<NP, NQ, false, false>(BPTe, v, o);
                        apply_eo_rect<NP, NQ, true, true>(DPTe, r1, o);
                        st_pencil<AX, NP, S1, S2>(TEN(CB, c), a, b, o);
                    });
                };
                bwd_o1(I0{}, I2{});
                bwd_o1(I1{}, I2{});
                bwd_o1(I2{}, I1{});
                wave_sync();
            }
            // o0: V <- BP^T V + DP^T r_o0 (NQ -> NP)
            auto bwd_o0 = [&](auto cb, auto ax, auto e0, auto e1, auto e2) {
                constexpr int CB = decltype(cb)::value, AX = decltype(ax)::value;
                constexpr int E0 = decltype(e0)::value, E1 = decltype(e1)::value, E2 = decltype(e2)::value;
                using O = Others<AX, E0, E1, E2>;
                pencils_part<C, O::P0, O::P1>(CB * SPAN, SPAN, [&](int c, int a, int b) {
                    T v[NQ], r0[NQ], o[NP];
                    ld_pencil<AX, NQ, S1, S2>(TEN(CB, c), a, b, v);
                    ld_pencil<AX, NQ, S1, S2>(TEN(3 + CB, c), a, b, r0);
                    apply_eo_rect<NP, NQ, false, false>(BPTe, v, o);
                    apply_eo_rect<NP, NQ, true, true>(DPTe, r0, o);
                    st_pencil<AX, NP, S1, S2>(TEN(CB, c), a, b, o);
                });
            };
            bwd_o0(I0{}, I1{}, INQ{}, INQ{}, INP{});
            bwd_o0(I1{}, I0{}, INQ{}, INQ{}, INP{});
            bwd_o0(I2{}, I0{}, INQ{}, INP{}, INQ{});
            wave_sync();
            // axis c: BD^T (NQ -> ND)
            bwd_d(I0{}, I0{}, INQ{}, INP{}, INP{});
            bwd_d(I1{}, I1{}, INP{}, INQ{}, INP{});
            bwd_d(I2{}, I2{}, INP{}, INP{}, INQ{});
            wave_sync();
        }

        // write this block's local results back through the staging map
        IO *const yg = y + cell0 * NF;
        const int lim = valid(g);
#pragma unroll
        for (int k = 0; k < KB; ++k)
            if (goff(k) < lim) yg[goff(k)] = IO(lds[soff(k)]);
        wave_sync(); // this wave's next staging overwrites its tensor
    }
}

namespace {

template <typename KF> int vec_grid(KF kernel, int nt, int64_t groups, int *cache)
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

template <int FAM, int K, typename T, typename IO, bool BOX>
int launch_fast_one(const LaunchArgs &a, const T *tab)
{
    constexpr int NQ = K + 1;
    constexpr int NT = 192;
    constexpr int C = 64 / (NQ * NQ) > 0 ? 64 / (NQ * NQ) : 1;
    static int cache = 0;
    const int64_t groups = (a.ncells + C - 1) / C;
    auto kern = action_vec_fast_kernel<FAM, K, T, IO, C, NT, BOX>;
    const int grid = vec_grid(kern, NT, groups, &cache);
    if (grid <= 0) return SF_ERR_HIP;
    const double al = (a.form == SF_MASS) ? 1.0 : a.alpha;
    const double be = (a.form == SF_MASS) ? 0.0 : a.beta;
    hipLaunchKernelGGL(kern, dim3(unsigned(grid)), dim3(NT), 0, a.stream, a.ncells, a.vert,
                       static_cast<const IO *>(a.kappa), static_cast<const IO *>(a.u), static_cast<IO *>(a.y), tab,
                       a.err, al, be);
    return hipGetLastError() == hipSuccess ? SF_OK : SF_ERR_HIP;
}

template <int FAM, int K, bool BOX>
int launch_fast_kb(const LaunchArgs &a)
{
    if (a.precision == SF_FP64)
        return a.io == SF_F64 ? launch_fast_one<FAM, K, double, double, BOX>(a, a.tab64)
                              : launch_fast_one<FAM, K, double, float, BOX>(a, a.tab64);
    if (a.precision == SF_FP32)
        return a.io == SF_F64 ? launch_fast_one<FAM, K, float, double, BOX>(a, a.tab32)
                              : launch_fast_one<FAM, K, float, float, BOX>(a, a.tab32);
    return SF_ERR_UNSUPPORTED;
}

// box contexts take the fused box-cell kernel unless variant 2 (the affine kernel) is asked for
template <int FAM, int K>
int launch_fast_k(const LaunchArgs &a)
{
    return (a.box && a.variant != 2) ? launch_fast_kb<FAM, K, true>(a) : launch_fast_kb<FAM, K, false>(a);
}

template <int FAM>
int launch_fast_fam(const LaunchArgs &a)
{
    switch (a.degree) {
    case 1: return launch_fast_k<FAM, 1>(a);
    case 2: return launch_fast_k<FAM, 2>(a);
    case 3: return launch_fast_k<FAM, 3>(a);
    case 4: return launch_fast_k<FAM, 4>(a);
    case 5: return launch_fast_k<FAM, 5>(a);
    case 6: return launch_fast_k<FAM, 6>(a);
    default: return SF_ERR_UNSUPPORTED;
    }
}

} // namespace

int launch_action_vec_fast(const LaunchArgs &a)
{
    if (a.nq != a.degree + 1 || a.trilinear) return SF_ERR_UNSUPPORTED;
    if (a.family == SF_NCF) return launch_fast_fam<SF_NCF>(a);
    if (a.family == SF_NCE) return launch_fast_fam<SF_NCE>(a);
    return SF_ERR_UNSUPPORTED;
}

} // namespace sf

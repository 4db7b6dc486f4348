// H(div) (NCF, "RTCF" on hexahedra) and H(curl) (NCE) elements of the Q^-
// family on gfx950: operator action (any affine cell, FP64 or FP32
// contractions; general trilinear cells with FP64 contractions and storage)
// and element matrices (axis-aligned boxes).
//
// Method.  The element is an enriched element of three tensor-product blocks
// (Sec. 2.6-2.7, eq. rtcf_impl); splitting the Concatenate node together with
// the indexed DOF buffer (Sec. 3.5, eq. rtcf_split_x/y) recovers the product
// structure of every block, which is then sum-factorised on its own.  Block c
// of NCF_k carries P_k (GLL_{k+1} nodes) on axis c and dP_{k-1} (GL_k nodes)
// on the other two axes; block c of NCE_k carries dP_{k-1} on axis c and P_k
// elsewhere.  The contraction order per block follows Alg. 1's criterion:
// factors shared by every quantity of the block are contracted first, so
//   NCF forward:  the two dP axes (B), then axis c with B and D (value, div);
//   NCE forward:  axis c (B of dP), then the first P axis with B and D, then
//                 the second P axis (value and the two derivatives);
// and the backward (transposed) contractions run in the reverse order, with
// the two terms of the first contraction merged by distributivity.
// Piola maps (FP64 per cell): contravariant for H(div)
//   v = alpha w kappa (J^T J / |J|) V,  s = beta w kappa div^ V / |J|,
// covariant for H(curl)
//   v = alpha w kappa |J| G G^T V,  c = beta w kappa (J^T J / |J|) curl^ V.
#include <type_traits>

#include "sf_device.hpp"
#include "sf_internal.hpp"
#include "vec_el.hpp"

namespace sf {

// ---------------------------------------------------------------------------
// action
// ---------------------------------------------------------------------------
// TRI: general trilinear cells, the Piola factors evaluated at every point from the
// eight vertices (J per point, Sec. 3.1) instead of once per affine cell
template <int FAM, int K, typename T, typename IO, int C, int NT, bool TRI = false>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(6, 8)))
    action_vec_kernel(const int64_t ncells, const double *__restrict__ vert, const IO *__restrict__ kappa,
                      const IO *__restrict__ u, IO *__restrict__ y, const T *__restrict__ tab, int *__restrict__ err,
                      const double alpha, const double beta)
{
    using E = VecEl<FAM, K>;
    constexpr int NQ = E::NQ, NP = E::NP, ND = E::ND, NF = E::NF;
    using L = Lds3<NQ>;
    constexpr int S1 = L::S1, S2 = L::S2, CS = L::CS;
    constexpr int NQ3 = NQ * NQ * NQ;
    // tensors per cell: NCF: V0 V1 V2 D0 D1 D2; NCE: V0 V1 V2 and dV_c along its two P axes
    constexpr int NTEN = (FAM == SF_NCF) ? 6 : 9;
    constexpr TabLayout TL(NP, ND, NQ);
    // the three blocks' contractions run side by side, one third of the threads each
    static_assert(NT % 3 == 0, "three equal thread ranges");
    constexpr int SPAN = NT / 3;
    const T *const BP = tab + TL.B0();
    const T *const DP = tab + TL.D0();
    const T *const BD = tab + TL.B1();
    const T *const BPT = tab + TL.B0T();
    const T *const DPT = tab + TL.D0T();
    const T *const BDT = tab + TL.B1T();
    const T *const tW = tab + TL.W();

    __shared__ T lds[NTEN * C * CS];
    __shared__ double sG[C][13];
    __shared__ T sWq[NQ]; // 1-D weights (lane-dependent reads in the pointwise stage)
    __shared__ double sXq[TRI ? NQ : 1], sVx[TRI ? C : 1][24]; // points and vertices (trilinear cells)
    static_assert(!TRI || std::is_same<T, double>::value, "trilinear cells: FP64 contractions");
    if (threadIdx.x < NQ) sWq[threadIdx.x] = tW[threadIdx.x]; // read after the staging barrier

    const int64_t cell0 = int64_t(blockIdx.x) * C;
    auto TEN = [&](int i, int c) { return lds + (i * C + c) * CS; };
    // the group's local DOFs, requested before the geometry work
    constexpr int KU = (C * NF + NT - 1) / NT;
    T uv[KU];
    ld_rows<C, NF, NT>(u, cell0, ncells, T(0), uv);

    if constexpr (TRI) {
        // the points (FP64 table block) and the group's vertices, for the per-point factors
        if (threadIdx.x < NQ) sXq[threadIdx.x] = reinterpret_cast<const double *>(tab)[TL.XQ() + threadIdx.x];
        for (int t = threadIdx.x; t < 24 * C; t += NT)
            sVx[t / 24][t % 24] = cell0 + t / 24 < ncells ? vert[cell0 * 24 + t] : 0.0;
    } else if (threadIdx.x < C) {
        const int64_t gc = cell0 + threadIdx.x;
        double M0[6] = {0, 0, 0, 0, 0, 0}, M1[6] = {0, 0, 0, 0, 0, 0}, rS = 0.0;
        if (gc < ncells) {
            const int f = vec_geometry(vert + gc * 24, M0, M1, rS);
            if (f) atomicOr(err, f);
        }
#pragma unroll
        for (int t = 0; t < 6; ++t) {
            sG[threadIdx.x][t] = M0[t];
            sG[threadIdx.x][6 + t] = M1[t];
        }
        sG[threadIdx.x][12] = rS;
    }
    // ---- stage the local DOFs into the three block tensors (coalesced over the flat index)
#pragma unroll
    for (int k = 0; k < KU; ++k) {
        const int t = threadIdx.x + k * NT;
        if (t >= C * NF) break;
        const int c = t / NF, d = t - c * NF;
        const T val = uv[k];
        int blk, r;
        if (d < E::off(1)) { blk = 0; r = d; }
        else if (d < E::off(2)) { blk = 1; r = d - E::off(1); }
        else { blk = 2; r = d - E::off(2); }
        int i0, i1, i2;
        if (blk == 0) { i2 = r % E::ext(0, 2); i1 = (r / E::ext(0, 2)) % E::ext(0, 1); i0 = r / (E::ext(0, 2) * E::ext(0, 1)); }
        else if (blk == 1) { i2 = r % E::ext(1, 2); i1 = (r / E::ext(1, 2)) % E::ext(1, 1); i0 = r / (E::ext(1, 2) * E::ext(1, 1)); }
        else { i2 = r % E::ext(2, 2); i1 = (r / E::ext(2, 2)) % E::ext(2, 1); i0 = r / (E::ext(2, 2) * E::ext(2, 1)); }
        TEN(blk, c)[i0 * S1 + i1 * S2 + i2] = val;
    }
    __syncthreads();

    // generic in-place contraction of one block tensor along AX (extents E0 E1 E2 before),
    // EI -> EO entries, matrix MT rows (EO x EI); optional second output (same pencil) into buf2
    auto fwd_block = [&](auto cblk, auto ax, auto e0, auto e1, auto e2, const T *M1p, const T *M2p, int ten2) {
        constexpr int CB = decltype(cblk)::value, AX = decltype(ax)::value;
        constexpr int E0 = decltype(e0)::value, E1 = decltype(e1)::value, E2 = decltype(e2)::value;
        constexpr int EI = AX == 0 ? E0 : (AX == 1 ? E1 : E2);
        using O = Others<AX, E0, E1, E2>;
        pencils_part<C, O::P0, O::P1>((CB) * SPAN, SPAN, [&](int c, int a, int b) {
            T in[EI], o1[NQ];
            ld_pencil<AX, EI, S1, S2>(TEN(CB, c), a, b, in);
            if (M2p) {
                T o2[NQ];
                mv<NQ, EI>(M2p, in, o2);
                st_pencil<AX, NQ, S1, S2>(TEN(ten2, c), a, b, o2);
            }
            mv<NQ, EI>(M1p, in, o1);
            st_pencil<AX, NQ, S1, S2>(TEN(CB, c), a, b, o1);
        });
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using INP = std::integral_constant<int, NP>;
    using IND = std::integral_constant<int, ND>;
    using INQ = std::integral_constant<int, NQ>;

    if constexpr (FAM == SF_NCF) {
        // block extents: c -> NP, others ND.  Forward: first dP axis, second dP axis, then axis c.
        // stage F1
        fwd_block(I0{}, I1{}, INP{}, IND{}, IND{}, BD, nullptr, 0);
        fwd_block(I1{}, I0{}, IND{}, INP{}, IND{}, BD, nullptr, 0);
        fwd_block(I2{}, I0{}, IND{}, IND{}, INP{}, BD, nullptr, 0);
        __syncthreads();
        // stage F2
        fwd_block(I0{}, I2{}, INP{}, INQ{}, IND{}, BD, nullptr, 0);
        fwd_block(I1{}, I2{}, INQ{}, INP{}, IND{}, BD, nullptr, 0);
        fwd_block(I2{}, I1{}, INQ{}, IND{}, INP{}, BD, nullptr, 0);
        __syncthreads();
        // stage F3: axis c, value (B) in place and derivative (D) into tensor 3 + c
        fwd_block(I0{}, I0{}, INP{}, INQ{}, INQ{}, BP, DP, 3);
        fwd_block(I1{}, I1{}, INQ{}, INP{}, INQ{}, BP, DP, 4);
        fwd_block(I2{}, I2{}, INQ{}, INQ{}, INP{}, BP, DP, 5);
        __syncthreads();
        // pointwise: v = alpha w kappa M1 V, s = beta w kappa div / |J|, one point per task
        // over all threads (the six values of a point are read, combined and written back)
        for (int t = threadIdx.x; t < C * NQ3; t += NT) {
            const int c = t / NQ3, q = t - c * NQ3;
            const int q0 = q / (NQ * NQ), q1 = (q / NQ) % NQ, q2 = q % NQ;
            const int64_t gc = cell0 + c;
            T m[6], sb;
            if constexpr (TRI) {
                double M0[6], M1[6], rS;
                const double det = vec_point_geometry(sVx[c], sXq[q0], sXq[q1], sXq[q2], M0, M1, rS);
                if (!(det > 0.0) && gc < ncells) atomicOr(err, SF_FLAG_DETJ);
#pragma unroll
                for (int e = 0; e < 6; ++e) m[e] = T(alpha * M1[e]);
                sb = T(beta * rS);
            } else {
#pragma unroll
                for (int e = 0; e < 6; ++e) m[e] = T(alpha * sG[c][6 + e]);
                sb = T(beta * sG[c][12]);
            }
            const T kq = (kappa != nullptr && gc < ncells) ? T(to_d(kappa[gc * NQ3 + q])) : T(1);
            const int o = q0 * S1 + q1 * S2 + q2;
            const T om = sWq[q0] * sWq[q1] * sWq[q2] * kq;
            T *t0 = TEN(0, c), *t1 = TEN(1, c), *t2 = TEN(2, c), *t3 = TEN(3, c), *t4 = TEN(4, c), *t5 = TEN(5, c);
            T x, yv, z;
            symmv(m, t0[o], t1[o], t2[o], x, yv, z);
            const T dv = t3[o] + t4[o] + t5[o];
            t0[o] = om * x;
            t1[o] = om * yv;
            t2[o] = om * z;
            t3[o] = om * sb * dv;
        }
        __syncthreads();
        // backward B1: axis c, T = BP^T v + DP^T s  (NQ -> NP), in place
        auto bwd_c = [&](auto cblk) {
            constexpr int CB = decltype(cblk)::value;
            pencils_part<C, NQ, NQ>((CB) * SPAN, SPAN, [&](int c, int a, int b) {
                T v[NQ], s[NQ], o[NP];
                ld_pencil<CB, NQ, S1, S2>(TEN(CB, c), a, b, v);
                ld_pencil<CB, NQ, S1, S2>(TEN(3, c), a, b, s);
                mtv<NQ, NP>(BPT, v, o);
                mtv_acc<NQ, NP>(DPT, s, o);
                st_pencil<CB, NP, S1, S2>(TEN(CB, c), a, b, o);
            });
        };
        bwd_c(I0{});
        bwd_c(I1{});
        bwd_c(I2{});
        __syncthreads();
        // backward B2, B3: the dP axes, reverse order of the forward pass (BD^T: NQ -> ND)
        auto bwd_d = [&](auto cblk, auto ax, auto e0, auto e1, auto e2) {
            constexpr int CB = decltype(cblk)::value, AX = decltype(ax)::value;
            constexpr int E0 = decltype(e0)::value, E1 = decltype(e1)::value, E2 = decltype(e2)::value;
            using O = Others<AX, E0, E1, E2>;
            pencils_part<C, O::P0, O::P1>((CB) * SPAN, SPAN, [&](int c, int a, int b) {
                T v[NQ], o[ND];
                ld_pencil<AX, NQ, S1, S2>(TEN(CB, c), a, b, v);
                mtv<NQ, ND>(BDT, v, o);
                st_pencil<AX, ND, S1, S2>(TEN(CB, c), a, b, o);
            });
        };
        bwd_d(I0{}, I2{}, INP{}, INQ{}, INQ{});
        bwd_d(I1{}, I2{}, INQ{}, INP{}, INQ{});
        bwd_d(I2{}, I1{}, INQ{}, INQ{}, INP{});
        __syncthreads();
        bwd_d(I0{}, I1{}, INP{}, INQ{}, IND{});
        bwd_d(I1{}, I0{}, INQ{}, INP{}, IND{});
        bwd_d(I2{}, I0{}, INQ{}, IND{}, INP{});
        __syncthreads();
    } else {
        // NCE: block extents c -> ND, others NP.  Tensors: V_c = c; dV_c along o0(c) = 3 + c,
        // along o1(c) = 6 + c, where o0 < o1 are the P axes of block c.
        // stage F1: axis c with BD (ND -> NQ)
        fwd_block(I0{}, I0{}, IND{}, INP{}, INP{}, BD, nullptr, 0);
        fwd_block(I1{}, I1{}, INP{}, IND{}, INP{}, BD, nullptr, 0);
        fwd_block(I2{}, I2{}, INP{}, INP{}, IND{}, BD, nullptr, 0);
        __syncthreads();
        // stage F2: first P axis o0 with BP (in place) and DP (-> 3 + c)
        fwd_block(I0{}, I1{}, INQ{}, INP{}, INP{}, BP, DP, 3); // block 0: o0 = 1
        fwd_block(I1{}, I0{}, INP{}, INQ{}, INP{}, BP, DP, 4); // block 1: o0 = 0
        fwd_block(I2{}, I0{}, INP{}, INP{}, INQ{}, BP, DP, 5); // block 2: o0 = 0
        __syncthreads();
        // stage F3: second P axis o1: V (BP in place), dV/d o1 (DP -> 6 + c); dV/d o0 (3 + c) by BP in place
        fwd_block(I0{}, I2{}, INQ{}, INQ{}, INP{}, BP, DP, 6); // block 0: o1 = 2
        fwd_block(I1{}, I2{}, INQ{}, INQ{}, INP{}, BP, DP, 7); // block 1: o1 = 2
        fwd_block(I2{}, I1{}, INQ{}, INP{}, INQ{}, BP, DP, 8); // block 2: o1 = 1
        {
            auto fwd_t = [&](int ten, auto ax, auto e0, auto e1, auto e2) {
                constexpr int AX = decltype(ax)::value;
                constexpr int E0 = decltype(e0)::value, E1 = decltype(e1)::value, E2 = decltype(e2)::value;
                constexpr int EI = AX == 0 ? E0 : (AX == 1 ? E1 : E2);
                using O = Others<AX, E0, E1, E2>;
                pencils_part<C, O::P0, O::P1>((ten - 3) * SPAN, SPAN, [&](int c, int a, int b) {
                    T in[EI], o[NQ];
                    ld_pencil<AX, EI, S1, S2>(TEN(ten, c), a, b, in);
                    mv<NQ, EI>(BP, in, o);
                    st_pencil<AX, NQ, S1, S2>(TEN(ten, c), a, b, o);
                });
            };
            fwd_t(3, I2{}, INQ{}, INQ{}, INP{});
            fwd_t(4, I2{}, INQ{}, INQ{}, INP{});
            fwd_t(5, I1{}, INQ{}, INP{}, INQ{});
        }
        __syncthreads();
        // pointwise, one point per task over all threads.  Derivatives present: block 0: d1 V0 (t3), d2 V0 (t6);
        // block 1: d0 V1 (t4), d2 V1 (t7); block 2: d0 V2 (t5), d1 V2 (t8).
        for (int t = threadIdx.x; t < C * NQ3; t += NT) {
            const int c = t / NQ3, q = t - c * NQ3;
            const int q0 = q / (NQ * NQ), q1 = (q / NQ) % NQ, q2 = q % NQ;
            const int64_t gc = cell0 + c;
            T m0[6], m1[6];
            if constexpr (TRI) {
                double M0[6], M1[6], rS;
                const double det = vec_point_geometry(sVx[c], sXq[q0], sXq[q1], sXq[q2], M0, M1, rS);
                if (!(det > 0.0) && gc < ncells) atomicOr(err, SF_FLAG_DETJ);
#pragma unroll
                for (int e = 0; e < 6; ++e) {
                    m0[e] = T(alpha * M0[e]);
                    m1[e] = T(beta * M1[e]);
                }
            } else {
#pragma unroll
                for (int e = 0; e < 6; ++e) {
                    m0[e] = T(alpha * sG[c][e]);
                    m1[e] = T(beta * sG[c][6 + e]);
                }
            }
            const T kq = (kappa != nullptr && gc < ncells) ? T(to_d(kappa[gc * NQ3 + q])) : T(1);
            {
                const int o = q0 * S1 + q1 * S2 + q2;
                const T om = sWq[q0] * sWq[q1] * sWq[q2] * kq;
                const T v0 = TEN(0, c)[o], v1 = TEN(1, c)[o], v2 = TEN(2, c)[o];
                const T d10 = TEN(3, c)[o], d20 = TEN(6, c)[o], d01 = TEN(4, c)[o];
                const T d21 = TEN(7, c)[o], d02 = TEN(5, c)[o], d12 = TEN(8, c)[o];
                // curl^ V = (d1 V2 - d2 V1, d2 V0 - d0 V2, d0 V1 - d1 V0)
                const T cr0 = d12 - d21, cr1 = d20 - d02, cr2 = d01 - d10;
                T x, yv, z, c0, c1, c2;
                symmv(m0, v0, v1, v2, x, yv, z);
                symmv(m1, cr0, cr1, cr2, c0, c1, c2);
                c0 *= om;
                c1 *= om;
                c2 *= om;
                TEN(0, c)[o] = om * x;
                TEN(1, c)[o] = om * yv;
                TEN(2, c)[o] = om * z;
                // test function phi e_c: curl^ contribution sum_b r_bc d_b phi, r_bc = sum_a eps_abc c_a
                TEN(3, c)[o] = -c2; // block 0, d1: r_10 = -c2
                TEN(6, c)[o] = c1;  // block 0, d2: r_20 =  c1
                TEN(4, c)[o] = c2;  // block 1, d0: r_01 =  c2
                TEN(7, c)[o] = -c0; // block 1, d2: r_21 = -c0
                TEN(5, c)[o] = -c1; // block 2, d0: r_02 = -c1
                TEN(8, c)[o] = c0;  // block 2, d1: r_12 =  c0
            }
        }
        __syncthreads();
        // backward B1: second P axis o1: V <- BP^T V + DP^T r_o1 ; r_o0 <- BP^T r_o0   (NQ -> NP)
        auto bwd_o1 = [&](auto cblk, auto ax) {
            constexpr int CB = decltype(cblk)::value, AX = decltype(ax)::value;
            pencils_part<C, NQ, NQ>((CB) * SPAN, SPAN, [&](int c, int a, int b) {
                T v[NQ], r1[NQ], r0[NQ], o[NP], o0[NP];
                ld_pencil<AX, NQ, S1, S2>(TEN(CB, c), a, b, v);
                ld_pencil<AX, NQ, S1, S2>(TEN(6 + CB, c), a, b, r1);
                ld_pencil<AX, NQ, S1, S2>(TEN(3 + CB, c), a, b, r0);
                mtv<NQ, NP>(BPT, v, o);
                mtv_acc<NQ, NP>(DPT, r1, o);
                mtv<NQ, NP>(BPT, r0, o0);
                st_pencil<AX, NP, S1, S2>(TEN(CB, c), a, b, o);
                st_pencil<AX, NP, S1, S2>(TEN(3 + CB, c), a, b, o0);
            });
        };
        bwd_o1(I0{}, I2{});
        bwd_o1(I1{}, I2{});
        bwd_o1(I2{}, I1{});
        __syncthreads();
        // backward B2: first P axis o0: V <- BP^T V + DP^T r_o0   (NQ -> NP)
        auto bwd_o0 = [&](auto cblk, auto ax, auto e0, auto e1, auto e2) {
            constexpr int CB = decltype(cblk)::value, AX = decltype(ax)::value;
            constexpr int E0 = decltype(e0)::value, E1 = decltype(e1)::value, E2 = decltype(e2)::value;
            using O = Others<AX, E0, E1, E2>;
            pencils_part<C, O::P0, O::P1>((CB) * SPAN, SPAN, [&](int c, int a, int b) {
                T v[NQ], r0[NQ], o[NP];
                ld_pencil<AX, NQ, S1, S2>(TEN(CB, c), a, b, v);
                ld_pencil<AX, NQ, S1, S2>(TEN(3 + CB, c), a, b, r0);
                mtv<NQ, NP>(BPT, v, o);
                mtv_acc<NQ, NP>(DPT, r0, o);
                st_pencil<AX, NP, S1, S2>(TEN(CB, c), a, b, o);
            });
        };
        bwd_o0(I0{}, I1{}, INQ{}, INQ{}, INP{});
        bwd_o0(I1{}, I0{}, INQ{}, INQ{}, INP{});
        bwd_o0(I2{}, I0{}, INQ{}, INP{}, INQ{});
        __syncthreads();
        // backward B3: axis c with BD^T (NQ -> ND)
        auto bwd_c = [&](auto cblk, auto e0, auto e1, auto e2) {
            constexpr int CB = decltype(cblk)::value;
            constexpr int E0 = decltype(e0)::value, E1 = decltype(e1)::value, E2 = decltype(e2)::value;
            using O = Others<CB, E0, E1, E2>;
            pencils_part<C, O::P0, O::P1>((CB) * SPAN, SPAN, [&](int c, int a, int b) {
                T v[NQ], o[ND];
                ld_pencil<CB, NQ, S1, S2>(TEN(CB, c), a, b, v);
                mtv<NQ, ND>(BDT, v, o);
                st_pencil<CB, ND, S1, S2>(TEN(CB, c), a, b, o);
            });
        };
        bwd_c(I0{}, INQ{}, INP{}, INP{});
        bwd_c(I1{}, INP{}, INQ{}, INP{});
        bwd_c(I2{}, INP{}, INP{}, INQ{});
        __syncthreads();
    }

    // ---- gather the three blocks back to the flat local index (coalesced store)
    for (int t = threadIdx.x; t < C * NF; t += NT) {
        const int c = t / NF, d = t - c * NF;
        const int64_t gc = cell0 + c;
        if (gc >= ncells) continue;
        int blk, r;
        if (d < E::off(1)) { blk = 0; r = d; }
        else if (d < E::off(2)) { blk = 1; r = d - E::off(1); }
        else { blk = 2; r = d - E::off(2); }
        int i0, i1, i2;
        if (blk == 0) { i2 = r % E::ext(0, 2); i1 = (r / E::ext(0, 2)) % E::ext(0, 1); i0 = r / (E::ext(0, 2) * E::ext(0, 1)); }
        else if (blk == 1) { i2 = r % E::ext(1, 2); i1 = (r / E::ext(1, 2)) % E::ext(1, 1); i0 = r / (E::ext(1, 2) * E::ext(1, 1)); }
        else { i2 = r % E::ext(2, 2); i1 = (r / E::ext(2, 2)) % E::ext(2, 1); i0 = r / (E::ext(2, 2) * E::ext(2, 1)); }
        y[gc * NF + d] = IO(TEN(blk, c)[i0 * S1 + i1 * S2 + i2]);
    }
}

// ---------------------------------------------------------------------------
// element matrices on boxes: a list of product terms per block pair
// ---------------------------------------------------------------------------
// Term t of block pair (c, c'): coefficient (per cell) times, on every axis a,
// the 1-D pair (test table of block c's space on axis a, B or D) x (trial table
// of block c''s space, B or D).  dt / ds: the axis carrying a derivative on the
// test / trial side (-1 = none).
struct TermShape {
    int dt, ds, kind; // kind: coefficient slot in the per-cell table
};

template <int FAM> struct Terms {
    // number of terms of pair (c, cp)
    static constexpr int count(int c, int cp)
    {
        if (FAM == SF_NCF) return c == cp ? 2 : 1;
        return c == cp ? 3 : 1;
    }
    static constexpr TermShape get(int c, int cp, int t)
    {
        if (FAM == SF_NCF) {
            if (c == cp && t == 0) return TermShape{-1, -1, c};    // alpha h_c^2 / S
            return TermShape{c, cp, 3};                            // beta / S (div-div)
        }
        if (c == cp) {
            if (t == 0) return TermShape{-1, -1, c};               // alpha S / h_c^2
            const int a = (t == 1) ? (c == 0 ? 1 : 0) : (c == 2 ? 1 : 2); // the two axes a != c
            const int b = 3 - a - c;
            return TermShape{b, b, 4 + a};                         // beta h_a^2 / S
        }
        const int a = 3 - c - cp;
        return TermShape{cp, c, 7 + a};                            // -beta h_a^2 / S
    }
};

template <int FAM, int K, typename IO, int NT>
__global__ void __launch_bounds__(NT)
    matrix_vec_kernel(const int64_t ncells, const double *__restrict__ vert, const IO *__restrict__ kappa,
                      IO *__restrict__ A, const double *__restrict__ tab, int *__restrict__ err, const double alpha,
                      const double beta)
{
    using E = VecEl<FAM, K>;
    constexpr int NQ = E::NQ, NP = E::NP, ND = E::ND, NF = E::NF;
    constexpr int NQ2 = NQ * NQ, NQ3 = NQ2 * NQ;
    constexpr TabLayout TL(NP, ND, NQ);
    constexpr int T1MAX = NQ2 * NP * NP; // per term
    constexpr int T2MAX = NQ * NP * NP;

    __shared__ double sT1[3 * T1MAX];
    __shared__ double sT2[2 * 3 * T2MAX];
    __shared__ double sK[NQ3];       // w_q kappa_q
    __shared__ double sTab[4][NQ * NP]; // BP, DP, BD, DD as [q][i]
    __shared__ double sCf[10];

    const int64_t gc = blockIdx.x;
    if (threadIdx.x == 0) {
        double J[3][3], det;
        int f = affine_jacobian(vert + gc * 24, J, det);
        const double off = fabs(J[0][1]) + fabs(J[0][2]) + fabs(J[1][0]) + fabs(J[1][2]) + fabs(J[2][0]) + fabs(J[2][1]);
        const double dia = fabs(J[0][0]) + fabs(J[1][1]) + fabs(J[2][2]);
        if (off > 1e-12 * dia) f |= SF_FLAG_NONBOX;
        if (f) atomicOr(err, f);
        const double S = fabs(det);
        const double h[3] = {J[0][0], J[1][1], J[2][2]};
        if (FAM == SF_NCF) {
            for (int c = 0; c < 3; ++c) sCf[c] = alpha * h[c] * h[c] / S;
            sCf[3] = beta / S;
        } else {
            for (int c = 0; c < 3; ++c) sCf[c] = alpha * S / (h[c] * h[c]);
            for (int a = 0; a < 3; ++a) {
                sCf[4 + a] = beta * h[a] * h[a] / S;
                sCf[7 + a] = -beta * h[a] * h[a] / S;
            }
        }
    }
    for (int t = threadIdx.x; t < NQ * NP; t += NT) {
        sTab[0][t] = tab[TL.B0() + t];
        sTab[1][t] = tab[TL.D0() + t];
    }
    for (int t = threadIdx.x; t < NQ * ND; t += NT) {
        sTab[2][t] = tab[TL.B1() + t];
        sTab[3][t] = tab[TL.D1() + t];
    }
    for (int t = threadIdx.x; t < NQ3; t += NT) {
        const int q0 = t / NQ2, q1 = (t / NQ) % NQ, q2 = t % NQ;
        const double w = tab[TL.W() + q0] * tab[TL.W() + q1] * tab[TL.W() + q2];
        sK[t] = w * (kappa ? to_d(kappa[gc * NQ3 + t]) : 1.0);
    }
    __syncthreads();

    // table of block c, axis a, derivative flag: sTab index and row length
    auto tsel = [](int c, int a, bool d) { return (E::pk(c, a) ? 0 : 2) + (d ? 1 : 0); };

    auto pair = [&](auto cc, auto ccp) {
        constexpr int c = decltype(cc)::value, cp = decltype(ccp)::value;
        constexpr int e0 = E::ext(c, 0), e1 = E::ext(c, 1), e2 = E::ext(c, 2);
        constexpr int f0 = E::ext(cp, 0), f1 = E::ext(cp, 1), f2 = E::ext(cp, 2);
        constexpr int NTm = Terms<FAM>::count(c, cp);
        constexpr int T1 = NQ2 * e2 * f2, T2 = NQ * f1 * f2;
        // stage 1: T1_t[q0 q1][i2][j2] = sum_q2 (w kappa) X2[q2][i2] Y2[q2][j2]
        for (int t = threadIdx.x; t < NTm * NQ2 * e2 * f2; t += NT) {
            const int tm = t / (NQ2 * e2 * f2);
            const int r = t - tm * (NQ2 * e2 * f2);
            const int q01 = r / (e2 * f2), ij = r - q01 * (e2 * f2);
            const int i2 = ij / f2, j2 = ij - i2 * f2;
            TermShape ts = Terms<FAM>::get(c, cp, tm);
            const double *X = sTab[tsel(c, 2, ts.dt == 2)];
            const double *Y = sTab[tsel(cp, 2, ts.ds == 2)];
            double acc = 0.0;
#pragma unroll
            for (int q2 = 0; q2 < NQ; ++q2) acc += sK[q01 * NQ + q2] * X[q2 * e2 + i2] * Y[q2 * f2 + j2];
            sT1[tm * T1MAX + r] = acc * sCf[ts.kind];
        }
        __syncthreads();
        for (int i1 = 0; i1 < e1; ++i1) {
            for (int i2 = 0; i2 < e2; ++i2) {
                const int buf = (i1 * e2 + i2) & 1;
                double *T2b = sT2 + buf * 3 * T2MAX;
                // phase A: T2_t[q0][j1][j2] = sum_q1 X1[q1][i1] Y1[q1][j1] T1_t[q0][q1][i2][j2]
                for (int t = threadIdx.x; t < NTm * NQ * f1 * f2; t += NT) {
                    const int tm = t / (NQ * f1 * f2);
                    const int r = t - tm * (NQ * f1 * f2);
                    const int q0 = r / (f1 * f2), jj = r - q0 * (f1 * f2);
                    const int j1 = jj / f2, j2 = jj - j1 * f2;
                    TermShape ts = Terms<FAM>::get(c, cp, tm);
                    const double *X = sTab[tsel(c, 1, ts.dt == 1)];
                    const double *Y = sTab[tsel(cp, 1, ts.ds == 1)];
                    const double *t1 = sT1 + tm * T1MAX + (q0 * NQ) * (e2 * f2) + i2 * f2 + j2;
                    double acc = 0.0;
#pragma unroll
                    for (int q1 = 0; q1 < NQ; ++q1) acc += X[q1 * e1 + i1] * Y[q1 * f1 + j1] * t1[q1 * e2 * f2];
                    T2b[tm * T2MAX + r] = acc;
                }
                __syncthreads();
                // phase B: rows (i0, i1, i2) of block c, columns of block cp
                for (int t = threadIdx.x; t < e0 * f0 * f1 * f2; t += NT) {
                    const int i0 = t / (f0 * f1 * f2);
                    const int j = t - i0 * (f0 * f1 * f2);
                    const int j0 = j / (f1 * f2), jj = j - j0 * (f1 * f2);
                    double acc = 0.0;
#pragma unroll
                    for (int tm = 0; tm < NTm; ++tm) {
                        TermShape ts = Terms<FAM>::get(c, cp, tm);
                        const double *X = sTab[tsel(c, 0, ts.dt == 0)];
                        const double *Y = sTab[tsel(cp, 0, ts.ds == 0)];
                        const double *t2 = T2b + tm * T2MAX + jj;
#pragma unroll
                        for (int q0 = 0; q0 < NQ; ++q0) acc += X[q0 * e0 + i0] * Y[q0 * f0 + j0] * t2[q0 * f1 * f2];
                    }
                    const int row = E::off(c) + (i0 * e1 + i1) * e2 + i2;
                    A[gc * int64_t(NF) * NF + int64_t(row) * NF + E::off(cp) + j] = IO(acc);
                }
            }
        }
        __syncthreads();
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    pair(I0{}, I0{});
    pair(I0{}, I1{});
    pair(I0{}, I2{});
    pair(I1{}, I0{});
    pair(I1{}, I1{});
    pair(I1{}, I2{});
    pair(I2{}, I0{});
    pair(I2{}, I1{});
    pair(I2{}, I2{});
}

namespace {

template <int FAM, int K, typename T, typename IO, bool TRI = false>
int launch_action_one(const LaunchArgs &a, const T *tab)
{
    // one or two waves per block, C cells so that a block's n^2 pencils fill them
    constexpr int NQ = K + 1;
    constexpr int WB = 1;
    constexpr int NT = 3 * 64 * WB;
    constexpr int C = (64 * WB) / (NQ * NQ) > 0 ? (64 * WB) / (NQ * NQ) : 1;
    const int64_t groups = (a.ncells + C - 1) / C;
    if (groups > 0x7fffffffLL) return SF_ERR_CAPACITY;
    const double al = (a.form == SF_MASS) ? 1.0 : a.alpha;
    const double be = (a.form == SF_MASS) ? 0.0 : a.beta;
    hipLaunchKernelGGL((action_vec_kernel<FAM, K, T, IO, C, NT, TRI>), dim3(unsigned(groups)), dim3(NT), 0, a.stream,
                       a.ncells, a.vert, static_cast<const IO *>(a.kappa), static_cast<const IO *>(a.u),
                       static_cast<IO *>(a.y), tab, a.err, al, be);
    return hipGetLastError() == hipSuccess ? SF_OK : SF_ERR_HIP;
}

template <int FAM, int K>
int launch_action_k(const LaunchArgs &a)
{
    if (a.trilinear) // per-point geometry: FP64 contractions and storage
        return (a.precision == SF_FP64 && a.io == SF_F64) ? launch_action_one<FAM, K, double, double, true>(a, a.tab64)
                                                         : SF_ERR_UNSUPPORTED;
    if (a.precision == SF_FP64)
        return a.io == SF_F64 ? launch_action_one<FAM, K, double, double>(a, a.tab64)
                              : launch_action_one<FAM, K, double, float>(a, a.tab64);
    if (a.precision == SF_FP32)
        return a.io == SF_F64 ? launch_action_one<FAM, K, float, double>(a, a.tab32)
                              : launch_action_one<FAM, K, float, float>(a, a.tab32);
    return SF_ERR_UNSUPPORTED;
}

template <int FAM>
int launch_action_fam(const LaunchArgs &a)
{
    switch (a.degree) {
    case 1: return launch_action_k<FAM, 1>(a);
    case 2: return launch_action_k<FAM, 2>(a);
    case 3: return launch_action_k<FAM, 3>(a);
    case 4: return launch_action_k<FAM, 4>(a);
    case 5: return launch_action_k<FAM, 5>(a);
    case 6: return launch_action_k<FAM, 6>(a);
    default: return SF_ERR_UNSUPPORTED;
    }
}

template <int FAM, int K, typename IO>
int launch_matrix_one(const LaunchArgs &a)
{
    constexpr int NT = K <= 2 ? 64 : (K <= 4 ? 128 : 256);
    if (a.ncells > 0x7fffffffLL) return SF_ERR_CAPACITY;
    const double al = (a.form == SF_MASS) ? 1.0 : a.alpha;
    const double be = (a.form == SF_MASS) ? 0.0 : a.beta;
    hipLaunchKernelGGL((matrix_vec_kernel<FAM, K, IO, NT>), dim3(unsigned(a.ncells)), dim3(NT), 0, a.stream,
                       a.ncells, a.vert, static_cast<const IO *>(a.kappa), static_cast<IO *>(a.A), a.tab64, a.err,
                       al, be);
    return hipGetLastError() == hipSuccess ? SF_OK : SF_ERR_HIP;
}

template <int FAM>
int launch_matrix_fam(const LaunchArgs &a)
{
    const bool f = a.io == SF_F32;
    switch (a.degree) {
    case 1: return f ? launch_matrix_one<FAM, 1, float>(a) : launch_matrix_one<FAM, 1, double>(a);
    case 2: return f ? launch_matrix_one<FAM, 2, float>(a) : launch_matrix_one<FAM, 2, double>(a);
    case 3: return f ? launch_matrix_one<FAM, 3, float>(a) : launch_matrix_one<FAM, 3, double>(a);
    case 4: return f ? launch_matrix_one<FAM, 4, float>(a) : launch_matrix_one<FAM, 4, double>(a);
    case 5: return f ? launch_matrix_one<FAM, 5, float>(a) : launch_matrix_one<FAM, 5, double>(a);
    case 6: return f ? launch_matrix_one<FAM, 6, float>(a) : launch_matrix_one<FAM, 6, double>(a);
    default: return SF_ERR_UNSUPPORTED;
    }
}

} // namespace

int launch_action_vec(const LaunchArgs &a)
{
    if (a.nq != a.degree + 1) return SF_ERR_UNSUPPORTED;
    // affine cells: the persistent even-odd kernel unless variant 1 (this file's kernel) is asked for
    if (!a.trilinear && a.variant != 1) return launch_action_vec_fast(a);
    if (a.family == SF_NCF) return launch_action_fam<SF_NCF>(a);
    if (a.family == SF_NCE) return launch_action_fam<SF_NCE>(a);
    return SF_ERR_UNSUPPORTED;
}

int launch_matrix_vec(const LaunchArgs &a)
{
    if (a.nq != a.degree + 1 || a.precision != SF_FP64) return SF_ERR_UNSUPPORTED;
    if (a.family == SF_NCF) return launch_matrix_fam<SF_NCF>(a);
    if (a.family == SF_NCE) return launch_matrix_fam<SF_NCE>(a);
    return SF_ERR_UNSUPPORTED;
}

} // namespace sf

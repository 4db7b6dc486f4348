// Host-side checks of the C ABI built with AddressSanitizer and UBSan (no GPU):
// the argument validation of every entry point, the 1-D rules and Lagrange
// tables, element dimensions, block layouts, the concatenated index and the
// axis-order planner.  Linked from api.cpp and tables.cpp; the kernel
// launchers are replaced by stubs that fail loudly, since validation must
// reject every bad call before any of them (or any HIP call) is reached.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "sf.h"
#include "../../paper_1711_02473_amd/csrc/sf_internal.hpp"

namespace sf {
#define STUB(name, ...)                                                      \
    int name(__VA_ARGS__)                                                    \
    {                                                                        \
        std::fprintf(stderr, "launcher %s reached without a GPU\n", #name); \
        std::abort();                                                        \
    }
STUB(launch_action_q, const LaunchArgs &)
STUB(launch_action_vq, const LaunchArgs &)
STUB(launch_matrix_svk, const LaunchArgs &)
STUB(launch_action_q_fast, const LaunchArgs &)
STUB(launch_action_q_global, const LaunchArgs &, int, int, int)
STUB(launch_matrix_q, const LaunchArgs &)
STUB(launch_action_vec, const LaunchArgs &)
STUB(launch_matrix_vec, const LaunchArgs &)
STUB(launch_action_mixed, const LaunchArgs &)
STUB(launch_dofmap_q, int, int, int, int, int32_t *, hipStream_t)
STUB(launch_matrix_qgen, const LaunchArgs &)
STUB(launch_matrix_coll, const LaunchArgs &)
STUB(noalloc_setup, int)
STUB(launch_action_box_noalloc, LaunchArgs, int)
#undef STUB
} // namespace sf

static int failures = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++failures;                                                       \
        }                                                                     \
    } while (0)

int main()
{
    // 1-D rules: weights sum to one, GL exact to degree 2m-1, GLL to 2m-3
    for (int kind = 0; kind < 2; ++kind)
        for (int m = (kind ? 2 : 1); m <= 17; ++m) {
            std::vector<double> x(m), w(m);
            CHECK(sf_rule_1d(kind, m, x.data(), w.data()) == SF_OK);
            const int deg = kind ? 2 * m - 3 : 2 * m - 1;
            for (int a = 0; a <= deg; ++a) {
                double s = 0.0;
                for (int q = 0; q < m; ++q) s += w[q] * std::pow(x[q], a);
                CHECK(std::fabs(s - 1.0 / (a + 1)) <= 1e-13);
            }
        }
    CHECK(sf_rule_1d(0, 0, nullptr, nullptr) != SF_OK);
    CHECK(sf_rule_1d(2, 3, nullptr, nullptr) != SF_OK);
    // Lagrange tables: delta at the nodes, partition of unity, derivative sums to zero
    for (int n = 1; n <= 12; ++n) {
        std::vector<double> xn(n), wn(n), xq(n + 3), wq(n + 3);
        CHECK(sf_rule_1d(n >= 2 ? 1 : 0, n, xn.data(), wn.data()) == SF_OK);
        CHECK(sf_rule_1d(0, n + 3, xq.data(), wq.data()) == SF_OK);
        std::vector<double> B(size_t(n) * n), D(size_t(n) * n), Bq(size_t(n + 3) * n), Dq(size_t(n + 3) * n);
        CHECK(sf_lagrange_table(n, xn.data(), n, xn.data(), B.data(), D.data()) == SF_OK);
        for (int p = 0; p < n; ++p)
            for (int i = 0; i < n; ++i) CHECK(std::fabs(B[p * n + i] - (p == i ? 1.0 : 0.0)) <= 1e-12);
        CHECK(sf_lagrange_table(n, xn.data(), n + 3, xq.data(), Bq.data(), Dq.data()) == SF_OK);
        for (int p = 0; p < n + 3; ++p) {
            double sb = 0.0, sd = 0.0;
            for (int i = 0; i < n; ++i) {
                sb += Bq[p * n + i];
                sd += Dq[p * n + i];
            }
            CHECK(std::fabs(sb - 1.0) <= 1e-11 && std::fabs(sd) <= 1e-9);
        }
    }
    // element dimensions and block layouts for every family, degree and form
    for (int fam = -1; fam <= 6; ++fam)
        for (int deg = 0; deg <= 10; ++deg)
            for (int form = -1; form <= 6; ++form)
                for (int prec = -1; prec <= 5; ++prec)
                    for (int io = -1; io <= 2; ++io) {
                        sf_op op{fam, deg, form, 0, prec, io, 1.0, 1.0};
                        int32_t nd = -7, nq = -7;
                        const int rc = sf_element_dims(&op, &nd, &nq);
                        if (rc == SF_OK) {
                            CHECK(nd > 0 && nq == (deg + 1) * (deg + 1) * (deg + 1));
                            int32_t nb = 0, ext[9], off[3];
                            CHECK(sf_block_layout(&op, &nb, ext, off) == SF_OK);
                            int64_t tot = 0;
                            for (int b = 0; b < nb; ++b) {
                                CHECK(off[b] == tot);
                                tot += int64_t(ext[3 * b]) * ext[3 * b + 1] * ext[3 * b + 2];
                            }
                            CHECK(tot == nd);
                        } else {
                            CHECK(rc == SF_ERR_UNSUPPORTED || rc == SF_ERR_ARG);
                        }
                    }
    CHECK(sf_element_dims(nullptr, nullptr, nullptr) == SF_ERR_ARG);
    sf_op bad{SF_Q, 2, SF_LAPLACE, 5, SF_FP64, SF_F64, 1.0, 1.0};
    CHECK(sf_element_dims(&bad, nullptr, nullptr) == SF_ERR_UNSUPPORTED);
    bad.nq1 = 0;
    bad.alpha = NAN;
    CHECK(sf_element_dims(&bad, nullptr, nullptr) == SF_ERR_ARG);
    // concatenated index: every multi-index of a 3-block element maps one to one
    {
        const int32_t ext[9] = {3, 2, 2, 2, 3, 2, 2, 2, 3};
        std::vector<int> seen(36, 0);
        for (int b = 0; b < 3; ++b)
            for (int i = 0; i < ext[3 * b]; ++i)
                for (int j = 0; j < ext[3 * b + 1]; ++j)
                    for (int k = 0; k < ext[3 * b + 2]; ++k) {
                        const int32_t m[3] = {i, j, k};
                        const int64_t r = sf_concat_index(3, 3, ext, b, m);
                        CHECK(r >= 0 && r < 36);
                        if (r >= 0 && r < 36) ++seen[r];
                    }
        for (int r = 0; r < 36; ++r) CHECK(seen[r] == 1);
        const int32_t out[3] = {3, 0, 0};
        CHECK(sf_concat_index(3, 3, ext, 0, out) == SF_ERR_ARG);
        CHECK(sf_concat_index(3, 3, ext, 3, out) == SF_ERR_ARG);
        CHECK(sf_concat_index(0, 3, ext, 0, out) == SF_ERR_ARG);
        CHECK(sf_concat_index(3, 3, nullptr, 0, out) == SF_ERR_ARG);
    }
    // axis-order planner
    {
        const int32_t in[3] = {9, 9, 9}, outq[3] = {9, 9, 9};
        int32_t order[3];
        CHECK(sf_plan_axis_order(in, outq, order) == 3 * 2 * 9 * 729);
        // the growing axis goes last: 2 (2*2*8) + 2*5*8 = 144 flops
        const int32_t in2[3] = {2, 2, 2}, out2[3] = {5, 2, 2};
        CHECK(sf_plan_axis_order(in2, out2, order) == 144);
        CHECK(order[2] == 0);
        const int32_t zero[3] = {0, 2, 2};
        CHECK(sf_plan_axis_order(zero, out2, order) == SF_ERR_ARG);
    }
    // validation before any HIP call: bad arguments never reach a launcher
    {
        sf_op op{SF_Q, 3, SF_LAPLACE, 0, SF_FP64, SF_F64, 1.0, 1.0};
        double dummy[8];
        CHECK(assemble_action(nullptr, &op, 4, dummy, nullptr, dummy, dummy + 1, nullptr) == SF_ERR_ARG);
        CHECK(assemble_element_matrix(nullptr, &op, 4, dummy, nullptr, dummy, nullptr) == SF_ERR_ARG);
        CHECK(assemble_action_global_q(nullptr, &op, 2, 2, 2, dummy, nullptr, dummy, dummy + 1, nullptr) ==
              SF_ERR_ARG);
        CHECK(sf_check_errors(nullptr, nullptr, nullptr) == SF_ERR_ARG);
        CHECK(sf_set_geometry(nullptr, SF_GEOM_BOX) == SF_ERR_ARG);
        CHECK(sf_context_destroy(nullptr) == SF_ERR_ARG);
        CHECK(sf_dof_map_q(nullptr, 2, 2, 2, 1, nullptr, nullptr) == SF_ERR_ARG);
        CHECK(sf_context_create(0, nullptr) == SF_ERR_ARG);
        // a host-side context (no device state) exercises the per-call checks
        sf_context ctx;
        CHECK(sf_set_geometry(&ctx, 9) == SF_ERR_ARG);
        CHECK(assemble_action(&ctx, &op, -1, dummy, nullptr, dummy, dummy + 1, nullptr) == SF_ERR_ARG);
        CHECK(assemble_action(&ctx, &op, 0, nullptr, nullptr, nullptr, nullptr, nullptr) == SF_OK);
        CHECK(assemble_action(&ctx, &op, 4, nullptr, nullptr, dummy, dummy + 1, nullptr) == SF_ERR_ARG);
        CHECK(assemble_action(&ctx, &op, 4, dummy, nullptr, dummy, dummy, nullptr) == SF_ERR_ARG);
        CHECK(assemble_action(&ctx, &op, 4, dummy, dummy + 1, dummy, dummy + 1, nullptr) == SF_ERR_ARG);
        sf_op res{SF_Q, 2, SF_SVK_RESIDUAL, 0, SF_FP64, SF_F64, 1.0, 1.0};
        CHECK(assemble_action(&ctx, &res, 4, dummy, dummy + 2, dummy, dummy + 1, nullptr) == SF_ERR_ARG);
        CHECK(sf_set_geometry(&ctx, SF_GEOM_TRILINEAR) == SF_OK);
        for (int prec = SF_FP32; prec <= SF_BF16X3; ++prec) {
            sf_op lo{SF_Q, 3, SF_LAPLACE, 0, prec, SF_F64, 1.0, 1.0};
            CHECK(assemble_action(&ctx, &lo, 4, dummy, nullptr, dummy, dummy + 1, nullptr) == SF_ERR_UNSUPPORTED);
        }
        sf_op lo32{SF_Q, 3, SF_LAPLACE, 0, SF_FP64, SF_F32, 1.0, 1.0};
        CHECK(assemble_action(&ctx, &lo32, 4, dummy, nullptr, dummy, dummy + 1, nullptr) == SF_ERR_UNSUPPORTED);
        sf_op mat{SF_Q, 3, SF_LAPLACE, 0, SF_BF16, SF_F64, 1.0, 1.0};
        CHECK(assemble_element_matrix(&ctx, &mat, 4, dummy, nullptr, dummy, nullptr) == SF_ERR_UNSUPPORTED);
        sf_op svk32{SF_Q, 5, SF_SVK, 0, SF_FP32, SF_F64, 1.0, 1.0};
        CHECK(assemble_element_matrix(&ctx, &svk32, 4, dummy, nullptr, dummy, nullptr) == SF_ERR_UNSUPPORTED);
        sf_op res2{SF_Q, 2, SF_SVK_RESIDUAL, 0, SF_FP64, SF_F64, 1.0, 1.0};
        CHECK(assemble_element_matrix(&ctx, &res2, 4, dummy, nullptr, dummy, nullptr) == SF_ERR_UNSUPPORTED);
        sf_op gll16{SF_QGLL, 3, SF_LAPLACE, 0, SF_FP16, SF_F64, 1.0, 1.0};
        CHECK(sf_set_geometry(&ctx, SF_GEOM_BOX) == SF_OK);
        CHECK(assemble_element_matrix(&ctx, &gll16, 4, dummy, nullptr, dummy, nullptr) == SF_ERR_UNSUPPORTED);
        CHECK(sf_set_geometry(&ctx, SF_GEOM_TRILINEAR) == SF_OK);
        CHECK(assemble_element_matrix(&ctx, &op, 4, dummy, dummy, dummy, nullptr) == SF_ERR_ARG);
        sf_op lowp{SF_Q, 3, SF_LAPLACE, 0, SF_BF16, SF_F64, 1.0, 1.0};
        CHECK(assemble_action_box_noalloc(&ctx, &lowp, 4, dummy, nullptr, dummy, dummy + 1, nullptr) ==
              SF_ERR_UNSUPPORTED);
        sf_op ncf{SF_NCF, 2, SF_HDIV, 0, SF_FP64, SF_F64, 1.0, 1.0};
        CHECK(assemble_action_box_noalloc(&ctx, &ncf, 4, dummy, nullptr, dummy, dummy + 1, nullptr) ==
              SF_ERR_UNSUPPORTED);
        CHECK(assemble_action_box_noalloc(&ctx, &op, 4, dummy, nullptr, dummy, dummy, nullptr) == SF_ERR_ARG);
        CHECK(assemble_action_box_noalloc(nullptr, &op, 4, dummy, nullptr, dummy, dummy + 1, nullptr) == SF_ERR_ARG);
        CHECK(assemble_action_box_noalloc(&ctx, &op, 0, nullptr, nullptr, nullptr, nullptr, nullptr) == SF_OK);
        sf_op glob{SF_DQ, 2, SF_LAPLACE, 0, SF_FP64, SF_F64, 1.0, 1.0};
        CHECK(assemble_action_global_q(&ctx, &glob, 2, 2, 2, dummy, nullptr, dummy, dummy + 1, nullptr) ==
              SF_ERR_UNSUPPORTED);
        CHECK(assemble_action_global_q(&ctx, &op, 0, 2, 2, dummy, nullptr, dummy, dummy + 1, nullptr) == SF_ERR_ARG);
        CHECK(assemble_action_global_q(&ctx, &op, 70000, 70000, 70000, dummy, nullptr, dummy, dummy + 1,
                                       nullptr) == SF_ERR_CAPACITY);
        CHECK(sf_dof_map_q(&ctx, 2000, 2000, 2000, 8, reinterpret_cast<int32_t *>(dummy), nullptr) ==
              SF_ERR_CAPACITY);
    }
    for (int s = -8; s <= 1; ++s) CHECK(sf_status_string(s) != nullptr);
    if (failures) {
        std::fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    std::printf("abi host checks ok\n");
    return 0;
}

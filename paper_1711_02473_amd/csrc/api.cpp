// Host side of the C ABI: validation, contexts, 1-D tables, dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "sf_internal.hpp"
#include "kron_layout.hpp"

using namespace sf;

namespace {

struct Dims {
    int nq1, ndof, nq, n0, n1;
};

bool scalar_family(int family) { return family == SF_Q || family == SF_DQ || family == SF_QGLL; }
int degree_max(int family) { return (scalar_family(family) || family == SF_VQ) ? 8 : 6; }

bool svk_form(int form) { return form == SF_SVK || form == SF_SVK_RESIDUAL; }

bool form_ok(int family, int form)
{
    if (svk_form(form)) return family == SF_Q || family == SF_QGLL;
    if (family == SF_VQ) return form == SF_MASS || form == SF_LAPLACE;
    if (scalar_family(family)) return form == SF_MASS || form == SF_LAPLACE;
    if (family == SF_NCF) return form == SF_MASS || form == SF_HDIV;
    if (family == SF_NCE) return form == SF_MASS || form == SF_HCURL;
    return false;
}

// common validation of an op; fills the element dimensions
int check_op(const sf_op *op, Dims *d)
{
    if (!op) return SF_ERR_ARG;
    if (op->family < SF_Q || op->family > SF_VQ) return SF_ERR_UNSUPPORTED;
    if (op->degree < 1 || op->degree > degree_max(op->family)) return SF_ERR_UNSUPPORTED;
    if (!form_ok(op->family, op->form)) return SF_ERR_UNSUPPORTED;
    if (op->nq1 < 0) return SF_ERR_ARG;
    if (op->precision < SF_FP64 || op->precision > SF_BF16X3) return SF_ERR_UNSUPPORTED;
    if (op->io_dtype != SF_F64 && op->io_dtype != SF_F32) return SF_ERR_UNSUPPORTED;
    if (!std::isfinite(op->alpha) || !std::isfinite(op->beta)) return SF_ERR_ARG;
    const int p = op->degree;
    const int nq1 = op->nq1 ? op->nq1 : p + 1;
    if (nq1 != p + 1) return SF_ERR_UNSUPPORTED; // kernels are built for p+1 Gauss points per axis
    if ((svk_form(op->form) || op->family == SF_VQ) && (op->precision != SF_FP64 || op->io_dtype != SF_F64))
        return SF_ERR_UNSUPPORTED;
    Dims r;
    r.nq1 = nq1;
    r.nq = nq1 * nq1 * nq1;
    if (scalar_family(op->family) || op->family == SF_VQ) {
        r.n0 = p + 1;
        r.n1 = 0;
        r.ndof = ((svk_form(op->form) || op->family == SF_VQ) ? 3 : 1) * (p + 1) * (p + 1) * (p + 1);
    } else {
        r.n0 = p + 1; // P_k factor
        r.n1 = p;     // dP_{k-1} factor
        r.ndof = (op->family == SF_NCF) ? 3 * p * p * (p + 1) : 3 * p * (p + 1) * (p + 1);
    }
    if (d) *d = r;
    return SF_OK;
}

// round-to-nearest-even conversions for the low-precision table planes
uint16_t bf16_bits(double v)
{
    float f = float(v);
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return uint16_t((u >> 16) | 0x40);
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return uint16_t(u >> 16);
}
double bf16_value(uint16_t b)
{
    uint32_t u = uint32_t(b) << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return double(f);
}
uint16_t fp16_bits(double v)
{
    _Float16 h = _Float16(float(v));
    uint16_t b;
    std::memcpy(&b, &h, 2);
    return b;
}

// Mixed-precision table planes (layout shared with mixed.hip): for the
// matrices B [nq][n], Dh [nq][nq], B^T [n][nq], Dh^T [nq][nq], four 16x16
// uint16 planes each: bf16 hi, mid, lo (v = hi + mid + lo to about 24 bits)
// and fp16.
std::vector<uint16_t> mixed_planes(const std::vector<double> &h, const TabLayout &L, int n, int nq)
{
    std::vector<uint16_t> m(4 * 4 * 256, 0);
    struct Mat { int off, rows, cols; } mats[4] = {{L.B0(), nq, n}, {L.Dh(), nq, nq}, {L.B0T(), n, nq}, {L.DhT(), nq, nq}};
    for (int k = 0; k < 4; ++k)
        for (int r = 0; r < mats[k].rows; ++r)
            for (int c = 0; c < mats[k].cols; ++c) {
                const double v = h[mats[k].off + size_t(r) * mats[k].cols + c];
                const uint16_t hi = bf16_bits(v);
                const double r1 = v - bf16_value(hi);
                const uint16_t mid = bf16_bits(r1);
                const uint16_t lo = bf16_bits(r1 - bf16_value(mid));
                uint16_t *base = m.data() + k * 1024 + r * 16 + c;
                base[0] = hi;
                base[256] = mid;
                base[512] = lo;
                base[768] = fp16_bits(v);
            }
    return m;
}

// Dense Kronecker table block of the low-degree mixed-precision action (layout in
// kron_layout.hpp) from the FP64 tables B = B0 [nq][n] and D = D0 [nq][n], n = nq <= 4.
std::vector<uint16_t> kron_block(const std::vector<double> &h, const TabLayout &L, int n)
{
    const KronLayout K(n);
    std::vector<uint16_t> out(K.total(), 0);
    const int nd = K.nd;
    auto B = [&](int q, int i) { return h[L.B0() + q * n + i]; };
    auto D = [&](int q, int i) { return h[L.D0() + q * n + i]; };
    // G_mat[q][i]; mat 0: B B B, 1: D B B, 2: B D B, 3: B B D (first factor on axis 0)
    auto G = [&](int mat, int q, int i) {
        if (q >= nd || i >= nd) return 0.0;
        const int q0 = q / (n * n), q1 = (q / n) % n, q2 = q % n;
        const int i0 = i / (n * n), i1 = (i / n) % n, i2 = i % n;
        return (mat == 1 ? D(q0, i0) : B(q0, i0)) * (mat == 2 ? D(q1, i1) : B(q1, i1)) *
               (mat == 3 ? D(q2, i2) : B(q2, i2));
    };
    auto planes = [&](double v, uint16_t p[4]) {
        p[0] = bf16_bits(v);
        const double r1 = v - bf16_value(p[0]);
        p[1] = bf16_bits(r1);
        p[2] = bf16_bits(r1 - bf16_value(p[1]));
        p[3] = fp16_bits(v);
    };
    for (int mat = 0; mat < 4; ++mat) {
        for (int m = 0; m < K.MT; ++m)
            for (int s = 0; s < K.KS; ++s)
                for (int l = 0; l < 64; ++l)
                    for (int j = 0; j < 8; ++j) {
                        uint16_t p[4];
                        planes(G(mat, 16 * m + l % 16, 32 * s + 8 * (l / 16) + j), p);
                        const int e = ((m * K.KS + s) * 64 + l) * 8 + j;
                        for (int pl = 0; pl < 4; ++pl) out[K.fwd(mat, pl) + e] = p[pl];
                    }
        for (int t = 0; t < K.NT; ++t)
            for (int m2 = 0; m2 < K.MT2; ++m2)
                for (int l = 0; l < 64; ++l)
                    for (int j = 0; j < 8; ++j) {
                        uint16_t p[4];
                        planes(G(mat, 32 * m2 + 16 * (j / 4) + 4 * (l / 16) + j % 4, 16 * t + l % 16), p);
                        const int e = ((t * K.MT2 + m2) * 64 + l) * 8 + j;
                        for (int pl = 0; pl < 4; ++pl) out[K.bwd(mat, pl) + e] = p[pl];
                    }
    }
    for (int q = 0; q < K.MT * 16; ++q) {
        float w = 0.0f;
        if (q < nd) {
            const int q0 = q / (n * n), q1 = (q / n) % n, q2 = q % n;
            w = float(h[L.W() + q0] * h[L.W() + q1] * h[L.W() + q2]);
        }
        std::memcpy(&out[K.w3() + 2 * q], &w, 4);
    }
    return out;
}

// Split Kronecker tables of the mixed-precision action at 5 <= n <= 9 (layout in
// kron_layout.hpp) from the FP64 tables B = B0 [nq][n] and D = D0 [nq][n], n = nq.
std::vector<uint16_t> kron2_block(const std::vector<double> &h, const TabLayout &L, int n)
{
    const Kron2Layout K(n);
    std::vector<uint16_t> out(K.total(), 0);
    const int q2 = K.q2;
    auto B = [&](int q, int i) { return h[L.B0() + q * n + i]; };
    auto D = [&](int q, int i) { return h[L.D0() + q * n + i]; };
    // plane matrix pm [q1 n + q2][i1 n + i2]: 0 B B, 1 D B, 2 B D (first factor on axis 1)
    auto Pm = [&](int pm, int q, int i) {
        if (q >= q2 || i >= q2) return 0.0;
        const int q1 = q / n, qq = q % n, i1 = i / n, ii = i % n;
        return (pm == 1 ? D(q1, i1) : B(q1, i1)) * (pm == 2 ? D(qq, ii) : B(qq, ii));
    };
    // block-diagonal axis-0 matrix am (0 B, 1 D) on tile rows (slot, q0) x (slot, i0)
    auto Mb = [&](int am, int r, int c) {
        if (r / K.rs != c / K.rs || r / K.rs >= K.cpt) return 0.0;
        const int q = r % K.rs, i = c % K.rs;
        if (q >= n || i >= n) return 0.0;
        return am == 1 ? D(q, i) : B(q, i);
    };
    auto planes = [&](double v, uint16_t p[4]) {
        p[0] = bf16_bits(v);
        const double r1 = v - bf16_value(p[0]);
        p[1] = bf16_bits(r1);
        p[2] = bf16_bits(r1 - bf16_value(p[1]));
        p[3] = fp16_bits(v);
    };
    for (int pm = 0; pm < 3; ++pm) {
        for (int c = 0; c < K.NQ; ++c)
            for (int k = 0; k < K.KS; ++k)
                for (int l = 0; l < 64; ++l)
                    for (int j = 0; j < 8; ++j) {
                        uint16_t p[4];
                        planes(Pm(pm, 16 * c + l % 16, 32 * k + 8 * (l / 16) + j), p);
                        const int e = ((c * K.KS + k) * 64 + l) * 8 + j;
                        for (int pl = 0; pl < 4; ++pl) out[K.s1f(pm, pl) + e] = p[pl];
                    }
        for (int t = 0; t < K.NQ; ++t)
            for (int m = 0; m < K.NQ2; ++m)
                for (int l = 0; l < 64; ++l)
                    for (int j = 0; j < 8; ++j) {
                        uint16_t p[4];
                        planes(Pm(pm, 32 * m + 16 * (j / 4) + 4 * (l / 16) + j % 4, 16 * t + l % 16), p);
                        const int e = ((t * K.NQ2 + m) * 64 + l) * 8 + j;
                        for (int pl = 0; pl < 4; ++pl) out[K.s1b(pm, pl) + e] = p[pl];
                    }
    }
    for (int am = 0; am < 2; ++am)
        for (int l = 0; l < 64; ++l)
            for (int j = 0; j < 4; ++j) {
                uint16_t pf[4], pb[4];
                planes(Mb(am, l % 16, 4 * (l / 16) + j), pf);
                planes(Mb(am, 4 * (l / 16) + j, l % 16), pb);
                for (int pl = 0; pl < 4; ++pl) {
                    out[K.s2f(am, pl) + l * 4 + j] = pf[pl];
                    out[K.s2b(am, pl) + l * 4 + j] = pb[pl];
                }
            }
    for (int q = 0; q < K.NQ * 16; ++q) {
        const float w = q < q2 ? float(h[L.W() + q / n] * h[L.W() + q % n]) : 0.0f;
        std::memcpy(&out[K.w2() + 2 * q], &w, 4);
    }
    for (int r = 0; r < 16; ++r) {
        const int q = r % K.rs;
        const float w = (r / K.rs < K.cpt && q < n) ? float(h[L.W() + q]) : 0.0f;
        std::memcpy(&out[K.w0() + 2 * r], &w, 4);
    }
    return out;
}

// Even-odd packing of a square n x n row-major matrix M at h[src] with
// M[n-1-q][n-1-i] = s M[q][i] (s = -1 when skew): for each row q < n/2 the
// entries (M[q][i] + M[q][n-1-i]) / 2 for i < n/2, M[q][n/2] when n is odd,
// then (M[q][i] - M[q][n-1-i]) / 2 for i < n/2; for odd n the middle row
// M[n/2][0..n/2] follows.  Returns false if M lacks the symmetry.
bool pack_eo(std::vector<double> &h, int src, int dst, int n, bool skew)
{
    const double s = skew ? -1.0 : 1.0;
    double scale = 0.0;
    for (int k = 0; k < n * n; ++k) scale = std::max(scale, std::fabs(h[src + k]));
    for (int q = 0; q < n; ++q)
        for (int i = 0; i < n; ++i)
            if (std::fabs(h[src + (n - 1 - q) * n + (n - 1 - i)] - s * h[src + q * n + i]) > 1e-12 * scale) return false;
    const int hh = n / 2, od = n % 2, rw = 2 * hh + od;
    auto M = [&](int q, int i) { return h[src + q * n + i]; };
    for (int q = 0; q < hh; ++q) {
        for (int i = 0; i < hh; ++i) h[dst + q * rw + i] = 0.5 * (M(q, i) + M(q, n - 1 - i));
        if (od) h[dst + q * rw + hh] = M(q, hh);
        for (int i = 0; i < hh; ++i) h[dst + q * rw + hh + od + i] = 0.5 * (M(q, i) - M(q, n - 1 - i));
    }
    if (od)
        for (int i = 0; i <= hh; ++i) h[dst + hh * rw + i] = M(hh, i);
    return true;
}

// The same packing for a rectangular no x ni matrix with M[no-1-q][ni-1-i] = s M[q][i]:
// rows q < no/2 hold the ni/2 half-sums, M[q][ni/2] when ni is odd, then the ni/2
// half-differences; for odd no the middle row's first ni/2 + ni%2 entries follow
// (the output equals pack_eo's when no == ni).  Returns false if M lacks the symmetry.
bool pack_eo_rect(std::vector<double> &h, int src, int dst, int no, int ni, bool skew)
{
    const double s = skew ? -1.0 : 1.0;
    double scale = 0.0;
    for (int k = 0; k < no * ni; ++k) scale = std::max(scale, std::fabs(h[src + k]));
    auto M = [&](int q, int i) { return h[src + size_t(q) * ni + i]; };
    for (int q = 0; q < no; ++q)
        for (int i = 0; i < ni; ++i)
            if (std::fabs(M(no - 1 - q, ni - 1 - i) - s * M(q, i)) > 1e-12 * scale) return false;
    const int hi = ni / 2, oi = ni % 2, ho = no / 2, rw = 2 * hi + oi;
    for (int q = 0; q < ho; ++q) {
        for (int i = 0; i < hi; ++i) h[dst + q * rw + i] = 0.5 * (M(q, i) + M(q, ni - 1 - i));
        if (oi) h[dst + q * rw + hi] = M(q, hi);
        for (int i = 0; i < hi; ++i) h[dst + q * rw + hi + oi + i] = 0.5 * (M(q, i) - M(q, ni - 1 - i));
    }
    if (no % 2)
        for (int i = 0; i < hi + oi; ++i) h[dst + ho * rw + i] = M(ho, i);
    return true;
}

} // namespace

namespace sf {
// The FP64 table block of one (family, degree, nq1) in the TabLayout order
// (host only, no device state).  Returns SF_OK or SF_ERR_UNSUPPORTED.
int host_table_block(int family, int n0, int n1, int nq1, std::vector<double> &h)
{
    TabLayout L(n0, n1, nq1);
    h.assign(L.size(), 0.0);
    std::vector<double> xq(nq1), wq(nq1), x0(n0), w0(n0), x1(std::max(n1, 1)), w1(std::max(n1, 1));
    // quadrature: GL, or GLL for the collocated variant (nodes = points, B = I)
    rule_1d(family == SF_QGLL ? 1 : 0, nq1, xq.data(), wq.data());
    if (family == SF_DQ) rule_1d(0, n0, x0.data(), w0.data());
    else rule_1d(1, n0, x0.data(), w0.data()); // Q_p and the P_k factor: GLL nodes
    lagrange_table(n0, x0.data(), nq1, xq.data(), h.data() + L.B0(), h.data() + L.D0());
    if (n1 > 0) {
        rule_1d(0, n1, x1.data(), w1.data()); // dP_{k-1}: GL nodes
        lagrange_table(n1, x1.data(), nq1, xq.data(), h.data() + L.B1(), h.data() + L.D1());
    }
    std::vector<double> tmpB(size_t(nq1) * nq1);
    lagrange_table(nq1, xq.data(), nq1, xq.data(), tmpB.data(), h.data() + L.Dh());
    std::copy(wq.begin(), wq.end(), h.begin() + L.W());
    std::copy(xq.begin(), xq.end(), h.begin() + L.XQ());
    auto transpose = [&](int src, int dst, int rows, int cols) {
        for (int r = 0; r < rows; ++r)
            for (int c = 0; c < cols; ++c) h[dst + size_t(c) * rows + r] = h[src + size_t(r) * cols + c];
    };
    transpose(L.B0(), L.B0T(), nq1, n0);
    transpose(L.D0(), L.D0T(), nq1, n0);
    transpose(L.B1(), L.B1T(), nq1, n1);
    transpose(L.D1(), L.D1T(), nq1, n1);
    transpose(L.Dh(), L.DhT(), nq1, nq1);
    if (n0 == nq1) {
        // node and point sets are symmetric about 1/2, so B and B^T are centrosymmetric and
        // Dh, Dh^T skew-centrosymmetric; pack their even-odd forms (see apply_eo)
        const bool ok = pack_eo(h, L.B0(), L.BEO(), nq1, false) && pack_eo(h, L.B0T(), L.BTEO(), nq1, false) &&
                        pack_eo(h, L.Dh(), L.DhEO(), nq1, true) && pack_eo(h, L.DhT(), L.DhTEO(), nq1, true);
        if (!ok) return SF_ERR_UNSUPPORTED;
    }
    if (n1 > 0) {
        // enriched elements: D0 (skew), B1 (node sets GLL_n0 / GL_n1, points GL) and their
        // transposes in even-odd form; the 3-D weight products
        const bool ok = pack_eo_rect(h, L.D0(), L.D0EO(), nq1, n0, true) &&
                        pack_eo_rect(h, L.D0T(), L.D0TEO(), n0, nq1, true) &&
                        pack_eo_rect(h, L.B1(), L.B1EO(), nq1, n1, false) &&
                        pack_eo_rect(h, L.B1T(), L.B1TEO(), n1, nq1, false);
        if (!ok) return SF_ERR_UNSUPPORTED;
        for (int a = 0; a < nq1; ++a)
            for (int b = 0; b < nq1; ++b)
                for (int c = 0; c < nq1; ++c) h[L.W3() + (a * nq1 + b) * nq1 + c] = wq[a] * wq[b] * wq[c];
    }
    return SF_OK;
}
} // namespace sf

namespace {

int build_tables(sf_context *ctx, const sf_op *op, const Dims &d, TableSet **out)
{
    auto key = std::make_tuple(int(op->family), int(op->degree), d.nq1);
    auto it = ctx->tables.find(key);
    if (it != ctx->tables.end()) {
        *out = &it->second;
        return SF_OK;
    }
    TabLayout L(d.n0, d.n1, d.nq1);
    std::vector<double> h;
    const int hrc = host_table_block(op->family, d.n0, d.n1, d.nq1, h);
    if (hrc) return hrc;

    TableSet ts;
    ts.len = L.size();
    std::vector<float> hf(h.begin(), h.end());
    if (hipMalloc(&ts.d64, sizeof(double) * h.size()) != hipSuccess) return SF_ERR_NOMEM;
    if (hipMalloc(&ts.f32, sizeof(float) * h.size()) != hipSuccess) {
        (void)hipFree(ts.d64);
        return SF_ERR_NOMEM;
    }
    if (hipMemcpy(ts.d64, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(ts.f32, hf.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(ts.d64);
        (void)hipFree(ts.f32);
        return SF_ERR_HIP;
    }
    if (scalar_family(op->family)) {
        std::vector<uint16_t> mp = mixed_planes(h, L, d.n0, d.nq1);
        if (hipMalloc(&ts.mixed, sizeof(uint16_t) * mp.size()) != hipSuccess) {
            (void)hipFree(ts.d64);
            (void)hipFree(ts.f32);
            return SF_ERR_NOMEM;
        }
        if (hipMemcpy(ts.mixed, mp.data(), sizeof(uint16_t) * mp.size(), hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(ts.d64);
            (void)hipFree(ts.f32);
            (void)hipFree(ts.mixed);
            return SF_ERR_HIP;
        }
        if (d.n0 == d.nq1 && d.nq1 <= kKron2MaxN) {
            std::vector<uint16_t> kb = d.nq1 <= kKronMaxN ? kron_block(h, L, d.nq1) : kron2_block(h, L, d.nq1);
            if (hipMalloc(&ts.kron, sizeof(uint16_t) * kb.size()) != hipSuccess ||
                hipMemcpy(ts.kron, kb.data(), sizeof(uint16_t) * kb.size(), hipMemcpyHostToDevice) != hipSuccess) {
                (void)hipFree(ts.d64);
                (void)hipFree(ts.f32);
                (void)hipFree(ts.mixed);
                (void)hipFree(ts.kron);
                return SF_ERR_NOMEM;
            }
        }
    }
    auto res = ctx->tables.emplace(key, ts);
    *out = &res.first->second;
    return SF_OK;
}

int make_args(sf_context *ctx, const sf_op *op, int64_t ncells, const double *vertices, const void *kappa,
              void *stream, LaunchArgs &a, Dims &d)
{
    int rc = check_op(op, &d);
    if (rc) return rc;
    TableSet *ts = nullptr;
    rc = build_tables(ctx, op, d, &ts);
    if (rc) return rc;
    a = LaunchArgs{};
    a.family = op->family;
    a.degree = op->degree;
    a.form = op->form;
    a.nq = d.nq1;
    a.n0 = d.n0;
    a.n1 = d.n1;
    a.precision = op->precision;
    a.io = op->io_dtype;
    a.alpha = op->alpha;
    a.beta = op->beta;
    a.ncells = ncells;
    a.vert = vertices;
    a.kappa = kappa;
    a.tab64 = ts->d64;
    a.tab32 = ts->f32;
    a.tabmix = ts->mixed;
    a.tabkron = ts->kron;
    a.err = ctx->d_err;
    a.stream = static_cast<hipStream_t>(stream);
    a.variant = 0;
    return SF_OK;
}

} // namespace

namespace sf {
std::string tune_key(const sf_op *op, const char *what)
{
    char b[160];
    snprintf(b, sizeof b, "gfx950|fam%d|p%d|form%d|nq%d|prec%d|io%d|%s", op->family, op->degree, op->form,
             op->nq1 ? op->nq1 : op->degree + 1, op->precision, op->io_dtype, what);
    return b;
}
int tuned_variant_of(sf_context *ctx, const sf_op *op, const char *what, int dflt)
{
    auto it = ctx->tuned.find(tune_key(op, what));
    return it == ctx->tuned.end() ? dflt : it->second;
}
int op_dims(const sf_op *op, int *ndof, int *nq)
{
    Dims d;
    int rc = check_op(op, &d);
    if (rc) return rc;
    *ndof = d.ndof;
    *nq = d.nq;
    return SF_OK;
}
int ensure_tables(sf_context *ctx, const sf_op *op, LaunchArgs &a)
{
    Dims d;
    return make_args(ctx, op, 0, nullptr, nullptr, nullptr, a, d);
}
} // namespace sf

extern "C" {

const char *sf_status_string(int status)
{
    switch (status) {
    case SF_OK: return "ok";
    case SF_ERR_ARG: return "invalid argument";
    case SF_ERR_UNSUPPORTED: return "unsupported family/degree/form/nq1/precision combination";
    case SF_ERR_NOMEM: return "out of memory";
    case SF_ERR_HIP: return "HIP runtime error";
    case SF_ERR_GEOMETRY: return "degenerate or unsupported cell geometry (det J <= 0, non-affine or non-box)";
    case SF_ERR_CAPACITY: return "size exceeds a documented maximum";
    default: return "unknown status";
    }
}

int sf_context_create(int hip_device, sf_context **out)
{
    if (!out) return SF_ERR_ARG;
    *out = nullptr;
    if (hipSetDevice(hip_device) != hipSuccess) return SF_ERR_HIP;
    sf_context *ctx = new (std::nothrow) sf_context();
    if (!ctx) return SF_ERR_NOMEM;
    ctx->device = hip_device;
    if (hipMalloc(&ctx->d_err, sizeof(int)) != hipSuccess) {
        delete ctx;
        return SF_ERR_NOMEM;
    }
    if (hipMemset(ctx->d_err, 0, sizeof(int)) != hipSuccess) {
        (void)hipFree(ctx->d_err);
        delete ctx;
        return SF_ERR_HIP;
    }
    // the allocation-free entry point's scratch array on this device (once per device)
    if (const int nrc = noalloc_setup(hip_device)) {
        (void)hipFree(ctx->d_err);
        delete ctx;
        return nrc;
    }
    if (hipMalloc(&ctx->d_sched, sizeof(int) * kSchedSlotInts * kSchedSlots) != hipSuccess) {
        (void)hipFree(ctx->d_err);
        delete ctx;
        return SF_ERR_NOMEM;
    }
    if (hipMemset(ctx->d_sched, 0, sizeof(int) * kSchedSlotInts * kSchedSlots) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        (void)hipFree(ctx->d_err);
        (void)hipFree(ctx->d_sched);
        delete ctx;
        return SF_ERR_HIP;
    }
    *out = ctx;
    return SF_OK;
}

int sf_context_destroy(sf_context *ctx)
{
    if (!ctx) return SF_ERR_ARG;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (auto &kv : ctx->tables) {
        (void)hipFree(kv.second.d64);
        (void)hipFree(kv.second.f32);
        if (kv.second.mixed) (void)hipFree(kv.second.mixed);
        if (kv.second.kron) (void)hipFree(kv.second.kron);
    }
    (void)hipFree(ctx->d_err);
    (void)hipFree(ctx->d_sched);
    delete ctx;
    return SF_OK;
}

int sf_set_geometry(sf_context *ctx, int32_t geometry)
{
    if (!ctx || (geometry != SF_GEOM_AFFINE && geometry != SF_GEOM_BOX && geometry != SF_GEOM_TRILINEAR))
        return SF_ERR_ARG;
    ctx->geometry = geometry;
    return SF_OK;
}

int sf_element_dims(const sf_op *op, int32_t *ndof_cell, int32_t *nq_cell)
{
    Dims d;
    int rc = check_op(op, &d);
    if (rc) return rc;
    if (ndof_cell) *ndof_cell = d.ndof;
    if (nq_cell) *nq_cell = d.nq;
    return SF_OK;
}

int assemble_action(sf_context *ctx, const sf_op *op, int64_t ncells, const double *vertices, const void *kappa,
                    const void *u, void *y, void *hip_stream)
{
    if (!ctx || !op || ncells < 0) return SF_ERR_ARG;
    Dims d;
    int rc = check_op(op, &d);
    if (rc) return rc;
    if (ncells == 0) return SF_OK;
    if (!vertices || !u || !y) return SF_ERR_ARG;
    if (y == u || y == kappa) return SF_ERR_ARG;
    // checks that need no device state come before make_args (which may allocate tables)
    if (op->form == SF_SVK_RESIDUAL && kappa) return SF_ERR_ARG;
    if (ctx->geometry == SF_GEOM_TRILINEAR && (op->precision != SF_FP64 || op->io_dtype != SF_F64))
        return SF_ERR_UNSUPPORTED; // per-point geometry is built for FP64 contractions and storage
    LaunchArgs a;
    rc = make_args(ctx, op, ncells, vertices, kappa, hip_stream, a, d);
    if (rc) return rc;
    a.u = u;
    a.y = y;
    if (svk_form(op->form) || op->family == SF_VQ) {
        a.trilinear = ctx->geometry == SF_GEOM_TRILINEAR;
        return launch_action_vq(a);
    }
    if (op->precision == SF_BF16 || op->precision == SF_FP16 || op->precision == SF_BF16X3) {
        // variant 0: the dense Kronecker form where it is built (n = p + 1 <= 4), else
        // the sum-factorised kernel; 1: always the sum-factorised kernel
        a.variant = tuned_variant_of(ctx, op, "standalone", 0);
        return launch_action_mixed(a);
    }
    if (scalar_family(op->family)) {
        if (ctx->geometry == SF_GEOM_TRILINEAR) {
            a.trilinear = true;
            return launch_action_q(a);
        }
        if (ctx->geometry == SF_GEOM_BOX) {
            // variants 0..2: box-cell kernels; 3: the general three-tensor kernel
            a.variant = tuned_variant_of(ctx, op, "standalone", 0);
            a.sched = ctx->d_sched + kSchedSlotInts * (ctx->sched_next++ % kSchedSlots);
            return a.variant == 3 ? launch_action_q(a) : launch_action_q_fast(a);
        }
        return launch_action_q(a);
    }
    a.trilinear = ctx->geometry == SF_GEOM_TRILINEAR;
    a.box = ctx->geometry == SF_GEOM_BOX;
    // variant 0: the fused box-cell kernel on box contexts, the persistent affine kernel
    // otherwise; 1: one group per workgroup; 2: the persistent affine kernel.  Untuned NCE_6
    // on boxes takes 2 (the fused form's registers spill at that degree).
    a.variant = tuned_variant_of(ctx, op, "standalone", a.box && op->family == SF_NCE && op->degree == 6 ? 2 : 0);
    return launch_action_vec(a);
}

int assemble_action_box_noalloc(sf_context *ctx, const sf_op *op, int64_t ncells, const double *vertices,
                                const void *kappa, const void *u, void *y, void *hip_stream)
{
    if (!ctx || !op || ncells < 0) return SF_ERR_ARG;
    Dims d;
    int rc = check_op(op, &d);
    if (rc) return rc;
    if (!scalar_family(op->family) || (op->form != SF_MASS && op->form != SF_LAPLACE) ||
        (op->precision != SF_FP64 && op->precision != SF_FP32))
        return SF_ERR_UNSUPPORTED;
    if (ncells == 0) return SF_OK;
    if (!vertices || !u || !y || y == u || y == kappa) return SF_ERR_ARG;
    // no make_args: its table cache allocates; the tables come from the scratch array
    LaunchArgs a{};
    a.family = op->family;
    a.degree = op->degree;
    a.form = op->form;
    a.nq = d.nq1;
    a.n0 = d.n0;
    a.n1 = d.n1;
    a.precision = op->precision;
    a.io = op->io_dtype;
    a.alpha = op->alpha;
    a.beta = op->beta;
    a.ncells = ncells;
    a.vert = vertices;
    a.kappa = kappa;
    a.u = u;
    a.y = y;
    a.err = ctx->d_err;
    a.stream = static_cast<hipStream_t>(hip_stream);
    a.variant = tuned_variant_of(ctx, op, "standalone", 0);
    return launch_action_box_noalloc(a, ctx->device);
}

int assemble_action_global_q(sf_context *ctx, const sf_op *op, int32_t nx, int32_t ny, int32_t nz,
                             const double *vertices, const void *kappa, const void *u_global, void *y_global,
                             void *hip_stream)
{
    if (!ctx || !op || nx < 1 || ny < 1 || nz < 1) return SF_ERR_ARG;
    Dims d;
    int rc = check_op(op, &d);
    if (rc) return rc;
    if (op->family != SF_Q || op->precision != SF_FP64 || op->io_dtype != SF_F64 ||
        (op->form != SF_LAPLACE && op->form != SF_MASS))
        return SF_ERR_UNSUPPORTED;
    const int64_t ncells = int64_t(nx) * ny * nz;
    const int64_t ng = (int64_t(nx) * op->degree + 1) * (int64_t(ny) * op->degree + 1) * (int64_t(nz) * op->degree + 1);
    if (ng > (int64_t(1) << 40)) return SF_ERR_CAPACITY;
    if (!vertices || !u_global || !y_global || y_global == u_global || y_global == kappa) return SF_ERR_ARG;
    LaunchArgs a;
    rc = make_args(ctx, op, ncells, vertices, kappa, hip_stream, a, d);
    if (rc) return rc;
    a.u = u_global;
    a.y = y_global;
    a.sched = ctx->d_sched + kSchedSlotInts * (ctx->sched_next++ % kSchedSlots);
    return launch_action_q_global(a, nx, ny, nz);
}

int assemble_element_matrix(sf_context *ctx, const sf_op *op, int64_t ncells, const double *vertices,
                            const void *kappa, void *A, void *hip_stream)
{
    if (!ctx || !op || ncells < 0) return SF_ERR_ARG;
    Dims d;
    int rc = check_op(op, &d);
    if (rc) return rc;
    if (op->form == SF_SVK_RESIDUAL) return SF_ERR_UNSUPPORTED;
    // lower-precision contractions: the box-cell kernel of Q_p / dQ_p (final contraction on MFMA)
    if (op->precision != SF_FP64 &&
        (op->precision == SF_FP32 || (op->family != SF_Q && op->family != SF_DQ) || ctx->geometry != SF_GEOM_BOX))
        return SF_ERR_UNSUPPORTED;
    if (ncells == 0) return SF_OK;
    if (!vertices || !A || A == kappa) return SF_ERR_ARG;
    LaunchArgs a;
    rc = make_args(ctx, op, ncells, vertices, kappa, hip_stream, a, d);
    if (rc) return rc;
    a.A = A;
    if (op->form == SF_SVK) {
        a.trilinear = ctx->geometry == SF_GEOM_TRILINEAR;
        return launch_matrix_svk(a);
    }
    a.trilinear = ctx->geometry == SF_GEOM_TRILINEAR;
    // collocated families (points = nodes, B = I): the O(n^5) structured assembly, any geometry
    if ((op->family == SF_QGLL || op->family == SF_DQ) && op->precision == SF_FP64) return launch_matrix_coll(a);
    if (scalar_family(op->family) || op->family == SF_VQ)
        return ctx->geometry == SF_GEOM_BOX ? launch_matrix_q(a) : launch_matrix_qgen(a);
    return launch_matrix_vec(a);
}

int sf_check_errors(sf_context *ctx, void *hip_stream, int32_t *flags)
{
    if (!ctx) return SF_ERR_ARG;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (hipStreamSynchronize(s) != hipSuccess) return SF_ERR_HIP;
    int h = 0;
    if (hipMemcpy(&h, ctx->d_err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return SF_ERR_HIP;
    if (h && hipMemset(ctx->d_err, 0, sizeof(int)) != hipSuccess) return SF_ERR_HIP;
    if (flags) *flags = h;
    return h ? SF_ERR_GEOMETRY : SF_OK;
}

int sf_dof_map_q(sf_context *ctx, int32_t nx, int32_t ny, int32_t nz, int32_t p, int32_t *map_device,
                 void *hip_stream)
{
    if (!ctx || nx < 1 || ny < 1 || nz < 1 || p < 1 || !map_device) return SF_ERR_ARG;
    const double nglob = (double(nx) * p + 1) * (double(ny) * p + 1) * (double(nz) * p + 1);
    const double nentries = double(nx) * ny * nz * double(p + 1) * (p + 1) * (p + 1);
    if (nglob > 2147483647.0 || nentries > 9.0e15) return SF_ERR_CAPACITY;
    return launch_dofmap_q(nx, ny, nz, p, map_device, static_cast<hipStream_t>(hip_stream));
}

int64_t sf_concat_index(int32_t ndim, int32_t nblocks, const int32_t *extents, int32_t block, const int32_t *multi)
{
    if (ndim < 1 || ndim > 16 || nblocks < 1 || !extents || !multi || block < 0 || block >= nblocks) return SF_ERR_ARG;
    int64_t off = 0;
    for (int b = 0; b < block; ++b) {
        int64_t sz = 1;
        for (int a = 0; a < ndim; ++a) {
            if (extents[b * ndim + a] < 1) return SF_ERR_ARG;
            sz *= extents[b * ndim + a];
        }
        off += sz;
    }
    int64_t idx = 0;
    for (int a = 0; a < ndim; ++a) {
        const int e = extents[block * ndim + a];
        if (e < 1 || multi[a] < 0 || multi[a] >= e) return SF_ERR_ARG;
        idx = idx * e + multi[a];
    }
    return off + idx;
}

int sf_block_layout(const sf_op *op, int32_t *nblocks, int32_t *extents, int32_t *offsets)
{
    Dims d;
    int rc = check_op(op, &d);
    if (rc) return rc;
    if (!nblocks || !extents || !offsets) return SF_ERR_ARG;
    const int p = op->degree;
    if (svk_form(op->form) || op->family == SF_VQ) { // vector element: one scalar block per component
        *nblocks = 3;
        for (int c = 0; c < 3; ++c) {
            extents[c * 3] = extents[c * 3 + 1] = extents[c * 3 + 2] = p + 1;
            offsets[c] = c * (p + 1) * (p + 1) * (p + 1);
        }
        return SF_OK;
    }
    if (scalar_family(op->family)) {
        *nblocks = 1;
        extents[0] = extents[1] = extents[2] = p + 1;
        offsets[0] = 0;
        return SF_OK;
    }
    *nblocks = 3;
    int off = 0;
    for (int c = 0; c < 3; ++c) {
        for (int a = 0; a < 3; ++a) {
            const bool pk = (op->family == SF_NCF) ? (a == c) : (a != c);
            extents[c * 3 + a] = pk ? p + 1 : p;
        }
        offsets[c] = off;
        off += extents[c * 3] * extents[c * 3 + 1] * extents[c * 3 + 2];
    }
    return SF_OK;
}

int64_t sf_plan_axis_order(const int32_t *in, const int32_t *out, int32_t *order)
{
    if (!in || !out || !order) return SF_ERR_ARG;
    for (int a = 0; a < 3; ++a)
        if (in[a] < 1 || out[a] < 1) return SF_ERR_ARG;
    int perm[3] = {0, 1, 2};
    int64_t best = -1;
    do {
        int64_t cur[3] = {in[0], in[1], in[2]};
        int64_t flops = 0;
        for (int s = 0; s < 3; ++s) {
            const int ax = perm[s];
            flops += 2 * int64_t(out[ax]) * cur[0] * cur[1] * cur[2];
            cur[ax] = out[ax];
        }
        if (best < 0 || flops < best) {
            best = flops;
            std::copy(perm, perm + 3, order);
        }
    } while (std::next_permutation(perm, perm + 3));
    return best;
}

} // extern "C"

// Internal declarations shared by the host API and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/sf.h"

namespace sf {

constexpr int kMaxRule = 32;

int rule_1d(int kind, int m, double *x, double *w);
int lagrange_table(int nn, const double *nodes, int np, const double *pts, double *B, double *D);

// Layout of the per-(family, degree, nq1) table block, identical for every
// storage type.  Space 0 has n0 functions (Q: GLL nodes; dQ: GL nodes; NCF /
// NCE: the P_k factor on GLL_{k+1}); space 1 has n1 functions (NCF / NCE: the
// dP_{k-1} factor on GL_k; 0 for scalar families).
//   B0[nq][n0]  values of space 0 at the GL points
//   D0[nq][n0]  derivatives of space 0
//   B1[nq][n1], D1[nq][n1]
//   Dh[nq][nq]  collocation derivative of the Lagrange basis on the GL points
//   w[nq]       GL weights on [0,1]
//   then the transposes B0T[n0][nq], D0T[n0][nq], B1T[n1][nq], D1T[n1][nq],
//   DhT[nq][nq], so that every contraction reads its matrix by contiguous rows.
struct TabLayout {
    int n0, n1, nq;
    __host__ __device__ constexpr TabLayout(int a, int b, int c) : n0(a), n1(b), nq(c) {}
    __host__ __device__ constexpr int B0() const { return 0; }
    __host__ __device__ constexpr int D0() const { return nq * n0; }
    __host__ __device__ constexpr int B1() const { return 2 * nq * n0; }
    __host__ __device__ constexpr int D1() const { return 2 * nq * n0 + nq * n1; }
    __host__ __device__ constexpr int Dh() const { return 2 * nq * (n0 + n1); }
    __host__ __device__ constexpr int W() const { return 2 * nq * (n0 + n1) + nq * nq; }
    __host__ __device__ constexpr int B0T() const { return W() + nq; }
    __host__ __device__ constexpr int D0T() const { return B0T() + nq * n0; }
    __host__ __device__ constexpr int B1T() const { return D0T() + nq * n0; }
    __host__ __device__ constexpr int D1T() const { return B1T() + nq * n1; }
    __host__ __device__ constexpr int DhT() const { return D1T() + nq * n1; }
    // even-odd packed forms of the square matrices B0 (when n0 == nq), B0^T, Dh, Dh^T
    __host__ __device__ static constexpr int eo_len(int n)
    {
        return (n / 2) * (2 * (n / 2) + n % 2) + (n % 2) * (n / 2 + 1);
    }
    __host__ __device__ constexpr int BEO() const { return DhT() + nq * nq; }
    __host__ __device__ constexpr int BTEO() const { return BEO() + eo_len(nq); }
    __host__ __device__ constexpr int DhEO() const { return BTEO() + eo_len(nq); }
    __host__ __device__ constexpr int DhTEO() const { return DhEO() + eo_len(nq); }
    __host__ __device__ constexpr int XQ() const { return DhTEO() + eo_len(nq); } // quadrature points
    // Enriched (two-factor) elements only, empty when n1 == 0: even-odd packed forms of
    // D0, D0^T (skew) and of the rectangular B1, B1^T, and the products w_q0 w_q1 w_q2
    // of the 1-D weights at the n_q^3 points (index (q0 nq + q1) nq + q2).
    __host__ __device__ static constexpr int eo_len2(int no, int ni)
    {
        return (no / 2) * (2 * (ni / 2) + ni % 2) + (no % 2) * (ni / 2 + ni % 2);
    }
    __host__ __device__ constexpr int D0EO() const { return XQ() + nq; }
    __host__ __device__ constexpr int D0TEO() const { return D0EO() + (n1 > 0 ? eo_len2(nq, n0) : 0); }
    __host__ __device__ constexpr int B1EO() const { return D0TEO() + (n1 > 0 ? eo_len2(n0, nq) : 0); }
    __host__ __device__ constexpr int B1TEO() const { return B1EO() + (n1 > 0 ? eo_len2(nq, n1) : 0); }
    __host__ __device__ constexpr int W3() const { return B1TEO() + (n1 > 0 ? eo_len2(n1, nq) : 0); }
    __host__ __device__ constexpr int size() const { return W3() + (n1 > 0 ? nq * nq * nq : 0); }
};

// Tables split into three bf16 terms (hi, mid, lo) and single fp16 / bf16
// copies live after the fp64 and fp32 blocks; see mixed.hip.
struct TableSet {
    int len = 0;
    double *d64 = nullptr;
    float *f32 = nullptr;
    void *mixed = nullptr; // low-precision tables (layout owned by mixed.hip)
    void *kron = nullptr;  // dense Kronecker tables for n <= 4 (layout in kron_layout.hpp)
};

struct LaunchArgs {
    int family, degree, form, nq, n0, n1, precision, io;
    double alpha, beta;
    int64_t ncells;
    const double *vert;
    const void *kappa;
    const void *u;
    void *y;
    void *A;
    const double *tab64;
    const float *tab32;
    const void *tabmix;
    const void *tabkron = nullptr;
    int *err;
    hipStream_t stream;
    int variant;
    // claim counters of a dynamically scheduled persistent launch: 8 claim counters
    // and one exit counter, each on its own 128-byte line (kSchedLine ints apart),
    // zero before the launch and reset to zero by the launch's last workgroup
    int *sched = nullptr;
    // cells are general trilinear hexahedra: geometry per quadrature point
    bool trilinear = false;
    // cells are axis-aligned boxes (the context's geometry): diagonal geometric factors
    bool box = false;
};

// ring of counter slots per context: consecutive launches take consecutive slots,
// so up to kSchedSlots launches from one context may run concurrently
constexpr int kSchedLine = 32;
constexpr int kSchedSlotInts = 9 * kSchedLine;
constexpr int kSchedSlots = 256;

// kernel launchers: return SF_OK, SF_ERR_UNSUPPORTED or SF_ERR_HIP
int launch_action_q(const LaunchArgs &a);
int launch_action_vq(const LaunchArgs &a);
int launch_matrix_svk(const LaunchArgs &a);
int launch_action_q_fast(const LaunchArgs &a);
int launch_action_q_global(const LaunchArgs &a, int nx, int ny, int nz);
int launch_matrix_q(const LaunchArgs &a);
int launch_matrix_qgen(const LaunchArgs &a);
int launch_matrix_coll(const LaunchArgs &a);
int launch_action_vec(const LaunchArgs &a);
int launch_action_vec_fast(const LaunchArgs &a);
int launch_matrix_vec(const LaunchArgs &a);
int launch_action_mixed(const LaunchArgs &a);
int launch_action_kron(const LaunchArgs &a);  // mixed precision, n = p + 1 <= 4
int launch_action_kron2(const LaunchArgs &a); // mixed precision, 5 <= n <= 9
int launch_dofmap_q(int nx, int ny, int nz, int p, int32_t *map, hipStream_t s);

// host-side table block of one element (TabLayout order, FP64)
int host_table_block(int family, int n0, int n1, int nq1, std::vector<double> &h);
// allocation-free box-cell action: per-device scratch set up once per device
// (called by sf_context_create with the device current), then launches that
// use only the scratch array's device address
int noalloc_setup(int device);
int launch_action_box_noalloc(LaunchArgs a, int device);

// tuning keys: what = "batch" (cell groups per tile) or "standalone" (kernel variant)
std::string tune_key(const sf_op *op, const char *what);
int tuned_variant_of(sf_context *ctx, const sf_op *op, const char *what, int dflt);

} // namespace sf

struct sf_context {
    int device = 0;
    int *d_sched = nullptr; // kSchedSlots slots of kSchedSlotInts counters
    unsigned sched_next = 0;
    int geometry = SF_GEOM_AFFINE;
    int *d_err = nullptr;
    std::map<std::tuple<int, int, int>, sf::TableSet> tables;
    std::map<std::string, int> tuned;
};

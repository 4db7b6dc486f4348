// Batched persistent launch: many meshes of different size and degree, actions
// and element matrices, in ONE kernel launch captured once in a hipGraph.
//
// Work is cut into tiles (job, first cell, cell count); tiles are ordered by
// an estimated cost (largest first) and the workgroups of one persistent
// kernel pop them from an atomic counter until the list is exhausted (every
// workgroup reaches the exit test, so the grid always drains).  Each tile runs
// the same per-cell-group device body as the stand-alone kernels; the bodies
// share one dynamic LDS buffer sized for the largest class present.  The
// counter is cleared by a one-thread kernel node in the same graph (no memset
// node).  Tile size (cell groups per tile) per class is chosen by a timing
// autotuner and cached per context and, optionally, in a JSON file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "sf_device.hpp"
#include "sf_internal.hpp"

namespace sf {

int op_dims(const sf_op *op, int *ndof, int *nq);
int ensure_tables(sf_context *ctx, const sf_op *op, LaunchArgs &a);

} // namespace sf

// the per-cell-group device bodies shared with the stand-alone kernels
#include "action_box_body.inc"
#include "action_q_body.inc"
#include "matrix_q_body.inc"
#include "mixed_body.inc"
#include "mixed_kron2_body.inc"
#include "mixed_kron_body.inc"

namespace sf {

// K_ACT_BOX: the FP64 action with the box-cell body (contexts declared SF_GEOM_BOX)
// K_MAT_BF16 / K_MAT_FP16 / K_MAT_BF16X3: element matrices with the final contraction on MFMA
enum {
    K_ACT_F64 = 0, K_ACT_BF16 = 1, K_ACT_FP16 = 2, K_ACT_BF16X3 = 3, K_MAT_F64 = 4, K_ACT_BOX = 5,
    K_MAT_BF16 = 6, K_MAT_FP16 = 7, K_MAT_BF16X3 = 8, K_NKIND = 9
};
constexpr bool is_mat(int kind) { return kind == K_MAT_F64 || kind >= K_MAT_BF16; }
constexpr int kNT = 256;
constexpr int kGroupVariants[5] = {1, 2, 4, 8, 16};

struct BatchJob {
    int cls; // kind * 8 + (degree - 1)
    int64_t ncells;
    const double *vert;
    const double *kappa;
    const double *u;
    double *y;
    double *A;
    int64_t arena;
    const double *tab64;
    const uint16_t *mix;
    const uint16_t *kron; // dense Kronecker tables (kron_layout.hpp)
};

struct BatchTile {
    int job;
    int pad;
    int64_t first, count;
};

// Mixed-precision action tiles run the dense Kronecker bodies except at n = 9 (BF16x3 and
// single term) where the sum-factorised MFMA body runs.  The tables are staged in LDS once
// per tile where they take at most 51.5 KB (three workgroups still fit per CU; the FP64
// classes take up to 56 KB): the single-term modes, and BF16x3 at n = 3 and 5; the other
// BF16x3 tiles read them from global memory.
template <int N, int KIND> constexpr bool kron_lds()
{
    return ((KIND == K_ACT_BF16 || KIND == K_ACT_FP16) && N <= 8) || (KIND == K_ACT_BF16X3 && (N == 3 || N == 5));
}
template <int N, int KIND> constexpr bool kron_tiles() { return (KIND == K_ACT_BF16X3 && N != 9) || kron_lds<N, KIND>(); }

template <int N> struct Cls {
    static constexpr int CA = (256 / (N * N)) > 0 ? 256 / (N * N) : 1; // FP64 action cells per group
    static constexpr int CM0 = (40 * 1024) / (4 * Lds3<N>::CS * 4);
    static constexpr int CMIX = CM0 < 1 ? 1 : (CM0 > 64 ? 64 : CM0);  // mixed action cells per group
    static constexpr int CMAT = (256 / (N * N * N)) > 0 ? 256 / (N * N * N) : 1;
    static constexpr int cells_per_group(int kind)
    {
        return (kind == K_ACT_F64 || kind == K_ACT_BOX) ? CA : (is_mat(kind) ? CMAT : CMIX);
    }
    static constexpr int smem(int kind)
    {
        if (kind == K_ACT_BF16X3 && (N == 3 || N == 5)) // the three-term tables in LDS
            return N <= 4 ? kron::KronSmem<N, SF_LAPLACE, SF_BF16X3>::bytes
                          : kron::K2Smem<N, SF_LAPLACE, SF_BF16X3>::bytes;
        if (kind == K_ACT_BF16X3 && N != 9) return 0; // the dense Kronecker bodies, global tables
        if ((kind == K_ACT_BF16 || kind == K_ACT_FP16) && N <= 8) // the tables (BF16 and FP16 planes alike)
            return N <= 4 ? kron::KronSmem<N, SF_LAPLACE, SF_BF16>::bytes : kron::K2Smem<N, SF_LAPLACE, SF_BF16>::bytes;
        return kind == K_ACT_BOX   ? BoxSmem<N, N, SF_LAPLACE, false, double, CA>::bytes
               : kind == K_ACT_F64 ? ActionQSmem<N, N, SF_LAPLACE, false, double, CA>::bytes
                                   : (is_mat(kind) ? MatrixQSmem<N, N, SF_LAPLACE, CMAT>::bytes
                                                        : ActionMixedSmem<N, N, SF_LAPLACE, CMIX>::bytes);
    }
};

// the dynamic LDS buffer of the persistent kernel; the tile functions use the
// symbol itself so that their accesses stay LDS instructions
extern __shared__ double batch_smem[];

// One class's tile loop.  Kept out of line so that every class gets its own
// register allocation (inlining all classes into one body exhausts the
// register file).
template <int N, int KIND>
__device__ __noinline__ void run_tile(const BatchJob *__restrict__ jobs, int job, int64_t first, int64_t count,
                                      int *__restrict__ err)
{
    const BatchJob j = jobs[job];
    const int64_t end = first + count < j.ncells ? first + count : j.ncells;
    if constexpr (kron_tiles<N, KIND>()) {
        // the tile's cells in 16-cell tiles (n <= 4) or geometry batches (n >= 5), one per
        // wave in turn, every product chained in registers
        using namespace kron;
        constexpr int MODE = KIND == K_ACT_BF16 ? SF_BF16 : (KIND == K_ACT_FP16 ? SF_FP16 : SF_BF16X3);
        constexpr int NW = kNT / 64;
        const int wave = threadIdx.x >> 6;
        unsigned char *const sm = reinterpret_cast<unsigned char *>(batch_smem);
        if constexpr (kron_lds<N, KIND>()) {
            // this tile's tables into LDS (the persistent loop's barrier before the next
            // tile keeps them until every wave is done)
            if constexpr (N <= 4) kron_stage<N, SF_LAPLACE, MODE, kNT>(j.kron, sm);
            else kron2_stage<N, SF_LAPLACE, MODE, kNT>(j.kron, sm);
            __syncthreads();
        }
        if constexpr (N <= 4) {
            constexpr KronLayout K(N);
            constexpr int NPL = KronMode<MODE>::NPL;
            auto plane = [](int p) { return NPL == 1 ? KronMode<MODE>::PLANE0 : p; };
            const uint16_t *kt = j.kron;
            using SM = KronSmem<N, SF_LAPLACE, MODE>;
            const uint16_t *const sF = reinterpret_cast<const uint16_t *>(sm);
            const uint16_t *const sB = reinterpret_cast<const uint16_t *>(sm + SM::off_bwd);
            auto ffrag = [&](int a, int p, int i) {
                if constexpr (kron_lds<N, KIND>())
                    return reinterpret_cast<const u32x4 *>(sF + (a * NPL + p) * K.fwd_elems())[i];
                else
                    return reinterpret_cast<const u32x4 *>(kt + K.fwd(1 + a, plane(p)))[i];
            };
            auto bfrag = [&](int a, int p, int i) {
                if constexpr (kron_lds<N, KIND>())
                    return reinterpret_cast<const u32x4 *>(sB + (a * NPL + p) * K.bwd_elems())[i];
                else
                    return reinterpret_cast<const u32x4 *>(kt + K.bwd(1 + a, plane(p)))[i];
            };
            const float *w3 = kron_lds<N, KIND>() ? reinterpret_cast<const float *>(sm + SM::off_w)
                                                  : reinterpret_cast<const float *>(kt + K.w3());
            for (int64_t c0 = first + 16 * wave; c0 < end; c0 += 16 * NW)
                kron_tile<N, SF_LAPLACE, MODE, double>(c0, end, ffrag, bfrag, w3, j.vert, j.kappa, j.u, j.y, err);
        } else {
            constexpr Kron2Layout K(N);
            constexpr int BATCH = K.cpt * (16 / K.cpt);
            constexpr bool PF = MODE != SF_BF16X3 && N <= 8;
            if constexpr (kron_lds<N, KIND>()) {
                const auto tabs = Kron2LdsTables<N, SF_LAPLACE, MODE>::at(sm);
                for (int64_t b0 = first + BATCH * wave; b0 < end; b0 += BATCH * NW)
                    kron2_batch<N, SF_LAPLACE, MODE, double, PF>(b0, end, tabs, j.vert, j.kappa, j.u, j.y, err);
            } else {
                const Kron2GlobalTables<N, MODE> tabs{j.kron};
                for (int64_t b0 = first + BATCH * wave; b0 < end; b0 += BATCH * NW)
                    kron2_batch<N, SF_LAPLACE, MODE, double, PF>(b0, end, tabs, j.vert, j.kappa, j.u, j.y, err);
            }
        }
        return;
    }
    constexpr int CPG = Cls<N>::cells_per_group(KIND);
    for (int64_t g = first; g < end; g += CPG) {
        if constexpr (KIND == K_ACT_BOX) {
            using SM = BoxSmem<N, N, SF_LAPLACE, false, double, CPG>;
            constexpr TabLayout TL(N, 0, N);
            unsigned char *sm = reinterpret_cast<unsigned char *>(batch_smem);
            const BoxPencil<N, CPG, kNT> pp;
            const BoxLattice<N> lat(0, 0);
            double vreg[BoxVR<CPG, kNT>::VR], ureg[N], kreg[N];
            if (threadIdx.x < N) reinterpret_cast<double *>(sm + SM::off_W)[threadIdx.x] = j.tab64[TL.W() + threadIdx.x];
            box_load<N, N, SF_LAPLACE, double, double, CPG, kNT, false>(g, end, j.vert, j.kappa, j.u, pp, lat, vreg,
                                                                       ureg, kreg);
            box_group<N, N, SF_LAPLACE, false, double, double, CPG, kNT, false>(g, end, j.kappa, j.y, j.tab64, err, sm, pp,
                                                                             lat, vreg, ureg, kreg, [] {});
        } else if constexpr (KIND == K_ACT_F64)
            action_q_body<N, N, SF_LAPLACE, false, double, double, CPG, kNT>(g, end, j.vert, j.kappa, j.u, j.y, j.tab64,
                                                                            err, batch_smem);
        else if constexpr (KIND == K_MAT_F64)
            matrix_q_body<N, N, SF_LAPLACE, double, CPG, kNT>(g, end, j.vert, j.kappa, j.A, j.arena, j.tab64, err,
                                                             batch_smem);
        else if constexpr (KIND == K_MAT_BF16)
            matrix_q_body<N, N, SF_LAPLACE, double, CPG, kNT, 1, SF_BF16>(g, end, j.vert, j.kappa, j.A, j.arena,
                                                                         j.tab64, err, batch_smem);
        else if constexpr (KIND == K_MAT_FP16)
            matrix_q_body<N, N, SF_LAPLACE, double, CPG, kNT, 1, SF_FP16>(g, end, j.vert, j.kappa, j.A, j.arena,
                                                                         j.tab64, err, batch_smem);
        else if constexpr (KIND == K_MAT_BF16X3)
            matrix_q_body<N, N, SF_LAPLACE, double, CPG, kNT, 1, SF_BF16X3>(g, end, j.vert, j.kappa, j.A, j.arena,
                                                                           j.tab64, err, batch_smem);
        else if constexpr (KIND == K_ACT_BF16)
            action_mixed_body<N, N, SF_LAPLACE, false, SF_BF16, double, CPG, kNT>(g, end, j.vert, j.kappa, j.u, j.y,
                                                                                 j.tab64, j.mix, err, batch_smem);
        else if constexpr (KIND == K_ACT_FP16)
            action_mixed_body<N, N, SF_LAPLACE, false, SF_FP16, double, CPG, kNT>(g, end, j.vert, j.kappa, j.u, j.y,
                                                                                 j.tab64, j.mix, err, batch_smem);
        else
            action_mixed_body<N, N, SF_LAPLACE, false, SF_BF16X3, double, CPG, kNT>(g, end, j.vert, j.kappa, j.u, j.y,
                                                                                   j.tab64, j.mix, err, batch_smem);
        __syncthreads();
    }
}

template <int N>
__device__ __forceinline__ void run_kind(int kind, const BatchJob *jobs, int job, int64_t first, int64_t count,
                                         int *err)
{
    switch (kind) {
    case K_ACT_F64: run_tile<N, K_ACT_F64>(jobs, job, first, count, err); break;
    case K_ACT_BF16: run_tile<N, K_ACT_BF16>(jobs, job, first, count, err); break;
    case K_ACT_FP16: run_tile<N, K_ACT_FP16>(jobs, job, first, count, err); break;
    case K_ACT_BF16X3: run_tile<N, K_ACT_BF16X3>(jobs, job, first, count, err); break;
    case K_MAT_F64: run_tile<N, K_MAT_F64>(jobs, job, first, count, err); break;
    case K_ACT_BOX: run_tile<N, K_ACT_BOX>(jobs, job, first, count, err); break;
    case K_MAT_BF16: run_tile<N, K_MAT_BF16>(jobs, job, first, count, err); break;
    case K_MAT_FP16: run_tile<N, K_MAT_FP16>(jobs, job, first, count, err); break;
    case K_MAT_BF16X3: run_tile<N, K_MAT_BF16X3>(jobs, job, first, count, err); break;
    default: break;
    }
}

__global__ void batch_reset_kernel(int *counter) { *counter = 0; }

// waves-per-EU target 3: the out-of-line tile functions inherit a register
// budget of 512/3 VGPRs instead of the whole file
__global__ void __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(3, 8))) batch_persistent_kernel(const BatchJob *__restrict__ jobs,
                                                               const BatchTile *__restrict__ tiles, const int ntiles,
                                                               int *__restrict__ counter, int *__restrict__ err)
{
    __shared__ int s_tile;
    for (;;) {
        if (threadIdx.x == 0) s_tile = atomicAdd(counter, 1);
        __syncthreads();
        const int t = s_tile;
        __syncthreads(); // everyone has read s_tile before it is overwritten
        if (t >= ntiles) break;
        const BatchTile tile = tiles[t];
        const int cls = jobs[tile.job].cls;
        const int kind = cls >> 3, n = (cls & 7) + 2;
        switch (n) {
        case 2: run_kind<2>(kind, jobs, tile.job, tile.first, tile.count, err); break;
        case 3: run_kind<3>(kind, jobs, tile.job, tile.first, tile.count, err); break;
        case 4: run_kind<4>(kind, jobs, tile.job, tile.first, tile.count, err); break;
        case 5: run_kind<5>(kind, jobs, tile.job, tile.first, tile.count, err); break;
        case 6: run_kind<6>(kind, jobs, tile.job, tile.first, tile.count, err); break;
        case 7: run_kind<7>(kind, jobs, tile.job, tile.first, tile.count, err); break;
        case 8: run_kind<8>(kind, jobs, tile.job, tile.first, tile.count, err); break;
        case 9: run_kind<9>(kind, jobs, tile.job, tile.first, tile.count, err); break;
        default: break;
        }
    }
}

namespace {

int cls_cells_per_group(int kind, int n)
{
    switch (n) {
    case 2: return Cls<2>::cells_per_group(kind);
    case 3: return Cls<3>::cells_per_group(kind);
    case 4: return Cls<4>::cells_per_group(kind);
    case 5: return Cls<5>::cells_per_group(kind);
    case 6: return Cls<6>::cells_per_group(kind);
    case 7: return Cls<7>::cells_per_group(kind);
    case 8: return Cls<8>::cells_per_group(kind);
    case 9: return Cls<9>::cells_per_group(kind);
    default: return 1;
    }
}

int cls_smem(int kind, int n)
{
    switch (n) {
    case 2: return Cls<2>::smem(kind);
    case 3: return Cls<3>::smem(kind);
    case 4: return Cls<4>::smem(kind);
    case 5: return Cls<5>::smem(kind);
    case 6: return Cls<6>::smem(kind);
    case 7: return Cls<7>::smem(kind);
    case 8: return Cls<8>::smem(kind);
    case 9: return Cls<9>::smem(kind);
    default: return 0;
    }
}

// estimated cost per cell (ns-like units): HBM bytes of the class
double cls_cost(int kind, int n)
{
    const double n3 = double(n) * n * n;
    if (is_mat(kind)) return 8.0 * n3 * n3 + 4.0 * n3 * n3 * n / 10.0;
    return 24.0 * n3 + 192.0 + 24.0 * n3 * n / 10.0;
}

int kind_of(const sf_job &j, bool box)
{
    if (j.A) {
        switch (j.op.precision) {
        case SF_FP64: return K_MAT_F64;
        case SF_BF16: return K_MAT_BF16;
        case SF_FP16: return K_MAT_FP16;
        case SF_BF16X3: return K_MAT_BF16X3;
        default: return -1;
        }
    }
    switch (j.op.precision) {
    case SF_FP64: return box ? K_ACT_BOX : K_ACT_F64;
    case SF_BF16: return K_ACT_BF16;
    case SF_FP16: return K_ACT_FP16;
    case SF_BF16X3: return K_ACT_BF16X3;
    default: return -1;
    }
}

int groups_for(sf_context *ctx, const sf_op *op, bool matrix)
{
    const int v = matrix ? tuned_variant_of(ctx, op, "batch_matrix", 0) : tuned_variant_of(ctx, op, "batch", 2);
    return kGroupVariants[std::min(std::max(v, 0), 4)];
}

} // namespace

} // namespace sf

using namespace sf;

struct sf_batch {
    sf_context *ctx = nullptr;
    BatchJob *d_jobs = nullptr;
    BatchTile *d_tiles = nullptr;
    int *d_counter = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t ntiles = 0;
    int nwg = 0;
    int smem = 0;
};

static void batch_free(sf_batch *b)
{
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->d_jobs) (void)hipFree(b->d_jobs);
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    if (b->d_counter) (void)hipFree(b->d_counter);
    delete b;
}

static int batch_build(sf_context *ctx, const sf_job *jobs, int32_t njobs, const int *groups_override, sf_batch **out)
{
    if (!ctx || !out || njobs < 0 || (njobs > 0 && !jobs)) return SF_ERR_ARG;
    *out = nullptr;
    std::vector<BatchJob> hj;
    std::vector<BatchTile> ht;
    std::vector<double> tcost;
    int smem = 0;
    for (int i = 0; i < njobs; ++i) {
        const sf_job &j = jobs[i];
        int nd, nq;
        int rc = op_dims(&j.op, &nd, &nq);
        if (rc) return rc;
        if (j.ncells < 0) return SF_ERR_ARG;
        if (j.op.family != SF_Q || j.op.form != SF_LAPLACE || j.op.io_dtype != SF_F64) return SF_ERR_UNSUPPORTED;
        const bool mat = j.A != nullptr;
        if (mat && (j.u || j.y)) return SF_ERR_ARG;
        if (!mat && (!j.u || !j.y || j.y == j.u)) return SF_ERR_ARG;
        if (j.ncells > 0 && !j.vertices) return SF_ERR_ARG;
        const int kind = kind_of(j, ctx->geometry == SF_GEOM_BOX);
        if (kind < 0) return SF_ERR_UNSUPPORTED;
        LaunchArgs a;
        rc = ensure_tables(ctx, &j.op, a);
        if (rc) return rc;
        const int n = j.op.degree + 1;
        BatchJob b;
        b.cls = kind * 8 + (n - 2);
        b.ncells = j.ncells;
        b.vert = j.vertices;
        b.kappa = static_cast<const double *>(j.kappa);
        b.u = static_cast<const double *>(j.u);
        b.y = static_cast<double *>(j.y);
        b.A = static_cast<double *>(j.A);
        b.arena = j.A_arena_cells > 0 ? j.A_arena_cells : 0;
        b.tab64 = a.tab64;
        b.mix = static_cast<const uint16_t *>(a.tabmix);
        b.kron = static_cast<const uint16_t *>(a.tabkron);
        if (!mat && kind != K_ACT_F64 && kind != K_ACT_BOX && !b.kron) return SF_ERR_UNSUPPORTED;
        hj.push_back(b);
        if (j.ncells == 0) continue;
        smem = std::max(smem, cls_smem(kind, n));
        const int cpg = cls_cells_per_group(kind, n);
        const int g = groups_override ? groups_override[i] : groups_for(ctx, &j.op, mat);
        const int64_t per = int64_t(cpg) * g;
        for (int64_t f = 0; f < j.ncells; f += per) {
            BatchTile t;
            t.job = i;
            t.pad = 0;
            t.first = f;
            t.count = std::min(per, j.ncells - f);
            ht.push_back(t);
            tcost.push_back(double(t.count) * cls_cost(kind, n));
        }
    }
    if (ht.size() > 0x7fffffff) return SF_ERR_CAPACITY;
    // largest estimated cost first (longest-processing-time order)
    std::vector<size_t> order(ht.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return tcost[x] > tcost[y]; });
    std::vector<BatchTile> sorted(ht.size());
    for (size_t i = 0; i < order.size(); ++i) sorted[i] = ht[order[i]];

    sf_batch *b = new (std::nothrow) sf_batch();
    if (!b) return SF_ERR_NOMEM;
    // a failing HIP call is reported on stderr with its step before the error code
    auto hip_fail = [&](const char *what) {
        std::fprintf(stderr, "sf_batch_create: %s failed (%s)\n", what, hipGetErrorString(hipGetLastError()));
        batch_free(b);
        return SF_ERR_HIP;
    };
    b->ctx = ctx;
    b->ntiles = int64_t(sorted.size());
    b->smem = smem;
    if (hipMalloc(&b->d_jobs, sizeof(BatchJob) * std::max<size_t>(1, hj.size())) != hipSuccess ||
        hipMalloc(&b->d_tiles, sizeof(BatchTile) * std::max<size_t>(1, sorted.size())) != hipSuccess ||
        hipMalloc(&b->d_counter, sizeof(int)) != hipSuccess) {
        batch_free(b);
        return SF_ERR_NOMEM;
    }
    if ((!hj.empty() && hipMemcpy(b->d_jobs, hj.data(), sizeof(BatchJob) * hj.size(), hipMemcpyHostToDevice) != hipSuccess) ||
        (!sorted.empty() &&
         hipMemcpy(b->d_tiles, sorted.data(), sizeof(BatchTile) * sorted.size(), hipMemcpyHostToDevice) != hipSuccess))
        return hip_fail("copying the job and tile lists");
    int per_cu = 0, ncu = 0;
    if (smem > 64 * 1024 &&
        hipFuncSetAttribute((const void *)batch_persistent_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, smem) !=
            hipSuccess)
        return hip_fail("raising the kernel's LDS limit");
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_persistent_kernel, kNT, size_t(smem)) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess)
        return hip_fail("the occupancy query");
    per_cu = std::max(per_cu, 1);
    b->nwg = int(std::min<int64_t>(std::max<int64_t>(b->ntiles, 1), int64_t(per_cu) * ncu));

    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return hip_fail("creating the capture stream");
    bool ok = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
        hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(1), 0, s, b->d_counter);
        hipLaunchKernelGGL(batch_persistent_kernel, dim3(b->nwg), dim3(kNT), size_t(smem), s, b->d_jobs, b->d_tiles,
                           int(b->ntiles), b->d_counter, ctx->d_err);
        ok = hipStreamEndCapture(s, &b->graph) == hipSuccess && b->graph;
    }
    ok = ok && hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) == hipSuccess;
    (void)hipStreamDestroy(s);
    if (!ok) return hip_fail("capturing and instantiating the graph");
    *out = b;
    return SF_OK;
}

namespace {

// minimal JSON object of string -> integer
std::map<std::string, int> read_json(const char *path)
{
    std::map<std::string, int> m;
    std::ifstream f(path);
    if (!f) return m;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    size_t i = 0;
    while (true) {
        size_t a = s.find('"', i);
        if (a == std::string::npos) break;
        size_t b2 = s.find('"', a + 1);
        if (b2 == std::string::npos) break;
        const std::string key = s.substr(a + 1, b2 - a - 1);
        size_t c = s.find(':', b2);
        if (c == std::string::npos) break;
        m[key] = std::atoi(s.c_str() + c + 1);
        i = c + 1;
    }
    return m;
}

bool write_json(const char *path, const std::map<std::string, int> &m)
{
    std::ofstream f(path, std::ios::trunc);
    if (!f) return false;
    f << "{\n";
    size_t k = 0;
    for (auto &kv : m) f << "  \"" << kv.first << "\": " << kv.second << (++k < m.size() ? ",\n" : "\n");
    f << "}\n";
    return bool(f);
}

template <typename IO>
__global__ void tune_fill_kernel(int64_t ncells, int n3, int nq3, double *vert, IO *u, IO *kap)
{
    const int64_t total = ncells * std::max(std::max(n3, nq3), 24);
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x) {
        if (t < ncells * n3) u[t] = IO(double((t * 2654435761LL) % 1000) * 1e-3 - 0.5);
        if (t < ncells * nq3) kap[t] = IO(1.0 + double((t * 40503LL) % 1000) * 1e-3);
        if (t < ncells * 24) {
            const int v = int((t % 24) / 3), a = int(t % 3);
            vert[t] = double((v >> (2 - a)) & 1);
        }
    }
}

} // namespace

extern "C" {

int sf_batch_create(sf_context *ctx, const sf_job *jobs, int32_t njobs, sf_batch **out)
{
    return batch_build(ctx, jobs, njobs, nullptr, out);
}

int sf_batch_launch(sf_batch *b, void *hip_stream)
{
    if (!b || !b->exec) return SF_ERR_ARG;
    return hipGraphLaunch(b->exec, static_cast<hipStream_t>(hip_stream)) == hipSuccess ? SF_OK : SF_ERR_HIP;
}

int sf_batch_destroy(sf_batch *b)
{
    if (!b) return SF_ERR_ARG;
    (void)hipDeviceSynchronize();
    batch_free(b);
    return SF_OK;
}

int sf_batch_info(const sf_batch *b, int64_t *ntiles, int32_t *nworkgroups)
{
    if (!b) return SF_ERR_ARG;
    if (ntiles) *ntiles = b->ntiles;
    if (nworkgroups) *nworkgroups = b->nwg;
    return SF_OK;
}

int sf_tuned_variant(sf_context *ctx, const sf_op *op, int32_t *variant)
{
    if (!ctx || !op || !variant) return SF_ERR_ARG;
    int nd, nq;
    int rc = op_dims(op, &nd, &nq);
    if (rc) return rc;
    *variant = tuned_variant_of(ctx, op, "batch", 2);
    return SF_OK;
}

int sf_load_tuning(sf_context *ctx, const char *path)
{
    if (!ctx || !path) return SF_ERR_ARG;
    for (auto &kv : read_json(path))
        if (kv.second >= 0 && kv.second <= 6) ctx->tuned[kv.first] = kv.second; // variants 0..6
    return SF_OK;
}

int sf_autotune(sf_context *ctx, const sf_op *op, int64_t ncells_hint, const char *cache_json_path)
{
    if (!ctx || !op || ncells_hint < 1) return SF_ERR_ARG;
    int nd, nq;
    int rc = op_dims(op, &nd, &nq);
    if (rc) return rc;
    const bool scalar = op->family == SF_Q || op->family == SF_DQ || op->family == SF_QGLL;
    // classes with a choice: the batched launch's tiles (Q_p Laplace, FP64 storage: actions in
    // every precision, element matrices in FP64) and the stand-alone box-cell action kernel
    // (scalar families, mass and Laplace, FP64 / FP32 contractions, either storage)
    const bool tune_batch = op->family == SF_Q && op->form == SF_LAPLACE && op->io_dtype == SF_F64 &&
                            op->precision != SF_FP32; // the batched launch has no FP32 kind
    const bool tune_matrix = tune_batch && op->precision == SF_FP64;
    const bool tune_sa = scalar && (op->form == SF_MASS || op->form == SF_LAPLACE) &&
                         (op->precision == SF_FP64 || op->precision == SF_FP32);
    // H(div) / H(curl) actions on box cells: fused box-cell kernel (0), one group per
    // workgroup (1) or the persistent affine kernel (2)
    const bool tune_vec = (op->family == SF_NCF || op->family == SF_NCE) &&
                          (op->precision == SF_FP64 || op->precision == SF_FP32);
    if (!tune_batch && !tune_sa && !tune_vec) return SF_ERR_UNSUPPORTED;
    const int64_t nc = std::min<int64_t>(ncells_hint, 1 << 20);
    const size_t esz = op->io_dtype == SF_F32 ? 4 : 8;
    // element matrices of at most 512 MiB for the matrix tiles
    const int64_t mat_cells = std::max<int64_t>(1, std::min<int64_t>(nc, (int64_t(512) << 20) / (8 * int64_t(nd) * nd)));
    // synthetic unit boxes, u and a kappa per quadrature point, as in a production call
    double *vert = nullptr, *A = nullptr;
    void *u = nullptr, *y = nullptr, *kap = nullptr;
    if (hipMalloc(&vert, sizeof(double) * 24 * nc) != hipSuccess || hipMalloc(&u, esz * nd * nc) != hipSuccess ||
        hipMalloc(&y, esz * nd * nc) != hipSuccess || hipMalloc(&kap, esz * nq * nc) != hipSuccess ||
        (tune_matrix && hipMalloc(&A, sizeof(double) * nd * nd * mat_cells) != hipSuccess)) {
        (void)hipFree(vert);
        (void)hipFree(u);
        (void)hipFree(y);
        (void)hipFree(kap);
        (void)hipFree(A);
        return SF_ERR_NOMEM;
    }
    if (esz == 4)
        hipLaunchKernelGGL(tune_fill_kernel<float>, dim3(1024), dim3(256), 0, 0, nc, nd, nq, vert,
                           static_cast<float *>(u), static_cast<float *>(kap));
    else
        hipLaunchKernelGGL(tune_fill_kernel<double>, dim3(1024), dim3(256), 0, 0, nc, nd, nq, vert,
                           static_cast<double *>(u), static_cast<double *>(kap));
    hipStream_t s;
    hipEvent_t e0, e1;
    bool ok = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
    ok = ok && hipDeviceSynchronize() == hipSuccess;
    // median-free, noise-robust timing: the sum of three launches after one warm-up;
    // a later variant must be 2% faster than the best so far (stable choices)
    auto time3 = [&](auto &&run) {
        float tot = -1.0f;
        if (!ok || !(ok = run())) return tot;
        tot = 0.0f;
        for (int r = 0; ok && r < 3; ++r) {
            ok = hipEventRecord(e0, s) == hipSuccess && run() && hipEventRecord(e1, s) == hipSuccess &&
                 hipEventSynchronize(e1) == hipSuccess;
            float ms = 0.0f;
            ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
            tot += ms;
        }
        return ok ? tot : -1.0f;
    };
    auto tune_tiles = [&](bool matrix, int &best) {
        float best_ms = 1e30f;
        for (int v = 0; ok && v < 5; ++v) {
            sf_job j;
            std::memset(&j, 0, sizeof j);
            j.op = *op;
            j.ncells = matrix ? mat_cells : nc;
            j.vertices = vert;
            j.kappa = kap;
            if (matrix) {
                j.A = A;
                j.A_arena_cells = mat_cells;
            } else {
                j.u = u;
                j.y = y;
            }
            int g = kGroupVariants[v];
            sf_batch *b = nullptr;
            const int brc = batch_build(ctx, &j, 1, &g, &b);
            if (brc != SF_OK) {
                std::fprintf(stderr, "sf_autotune: building the %s tile variant %d failed (%s)\n",
                             matrix ? "matrix" : "action", v, sf_status_string(brc));
                ok = false;
                break;
            }
            const float t = time3([&] { return hipGraphLaunch(b->exec, s) == hipSuccess; });
            if (!ok)
                std::fprintf(stderr, "sf_autotune: timing the %s tile variant %d failed (%s)\n",
                             matrix ? "matrix" : "action", v, hipGetErrorString(hipGetLastError()));
            (void)hipStreamSynchronize(s);
            batch_free(b);
            if (ok && t < 0.98f * best_ms) {
                best_ms = t;
                best = v;
            }
        }
    };
    int best = 2, best_mat = 0, best_sa = 0, best_vec = 0;
    if (tune_batch) tune_tiles(false, best);
    if (tune_matrix) tune_tiles(true, best_mat);
    if (ok && tune_sa) {
        // stand-alone box-cell action kernel variants (prefetch / occupancy; 3 = the general kernel)
        LaunchArgs a;
        ok = ensure_tables(ctx, op, a) == SF_OK;
        float best_sa_ms = 1e30f;
        for (int v = 0; ok && v < 7; ++v) {
            if (v == 6 && op->degree != 1) continue; // one cell per thread: p = 1 only
            a.ncells = nc;
            a.vert = vert;
            a.kappa = kap;
            a.u = u;
            a.y = y;
            a.stream = s;
            a.variant = v;
            const float t = time3([&] {
                a.sched = ctx->d_sched + kSchedSlotInts * (ctx->sched_next++ % kSchedSlots);
                return (v == 3 ? launch_action_q(a) : launch_action_q_fast(a)) == SF_OK;
            });
            if (!ok)
                std::fprintf(stderr, "sf_autotune: timing the stand-alone variant %d failed (%s)\n", v,
                             hipGetErrorString(hipGetLastError()));
            if (ok && t < 0.98f * best_sa_ms) {
                best_sa_ms = t;
                best_sa = v;
            }
        }
    }
    if (ok && tune_vec) {
        LaunchArgs a;
        ok = ensure_tables(ctx, op, a) == SF_OK;
        float best_vec_ms = 1e30f;
        const int order[3] = {0, 2, 1};
        for (int i = 0; ok && i < 3; ++i) {
            const int v = order[i];
            a.ncells = nc;
            a.vert = vert;
            a.kappa = nullptr;
            a.u = u;
            a.y = y;
            a.stream = s;
            a.box = true;
            a.trilinear = false;
            a.variant = v;
            const float t = time3([&] { return launch_action_vec(a) == SF_OK; });
            if (!ok)
                std::fprintf(stderr, "sf_autotune: timing the H(div)/H(curl) variant %d failed (%s)\n", v,
                             hipGetErrorString(hipGetLastError()));
            if (ok && t < 0.98f * best_vec_ms) {
                best_vec_ms = t;
                best_vec = v;
            }
        }
    }
    (void)hipStreamSynchronize(s);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(s);
    (void)hipFree(vert);
    (void)hipFree(u);
    (void)hipFree(y);
    (void)hipFree(kap);
    (void)hipFree(A);
    if (!ok) return SF_ERR_HIP;
    std::map<std::string, int> got;
    if (tune_batch) got[tune_key(op, "batch")] = best;
    if (tune_matrix) got[tune_key(op, "batch_matrix")] = best_mat;
    if (tune_sa) got[tune_key(op, "standalone")] = best_sa;
    if (tune_vec) got[tune_key(op, "standalone")] = best_vec;
    for (auto &kv : got) ctx->tuned[kv.first] = kv.second;
    if (cache_json_path) {
        auto m = read_json(cache_json_path);
        for (auto &kv : got) m[kv.first] = kv.second;
        if (!write_json(cache_json_path, m)) return SF_ERR_ARG;
    }
    return SF_OK;
}

} // extern "C"

// Allocation-free variant of the box-cell action (assemble_action_box_noalloc).
//
// The persistent box-cell kernel needs device memory beyond its inputs and
// outputs: one slot of claim counters and the 1-D table block of its
// (family, degree).  For callers that cannot allocate, both live here in a
// file-scope device array of fixed size: the counters at offset 0, then the
// FP64 and FP32 table blocks of every scalar family (Q_p, dQ_p, collocated
// Q_p) and degree p = 1..8.  The array's device address is taken once per
// device at context creation (hipGetSymbolAddress), where the tables are also
// uploaded; launches use only that address.  Every call on a device shares
// the one counter slot: the counters are cleared by a fill kernel before each
// launch (the kernel's last workgroup also resets them), and calls that
// overlap on one device race.
#include <mutex>
#include <vector>

#include "sf_internal.hpp"

namespace sf {

namespace {

constexpr int kScratchBytes = 96 * 1024;
constexpr int kMaxDevices = 64;
constexpr int kCounterBytes = kSchedSlotInts * 4;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

int family_slot(int family) { return family == SF_Q ? 0 : family == SF_DQ ? 1 : family == SF_QGLL ? 2 : -1; }

struct ScratchLayout {
    int off64[3][10] = {}, off32[3][10] = {}, end = 0;
    ScratchLayout()
    {
        const int fams[3] = {SF_Q, SF_DQ, SF_QGLL};
        int o = (kCounterBytes + 255) / 256 * 256;
        for (int f = 0; f < 3; ++f)
            for (int n = 2; n <= 9; ++n) {
                const int len = TabLayout(n, 0, n).size();
                off64[family_slot(fams[f])][n] = o;
                o += (len * 8 + 255) / 256 * 256;
                off32[family_slot(fams[f])][n] = o;
                o += (len * 4 + 255) / 256 * 256;
            }
        end = o;
    }
};
const ScratchLayout kLayout;

struct DeviceScratch {
    bool ready = false;
    unsigned char *ptr = nullptr; // device address of `scratch` on this device
};
DeviceScratch g_dev[kMaxDevices];
std::mutex g_mu;

__global__ void clear_counters_kernel(int *c, int n)
{
    for (int t = threadIdx.x; t < n; t += blockDim.x) c[t] = 0;
}

} // namespace

int noalloc_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return SF_ERR_CAPACITY;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_dev[device].ready) return SF_OK;
    static_assert(kScratchBytes >= 8192, "scratch holds the counters and the tables");
    if (kLayout.end > kScratchBytes) return SF_ERR_CAPACITY;
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return SF_ERR_HIP;
    unsigned char *base = static_cast<unsigned char *>(p);
    if (hipMemset(base, 0, kCounterBytes) != hipSuccess) return SF_ERR_HIP;
    const int fams[3] = {SF_Q, SF_DQ, SF_QGLL};
    std::vector<double> h;
    for (int f = 0; f < 3; ++f)
        for (int n = 2; n <= 9; ++n) {
            if (host_table_block(fams[f], n, 0, n, h) != SF_OK) return SF_ERR_UNSUPPORTED;
            std::vector<float> hf(h.begin(), h.end());
            const int s = family_slot(fams[f]);
            if (hipMemcpy(base + kLayout.off64[s][n], h.data(), h.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
                hipMemcpy(base + kLayout.off32[s][n], hf.data(), hf.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
                return SF_ERR_HIP;
        }
    if (hipDeviceSynchronize() != hipSuccess) return SF_ERR_HIP;
    g_dev[device].ptr = base;
    g_dev[device].ready = true;
    return SF_OK;
}

int launch_action_box_noalloc(LaunchArgs a, int device)
{
    if (device < 0 || device >= kMaxDevices) return SF_ERR_CAPACITY;
    unsigned char *base;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if (!g_dev[device].ready) return SF_ERR_HIP; // set up by sf_context_create on this device
        base = g_dev[device].ptr;
    }
    const int s = family_slot(a.family);
    const int n = a.degree + 1;
    if (s < 0 || n < 2 || n > 9 || a.nq != n) return SF_ERR_UNSUPPORTED;
    a.sched = reinterpret_cast<int *>(base);
    a.tab64 = reinterpret_cast<const double *>(base + kLayout.off64[s][n]);
    a.tab32 = reinterpret_cast<const float *>(base + kLayout.off32[s][n]);
    a.tabmix = nullptr;
    if (a.variant == 3) a.variant = 0; // the general kernel is not this entry point's kernel
    hipLaunchKernelGGL(clear_counters_kernel, dim3(1), dim3(256), 0, a.stream, a.sched, kSchedSlotInts);
    if (hipGetLastError() != hipSuccess) return SF_ERR_HIP;
    return launch_action_q_fast(a);
}

} // namespace sf

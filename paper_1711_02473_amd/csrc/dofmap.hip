// Global continuous Q_p numbering of a tensor grid of cells (integer work,
// bit-exact).  Local node (i0,i1,i2) of cell (i,j,k) is the lattice point
// (i*p+i0, j*p+i1, k*p+i2); shared nodes of neighbouring cells are the same
// lattice point and so receive the same number (Sec. 4.1: unique DOFs n^d per
// cell against (n+1)^d local ones).
#include "sf_device.hpp"
#include "sf_internal.hpp"

namespace sf {

__global__ void dofmap_q_kernel(int nx, int ny, int nz, int p, int64_t total, int32_t *__restrict__ map)
{
    const int n = p + 1;
    const int nloc = n * n * n;
    const int64_t my = int64_t(ny) * p + 1, mz = int64_t(nz) * p + 1;
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += int64_t(gridDim.x) * blockDim.x) {
        const int64_t cell = t / nloc;
        const int loc = int(t - cell * nloc);
        const int i0 = loc / (n * n), i1 = (loc / n) % n, i2 = loc % n;
        const int64_t k = cell % nz, j = (cell / nz) % ny, i = cell / (int64_t(ny) * nz);
        const int64_t a = i * p + i0, b = j * p + i1, c = k * p + i2;
        map[t] = int32_t((a * my + b) * mz + c);
    }
}

int launch_dofmap_q(int nx, int ny, int nz, int p, int32_t *map, hipStream_t s)
{
    const int64_t total = int64_t(nx) * ny * nz * int64_t(p + 1) * (p + 1) * (p + 1);
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(dofmap_q_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, nx, ny, nz, p, total, map);
    return hipGetLastError() == hipSuccess ? SF_OK : SF_ERR_HIP;
}

} // namespace sf

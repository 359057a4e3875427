// Spatial cells for the Metropolis scan: atoms sorted by the cell of their
// position (x fastest), so every row of cells along x is one contiguous range
// of the sorted arrays.  The sort is a stable radix sort of the keys
// (cell << abits | atom), so the order inside a cell is the atom order and
// every rebuild is deterministic.  Between rebuilds atoms keep their sorted
// slot while they move; the distance any atom has moved from its position at
// the last rebuild ("drift", fractional units) is tracked by the commit step
// and widens the cell search so no neighbour is missed.
#include "nd_internal.h"

#include <rocprim/device/device_radix_sort.hpp>

#include <algorithm>
#include <cmath>

namespace {

__global__ void k_cell_keys(const float4 *__restrict__ pos4, int N, int nc, int abits, uint64_t *__restrict__ keys)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const float4 p = pos4[i];
    const int cx = min(max((int)(p.x * (float)nc), 0), nc - 1);
    const int cy = min(max((int)(p.y * (float)nc), 0), nc - 1);
    const int cz = min(max((int)(p.z * (float)nc), 0), nc - 1);
    const uint64_t c = (uint64_t)((cz * nc + cy) * nc + cx);
    keys[i] = (c << abits) | (uint64_t)i;
}

__global__ void k_cell_gather(const uint64_t *__restrict__ keys, int N, int abits, int ncell,
                              const float4 *__restrict__ pos4, const float4 *__restrict__ poslo,
                              int32_t *__restrict__ sorted, int32_t *__restrict__ slot, float4 *__restrict__ spos4,
                              float4 *__restrict__ sposlo, float4 *__restrict__ sref, int32_t *__restrict__ start)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= N) return;
    const uint64_t key = keys[s];
    const int atom = (int)(key & ((1ull << abits) - 1ull));
    const int c = (int)(key >> abits);
    sorted[s] = atom;
    slot[atom] = s;
    const float4 p = pos4[atom];
    spos4[s] = p;
    sposlo[s] = poslo[atom];
    sref[s] = p;
    // start[cc] = first slot of cell cc; cells between the previous atom's
    // cell and this one are empty and start here
    const int cprev = s > 0 ? (int)(keys[s - 1] >> abits) : -1;
    for (int cc = cprev + 1; cc <= c; ++cc) start[cc] = s;
    if (s == N - 1)
        for (int cc = c + 1; cc <= ncell; ++cc) start[cc] = N;
}

__global__ void k_zero_f32(float *p) { *p = 0.0f; }

}  // namespace

namespace nd {

void cells_free(nd_box *b)
{
    Cells &c = b->cells;
    dfree(c.start);
    dfree(c.sorted);
    dfree(c.slot);
    dfree(c.spos4);
    dfree(c.sposlo);
    dfree(c.sref);
    dfree(c.keys_in);
    dfree(c.keys_out);
    dfree(c.sort_tmp);
    dfree(c.drift);
    c = Cells();
}

void cells_build(nd_box *b)
{
    Cells &c = b->cells;
    const int N = b->N;
    // about four atoms per cell, at least one cell per axis
    const double rho = (double)N / (b->L * b->L * b->L);
    const double edge = std::cbrt(4.0 / rho);
    int nc = (int)std::floor(b->L / edge);
    nc = std::max(1, std::min(nc, 128));
    const int ncell = nc * nc * nc;
    int abits = 1;
    while ((1ll << abits) < (long long)N) ++abits;
    int cbits = 1;
    while ((1ll << cbits) < (long long)ncell) ++cbits;
    if (c.cap_n < N || c.ncell != ncell) {
        ND_HIP(hipStreamSynchronize(b->stream));
        cells_free(b);
        c.start = static_cast<int32_t *>(dmalloc(sizeof(int32_t) * (ncell + 1)));
        c.sorted = static_cast<int32_t *>(dmalloc(sizeof(int32_t) * N));
        c.slot = static_cast<int32_t *>(dmalloc(sizeof(int32_t) * N));
        c.spos4 = static_cast<float4 *>(dmalloc(sizeof(float4) * N));
        c.sposlo = static_cast<float4 *>(dmalloc(sizeof(float4) * N));
        c.sref = static_cast<float4 *>(dmalloc(sizeof(float4) * N));
        c.keys_in = static_cast<uint64_t *>(dmalloc(sizeof(uint64_t) * N));
        c.keys_out = static_cast<uint64_t *>(dmalloc(sizeof(uint64_t) * N));
        c.drift = static_cast<float *>(dmalloc(sizeof(float)));
        size_t tmp = 0;
        ND_HIP(rocprim::radix_sort_keys(nullptr, tmp, c.keys_in, c.keys_out, (unsigned)N, 0u,
                                        (unsigned)(abits + cbits), b->stream));
        c.sort_tmp = dmalloc(tmp);
        c.sort_tmp_bytes = tmp;
        c.cap_n = N;
        c.ncell = ncell;
    }
    c.nc = nc;
    const int threads = 256, blocks = (N + threads - 1) / threads;
    hipLaunchKernelGGL(k_cell_keys, dim3(blocks), dim3(threads), 0, b->stream, b->pos4, N, nc, abits, c.keys_in);
    ND_HIP(hipGetLastError());
    size_t tmp = c.sort_tmp_bytes;
    ND_HIP(rocprim::radix_sort_keys(c.sort_tmp, tmp, c.keys_in, c.keys_out, (unsigned)N, 0u,
                                    (unsigned)(abits + cbits), b->stream));
    hipLaunchKernelGGL(k_cell_gather, dim3(blocks), dim3(threads), 0, b->stream, c.keys_out, N, abits, ncell, b->pos4,
                       b->poslo, c.sorted, c.slot, c.spos4, c.sposlo, c.sref, c.start);
    ND_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(1), 0, b->stream, c.drift);
    ND_HIP(hipGetLastError());
    c.valid = true;
    c.trials_since_build = 0;
}

}  // namespace nd

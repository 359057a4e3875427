// Intramolecular harmonic terms of flexible molecules (Sec. "Correctness":
// the molecule's shape is kept by harmonic oscillator potentials between
// every two of its atoms):  V_intra = sum over pairs a < b of one unit of
// k_p (r_ab - r0_ab)^2, with r0_ab the pair's length in a reference geometry
// (the coordinates when the terms are set).  Distances are nearest-image
// lengths in FP64 of the float32 coordinates (displacement by comparison
// with L/2).  The energy change of a trial is computed by the proposal
// (k_mc.hip); here: the reference lengths, the total, and the gradient.
#include "nd_internal.h"

#include <cmath>

namespace {

constexpr int IN_THREADS = 256;

struct IntraArgs {
    const float *xyz;
    const uint8_t *sp;
    const int32_t *uoff, *unit_of;
    const double *r0;  // [N][ND_MAX_UNIT_ATOMS]
    int N, M, n_units;
    double L;
    double kint[ND_MAX_SPECIES * (ND_MAX_SPECIES + 1) / 2];
};

__device__ __forceinline__ double mi(double d, double L)
{
    const double half = 0.5 * L;
    if (d > half) return d - L;
    if (d < -half) return d + L;
    return d;
}

__global__ void k_intra_reference(IntraArgs a, double *__restrict__ r0)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.N) return;
    const int u = a.unit_of[i], u0 = a.uoff[u], u1 = a.uoff[u + 1];
    const int N = a.N;
    for (int s = 0; s < ND_MAX_UNIT_ATOMS; ++s) {
        const int j = u0 + s;
        double v = 0.0;
        if (j < u1 && j != i) {
            const double dx = mi((double)a.xyz[j] - (double)a.xyz[i], a.L);
            const double dy = mi((double)a.xyz[N + j] - (double)a.xyz[N + i], a.L);
            const double dz = mi((double)a.xyz[2 * N + j] - (double)a.xyz[2 * N + i], a.L);
            v = sqrt(dx * dx + dy * dy + dz * dz);
        }
        r0[(size_t)i * ND_MAX_UNIT_ATOMS + s] = v;
    }
}

// One block: every unit's energy in unit order, summed per thread in a
// fixed order and over the block in a fixed order, added to *E (and the
// |terms| to *S).
__global__ __launch_bounds__(IN_THREADS) void k_intra_energy(IntraArgs a, double *__restrict__ E,
                                                             double *__restrict__ S)
{
    __shared__ double se[IN_THREADS], ss[IN_THREADS];
    const int N = a.N;
    double e = 0.0, s = 0.0;
    for (int u = threadIdx.x; u < a.n_units; u += IN_THREADS) {
        const int u0 = a.uoff[u], u1 = a.uoff[u + 1];
        for (int p = u0; p < u1; ++p)
            for (int q = p + 1; q < u1; ++q) {
                const double dx = mi((double)a.xyz[q] - (double)a.xyz[p], a.L);
                const double dy = mi((double)a.xyz[N + q] - (double)a.xyz[N + p], a.L);
                const double dz = mi((double)a.xyz[2 * N + q] - (double)a.xyz[2 * N + p], a.L);
                const double d = sqrt(dx * dx + dy * dy + dz * dz) - a.r0[(size_t)p * ND_MAX_UNIT_ATOMS + (q - u0)];
                const double v = a.kint[nd::pair_index(a.sp[p], a.sp[q], a.M)] * d * d;
                e += v;
                s += fabs(v);
            }
    }
    se[threadIdx.x] = e;
    ss[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double te = 0.0, ts = 0.0;
        for (int t = 0; t < IN_THREADS; ++t) {
            te += se[t];
            ts += ss[t];
        }
        *E += te;
        if (S) *S += ts;
    }
}

// dV/dx_i = sum over the other atoms b of i's unit of 2 k (r - r0) (x_i - x_b) / r
__global__ void k_intra_forces(IntraArgs a, double *__restrict__ grad)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.N) return;
    const int N = a.N;
    const int u = a.unit_of[i], u0 = a.uoff[u], u1 = a.uoff[u + 1];
    double gx = 0.0, gy = 0.0, gz = 0.0;
    for (int b = u0; b < u1; ++b) {
        if (b == i) continue;
        const double dx = mi((double)a.xyz[i] - (double)a.xyz[b], a.L);
        const double dy = mi((double)a.xyz[N + i] - (double)a.xyz[N + b], a.L);
        const double dz = mi((double)a.xyz[2 * N + i] - (double)a.xyz[2 * N + b], a.L);
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        if (r == 0.0) continue;
        const double c = 2.0 * a.kint[nd::pair_index(a.sp[i], a.sp[b], a.M)] *
                         (r - a.r0[(size_t)i * ND_MAX_UNIT_ATOMS + (b - u0)]) / r;
        gx += c * dx;
        gy += c * dy;
        gz += c * dz;
    }
    grad[i] += gx;
    grad[N + i] += gy;
    grad[2 * N + i] += gz;
}

IntraArgs intra_args(const nd_box *b)
{
    IntraArgs a{};
    a.xyz = b->xyz;
    a.sp = b->species;
    a.uoff = b->uoff;
    a.unit_of = b->unit_of;
    a.r0 = b->r0;
    a.N = b->N;
    a.M = b->M;
    a.n_units = b->n_units;
    a.L = b->L;
    for (int q = 0; q < ND_MAX_SPECIES * (ND_MAX_SPECIES + 1) / 2; ++q) a.kint[q] = b->kint[q];
    return a;
}

}  // namespace

namespace nd {

void launch_intra_reference(nd_box *b)
{
    if (!b->r0) b->r0 = static_cast<double *>(dmalloc(sizeof(double) * (size_t)b->N * ND_MAX_UNIT_ATOMS));
    hipLaunchKernelGGL(k_intra_reference, dim3((b->N + 255) / 256), dim3(256), 0, b->stream, intra_args(b), b->r0);
    ND_HIP(hipGetLastError());
}

void launch_intra_energy_add(nd_box *b, double *d_E, double *d_S)
{
    if (!b->has_intra) return;
    hipLaunchKernelGGL(k_intra_energy, dim3(1), dim3(IN_THREADS), 0, b->stream, intra_args(b), d_E, d_S);
    ND_HIP(hipGetLastError());
}

void launch_intra_forces_add(nd_box *b, double *d_grad)
{
    if (!b->has_intra) return;
    hipLaunchKernelGGL(k_intra_forces, dim3((b->N + 255) / 256), dim3(256), 0, b->stream, intra_args(b), d_grad);
    ND_HIP(hipGetLastError());
}

}  // namespace nd

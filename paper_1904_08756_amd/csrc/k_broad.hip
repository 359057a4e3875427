// Differentiated form: a Gaussian-broadened pair histogram (forward), the
// gradient of a loss on that histogram with respect to every coordinate
// (backward), and the gradient of the tabulated total energy (forces).
//
// Broadening: a pair at distance r adds to bin k the Gaussian mass between
// its edges, w_k(r) = Phi((e_{k+1}-r)/s) - Phi((e_k-r)/s), e_k = k dr, for
// the bins that intersect [r - 6s, r + 6s].  Each edge needs one tail mass
// T(e) = Phi(-|e - r|/s) = erfc(|e - r|/(s sqrt 2))/2, from which every bin
// weight follows without cancellation:
//   bin right of r: T(e_k) - T(e_{k+1});  left of r: T(e_{k+1}) - T(e_k);
//   bin containing r: 1 - T(e_k) - T(e_{k+1}).
// Distances are FP64 from the float32 coordinates; per-pair weights FP32;
// sums FP64.
#include "nd_internal.h"
#include "nd_pair.h"

#include <algorithm>
#include <cmath>

namespace {

constexpr int TILE = 256;

__device__ __forceinline__ void tri_index(long long t, int nt, int &I, int &J)
{
    double a = 2.0 * nt + 1.0;
    int r = (int)floor((a - sqrt(a * a - 8.0 * (double)t)) * 0.5);
    if (r < 0) r = 0;
    if (r > nt - 1) r = nt - 1;
    auto off = [nt](long long i) { return i * nt - i * (i - 1) / 2; };
    while (r > 0 && off(r) > t) --r;
    while (r < nt - 1 && off(r + 1) <= t) ++r;
    I = r;
    J = r + (int)(t - off(r));
}

struct BroadArgs {
    const float *xyz;
    const uint8_t *sp;
    int N, M, P, nbins, nt;
    long long ntp;
    double L, invL, half2;  // half2 = (L/2)^2
    double dr, inv_dr, inv_sigma_sqrt2, six_sigma;
    double *partial;  // [gridDim.x][P*nbins]
};

__global__ __launch_bounds__(TILE) void k_hist_broad(BroadArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    double *hist = reinterpret_cast<double *>(smem);                   // [P*nbins]
    double *jx = hist + (size_t)a.P * a.nbins;                          // [3][TILE]
    int *js = reinterpret_cast<int *>(jx + 3 * TILE);                  // [TILE]
    int *prow = js + TILE;                                              // [16]
    const int tid = threadIdx.x;
    const int nq = a.P * a.nbins;
    for (int q = tid; q < nq; q += TILE) hist[q] = 0.0;
    if (tid < a.M * a.M) prow[tid] = nd::pair_index(tid / a.M, tid % a.M, a.M) * a.nbins;
    __syncthreads();
    const int N = a.N;
    const double rmax_win = (double)a.nbins * a.dr + a.six_sigma;
    for (long long t = blockIdx.x; t < a.ntp; t += gridDim.x) {
        int I, J;
        tri_index(t, a.nt, I, J);
        const int i = I * TILE + tid;
        const bool iv = i < N;
        double xi = 0.0, yi = 0.0, zi = 0.0;
        int si = 0;
        if (iv) {
            xi = a.xyz[i];
            yi = a.xyz[N + i];
            zi = a.xyz[2 * N + i];
            si = a.sp[i];
        }
        __syncthreads();
        const int j = J * TILE + tid;
        if (j < N) {
            jx[tid] = a.xyz[j];
            jx[TILE + tid] = a.xyz[N + j];
            jx[2 * TILE + tid] = a.xyz[2 * N + j];
            js[tid] = a.sp[j];
        }
        __syncthreads();
        const int jn = min(TILE, N - J * TILE);
        const int jstart = (I == J) ? tid + 1 : 0;
        if (!iv) continue;
        const int rowbase = si * a.M;
        for (int jj = jstart; jj < jn; ++jj) {
            double dx = jx[jj] - xi, dy = jx[TILE + jj] - yi, dz = jx[2 * TILE + jj] - zi;
            dx = fma(-rint(dx * a.invL), a.L, dx);
            dy = fma(-rint(dy * a.invL), a.L, dy);
            dz = fma(-rint(dz * a.invL), a.L, dz);
            const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
            if (!(r2 < a.half2)) continue;
            const double r = sqrt(r2);
            if (!(r < rmax_win)) continue;
            int k0 = (int)floor((r - a.six_sigma) * a.inv_dr);
            int k1 = (int)floor((r + a.six_sigma) * a.inv_dr);
            k0 = max(k0, 0);
            k1 = min(k1, a.nbins - 1);
            double *row = hist + prow[rowbase + js[jj]];
            // tail mass at edge k0; offsets from r in FP64, tails in FP32
            float xe = (float)(((double)k0 * a.dr - r) * a.inv_sigma_sqrt2);
            float Tlo = 0.5f * erfcf(fabsf(xe));
            bool lo_right = xe >= 0.0f;
            for (int k = k0; k <= k1; ++k) {
                const float xh = (float)(((double)(k + 1) * a.dr - r) * a.inv_sigma_sqrt2);
                const float Thi = 0.5f * erfcf(fabsf(xh));
                const bool hi_right = xh >= 0.0f;
                float wk;
                if (lo_right) wk = Tlo - Thi;
                else if (!hi_right) wk = Thi - Tlo;
                else wk = 1.0f - Tlo - Thi;
                atomicAdd(&row[k], (double)wk);
                Tlo = Thi;
                lo_right = hi_right;
            }
        }
    }
    __syncthreads();
    double *out = a.partial + (size_t)blockIdx.x * nq;
    for (int q = tid; q < nq; q += TILE) out[q] = hist[q];
}

__global__ void k_reduce_f64(const double *__restrict__ partial, int G, int n, double *__restrict__ out)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    double s = 0.0;
    for (int g = 0; g < G; ++g) s += partial[(size_t)g * n + q];
    out[q] = s;
}

// ---------------------------------------------------------------- backward
struct BackArgs {
    const float *xyz;
    const uint8_t *sp;
    const double *A;  // [P][nbins]
    int N, M, P, nbins;
    double L, invL, half2;
    double dr, inv_dr, inv_sigma, six_sigma;
    float norm;       // 1 / (sigma sqrt(2 pi))
    int jchunk;
    double *partial;  // [gridDim.y][3][N]
};

// grid (i-blocks, j-chunks): each thread owns atom i and sums over the j of
// its chunk (j != i); no atomics, partial gradients reduced afterwards.
__global__ __launch_bounds__(TILE) void k_hist_broad_bwd(BackArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    double *dA = reinterpret_cast<double *>(smem);                      // [P*nbins]
    double *jx = dA + (size_t)a.P * a.nbins;                            // [3][TILE]
    int *js = reinterpret_cast<int *>(jx + 3 * TILE);                  // [TILE]
    int *prow = js + TILE;                                              // [16]
    const int tid = threadIdx.x;
    const int nq = a.P * a.nbins;
    for (int q = tid; q < nq; q += TILE) dA[q] = a.A[q];
    if (tid < a.M * a.M) prow[tid] = nd::pair_index(tid / a.M, tid % a.M, a.M) * a.nbins;
    const int N = a.N;
    const int i = blockIdx.x * TILE + tid;
    const bool iv = i < N;
    double xi = 0.0, yi = 0.0, zi = 0.0;
    int si = 0;
    if (iv) {
        xi = a.xyz[i];
        yi = a.xyz[N + i];
        zi = a.xyz[2 * N + i];
        si = a.sp[i];
    }
    const double rmax_win = (double)a.nbins * a.dr + a.six_sigma;
    const float norm = a.norm;
    double gx = 0.0, gy = 0.0, gz = 0.0;
    const int jbeg = blockIdx.y * a.jchunk;
    const int jend = min(N, jbeg + a.jchunk);
    for (int jt = jbeg; jt < jend; jt += TILE) {
        __syncthreads();
        const int j = jt + tid;
        if (j < jend) {
            jx[tid] = a.xyz[j];
            jx[TILE + tid] = a.xyz[N + j];
            jx[2 * TILE + tid] = a.xyz[2 * N + j];
            js[tid] = a.sp[j];
        }
        __syncthreads();
        if (!iv) continue;
        const int jn = min(TILE, jend - jt);
        const int rowbase = si * a.M;
        for (int jj = 0; jj < jn; ++jj) {
            if (jt + jj == i) continue;
            double dx = xi - jx[jj], dy = yi - jx[TILE + jj], dz = zi - jx[2 * TILE + jj];
            dx = fma(-rint(dx * a.invL), a.L, dx);
            dy = fma(-rint(dy * a.invL), a.L, dy);
            dz = fma(-rint(dz * a.invL), a.L, dz);
            const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
            if (!(r2 < a.half2) || r2 == 0.0) continue;
            const double r = sqrt(r2);
            if (!(r < rmax_win)) continue;
            int k0 = (int)floor((r - a.six_sigma) * a.inv_dr);
            int k1 = (int)floor((r + a.six_sigma) * a.inv_dr);
            k0 = max(k0, 0);
            k1 = min(k1, a.nbins - 1);
            const double *row = dA + prow[rowbase + js[jj]];
            // dL/dr = sum_k A(k) (phi(x_k) - phi(x_{k+1})) / s, x_e = (e - r)/s
            float xe = (float)(((double)k0 * a.dr - r) * a.inv_sigma);
            float plo = __expf(-0.5f * xe * xe);
            double dLdr = 0.0;
            for (int k = k0; k <= k1; ++k) {
                const float xh = (float)(((double)(k + 1) * a.dr - r) * a.inv_sigma);
                const float phi_hi = __expf(-0.5f * xh * xh);
                dLdr += row[k] * (double)(norm * (plo - phi_hi));
                plo = phi_hi;
            }
            const double c = dLdr / r;
            gx += c * dx;
            gy += c * dy;
            gz += c * dz;
        }
    }
    if (iv) {
        double *out = a.partial + (size_t)blockIdx.y * 3 * N;
        out[i] = gx;
        out[N + i] = gy;
        out[2 * N + i] = gz;
    }
}

// ---------------------------------------------------------------- forces
struct ForceArgs {
    const float *xyz;
    const uint8_t *sp;
    const int32_t *unit_of;
    const float *tab;
    int N, M, n_pts;
    double L, invL, rc2, inv_h;
    int jchunk;
    double *partial;   // [gridDim.y][3][N]
    double *epart;     // [gridDim.y][gridDim.x]
};

__global__ __launch_bounds__(TILE) void k_forces(ForceArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    float *tab = reinterpret_cast<float *>(smem);                          // [P][n_pts]
    const int P = a.M * (a.M + 1) / 2;
    double *jx = reinterpret_cast<double *>(tab + ((P * a.n_pts + 3) & ~3)); // [3][TILE]
    int *ju = reinterpret_cast<int *>(jx + 3 * TILE);                      // [TILE]
    int *js = ju + TILE;                                                    // [TILE]
    int *prow = js + TILE;                                                  // [16]
    __shared__ double red[TILE / 64];
    const int tid = threadIdx.x;
    nd::stage_floats<TILE>(tab, a.tab, P * a.n_pts);
    if (tid < a.M * a.M) prow[tid] = nd::pair_index(tid / a.M, tid % a.M, a.M) * a.n_pts;
    const int N = a.N;
    const int i = blockIdx.x * TILE + tid;
    const bool iv = i < N;
    double xi = 0.0, yi = 0.0, zi = 0.0;
    int si = 0, ui = -1;
    if (iv) {
        xi = a.xyz[i];
        yi = a.xyz[N + i];
        zi = a.xyz[2 * N + i];
        si = a.sp[i];
        ui = a.unit_of[i];
    }
    double gx = 0.0, gy = 0.0, gz = 0.0, e = 0.0;
    const int jbeg = blockIdx.y * a.jchunk;
    const int jend = min(N, jbeg + a.jchunk);
    for (int jt = jbeg; jt < jend; jt += TILE) {
        __syncthreads();
        const int j = jt + tid;
        if (j < jend) {
            jx[tid] = a.xyz[j];
            jx[TILE + tid] = a.xyz[N + j];
            jx[2 * TILE + tid] = a.xyz[2 * N + j];
            ju[tid] = a.unit_of[j];
            js[tid] = a.sp[j];
        }
        __syncthreads();
        if (!iv) continue;
        const int jn = min(TILE, jend - jt);
        const int rowbase = si * a.M;
        for (int jj = 0; jj < jn; ++jj) {
            double dx = xi - jx[jj], dy = yi - jx[TILE + jj], dz = zi - jx[2 * TILE + jj];
            dx = fma(-rint(dx * a.invL), a.L, dx);
            dy = fma(-rint(dy * a.invL), a.L, dy);
            dz = fma(-rint(dz * a.invL), a.L, dz);
            const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
            if (r2 < a.rc2 && r2 > 0.0 && ju[jj] != ui) {
                const double r = sqrt(r2);
                const double t = r * a.inv_h;
                int i0 = (int)t;
                i0 = min(i0, a.n_pts - 2);
                const float *row = tab + prow[rowbase + js[jj]];
                const double u0 = row[i0], u1 = row[i0 + 1];
                const double slope = (u1 - u0) * a.inv_h;
                const double f = t - (double)i0;
                e += 0.5 * (u0 + f * (u1 - u0));
                const double c = slope / r;
                gx += c * dx;
                gy += c * dy;
                gz += c * dz;
            }
        }
    }
    if (iv) {
        double *out = a.partial + (size_t)blockIdx.y * 3 * N;
        out[i] = gx;
        out[N + i] = gy;
        out[2 * N + i] = gz;
    }
    for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o);
    if ((tid & 63) == 0) red[tid >> 6] = e;
    __syncthreads();
    if (tid == 0) a.epart[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void k_sum_serial(const double *__restrict__ v, int n, double *__restrict__ out)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int q = threadIdx.x; q < n; q += 256) s += v[q];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

int n_jchunks(nd_box *b)
{
    // enough blocks to fill the chip with about 4 blocks per CU
    const int nib = (b->N + TILE - 1) / TILE;
    int want = (4 * nd::cu_count(b->device) + nib - 1) / nib;
    want = std::max(1, std::min(want, 64));
    return want;
}

}  // namespace

namespace nd {

void launch_hist_broad(nd_box *b, double dr, int nbins, double sigma, double *d_nhat)
{
    BroadArgs a;
    a.xyz = b->xyz;
    a.sp = b->species;
    a.N = b->N;
    a.M = b->M;
    a.P = b->P;
    a.nbins = nbins;
    a.nt = (b->N + TILE - 1) / TILE;
    a.ntp = (long long)a.nt * (a.nt + 1) / 2;
    a.L = b->L;
    a.invL = 1.0 / b->L;
    a.half2 = 0.25 * b->L * b->L;
    a.dr = dr;
    a.inv_dr = 1.0 / dr;
    a.inv_sigma_sqrt2 = 1.0 / (sigma * std::sqrt(2.0));
    a.six_sigma = 6.0 * sigma;
    const int nq = a.P * nbins;
    size_t lds = sizeof(double) * ((size_t)nq + 3 * TILE) + sizeof(int) * (TILE + 16);
    if (lds > 160 * 1024) fail(ND_E_UNSUPPORTED, "broadened histogram does not fit in LDS");
    int per_cu = (int)std::max<size_t>(1, std::min<size_t>(4, (160 * 1024) / (lds + 1024)));
    long long G = (long long)cu_count(b->device) * per_cu;
    if (G > a.ntp) G = a.ntp;
    a.partial = static_cast<double *>(workspace(b, sizeof(double) * (size_t)G * nq));
    {
        ProfScope ps(b, ND_PROF_HIST_BROAD);
        hipLaunchKernelGGL(k_hist_broad, dim3((unsigned)G), dim3(TILE), lds, b->stream, a);
        ND_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_reduce_f64, dim3((nq + 255) / 256), dim3(256), 0, b->stream, a.partial, (int)G, nq, d_nhat);
    ND_HIP(hipGetLastError());
}

void launch_hist_broad_backward(nd_box *b, double dr, int nbins, double sigma, const double *d_A, double *d_grad)
{
    BackArgs a;
    a.xyz = b->xyz;
    a.sp = b->species;
    a.A = d_A;
    a.N = b->N;
    a.M = b->M;
    a.P = b->P;
    a.nbins = nbins;
    a.L = b->L;
    a.invL = 1.0 / b->L;
    a.half2 = 0.25 * b->L * b->L;
    a.dr = dr;
    a.inv_dr = 1.0 / dr;
    a.inv_sigma = 1.0 / sigma;
    a.six_sigma = 6.0 * sigma;
    a.norm = (float)(1.0 / (sigma * std::sqrt(2.0 * M_PI)));
    const int nch = n_jchunks(b);
    a.jchunk = (b->N + nch - 1) / nch;
    const int nib = (b->N + TILE - 1) / TILE;
    size_t lds = sizeof(double) * ((size_t)b->P * nbins + 3 * TILE) + sizeof(int) * (TILE + 16);
    if (lds > 160 * 1024) fail(ND_E_UNSUPPORTED, "adjoint table does not fit in LDS");
    a.partial = static_cast<double *>(workspace(b, sizeof(double) * (size_t)nch * 3 * b->N));
    {
        ProfScope ps(b, ND_PROF_HIST_BROAD_BWD);
        hipLaunchKernelGGL(k_hist_broad_bwd, dim3(nib, nch), dim3(TILE), lds, b->stream, a);
        ND_HIP(hipGetLastError());
    }
    const int n = 3 * b->N;
    hipLaunchKernelGGL(k_reduce_f64, dim3((n + 255) / 256), dim3(256), 0, b->stream, a.partial, nch, n, d_grad);
    ND_HIP(hipGetLastError());
}

void launch_forces(nd_box *b, double *d_grad, double *d_E)
{
    ForceArgs a;
    a.xyz = b->xyz;
    a.sp = b->species;
    a.unit_of = b->unit_of;
    a.tab = b->tab;
    a.N = b->N;
    a.M = b->M;
    a.n_pts = b->n_pts;
    a.L = b->L;
    a.invL = 1.0 / b->L;
    a.rc2 = b->rc * b->rc;
    a.inv_h = 1.0 / b->h;
    const int nch = n_jchunks(b);
    a.jchunk = (b->N + nch - 1) / nch;
    const int nib = (b->N + TILE - 1) / TILE;
    const int P = b->P;
    size_t lds = sizeof(float) * (size_t)((P * b->n_pts + 3) & ~3) + sizeof(double) * 3 * TILE +
                 sizeof(int) * (2 * TILE + 16);
    if (lds > 160 * 1024) fail(ND_E_UNSUPPORTED, "potential table does not fit in LDS");
    size_t gbytes = sizeof(double) * (size_t)nch * 3 * b->N;
    size_t ebytes = sizeof(double) * (size_t)nch * nib;
    char *ws = static_cast<char *>(workspace(b, gbytes + ebytes));
    a.partial = reinterpret_cast<double *>(ws);
    a.epart = reinterpret_cast<double *>(ws + gbytes);
    {
        ProfScope ps(b, ND_PROF_FORCES);
        hipLaunchKernelGGL(k_forces, dim3(nib, nch), dim3(TILE), lds, b->stream, a);
        ND_HIP(hipGetLastError());
    }
    const int n = 3 * b->N;
    hipLaunchKernelGGL(k_reduce_f64, dim3((n + 255) / 256), dim3(256), 0, b->stream, a.partial, nch, n, d_grad);
    ND_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sum_serial, dim3(1), dim3(256), 0, b->stream, a.epart, nch * nib, d_E);
    ND_HIP(hipGetLastError());
}

}  // namespace nd

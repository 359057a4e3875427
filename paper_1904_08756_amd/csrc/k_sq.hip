// g(r) normalisation and the Eq. 1 sine transform to S(Q), plus the adjoint
// of both (for the chi^2 gradient).  All FP64.
//
//   g_p(k)  = n_p(k) / (npairs_p Vshell(k) / V),  Vshell(k) = (4 pi/3)((k+1)^3 - k^3) dr^3
//   S(Q_i)  = self + 4 pi rho sum_k h(k) sinc(Q_i r_k),  r_k = (k + 1/2) dr,
//   h(k)    = r_k^2 dr sum_p w_p (g_p(k) - 1)
// The partial-type sum is folded into h(k) first, so each (Q, r) pair needs
// one sine instead of one per pair type.
#include "nd_internal.h"

#include <algorithm>
#include <cmath>

namespace {

constexpr int MAXP = ND_MAX_SPECIES * (ND_MAX_SPECIES + 1) / 2;

struct PVec {
    double v[MAXP];
};

__device__ __forceinline__ double shell_volume(int k, double dr)
{
    const double k0 = (double)k, k1 = (double)(k + 1);
    return (4.0 * M_PI / 3.0) * (k1 * k1 * k1 - k0 * k0 * k0) * dr * dr * dr;
}

template <class T>
__global__ void k_gr_normalize(const T *__restrict__ counts, int P, int nbins, double dr, double V, PVec npairs,
                               double *__restrict__ g)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= P * nbins) return;
    const int p = q / nbins, k = q - p * nbins;
    g[q] = (double)counts[q] / (npairs.v[p] * shell_volume(k, dr) / V);
}

__device__ __forceinline__ double sinc(double x) { return x == 0.0 ? 1.0 : sin(x) / x; }

// S at one Q point by one block of 256 threads (threads over r); the
// partial-type sum h(k) = r_k^2 dr sum_p w_p (g_p(k) - 1) is formed on the fly
__device__ __forceinline__ void sq_point(const double *__restrict__ g, int P, int nbins, double dr, const double *w,
                                         double four_pi_rho, double self_term, double q, double *out)
{
    __shared__ double red[256 / 64];
    double s = 0.0;
    for (int k = threadIdx.x; k < nbins; k += 256) {
        const double r = ((double)k + 0.5) * dr;
        double hk = 0.0;
        for (int p = 0; p < P; ++p) hk += w[p] * (g[(size_t)p * nbins + k] - 1.0);
        s += r * r * dr * hk * sinc(q * r);
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) *out = self_term + four_pi_rho * ((red[0] + red[1]) + (red[2] + red[3]));
}

// one block per Q point
__global__ __launch_bounds__(256) void k_sq(const double *__restrict__ g, int P, int nbins, double dr, PVec w,
                                            double four_pi_rho, double self_term, const double *__restrict__ Q,
                                            double *__restrict__ S)
{
    sq_point(g, P, nbins, dr, w.v, four_pi_rho, self_term, Q[blockIdx.x], S + blockIdx.x);
}

// Several boxes per launch: blockIdx.y selects the box.
__global__ void k_gr_normalize_multi(const nd::SqBoxDesc *__restrict__ d)
{
    const nd::SqBoxDesc &b = d[blockIdx.y];
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= b.P * b.nbins) return;
    const int p = q / b.nbins, k = q - p * b.nbins;
    b.g[q] = (double)b.counts[q] / (b.npairs[p] * shell_volume(k, b.dr) / b.V);
}

__global__ __launch_bounds__(256) void k_sq_multi(const nd::SqBoxDesc *__restrict__ d, const double *__restrict__ Q)
{
    const nd::SqBoxDesc &b = d[blockIdx.y];
    sq_point(b.g, b.P, b.nbins, b.dr, b.w, b.four_pi_rho, b.self_term, Q[blockIdx.x], b.S + blockIdx.x);
}

// A_p(k) = [sum_i dLdS_i sinc(Q_i r_k)] w_p 4 pi rho r_k^2 dr / (npairs_p Vshell(k)/V)
__global__ __launch_bounds__(256) void k_sq_adjoint(const double *__restrict__ dLdS, const double *__restrict__ Q,
                                                    int nQ, int P, int nbins, double dr, double four_pi_rho,
                                                    double V, PVec w, PVec npairs, double *__restrict__ A)
{
    __shared__ double red[256 / 64];
    const int k = blockIdx.x;
    const double r = ((double)k + 0.5) * dr;
    double s = 0.0;
    for (int i = threadIdx.x; i < nQ; i += 256) s += dLdS[i] * sinc(Q[i] * r);
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x < P) {
        const int p = threadIdx.x;
        const double tot = (red[0] + red[1]) + (red[2] + red[3]);
        A[(size_t)p * nbins + k] = tot * w.v[p] * four_pi_rho * r * r * dr / (npairs.v[p] * shell_volume(k, dr) / V);
    }
}

__global__ __launch_bounds__(256) void k_chi2(const double *__restrict__ S, const double *__restrict__ T, int n,
                                              double *__restrict__ chi2, double *__restrict__ grad)
{
    __shared__ double red[256 / 64];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        const double d = S[i] - T[i];
        s += d * d;
        if (grad) grad[i] = 2.0 * d;
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) *chi2 = (red[0] + red[1]) + (red[2] + red[3]);
}

PVec make_pvec(const double *v, int P)
{
    PVec x;
    for (int p = 0; p < MAXP; ++p) x.v[p] = p < P ? v[p] : 0.0;
    return x;
}

}  // namespace

namespace nd {

void launch_gr_normalize(const uint64_t *counts, int P, int nbins, double dr, double V, const double *npairs_host,
                         double *g, hipStream_t s)
{
    const int n = P * nbins;
    hipLaunchKernelGGL(k_gr_normalize<uint64_t>, dim3((n + 255) / 256), dim3(256), 0, s, counts, P, nbins, dr, V,
                       make_pvec(npairs_host, P), g);
    ND_HIP(hipGetLastError());
}

void launch_gr_normalize_f64(const double *counts, int P, int nbins, double dr, double V, const double *npairs_host,
                             double *g, hipStream_t s)
{
    const int n = P * nbins;
    hipLaunchKernelGGL(k_gr_normalize<double>, dim3((n + 255) / 256), dim3(256), 0, s, counts, P, nbins, dr, V,
                       make_pvec(npairs_host, P), g);
    ND_HIP(hipGetLastError());
}

void launch_chi2(const double *S, const double *T, int nQ, double *chi2, double *grad, hipStream_t s)
{
    hipLaunchKernelGGL(k_chi2, dim3(1), dim3(256), 0, s, S, T, nQ, chi2, grad);
    ND_HIP(hipGetLastError());
}

void launch_sq(const double *g, int P, int nbins, double dr, double rho, const double *w_host, double self_term,
               const double *Q, int nQ, double *S, hipStream_t s)
{
    hipLaunchKernelGGL(k_sq, dim3(nQ), dim3(256), 0, s, g, P, nbins, dr, make_pvec(w_host, P), 4.0 * M_PI * rho,
                       self_term, Q, S);
    ND_HIP(hipGetLastError());
}

void launch_sq_adjoint(const double *dLdS, int P, int nbins, double dr, double rho, double V, const double *w_host,
                       const double *npairs_host, const double *Q, int nQ, double *A, hipStream_t s)
{
    hipLaunchKernelGGL(k_sq_adjoint, dim3(nbins), dim3(256), 0, s, dLdS, Q, nQ, P, nbins, dr, 4.0 * M_PI * rho, V,
                       make_pvec(w_host, P), make_pvec(npairs_host, P), A);
    ND_HIP(hipGetLastError());
}

// ---- several boxes (the batched form)
struct SqMulti {
    std::vector<SqBoxDesc> boxes;
    SqBoxDesc *d_boxes = nullptr;
    size_t cap = 0;
    const double *Q = nullptr;
    int nQ = 0, max_nq = 0;
};

SqMulti *sq_multi_create() { return new SqMulti(); }

void sq_multi_destroy(SqMulti *m)
{
    if (!m) return;
    dfree(m->d_boxes);
    delete m;
}

void sq_multi_plan(SqMulti *m, const SqBoxDesc *descs, int n, const double *Q, int nQ, std::vector<long long> &sig)
{
    m->boxes.assign(descs, descs + n);
    m->Q = Q;
    m->nQ = nQ;
    m->max_nq = 0;
    for (int i = 0; i < n; ++i) m->max_nq = std::max(m->max_nq, descs[i].P * descs[i].nbins);
    if (m->cap < (size_t)n || !m->d_boxes) {
        dfree(m->d_boxes);
        m->d_boxes = static_cast<SqBoxDesc *>(dmalloc(sizeof(SqBoxDesc) * n));
        m->cap = n;
    }
    sig.push_back(0x5351);
    sig.push_back(n);
    sig.push_back(nQ);
    sig.push_back(m->max_nq);
    sig.push_back((long long)(uintptr_t)Q);
    sig.push_back((long long)(uintptr_t)m->d_boxes);
}

void sq_multi_upload(SqMulti *m, hipStream_t s)
{
    ND_HIP(hipMemcpyAsync(m->d_boxes, m->boxes.data(), sizeof(SqBoxDesc) * m->boxes.size(), hipMemcpyHostToDevice, s));
    ND_HIP(hipStreamSynchronize(s));
}

void sq_multi_enqueue(SqMulti *m, hipStream_t s)
{
    const int n = (int)m->boxes.size();
    hipLaunchKernelGGL(k_gr_normalize_multi, dim3((m->max_nq + 255) / 256, n), dim3(256), 0, s, m->d_boxes);
    ND_HIP(hipGetLastError());
    if (m->nQ > 0) {
        hipLaunchKernelGGL(k_sq_multi, dim3(m->nQ, n), dim3(256), 0, s, m->d_boxes, m->Q);
        ND_HIP(hipGetLastError());
    }
}

}  // namespace nd

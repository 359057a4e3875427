// Running pair-count histogram: N(r) kept current by the Delta N(r) of every
// accepted trial move (Sec. "Acceleration method": Delta N(r) is recomputed
// after every Monte Carlo step at a cost proportional to N, while the full
// N(r) costs N^2), and the accumulation of N(r) over samples for averaged
// g(r) and S(Q) (Sec. "NeuDATool Algorithmic Flow", steps EPMC and
// "Accumulate g(r) and S(Q)").
//
// After a batch's decision has committed its accepted trials, the batch's
// Delta N is the change of every pair that has at least one atom in a moved
// unit:
//   pairs (a moved, j not moved):      bin(x'_a, x_j)  - bin(x_a, x_j)
//   pairs (a, b moved, a < b by trial, or a < b in one unit):
//                                      bin(x'_a, x'_b) - bin(x_a, x_b)
// with the histogram's exact bin rule (FP64 r^2 of the float32
// coordinates, bin = max{k : (k dr)^2 <= r^2}, counted iff k < nbins), so
// the running counts equal a fresh histogram bit for bit.  The decision
// tags each moved unit with the batch's tag plus the trial's index, which
// tells a j atom whether (and by which trial) it moved in this batch; the
// positions before the move come from the trial records.
//
// One block per group of j atoms loops over the batch's accepted trials,
// counting +1/-1 in an LDS histogram; the blocks' histograms are written to
// per-block slices and summed by a second kernel into the running u64
// counts (integer sums, independent of order).
#include "nd_internal.h"
#include "nd_pair.h"

#include <algorithm>
#include <cmath>

namespace {

using nd::ldg;

constexpr int DN_THREADS = 256;
constexpr int DN_KMAX = 2048;  // trials per batch (as the Metropolis kernels)

struct DnArgs {
    const float *xyz;           // [3][N] after the batch's commit
    const uint8_t *sp;          // [N]
    const int32_t *unit_of;     // [N]
    const long long *moved;     // [n_units] tags
    const nd::Trial *trials;    // the batch's trial records
    const uint8_t *acc;         // [kb] decisions
    int N, M, P, nbins, kb;
    double L, dr;
    float inv_dr;
    long long tag_base;
    int32_t *partial;           // [gridDim.x][P * nbins]
};

// The histogram's exact rule: nearest-image length min(|d|, L - |d|) per
// axis (equal to the d -/+ L form for coordinates in [0, L)), r2 =
// fma(dz,dz, fma(dy,dy, dx*dx)) in FP64, bin = max{k : (k dr)^2 <= r2}.  The
// FP32 root gives a candidate within one bin; the FP64 edges decide.
__device__ __forceinline__ int exact_bin(float xi, float yi, float zi, float xj, float yj, float zj, double L,
                                         double dr, float inv_dr)
{
    const double ax = fabs((double)xj - (double)xi);
    const double ay = fabs((double)yj - (double)yi);
    const double az = fabs((double)zj - (double)zi);
    const double mx = fmin(ax, L - ax), my = fmin(ay, L - ay), mz = fmin(az, L - az);
    const double r2 = fma(mz, mz, fma(my, my, mx * mx));
    int k = (int)(sqrtf((float)r2) * inv_dr);
    const double e = (double)k * dr;
    if (r2 < e * e) {
        --k;
    } else {
        const double e1 = (double)(k + 1) * dr;
        if (r2 >= e1 * e1) ++k;
    }
    return k;
}

__device__ __forceinline__ void dn_count(int *hist, int row, int k, int nbins, int v)
{
    if (k >= 0 && k < nbins) atomicAdd(&hist[row + k], v);
}

__global__ __launch_bounds__(DN_THREADS) void k_mc_dn(DnArgs a)
{
    extern __shared__ __align__(16) int s_hist[];  // [P * nbins], then the accepted list
    __shared__ int s_n;
    __shared__ int s_prow[16];
    unsigned short *s_list = reinterpret_cast<unsigned short *>(s_hist + a.P * a.nbins);
    const int tid = threadIdx.x, lane = tid & 63;
    const int nq = a.P * a.nbins;
    for (int q = tid; q < nq; q += DN_THREADS) s_hist[q] = 0;
    if (tid == 0) s_n = 0;
    if (tid < a.M * a.M) s_prow[tid] = nd::pair_index(tid / a.M, tid % a.M, a.M) * a.nbins;
    __syncthreads();
    // the accepted trials in trial order
    for (int k0 = 0; k0 < a.kb; k0 += DN_THREADS) {
        const int k = k0 + tid;
        const bool acc = k < a.kb && ldg(a.acc + k) != 0;
        const unsigned long long m = __ballot(acc);
        __shared__ int s_wbase[DN_THREADS / 64];
        if (lane == 0) s_wbase[tid >> 6] = __popcll(m);
        __syncthreads();
        int base = s_n;
        for (int w = 0; w < (tid >> 6); ++w) base += s_wbase[w];
        if (acc) s_list[base + __popcll(m & ((1ull << lane) - 1ull))] = (unsigned short)k;
        __syncthreads();
        if (tid == 0)
            for (int w = 0; w < DN_THREADS / 64; ++w) s_n += s_wbase[w];
        __syncthreads();
    }
    const int n_acc = s_n;
    const int N = a.N;
    for (int j = blockIdx.x * DN_THREADS + tid; j < N; j += gridDim.x * DN_THREADS) {
        const float xj = a.xyz[j], yj = a.xyz[N + j], zj = a.xyz[2 * N + j];
        const int sj = a.sp[j];
        const long long tag = a.moved[a.unit_of[j]];
        // trial of this batch that moved j (a whole unit, or one atom of a
        // flexible unit), or -1
        int mj = (tag >= a.tag_base && tag < a.tag_base + nd::TRACK_TAG_STRIDE) ? (int)(tag - a.tag_base) : -1;
        float ojx = xj, ojy = yj, ojz = zj;  // j before the batch
        if (mj >= 0) {
            const nd::Trial &Tm = a.trials[mj];
            const int at = j - Tm.a0;
            if (at >= 0 && at < Tm.na) {
                ojx = Tm.old_x[at][0];
                ojy = Tm.old_x[at][1];
                ojz = Tm.old_x[at][2];
            } else {
                mj = -1;  // j's unit moved only one of its other atoms
            }
        }
        for (int li = 0; li < n_acc; ++li) {
            const int k = __builtin_amdgcn_readfirstlane(s_list[li]);
            const nd::Trial &T = a.trials[k];
            const int na = T.na, a0 = T.a0;
            if (mj >= 0 && (mj < k)) continue;  // counted from the earlier trial
            for (int at = 0; at < na; ++at) {
                const int ia = a0 + at;
                if (mj == k && j <= ia) continue;  // one unit: each pair once, no self pair
                const int row = s_prow[a.sp[ia] * a.M + sj];
                const int kn = exact_bin(T.new_x[at][0], T.new_x[at][1], T.new_x[at][2], xj, yj, zj, a.L, a.dr,
                                         a.inv_dr);
                const int ko = exact_bin(T.old_x[at][0], T.old_x[at][1], T.old_x[at][2], ojx, ojy, ojz, a.L, a.dr,
                                         a.inv_dr);
                if (kn != ko) {
                    dn_count(s_hist, row, kn, a.nbins, 1);
                    dn_count(s_hist, row, ko, a.nbins, -1);
                }
            }
        }
    }
    __syncthreads();
    int32_t *out = a.partial + (size_t)blockIdx.x * nq;
    for (int q = tid; q < nq; q += DN_THREADS) out[q] = s_hist[q];
}

// counts[q] += sum over blocks of partial[g][q] (u64 arithmetic modulo 2^64,
// so negative block sums subtract; the result is a count again).
__global__ void k_dn_reduce(const int32_t *__restrict__ partial, int G, int nq, unsigned long long *__restrict__ counts)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    long long s = 0;
    for (int g = 0; g < G; ++g) s += partial[(size_t)g * nq + q];
    counts[q] += (unsigned long long)s;
}

__global__ void k_fill_i64(long long *__restrict__ p, long long n, long long v)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_add_u64(const unsigned long long *__restrict__ x, unsigned long long *__restrict__ sum, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) sum[i] += x[i];
}

__global__ void k_mean_u64(const unsigned long long *__restrict__ sum, double inv_n, int n, double *__restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (double)sum[i] * inv_n;
}

}  // namespace

namespace nd {

void track_stop(nd_box *b)
{
    Track &t = b->track;
    if (t.counts || t.sum || t.partial || t.moved) ND_HIP(hipStreamSynchronize(b->stream));
    dfree(t.counts);
    dfree(t.sum);
    dfree(t.partial);
    dfree(t.moved);
    t = Track();
}

void track_start(nd_box *b, double dr, int nbins)
{
    track_stop(b);
    Track &t = b->track;
    const int nq = b->P * nbins;
    const size_t lds = sizeof(int) * (size_t)nq + sizeof(unsigned short) * DN_KMAX;
    if (lds > 160 * 1024) fail(ND_E_UNSUPPORTED, "running histogram does not fit in LDS (P*nbins too large)");
    t.G = (int)std::min<long long>((b->N + DN_THREADS - 1) / DN_THREADS, 4LL * cu_count(b->device));
    try {
        t.counts = static_cast<uint64_t *>(dmalloc(sizeof(uint64_t) * (size_t)nq));
        t.sum = static_cast<uint64_t *>(dmalloc(sizeof(uint64_t) * (size_t)nq));
        t.partial = static_cast<int32_t *>(dmalloc(sizeof(int32_t) * (size_t)t.G * nq));
        t.moved = static_cast<long long *>(dmalloc(sizeof(long long) * (size_t)b->n_units));
    } catch (...) {
        track_stop(b);
        throw;
    }
    t.dr = dr;
    t.nbins = nbins;
    t.on = true;
    hipLaunchKernelGGL(k_fill_i64, dim3((b->n_units + 255) / 256), dim3(256), 0, b->stream, t.moved,
                       (long long)b->n_units, -1LL);
    ND_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_fill_i64, dim3((nq + 255) / 256), dim3(256), 0, b->stream,
                       reinterpret_cast<long long *>(t.sum), (long long)nq, 0LL);
    ND_HIP(hipGetLastError());
    track_refresh(b);
}

// The running counts from scratch (after the coordinates changed other
// than by tracked moves).
void track_refresh(nd_box *b)
{
    Track &t = b->track;
    if (!t.on) return;
    launch_pair_histogram(b, t.dr, t.nbins, t.counts);
    t.valid = true;
}

void track_launch(nd_box *b, const Trial *trials, const uint8_t *acc, int kb, long long tag_base)
{
    Track &t = b->track;
    if (kb <= 0) return;
    DnArgs a;
    a.xyz = b->xyz;
    a.sp = b->species;
    a.unit_of = b->unit_of;
    a.moved = t.moved;
    a.trials = trials;
    a.acc = acc;
    a.N = b->N;
    a.M = b->M;
    a.P = b->P;
    a.nbins = t.nbins;
    a.kb = kb;
    a.L = b->L;
    a.dr = t.dr;
    a.inv_dr = (float)(1.0 / t.dr);
    a.tag_base = tag_base;
    a.partial = t.partial;
    const int nq = b->P * t.nbins;
    const size_t lds = sizeof(int) * (size_t)nq + sizeof(unsigned short) * DN_KMAX;
    hipLaunchKernelGGL(k_mc_dn, dim3(t.G), dim3(DN_THREADS), lds, b->stream, a);
    ND_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_dn_reduce, dim3((nq + 255) / 256), dim3(256), 0, b->stream, t.partial, t.G, nq,
                       reinterpret_cast<unsigned long long *>(t.counts));
    ND_HIP(hipGetLastError());
}

void track_accumulate(nd_box *b)
{
    Track &t = b->track;
    const int nq = b->P * t.nbins;
    hipLaunchKernelGGL(k_add_u64, dim3((nq + 255) / 256), dim3(256), 0, b->stream,
                       reinterpret_cast<const unsigned long long *>(t.counts),
                       reinterpret_cast<unsigned long long *>(t.sum), nq);
    ND_HIP(hipGetLastError());
    ++t.n_samples;
}

void track_mean(nd_box *b, double *d_mean)
{
    Track &t = b->track;
    const int nq = b->P * t.nbins;
    hipLaunchKernelGGL(k_mean_u64, dim3((nq + 255) / 256), dim3(256), 0, b->stream,
                       reinterpret_cast<const unsigned long long *>(t.sum), 1.0 / (double)t.n_samples, nq, d_mean);
    ND_HIP(hipGetLastError());
}

}  // namespace nd

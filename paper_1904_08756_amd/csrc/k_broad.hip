// Differentiated form: a Gaussian-broadened pair histogram (forward), the
// gradient of a loss on that histogram with respect to every coordinate
// (backward), and the gradient of the tabulated total energy (forces).
//
// Broadening: a pair at distance r adds to bin k the Gaussian mass between
// its edges, w_k(r) = Phi((e_{k+1}-r)/s) - Phi((e_k-r)/s), e_k = k dr, for
// the bins that intersect [r - 6s, r + 6s].  Each edge needs one tail mass
// T(x) = Phi(-|x|), x = (e - r)/s, from which every bin weight follows
// without cancellation:
//   bin right of r: T(x_k) - T(x_{k+1});  left of r: T(x_{k+1}) - T(x_k);
//   bin containing r: 1 - T(x_k) - T(x_{k+1}).
// The tail is taken as T(x) = phi(x) R(x) with phi the Gaussian density
// and R the Mills ratio T/phi, a smooth function tabulated on [0, 8] (step
// 1/32, cubic Taylor coefficients from R' = xR - 1; beyond 8, T < 7e-16 is
// dropped).  Edge offsets x = (k - k_r - f) dr/s come from the pair's bin
// k_r and fraction f of r/dr.  Distances are FP64 from the float32
// coordinates; per-pair weights FP32; a block sums them as integers in
// units of 2^-32 (exact and independent of order), the blocks' sums are
// added in FP64.
#include "nd_internal.h"
#include "nd_pair.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <vector>

namespace {

constexpr int MILLS_PER_UNIT = 32;                   // table points per unit of x
constexpr float MILLS_XMAX = 8.0f;
constexpr int MILLS_N = 8 * MILLS_PER_UNIT + 1;      // points 0, 1/32, ..., 8
constexpr float NEG_HALF_LOG2E = -0.72134752044448170f;  // -log2(e)/2
constexpr float INV_SQRT_2PI = 0.39894228040143268f;

// Upper-tail mass Phi(-ax) for ax >= 0 from the Mills-ratio table in LDS
// (c.x..c.w: R and its first three Taylor coefficients at the nearest point).
__device__ __forceinline__ float gauss_tail(float ax, const float4 *mills)
{
    const float phi = __builtin_amdgcn_exp2f(ax * ax * NEG_HALF_LOG2E) * INV_SQRT_2PI;
    const int i = min((int)fmaf(ax, (float)MILLS_PER_UNIT, 0.5f), MILLS_N - 1);
    const float4 c = mills[i];
    const float d = ax - (float)i * (1.0f / MILLS_PER_UNIT);
    const float R = fmaf(d, fmaf(d, fmaf(d, c.w, c.z), c.y), c.x);
    return ax < MILLS_XMAX ? phi * R : 0.0f;
}

// Tail mass phi R(ax) for ax >= 0 given the density phi at ax.
__device__ __forceinline__ float gauss_tail_phi(float ax, float phi, const float4 *mills)
{
    const int i = min((int)fmaf(ax, (float)MILLS_PER_UNIT, 0.5f), MILLS_N - 1);
    const float4 c = mills[i];
    const float d = ax - (float)i * (1.0f / MILLS_PER_UNIT);
    const float R = fmaf(d, fmaf(d, fmaf(d, c.w, c.z), c.y), c.x);
    return ax < MILLS_XMAX ? phi * R : 0.0f;
}

// Gaussian density at x (any sign).
__device__ __forceinline__ float gauss_pdf(float x)
{
    return __builtin_amdgcn_exp2f(x * x * NEG_HALF_LOG2E) * INV_SQRT_2PI;
}

// Nearest-image distance of float32 positions in FP64 (min(|d|, L - |d|)
// per axis) and the displacement d = x_i - x_j with the sign of that image.
__device__ __forceinline__ double nearest_r2(double dx, double dy, double dz, double L)
{
    const double ax = fabs(dx), ay = fabs(dy), az = fabs(dz);
    const double mx = fmin(ax, L - ax), my = fmin(ay, L - ay), mz = fmin(az, L - az);
    return fma(mz, mz, fma(my, my, mx * mx));
}

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
    double dr, inv_dr, six_sigma;
    float beta;              // dr / sigma
    const float4 *mills;     // [MILLS_N] Mills-ratio table
    // bin-mass table (wt_nm > 0): the mass of bin kr + m, m = wt_m0 + mi, of
    // a unit Gaussian at fraction f of bin kr, as a quadratic in f about the
    // centre of each of WT_NP pieces: (value as two floats, hi + lo, and the
    // first two Taylor coefficients), one 16-byte read per bin
    const float4 *wt;        // [wt_nm][WT_NP]
    int wt_m0, wt_nm;
    double *partial;  // [gridDim.x][P*nbins]
};

constexpr int WT_NP = 64;             // pieces of the bin-mass table per unit of f
constexpr int WT_MAX_BYTES = 16384;   // the table path is taken when the table fits this

constexpr int BQ = 128;     // pairs queued per wave
constexpr int FTILE = 512;  // atoms per tile of the forward: eight waves share one LDS histogram

// The window of one pair at distance r (r < L/2) into the u64 row h from the
// bin-mass table: one entry per bin of the window, the value (hi + lo,
// summed in FP64) plus the FP32 Taylor terms (at most a few 1e-3), in units
// of 2^-32.  Bins past the table (masses below 1e-13) are left out.
__device__ __forceinline__ void broad_pair_tab(const BroadArgs &a, const float4 *t, unsigned long long *h, double r2)
{
    const double r = nd::sqrt_nr(r2);
    int k0 = (int)floor((r - a.six_sigma) * a.inv_dr);
    int k1 = (int)floor((r + a.six_sigma) * a.inv_dr);
    k0 = max(k0, 0);
    k1 = min(k1, a.nbins - 1);
    const double u = r * a.inv_dr;
    const int kr = (int)u;
    const float f = (float)(u - (double)kr);
    const int pc = min((int)(f * (float)WT_NP), WT_NP - 1);
    const float d = f - ((float)pc + 0.5f) * (1.0f / WT_NP);
    // offsets k - kr stay inside the table's range (it has a bin of margin
    // on each side); the clamps only guard that
    int m = k0 - kr - a.wt_m0;
    if (m < 0) {
        k0 -= m;
        m = 0;
    }
    k1 = min(k1, k0 + (a.wt_nm - 1 - m));
    const float4 *tp = t + m * WT_NP + pc;
    auto bin = [&](const float4 c) {
        const double w = (double)c.x + ((double)c.y + (double)(d * fmaf(d, c.w, c.z)));
        return (unsigned long long)__double2uint_rn(w * 4294967296.0);
    };
    int k = k0;
    for (; k < k1; k += 2, tp += 2 * WT_NP) {
        const float4 c0 = tp[0], c1 = tp[WT_NP];
        atomicAdd(&h[k], bin(c0));
        atomicAdd(&h[k + 1], bin(c1));
    }
    if (k == k1) atomicAdd(&h[k], bin(tp[0]));
}

// The window of one pair at distance r (r < L/2) into the u64 row h: bin
// weights as differences of the edges' tail masses, in units of 2^-32.  Each
// edge's density is evaluated directly: a recurrence along the window would
// raise the rounding of its first factor to the power of the step count,
// which biases every pair's far bins alike.
__device__ __forceinline__ void broad_pair(const BroadArgs &a, const float4 *mills, unsigned long long *h, double r2)
{
    const double r = nd::sqrt_nr(r2);
    int k0 = (int)floor((r - a.six_sigma) * a.inv_dr);
    int k1 = (int)floor((r + a.six_sigma) * a.inv_dr);
    k0 = max(k0, 0);
    k1 = min(k1, a.nbins - 1);
    const double u = r * a.inv_dr;
    const int kr = (int)u;
    const float f = (float)(u - (double)kr);
    const float beta = a.beta;
    const float x = ((float)(k0 - kr) - f) * beta;
    float T = gauss_tail_phi(fabsf(x), gauss_pdf(x), mills);
    bool right = x >= 0.0f;
    for (int k = k0; k <= k1; ++k) {
        const float xh = ((float)(k + 1 - kr) - f) * beta;
        const float Th = gauss_tail_phi(fabsf(xh), gauss_pdf(xh), mills);
        const bool rh = xh >= 0.0f;
        const float wk = right ? T - Th : (rh ? 1.0f - T - Th : Th - T);
        // weight in units of 2^-32 (exact integer sums, deterministic)
        atomicAdd(&h[k], (unsigned long long)__float2uint_rn(wk * 4294967296.0f));
        T = Th;
        right = rh;
    }
}

// Each lane owns atom i of the I tile and tests it against the J tile; the
// pairs inside the window range are queued per wave in LDS and their windows
// are evaluated 64 at a time, one per lane, so no lane idles on the pairs
// past L/2.  Integer sums: the result does not depend on the order.
template <bool TAB>
__global__ __launch_bounds__(FTILE) void k_hist_broad(BroadArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned long long *hist = reinterpret_cast<unsigned long long *>(smem);  // [P*nbins] weights x 2^32
    double *jx = reinterpret_cast<double *>(hist + (size_t)a.P * a.nbins);   // [3][FTILE]
    // the bin-mass table (TAB) or the Mills-ratio table
    const int ntab = TAB ? a.wt_nm * WT_NP : MILLS_N;
    float4 *tab = reinterpret_cast<float4 *>(jx + 3 * FTILE);                 // [ntab]
    int *js = reinterpret_cast<int *>(tab + ntab);                            // [FTILE]
    int *prow = js + FTILE;                                                    // [16]
    __shared__ double s_qr[FTILE / 64][BQ];
    __shared__ int s_qrow[FTILE / 64][BQ];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const unsigned long long lt = (1ull << lane) - 1ull;
    const int nq = a.P * a.nbins;
    for (int q = tid; q < nq; q += FTILE) hist[q] = 0ull;
    for (int q = tid; q < ntab; q += FTILE) tab[q] = nd::ld4((TAB ? a.wt : a.mills) + q);
    if (tid < a.M * a.M) prow[tid] = nd::pair_index(tid / a.M, tid % a.M, a.M) * a.nbins;
    __syncthreads();
    const int N = a.N;
    const double rmax_win = (double)a.nbins * a.dr + a.six_sigma;
    const double rwin2 = rmax_win * rmax_win;
    double *qr = s_qr[wave];  // r^2 of the queued pairs (a ring of BQ)
    int *qrow = s_qrow[wave];
    int nqw = 0, qh = 0;  // queued pairs of this wave, first slot of the ring
    for (long long t = blockIdx.x; t < a.ntp; t += gridDim.x) {
        int I, J;
        tri_index(t, a.nt, I, J);
        const int i = I * FTILE + tid;
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
        const int j = J * FTILE + tid;
        if (j < N) {
            jx[tid] = a.xyz[j];
            jx[FTILE + tid] = a.xyz[N + j];
            jx[2 * FTILE + tid] = a.xyz[2 * N + j];
            js[tid] = a.sp[j];
        }
        __syncthreads();
        const int jn = min(FTILE, N - J * FTILE);
        const int jstart = (I == J) ? tid + 1 : 0;
        const int rowbase = si * a.M;
        for (int jj = 0; jj < jn; ++jj) {
            const double r2 = nearest_r2(jx[jj] - xi, jx[FTILE + jj] - yi, jx[2 * FTILE + jj] - zi, a.L);
            const bool in = iv && jj >= jstart && r2 < a.half2 && r2 < rwin2;
            const unsigned long long bal = __ballot(in);
            if (in) {
                const int q = (qh + nqw + __popcll(bal & lt)) & (BQ - 1);
                qr[q] = r2;
                qrow[q] = prow[rowbase + js[jj]];
            }
            nqw += __popcll(bal);
            if (nqw >= 64) {
                __builtin_amdgcn_wave_barrier();
                const int q = (qh + lane) & (BQ - 1);
                const double rq = qr[q];
                const int rowq = qrow[q];
                qh = (qh + 64) & (BQ - 1);
                nqw -= 64;
                __builtin_amdgcn_wave_barrier();
                if (TAB)
                    broad_pair_tab(a, tab, hist + rowq, rq);
                else
                    broad_pair(a, tab, hist + rowq, rq);
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
    if (lane < nqw) {
        const int q = (qh + lane) & (BQ - 1);
        if (TAB)
            broad_pair_tab(a, tab, hist + qrow[q], qr[q]);
        else
            broad_pair(a, tab, hist + qrow[q], qr[q]);
    }
    __syncthreads();
    double *out = a.partial + (size_t)blockIdx.x * nq;
    for (int q = tid; q < nq; q += FTILE) out[q] = (double)hist[q] * 2.3283064365386963e-10;
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
constexpr int BTILE = 256;  // atoms per tile of the backward: four waves
constexpr int BBQ = 128;    // pairs queued per wave

struct BackArgs {
    const float *xyz;
    const uint8_t *sp;
    const double *A;  // [P][nbins]
    int N, M, P, nbins, nt;
    long long ntp;
    double L, invL, half2;  // half2 = (L/2)^2
    double dr, inv_dr, inv_sigma, six_sigma;
    float beta;       // dr / sigma
    float rho_step;   // exp(-beta^2)
    int recur;        // 1: Gaussian density by recurrence along the edges (beta <= 4)
    int kp;           // a pair's scaled term stays below 2^kp, an atom's total below 2^62
    long long *gsum;  // [3][N] gradient in units of 2^-sh, cleared before the launch
    int *shift;       // sh, written by block 0 (INT_MIN: the adjoint is not finite)
};

// Nearest integer of y for |y| < 2^51: adding 1.5 * 2^52 leaves the rounded
// value in the low bits of the FP64 sum.
__device__ __forceinline__ long long nearest_ll(double y)
{
    return __double_as_longlong(y + 6755399441055744.0) - 0x4338000000000000LL;
}

// dL/dr of one pair at distance r (r < L/2) and its gradient on both atoms:
// dL/dr = sum_k A(k) (phi(x_k) - phi(x_{k+1})) / s with x = (e - r)/s, then
// +c d on atom i (LDS row il of the I tile) and -c d on atom j (row jl of
// the J tile), c = (dL/dr) / r and d = x_i - x_j (nearest image, FP64 from
// the tiles' coordinates), each as an integer in units of 1/S.
__device__ __forceinline__ void bwd_pair(const BackArgs &a, const float *dA, int ibase, const double *jx,
                                         unsigned long long *gacc, double S, double r2, int row, int ij)
{
    const double r = nd::sqrt_nr(r2);
    int k0 = (int)floor((r - a.six_sigma) * a.inv_dr);
    int k1 = (int)floor((r + a.six_sigma) * a.inv_dr);
    k0 = max(k0, 0);
    k1 = min(k1, a.nbins - 1);
    const double u = r * a.inv_dr;
    const int kr = (int)u;
    const float f = (float)(u - (double)kr);
    const float beta = a.beta;
    const float *rowp = dA + row;
    const float x0 = ((float)(k0 - kr) - f) * beta;
    float plo = gauss_pdf(x0);
    float dLdr = 0.0f;
    if (a.recur) {
        // phi(x + beta) = phi(x) rho, rho = exp(-beta x - beta^2/2); rho
        // itself steps by the constant factor exp(-beta^2); two bins a trip
        float rho = __builtin_amdgcn_exp2f((x0 + 0.5f * beta) * beta * -1.4426950408889634f);
        const float step = a.rho_step;
        int k = k0;
        for (; k < k1; k += 2) {
            const float A0 = rowp[k], A1 = rowp[k + 1];
            const float p1 = plo * rho;
            rho *= step;
            const float p2 = p1 * rho;
            rho *= step;
            dLdr = fmaf(A0, plo - p1, dLdr);
            dLdr = fmaf(A1, p1 - p2, dLdr);
            plo = p2;
        }
        if (k == k1) dLdr = fmaf(rowp[k], plo - plo * rho, dLdr);
    } else {
        for (int k = k0; k <= k1; ++k) {
            const float phi_hi = gauss_pdf(((float)(k + 1 - kr) - f) * beta);
            dLdr = fmaf(rowp[k], plo - phi_hi, dLdr);
            plo = phi_hi;
        }
    }
    // 1/r from the FP32 reciprocal: relative error ~1e-7, far below the
    // gradient's FP32 pair weights
    const double c = (double)dLdr * a.inv_sigma * (double)__builtin_amdgcn_rcpf((float)r);
    const double cs = c * S;
    const int il = ij & 0xffff, jl = ij >> 16;
    const int i = ibase + il;
    double dx = (double)a.xyz[i] - jx[jl], dy = (double)a.xyz[a.N + i] - jx[BTILE + jl],
           dz = (double)a.xyz[2 * a.N + i] - jx[2 * BTILE + jl];
    dx = fma(-rint(dx * a.invL), a.L, dx);
    dy = fma(-rint(dy * a.invL), a.L, dy);
    dz = fma(-rint(dz * a.invL), a.L, dz);
    const unsigned long long qx = (unsigned long long)nearest_ll(cs * dx);
    const unsigned long long qy = (unsigned long long)nearest_ll(cs * dy);
    const unsigned long long qz = (unsigned long long)nearest_ll(cs * dz);
    __hip_atomic_fetch_add(gacc + il, qx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_add(gacc + BTILE + il, qy, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_add(gacc + 2 * BTILE + il, qz, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_add(gacc + 3 * BTILE + jl, 0ull - qx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_add(gacc + 4 * BTILE + jl, 0ull - qy, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_add(gacc + 5 * BTILE + jl, 0ull - qz, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Each unordered pair once: blocks take tile pairs (I <= J) as the forward
// does, each lane owns atom i of the I tile and tests it against the J
// tile; the pairs inside the window range are queued per wave in LDS and
// evaluated 64 at a time, one per lane.  A pair's gradient goes to both of
// its atoms as integers in units of 1/S, S = 2^sh a power of two chosen from
// max |A| so that no sum can overflow: summed in LDS per tile and added to
// the [3][N] totals with device atomics when the tile pair is done.  Integer
// sums: the result does not depend on the order.
__global__ __launch_bounds__(BTILE) void k_hist_broad_bwd(BackArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned long long *gacc = reinterpret_cast<unsigned long long *>(smem);  // [2][3][BTILE] I tile, J tile
    double *jx = reinterpret_cast<double *>(gacc + 6 * BTILE);               // [3][BTILE]
    int *js = reinterpret_cast<int *>(jx + 3 * BTILE);               // [BTILE]
    int *prow = js + BTILE;                                           // [16]
    float *dA = reinterpret_cast<float *>(prow + 16);                // [P*nbins]
    __shared__ double s_qr[BTILE / 64][BBQ];
    __shared__ int s_qrow[BTILE / 64][BBQ];
    __shared__ int s_qij[BTILE / 64][BBQ];
    __shared__ double s_amax[BTILE / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const unsigned long long lt = (1ull << lane) - 1ull;
    const int nq = a.P * a.nbins;
    // the adjoint in FP32: each pair's dL/dr is a sum of ~10 such terms
    // (relative error ~1e-7 of the sum of their magnitudes); its largest
    // magnitude (infinite if any entry is not finite) sets the scale
    double amax = 0.0;
    for (int q = tid; q < nq; q += BTILE) {
        const double v = a.A[q];
        dA[q] = (float)v;
        amax = fmax(amax, v == v ? fabs(v) : HUGE_VAL);
    }
    for (int o = 32; o > 0; o >>= 1) amax = fmax(amax, __shfl_xor(amax, o));
    if (lane == 0) s_amax[wave] = amax;
    if (tid < a.M * a.M) prow[tid] = nd::pair_index(tid / a.M, tid % a.M, a.M) * a.nbins;
    __syncthreads();
    amax = s_amax[0];
    for (int w = 1; w < BTILE / 64; ++w) amax = fmax(amax, s_amax[w]);
    // |a pair's term| <= |dL/dr| / s <= max|A| 2 phi(0) / s < 2^e
    const double bound = amax * a.inv_sigma;
    const bool finite = bound <= 1.0e300;
    const int e = finite && bound > 0.0 ? ilogb(bound) + 1 : 0;
    const int sh = a.kp - e;
    const double S = ldexp(1.0, sh);
    if (blockIdx.x == 0 && tid == 0) *a.shift = finite ? sh : INT_MIN;
    if (!finite) return;
    const int N = a.N;
    const double rmax_win = (double)a.nbins * a.dr + a.six_sigma;
    const double rwin2 = rmax_win * rmax_win;
    double *qr = s_qr[wave];  // r^2 of the queued pairs
    int *qrow = s_qrow[wave], *qij = s_qij[wave];
    for (long long t = blockIdx.x; t < a.ntp; t += gridDim.x) {
        int I, J;
        tri_index(t, a.nt, I, J);
        const int i = I * BTILE + tid;
        const bool iv = i < N;
        double xi = 0.0, yi = 0.0, zi = 0.0;
        int si = 0;
        if (iv) {
            xi = a.xyz[i];
            yi = a.xyz[N + i];
            zi = a.xyz[2 * N + i];
            si = a.sp[i];
        }
        __syncthreads();  // the previous tile pair's sums are out
        const int j = J * BTILE + tid;
        if (j < N) {
            jx[tid] = a.xyz[j];
            jx[BTILE + tid] = a.xyz[N + j];
            jx[2 * BTILE + tid] = a.xyz[2 * N + j];
            js[tid] = a.sp[j];
        }
        for (int q = tid; q < 6 * BTILE; q += BTILE) gacc[q] = 0ull;
        __syncthreads();
        const int jn = min(BTILE, N - J * BTILE);
        const int rowbase = si * a.M;
        int nqw = 0, qh = 0;  // queued pairs of this wave, first slot of the ring
        // the J tile in blocks of 64, each walked along its diagonals: at
        // step st lane l takes j = jb + (l + st) mod 64, so the pairs of one
        // step have distinct i and distinct j and the sums of a batch of 64
        // queued pairs meet at most two to an address
        for (int jb = 0; jb < jn; jb += 64) {
            for (int st = 0; st < 64; ++st) {
                const int jj = jb + ((lane + st) & 63);
                const double dx = xi - jx[jj], dy = yi - jx[BTILE + jj], dz = zi - jx[2 * BTILE + jj];
                const double r2 = nearest_r2(dx, dy, dz, a.L);
                // coincident atoms (r = 0) have no direction and are left out
                const bool in = iv && jj < jn && (I != J || jj > tid) && r2 < a.half2 && r2 < rwin2 && r2 > 0.0;
                const unsigned long long bal = __ballot(in);
                if (in) {
                    const int q = (qh + nqw + __popcll(bal & lt)) & (BBQ - 1);
                    qr[q] = r2;
                    qrow[q] = prow[rowbase + js[jj]];
                    qij[q] = tid | (jj << 16);
                }
                nqw += __popcll(bal);
                if (nqw >= 64) {
                    __builtin_amdgcn_wave_barrier();
                    const int q = (qh + lane) & (BBQ - 1);
                    const double rq = qr[q];
                    const int rowq = qrow[q], ijq = qij[q];
                    qh = (qh + 64) & (BBQ - 1);
                    nqw -= 64;
                    __builtin_amdgcn_wave_barrier();
                    bwd_pair(a, dA, I * BTILE, jx, gacc, S, rq, rowq, ijq);
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        if (lane < nqw) {
            const int q = (qh + lane) & (BBQ - 1);
            bwd_pair(a, dA, I * BTILE, jx, gacc, S, qr[q], qrow[q], qij[q]);
        }
        __syncthreads();
        unsigned long long *gs = reinterpret_cast<unsigned long long *>(a.gsum);
        if (iv)
            for (int c = 0; c < 3; ++c) atomicAdd(gs + (size_t)c * N + i, gacc[c * BTILE + tid]);
        if (j < N)
            for (int c = 0; c < 3; ++c) atomicAdd(gs + (size_t)c * N + j, gacc[(3 + c) * BTILE + tid]);
    }
}

// Two-word integer totals (hi 2^32 + lo, units of 2^ue) back to FP64 (NaN
// where the table was not finite).
__global__ void k_words_to_f64(const long long *__restrict__ v, long long n, const int *__restrict__ shift,
                               double *__restrict__ out)
{
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int ue = *shift;
    out[q] = ue == INT_MIN ? __builtin_nan("") : ldexp((double)v[q], 32 + ue) + ldexp((double)v[n + q], ue);
}

// The integer totals back to FP64 (NaN where the adjoint was not finite).
__global__ void k_fixed_to_f64(const long long *__restrict__ v, long long n, const int *__restrict__ shift,
                               double *__restrict__ out)
{
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int sh = *shift;
    out[q] = sh == INT_MIN ? __builtin_nan("") : ldexp((double)v[q], -sh);
}

__global__ void k_fill_zero_f64(double *__restrict__ p, long long n)
{
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) p[q] = 0.0;
}

// ---------------------------------------------------------------- forces
constexpr int GTILE = 256;  // atoms per tile of the forces: four waves
constexpr int GQ = 128;     // pairs queued per wave

struct ForceArgs {
    const float *xyz;
    const uint8_t *sp;
    const int32_t *unit_of;
    const float *tab;
    int N, M, P, n_pts, nt;
    long long ntp;
    double L, invL, half2, rc2, inv_h;
    long long *gsum;  // [2][3][N] gradient as two integer words (hi 2^32 + lo) in units of 2^ue
    int *shift;       // ue, written by block 0 (INT_MIN: the table is not finite)
    double *epart;    // [gridDim.x] energy of each block's pairs
};

// y = hi 2^32 + lo with hi, lo integers and 0 <= lo <= 2^32 (|y| < 2^70):
// each word is summed on its own, so no carry passes between them.
__device__ __forceinline__ void split_words(double y, unsigned long long &hi, unsigned long long &lo)
{
    const double h = floor(y * 2.3283064365386963e-10);
    hi = (unsigned long long)nearest_ll(h);
    lo = (unsigned long long)nearest_ll(fma(-h, 4294967296.0, y));
}

// One queued pair within the cutoff: the tabulated U(r) (linear between
// points) into e, and +dU/dr (x_i - x_j)/r on atom i, the negative on atom
// j, as two integer words in units of 1/S.  The displacement is taken again
// in FP64 from the tiles' coordinates.
__device__ __forceinline__ void force_pair(const ForceArgs &a, const float *tab, int ibase, const double *jx,
                                           unsigned long long *gacc, double S, double r2, int row, int ij,
                                           double &e)
{
    const int il = ij & 0xffff, jl = ij >> 16, i = ibase + il;
    double dx = (double)a.xyz[i] - jx[jl], dy = (double)a.xyz[a.N + i] - jx[GTILE + jl],
           dz = (double)a.xyz[2 * a.N + i] - jx[2 * GTILE + jl];
    dx = fma(-rint(dx * a.invL), a.L, dx);
    dy = fma(-rint(dy * a.invL), a.L, dy);
    dz = fma(-rint(dz * a.invL), a.L, dz);
    const double r = sqrt(r2);
    const double t = r * a.inv_h;
    const int i0 = min((int)t, a.n_pts - 2);
    const float *rowp = tab + row;
    const double u0 = rowp[i0], u1 = rowp[i0 + 1];
    const double slope = (u1 - u0) * a.inv_h;
    const double f = t - (double)i0;
    e += u0 + f * (u1 - u0);
    const double cs = slope / r * S;
    const double comp[3] = {cs * dx, cs * dy, cs * dz};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        unsigned long long hi, lo;
        split_words(comp[c], hi, lo);
        __hip_atomic_fetch_add(gacc + c * GTILE + il, hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_fetch_add(gacc + (6 + c) * GTILE + il, lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_fetch_add(gacc + (3 + c) * GTILE + jl, 0ull - hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_fetch_add(gacc + (9 + c) * GTILE + jl, 0ull - lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
}

// Gradient of the tabulated total energy and the energy itself, each
// unordered pair of different units once: tile pairs I <= J as in the
// broadened backward, the J tile walked along its diagonals, the pairs
// within the cutoff queued per wave and evaluated 64 at a time.  Gradient
// terms are integers in units of 2^ue, ue = e - 70 with 2^e above the
// table's steepest step, held as two words (hi 2^32 + lo) summed
// separately: 70 bits of range for the steep short-range end of the table
// and a quantum of 2^-71 of that bound, sums exact and independent of
// order; the energy is summed per lane in queue order, per block, then
// over blocks in block order.
__global__ __launch_bounds__(GTILE) void k_forces(ForceArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned long long *gacc = reinterpret_cast<unsigned long long *>(smem);  // [hi, lo][I, J tile][3][GTILE]
    double *jx = reinterpret_cast<double *>(gacc + 12 * GTILE);               // [3][GTILE]
    int *js = reinterpret_cast<int *>(jx + 3 * GTILE);                       // [GTILE]
    int *ju = js + GTILE;                                                       // [GTILE]
    int *prow = ju + GTILE;                                                     // [16]
    float *tab = reinterpret_cast<float *>(prow + 16);                        // [P][n_pts]
    __shared__ double s_qr[GTILE / 64][GQ];
    __shared__ int s_qrow[GTILE / 64][GQ];
    __shared__ int s_qij[GTILE / 64][GQ];
    __shared__ double s_red[GTILE / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const unsigned long long lt = (1ull << lane) - 1ull;
    // the tables, and their steepest step (infinite if any value is not finite)
    const int ntab = a.P * a.n_pts;
    double smax = 0.0;
    for (int q = tid; q < ntab; q += GTILE) {
        const float v = a.tab[q];
        tab[q] = v;
        if (q % a.n_pts != a.n_pts - 1) {
            const double s = fabs(((double)a.tab[q + 1] - (double)v) * a.inv_h);
            smax = fmax(smax, s == s ? s : HUGE_VAL);
        }
    }
    for (int o = 32; o > 0; o >>= 1) smax = fmax(smax, __shfl_xor(smax, o));
    if (lane == 0) s_red[wave] = smax;
    if (tid < a.M * a.M) prow[tid] = nd::pair_index(tid / a.M, tid % a.M, a.M) * a.n_pts;
    __syncthreads();
    smax = s_red[0];
    for (int w = 1; w < GTILE / 64; ++w) smax = fmax(smax, s_red[w]);
    // |a pair's term| <= |dU/dr| <= smax < 2^e
    const bool finite = smax <= 1.0e300;
    const int e2 = finite && smax > 0.0 ? ilogb(smax) + 1 : 0;
    const int ue = e2 - 70;
    const double S = ldexp(1.0, -ue);
    if (blockIdx.x == 0 && tid == 0) *a.shift = finite ? ue : INT_MIN;
    const int N = a.N;
    double *qr = s_qr[wave];
    int *qrow = s_qrow[wave], *qij = s_qij[wave];
    double e = 0.0;
    for (long long t = finite ? blockIdx.x : a.ntp; t < a.ntp; t += gridDim.x) {
        int I, J;
        tri_index(t, a.nt, I, J);
        const int i = I * GTILE + tid;
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
        __syncthreads();  // the previous tile pair's sums are out
        const int j = J * GTILE + tid;
        if (j < N) {
            jx[tid] = a.xyz[j];
            jx[GTILE + tid] = a.xyz[N + j];
            jx[2 * GTILE + tid] = a.xyz[2 * N + j];
            js[tid] = a.sp[j];
            ju[tid] = a.unit_of[j];
        }
        for (int q = tid; q < 12 * GTILE; q += GTILE) gacc[q] = 0ull;
        __syncthreads();
        const int jn = min(GTILE, N - J * GTILE);
        const int rowbase = si * a.M;
        int nqw = 0, qh = 0;  // queued pairs of this wave, first slot of the ring
        for (int jb = 0; jb < jn; jb += 64) {
            for (int st = 0; st < 64; ++st) {
                const int jj = jb + ((lane + st) & 63);
                const double r2 = nearest_r2(xi - jx[jj], yi - jx[GTILE + jj], zi - jx[2 * GTILE + jj], a.L);
                const bool in = iv && jj < jn && (I != J || jj > tid) && r2 < a.rc2 && r2 > 0.0 && ju[jj] != ui;
                const unsigned long long bal = __ballot(in);
                if (in) {
                    const int q = (qh + nqw + __popcll(bal & lt)) & (GQ - 1);
                    qr[q] = r2;
                    qrow[q] = prow[rowbase + js[jj]];
                    qij[q] = tid | (jj << 16);
                }
                nqw += __popcll(bal);
                if (nqw >= 64) {
                    __builtin_amdgcn_wave_barrier();
                    const int q = (qh + lane) & (GQ - 1);
                    const double rq = qr[q];
                    const int rowq = qrow[q], ijq = qij[q];
                    qh = (qh + 64) & (GQ - 1);
                    nqw -= 64;
                    __builtin_amdgcn_wave_barrier();
                    force_pair(a, tab, I * GTILE, jx, gacc, S, rq, rowq, ijq, e);
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        if (lane < nqw) {
            const int q = (qh + lane) & (GQ - 1);
            force_pair(a, tab, I * GTILE, jx, gacc, S, qr[q], qrow[q], qij[q], e);
        }
        __syncthreads();
        unsigned long long *gs = reinterpret_cast<unsigned long long *>(a.gsum);
        for (int w = 0; w < 2; ++w) {
            unsigned long long *gw = gs + (size_t)w * 3 * N;
            const unsigned long long *aw = gacc + w * 6 * GTILE;
            for (int c = 0; c < 3; ++c) {
                const unsigned long long vi = aw[c * GTILE + tid], vj = aw[(3 + c) * GTILE + tid];
                if (iv && vi) atomicAdd(gw + (size_t)c * N + i, vi);
                if (j < N && vj) atomicAdd(gw + (size_t)c * N + j, vj);
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o);
    __syncthreads();
    if (lane == 0) s_red[wave] = e;
    __syncthreads();
    if (tid == 0) {
        double eb = s_red[0];
        for (int w = 1; w < GTILE / 64; ++w) eb += s_red[w];
        a.epart[blockIdx.x] = finite ? eb : __builtin_nan("");
    }
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

// Mills ratio R(x) = T(x)/phi(x), T the upper Gaussian tail, with its Taylor
// coefficients R', R''/2 and R'''/6 at x = i/32, from R' = xR - 1,
// R'' = (1 + x^2) R - x and R''' = (x^3 + 3x) R - x^2 - 2; computed in FP64
// on the host and kept on each device for the life of the process.
const float4 *mills_table(nd_box *b)
{
    static const float4 *dev_table[64] = {nullptr};
    if (b->device < 0 || b->device >= 64) nd::fail(ND_E_INVALID, "device index out of range");
    if (dev_table[b->device]) return dev_table[b->device];
    std::vector<float4> h(MILLS_N);
    for (int i = 0; i < MILLS_N; ++i) {
        const double x = (double)i / MILLS_PER_UNIT;
        const double T = 0.5 * std::erfc(x / std::sqrt(2.0));
        const double phi = std::exp(-0.5 * x * x) / std::sqrt(2.0 * M_PI);
        const double R = T / phi;
        const double R1 = x * R - 1.0;
        const double R2 = (1.0 + x * x) * R - x;
        const double R3 = (x * x * x + 3.0 * x) * R - x * x - 2.0;
        h[i] = make_float4((float)R, (float)R1, (float)(R2 / 2.0), (float)(R3 / 6.0));
    }
    float4 *d = static_cast<float4 *>(nd::dmalloc(sizeof(float4) * MILLS_N));
    ND_HIP(hipMemcpy(d, h.data(), sizeof(float4) * MILLS_N, hipMemcpyHostToDevice));
    dev_table[b->device] = d;
    return d;
}

// Mass of [b, a] under the unit Gaussian, from the tails so that neither
// side cancels.
double gauss_mass(double b, double a)
{
    auto Q = [](double x) { return 0.5 * std::erfc(x / std::sqrt(2.0)); };  // upper tail
    if (b >= 0.0) return Q(b) - Q(a);
    if (a <= 0.0) return Q(-a) - Q(-b);
    return 1.0 - Q(a) - Q(-b);
}

// The bin-mass table for beta = dr/sigma and s = 6 sigma/dr (FP64 on the
// host, kept per box until the parameters change): for bin offset m and
// piece centre fc, w(f) = Phi((m+1-f) beta) - Phi((m-f) beta) and its
// derivatives in f, w' = -beta [phi(a) - phi(b)] and w'' = beta^2 [phi'(a) -
// phi'(b)], with a = (m+1-fc) beta, b = (m-fc) beta, phi' = -x phi.  The
// cubic term left out, w''' d^3 / 6 with |d| <= 1/128 and |w'''| <= 0.8
// beta^3, is odd in d (no mean over a piece) and at most 6.4e-8 beta^3 of a
// pair's mass in a bin; the table is taken for beta <= 2 (5e-7).  Returns
// false for sharper windows or when the table would not fit.
bool bin_mass_table(nd_box *b, double dr, double sigma, BroadArgs &a)
{
    const double beta = dr / sigma, s = 6.0 * sigma / dr;
    if (beta > 2.0) return false;
    const int m0 = (int)std::floor(-s) - 1, m1 = (int)std::ceil(s) + 1;
    const int nm = m1 - m0 + 1;
    const size_t bytes = sizeof(float4) * (size_t)nm * WT_NP;
    if (bytes > (size_t)WT_MAX_BYTES) return false;
    if (!(b->bt_dev && b->bt_beta == beta && b->bt_s == s)) {
        std::vector<float4> h((size_t)nm * WT_NP);
        const double c = 1.0 / std::sqrt(2.0 * M_PI);
        auto phi = [c](double x) { return c * std::exp(-0.5 * x * x); };
        for (int mi = 0; mi < nm; ++mi) {
            const int m = m0 + mi;
            for (int p = 0; p < WT_NP; ++p) {
                const double fc = (p + 0.5) / WT_NP;
                const double xa = (m + 1 - fc) * beta, xb = (m - fc) * beta;
                const double pa = phi(xa), pb = phi(xb);
                const double w0 = gauss_mass(xb, xa);
                const double w1 = -beta * (pa - pb);
                const double w2 = beta * beta * (-xa * pa + xb * pb);
                const float hi = (float)w0;
                h[(size_t)mi * WT_NP + p] = make_float4(hi, (float)(w0 - (double)hi), (float)w1, (float)(w2 / 2.0));
            }
        }
        ND_HIP(hipStreamSynchronize(b->stream));
        nd::dfree(b->bt_dev);
        b->bt_dev = nd::dmalloc(bytes);
        ND_HIP(hipMemcpy(b->bt_dev, h.data(), bytes, hipMemcpyHostToDevice));
        b->bt_beta = beta;
        b->bt_s = s;
    }
    a.wt = static_cast<const float4 *>(b->bt_dev);
    a.wt_m0 = m0;
    a.wt_nm = nm;
    return true;
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
    a.nt = (b->N + FTILE - 1) / FTILE;
    a.ntp = (long long)a.nt * (a.nt + 1) / 2;
    a.L = b->L;
    a.invL = 1.0 / b->L;
    a.half2 = 0.25 * b->L * b->L;
    a.dr = dr;
    a.inv_dr = 1.0 / dr;
    a.six_sigma = 6.0 * sigma;
    a.beta = (float)(dr / sigma);
    a.mills = mills_table(b);
    a.wt = nullptr;
    a.wt_m0 = 0;
    a.wt_nm = 0;
    const bool tab = bin_mass_table(b, dr, sigma, a);
    const int nq = a.P * nbins;
    const size_t lds_tab = sizeof(float4) * (tab ? (size_t)a.wt_nm * WT_NP : (size_t)MILLS_N);
    size_t lds = sizeof(double) * ((size_t)nq + 3 * FTILE) + lds_tab + sizeof(int) * (FTILE + 16);
    const size_t lds_queue = (sizeof(double) + sizeof(int)) * BQ * (FTILE / 64);  // static, in the kernel
    if (lds + lds_queue > 160 * 1024) fail(ND_E_UNSUPPORTED, "broadened histogram does not fit in LDS");
    int per_cu = (int)std::max<size_t>(1, std::min<size_t>(4, (160 * 1024) / (lds + lds_queue + 1024)));
    long long G = (long long)cu_count(b->device) * per_cu;
    if (G > a.ntp) G = a.ntp;
    // a block's integer sum of weights < 1 per pair stays below 2^64
    if ((double)((a.ntp + G - 1) / G) * FTILE * FTILE >= 4294967295.0)
        fail(ND_E_UNSUPPORTED, "box too large for the broadened histogram's block sums");
    a.partial = static_cast<double *>(workspace(b, sizeof(double) * (size_t)G * nq));
    {
        ProfScope ps(b, ND_PROF_HIST_BROAD);
        if (tab)
            hipLaunchKernelGGL(k_hist_broad<true>, dim3((unsigned)G), dim3(FTILE), lds, b->stream, a);
        else
            hipLaunchKernelGGL(k_hist_broad<false>, dim3((unsigned)G), dim3(FTILE), lds, b->stream, a);
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
    a.nt = (b->N + BTILE - 1) / BTILE;
    a.ntp = (long long)a.nt * (a.nt + 1) / 2;
    a.L = b->L;
    a.invL = 1.0 / b->L;
    a.half2 = 0.25 * b->L * b->L;
    a.dr = dr;
    a.inv_dr = 1.0 / dr;
    a.inv_sigma = 1.0 / sigma;
    a.six_sigma = 6.0 * sigma;
    a.beta = (float)(dr / sigma);
    a.rho_step = (float)std::exp(-(dr / sigma) * (dr / sigma));
    // the first step factor exp(beta (6 + beta/2 + 1)) stays far inside FP32 range
    a.recur = dr / sigma <= 4.0 ? 1 : 0;
    // a pair's term below 2^kp, so that the N - 1 terms of an atom stay
    // below 2^62 and nearest_ll stays exact
    int lg = 0;
    while ((1LL << lg) < (long long)b->N) ++lg;
    a.kp = std::min(51, 62 - lg);
    // summed in the box's workspace, then converted into the caller's array
    char *ws = static_cast<char *>(workspace(b, sizeof(long long) * 3 * (size_t)b->N + 256));
    a.gsum = reinterpret_cast<long long *>(ws);
    a.shift = reinterpret_cast<int *>(ws + sizeof(long long) * 3 * (size_t)b->N);
    const size_t lds = sizeof(double) * 9 * BTILE + sizeof(int) * (BTILE + 16) + sizeof(float) * (size_t)b->P * nbins;
    const size_t lds_queue = (sizeof(double) + 2 * sizeof(int)) * BBQ * (BTILE / 64) +
                             sizeof(double) * (BTILE / 64);  // static
    if (lds + lds_queue > 160 * 1024) fail(ND_E_UNSUPPORTED, "adjoint table does not fit in LDS");
    const int per_cu = (int)std::max<size_t>(1, std::min<size_t>(4, (160 * 1024) / (lds + lds_queue + 1024)));
    long long G = (long long)cu_count(b->device) * per_cu;
    if (G > a.ntp) G = a.ntp;
    const long long n = 3LL * b->N;
    hipLaunchKernelGGL(k_fill_zero_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, b->stream,
                       reinterpret_cast<double *>(a.gsum), n);
    ND_HIP(hipGetLastError());
    {
        ProfScope ps(b, ND_PROF_HIST_BROAD_BWD);
        hipLaunchKernelGGL(k_hist_broad_bwd, dim3((unsigned)G), dim3(BTILE), lds, b->stream, a);
        ND_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_fixed_to_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, b->stream, a.gsum, n, a.shift,
                       d_grad);
    ND_HIP(hipGetLastError());
}

// Scratch bytes of the forces for N atoms and a grid of G blocks: the two
// integer words of the [3][N] gradient sums, the blocks' energies, the shift.
size_t forces_scratch_bytes(int N, long long G)
{
    return sizeof(long long) * 2 * 3 * (size_t)N + sizeof(double) * (size_t)G + 256;
}

// Grid of the forces kernel and its LDS bytes for box b.
static long long forces_grid(const nd_box *b, size_t &lds_total)
{
    const int P = b->P;
    const size_t lds = sizeof(unsigned long long) * 12 * GTILE + sizeof(double) * 3 * GTILE +
                       sizeof(int) * (2 * GTILE + 16) + sizeof(float) * (size_t)P * b->n_pts;
    const size_t lds_queue = (sizeof(double) + 2 * sizeof(int)) * GQ * (GTILE / 64) + sizeof(double) * (GTILE / 64);
    if (lds + lds_queue > 160 * 1024) fail(ND_E_UNSUPPORTED, "potential table does not fit in LDS");
    const int per_cu = (int)std::max<size_t>(1, std::min<size_t>(8, (160 * 1024) / (lds + lds_queue + 1024)));
    const int nt = (b->N + GTILE - 1) / GTILE;
    const long long ntp = (long long)nt * (nt + 1) / 2;
    long long G = (long long)cu_count(b->device) * per_cu;
    if (G > ntp) G = ntp;
    lds_total = lds;
    return G;
}

void launch_forces(nd_box *b, double *d_grad, double *d_E)
{
    size_t lds = 0;
    const long long G = forces_grid(b, lds);
    char *ws = static_cast<char *>(workspace(b, forces_scratch_bytes(b->N, G)));
    launch_forces_in(b, d_grad, d_E, ws, G, true);
}

// The forces with a caller-provided scratch of forces_scratch_bytes(N, G)
// bytes (G at most max_grid); profiling events only when `prof`.
void launch_forces_in(nd_box *b, double *d_grad, double *d_E, char *ws, long long max_grid, bool prof)
{
    ForceArgs a;
    a.xyz = b->xyz;
    a.sp = b->species;
    a.unit_of = b->unit_of;
    a.tab = b->tab;
    a.N = b->N;
    a.M = b->M;
    a.P = b->P;
    a.n_pts = b->n_pts;
    a.nt = (b->N + GTILE - 1) / GTILE;
    a.ntp = (long long)a.nt * (a.nt + 1) / 2;
    a.L = b->L;
    a.invL = 1.0 / b->L;
    a.half2 = 0.25 * b->L * b->L;
    a.rc2 = b->rc * b->rc;
    a.inv_h = 1.0 / b->h;
    // a word's sum over an atom's N - 1 pairs: hi below 2^38 N, lo below 2^32 N
    if (b->N > (1 << 24)) fail(ND_E_UNSUPPORTED, "too many atoms for the forces' gradient sums");
    size_t lds = 0;
    long long G = forces_grid(b, lds);
    if (G > max_grid) G = max_grid;  // a persistent grid: fewer blocks take more tile pairs each
    const long long n = 3LL * b->N;
    a.gsum = reinterpret_cast<long long *>(ws);
    a.epart = reinterpret_cast<double *>(ws + sizeof(long long) * 2 * (size_t)n);
    a.shift = reinterpret_cast<int *>(ws + sizeof(long long) * 2 * (size_t)n + sizeof(double) * (size_t)G);
    hipLaunchKernelGGL(k_fill_zero_f64, dim3((unsigned)((2 * n + 255) / 256)), dim3(256), 0, b->stream,
                       reinterpret_cast<double *>(a.gsum), 2 * n);
    ND_HIP(hipGetLastError());
    {
        ProfScope ps(b, prof ? ND_PROF_FORCES : -1);
        hipLaunchKernelGGL(k_forces, dim3((unsigned)G), dim3(GTILE), lds, b->stream, a);
        ND_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_words_to_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, b->stream, a.gsum, n, a.shift,
                       d_grad);
    ND_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sum_serial, dim3(1), dim3(256), 0, b->stream, a.epart, (int)G, d_E);
    ND_HIP(hipGetLastError());
    // flexible molecules: the intramolecular harmonic terms
    launch_intra_forces_add(b, d_grad);
    launch_intra_energy_add(b, d_E, nullptr);
}

}  // namespace nd

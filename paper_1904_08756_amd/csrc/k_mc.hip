// Metropolis Monte Carlo over rigid units (Sec. "Algorithmic Flow" III)
// with the per-trial energy change computed as a minimum-image pair sum
// against every atom (Sec. "Acceleration method": the per-step work that is
// proportional to N).
//
// Trials are processed in batches of K consecutive trials.  In sequential
// order consecutive trials move distinct units, and a trial's proposal
// depends only on (seed, trial) and its own unit's positions, so the K
// proposals and their energy changes dE0_k against the configuration at the
// start of the batch can be computed together.  The sequential chain is then
// recovered exactly: if an earlier trial m of the batch was accepted, trial k
// sees m at its new position, which changes k's energy change by
//   C_km = [U(k',m') - U(k,m')] - [U(k',m) - U(k,m)]
// (primes = proposed positions, sums over the atom pairs of the two units).
// Only unit pairs whose bounding spheres come within the cutoff have
// C_km != 0.  The decision kernel resolves acc_k = metropolis(dE0_k +
// sum_{m<k} acc_m C_km) for the whole batch by fixed-point iteration on this
// lower-triangular system, which reaches the sequential answer because
// trial k only depends on trials before it.
//
// Kernels per batch: propose -> scan (the hot pair sum) -> corrections ->
// decide (+ commit).  Pair terms are FP32 (fractional coordinates, table
// interpolation); every sum is FP64.
#include "nd_internal.h"
#include "nd_pair.h"

#include <algorithm>
#include <cmath>

namespace {

using nd::PairCtx;

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_JPT = 8;                         // j atoms held per thread
constexpr int SCAN_JB = SCAN_THREADS * SCAN_JPT;    // atoms per j-block
constexpr int MAX_TG = 64;                          // trials per scan block
constexpr int DECIDE_THREADS = 1024;
constexpr int KMAX = 2048;                          // trials per batch
constexpr double TWO_PI = 6.283185307179586;

// ---------------------------------------------------------------- RNG
// SplitMix64 (Steele, Lea, Flood 2014): output i of the generator seeded
// with s is the 64-bit finalizer applied to s + (i + 1) * gamma.  Draw d of
// trial t is output 16 t + d, mapped to [0, 1) with 53 bits.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (i + 1ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double draw(uint64_t seed, uint64_t t, int d)
{
    return (double)(splitmix64(seed, 16ull * t + (uint64_t)d) >> 11) * (1.0 / 9007199254740992.0);
}

// Wrap into [0, L) and round to float32; a value that rounds to L is 0.
__device__ __forceinline__ float wrap_round(double x, double L)
{
    const double w = x - L * floor(x / L);
    float f = (float)w;
    if ((double)f >= L || f < 0.0f) f = 0.0f;
    return f;
}

__device__ __forceinline__ double min_image_cmp(double d, double L)
{
    const double half = 0.5 * L;
    if (d > half) return d - L;
    if (d < -half) return d + L;
    return d;
}

struct ProposeArgs {
    const float *xyz;
    const float4 *pos4;
    const float4 *poslo;
    const int32_t *uoff;
    int N, n_units;
    double L, invL, max_disp, max_rot;
    uint64_t seed, t0;
    int kb;
    nd::Trial *trials;
};

// One thread per trial: translation tau = d (2u - 1) per axis; for units of
// several atoms a rotation by theta = r (2u_5 - 1) about the axis
// (sqrt(1-z^2) cos phi, sqrt(1-z^2) sin phi, z), z = 2u_3 - 1, phi = 2 pi u_4,
// through the unweighted centroid of the unit unwrapped around its first
// atom (Rodrigues' formula).  FP64, then wrapped and rounded to float32.
__global__ __launch_bounds__(64) void k_mc_propose(ProposeArgs a)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.kb) return;
    const uint64_t t = a.t0 + (uint64_t)k;
    const int u = (int)(t % (uint64_t)a.n_units);
    const int a0 = a.uoff[u];
    const int na = a.uoff[u + 1] - a0;
    const int N = a.N;
    const double L = a.L;

    double tau[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) tau[c] = a.max_disp * (2.0 * draw(a.seed, t, c) - 1.0);

    nd::Trial T;
    T.unit = u;
    T.a0 = a0;
    T.na = na;
    T.pad = 0;
    T.u_acc = draw(a.seed, t, 6);

    float nx[ND_MAX_UNIT_ATOMS][3];
    if (na == 1) {
#pragma unroll
        for (int c = 0; c < 3; ++c) nx[0][c] = wrap_round((double)a.xyz[c * N + a0] + tau[c], L);
    } else {
        double p[ND_MAX_UNIT_ATOMS][3];
        double cen[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double x0 = (double)a.xyz[c * N + a0];
            double s = 0.0;
#pragma unroll
            for (int at = 0; at < ND_MAX_UNIT_ATOMS; ++at) {
                if (at < na) {
                    p[at][c] = x0 + min_image_cmp((double)a.xyz[c * N + a0 + at] - x0, L);
                    s += p[at][c];
                }
            }
            cen[c] = s / (double)na;
        }
        const double zc = 2.0 * draw(a.seed, t, 3) - 1.0;
        const double phi = TWO_PI * draw(a.seed, t, 4);
        const double sr = sqrt(1.0 - zc * zc);
        const double n0 = sr * cos(phi), n1 = sr * sin(phi), n2 = zc;
        const double th = a.max_rot * (2.0 * draw(a.seed, t, 5) - 1.0);
        const double ct = cos(th), st = sin(th), omc = 1.0 - ct;
#pragma unroll
        for (int at = 0; at < ND_MAX_UNIT_ATOMS; ++at) {
            if (at < na) {
                const double v0 = p[at][0] - cen[0], v1 = p[at][1] - cen[1], v2 = p[at][2] - cen[2];
                const double c0 = n1 * v2 - n2 * v1, c1 = n2 * v0 - n0 * v2, c2 = n0 * v1 - n1 * v0;
                const double dot = n0 * v0 + n1 * v1 + n2 * v2;
                const double kk = dot * omc;
                const double w0 = v0 * ct + c0 * st + n0 * kk;
                const double w1 = v1 * ct + c1 * st + n1 * kk;
                const double w2 = v2 * ct + c2 * st + n2 * kk;
                nx[at][0] = wrap_round(cen[0] + w0 + tau[0], L);
                nx[at][1] = wrap_round(cen[1] + w1 + tau[1], L);
                nx[at][2] = wrap_round(cen[2] + w2 + tau[2], L);
            }
        }
    }

    // fractional positions (hi + lo) and the bounding sphere of old + new atoms
    const float4 ref = a.pos4[a0];
    float sx = 0.f, sy = 0.f, sz = 0.f;
#pragma unroll
    for (int at = 0; at < ND_MAX_UNIT_ATOMS; ++at) {
        if (at < na) {
            const float4 o = a.pos4[a0 + at];
            const double fx = (double)nx[at][0] * a.invL, fy = (double)nx[at][1] * a.invL,
                         fz = (double)nx[at][2] * a.invL;
            float4 q, ql;
            q.x = (float)fx;
            q.y = (float)fy;
            q.z = (float)fz;
            q.w = o.w;
            ql.x = (float)(fx - (double)q.x);
            ql.y = (float)(fy - (double)q.y);
            ql.z = (float)(fz - (double)q.z);
            ql.w = 0.0f;
            T.old_hi[at] = o;
            T.old_lo[at] = a.poslo[a0 + at];
            T.new_hi[at] = q;
            T.new_lo[at] = ql;
            T.new_x[at][0] = nx[at][0];
            T.new_x[at][1] = nx[at][1];
            T.new_x[at][2] = nx[at][2];
            float d;
            d = o.x - ref.x; sx += d - rintf(d);
            d = o.y - ref.y; sy += d - rintf(d);
            d = o.z - ref.z; sz += d - rintf(d);
            d = q.x - ref.x; sx += d - rintf(d);
            d = q.y - ref.y; sy += d - rintf(d);
            d = q.z - ref.z; sz += d - rintf(d);
        } else {
            const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
            T.old_hi[at] = zero;
            T.old_lo[at] = zero;
            T.new_hi[at] = zero;
            T.new_lo[at] = zero;
            T.new_x[at][0] = T.new_x[at][1] = T.new_x[at][2] = 0.f;
        }
    }
    const float inv2n = 1.0f / (float)(2 * na);
    const float cx = ref.x + sx * inv2n, cy = ref.y + sy * inv2n, cz = ref.z + sz * inv2n;
    float r2max = 0.f;
#pragma unroll
    for (int at = 0; at < ND_MAX_UNIT_ATOMS; ++at) {
        if (at < na) {
            float dx = T.old_hi[at].x - cx, dy = T.old_hi[at].y - cy, dz = T.old_hi[at].z - cz;
            dx -= rintf(dx); dy -= rintf(dy); dz -= rintf(dz);
            r2max = fmaxf(r2max, dx * dx + dy * dy + dz * dz);
            dx = T.new_hi[at].x - cx; dy = T.new_hi[at].y - cy; dz = T.new_hi[at].z - cz;
            dx -= rintf(dx); dy -= rintf(dy); dz -= rintf(dz);
            r2max = fmaxf(r2max, dx * dx + dy * dy + dz * dz);
        }
    }
    T.cen[0] = cx;
    T.cen[1] = cy;
    T.cen[2] = cz;
    T.rad = sqrtf(r2max) * 1.0001f + 2e-6f;
    a.trials[k] = T;
}

struct ScanArgs {
    const float4 *pos4;
    const float4 *poslo;
    const float *tab;
    const nd::Trial *trials;
    int N, M, n_pts, kb, tg, kcap;
    float rcf2_filter;
    double rcf2, tscale;
    double *partial;  // [n_jb][2][kcap]
};

template <int MAXNU, bool EXCL>
__device__ __forceinline__ void scan_trial(const PairCtx &c, const nd::Trial *__restrict__ T, int na,
                                           const float4 (&pj)[SCAN_JPT], const float4 (&pl)[SCAN_JPT],
                                           unsigned exmask, double &e, double &s)
{
#pragma unroll
    for (int at = 0; at < MAXNU; ++at) {
        if (at < na) {
            const float4 po = T->old_hi[at], pol = T->old_lo[at];
            const float4 pn = T->new_hi[at], pnl = T->new_lo[at];
            const double ox = (double)po.x + (double)pol.x, oy = (double)po.y + (double)pol.y,
                         oz = (double)po.z + (double)pol.z;
            const double nx = (double)pn.x + (double)pnl.x, ny = (double)pn.y + (double)pnl.y,
                         nz = (double)pn.z + (double)pnl.z;
            const int rb = __float_as_int(po.w) * c.M;
#pragma unroll
            for (int m = 0; m < SCAN_JPT; ++m) {
                if (EXCL && ((exmask >> m) & 1u)) continue;
                float u;
                if (nd::pair_u(c, pn, nx, ny, nz, rb, pj[m], pl[m], u)) {
                    e += (double)u;
                    s += (double)fabsf(u);
                }
                if (nd::pair_u(c, po, ox, oy, oz, rb, pj[m], pl[m], u)) {
                    e -= (double)u;
                    s += (double)fabsf(u);
                }
            }
        }
    }
}

// grid (n_jb, n_groups): block (jb, g) sums the pair terms of trials
// g*tg .. g*tg+tg-1 against atoms jb*SCAN_JB .. +SCAN_JB (SCAN_JPT per thread,
// in registers), tables in LDS, one FP64 wave reduction per trial.
template <int MAXNU>
__global__ __launch_bounds__(SCAN_THREADS) void k_mc_scan(ScanArgs a)
{
    extern __shared__ float s_tab[];  // [P][n_pts]
    __shared__ int s_prow[16];
    __shared__ double s_red[2][SCAN_THREADS / 64][MAX_TG];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int P = a.M * (a.M + 1) / 2;
    for (int q = tid; q < P * a.n_pts; q += SCAN_THREADS) s_tab[q] = a.tab[q];
    if (tid < a.M * a.M) s_prow[tid] = nd::pair_index(tid / a.M, tid % a.M, a.M) * a.n_pts;

    const int jstart = blockIdx.x * SCAN_JB;
    float4 pj[SCAN_JPT], pl[SCAN_JPT];
    const float qnan = __int_as_float(0x7fc00000);
#pragma unroll
    for (int m = 0; m < SCAN_JPT; ++m) {
        const int j = jstart + m * SCAN_THREADS + tid;
        pj[m] = (j < a.N) ? a.pos4[j] : make_float4(qnan, qnan, qnan, 0.f);
        pl[m] = (j < a.N) ? a.poslo[j] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    __syncthreads();

    PairCtx c{s_tab, s_prow, a.M, a.n_pts, a.rcf2_filter, a.rcf2, a.tscale};
    const int k0 = blockIdx.y * a.tg;
    const int k1 = min(a.kb, k0 + a.tg);
    for (int k = k0; k < k1; ++k) {
        const nd::Trial *T = a.trials + k;
        const int ta0 = T->a0, tna = T->na;
        double e = 0.0, s = 0.0;
        const bool own = (ta0 < jstart + SCAN_JB) && (ta0 + tna > jstart);
        if (!own) {
            scan_trial<MAXNU, false>(c, T, tna, pj, pl, 0u, e, s);
        } else {
            unsigned ex = 0u;
#pragma unroll
            for (int m = 0; m < SCAN_JPT; ++m) {
                const int j = jstart + m * SCAN_THREADS + tid;
                if ((unsigned)(j - ta0) < (unsigned)tna) ex |= 1u << m;
            }
            scan_trial<MAXNU, true>(c, T, tna, pj, pl, ex, e, s);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            e += __shfl_xor(e, o);
            s += __shfl_xor(s, o);
        }
        if (lane == 0) {
            s_red[0][wave][k - k0] = e;
            s_red[1][wave][k - k0] = s;
        }
    }
    __syncthreads();
    for (int q = tid; q < k1 - k0; q += SCAN_THREADS) {
        double e = 0.0, s = 0.0;
#pragma unroll
        for (int w = 0; w < SCAN_THREADS / 64; ++w) {
            e += s_red[0][w][q];
            s += s_red[1][w][q];
        }
        a.partial[((size_t)blockIdx.x * 2 + 0) * a.kcap + k0 + q] = e;
        a.partial[((size_t)blockIdx.x * 2 + 1) * a.kcap + k0 + q] = s;
    }
}

// ---------------------------------------------------------------- corrections
struct CorrArgs {
    const float *tab;
    const nd::Trial *trials;
    int M, n_pts, kb;
    float rcf, rcf2_filter;
    double rcf2, tscale;
    int32_t *corr_n, *corr_off, *pool_m;
    double *pool_c, *pool_s;
    long long *pool_fill;
};

__device__ __forceinline__ bool spheres_meet(const nd::Trial *A, const nd::Trial *B, float rcf)
{
    float dx = B->cen[0] - A->cen[0], dy = B->cen[1] - A->cen[1], dz = B->cen[2] - A->cen[2];
    dx -= rintf(dx);
    dy -= rintf(dy);
    dz -= rintf(dz);
    const float lim = rcf + A->rad + B->rad;
    return dx * dx + dy * dy + dz * dz < lim * lim;
}

// One wave per trial k: entries (m, C_km, S_km) for every earlier trial m of
// the batch whose unit can interact with k's, in increasing m.
template <int MAXNU>
__global__ __launch_bounds__(64) void k_mc_corr(CorrArgs a)
{
    __shared__ int s_prow[16];
    const int k = blockIdx.x, lane = threadIdx.x;
    if (lane < a.M * a.M) s_prow[lane] = nd::pair_index(lane / a.M, lane % a.M, a.M) * a.n_pts;
    __syncthreads();
    const nd::Trial *Tk = a.trials + k;
    // pass 1: count
    int cnt = 0;
    for (int m0 = 0; m0 < k; m0 += 64) {
        const int m = m0 + lane;
        const bool hit = (m < k) && spheres_meet(Tk, a.trials + m, a.rcf);
        cnt += __popcll(__ballot(hit));
    }
    int off = 0;
    if (lane == 0 && cnt > 0) off = (int)atomicAdd(reinterpret_cast<unsigned long long *>(a.pool_fill),
                                                   (unsigned long long)cnt);
    off = __shfl(off, 0);
    if (lane == 0) {
        a.corr_n[k] = cnt;
        a.corr_off[k] = off;
    }
    if (cnt == 0) return;
    // pass 2: exact corrections, written in m order
    PairCtx c{a.tab, s_prow, a.M, a.n_pts, a.rcf2_filter, a.rcf2, a.tscale};
    const int nak = Tk->na;
    int base = off;
    for (int m0 = 0; m0 < k; m0 += 64) {
        const int m = m0 + lane;
        const bool hit = (m < k) && spheres_meet(Tk, a.trials + m, a.rcf);
        const unsigned long long bal = __ballot(hit);
        if (hit) {
            const nd::Trial *Tm = a.trials + m;
            const int nam = Tm->na;
            double C = 0.0, S = 0.0;
#pragma unroll
            for (int x = 0; x < MAXNU; ++x) {
                if (x < nak) {
                    const float4 ko = Tk->old_hi[x], kol = Tk->old_lo[x];
                    const float4 kn = Tk->new_hi[x], knl = Tk->new_lo[x];
                    const double kox = (double)ko.x + (double)kol.x, koy = (double)ko.y + (double)kol.y,
                                 koz = (double)ko.z + (double)kol.z;
                    const double knx = (double)kn.x + (double)knl.x, kny = (double)kn.y + (double)knl.y,
                                 knz = (double)kn.z + (double)knl.z;
                    const int rb = __float_as_int(ko.w) * a.M;
#pragma unroll
                    for (int y = 0; y < MAXNU; ++y) {
                        if (y < nam) {
                            const float4 mo = Tm->old_hi[y], mol = Tm->old_lo[y];
                            const float4 mn = Tm->new_hi[y], mnl = Tm->new_lo[y];
                            float u;
                            if (nd::pair_u(c, kn, knx, kny, knz, rb, mn, mnl, u)) { C += (double)u; S += (double)fabsf(u); }
                            if (nd::pair_u(c, ko, kox, koy, koz, rb, mn, mnl, u)) { C -= (double)u; S += (double)fabsf(u); }
                            if (nd::pair_u(c, kn, knx, kny, knz, rb, mo, mol, u)) { C -= (double)u; S += (double)fabsf(u); }
                            if (nd::pair_u(c, ko, kox, koy, koz, rb, mo, mol, u)) { C += (double)u; S += (double)fabsf(u); }
                        }
                    }
                }
            }
            const int rank = __popcll(bal & ((1ull << lane) - 1ull));
            a.pool_m[base + rank] = m;
            a.pool_c[base + rank] = C;
            a.pool_s[base + rank] = S;
        }
        base += __popcll(bal);
    }
}

// ---------------------------------------------------------------- decide
struct DecideArgs {
    float *xyz;
    float4 *pos4;
    float4 *poslo;
    double *E;
    const nd::Trial *trials;
    const double *partial;
    const int32_t *corr_n, *corr_off, *pool_m;
    const double *pool_c, *pool_s;
    int N, kb, n_jb, kcap;
    double kT, tie_rel;
    long long *counters;  // [0] accepted, [1] near ties, [2] pool fill (reset here)
    double *dsum;
    double *tr_dE, *tr_sabs;
    uint8_t *tr_acc;
    int32_t *tr_unit;
};

__device__ __forceinline__ bool metropolis(double dE, double u, double kT)
{
    return (dE <= 0.0) || (u < exp(-dE / kT));
}

__global__ __launch_bounds__(DECIDE_THREADS) void k_mc_decide(DecideArgs a)
{
    __shared__ double s_dE[KMAX];
    __shared__ double s_S[KMAX];
    __shared__ unsigned char s_acc[KMAX];
    __shared__ int s_changed;
    __shared__ double s_red_d[DECIDE_THREADS / 64];
    __shared__ long long s_red_a[DECIDE_THREADS / 64], s_red_t[DECIDE_THREADS / 64];
    const int tid = threadIdx.x;
    const int kb = a.kb;

    for (int k = tid; k < kb; k += DECIDE_THREADS) {
        double e = 0.0, s = 0.0;
        for (int jb = 0; jb < a.n_jb; ++jb) {
            e += a.partial[((size_t)jb * 2 + 0) * a.kcap + k];
            s += a.partial[((size_t)jb * 2 + 1) * a.kcap + k];
        }
        s_dE[k] = e;
        s_S[k] = s;
        s_acc[k] = metropolis(e, a.trials[k].u_acc, a.kT) ? 1 : 0;
    }
    __syncthreads();

    // fixed point of acc_k = metropolis(dE0_k + sum_{m<k} acc_m C_km)
    for (int it = 0; it <= kb + 1; ++it) {
        if (tid == 0) s_changed = 0;
        __syncthreads();
        for (int k = tid; k < kb; k += DECIDE_THREADS) {
            const int n = a.corr_n[k];
            if (n == 0) continue;
            const int off = a.corr_off[k];
            double e = s_dE[k];
            for (int i = 0; i < n; ++i)
                if (s_acc[a.pool_m[off + i]]) e += a.pool_c[off + i];
            const unsigned char acc = metropolis(e, a.trials[k].u_acc, a.kT) ? 1 : 0;
            if (acc != s_acc[k]) {
                s_acc[k] = acc;
                s_changed = 1;
            }
        }
        __syncthreads();
        const int ch = s_changed;
        __syncthreads();
        if (!ch) break;
    }

    // finalize: energies, ties, commit, trace
    double dsum = 0.0;
    long long nacc = 0, ntie = 0;
    for (int k = tid; k < kb; k += DECIDE_THREADS) {
        const int n = a.corr_n[k];
        const int off = a.corr_off[k];
        double e = s_dE[k], S = s_S[k];
        for (int i = 0; i < n; ++i)
            if (s_acc[a.pool_m[off + i]]) {
                e += a.pool_c[off + i];
                S += a.pool_s[off + i];
            }
        const nd::Trial &T = a.trials[k];
        const bool acc = s_acc[k] != 0;
        const double u = T.u_acc;
        if (u > 0.0 && fabs(log(u) + e / a.kT) < a.tie_rel * S / a.kT) ++ntie;
        if (acc) {
            ++nacc;
            dsum += e;
            for (int at = 0; at < T.na; ++at) {
                const int i = T.a0 + at;
                a.xyz[i] = T.new_x[at][0];
                a.xyz[a.N + i] = T.new_x[at][1];
                a.xyz[2 * a.N + i] = T.new_x[at][2];
                a.pos4[i] = T.new_hi[at];
                a.poslo[i] = T.new_lo[at];
            }
        }
        if (a.tr_dE) a.tr_dE[k] = e;
        if (a.tr_sabs) a.tr_sabs[k] = S;
        if (a.tr_acc) a.tr_acc[k] = acc ? 1 : 0;
        if (a.tr_unit) a.tr_unit[k] = T.unit;
    }
    // block reduction in a fixed order
    for (int o = 32; o > 0; o >>= 1) {
        dsum += __shfl_xor(dsum, o);
        nacc += __shfl_xor(nacc, o);
        ntie += __shfl_xor(ntie, o);
    }
    if ((tid & 63) == 0) {
        s_red_d[tid >> 6] = dsum;
        s_red_a[tid >> 6] = nacc;
        s_red_t[tid >> 6] = ntie;
    }
    __syncthreads();
    if (tid == 0) {
        double d = 0.0;
        long long na = 0, nt = 0;
        for (int w = 0; w < DECIDE_THREADS / 64; ++w) {
            d += s_red_d[w];
            na += s_red_a[w];
            nt += s_red_t[w];
        }
        *a.E += d;
        *a.dsum += d;
        a.counters[0] += na;
        a.counters[1] += nt;
        a.counters[2] = 0;  // pool is free for the next batch
    }
}

__global__ void k_mc_reset(long long *counters, double *dsum)
{
    if (threadIdx.x < 3) counters[threadIdx.x] = 0;
    if (threadIdx.x == 0) *dsum = 0.0;
}

int pick_maxnu(int max_na)
{
    if (max_na <= 1) return 1;
    if (max_na <= 2) return 2;
    if (max_na <= 3) return 3;
    if (max_na <= 4) return 4;
    return 8;
}

template <int MAXNU>
void launch_batch(nd_box *b, const ScanArgs &sa, dim3 sgrid, size_t slds, const CorrArgs &ca)
{
    {
        nd::ProfScope ps(b, ND_PROF_MC_SCAN);
        hipLaunchKernelGGL(k_mc_scan<MAXNU>, sgrid, dim3(SCAN_THREADS), slds, b->stream, sa);
        ND_HIP(hipGetLastError());
    }
    {
        nd::ProfScope ps(b, ND_PROF_MC_CORR);
        hipLaunchKernelGGL(k_mc_corr<MAXNU>, dim3(ca.kb), dim3(64), 0, b->stream, ca);
        ND_HIP(hipGetLastError());
    }
}

void ensure_work(nd_box *b, int K, int n_jb)
{
    nd::McWork &w = b->mc;
    size_t pool = (size_t)K * (K - 1) / 2 + 1;
    if (w.trials && w.cap_k >= K && w.cap_jb >= n_jb && w.cap_pool >= pool) return;
    ND_HIP(hipStreamSynchronize(b->stream));
    nd::dfree(w.trials);
    nd::dfree(w.partial);
    nd::dfree(w.corr_n);
    nd::dfree(w.corr_off);
    nd::dfree(w.pool_m);
    nd::dfree(w.pool_c);
    nd::dfree(w.pool_s);
    w.trials = nullptr;
    w.partial = nullptr;
    w.corr_n = w.corr_off = w.pool_m = nullptr;
    w.pool_c = w.pool_s = nullptr;
    w.cap_k = w.cap_jb = 0;
    w.cap_pool = 0;
    w.trials = static_cast<nd::Trial *>(nd::dmalloc(sizeof(nd::Trial) * K));
    w.partial = static_cast<double *>(nd::dmalloc(sizeof(double) * 2 * (size_t)n_jb * K));
    w.corr_n = static_cast<int32_t *>(nd::dmalloc(sizeof(int32_t) * K));
    w.corr_off = static_cast<int32_t *>(nd::dmalloc(sizeof(int32_t) * K));
    w.pool_m = static_cast<int32_t *>(nd::dmalloc(sizeof(int32_t) * pool));
    w.pool_c = static_cast<double *>(nd::dmalloc(sizeof(double) * pool));
    w.pool_s = static_cast<double *>(nd::dmalloc(sizeof(double) * pool));
    if (!w.counters) w.counters = static_cast<long long *>(nd::dmalloc(sizeof(long long) * 4));
    if (!w.dsum) w.dsum = static_cast<double *>(nd::dmalloc(sizeof(double)));
    w.cap_k = K;
    w.cap_jb = n_jb;
    w.cap_pool = pool;
}

}  // namespace

namespace nd {

void mc_run(nd_box *b, const nd_mc_params *p, uint64_t seed, uint64_t first, int64_t n, const nd_mc_trace *trace)
{
    const int n_jb = (b->N + SCAN_JB - 1) / SCAN_JB;
    // Batch size: expected number of interacting earlier trials per trial
    // about 16, at most KMAX and the number of units.
    int K;
    if (p->k_batch > 0) {
        K = p->k_batch;
    } else {
        const double ext = (b->max_na > 1 ? 1.2 : 0.0) + p->max_disp * 1.8;
        const double reach = b->rc + 2.0 * ext;
        const double f = (4.0 / 3.0) * M_PI * reach * reach * reach / (b->L * b->L * b->L);
        K = (int)std::min(1e9, 16.0 / std::max(f, 1e-9));
    }
    K = std::max(1, std::min({K, KMAX, b->n_units}));
    ensure_work(b, K, n_jb);
    McWork &w = b->mc;
    const size_t lds = sizeof(float) * (size_t)b->P * b->n_pts;
    if (lds > 64 * 1024) fail(ND_E_UNSUPPORTED, "potential table larger than 64 KB");
    const double tie_rel = p->tie_rel > 0.0 ? p->tie_rel : 1e-6;
    const int maxnu = pick_maxnu(b->max_na);
    const int ncu = cu_count(b->device);

    hipLaunchKernelGGL(k_mc_reset, dim3(1), dim3(64), 0, b->stream, w.counters, w.dsum);
    ND_HIP(hipGetLastError());

    const float rcf = (float)(b->rc / b->L);
    for (int64_t done = 0; done < n;) {
        const int kb = (int)std::min<int64_t>(K, n - done);
        const uint64_t t0 = first + (uint64_t)done;

        ProposeArgs pa;
        pa.xyz = b->xyz;
        pa.pos4 = b->pos4;
        pa.poslo = b->poslo;
        pa.uoff = b->uoff;
        pa.N = b->N;
        pa.n_units = b->n_units;
        pa.L = b->L;
        pa.invL = 1.0 / b->L;
        pa.max_disp = p->max_disp;
        pa.max_rot = p->max_rot;
        pa.seed = seed;
        pa.t0 = t0;
        pa.kb = kb;
        pa.trials = w.trials;
        {
            ProfScope ps(b, ND_PROF_MC_PROPOSE);
            hipLaunchKernelGGL(k_mc_propose, dim3((kb + 63) / 64), dim3(64), 0, b->stream, pa);
            ND_HIP(hipGetLastError());
        }

        int tg = (int)std::max<long long>(1, std::min<long long>(MAX_TG, ((long long)kb * n_jb) / (2LL * ncu)));
        ScanArgs sa;
        sa.pos4 = b->pos4;
        sa.poslo = b->poslo;
        sa.tab = b->tab;
        sa.trials = w.trials;
        sa.N = b->N;
        sa.M = b->M;
        sa.n_pts = b->n_pts;
        sa.kb = kb;
        sa.tg = tg;
        sa.kcap = w.cap_k;
        sa.rcf2_filter = nd::filter_r2(b->rc / b->L);
        sa.rcf2 = (b->rc / b->L) * (b->rc / b->L);
        sa.tscale = b->L / b->h;
        sa.partial = w.partial;
        dim3 sgrid(n_jb, (kb + tg - 1) / tg);

        CorrArgs ca;
        ca.tab = b->tab;
        ca.trials = w.trials;
        ca.M = b->M;
        ca.n_pts = b->n_pts;
        ca.kb = kb;
        ca.rcf = rcf + 2e-6f;
        ca.rcf2_filter = sa.rcf2_filter;
        ca.rcf2 = sa.rcf2;
        ca.tscale = sa.tscale;
        ca.corr_n = w.corr_n;
        ca.corr_off = w.corr_off;
        ca.pool_m = w.pool_m;
        ca.pool_c = w.pool_c;
        ca.pool_s = w.pool_s;
        ca.pool_fill = w.counters + 2;

        switch (maxnu) {
        case 1: launch_batch<1>(b, sa, sgrid, lds, ca); break;
        case 2: launch_batch<2>(b, sa, sgrid, lds, ca); break;
        case 3: launch_batch<3>(b, sa, sgrid, lds, ca); break;
        case 4: launch_batch<4>(b, sa, sgrid, lds, ca); break;
        default: launch_batch<8>(b, sa, sgrid, lds, ca); break;
        }

        DecideArgs da;
        da.xyz = b->xyz;
        da.pos4 = b->pos4;
        da.poslo = b->poslo;
        da.E = b->E;
        da.trials = w.trials;
        da.partial = w.partial;
        da.corr_n = w.corr_n;
        da.corr_off = w.corr_off;
        da.pool_m = w.pool_m;
        da.pool_c = w.pool_c;
        da.pool_s = w.pool_s;
        da.N = b->N;
        da.kb = kb;
        da.n_jb = n_jb;
        da.kcap = w.cap_k;
        da.kT = p->kT;
        da.tie_rel = tie_rel;
        da.counters = w.counters;
        da.dsum = w.dsum;
        da.tr_dE = trace && trace->dE ? trace->dE + done : nullptr;
        da.tr_sabs = trace && trace->sabs ? trace->sabs + done : nullptr;
        da.tr_acc = trace && trace->accepted ? trace->accepted + done : nullptr;
        da.tr_unit = trace && trace->unit ? trace->unit + done : nullptr;
        {
            ProfScope ps(b, ND_PROF_MC_DECIDE);
            hipLaunchKernelGGL(k_mc_decide, dim3(1), dim3(DECIDE_THREADS), 0, b->stream, da);
            ND_HIP(hipGetLastError());
        }
        done += kb;
    }
}

}  // namespace nd

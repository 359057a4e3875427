// Metropolis Monte Carlo over rigid units (Sec. "Algorithmic Flow" III)
// with the per-trial energy change computed as a minimum-image pair sum
// against every atom (Sec. "Acceleration method": the per-step work that is
// proportional to N).
//
// Trials are processed in batches of up to K consecutive trials that move
// distinct units: in sequential order any K <= n_units consecutive trials
// do; in random order a batch is cut before the first trial whose unit is
// already in it.  A trial's proposal
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
#include <type_traits>

namespace {

using nd::PairCtx;
using nd::ld4;
using nd::ld_lds4;
using nd::ldg;
using nd::ld_i4;
using nd::ld_d2;
using nd::stg;

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_JPT = 8;                         // j atoms held per thread
constexpr int SCAN_JB = SCAN_THREADS * SCAN_JPT;    // atoms per j-block
constexpr int MAX_TG = 64;                          // trials per scan block
constexpr int KMAX = 2048;                          // trials per batch
constexpr int N_SLAB = 8;                           // spatial slabs along z, one per XCD
constexpr double TWO_PI = 6.283185307179586;

// ---------------------------------------------------------------- RNG
// SplitMix64 (Steele, Lea, Flood 2014): output i of the generator seeded
// with s is the 64-bit finalizer applied to s + (i + 1) * gamma.  Draw d of
// trial t is output 16 t + d, mapped to [0, 1) with 53 bits.
__host__ __device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (i + 1ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__host__ __device__ __forceinline__ double draw(uint64_t seed, uint64_t t, int d)
{
    return (double)(splitmix64(seed, 16ull * t + (uint64_t)d) >> 11) * (1.0 / 9007199254740992.0);
}

// Unit moved by trial t: t mod n_units in sequential order; in random order
// floor(u_7 n_units) of the trial's draw 7 (the last unit if the product
// rounds up to n_units).  The host plans batches with the same function.
__host__ __device__ __forceinline__ int trial_unit(int order, uint64_t seed, uint64_t t, int n_units)
{
    if (order == ND_ORDER_SEQ) return (int)(t % (uint64_t)n_units);
    const int u = (int)floor(draw(seed, t, 7) * (double)n_units);
    return u < n_units ? u : n_units - 1;
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
    int N, n_units, order;
    double L, invL, max_disp, max_rot, kT;
    uint64_t seed, t0;
    int kb, kcap;
    nd::Trial *trials;
    float4 *spheres;
    int32_t *slab;  // [N_SLAB] counts (zero beforehand), then [N_SLAB][kcap] trial lists
    int4 *head;     // [kb] unit, first atom, atoms, 0 of each trial (compact copy for the decision)
    double *hthr;   // [kb] acceptance threshold of each trial (compact copy)
    // flexible molecules: single-atom moves and intramolecular harmonic terms
    double atom_frac, atom_disp;
    const double *r0;       // [N][ND_MAX_UNIT_ATOMS] reference lengths (null: no intramolecular terms)
    const uint8_t *sp;      // [N] species
    int M;
    double kint[ND_MAX_SPECIES * (ND_MAX_SPECIES + 1) / 2];
};

// Nearest-image distance in FP64 of two positions (displacement by
// comparison with L/2, the oracle's form).
__device__ __forceinline__ double dist_fp64(double ax, double ay, double az, double bx, double by, double bz, double L)
{
    const double dx = min_image_cmp(bx - ax, L), dy = min_image_cmp(by - ay, L), dz = min_image_cmp(bz - az, L);
    return sqrt(dx * dx + dy * dy + dz * dz);
}

// Change of unit u's intramolecular energy sum_{a<b} k (r_ab - r0_ab)^2 when
// atoms a0 .. a0 + na - 1 move to new_x (the others stay), and its |terms|.
__device__ void intra_delta(const ProposeArgs &a, int u0, int u1, int a0, int na, const float (*new_x)[3],
                            double &dE, double &S)
{
    const int N = a.N;
    double e = 0.0, s = 0.0;
    for (int p = u0; p < u1; ++p)
        for (int q = p + 1; q < u1; ++q) {
            const bool mp = p >= a0 && p < a0 + na, mq = q >= a0 && q < a0 + na;
            if (!mp && !mq) continue;
            const double px = a.xyz[p], py = a.xyz[N + p], pz = a.xyz[2 * N + p];
            const double qx = a.xyz[q], qy = a.xyz[N + q], qz = a.xyz[2 * N + q];
            const double npx = mp ? (double)new_x[p - a0][0] : px, npy = mp ? (double)new_x[p - a0][1] : py,
                         npz = mp ? (double)new_x[p - a0][2] : pz;
            const double nqx = mq ? (double)new_x[q - a0][0] : qx, nqy = mq ? (double)new_x[q - a0][1] : qy,
                         nqz = mq ? (double)new_x[q - a0][2] : qz;
            const double k = a.kint[nd::pair_index(a.sp[p], a.sp[q], a.M)];
            const double r0 = a.r0[(size_t)p * ND_MAX_UNIT_ATOMS + (q - u0)];
            const double dn = dist_fp64(npx, npy, npz, nqx, nqy, nqz, a.L) - r0;
            const double dold = dist_fp64(px, py, pz, qx, qy, qz, a.L) - r0;
            const double vn = k * dn * dn, vo = k * dold * dold;
            e += vn - vo;
            s += fabs(vn) + fabs(vo);
        }
    dE = e;
    S = s;
}

// Threshold form of the Metropolis test: with u > 0, u < exp(-dE/kT)
// exactly when dE < -kT ln u (they can differ only by rounding, far inside
// the near-tie band); u = 0 accepts while exp(-dE/kT) is not 0.
__device__ __forceinline__ double accept_threshold(double u, double kT)
{
    return u > 0.0 ? -kT * log(u) : 745.13321910194122 * kT;
}

// One thread per trial: translation tau = d (2u - 1) per axis; for units of
// several atoms a rotation by theta = r (2u_5 - 1) about the axis
// (sqrt(1-z^2) cos phi, sqrt(1-z^2) sin phi, z), z = 2u_3 - 1, phi = 2 pi u_4,
// through the unweighted centroid of the unit unwrapped around its first
// atom (Rodrigues' formula).  FP64, then wrapped and rounded to float32.
__device__ __forceinline__ void propose_one(const ProposeArgs &a, int k)
{
    const uint64_t t = a.t0 + (uint64_t)k;
    const int u = trial_unit(a.order, a.seed, t, a.n_units);
    const int u0 = a.uoff[u], u1 = a.uoff[u + 1];
    int a0 = u0;
    int na = u1 - u0;
    const int N = a.N;
    const double L = a.L;
    nd::Trial *T = a.trials + k;

    // a single-atom move (draw 8 below atom_frac): atom floor(u_9 na) of the
    // unit translates by up to atom_disp per axis
    double disp = a.max_disp;
    if (a.atom_frac > 0.0 && draw(a.seed, t, 8) < a.atom_frac) {
        int ai = (int)floor(draw(a.seed, t, 9) * (double)na);
        if (ai >= na) ai = na - 1;
        a0 = u0 + ai;
        na = 1;
        disp = a.atom_disp;
    }
    double tau[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) tau[c] = disp * (2.0 * draw(a.seed, t, c) - 1.0);
    T->unit = u;
    T->a0 = a0;
    T->na = na;
    T->pad = 0;
    T->thr = accept_threshold(draw(a.seed, t, 6), a.kT);
    a.head[k] = make_int4(u, a0, na, 0);
    a.hthr[k] = T->thr;

    // centroid of the unit unwrapped around its first atom, rotation
    double x0[3] = {0.0, 0.0, 0.0}, cen[3] = {0.0, 0.0, 0.0};
    double n0 = 0.0, n1 = 0.0, n2 = 0.0, ct = 1.0, st = 0.0, omc = 0.0;
    if (na > 1) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            x0[c] = (double)a.xyz[c * N + a0];
            double s = 0.0;
            for (int at = 0; at < na; ++at) s += x0[c] + min_image_cmp((double)a.xyz[c * N + a0 + at] - x0[c], L);
            cen[c] = s / (double)na;
        }
        const double zc = 2.0 * draw(a.seed, t, 3) - 1.0;
        const double phi = TWO_PI * draw(a.seed, t, 4);
        const double sr = sqrt(1.0 - zc * zc);
        n0 = sr * cos(phi);
        n1 = sr * sin(phi);
        n2 = zc;
        const double th = a.max_rot * (2.0 * draw(a.seed, t, 5) - 1.0);
        ct = cos(th);
        st = sin(th);
        omc = 1.0 - ct;
    }

    // new positions, atom by atom, written straight into the trial record
    const float4 ref = a.pos4[a0];
    float sx = 0.f, sy = 0.f, sz = 0.f;
    for (int at = 0; at < na; ++at) {
        float nx0, nx1, nx2;
        if (na == 1) {
            nx0 = wrap_round((double)a.xyz[a0] + tau[0], L);
            nx1 = wrap_round((double)a.xyz[N + a0] + tau[1], L);
            nx2 = wrap_round((double)a.xyz[2 * N + a0] + tau[2], L);
        } else {
            const double v0 = (x0[0] + min_image_cmp((double)a.xyz[a0 + at] - x0[0], L)) - cen[0];
            const double v1 = (x0[1] + min_image_cmp((double)a.xyz[N + a0 + at] - x0[1], L)) - cen[1];
            const double v2 = (x0[2] + min_image_cmp((double)a.xyz[2 * N + a0 + at] - x0[2], L)) - cen[2];
            // Rodrigues: v cos + (n x v) sin + n (n.v)(1 - cos)
            const double c0 = n1 * v2 - n2 * v1, c1 = n2 * v0 - n0 * v2, c2 = n0 * v1 - n1 * v0;
            const double dot = n0 * v0 + n1 * v1 + n2 * v2;
            const double kk = dot * omc;
            const double w0 = v0 * ct + c0 * st + n0 * kk;
            const double w1 = v1 * ct + c1 * st + n1 * kk;
            const double w2 = v2 * ct + c2 * st + n2 * kk;
            nx0 = wrap_round(cen[0] + w0 + tau[0], L);
            nx1 = wrap_round(cen[1] + w1 + tau[1], L);
            nx2 = wrap_round(cen[2] + w2 + tau[2], L);
        }
        const float4 o = a.pos4[a0 + at];
        const double f0 = (double)nx0 * a.invL, f1 = (double)nx1 * a.invL, f2 = (double)nx2 * a.invL;
        float4 q, ql;
        q.x = (float)f0;
        q.y = (float)f1;
        q.z = (float)f2;
        q.w = o.w;
        ql.x = (float)(f0 - (double)q.x);
        ql.y = (float)(f1 - (double)q.y);
        ql.z = (float)(f2 - (double)q.z);
        ql.w = __int_as_float(u);
        T->old_hi[at] = o;
        T->old_lo[at] = a.poslo[a0 + at];
        T->new_hi[at] = q;
        T->new_lo[at] = ql;
        T->new_x[at][0] = nx0;
        T->new_x[at][1] = nx1;
        T->new_x[at][2] = nx2;
        T->old_x[at][0] = a.xyz[a0 + at];
        T->old_x[at][1] = a.xyz[N + a0 + at];
        T->old_x[at][2] = a.xyz[2 * N + a0 + at];
        float d;
        d = o.x - ref.x; sx += d - rintf(d);
        d = o.y - ref.y; sy += d - rintf(d);
        d = o.z - ref.z; sz += d - rintf(d);
        d = q.x - ref.x; sx += d - rintf(d);
        d = q.y - ref.y; sy += d - rintf(d);
        d = q.z - ref.z; sz += d - rintf(d);
    }
    // bounding sphere of the old and new atoms (fractional)
    const float inv2n = 1.0f / (float)(2 * na);
    const float cx = ref.x + sx * inv2n, cy = ref.y + sy * inv2n, cz = ref.z + sz * inv2n;
    float r2max = 0.f;
    for (int at = 0; at < na; ++at) {
        const float4 o = T->old_hi[at], q = T->new_hi[at];
        float dx = o.x - cx, dy = o.y - cy, dz = o.z - cz;
        dx -= rintf(dx); dy -= rintf(dy); dz -= rintf(dz);
        r2max = fmaxf(r2max, dx * dx + dy * dy + dz * dz);
        dx = q.x - cx; dy = q.y - cy; dz = q.z - cz;
        dx -= rintf(dx); dy -= rintf(dy); dz -= rintf(dz);
        r2max = fmaxf(r2max, dx * dx + dy * dy + dz * dz);
    }
    const float rad = sqrtf(r2max) * 1.0001f + 2e-6f;
    T->dintra = 0.0;
    T->sintra = 0.0;
    if (a.r0) intra_delta(a, u0, u1, a0, na, T->new_x, T->dintra, T->sintra);
    T->cen[0] = cx;
    T->cen[1] = cy;
    T->cen[2] = cz;
    T->rad = rad;
    a.spheres[k] = make_float4(cx, cy, cz, rad);
    // z-slab of the centre, for the XCD-aware assignment of scan blocks; the
    // trials of a wave are listed with one atomic per slab they fall in
    // (the lanes calling this may be any subset of the wave)
    const float zw = cz - floorf(cz);
    const int sb = min(max((int)(zw * (float)N_SLAB), 0), N_SLAB - 1);
    const int lane = threadIdx.x & 63;
    const unsigned long long lt = (1ull << lane) - 1ull;
    int pos = 0;
#pragma unroll
    for (int q = 0; q < N_SLAB; ++q) {
        const unsigned long long m = __ballot(sb == q);
        if (m != 0ull && sb == q) {
            const int leader = __ffsll((long long)m) - 1;
            int base = 0;
            if (lane == leader) base = atomicAdd(&a.slab[q], __popcll(m));
            base = __shfl(base, leader);
            pos = base + __popcll(m & lt);
        }
    }
    a.slab[N_SLAB + sb * a.kcap + pos] = k;
}

__global__ __launch_bounds__(64) void k_mc_propose(ProposeArgs a)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < a.kb) propose_one(a, k);
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
__global__ __launch_bounds__(SCAN_THREADS, 4) void k_mc_scan(ScanArgs a)
{
    extern __shared__ __align__(16) float s_tab[];  // [P][n_pts]
    __shared__ int s_prow[16];
    __shared__ double s_red[2][SCAN_THREADS / 64][MAX_TG];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int P = a.M * (a.M + 1) / 2;
    nd::stage_floats<SCAN_THREADS>(s_tab, a.tab, P * a.n_pts);
    if (tid < a.M * a.M) s_prow[tid] = nd::pair_index(tid / a.M, tid % a.M, a.M) * a.n_pts;

    const int jstart = blockIdx.x * SCAN_JB;
    float4 pj[SCAN_JPT], pl[SCAN_JPT];
    const float qnan = __int_as_float(0x7fc00000);
#pragma unroll
    for (int m = 0; m < SCAN_JPT; ++m) {
        const int j = jstart + m * SCAN_THREADS + tid;
        pj[m] = (j < a.N) ? a.pos4[j] : make_float4(qnan, qnan, qnan, 0.f);
        pl[m] = (j < a.N) ? a.poslo[j] : make_float4(0.f, 0.f, 0.f, __int_as_float(-1));
    }
    __syncthreads();

    PairCtx c{s_tab, s_prow, a.M, a.n_pts, a.rcf2_filter, a.rcf2, a.tscale};
    const int k0 = blockIdx.y * a.tg;
    const int k1 = min(a.kb, k0 + a.tg);
    for (int k = k0; k < k1; ++k) {
        const nd::Trial *T = a.trials + k;
        const int tna = T->na, tunit = T->unit;
        double e = 0.0, s = 0.0;
        // every atom of the moved unit is left out (all of them when the unit
        // moves, its other atoms when one atom of a flexible unit moves)
        unsigned ex = 0u;
#pragma unroll
        for (int m = 0; m < SCAN_JPT; ++m)
            if (__float_as_int(pl[m].w) == tunit) ex |= 1u << m;
        scan_trial<MAXNU, true>(c, T, tna, pj, pl, ex, e, s);
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

// ---------------------------------------------------------------- partial sums
// full scan: dE0_k = sum over j-blocks of the partial sums (fixed order)
__global__ void k_mc_reduce(const double *__restrict__ partial, int n_jb, int kcap, int kb, double *__restrict__ dE0,
                            double *__restrict__ S0, const nd::Trial *__restrict__ trials)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kb) return;
    // the intramolecular change of flexible molecules first, then the pair sums
    double e = trials[k].dintra, s = trials[k].sintra;
    for (int jb = 0; jb < n_jb; ++jb) {
        e += partial[((size_t)jb * 2 + 0) * kcap + k];
        s += partial[((size_t)jb * 2 + 1) * kcap + k];
    }
    dE0[k] = e;
    S0[k] = s;
}

// Exact pair energy from the FP64 fractional displacement d = s_j - s_a
// (the same arithmetic as pair_u_exact); false beyond r_cut.
__device__ __forceinline__ bool pair_u_img(const PairCtx &c, double ex, double ey, double ez, int row, float &u)
{
    const double r2 = fma(ez, ez, fma(ey, ey, ex * ex));
    if (!(r2 < c.rcf2)) return false;
    const double t = nd::sqrt_nr(r2) * c.tscale;
    int i0 = (int)t;
    i0 = min(i0, c.n_pts - 2);
    const float f = (float)(t - (double)i0);
    const float *tr = c.tab + row;
    const float u0 = tr[i0];
    const float u1 = tr[i0 + 1];
    u = fmaf(f, u1 - u0, u0);
    return true;
}

__device__ __forceinline__ bool pair_u_disp(const PairCtx &c, double ex, double ey, double ez, int row, float &u)
{
    ex -= rint(ex);
    ey -= rint(ey);
    ez -= rint(ez);
    return pair_u_img(c, ex, ey, ez, row, u);
}

// ---------------------------------------------------------------- corrections
constexpr int CORR_CAP = 24;  // fixed entry slots per trial (more go to an overflow area)
constexpr int CORR_TPB = 4;   // trials per correction block (one per wave)

struct CorrArgs {
    const float *tab;  // table rows read through the caches
    const nd::Trial *trials;
    const float4 *spheres;
    int M, n_pts, kb;
    float rcf, rcf2_filter;
    double rcf2, tscale;
    int32_t *corr_n, *corr_ptr;  // [K] entries of trial k and where they start
    float *corr_s;               // [K] sum of |U| over all of trial k's correction terms
    double2 *corr_b;             // [2K] (lo, hi), (mag, count) of trial k's entries with m >= 0
    int32_t *pool_m;             // earlier trial m (increasing within a trial); -1: C_km = 0
    double *pool_c;              // C_km, the change of k's dE if m was accepted
    int32_t *ovf_fill;           // overflow entries used in this batch
    int ovf_base;
    int per_block;               // decision launch: trials per correction block (one per wave, <= 16)
};

// A decided batch's final dE sums, counters and trace (k_mc_final's body,
// run as the first block of the next scan launch): its entries, ΔE⁰ and
// |U| sums by buffer, and what the decision stored.
struct FinalArgs {
    const double *dE0, *S0, *thr;
    const float *corr_s;
    const int32_t *corr_n, *corr_ptr, *pool_m;
    const double *pool_c;
    const uint8_t *acc;
    int kb;  // 0: nothing to do
    double kT, tie_rel;
    double *E, *dsum;
    long long *counters;
    double *tr_dE, *tr_sabs;
    uint8_t *tr_acc;
};
constexpr int FIN_THREADS = 256;
__device__ void final_body(const FinalArgs &f, unsigned char *lds);

constexpr int CORR_LIST = 256;  // hits listed per wave at a time

// Per-wave LDS scratch of the correction step: the hit list, per-lane
// partial sums, and trial k's atoms (FP64 fractional positions and species,
// old at 2a, new at 2a + 1).
struct CorrScratch {
    int wl[CORR_LIST];
    double pc[64], ps[64];
    double x[2 * ND_MAX_UNIT_ATOMS], y[2 * ND_MAX_UNIT_ATOMS], z[2 * ND_MAX_UNIT_ATOMS];
    int sp[2 * ND_MAX_UNIT_ATOMS];
};

// List the hits of ranks [first, first + CORR_LIST): earlier trials m < k of
// the batch whose bounding sphere comes within r_cut of k's, in increasing m.
// Returns the total number of hits.  The spheres are read from `lds` (a copy
// of the batch's spheres in LDS) when it is not null, else from memory.
__device__ __forceinline__ int corr_collect(const CorrArgs &a, const float4 *lds, float4 A, int k, int lane, int first,
                                            int *wl)
{
    const unsigned long long lt = (1ull << lane) - 1ull;
    int n = 0;
    constexpr int CB = 8;  // spheres per lane per round, their loads in flight together
    const float rA = a.rcf + A.w;
    for (int m0 = 0; m0 < k; m0 += 64 * CB) {
        float4 B[CB];
#pragma unroll
        for (int h = 0; h < CB; ++h) {
            const int m = min(m0 + 64 * h + lane, k - 1);
            B[h] = lds ? ld_lds4(lds + m) : ld4(a.spheres + m);
        }
        // the lane's hits of the round as a bit mask; hits are rare, so the
        // listing (in increasing m) runs only for rounds that have one
        unsigned int hm = 0u;
#pragma unroll
        for (int h = 0; h < CB; ++h) {
            float dx = B[h].x - A.x, dy = B[h].y - A.y, dz = B[h].z - A.z;
            dx -= rintf(dx);
            dy -= rintf(dy);
            dz -= rintf(dz);
            const float lim = rA + B[h].w;
            // both conditions evaluated (no branch per sphere)
            const unsigned int in = (unsigned int)(m0 + 64 * h + lane < k);
            const unsigned int near = (unsigned int)(dx * dx + dy * dy + dz * dz < lim * lim);
            hm |= (in & near) << h;
        }
        if (__ballot(hm != 0u) == 0ull) continue;
#pragma unroll
        for (int h = 0; h < CB; ++h) {
            const bool hit = (hm >> h) & 1u;
            const unsigned long long bal = __ballot(hit);
            const int idx = n + __popcll(bal & lt) - first;
            if (hit && idx >= 0 && idx < CORR_LIST) wl[idx] = m0 + 64 * h + lane;
            n += __popcll(bal);
        }
    }
    __builtin_amdgcn_wave_barrier();
    return n;
}

// One wave: the entries (m, C_km) of trial k for every hit m, in increasing
// m, with C_km = [U(k',m') - U(k,m')] - [U(k',m) - U(k,m)].  The pair terms
// are spread over the lanes: one lane per (hit, atom of m, old/new of m),
// each summing over k's atoms old and new; the lane of each hit then adds
// its items' partial sums in a fixed order.
template <int MAXNU>
__device__ __forceinline__ void corr_trial(const CorrArgs &a, const PairCtx &c, int k, int lane, CorrScratch &cs,
                                           const float4 *lds = nullptr)
{
    const float4 A = lds ? ld_lds4(lds + k) : a.spheres[k];
    // trial k's own atoms (old and new), loaded before the collection so
    // that their latency overlaps it; slots past na are read but not used
    const nd::Trial *Tk = a.trials + k;
    float4 kh = make_float4(0.f, 0.f, 0.f, 0.f), kl = kh;
    if (lane < 2 * MAXNU) {
        const int at = lane >> 1;
        kh = ld4((lane & 1) ? &Tk->new_hi[at] : &Tk->old_hi[at]);
        kl = ld4((lane & 1) ? &Tk->new_lo[at] : &Tk->old_lo[at]);
    }
    const int nak = ldg(&Tk->na);
    const int n = k > 0 ? corr_collect(a, lds, A, k, lane, 0, cs.wl) : 0;
    int base;
    if (n <= CORR_CAP) {
        base = k * CORR_CAP;
    } else {
        int o = 0;
        if (lane == 0) o = atomicAdd(a.ovf_fill, n);
        base = a.ovf_base + __shfl(o, 0);
    }
    if (lane == 0) {
        a.corr_n[k] = n;
        a.corr_ptr[k] = base;
    }
    if (n == 0) {
        if (lane == 0) {
            a.corr_s[k] = 0.0f;
            nd::st_d2(a.corr_b + 2 * k, make_double2(0.0, 0.0));
            nd::st_d2(a.corr_b + 2 * k + 1, make_double2(0.0, 0.0));
        }
        return;
    }
    if (lane < 2 * MAXNU) {
        cs.x[lane] = (double)kh.x + (double)kl.x;
        cs.y[lane] = (double)kh.y + (double)kl.y;
        cs.z[lane] = (double)kh.z + (double)kl.z;
        cs.sp[lane] = __float_as_int(kh.w);
    }
    __builtin_amdgcn_wave_barrier();
    constexpr int IPH = 2 * MAXNU;   // items per hit
    constexpr int HPR = 64 / IPH;    // hits per round
    const int hl = lane / IPH, r = lane - hl * IPH;
    const int y = r >> 1, om = r & 1;  // atom of m; 0: m old, 1: m new
    double Sk = 0.0;
    double blo = 0.0, bhi = 0.0, bmag = 0.0, bnv = 0.0;  // bracket summary of the entries with m >= 0
    int wbase = 0;
    // two rounds of hits at a time, the loads of both issued together
    for (int h0 = 0; h0 < n; h0 += 2 * HPR) {
        if (h0 + 2 * HPR > wbase + CORR_LIST) {
            // more hits than the list holds (rare): list the next window
            wbase = h0;
            corr_collect(a, lds, A, k, lane, wbase, cs.wl);
        }
        int nam[2];
        float4 q[2], ql[2];
#pragma unroll
        for (int rr = 0; rr < 2; ++rr) {
            // a lane past the hits reads hit h0 again (unused): no condition
            // between the loads of both rounds
            const int h = h0 + rr * HPR + hl;
            const bool hv = hl < HPR && h < n;
            const nd::Trial *Tm = a.trials + cs.wl[(hv ? h : h0) - wbase];
            const int na_m = ldg(&Tm->na);
            q[rr] = ld4(om ? &Tm->new_hi[y] : &Tm->old_hi[y]);
            ql[rr] = ld4(om ? &Tm->new_lo[y] : &Tm->old_lo[y]);
            nam[rr] = hv ? na_m : 0;
        }
#pragma unroll
        for (int rr = 0; rr < 2; ++rr) {
            const int hr0 = h0 + rr * HPR;
            if (hr0 >= n) break;
            // the item's pair terms with k's atoms (old and new): every
            // table index first, then all their table loads in flight
            // together, then the sums in the order atom, old/new
            constexpr int NT = 2 * MAXNU;
            float tu0[NT], tu1[NT], tf[NT];
            bool tin[NT];
            {
                const double qx = (double)q[rr].x + (double)ql[rr].x, qy = (double)q[rr].y + (double)ql[rr].y,
                             qz = (double)q[rr].z + (double)ql[rr].z;
                const int sq = __float_as_int(q[rr].w);
#pragma unroll
                for (int ia = 0; ia < NT; ++ia) {  // atom ia / 2 of k, old (even) or new (odd)
                    const bool v = y < nam[rr] && (ia >> 1) < nak;
                    double ex = qx - cs.x[ia], ey = qy - cs.y[ia], ez = qz - cs.z[ia];
                    ex -= rint(ex);
                    ey -= rint(ey);
                    ez -= rint(ez);
                    const double r2 = fma(ez, ez, fma(ey, ey, ex * ex));
                    tin[ia] = v && r2 < c.rcf2;
                    const double t = nd::sqrt_nr(r2) * c.tscale;
                    // in range for any r2 (also NaN from unused slots): the
                    // index is clamped before the conversion
                    const int i0 = min((int)fmin(t, 1e9), c.n_pts - 2);
                    tf[ia] = (float)(t - (double)i0);
                    const float *tr = c.tab + (v ? c.prow[cs.sp[ia] * c.M + sq] : 0) + i0;
                    tu0[ia] = tr[0];
                    tu1[ia] = tr[1];
                }
            }
            double pc = 0.0, ps = 0.0;
#pragma unroll
            for (int ia = 0; ia < NT; ++ia) {
                if (tin[ia]) {
                    const float u = fmaf(tf[ia], tu1[ia] - tu0[ia], tu0[ia]);
                    // + (k', m') and (k, m); - (k, m') and (k', m)
                    pc += ((ia & 1) == om) ? (double)u : -(double)u;
                    ps += (double)fabsf(u);
                }
            }
            cs.pc[lane] = pc;
            cs.ps[lane] = ps;
            __builtin_amdgcn_wave_barrier();
            if (lane < HPR && hr0 + lane < n) {
                double C = 0.0, S = 0.0;
#pragma unroll
                for (int qq = 0; qq < IPH; ++qq) {
                    C += cs.pc[lane * IPH + qq];
                    S += cs.ps[lane * IPH + qq];
                }
                const int m = cs.wl[hr0 + lane - wbase];
                const bool v = S > 0.0;
                stg(a.pool_m + base + hr0 + lane, v ? m : -1);
                stg(a.pool_c + base + hr0 + lane, C);
                Sk += S;
                blo += v ? fmin(C, 0.0) : 0.0;
                bhi += v ? fmax(C, 0.0) : 0.0;
                bmag += v ? fabs(C) : 0.0;
                bnv += v ? 1.0 : 0.0;
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        Sk += __shfl_xor(Sk, o);
        blo += __shfl_xor(blo, o);
        bhi += __shfl_xor(bhi, o);
        bmag += __shfl_xor(bmag, o);
        bnv += __shfl_xor(bnv, o);
    }
    if (lane == 0) {
        a.corr_s[k] = (float)Sk;
        nd::st_d2(a.corr_b + 2 * k, make_double2(blo, bhi));
        nd::st_d2(a.corr_b + 2 * k + 1, make_double2(bmag, bnv));
    }
}

template <int MAXNU>
__global__ __launch_bounds__(256) void k_mc_corr(CorrArgs a)
{
    __shared__ int s_prow[16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid < a.M * a.M) s_prow[tid] = nd::pair_index(tid / a.M, tid % a.M, a.M) * a.n_pts;
    __syncthreads();
    const PairCtx c{a.tab, s_prow, a.M, a.n_pts, a.rcf2_filter, a.rcf2, a.tscale};
    __shared__ CorrScratch s_cs[4];
    const int k_begin = blockIdx.x * CORR_TPB, k_end = min(a.kb, k_begin + CORR_TPB);
    for (int k = k_begin + wave; k < k_end; k += 4) corr_trial<MAXNU>(a, c, k, lane, s_cs[wave]);
}

// ---------------------------------------------------------------- cell scan
constexpr int CS_LIST = 192;  // survivors buffered per wave

struct CellScanArgs {
    const float4 *spos4;
    const float4 *sposlo;    // .w: unit
    const int32_t *cstart;
    const float *tab;
    const nd::Trial *trials;
    const float *drift;
    const int32_t *slab;     // [N_SLAB] counts, then [N_SLAB][kcap] trial lists
    int M, n_pts, kb, nc, kcap, per_slab;
    int nw;                  // waves per trial (1, 2 or 4; picks the kernel)
    float rcf, rcf2_filter;
    double rcf2, tscale;
    double *dE0, *S0;
    unsigned long long *count;  // null, or [0] candidates tested, [1] survivors (measurement)
};

// Trial atoms staged in LDS for the scan: FP64 fractional position and the
// table-row base of the atom's species, for the old (index 2a) and new
// (2a + 1) position of atom a.
struct TrialAtoms {
    double x[2 * ND_MAX_UNIT_ATOMS], y[2 * ND_MAX_UNIT_ATOMS], z[2 * ND_MAX_UNIT_ATOMS];
    int rb[2 * ND_MAX_UNIT_ATOMS];
};

// Survivors are kept in LDS as their current position, hi (with .w =
// species) and lo.  CIMG: the trial's atoms (taken
// at their images nearest the centre) lie within rad of the centre and
// r_cut + 2 rad < L/2, so the survivor's image nearest the centre is its
// nearest image to every atom of the trial along each axis, and the
// per-pair image shift is dropped (the displacements differ from the
// per-pair ones only by the rounding of the shifted positions, ~1e-16).
template <int MAXNU, bool CIMG>
__device__ __forceinline__ void cell_flush(const PairCtx &c, const TrialAtoms &ta, int tna, const float4 *list,
                                           const float4 *listlo, int nlist, int lane, double &e, double &s,
                                           double cx, double cy, double cz)
{
    for (int i = lane; i < nlist; i += 64) {
        const float4 q = list[i];
        const int w = __float_as_int(q.w);
        const float4 ql = listlo[i];
        double sx = (double)q.x + (double)ql.x, sy = (double)q.y + (double)ql.y, sz = (double)q.z + (double)ql.z;
        if (CIMG) {
            sx -= rint(sx - cx);
            sy -= rint(sy - cy);
            sz -= rint(sz - cz);
        }
        const int sj = w;
#pragma unroll
        for (int at = 0; at < MAXNU; ++at) {
            if (at < tna) {
                float u;
                // one table row for the atom's old and new position (its species)
                const int rn = c.prow[ta.rb[2 * at + 1] + sj];
                const double nx = sx - ta.x[2 * at + 1], ny = sy - ta.y[2 * at + 1], nz = sz - ta.z[2 * at + 1];
                if (CIMG ? pair_u_img(c, nx, ny, nz, rn, u) : pair_u_disp(c, nx, ny, nz, rn, u)) {
                    e += (double)u;
                    s += (double)fabsf(u);
                }
                const double ox = sx - ta.x[2 * at], oy = sy - ta.y[2 * at], oz = sz - ta.z[2 * at];
                if (CIMG ? pair_u_img(c, ox, oy, oz, rn, u) : pair_u_disp(c, ox, oy, oz, rn, u)) {
                    e -= (double)u;
                    s += (double)fabsf(u);
                }
            }
        }
    }
}

template <int MAXNU>
__device__ __forceinline__ void cell_flush_any(bool cimg, const PairCtx &c, const TrialAtoms &ta, int tna,
                                               const float4 *list, const float4 *listlo, int nlist, int lane,
                                               double &e, double &s, double cx, double cy, double cz)
{
    if (cimg)
        cell_flush<MAXNU, true>(c, ta, tna, list, listlo, nlist, lane, e, s, cx, cy, cz);
    else
        cell_flush<MAXNU, false>(c, ta, tna, list, listlo, nlist, lane, e, s, cx, cy, cz);
}

// Distance from c to the nearest periodic image of the cell interval
// [i/nc, (i+1)/nc) along one axis.
__device__ __forceinline__ float gap_to_cell(float c, int i, float inv_nc)
{
    float d = ((float)i + 0.5f) * inv_nc - c;
    d -= rintf(d);
    return fmaxf(0.0f, fabsf(d) - 0.5f * inv_nc);
}

// Trial k by NW waves (wsub = the wave's rank among them).  The cell rows
// (z, y) within reach of the trial's bounding sphere are dealt round-robin
// to the waves; each row is cut to the chord of the reach sphere at the row's nearest point
// (rows that miss the sphere are skipped) and split in two slot ranges
// where it wraps.  A wave fetches up to 64 rows at once (one per lane),
// concatenates their slot ranges with a prefix sum, and walks the
// concatenation 128 candidates at a time; candidates whose current position
// lies within r_cut + radius of the centre (atoms of the moved unit, known
// by the unit in lo.w, aside) are compacted into LDS and their exact pair
// terms summed.
template <int NW>
__device__ __forceinline__ void scan_sync()
{
    if (NW == 1)
        __builtin_amdgcn_wave_barrier();
    else
        __syncthreads();
}

// With NW > 1 every wave of the block calls this the same number of times
// (active false: a wave with no trial in this round, which only takes part
// in the barriers).
template <int MAXNU, int NW>
__device__ __forceinline__ void scan_cells_group(const CellScanArgs &a, const PairCtx &c, int k, bool active, int wsub,
                                                 int lane, float4 *list, float4 *listlo, double *red, TrialAtoms &ta,
                                                 unsigned long long *cnt)
{
    scan_sync<NW>();  // the previous trial is done with ta, red and the lists
    if (!active) {
        scan_sync<NW>();
        scan_sync<NW>();
        return;
    }
    const nd::Trial *T = a.trials + k;
    const int tna = T->na, tunit = T->unit;
    const float cx = T->cen[0], cy = T->cen[1], cz = T->cen[2];
    const float surv = a.rcf + T->rad + 4e-6f;
    const float surv2 = surv * surv;
    // r_cut + 2 rad < L/2: every pair term of the trial can take the nearest
    // image of its survivor relative to the centre (see cell_flush)
    const bool cimg = a.rcf + 2.0f * T->rad + 1e-4f < 0.5f;
    // every slot up to MAXNU is read (in bounds, unused past na), so these
    // loads do not wait for na
    if (wsub == 0 && lane < 2 * MAXNU) {
        const int at = lane >> 1;
        const float4 h = ld4((lane & 1) ? &T->new_hi[at] : &T->old_hi[at]);
        const float4 l = ld4((lane & 1) ? &T->new_lo[at] : &T->old_lo[at]);
        double x = (double)h.x + (double)l.x, y = (double)h.y + (double)l.y, z = (double)h.z + (double)l.z;
        if (cimg) {
            // the atom's image nearest the centre (atoms are wrapped one by one)
            x -= rint(x - (double)cx);
            y -= rint(y - (double)cy);
            z -= rint(z - (double)cz);
        }
        ta.x[lane] = x;
        ta.y[lane] = y;
        ta.z[lane] = z;
        ta.rb[lane] = __float_as_int(h.w) * c.M;
    }
    scan_sync<NW>();
    const float reach = surv + *a.drift + 1e-6f;
    const float reach2 = reach * reach;
    const int nc = a.nc;
    const float fnc = (float)nc, inv_nc = 1.0f / fnc;
    // rows: z in [lz, hz], y in [ly, hy] (unwrapped cell indices)
    const int lz = (int)floorf((cz - reach) * fnc), hz = min((int)floorf((cz + reach) * fnc), lz + nc - 1);
    const int ly = (int)floorf((cy - reach) * fnc), hy = min((int)floorf((cy + reach) * fnc), ly + nc - 1);
    const int cnty = hy - ly + 1;
    const int nrows = (hz - lz + 1) * cnty;
    const int my_rows = nrows > wsub ? (nrows - wsub + NW - 1) / NW : 0;
    const unsigned long long lt = (1ull << lane) - 1ull;
    double e = 0.0, s = 0.0;
    int nlist = 0;
    for (int sp = 0; sp < my_rows; sp += 64) {
        // row sp + lane: slot ranges [b0, b0 + n0) and [b1, b1 + n1)
        const int sid = sp + lane;
        int b0 = 0, n0 = 0, b1 = 0, n1 = 0;
        if (sid < my_rows) {
            const int r = wsub + NW * sid;
            const int zu = lz + r / cnty, yu = ly + r % cnty;
            const float gz = gap_to_cell(cz, zu, inv_nc), gy = gap_to_cell(cy, yu, inv_nc);
            const float d2 = gz * gz + gy * gy;
            if (d2 < reach2) {
                const float half = sqrtf(reach2 - d2) * 1.0000005f + 1e-7f;
                int l = (int)floorf((cx - half) * fnc);
                int h = (int)floorf((cx + half) * fnc);
                int lo, cnt;
                if (h - l + 1 >= nc) {
                    lo = 0;
                    cnt = nc;
                } else {
                    lo = ((l % nc) + nc) % nc;
                    cnt = h - l + 1;
                }
                const int zz = ((zu % nc) + nc) % nc, yy = ((yu % nc) + nc) % nc;
                const int rowc = (zz * nc + yy) * nc;
                const int e0 = min(lo + cnt, nc);
                b0 = ldg(a.cstart + rowc + lo);
                n0 = ldg(a.cstart + rowc + e0) - b0;
                if (lo + cnt > nc) {
                    b1 = ldg(a.cstart + rowc);
                    n1 = ldg(a.cstart + rowc + lo + cnt - nc) - b1;
                }
            }
        }
        const int len = n0 + n1;
        // inclusive prefix of the lengths across the wave
        int incl = len;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(incl, o);
            if (lane >= o) incl += y;
        }
        const int total = __shfl(incl, 63);
        const int excl = incl - len;
        if (a.count && lane == 0) atomicAdd(&cnt[0], (unsigned long long)total);  // measurement only
        // two candidates per lane per trip, so two loads are in flight
        for (int c0 = 0; c0 < total; c0 += 128) {
            int sl[2];
            bool live[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int cidx = c0 + 64 * h + lane;
                // row of candidate cidx: the largest j with excl_j <= cidx
                // (binary search over lanes; every lane takes part in the shuffles)
                const int cc = min(cidx, total - 1);
                int j = 0;
#pragma unroll
                for (int step = 32; step > 0; step >>= 1) {
                    const int cand = j + step;
                    const int ex = __shfl(excl, cand < 64 ? cand : 63);
                    if (cand < 64 && ex <= cc) j = cand;
                }
                // every lane shuffles every value: no shuffle under a branch
                const int off = cc - __shfl(excl, j);
                const int jn0 = __shfl(n0, j);
                const int jb0 = __shfl(b0, j);
                const int jb1 = __shfl(b1, j);
                sl[h] = off < jn0 ? jb0 + off : jb1 + (off - jn0);
                live[h] = cidx < total;
            }
            float4 q[2], ql[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                q[h] = ld4(a.spos4 + sl[h]);
                ql[h] = ld4(a.sposlo + sl[h]);
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                float dx = q[h].x - cx, dy = q[h].y - cy, dz = q[h].z - cz;
                dx -= rintf(dx);
                dy -= rintf(dy);
                dz -= rintf(dz);
                const bool mine = __float_as_int(ql[h].w) == tunit;
                const bool hit = live[h] && !mine && fmaf(dz, dz, fmaf(dy, dy, dx * dx)) < surv2;
                const unsigned long long bal = __ballot(hit);
                if (a.count && lane == 0) atomicAdd(&cnt[1], (unsigned long long)__popcll(bal));
                if (hit) {
                    const int idx = nlist + __popcll(bal & lt);
                    list[idx] = q[h];
                    listlo[idx] = ql[h];
                }
                nlist += __popcll(bal);
            }
            if (nlist > CS_LIST - 128) {
                __builtin_amdgcn_wave_barrier();
                cell_flush_any<MAXNU>(cimg, c, ta, tna, list, listlo, nlist, lane, e, s, cx, cy, cz);
                __builtin_amdgcn_wave_barrier();
                nlist = 0;
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
    cell_flush_any<MAXNU>(cimg, c, ta, tna, list, listlo, nlist, lane, e, s, cx, cy, cz);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        e += __shfl_xor(e, o);
        s += __shfl_xor(s, o);
    }
    if (NW == 1) {
        if (lane == 0) {
            const nd::Trial &T = a.trials[k];
            a.dE0[k] = T.dintra + e;
            a.S0[k] = T.sintra + s;
        }
        return;
    }
    if (lane == 0) {
        red[2 * wsub] = e;
        red[2 * wsub + 1] = s;
    }
    scan_sync<NW>();
    if (wsub == 0 && lane == 0) {
        double E = red[0], S = red[1];
        for (int w = 1; w < NW; ++w) {
            E += red[2 * w];
            S += red[2 * w + 1];
        }
        const nd::Trial &T = a.trials[k];
        a.dE0[k] = T.dintra + E;
        a.S0[k] = T.sintra + S;
    }
}

// Blocks of one launch, in dispatch order: the previous batch's final sums
// (when the decision left them), the proposals of the next batch (its units
// are disjoint from this batch's) and the in-batch corrections, which are
// few and long, so they start first; padding to a
// multiple of 8; then the cell scans, 4/NW trials per block (NW waves
// each, sharing the staged tables), block b of them on XCD b mod 8 taking
// the trials whose centre lies in z-slab b mod 8, so each XCD's L2 holds
// about one slab of the cell data instead of all of it.
__host__ __device__ inline int scan_front_blocks(int kb_corr, int kb_next, int n_fin)
{
    const int n = n_fin + (kb_next + 255) / 256 + (kb_corr + CORR_TPB - 1) / CORR_TPB;
    return (n + N_SLAB - 1) / N_SLAB * N_SLAB;
}

static_assert(sizeof(CorrScratch) <= 2 * sizeof(float4) * CS_LIST, "correction scratch must fit a wave's survivor lists");

template <int MAXNU, int NW>
__device__ __forceinline__ void scan_corr_body(const CellScanArgs &a, const CorrArgs &ca, const ProposeArgs &next,
                                               const FinalArgs &fin, int bx)
{
    constexpr int TPB = 4 / NW;  // trials per block
    extern __shared__ __align__(16) float s_tab[];  // [P][n_pts]
    __shared__ int s_prow[16];
    __shared__ float4 s_list[4][2][CS_LIST];  // per wave: survivors hi, then lo
    __shared__ TrialAtoms s_ta[TPB];
    __shared__ double s_red[TPB][2 * NW];
    __shared__ unsigned long long s_cnt[2];  // candidates, survivors (measurement)
    const int tid = threadIdx.x;
    const int n_fin = fin.kb > 0 ? 1 : 0;
    const int n_prop = (next.kb + 255) / 256;
    const int n_corr = (ca.kb + CORR_TPB - 1) / CORR_TPB;
    const int n_front = scan_front_blocks(ca.kb, next.kb, n_fin);
    if (bx < n_fin) {
        final_body(fin, reinterpret_cast<unsigned char *>(&s_list[0][0][0]));
        return;
    }
    if (bx < n_fin + n_prop) {
        const int k = (bx - n_fin) * 256 + tid;
        if (k < next.kb) propose_one(next, k);
        return;
    }
    if (bx < n_fin + n_prop + n_corr) {
        if (tid < a.M * a.M) s_prow[tid] = nd::pair_index(tid / a.M, tid % a.M, a.M) * a.n_pts;
        __syncthreads();
        const PairCtx c{ca.tab, s_prow, ca.M, ca.n_pts, ca.rcf2_filter, ca.rcf2, ca.tscale};
        CorrScratch &cs = *reinterpret_cast<CorrScratch *>(&s_list[tid >> 6][0][0]);
        // trials interleaved over the correction blocks (late trials are the
        // heavy ones)
        const int k = (tid >> 6) * n_corr + (bx - n_fin - n_prop);
        if (k < ca.kb) corr_trial<MAXNU>(ca, c, k, tid & 63, cs);
        return;
    }
    if (bx < n_front) return;
    const int sb = bx - n_front;
    const int slab = sb & (N_SLAB - 1);
    const int cnt = a.slab[slab];
    const int i0 = (sb >> 3) * TPB;
    if (i0 >= cnt) return;
    const int P = a.M * (a.M + 1) / 2;
    nd::stage_floats<256>(s_tab, a.tab, P * a.n_pts);
    if (tid < a.M * a.M) s_prow[tid] = nd::pair_index(tid / a.M, tid % a.M, a.M) * a.n_pts;
    if (tid < 2) s_cnt[tid] = 0ull;
    __syncthreads();  // tables staged
    const PairCtx c{s_tab, s_prow, a.M, a.n_pts, a.rcf2_filter, a.rcf2, a.tscale};
    const int32_t *lst = a.slab + N_SLAB + slab * a.kcap;
    const int wave = tid >> 6, grp = wave / NW, wsub = wave % NW;
    const int stride = a.per_slab * TPB;
    // rounds of the block (the same for all its waves): group 0 has the most
    const int rounds = (cnt - i0 + stride - 1) / stride;
    for (int it = 0; it < rounds; ++it) {
        const int i = i0 + grp + it * stride;
        const bool active = i < cnt;
        scan_cells_group<MAXNU, NW>(a, c, active ? lst[i] : 0, active, wsub, tid & 63, s_list[wave][0],
                                     s_list[wave][1], s_red[grp], s_ta[grp], s_cnt);
    }
    if (a.count) {
        __syncthreads();
        if (tid < 2) atomicAdd(a.count + tid, s_cnt[tid]);
    }
}

template <int MAXNU, int NW>
__global__ __launch_bounds__(256, (MAXNU <= 3 ? 4 : (MAXNU <= 4 ? 3 : 2))) void k_mc_scan_corr(CellScanArgs a, CorrArgs ca, ProposeArgs next,
                                                                                         FinalArgs fin)
{
    scan_corr_body<MAXNU, NW>(a, ca, next, fin, blockIdx.x);
}

// ---------------------------------------------------------------- decide
constexpr int DEC_THREADS = 1024;
static_assert(KMAX == 2 * DEC_THREADS, "a decide thread holds two trial rows");

struct DecideArgs {
    float *xyz;
    float4 *pos4;
    float4 *poslo;
    double *E;
    const nd::Trial *trials;
    const double *dE0, *S0;
    const int32_t *corr_n, *corr_ptr, *pool_m;
    const float *corr_s;
    const double2 *corr_b;
    const double *pool_c;
    int32_t *ovf_fill;
    // cell copies (null when cells are not in use)
    const int32_t *cell_slot;
    float4 *spos4, *sposlo;
    const float4 *sref;
    float *drift;
    int32_t *slab_cnt;  // [N_SLAB] slab counts of this batch's buffer, cleared here
    const int4 *head;   // [kb] unit, first atom, atoms of each trial
    const double *hthr; // [kb] acceptance thresholds
    int N, kb, max_na;
    double kT, tie_rel;
    long long *counters;  // [0] accepted, [1] near ties
    double *dsum;
    double *tr_dE, *tr_sabs;
    uint8_t *tr_acc;
    int32_t *tr_unit;
    // defer: the final dE sums, counters and trace are left to a later launch
    // (k_mc_final's body); the decision stores what they need
    int defer;
    uint8_t *acc_out;  // [kb] 1: accepted (written when not null)
    double *thr_out;   // [kb] acceptance threshold -kT ln u
    // running histogram: the unit of each accepted trial k is tagged
    // tag_base + k (null when no histogram is tracked)
    long long *moved_tag;
    long long tag_base;
    // blocks 1 .. n_cm of the decision launch commit the trials accepted in
    // the first pass, and block 0 the rest (0: block 0 commits all)
    int n_cm;
};

// exclusive prefix sum over the block of one value per thread
__device__ __forceinline__ int block_exscan(int v, int *s_wave)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_wave[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int w = 0; w < DEC_THREADS / 64; ++w) {
            const int t = s_wave[w];
            s_wave[w] = acc;
            acc += t;
        }
        s_wave[DEC_THREADS / 64] = acc;
    }
    __syncthreads();
    return s_wave[wave] + x - v;
}

__device__ __forceinline__ bool metropolis(double e, double thr) { return e <= 0.0 || e < thr; }

constexpr unsigned char ST_OPEN = 0, ST_REJ = 1, ST_ACC = 2;
constexpr int ST_NONE = 3;  // an entry with no pair term (m < 0)

// The first pass's state of a trial from per-trial values only: ΔE⁰, the
// threshold and the bracket summary of its entries (lo, hi), (mag, count).
// Without entries the test is exact; otherwise the trial is decided when
// the test gives the same answer at both ends of the bracket, with a margin
// far above the rounding of the sums.  The commit blocks evaluate the same
// function on the same values, so they agree with the decision bit for bit.
__device__ __forceinline__ unsigned char first_pass_state(double e0, double thr, double2 blh, double2 bmc)
{
    if (!(bmc.y > 0.0)) return metropolis(e0, thr) ? ST_ACC : ST_REJ;
    const double eps = 1e-12 * (fabs(e0) + bmc.x);
    const bool alo = metropolis(e0 + blh.x - eps, thr), ahi = metropolis(e0 + blh.y + eps, thr);
    return alo == ahi ? (alo ? ST_ACC : ST_REJ) : ST_OPEN;
}

// Correction entries of trial k: fixed slots [k CORR_CAP, k CORR_CAP + n)
// when n <= CORR_CAP (read with wide loads, all at once), else n entries at
// ptr in the overflow area.  f(m, c) is called for every entry in order.
template <class F>
__device__ __forceinline__ void for_entries(const int32_t *pool_m, const double *pool_c, int k, int n, int ptr, F &&f)
{
    if (n <= CORR_CAP) {
        int m[CORR_CAP];
        double c[CORR_CAP];
        const int4 *pm = reinterpret_cast<const int4 *>(pool_m + (size_t)k * CORR_CAP);
        const double2 *pc = reinterpret_cast<const double2 *>(pool_c + (size_t)k * CORR_CAP);
#pragma unroll
        for (int i = 0; i < CORR_CAP / 4; ++i) {
            if (4 * i < n) {
                const int4 v = ld_i4(pm + i);
                m[4 * i] = v.x;
                m[4 * i + 1] = v.y;
                m[4 * i + 2] = v.z;
                m[4 * i + 3] = v.w;
            }
        }
#pragma unroll
        for (int i = 0; i < CORR_CAP / 2; ++i) {
            if (2 * i < n) {
                const double2 v = ld_d2(pc + i);
                c[2 * i] = v.x;
                c[2 * i + 1] = v.y;
            }
        }
#pragma unroll
        for (int i = 0; i < CORR_CAP; ++i)
            if (i < n) f(m[i], c[i]);
    } else {
        for (int i = 0; i < n; ++i) f(ldg(pool_m + ptr + i), ldg(pool_c + ptr + i));
    }
}

// As for_entries, with f(st, c) taking the state of the earlier trial m
// (ST_NONE when m < 0) instead of m.  For n <= CORR_CAP every state is read
// from LDS before any is used (indexes clamped, no branches), so the reads
// are in flight together rather than one after another.
template <class F>
__device__ __forceinline__ void for_entries_st(const int32_t *pool_m, const double *pool_c, const unsigned char *st,
                                               int k, int n, int ptr, F &&f)
{
    if (n <= CORR_CAP) {
        int m[CORR_CAP];
        double c[CORR_CAP];
        const int4 *pm = reinterpret_cast<const int4 *>(pool_m + (size_t)k * CORR_CAP);
        const double2 *pc = reinterpret_cast<const double2 *>(pool_c + (size_t)k * CORR_CAP);
#pragma unroll
        for (int i = 0; i < CORR_CAP / 4; ++i) {
            int4 v = make_int4(-1, -1, -1, -1);
            if (4 * i < n) v = ld_i4(pm + i);
            m[4 * i] = 4 * i < n ? v.x : -1;
            m[4 * i + 1] = 4 * i + 1 < n ? v.y : -1;
            m[4 * i + 2] = 4 * i + 2 < n ? v.z : -1;
            m[4 * i + 3] = 4 * i + 3 < n ? v.w : -1;
        }
#pragma unroll
        for (int i = 0; i < CORR_CAP / 2; ++i) {
            if (2 * i < n) {
                const double2 v = ld_d2(pc + i);
                c[2 * i] = v.x;
                c[2 * i + 1] = v.y;
            }
        }
#pragma unroll
        for (int i = 0; i < CORR_CAP; ++i) {
            const int s = st[m[i] >= 0 ? m[i] : 0];
            m[i] = m[i] >= 0 ? s : ST_NONE;
        }
#pragma unroll
        for (int i = 0; i < CORR_CAP; ++i)
            if (i < n) f(m[i], c[i]);
    } else {
        for (int i = 0; i < n; ++i) {
            const int mi = ldg(pool_m + ptr + i);
            f(mi >= 0 ? (int)st[mi] : ST_NONE, ldg(pool_c + ptr + i));
        }
    }
}

// The open trials s_open[0 .. n_open) of a batch, resolved by one wave:
// lane l takes trial s_open[l] and reads its entries once.  Entries whose
// earlier trial is already decided are summed into a base (ΔE⁰ plus the
// accepted ones), and those whose trial is still open are kept in LDS
// (kept entry i of lane l at [i][l]); each pass then reads only the states
// of the kept entries, until the trial is decided.  Each pass decides at
// least the earliest open trial (its earlier trials are all decided, so its
// dE is exact), so at most n_open passes run; states written in a pass are
// visible to the wave in the next.  A trial with more entries than the
// fixed slots (rare) reads all of them from memory in every pass.  `pool`
// holds 64 CORR_CAP (int, double).
constexpr int RESOLVE_POOL_BYTES = 64 * CORR_CAP * (int)(sizeof(int) + sizeof(double));

__device__ __forceinline__ void resolve_in_wave(const DecideArgs &a, const double *s_e, const double *s_u,
                                                const int *s_n, const int *s_ptr, unsigned char *s_st,
                                                const unsigned short *s_open, int n_open, int lane,
                                                unsigned char *pool)
{
    double *ec = reinterpret_cast<double *>(pool);        // [CORR_CAP][64]
    int *em = reinterpret_cast<int *>(ec + CORR_CAP * 64);  // [CORR_CAP][64]
    const bool has = lane < n_open;
    const int k = has ? s_open[lane] : 0;
    const int nk = has ? s_n[k] : 0, pk = s_ptr[k];
    const bool big = nk > CORR_CAP;
    const double e0 = s_e[k], thr = s_u[k];
    double eb = e0, mag = fabs(e0);  // base and scale of the kept entries' sums
    int nkeep = 0;
    if (!big) {
        // every fixed slot of trial k is read (they are always allocated;
        // those past nk are not used), with no condition between the loads,
        // so that all of them are in flight together; then the states of
        // all the entries' trials, also together
        const int4 *pm = reinterpret_cast<const int4 *>(a.pool_m + (size_t)k * CORR_CAP);
        const double2 *pc = reinterpret_cast<const double2 *>(a.pool_c + (size_t)k * CORR_CAP);
        int4 vm[CORR_CAP / 4];
        double2 vc[CORR_CAP / 2];
#pragma unroll
        for (int i = 0; i < CORR_CAP / 4; ++i) vm[i] = ld_i4(pm + i);
#pragma unroll
        for (int i = 0; i < CORR_CAP / 2; ++i) vc[i] = ld_d2(pc + i);
        int mm[CORR_CAP], st[CORR_CAP];
#pragma unroll
        for (int i = 0; i < CORR_CAP / 4; ++i) {
            mm[4 * i] = 4 * i < nk ? vm[i].x : -1;
            mm[4 * i + 1] = 4 * i + 1 < nk ? vm[i].y : -1;
            mm[4 * i + 2] = 4 * i + 2 < nk ? vm[i].z : -1;
            mm[4 * i + 3] = 4 * i + 3 < nk ? vm[i].w : -1;
        }
#pragma unroll
        for (int i = 0; i < CORR_CAP; ++i) st[i] = s_st[mm[i] >= 0 ? mm[i] : 0];
        // fold the decided entries into the base; keep the open ones, in
        // order.  No branches: every entry is written at the next kept
        // slot, which only an open one advances (nkeep <= i < CORR_CAP)
#pragma unroll
        for (int i = 0; i < CORR_CAP; ++i) {
            const double cv = (i & 1) ? vc[i >> 1].y : vc[i >> 1].x;
            const bool v = mm[i] >= 0;
            mag += v ? fabs(cv) : 0.0;
            eb += v && st[i] == ST_ACC ? cv : 0.0;
            em[nkeep * 64 + lane] = mm[i];
            ec[nkeep * 64 + lane] = cv;
            nkeep += v && st[i] == ST_OPEN ? 1 : 0;
        }
    }
    bool open = has;
    for (int pass = 0; pass < 64; ++pass) {
        if (__ballot(open) == 0ull) break;
        unsigned char d = ST_OPEN;
        if (open) {
            double e = eb, lo = 0.0, hi = 0.0, sc = mag;
            bool all = true;
            auto visit = [&](int st, double cv) {
                const bool op = st == ST_OPEN;
                e += st == ST_ACC ? cv : 0.0;
                all &= !op;
                lo += op ? fmin(cv, 0.0) : 0.0;
                hi += op ? fmax(cv, 0.0) : 0.0;
            };
            if (!big) {
                // the kept entries, four at a time (their reads in flight together)
                for (int i0 = 0; i0 < nkeep; i0 += 4) {
                    int mm[4], st[4];
                    double cc[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int j = i0 + i < nkeep ? i0 + i : i0;
                        mm[i] = em[j * 64 + lane];
                        cc[i] = ec[j * 64 + lane];
                    }
#pragma unroll
                    for (int i = 0; i < 4; ++i) st[i] = s_st[mm[i]];
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (i0 + i < nkeep) visit(st[i], cc[i]);
                }
            } else {
                e = e0;
                sc = fabs(e0);
                for (int i = 0; i < nk; ++i) {
                    const int mi = ldg(a.pool_m + pk + i);
                    const double cv = ldg(a.pool_c + pk + i);
                    visit(mi >= 0 ? (int)s_st[mi] : ST_NONE, cv);
                    sc += mi >= 0 ? fabs(cv) : 0.0;
                }
            }
            if (all) {
                d = metropolis(e, thr) ? ST_ACC : ST_REJ;
            } else {
                const double eps = 1e-12 * sc;
                const bool alo = metropolis(e + lo - eps, thr), ahi = metropolis(e + hi + eps, thr);
                if (alo == ahi) d = alo ? ST_ACC : ST_REJ;
            }
        }
        // every lane has read this pass's states before any is written
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (open && d != ST_OPEN) {
            s_st[k] = d;
            open = false;
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

// One atom of an accepted trial, committed in two halves: the loads (the
// trial record's new position and, with cell lists, the atom's slot in the
// sorted copies and its cell reference), then the stores of the new position
// to xyz, pos4/poslo and the sorted copies, with the atom's displacement from
// the cell reference taken into dmax.  Each trial writes only its own atoms,
// so the order is free.
struct CommitItem {
    int i, slot, unit, at;
    float4 hi, lo, ref;
    float x[3];
};

__device__ __forceinline__ void commit_load(const DecideArgs &a, int k, int at, int a0, CommitItem &c)
{
    const nd::Trial &T = a.trials[k];
    c.i = a0 + at;
    c.at = at;
    c.unit = ldg(&T.unit);
    c.hi = ld4(&T.new_hi[at]);
    c.lo = ld4(&T.new_lo[at]);
    c.x[0] = ldg(&T.new_x[at][0]);
    c.x[1] = ldg(&T.new_x[at][1]);
    c.x[2] = ldg(&T.new_x[at][2]);
    c.slot = 0;
    c.ref = make_float4(0.f, 0.f, 0.f, 0.f);
    if (a.cell_slot) {
        c.slot = ldg(a.cell_slot + c.i);
        c.ref = ld4(a.sref + c.i);
    }
}

__device__ __forceinline__ void commit_store(const DecideArgs &a, int k, const CommitItem &c, float &dmax)
{
    const int i = c.i;
    if (a.moved_tag && c.at == 0) a.moved_tag[c.unit] = a.tag_base + k;
    a.xyz[i] = c.x[0];
    a.xyz[a.N + i] = c.x[1];
    a.xyz[2 * a.N + i] = c.x[2];
    a.pos4[i] = c.hi;
    a.poslo[i] = c.lo;
    if (a.cell_slot) {
        a.spos4[c.slot] = c.hi;
        a.sposlo[c.slot] = c.lo;
        float dx = c.hi.x - c.ref.x, dy = c.hi.y - c.ref.y, dz = c.hi.z - c.ref.z;
        dx -= rintf(dx);
        dy -= rintf(dy);
        dz -= rintf(dz);
        dmax = fmaxf(dmax, sqrtf(dx * dx + dy * dy + dz * dz) * 1.0001f + 1e-6f);
    }
}

// Commit the trials list[0 .. n) (only those in state ST_ACC when `filter`):
// one item per (trial, atom), consecutive items on consecutive threads t of
// nt (a trial's atoms share cache lines), the loads of four items issued
// together.
__device__ __forceinline__ void commit_trials(const DecideArgs &a, const unsigned short *list, int n, bool filter,
                                              const unsigned char *s_st, const int *s_a0, const unsigned char *s_na,
                                              int t, int nt, float &dmax)
{
    const int max_na = a.max_na;
    const int n_items = n * max_na;
    constexpr int CU = 4;
    for (int base = t; base < n_items; base += CU * nt) {
        int kk[CU];
        CommitItem ci[CU];
#pragma unroll
        for (int u = 0; u < CU; ++u) {
            const int it = base + u * nt;
            kk[u] = -1;
            if (it < n_items) {
                const int li = it / max_na, at = it - li * max_na;
                const int k = list[li];
                if (at < s_na[k] && (!filter || s_st[k] == ST_ACC)) {
                    kk[u] = k;
                    commit_load(a, k, at, s_a0[k], ci[u]);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < CU; ++u)
            if (kk[u] >= 0) commit_store(a, kk[u], ci[u], dmax);
    }
}

// Decide batch b -- acc_k = metropolis(dE0_k + sum_{m<k} acc_m C_km), which
// is the sequential chain -- and commit it.
//
// A trial whose earlier interacting trials are all decided gets its exact
// dE and is decided; otherwise its dE lies between the sums with the open
// terms' negative (resp. positive) parts, and when the test gives the same
// answer at both ends (with a margin far above the rounding of the sums)
// that is its decision whatever the open trials do.  The first pass needs
// no other decision and runs while the entries are loaded; later passes
// visit only the open trials.  Every pass decides at least the earliest
// open trial, so the loop ends; decisions do not depend on the pass in which
// they are made, so the result is deterministic and equals the in-order
// chain.  When `next.kb` > 0 the next batch is proposed afterwards (used
// when its units may overlap this batch's).
__device__ __forceinline__ void decide_body(const DecideArgs &a, const ProposeArgs &next, unsigned char *pool)
{
    __shared__ double s_e[KMAX];      // dE0, then the final dE
    __shared__ double s_u[KMAX];      // acceptance threshold -kT ln u
    __shared__ double s_S[KMAX];      // sum of |U| over the trial's pair terms
    __shared__ int s_n[KMAX];         // entries to read (0 when none has m >= 0)
    __shared__ int s_ptr[KMAX];
    __shared__ int s_a0[KMAX];
    __shared__ unsigned char s_na[KMAX];
    __shared__ unsigned char s_st[KMAX];
    __shared__ unsigned char s_nx[KMAX];
    __shared__ unsigned short s_open[KMAX];
    __shared__ int s_wave[DEC_THREADS / 64 + 1];
    __shared__ double s_red_d[DEC_THREADS / 64];
    __shared__ long long s_red_a[DEC_THREADS / 64], s_red_t[DEC_THREADS / 64];
    __shared__ float s_red_f[DEC_THREADS / 64];
    __shared__ unsigned short s_alist[KMAX];  // trials accepted in the first pass, then the first open list
    __shared__ int s_nopen, s_nacc0;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int kb = a.kb;

    if (kb > 0) {
        if (tid == 0) {
            s_nopen = 0;
            s_nacc0 = 0;
        }
        // trial data and the first pass (needs no other decision): a thread
        // holds trials tid and tid + DEC_THREADS and issues all their loads
        // before using any; the bracket of the open terms is the summary the
        // correction step wrote, so no entry is read here
        int my_open = 0;
        int n[2], ptr[2];
        double e0[2], thr_k[2], S[2];
        double2 blh[2], bmc[2];
        int4 ids[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            // past kb the last trial is read again (unused): no condition
            // between the loads, so all of them are in flight together
            const int k = min(tid + h * DEC_THREADS, kb - 1);
            n[h] = ldg(a.corr_n + k);
            ptr[h] = ldg(a.corr_ptr + k);
            e0[h] = ldg(a.dE0 + k);
            ids[h] = ld_i4(a.head + k);  // compact per-trial copies: coalesced loads
            thr_k[h] = ldg(a.hthr + k);
            S[h] = ldg(a.S0 + k) + (double)ldg(a.corr_s + k);
            blh[h] = ld_d2(a.corr_b + 2 * k);
            bmc[h] = ld_d2(a.corr_b + 2 * k + 1);
        }
        __syncthreads();  // s_nopen cleared (the loads above are in flight meanwhile)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            // k < KMAX: the LDS rows past kb are written too (never read),
            // so only the global stores wait on k < kb
            const int k = tid + h * DEC_THREADS;
            const bool in = k < kb;
            const double thr = thr_k[h];
            const bool any = bmc[h].y > 0.0;
            const unsigned char d = in ? first_pass_state(e0[h], thr, blh[h], bmc[h]) : ST_REJ;
            s_e[k] = e0[h];
            s_u[k] = thr;
            if (in && a.defer) {
                a.thr_out[k] = thr;
                if (a.tr_unit) a.tr_unit[k] = ids[h].x;
            }
            s_S[k] = S[h];
            s_n[k] = any ? n[h] : 0;
            s_ptr[k] = ptr[h];
            s_a0[k] = ids[h].y;
            s_na[k] = (unsigned char)ids[h].z;
            s_st[k] = d;
            my_open += d == ST_OPEN;
            // the open and the accepted trials listed, in any order (one
            // LDS atomic per wave for each list)
            const unsigned long long mo = __ballot(d == ST_OPEN), ma = __ballot(d == ST_ACC);
            const unsigned long long lt = (1ull << lane) - 1ull;
            int bo = 0, ba = 0;
            if (lane == 0) {
                if (mo) bo = atomicAdd(&s_nopen, __popcll(mo));
                if (ma) ba = atomicAdd(&s_nacc0, __popcll(ma));
            }
            bo = __shfl(bo, 0);
            ba = __shfl(ba, 0);
            if (d == ST_OPEN) s_open[bo + __popcll(mo & lt)] = (unsigned short)k;
            if (d == ST_ACC) s_alist[ba + __popcll(ma & lt)] = (unsigned short)k;
        }
        if (tid == 0) *a.ovf_fill = 0;  // overflow area is free for the next batch
        if (tid < N_SLAB) a.slab_cnt[tid] = 0;  // the scan of this batch is done with its lists
        __syncthreads();
        const int n_open0 = s_nopen, n_acc0 = s_nacc0;

        // Later passes over the open trials, and the commits.  Trials
        // accepted in the first pass are committed at once: nothing in this
        // launch reads the positions they write (the decisions use dE0 and
        // the entries; the next batch's corrections read trial records).
        // Few open trials (the usual case): one wave resolves them, a lane
        // per trial, its passes synchronised within the wave only, while the
        // other waves commit.  Many: the commits, then passes in which every
        // thread takes part, separated by barriers.
        // With commit blocks, the waves other than the resolving one read
        // the commit data of the open trials' atoms meanwhile (one atom per
        // thread) and store it after the barrier if the trial was accepted.
        float dmax = 0.0f;
        const bool pre = n_open0 <= 64 && a.n_cm > 0 && n_open0 * a.max_na <= DEC_THREADS - 64;
        int pk = -1;
        CommitItem pci;
        if (n_open0 <= 64) {
            if (wave == 0) {
                if (n_open0 > 0) resolve_in_wave(a, s_e, s_u, s_n, s_ptr, s_st, s_open, n_open0, lane, pool);
            } else if (a.n_cm == 0) {
                commit_trials(a, s_alist, n_acc0, false, s_st, s_a0, s_na, tid - 64, DEC_THREADS - 64, dmax);
            } else if (pre) {
                const int it = tid - 64, li = it / a.max_na, at = it - li * a.max_na;
                if (li < n_open0) {
                    const int k = s_open[li];
                    if (at < s_na[k]) {
                        pk = k;
                        commit_load(a, k, at, s_a0[k], pci);
                    }
                }
            }
            __syncthreads();
            // the open trials are all decided
            if (pk >= 0 && s_st[pk] == ST_ACC) commit_store(a, pk, pci, dmax);
        } else {
            if (a.n_cm == 0) commit_trials(a, s_alist, n_acc0, false, s_st, s_a0, s_na, tid, DEC_THREADS, dmax);
            for (int i = tid; i < n_open0; i += DEC_THREADS) s_alist[n_acc0 + i] = s_open[i];
        }
        for (; n_open0 > 64;) {
            // list the open trials (in trial order)
            const int off = block_exscan(my_open, s_wave);  // ends with a barrier
            const int n_open = s_wave[DEC_THREADS / 64];
            if (n_open == 0) break;
            {
                int o = off;
                for (int k = tid; k < kb; k += DEC_THREADS)
                    if (s_st[k] == ST_OPEN) s_open[o++] = (unsigned short)k;
            }
            __syncthreads();
            for (int i = tid; i < n_open; i += DEC_THREADS) {
                const int k = s_open[i];
                double e = s_e[k], lo = 0.0, hi = 0.0, mag = fabs(e);
                bool all = true;
                for_entries_st(a.pool_m, a.pool_c, s_st, k, s_n[k], s_ptr[k], [&](int st, double c) {
                    const bool open = st == ST_OPEN;
                    e += st == ST_ACC ? c : 0.0;
                    all &= !open;
                    lo += open ? fmin(c, 0.0) : 0.0;
                    hi += open ? fmax(c, 0.0) : 0.0;
                    mag += st != ST_NONE ? fabs(c) : 0.0;
                });
                const double thr = s_u[k];
                unsigned char d = ST_OPEN;
                if (all) {
                    d = metropolis(e, thr) ? ST_ACC : ST_REJ;
                } else {
                    const double eps = 1e-12 * mag;
                    const bool alo = metropolis(e + lo - eps, thr), ahi = metropolis(e + hi + eps, thr);
                    if (alo == ahi) d = alo ? ST_ACC : ST_REJ;
                }
                s_nx[k] = d;
            }
            __syncthreads();
            my_open = 0;
            for (int i = tid; i < n_open; i += DEC_THREADS) {
                const int k = s_open[i];
                s_st[k] = s_nx[k];
            }
            __syncthreads();
            for (int k = tid; k < kb; k += DEC_THREADS) my_open += s_st[k] == ST_OPEN;
        }

        // the first pass's open trials that were accepted (already done when
        // their commit data was read during the resolve)
        if (!pre) {
            if (n_open0 <= 64)
                commit_trials(a, s_open, n_open0, true, s_st, s_a0, s_na, tid, DEC_THREADS, dmax);
            else
                commit_trials(a, s_alist + n_acc0, n_open0, true, s_st, s_a0, s_na, tid, DEC_THREADS, dmax);
        }

        // final dE (the same in-order sum as an exact decision), counters, trace
        double dsum = 0.0;
        long long nacc = 0, ntie = 0;
        if (a.acc_out)
            for (int k = tid; k < kb; k += DEC_THREADS) a.acc_out[k] = s_st[k] == ST_ACC ? 1 : 0;
        for (int k = tid; k < kb && !a.defer; k += DEC_THREADS) {
            double e = s_e[k];
            for_entries_st(a.pool_m, a.pool_c, s_st, k, s_n[k], s_ptr[k],
                           [&](int st, double c) { e += st == ST_ACC ? c : 0.0; });
            const bool acc = s_st[k] == ST_ACC;
            const double S = s_S[k];
            const double thr = s_u[k];
            // |ln u + dE/kT| < tie_rel S / kT, i.e. |dE - (-kT ln u)| < tie_rel S (u > 0)
            if (thr != 745.13321910194122 * a.kT && fabs(e - thr) < a.tie_rel * S) ++ntie;
            if (acc) {
                ++nacc;
                dsum += e;
            }
            if (a.tr_dE) a.tr_dE[k] = e;
            if (a.tr_sabs) a.tr_sabs[k] = S;
            if (a.tr_acc) a.tr_acc[k] = acc ? 1 : 0;
            if (a.tr_unit) a.tr_unit[k] = a.trials[k].unit;
        }
        if (a.defer) {
            // the sums wait for a later launch; the drift is a maximum, so
            // each wave adds its own with one atomic and no block reduction
            for (int o2 = 32; o2 > 0; o2 >>= 1) dmax = fmaxf(dmax, __shfl_xor(dmax, o2));
            if (lane == 0 && a.drift && dmax > 0.0f)
                atomicMax(reinterpret_cast<unsigned int *>(a.drift), __float_as_uint(dmax));
        } else {
            for (int o2 = 32; o2 > 0; o2 >>= 1) {
                dsum += __shfl_xor(dsum, o2);
                nacc += __shfl_xor(nacc, o2);
                ntie += __shfl_xor(ntie, o2);
                dmax = fmaxf(dmax, __shfl_xor(dmax, o2));
            }
            if (lane == 0) {
                s_red_d[wave] = dsum;
                s_red_a[wave] = nacc;
                s_red_t[wave] = ntie;
                s_red_f[wave] = dmax;
            }
            __syncthreads();
            if (tid == 0) {
                double d = 0.0;
                long long na = 0, nt = 0;
                float dm = 0.0f;
                for (int w = 0; w < DEC_THREADS / 64; ++w) {
                    d += s_red_d[w];
                    na += s_red_a[w];
                    nt += s_red_t[w];
                    dm = fmaxf(dm, s_red_f[w]);
                }
                *a.E += d;
                *a.dsum += d;
                a.counters[0] += na;
                a.counters[1] += nt;
                if (a.drift && dm > 0.0f) atomicMax(reinterpret_cast<unsigned int *>(a.drift), __float_as_uint(dm));
            }
        }
        if (next.kb > 0) __syncthreads();  // commits are visible to the proposals below
    }
    for (int k = tid; k < next.kb; k += DEC_THREADS) propose_one(next, k);
}

// Commit blocks of a decision launch (blocks 1 .. n_cm): block cb takes the
// items (trial, atom) [cb CM_ITEMS, (cb + 1) CM_ITEMS) of the batch, one per
// thread, evaluates the first-pass state of the item's trial from the same
// values as the decision, and commits the atom when the trial is accepted
// there.  Nothing else in the launch reads the positions they write (the
// decision reads ΔE⁰ and entries, the correction blocks trial records);
// spread over many CUs, the scattered loads and stores of the commit take a
// fraction of the time they take on the deciding block's one CU.
constexpr int CM_ITEMS = 256;

__device__ __forceinline__ void commit_block(const DecideArgs &a, int cb)
{
    const int t = threadIdx.x;
    if (t >= CM_ITEMS) return;
    const int lane = t & 63;
    const int max_na = a.max_na;
    const int item = cb * CM_ITEMS + t;
    const int k = item / max_na, at = item - k * max_na;
    bool ok = false;
    int idx = 0;
    if (k < a.kb) {
        const int4 id = ld_i4(a.head + k);  // unit, first atom, atoms
        const double2 blh = ld_d2(a.corr_b + 2 * k), bmc = ld_d2(a.corr_b + 2 * k + 1);
        const double e0 = ldg(a.dE0 + k), thr = ldg(a.hthr + k);
        ok = at < id.z && first_pass_state(e0, thr, blh, bmc) == ST_ACC;
        idx = id.y + at;
    }
    float dmax = 0.0f;
    if (ok) {
        CommitItem ci;
        commit_load(a, k, at, idx - at, ci);
        commit_store(a, k, ci, dmax);
    }
    for (int o = 32; o > 0; o >>= 1) dmax = fmaxf(dmax, __shfl_xor(dmax, o));
    if (lane == 0 && a.drift && dmax > 0.0f) atomicMax(reinterpret_cast<unsigned int *>(a.drift), __float_as_uint(dmax));
}

// Blocks 1.. of a decision launch: the corrections of the next batch, one
// trial per wave.  They need only the next batch's trial records (its units
// are disjoint from this batch's, so the commit does not touch them) and
// run on the CUs the one-block decision leaves idle.
constexpr int DEC_CORR_TRIALS = DEC_THREADS / 64;

// LDS shared by the roles of a decision launch: the correction blocks'
// scratch, and block 0's entries of the trials it resolves in one wave.
constexpr int DEC_POOL_BYTES = (int)sizeof(CorrScratch) * DEC_CORR_TRIALS + (int)sizeof(float4) * KMAX;
static_assert(RESOLVE_POOL_BYTES <= DEC_POOL_BYTES, "resolve area must fit the shared pool");

template <int MAXNU>
__device__ __forceinline__ void next_corr_block(const CorrArgs &cn, int bx, CorrScratch *s_cs)
{
    __shared__ int s_prow[16];
    const int tid = threadIdx.x;
    // trials interleaved over the blocks (block bx - 1 of nb takes trials
    // bx - 1, bx - 1 + nb, ...): a trial's work grows with its rank in the
    // batch, and a block of consecutive late trials would load its CU's SIMDs
    // with the heaviest ones at once
    const int tpb = cn.per_block;
    // Waves w, w + 4, w + 8, ... share a SIMD, so the ranks go up in the
    // first group of four waves and down in the next (0 1 2 3 7 6 5 4 ...):
    // every SIMD then holds trials whose ranks sum alike, and no SIMD takes
    // two late, heavy ones.
    const int nb = (cn.kb + tpb - 1) / tpb;
    const int w = tid >> 6, wg = w >> 2, ws = w & 3;
    const int rank = 4 * wg + ((wg & 1) ? 3 - ws : ws);
    const int k = w < tpb ? rank * nb + (bx - 1) : cn.kb;
    // the batch's spheres, staged in LDS (after the scratch): every wave
    // tests its trial against all earlier ones
    float4 *s_sph = reinterpret_cast<float4 *>(s_cs + DEC_CORR_TRIALS);
    const int k_end = min(cn.kb, (tpb - 1) * nb + bx);
    for (int m = tid; m < k_end; m += DEC_THREADS) s_sph[m] = ld4(cn.spheres + m);
    if (tid < cn.M * cn.M) s_prow[tid] = nd::pair_index(tid / cn.M, tid % cn.M, cn.M) * cn.n_pts;
    __syncthreads();
    const PairCtx c{cn.tab, s_prow, cn.M, cn.n_pts, cn.rcf2_filter, cn.rcf2, cn.tscale};
    if (k < cn.kb) corr_trial<MAXNU>(cn, c, k, tid & 63, s_cs[tid >> 6], s_sph);
}

// The final dE of every trial of a decided batch (the same in-order sum as
// the decision's own final pass: ΔE⁰ plus the entries of accepted earlier
// trials), the near-tie count, the trace, and the running energy and
// counters, updated by one thread after a fixed-order block reduction.
__device__ void final_body(const FinalArgs &f, unsigned char *lds)
{
    unsigned char *s_acc = lds;                                        // [KMAX]
    double *s_rd = reinterpret_cast<double *>(lds + KMAX);             // [FIN_THREADS / 64]
    long long *s_ra = reinterpret_cast<long long *>(s_rd + FIN_THREADS / 64);
    long long *s_rt = s_ra + FIN_THREADS / 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int k = tid; k < f.kb; k += FIN_THREADS) s_acc[k] = ldg(f.acc + k);
    __syncthreads();
    double dsum = 0.0;
    long long nacc = 0, ntie = 0;
    for (int k = tid; k < f.kb; k += FIN_THREADS) {
        double e = ldg(f.dE0 + k);
        for_entries(f.pool_m, f.pool_c, k, ldg(f.corr_n + k), ldg(f.corr_ptr + k),
                    [&](int m, double c) { e += (m >= 0 && s_acc[m]) ? c : 0.0; });
        const bool acc = s_acc[k] != 0;
        const double S = ldg(f.S0 + k) + (double)ldg(f.corr_s + k);
        const double thr = ldg(f.thr + k);
        // |ln u + dE/kT| < tie_rel S / kT, i.e. |dE - (-kT ln u)| < tie_rel S (u > 0)
        if (thr != 745.13321910194122 * f.kT && fabs(e - thr) < f.tie_rel * S) ++ntie;
        if (acc) {
            ++nacc;
            dsum += e;
        }
        if (f.tr_dE) f.tr_dE[k] = e;
        if (f.tr_sabs) f.tr_sabs[k] = S;
        if (f.tr_acc) f.tr_acc[k] = acc ? 1 : 0;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        dsum += __shfl_xor(dsum, o);
        nacc += __shfl_xor(nacc, o);
        ntie += __shfl_xor(ntie, o);
    }
    if (lane == 0) {
        s_rd[wave] = dsum;
        s_ra[wave] = nacc;
        s_rt[wave] = ntie;
    }
    __syncthreads();
    if (tid == 0) {
        double d = 0.0;
        long long na = 0, nt = 0;
        for (int w = 0; w < FIN_THREADS / 64; ++w) {
            d += s_rd[w];
            na += s_ra[w];
            nt += s_rt[w];
        }
        *f.E += d;
        *f.dsum += d;
        f.counters[0] += na;
        f.counters[1] += nt;
    }
}

// The last batch's final sums (no scan launch follows it).
__global__ __launch_bounds__(FIN_THREADS) void k_mc_final(FinalArgs f)
{
    __shared__ __align__(16) unsigned char s_lds[KMAX + 3 * sizeof(double) * (FIN_THREADS / 64)];
    final_body(f, s_lds);
}

template <int MAXNU>
__global__ __launch_bounds__(DEC_THREADS) void k_mc_decide(DecideArgs a, ProposeArgs next, CorrArgs cn)
{
    __shared__ __align__(16) unsigned char s_pool[DEC_POOL_BYTES];
    if (blockIdx.x == 0)
        decide_body(a, next, s_pool);
    else if ((int)blockIdx.x <= a.n_cm)
        commit_block(a, blockIdx.x - 1);
    else
        next_corr_block<MAXNU>(cn, blockIdx.x - a.n_cm, reinterpret_cast<CorrScratch *>(s_pool));
}

__global__ void k_mc_reset(long long *counters, double *dsum, int32_t *ovf_fill, int32_t *slab0, int32_t *slab1)
{
    if (threadIdx.x < N_SLAB) {
        slab0[threadIdx.x] = 0;
        slab1[threadIdx.x] = 0;
    }
    if (threadIdx.x < 2) {
        counters[threadIdx.x] = 0;
        ovf_fill[threadIdx.x] = 0;  // one per correction buffer
    }
    if (threadIdx.x == 0) *dsum = 0.0;
}

// ---------------------------------------------------------------- several boxes
// One batch of one box: the arguments of its scan launch (cell scan,
// corrections, early proposals of the next batch) and of its decision launch.
struct McLaunch {
    CellScanArgs ca;
    CorrArgs cr;
    ProposeArgs next;  // next batch proposed by the scan launch (kb = 0: not there)
    DecideArgs da;
    ProposeArgs late;  // next batch proposed after the commit (kb = 0: not there)
    CorrArgs cn;       // corrections of the next batch, run by the decision launch (kb = 0: none)
    FinalArgs fin;     // the previous batch's final sums, run by the scan launch (kb = 0: none)
    int32_t *ovf0;     // overflow fills of the two correction buffers (cleared by the reset)
    int32_t *slab0, *slab1;  // slab counts of the two trial buffers (cleared by the reset)
    int nblk;          // blocks of the scan launch
    int dblk;          // blocks of the decision launch
    int rebuild;       // cells rebuilt before this batch
};

// The same kernels over several boxes at once: blockIdx.y selects the box's
// batch descriptor, blocks past a box's own grid return at once.
template <int MAXNU, int NW>
__global__ __launch_bounds__(256, (MAXNU <= 3 ? 4 : (MAXNU <= 4 ? 3 : 2))) void k_mc_scan_corr_multi(const McLaunch *__restrict__ L)
{
    const McLaunch &e = L[blockIdx.y];
    if ((int)blockIdx.x >= e.nblk) return;
    scan_corr_body<MAXNU, NW>(e.ca, e.cr, e.next, e.fin, blockIdx.x);
}

// blockIdx.x selects the box and blockIdx.y the role (0: its decision), so
// the decisions of every box are dispatched before any correction block.
template <int MAXNU>
__global__ __launch_bounds__(DEC_THREADS) void k_mc_decide_multi(const McLaunch *__restrict__ L)
{
    const McLaunch &e = L[blockIdx.x];
    __shared__ __align__(16) unsigned char s_pool[DEC_POOL_BYTES];
    if (blockIdx.y == 0)
        decide_body(e.da, e.late, s_pool);
    else if ((int)blockIdx.y < e.dblk)
        next_corr_block<MAXNU>(e.cn, blockIdx.y, reinterpret_cast<CorrScratch *>(s_pool));
}

__global__ __launch_bounds__(64) void k_mc_propose_multi(const ProposeArgs *__restrict__ P)
{
    const ProposeArgs &a = P[blockIdx.y];
    const int k = blockIdx.x * 64 + threadIdx.x;
    if (k < a.kb) propose_one(a, k);
}

__global__ void k_mc_reset_multi(const McLaunch *__restrict__ L)
{
    const McLaunch &e = L[blockIdx.y];
    const DecideArgs &d = e.da;
    if (threadIdx.x < N_SLAB) {
        e.slab0[threadIdx.x] = 0;
        e.slab1[threadIdx.x] = 0;
    }
    if (threadIdx.x < 2) {
        d.counters[threadIdx.x] = 0;
        e.ovf0[threadIdx.x] = 0;  // one per correction buffer
    }
    if (threadIdx.x == 0) *d.dsum = 0.0;
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
void launch_scan_corr(nd_box *b, const CellScanArgs &ca, const CorrArgs &cr, const ProposeArgs &next,
                      const FinalArgs &fin, size_t slds)
{
    nd::ProfScope ps(b, ND_PROF_MC_SCAN);
    const int nblk = scan_front_blocks(cr.kb, next.kb, fin.kb > 0 ? 1 : 0) + N_SLAB * ca.per_slab;
    const dim3 g(nblk), t(256);
    switch (ca.nw) {
    case 1: hipLaunchKernelGGL((k_mc_scan_corr<MAXNU, 1>), g, t, slds, b->stream, ca, cr, next, fin); break;
    case 2: hipLaunchKernelGGL((k_mc_scan_corr<MAXNU, 2>), g, t, slds, b->stream, ca, cr, next, fin); break;
    default: hipLaunchKernelGGL((k_mc_scan_corr<MAXNU, 4>), g, t, slds, b->stream, ca, cr, next, fin); break;
    }
    ND_HIP(hipGetLastError());
}

template <int MAXNU>
void launch_corr(nd_box *b, const CorrArgs &cr)
{
    nd::ProfScope ps(b, ND_PROF_MC_CORR);
    hipLaunchKernelGGL(k_mc_corr<MAXNU>, dim3((cr.kb + CORR_TPB - 1) / CORR_TPB), dim3(256), 0, b->stream, cr);
    ND_HIP(hipGetLastError());
}

void ensure_work(nd_box *b, int K, int n_jb)
{
    nd::McWork &w = b->mc;
    size_t pool = (size_t)K * CORR_CAP + (size_t)K * (K - 1) / 2 + 1;
    if (w.trials && w.cap_k >= K && w.cap_jb >= n_jb && w.cap_pool >= pool) return;
    ND_HIP(hipStreamSynchronize(b->stream));
    nd::dfree(w.trials);
    nd::dfree(w.spheres);
    nd::dfree(w.head);
    nd::dfree(w.hthr);
    nd::dfree(w.partial);
    nd::dfree(w.dE0);
    nd::dfree(w.S0);
    nd::dfree(w.thr);
    nd::dfree(w.acc_flags);
    nd::dfree(w.corr_n);
    nd::dfree(w.corr_ptr);
    nd::dfree(w.pool_m);
    nd::dfree(w.pool_c);
    nd::dfree(w.corr_s);
    nd::dfree(w.corr_b);
    nd::dfree(w.slab);
    long long *counters = w.counters;
    double *dsum = w.dsum;
    int32_t *ovf = w.ovf_fill;
    w = nd::McWork();
    w.counters = counters;
    w.dsum = dsum;
    w.ovf_fill = ovf;
    // two trial buffers: the batch being decided and the next one
    w.trials = static_cast<nd::Trial *>(nd::dmalloc(sizeof(nd::Trial) * 2 * K));
    w.spheres = static_cast<float4 *>(nd::dmalloc(sizeof(float4) * 2 * K));
    w.head = static_cast<int4 *>(nd::dmalloc(sizeof(int4) * 2 * K));
    w.hthr = static_cast<double *>(nd::dmalloc(sizeof(double) * 2 * K));
    w.partial = static_cast<double *>(nd::dmalloc(sizeof(double) * 2 * (size_t)n_jb * K));
    // by buffer: the final sums of a batch read them beside the next batch's scan
    w.dE0 = static_cast<double *>(nd::dmalloc(sizeof(double) * 2 * K));
    w.S0 = static_cast<double *>(nd::dmalloc(sizeof(double) * 2 * K));
    w.thr = static_cast<double *>(nd::dmalloc(sizeof(double) * 2 * K));
    w.acc_flags = static_cast<uint8_t *>(nd::dmalloc(sizeof(uint8_t) * 2 * K));
    // two correction buffers: the batch being decided and the next one
    w.corr_n = static_cast<int32_t *>(nd::dmalloc(sizeof(int32_t) * 2 * K));
    w.corr_ptr = static_cast<int32_t *>(nd::dmalloc(sizeof(int32_t) * 2 * K));
    w.pool_m = static_cast<int32_t *>(nd::dmalloc(sizeof(int32_t) * 2 * pool));
    w.pool_c = static_cast<double *>(nd::dmalloc(sizeof(double) * 2 * pool));
    w.corr_s = static_cast<float *>(nd::dmalloc(sizeof(float) * 2 * K));
    w.corr_b = static_cast<double2 *>(nd::dmalloc(sizeof(double2) * 4 * K));
    w.slab = static_cast<int32_t *>(nd::dmalloc(sizeof(int32_t) * 2 * (size_t)(N_SLAB + N_SLAB * K)));
    if (!w.counters) w.counters = static_cast<long long *>(nd::dmalloc(sizeof(long long) * 4));
    if (!w.dsum) w.dsum = static_cast<double *>(nd::dmalloc(sizeof(double)));
    if (!w.ovf_fill) w.ovf_fill = static_cast<int32_t *>(nd::dmalloc(sizeof(int32_t) * 2));
    w.cap_k = K;
    w.cap_jb = n_jb;
    w.cap_pool = pool;
}

}  // namespace

namespace nd {

int mc_batch_size(nd_box *b, const nd_mc_params *p, double target)
{
    // about `target` (18 unless tuned) interacting earlier trials expected
    // for the last trial of a batch; at most KMAX and half the number of units
    int K;
    if (p->k_batch > 0) {
        K = p->k_batch;
    } else {
        if (!(target > 0.0)) {
            nd_tuning e;
            target = (tune_lookup(ND_TUNE_BOX, b->N, &e) && e.batch_target > 0.0) ? e.batch_target : 18.0;
        }
        const double disp = std::max(p->max_disp, p->atom_frac > 0.0 ? p->atom_disp : 0.0);
        const double ext = (b->max_na > 1 ? 1.2 : 0.0) + disp * 1.8;
        const double reach = b->rc + 2.0 * ext;
        const double f = (4.0 / 3.0) * M_PI * reach * reach * reach / (b->L * b->L * b->L);
        K = (int)std::min(1e9, target / std::max(f, 1e-9));
        K = std::min(K, std::max(1, b->n_units / 2));
    }
    return std::max(1, std::min({K, KMAX, b->n_units}));
}

}  // namespace nd

namespace {

using nd::McWork;

struct McConsts {
    float rcf, rcf2_filter;
    double rcf2, tscale, tie_rel;
};

McConsts mc_consts(const nd_box *b, const nd_mc_params *p)
{
    McConsts c;
    c.rcf = (float)(b->rc / b->L);
    c.rcf2_filter = nd::filter_r2(b->rc / b->L);
    c.rcf2 = (b->rc / b->L) * (b->rc / b->L);
    c.tscale = b->L / b->h;
    c.tie_rel = p->tie_rel > 0.0 ? p->tie_rel : 1e-6;
    return c;
}

size_t mc_table_lds(const nd_box *b)
{
    const size_t lds_tab = sizeof(float) * (size_t)b->P * b->n_pts;
    if (lds_tab > 64 * 1024) nd::fail(ND_E_UNSUPPORTED, "potential table larger than 64 KB");
    return lds_tab;
}

int32_t *slab_buffer(const nd_box *b, int buf)
{
    const McWork &w = b->mc;
    return w.slab + (size_t)buf * (N_SLAB + (size_t)N_SLAB * w.cap_k);
}

// Scan blocks per slab: room for the mean count of a slab plus three
// standard deviations, so that a wave rarely takes a second trial.
int per_slab_blocks(int kb, int nw)
{
    const double m = (double)kb / N_SLAB;
    return std::max(1, (int)std::ceil((m + 3.0 * std::sqrt(m)) * nw / 4.0));
}

// Waves per trial of a scan launch holding `trials` trials: the most of
// 4, 2, 1 that keeps all of them in flight at once (16 waves per CU at the
// kernel's register use, with a quarter to spare for the correction
// blocks).  A trial's chain of dependent loads is shorter with more waves;
// more trials at once beat that when the GPU would otherwise take them in
// several rounds.
int pick_scan_nw(long long trials, int ncu, int tuned = 0)
{
    if (tuned > 0) return tuned;
    const long long slots = 16LL * ncu * 5 / 4;
    if (4 * trials <= slots) return 4;
    if (2 * trials <= slots) return 2;
    return 1;
}

ProposeArgs proposal_args(const nd_box *b, const nd_mc_params *p, uint64_t seed, uint64_t t0, int kb, int buf, int K)
{
    const McWork &w = b->mc;
    ProposeArgs pa;
    pa.xyz = b->xyz;
    pa.pos4 = b->pos4;
    pa.poslo = b->poslo;
    pa.uoff = b->uoff;
    pa.N = b->N;
    pa.n_units = b->n_units;
    pa.order = p->order;
    pa.L = b->L;
    pa.invL = 1.0 / b->L;
    pa.max_disp = p->max_disp;
    pa.max_rot = p->max_rot;
    pa.kT = p->kT;
    pa.seed = seed;
    pa.t0 = t0;
    pa.kb = kb;
    pa.trials = w.trials + (size_t)buf * K;
    pa.spheres = w.spheres + (size_t)buf * K;
    pa.kcap = w.cap_k;
    pa.slab = slab_buffer(b, buf);
    pa.head = w.head + (size_t)buf * K;
    pa.hthr = w.hthr + (size_t)buf * K;
    pa.atom_frac = p->atom_frac;
    pa.atom_disp = p->atom_disp;
    pa.r0 = b->has_intra ? b->r0 : nullptr;
    pa.sp = b->species;
    pa.M = b->M;
    for (int q = 0; q < ND_MAX_SPECIES * (ND_MAX_SPECIES + 1) / 2; ++q) pa.kint[q] = b->kint[q];
    return pa;
}

CorrArgs corr_args(const nd_box *b, const McConsts &k, const nd::Trial *trials, const float4 *spheres, int kb, int K,
                   int buf)
{
    const McWork &w = b->mc;
    CorrArgs cr;
    cr.tab = b->tab;
    cr.trials = trials;
    cr.spheres = spheres;
    cr.M = b->M;
    cr.n_pts = b->n_pts;
    cr.kb = kb;
    cr.rcf = k.rcf + 2e-6f;
    cr.rcf2_filter = k.rcf2_filter;
    cr.rcf2 = k.rcf2;
    cr.tscale = k.tscale;
    cr.corr_n = w.corr_n + (size_t)buf * w.cap_k;
    cr.corr_ptr = w.corr_ptr + (size_t)buf * w.cap_k;
    cr.corr_s = w.corr_s + (size_t)buf * w.cap_k;
    cr.corr_b = w.corr_b + (size_t)buf * 2 * w.cap_k;
    cr.pool_m = w.pool_m + (size_t)buf * w.cap_pool;
    cr.pool_c = w.pool_c + (size_t)buf * w.cap_pool;
    cr.ovf_fill = w.ovf_fill + buf;
    cr.ovf_base = K * CORR_CAP;
    cr.per_block = DEC_CORR_TRIALS;
    return cr;
}

DecideArgs decide_args(const nd_box *b, const nd_mc_params *p, const McConsts &k, const nd::Trial *trials, int kb,
                       int64_t done, const nd_mc_trace *trace, bool cells_live, int buf)
{
    const McWork &w = b->mc;
    DecideArgs da;
    da.xyz = b->xyz;
    da.pos4 = b->pos4;
    da.poslo = b->poslo;
    da.E = b->E;
    da.trials = trials;
    da.dE0 = w.dE0 + (size_t)buf * w.cap_k;
    da.S0 = w.S0 + (size_t)buf * w.cap_k;
    da.corr_n = w.corr_n + (size_t)buf * w.cap_k;
    da.corr_ptr = w.corr_ptr + (size_t)buf * w.cap_k;
    da.pool_m = w.pool_m + (size_t)buf * w.cap_pool;
    da.pool_c = w.pool_c + (size_t)buf * w.cap_pool;
    da.corr_s = w.corr_s + (size_t)buf * w.cap_k;
    da.corr_b = w.corr_b + (size_t)buf * 2 * w.cap_k;
    da.ovf_fill = w.ovf_fill + buf;
    da.cell_slot = cells_live ? b->cells.slot : nullptr;
    da.spos4 = cells_live ? b->cells.spos4 : nullptr;
    da.sposlo = cells_live ? b->cells.sposlo : nullptr;
    da.sref = cells_live ? b->cells.sref : nullptr;
    da.drift = cells_live ? b->cells.drift : nullptr;
    da.slab_cnt = slab_buffer(b, buf);
    // the compact copies sit at the trial records' own offset (buffer x K)
    da.head = w.head + (trials - w.trials);
    da.hthr = w.hthr + (trials - w.trials);
    da.N = b->N;
    da.max_na = b->max_na;
    da.kb = kb;
    da.kT = p->kT;
    da.tie_rel = k.tie_rel;
    da.counters = w.counters;
    da.dsum = w.dsum;
    da.tr_dE = trace && trace->dE ? trace->dE + done : nullptr;
    da.tr_sabs = trace && trace->sabs ? trace->sabs + done : nullptr;
    da.tr_acc = trace && trace->accepted ? trace->accepted + done : nullptr;
    da.tr_unit = trace && trace->unit ? trace->unit + done : nullptr;
    da.defer = 0;
    da.acc_out = nullptr;
    da.thr_out = nullptr;
    da.moved_tag = nullptr;
    da.tag_base = 0;
    da.n_cm = 0;
    if (b->track.on) {
        da.acc_out = w.acc_flags + (size_t)buf * w.cap_k;
        da.moved_tag = b->track.moved;
        da.tag_base = nd::TRACK_TAG_STRIDE * (b->track.serial++);
    }
    return da;
}

FinalArgs final_args(const nd_box *b, const nd_mc_params *p, const McConsts &k, int kb, int64_t done,
                     const nd_mc_trace *trace, int buf)
{
    const McWork &w = b->mc;
    const size_t o = (size_t)buf * w.cap_k;
    FinalArgs f;
    f.dE0 = w.dE0 + o;
    f.S0 = w.S0 + o;
    f.thr = w.thr + o;
    f.corr_s = w.corr_s + o;
    f.corr_n = w.corr_n + o;
    f.corr_ptr = w.corr_ptr + o;
    f.pool_m = w.pool_m + (size_t)buf * w.cap_pool;
    f.pool_c = w.pool_c + (size_t)buf * w.cap_pool;
    f.acc = w.acc_flags + o;
    f.kb = kb;
    f.kT = p->kT;
    f.tie_rel = k.tie_rel;
    f.E = b->E;
    f.dsum = w.dsum;
    f.counters = w.counters;
    f.tr_dE = trace && trace->dE ? trace->dE + done : nullptr;
    f.tr_sabs = trace && trace->sabs ? trace->sabs + done : nullptr;
    f.tr_acc = trace && trace->accepted ? trace->accepted + done : nullptr;
    return f;
}

// Sizes of the batches of trials first .. first + n - 1: at most K each; in
// random order a batch also ends before the first trial whose unit it
// already holds, so the trials of a batch always move distinct units.
std::vector<int> batch_sizes(const nd_box *b, const nd_mc_params *p, uint64_t seed, uint64_t first, int64_t n, int K)
{
    std::vector<int> out;
    if (p->order == ND_ORDER_SEQ) {
        for (int64_t done = 0; done < n; done += K) out.push_back((int)std::min<int64_t>(K, n - done));
        return out;
    }
    std::vector<int64_t> stamp((size_t)b->n_units, -1);
    int64_t batch = 0;
    int size = 0;
    for (int64_t k = 0; k < n; ++k) {
        const int u = trial_unit(p->order, seed, first + (uint64_t)k, b->n_units);
        if (size == K || stamp[(size_t)u] == batch) {
            out.push_back(size);
            ++batch;
            size = 0;
        }
        stamp[(size_t)u] = batch;
        ++size;
    }
    if (size > 0) out.push_back(size);
    return out;
}

// Plan of n trials of one box with the cell scan.
struct McPlan {
    int K = 0, maxnu = 1;
    size_t lds = 0;
    ProposeArgs first;               // proposals of the first batch
    std::vector<McLaunch> batches;
    FinalArgs last_fin;              // the last batch's final sums (kb = 0: none)
};

// Every batch's launch arguments and cell rebuild points, in order.  The
// box's cell bookkeeping is advanced as the launches will advance it.
void mc_plan_cells(nd_box *b, const nd_mc_params *p, uint64_t seed, uint64_t first, int64_t n,
                   const nd_mc_trace *trace, bool force_rebuild, McPlan &pl, double target = 0.0)
{
    const int K = nd::mc_batch_size(b, p, target);
    nd_tuning te;
    const int tuned_nw = nd::tune_lookup(ND_TUNE_BOX, b->N, &te) ? te.scan_waves : 0;
    ensure_work(b, K, 1);
    nd::cells_ensure(b);
    const McWork &w = b->mc;
    const McConsts k = mc_consts(b, p);
    pl.K = K;
    pl.maxnu = pick_maxnu(b->max_na);
    pl.lds = mc_table_lds(b);
    pl.batches.clear();
    const std::vector<int> sizes = batch_sizes(b, p, seed, first, n, K);
    pl.first = proposal_args(b, p, seed, first, sizes.empty() ? 0 : sizes[0], 0, K);
    if (force_rebuild) b->cells.valid = false;
    // in sequential order the next batch's units are disjoint from this
    // batch's when 2K <= n_units: propose it alongside this batch's scan
    // instead of after the commit (in random order they may repeat)
    const bool early_propose = p->order == ND_ORDER_SEQ && 2 * K <= b->n_units;
    FinalArgs prev_fin{};
    prev_fin.kb = 0;
    int buf = 0;
    size_t bi = 0;
    for (int64_t done = 0; done < n; ++bi) {
        const int kb = sizes[bi];
        const nd::Trial *trials = w.trials + (size_t)buf * K;
        const float4 *spheres = w.spheres + (size_t)buf * K;
        McLaunch L;
        L.rebuild = (!b->cells.valid || b->cells.trials_since_build >= b->n_units) ? 1 : 0;
        if (L.rebuild) {
            b->cells.valid = true;
            b->cells.trials_since_build = 0;
        }
        // with early proposals a batch's corrections (but the first's) run in
        // the previous batch's decision launch
        L.cr = corr_args(b, k, trials, spheres, kb, K, buf);
        if (early_propose && done > 0) L.cr.kb = 0;
        CellScanArgs &ca = L.ca;
        ca.spos4 = b->cells.spos4;
        ca.sposlo = b->cells.sposlo;
        ca.slab = slab_buffer(b, buf);
        ca.kcap = w.cap_k;
        ca.nw = pick_scan_nw(kb, nd::cu_count(b->device), tuned_nw);
        ca.per_slab = per_slab_blocks(kb, ca.nw);
        ca.cstart = b->cells.start;
        ca.tab = b->tab;
        ca.trials = trials;
        ca.drift = b->cells.drift;
        ca.M = b->M;
        ca.n_pts = b->n_pts;
        ca.kb = kb;
        ca.nc = b->cells.nc;
        ca.rcf = k.rcf;
        ca.rcf2_filter = k.rcf2_filter;
        ca.rcf2 = k.rcf2;
        ca.tscale = k.tscale;
        ca.dE0 = w.dE0 + (size_t)buf * w.cap_k;
        ca.S0 = w.S0 + (size_t)buf * w.cap_k;
        ca.count = b->scan_count;
        const int64_t done_next = done + kb;
        const int kb_next = bi + 1 < sizes.size() ? sizes[bi + 1] : 0;
        const ProposeArgs nx = proposal_args(b, p, seed, first + (uint64_t)done_next, kb_next, buf ^ 1, K);
        L.next = nx;
        L.late = nx;
        if (early_propose)
            L.late.kb = 0;
        else
            L.next.kb = 0;
        L.da = decide_args(b, p, k, trials, kb, done, trace, true, buf);
        L.cn = corr_args(b, k, w.trials + (size_t)(buf ^ 1) * K, w.spheres + (size_t)(buf ^ 1) * K, kb_next, K,
                         buf ^ 1);
        if (!early_propose) L.cn.kb = 0;
        // the first pass's acceptances are committed by blocks of their own,
        // unless the decision block proposes the next batch after its commit
        // (those proposals read positions this batch may have moved)
        L.da.n_cm = L.late.kb > 0 ? 0 : (kb * b->max_na + CM_ITEMS - 1) / CM_ITEMS;
        // correction blocks of 8 trials (two waves per SIMD) when the
        // launch then still fits one block per CU, else 16
        L.cn.per_block = DEC_CORR_TRIALS / 2;
        if (1 + L.da.n_cm + (L.cn.kb + L.cn.per_block - 1) / L.cn.per_block > nd::cu_count(b->device))
            L.cn.per_block = DEC_CORR_TRIALS;
        L.dblk = 1 + L.da.n_cm + (L.cn.kb + L.cn.per_block - 1) / L.cn.per_block;
        L.ovf0 = w.ovf_fill;
        // the final sums of each batch run beside the next batch's scan
        L.da.defer = 1;
        L.da.acc_out = w.acc_flags + (size_t)buf * w.cap_k;
        L.da.thr_out = w.thr + (size_t)buf * w.cap_k;
        L.fin = prev_fin;
        prev_fin = final_args(b, p, k, kb, done, trace, buf);
        L.nblk = scan_front_blocks(L.cr.kb, L.next.kb, L.fin.kb > 0 ? 1 : 0) + N_SLAB * ca.per_slab;
        L.slab0 = slab_buffer(b, 0);
        L.slab1 = slab_buffer(b, 1);
        b->cells.trials_since_build += kb;
        pl.batches.push_back(L);
        done = done_next;
        buf ^= 1;
    }
    pl.last_fin = prev_fin;
}

template <int MAXNU>
void launch_scan_corr_multi(hipStream_t s, int nw, const McLaunch *d_L, int n_boxes, int max_blk, size_t lds)
{
    const dim3 grid(max_blk, n_boxes);
    switch (nw) {
    case 1: hipLaunchKernelGGL((k_mc_scan_corr_multi<MAXNU, 1>), grid, dim3(256), lds, s, d_L); break;
    case 2: hipLaunchKernelGGL((k_mc_scan_corr_multi<MAXNU, 2>), grid, dim3(256), lds, s, d_L); break;
    default: hipLaunchKernelGGL((k_mc_scan_corr_multi<MAXNU, 4>), grid, dim3(256), lds, s, d_L); break;
    }
    ND_HIP(hipGetLastError());
}

void scan_corr_multi(int maxnu, int nw, hipStream_t s, const McLaunch *d_L, int n_boxes, int max_blk, size_t lds)
{
    switch (maxnu) {
    case 1: launch_scan_corr_multi<1>(s, nw, d_L, n_boxes, max_blk, lds); break;
    case 2: launch_scan_corr_multi<2>(s, nw, d_L, n_boxes, max_blk, lds); break;
    case 3: launch_scan_corr_multi<3>(s, nw, d_L, n_boxes, max_blk, lds); break;
    case 4: launch_scan_corr_multi<4>(s, nw, d_L, n_boxes, max_blk, lds); break;
    default: launch_scan_corr_multi<8>(s, nw, d_L, n_boxes, max_blk, lds); break;
    }
}

void launch_decide(nd_box *b, int maxnu, int nblk, const DecideArgs &da, const ProposeArgs &late, const CorrArgs &cn)
{
    nd::ProfScope ps(b, ND_PROF_MC_DECIDE);
    const dim3 g(nblk), t(DEC_THREADS);
    switch (maxnu) {
    case 1: hipLaunchKernelGGL(k_mc_decide<1>, g, t, 0, b->stream, da, late, cn); break;
    case 2: hipLaunchKernelGGL(k_mc_decide<2>, g, t, 0, b->stream, da, late, cn); break;
    case 3: hipLaunchKernelGGL(k_mc_decide<3>, g, t, 0, b->stream, da, late, cn); break;
    case 4: hipLaunchKernelGGL(k_mc_decide<4>, g, t, 0, b->stream, da, late, cn); break;
    default: hipLaunchKernelGGL(k_mc_decide<8>, g, t, 0, b->stream, da, late, cn); break;
    }
    ND_HIP(hipGetLastError());
}

void decide_multi(int maxnu, hipStream_t s, const McLaunch *d_L, int n_boxes, int nblk)
{
    const dim3 g(n_boxes, nblk), t(DEC_THREADS);
    switch (maxnu) {
    case 1: hipLaunchKernelGGL(k_mc_decide_multi<1>, g, t, 0, s, d_L); break;
    case 2: hipLaunchKernelGGL(k_mc_decide_multi<2>, g, t, 0, s, d_L); break;
    case 3: hipLaunchKernelGGL(k_mc_decide_multi<3>, g, t, 0, s, d_L); break;
    case 4: hipLaunchKernelGGL(k_mc_decide_multi<4>, g, t, 0, s, d_L); break;
    default: hipLaunchKernelGGL(k_mc_decide_multi<8>, g, t, 0, s, d_L); break;
    }
    ND_HIP(hipGetLastError());
}

// The O(N) scan of every atom per trial (ND_SCAN_FULL).
void mc_run_full(nd_box *b, const nd_mc_params *p, uint64_t seed, uint64_t first, int64_t n, const nd_mc_trace *trace)
{
    const int n_jb = (b->N + SCAN_JB - 1) / SCAN_JB;
    const int K = nd::mc_batch_size(b, p);
    ensure_work(b, K, n_jb);
    McWork &w = b->mc;
    const size_t lds_tab = mc_table_lds(b);
    const McConsts k = mc_consts(b, p);
    const int maxnu = pick_maxnu(b->max_na);
    const int ncu = nd::cu_count(b->device);

    hipLaunchKernelGGL(k_mc_reset, dim3(1), dim3(64), 0, b->stream, w.counters, w.dsum, w.ovf_fill,
                       slab_buffer(b, 0), slab_buffer(b, 1));
    ND_HIP(hipGetLastError());
    if (n == 0) return;
    int buf = 0;
    const std::vector<int> sizes = batch_sizes(b, p, seed, first, n, K);
    {
        ProposeArgs pa = proposal_args(b, p, seed, first, sizes[0], buf, K);
        nd::ProfScope ps(b, ND_PROF_MC_PROPOSE);
        hipLaunchKernelGGL(k_mc_propose, dim3((pa.kb + 63) / 64), dim3(64), 0, b->stream, pa);
        ND_HIP(hipGetLastError());
    }
    size_t bi = 0;
    for (int64_t done = 0; done < n; ++bi) {
        const int kb = sizes[bi];
        nd::Trial *trials = w.trials + (size_t)buf * K;
        float4 *spheres = w.spheres + (size_t)buf * K;
        const CorrArgs cr = corr_args(b, k, trials, spheres, kb, K, buf);
        const int64_t done_next = done + kb;
        const int kb_next = bi + 1 < sizes.size() ? sizes[bi + 1] : 0;
        const ProposeArgs late = proposal_args(b, p, seed, first + (uint64_t)done_next, kb_next, buf ^ 1, K);
        const int tg = (int)std::max<long long>(1, std::min<long long>(MAX_TG, ((long long)kb * n_jb) / (2LL * ncu)));
        ScanArgs sa;
        sa.pos4 = b->pos4;
        sa.poslo = b->poslo;
        sa.tab = b->tab;
        sa.trials = trials;
        sa.N = b->N;
        sa.M = b->M;
        sa.n_pts = b->n_pts;
        sa.kb = kb;
        sa.tg = tg;
        sa.kcap = w.cap_k;
        sa.rcf2_filter = k.rcf2_filter;
        sa.rcf2 = k.rcf2;
        sa.tscale = k.tscale;
        sa.partial = w.partial;
        const dim3 sgrid(n_jb, (kb + tg - 1) / tg);
        {
            nd::ProfScope ps(b, ND_PROF_MC_SCAN);
            switch (maxnu) {
            case 1: hipLaunchKernelGGL(k_mc_scan<1>, sgrid, dim3(SCAN_THREADS), lds_tab, b->stream, sa); break;
            case 2: hipLaunchKernelGGL(k_mc_scan<2>, sgrid, dim3(SCAN_THREADS), lds_tab, b->stream, sa); break;
            case 3: hipLaunchKernelGGL(k_mc_scan<3>, sgrid, dim3(SCAN_THREADS), lds_tab, b->stream, sa); break;
            case 4: hipLaunchKernelGGL(k_mc_scan<4>, sgrid, dim3(SCAN_THREADS), lds_tab, b->stream, sa); break;
            default: hipLaunchKernelGGL(k_mc_scan<8>, sgrid, dim3(SCAN_THREADS), lds_tab, b->stream, sa); break;
            }
            ND_HIP(hipGetLastError());
        }
        hipLaunchKernelGGL(k_mc_reduce, dim3((kb + 255) / 256), dim3(256), 0, b->stream, w.partial, n_jb, w.cap_k, kb,
                           w.dE0 + (size_t)buf * w.cap_k, w.S0 + (size_t)buf * w.cap_k, trials);
        ND_HIP(hipGetLastError());
        switch (maxnu) {
        case 1: launch_corr<1>(b, cr); break;
        case 2: launch_corr<2>(b, cr); break;
        case 3: launch_corr<3>(b, cr); break;
        case 4: launch_corr<4>(b, cr); break;
        default: launch_corr<8>(b, cr); break;
        }
        // cells kept consistent when they are live from an earlier cell-scan call
        const DecideArgs da = decide_args(b, p, k, trials, kb, done, trace, b->cells.valid, buf);
        CorrArgs none{};
        none.kb = 0;
        launch_decide(b, maxnu, 1, da, late, none);
        if (da.moved_tag) nd::track_launch(b, da.trials, da.acc_out, da.kb, da.tag_base);
        if (b->cells.valid) b->cells.trials_since_build += kb;
        done = done_next;
        buf ^= 1;
    }
}

}  // namespace

namespace nd {

void mc_run(nd_box *b, const nd_mc_params *p, uint64_t seed, uint64_t first, int64_t n, const nd_mc_trace *trace)
{
    if (p->scan == ND_SCAN_FULL) {
        mc_run_full(b, p, seed, first, n, trace);
        return;
    }
    McPlan pl;
    mc_plan_cells(b, p, seed, first, n, trace, false, pl);
    McWork &w = b->mc;
    hipLaunchKernelGGL(k_mc_reset, dim3(1), dim3(64), 0, b->stream, w.counters, w.dsum, w.ovf_fill,
                       slab_buffer(b, 0), slab_buffer(b, 1));
    ND_HIP(hipGetLastError());
    if (pl.batches.empty()) return;
    {
        ProfScope ps(b, ND_PROF_MC_PROPOSE);
        hipLaunchKernelGGL(k_mc_propose, dim3((pl.first.kb + 63) / 64), dim3(64), 0, b->stream, pl.first);
        ND_HIP(hipGetLastError());
    }
    for (const McLaunch &L : pl.batches) {
        if (L.rebuild) cells_rebuild_launch(b->stream, b->cells.d_args, 1, b->N, b->cells.ncell);
        switch (pl.maxnu) {
        case 1: launch_scan_corr<1>(b, L.ca, L.cr, L.next, L.fin, pl.lds); break;
        case 2: launch_scan_corr<2>(b, L.ca, L.cr, L.next, L.fin, pl.lds); break;
        case 3: launch_scan_corr<3>(b, L.ca, L.cr, L.next, L.fin, pl.lds); break;
        case 4: launch_scan_corr<4>(b, L.ca, L.cr, L.next, L.fin, pl.lds); break;
        default: launch_scan_corr<8>(b, L.ca, L.cr, L.next, L.fin, pl.lds); break;
        }
        launch_decide(b, pl.maxnu, L.dblk, L.da, L.late, L.cn);
        if (L.da.moved_tag) track_launch(b, L.da.trials, L.da.acc_out, L.da.kb, L.da.tag_base);
    }
    if (pl.last_fin.kb > 0) {
        hipLaunchKernelGGL(k_mc_final, dim3(1), dim3(FIN_THREADS), 0, b->stream, pl.last_fin);
        ND_HIP(hipGetLastError());
    }
}

// ---- several boxes in one stream of launches (the batched form)
struct McMulti {
    int maxnu = 1, n_rounds = 0, n_first = 0, max_kb0 = 0;
    size_t lds = 0;
    std::vector<McLaunch> launches;  // round after round, the active boxes of each
    std::vector<int> r_off, r_n, r_maxblk, r_nw, r_dblk;
    std::vector<CellBuildArgs> cb;   // per round, the boxes whose cells are rebuilt first
    std::vector<int> cb_off, cb_n, cb_maxn, cb_maxcell;
    std::vector<ProposeArgs> first;  // first proposals of every box with trials
    McLaunch *d_launch = nullptr;
    CellBuildArgs *d_cb = nullptr;
    ProposeArgs *d_first = nullptr;
    size_t cap_launch = 0, cap_cb = 0, cap_first = 0;
};

McMulti *mc_multi_create() { return new McMulti(); }

void mc_multi_destroy(McMulti *m)
{
    if (!m) return;
    dfree(m->d_launch);
    dfree(m->d_cb);
    dfree(m->d_first);
    delete m;
}

void mc_multi_plan(McMulti *m, nd_box *const *boxes, int n, const nd_mc_params *params, const uint64_t *seed,
                   const uint64_t *first, const int64_t *n_trials, const nd_mc_trace *trace,
                   std::vector<long long> &sig)
{
    std::vector<McPlan> plans(n);
    m->maxnu = 1;
    m->lds = 0;
    int n_rounds = 0;
    long long total_atoms = 0;
    for (int i = 0; i < n; ++i) total_atoms += boxes[i]->N;
    nd_tuning te;
    const bool tuned = tune_lookup(ND_TUNE_BATCH, total_atoms, &te);
    for (int i = 0; i < n; ++i) {
        nd_box *b = boxes[i];
        // every run starts from freshly built cells, so the launch structure
        // depends only on the trial counts and batch sizes
        mc_plan_cells(b, &params[i], seed[i], first[i], n_trials[i], trace ? &trace[i] : nullptr, true, plans[i],
                      tuned ? te.batch_target : 0.0);
        m->maxnu = std::max(m->maxnu, plans[i].maxnu);
        m->lds = std::max(m->lds, plans[i].lds);
        n_rounds = std::max(n_rounds, (int)plans[i].batches.size());
    }
    m->n_rounds = n_rounds;
    m->launches.clear();
    m->r_off.assign(n_rounds, 0);
    m->r_n.assign(n_rounds, 0);
    m->r_maxblk.assign(n_rounds, 0);
    m->r_nw.assign(n_rounds, 4);
    m->r_dblk.assign(n_rounds, 1);
    const int ncu = n > 0 ? cu_count(boxes[0]->device) : 1;
    m->cb.clear();
    m->cb_off.assign(n_rounds, 0);
    m->cb_n.assign(n_rounds, 0);
    m->cb_maxn.assign(n_rounds, 0);
    m->cb_maxcell.assign(n_rounds, 0);
    m->first.clear();
    m->max_kb0 = 0;
    for (int i = 0; i < n; ++i) {
        if (plans[i].batches.empty()) continue;
        m->first.push_back(plans[i].first);
        m->max_kb0 = std::max(m->max_kb0, plans[i].first.kb);
    }
    m->n_first = (int)m->first.size();
    for (int r = 0; r < n_rounds; ++r) {
        m->r_off[r] = (int)m->launches.size();
        m->cb_off[r] = (int)m->cb.size();
        // one scan launch takes the round's trials of every box: its waves
        // per trial follow their total
        long long round_trials = 0;
        for (int i = 0; i < n; ++i)
            if (r < (int)plans[i].batches.size()) round_trials += plans[i].batches[r].ca.kb;
        const int nw = pick_scan_nw(round_trials, ncu, tuned ? te.scan_waves : 0);
        m->r_nw[r] = nw;
        for (int i = 0; i < n; ++i) {
            if (r >= (int)plans[i].batches.size()) continue;
            McLaunch L = plans[i].batches[r];
            // corrections stay in the scan launch: there they run as small
            // blocks, four per CU, while a decision-launch block takes a whole
            // CU, and a round's boxes bring thousands of them
            L.cr.kb = L.ca.kb;
            L.cn.kb = 0;
            L.dblk = 1;
            L.da.n_cm = 0;  // each box's decision block commits its own trials
            // each box's decision keeps its own final sums
            L.da.defer = 0;
            L.fin.kb = 0;
            L.da.moved_tag = nullptr;
            L.ca.count = nullptr;
            L.ca.nw = nw;
            L.ca.per_slab = per_slab_blocks(L.ca.kb, nw);
            L.nblk = scan_front_blocks(L.cr.kb, L.next.kb, 0) + N_SLAB * L.ca.per_slab;
            m->launches.push_back(L);
            // a multiple of N_SLAB, so block x of every box row lands on XCD x mod 8
            m->r_maxblk[r] = std::max(m->r_maxblk[r], (L.nblk + N_SLAB - 1) / N_SLAB * N_SLAB);
            m->r_dblk[r] = std::max(m->r_dblk[r], L.dblk);
            if (L.rebuild) {
                m->cb.push_back(boxes[i]->cells.args);
                m->cb_maxn[r] = std::max(m->cb_maxn[r], boxes[i]->N);
                m->cb_maxcell[r] = std::max(m->cb_maxcell[r], boxes[i]->cells.ncell);
            }
        }
        m->r_n[r] = (int)m->launches.size() - m->r_off[r];
        m->cb_n[r] = (int)m->cb.size() - m->cb_off[r];
    }
    // device copies of the descriptors (grow only; the addresses are part of
    // the launch structure)
    auto grow = [](auto *&ptr, size_t &cap, size_t need) {
        using T = std::remove_reference_t<decltype(*ptr)>;
        if (cap >= need && ptr) return;
        dfree(ptr);
        ptr = static_cast<T *>(dmalloc(sizeof(T) * std::max<size_t>(need, 1)));
        cap = std::max<size_t>(need, 1);
    };
    grow(m->d_launch, m->cap_launch, m->launches.size());
    grow(m->d_cb, m->cap_cb, m->cb.size());
    grow(m->d_first, m->cap_first, m->first.size());
    sig.push_back(0x4d43);
    sig.push_back(m->maxnu);
    sig.push_back((long long)m->lds);
    sig.push_back(n_rounds);
    sig.push_back(m->n_first);
    sig.push_back(m->max_kb0);
    sig.push_back((long long)(uintptr_t)m->d_launch);
    sig.push_back((long long)(uintptr_t)m->d_cb);
    sig.push_back((long long)(uintptr_t)m->d_first);
    for (int r = 0; r < n_rounds; ++r) {
        sig.push_back(m->r_off[r]);
        sig.push_back(m->r_n[r]);
        sig.push_back(m->r_maxblk[r]);
        sig.push_back(m->r_nw[r]);
        sig.push_back(m->r_dblk[r]);
        sig.push_back(m->cb_off[r]);
        sig.push_back(m->cb_n[r]);
        sig.push_back(m->cb_maxn[r]);
        sig.push_back(m->cb_maxcell[r]);
    }
}

void mc_multi_upload(McMulti *m, hipStream_t s)
{
    if (!m->launches.empty())
        ND_HIP(hipMemcpyAsync(m->d_launch, m->launches.data(), sizeof(McLaunch) * m->launches.size(),
                              hipMemcpyHostToDevice, s));
    if (!m->cb.empty())
        ND_HIP(hipMemcpyAsync(m->d_cb, m->cb.data(), sizeof(CellBuildArgs) * m->cb.size(), hipMemcpyHostToDevice, s));
    if (!m->first.empty())
        ND_HIP(hipMemcpyAsync(m->d_first, m->first.data(), sizeof(ProposeArgs) * m->first.size(),
                              hipMemcpyHostToDevice, s));
    // the host vectors are reused by the next plan: wait for the copies
    ND_HIP(hipStreamSynchronize(s));
}

void mc_multi_enqueue(McMulti *m, hipStream_t s)
{
    if (m->n_rounds == 0) return;
    // round 0 holds every box that has trials
    hipLaunchKernelGGL(k_mc_reset_multi, dim3(1, m->r_n[0]), dim3(64), 0, s, m->d_launch);
    ND_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_mc_propose_multi, dim3((m->max_kb0 + 63) / 64, m->n_first), dim3(64), 0, s, m->d_first);
    ND_HIP(hipGetLastError());
    for (int r = 0; r < m->n_rounds; ++r) {
        const McLaunch *Lr = m->d_launch + m->r_off[r];
        if (m->cb_n[r] > 0)
            cells_rebuild_launch(s, m->d_cb + m->cb_off[r], m->cb_n[r], m->cb_maxn[r], m->cb_maxcell[r]);
        scan_corr_multi(m->maxnu, m->r_nw[r], s, Lr, m->r_n[r], m->r_maxblk[r], m->lds);
        decide_multi(m->maxnu, s, Lr, m->r_n[r], m->r_dblk[r]);
    }
}

}  // namespace nd

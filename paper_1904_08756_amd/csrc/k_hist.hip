// Pair-count histogram N_p(k) over all unordered atom pairs (the paper's
// N(r), Sec. "Acceleration method") and the full-box total energy.
//
// Layout: the i side of a tile pair is held one atom per thread in
// registers; the j side is staged in LDS (fixed-point and float32
// coordinates plus the histogram row offsets) and read by broadcast.
// A block is GRP groups of TILE threads; each group takes its own tile
// pair per round and all of them count into one LDS-private u32 histogram
// of the block (one copy per CU's worth of groups instead of one per group,
// so fewer counters to merge).  Blocks visit many tile pairs (persistent
// grid) and add their nonzero counters with integer atomics when done, and
// after every FLUSH_TILES tile pairs counted into a counter, before a u32
// could overflow, into the u64 counts (the several-box kernel into each
// box's counts).  Integer sums are exact in any order, so the counts do not
// depend on scheduling.
#include "nd_internal.h"
#include "nd_pair.h"

#include <algorithm>
#include <cmath>

namespace {

constexpr int TILE = 256;  // atoms per tile = threads per block
// A tile pair adds at most TILE * TILE counts, so a u32 LDS counter holds
// the counts of this many tile pairs (65535 * 65536 < 2^32).
constexpr long long FLUSH_TILES = 65535;

// Fractional coordinates s = x / L in FP64, stored as float32 hi + lo;
// hi.w holds the species and lo.w the atom's rigid unit, both as int bits.
__global__ void k_pos4_from_xyz(const float *__restrict__ xyz, const uint8_t *__restrict__ sp,
                                const int32_t *__restrict__ unit_of, int N, double invL, float4 *__restrict__ pos4,
                                float4 *__restrict__ poslo)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double sx = (double)xyz[i] * invL, sy = (double)xyz[N + i] * invL, sz = (double)xyz[2 * N + i] * invL;
    float4 p, q;
    p.x = (float)sx;
    p.y = (float)sy;
    p.z = (float)sz;
    p.w = __int_as_float((int)sp[i]);
    q.x = (float)(sx - (double)p.x);
    q.y = (float)(sy - (double)p.y);
    q.z = (float)(sz - (double)p.z);
    q.w = __int_as_float(unit_of[i]);  // read by the Metropolis cell scan
    pos4[i] = p;
    poslo[i] = q;
}

// Coordinates given in device memory: each value wrapped into [0, L) as
// x - L floor(x / L) in FP64 and rounded to float32 (a result of L is 0);
// a value that is not finite sets *bad.
__global__ void k_wrap_coords(const float *__restrict__ in, float *__restrict__ out, long long n, double L,
                              int *__restrict__ bad)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float v = in[i];
    if (!isfinite(v)) {
        atomicOr(bad, 1);
        out[i] = 0.0f;
        return;
    }
    const double x = (double)v;
    const double w = x - L * floor(x / L);
    float f = (float)w;
    if ((double)f >= L || f < 0.0f) f = 0.0f;
    out[i] = f;
}

// Upper-triangle tile pair t -> (I, J), I <= J < nt, row-major.
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

struct HistArgs {
    const float *xyz;
    const uint8_t *sp;
    int N, M, P, nbins, nt;
    long long ntp;
    double L, invL, dr;
    float fix_scale;        // (L / 2^32) / dr: fixed-point length to bins
    float nb_hi;            // nbins + 2 edge_eps: shifted candidates beyond are out of range
    float edge_eps;
    unsigned long long *out;  // [P * nbins] counts (cleared beforehand), accumulated atomically
    long long tile0;        // first global tile-pair index of this box (several boxes per launch)
};

// LDS layout of the histogram kernels.  A block is GRP groups of TILE
// threads; each group stages its own j tile, and the groups share one
// histogram (so a block's flush covers the pairs of GRP groups).
struct HistLds {
    int4 *jq;        // [TILE] j-tile fixed-point coordinates; .w: row word offsets (16 bits per species, M <= 2)
    float *jf;       // [3][TILE] j-tile float32 coordinates
    int *jrow;       // [ND_MAX_SPECIES][TILE] word offset of the histogram row of (species s, atom j)
    int *prow;       // [16] partial row offset of each species pair
    unsigned *hist;  // [P * nbins + 1]: the last word takes pairs just past the range
};

constexpr size_t HIST_LDS_GROUP = sizeof(int4) * TILE + sizeof(float) * 3 * TILE + sizeof(int) * ND_MAX_SPECIES * TILE;

__device__ __forceinline__ HistLds hist_lds(unsigned char *smem, int grp, int n_grp)
{
    HistLds h;
    unsigned char *g = smem + HIST_LDS_GROUP * (size_t)grp;
    h.jq = reinterpret_cast<int4 *>(g);
    h.jf = reinterpret_cast<float *>(h.jq + TILE);
    h.jrow = reinterpret_cast<int *>(h.jf + 3 * TILE);
    h.prow = reinterpret_cast<int *>(smem + HIST_LDS_GROUP * (size_t)n_grp);
    h.hist = reinterpret_cast<unsigned *>(h.prow + 16);
    return h;
}

constexpr size_t hist_lds_fixed(int n_grp) { return HIST_LDS_GROUP * (size_t)n_grp + sizeof(int) * 16; }

// Fixed-point fractional coordinate: round(x / L 2^32) mod 2^32.  The
// difference of two of them, read as a signed 32-bit integer, is the
// nearest-image displacement in units of L / 2^32.
__device__ __forceinline__ int fixed_coord(float x, double invL)
{
    return (int)(unsigned)(long long)rint((double)x * invL * 4294967296.0);
}

// Zero the LDS histogram and set the species-pair row offsets of box a.
__device__ __forceinline__ void hist_begin(const HistArgs &a, const HistLds &h)
{
    const int tid = threadIdx.x;
    for (int q = tid; q < a.P * a.nbins; q += blockDim.x) h.hist[q] = 0u;
    if (tid < a.M * a.M) {
        int s0 = tid / a.M, s1 = tid % a.M;
        int lo = s0 < s1 ? s0 : s1, hi = s0 < s1 ? s1 : s0;
        h.prow[tid] = (lo * a.M - lo * (lo - 1) / 2 + (hi - lo)) * a.nbins;
    }
    __syncthreads();
}

// Every pair (i, j) of tile pair (I, J), i < j on the diagonal.  The bin
// is the exact rule: k = max{k : (k dr)^2 <= r2}, counted iff k < nbins,
// with r2 = fma(dz,dz, fma(dy,dy, dx*dx)) in FP64 from the float32
// coordinates, d per axis taken at its nearest-image length min(|d|, L-|d|).
// A candidate comes from the fixed-point coordinates: the 32-bit difference
// is the nearest-image displacement, and its FP32 length times (L/2^32)/dr
// is r/dr to within the error bound below edge_eps (make_hist_args).  When
// the candidate lies within edge_eps of an integer K (a bin edge or the end
// of the range) the bin is K - 1 or K, and the FP64 r2 compared with
// (K dr)^2 decides; otherwise the candidate's floor is the bin.  One LDS
// atomic per counted pair.
// tid: the thread's rank in its group; valid false: the group has no tile
// pair in this round and only takes part in the barriers.
template <bool PACKED>
__device__ __forceinline__ void hist_tile(const HistArgs &a, const HistLds &h, int I, int J, int tid, bool valid)
{
    const int N = a.N;
    const int i = I * TILE + tid;
    const bool iv = valid && i < N;
    float xi = 0.f, yi = 0.f, zi = 0.f;
    int si = 0;
    if (iv) {
        xi = a.xyz[i];
        yi = a.xyz[N + i];
        zi = a.xyz[2 * N + i];
        si = a.sp[i];
    }
    const int qx = fixed_coord(xi, a.invL), qy = fixed_coord(yi, a.invL), qz = fixed_coord(zi, a.invL);
    __syncthreads();  // previous tile's readers are done with the j arrays
    const int j = J * TILE + tid;
    if (valid && j < N) {
        const float x = a.xyz[j], y = a.xyz[N + j], z = a.xyz[2 * N + j];
        const int sj = a.sp[j];
        int w = 0;
        if (PACKED) {
            for (int s = 0; s < a.M; ++s) w |= h.prow[s * a.M + sj] << (16 * s);
        } else {
            for (int s = 0; s < a.M; ++s) h.jrow[s * TILE + tid] = h.prow[s * a.M + sj];
        }
        h.jq[tid] = make_int4(fixed_coord(x, a.invL), fixed_coord(y, a.invL), fixed_coord(z, a.invL), w);
        h.jf[tid] = x;
        h.jf[TILE + tid] = y;
        h.jf[2 * TILE + tid] = z;
    }
    __syncthreads();
    const int jn = min(TILE, N - J * TILE);
    const int jstart = (I == J) ? tid + 1 : 0;  // diagonal tile: pairs j > i only
    if (!iv) return;
    const int *jrow = h.jrow + si * TILE;
    const int sh = 16 * si;
    const float scale = a.fix_scale, nb_hi = a.nb_hi, eps2 = 2.0f * a.edge_eps;
    float eps = a.edge_eps;
    asm volatile("" : "+v"(eps));  // held in a vector register: the fma below takes one scalar operand
#pragma unroll 4
    for (int jj = jstart; jj < jn; ++jj) {
        const int4 q = h.jq[jj];
        // 32-bit wrap-around differences
        const float dx = (float)(int)((unsigned)q.x - (unsigned)qx);
        const float dy = (float)(int)((unsigned)q.y - (unsigned)qy);
        const float dz = (float)(int)((unsigned)q.z - (unsigned)qz);
        // the candidate r/dr shifted up by eps: within eps of an integer K
        // exactly when its fraction is below 2 eps, and otherwise its floor
        // is the floor of the candidate
        const float tb = fmaf(__builtin_amdgcn_sqrtf(fmaf(dz, dz, fmaf(dy, dy, dx * dx))), scale, eps);
        if (tb < nb_hi) {
            // word offset of the (si, sj) histogram row, plus the bin
            const int rw = PACKED ? (int)__builtin_amdgcn_ubfe((unsigned)q.w, (unsigned)sh, 16u) : jrow[jj];
            const int kk = (int)tb;
            int idx = rw + kk;
            if (__builtin_amdgcn_fractf(tb) < eps2) {
                // near an edge: the exact FP64 rule
                const double L = a.L;
                const double ax = fabs((double)h.jf[jj] - (double)xi);
                const double ay = fabs((double)h.jf[TILE + jj] - (double)yi);
                const double az = fabs((double)h.jf[2 * TILE + jj] - (double)zi);
                const double mx = fmin(ax, L - ax), my = fmin(ay, L - ay), mz = fmin(az, L - az);
                const double r2 = fma(mz, mz, fma(my, my, mx * mx));
                const double e = (double)kk * a.dr;
                const int k = (r2 >= e * e) ? kk : kk - 1;
                // past the range: count into the spare word after the histogram
                idx = k < a.nbins ? rw + k : a.P * a.nbins;
            }
            atomicAdd(reinterpret_cast<unsigned *>(reinterpret_cast<unsigned char *>(h.hist) + ((unsigned)idx << 2)), 1u);
        }
    }
}

// Adds the block's nonzero LDS counters to the u64 counts and clears them.
__device__ __forceinline__ void hist_flush(const HistArgs &a, const HistLds &h)
{
    __syncthreads();
    const int nq = a.P * a.nbins;
    for (int q = threadIdx.x; q < nq; q += blockDim.x) {
        const unsigned v = h.hist[q];
        if (v) {
            atomicAdd(&a.out[q], (unsigned long long)v);
            h.hist[q] = 0u;
        }
    }
    __syncthreads();
}

// Block b takes the rounds of tile pairs t = (b + r gridDim) GRP + g, group
// g one pair per round; a round adds at most GRP TILE^2 counts to a
// counter, so the LDS counters are flushed every FLUSH_TILES / GRP rounds.
template <bool PACKED, int GRP>
__global__ __launch_bounds__(TILE * GRP, 8) void k_pair_hist(HistArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int grp = threadIdx.x / TILE, tid = threadIdx.x - grp * TILE;
    const HistLds h = hist_lds(smem, grp, GRP);
    hist_begin(a, h);
    long long since = 0;
    for (long long t0 = (long long)blockIdx.x * GRP; t0 < a.ntp; t0 += (long long)gridDim.x * GRP) {
        const long long t = t0 + grp;
        int I = 0, J = 0;
        if (t < a.ntp) tri_index(t, a.nt, I, J);
        hist_tile<PACKED>(a, h, I, J, tid, t < a.ntp);
        if (++since == FLUSH_TILES / GRP) {
            hist_flush(a, h);
            since = 0;
        }
    }
    hist_flush(a, h);
}

// Several boxes in one persistent launch.  The tile pairs of all boxes form
// one index range (box after box); block b takes the contiguous slice
// [b per, (b + 1) per) of it, so it meets one or two boxes, its GRP groups
// taking consecutive tile pairs of a box in rounds, and adds its LDS
// histogram to a box's counts with integer atomics when it leaves the box
// (exact, so the counts do not depend on the order of the blocks).
template <bool PACKED, int GRP>
__global__ __launch_bounds__(TILE * GRP, 8) void k_pair_hist_multi(const HistArgs *__restrict__ boxes, int n_boxes,
                                                                   long long total, long long per)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int grp = threadIdx.x / TILE, tid = threadIdx.x - grp * TILE;
    const HistLds h = hist_lds(smem, grp, GRP);
    long long t = (long long)blockIdx.x * per;
    const long long t_end = min(total, t + per);
    if (t >= t_end) return;
    // box holding tile pair t: the last box whose first tile is <= t
    int bi = 0;
    {
        int lo = 0, hi = n_boxes - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (boxes[mid].tile0 <= t) lo = mid; else hi = mid - 1;
        }
        bi = lo;
    }
    while (t < t_end) {
        const HistArgs &a = boxes[bi];
        const long long box_end = min(t_end, a.tile0 + a.ntp);
        if (t < box_end) {
            hist_begin(a, h);
            long long since = 0;
            for (; t < box_end; t += GRP) {
                const long long tg = t + grp;
                const bool valid = tg < box_end;
                int I = 0, J = 0;
                if (valid) tri_index(tg - a.tile0, a.nt, I, J);
                hist_tile<PACKED>(a, h, I, J, tid, valid);
                if (++since == FLUSH_TILES / GRP) {
                    hist_flush(a, h);
                    since = 0;
                }
            }
            t = box_end;
            hist_flush(a, h);
        }
        ++bi;
        if (bi >= n_boxes) break;
    }
}

__global__ void k_zero_u64_multi(const HistArgs *__restrict__ boxes)
{
    const HistArgs &a = boxes[blockIdx.y];
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < a.P * a.nbins) a.out[q] = 0ull;
}

// Clears n u64 counters (a fill kernel rather than a memset node, so the
// sequence can be captured into a graph).
__global__ void k_zero_u64(unsigned long long *__restrict__ p, int n)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) p[q] = 0ull;
}

// ---------------------------------------------------------------- energy
struct EnergyArgs {
    const float4 *pos4;
    const float4 *poslo;
    const int32_t *unit_of;
    const float *tab;
    int N, M, n_pts, nt;
    long long ntp;
    float rcf2_filter;
    double rcf2, tscale;
    double *partial;  // [gridDim.x][2]
};

// Sum over pairs i < j in different units of the tabulated energy (the
// same pair evaluation as the Metropolis kernels), FP64 sums.
__global__ __launch_bounds__(TILE) void k_total_energy(EnergyArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    float4 *jp = reinterpret_cast<float4 *>(smem);      // [TILE]
    float4 *jl = jp + TILE;                              // [TILE]
    int *ju = reinterpret_cast<int *>(jl + TILE);        // [TILE]
    int *prow = ju + TILE;                               // [16]
    float *tab = reinterpret_cast<float *>(prow + 16);   // [P][n_pts]
    __shared__ double red[2][TILE / 64];
    const int tid = threadIdx.x;
    const int P = a.M * (a.M + 1) / 2;
    nd::stage_floats<TILE>(tab, a.tab, P * a.n_pts);
    if (tid < a.M * a.M) prow[tid] = nd::pair_index(tid / a.M, tid % a.M, a.M) * a.n_pts;
    const nd::PairCtx c{tab, prow, a.M, a.n_pts, a.rcf2_filter, a.rcf2, a.tscale};
    double e = 0.0, s = 0.0;
    for (long long t = blockIdx.x; t < a.ntp; t += gridDim.x) {
        int I, J;
        tri_index(t, a.nt, I, J);
        const int i = I * TILE + tid;
        const bool iv = i < a.N;
        float4 pi = make_float4(0.f, 0.f, 0.f, 0.f), pil = pi;
        int ui = -1;
        if (iv) {
            pi = a.pos4[i];
            pil = a.poslo[i];
            ui = a.unit_of[i];
        }
        const double sx = (double)pi.x + (double)pil.x, sy = (double)pi.y + (double)pil.y,
                     sz = (double)pi.z + (double)pil.z;
        __syncthreads();
        const int j = J * TILE + tid;
        if (j < a.N) {
            jp[tid] = a.pos4[j];
            jl[tid] = a.poslo[j];
            ju[tid] = a.unit_of[j];
        }
        __syncthreads();
        const int jn = min(TILE, a.N - J * TILE);
        const int jstart = (I == J) ? tid + 1 : 0;
        if (!iv) continue;
        const int rb = __float_as_int(pi.w) * a.M;
        for (int jj = jstart; jj < jn; ++jj) {
            const float4 pj = jp[jj];
            if (nd::r2_hi(pi, pj) < c.rcf2_filter && ju[jj] != ui) {
                float u;
                if (nd::pair_u_exact(c, sx, sy, sz, rb, pj, jl[jj], u)) {
                    e += (double)u;
                    s += (double)fabsf(u);
                }
            }
        }
    }
    // block reduction in a fixed order
    for (int o = 32; o > 0; o >>= 1) {
        e += __shfl_xor(e, o);
        s += __shfl_xor(s, o);
    }
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = e;
        red[1][tid >> 6] = s;
    }
    __syncthreads();
    if (tid == 0) {
        double te = 0.0, ts = 0.0;
        for (int w = 0; w < TILE / 64; ++w) {
            te += red[0][w];
            ts += red[1][w];
        }
        a.partial[2 * blockIdx.x] = te;
        a.partial[2 * blockIdx.x + 1] = ts;
    }
}

__global__ void k_energy_reduce(const double *__restrict__ partial, int G, double *__restrict__ E,
                                double *__restrict__ S)
{
    __shared__ double re[256], rs[256];
    double e = 0.0, s = 0.0;
    for (int g = threadIdx.x; g < G; g += 256) {
        e += partial[2 * g];
        s += partial[2 * g + 1];
    }
    re[threadIdx.x] = e;
    rs[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            re[threadIdx.x] += re[threadIdx.x + w];
            rs[threadIdx.x] += rs[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (E) *E = re[0];
        if (S) *S = rs[0];
    }
}

}  // namespace

namespace nd {

void launch_pos4_from_xyz(nd_box *b)
{
    int threads = 256;
    int blocks = (b->N + threads - 1) / threads;
    hipLaunchKernelGGL(k_pos4_from_xyz, dim3(blocks), dim3(threads), 0, b->stream, b->xyz, b->species, b->unit_of,
                       b->N, 1.0 / b->L, b->pos4, b->poslo);
    ND_HIP(hipGetLastError());
}

void launch_wrap_coords(nd_box *b, const float *d_in, float *d_out, int *d_bad)
{
    const long long n = 3LL * b->N;
    hipLaunchKernelGGL(k_wrap_coords, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, b->stream, d_in, d_out, n, b->L,
                       d_bad);
    ND_HIP(hipGetLastError());
}

}  // namespace nd

namespace {

HistArgs make_hist_args(const nd_box *b, double dr, int nbins)
{
    HistArgs a{};
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
    a.dr = dr;
    a.fix_scale = (float)(b->L / 4294967296.0 / dr);
    // |candidate - r/dr| <= 8.5 u tb + sqrt(3) (L / 2^32) / dr, u = 2^-24:
    // conversion (squared: 2u), the square and two fma (3u), square root
    // (2 ulp: 2u, halved by the root of the rest), scale and product (2u);
    // the second term is the fixed-point rounding of the coordinates
    a.edge_eps = (float)(6e-7 * ((double)nbins + 1.0) + 2.0 * b->L / 4294967296.0 / dr + 1e-5);
    if (!(a.edge_eps < 0.25f)) nd::fail(ND_E_UNSUPPORTED, "nbins too large for the binning kernel");
    a.nb_hi = (float)nbins + 2.0f * a.edge_eps;
    return a;
}

// Whether the packed layout holds: at most two species, row offsets < 2^16.
bool hist_packed(int M, int nq) { return M <= 2 && nq < 65536; }

size_t hist_lds_bytes(int nq, int n_grp = 1)
{
    const size_t lds = hist_lds_fixed(n_grp) + sizeof(unsigned) * ((size_t)nq + 1);
    if (lds > 160 * 1024) nd::fail(ND_E_UNSUPPORTED, "histogram does not fit in LDS (P*nbins too large)");
    return lds;
}

constexpr int HIST_GRP = 4;  // groups per block sharing one LDS histogram

}  // namespace

namespace nd {

void launch_pair_histogram(nd_box *b, double dr, int nbins, uint64_t *d_counts)
{
    HistArgs a = make_hist_args(b, dr, nbins);
    const int nq = a.P * nbins;
    // tuned: groups of TILE threads per CU; blocks of HIST_GRP groups share
    // a histogram when two such blocks fit a CU's LDS, else one group each
    nd_tuning te;
    const int want = (tune_lookup(ND_TUNE_BOX, b->N, &te) && te.hist_blocks_per_cu > 0) ? te.hist_blocks_per_cu : 8;
    const size_t lds_g = hist_lds_bytes(nq, HIST_GRP);
    const int grp = 2 * lds_g <= 160 * 1024 ? HIST_GRP : 1;
    const size_t lds = grp == 1 ? hist_lds_bytes(nq, 1) : lds_g;
    const int want_blk = std::max(1, (want + grp - 1) / grp);
    const int per_cu = (int)std::max<size_t>(1, std::min<size_t>((size_t)want_blk, (160 * 1024) / lds));
    long long G = (long long)cu_count(b->device) * per_cu;
    G = std::min<long long>(G, (a.ntp + grp - 1) / grp);
    a.out = reinterpret_cast<unsigned long long *>(d_counts);
    hipLaunchKernelGGL(k_zero_u64, dim3((nq + 255) / 256), dim3(256), 0, b->stream, a.out, nq);
    ND_HIP(hipGetLastError());
    {
        ProfScope ps(b, ND_PROF_PAIR_HIST);
        // row offsets of up to two species fit the spare lane of the j records
        const bool packed = hist_packed(a.M, nq);
        const dim3 g((unsigned)G), t(TILE * grp);
        if (grp == HIST_GRP) {
            if (packed)
                hipLaunchKernelGGL((k_pair_hist<true, HIST_GRP>), g, t, lds, b->stream, a);
            else
                hipLaunchKernelGGL((k_pair_hist<false, HIST_GRP>), g, t, lds, b->stream, a);
        } else {
            if (packed)
                hipLaunchKernelGGL((k_pair_hist<true, 1>), g, t, lds, b->stream, a);
            else
                hipLaunchKernelGGL((k_pair_hist<false, 1>), g, t, lds, b->stream, a);
        }
        ND_HIP(hipGetLastError());
    }
}

// ---- several boxes in one launch (the batched form)
struct HistMulti {
    std::vector<HistArgs> boxes;
    HistArgs *d_boxes = nullptr;
    size_t cap = 0;
    long long total = 0, per = 0;
    int G = 0, max_nq = 0, max_m = 0, grp = 1;
    size_t lds = 0;
};

HistMulti *hist_multi_create() { return new HistMulti(); }

void hist_multi_destroy(HistMulti *m)
{
    if (!m) return;
    dfree(m->d_boxes);
    delete m;
}

void hist_multi_plan(HistMulti *m, nd_box *const *boxes, int n, double dr, const int32_t *nbins,
                     uint64_t *const *counts, std::vector<long long> &sig)
{
    m->boxes.clear();
    m->total = 0;
    m->max_nq = 0;
    m->max_m = 0;
    for (int i = 0; i < n; ++i) {
        HistArgs a = make_hist_args(boxes[i], dr, nbins[i]);
        a.out = reinterpret_cast<unsigned long long *>(counts[i]);
        a.tile0 = m->total;
        m->total += a.ntp;
        m->max_nq = std::max(m->max_nq, a.P * a.nbins);
        m->max_m = std::max(m->max_m, a.M);
        m->boxes.push_back(a);
    }
    long long total_atoms = 0;
    for (int i = 0; i < n; ++i) total_atoms += boxes[i]->N;
    // tuned: groups of TILE threads per CU; blocks of HIST_GRP groups when
    // two of them fit a CU's LDS, else one group per block
    nd_tuning te;
    const int want =
        (tune_lookup(ND_TUNE_BATCH, total_atoms, &te) && te.hist_blocks_per_cu > 0) ? te.hist_blocks_per_cu : 8;
    const size_t lds_g = hist_lds_bytes(m->max_nq, HIST_GRP);
    m->grp = 2 * lds_g <= 160 * 1024 ? HIST_GRP : 1;
    m->lds = m->grp == 1 ? hist_lds_bytes(m->max_nq, 1) : lds_g;
    const int want_blk = std::max(1, (want + m->grp - 1) / m->grp);
    const int per_cu = (int)std::max<size_t>(1, std::min<size_t>((size_t)want_blk, (160 * 1024) / m->lds));
    long long G = (long long)cu_count(boxes[0]->device) * per_cu;
    if (G > m->total) G = m->total;
    m->per = (m->total + G - 1) / G;
    m->G = (int)((m->total + m->per - 1) / m->per);
    if (m->cap < m->boxes.size() || !m->d_boxes) {
        dfree(m->d_boxes);
        m->d_boxes = static_cast<HistArgs *>(dmalloc(sizeof(HistArgs) * m->boxes.size()));
        m->cap = m->boxes.size();
    }
    sig.push_back(0x4849);
    sig.push_back(n);
    sig.push_back(m->G);
    sig.push_back(m->per);
    sig.push_back(m->total);
    sig.push_back(m->max_nq);
    sig.push_back(m->max_m);
    sig.push_back(m->grp);
    sig.push_back((long long)m->lds);
    sig.push_back((long long)(uintptr_t)m->d_boxes);
}

void hist_multi_upload(HistMulti *m, hipStream_t s)
{
    ND_HIP(hipMemcpyAsync(m->d_boxes, m->boxes.data(), sizeof(HistArgs) * m->boxes.size(), hipMemcpyHostToDevice, s));
    ND_HIP(hipStreamSynchronize(s));
}

void hist_multi_enqueue(HistMulti *m, hipStream_t s)
{
    const int n = (int)m->boxes.size();
    hipLaunchKernelGGL(k_zero_u64_multi, dim3((m->max_nq + 255) / 256, n), dim3(256), 0, s, m->d_boxes);
    ND_HIP(hipGetLastError());
    const bool packed = hist_packed(m->max_m, m->max_nq);
    const dim3 g(m->G), t(TILE * m->grp);
    if (m->grp == HIST_GRP) {
        if (packed)
            hipLaunchKernelGGL((k_pair_hist_multi<true, HIST_GRP>), g, t, m->lds, s, m->d_boxes, n, m->total, m->per);
        else
            hipLaunchKernelGGL((k_pair_hist_multi<false, HIST_GRP>), g, t, m->lds, s, m->d_boxes, n, m->total, m->per);
    } else {
        if (packed)
            hipLaunchKernelGGL((k_pair_hist_multi<true, 1>), g, t, m->lds, s, m->d_boxes, n, m->total, m->per);
        else
            hipLaunchKernelGGL((k_pair_hist_multi<false, 1>), g, t, m->lds, s, m->d_boxes, n, m->total, m->per);
    }
    ND_HIP(hipGetLastError());
}

void launch_total_energy(nd_box *b, double *d_E_out, double *d_sabs_out)
{
    EnergyArgs a;
    a.pos4 = b->pos4;
    a.poslo = b->poslo;
    a.unit_of = b->unit_of;
    a.tab = b->tab;
    a.N = b->N;
    a.M = b->M;
    a.n_pts = b->n_pts;
    a.nt = (b->N + TILE - 1) / TILE;
    a.ntp = (long long)a.nt * (a.nt + 1) / 2;
    a.rcf2_filter = nd::filter_r2(b->rc / b->L);
    a.rcf2 = (b->rc / b->L) * (b->rc / b->L);
    a.tscale = b->L / b->h;
    size_t lds = sizeof(float4) * 2 * TILE + sizeof(int) * (TILE + 16) + sizeof(float) * (size_t)b->P * b->n_pts;
    if (lds > 160 * 1024) fail(ND_E_UNSUPPORTED, "potential table does not fit in LDS");
    long long G = (long long)cu_count(b->device) * 4;
    if (G > a.ntp) G = a.ntp;
    a.partial = static_cast<double *>(workspace(b, sizeof(double) * 2 * (size_t)G));
    hipLaunchKernelGGL(k_total_energy, dim3((unsigned)G), dim3(TILE), lds, b->stream, a);
    ND_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_energy_reduce, dim3(1), dim3(256), 0, b->stream, a.partial, (int)G, d_E_out, d_sabs_out);
    ND_HIP(hipGetLastError());
}

}  // namespace nd

// Spatial cells for the Metropolis scan: atoms sorted by the cell of their
// position (x fastest), so every row of cells along x is one contiguous range
// of the sorted arrays.  Inside a cell the atoms are in increasing atom
// order, so every rebuild is deterministic.  Between rebuilds atoms keep
// their sorted slot while they move; the distance any atom has moved from
// its position at the last rebuild ("drift", fractional units) is tracked by
// the commit step and widens the cell search so no neighbour is missed.
//
// The build is a counting sort in four launches with no library calls, no
// memset and no host synchronisation, so it can be captured in a graph:
// count (atomic arrival rank per cell), scan (cell starts; the counters are
// cleared for the next build), scatter in arrival order, and a pass with one
// thread per atom that finds the atom's place in atom order inside its cell
// by ranking it among the cell's atoms, and gathers the sorted copies.  Every kernel
// takes an array of box descriptors indexed by blockIdx.y, so one launch
// rebuilds the cells of several boxes.
#include "nd_internal.h"
#include "nd_pair.h"

#include <algorithm>
#include <cmath>

namespace {

constexpr int CB_THREADS = 256;
constexpr int CB_SCAN_THREADS = 1024;
// A cell holding more atoms than this keeps its atomic arrival order (still
// a valid cell list; only the summation order, hence the last bits of the
// energy sums, then depends on scheduling).  Bounds the per-atom ranking.
constexpr int CB_SORT_MAX = 512;

__device__ __forceinline__ int cell_of(float4 p, int nc)
{
    const int cx = min(max((int)(p.x * (float)nc), 0), nc - 1);
    const int cy = min(max((int)(p.y * (float)nc), 0), nc - 1);
    const int cz = min(max((int)(p.z * (float)nc), 0), nc - 1);
    return (cz * nc + cy) * nc + cx;
}

__global__ __launch_bounds__(CB_THREADS) void k_cb_count(const nd::CellBuildArgs *__restrict__ args)
{
    const nd::CellBuildArgs &A = args[blockIdx.y];
    const int i = blockIdx.x * CB_THREADS + threadIdx.x;
    if (i >= A.N) return;
    const int c = cell_of(A.pos4[i], A.nc);
    A.cellof[i] = c;
    A.rank[i] = atomicAdd(&A.count[c], 1);
}

// One block per box: start[c] = sum of count[0..c), start[ncell] = N; the
// counters are cleared behind the scan and the drift is reset.  The cells
// go in tiles of CB_SCAN_PER per thread: coalesced loads into LDS, each
// thread's contiguous run summed from LDS (one pad word per run spreads the
// runs over the banks), one block-wide exclusive scan of the run totals,
// the starts written back in place, then coalesced stores.
constexpr int CB_SCAN_PER = 16;
constexpr int CB_SCAN_TILE = CB_SCAN_THREADS * CB_SCAN_PER;

__device__ __forceinline__ int cb_pad(int p) { return p + p / CB_SCAN_PER; }

__global__ __launch_bounds__(CB_SCAN_THREADS) void k_cb_scan(const nd::CellBuildArgs *__restrict__ args)
{
    __shared__ int s_w[CB_SCAN_THREADS / 64];
    __shared__ int s_c[CB_SCAN_TILE + CB_SCAN_TILE / CB_SCAN_PER];
    const nd::CellBuildArgs &A = args[blockIdx.y];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ncell = A.ncell;
    int32_t *cnt = A.count;
    int32_t *start = A.start;
    int carry = 0;
    for (int t0 = 0; t0 < ncell; t0 += CB_SCAN_TILE) {
        int t[CB_SCAN_PER];
#pragma unroll
        for (int u = 0; u < CB_SCAN_PER; ++u) {
            const int c = t0 + u * CB_SCAN_THREADS + tid;
            t[u] = c < ncell ? cnt[c] : 0;
        }
#pragma unroll
        for (int u = 0; u < CB_SCAN_PER; ++u) s_c[cb_pad(u * CB_SCAN_THREADS + tid)] = t[u];
        __syncthreads();
        const int r0 = cb_pad(tid * CB_SCAN_PER);  // the run's CB_SCAN_PER words are contiguous
        int v = 0;
#pragma unroll
        for (int u = 0; u < CB_SCAN_PER; ++u) v += s_c[r0 + u];
        int x = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        if (lane == 63) s_w[wave] = x;
        __syncthreads();
        int wbase = 0, total = 0;
        for (int w = 0; w < CB_SCAN_THREADS / 64; ++w) {
            const int tw = s_w[w];
            wbase += w < wave ? tw : 0;
            total += tw;
        }
        int run = carry + wbase + x - v;
#pragma unroll
        for (int u = 0; u < CB_SCAN_PER; ++u) {
            const int n = s_c[r0 + u];
            s_c[r0 + u] = run;
            run += n;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < CB_SCAN_PER; ++u) {
            const int c = t0 + u * CB_SCAN_THREADS + tid;
            if (c < ncell) {
                start[c] = s_c[cb_pad(u * CB_SCAN_THREADS + tid)];
                cnt[c] = 0;
            }
        }
        carry += total;
        __syncthreads();  // s_c and s_w are reused by the next tile
    }
    if (tid == 0) {
        start[ncell] = carry;
        *A.drift = 0.0f;
    }
}

__global__ __launch_bounds__(CB_THREADS) void k_cb_scatter(const nd::CellBuildArgs *__restrict__ args)
{
    const nd::CellBuildArgs &A = args[blockIdx.y];
    const int i = blockIdx.x * CB_THREADS + threadIdx.x;
    if (i >= A.N) return;
    A.arrival[A.start[A.cellof[i]] + A.rank[i]] = i;
}

// One thread per atom: its slot is the cell's start plus the number of the
// cell's atoms with a smaller index (arrival order for a cell too large to
// rank); then the inverse map and the sorted copies of the positions.
__global__ __launch_bounds__(CB_THREADS) void k_cb_finish(const nd::CellBuildArgs *__restrict__ args)
{
    const nd::CellBuildArgs &A = args[blockIdx.y];
    const int i = blockIdx.x * CB_THREADS + threadIdx.x;
    if (i >= A.N) return;
    const int c = A.cellof[i];
    const int b = A.start[c], e = A.start[c + 1];
    int x = b + A.rank[i];
    if (e - b <= CB_SORT_MAX) {
        x = b;
        for (int y = b; y < e; ++y) x += A.arrival[y] < i;
    }
    A.sorted[x] = i;
    A.slot[i] = x;
    const float4 p = A.pos4[i];
    A.spos4[x] = p;
    A.sposlo[x] = A.poslo[i];
    A.sref[i] = p;
}

// Sorted copies of the current positions for a restored slot order.
__global__ void k_cb_gather(const nd::CellBuildArgs *__restrict__ args)
{
    const nd::CellBuildArgs &A = args[blockIdx.y];
    const int x = blockIdx.x * CB_THREADS + threadIdx.x;
    if (x >= A.N) return;
    const int atom = A.sorted[x];
    A.spos4[x] = A.pos4[atom];
    A.sposlo[x] = A.poslo[atom];
}

__global__ void k_fill_i32(int32_t *p, int n, int v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Total energy from freshly built cells: one thread per sorted slot i sums
// the pair terms with every slot j > i of a different unit in the cells
// within reach (R cells per axis; the whole axis when 2R + 1 >= nc, so no
// cell is visited twice), with the same pair evaluation as the Metropolis
// kernels; FP64 sums per thread, per block in a fixed order.
struct CellEnergyArgs {
    const float4 *spos4, *sposlo;
    const int32_t *start;
    const float *tab;
    int N, M, n_pts, nc, R;
    float rcf2_filter;
    double rcf2, tscale;
    double *partial;  // [gridDim.x][2]
};

constexpr int CE_THREADS = 256;

__global__ __launch_bounds__(CE_THREADS) void k_energy_cells(CellEnergyArgs a)
{
    extern __shared__ __align__(16) float s_tab[];
    __shared__ int prow[16];
    __shared__ double red[2][CE_THREADS / 64];
    const int tid = threadIdx.x;
    const int P = a.M * (a.M + 1) / 2;
    nd::stage_floats<CE_THREADS>(s_tab, a.tab, P * a.n_pts);
    if (tid < a.M * a.M) prow[tid] = nd::pair_index(tid / a.M, tid % a.M, a.M) * a.n_pts;
    __syncthreads();
    const nd::PairCtx c{s_tab, prow, a.M, a.n_pts, a.rcf2_filter, a.rcf2, a.tscale};
    const int i = blockIdx.x * CE_THREADS + tid;
    double e = 0.0, s = 0.0;
    if (i < a.N) {
        const int nc = a.nc, R = a.R;
        const float4 pi = a.spos4[i], pil = a.sposlo[i];
        const int ui = __float_as_int(pil.w);
        const double sx = (double)pi.x + (double)pil.x, sy = (double)pi.y + (double)pil.y,
                     sz = (double)pi.z + (double)pil.z;
        const int rb = __float_as_int(pi.w) * a.M;
        const int cx = min(max((int)(pi.x * (float)nc), 0), nc - 1);
        const int cy = min(max((int)(pi.y * (float)nc), 0), nc - 1);
        const int cz = min(max((int)(pi.z * (float)nc), 0), nc - 1);
        const bool all = 2 * R + 1 >= nc;
        const int lo = all ? 0 : -R, hi = all ? nc - 1 : R;
        for (int dz = lo; dz <= hi; ++dz) {
            const int z = all ? dz : (cz + dz + nc) % nc;
            for (int dy = lo; dy <= hi; ++dy) {
                const int y = all ? dy : (cy + dy + nc) % nc;
                const int row = (z * nc + y) * nc;
                // the row's cells cx - R .. cx + R as at most two slot ranges
                int r0a, r0b, r1a = 0, r1b = 0;
                if (all) {
                    r0a = a.start[row];
                    r0b = a.start[row + nc];
                } else {
                    const int xl = cx - R, xh = cx + R;
                    if (xl < 0) {
                        r0a = a.start[row + xl + nc];
                        r0b = a.start[row + nc];
                        r1a = a.start[row];
                        r1b = a.start[row + xh + 1];
                    } else if (xh >= nc) {
                        r0a = a.start[row + xl];
                        r0b = a.start[row + nc];
                        r1a = a.start[row];
                        r1b = a.start[row + xh - nc + 1];
                    } else {
                        r0a = a.start[row + xl];
                        r0b = a.start[row + xh + 1];
                    }
                }
                for (int part = 0; part < 2; ++part) {
                    const int ja = part ? r1a : r0a, jb = part ? r1b : r0b;
                    for (int j = max(ja, i + 1); j < jb; ++j) {
                        const float4 pj = a.spos4[j], pjl = a.sposlo[j];
                        if (__float_as_int(pjl.w) == ui) continue;
                        float u;
                        if (nd::pair_u(c, pi, sx, sy, sz, rb, pj, pjl, u)) {
                            e += (double)u;
                            s += (double)fabsf(u);
                        }
                    }
                }
            }
        }
    }
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
        for (int w = 0; w < CE_THREADS / 64; ++w) {
            te += red[0][w];
            ts += red[1][w];
        }
        a.partial[2 * blockIdx.x] = te;
        a.partial[2 * blockIdx.x + 1] = ts;
    }
}

// Fixed-order sum of the block partials: thread t adds blocks t, t + 256, ...,
// then thread 0 adds the 256 sums in order.
__global__ void k_energy_cells_sum(const double *__restrict__ partial, int G, double *__restrict__ E)
{
    __shared__ double re[256];
    double e = 0.0;
    for (int g = threadIdx.x; g < G; g += 256) e += partial[2 * g];
    re[threadIdx.x] = e;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < 256; ++k) t += re[k];
        *E = t;
    }
}

}  // namespace

namespace nd {

// The box's energy over pairs in different units within r_cut in O(N),
// from cell lists rebuilt here (the same pair terms as launch_total_energy,
// summed in another order).
void launch_energy_cells(nd_box *b, double *d_E)
{
    cells_build(b);
    const Cells &cl = b->cells;
    CellEnergyArgs a;
    a.spos4 = cl.spos4;
    a.sposlo = cl.sposlo;
    a.start = cl.start;
    a.tab = b->tab;
    a.N = b->N;
    a.M = b->M;
    a.n_pts = b->n_pts;
    a.nc = cl.nc;
    a.R = (int)std::floor(b->rc / b->L * cl.nc) + 1;
    a.rcf2_filter = filter_r2(b->rc / b->L);
    a.rcf2 = (b->rc / b->L) * (b->rc / b->L);
    a.tscale = b->L / b->h;
    const int G = (b->N + CE_THREADS - 1) / CE_THREADS;
    a.partial = static_cast<double *>(workspace(b, sizeof(double) * 2 * (size_t)G));
    const size_t lds = sizeof(float) * (size_t)b->P * b->n_pts;
    hipLaunchKernelGGL(k_energy_cells, dim3(G), dim3(CE_THREADS), lds, b->stream, a);
    ND_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_energy_cells_sum, dim3(1), dim3(256), 0, b->stream, a.partial, G, d_E);
    ND_HIP(hipGetLastError());
}

void cells_free(nd_box *b)
{
    Cells &c = b->cells;
    dfree(c.start);
    dfree(c.sorted);
    dfree(c.slot);
    dfree(c.spos4);
    dfree(c.sposlo);
    dfree(c.sref);
    dfree(c.cellof);
    dfree(c.rank);
    dfree(c.arrival);
    dfree(c.count);
    dfree(c.drift);
    dfree(c.d_args);
    c = Cells();
}

// Cell grid of about four atoms per cell, at least one and at most 256 cells
// per axis.
static int cells_per_axis(const nd_box *b)
{
    const double rho = (double)b->N / (b->L * b->L * b->L);
    const double edge = std::cbrt(4.0 / rho);
    const int nc = (int)std::floor(b->L / edge);
    return std::max(1, std::min(nc, 256));
}

void cells_ensure(nd_box *b)
{
    Cells &c = b->cells;
    const int N = b->N;
    const int nc = cells_per_axis(b);
    const int ncell = nc * nc * nc;
    if (c.d_args && c.cap_n >= N && c.ncell == ncell) return;
    ND_HIP(hipStreamSynchronize(b->stream));
    cells_free(b);
    c.start = static_cast<int32_t *>(dmalloc(sizeof(int32_t) * (ncell + 1)));
    c.sorted = static_cast<int32_t *>(dmalloc(sizeof(int32_t) * N));
    c.slot = static_cast<int32_t *>(dmalloc(sizeof(int32_t) * N));
    c.spos4 = static_cast<float4 *>(dmalloc(sizeof(float4) * N));
    c.sposlo = static_cast<float4 *>(dmalloc(sizeof(float4) * N));
    c.sref = static_cast<float4 *>(dmalloc(sizeof(float4) * N));
    c.cellof = static_cast<int32_t *>(dmalloc(sizeof(int32_t) * N));
    c.rank = static_cast<int32_t *>(dmalloc(sizeof(int32_t) * N));
    c.arrival = static_cast<int32_t *>(dmalloc(sizeof(int32_t) * N));
    c.count = static_cast<int32_t *>(dmalloc(sizeof(int32_t) * ncell));
    c.drift = static_cast<float *>(dmalloc(sizeof(float)));
    c.d_args = static_cast<CellBuildArgs *>(dmalloc(sizeof(CellBuildArgs)));
    c.cap_n = N;
    c.nc = nc;
    c.ncell = ncell;
    c.args = CellBuildArgs{b->pos4, b->poslo, N, nc, ncell, 0, c.cellof, c.rank, c.count, c.start,
                           c.arrival, c.sorted, c.slot, c.spos4, c.sposlo, c.sref, c.drift};
    hipLaunchKernelGGL(k_fill_i32, dim3((ncell + 255) / 256), dim3(256), 0, b->stream, c.count, ncell, 0);
    ND_HIP(hipGetLastError());
    ND_HIP(hipMemcpyAsync(c.d_args, &c.args, sizeof(CellBuildArgs), hipMemcpyHostToDevice, b->stream));
    ND_HIP(hipStreamSynchronize(b->stream));
}

void cells_rebuild_launch(hipStream_t s, const CellBuildArgs *d_args, int n_boxes, int max_n, int max_ncell)
{
    if (n_boxes <= 0) return;
    (void)max_ncell;
    const dim3 ga((max_n + CB_THREADS - 1) / CB_THREADS, n_boxes);
    hipLaunchKernelGGL(k_cb_count, ga, dim3(CB_THREADS), 0, s, d_args);
    ND_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_cb_scan, dim3(1, n_boxes), dim3(CB_SCAN_THREADS), 0, s, d_args);
    ND_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_cb_scatter, ga, dim3(CB_THREADS), 0, s, d_args);
    ND_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_cb_finish, ga, dim3(CB_THREADS), 0, s, d_args);
    ND_HIP(hipGetLastError());
}

void cells_build(nd_box *b)
{
    cells_ensure(b);
    Cells &c = b->cells;
    cells_rebuild_launch(b->stream, c.d_args, 1, b->N, c.ncell);
    c.valid = true;
    c.trials_since_build = 0;
}

void cells_restore(nd_box *b, const CellState &st)
{
    cells_ensure(b);
    Cells &c = b->cells;
    if (st.nc != c.nc) fail(ND_E_INVALID, "checkpoint cell grid does not match the box");
    const size_t N = (size_t)b->N;
    ND_HIP(hipMemcpyAsync(c.sorted, st.sorted, sizeof(int32_t) * N, hipMemcpyHostToDevice, b->stream));
    ND_HIP(hipMemcpyAsync(c.slot, st.slot, sizeof(int32_t) * N, hipMemcpyHostToDevice, b->stream));
    ND_HIP(hipMemcpyAsync(c.sref, st.sref, sizeof(float4) * N, hipMemcpyHostToDevice, b->stream));
    ND_HIP(hipMemcpyAsync(c.start, st.start, sizeof(int32_t) * (c.ncell + 1), hipMemcpyHostToDevice, b->stream));
    ND_HIP(hipMemcpyAsync(c.drift, &st.drift, sizeof(float), hipMemcpyHostToDevice, b->stream));
    hipLaunchKernelGGL(k_cb_gather, dim3((b->N + CB_THREADS - 1) / CB_THREADS, 1), dim3(CB_THREADS), 0, b->stream,
                       c.d_args);
    ND_HIP(hipGetLastError());
    ND_HIP(hipStreamSynchronize(b->stream));
    c.valid = true;
    c.trials_since_build = st.trials_since_build;
}

}  // namespace nd

// Internal declarations shared by the host runtime and the kernel files of
// the neuda library.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "neuda.h"

namespace nd {

// Error reporting: the entry points catch nd::Error and turn it into a
// status plus the thread-local message.
struct Error {
    nd_status code;
    std::string msg;
};

[[noreturn]] void fail(nd_status code, const std::string &msg);
void check_hip(hipError_t e, const char *what);

#define ND_HIP(call) ::nd::check_hip((call), #call)

__host__ __device__ inline int pair_index(int a, int b, int M)
{
    if (a > b) { int t = a; a = b; b = t; }
    return a * M - a * (a - 1) / 2 + (b - a);
}

// Trial record written by the proposal kernel and read by the scan,
// correction and decision kernels.  Fractional coordinates s = x / L are
// held as a float32 pair: hi = (float)s (species in .w as int bits) and
// lo = (float)(s - hi) (the atom's unit in .w as int bits), so (double)hi +
// (double)lo carries s to ~2^-48.
struct Trial {
    float4 old_hi[ND_MAX_UNIT_ATOMS];
    float4 old_lo[ND_MAX_UNIT_ATOMS];
    float4 new_hi[ND_MAX_UNIT_ATOMS];
    float4 new_lo[ND_MAX_UNIT_ATOMS];
    float new_x[ND_MAX_UNIT_ATOMS][3];  // absolute float32 new positions
    float old_x[ND_MAX_UNIT_ATOMS][3];  // absolute float32 positions before the move
    float cen[3];                       // fractional centre of old+new atoms
    float rad;                          // fractional radius about cen
    int32_t unit, a0, na, pad;           // moved atoms a0 .. a0 + na - 1 of the unit
    double thr;                         // acceptance threshold -kT ln u of the trial's draw u
    double dintra, sintra;              // intramolecular energy change and its sum of |terms|
};

struct McWork {
    int cap_k = 0;
    int cap_jb = 0;
    size_t cap_pool = 0;
    Trial *trials = nullptr;      // [2][cap_k] batch being decided, next batch
    float4 *spheres = nullptr;    // [2][cap_k] bounding sphere of each trial (fractional)
    int4 *head = nullptr;         // [2][cap_k] unit, first atom, atoms of each trial (compact)
    double *hthr = nullptr;       // [2][cap_k] acceptance thresholds (compact)
    double *partial = nullptr;    // [cap_jb][2][cap_k]  (dE, sum |U|) per j-block (full scan)
    double *dE0 = nullptr;        // [2][cap_k] energy change against the batch-start configuration
    double *S0 = nullptr;         // [2][cap_k] sum of |U| of those pair terms
    double *thr = nullptr;        // [2][cap_k] acceptance threshold -kT ln u, stored by the decision
    uint8_t *acc_flags = nullptr; // [2][cap_k] decisions, for the deferred final sums
    // correction buffers, one per batch parity: [2][cap_k] unless stated
    int32_t *corr_n = nullptr;    // correction entries of trial k
    int32_t *corr_ptr = nullptr;  // first entry of trial k in its buffer's pool
    float *corr_s = nullptr;      // sum |U| over trial k's correction terms
    double2 *corr_b = nullptr;    // [2][2 cap_k] (lo, hi), (mag, count) of trial k's entries with m >= 0
    int32_t *pool_m = nullptr;    // [2][cap_pool] earlier trial m of each entry (increasing), -1 if C = 0
    double *pool_c = nullptr;     // [2][cap_pool] energy correction if m was accepted
    int32_t *ovf_fill = nullptr;  // [2] entries used in each pool's overflow area
    int32_t *slab = nullptr;      // [2][8 + 8 cap_k] per buffer: z-slab counts, then trial lists
    long long *counters = nullptr;   // [0] accepted, [1] near ties
    double *dsum = nullptr;       // accepted dE sum
};

// Device view of one box's cell arrays, read by the cell-build kernels
// (one descriptor per box, so a launch can rebuild several boxes).
struct CellBuildArgs {
    const float4 *pos4, *poslo;
    int N, nc, ncell, pad;
    int32_t *cellof;  // [N] cell of each atom
    int32_t *rank;    // [N] arrival rank inside the cell
    int32_t *count;   // [ncell] atoms per cell; zero between builds
    int32_t *start;   // [ncell + 1] first sorted slot of each cell
    int32_t *arrival; // [N] atoms in cell order, arrival order inside a cell
    int32_t *sorted, *slot;
    float4 *spos4, *sposlo, *sref;
    float *drift;
};

// Running pair-count histogram kept current by the Delta N(r) of every
// accepted move (see k_track.hip), and the sum of its samples.
struct Track {
    bool on = false, valid = false;
    double dr = 0.0;
    int nbins = 0;
    uint64_t *counts = nullptr;  // [P][nbins] running N(r)
    uint64_t *sum = nullptr;     // [P][nbins] sum of the accumulated samples
    long long n_samples = 0;
    int32_t *partial = nullptr;  // [G][P][nbins] per-block Delta N of one batch
    int G = 0;
    long long *moved = nullptr;  // [n_units] tag of the last batch (and trial) that moved the unit
    mutable long long serial = 0;  // batches tagged so far (advanced while planning)
};

// Atoms sorted into spatial cells (see k_cells.hip).
struct Cells {
    int nc = 0, ncell = 0, cap_n = 0;
    int32_t *start = nullptr;     // [ncell + 1] first sorted slot of each cell
    int32_t *sorted = nullptr;    // [N] slot -> atom
    int32_t *slot = nullptr;      // [N] atom -> slot
    float4 *spos4 = nullptr;      // [N] current hi + species, sorted order
    float4 *sposlo = nullptr;     // [N] current lo, sorted order
    float4 *sref = nullptr;       // [N] hi at the last rebuild, by atom
    int32_t *cellof = nullptr, *rank = nullptr, *count = nullptr, *arrival = nullptr;
    float *drift = nullptr;       // device: max distance moved since the rebuild (fractional)
    CellBuildArgs args;           // host copy of the descriptor
    CellBuildArgs *d_args = nullptr;  // device copy
    bool valid = false;
    long long trials_since_build = 0;
};

}  // namespace nd

struct nd_box {
    int device = 0;
    hipStream_t stream = nullptr;
    int N = 0, M = 0, P = 0, n_units = 0, max_na = 0;
    double L = 0.0;
    // device
    float *xyz = nullptr;        // [3][N] absolute float32 (canonical state)
    float4 *pos4 = nullptr;      // [N] fractional float32 (hi) + species bits
    float4 *poslo = nullptr;     // [N] fractional remainder (lo), .w = unit (int bits)
    uint8_t *species = nullptr;  // [N]
    int32_t *uoff = nullptr;     // [n_units + 1]
    int32_t *unit_of = nullptr;  // [N]
    // host copies
    int32_t *h_uoff = nullptr;
    uint8_t *h_species = nullptr;
    int64_t species_count[ND_MAX_SPECIES] = {0, 0, 0, 0};
    // potential tables
    float *tab = nullptr;        // [P][n_pts] reference potential + EMP, used by every energy kernel
    float *rp = nullptr;         // [P][n_pts] reference potential as given to nd_box_set_tables
    double *emp = nullptr;       // [P][n_pts] accumulated empirical potential (null: none yet)
    int n_pts = 0;
    double h = 0.0, rc = 0.0;
    bool has_tables = false;
    // intramolecular harmonic terms (flexible molecules)
    double kint[ND_MAX_SPECIES * (ND_MAX_SPECIES + 1) / 2] = {};
    double *r0 = nullptr;        // device [N][ND_MAX_UNIT_ATOMS]: reference length to each atom of the unit
    bool has_intra = false;
    // running energy
    double *E = nullptr;         // device [1]
    bool energy_valid = false;
    nd::McWork mc;
    nd::Cells cells;
    nd::Track track;
    // measurement: candidates tested and survivors of the cell scan (null: off)
    unsigned long long *scan_count = nullptr;
    // reusable device workspace for per-block partial results
    void *ws = nullptr;
    size_t ws_bytes = 0;
    // per-kernel event timing
    uint32_t prof_mask = 0;  // bit k: event pairs around launches of kernel id k
    // bin-mass table of the broadened histogram, for (beta, s) = (dr/sigma, 6 sigma/dr)
    void *bt_dev = nullptr;
    double bt_beta = 0.0, bt_s = 0.0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_pending[ND_PROF_KINDS];
    std::vector<hipEvent_t> prof_free;
    double prof_ms[ND_PROF_KINDS] = {0, 0, 0, 0, 0, 0, 0, 0};
    long long prof_n[ND_PROF_KINDS] = {0, 0, 0, 0, 0, 0, 0, 0};
};

namespace nd {

// ---- kernel launchers (defined in the .hip files) ----
void launch_pos4_from_xyz(nd_box *b);
void launch_wrap_coords(nd_box *b, const float *d_in, float *d_out, int *d_bad);
void launch_pair_histogram(nd_box *b, double dr, int nbins, uint64_t *d_counts);
void launch_total_energy(nd_box *b, double *d_E_out, double *d_sabs_out);
// Intramolecular terms (k_intra in k_track.hip): reference lengths from the
// current coordinates; energy added to *d_E (and |terms| to *d_S if not
// null); gradient added to d_grad [3][N].
void launch_intra_reference(nd_box *b);
void launch_intra_energy_add(nd_box *b, double *d_E, double *d_S);
void launch_intra_forces_add(nd_box *b, double *d_grad);
void launch_gr_normalize(const uint64_t *counts, int P, int nbins, double dr, double V,
                         const double *npairs_host, double *g, hipStream_t s);
void launch_gr_normalize_f64(const double *counts, int P, int nbins, double dr, double V,
                             const double *npairs_host, double *g, hipStream_t s);
void launch_chi2(const double *S, const double *T, int nQ, double *chi2, double *grad, hipStream_t s);
void launch_sq(const double *g, int P, int nbins, double dr, double rho, const double *w_host,
               double self_term, const double *Q, int nQ, double *S, hipStream_t s);
void launch_sq_adjoint(const double *dLdS, int P, int nbins, double dr, double rho, double V,
                       const double *w_host, const double *npairs_host, const double *Q, int nQ,
                       double *A, hipStream_t s);
void launch_hist_broad(nd_box *b, double dr, int nbins, double sigma, double *d_nhat);
void launch_hist_broad_backward(nd_box *b, double dr, int nbins, double sigma, const double *d_A,
                                double *d_grad);
void launch_forces(nd_box *b, double *d_grad, double *d_E);
size_t forces_scratch_bytes(int N, long long G);
void launch_forces_in(nd_box *b, double *d_grad, double *d_E, char *ws, long long max_grid, bool prof);
void mc_run(nd_box *b, const nd_mc_params *p, uint64_t seed, uint64_t first, int64_t n,
            const nd_mc_trace *trace);
int mc_batch_size(nd_box *b, const nd_mc_params *p, double target = 0.0);

// Metropolis runs of several boxes as one sequence of launches, each launch
// covering every box that still has batches (k_mc.hip).  plan: host-side
// descriptors of every batch of every box (allocates workspaces; appends the
// launch structure to sig); upload: descriptors to the device (synchronous);
// enqueue: the launches only, so they can be captured in a graph.
struct McMulti;
McMulti *mc_multi_create();
void mc_multi_destroy(McMulti *m);
void mc_multi_plan(McMulti *m, nd_box *const *boxes, int n, const nd_mc_params *params, const uint64_t *seed,
                   const uint64_t *first, const int64_t *n_trials, const nd_mc_trace *trace,
                   std::vector<long long> &sig);
void mc_multi_upload(McMulti *m, hipStream_t s);
void mc_multi_enqueue(McMulti *m, hipStream_t s);

// Pair histograms of several boxes in one persistent launch (k_hist.hip);
// counts[i] is a device array [P][nbins[i]] of box i, cleared by the launch.
struct HistMulti;
HistMulti *hist_multi_create();
void hist_multi_destroy(HistMulti *m);
void hist_multi_plan(HistMulti *m, nd_box *const *boxes, int n, double dr, const int32_t *nbins,
                     uint64_t *const *counts, std::vector<long long> &sig);
void hist_multi_upload(HistMulti *m, hipStream_t s);
void hist_multi_enqueue(HistMulti *m, hipStream_t s);

// g(r) and S(Q) of several boxes, one launch each (k_sq.hip).
constexpr int MAX_PARTIALS = ND_MAX_SPECIES * (ND_MAX_SPECIES + 1) / 2;
struct SqBoxDesc {
    const uint64_t *counts;  // [P][nbins]
    double *g;               // [P][nbins]
    double *S;               // [nQ]
    int P, nbins;
    double dr, V, four_pi_rho, self_term;
    double npairs[MAX_PARTIALS];
    double w[MAX_PARTIALS];
};
struct SqMulti;
SqMulti *sq_multi_create();
void sq_multi_destroy(SqMulti *m);
void sq_multi_plan(SqMulti *m, const SqBoxDesc *descs, int n, const double *Q, int nQ, std::vector<long long> &sig);
void sq_multi_upload(SqMulti *m, hipStream_t s);
void sq_multi_enqueue(SqMulti *m, hipStream_t s);
// Running histogram (k_track.hip).  track_launch: the Delta N(r) of the
// accepted trials of one decided batch, added to the running counts.
constexpr long long TRACK_TAG_STRIDE = 4096;  // > trials per batch
void track_start(nd_box *b, double dr, int nbins);
void track_stop(nd_box *b);
void track_refresh(nd_box *b);
void track_launch(nd_box *b, const Trial *trials, const uint8_t *acc, int kb, long long tag_base);
void track_accumulate(nd_box *b);
void track_mean(nd_box *b, double *d_mean);
void emp_reset(nd_box *b);
void launch_emp_update(nd_box *b, const nd_emp_params *prm, int n_prof, const double *W_host,
                       const double *self_host, const double *g, int nbins, double dr, const double *Q, int nQ,
                       const double *S_exp, double *dS_out, double *emp_out, double *C_out);
void cells_build(nd_box *b);
void launch_energy_cells(nd_box *b, double *d_E);
void cells_ensure(nd_box *b);
void cells_rebuild_launch(hipStream_t s, const CellBuildArgs *d_args, int n_boxes, int max_n, int max_ncell);
void cells_free(nd_box *b);
// Host image of a box's cell lists (checkpoint).
struct CellState {
    int nc;
    long long trials_since_build;
    float drift;
    const int32_t *sorted, *slot, *start;  // [N], [N], [ncell + 1]
    const float4 *sref;                    // [N] by atom
};
void cells_restore(nd_box *b, const CellState &st);

// Tuning table (nd_set_tuning): the entry of `kind` for n atoms, copied
// into *out; false when the table has none.
bool tune_lookup(int kind, long long n, nd_tuning *out);

// device memory helpers
void *dmalloc(size_t bytes);
void dfree(void *p);
// Workspace owned by the box, grown on demand (calls on a box are ordered
// on one stream, so one buffer serves every call).
void *workspace(nd_box *b, size_t bytes);
int cu_count(int device);

// Event pair around one kernel launch when profiling is on.
struct ProfScope {
    nd_box *b;
    int kind;
    hipEvent_t e1 = nullptr, e2 = nullptr;
    ProfScope(nd_box *box, int k);
    ~ProfScope();
};
void prof_harvest(nd_box *b);
void prof_release(nd_box *b);

}  // namespace nd

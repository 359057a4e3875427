/*
 * neuda.h - C ABI of the MI355X pair-sum library for EPSR-style structure
 * refinement (Ma et al., "NeuDATool", arXiv 1904.08756).
 *
 * The library computes the data-parallel hot path of the method on one
 * gfx950 GPU:
 *   - the minimum-image pair sum that gives the energy change of a trial
 *     move of one rigid unit against every other atom, followed by the
 *     Metropolis test (Sec. "Algorithmic Flow", step III; Sec. "Acceleration
 *     method": the per-step Delta N(r) work that is proportional to N);
 *   - the all-pairs partial histograms N_ab(r) (Sec. "Acceleration method":
 *     the N(r) work that is proportional to N^2), their normalisation to
 *     g_ab(r), and the sine transform to S(Q) of Eq. 1;
 *   - a Gaussian-broadened histogram with the gradient of a chi^2 misfit in
 *     S(Q) with respect to every coordinate, and the energy gradient.
 *
 * Conventions shared by every entry point
 *   - Every function returns an nd_status; ND_OK is 0, errors are negative.
 *     nd_last_error() returns a thread-local description of the last error
 *     (valid until the next call on the same thread).  No C++ exception
 *     crosses this boundary.
 *   - All arguments are validated before any device work is enqueued.  A
 *     call that fails leaves the box unchanged unless stated otherwise.
 *   - Coordinates are float32 in structure-of-arrays order [3][N]: all x,
 *     then all y, then all z, each in [0, L) of a cubic periodic box.
 *   - `where` says where a caller pointer lives: ND_HOST (pageable or pinned
 *     host memory; the call copies and synchronises) or ND_DEVICE (device
 *     memory on the machine's GPU; the call is asynchronous on the box's stream
 *     and the caller synchronises before reading results).
 *   - The caller owns every array it passes.  Host inputs are copied; the
 *     library keeps no caller pointer after a call returns.
 *   - Species are 0 .. M-1 with M <= ND_MAX_SPECIES.  The P = M(M+1)/2 pair
 *     types (a <= b) are ordered (0,0), (0,1), ..., (0,M-1), (1,1), ...: the
 *     index of (a, b) is a*M - a(a-1)/2 + (b - a).
 *   - A box is used by one host thread at a time.
 */
#ifndef NEUDA_H
#define NEUDA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t nd_status;

#define ND_OK 0
#define ND_E_INVALID (-1)     /* NULL pointer, NaN input, bad size or flag       */
#define ND_E_RANGE (-2)       /* cutoff or histogram range beyond L/2, species  */
#define ND_E_OOM (-3)         /* device allocation failed                        */
#define ND_E_HIP (-4)         /* HIP runtime or kernel launch failure            */
#define ND_E_STATE (-5)       /* call not valid in the box's state (no tables)   */
#define ND_E_UNSUPPORTED (-6) /* valid request the library does not implement    */

#define ND_HOST 0
#define ND_DEVICE 1

#define ND_ORDER_SEQ 0    /* trial t moves unit t mod n_units                    */
#define ND_ORDER_RANDOM 1 /* trial t moves unit floor(u_7 n_units), u_7 its draw 7 */

#define ND_MAX_SPECIES 4
#define ND_MAX_UNIT_ATOMS 8
#define ND_ABI_VERSION 1

typedef struct nd_box nd_box;

/* Description of a periodic box of atoms grouped into rigid units (the
 * paper's Atom / Molecule / SimBox classes, Sec. "Algorithmic Flow" I).
 * All pointers are host pointers and are copied by nd_box_create. */
typedef struct nd_box_desc {
    int32_t n_atoms;              /* N >= 2                                     */
    int32_t n_species;            /* M, 1 .. ND_MAX_SPECIES                      */
    double L;                     /* box edge in Angstrom, > 0                   */
    const uint8_t *species;       /* [N], values < M                             */
    int32_t n_units;              /* >= 1                                        */
    const int32_t *unit_offsets;  /* [n_units + 1], 0 = off[0] < off[1] < ... = N,
                                     at most ND_MAX_UNIT_ATOMS atoms per unit    */
    const float *xyz;             /* [3][N] in [0, L)                            */
    int32_t device;               /* HIP device ordinal                          */
    void *stream;                 /* hipStream_t for all work, NULL = default   */
} nd_box_desc;

/* Parameters of a Metropolis run (Sec. "Algorithmic Flow" III). */
typedef struct nd_mc_params {
    double kT;          /* kJ/mol, > 0                                            */
    double max_disp;    /* translation half-width per axis, Angstrom, >= 0        */
    double max_rot;     /* rotation half-angle, radians, >= 0 (units of >1 atom)  */
    int32_t order;      /* ND_ORDER_SEQ or ND_ORDER_RANDOM                        */
    int32_t k_batch;    /* trials evaluated together; 0 = chosen by the library   */
    double tie_rel;     /* near-tie threshold (see nd_mc_sweep); 0 = 1e-6         */
    int32_t scan;       /* ND_SCAN_CELLS (default) or ND_SCAN_FULL                 */
    double atom_frac;   /* share of single-atom moves (flexible molecules), 0..1  */
    double atom_disp;   /* their translation half-width per axis, Angstrom, >= 0  */
} nd_mc_params;

/* How nd_mc_sweep finds the atoms within the cutoff of a moved unit.  Both
 * give the same energy changes (pairs beyond r_cut contribute exactly 0):
 * ND_SCAN_CELLS visits only atoms in spatial cells that can be within reach
 * (atoms sorted by cell, rebuilt once per sweep); ND_SCAN_FULL tests every
 * atom of the box for every trial, the O(N) scan of the paper. */
#define ND_SCAN_CELLS 0
#define ND_SCAN_FULL 1

/* Counters of one nd_mc_sweep call. */
typedef struct nd_mc_stats {
    int64_t trials;     /* trials evaluated                                       */
    int64_t accepted;   /* trials accepted                                        */
    int64_t near_ties;  /* decisions within the near-tie band                     */
    double E_total;     /* running total energy after the call                    */
    double dE_sum;      /* sum of accepted energy changes                         */
} nd_mc_stats;

/* Optional per-trial record of nd_mc_sweep: device arrays of n_trials. */
typedef struct nd_mc_trace {
    double *dE;         /* energy change of each trial (accepted or not)          */
    double *sabs;       /* sum over the trial's pair terms of |U| (old and new)  */
    uint8_t *accepted;  /* 1 if accepted                                          */
    int32_t *unit;      /* unit moved by the trial                                */
} nd_mc_trace;

int32_t nd_abi_version(void);
const char *nd_last_error(void);

/* Creates a box on desc->device.  Copies species, units and coordinates to
 * the device.  *out receives the handle; nd_box_destroy releases it.
 * Errors: ND_E_INVALID (bad sizes, NULL, NaN or out-of-box coordinates,
 * species >= M, non-increasing offsets, units larger than
 * ND_MAX_UNIT_ATOMS), ND_E_OOM, ND_E_HIP. */
nd_status nd_box_create(const nd_box_desc *desc, nd_box **out);

/* Releases the box and its device memory after its stream drains.
 * NULL is accepted.  Reached when the HIP runtime is no longer usable (a
 * release during process teardown), it frees the host side only and leaves
 * the device memory to the end of the process. */
nd_status nd_box_destroy(nd_box *box);

/* Sets the stream used by later calls on the box (NULL = default stream). */
nd_status nd_box_set_stream(nd_box *box, void *stream);

/* Replaces all coordinates ([3][N], where = ND_HOST or ND_DEVICE).  Host
 * input must be finite and in [0, L) (ND_E_INVALID otherwise).  Device
 * input is wrapped into the box, x - L floor(x/L) rounded to float32 (a
 * result of L becomes 0), in a staging copy; a value that is not finite
 * gives ND_E_INVALID and leaves the box unchanged.  The device path
 * synchronises the box's stream.  keep_energy = 0 marks the running energy
 * stale (the next nd_mc_sweep, nd_batch_run or nd_box_total_energy
 * recomputes it); 1 keeps the running value (the caller asserts the energy
 * did not change, e.g. when restoring the same coordinates). */
nd_status nd_box_set_coords(nd_box *box, const float *xyz, int32_t where, int32_t keep_energy);

/* Copies the current coordinates ([3][N]) out. */
nd_status nd_box_get_coords(nd_box *box, float *xyz, int32_t where);

/* Sets the tabulated pair potentials U_p(k h), k = 0 .. n_pts-1 (host
 * float32 [P][n_pts]): reference potential plus empirical potential per
 * pair type (Sec. "Algorithmic Principle").  Between grid points the
 * energy is the linear interpolant; it is zero for r >= r_cut.
 * Requires h > 0, r_cut <= L/2 and n_pts >= r_cut/h + 1.  Pairs inside one
 * unit are excluded from all energies.  Errors: ND_E_INVALID, ND_E_RANGE. */
nd_status nd_box_set_tables(nd_box *box, const float *U, int32_t n_pts, double h, double r_cut);

/* Intramolecular harmonic terms between every two atoms of a unit (the
 * flexible molecules of Sec. "Correctness", whose shape is kept by harmonic
 * oscillator potentials between every two atoms):
 *   V_intra = sum over pairs a < b of one unit of k_p (r_ab - r0_ab)^2,
 * k host double [P] per pair type (kJ/mol/A^2, >= 0), r0_ab the pair's
 * nearest-image length in the box's current coordinates (taken in FP64 when
 * this is called: the reference geometry).  Every energy of the library
 * (nd_mc_sweep's energy changes, nd_box_total_energy, nd_forces) then
 * includes V_intra.  k = NULL removes the terms.  The running energy becomes
 * stale.  Errors: ND_E_INVALID (negative or non-finite k). */
nd_status nd_box_set_intra(nd_box *box, const double *k);

/* Recomputes the total energy over all pairs in different units from
 * scratch (FP32 pair terms, FP64 sum), stores it as the running total and
 * writes it to *E (host).  Synchronises the box's stream. */
nd_status nd_box_total_energy(nd_box *box, double *E);

/* Reads the running total energy (host).  Synchronises the stream. */
nd_status nd_box_energy(nd_box *box, double *E);

/* Runs trials first_trial .. first_trial + n_trials - 1 of the Metropolis
 * chain (Sec. "Algorithmic Flow" III, where units move in sequence or at
 * random): trial t moves unit t mod n_units (ND_ORDER_SEQ) or unit
 * floor(u_7 n_units) of its draw 7 (ND_ORDER_RANDOM).  It proposes a
 * translation (uniform in [-max_disp, max_disp] per axis) and, for units of more than
 * one atom, a rotation by an angle uniform in [-max_rot, max_rot] about a
 * uniform axis through the unit's unweighted centroid.  With atom_frac > 0,
 * a trial whose draw 8 is below atom_frac instead translates one atom of the
 * unit, floor(u_9 na), by up to atom_disp per axis (flexible molecules,
 * Sec. "Correctness": the molecule's translation and rotation, and the
 * translation of one of its atoms).  The energy change
 * dE of the unit against every atom outside it decides acceptance:
 * accept iff dE <= 0 or u < exp(-dE/kT).  Random draws come from
 * SplitMix64 seeded with `seed` (output 16 t + d is draw d of trial t), so
 * a run split over several calls equals one call over the same trials.
 * The result equals the sequential chain; trials are evaluated in batches
 * of distinct units whose interactions are corrected exactly (in random
 * order a batch ends before the first repeated unit, so batches are
 * shorter, about sqrt(pi n_units / 2) trials).  A decision with
 * |ln u + dE/kT| < tie_rel * sabs / kT is counted as a near tie.
 * A running energy made stale by nd_box_set_coords or nd_box_set_tables is
 * recomputed over all pairs before the first trial, so stats->E_total is
 * always the energy of the final configuration.
 * stats (host, may be NULL) synchronises; trace (device arrays, may be
 * NULL) records every trial.  Errors: ND_E_INVALID, ND_E_STATE (no
 * tables), ND_E_HIP. */
nd_status nd_mc_sweep(nd_box *box, const nd_mc_params *params, uint64_t seed,
                      uint64_t first_trial, int64_t n_trials, nd_mc_stats *stats,
                      const nd_mc_trace *trace);

/* Pair-count histogram N_p(k) of every unordered pair i < j (atoms of one
 * unit included), counts uint64 [P][nbins].  Per pair, in FP64: the
 * nearest-image displacement of the float32 coordinates, r2 =
 * fma(dz,dz, fma(dy,dy, dx*dx)), and bin k = max{k : (k dr)^2 <= r2},
 * counted iff r2 < (nbins dr)^2.  Counts are exact.  Requires dr > 0,
 * nbins >= 1 and nbins*dr < L/2 (1 - 1e-9).  Errors: ND_E_INVALID,
 * ND_E_RANGE, ND_E_OOM, ND_E_HIP. */
nd_status nd_pair_histogram(nd_box *box, double dr, int32_t nbins, uint64_t *counts, int32_t where);

/* g_p(k) = n_p(k) / (npairs_p Vshell(k) / V), Vshell(k) = (4 pi/3)((k+1)^3 -
 * k^3) dr^3, for counts uint64 [P][nbins] and npairs double [P] (host).
 * Output g double [P][nbins].  counts and g live in `where`. */
nd_status nd_gr_normalize(const uint64_t *counts, int32_t P, int32_t nbins, double dr, double V,
                          const double *npairs, double *g, int32_t where, void *stream);

/* As nd_gr_normalize for real-valued counts (double [P][nbins]), such as the
 * Gaussian-broadened histogram of nd_hist_broad. */
nd_status nd_gr_normalize_f64(const double *counts, int32_t P, int32_t nbins, double dr, double V,
                              const double *npairs, double *g, int32_t where, void *stream);

/* Number of distinct atom pairs of each pair type (host double [P]):
 * N_a (N_a - 1)/2 for like species, N_a N_b for unlike species (the pair
 * counts that normalise g_ab(r), Eq. 1). */
nd_status nd_box_pair_counts(nd_box *box, double *npairs);

/* ---- Running histogram and its accumulation (Sec. "Acceleration method":
 * Delta N(r) is recomputed after every Monte Carlo step at a cost
 * proportional to N, the full N(r) at a cost proportional to N^2; Sec.
 * "NeuDATool Algorithmic Flow", steps EPMC and "Accumulate g(r) and S(Q)").
 *
 * nd_box_track_histogram starts keeping a running N(r) of the box: the
 * counts of nd_pair_histogram(dr, nbins) of the current coordinates, to
 * which every later nd_mc_sweep adds the Delta N(r) of each accepted move
 * (the change of every pair with an atom in a moved unit, by the same
 * exact bin rule), so the running counts stay equal to a fresh
 * nd_pair_histogram bit for bit.  Coordinates changed otherwise
 * (nd_box_set_coords, nd_box_load, the batched form's sweeps) are counted
 * afresh before the next use.  nbins = 0 stops tracking and frees its
 * memory; restarting clears the accumulated samples.  Requires dr > 0 and
 * nbins * dr < L/2.  Errors: ND_E_INVALID, ND_E_RANGE, ND_E_UNSUPPORTED
 * (P * nbins beyond the kernel's LDS), ND_E_OOM, ND_E_HIP. */
nd_status nd_box_track_histogram(nd_box *box, double dr, int32_t nbins);

/* Copies the running counts (uint64 [P][nbins]) to `where`.  Errors:
 * ND_E_STATE when no histogram is tracked. */
nd_status nd_box_tracked_histogram(nd_box *box, uint64_t *counts, int32_t where);

/* Adds the running counts to the box's sum of samples (one sample), on the
 * box's stream.  Errors: ND_E_STATE when no histogram is tracked. */
nd_status nd_box_accumulate(nd_box *box);

/* Mean of the accumulated samples, double [P][nbins] in `where`, and the
 * number of samples (host, may be NULL).  g(r) and S(Q) are linear in the
 * counts, so nd_gr_normalize_f64 and nd_sq_transform of the mean give the
 * averaged g(r) and S(Q).  Errors: ND_E_STATE when no histogram is tracked
 * or no sample was taken. */
nd_status nd_box_accumulated(nd_box *box, double *mean_counts, int64_t *n_samples, int32_t where);

/* Volume V = L^3 (Angstrom^3) and number density rho = N / V (atoms per
 * Angstrom^3) of the box (host doubles): the V of the g(r) normalisation
 * and the rho of Eq. 1. */
nd_status nd_box_density(nd_box *box, double *V, double *rho);

/* Eq. 1 coefficients of the box for scattering lengths b (host double [M]):
 * w_p = (2 - delta_ab) c_a c_b b_a b_b (host double [P]) and the flat term
 * sum_a c_a b_a^2, with c_a = N_a / N the atomic fractions. */
nd_status nd_eq1_weights(nd_box *box, const double *b, double *w, double *self_term);

/* chi^2 = sum_i (S_i - T_i)^2 over nQ points and its gradient
 * dchi^2/dS_i = 2 (S_i - T_i).  S, T, grad (double [nQ], grad may be NULL)
 * and chi2 (double [1]) live in `where`. */
nd_status nd_chi2(const double *S, const double *T, int32_t nQ, double *chi2, double *grad,
                  int32_t where, void *stream);

/* Eq. 1 by the midpoint rule on r_k = (k + 1/2) dr:
 *   S(Q_i) = self_term + sum_p w_p 4 pi rho sum_k r_k^2 (g_p(k) - 1) sinc(Q_i r_k) dr
 * with w_p = (2 - delta_ab) c_a c_b b_a b_b (host double [P]) and
 * self_term = sum_a c_a b_a^2.  g double [P][nbins], Q double [nQ] and
 * S double [nQ] live in `where`.  FP64 throughout. */
nd_status nd_sq_transform(const double *g, int32_t P, int32_t nbins, double dr, double rho,
                          const double *w, double self_term, const double *Q, int32_t nQ,
                          double *S, int32_t where, void *stream);

/* Gaussian-broadened histogram: each pair with r < L/2 adds
 * Phi((e_{k+1} - r)/sigma) - Phi((e_k - r)/sigma), e_k = k dr, to the bins
 * that intersect [r - 6 sigma, r + 6 sigma].  nhat double [P][nbins]. */
nd_status nd_hist_broad(nd_box *box, double dr, int32_t nbins, double sigma, double *nhat,
                        int32_t where);

/* Adjoint of nd_gr_normalize followed by nd_sq_transform: given dL/dS
 * (double [nQ]), A_p(k) = sum_i dL/dS_i w_p 4 pi rho r_k^2 sinc(Q_i r_k) dr /
 * (npairs_p Vshell(k)/V).  dLdS, Q and A ([P][nbins]) live in `where`. */
nd_status nd_sq_adjoint(const double *dLdS, int32_t P, int32_t nbins, double dr, double rho,
                        double V, const double *w, const double *npairs, const double *Q,
                        int32_t nQ, double *A, int32_t where, void *stream);

/* Backward of nd_hist_broad: given A = dL/dnhat (double [P][nbins]), writes
 * dL/dx (double [3][N]) = sum over pairs of dL/dr (x_i - x_j)/r with
 * dL/dr = sum_k A_p(k) (phi((e_k - r)/sigma) - phi((e_{k+1} - r)/sigma))/sigma
 * (coincident atoms, r = 0, contribute nothing).  The pair terms are summed
 * as integers in units of a power of two set by max |A| (a quantum of
 * 2^-45 of the largest possible term at 1e5 atoms), so the result does not
 * depend on the order of the sums (repeated calls agree bit for bit);
 * if A holds a NaN or an infinity every output is NaN. */
nd_status nd_hist_broad_backward(nd_box *box, double dr, int32_t nbins, double sigma,
                                 const double *A, double *dLdx, int32_t where);

/* Energy gradient dE/dx (double [3][N]) over pairs in different units with
 * r < r_cut, using the slope of the interpolated table, and the total
 * energy E (host double, may be NULL).  The gradient's pair terms are summed
 * as integers in units of a power of two set by the table's steepest step
 * and the energy in a fixed order, so repeated calls agree bit for bit; a
 * table holding a NaN or an infinity gives NaN everywhere. */
nd_status nd_forces(nd_box *box, double *dEdx, double *E, int32_t where);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving or optimisation loops, harnesses that forbid
 * hipMalloc): nd_forces with device outputs only -- dEdx device double
 * [3][N], E device double [1] or NULL -- that allocates nothing.  Its
 * kernels use a fixed scratch array built into the library instead of the
 * box's workspace: one per GPU, 12.6 MB (ND_NOALLOC_MAX_ATOMS atoms), held
 * until the process ends, its address looked up on a device's first call.
 * Every call on a GPU shares that GPU's array (each call clears what it
 * sums), so calls that overlap in time on one GPU -- on different streams
 * or from different host threads -- race and must not be issued.
 * Asynchronous on the box's stream; results equal nd_forces bit for bit.
 * Errors: ND_E_INVALID (NULL dEdx), ND_E_STATE (no tables), ND_E_RANGE
 * (N > ND_NOALLOC_MAX_ATOMS), ND_E_HIP. */
#define ND_NOALLOC_MAX_ATOMS 262144
nd_status nd_forces_noalloc(nd_box *box, double *dEdx, double *E);

/* Checkpoint of a box's Metropolis state: coordinates, running energy and
 * (when live) the cell lists, so that a run resumed from the checkpoint
 * repeats the uninterrupted run bit for bit.  The image is a flat byte
 * buffer owned by the caller, ending in an FNV-1a 64-bit hash.
 * nd_box_save with buf = NULL stores the needed size in *len; otherwise
 * *len is the buffer size on entry and the bytes written on return
 * (ND_E_INVALID if too small).  Synchronises the box's stream.
 * nd_box_load restores an image into a box with the same atom count,
 * species count, unit count and L (tables are not part of the image);
 * errors: ND_E_INVALID (not an image, other box, truncated, hash mismatch,
 * corrupt cell order), ND_E_HIP. */
nd_status nd_box_save(nd_box *box, void *buf, size_t *len);
nd_status nd_box_load(nd_box *box, const void *buf, size_t len);

/* ---- Batched form: several independent boxes in one graph launch.
 * The boxes may differ in size, box length, tables and Eq. 1 weighting
 * (e.g. isotope substitutions; Sec. "Neutron scattering" and Eq. 1).  One
 * run does, for every box, `sweeps` Metropolis sweeps (n_units trials per
 * sweep, as nd_mc_sweep with the cell scan), then the pair histogram, g(r)
 * and S(Q) as nd_pair_histogram, nd_gr_normalize and nd_sq_transform.  Each
 * launch of the run covers every box at once (one grid row per box; the
 * histogram is one persistent launch over the tile pairs of all boxes).
 * The launches are captured into a HIP graph on the first run and the graph
 * is replayed by later runs with the same launch structure (same boxes,
 * sweeps, batch sizes, bin counts and output arrays); other arguments
 * (seeds, trial counters, weights) may change between replays.  Every run
 * rebuilds the boxes' cell lists first.
 *
 * The batch keeps pointers to the boxes: destroy the batch before any of
 * its boxes, and do not run nd_* calls on its boxes while a run is in
 * flight except on the boxes' own streams (the run waits for work already
 * queued on each box's stream and work queued on them afterwards waits for
 * the run). */
typedef struct nd_batch nd_batch;

typedef struct nd_batch_plan {
    int32_t sweeps;               /* Metropolis sweeps per box, 0 = none          */
    const nd_mc_params *mc;       /* host [n]: scan must be ND_SCAN_CELLS         */
    const uint64_t *seed;         /* host [n]                                     */
    const uint64_t *first_trial;  /* host [n]: counter of each box's first trial  */
    double dr;                    /* histogram bin width (Angstrom)               */
    const int32_t *nbins;         /* host [n]: bins of box i, nbins*dr < L_i/2    */
    const double *w;              /* host [n][P]: Eq. 1 weights of box i          */
    const double *self_term;      /* host [n]: sum_a c_a b_a^2 of box i           */
    const double *Q;              /* device [nQ], shared by all boxes             */
    int32_t nQ;
    uint64_t *const *counts;      /* host [n] of device [P][nbins_i]; NULL: no histogram */
    double *const *g;             /* host [n] of device [P][nbins_i]; NULL: no g or S    */
    double *const *S;             /* host [n] of device [nQ]; NULL or nQ = 0: no S       */
    const nd_mc_trace *trace;     /* host [n] or NULL: per-trial record of box i's sweeps
                                     (device arrays of sweeps * n_units_i entries, as for
                                     nd_mc_sweep; any member may be NULL)              */
} nd_batch_plan;

/* Groups n >= 1 distinct boxes on one device with the same number of
 * species.  Errors: ND_E_INVALID, ND_E_HIP. */
nd_status nd_batch_create(nd_box *const *boxes, int32_t n, nd_batch **out);

/* NULL-safe; waits for the batch's work to finish. */
nd_status nd_batch_destroy(nd_batch *batch);

/* One run of the plan (see above), asynchronous on the batch's own stream.
 * stats: host [n] or NULL; when given, the call waits for the run and fills
 * the counters of each box's sweeps.  Errors: ND_E_INVALID, ND_E_RANGE,
 * ND_E_STATE (a box without tables), ND_E_UNSUPPORTED (ND_SCAN_FULL),
 * ND_E_OOM, ND_E_HIP. */
nd_status nd_batch_run(nd_batch *batch, const nd_batch_plan *plan, nd_mc_stats *stats);

/* Number of graph captures and of graph launches of the batch so far. */
nd_status nd_batch_info(const nd_batch *batch, int64_t *captures, int64_t *launches);

/* ---- Empirical-potential refinement (Sec. "Algorithmic Principle": the
 * EMP is the Fourier counterpart of the difference dS(Q) between measured
 * and simulated S(Q), fitted by a series of Poisson functions in Q space and
 * added to the reference potential; Sec. "Correctness", Eq. 2: the EMP of
 * each pair type through the inverse of the Eq. 1 weight matrix of the
 * measured profiles, enlarged by a unit matrix when there are fewer profiles
 * than pair types; Sec. "NeuDATool Algorithmic Flow", step EPMC: update,
 * re-equilibrate, repeat).
 *
 * Poisson functions, normalised so that 4 pi rho int r^2 p_n dr = 1:
 *   p_n(r) = (r/s)^n exp(-r/s) / (4 pi rho s^3 (n+2)!),  n = 1 .. n_terms,
 * with the Eq. 1 transform 4 pi rho int r^2 p_n(r) sin(Qr)/(Qr) dr
 *   P_n(Q) = sin((n+2) a) / ((n+2) Q s (1 + Q^2 s^2)^((n+2)/2)),  a = atan(Q s).
 * One update: S_sim,i by Eq. 1 from the model's g(r) with profile i's
 * weights W[i][.] and flat term; dS_i = S_exp,i - S_sim,i; least-squares
 * coefficients c_i of dS_i in the P_n (normal equations plus ridge * tr/n
 * on the diagonal); the pair types' coefficients C_p = sum_i W+[p][i] c_i
 * (W+ = W^-1 when there are as many profiles as pair types, else the
 * pseudo-inverse of W stacked over id_weight times the unit matrix); the
 * update dU_p(r) = -feedback kT sum_n C_pn p_n(r), shifted to zero at the
 * cutoff and zero beyond, added to the box's EMP (which nd_box_set_tables
 * resets to zero); if emp_max > 0 the EMP is then scaled so that
 * max |EMP| <= emp_max; the box's tables become (float)(reference + EMP).
 * The running energy becomes stale (the next sweep recomputes it). */
#define ND_EMP_MAX_TERMS 64
#define ND_EMP_MAX_PROFILES 8

typedef struct nd_emp_params {
    double sigma;       /* width s of the Poisson functions, Angstrom, > 0        */
    int32_t n_terms;    /* number of Poisson functions, 1 .. ND_EMP_MAX_TERMS     */
    int32_t pad;
    double feedback;    /* fraction of the fitted potential applied, > 0          */
    double kT;          /* energy scale, kJ/mol, > 0                              */
    double ridge;       /* relative ridge of the fit, >= 0                        */
    double id_weight;   /* weight of the unit-matrix rows (fewer profiles), > 0   */
    double emp_max;     /* cap on max |EMP| in kJ/mol, 0 = none                   */
} nd_emp_params;

/* One EMP update of `box` from n_prof measured profiles: W host double
 * [n_prof][P] (Eq. 1 weights of each profile, as nd_eq1_weights gives for its
 * scattering lengths), self_terms host double [n_prof]; g device double
 * [P][nbins] (the model's g(r), bins of width dr); Q device double [nQ];
 * S_exp device double [n_prof][nQ].  Optional device outputs (NULL to skip):
 * dS [n_prof][nQ], the EMP after the update [P][n_pts], the update's
 * coefficients C [P][n_terms].  Asynchronous on the box's stream.  Errors:
 * ND_E_INVALID (bad sizes or parameters, W singular when square),
 * ND_E_STATE (no tables), ND_E_HIP. */
nd_status nd_emp_update(nd_box *box, const nd_emp_params *params, int32_t n_prof, const double *W,
                        const double *self_terms, const double *g, int32_t nbins, double dr, const double *Q,
                        int32_t nQ, const double *S_exp, double *dS, double *emp, double *C);

/* Copies the box's tables as used by the energy kernels (float32 [P][n_pts]:
 * reference potential plus EMP) to `where`.  Errors: ND_E_STATE (no tables). */
nd_status nd_box_get_tables(nd_box *box, float *U, int32_t where);

/* ---- Tuning table.  Launch parameters chosen per size class by a tuner
 * (the package's autotune module writes them to a text file that the
 * binding loads at start-up); without an entry the library's built-in
 * choices apply.  Entries of one kind are looked up by atom count: the
 * first entry (in the order given) with n <= n_max applies.  The table is
 * process-wide; set it before the calls it should affect (a batched run
 * captured earlier keeps its launch structure until that changes). */
#define ND_TUNE_BOX 0    /* nd_mc_sweep and nd_pair_histogram of a box of n atoms */
#define ND_TUNE_BATCH 1  /* nd_batch_run over boxes of n atoms in total           */

typedef struct nd_tuning {
    int32_t kind;               /* ND_TUNE_BOX or ND_TUNE_BATCH                        */
    int32_t scan_waves;         /* waves per trial of the cell scan: 1, 2 or 4; 0 = built in */
    int64_t n_max;              /* largest atom count the entry applies to             */
    double batch_target;        /* expected interacting earlier trials per trial at the
                                   end of a Metropolis batch; sets the batch size
                                   K = target / f (f the share of the box within reach,
                                   K <= 2048 and <= n_units / 2); 0 = built in (18)    */
    int32_t hist_blocks_per_cu; /* pair histogram: 256-thread groups per compute unit,
                                   1..8, capped by LDS.  The single-box kernel packs
                                   four groups into a block that shares one LDS
                                   histogram (1..4: one block per CU, 5..8: two); the
                                   several-box kernel runs one group per block.
                                   0 = built in (8 single-box, 5 several-box)          */
    int32_t pad;
} nd_tuning;

/* Replaces the table with n entries (n = 0 clears it).  Errors:
 * ND_E_INVALID (bad kind, scan_waves, negative target, blocks per CU). */
nd_status nd_set_tuning(const nd_tuning *entries, int32_t n);

/* Copies at most cap entries to `entries` (may be NULL when cap = 0) and the
 * table's size to *n. */
nd_status nd_get_tuning(nd_tuning *entries, int32_t cap, int32_t *n);

/* Replaces the table with the entries of a text file: one entry per line,
 * "box|batch n_max scan_waves batch_target hist_blocks_per_cu", blank lines
 * and lines starting with '#' ignored.  Errors: ND_E_INVALID (unreadable
 * file or malformed line; the table is then unchanged). */
nd_status nd_load_tuning(const char *path);

/* Per-kernel timing with HIP events on the box's stream, for measurement.
 * Kernel ids for nd_box_profile. */
#define ND_PROF_MC_SCAN 0       /* pair-sum scan of a batch of trials        */
#define ND_PROF_MC_CORR 1       /* in-batch interaction corrections           */
#define ND_PROF_MC_DECIDE 2     /* Metropolis decisions and commit            */
#define ND_PROF_MC_PROPOSE 3    /* trial proposals                            */
#define ND_PROF_PAIR_HIST 4     /* pair-count histogram (main kernel)         */
#define ND_PROF_HIST_BROAD 5    /* broadened histogram (main kernel)          */
#define ND_PROF_HIST_BROAD_BWD 6 /* broadened histogram backward              */
#define ND_PROF_FORCES 7        /* energy gradient                            */
#define ND_PROF_KINDS 8

/* enable = 1 starts recording an event pair around every launch of the
 * kernels above on this machine and clears the totals; 0 stops recording. */
nd_status nd_box_set_profiling(nd_box *box, int32_t enable);

/* The same for a subset: bit k of `kernels` (1 << ND_PROF_*) selects kernel
 * id k; the other kernels launch without events (an event pair adds a few
 * microseconds to a launch on the stream).  0 stops recording.  Errors:
 * ND_E_INVALID for bits past ND_PROF_KINDS. */
nd_status nd_box_set_profiling_mask(nd_box *box, uint32_t kernels);

/* Counts, for measurement, the work of the cell scan of later nd_mc_sweep
 * calls on the box: the candidate atoms tested against each trial's reach
 * sphere and the survivors whose pair terms are evaluated.  Each call first
 * returns the counts since the last call (host, may be NULL; zero when
 * counting was off), then restarts them (enable = 1) or stops counting
 * (enable = 0).  Counting adds device atomics to the scan; leave it off in
 * timed runs.  Synchronises the box's stream. */
nd_status nd_box_count_scan(nd_box *box, int32_t enable, int64_t *candidates, int64_t *survivors);

/* Synchronises the box's stream and returns the number of recorded launches
 * of `kernel` and their summed duration in milliseconds since profiling was
 * enabled.  Errors: ND_E_INVALID for an unknown kernel id. */
nd_status nd_box_profile(nd_box *box, int32_t kernel, int64_t *launches, double *ms);

#ifdef __cplusplus
}
#endif

#endif /* NEUDA_H */

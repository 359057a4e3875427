/*
 * FP64 CPU oracle for the pair-sum path of the EPSR-style refinement in
 * "NeuDATool" (arXiv 1904.08756).
 *
 * TEST INFRASTRUCTURE ONLY.  This file exists to check the HIP library; it
 * is loaded by the tests, by the smoke check and by the CPU-baseline leg of
 * the benchmark, and by nothing else.  It shares no code, header, table or
 * constant generator with the library: both sides are written separately
 * from the paper's definitions and only consume the same seeded inputs.
 *
 * Everything is plain double precision, loop by loop, in the order of the
 * definitions.  Build with -ffp-contract=off so no multiply-add is fused
 * unless written as fma() explicitly.
 *
 * Conventions
 *   xyz      float32 [3][N] (x row, y row, z row), wrapped into [0, L)
 *   species  uint8 [N], values < M
 *   uoff     int32 [n_units + 1], atoms of unit u are uoff[u] .. uoff[u+1]-1
 *   tables   float32 [P][n_pts], P = M(M+1)/2, U_p(k h) for k < n_pts
 *   pair type index of species (a <= b): a*M - a(a-1)/2 + (b - a)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_TWO_PI 6.283185307179586

int orc_abi_version(void) { return 1; }

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------ */
/* Random numbers.  The paper does not specify a generator; the trial  */
/* draws use SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): the i-th     */
/* output of the generator seeded with s is mix(s + (i+1) * gamma).     */
/* Draw d of trial t is output number 16 t + d.                         */
/* ------------------------------------------------------------------ */
uint64_t orc_splitmix64(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + 0x9E3779B97F4A7C15ULL * (i + 1u);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

double orc_uniform(uint64_t seed, uint64_t trial, int draw)
{
    uint64_t x = orc_splitmix64(seed, 16u * trial + (uint64_t)draw);
    return (double)(x >> 11) * (1.0 / 9007199254740992.0);
}

/* ------------------------------------------------------------------ */
/* Geometry and pair energy.                                           */
/* ------------------------------------------------------------------ */
int orc_pair_index(int a, int b, int M)
{
    if (a > b) { int t = a; a = b; b = t; }
    return a * M - a * (a - 1) / 2 + (b - a);
}

/* Nearest periodic image of a displacement d in (-L, L). */
static double min_image(double d, double L)
{
    double half = 0.5 * L;
    if (d > half) return d - L;
    if (d < -half) return d + L;
    return d;
}

/* Linear interpolation in a tabulated potential row; zero from r_cut on. */
double orc_table_u(const float *row, int n_pts, double h, double r_cut, double r)
{
    if (!(r < r_cut)) return 0.0;
    double t = r / h;
    int i0 = (int)floor(t);
    if (i0 > n_pts - 2) i0 = n_pts - 2;
    double f = t - (double)i0;
    double a = (double)row[i0];
    double b = (double)row[i0 + 1];
    return a + f * (b - a);
}

/* Slope of the interpolant used by orc_table_u (0 from r_cut on). */
double orc_table_du(const float *row, int n_pts, double h, double r_cut, double r)
{
    if (!(r < r_cut)) return 0.0;
    double t = r / h;
    int i0 = (int)floor(t);
    if (i0 > n_pts - 2) i0 = n_pts - 2;
    return ((double)row[i0 + 1] - (double)row[i0]) / h;
}

/* Closed form of the reference potential the tables sample: Lennard-Jones
 * (optionally shifted to zero at r_cut) plus Coulomb shifted to zero at
 * r_cut, in kJ/mol with k_C in kJ mol^-1 A e^-2.  Used only to pin the
 * tabulation and the interpolation. */
double orc_analytic_u(double r, double sigma, double eps, double qq, double kc,
                      double r_cut, int shift_lj)
{
    if (!(r < r_cut)) return 0.0;
    double u = 0.0;
    if (eps != 0.0) {
        double s6 = pow(sigma / r, 6.0);
        double c6 = pow(sigma / r_cut, 6.0);
        u += 4.0 * eps * (s6 * s6 - s6);
        if (shift_lj) u -= 4.0 * eps * (c6 * c6 - c6);
    }
    if (qq != 0.0) u += kc * qq * (1.0 / r - 1.0 / r_cut);
    return u;
}

static double pair_dist(const float *xyz, int N, double L, int i, double px, double py, double pz)
{
    double dx = min_image((double)xyz[i] - px, L);
    double dy = min_image((double)xyz[N + i] - py, L);
    double dz = min_image((double)xyz[2 * N + i] - pz, L);
    return sqrt(dx * dx + dy * dy + dz * dz);
}

/* Total potential energy: every pair of atoms in different units, once.
 * Pairs inside a unit are excluded (rigid units).  Sabs collects the sum
 * of |U| over the contributing pairs. */
void orc_total_energy(int N, double L, int M, const uint8_t *species, const int32_t *unit_of,
                      const float *xyz, const float *tab, int n_pts, double h, double r_cut,
                      double *E_out, double *Sabs_out)
{
    double E = 0.0, S = 0.0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : E, S)
    for (int i = 0; i < N; ++i) {
        double xi = xyz[i], yi = xyz[N + i], zi = xyz[2 * N + i];
        for (int j = i + 1; j < N; ++j) {
            if (unit_of[i] == unit_of[j]) continue;
            double r = pair_dist(xyz, N, L, j, xi, yi, zi);
            const float *row = tab + (size_t)orc_pair_index(species[i], species[j], M) * n_pts;
            double u = orc_table_u(row, n_pts, h, r_cut, r);
            E += u;
            S += fabs(u);
        }
    }
    *E_out = E;
    *Sabs_out = S;
}

/* Energy change when the atoms of unit u move from their positions in xyz
 * to newpos (double [na][3], already float32-representable):
 *   dE = sum_{a in u} sum_{j not in u} U(new_a, x_j) - U(old_a, x_j). */
void orc_delta_e(int N, double L, int M, const uint8_t *species, const int32_t *uoff, int u,
                 const float *xyz, const double *newpos, const float *tab, int n_pts, double h,
                 double r_cut, double *dE_out, double *Sabs_out)
{
    int a0 = uoff[u], a1 = uoff[u + 1];
    double dE = 0.0, S = 0.0;
    for (int a = a0; a < a1; ++a) {
        double ox = xyz[a], oy = xyz[N + a], oz = xyz[2 * N + a];
        const double *np_ = newpos + 3 * (a - a0);
        double sum = 0.0, sabs = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : sum, sabs)
        for (int j = 0; j < N; ++j) {
            if (j >= a0 && j < a1) continue;
            const float *row = tab + (size_t)orc_pair_index(species[a], species[j], M) * n_pts;
            double un = orc_table_u(row, n_pts, h, r_cut, pair_dist(xyz, N, L, j, np_[0], np_[1], np_[2]));
            double uo = orc_table_u(row, n_pts, h, r_cut, pair_dist(xyz, N, L, j, ox, oy, oz));
            sum += un - uo;
            sabs += fabs(un) + fabs(uo);
        }
        dE += sum;
        S += sabs;
    }
    *dE_out = dE;
    *Sabs_out = S;
}

/* Round a position into [0, L) as float32; a result equal to L becomes 0. */
static double wrap_round(double x, double L)
{
    double w = x - L * floor(x / L);
    float f = (float)w;
    if ((double)f >= L || f < 0.0f) f = 0.0f;
    return (double)f;
}

/* Trial move t (paper Sec. "Algorithmic Flow" III: units move in sequence or
 * at random; Sec. "Correctness": molecule translation and rotation, single
 * atom translation).  Writes the proposed positions of the unit's atoms to
 * newpos[na][3] and returns the unit index.  Draws: 0-2 translation, 3-4
 * rotation axis, 5 angle, 7 unit (random order only). */
int orc_propose(int N, double L, int n_units, const int32_t *uoff, const float *xyz,
                double max_disp, double max_rot, int order, uint64_t seed, uint64_t t,
                double *newpos)
{
    int u;
    if (order == 0) u = (int)(t % (uint64_t)n_units);
    else {
        u = (int)floor(orc_uniform(seed, t, 7) * (double)n_units);
        if (u >= n_units) u = n_units - 1;
    }
    int a0 = uoff[u], na = uoff[u + 1] - a0;
    double tau[3];
    for (int c = 0; c < 3; ++c) tau[c] = max_disp * (2.0 * orc_uniform(seed, t, c) - 1.0);

    if (na == 1) {
        for (int c = 0; c < 3; ++c)
            newpos[c] = wrap_round((double)xyz[c * N + a0] + tau[c], L);
        return u;
    }

    /* unwrap the unit around its first atom */
    double p[64][3];
    if (na > 64) return -1;
    for (int a = 0; a < na; ++a)
        for (int c = 0; c < 3; ++c) {
            double x0 = xyz[c * N + a0];
            p[a][c] = x0 + min_image((double)xyz[c * N + a0 + a] - x0, L);
        }
    /* unweighted centroid */
    double cen[3];
    for (int c = 0; c < 3; ++c) {
        double s = 0.0;
        for (int a = 0; a < na; ++a) s += p[a][c];
        cen[c] = s / (double)na;
    }
    /* uniform axis on the sphere, uniform angle in [-max_rot, max_rot] */
    double zc = 2.0 * orc_uniform(seed, t, 3) - 1.0;
    double phi = ORC_TWO_PI * orc_uniform(seed, t, 4);
    double sr = sqrt(1.0 - zc * zc);
    double n[3] = {sr * cos(phi), sr * sin(phi), zc};
    double th = max_rot * (2.0 * orc_uniform(seed, t, 5) - 1.0);
    double ct = cos(th), st = sin(th), omc = 1.0 - ct;
    for (int a = 0; a < na; ++a) {
        double v[3] = {p[a][0] - cen[0], p[a][1] - cen[1], p[a][2] - cen[2]};
        /* Rodrigues: v cos + (n x v) sin + n (n.v)(1 - cos) */
        double cr[3] = {n[1] * v[2] - n[2] * v[1], n[2] * v[0] - n[0] * v[2],
                        n[0] * v[1] - n[1] * v[0]};
        double dot = n[0] * v[0] + n[1] * v[1] + n[2] * v[2];
        double k = dot * omc;
        for (int c = 0; c < 3; ++c) {
            double w = v[c] * ct + cr[c] * st + n[c] * k;
            newpos[3 * a + c] = wrap_round(cen[c] + w + tau[c], L);
        }
    }
    return u;
}

/* Metropolis chain (Sec. "Algorithmic Flow" III): trial t proposes a move,
 * dE is computed against the current configuration, and the move is
 * accepted iff dE <= 0 or u_6 < exp(-dE/kT).  Accepted positions are
 * written back (float32) and E_total advances by dE.
 *
 * Near ties: when |ln u_6 + dE/kT| < tie_rel * Sabs / kT the decision
 * depends on rounding; if `forced` is given, its entry is taken there
 * (the decision of the implementation under test) and the tie is flagged.
 * Per-trial outputs (dE, Sabs, accepted, tie, unit) are optional. */
int64_t orc_mc_run(int N, double L, int M, const uint8_t *species, int n_units,
                   const int32_t *uoff, float *xyz, const float *tab, int n_pts, double h,
                   double r_cut, double kT, double max_disp, double max_rot, int order,
                   uint64_t seed, uint64_t first_trial, int64_t n_trials, double tie_rel,
                   const uint8_t *forced, double *dE_out, double *sabs_out, uint8_t *acc_out,
                   uint8_t *tie_out, int32_t *unit_out, double *E_total)
{
    int64_t n_acc = 0;
    double newpos[64 * 3];
    for (int64_t k = 0; k < n_trials; ++k) {
        uint64_t t = first_trial + (uint64_t)k;
        int u = orc_propose(N, L, n_units, uoff, xyz, max_disp, max_rot, order, seed, t, newpos);
        if (u < 0) return -1;
        double dE, sabs;
        orc_delta_e(N, L, M, species, uoff, u, xyz, newpos, tab, n_pts, h, r_cut, &dE, &sabs);
        double u6 = orc_uniform(seed, t, 6);
        int acc = (dE <= 0.0) || (u6 < exp(-dE / kT));
        int tie = 0;
        if (u6 > 0.0 && fabs(log(u6) + dE / kT) < tie_rel * sabs / kT) {
            tie = 1;
            if (forced) acc = forced[k] ? 1 : 0;
        }
        if (acc) {
            int a0 = uoff[u], a1 = uoff[u + 1];
            for (int a = a0; a < a1; ++a)
                for (int c = 0; c < 3; ++c) xyz[c * N + a] = (float)newpos[3 * (a - a0) + c];
            if (E_total) *E_total += dE;
            ++n_acc;
        }
        if (dE_out) dE_out[k] = dE;
        if (sabs_out) sabs_out[k] = sabs;
        if (acc_out) acc_out[k] = (uint8_t)acc;
        if (tie_out) tie_out[k] = (uint8_t)tie;
        if (unit_out) unit_out[k] = u;
    }
    return n_acc;
}

/* ------------------------------------------------------------------ */
/* Flexible molecules (Sec. "Correctness": the molecule's shape is kept */
/* by harmonic oscillator potentials between every two of its atoms, and */
/* single atoms move besides whole-molecule translations and rotations). */
/*   V_intra = sum over unit pairs a < b of k_p (r_ab - r0_ab)^2,        */
/* k_p per pair type, r0_ab the pair's length in a reference geometry.  */
/* r0 is stored per atom as r0[a * 8 + (b - first atom of the unit)].   */
/* ------------------------------------------------------------------ */
static double dist_pts(double L, const double *p, const double *q)
{
    double dx = min_image(q[0] - p[0], L), dy = min_image(q[1] - p[1], L), dz = min_image(q[2] - p[2], L);
    return sqrt(dx * dx + dy * dy + dz * dz);
}

static void atom_pos(const float *xyz, int N, int a, double p[3])
{
    p[0] = xyz[a];
    p[1] = xyz[N + a];
    p[2] = xyz[2 * N + a];
}

/* Reference lengths r0 of every intramolecular pair from coordinates xyz. */
void orc_intra_reference(int N, double L, int n_units, const int32_t *uoff, const float *xyz, double *r0)
{
    for (size_t q = 0; q < (size_t)N * 8; ++q) r0[q] = 0.0;
    for (int u = 0; u < n_units; ++u)
        for (int a = uoff[u]; a < uoff[u + 1]; ++a)
            for (int b = uoff[u]; b < uoff[u + 1]; ++b) {
                if (a == b) continue;
                double pa[3], pb[3];
                atom_pos(xyz, N, a, pa);
                atom_pos(xyz, N, b, pb);
                r0[(size_t)a * 8 + (b - uoff[u])] = dist_pts(L, pa, pb);
            }
}

/* Total intramolecular energy and the sum of its |terms|. */
void orc_intra_energy(int N, double L, int M, const uint8_t *species, int n_units, const int32_t *uoff,
                      const float *xyz, const double *kint, const double *r0, double *E_out, double *S_out)
{
    double E = 0.0, S = 0.0;
    for (int u = 0; u < n_units; ++u)
        for (int a = uoff[u]; a < uoff[u + 1]; ++a)
            for (int b = a + 1; b < uoff[u + 1]; ++b) {
                double pa[3], pb[3];
                atom_pos(xyz, N, a, pa);
                atom_pos(xyz, N, b, pb);
                double d = dist_pts(L, pa, pb) - r0[(size_t)a * 8 + (b - uoff[u])];
                double v = kint[orc_pair_index(species[a], species[b], M)] * d * d;
                E += v;
                S += fabs(v);
            }
    *E_out = E;
    *S_out = S;
}

/* Gradient of the intramolecular energy added to grad [3][N]:
 * dV/dx_a = sum over the other atoms b of a's unit of 2 k (r - r0) (x_a - x_b) / r. */
void orc_intra_forces(int N, double L, int M, const uint8_t *species, int n_units, const int32_t *uoff,
                      const float *xyz, const double *kint, const double *r0, double *grad)
{
    for (int u = 0; u < n_units; ++u)
        for (int a = uoff[u]; a < uoff[u + 1]; ++a)
            for (int b = uoff[u]; b < uoff[u + 1]; ++b) {
                if (a == b) continue;
                double d[3] = {min_image((double)xyz[a] - (double)xyz[b], L),
                               min_image((double)xyz[N + a] - (double)xyz[N + b], L),
                               min_image((double)xyz[2 * N + a] - (double)xyz[2 * N + b], L)};
                double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                if (r == 0.0) continue;
                double c = 2.0 * kint[orc_pair_index(species[a], species[b], M)] *
                           (r - r0[(size_t)a * 8 + (b - uoff[u])]) / r;
                for (int q = 0; q < 3; ++q) grad[(size_t)q * N + a] += c * d[q];
            }
}

/* Energy change of unit u's intramolecular terms when atoms a0 .. a0+na-1
 * of it move to newpos[na][3] (the others stay). */
static void intra_delta(int N, double L, int M, const uint8_t *species, const int32_t *uoff, int u, int a0,
                        int na, const float *xyz, const double *newpos, const double *kint, const double *r0,
                        double *dE, double *S)
{
    int u0 = uoff[u], u1 = uoff[u + 1];
    double e = 0.0, s = 0.0;
    for (int a = u0; a < u1; ++a)
        for (int b = a + 1; b < u1; ++b) {
            int ma = a >= a0 && a < a0 + na, mb = b >= a0 && b < a0 + na;
            if (!ma && !mb) continue;
            double pa[3], pb[3], qa[3], qb[3];
            atom_pos(xyz, N, a, pa);
            atom_pos(xyz, N, b, pb);
            for (int c = 0; c < 3; ++c) {
                qa[c] = ma ? newpos[3 * (a - a0) + c] : pa[c];
                qb[c] = mb ? newpos[3 * (b - a0) + c] : pb[c];
            }
            double k = kint[orc_pair_index(species[a], species[b], M)];
            double r0ab = r0[(size_t)a * 8 + (b - u0)];
            double dn = dist_pts(L, qa, qb) - r0ab, dold = dist_pts(L, pa, pb) - r0ab;
            double vn = k * dn * dn, vo = k * dold * dold;
            e += vn - vo;
            s += fabs(vn) + fabs(vo);
        }
    *dE = e;
    *S = s;
}

/* Energy change of atoms a0 .. a0+na-1 (all of one unit u) moving to
 * newpos: intermolecular pair terms against every atom outside u. */
static void inter_delta(int N, double L, int M, const uint8_t *species, const int32_t *uoff, int u, int a0, int na,
                        const float *xyz, const double *newpos, const float *tab, int n_pts, double h, double r_cut,
                        double *dE_out, double *Sabs_out)
{
    int u0 = uoff[u], u1 = uoff[u + 1];
    double dE = 0.0, S = 0.0;
    for (int a = a0; a < a0 + na; ++a) {
        double ox = xyz[a], oy = xyz[N + a], oz = xyz[2 * N + a];
        const double *np_ = newpos + 3 * (a - a0);
        double sum = 0.0, sabs = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : sum, sabs)
        for (int j = 0; j < N; ++j) {
            if (j >= u0 && j < u1) continue;
            const float *row = tab + (size_t)orc_pair_index(species[a], species[j], M) * n_pts;
            double un = orc_table_u(row, n_pts, h, r_cut, pair_dist(xyz, N, L, j, np_[0], np_[1], np_[2]));
            double uo = orc_table_u(row, n_pts, h, r_cut, pair_dist(xyz, N, L, j, ox, oy, oz));
            sum += un - uo;
            sabs += fabs(un) + fabs(uo);
        }
        dE += sum;
        S += sabs;
    }
    *dE_out = dE;
    *Sabs_out = S;
}

/* Trial t of a flexible-molecule run: with probability atom_frac (draw 8)
 * one atom of the unit, floor(u_9 na), translates by up to atom_disp per
 * axis (draws 0-2); otherwise the whole unit moves as in orc_propose.
 * Writes the moved atoms' new positions and returns the unit; *a0_out and
 * *na_out give the moved atoms. */
int orc_propose_flex(int N, double L, int n_units, const int32_t *uoff, const float *xyz, double max_disp,
                     double max_rot, int order, double atom_frac, double atom_disp, uint64_t seed, uint64_t t,
                     double *newpos, int *a0_out, int *na_out)
{
    int u;
    if (order == 0) u = (int)(t % (uint64_t)n_units);
    else {
        u = (int)floor(orc_uniform(seed, t, 7) * (double)n_units);
        if (u >= n_units) u = n_units - 1;
    }
    int na = uoff[u + 1] - uoff[u];
    if (orc_uniform(seed, t, 8) < atom_frac) {
        int ai = (int)floor(orc_uniform(seed, t, 9) * (double)na);
        if (ai >= na) ai = na - 1;
        int a = uoff[u] + ai;
        for (int c = 0; c < 3; ++c)
            newpos[c] = wrap_round((double)xyz[c * N + a] + atom_disp * (2.0 * orc_uniform(seed, t, c) - 1.0), L);
        *a0_out = a;
        *na_out = 1;
        return u;
    }
    orc_propose(N, L, n_units, uoff, xyz, max_disp, max_rot, order, seed, t, newpos);
    *a0_out = uoff[u];
    *na_out = na;
    return u;
}

/* The Metropolis chain of orc_mc_run with intramolecular harmonic terms
 * (kint [P], r0 as orc_intra_reference) and single-atom moves. */
int64_t orc_mc_run_flex(int N, double L, int M, const uint8_t *species, int n_units, const int32_t *uoff,
                        float *xyz, const float *tab, int n_pts, double h, double r_cut, double kT, double max_disp,
                        double max_rot, int order, double atom_frac, double atom_disp, const double *kint,
                        const double *r0, uint64_t seed, uint64_t first_trial, int64_t n_trials, double tie_rel,
                        const uint8_t *forced, double *dE_out, double *sabs_out, uint8_t *acc_out, uint8_t *tie_out,
                        int32_t *unit_out, int32_t *atom_out, double *E_total)
{
    int64_t n_acc = 0;
    double newpos[64 * 3];
    for (int64_t k = 0; k < n_trials; ++k) {
        uint64_t t = first_trial + (uint64_t)k;
        int a0, na;
        int u = orc_propose_flex(N, L, n_units, uoff, xyz, max_disp, max_rot, order, atom_frac, atom_disp, seed, t,
                                 newpos, &a0, &na);
        if (u < 0 || na > 64) return -1;
        double dEi, Si, dEa, Sa;
        inter_delta(N, L, M, species, uoff, u, a0, na, xyz, newpos, tab, n_pts, h, r_cut, &dEi, &Si);
        intra_delta(N, L, M, species, uoff, u, a0, na, xyz, newpos, kint, r0, &dEa, &Sa);
        double dE = dEi + dEa, sabs = Si + Sa;
        double u6 = orc_uniform(seed, t, 6);
        int acc = (dE <= 0.0) || (u6 < exp(-dE / kT));
        int tie = 0;
        if (u6 > 0.0 && fabs(log(u6) + dE / kT) < tie_rel * sabs / kT) {
            tie = 1;
            if (forced) acc = forced[k] ? 1 : 0;
        }
        if (acc) {
            for (int a = a0; a < a0 + na; ++a)
                for (int c = 0; c < 3; ++c) xyz[c * N + a] = (float)newpos[3 * (a - a0) + c];
            if (E_total) *E_total += dE;
            ++n_acc;
        }
        if (dE_out) dE_out[k] = dE;
        if (sabs_out) sabs_out[k] = sabs;
        if (acc_out) acc_out[k] = (uint8_t)acc;
        if (tie_out) tie_out[k] = (uint8_t)tie;
        if (unit_out) unit_out[k] = u;
        if (atom_out) atom_out[k] = na == 1 && uoff[u + 1] - uoff[u] > 1 ? a0 : -1;
    }
    return n_acc;
}

/* ------------------------------------------------------------------ */
/* Pair-count histogram N_ab(r) (Sec. "Acceleration method").           */
/* For every unordered pair i < j (same unit included):                */
/*   d = x_j - x_i per axis in double, nearest image by comparison     */
/*   with L/2; r2 = fma(dz,dz, fma(dy,dy, dx*dx));                      */
/*   edge2[k] = (k dr)(k dr); bin = max{k : edge2[k] <= r2};            */
/*   counted iff r2 < edge2[nbins].                                     */
/* ------------------------------------------------------------------ */
double orc_edge2(int k, double dr)
{
    double e = (double)k * dr;
    return e * e;
}

double orc_r2(double xi, double yi, double zi, double xj, double yj, double zj, double L)
{
    double dx = min_image(xj - xi, L);
    double dy = min_image(yj - yi, L);
    double dz = min_image(zj - zi, L);
    return fma(dz, dz, fma(dy, dy, dx * dx));
}

static int bin_of(const double *edge2, int nbins, double r2)
{
    /* largest k in [0, nbins) with edge2[k] <= r2; caller ensures r2 < edge2[nbins] */
    int lo = 0, hi = nbins; /* edge2[lo] <= r2 < edge2[hi] */
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (edge2[mid] <= r2) lo = mid; else hi = mid;
    }
    return lo;
}

void orc_pair_histogram(int N, double L, int M, const uint8_t *species, const float *xyz,
                        double dr, int nbins, uint64_t *counts, uint64_t *n_out)
{
    int P = M * (M + 1) / 2;
    double *edge2 = (double *)malloc(sizeof(double) * (size_t)(nbins + 1));
    for (int k = 0; k <= nbins; ++k) edge2[k] = orc_edge2(k, dr);
    memset(counts, 0, sizeof(uint64_t) * (size_t)P * nbins);
    if (n_out) memset(n_out, 0, sizeof(uint64_t) * (size_t)P);
#pragma omp parallel
    {
        uint64_t *loc = (uint64_t *)calloc((size_t)P * nbins + P, sizeof(uint64_t));
#pragma omp for schedule(dynamic, 16)
        for (int i = 0; i < N; ++i) {
            double xi = xyz[i], yi = xyz[N + i], zi = xyz[2 * N + i];
            for (int j = i + 1; j < N; ++j) {
                double r2 = orc_r2(xi, yi, zi, xyz[j], xyz[N + j], xyz[2 * N + j], L);
                int p = orc_pair_index(species[i], species[j], M);
                if (r2 < edge2[nbins]) loc[(size_t)p * nbins + bin_of(edge2, nbins, r2)] += 1;
                else loc[(size_t)P * nbins + p] += 1;
            }
        }
#pragma omp critical
        {
            for (size_t q = 0; q < (size_t)P * nbins; ++q) counts[q] += loc[q];
            if (n_out) for (int p = 0; p < P; ++p) n_out[p] += loc[(size_t)P * nbins + p];
        }
        free(loc);
    }
    free(edge2);
}

/* ------------------------------------------------------------------ */
/* g(r) and S(Q) (Eq. 1).                                               */
/* ------------------------------------------------------------------ */
/* g_p(k) = n_p(k) / (npairs_p * Vshell(k) / V),
 * Vshell(k) = (4 pi / 3) ((k+1)^3 - k^3) dr^3. */
void orc_gr_normalize(const double *counts, int P, int nbins, double dr, double V,
                      const double *npairs, double *g)
{
    for (int p = 0; p < P; ++p)
        for (int k = 0; k < nbins; ++k) {
            double k0 = (double)k, k1 = (double)(k + 1);
            double shell = (4.0 * M_PI / 3.0) * (k1 * k1 * k1 - k0 * k0 * k0) * dr * dr * dr;
            g[(size_t)p * nbins + k] = counts[(size_t)p * nbins + k] / (npairs[p] * shell / V);
        }
}

static double sinc(double x) { return x == 0.0 ? 1.0 : sin(x) / x; }

/* Eq. 1 by the midpoint rule on r_k = (k + 1/2) dr, k < nbins:
 *   S(Q) = self + sum_p w_p 4 pi rho sum_k r_k^2 (g_p(k) - 1) sinc(Q r_k) dr */
void orc_sq(const double *g, int P, int nbins, double dr, double rho, const double *w,
            double self_term, const double *Q, int nQ, double *S)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nQ; ++i) {
        double total = self_term;
        for (int p = 0; p < P; ++p) {
            double acc = 0.0;
            for (int k = 0; k < nbins; ++k) {
                double r = ((double)k + 0.5) * dr;
                acc += r * r * (g[(size_t)p * nbins + k] - 1.0) * sinc(Q[i] * r) * dr;
            }
            total += w[p] * 4.0 * M_PI * rho * acc;
        }
        S[i] = total;
    }
}

/* ------------------------------------------------------------------ */
/* Gaussian-broadened histogram, its chi^2 gradient, and forces.        */
/* Bin k gets w_k(r) = Phi((e_{k+1} - r)/s) - Phi((e_k - r)/s) from     */
/* each pair with r < L/2, for the bins that intersect [r-6s, r+6s].    */
/* ------------------------------------------------------------------ */
static double Phi(double x) { return 0.5 * (1.0 + erf(x / sqrt(2.0))); }
static double phi(double x) { return exp(-0.5 * x * x) / sqrt(2.0 * M_PI); }

static void bin_window(double r, double dr, double sigma, int nbins, int *k0, int *k1)
{
    /* bins k with e_{k+1} > r - 6s and e_k < r + 6s */
    int lo = (int)floor((r - 6.0 * sigma) / dr);
    int hi = (int)floor((r + 6.0 * sigma) / dr);
    if (lo < 0) lo = 0;
    if (hi > nbins - 1) hi = nbins - 1;
    *k0 = lo;
    *k1 = hi;
}

static double pair_r(const float *xyz, int N, double L, int i, int j, double d[3])
{
    d[0] = min_image((double)xyz[i] - (double)xyz[j], L);
    d[1] = min_image((double)xyz[N + i] - (double)xyz[N + j], L);
    d[2] = min_image((double)xyz[2 * N + i] - (double)xyz[2 * N + j], L);
    return sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
}

void orc_hist_broad(int N, double L, int M, const uint8_t *species, const float *xyz, double dr,
                    int nbins, double sigma, double *nhat)
{
    int P = M * (M + 1) / 2;
    memset(nhat, 0, sizeof(double) * (size_t)P * nbins);
#pragma omp parallel
    {
        double *loc = (double *)calloc((size_t)P * nbins, sizeof(double));
#pragma omp for schedule(dynamic, 16)
        for (int i = 0; i < N; ++i)
            for (int j = i + 1; j < N; ++j) {
                double d[3];
                double r = pair_r(xyz, N, L, i, j, d);
                if (!(r < 0.5 * L)) continue;
                int k0, k1;
                bin_window(r, dr, sigma, nbins, &k0, &k1);
                int p = orc_pair_index(species[i], species[j], M);
                for (int k = k0; k <= k1; ++k) {
                    double e0 = (double)k * dr, e1 = (double)(k + 1) * dr;
                    loc[(size_t)p * nbins + k] += Phi((e1 - r) / sigma) - Phi((e0 - r) / sigma);
                }
            }
#pragma omp critical
        for (size_t q = 0; q < (size_t)P * nbins; ++q) nhat[q] += loc[q];
        free(loc);
    }
}

/* dL/dx for L a function of the broadened histogram: given A = dL/dnhat
 * [P][nbins], each pair contributes dL/dr = sum_k A_p(k) dw_k/dr with
 * dw_k/dr = (phi((e_k - r)/s) - phi((e_{k+1} - r)/s)) / s, and
 * dL/dx_i += dL/dr (x_i - x_j)/r, dL/dx_j -= the same.  grad [3][N]. */
static void broad_grad_atom(int i, int N, double L, int M, const uint8_t *species, const float *xyz,
                            double dr, int nbins, double sigma, const double *A, double g[3])
{
    double gx = 0.0, gy = 0.0, gz = 0.0;
    for (int j = 0; j < N; ++j) {
        if (j == i) continue;
        double d[3];
        double r = pair_r(xyz, N, L, i, j, d);
        if (!(r < 0.5 * L) || r == 0.0) continue;
        int k0, k1;
        bin_window(r, dr, sigma, nbins, &k0, &k1);
        int p = orc_pair_index(species[i], species[j], M);
        double dLdr = 0.0;
        for (int k = k0; k <= k1; ++k) {
            double e0 = (double)k * dr, e1 = (double)(k + 1) * dr;
            dLdr += A[(size_t)p * nbins + k] * (phi((e0 - r) / sigma) - phi((e1 - r) / sigma)) / sigma;
        }
        gx += dLdr * d[0] / r;
        gy += dLdr * d[1] / r;
        gz += dLdr * d[2] / r;
    }
    g[0] = gx;
    g[1] = gy;
    g[2] = gz;
}

void orc_hist_broad_backward(int N, double L, int M, const uint8_t *species, const float *xyz,
                             double dr, int nbins, double sigma, const double *A, double *grad)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < N; ++i) {
        double g[3];
        broad_grad_atom(i, N, L, M, species, xyz, dr, nbins, sigma, A, g);
        grad[i] = g[0];
        grad[N + i] = g[1];
        grad[2 * N + i] = g[2];
    }
}

/* The same gradient for the atoms sel[0 .. n_sel-1] only (each is a sum over
 * all N partners): grad_sel [3][n_sel]. */
void orc_hist_broad_backward_atoms(int N, double L, int M, const uint8_t *species, const float *xyz,
                                   double dr, int nbins, double sigma, const double *A, int n_sel,
                                   const int32_t *sel, double *grad_sel)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int q = 0; q < n_sel; ++q) {
        double g[3];
        broad_grad_atom(sel[q], N, L, M, species, xyz, dr, nbins, sigma, A, g);
        grad_sel[q] = g[0];
        grad_sel[n_sel + q] = g[1];
        grad_sel[2 * n_sel + q] = g[2];
    }
}

/* Adjoint of g-normalisation followed by Eq. 1:
 * A_p(k) = sum_i dL/dS_i * w_p 4 pi rho r_k^2 sinc(Q_i r_k) dr / (npairs_p Vshell(k)/V). */
void orc_sq_adjoint(const double *dLdS, int P, int nbins, double dr, double rho, double V,
                    const double *w, const double *npairs, const double *Q, int nQ, double *A)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nbins; ++k) {
        double r = ((double)k + 0.5) * dr;
        double k0 = (double)k, k1 = (double)(k + 1);
        double shell = (4.0 * M_PI / 3.0) * (k1 * k1 * k1 - k0 * k0 * k0) * dr * dr * dr;
        double s = 0.0;
        for (int i = 0; i < nQ; ++i) s += dLdS[i] * sinc(Q[i] * r);
        for (int p = 0; p < P; ++p)
            A[(size_t)p * nbins + k] = s * w[p] * 4.0 * M_PI * rho * r * r * dr / (npairs[p] * shell / V);
    }
}

/* dE/dx of atom i and half its pair energy (see orc_forces). */
static void force_atom(int i, int N, double L, int M, const uint8_t *species, const int32_t *unit_of,
                       const float *xyz, const float *tab, int n_pts, double h, double r_cut, double g[3],
                       double *e_half)
{
    double gx = 0.0, gy = 0.0, gz = 0.0, e = 0.0;
    for (int j = 0; j < N; ++j) {
        if (unit_of[i] == unit_of[j]) continue;
        double d[3];
        double r = pair_r(xyz, N, L, i, j, d);
        if (!(r < r_cut) || r == 0.0) continue;
        const float *row = tab + (size_t)orc_pair_index(species[i], species[j], M) * n_pts;
        double du = orc_table_du(row, n_pts, h, r_cut, r);
        e += 0.5 * orc_table_u(row, n_pts, h, r_cut, r);
        gx += du * d[0] / r;
        gy += du * d[1] / r;
        gz += du * d[2] / r;
    }
    g[0] = gx;
    g[1] = gy;
    g[2] = gz;
    *e_half = e;
}

/* Gradient of the total energy: dE/dx_i = sum over j in other units of
 * U'(r) (x_i - x_j)/r, with U' the slope of the table interpolant. */
void orc_forces(int N, double L, int M, const uint8_t *species, const int32_t *unit_of,
                const float *xyz, const float *tab, int n_pts, double h, double r_cut,
                double *grad, double *E_out)
{
    double E = 0.0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : E)
    for (int i = 0; i < N; ++i) {
        double g[3], e;
        force_atom(i, N, L, M, species, unit_of, xyz, tab, n_pts, h, r_cut, g, &e);
        E += e;
        grad[i] = g[0];
        grad[N + i] = g[1];
        grad[2 * N + i] = g[2];
    }
    if (E_out) *E_out = E;
}

/* The same gradient for the atoms sel[0 .. n_sel-1] only: grad_sel [3][n_sel]. */
void orc_forces_atoms(int N, double L, int M, const uint8_t *species, const int32_t *unit_of, const float *xyz,
                      const float *tab, int n_pts, double h, double r_cut, int n_sel, const int32_t *sel,
                      double *grad_sel)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int q = 0; q < n_sel; ++q) {
        double g[3], e;
        force_atom(sel[q], N, L, M, species, unit_of, xyz, tab, n_pts, h, r_cut, g, &e);
        grad_sel[q] = g[0];
        grad_sel[n_sel + q] = g[1];
        grad_sel[2 * n_sel + q] = g[2];
    }
}

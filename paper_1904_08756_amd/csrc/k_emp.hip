// Empirical-potential (EMP) update of the refinement loop (Sec. "Algorithmic
// Principle": the EMP is the Fourier counterpart of the difference between
// measured and simulated S(Q), fitted by a series of Poisson functions in Q
// space; Sec. "Correctness", Eq. 2: the partials' EMPs through the inverse
// of the Eq. 1 weight matrix, a pseudo-inverse of the matrix enlarged by a
// unit matrix when there are fewer profiles than partials).
//
// Poisson functions in r, normalised so that 4 pi rho int r^2 p_n dr = 1:
//   p_n(r) = (r/s)^n exp(-r/s) / (4 pi rho s^3 (n+2)!),  n = 1 .. n_terms,
// whose Eq. 1-style transform 4 pi rho int r^2 p_n(r) sinc(Q r) dr is
//   P_n(Q) = sin((n+2) a) / ((n+2) Q s (1 + Q^2 s^2)^((n+2)/2)),  a = atan(Q s)
// (P_n(0) = 1).  Steps: S_sim of every profile by Eq. 1 (k_sq), dS = S_exp -
// S_sim, least-squares Poisson coefficients of each dS (normal equations with
// a relative ridge, Cholesky), the partials' coefficients through W+ (Gauss-
// Jordan inverse of W, or of the normal matrix of W enlarged by the scaled
// unit matrix), the update dU_p(r) = -feedback kT sum_n C_pn p_n(r) shifted to
// zero at the cutoff, added to the EMP (then scaled to max |EMP| <= emp_max
// when asked), and the tables rewritten as reference potential + EMP.  All
// FP64; the tables are rounded to float32 at the end.
#include "nd_internal.h"

#include <algorithm>
#include <cmath>

namespace {

constexpr int EMP_THREADS = 1024;

struct EmpArgs {
    const double *basis;  // [n_terms][nQ] P_n(Q)
    const double *dS;     // [n_prof][nQ]
    int n_terms, nQ, n_prof, P, n_pts;
    double W[ND_EMP_MAX_PROFILES * nd::MAX_PARTIALS];  // [n_prof][P]
    double ridge, id_weight, feedback, kT, sigma, rho, h, r_cut, emp_max;
    const float *rp;     // [P][n_pts] reference potential
    double *emp;         // [P][n_pts] accumulated EMP (updated)
    float *tab;          // [P][n_pts] tables = rp + emp (written)
    double *C_out;       // [P][n_terms] partials' coefficients of this update
};

__global__ void k_emp_basis(const double *__restrict__ Q, int nQ, int n_terms, double sigma, double *__restrict__ B)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nQ * n_terms) return;
    const int n = i / nQ + 1, q = i % nQ;
    const double x = Q[q] * sigma;
    double v = 1.0;
    if (x != 0.0) {
        const double a = atan(x);
        v = sin((n + 2) * a) / ((double)(n + 2) * x * pow(1.0 + x * x, 0.5 * (n + 2)));
    }
    B[i] = v;
}

__global__ void k_emp_diff(const double *__restrict__ S_exp, const double *__restrict__ S_sim, int n,
                           double *__restrict__ dS)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dS[i] = S_exp[i] - S_sim[i];
}

// log of p_n(r) without the normalisation constant: n ln(r/s) - r/s
__device__ __forceinline__ double poisson_r(int n, double r, double sigma, double lognorm_n)
{
    if (!(r > 0.0)) return 0.0;
    const double x = r / sigma;
    return exp((double)n * log(x) - x - lognorm_n);
}

// One block: the fit, the weight inverse, the real-space update and the tables.
__global__ __launch_bounds__(EMP_THREADS) void k_emp_fit(EmpArgs a)
{
    constexpr int NT = ND_EMP_MAX_TERMS;
    constexpr int NP = ND_EMP_MAX_PROFILES;
    constexpr int MP = nd::MAX_PARTIALS;
    __shared__ double G[NT * NT];
    __shared__ double rhs[NP * NT];
    __shared__ double Wp[MP * (NP + MP)];  // W+ [P][n_prof]
    __shared__ double Cp[MP * NT];
    __shared__ double lognorm[NT];
    __shared__ double red[EMP_THREADS / 64];
    const int tid = threadIdx.x;
    const int nt = a.n_terms, nQ = a.nQ, np = a.n_prof, P = a.P;
    // Gram matrix and right-hand sides, each a fixed-order sum over Q
    for (int e = tid; e < nt * nt + np * nt; e += EMP_THREADS) {
        if (e < nt * nt) {
            const int n = e / nt, m = e % nt;
            const double *bn = a.basis + (size_t)n * nQ, *bm = a.basis + (size_t)m * nQ;
            double s = 0.0;
            for (int q = 0; q < nQ; ++q) s += bn[q] * bm[q];
            G[e] = s;
        } else {
            const int f = e - nt * nt, i = f / nt, n = f % nt;
            const double *bn = a.basis + (size_t)n * nQ, *d = a.dS + (size_t)i * nQ;
            double s = 0.0;
            for (int q = 0; q < nQ; ++q) s += bn[q] * d[q];
            rhs[i * nt + n] = s;
        }
    }
    if (tid < nt) lognorm[tid] = lgamma((double)(tid + 4)) + log(4.0 * M_PI * a.rho * a.sigma * a.sigma * a.sigma);
    __syncthreads();
    if (tid == 0) {
        // relative ridge, Cholesky G = L L^T (in place, lower), solve per profile
        double tr = 0.0;
        for (int n = 0; n < nt; ++n) tr += G[n * nt + n];
        const double lam = a.ridge * tr / nt;
        for (int n = 0; n < nt; ++n) G[n * nt + n] += lam;
        for (int j = 0; j < nt; ++j) {
            double d = G[j * nt + j];
            for (int k = 0; k < j; ++k) d -= G[j * nt + k] * G[j * nt + k];
            d = sqrt(d);
            G[j * nt + j] = d;
            for (int i = j + 1; i < nt; ++i) {
                double s = G[i * nt + j];
                for (int k = 0; k < j; ++k) s -= G[i * nt + k] * G[j * nt + k];
                G[i * nt + j] = s / d;
            }
        }
        for (int p = 0; p < np; ++p) {
            double *y = rhs + p * nt;
            for (int i = 0; i < nt; ++i) {
                double s = y[i];
                for (int k = 0; k < i; ++k) s -= G[i * nt + k] * y[k];
                y[i] = s / G[i * nt + i];
            }
            for (int i = nt - 1; i >= 0; --i) {
                double s = y[i];
                for (int k = i + 1; k < nt; ++k) s -= G[k * nt + i] * y[k];
                y[i] = s / G[i * nt + i];
            }
        }
        // W+: the inverse of W (square), else (Wa^T Wa)^-1 Wa^T restricted to
        // the data rows, Wa = [W; id_weight I]; Gauss-Jordan with partial pivots
        double A[MP * 2 * MP];
        for (int r = 0; r < P; ++r)
            for (int c = 0; c < P; ++c) {
                double v;
                if (np == P) {
                    v = a.W[r * P + c];
                } else {
                    v = (r == c) ? a.id_weight * a.id_weight : 0.0;
                    for (int i = 0; i < np; ++i) v += a.W[i * P + r] * a.W[i * P + c];
                }
                A[r * 2 * P + c] = v;
                A[r * 2 * P + P + c] = (r == c) ? 1.0 : 0.0;
            }
        for (int c = 0; c < P; ++c) {
            int piv = c;
            for (int r = c + 1; r < P; ++r)
                if (fabs(A[r * 2 * P + c]) > fabs(A[piv * 2 * P + c])) piv = r;
            if (piv != c)
                for (int k = 0; k < 2 * P; ++k) {
                    const double t = A[c * 2 * P + k];
                    A[c * 2 * P + k] = A[piv * 2 * P + k];
                    A[piv * 2 * P + k] = t;
                }
            const double d = A[c * 2 * P + c];
            for (int k = 0; k < 2 * P; ++k) A[c * 2 * P + k] /= d;
            for (int r = 0; r < P; ++r) {
                if (r == c) continue;
                const double f = A[r * 2 * P + c];
                if (f != 0.0)
                    for (int k = 0; k < 2 * P; ++k) A[r * 2 * P + k] -= f * A[c * 2 * P + k];
            }
        }
        for (int p = 0; p < P; ++p)
            for (int i = 0; i < np; ++i) {
                double v;
                if (np == P) {
                    v = A[p * 2 * P + P + i];
                } else {
                    v = 0.0;  // ((Wa^T Wa)^-1 W^T)[p][i]
                    for (int k = 0; k < P; ++k) v += A[p * 2 * P + P + k] * a.W[i * P + k];
                }
                Wp[p * np + i] = v;
            }
        for (int p = 0; p < P; ++p)
            for (int n = 0; n < nt; ++n) {
                double v = 0.0;
                for (int i = 0; i < np; ++i) v += Wp[p * np + i] * rhs[i * nt + n];
                Cp[p * nt + n] = v;
            }
    }
    __syncthreads();
    if (a.C_out)
        for (int e = tid; e < P * nt; e += EMP_THREADS) a.C_out[e] = Cp[e];
    // real-space update, shifted to zero at the cutoff
    const int n_pts = a.n_pts;
    const double scale = -a.feedback * a.kT;
    double mx = 0.0;
    for (int e = tid; e < P * n_pts; e += EMP_THREADS) {
        const int p = e / n_pts, k = e % n_pts;
        const double r = (double)k * a.h;
        double du = 0.0;
        if (r < a.r_cut) {
            double hr = 0.0, hc = 0.0;
            for (int n = 0; n < nt; ++n) {
                hr += Cp[p * nt + n] * poisson_r(n + 1, r, a.sigma, lognorm[n]);
                hc += Cp[p * nt + n] * poisson_r(n + 1, a.r_cut, a.sigma, lognorm[n]);
            }
            du = scale * (hr - hc);
        }
        const double v = a.emp[e] + du;
        a.emp[e] = v;
        mx = fmax(mx, fabs(v));
    }
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
    if ((tid & 63) == 0) red[tid >> 6] = mx;
    __syncthreads();
    if (tid == 0) {
        double m = 0.0;
        for (int w = 0; w < EMP_THREADS / 64; ++w) m = fmax(m, red[w]);
        red[0] = m;
    }
    __syncthreads();
    const double m = red[0];
    const double f = (a.emp_max > 0.0 && m > a.emp_max) ? a.emp_max / m : 1.0;
    for (int e = tid; e < P * n_pts; e += EMP_THREADS) {
        double v = a.emp[e];
        if (f != 1.0) {
            v *= f;
            a.emp[e] = v;
        }
        a.tab[e] = (float)((double)a.rp[e] + v);
    }
}

__global__ void k_fill_zero_d(double *__restrict__ p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

}  // namespace

namespace nd {

void emp_reset(nd_box *b)
{
    if (!b->emp) return;
    const int n = b->P * b->n_pts;
    hipLaunchKernelGGL(k_fill_zero_d, dim3((n + 255) / 256), dim3(256), 0, b->stream, b->emp, n);
    ND_HIP(hipGetLastError());
}

void launch_emp_update(nd_box *b, const nd_emp_params *prm, int n_prof, const double *W_host,
                       const double *self_host, const double *g, int nbins, double dr, const double *Q, int nQ,
                       const double *S_exp, double *dS_out, double *emp_out, double *C_out)
{
    const int P = b->P, n_pts = b->n_pts, nt = prm->n_terms;
    if (!b->emp) {
        b->emp = static_cast<double *>(dmalloc(sizeof(double) * (size_t)P * n_pts));
        emp_reset(b);
    }
    const double V = b->L * b->L * b->L, rho = (double)b->N / V;
    // workspace: basis [nt][nQ], S_sim [n_prof][nQ], dS [n_prof][nQ]
    const size_t nb = (size_t)nt * nQ, ns = (size_t)n_prof * nQ;
    double *ws = static_cast<double *>(workspace(b, sizeof(double) * (nb + 2 * ns)));
    double *B = ws, *S_sim = ws + nb, *dS = dS_out ? dS_out : ws + nb + ns;
    hipLaunchKernelGGL(k_emp_basis, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, b->stream, Q, nQ, nt,
                       prm->sigma, B);
    ND_HIP(hipGetLastError());
    for (int i = 0; i < n_prof; ++i)
        launch_sq(g, P, nbins, dr, rho, W_host + (size_t)i * P, self_host[i], Q, nQ, S_sim + (size_t)i * nQ,
                  b->stream);
    hipLaunchKernelGGL(k_emp_diff, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, b->stream, S_exp, S_sim,
                       (int)ns, dS);
    ND_HIP(hipGetLastError());
    EmpArgs a{};
    a.basis = B;
    a.dS = dS;
    a.n_terms = nt;
    a.nQ = nQ;
    a.n_prof = n_prof;
    a.P = P;
    a.n_pts = n_pts;
    for (int i = 0; i < n_prof * P; ++i) a.W[i] = W_host[i];
    a.ridge = prm->ridge;
    a.id_weight = prm->id_weight;
    a.feedback = prm->feedback;
    a.kT = prm->kT;
    a.sigma = prm->sigma;
    a.rho = rho;
    a.h = b->h;
    a.r_cut = b->rc;
    a.emp_max = prm->emp_max;
    a.rp = b->rp;
    a.emp = b->emp;
    a.tab = b->tab;
    a.C_out = C_out;
    hipLaunchKernelGGL(k_emp_fit, dim3(1), dim3(EMP_THREADS), 0, b->stream, a);
    ND_HIP(hipGetLastError());
    if (emp_out)
        ND_HIP(hipMemcpyAsync(emp_out, b->emp, sizeof(double) * (size_t)P * n_pts, hipMemcpyDeviceToDevice, b->stream));
}

}  // namespace nd

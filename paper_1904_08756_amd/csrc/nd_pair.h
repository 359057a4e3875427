// Device-side pair energy shared by the Metropolis and total-energy kernels.
//
// Positions are fractional (s = x / L).  Each atom carries a float32 pair
// (hi, lo) with s = hi + lo to about 2^-48.  The cutoff is first tested in
// FP32 on the hi parts with a margin that covers their rounding; a pair
// that passes is re-evaluated from the FP64 positions, so the distance and
// the table coordinate r/h are as accurate as FP64 arithmetic on the
// float32 input coordinates.  The energy itself is the float32 linear
// interpolation of the tabulated potential.
#pragma once

#include "nd_internal.h"

namespace nd {

// Loads and stores through the global address space.  Pointers read from a
// descriptor in device memory (rather than from kernel arguments) are
// generic to the compiler, and generic (flat) accesses also count against
// the LDS wait counter, so every LDS wait would wait for them too.
#define ND_GLOBAL_AS __attribute__((address_space(1)))
typedef float nd_v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float4 ld4(const float4 *p)
{
    const nd_v4f v = *(const ND_GLOBAL_AS nd_v4f *)p;
    return make_float4(v.x, v.y, v.z, v.w);
}

// A float4 from LDS through a generic pointer into shared memory (an LDS
// read rather than a flat one).
__device__ __forceinline__ float4 ld_lds4(const float4 *p)
{
    const nd_v4f v = *(const __attribute__((address_space(3))) nd_v4f *)p;
    return make_float4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ int4 ld_i4(const int4 *p)
{
    typedef int v4i __attribute__((ext_vector_type(4)));
    const v4i v = *(const ND_GLOBAL_AS v4i *)p;
    return make_int4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ double2 ld_d2(const double2 *p)
{
    typedef double v2d __attribute__((ext_vector_type(2)));
    const v2d v = *(const ND_GLOBAL_AS v2d *)p;
    return make_double2(v.x, v.y);
}

template <class T>
__device__ __forceinline__ T ldg(const T *p)
{
    return *(const ND_GLOBAL_AS T *)p;
}

template <class T>
__device__ __forceinline__ void stg(T *p, T v)
{
    *(ND_GLOBAL_AS T *)p = v;
}

__device__ __forceinline__ void st_d2(double2 *p, double2 v)
{
    typedef double v2d __attribute__((ext_vector_type(2)));
    v2d x;
    x.x = v.x;
    x.y = v.y;
    *(ND_GLOBAL_AS v2d *)p = x;
}

// Block-wide copy of n floats from global memory to 16-byte aligned LDS
// (src 16-byte aligned): all wide loads of a thread are issued before its
// LDS writes, so the copy costs about one memory latency, not one per
// element.
template <int THREADS>
__device__ __forceinline__ void stage_floats(float *dst, const float *src, int n)
{
    constexpr int U = 4;
    const int n4 = n >> 2;
    const float4 *s4 = reinterpret_cast<const float4 *>(src);
    float4 *d4 = reinterpret_cast<float4 *>(dst);
    for (int base = (int)threadIdx.x; base < n4; base += THREADS * U) {
        float4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (base + u * THREADS < n4) v[u] = ld4(s4 + base + u * THREADS);
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (base + u * THREADS < n4) d4[base + u * THREADS] = v[u];
    }
    for (int i = 4 * n4 + (int)threadIdx.x; i < n; i += THREADS) dst[i] = ldg(src + i);
}

struct PairCtx {
    const float *tab;   // [P][n_pts] table rows (LDS or global)
    const int *prow;    // [M*M] row offset of each species pair
    int M, n_pts;
    float rcf2_filter;  // (r_cut/L + margin)^2, FP32 filter on hi parts
    double rcf2;        // (r_cut/L)^2
    double tscale;      // L / h
};

// Nearest-image squared distance of the hi parts, FP32 (the filter).
__device__ __forceinline__ float r2_hi(float4 p, float4 q)
{
    float dx = q.x - p.x, dy = q.y - p.y, dz = q.z - p.z;
    dx -= rintf(dx);
    dy -= rintf(dy);
    dz -= rintf(dz);
    return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
}

// Square root of a non-negative FP64 value to about 1e-13 relative, from one
// hardware FP64 reciprocal square root y (one transcendental, no
// conversions): r0 = r2 y, then one Newton step r = r0 + (r2 - r0^2) y / 2,
// which squares y's relative error.  The argument is held at or above the
// least normal double, so r2 = 0 gives y finite and r = 0.
__device__ __forceinline__ double sqrt_nr(double r2)
{
    const double y = __builtin_amdgcn_rsq(fmax(r2, 2.2250738585072014e-308));
    const double r0 = r2 * y;
    const double d = fma(-r0, r0, r2);
    return fma(d, 0.5 * y, r0);
}

// Exact-path pair energy of trial atom p (FP64 fractional position ps,
// species row base rb) with atom q (hi, lo).  Returns false beyond r_cut.
__device__ __forceinline__ bool pair_u_exact(const PairCtx &c, double psx, double psy, double psz, int rb,
                                             float4 q, float4 ql, float &u)
{
    double ex = ((double)q.x + (double)ql.x) - psx;
    double ey = ((double)q.y + (double)ql.y) - psy;
    double ez = ((double)q.z + (double)ql.z) - psz;
    ex -= rint(ex);
    ey -= rint(ey);
    ez -= rint(ez);
    const double r2 = fma(ez, ez, fma(ey, ey, ex * ex));
    if (!(r2 < c.rcf2)) return false;
    const double t = sqrt_nr(r2) * c.tscale;
    int i0 = (int)t;
    i0 = min(i0, c.n_pts - 2);
    const float f = (float)(t - (double)i0);
    const float *row = c.tab + c.prow[rb + __float_as_int(q.w)];
    const float u0 = row[i0];
    const float u1 = row[i0 + 1];
    u = fmaf(f, u1 - u0, u0);
    return true;
}

// Full pair energy: FP32 filter, then the exact path.
__device__ __forceinline__ bool pair_u(const PairCtx &c, float4 p, double psx, double psy, double psz, int rb,
                                       float4 q, float4 ql, float &u)
{
    if (r2_hi(p, q) < c.rcf2_filter) return pair_u_exact(c, psx, psy, psz, rb, q, ql, u);
    return false;
}

// Filter margin: each hi coordinate is within 2^-24 of s and the FP32
// nearest-image arithmetic adds a few ulps, so |r_hi - r| < 1e-6 (fractional).
inline float filter_r2(double rcf) { const double m = rcf + 1e-6; return (float)(m * m * (1.0 + 1e-6)); }

}  // namespace nd

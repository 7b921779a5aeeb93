// Device helpers shared by the lattice kernels of libmdlbm (forward and
// adjoint): storage formats, D3Q19 equilibrium, moments, BGK collision with
// Guo forcing, and lattice indexing.  Internal to the library.
#pragma once

#include "lbm_internal.h"
#include "lbm_stencil.h"

namespace mdlbm {


// Per-node moments (rho - 1, u) in the storage's arithmetic.
struct alignas(16) Mom64 {
    double d, x, y, z;
};
struct alignas(8) Mom16 {
    __half2 a, b;
};

template <int S>
struct St;
template <>
struct St<LBM_STORE_F64> {
    using T = double;
    using A = double;
    using M = Mom64;
    static constexpr bool dev = false;
    static __device__ __forceinline__ double ld(const double* p, float) { return *p; }
    static __device__ __forceinline__ void st(double* p, double v, float) { *p = v; }
    static __device__ __forceinline__ void st_mom(M* p, double d, double x, double y, double z, float)
    {
        *p = Mom64{d, x, y, z};
    }
    static __device__ __forceinline__ void ld_mom(const M* p, float, double& d, double& x, double& y,
                                                  double& z)
    {
        const Mom64 m = *p;
        d = m.d, x = m.x, y = m.y, z = m.z;
    }
};
template <>
struct St<LBM_STORE_F32> {
    using T = float;
    using A = float;
    using M = float4;
    static constexpr bool dev = true;
    static __device__ __forceinline__ float ld(const float* p, float) { return *p; }
    static __device__ __forceinline__ void st(float* p, float v, float) { *p = v; }
    static __device__ __forceinline__ void st_mom(M* p, float d, float x, float y, float z, float)
    {
        *p = make_float4(d, x, y, z);
    }
    static __device__ __forceinline__ void ld_mom(const M* p, float, float& d, float& x, float& y,
                                                  float& z)
    {
        const float4 m = *p;
        d = m.x, x = m.y, y = m.z, z = m.w;
    }
};
template <>
struct St<LBM_STORE_F16> {
    using T = __half;
    using A = float;
    using M = Mom16;
    static constexpr bool dev = true;
    static __device__ __forceinline__ float ld(const __half* p, float inv)
    {
        return __half2float(*p) * inv;
    }
    static __device__ __forceinline__ void st(__half* p, float v, float sc)
    {
        *p = __float2half_rn(v * sc);
    }
    static __device__ __forceinline__ void st_mom(M* p, float d, float x, float y, float z, float sc)
    {
        Mom16 m;
        m.a = __floats2half2_rn(d * sc, x * sc);
        m.b = __floats2half2_rn(y * sc, z * sc);
        *p = m;
    }
    static __device__ __forceinline__ void ld_mom(const M* p, float inv, float& d, float& x, float& y,
                                                  float& z)
    {
        const Mom16 m = *p;
        const float2 a = __half22float2(m.a), b = __half22float2(m.b);
        d = a.x * inv, x = a.y * inv, y = b.x * inv, z = b.y * inv;
    }
};

template <class A>
__device__ __forceinline__ A W(int i);
template <>
__device__ __forceinline__ double W<double>(int i) { return wgt(i); }
template <>
__device__ __forceinline__ float W<float>(int i) { return wgtf(i); }

// Equilibrium of direction i in the storage's form:
//   plain:      feq = w rho (1 + 3 e.u + 4.5 (e.u)^2 - 1.5 u.u)
//   deviation:  feq - w = w (drho + rho (3 e.u + 4.5 (e.u)^2 - 1.5 u.u)).
template <bool DEV, class A>
__device__ __forceinline__ A eq_i(int i, A drho, A rho, A ux, A uy, A uz)
{
    const A eu = A(cx(i)) * ux + A(cy(i)) * uy + A(cz(i)) * uz;
    const A uu = ux * ux + uy * uy + uz * uz;
    const A poly = A(3) * eu + A(4.5) * eu * eu - A(1.5) * uu;
    if constexpr (DEV)
        return W<A>(i) * (drho + rho * poly);
    else
        return W<A>(i) * rho * (A(1) + poly);
}

// Moments of the values v[19] in the storage's form; `shift` is +1/2 for
// pre-collision populations (u = (sum f e + F/2)/rho) and -1/2 for
// post-collision ones (the collision turned the momentum into rho u + F/2).
template <bool DEV, class A>
__device__ __forceinline__ void moments(const A* v, A shift, const A* F, A& drho, A& rho, A& ux,
                                        A& uy, A& uz)
{
    A s = A(0), jx = A(0), jy = A(0), jz = A(0);
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        s += v[i];
        if (cx(i)) jx += A(cx(i)) * v[i];
        if (cy(i)) jy += A(cy(i)) * v[i];
        if (cz(i)) jz += A(cz(i)) * v[i];
    }
    if constexpr (DEV) {
        drho = s;
        rho = A(1) + s;
    } else {
        rho = s;
        drho = s - A(1);
    }
    const A ir = A(1) / rho;
    ux = (jx + shift * F[0]) * ir;
    uy = (jy + shift * F[1]) * ir;
    uz = (jz + shift * F[2]) * ir;
}

// BGK collision with Guo forcing, in place:
//   f+ = f + omega (feq - f) + (1 - omega/2) w [3 (e - u) + 9 (e.u) e].F
template <bool DEV, class A>
__device__ __forceinline__ void collide(A* v, A omega, const A* F, A& drho, A& ux, A& uy, A& uz)
{
    A rho;
    moments<DEV, A>(v, A(0.5), F, drho, rho, ux, uy, uz);
    const A uF = ux * F[0] + uy * F[1] + uz * F[2];
    const A gf = A(1) - A(0.5) * omega;
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        const A eu = A(cx(i)) * ux + A(cy(i)) * uy + A(cz(i)) * uz;
        const A eF = A(cx(i)) * F[0] + A(cy(i)) * F[1] + A(cz(i)) * F[2];
        const A src = gf * W<A>(i) * (A(3) * (eF - uF) + A(9) * eu * eF);
        v[i] = v[i] + omega * (eq_i<DEV, A>(i, drho, rho, ux, uy, uz) - v[i]) + src;
    }
}

// Offsets of (c-1, c, c+1) along one axis and whether each lies in the domain.
__device__ __forceinline__ void axis3(uint32_t c, uint32_t n, int per, uint32_t mul,
                                      uint32_t o[3], bool v[3])
{
    o[1] = c * mul;
    v[1] = true;
    if (c > 0) {
        o[0] = (c - 1) * mul;
        v[0] = true;
    } else {
        o[0] = (n - 1) * mul;
        v[0] = per != 0;
    }
    if (c + 1 < n) {
        o[2] = (c + 1) * mul;
        v[2] = true;
    } else {
        o[2] = 0;
        v[2] = per != 0;
    }
}

__device__ __forceinline__ double image_coord(int c, int L, int per, double center)
{
    if (!per) return (double)c;
    const double d = (double)c - center;
    if (d > 0.5 * L) return (double)(c - L);
    if (d < -0.5 * L) return (double)(c + L);
    return (double)c;
}

__device__ __forceinline__ bool wrap3(int c[3], const Geom& g)
{
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (c[a] < 0 || c[a] >= g.n[a]) {
            if (g.per[a])
                c[a] = c[a] < 0 ? c[a] + g.n[a] : c[a] - g.n[a];
            else
                ok = false;
        }
    }
    return ok;
}

__device__ __forceinline__ uint32_t node_of(const int c[3], const Geom& g)
{
    return (uint32_t)c[0] + (uint32_t)g.n[0] * ((uint32_t)c[1] + (uint32_t)g.n[1] * (uint32_t)c[2]);
}

__device__ __forceinline__ double dsum_wave(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}


}  // namespace mdlbm

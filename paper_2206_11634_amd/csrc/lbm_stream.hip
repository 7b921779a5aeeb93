// Lattice kernels of libmdlbm for gfx950: fused pull-stream + BGK collision,
// link reconstruction (VIBB / halfway) with momentum-exchange forces, local
// refilling, and population import/export.
//
// Storage formats (template parameter S):
//   LBM_STORE_F64  f_i in double, arithmetic in double (the plain method);
//   LBM_STORE_F32  h_i = f_i - w_i in float, arithmetic in float;
//   LBM_STORE_F16  h_i * scale in half, arithmetic in float.
// Deviations keep the O(1) weights out of the stored values, so the rounding
// error of a stored population is relative to |f - w| (a few 1e-3 at the
// Mach numbers of interest) rather than to f.
//
// Layout: plane i of a buffer starts at element i * stride, x fastest.  Every
// collision also stores the node's moments (rho - 1, u) into a moment plane,
// so a link needs two populations and two moment vectors instead of the 38
// populations of x_f and x_ff.  Every kernel is bound by HBM traffic; none of
// them is a contraction, so there is no MFMA here.  A solid node's plane-i slot serves as the "ghost" that holds
// the reconstructed population f_i(x_f, t+1) of the one fluid node
// x_f = x_s + e_i that pulls from it, so the bulk kernel needs no link lookup.
#include <algorithm>

#include "lbm_internal.h"
#include "lbm_stencil.h"
#include "lbm_kernels.h"

namespace mdlbm {
namespace {

// Workgroups are dispatched round-robin over the 8 XCDs.  Each XCD takes
// runs of 128 consecutive workgroups (32768 nodes), the runs of the 8 XCDs
// interleaved: the cache lines neighbouring workgroups share (the +-1 shifts
// in x) mostly stay in one XCD's L2, while the workgroups in flight still
// cover one window of each plane.  Measured on the 512^3 step: 1.9% faster
// than one contiguous eighth of the lattice per XCD, 4% faster than plain
// round-robin.  Grids not divisible into such runs keep the eighths.
__device__ __forceinline__ uint32_t xcd_block()
{
    constexpr uint32_t kRun = 128u;
    const uint32_t per = gridDim.x >> 3;
    const uint32_t k = blockIdx.x >> 3;
    if (per % kRun) return (blockIdx.x & 7u) * per + k;
    return (k / kRun) * (8u * kRun) + (blockIdx.x & 7u) * kRun + (k % kRun);
}

// ---------------------------------------------------------------------------
// Bulk: one thread per node, pull f_i(x - e_i), collide, store.
// ---------------------------------------------------------------------------
template <int S>
__global__ __launch_bounds__(256) void k_stream_collide(const typename St<S>::T* __restrict__ src,
                                                        typename St<S>::T* __restrict__ dst,
                                                        typename St<S>::M* __restrict__ mom,
                                                        const uint8_t* __restrict__ flag, Geom g,
                                                        Phys ph)
{
    using A = typename St<S>::A;
    constexpr bool DEV = St<S>::dev;
    const uint32_t cell = xcd_block() * 256u + threadIdx.x;
    if (cell >= g.ncell) return;
    if (flag[cell]) {
        // A solid node's slots are only ever read as link ghosts, which the
        // boundary kernel writes before they are pulled.  Storing the rest
        // state keeps every cache line of the wave fully written (partially
        // written lines cost far more HBM time than the bytes saved) and keeps
        // stale values from evolving inside the bodies.
        const A rest = DEV ? A(0) : A(1);
#pragma unroll
        for (int i = 0; i < kQ; ++i)
            St<S>::st(dst + (int64_t)i * g.stride + cell, DEV ? A(0) : A(wgt(i)) * rest, ph.scale);
        St<S>::st_mom(mom + cell, A(0), A(0), A(0), A(0), ph.scale);
        return;
    }
    const uint32_t nx = g.n[0], ny = g.n[1];
    const uint32_t x = cell % nx, yz = cell / nx, y = yz % ny, z = yz / ny;
    uint32_t ox[3], oy[3], oz[3];
    bool vx[3], vy[3], vz[3];
    axis3(x, nx, g.per[0], 1u, ox, vx);
    axis3(y, ny, g.per[1], nx, oy, vy);
    axis3(z, g.n[2], g.per[2], nx * ny, oz, vz);
    A f[kQ];
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        const int sx = 1 - cx(i), sy = 1 - cy(i), sz = 1 - cz(i);
        const bool ok = vx[sx] && vy[sy] && vz[sz];
        // a source beyond a wall: static halfway bounce-back, f_i = f+_opp(i)(x)
        const uint32_t s = ok ? ox[sx] + oy[sy] + oz[sz] : cell;
        const int64_t plane = ok ? i : opp(i);
        f[i] = St<S>::ld(src + plane * g.stride + s, ph.inv_scale);
    }
    A F[3];
    A om;
    if constexpr (DEV) {
        F[0] = ph.Ff[0], F[1] = ph.Ff[1], F[2] = ph.Ff[2];
        om = ph.omegaf;
    } else {
        F[0] = ph.F[0], F[1] = ph.F[1], F[2] = ph.F[2];
        om = ph.omega;
    }
    A drho, ux, uy, uz;
    collide<DEV, A>(f, om, F, drho, ux, uy, uz);
#pragma unroll
    for (int i = 0; i < kQ; ++i) St<S>::st(dst + (int64_t)i * g.stride + cell, f[i], ph.scale);
    St<S>::st_mom(mom + cell, drho, ux, uy, uz, ph.scale);
}

// FP16 deviation storage, two x-neighbouring nodes per thread: the stores
// and the pulls along directions with e_x = 0 move a pair of values per lane
// (half2) instead of one.  Pulls with e_x != 0 start at an odd node and
// are loaded per node.  The arithmetic per node is that of k_stream_collide,
// bit for bit.  Requires an even nx (pairs never straddle a row).
template <int S>
struct Pair;
template <>
struct Pair<LBM_STORE_F16> {
    using T = __half;
    static __device__ __forceinline__ void ld2(const __half* p, float inv, float& a, float& b)
    {
        const float2 v = __half22float2(*reinterpret_cast<const __half2*>(p));
        a = v.x * inv;
        b = v.y * inv;
    }
    static __device__ __forceinline__ void st2(__half* p, float a, float b, float sc)
    {
        *reinterpret_cast<__half2*>(p) = __floats2half2_rn(a * sc, b * sc);
    }
    static __device__ __forceinline__ void st_mom2(Mom16* p, const float m0[4], const float m1[4],
                                                   float sc)
    {
        struct alignas(16) M2 {
            Mom16 a, b;
        } m;
        m.a.a = __floats2half2_rn(m0[0] * sc, m0[1] * sc);
        m.a.b = __floats2half2_rn(m0[2] * sc, m0[3] * sc);
        m.b.a = __floats2half2_rn(m1[0] * sc, m1[1] * sc);
        m.b.b = __floats2half2_rn(m1[2] * sc, m1[3] * sc);
        *reinterpret_cast<M2*>(p) = m;
    }
};
// (a bound of six waves per SIMD: 78 registers instead of 96 and five waves,
// 3% faster on 512^3; dword loads of the shifted pairs at 2-byte aligned
// addresses instead of two 2-byte loads ran 30% slower and are not used)
template <int S>
__global__ __launch_bounds__(256, 6) void k_stream_collide_x2(const typename St<S>::T* __restrict__ src,
                                                           typename St<S>::T* __restrict__ dst,
                                                           typename St<S>::M* __restrict__ mom,
                                                           const uint8_t* __restrict__ flag,
                                                           Geom g, Phys ph)
{
    using P2 = Pair<S>;
    const uint32_t pair = xcd_block() * 256u + threadIdx.x;
    const uint32_t cell = 2u * pair;
    if (cell >= g.ncell) return;
    const uint16_t fl = *reinterpret_cast<const uint16_t*>(flag + cell);
    const bool solid0 = (fl & 0xFFu) != 0, solid1 = (fl >> 8) != 0;
    const float zero4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (solid0 && solid1) {
#pragma unroll
        for (int i = 0; i < kQ; ++i) P2::st2(dst + (int64_t)i * g.stride + cell, 0.0f, 0.0f, ph.scale);
        P2::st_mom2(mom + cell, zero4, zero4, ph.scale);
        return;
    }
    const uint32_t nx = g.n[0], ny = g.n[1];
    const uint32_t x = cell % nx, yz = cell / nx, y = yz % ny, z = yz / ny;
    uint32_t ox0[3], ox1[3], oy[3], oz[3];
    bool vx0[3], vx1[3], vy[3], vz[3];
    axis3(x, nx, g.per[0], 1u, ox0, vx0);
    axis3(x + 1u, nx, g.per[0], 1u, ox1, vx1);
    axis3(y, ny, g.per[1], nx, oy, vy);
    axis3(z, g.n[2], g.per[2], nx * ny, oz, vz);
    float f0[kQ], f1[kQ];
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        const int sy = 1 - cy(i), sz = 1 - cz(i);
        if (cx(i) == 0) {
            // both sources in one aligned pair: x and x + 1 of the source row,
            // or, beyond a wall, the nodes' own opposite populations
            const bool ok = vy[sy] && vz[sz];
            const uint32_t s = ok ? ox0[1] + oy[sy] + oz[sz] : cell;
            const int64_t plane = ok ? i : opp(i);
            P2::ld2(src + plane * g.stride + s, ph.inv_scale, f0[i], f1[i]);
        } else {
            const int sx = 1 - cx(i);
            const bool ok0 = vx0[sx] && vy[sy] && vz[sz];
            const bool ok1 = vx1[sx] && vy[sy] && vz[sz];
            const uint32_t s0 = ok0 ? ox0[sx] + oy[sy] + oz[sz] : cell;
            const uint32_t s1 = ok1 ? ox1[sx] + oy[sy] + oz[sz] : cell + 1u;
            f0[i] = St<S>::ld(src + (int64_t)(ok0 ? i : opp(i)) * g.stride + s0, ph.inv_scale);
            f1[i] = St<S>::ld(src + (int64_t)(ok1 ? i : opp(i)) * g.stride + s1, ph.inv_scale);
        }
    }
    const float F[3] = {ph.Ff[0], ph.Ff[1], ph.Ff[2]};
    float m0[4], m1[4];
    collide<true, float>(f0, ph.omegaf, F, m0[0], m0[1], m0[2], m0[3]);
    collide<true, float>(f1, ph.omegaf, F, m1[0], m1[1], m1[2], m1[3]);
    if (solid0) {
        // rest state, as k_stream_collide stores at solid nodes
#pragma unroll
        for (int i = 0; i < kQ; ++i) f0[i] = 0.0f;
        m0[0] = m0[1] = m0[2] = m0[3] = 0.0f;
    }
    if (solid1) {
#pragma unroll
        for (int i = 0; i < kQ; ++i) f1[i] = 0.0f;
        m1[0] = m1[1] = m1[2] = m1[3] = 0.0f;
    }
#pragma unroll
    for (int i = 0; i < kQ; ++i) P2::st2(dst + (int64_t)i * g.stride + cell, f0[i], f1[i], ph.scale);
    P2::st_mom2(mom + cell, m0, m1, ph.scale);
}

// ---------------------------------------------------------------------------
// Links: one thread per link record of one particle (blockIdx.y).
// ---------------------------------------------------------------------------
// Exact force sums: a term v becomes the 128-bit two's-complement integer
// v * 2^80 rounded toward zero (hi: the signed upper word, lo: the lower);
// integer sums do not depend on their order.  Returns true, with v taken as
// zero, for a term that is not finite or not below 2^46.
__device__ __forceinline__ bool to_fixed(double v, uint64_t& lo, int64_t& hi)
{
    const bool bad = !(fabs(v) < 0x1p46);
    const double a = bad ? 0.0 : fabs(v) * 0x1p16;  // exact: a power of two
    const double h = floor(a);
    const uint64_t H = (uint64_t)h;
    const uint64_t L = (uint64_t)((a - h) * 0x1p64);  // a - h in [0, 1), exact for a >= 0
    if (v < 0.0 && !bad) {
        lo = 0ull - L;
        hi = (int64_t)(0ull - H - (L != 0ull ? 1ull : 0ull));
    } else {
        lo = L;
        hi = (int64_t)H;
    }
    return bad;
}
__device__ __forceinline__ void add128(uint64_t& lo, int64_t& hi, uint64_t blo, int64_t bhi)
{
    const uint64_t s = lo + blo;
    hi = (int64_t)((uint64_t)hi + (uint64_t)bhi + (s < lo ? 1u : 0u));
    lo = s;
}

template <int S, bool EXACT>
__global__ __launch_bounds__(256) void k_boundary(typename St<S>::T* __restrict__ f,
                                                  const typename St<S>::M* __restrict__ mom,
                                                  const LinkRec* __restrict__ links,
                                                  const uint32_t* __restrict__ cursor,
                                                  const int64_t* __restrict__ loff,
                                                  const uint32_t* __restrict__ chunk,
                                                  PartDev P, double* __restrict__ FT,
                                                  unsigned long long* __restrict__ FX, Geom g,
                                                  Phys ph, uint32_t* __restrict__ numeric)
{
    using A = typename St<S>::A;
    constexpr bool DEV = St<S>::dev;
    // one workgroup per 256-record chunk of the link layout (chunks do not
    // straddle particles)
    const int p = (int)chunk[blockIdx.x];
    const int64_t g0 = (int64_t)blockIdx.x * 256;
    const int64_t cnt = min(loff[p + 1] - loff[p], (int64_t)cursor[(int64_t)p * kCursorPad]);
    if (g0 - loff[p] >= cnt) return;  // uniform over the block
    const int64_t l = g0 - loff[p] + threadIdx.x;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    if (l < cnt) {
        const LinkRec r = links[g0 + threadIdx.x];
        const int d = r.d, db = opp(d);
        const int e[3] = {cx(d), cy(d), cz(d)};
        const uint32_t nx = g.n[0], ny = g.n[1];
        const int cs[3] = {(int)(r.node % nx), (int)((r.node / nx) % ny), (int)(r.node / (nx * ny))};
        int cn[3] = {cs[0] - e[0], cs[1] - e[1], cs[2] - e[2]};
        const double xp[3] = {P.pos[3 * p], P.pos[3 * p + 1], P.pos[3 * p + 2]};
        const double vp[3] = {P.vel[3 * p], P.vel[3 * p + 1], P.vel[3 * p + 2]};
        const double wp[3] = {P.omega[3 * p], P.omega[3 * p + 1], P.omega[3 * p + 2]};
        wrap3(cn, g);  // for a missing point beyond a wall the node is virtual
        double Xw[3], rr[3], uw[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            // periodic axes are wrapped by wrap3; a node beyond a wall keeps
            // its raw coordinate (a virtual missing force point)
            const double Xn = image_coord(cn[a], g.n[a], g.per[a], xp[a]);
            Xw[a] = Xn + r.q * (double)e[a];
            rr[a] = Xw[a] - xp[a];
        }
        uw[0] = vp[0] + (wp[1] * rr[2] - wp[2] * rr[1]);
        uw[1] = vp[1] + (wp[2] * rr[0] - wp[0] * rr[2]);
        uw[2] = vp[2] + (wp[0] * rr[1] - wp[1] * rr[0]);
        double out, in;
        if (r.kind == LBM_LINK_MISSING) {
            // treatment 2: equilibrium at (rho0, u_w) on both sides
            out = eq_i<false, double>(d, ph.rho0 - 1.0, ph.rho0, uw[0], uw[1], uw[2]);
            in = eq_i<false, double>(db, ph.rho0 - 1.0, ph.rho0, uw[0], uw[1], uw[2]);
        } else {
            // x_f: its outgoing population and moments at time t
            const uint32_t xf = node_of(cn, g);
            const A fdf = St<S>::ld(f + (int64_t)d * g.stride + xf, ph.inv_scale);
            A drf, uf[3];
            St<S>::ld_mom(mom + xf, ph.inv_scale, drf, uf[0], uf[1], uf[2]);
            const A rf = A(1) + drf;
            const A uwa[3] = {A(uw[0]), A(uw[1]), A(uw[2])};
            const A ebu = -(A(e[0]) * uwa[0] + A(e[1]) * uwa[1] + A(e[2]) * uwa[2]);
            A unk;
            if (r.kind == LBM_LINK_VIBB) {
                int cf[3] = {cn[0] - e[0], cn[1] - e[1], cn[2] - e[2]};
                wrap3(cf, g);
                const uint32_t xff = node_of(cf, g);
                const A fdff = St<S>::ld(f + (int64_t)d * g.stride + xff, ph.inv_scale);
                A drff, uff[3];
                St<S>::ld_mom(mom + xff, ph.inv_scale, drff, uff[0], uff[1], uff[2]);
                const A rff = A(1) + drff;
                const A q = A(r.q);
                const A tq = A(2) * q, oq = A(1) - A(2) * q;
                // non-equilibrium part extrapolated to x_d (Eq. neqd), or for
                // q > 1/2 under treatment bit 8 held at its x_f value
                const bool hold = ph.neq_split && q > A(0.5);
                const A fneq = (hold ? A(1) : tq) * (fdf - eq_i<DEV, A>(d, drf, rf, uf[0], uf[1], uf[2])) +
                               (hold ? A(0) : oq) *
                                   (fdff - eq_i<DEV, A>(d, drff, rff, uff[0], uff[1], uff[2]));
                // density at x_d (Eq. rhod)
                A drd, rd;
                if (q <= A(0.5)) {
                    drd = tq * drf + oq * drff;
                    rd = tq * rf + oq * rff;
                } else {
                    drd = drf;
                    rd = rf;
                }
                A ud[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const A us = (q <= A(0.5)) ? tq * uf[a] + oq * uff[a]
                                               : (A(1) - q) / q * uf[a] + (tq - A(1)) / q * uwa[a];
                    const A uss = (A(1) - q) / (A(1) + q) * uff[a] + tq / (A(1) + q) * uwa[a];
                    ud[a] = us / A(3) + A(2) * uss / A(3);
                }
                unk = eq_i<DEV, A>(d, drd, rd, ud[0], ud[1], ud[2]) + fneq +
                      A(6) * W<A>(d) * rf * ebu;
            } else {
                // treatment 1: halfway bounce-back with the moving-wall term
                unk = fdf + A(6) * W<A>(d) * rf * ebu;
            }
            St<S>::st(f + (int64_t)db * g.stride + r.node, unk, ph.scale);
            out = (double)fdf;
            in = (double)unk;
            if constexpr (DEV) {
                out += wgt(d);
                in += wgt(db);
            }
        }
        // Galilean-invariant momentum exchange (Eq. mem)
        double t[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) t[a] = ((double)e[a] - uw[a]) * out - (-(double)e[a] - uw[a]) * in;
        acc[0] = t[0];
        acc[1] = t[1];
        acc[2] = t[2];
        acc[3] = rr[1] * t[2] - rr[2] * t[1];
        acc[4] = rr[2] * t[0] - rr[0] * t[2];
        acc[5] = rr[0] * t[1] - rr[1] * t[0];
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if constexpr (EXACT) {
        // per link in 128-bit integers, then wave, workgroup and the
        // particle's accumulator (the carry of the low word's atomic goes
        // into the high word's)
        __shared__ uint64_t rlo[4][6];
        __shared__ int64_t rhi[4][6];
        bool bad = false;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            uint64_t lo;
            int64_t hi;
            bad = to_fixed(acc[k], lo, hi) || bad;
            for (int m = 32; m >= 1; m >>= 1) {
                const uint64_t blo = __shfl_xor((unsigned long long)lo, m, 64);
                const int64_t bhi = __shfl_xor((long long)hi, m, 64);
                add128(lo, hi, blo, bhi);
            }
            if (lane == 0) {
                rlo[wv][k] = lo;
                rhi[wv][k] = hi;
            }
        }
        if (__ballot(bad) && lane == 0) atomicOr(numeric, 1u);  // reported by the next classification
        __syncthreads();
        if (threadIdx.x < 6) {
            uint64_t lo = rlo[0][threadIdx.x];
            int64_t hi = rhi[0][threadIdx.x];
            for (int w = 1; w < 4; ++w) add128(lo, hi, rlo[w][threadIdx.x], rhi[w][threadIdx.x]);
            unsigned long long* a = FX + 2 * (6 * (int64_t)p + threadIdx.x);
            const unsigned long long old = atomicAdd(a, (unsigned long long)lo);
            const unsigned long long carry = old + lo < old ? 1ull : 0ull;
            atomicAdd(a + 1, (unsigned long long)hi + carry);
        }
    } else {
        __shared__ double red[4][6];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const double s = dsum_wave(acc[k]);
            if (lane == 0) red[wv][k] = s;
        }
        __syncthreads();
        if (threadIdx.x < 6) {
            const double s = (red[0][threadIdx.x] + red[1][threadIdx.x]) +
                             (red[2][threadIdx.x] + red[3][threadIdx.x]);
            atomicAdd(FT + 6 * p + threadIdx.x, s);
            if (!isfinite(s)) atomicOr(numeric, 1u);  // reported by the next classification
        }
    }
}

// The exact sums as doubles (rounded once each word).
__global__ __launch_bounds__(256) void k_fixed_to_f64(const unsigned long long* __restrict__ FX,
                                                      double* __restrict__ FT, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    FT[i] = (double)(int64_t)FX[2 * i + 1] * 0x1p-16 + (double)FX[2 * i] * 0x1p-80;
}

// ---------------------------------------------------------------------------
// Refill: one thread per node uncovered since the previous classification.
// The count is read on the device (the list's cursor, at most cap), so the
// launch needs no read-back; a grid of at most a few thousand workgroups
// strides over the list.  Each node reads only the previous populations and
// owners and writes only its own populations and moments, so running the
// kernel again over a longer list (after the list has grown) gives the same
// values at the nodes of the first run.
// ---------------------------------------------------------------------------
template <int S>
__device__ __forceinline__ void refill_node(const typename St<S>::T* __restrict__ prev,
                                            typename St<S>::T* __restrict__ cur,
                                            typename St<S>::M* __restrict__ mom,
                                            const RefillRec r,
                                            const uint32_t* __restrict__ own_prev,
                                            const PartDev& P, const Geom& g, const Phys& ph)
{
    using A = typename St<S>::A;
    constexpr bool DEV = St<S>::dev;
    const int p = r.part;
    const uint32_t nx = g.n[0], ny = g.n[1];
    const int c[3] = {(int)(r.node % nx), (int)((r.node / nx) % ny), (int)(r.node / (nx * ny))};
    double rr[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double xp = P.pos[3 * p + a];
        rr[a] = image_coord(c[a], g.n[a], g.per[a], xp) - xp;
    }
    const double wp[3] = {P.omega[3 * p], P.omega[3 * p + 1], P.omega[3 * p + 2]};
    const A un[3] = {A(P.vel[3 * p] + (wp[1] * rr[2] - wp[2] * rr[1])),
                     A(P.vel[3 * p + 1] + (wp[2] * rr[0] - wp[0] * rr[2])),
                     A(P.vel[3 * p + 2] + (wp[0] * rr[1] - wp[1] * rr[0]))};
    const A r0 = A(ph.rho0), dr0 = A(ph.rho0 - 1.0);
    A v[kQ];
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        int cu[3] = {c[0] - cx(i), c[1] - cy(i), c[2] - cz(i)};
        int cd[3] = {c[0] + cx(i), c[1] + cy(i), c[2] + cz(i)};
        const bool iu = i > 0 && wrap3(cu, g);
        const bool id = i > 0 && wrap3(cd, g);
        const uint32_t nu = iu ? node_of(cu, g) : r.node;
        const uint32_t nd = id ? node_of(cd, g) : r.node;
        // both candidate populations load beside the owners (both indices
        // are nodes of the lattice), the owners then pick
        const A a_up = St<S>::ld(prev + (int64_t)i * g.stride + nu, ph.inv_scale);
        const A a_dn = St<S>::ld(prev + (int64_t)opp(i) * g.stride + nd, ph.inv_scale);
        const bool up = iu && own_prev[nu] == kFluid;
        const bool dn = id && own_prev[nd] == kFluid;
        if (up) {
            v[i] = a_up;  // streamed
        } else if (dn) {
            const A eu = A(cx(i)) * un[0] + A(cy(i)) * un[1] + A(cz(i)) * un[2];
            v[i] = a_dn + A(6) * W<A>(i) * r0 * eu;  // bounce-back of the streamed opposite
        } else {
            v[i] = eq_i<DEV, A>(i, dr0, r0, un[0], un[1], un[2]);
        }
    }
    A F[3];
    A om;
    if constexpr (DEV) {
        F[0] = ph.Ff[0], F[1] = ph.Ff[1], F[2] = ph.Ff[2];
        om = ph.omegaf;
    } else {
        F[0] = ph.F[0], F[1] = ph.F[1], F[2] = ph.F[2];
        om = ph.omega;
    }
    A drho, ux, uy, uz;
    collide<DEV, A>(v, om, F, drho, ux, uy, uz);
#pragma unroll
    for (int i = 0; i < kQ; ++i) St<S>::st(cur + (int64_t)i * g.stride + r.node, v[i], ph.scale);
    St<S>::st_mom(mom + r.node, drho, ux, uy, uz, ph.scale);
}

template <int S>
__global__ __launch_bounds__(256) void k_refill(const typename St<S>::T* __restrict__ prev,
                                                typename St<S>::T* __restrict__ cur,
                                                typename St<S>::M* __restrict__ mom,
                                                const RefillRec* __restrict__ rec,
                                                const uint32_t* __restrict__ cursor, uint32_t cap,
                                                const uint32_t* __restrict__ err,
                                                const uint32_t* __restrict__ own_prev, PartDev P,
                                                Geom g, Phys ph)
{
    if (*err) return;  // the classification's box check failed: nothing was listed
    const uint32_t cnt = min(*cursor, cap);
    for (uint32_t l = blockIdx.x * 256u + threadIdx.x; l < cnt; l += gridDim.x * 256u)
        refill_node<S>(prev, cur, mom, rec[l], own_prev, P, g, ph);
}

// ---------------------------------------------------------------------------
// Import / export
// ---------------------------------------------------------------------------
template <int S>
__global__ void k_init_eq(typename St<S>::T* f, typename St<S>::M* mom, Geom g, Phys ph, double u0x,
                          double u0y, double u0z)
{
    using A = typename St<S>::A;
    constexpr bool DEV = St<S>::dev;
    const uint32_t cell = blockIdx.x * 256u + threadIdx.x;
    if (cell >= g.ncell) return;
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        const A v = eq_i<DEV, A>(i, A(ph.rho0 - 1.0), A(ph.rho0), A(u0x), A(u0y), A(u0z));
        St<S>::st(f + (int64_t)i * g.stride + cell, v, ph.scale);
    }
    // the initial populations count as post-collision ones: u = (rho0 u0 - F/2) / rho0
    St<S>::st_mom(mom + cell, A(ph.rho0 - 1.0), A(u0x - 0.5 * ph.F[0] / ph.rho0),
                  A(u0y - 0.5 * ph.F[1] / ph.rho0), A(u0z - 0.5 * ph.F[2] / ph.rho0), ph.scale);
}

template <int S>
__global__ void k_get(const typename St<S>::T* f, double* out, Geom g, Phys ph)
{
    const uint32_t cell = blockIdx.x * 256u + threadIdx.x;
    if (cell >= g.ncell) return;
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        double v = (double)St<S>::ld(f + (int64_t)i * g.stride + cell, ph.inv_scale);
        if constexpr (St<S>::dev) v += wgt(i);
        out[(int64_t)i * g.ncell + cell] = v;
    }
}

template <int S>
__global__ void k_set(typename St<S>::T* f, typename St<S>::M* mom, const double* in, Geom g,
                      Phys ph)
{
    using A = typename St<S>::A;
    const uint32_t cell = blockIdx.x * 256u + threadIdx.x;
    if (cell >= g.ncell) return;
    double rho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        const double fi = in[(int64_t)i * g.ncell + cell];
        rho += fi;
        jx += cx(i) * fi;
        jy += cy(i) * fi;
        jz += cz(i) * fi;
        double v = fi;
        if constexpr (St<S>::dev) v -= wgt(i);
        St<S>::st(f + (int64_t)i * g.stride + cell, A(v), ph.scale);
    }
    // the given populations are post-collision: u = (sum f e - F/2) / rho
    St<S>::st_mom(mom + cell, A(rho - 1.0), A((jx - 0.5 * ph.F[0]) / rho),
                  A((jy - 0.5 * ph.F[1]) / rho), A((jz - 0.5 * ph.F[2]) / rho), ph.scale);
}

__global__ void k_zero(double* p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

__global__ void k_split(const double* FT, double* F, double* T, int n)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    for (int a = 0; a < 3; ++a) {
        F[3 * i + a] = FT[6 * i + a];
        T[3 * i + a] = FT[6 * i + 3 + a];
    }
}

inline uint32_t blocks_for(int64_t n) { return (uint32_t)((n + 255) / 256); }

template <template <int> class Fn, class... Args>
hipError_t dispatch(int storage, Args&&... args)
{
    switch (storage) {
    case LBM_STORE_F64: return Fn<LBM_STORE_F64>::run(args...);
    case LBM_STORE_F32: return Fn<LBM_STORE_F32>::run(args...);
    case LBM_STORE_F16: return Fn<LBM_STORE_F16>::run(args...);
    default: return hipErrorInvalidValue;
    }
}

template <int S>
struct RunInit {
    static hipError_t run(lbm_ctx* c, void* f)
    {
        hipLaunchKernelGGL(k_init_eq<S>, dim3(blocks_for(c->geom.ncell)), dim3(256), 0, c->stream,
                           (typename St<S>::T*)f, (typename St<S>::M*)c->mom, c->geom, c->phys,
                           c->cfg.u0[0], c->cfg.u0[1], c->cfg.u0[2]);
        return hipGetLastError();
    }
};

template <int S>
struct RunSC {
    static hipError_t run(lbm_ctx* c, const void* src, void* dst)
    {
        // FP16 only: for FP32 the pair kernel was measured slower (4.8 against
        // 4.4 ms on 512^3), the single-node pass already runs at copy speed
        if constexpr (S == LBM_STORE_F16) {
            if (c->geom.n[0] % 2 == 0) {
                uint32_t nb = blocks_for(c->geom.ncell / 2);
                nb = (nb + 7u) & ~7u;
                hipLaunchKernelGGL(k_stream_collide_x2<S>, dim3(nb), dim3(256), 0, c->stream,
                                   (const typename St<S>::T*)src, (typename St<S>::T*)dst,
                                   (typename St<S>::M*)c->mom, c->flag, c->geom, c->phys);
                return hipGetLastError();
            }
        }
        uint32_t nb = blocks_for(c->geom.ncell);
        nb = (nb + 7u) & ~7u;  // whole rounds over the 8 XCDs
        hipLaunchKernelGGL(k_stream_collide<S>, dim3(nb), dim3(256), 0, c->stream,
                           (const typename St<S>::T*)src, (typename St<S>::T*)dst,
                           (typename St<S>::M*)c->mom, c->flag, c->geom, c->phys);
        return hipGetLastError();
    }
};

template <int S>
struct RunBC {
    static hipError_t run(lbm_ctx* c, void* f, const PartDev& P)
    {
        if (c->cfg.n_particles == 0 || c->link_max == 0 || c->lay->chunks() == 0)
            return hipSuccess;
        const dim3 grid((uint32_t)c->lay->chunks());
        if (c->FX) {
            const int64_t n6 = 6 * (int64_t)c->cfg.n_particles;
            hipLaunchKernelGGL(k_zero, dim3(blocks_for(2 * n6)), dim3(256), 0, c->stream,
                               reinterpret_cast<double*>(c->FX), 2 * n6);
            hipLaunchKernelGGL((k_boundary<S, true>), grid, dim3(256), 0, c->stream,
                               (typename St<S>::T*)f, (const typename St<S>::M*)c->mom, c->links,
                               c->link_cursor, c->lay->off_dev, c->lay->chunk_dev, P, c->FT, c->FX,
                               c->geom, c->phys, c->numeric);
            hipLaunchKernelGGL(k_fixed_to_f64, dim3(blocks_for(n6)), dim3(256), 0, c->stream, c->FX,
                               c->FT, n6);
        } else {
            hipLaunchKernelGGL((k_boundary<S, false>), grid, dim3(256), 0, c->stream,
                               (typename St<S>::T*)f, (const typename St<S>::M*)c->mom, c->links,
                               c->link_cursor, c->lay->off_dev, c->lay->chunk_dev, P, c->FT,
                               nullptr, c->geom, c->phys, c->numeric);
        }
        return hipGetLastError();
    }
};

template <int S>
struct RunRefill {
    static hipError_t run(lbm_ctx* c, const void* fprev, void* fcur, const uint32_t* own_prev,
                          const PartDev& P)
    {
        const uint32_t nb = std::min<uint32_t>(blocks_for(c->refill_cap), 2048u);
        hipLaunchKernelGGL(k_refill<S>, dim3(nb), dim3(256), 0, c->stream,
                           (const typename St<S>::T*)fprev, (typename St<S>::T*)fcur,
                           (typename St<S>::M*)c->mom, c->refill, c->refill_cursor,
                           (uint32_t)c->refill_cap, c->err, own_prev, P, c->geom, c->phys);
        return hipGetLastError();
    }
};

template <int S>
struct RunGet {
    static hipError_t run(lbm_ctx* c, const void* f, double* out)
    {
        hipLaunchKernelGGL(k_get<S>, dim3(blocks_for(c->geom.ncell)), dim3(256), 0, c->stream,
                           (const typename St<S>::T*)f, out, c->geom, c->phys);
        return hipGetLastError();
    }
};

// Density and velocity of every node from the moment plane, in FP64.
template <int S>
__global__ __launch_bounds__(256) void k_get_moments(const typename St<S>::M* __restrict__ mom,
                                                     double* __restrict__ rho,
                                                     double* __restrict__ u, Geom g, Phys ph)
{
    using A = typename St<S>::A;
    const uint32_t cell = blockIdx.x * 256u + threadIdx.x;
    if (cell >= g.ncell) return;
    A d, ux, uy, uz;
    St<S>::ld_mom(mom + cell, ph.inv_scale, d, ux, uy, uz);
    rho[cell] = 1.0 + (double)d;
    u[3 * (int64_t)cell] = (double)ux;
    u[3 * (int64_t)cell + 1] = (double)uy;
    u[3 * (int64_t)cell + 2] = (double)uz;
}

template <int S>
struct RunMoments {
    static hipError_t run(lbm_ctx* c, double* rho, double* u)
    {
        hipLaunchKernelGGL(k_get_moments<S>, dim3(blocks_for(c->geom.ncell)), dim3(256), 0,
                           c->stream, (const typename St<S>::M*)c->mom, rho, u, c->geom, c->phys);
        return hipGetLastError();
    }
};

template <int S>
struct RunSet {
    static hipError_t run(lbm_ctx* c, void* f, const double* in)
    {
        hipLaunchKernelGGL(k_set<S>, dim3(blocks_for(c->geom.ncell)), dim3(256), 0, c->stream,
                           (typename St<S>::T*)f, (typename St<S>::M*)c->mom, in, c->geom, c->phys);
        return hipGetLastError();
    }
};

}  // namespace

namespace MDLBM_QNS {

hipError_t launch_init_equilibrium(lbm_ctx* c, void* f)
{
    return dispatch<RunInit>(c->cfg.storage, c, f);
}
hipError_t launch_stream_collide(lbm_ctx* c, const void* src, void* dst)
{
    return dispatch<RunSC>(c->cfg.storage, c, src, dst);
}
hipError_t launch_boundary(lbm_ctx* c, void* f, const PartDev& P)
{
    return dispatch<RunBC>(c->cfg.storage, c, f, P);
}
hipError_t launch_refill(lbm_ctx* c, const void* fprev, void* fcur, const uint32_t* own_prev,
                         const PartDev& P)
{
    return dispatch<RunRefill>(c->cfg.storage, c, fprev, fcur, own_prev, P);
}
hipError_t launch_get_populations(lbm_ctx* c, const void* f, double* out)
{
    return dispatch<RunGet>(c->cfg.storage, c, f, out);
}
hipError_t launch_set_populations(lbm_ctx* c, void* f, const double* in)
{
    return dispatch<RunSet>(c->cfg.storage, c, f, in);
}
hipError_t launch_get_moments(lbm_ctx* c, double* rho, double* u)
{
    return dispatch<RunMoments>(c->cfg.storage, c, rho, u);
}
hipError_t launch_zero_f64(lbm_ctx* c, double* p, int64_t n)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3(blocks_for(n)), dim3(256), 0, c->stream, p, n);
    return hipGetLastError();
}
hipError_t launch_split_forces(const lbm_ctx* c, double* F, double* T)
{
    const int n = c->cfg.n_particles;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_split, dim3(blocks_for(n)), dim3(256), 0, c->stream, c->FT, F, T, n);
    return hipGetLastError();
}

}  // namespace MDLBM_QNS
}  // namespace mdlbm

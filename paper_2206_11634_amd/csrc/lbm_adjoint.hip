// Adjoint of the lattice step (differentiation form; not part of the paper).
//
// With the geometry schedule held fixed, one taped step maps the populations
// f(n) (fluid nodes of the owners at n) to f(n+1) (fluid nodes of the owners
// at n+1): link reconstruction from f(n), pull streaming and BGK + Guo
// collision of the fluid nodes of n, and refilling + collision of the nodes
// uncovered between n and n+1.  The objective adds, per step, the momentum
// exchange force and torque of every particle weighted by (wF, wT).
//
// One adjoint step n <- n+1 runs three kernels:
//  1. k_adj_node   per node x fluid at n: recompute its pulled pre-collision
//                  populations, apply the transposed collision Jacobian to
//                  lambda(n+1) -> Lambda (the adjoint of the pre-collision
//                  populations), accumulate dJ/dtau, dJ/dF; then (every node)
//                  push Lambda to the entries of lambda(n) that x read: entry
//                  (j, x - e_j), of which x is the only writer (x itself for
//                  entries read through a wall); and list the nodes refilled
//                  between n and n+1;
//     k_adj_refill the same for the listed nodes, whose pre-collision
//                  populations come from the refill rules; also dJ/dv of the
//                  wall velocity in those rules;
//  2. k_adj_links  per link: adjoint of its reconstructed population (Lambda
//                  of the fluid node that pulled the ghost slot, left in
//                  lambda(n) at the solid node, plus the objective), transposed
//                  through VIBB / halfway by forward-mode dual numbers and
//                  added to lambda(n) at x_f and x_ff with atomics; momentum-
//                  exchange and missing-point objective terms; dJ/dv, dJ/dF.
// Arithmetic is that of the storage (double for FP64, float otherwise);
// parameter gradients are summed in FP64.
#include <algorithm>

#include "lbm_internal.h"
#include "lbm_stencil.h"
#include "lbm_kernels.h"

namespace mdlbm {
namespace {

// ---------------------------------------------------------------------------
// forward-mode dual numbers with N tangents
// ---------------------------------------------------------------------------
template <class A, int N>
struct Dual {
    A v;
    A d[N];
    __device__ Dual() = default;
    __device__ Dual(A x) : v(x)
    {
#pragma unroll
        for (int k = 0; k < N; ++k) d[k] = A(0);
    }
};
template <class A, int N>
__device__ __forceinline__ Dual<A, N> var(A v, int k)
{
    Dual<A, N> r(v);
    r.d[k] = A(1);
    return r;
}
template <class A, int N>
__device__ __forceinline__ Dual<A, N> operator+(const Dual<A, N>& a, const Dual<A, N>& b)
{
    Dual<A, N> r;
    r.v = a.v + b.v;
#pragma unroll
    for (int k = 0; k < N; ++k) r.d[k] = a.d[k] + b.d[k];
    return r;
}
template <class A, int N>
__device__ __forceinline__ Dual<A, N> operator-(const Dual<A, N>& a, const Dual<A, N>& b)
{
    Dual<A, N> r;
    r.v = a.v - b.v;
#pragma unroll
    for (int k = 0; k < N; ++k) r.d[k] = a.d[k] - b.d[k];
    return r;
}
template <class A, int N>
__device__ __forceinline__ Dual<A, N> operator*(const Dual<A, N>& a, const Dual<A, N>& b)
{
    Dual<A, N> r;
    r.v = a.v * b.v;
#pragma unroll
    for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
    return r;
}
template <class A, int N>
__device__ __forceinline__ Dual<A, N> operator/(const Dual<A, N>& a, const Dual<A, N>& b)
{
    Dual<A, N> r;
    const A ib = A(1) / b.v;
    r.v = a.v * ib;
#pragma unroll
    for (int k = 0; k < N; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) * ib;
    return r;
}

// Equilibrium of direction d at (rho, u), in the deviation form (feq - w) when
// DEV, generic scalar T.
template <bool DEV, class A, class T>
__device__ __forceinline__ T eq_t(int d, const int e[3], const T& rho, const T u[3])
{
    const T eu = T(A(e[0])) * u[0] + T(A(e[1])) * u[1] + T(A(e[2])) * u[2];
    const T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const T poly = T(A(3)) * eu + T(A(4.5)) * (eu * eu) - T(A(1.5)) * uu;
    const T w = T(W<A>(d));
    if constexpr (DEV)
        return w * ((rho - T(A(1))) + rho * poly);
    else
        return w * (rho + rho * poly);
}

// The reconstructed population of a link from its inputs: the formulas of
// the forward link kernel (VIBB, Eqs. eqneq, neqd, rhod, u*_d, u**_d, u_d; or
// halfway bounce-back), written for a generic scalar; q is a scalar of the
// same kind so that its derivative can be carried too.
template <class A>
__device__ __forceinline__ A val(const A& x)
{
    return x;
}
template <class A, int N>
__device__ __forceinline__ A val(const Dual<A, N>& x)
{
    return x.v;
}

template <bool DEV, class A, class T>
__device__ T link_value(int kind, int d, const int e[3], const T& q, const T& fdf, const T& rf,
                        const T* uf, const T& fdff, const T& rff, const T* uff, const T* uw,
                        bool neq_split)
{
    const T ebu = T(A(-e[0])) * uw[0] + T(A(-e[1])) * uw[1] + T(A(-e[2])) * uw[2];
    const T mw = T(A(6) * W<A>(d)) * rf * ebu;
    if (kind != LBM_LINK_VIBB) return fdf + mw;
    const A qv = val(q);
    const T one = T(A(1));
    const T tq = T(A(2)) * q, oq = one - tq;
    const bool hold = neq_split && qv > A(0.5);
    const T fneq = (hold ? one : tq) * (fdf - eq_t<DEV, A>(d, e, rf, uf)) +
                   (hold ? T(A(0)) : oq) * (fdff - eq_t<DEV, A>(d, e, rff, uff));
    const T rd = (qv <= A(0.5)) ? tq * rf + oq * rff : rf;
    const T c1 = (one - q) / q, c2 = (tq - one) / q;
    const T c3 = (one - q) / (one + q), c4 = tq / (one + q);
    T ud[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const T us = (qv <= A(0.5)) ? tq * uf[a] + oq * uff[a] : c1 * uf[a] + c2 * uw[a];
        const T uss = c3 * uff[a] + c4 * uw[a];
        ud[a] = us / T(A(3)) + T(A(2)) * uss / T(A(3));
    }
    return eq_t<DEV, A>(d, e, rd, ud) + fneq + mw;
}

// Metaball sum of one particle at X (world coordinates of the image nearest
// the particle), its gradient in X, and its derivative for a small rotation
// of the body about its centre xp: each point x_i moves by dtheta x (x_i - xp),
// so dM/dtheta = sum_i (x_i - xp) x dm_i/dx_i with dm_i/dx_i = -grad_X m_i.
__device__ __forceinline__ void metaball_grad(const double* pts, const double* K, int i0, int i1,
                                              const double X[3], const double xp[3], double& M,
                                              double gM[3], double gR[3])
{
    M = 0.0;
    gM[0] = gM[1] = gM[2] = 0.0;
    gR[0] = gR[1] = gR[2] = 0.0;
    for (int i = i0; i < i1; ++i) {
        const double r[3] = {X[0] - pts[3 * i], X[1] - pts[3 * i + 1], X[2] - pts[3 * i + 2]};
        const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        const double t = K[i] / r2;
        M += t;
        const double s = -2.0 * t / r2;
        gM[0] += s * r[0];
        gM[1] += s * r[1];
        gM[2] += s * r[2];
        const double b[3] = {pts[3 * i] - xp[0], pts[3 * i + 1] - xp[1], pts[3 * i + 2] - xp[2]};
        // (x_i - xp) x (-s r)
        gR[0] -= s * (b[1] * r[2] - b[2] * r[1]);
        gR[1] -= s * (b[2] * r[0] - b[0] * r[2]);
        gR[2] -= s * (b[0] * r[1] - b[1] * r[0]);
    }
}

// Pose data of one taped step for the geometry terms of the adjoint, and
// where the per-particle derivatives go.  Prescribed trajectories: the pose
// gradients of each step (stride 6: x, theta) and one dJ/dv for all steps
// (stride 3); free motion: the state adjoints of the steps (stride 12: x,
// theta, v, omega).
struct GeoArgs {
    const double* wpts = nullptr;   // world control points of the step's pose
    const double* K = nullptr;
    const double* c0 = nullptr;
    const int32_t* off = nullptr;
    int exact_q = 0;
    double* g_links = nullptr;      // dJ/d(x_p, theta_p) of the pose the links used
    double* g_refill = nullptr;     // dJ/dx_p of the pose the refill used
    int gstride = 6;
    double* v_links = nullptr;      // dJ/dv_p seen by the links (null: grad + 4)
    double* v_refill = nullptr;     // dJ/dv_p seen by the refill (null: grad + 4)
    int vstride = 3;
    double* w_links = nullptr;      // dJ/domega_p seen by the links (null: not kept)
    double* w_refill = nullptr;     // dJ/domega_p seen by the refill (null: not kept)
};

__device__ __forceinline__ void dir_of(int d, int e[3])
{
    e[0] = cx(d);
    e[1] = cy(d);
    e[2] = cz(d);
}

// Sum n doubles over the block and add them to out[] (one atomic each).
template <int NV>
__device__ __forceinline__ void block_add(double (&v)[NV], double* const* out)
{
    __shared__ double red[4][NV];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double s = dsum_wave(v[k]);
        if (lane == 0) red[wv][k] = s;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        const double s = (red[0][threadIdx.x] + red[1][threadIdx.x]) +
                         (red[2][threadIdx.x] + red[3][threadIdx.x]);
        if (s != 0.0) atomicAdd(out[threadIdx.x], s);
    }
}

// ---------------------------------------------------------------------------
// 1. transposed collision per node, pushed to lambda(n)
// ---------------------------------------------------------------------------

// Lambda = (d post / d pre)^T lambda for BGK + Guo at the pre-collision state
// pre, in closed form: Lambda_j = (1 - omega) lambda_j + omega a
// + H . (e_j - u) / rho.  Returns the coefficients; adds dJ/dF (3) and dJ/dtau
// to acc.
template <class A>
struct AdjCoef {
    A om, a, H[3], u[3], ir;
    __device__ __forceinline__ A operator()(int j, A lam_j) const
    {
        return (A(1) - om) * lam_j + om * a +
               (H[0] * (A(cx(j)) - u[0]) + H[1] * (A(cy(j)) - u[1]) + H[2] * (A(cz(j)) - u[2])) * ir;
    }
};

template <bool DEV, class A>
__device__ __forceinline__ AdjCoef<A> adj_collide(const A lam[kQ], const A pre[kQ], const Phys& ph,
                                                  double acc[4])
{
    A F[3];
    A om;
    if constexpr (DEV) {
        F[0] = ph.Ff[0], F[1] = ph.Ff[1], F[2] = ph.Ff[2];
        om = ph.omegaf;
    } else {
        F[0] = ph.F[0], F[1] = ph.F[1], F[2] = ph.F[2];
        om = ph.omega;
    }
    A drho, rho, u[3];
    moments<DEV, A>(pre, A(0.5), F, drho, rho, u[0], u[1], u[2]);
    const A uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const A uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
    const A gf = A(1) - A(0.5) * om;
    // feq - pre - S/2 sums to zero over i, so its weight in dJ/domega may be
    // centred on the mean of lambda, which keeps the sum free of the
    // cancellation of a large common adjoint density
    A lbar = A(0);
#pragma unroll
    for (int i = 0; i < kQ; ++i) lbar += lam[i];
    lbar *= A(1.0 / kQ);
    // weighted moments of lambda, m0 = sum w l, m1 = sum w l e, m2 = sum w l e e:
    // the sums over i of the equilibrium's and the forcing's derivatives are
    // polynomials in u and F with these coefficients
    A m0 = A(0), m1[3] = {A(0), A(0), A(0)};
    A mxx = A(0), myy = A(0), mzz = A(0), mxy = A(0), mxz = A(0), myz = A(0);
    A dom = A(0);
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        const A wl = W<A>(i) * lam[i];
        m0 += wl;
        if (cx(i)) {
            m1[0] += A(cx(i)) * wl;
            mxx += wl;
        }
        if (cy(i)) {
            m1[1] += A(cy(i)) * wl;
            myy += wl;
        }
        if (cz(i)) {
            m1[2] += A(cz(i)) * wl;
            mzz += wl;
        }
        if (cx(i) && cy(i)) mxy += A(cx(i) * cy(i)) * wl;
        if (cx(i) && cz(i)) mxz += A(cx(i) * cz(i)) * wl;
        if (cy(i) && cz(i)) myz += A(cy(i) * cz(i)) * wl;
        const A eu = A(cx(i)) * u[0] + A(cy(i)) * u[1] + A(cz(i)) * u[2];
        const A eF = A(cx(i)) * F[0] + A(cy(i)) * F[1] + A(cz(i)) * F[2];
        const A St_i = W<A>(i) * (A(3) * (eF - uF) + A(9) * eu * eF);
        const A feq = eq_i<DEV, A>(i, drho, rho, u[0], u[1], u[2]);
        dom += (lam[i] - lbar) * (feq - pre[i] - A(0.5) * St_i);
    }
    const A m2u[3] = {mxx * u[0] + mxy * u[1] + mxz * u[2], mxy * u[0] + myy * u[1] + myz * u[2],
                      mxz * u[0] + myz * u[1] + mzz * u[2]};
    const A m2F[3] = {mxx * F[0] + mxy * F[1] + mxz * F[2], mxy * F[0] + myy * F[1] + myz * F[2],
                      mxz * F[0] + myz * F[1] + mzz * F[2]};
    const A m1u = m1[0] * u[0] + m1[1] * u[1] + m1[2] * u[2];
    const A um2u = u[0] * m2u[0] + u[1] * m2u[1] + u[2] * m2u[2];
    // a = sum w l P_i with P_i = 1 + 3 e.u + 4.5 (e.u)^2 - 1.5 u.u
    const A a = m0 * (A(1) - A(1.5) * uu) + A(3) * m1u + A(4.5) * um2u;
    A B[3], G[3], Fd[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        B[k] = rho * (A(3) * m1[k] + A(9) * m2u[k] - A(3) * u[k] * m0);
        G[k] = A(-3) * F[k] * m0 + A(9) * m2F[k];
        Fd[k] = A(3) * m1[k] - A(3) * u[k] * m0 + A(9) * m2u[k];
    }
    AdjCoef<A> co;
    co.om = om;
    co.a = a;
    co.ir = A(1) / rho;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        co.H[k] = om * B[k] + gf * G[k];
        co.u[k] = u[k];
        acc[k] += (double)(co.H[k] * A(0.5) * co.ir + gf * Fd[k]);
    }
    acc[3] += -(double)om * (double)om * (double)dom;  // dtau = -omega^2 domega
    return co;
}

// Every node x.  A node fluid at n and n + 1 recomputes its pulled
// pre-collision populations and takes the transposed collision; then x pushes
// Lambda to the entries of lambda(n) it read.  Entry (j, y) is written by
// exactly one node: x = y + e_j when that lies inside the lattice, else y
// itself (read through a wall).  Its value is Lambda_j(x) for a node x fluid
// at n (for a solid y that is the adjoint of the ghost slot, which the link
// kernel takes and clears), and zero otherwise; k_adj_refill then rewrites the
// entries its refilled nodes read.
template <int S>
// (the moment form of the transposed collision keeps the FP32 kernel at 85
// registers, five waves per SIMD; a bound of six spills)
__global__ __launch_bounds__(256) void k_adj_node(const typename St<S>::T* __restrict__ f,
                                                  const uint32_t* __restrict__ own0,
                                                  const uint32_t* __restrict__ own1,
                                                  const typename St<S>::A* __restrict__ lam1,
                                                  typename St<S>::A* __restrict__ lam0, Geom g,
                                                  Phys ph, double* grad, AdjList list)
{
    using A = typename St<S>::A;
    constexpr bool DEV = St<S>::dev;
    const uint32_t cell = blockIdx.x * 256u + threadIdx.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};  // dJ/dF (3), dJ/dtau
    bool refilled = false;
    if (cell < g.ncell) {
        const uint32_t nx = g.n[0], ny = g.n[1];
        const uint32_t x = cell % nx, y = (cell / nx) % ny, z = cell / (nx * ny);
        uint32_t ox[3], oy[3], oz[3];
        bool vx[3], vy[3], vz[3];
        axis3(x, nx, g.per[0], 1u, ox, vx);
        axis3(y, ny, g.per[1], nx, oy, vy);
        axis3(z, g.n[2], g.per[2], nx * ny, oz, vz);
        const bool live = own0[cell] == kFluid && own1[cell] == kFluid;
        A lam[kQ] = {};
        AdjCoef<A> co{};
        if (live) {
            A pre[kQ];
#pragma unroll
            for (int i = 0; i < kQ; ++i) {
                lam[i] = lam1[(int64_t)i * g.stride + cell];
                const int sx = 1 - cx(i), sy = 1 - cy(i), sz = 1 - cz(i);
                const bool ok = vx[sx] && vy[sy] && vz[sz];
                const uint32_t s = ok ? ox[sx] + oy[sy] + oz[sz] : cell;
                const int64_t plane = ok ? i : opp(i);
                pre[i] = St<S>::ld(f + plane * g.stride + s, ph.inv_scale);
            }
            co = adj_collide<DEV, A>(lam, pre, ph, acc);
        }
        // a node refilled between n and n + 1 leaves the entries it read from
        // nodes fluid at n to k_adj_refill, so the two kernels write
        // disjoint entries
        refilled = own0[cell] != kFluid && own1[cell] == kFluid;
#pragma unroll
        for (int j = 0; j < kQ; ++j) {
            const A v = live ? co(j, lam[j]) : A(0);
            const int sx = 1 - cx(j), sy = 1 - cy(j), sz = 1 - cz(j);  // x - e_j
            if (vx[sx] && vy[sy] && vz[sz]) {
                const uint32_t y = ox[sx] + oy[sy] + oz[sz];
                if (!(refilled && j > 0 && own0[y] == kFluid))
                    lam0[(int64_t)j * g.stride + y] = v;
            } else {  // x pulled f_j through a wall: its own f_opp(j)
                lam0[(int64_t)opp(j) * g.stride + cell] = v;
            }
        }
    }
    // list the refilled nodes for k_adj_refill (one atomic per wave); the
    // count may pass the capacity, which the host checks after the adjoint
    const uint64_t m = __ballot(refilled);
    if (m) {  // uniform over the wave
        const int lane = threadIdx.x & 63;
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(list.count, (uint32_t)__popcll(m));
        base = __shfl(base, 0, 64);
        const uint32_t idx = base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
        if (refilled && idx < list.cap) list.node[idx] = cell;
    }
    double* outs[4] = {grad + 0, grad + 1, grad + 2, grad + 3};
    block_add<4>(acc, outs);
}

// Nodes refilled between n and n + 1 (solid at n, fluid at n + 1): their
// pre-collision populations follow the refill rules (streamed from a node
// fluid at n, bounce-back of the opposite streamed population with the wall
// term, or the equilibrium at (rho0, u_wall)); transposed collision, dJ/dF,
// dJ/dtau, and dJ/dv of the wall velocity in the bounce-back and equilibrium
// rules.  The entries (j, x - e_j) of lambda(n) at nodes fluid at n get the
// adjoint of the streamed f_j, plus that of the bounce-back of direction
// opp(j) unless x + e_j was fluid.
template <int S>
__global__ __launch_bounds__(256) void k_adj_refill(const typename St<S>::T* __restrict__ f,
                                                    const uint32_t* __restrict__ own0,
                                                    const typename St<S>::A* __restrict__ lam1,
                                                    typename St<S>::A* __restrict__ lam0,
                                                    const double* pos1, const double* vel1,
                                                    const double* om1, Geom g, Phys ph,
                                                    double* grad, GeoArgs ga, AdjList list)
{
    using A = typename St<S>::A;
    constexpr bool DEV = St<S>::dev;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const uint32_t cnt = min(*list.count, list.cap);
    for (uint32_t l = blockIdx.x * 256u + threadIdx.x; l < cnt; l += gridDim.x * 256u) {
        const uint32_t cell = list.node[l];
        const uint32_t o0 = own0[cell];
        const uint32_t nx = g.n[0], ny = g.n[1];
        const int c[3] = {(int)(cell % nx), (int)((cell / nx) % ny), (int)(cell / (nx * ny))};
        const int p = (int)o0;
        double rr[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double xp = pos1[3 * p + a];
            rr[a] = image_coord(c[a], g.n[a], g.per[a], xp) - xp;
        }
        const double* wp = om1 + 3 * p;
        const A un[3] = {A(vel1[3 * p] + (wp[1] * rr[2] - wp[2] * rr[1])),
                         A(vel1[3 * p + 1] + (wp[2] * rr[0] - wp[0] * rr[2])),
                         A(vel1[3 * p + 2] + (wp[0] * rr[1] - wp[1] * rr[0]))};
        const A r0 = A(ph.rho0), dr0 = A(ph.rho0 - 1.0);
        A lam[kQ], pre[kQ];
        uint32_t nu[kQ];
        uint64_t rule = 0;  // per direction: 0 streamed, 1 bounce-back, 2 equilibrium
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            lam[i] = lam1[(int64_t)i * g.stride + cell];
            int cuu[3] = {c[0] - cx(i), c[1] - cy(i), c[2] - cz(i)};
            int cdd[3] = {c[0] + cx(i), c[1] + cy(i), c[2] + cz(i)};
            const bool iu = i > 0 && wrap3(cuu, g);
            const bool id = i > 0 && wrap3(cdd, g);
            // both candidate populations load beside the owners (both indices
            // are nodes of the lattice), the owners then pick
            const uint32_t su = iu ? node_of(cuu, g) : cell;
            const uint32_t nd = id ? node_of(cdd, g) : cell;
            const A a_up = St<S>::ld(f + (int64_t)i * g.stride + su, ph.inv_scale);
            const A a_dn = St<S>::ld(f + (int64_t)opp(i) * g.stride + nd, ph.inv_scale);
            const bool up = iu && own0[su] == kFluid;
            const bool dn = id && own0[nd] == kFluid;
            nu[i] = up ? su : kFluid;
            const A eu = A(cx(i)) * un[0] + A(cy(i)) * un[1] + A(cz(i)) * un[2];
            if (up) {
                pre[i] = a_up;
            } else if (dn) {
                pre[i] = a_dn + A(6) * W<A>(i) * r0 * eu;
                rule |= 1ull << (2 * i);
            } else {
                pre[i] = eq_i<DEV, A>(i, dr0, r0, un[0], un[1], un[2]);
                rule |= 2ull << (2 * i);
            }
        }
        const AdjCoef<A> co = adj_collide<DEV, A>(lam, pre, ph, acc);
        A Lp[kQ];
#pragma unroll
        for (int j = 0; j < kQ; ++j) Lp[j] = co(j, lam[j]);
        // d pre_j / d u_new: 6 w rho0 e_j for the bounce-back rule, d feq_j(rho0,
        // u_new)/du for the equilibrium
        double dv[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int j = 0; j < kQ; ++j) {
            const uint32_t rj = (uint32_t)(rule >> (2 * j)) & 3u;
            if (rj) {
                const A ej[3] = {A(cx(j)), A(cy(j)), A(cz(j))};
                const A eun = ej[0] * un[0] + ej[1] * un[1] + ej[2] * un[2];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const A cuk = (rj == 1u) ? A(6) * W<A>(j) * r0 * ej[k]
                                             : W<A>(j) * r0 * (A(3) * ej[k] + A(9) * eun * ej[k] - A(3) * un[k]);
                    dv[k] += (double)(Lp[j] * cuk);
                }
            }
        }
        double* vout = ga.v_refill ? ga.v_refill + (int64_t)ga.vstride * p : grad + 4 + 3 * p;
        for (int k = 0; k < 3; ++k)
            if (dv[k] != 0.0) atomicAdd(vout + k, dv[k]);
        if (ga.g_refill) {
            // u_new = v + omega x (x - x_p): dJ/dx_p = -(dJ/du_new) x omega
            const double gx[3] = {-(dv[1] * wp[2] - dv[2] * wp[1]), -(dv[2] * wp[0] - dv[0] * wp[2]),
                                  -(dv[0] * wp[1] - dv[1] * wp[0])};
            for (int k = 0; k < 3; ++k)
                if (gx[k] != 0.0) atomicAdd(ga.g_refill + (int64_t)ga.gstride * p + k, gx[k]);
        }
        if (ga.w_refill) {
            // dJ/domega = (x - x_p) x dJ/du_new
            const double gw[3] = {rr[1] * dv[2] - rr[2] * dv[1], rr[2] * dv[0] - rr[0] * dv[2],
                                  rr[0] * dv[1] - rr[1] * dv[0]};
            for (int k = 0; k < 3; ++k)
                if (gw[k] != 0.0) atomicAdd(ga.w_refill + (int64_t)ga.vstride * p + k, gw[k]);
        }
        // entries read through the streaming rule of direction j (x - e_j fluid
        // at n): f_j(x - e_j) also fed the bounce-back of opp(j) when x + e_j
        // was not fluid
#pragma unroll
        for (int j = 1; j < kQ; ++j)
            if (nu[j] != kFluid) {
                const bool bb = ((rule >> (2 * opp(j))) & 3u) == 1u;
                lam0[(int64_t)j * g.stride + nu[j]] = bb ? Lp[j] + Lp[opp(j)] : Lp[j];
            }
    }
    double* outs[4] = {grad + 0, grad + 1, grad + 2, grad + 3};
    block_add<4>(acc, outs);
}

// ---------------------------------------------------------------------------
// 2. links: reconstruction, momentum exchange and missing points
// ---------------------------------------------------------------------------
template <class A>
__device__ __forceinline__ void atomic_add_a(A* p, A v)
{
    if (v != A(0)) atomicAdd(p, v);
}

// With GEO, also dJ/dx_p of the pose the links were built from, with the
// link set held fixed: through q (Eq. appq, or Eq. calq by the implicit
// function theorem), which moves the VIBB weights and the wall point
// x_w = x_n + q e, and through the lever arm r = x_w - x_p of the torque
// weight and of u_w = v + omega x r.
template <int S, bool GEO>
__global__ __launch_bounds__(256) void k_adj_links(const typename St<S>::T* __restrict__ f,
                                                   const LinkRec* __restrict__ links,
                                                   const uint32_t* __restrict__ cursor,
                                                   const int64_t* __restrict__ loff,
                                                   const uint32_t* __restrict__ chunk,
                                                   const double* pos,
                                                   const double* vel, const double* om,
                                                   typename St<S>::A* lam0, const double* wts,
                                                   Geom g, Phys ph, double* grad, GeoArgs ga)
{
    using A = typename St<S>::A;
    constexpr bool DEV = St<S>::dev;
    constexpr int N = GEO ? 14 : 13;  // tangents: 13 link inputs (+ q)
    using DN = Dual<A, N>;
    // one workgroup per 256-record chunk of the step's link layout
    const int p = (int)chunk[blockIdx.x];
    const int64_t g0 = (int64_t)blockIdx.x * 256;
    const int64_t cnt = min(loff[p + 1] - loff[p], (int64_t)cursor[(int64_t)p * kCursorPad]);
    if (g0 - loff[p] >= cnt) return;  // uniform over the block
    const int64_t l = g0 - loff[p] + threadIdx.x;
    // dJ/dF (3), dJ/dv_p (3), dJ/dx_p (3, GEO), dJ/dtheta_p (3, GEO),
    // dJ/domega_p (3, GEO)
    double acc[15] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (l < cnt) {
        const LinkRec r = links[g0 + threadIdx.x];
        const int d = r.d, db = opp(d);
        int e[3];
        dir_of(d, e);
        const uint32_t nx = g.n[0], ny = g.n[1];
        const int cs[3] = {(int)(r.node % nx), (int)((r.node / nx) % ny), (int)(r.node / (nx * ny))};
        int cn[3] = {cs[0] - e[0], cs[1] - e[1], cs[2] - e[2]};
        wrap3(cn, g);
        double rr[3], uw[3], Wv[3], Xn[3];
        const double* xp = pos + 3 * p;
        const double* wp = om + 3 * p;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            Xn[a] = image_coord(cn[a], g.n[a], g.per[a], xp[a]);
            rr[a] = Xn[a] + r.q * (double)e[a] - xp[a];
        }
        uw[0] = vel[3 * p] + (wp[1] * rr[2] - wp[2] * rr[1]);
        uw[1] = vel[3 * p + 1] + (wp[2] * rr[0] - wp[0] * rr[2]);
        uw[2] = vel[3 * p + 2] + (wp[0] * rr[1] - wp[1] * rr[0]);
        // objective weight of this force point: wF + wT x r (J = F.wF + (r x F).wT)
        const double* wF = wts + 6 * p;
        const double* wT = wts + 6 * p + 3;
        Wv[0] = wF[0] + (wT[1] * rr[2] - wT[2] * rr[1]);
        Wv[1] = wF[1] + (wT[2] * rr[0] - wT[0] * rr[2]);
        Wv[2] = wF[2] + (wT[0] * rr[1] - wT[1] * rr[0]);
        // geometry terms: t = the link's momentum-exchange vector, G = dJ/du_w
        // of the link (all paths), dq = dJ/dq through the reconstruction
        double tv[3] = {0, 0, 0}, G[3] = {0, 0, 0}, dq = 0.0;
        if (r.kind == LBM_LINK_MISSING) {
            // J = [(e_d - u_w) feq_d(rho0, u_w) - (e_db - u_w) feq_db(rho0, u_w)] . W
            using D3 = Dual<double, 3>;
            D3 u3[3] = {var<double, 3>(uw[0], 0), var<double, 3>(uw[1], 1), var<double, 3>(uw[2], 2)};
            int eb[3] = {-e[0], -e[1], -e[2]};
            const D3 r0 = D3(ph.rho0);
            const D3 fo = eq_t<false, double>(d, e, r0, u3);
            const D3 fi = eq_t<false, double>(db, eb, r0, u3);
            D3 J = D3(0.0);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const D3 ta = (D3((double)e[a]) - u3[a]) * fo - (D3((double)eb[a]) - u3[a]) * fi;
                J = J + D3(Wv[a]) * ta;
                tv[a] = ta.v;
            }
            acc[3] = J.d[0], acc[4] = J.d[1], acc[5] = J.d[2];
            G[0] = J.d[0], G[1] = J.d[1], G[2] = J.d[2];
        } else {
            A F[3];
            if constexpr (DEV) {
                F[0] = ph.Ff[0], F[1] = ph.Ff[1], F[2] = ph.Ff[2];
            } else {
                F[0] = ph.F[0], F[1] = ph.F[1], F[2] = ph.F[2];
            }
            const uint32_t xf = node_of(cn, g);
            A v[kQ];
#pragma unroll
            for (int i = 0; i < kQ; ++i) v[i] = St<S>::ld(f + (int64_t)i * g.stride + xf, ph.inv_scale);
            A drf, rf, uf[3];
            moments<DEV, A>(v, A(-0.5), F, drf, rf, uf[0], uf[1], uf[2]);
            A fdf = A(0);
#pragma unroll
            for (int i = 0; i < kQ; ++i) fdf = (i == d) ? v[i] : fdf;
            uint32_t xff = xf;
            A rff = A(1), uff[3] = {A(0), A(0), A(0)}, fdff = A(0), drff = A(0);
            if (r.kind == LBM_LINK_VIBB) {
                int cf[3] = {cn[0] - e[0], cn[1] - e[1], cn[2] - e[2]};
                wrap3(cf, g);
                xff = node_of(cf, g);
#pragma unroll
                for (int i = 0; i < kQ; ++i) v[i] = St<S>::ld(f + (int64_t)i * g.stride + xff, ph.inv_scale);
                moments<DEV, A>(v, A(-0.5), F, drff, rff, uff[0], uff[1], uff[2]);
#pragma unroll
                for (int i = 0; i < kQ; ++i) fdff = (i == d) ? v[i] : fdff;
            }
            // value and gradient of the reconstructed population
            DN x_fdf = var<A, N>(fdf, 0), x_rf = var<A, N>(rf, 1);
            DN x_uf[3] = {var<A, N>(uf[0], 2), var<A, N>(uf[1], 3), var<A, N>(uf[2], 4)};
            DN x_fdff = var<A, N>(fdff, 5), x_rff = var<A, N>(rff, 6);
            DN x_uff[3] = {var<A, N>(uff[0], 7), var<A, N>(uff[1], 8), var<A, N>(uff[2], 9)};
            DN x_uw[3] = {var<A, N>(A(uw[0]), 10), var<A, N>(A(uw[1]), 11),
                          var<A, N>(A(uw[2]), 12)};
            DN x_q;
            if constexpr (GEO)
                x_q = var<A, N>(A(r.q), 13);
            else
                x_q = DN(A(r.q));
            const DN unk = link_value<DEV, A>(r.kind, d, e, x_q, x_fdf, x_rf, x_uf, x_fdff,
                                              x_rff, x_uff, x_uw, ph.neq_split != 0);
            // momentum exchange of this link: [(e_d - u_w) out - (e_db - u_w) in] . W
            double out = (double)fdf, in = (double)unk.v;
            if constexpr (DEV) {
                out += wgt(d);
                in += wgt(db);
            }
            double d_out = 0.0, d_in = 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                d_out += ((double)e[a] - uw[a]) * Wv[a];
                d_in += ((double)e[a] + uw[a]) * Wv[a];
                acc[3 + a] += -(out - in) * Wv[a];
                tv[a] = ((double)e[a] - uw[a]) * out + ((double)e[a] + uw[a]) * in;
                G[a] = -(out - in) * Wv[a];
            }
            // adjoint of the reconstructed value: the fluid node that pulled
            // the ghost slot, plus the objective
            // the node kernel left the adjoint of the ghost slot (x_s, opp d),
            // which x_f pulled, in lambda(n) at x_s; take it and clear it
            A* ghost = lam0 + (int64_t)db * g.stride + r.node;
            const A lu = *ghost + A(d_in);
            *ghost = A(0);
            A gk[N];
#pragma unroll
            for (int k = 0; k < N; ++k) gk[k] = lu * unk.d[k];
            atomic_add_a(lam0 + (int64_t)d * g.stride + xf, gk[0] + A(d_out));
            const A irf = A(1) / rf;
#pragma unroll
            for (int j = 0; j < kQ; ++j) {
                const A t = gk[1] + (gk[2] * (A(cx(j)) - uf[0]) + gk[3] * (A(cy(j)) - uf[1]) +
                                     gk[4] * (A(cz(j)) - uf[2])) * irf;
                atomic_add_a(lam0 + (int64_t)j * g.stride + xf, t);
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) acc[a] += -(double)(gk[2 + a] * A(0.5) * irf);
            if (r.kind == LBM_LINK_VIBB) {
                atomic_add_a(lam0 + (int64_t)d * g.stride + xff, gk[5]);
                const A irff = A(1) / rff;
#pragma unroll
                for (int j = 0; j < kQ; ++j) {
                    const A t = gk[6] + (gk[7] * (A(cx(j)) - uff[0]) + gk[8] * (A(cy(j)) - uff[1]) +
                                         gk[9] * (A(cz(j)) - uff[2])) * irff;
                    atomic_add_a(lam0 + (int64_t)j * g.stride + xff, t);
                }
#pragma unroll
                for (int a = 0; a < 3; ++a) acc[a] += -(double)(gk[7 + a] * A(0.5) * irff);
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                acc[3 + a] += (double)gk[10 + a];
                G[a] += (double)gk[10 + a];
            }
            if constexpr (GEO) dq = (double)gk[13];
            (void)drf;
            (void)drff;
        }
        if constexpr (GEO) {
            // dJ/dr: torque weight (wT x r).t and u_w = v + omega x r
            double Jr[3];
            Jr[0] = (tv[1] * wT[2] - tv[2] * wT[1]) + (G[1] * wp[2] - G[2] * wp[1]);
            Jr[1] = (tv[2] * wT[0] - tv[0] * wT[2]) + (G[2] * wp[0] - G[0] * wp[2]);
            Jr[2] = (tv[0] * wT[1] - tv[1] * wT[0]) + (G[0] * wp[1] - G[1] * wp[0]);
            dq += Jr[0] * e[0] + Jr[1] * e[1] + Jr[2] * e[2];
            // dq/dx_p and dq/dtheta_p: translating the body by dx moves M(X)
            // by -grad M(X).dx; a small rotation moves it by dM/dtheta
            const int i0 = ga.off[p], i1 = ga.off[p + 1];
            const double c0 = ga.c0[p];
            double qx[3], qt[3];
            if (ga.exact_q) {
                const double Xw[3] = {Xn[0] + r.q * e[0], Xn[1] + r.q * e[1], Xn[2] + r.q * e[2]};
                double M, gM[3], gR[3];
                metaball_grad(ga.wpts, ga.K, i0, i1, Xw, xp, M, gM, gR);
                const double ge = gM[0] * e[0] + gM[1] * e[1] + gM[2] * e[2];
                for (int a = 0; a < 3; ++a) {
                    qx[a] = gM[a] / ge;
                    qt[a] = -gR[a] / ge;
                }
            } else {
                const double Xs[3] = {Xn[0] + e[0], Xn[1] + e[1], Xn[2] + e[2]};
                double Mn, Ms, gn[3], gs[3], rn[3], rs[3];
                metaball_grad(ga.wpts, ga.K, i0, i1, Xn, xp, Mn, gn, rn);
                metaball_grad(ga.wpts, ga.K, i0, i1, Xs, xp, Ms, gs, rs);
                const double den = (Ms - Mn) * (Ms - Mn);
                const double an = (c0 - Ms) / den, as = (Mn - c0) / den;
                for (int a = 0; a < 3; ++a) {
                    qx[a] = -(an * gn[a] + as * gs[a]);
                    qt[a] = an * rn[a] + as * rs[a];
                }
            }
            for (int a = 0; a < 3; ++a) {
                acc[6 + a] = dq * qx[a] - Jr[a];
                acc[9 + a] = dq * qt[a];
            }
            // u_w = v + omega x r: dJ/domega = r x G
            acc[12] = rr[1] * G[2] - rr[2] * G[1];
            acc[13] = rr[2] * G[0] - rr[0] * G[2];
            acc[14] = rr[0] * G[1] - rr[1] * G[0];
        }
    }
    if constexpr (GEO) {
        double* gl = ga.g_links + (int64_t)ga.gstride * p;
        double* vl = ga.v_links ? ga.v_links + (int64_t)ga.vstride * p : grad + 4 + 3 * p;
        if (ga.w_links) {
            double* wl = ga.w_links + (int64_t)ga.vstride * p;
            double* outs[15] = {grad + 0, grad + 1, grad + 2, vl, vl + 1, vl + 2, gl, gl + 1, gl + 2,
                                gl + 3, gl + 4, gl + 5, wl, wl + 1, wl + 2};
            block_add<15>(acc, outs);
        } else {
            double a12[12];
            for (int k = 0; k < 12; ++k) a12[k] = acc[k];
            double* outs[12] = {grad + 0, grad + 1, grad + 2, vl, vl + 1, vl + 2, gl, gl + 1, gl + 2,
                                gl + 3, gl + 4, gl + 5};
            block_add<12>(a12, outs);
        }
    } else {
        double a6[6] = {acc[0], acc[1], acc[2], acc[3], acc[4], acc[5]};
        double* outs[6] = {grad + 0, grad + 1, grad + 2, grad + 4 + 3 * p, grad + 5 + 3 * p,
                           grad + 6 + 3 * p};
        block_add<6>(a6, outs);
    }
}

inline uint32_t blocks_for(int64_t n) { return (uint32_t)((n + 255) / 256); }

template <int S>
struct RunAdj {
    static hipError_t run(lbm_ctx* c, const TapeStep& ts, const uint32_t* own1, const double* pos1,
                          const double* vel1, const double* om1, const void* lam1,
                          void* lam0, const double* wts, double* grad, const GeoArgs& ga,
                          const AdjList& list, int parts)
    {
        using T = typename St<S>::T;
        using A = typename St<S>::A;
        if (parts & kAdjNode)
            hipLaunchKernelGGL(k_adj_node<S>, dim3(blocks_for(c->geom.ncell)), dim3(256), 0,
                               c->stream, (const T*)ts.f, ts.own_use, own1, (const A*)lam1, (A*)lam0,
                               c->geom, c->phys, grad, list);
        if (parts & kAdjRefill) {
            // a grid that one round of resident workgroups covers
            const uint32_t nb = std::min<uint32_t>(blocks_for(list.cap), 512u);
            hipLaunchKernelGGL(k_adj_refill<S>, dim3(nb), dim3(256), 0, c->stream, (const T*)ts.f,
                               ts.own_use, (const A*)lam1, (A*)lam0, pos1, vel1, om1, c->geom, c->phys,
                               grad, ga, list);
        }
        if ((parts & kAdjLinks) && c->cfg.n_particles > 0 && ts.link_max > 0 && ts.lay &&
            ts.lay->chunks() > 0) {
            const int np = c->cfg.n_particles;
            const dim3 grid((uint32_t)ts.lay->chunks());
            if (ga.g_links)
                hipLaunchKernelGGL((k_adj_links<S, true>), grid, dim3(256), 0, c->stream,
                                   (const T*)ts.f, ts.links_use, ts.cursor, ts.lay->off_dev,
                                   ts.lay->chunk_dev, ts.part, ts.part + 3 * np,
                                   ts.part + 6 * np, (A*)lam0, wts, c->geom, c->phys, grad, ga);
            else
                hipLaunchKernelGGL((k_adj_links<S, false>), grid, dim3(256), 0, c->stream,
                                   (const T*)ts.f, ts.links_use, ts.cursor, ts.lay->off_dev,
                                   ts.lay->chunk_dev, ts.part, ts.part + 3 * np,
                                   ts.part + 6 * np, (A*)lam0, wts, c->geom, c->phys, grad, ga);
        }
        return hipGetLastError();
    }
};

// The small arrays of one taped step in one launch: the first word of every
// link cursor line, the particle state (position, velocity, angular
// velocity, world control points, quaternion, F^h and T^h of the step), and
// the DEM state the next dem_step starts from (pair records, wall records,
// carried contact sums; the pair records' keys).
__global__ void k_tape_small(uint32_t* __restrict__ tcur, const uint32_t* __restrict__ cur,
                             double* __restrict__ part, const double* __restrict__ pos,
                             const double* __restrict__ vel, const double* __restrict__ om,
                             const double* __restrict__ wpts, const double* __restrict__ quat,
                             const double* __restrict__ FT, int np, int nctrl,
                             double* __restrict__ dem, int32_t* __restrict__ dem_key,
                             const double* __restrict__ hpp, const double* __restrict__ hpw,
                             const double* __restrict__ fc, const int32_t* __restrict__ hkey)
{
    const int i = (int)(blockIdx.x * 256u + threadIdx.x);
    if (i < np) tcur[(int64_t)i * kCursorPad] = cur[(int64_t)i * kCursorPad];
    if (i < 3 * np) {
        part[i] = pos[i];
        part[3 * np + i] = vel[i];
        part[6 * np + i] = om[i];
    }
    if (i < 3 * nctrl) part[9 * np + i] = wpts[i];
    double* tq = part + 9 * np + 3 * nctrl;
    if (quat && i < 4 * np) tq[i] = quat[i];
    if (i < 6 * np) tq[4 * np + i] = FT[i];
    const int npp = np * kPairSlots;
    if (i < 8 * npp) dem[i] = hpp[i];
    if (i < 48 * np) dem[8 * npp + i] = hpw[i];
    if (i < 6 * np) dem[8 * npp + 48 * np + i] = fc[i];
    if (i < npp) dem_key[i] = hkey[i];
}

}  // namespace

namespace MDLBM_QNS {

hipError_t launch_tape_small(lbm_ctx* c, TapeStep& t, const lbm_particles* P)
{
    const int np = c->cfg.n_particles, nctrl = c->cfg.n_ctrl;
    if (np == 0) return hipSuccess;
    const int64_t n = std::max<int64_t>({8 * (int64_t)np * kPairSlots, 48 * (int64_t)np,
                                         3 * (int64_t)nctrl});
    hipLaunchKernelGGL(k_tape_small, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, c->stream,
                       t.cursor, c->link_cursor, t.part, P->pos, P->vel, P->omega, P->world_pts,
                       P->quat, c->FT, np, nctrl, t.dem, t.dem_key, c->hist_pp, c->hist_pw, c->fc,
                       c->hist_key);
    return hipGetLastError();
}

hipError_t launch_adjoint_step(lbm_ctx* c, const TapeStep& ts, const uint32_t* own1,
                               const double* pos1, const double* vel1, const double* om1,
                               const void* lam1, void* lam0, const double* wts,
                               double* grad, const lbm_particles* P, const AdjOut& out,
                               const AdjList& list, int parts)
{
    GeoArgs ga;
    const int np = c->cfg.n_particles;
    ga.wpts = ts.part + 9 * np;
    ga.K = P->K;
    ga.c0 = P->c0;
    ga.off = P->ctrl_off;
    ga.exact_q = (c->cfg.treatments & LBM_TREAT_EXACT_Q) ? 1 : 0;
    ga.g_links = out.g_links;
    ga.g_refill = out.g_refill;
    ga.gstride = out.gstride;
    ga.v_links = out.v_links;
    ga.v_refill = out.v_refill;
    ga.w_links = out.w_links;
    ga.w_refill = out.w_refill;
    ga.vstride = out.vstride;
    switch (c->cfg.storage) {
    case LBM_STORE_F64:
        return RunAdj<LBM_STORE_F64>::run(c, ts, own1, pos1, vel1, om1, lam1, lam0, wts, grad, ga,
                                          list, parts);
    case LBM_STORE_F32:
        return RunAdj<LBM_STORE_F32>::run(c, ts, own1, pos1, vel1, om1, lam1, lam0, wts, grad, ga,
                                          list, parts);
    case LBM_STORE_F16:
        return RunAdj<LBM_STORE_F16>::run(c, ts, own1, pos1, vel1, om1, lam1, lam0, wts, grad, ga,
                                          list, parts);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace MDLBM_QNS
}  // namespace mdlbm

// Adjoint of one dem_step call for free motion (differentiation form; not
// part of the paper).
//
// One call advances each particle's state s = (x, q, v, omega) by n_sub
// velocity-Verlet substeps under the hydrodynamic force and torque (F, T) of
// the lattice step, relative gravity and no contact forces: a half kick
// (explicit Euler half step of Euler's equations in the body frame), the
// drift x += dt v and rotation q <- exp(omega dt / 2) q, and a second half
// kick whose rotational part takes four fixed-point sweeps in the new frame.
// The kernel runs those substeps in forward-mode dual numbers, one thread per
// particle and input: each of the 18 inputs (x, theta, v, omega, F, T), theta
// being a small world-frame rotation of the pose (q -> exp(theta / 2) q),
// gives one column of the Jacobian, and its product with the adjoint of the
// state after the call is that input's adjoint:
//   sigma(s_k) = (d s_{k+1} / d s_k)^T sigma(s_{k+1}),
//   dJ/d(F, T)_k = (d s_{k+1} / d(F, T)_k)^T sigma(s_{k+1}),
// with sigma ordered (x, theta, v, omega).  The second line becomes the
// objective weights of the step's momentum-exchange forces.  Contact forces
// are not differentiated.
#include <cmath>

#include "lbm_internal.h"

namespace mdlbm {
namespace {

constexpr int NIN = 18;  // inputs: x 0-2, theta 3-5, v 6-8, omega 9-11, F 12-14, T 15-17
constexpr int NT = 1;    // one tangent per thread

struct D {
    double v;
    double d[NT];
    __device__ D() = default;
    __device__ D(double x) : v(x)
    {
#pragma unroll
        for (int k = 0; k < NT; ++k) d[k] = 0.0;
    }
};
// x, with tangent 1 when it is the thread's input k
__device__ __forceinline__ D var(double x, int k, int seed)
{
    D r(x);
    r.d[0] = (k == seed) ? 1.0 : 0.0;
    return r;
}
__device__ __forceinline__ D operator+(const D& a, const D& b)
{
    D r;
    r.v = a.v + b.v;
#pragma unroll
    for (int k = 0; k < NT; ++k) r.d[k] = a.d[k] + b.d[k];
    return r;
}
__device__ __forceinline__ D operator-(const D& a, const D& b)
{
    D r;
    r.v = a.v - b.v;
#pragma unroll
    for (int k = 0; k < NT; ++k) r.d[k] = a.d[k] - b.d[k];
    return r;
}
__device__ __forceinline__ D operator*(const D& a, const D& b)
{
    D r;
    r.v = a.v * b.v;
#pragma unroll
    for (int k = 0; k < NT; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
    return r;
}
__device__ __forceinline__ D operator*(double s, const D& b)
{
    D r;
    r.v = s * b.v;
#pragma unroll
    for (int k = 0; k < NT; ++k) r.d[k] = s * b.d[k];
    return r;
}
__device__ __forceinline__ D operator/(const D& a, const D& b)
{
    D r;
    const double ib = 1.0 / b.v;
    r.v = a.v * ib;
#pragma unroll
    for (int k = 0; k < NT; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) * ib;
    return r;
}
__device__ __forceinline__ D dsqrt(const D& a)
{
    D r;
    r.v = sqrt(a.v);
    const double h = r.v > 0.0 ? 0.5 / r.v : 0.0;
#pragma unroll
    for (int k = 0; k < NT; ++k) r.d[k] = h * a.d[k];
    return r;
}
// f(a) with f(a.v) = fv and f'(a.v) = fp
__device__ __forceinline__ D chain(const D& a, double fv, double fp)
{
    D r;
    r.v = fv;
#pragma unroll
    for (int k = 0; k < NT; ++k) r.d[k] = fp * a.d[k];
    return r;
}

// c = a (x) b for quaternions (w, x, y, z)
__device__ __forceinline__ void qmul(const D a[4], const D b[4], D c[4])
{
    c[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    c[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    c[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    c[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}

__device__ __forceinline__ void rot(const D q[4], D R[9])
{
    const D w = q[0], x = q[1], y = q[2], z = q[3];
    const D one(1.0);
    R[0] = one - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = one - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = one - 2.0 * (x * x + y * y);
}

// Half kick of the rotation: body-frame Euler equations with `iters`
// fixed-point sweeps, as in the forward integrator.
__device__ __forceinline__ void spin_kick(const D q[4], D w[3], const D T[3], const double I[3],
                                          double h, int iters)
{
    D R[9];
    rot(q, R);
    D w0[3], Tb[3], wb[3];
    for (int i = 0; i < 3; ++i) {
        w0[i] = R[i] * w[0] + R[3 + i] * w[1] + R[6 + i] * w[2];
        Tb[i] = R[i] * T[0] + R[3 + i] * T[1] + R[6 + i] * T[2];
        wb[i] = w0[i];
    }
    for (int it = 0; it < iters; ++it) {
        const D Iw[3] = {I[0] * wb[0], I[1] * wb[1], I[2] * wb[2]};
        const D cc[3] = {wb[1] * Iw[2] - wb[2] * Iw[1], wb[2] * Iw[0] - wb[0] * Iw[2],
                         wb[0] * Iw[1] - wb[1] * Iw[0]};
        D nw[3];
        for (int a = 0; a < 3; ++a) nw[a] = w0[a] + (h / I[a]) * (Tb[a] - cc[a]);
        for (int a = 0; a < 3; ++a) wb[a] = nw[a];
    }
    for (int i = 0; i < 3; ++i) w[i] = R[3 * i] * wb[0] + R[3 * i + 1] * wb[1] + R[3 * i + 2] * wb[2];
}

__global__ __launch_bounds__(64) void k_dem_adjoint(int np, const double* mass, const double* volume,
                                                    const double* inertia, const double* pos,
                                                    const double* vel, const double* om,
                                                    const double* quat, const double* FT,
                                                    double g0, double g1, double g2, double rhof,
                                                    int n_sub, double dt, const double* sig1,
                                                    double* sig0, const double* wJ, double* wts)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= np * NIN) return;
    const int p = t / NIN, seed = t % NIN;
    D x[3], v[3], w[3], F[3], T[3], q[4];
    for (int a = 0; a < 3; ++a) {
        x[a] = var(pos[3 * p + a], a, seed);
        v[a] = var(vel[3 * p + a], 6 + a, seed);
        w[a] = var(om[3 * p + a], 9 + a, seed);
        F[a] = var(FT[6 * p + a], 12 + a, seed);
        T[a] = var(FT[6 * p + 3 + a], 15 + a, seed);
    }
    // q(theta) = exp(theta / 2) q: dq/dtheta_a = (0, e_a)/2 (x) q
    for (int c = 0; c < 4; ++c) q[c] = D(quat[4 * p + c]);
    {
        const double* qq = quat + 4 * p;
        const double e[3][4] = {{0, 1, 0, 0}, {0, 0, 1, 0}, {0, 0, 0, 1}};
        for (int a = 0; a < 3; ++a) {
            const double* u = e[a];
            const double r[4] = {u[0] * qq[0] - u[1] * qq[1] - u[2] * qq[2] - u[3] * qq[3],
                                 u[0] * qq[1] + u[1] * qq[0] + u[2] * qq[3] - u[3] * qq[2],
                                 u[0] * qq[2] - u[1] * qq[3] + u[2] * qq[0] + u[3] * qq[1],
                                 u[0] * qq[3] + u[1] * qq[2] - u[2] * qq[1] + u[3] * qq[0]};
            if (seed == 3 + a)
                for (int c = 0; c < 4; ++c) q[c].d[0] = 0.5 * r[c];
        }
    }
    const double m = mass[p];
    const double mrel = m - rhof * volume[p];
    const double gv[3] = {g0, g1, g2};
    const double I[3] = {inertia[3 * p], inertia[3 * p + 1], inertia[3 * p + 2]};
    const double h = 0.5 * dt;
    for (int s = 0; s < n_sub; ++s) {
        for (int a = 0; a < 3; ++a) v[a] = v[a] + (h / m) * (F[a] + D(mrel * gv[a]));
        spin_kick(q, w, T, I, h, 1);
        for (int a = 0; a < 3; ++a) x[a] = x[a] + dt * v[a];
        // dq = (cos(|w| dt / 2), sin(|w| dt / 2) w / |w|), smooth through w = 0
        const D ww = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
        D c, sn;
        if (sqrt(ww.v) * dt < 1e-4) {
            const D z = (0.25 * dt * dt) * ww;  // (|w| dt / 2)^2
            c = D(1.0) - 0.5 * z + (1.0 / 24.0) * (z * z);
            sn = (0.5 * dt) * (D(1.0) - (1.0 / 6.0) * z);
        } else {
            const D wn = dsqrt(ww);
            const double ang = 0.5 * wn.v * dt;
            c = chain(wn, cos(ang), -0.5 * dt * sin(ang));
            const D sa = chain(wn, sin(ang), 0.5 * dt * cos(ang));
            sn = sa / wn;
        }
        const D dq[4] = {c, sn * w[0], sn * w[1], sn * w[2]};
        D qn[4];
        qmul(dq, q, qn);
        const D nrm = dsqrt(qn[0] * qn[0] + qn[1] * qn[1] + qn[2] * qn[2] + qn[3] * qn[3]);
        for (int a = 0; a < 4; ++a) q[a] = qn[a] / nrm;
        for (int a = 0; a < 3; ++a) v[a] = v[a] + (h / m) * (F[a] + D(mrel * gv[a]));
        spin_kick(q, w, T, I, h, 4);
    }
    // this input's column of the Jacobian of the output state in (x, theta,
    // v, omega), the rotation tangent being 2 vec(dq (x) conj(q)), times the
    // adjoint of the output
    double col[12];
    for (int a = 0; a < 3; ++a) {
        col[a] = x[a].d[0];
        col[6 + a] = v[a].d[0];
        col[9 + a] = w[a].d[0];
    }
    {
        const double dw = q[0].d[0], dx = q[1].d[0], dy = q[2].d[0], dz = q[3].d[0];
        const double cw = q[0].v, cx_ = -q[1].v, cy_ = -q[2].v, cz_ = -q[3].v;
        col[3] = 2.0 * (dw * cx_ + dx * cw + dy * cz_ - dz * cy_);
        col[4] = 2.0 * (dw * cy_ - dx * cz_ + dy * cw + dz * cx_);
        col[5] = 2.0 * (dw * cz_ + dx * cy_ - dy * cx_ + dz * cw);
    }
    const double* s1 = sig1 + 12 * p;
    double acc = 0.0;
    for (int i = 0; i < 12; ++i) acc += col[i] * s1[i];
    if (seed < 12)
        sig0[12 * p + seed] = acc;
    else
        wts[6 * p + (seed - 12)] = wJ[6 * p + (seed - 12)] + acc;
}

}  // namespace

hipError_t launch_dem_adjoint(lbm_ctx* c, const TapeStep& ts, const lbm_particles* P,
                              const dem_params& prm, int n_sub, double dt, const double* sig1,
                              double* sig0, const double* wJ, double* wts)
{
    const int np = c->cfg.n_particles;
    if (np == 0) return hipSuccess;
    const double* st = ts.part;
    const double* quat = st + 9 * np + 3 * c->cfg.n_ctrl;
    const double* FT = quat + 4 * np;
    hipLaunchKernelGGL(k_dem_adjoint, dim3((np * NIN + 63) / 64), dim3(64), 0, c->stream, np, P->mass,
                       P->volume, P->inertia, st, st + 3 * np, st + 6 * np, quat, FT,
                       prm.gravity[0], prm.gravity[1], prm.gravity[2], prm.rho_f, n_sub, dt,
                       sig1, sig0, wJ, wts);
    return hipGetLastError();
}

}  // namespace mdlbm

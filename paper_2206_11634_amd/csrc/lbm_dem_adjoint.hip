// Adjoint of one dem_step call (differentiation form; not part of the paper).
//
// One call advances the DEM state by n_sub velocity-Verlet substeps under the
// hydrodynamic force and torque (F, T) of the lattice step, relative gravity
// and the contact forces of Sec. 2.1.1: per particle s = (x, q, v, omega)
// and the contact sum (force, torque) of the last substep, which the next
// call's first half kick uses; per contact record (pair or particle-wall) the
// tangential spring xi.  A substep is: half kick with the carried contact sum
// (explicit Euler half step of Euler's equations in the body frame), drift
// x += dt v and rotation q <- exp(omega dt / 2) q, the contacts at the new
// pose (metaball-wall and metaball-metaball: the Newton search for the
// contact point, the overlap, the spring-dashpot normal force, the spring
// and the Coulomb limit), and a second half kick with the new sum whose
// rotational part takes four fixed-point sweeps in the new frame.
//
// The kernel runs the call in forward-mode dual numbers, one thread per
// input: each of a particle's 24 inputs (x, theta, v, omega, F, T and the
// carried contact force and torque), theta being a small world-frame
// rotation of the pose (q -> exp(theta / 2) q), and each component of the
// springs of its contact records, gives one column of the Jacobian, and its
// product with the adjoint of the state after the call is that input's
// adjoint:
//   sigma(s_k) = (d s_{k+1} / d s_k)^T sigma(s_{k+1}),
//   dJ/d(F, T)_k = (d s_{k+1} / d(F, T)_k)^T sigma(s_{k+1}).
// A thread simulates the cluster of its particle: the particles linked to it
// through pairs that are broad-phase candidates of the call (only those can
// touch it within the call), at most kAdjCluster of them.  The contact point
// of a pair is the root of grad(M_i + M_j) = 0: the iteration runs on values
// from the recorded warm start, as in dem_step, and one more Newton step in
// dual numbers from the converged point gives its derivative by the
// implicit function theorem (the step's tangent is -H^{-1} dg, g = 0 there);
// the in-plane point of a wall contact likewise.  Branches (contact on or
// off, the clamp of the normal force, the Coulomb limit) follow the values,
// as in dem_step.
#include <cmath>

#include "lbm_internal.h"

namespace mdlbm {
namespace {

constexpr int kHist = 8;   // active, xi[3], warm start[3], pad
constexpr int NPIN = 24;   // particle inputs: x 0-2, theta 3-5, v 6-8, omega 9-11, F 12-14,
                           // T 15-17, carried contact force 18-20 and torque 21-23
constexpr int NSEED = NPIN + 3 * kPairSlots + 3 * 6;
constexpr int kMaxPairs = kAdjCluster * (kAdjCluster - 1) / 2;

struct D {
    double v, d;
    __device__ D() = default;
    __device__ D(double x) : v(x), d(0.0) {}
    __device__ D(double x, double t) : v(x), d(t) {}
};
__device__ __forceinline__ D var(double x, bool seeded) { return D(x, seeded ? 1.0 : 0.0); }
__device__ __forceinline__ D operator+(const D& a, const D& b) { return D(a.v + b.v, a.d + b.d); }
__device__ __forceinline__ D operator-(const D& a, const D& b) { return D(a.v - b.v, a.d - b.d); }
__device__ __forceinline__ D operator-(const D& a) { return D(-a.v, -a.d); }
__device__ __forceinline__ D operator*(const D& a, const D& b)
{
    return D(a.v * b.v, a.d * b.v + a.v * b.d);
}
__device__ __forceinline__ D operator*(double s, const D& b) { return D(s * b.v, s * b.d); }
__device__ __forceinline__ D operator/(const D& a, const D& b)
{
    const double ib = 1.0 / b.v, r = a.v * ib;
    return D(r, (a.d - r * b.d) * ib);
}
__device__ __forceinline__ D dsqrt(const D& a)
{
    const double r = sqrt(a.v);
    return D(r, r > 0.0 ? 0.5 * a.d / r : 0.0);
}
// f(a) with f(a.v) = fv and f'(a.v) = fp
__device__ __forceinline__ D chain(const D& a, double fv, double fp) { return D(fv, fp * a.d); }
__device__ __forceinline__ D dot3(const D a[3], const D b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
__device__ __forceinline__ void cross3(const D a[3], const D b[3], D c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
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
__device__ void spin_kick(const D q[4], D w[3], const D T[3], const double I[3], double h, int iters)
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
        D cc[3];
        cross3(wb, Iw, cc);
        D nw[3];
        for (int a = 0; a < 3; ++a) nw[a] = w0[a] + (h / I[a]) * (Tb[a] - cc[a]);
        for (int a = 0; a < 3; ++a) wb[a] = nw[a];
    }
    for (int i = 0; i < 3; ++i) w[i] = R[3 * i] * wb[0] + R[3 * i + 1] * wb[1] + R[3 * i + 2] * wb[2];
}

// What the kernel reads of the particles: shapes and rigid-body constants.
struct Shapes {
    const int32_t* off;
    const double* body_pts;
    const double* K;
    const double* rs;
    const double* mass;
    const double* volume;
    const double* inertia;
};

// DEM state of one taped step (the start of the call that followed it).
struct DemTape {
    const double* pos;
    const double* vel;
    const double* om;
    const double* quat;
    const double* FT;
    const double* hist;     // [np][kPairSlots][kHist]
    const int32_t* key;     // [np][kPairSlots]: partner + 1, 0 free
    const double* hist_w;   // [np][6][kHist]
    const double* fc;       // [np][6]
};

struct Consts {
    double kn, etan, kt, etat, mu, ctol, ntol;
    int niter;
    double g[3];
    double rhof;
};

__device__ double body_reach(const Shapes& S, int p)
{
    double sk = 0.0, r = 0.0;
    for (int i = S.off[p]; i < S.off[p + 1]; ++i) {
        const double* b = S.body_pts + 3 * (int64_t)i;
        r = fmax(r, sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]));
        sk += S.K[i];
    }
    return r + sqrt(sk);
}

// The broad-phase test of dem_step for pair (i, j) at the start of the call.
__device__ bool candidate(const Shapes& S, const DemTape& s, int i, int j, double T, const Geom& g)
{
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        double d = s.pos[3 * j + a] - s.pos[3 * i + a];
        if (g.per[a]) {
            const double L = g.n[a];
            if (d > 0.5 * L) d -= L;
            else if (d < -0.5 * L) d += L;
        }
        d2 += d * d;
    }
    const double* vi = s.vel + 3 * i;
    const double* vj = s.vel + 3 * j;
    const double skin = (sqrt(vi[0] * vi[0] + vi[1] * vi[1] + vi[2] * vi[2]) +
                         sqrt(vj[0] * vj[0] + vj[1] * vj[1] + vj[2] * vj[2])) * T + 0.5;
    const double thr = body_reach(S, i) + body_reach(S, j) + S.rs[i] + S.rs[j] + skin;
    return sqrt(d2) <= thr;
}

// One particle of the cluster.
struct Body {
    int gi;               // global index
    int a0, n;            // control points
    D x[3], q[4], v[3], w[3], F[3], T[3], fc[6];
    D R[9];
    double m, mrel, I[3], rs, reach;
};

// M, grad M and the Hessian of body b (world points x + R b_i, shifted by
// sh) at X, in dual numbers.
__device__ void mb_d2(const Shapes& S, const Body& b, const double sh[3], const D X[3], D& M,
                      D g[3], D H[9])
{
    M = D(0.0);
    for (int a = 0; a < 3; ++a) g[a] = D(0.0);
    for (int a = 0; a < 9; ++a) H[a] = D(0.0);
    for (int i = 0; i < b.n; ++i) {
        const double* bp = S.body_pts + 3 * (int64_t)(b.a0 + i);
        const double K = S.K[b.a0 + i];
        D r[3];
        for (int a = 0; a < 3; ++a) {
            const D wp = b.x[a] + (b.R[3 * a] * D(bp[0]) + b.R[3 * a + 1] * D(bp[1]) +
                                   b.R[3 * a + 2] * D(bp[2]));
            r[a] = X[a] - (wp + D(sh[a]));
        }
        const D r2 = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
        const D i2 = D(1.0) / r2, i4 = i2 * i2, i6 = i4 * i2;
        M = M + K * i2;
        for (int a = 0; a < 3; ++a) {
            g[a] = g[a] + (-2.0 * K) * (r[a] * i4);
            for (int c = 0; c < 3; ++c)
                H[3 * a + c] = H[3 * a + c] + K * (8.0 * (r[a] * r[c] * i6) - (a == c ? 2.0 * i4 : D(0.0)));
        }
    }
}

// The same on values only (the Newton iterations).
__device__ void mb_d2v(const Shapes& S, const Body& b, const double sh[3], const double X[3],
                       double& M, double g[3], double H[9])
{
    M = 0.0;
    for (int a = 0; a < 3; ++a) g[a] = 0.0;
    for (int a = 0; a < 9; ++a) H[a] = 0.0;
    for (int i = 0; i < b.n; ++i) {
        const double* bp = S.body_pts + 3 * (int64_t)(b.a0 + i);
        const double K = S.K[b.a0 + i];
        double r[3];
        for (int a = 0; a < 3; ++a) {
            const double wp = b.x[a].v + (b.R[3 * a].v * bp[0] + b.R[3 * a + 1].v * bp[1] +
                                          b.R[3 * a + 2].v * bp[2]);
            r[a] = X[a] - (wp + sh[a]);
        }
        const double r2 = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
        const double i2 = 1.0 / r2, i4 = i2 * i2, i6 = i4 * i2;
        M += K * i2;
        for (int a = 0; a < 3; ++a) {
            g[a] += -2.0 * K * r[a] * i4;
            for (int c = 0; c < 3; ++c)
                H[3 * a + c] += K * (8.0 * r[a] * r[c] * i6 - (a == c ? 2.0 * i4 : 0.0));
        }
    }
}

// World control point u of body b (values).
__device__ void world_pt(const Shapes& S, const Body& b, int u, double out[3])
{
    const double* bp = S.body_pts + 3 * (int64_t)(b.a0 + u);
    for (int a = 0; a < 3; ++a)
        out[a] = b.x[a].v + (b.R[3 * a].v * bp[0] + b.R[3 * a + 1].v * bp[1] + b.R[3 * a + 2].v * bp[2]);
}

template <class T>
__device__ bool solve3(const T H[9], const T g[3], T dx[3])
{
    T c[9];
    c[0] = H[4] * H[8] - H[5] * H[7];
    c[1] = H[2] * H[7] - H[1] * H[8];
    c[2] = H[1] * H[5] - H[2] * H[4];
    c[3] = H[5] * H[6] - H[3] * H[8];
    c[4] = H[0] * H[8] - H[2] * H[6];
    c[5] = H[2] * H[3] - H[0] * H[5];
    c[6] = H[3] * H[7] - H[4] * H[6];
    c[7] = H[1] * H[6] - H[0] * H[7];
    c[8] = H[0] * H[4] - H[1] * H[3];
    const T det = H[0] * c[0] + H[1] * c[3] + H[2] * c[6];
    double dv;
    if constexpr (sizeof(T) == sizeof(double)) dv = det; else dv = det.v;
    if (!(fabs(dv) > 0.0) || !isfinite(dv)) return false;
    for (int i = 0; i < 3; ++i) dx[i] = -((c[3 * i] * g[0] + c[3 * i + 1] * g[1] + c[3 * i + 2] * g[2]) / det);
    return true;
}

// A contact record: the spring (dual) and the values that steer the search.
struct Rec {
    double active, warm[3];
    D xi[3];
    __device__ void clear()
    {
        active = 0.0;
        for (int a = 0; a < 3; ++a) {
            warm[a] = 0.0;
            xi[a] = D(0.0);
        }
    }
};

// Spring-dashpot normal force (clamped at zero) and the tangential spring
// with the Coulomb limit, as dem_step evaluates them; updates the spring.
__device__ void contact_force(const Consts& c, const D& delta, const D n[3], const D vrel[3],
                              double dt, Rec& h, D Fi[3])
{
    const D vn = dot3(vrel, n);
    D Fn = c.kn * delta - c.etan * vn;
    if (Fn.v < 0.0) Fn = D(0.0);
    D vt[3], xi[3], Ft[3];
    for (int a = 0; a < 3; ++a) vt[a] = vrel[a] - vn * n[a];
    const D xin = h.xi[0] * n[0] + h.xi[1] * n[1] + h.xi[2] * n[2];
    for (int a = 0; a < 3; ++a) xi[a] = h.xi[a] - xin * n[a] + dt * vt[a];
    for (int a = 0; a < 3; ++a) Ft[a] = (-c.kt) * xi[a] - c.etat * vt[a];
    const D ftn = dsqrt(dot3(Ft, Ft));
    if (ftn.v > c.mu * Fn.v && ftn.v > 0.0) {
        const D s = (c.mu * Fn) / ftn;
        for (int a = 0; a < 3; ++a) {
            Ft[a] = s * Ft[a];
            xi[a] = (-1.0 / c.kt) * (Ft[a] + c.etat * vt[a]);
        }
    }
    for (int a = 0; a < 3; ++a) {
        h.xi[a] = xi[a];
        Fi[a] = Fn * n[a] + Ft[a];
    }
}

__device__ void half_kick(Body& b, const Consts& c, double h, bool implicit)
{
    D T[3];
    for (int a = 0; a < 3; ++a) {
        b.v[a] = b.v[a] + (h / b.m) * (b.F[a] + D(b.mrel * c.g[a]) + b.fc[a]);
        T[a] = b.T[a] + b.fc[3 + a];
    }
    spin_kick(b.q, b.w, T, b.I, h, implicit ? 4 : 1);
}

__device__ void drift_rotate(Body& b, double dt, const Geom& g)
{
    for (int a = 0; a < 3; ++a) {
        D x = b.x[a] + dt * b.v[a];
        if (g.per[a]) {
            if (x.v >= (double)g.n[a]) x.v -= g.n[a];
            else if (x.v < 0.0) x.v += g.n[a];
        }
        b.x[a] = x;
    }
    // dq = (cos(|w| dt / 2), sin(|w| dt / 2) w / |w|), smooth through w = 0
    const D ww = b.w[0] * b.w[0] + b.w[1] * b.w[1] + b.w[2] * b.w[2];
    D cs, sn;
    if (sqrt(ww.v) * dt < 1e-4) {
        const D z = (0.25 * dt * dt) * ww;
        cs = D(1.0) - 0.5 * z + (1.0 / 24.0) * (z * z);
        sn = (0.5 * dt) * (D(1.0) - (1.0 / 6.0) * z);
    } else {
        const D wn = dsqrt(ww);
        const double ang = 0.5 * wn.v * dt;
        cs = chain(wn, cos(ang), -0.5 * dt * sin(ang));
        const D sa = chain(wn, sin(ang), 0.5 * dt * cos(ang));
        sn = sa / wn;
    }
    const D dq[4] = {cs, sn * b.w[0], sn * b.w[1], sn * b.w[2]};
    D qn[4];
    qmul(dq, b.q, qn);
    const D nrm = dsqrt(qn[0] * qn[0] + qn[1] * qn[1] + qn[2] * qn[2] + qn[3] * qn[3]);
    for (int a = 0; a < 4; ++a) b.q[a] = qn[a] / nrm;
    rot(b.q, b.R);
}

// Metaball-wall contact of body b with wall (ax, side), as dem_step.
__device__ void wall_item(const Shapes& S, Body& b, int ax, int side, Rec& h, const Consts& c,
                          double dt, const Geom& g)
{
    const double plane = side ? g.n[ax] - 0.5 : -0.5, sgn = side ? -1.0 : 1.0;
    if (sgn * (b.x[ax].v - plane) > b.reach + b.rs) {
        h.clear();
        return;
    }
    const int t1 = (ax + 1) % 3, t2 = (ax + 2) % 3;
    const double z3[3] = {0.0, 0.0, 0.0};
    double x[3];
    if (h.active != 0.0) {
        for (int a = 0; a < 3; ++a) x[a] = b.x[a].v + h.warm[a];
    } else {
        double best = INFINITY;
        for (int u = 0; u < b.n; ++u) {
            double p[3];
            world_pt(S, b, u, p);
            const double dd = fabs(p[ax] - plane);
            if (dd < best) {
                best = dd;
                for (int a = 0; a < 3; ++a) x[a] = p[a];
            }
        }
    }
    x[ax] = plane;
    bool conv = false;
    for (int it = 0; it < c.niter; ++it) {
        double M, gr[3], H[9];
        mb_d2v(S, b, z3, x, M, gr, H);
        const double h11 = H[3 * t1 + t1], h12 = H[3 * t1 + t2], h22 = H[3 * t2 + t2];
        const double det = h11 * h22 - h12 * h12;
        if (!(fabs(det) > 0.0) || !isfinite(det)) break;
        const double d1 = -(h22 * gr[t1] - h12 * gr[t2]) / det;
        const double d2 = -(-h12 * gr[t1] + h11 * gr[t2]) / det;
        x[t1] += d1;
        x[t2] += d2;
        if (sqrt(d1 * d1 + d2 * d2) < c.ntol) {
            conv = true;
            break;
        }
    }
    if (!conv) {
        h.clear();
        return;
    }
    // one Newton step in dual numbers from the converged point
    D X[3] = {D(x[0]), D(x[1]), D(x[2])};
    D M, gr[3], H[9];
    mb_d2(S, b, z3, X, M, gr, H);
    {
        const D h11 = H[3 * t1 + t1], h12 = H[3 * t1 + t2], h22 = H[3 * t2 + t2];
        const D det = h11 * h22 - h12 * h12;
        const D d1 = -((h22 * gr[t1] - h12 * gr[t2]) / det);
        const D d2 = -((-h12 * gr[t1] + h11 * gr[t2]) / det);
        X[t1] = D(x[t1], d1.d);
        X[t2] = D(x[t2], d2.d);
    }
    mb_d2(S, b, z3, X, M, gr, H);
    if (!(sgn * gr[ax].v > 0.0)) {
        h.clear();
        return;
    }
    h.active = 1.0;
    for (int a = 0; a < 3; ++a) h.warm[a] = x[a] - b.x[a].v;
    const D qR = (D(1.0) - M) / dot3(gr, gr);
    const D delta = D(b.rs) - sgn * (qR * gr[ax]);
    if (delta.v <= 0.0) {
        for (int a = 0; a < 3; ++a) h.xi[a] = D(0.0);
        return;
    }
    D n[3] = {D(0.0), D(0.0), D(0.0)}, xcp[3], ra[3];
    n[ax] = D(sgn);
    for (int a = 0; a < 3; ++a) {
        xcp[a] = X[a] - 0.5 * (delta * n[a]);
        ra[a] = xcp[a] - b.x[a];
    }
    D ca[3], vrel[3], Fi[3], tq[3];
    cross3(b.w, ra, ca);
    for (int a = 0; a < 3; ++a) vrel[a] = b.v[a] + ca[a];
    contact_force(c, delta, n, vrel, dt, h, Fi);
    cross3(ra, Fi, tq);
    for (int a = 0; a < 3; ++a) {
        b.fc[a] = b.fc[a] + Fi[a];
        b.fc[3 + a] = b.fc[3 + a] + tq[a];
    }
}

// Metaball-metaball contact of the pair (A, B), A of lower index, as dem_step.
__device__ void pair_item(const Shapes& S, Body& A, Body& B, Rec& h, const Consts& c, double dt,
                          const Geom& g)
{
    double sh[3], dv[3];
    for (int a = 0; a < 3; ++a) {
        const double d = B.x[a].v - A.x[a].v;
        sh[a] = 0.0;
        if (g.per[a]) {
            const double L = g.n[a];
            if (d > 0.5 * L) sh[a] = -L;
            else if (d < -0.5 * L) sh[a] = L;
        }
        dv[a] = d + sh[a];
    }
    if (sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]) > A.reach + B.reach + A.rs + B.rs) {
        h.clear();
        return;
    }
    const double z3[3] = {0.0, 0.0, 0.0};
    double x[3];
    if (h.active != 0.0) {
        for (int a = 0; a < 3; ++a) x[a] = A.x[a].v + h.warm[a];
    } else {
        double best = INFINITY;
        for (int u = 0; u < A.n; ++u)
            for (int w = 0; w < B.n; ++w) {
                double pa[3], pb[3], d2 = 0.0;
                world_pt(S, A, u, pa);
                world_pt(S, B, w, pb);
                for (int a = 0; a < 3; ++a) d2 += (pa[a] - (pb[a] + sh[a])) * (pa[a] - (pb[a] + sh[a]));
                if (d2 < best) {
                    best = d2;
                    for (int a = 0; a < 3; ++a) x[a] = 0.5 * (pa[a] + pb[a] + sh[a]);
                }
            }
    }
    bool conv = false;
    for (int it = 0; it < c.niter; ++it) {
        double MA, MB, gA[3], gB[3], HA[9], HB[9], gg[3], H[9], dx[3];
        mb_d2v(S, A, z3, x, MA, gA, HA);
        mb_d2v(S, B, sh, x, MB, gB, HB);
        for (int a = 0; a < 3; ++a) gg[a] = gA[a] + gB[a];
        for (int a = 0; a < 9; ++a) H[a] = HA[a] + HB[a];
        if (!solve3(H, gg, dx)) break;
        for (int a = 0; a < 3; ++a) x[a] += dx[a];
        if (sqrt(dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2]) < c.ntol) {
            conv = true;
            break;
        }
    }
    if (!conv) {
        h.clear();
        return;
    }
    // one Newton step in dual numbers from the converged point
    D X[3] = {D(x[0]), D(x[1]), D(x[2])};
    D MA, MB, gA[3], gB[3], HA[9], HB[9];
    {
        mb_d2(S, A, z3, X, MA, gA, HA);
        mb_d2(S, B, sh, X, MB, gB, HB);
        D gg[3], H[9], dx[3];
        for (int a = 0; a < 3; ++a) gg[a] = gA[a] + gB[a];
        for (int a = 0; a < 9; ++a) H[a] = HA[a] + HB[a];
        if (solve3(H, gg, dx))
            for (int a = 0; a < 3; ++a) X[a] = D(x[a], dx[a].d);
    }
    mb_d2(S, A, z3, X, MA, gA, HA);
    mb_d2(S, B, sh, X, MB, gB, HB);
    if (!(MA.v > c.ctol && MB.v > c.ctol)) {
        h.clear();
        return;
    }
    const D qA = (D(1.0) - MA) / dot3(gA, gA), qB = (D(1.0) - MB) / dot3(gB, gB);
    D xa[3], dd[3], n[3];
    for (int a = 0; a < 3; ++a) {
        xa[a] = X[a] + qA * gA[a];
        dd[a] = xa[a] - (X[a] + qB * gB[a]);
        n[a] = gA[a] - gB[a];
    }
    const D un = dsqrt(dot3(n, n));
    if (!(un.v > 0.0)) {
        h.clear();
        return;
    }
    for (int a = 0; a < 3; ++a) n[a] = n[a] / un;
    const D delta = D(A.rs + B.rs) - dot3(dd, n);
    if (!(delta.v <= 2.0 * (A.rs + B.rs))) {
        h.clear();
        return;
    }
    h.active = 1.0;
    for (int a = 0; a < 3; ++a) h.warm[a] = x[a] - A.x[a].v;
    if (delta.v <= 0.0) {
        for (int a = 0; a < 3; ++a) h.xi[a] = D(0.0);
        return;
    }
    D xcp[3], ra[3], rb[3];
    for (int a = 0; a < 3; ++a) {
        xcp[a] = xa[a] - (D(A.rs) - 0.5 * delta) * n[a];
        ra[a] = xcp[a] - A.x[a];
        rb[a] = xcp[a] - (B.x[a] + D(sh[a]));
    }
    D ca[3], cb[3], vrel[3], Fi[3], tq[3];
    cross3(A.w, ra, ca);
    cross3(B.w, rb, cb);
    for (int a = 0; a < 3; ++a) vrel[a] = (A.v[a] + ca[a]) - (B.v[a] + cb[a]);
    contact_force(c, delta, n, vrel, dt, h, Fi);
    for (int a = 0; a < 3; ++a) {
        A.fc[a] = A.fc[a] + Fi[a];
        B.fc[a] = B.fc[a] - Fi[a];
    }
    cross3(ra, Fi, tq);
    for (int a = 0; a < 3; ++a) A.fc[3 + a] = A.fc[3 + a] + tq[a];
    cross3(rb, Fi, tq);
    for (int a = 0; a < 3; ++a) B.fc[3 + a] = B.fc[3 + a] - tq[a];
}

__device__ int find_slot(const int32_t* key, int i, int j)
{
    for (int s = 0; s < kPairSlots; ++s)
        if (key[(int64_t)i * kPairSlots + s] == j + 1) return s;
    return -1;
}

// One thread per (particle p, input).  sig: [np][12] state adjoints (x,
// theta, v, omega); sc: [np][kAdjContact] contact-state adjoints (carried
// force and torque, then the springs of the kPairSlots pair records and of
// the six wall records); key_next: the pair records' keys after the call.
__global__ __launch_bounds__(64) void k_dem_adjoint(int np, Shapes S, DemTape st,
                                                    const int32_t* key_next, Consts c, Geom g,
                                                    int n_sub, double dt, const double* sig1,
                                                    const double* sc1, double* sig0, double* sc0,
                                                    const double* wJ, double* wts, uint32_t* err)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= np * NSEED) return;
    const int p = t / NSEED, seed = t % NSEED;
    const double Tcall = (double)n_sub * dt;
    int pslot = -1, pwall = -1, pa = 0;
    if (seed >= NPIN && seed < NPIN + 3 * kPairSlots) {
        pslot = (seed - NPIN) / 3;
        pa = (seed - NPIN) % 3;
        const int key = st.key[(int64_t)p * kPairSlots + pslot];
        // a free record, or one that the call releases (its partner no longer
        // a candidate), does not enter the call
        if (key == 0 || key - 1 >= np || !candidate(S, st, p, key - 1, Tcall, g)) {
            sc0[(int64_t)p * kAdjContact + 6 + 3 * pslot + pa] = 0.0;
            return;
        }
    } else if (seed >= NPIN + 3 * kPairSlots) {
        pwall = (seed - NPIN - 3 * kPairSlots) / 3;
        pa = (seed - NPIN - 3 * kPairSlots) % 3;
    }

    // the cluster: particles linked to p through candidate pairs
    int mem[kAdjCluster];
    int nm = 1;
    mem[0] = p;
    for (int hd = 0; hd < nm; ++hd) {
        for (int j = 0; j < np; ++j) {
            bool in = false;
            for (int k = 0; k < nm; ++k) in |= mem[k] == j;
            if (in || !candidate(S, st, mem[hd], j, Tcall, g)) continue;
            if (nm == kAdjCluster) {
                atomicOr(err, 1u);
                return;
            }
            mem[nm++] = j;
        }
    }
    for (int a = 1; a < nm; ++a)  // ascending global index
        for (int b = a; b > 0 && mem[b - 1] > mem[b]; --b) {
            const int tmp = mem[b];
            mem[b] = mem[b - 1];
            mem[b - 1] = tmp;
        }

    Body B[kAdjCluster];
    for (int m = 0; m < nm; ++m) {
        Body& b = B[m];
        const int gi = mem[m];
        const bool me = gi == p;
        b.gi = gi;
        b.a0 = S.off[gi];
        b.n = S.off[gi + 1] - b.a0;
        b.m = S.mass[gi];
        b.mrel = b.m - c.rhof * S.volume[gi];
        for (int a = 0; a < 3; ++a) b.I[a] = S.inertia[3 * gi + a];
        b.rs = S.rs[gi];
        b.reach = body_reach(S, gi);
        for (int a = 0; a < 3; ++a) {
            b.x[a] = var(st.pos[3 * gi + a], me && seed == a);
            b.v[a] = var(st.vel[3 * gi + a], me && seed == 6 + a);
            b.w[a] = var(st.om[3 * gi + a], me && seed == 9 + a);
            b.F[a] = var(st.FT[6 * gi + a], me && seed == 12 + a);
            b.T[a] = var(st.FT[6 * gi + 3 + a], me && seed == 15 + a);
        }
        for (int k = 0; k < 6; ++k) b.fc[k] = var(st.fc[6 * gi + k], me && seed == 18 + k);
        // q(theta) = exp(theta / 2) q: dq/dtheta_a = (0, e_a)/2 (x) q
        const double* qq = st.quat + 4 * gi;
        for (int k = 0; k < 4; ++k) b.q[k] = D(qq[k]);
        if (me && seed >= 3 && seed < 6) {
            const int a = seed - 3;
            double u[4] = {0.0, 0.0, 0.0, 0.0};
            u[1 + a] = 1.0;
            const double r[4] = {u[0] * qq[0] - u[1] * qq[1] - u[2] * qq[2] - u[3] * qq[3],
                                 u[0] * qq[1] + u[1] * qq[0] + u[2] * qq[3] - u[3] * qq[2],
                                 u[0] * qq[2] - u[1] * qq[3] + u[2] * qq[0] + u[3] * qq[1],
                                 u[0] * qq[3] + u[1] * qq[2] - u[2] * qq[1] + u[3] * qq[0]};
            for (int k = 0; k < 4; ++k) b.q[k].d = 0.5 * r[k];
        }
        rot(b.q, B[m].R);
    }
    // contact records: the candidate pairs of the cluster (as the call keeps
    // or claims them) and the walls of every member
    int pi_[kMaxPairs], pj_[kMaxPairs];
    Rec pr[kMaxPairs];
    int npair = 0;
    for (int u = 0; u < nm; ++u)
        for (int w = u + 1; w < nm; ++w) {
            const int gi = mem[u], gj = mem[w];
            if (!candidate(S, st, gi, gj, Tcall, g)) continue;
            Rec& h = pr[npair];
            h.clear();
            const int s = find_slot(st.key, gi, gj);
            if (s >= 0) {
                const double* src = st.hist + ((int64_t)gi * kPairSlots + s) * kHist;
                h.active = src[0];
                for (int a = 0; a < 3; ++a) {
                    h.xi[a] = var(src[1 + a], gi == p && s == pslot && a == pa);
                    h.warm[a] = src[4 + a];
                }
            }
            pi_[npair] = u;
            pj_[npair] = w;
            ++npair;
        }
    Rec wr[kAdjCluster][6];
    for (int m = 0; m < nm; ++m)
        for (int k = 0; k < 6; ++k) {
            Rec& h = wr[m][k];
            const double* src = st.hist_w + ((int64_t)mem[m] * 6 + k) * kHist;
            h.active = src[0];
            for (int a = 0; a < 3; ++a) {
                h.xi[a] = var(src[1 + a], mem[m] == p && k == pwall && a == pa);
                h.warm[a] = src[4 + a];
            }
        }

    // the call's substeps
    for (int s = 0; s < n_sub; ++s) {
        for (int m = 0; m < nm; ++m) {
            half_kick(B[m], c, 0.5 * dt, false);
            for (int k = 0; k < 6; ++k) B[m].fc[k] = D(0.0);
            drift_rotate(B[m], dt, g);
        }
        for (int m = 0; m < nm; ++m)
            for (int ax = 0; ax < 3; ++ax) {
                if (g.per[ax]) continue;
                for (int side = 0; side < 2; ++side)
                    wall_item(S, B[m], ax, side, wr[m][2 * ax + side], c, dt, g);
            }
        for (int k = 0; k < npair; ++k) pair_item(S, B[pi_[k]], B[pj_[k]], pr[k], c, dt, g);
        for (int m = 0; m < nm; ++m) half_kick(B[m], c, 0.5 * dt, true);
    }

    // this input's column of the Jacobian times the adjoint of the output
    double acc = 0.0;
    for (int m = 0; m < nm; ++m) {
        const Body& b = B[m];
        const double* s1 = sig1 + 12 * (int64_t)b.gi;
        for (int a = 0; a < 3; ++a)
            acc += b.x[a].d * s1[a] + b.v[a].d * s1[6 + a] + b.w[a].d * s1[9 + a];
        {
            // rotation tangent 2 vec(dq (x) conj(q))
            const double dw = b.q[0].d, dx = b.q[1].d, dy = b.q[2].d, dz = b.q[3].d;
            const double cw = b.q[0].v, cx_ = -b.q[1].v, cy_ = -b.q[2].v, cz_ = -b.q[3].v;
            acc += 2.0 * (dw * cx_ + dx * cw + dy * cz_ - dz * cy_) * s1[3];
            acc += 2.0 * (dw * cy_ - dx * cz_ + dy * cw + dz * cx_) * s1[4];
            acc += 2.0 * (dw * cz_ + dx * cy_ - dy * cx_ + dz * cw) * s1[5];
        }
        const double* c1 = sc1 + (int64_t)kAdjContact * b.gi;
        for (int k = 0; k < 6; ++k) acc += b.fc[k].d * c1[k];
        for (int k = 0; k < 6; ++k)
            for (int a = 0; a < 3; ++a) acc += wr[m][k].xi[a].d * c1[6 + 3 * kPairSlots + 3 * k + a];
    }
    for (int k = 0; k < npair; ++k) {
        const int gi = mem[pi_[k]], gj = mem[pj_[k]];
        const int s = find_slot(key_next, gi, gj);
        if (s < 0) continue;
        const double* c1 = sc1 + (int64_t)kAdjContact * gi + 6 + 3 * s;
        for (int a = 0; a < 3; ++a) acc += pr[k].xi[a].d * c1[a];
    }
    if (seed < 12)
        sig0[12 * (int64_t)p + seed] = acc;
    else if (seed < 18)
        wts[6 * (int64_t)p + (seed - 12)] = wJ[6 * (int64_t)p + (seed - 12)] + acc;
    else if (seed < NPIN)
        sc0[(int64_t)kAdjContact * p + (seed - 18)] = acc;
    else if (pslot >= 0)
        sc0[(int64_t)kAdjContact * p + 6 + 3 * pslot + pa] = acc;
    else
        sc0[(int64_t)kAdjContact * p + 6 + 3 * kPairSlots + 3 * pwall + pa] = acc;
}

}  // namespace

hipError_t launch_dem_adjoint(lbm_ctx* c, const TapeStep& ts, const int32_t* key_next,
                              const lbm_particles* P, const dem_params& prm, int n_sub, double dt,
                              const double* sig1, const double* sc1, double* sig0, double* sc0,
                              const double* wJ, double* wts, uint32_t* err)
{
    const int np = c->cfg.n_particles;
    if (np == 0) return hipSuccess;
    Shapes S{P->ctrl_off, P->body_pts, P->K, P->rs, P->mass, P->volume, P->inertia};
    const double* part = ts.part;
    const double* quat = part + 9 * np + 3 * c->cfg.n_ctrl;
    DemTape st{part,           part + 3 * np,      part + 6 * np, quat, quat + 4 * np,
               ts.dem,         ts.dem_key,         ts.dem + (int64_t)np * kPairSlots * kHist,
               ts.dem + (int64_t)np * kPairSlots * kHist + (int64_t)np * 6 * kHist};
    Consts k;
    k.kn = prm.kn;
    k.etan = prm.eta_n;
    k.kt = prm.kt;
    k.etat = prm.eta_t;
    k.mu = prm.mu_s;
    k.ctol = prm.ctol;
    k.ntol = prm.newton_tol;
    k.niter = prm.newton_iter;
    for (int a = 0; a < 3; ++a) k.g[a] = prm.gravity[a];
    k.rhof = prm.rho_f;
    const int64_t n = (int64_t)np * NSEED;
    hipLaunchKernelGGL(k_dem_adjoint, dim3((uint32_t)((n + 63) / 64)), dim3(64), 0, c->stream, np, S,
                       st, key_next, k, c->geom, n_sub, dt, sig1, sc1, sig0, sc0, wJ, wts, err);
    return hipGetLastError();
}

}  // namespace mdlbm

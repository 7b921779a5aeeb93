// Metaball DEM of libmdlbm in FP64 on the GPU (Sec. 2.1, with the
// sub-cycling of Sec. 2.3.4): velocity Verlet for translation, Euler's
// equations in the principal body frame for rotation, linear spring-dashpot
// normal force and Coulomb-limited tangential spring, metaball-metaball
// contacts by Newton-Raphson on grad(M_i + M_j) = 0 (Eqs. opt, grad, cp, k0,
// contactprop) and metaball-wall contacts by Newton on the in-plane gradient
// (Eqs. metawall, metawallcp, k, contactprop2).
//
// One substep = three launches: half kick + drift + rotation + reset of the
// contact sums (one thread per particle), contacts (one thread per pair i < j
// and one per particle-wall pair, FP64 atomics into the sums), second half
// kick.
// The work is latency-bound (a few thousand particles at most), not HBM-bound.
#include <mutex>

#include "lbm_internal.h"

namespace mdlbm {
namespace {

constexpr int kHist = 8;  // active, xi[3], warm start[3], pad
constexpr int kMaxPts = 64;

struct DemP {
    double kn, etan, kt, etat, mu, ctol, ntol;
    int niter;
    double g[3];
    double rhof;
};

__device__ __forceinline__ void cross3(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ __forceinline__ double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

__device__ void rotmat(const double* q, double R[9])
{
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z);
    R[1] = 2 * (x * y - w * z);
    R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);
    R[4] = 1 - 2 * (x * x + z * z);
    R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);
    R[7] = 2 * (y * z + w * x);
    R[8] = 1 - 2 * (x * x + y * y);
}

// M, grad M and the Hessian of a metaball with n points at X; pts may be
// shifted by `sh` (a periodic image).
__device__ void mb_d2(const double* pts, const double* K, int n, const double sh[3],
                      const double X[3], double& M, double g[3], double H[9])
{
    M = 0.0;
    for (int a = 0; a < 3; ++a) g[a] = 0.0;
    for (int a = 0; a < 9; ++a) H[a] = 0.0;
    for (int i = 0; i < n; ++i) {
        double r[3];
        for (int a = 0; a < 3; ++a) r[a] = X[a] - (pts[3 * i + a] + sh[a]);
        const double r2 = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
        const double i2 = 1.0 / r2, i4 = i2 * i2, i6 = i4 * i2;
        M += K[i] * i2;
        for (int a = 0; a < 3; ++a) {
            g[a] += -2.0 * K[i] * r[a] * i4;
            for (int b = 0; b < 3; ++b)
                H[3 * a + b] += K[i] * (8.0 * r[a] * r[b] * i6 - (a == b ? 2.0 * i4 : 0.0));
        }
    }
}

// A body's control points for the Newton iterations: read from global
// memory each time, or (up to kRegPts points) held in registers, which
// removes the memory latency from the serial iteration.  Both evaluate
// exactly the sums of mb_d2 in the same order.
struct BodyG {
    const double* pts;
    const double* K;
    int n;
    __device__ void eval(const double sh[3], const double X[3], double& M, double g[3],
                         double H[9]) const
    {
        mb_d2(pts, K, n, sh, X, M, g, H);
    }
};

constexpr int kRegPts = 6;
struct BodyR {
    double p[kRegPts][3], k[kRegPts];
    int n;
    __device__ BodyR(const double* pts, const double* K, int n_) : n(n_)
    {
#pragma unroll
        for (int i = 0; i < kRegPts; ++i) {
            const bool on = i < n;
            for (int a = 0; a < 3; ++a) p[i][a] = on ? pts[3 * i + a] : 0.0;
            k[i] = on ? K[i] : 0.0;
        }
    }
    __device__ __forceinline__ void eval(const double sh[3], const double X[3], double& M,
                                         double g[3], double H[9]) const
    {
        M = 0.0;
        for (int a = 0; a < 3; ++a) g[a] = 0.0;
        for (int a = 0; a < 9; ++a) H[a] = 0.0;
#pragma unroll
        for (int i = 0; i < kRegPts; ++i) {
            if (i >= n) break;
            double r[3];
            for (int a = 0; a < 3; ++a) r[a] = X[a] - (p[i][a] + sh[a]);
            const double r2 = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
            const double i2 = 1.0 / r2, i4 = i2 * i2, i6 = i4 * i2;
            M += k[i] * i2;
            for (int a = 0; a < 3; ++a) {
                g[a] += -2.0 * k[i] * r[a] * i4;
                for (int b = 0; b < 3; ++b)
                    H[3 * a + b] += k[i] * (8.0 * r[a] * r[b] * i6 - (a == b ? 2.0 * i4 : 0.0));
            }
        }
    }
};

__device__ bool solve3(const double H[9], const double g[3], double dx[3])
{
    double c[9];
    c[0] = H[4] * H[8] - H[5] * H[7];
    c[1] = H[2] * H[7] - H[1] * H[8];
    c[2] = H[1] * H[5] - H[2] * H[4];
    c[3] = H[5] * H[6] - H[3] * H[8];
    c[4] = H[0] * H[8] - H[2] * H[6];
    c[5] = H[2] * H[3] - H[0] * H[5];
    c[6] = H[3] * H[7] - H[4] * H[6];
    c[7] = H[1] * H[6] - H[0] * H[7];
    c[8] = H[0] * H[4] - H[1] * H[3];
    const double det = H[0] * c[0] + H[1] * c[3] + H[2] * c[6];
    if (!(fabs(det) > 0.0) || !isfinite(det)) return false;
    for (int i = 0; i < 3; ++i) dx[i] = -(c[3 * i] * g[0] + c[3 * i + 1] * g[1] + c[3 * i + 2] * g[2]) / det;
    return true;
}

__device__ double reach(const PartDev& P, int p)
{
    double sk = 0.0, r = 0.0;
    for (int i = P.off[p]; i < P.off[p + 1]; ++i) {
        const double* b = P.body_pts + 3 * (int64_t)i;
        r = fmax(r, sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]));
        sk += P.K[i];
    }
    return r + sqrt(sk);
}

// Normal spring-dashpot (clamped at zero) and tangential spring with Coulomb
// limit; updates the spring xi in h[1..3]; returns the force on body i.
__device__ void contact_force(const DemP& c, double delta, const double n[3], const double vrel[3],
                              double dt, double* h, double Fi[3])
{
    const double vn = dot3(vrel, n);
    double Fn = c.kn * delta - c.etan * vn;
    if (Fn < 0.0) Fn = 0.0;
    double vt[3], xi[3], Ft[3];
    for (int a = 0; a < 3; ++a) vt[a] = vrel[a] - vn * n[a];
    const double xin = h[1] * n[0] + h[2] * n[1] + h[3] * n[2];
    for (int a = 0; a < 3; ++a) xi[a] = h[1 + a] - xin * n[a] + vt[a] * dt;
    for (int a = 0; a < 3; ++a) Ft[a] = -c.kt * xi[a] - c.etat * vt[a];
    const double ftn = sqrt(dot3(Ft, Ft));
    if (ftn > c.mu * Fn && ftn > 0.0) {
        const double s = c.mu * Fn / ftn;
        for (int a = 0; a < 3; ++a) {
            Ft[a] *= s;
            xi[a] = -(Ft[a] + c.etat * vt[a]) / c.kt;
        }
    }
    for (int a = 0; a < 3; ++a) {
        h[1 + a] = xi[a];
        Fi[a] = Fn * n[a] + Ft[a];
    }
}

__device__ void half_kick(const PartDev& P, int p, const double* FTh, const double* fc,
                          const DemP& c, double h, bool implicit)
{
    const double m = P.mass[p];
    const double mrel = m - c.rhof * P.volume[p];
    double T[3];
    for (int a = 0; a < 3; ++a) {
        const double F = FTh[6 * p + a] + mrel * c.g[a] + fc[6 * p + a];
        P.vel[3 * p + a] += h * F / m;
        T[a] = FTh[6 * p + 3 + a] + fc[6 * p + 3 + a];
    }
    double R[9];
    rotmat(P.quat + 4 * p, R);
    double w0[3], Tb[3], wb[3];
    const double* om = P.omega + 3 * p;
    for (int i = 0; i < 3; ++i) {
        w0[i] = R[i] * om[0] + R[3 + i] * om[1] + R[6 + i] * om[2];
        Tb[i] = R[i] * T[0] + R[3 + i] * T[1] + R[6 + i] * T[2];
        wb[i] = w0[i];
    }
    const double* I = P.inertia + 3 * p;
    const int iters = implicit ? 4 : 1;
    for (int it = 0; it < iters; ++it) {
        const double Iw[3] = {I[0] * wb[0], I[1] * wb[1], I[2] * wb[2]};
        double cc[3];
        cross3(wb, Iw, cc);
        double nw[3];
        for (int a = 0; a < 3; ++a) nw[a] = w0[a] + h * (Tb[a] - cc[a]) / I[a];
        for (int a = 0; a < 3; ++a) wb[a] = nw[a];
    }
    for (int i = 0; i < 3; ++i) P.omega[3 * p + i] = R[3 * i] * wb[0] + R[3 * i + 1] * wb[1] + R[3 * i + 2] * wb[2];
}

// First half kick, drift, rotation and world control points of particle p;
// also its broad-phase reach and the reset of its contact sums.
__device__ void first_half(const PartDev& P, int p, const double* FTh, double* fc,
                           double* reach_out, const DemP& c, double dt, const Geom& g)
{
    half_kick(P, p, FTh, fc, c, 0.5 * dt, false);
    for (int k = 0; k < 6; ++k) fc[6 * p + k] = 0.0;
    reach_out[p] = reach(P, p);
    for (int a = 0; a < 3; ++a) {
        double x = P.pos[3 * p + a] + dt * P.vel[3 * p + a];
        if (g.per[a]) {
            if (x >= (double)g.n[a]) x -= g.n[a];
            else if (x < 0.0) x += g.n[a];
        }
        P.pos[3 * p + a] = x;
    }
    const double* om = P.omega + 3 * p;
    const double wn = sqrt(om[0] * om[0] + om[1] * om[1] + om[2] * om[2]);
    double dq[4];
    dq[0] = cos(0.5 * wn * dt);
    const double s = wn > 0.0 ? sin(0.5 * wn * dt) / wn : 0.0;
    dq[1] = s * om[0];
    dq[2] = s * om[1];
    dq[3] = s * om[2];
    double* q = P.quat + 4 * p;
    double qn[4];
    qn[0] = dq[0] * q[0] - dq[1] * q[1] - dq[2] * q[2] - dq[3] * q[3];
    qn[1] = dq[0] * q[1] + dq[1] * q[0] + dq[2] * q[3] - dq[3] * q[2];
    qn[2] = dq[0] * q[2] - dq[1] * q[3] + dq[2] * q[0] + dq[3] * q[1];
    qn[3] = dq[0] * q[3] + dq[1] * q[2] - dq[2] * q[1] + dq[3] * q[0];
    const double nrm = sqrt(qn[0] * qn[0] + qn[1] * qn[1] + qn[2] * qn[2] + qn[3] * qn[3]);
    for (int a = 0; a < 4; ++a) q[a] = qn[a] / nrm;
    double R[9];
    rotmat(q, R);
    for (int i = P.off[p]; i < P.off[p + 1]; ++i) {
        const double* b = P.body_pts + 3 * (int64_t)i;
        for (int a = 0; a < 3; ++a)
            P.wpts[3 * (int64_t)i + a] = P.pos[3 * p + a] + (R[3 * a] * b[0] + R[3 * a + 1] * b[1] + R[3 * a + 2] * b[2]);
    }
}

__global__ void k_first_half(PartDev P, const double* FTh, double* fc, double* reach_out, DemP c,
                             double dt, Geom g)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P.n) return;
    first_half(P, p, FTh, fc, reach_out, c, dt, g);
}

__device__ void wall_contact(const PartDev& P, int t, double* hist, double* fc, const double* rch,
                             const DemP& c, double dt, const Geom& g);

// Newton on grad(M_A + M_B) = 0 from x, the contact test and the force of
// pair (i, j); A and B supply the two bodies' metaball sums.
template <class BA, class BB>
__device__ __forceinline__ void pair_contact(const BA& A, const BB& B, double x[3], double* h, const double* xi,
                             const double* xj, const double sh[3], int i, int j, double rsi,
                             double rsj, const PartDev& P, const DemP& c, double dt, double* fc)
{
    const double z3[3] = {0.0, 0.0, 0.0};
    double MA, MB, gA[3], gB[3], HA[9], HB[9];
    bool conv = false;
    for (int it = 0; it < c.niter; ++it) {
        A.eval(z3, x, MA, gA, HA);
        B.eval(sh, x, MB, gB, HB);
        double gg[3], H[9], dx[3];
        for (int a = 0; a < 3; ++a) gg[a] = gA[a] + gB[a];
        for (int a = 0; a < 9; ++a) H[a] = HA[a] + HB[a];
        if (!solve3(H, gg, dx)) break;
        for (int a = 0; a < 3; ++a) x[a] += dx[a];
        if (sqrt(dot3(dx, dx)) < c.ntol) {
            conv = true;
            break;
        }
    }
    if (!conv) {
        for (int k = 0; k < kHist; ++k) h[k] = 0.0;
        return;
    }
    A.eval(z3, x, MA, gA, HA);
    B.eval(sh, x, MB, gB, HB);
    // both bodies' fields above ctol at the stationary point (Eq. opt); the
    // separation is signed along the common line of the two projections of
    // Eq. cp, n = (grad M_i - grad M_j)/|.| from body j to body i, so that a
    // stationary point already inside one internal body (two flat faces
    // meeting at an angle) reads as an overlap rather than as no contact;
    // overlaps beyond 2 (R_si + R_sj) are stationary points inside a body,
    // where the projection of Eq. k0 does not hold, and are not contacts
    if (!(MA > c.ctol && MB > c.ctol)) {
        for (int k = 0; k < kHist; ++k) h[k] = 0.0;
        return;
    }
    const double qA = (1.0 - MA) / dot3(gA, gA), qB = (1.0 - MB) / dot3(gB, gB);
    double xa[3], dd[3], n[3];
    for (int a = 0; a < 3; ++a) {
        xa[a] = x[a] + qA * gA[a];
        dd[a] = xa[a] - (x[a] + qB * gB[a]);
        n[a] = gA[a] - gB[a];
    }
    const double un = sqrt(dot3(n, n));
    if (!(un > 0.0)) {
        for (int k = 0; k < kHist; ++k) h[k] = 0.0;
        return;
    }
    for (int a = 0; a < 3; ++a) n[a] = n[a] / un;
    const double delta = rsi + rsj - dot3(dd, n);
    if (!(delta <= 2.0 * (rsi + rsj))) {
        for (int k = 0; k < kHist; ++k) h[k] = 0.0;
        return;
    }
    h[0] = 1.0;
    for (int a = 0; a < 3; ++a) h[4 + a] = x[a] - xi[a];
    if (delta <= 0.0) {
        h[1] = h[2] = h[3] = 0.0;
        return;
    }
    double xcp[3], ra[3], rb[3];
    for (int a = 0; a < 3; ++a) {
        xcp[a] = xa[a] - (rsi - 0.5 * delta) * n[a];
        ra[a] = xcp[a] - xi[a];
        rb[a] = xcp[a] - (xj[a] + sh[a]);
    }
    double ca[3], cb[3], vrel[3], Fi[3], tq[3];
    cross3(P.omega + 3 * i, ra, ca);
    cross3(P.omega + 3 * j, rb, cb);
    for (int a = 0; a < 3; ++a) vrel[a] = (P.vel[3 * i + a] + ca[a]) - (P.vel[3 * j + a] + cb[a]);
    contact_force(c, delta, n, vrel, dt, h, Fi);
    for (int a = 0; a < 3; ++a) {
        atomicAdd(fc + 6 * i + a, Fi[a]);
        atomicAdd(fc + 6 * j + a, -Fi[a]);
    }
    cross3(ra, Fi, tq);
    for (int a = 0; a < 3; ++a) atomicAdd(fc + 6 * i + 3 + a, tq[a]);
    cross3(rb, Fi, tq);
    for (int a = 0; a < 3; ++a) atomicAdd(fc + 6 * j + 3 + a, -tq[a]);
}

// Contact of pair (i < j): broad-phase test on the reach radii, then the
// Newton search and force; the pair's history is record `slot` of particle i.
__device__ __forceinline__ void pair_item(const PartDev& P, double* hist, double* fc,
                                          const double* rch, const DemP& c, double dt,
                                          const Geom& g, int i, int j, int slot)
{
    double* h = hist + ((int64_t)i * kPairSlots + slot) * kHist;
    const double* xi = P.pos + 3 * i;
    const double* xj = P.pos + 3 * j;
    double sh[3], dv[3];
    for (int a = 0; a < 3; ++a) {
        const double d = xj[a] - xi[a];
        sh[a] = 0.0;
        if (g.per[a]) {
            const double L = g.n[a];
            if (d > 0.5 * L) sh[a] = -L;
            else if (d < -0.5 * L) sh[a] = L;
        }
        dv[a] = d + sh[a];
    }
    const double rsi = P.rs[i], rsj = P.rs[j];
    if (sqrt(dot3(dv, dv)) > rch[i] + rch[j] + rsi + rsj) {
        // out of reach: forget the pair's contact (read one double instead of
        // writing eight when the record is zero already)
        if (h[0] != 0.0)
            for (int k = 0; k < kHist; ++k) h[k] = 0.0;
        return;
    }
    const int ai = P.off[i], ni = min(P.off[i + 1] - ai, kMaxPts);
    const int aj = P.off[j], nj = min(P.off[j + 1] - aj, kMaxPts);
    const double* pi = P.wpts + 3 * (int64_t)ai;
    const double* pj = P.wpts + 3 * (int64_t)aj;
    double x[3];
    if (h[0] != 0.0) {
        for (int a = 0; a < 3; ++a) x[a] = xi[a] + h[4 + a];
    } else {
        double best = INFINITY;
        for (int u = 0; u < ni; ++u)
            for (int v = 0; v < nj; ++v) {
                double d2 = 0.0;
                for (int a = 0; a < 3; ++a) {
                    const double dd = pi[3 * u + a] - (pj[3 * v + a] + sh[a]);
                    d2 += dd * dd;
                }
                if (d2 < best) {
                    best = d2;
                    for (int a = 0; a < 3; ++a) x[a] = 0.5 * (pi[3 * u + a] + pj[3 * v + a] + sh[a]);
                }
            }
    }
    if (ni <= kRegPts && nj <= kRegPts)
        pair_contact(BodyR(pi, P.K + ai, ni), BodyR(pj, P.K + aj, nj), x, h, xi, xj, sh, i, j, rsi,
                     rsj, P, c, dt, fc);
    else
        pair_contact(BodyG{pi, P.K + ai, ni}, BodyG{pj, P.K + aj, nj}, x, h, xi, xj, sh, i, j,
                     rsi, rsj, P, c, dt, fc);
}

// Whether pair (i, j) is a candidate of a dem_step call of duration T: the
// centres are within the reach radii, R_s and a skin that covers the
// relative displacement of the call, (|v_i| + |v_j|) T + 1/2 (velocities
// change by far less than 1/4 lu per lattice step under the accelerations of
// a stable run).  A pair outside it cannot come into reach during the call.
__device__ bool pair_candidate(const PartDev& P, int i, int j, double T, const Geom& g)
{
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        double d = P.pos[3 * j + a] - P.pos[3 * i + a];
        if (g.per[a]) {
            const double L = g.n[a];
            if (d > 0.5 * L) d -= L;
            else if (d < -0.5 * L) d += L;
        }
        d2 += d * d;
    }
    const double* vi = P.vel + 3 * i;
    const double* vj = P.vel + 3 * j;
    const double skin = (sqrt(dot3(vi, vi)) + sqrt(dot3(vj, vj))) * T + 0.5;
    const double thr = reach(P, i) + reach(P, j) + P.rs[i] + P.rs[j] + skin;
    return sqrt(d2) <= thr;
}

// The history records of pairs that are no longer candidates are released
// (zeroed, slot freed): one thread per (particle, slot).  A slot's key is
// the partner's index + 1, 0 when free, so zeroed state is empty.
__global__ __launch_bounds__(256) void k_pair_release(PartDev P, double* hist, int32_t* key,
                                                      double T, Geom g, uint32_t* count)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (count && t == 0) *count = 0u;  // the pair list of this call starts empty
    if (t >= (int64_t)P.n * kPairSlots) return;
    const int j = key[t] - 1;
    if (j < 0) return;
    const int i = (int)(t / kPairSlots);
    if (pair_candidate(P, i, j, T, g)) return;
    double* h = hist + t * kHist;
    for (int k = 0; k < kHist; ++k) h[k] = 0.0;
    key[t] = 0;
}

// Candidate pairs of one dem_step call, one thread per (i, j): a candidate
// pair i < j finds its history record among particle i's slots, or claims a
// free one (released records are zero), and is appended as
// slot << 32 | i << 16 | j, one atomic per wave.  A particle with more
// candidate partners than slots latches kDeferredSlots (the pair is left
// out).
__global__ __launch_bounds__(256) void k_pairs(PartDev P, int32_t* key, double T, Geom g,
                                               uint64_t* list, uint32_t* count, uint32_t* deferred)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int np = P.n;
    bool take = false;
    int i = 0, j = 0, slot = -1;
    if (t < (int64_t)np * np) {
        i = (int)(t / np);
        j = (int)(t % np);
        take = i < j && pair_candidate(P, i, j, T, g);
    }
    if (take) {
        int32_t* ki = key + (int64_t)i * kPairSlots;
        for (int s = 0; s < kPairSlots && slot < 0; ++s)
            if (ki[s] == j + 1) slot = s;
        for (int s = 0; s < kPairSlots && slot < 0; ++s)
            if (atomicCAS(ki + s, 0, j + 1) == 0) slot = s;
        if (slot < 0) {
            atomicOr(deferred, kDeferredSlots);
            take = false;
        }
    }
    const uint64_t m = __ballot(take);
    if (m == 0) return;
    const int lane = threadIdx.x & 63;
    uint32_t base = 0;
    if (lane == __ffsll((unsigned long long)m) - 1) base = atomicAdd(count, (uint32_t)__popcll(m));
    base = __shfl(base, __ffsll((unsigned long long)m) - 1, 64);
    if (take) {
        const uint32_t below = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
        list[base + below] = ((uint64_t)slot << 32) | ((uint64_t)i << 16) | (uint64_t)j;
    }
}

// ---------------------------------------------------------------------------
// Broad phase on a cell grid (many particles): every pair that
// pair_candidate accepts is at most H = 2 max_p (reach_p + R_s,p) + 2 max_p
// |v_p| T + 1/2 apart, so with cells at least H wide (fewer cells than the
// arrays hold: wider) its particles lie in the same or adjacent cells.  The
// same pairs, records and latch as k_pairs; only the list's order differs,
// and the contact forces are summed by atomics in any order either way.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int grid_cell(const PartDev& P, int p, const Geom& g,
                                         const int32_t* gdim, const double* gsize, int c3[3])
{
    for (int a = 0; a < 3; ++a) {
        double x = P.pos[3 * p + a];
        if (g.per[a]) x -= (double)g.n[a] * floor(x / (double)g.n[a]);  // into [0, n]
        int k = (int)floor(x / gsize[a]);
        c3[a] = min(max(k, 0), gdim[a] - 1);
    }
    return c3[0] + gdim[0] * (c3[1] + gdim[1] * c3[2]);
}

// One workgroup: the cell width from the particles, the grid's shape, and
// the counts cleared.
__global__ __launch_bounds__(1024) void k_grid_setup(PartDev P, double T, Geom g, int32_t* gdim,
                                                     double* gsize, uint32_t* gcount, int64_t gcap)
{
    __shared__ double red[2][16];
    __shared__ int ncell;
    double h = 0.0, v = 0.0;
    for (int p = (int)threadIdx.x; p < P.n; p += (int)blockDim.x) {
        h = fmax(h, reach(P, p) + P.rs[p]);
        const double* vp = P.vel + 3 * p;
        v = fmax(v, sqrt(dot3(vp, vp)));
    }
    for (int m = 32; m >= 1; m >>= 1) {
        h = fmax(h, __shfl_xor(h, m, 64));
        v = fmax(v, __shfl_xor(v, m, 64));
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wv] = h;
        red[1][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double hm = 0.0, vm = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            hm = fmax(hm, red[0][w]);
            vm = fmax(vm, red[1][w]);
        }
        // the largest accepted distance, with a margin for rounding
        double H = (2.0 * hm + 2.0 * vm * T + 0.5) * (1.0 + 1e-9) + 1e-9;
        int nc[3];
        int64_t total = 1;
        for (int it = 0; it < 64; ++it) {
            total = 1;
            for (int a = 0; a < 3; ++a) {
                nc[a] = max(1, (int)floor((double)g.n[a] / H));
                total *= nc[a];
            }
            if (total <= gcap) break;
            H *= 1.25;  // more cells than the arrays hold: wider cells
        }
        for (int a = 0; a < 3; ++a) {
            gdim[a] = nc[a];
            gsize[a] = (double)g.n[a] / (double)nc[a];
        }
        gsize[3] = H;
        gdim[3] = (int32_t)total;
        ncell = (int)total;
    }
    __syncthreads();
    for (int i = (int)threadIdx.x; i <= ncell; i += (int)blockDim.x) gcount[i] = 0u;
}

__global__ __launch_bounds__(256) void k_grid_count(PartDev P, Geom g, const int32_t* gdim,
                                                    const double* gsize, uint32_t* gcount)
{
    const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (p >= P.n) return;
    int c3[3];
    atomicAdd(gcount + grid_cell(P, p, g, gdim, gsize, c3), 1u);
}

// One workgroup: exclusive starts of the cells in place (gcount[C] = n),
// and the scatter cursors.
__global__ __launch_bounds__(1024) void k_grid_scan(const int32_t* gdim, uint32_t* gcount,
                                                    uint32_t* gcursor)
{
    __shared__ uint32_t wsum[16];
    __shared__ uint32_t carry;
    const int C = gdim[3];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (threadIdx.x == 0) carry = 0u;
    __syncthreads();
    for (int b0 = 0; b0 < C; b0 += (int)blockDim.x) {
        const int i = b0 + (int)threadIdx.x;
        const uint32_t x = i < C ? gcount[i] : 0u;
        uint32_t incl = x;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t t = __shfl_up(incl, o, 64);
            if (lane >= o) incl += t;
        }
        if (lane == 63) wsum[wv] = incl;
        __syncthreads();
        uint32_t before = carry;
        for (int w = 0; w < wv; ++w) before += wsum[w];
        const uint32_t excl = before + incl - x;
        __syncthreads();  // every thread has read carry and wsum
        if (i < C) {
            gcount[i] = excl;
            gcursor[i] = excl;
        }
        if (threadIdx.x == blockDim.x - 1) carry = excl + x;
        __syncthreads();
    }
    if (threadIdx.x == 0) gcount[C] = carry;
}

__global__ __launch_bounds__(256) void k_grid_scatter(PartDev P, Geom g, const int32_t* gdim,
                                                      const double* gsize, uint32_t* gcursor,
                                                      uint32_t* gitem)
{
    const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (p >= P.n) return;
    int c3[3];
    const uint32_t slot = atomicAdd(gcursor + grid_cell(P, p, g, gdim, gsize, c3), 1u);
    gitem[slot] = (uint32_t)p;
}

// The cells around one along an axis: c - 1, c, c + 1, wrapped on a
// periodic axis, clipped at walls, each once.
__device__ __forceinline__ int around(int c, int nc, int per, int out[3])
{
    int m = 0;
    for (int d = -1; d <= 1; ++d) {
        int k = c + d;
        if (k < 0 || k >= nc) {
            if (!per) continue;
            k = (k + nc) % nc;
        }
        bool seen = false;
        for (int t = 0; t < m; ++t) seen = seen || out[t] == k;
        if (!seen) out[m++] = k;
    }
    return m;
}

// One thread per particle i: the partners j > i in the cells around i's.
__global__ __launch_bounds__(256) void k_pairs_grid(PartDev P, int32_t* key, double T, Geom g,
                                                    const int32_t* gdim, const double* gsize,
                                                    const uint32_t* gstart, const uint32_t* gitem,
                                                    uint64_t* list, uint32_t* count,
                                                    uint32_t* deferred)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= P.n) return;
    int c3[3];
    grid_cell(P, i, g, gdim, gsize, c3);
    int ax[3][3], na[3];
    for (int a = 0; a < 3; ++a) na[a] = around(c3[a], gdim[a], g.per[a], ax[a]);
    int32_t* ki = key + (int64_t)i * kPairSlots;
    // every accepted pair lies within H (gsize[3]): a cheaper distance test
    // first, then pair_candidate's own decision
    const double hb2 = gsize[3] * gsize[3];
    for (int u = 0; u < na[2]; ++u)
        for (int t = 0; t < na[1]; ++t)
            for (int s = 0; s < na[0]; ++s) {
                const int cell = ax[0][s] + gdim[0] * (ax[1][t] + gdim[1] * ax[2][u]);
                for (uint32_t k = gstart[cell]; k < gstart[cell + 1]; ++k) {
                    const int j = (int)gitem[k];
                    if (j <= i) continue;
                    double d2 = 0.0;
                    for (int a = 0; a < 3; ++a) {
                        double d = P.pos[3 * j + a] - P.pos[3 * i + a];
                        if (g.per[a]) {
                            const double L = g.n[a];
                            if (d > 0.5 * L) d -= L;
                            else if (d < -0.5 * L) d += L;
                        }
                        d2 += d * d;
                    }
                    if (!(d2 <= hb2) || !pair_candidate(P, i, j, T, g)) continue;
                    int slot = -1;
                    for (int q = 0; q < kPairSlots && slot < 0; ++q)
                        if (ki[q] == j + 1) slot = q;
                    for (int q = 0; q < kPairSlots && slot < 0; ++q)
                        if (atomicCAS(ki + q, 0, j + 1) == 0) slot = q;
                    if (slot < 0) {
                        atomicOr(deferred, kDeferredSlots);
                        continue;
                    }
                    const uint32_t at = atomicAdd(count, 1u);
                    list[at] = ((uint64_t)slot << 32) | ((uint64_t)i << 16) | (uint64_t)j;
                }
            }
}

// One substep's contacts: the walls of every body (6 n items), then the
// listed pairs; thread t of nthreads strides over both.
__device__ void contacts(const PartDev& P, double* hist, double* hist_w, double* fc,
                         const double* rch, const DemP& c, double dt, const Geom& g,
                         const uint64_t* list, const uint32_t* count, int64_t t0, int64_t nthreads)
{
    const int64_t nw = (int64_t)P.n * 6;
    const int64_t total = nw + (int64_t)*count;
    for (int64_t t = t0; t < total; t += nthreads) {
        if (t < nw) {
            wall_contact(P, (int)t, hist_w, fc, rch, c, dt, g);
        } else {
            const uint64_t e = list[t - nw];
            pair_item(P, hist, fc, rch, c, dt, g, (int)((e >> 16) & 0xffffu), (int)(e & 0xffffu),
                      (int)(e >> 32));
        }
    }
}

__global__ __launch_bounds__(256) void k_contacts(PartDev P, double* hist, double* hist_w, double* fc,
                                                  const double* rch, DemP c, double dt, Geom g,
                                                  const uint64_t* list, const uint32_t* count)
{
    contacts(P, hist, hist_w, fc, rch, c, dt, g, list, count,
             (int64_t)blockIdx.x * blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x);
}

// In-plane Newton for the point of the wall plane where M is largest, the
// contact test and the force of body i on wall (ax, side); A supplies the
// body's metaball sums.
template <class BA>
__device__ __forceinline__ void wall_newton(const BA& A, double x[3], double* h, const double* xi, int i, int ax,
                            int t1, int t2, double sgn, const PartDev& P, const DemP& c, double dt,
                            double* fc)
{
    const double z3[3] = {0.0, 0.0, 0.0};
    double M, gr[3], H[9];
    bool conv = false;
    for (int it = 0; it < c.niter; ++it) {
        A.eval(z3, x, M, gr, H);
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
        for (int k = 0; k < kHist; ++k) h[k] = 0.0;
        return;
    }
    A.eval(z3, x, M, gr, H);
    if (!(sgn * gr[ax] > 0.0)) {
        for (int k = 0; k < kHist; ++k) h[k] = 0.0;
        return;
    }
    h[0] = 1.0;
    for (int a = 0; a < 3; ++a) h[4 + a] = x[a] - xi[a];
    const double qR = (1.0 - M) / dot3(gr, gr);
    const double delta = P.rs[i] - sgn * (qR * gr[ax]);
    if (delta <= 0.0) {
        h[1] = h[2] = h[3] = 0.0;
        return;
    }
    double n[3] = {0.0, 0.0, 0.0}, xcp[3], ra[3];
    n[ax] = sgn;
    for (int a = 0; a < 3; ++a) {
        xcp[a] = x[a] - 0.5 * delta * n[a];
        ra[a] = xcp[a] - xi[a];
    }
    double ca[3], vrel[3], Fi[3], tq[3];
    cross3(P.omega + 3 * i, ra, ca);
    for (int a = 0; a < 3; ++a) vrel[a] = P.vel[3 * i + a] + ca[a];
    contact_force(c, delta, n, vrel, dt, h, Fi);
    cross3(ra, Fi, tq);
    for (int a = 0; a < 3; ++a) {
        atomicAdd(fc + 6 * i + a, Fi[a]);
        atomicAdd(fc + 6 * i + 3 + a, tq[a]);
    }
}

__device__ void wall_contact(const PartDev& P, int t, double* hist, double* fc, const double* rch,
                             const DemP& c, double dt, const Geom& g)
{
    const int i = t / 6, ax = (t % 6) / 2, side = t % 2;
    if (g.per[ax]) return;
    double* h = hist + (int64_t)t * kHist;
    const double plane = side ? g.n[ax] - 0.5 : -0.5, sgn = side ? -1.0 : 1.0;
    const double* xi = P.pos + 3 * i;
    if (sgn * (xi[ax] - plane) > rch[i] + P.rs[i]) {
        if (h[0] != 0.0)
            for (int k = 0; k < kHist; ++k) h[k] = 0.0;
        return;
    }
    const int ai = P.off[i], ni = min(P.off[i + 1] - ai, kMaxPts);
    const double* pi = P.wpts + 3 * (int64_t)ai;
    const int t1 = (ax + 1) % 3, t2 = (ax + 2) % 3;
    double x[3];
    if (h[0] != 0.0) {
        for (int a = 0; a < 3; ++a) x[a] = xi[a] + h[4 + a];
    } else {
        double best = INFINITY;
        for (int u = 0; u < ni; ++u) {
            const double dd = fabs(pi[3 * u + ax] - plane);
            if (dd < best) {
                best = dd;
                for (int a = 0; a < 3; ++a) x[a] = pi[3 * u + a];
            }
        }
    }
    x[ax] = plane;
    if (ni <= kRegPts)
        wall_newton(BodyR(pi, P.K + ai, ni), x, h, xi, i, ax, t1, t2, sgn, P, c, dt, fc);
    else
        wall_newton(BodyG{pi, P.K + ai, ni}, x, h, xi, i, ax, t1, t2, sgn, P, c, dt, fc);
}

__global__ void k_second_half(PartDev P, const double* FTh, const double* fc, DemP c, double dt)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P.n) return;
    half_kick(P, p, FTh, fc, c, 0.5 * dt, true);
}

// The second half kick of substep s and the first half of substep s + 1 of
// particle p in one launch: both read the contact sum of substep s, which
// the first half then clears.
__global__ void k_between(PartDev P, const double* FTh, double* fc, double* reach_out, DemP c,
                          double dt, Geom g)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P.n) return;
    half_kick(P, p, FTh, fc, c, 0.5 * dt, true);
    first_half(P, p, FTh, fc, reach_out, c, dt, g);
}

}  // namespace

hipError_t launch_dem(lbm_ctx* ctx, const PartDev& P, int n_sub, double dt, const dem_params& prm,
                      const DemScratch& ws)
{
    const int np = P.n;
    if (np == 0) return hipSuccess;
    DemP c;
    c.kn = prm.kn;
    c.etan = prm.eta_n;
    c.kt = prm.kt;
    c.etat = prm.eta_t;
    c.mu = prm.mu_s;
    c.ctol = prm.ctol;
    c.ntol = prm.newton_tol;
    c.niter = prm.newton_iter;
    for (int a = 0; a < 3; ++a) c.g[a] = prm.gravity[a];
    c.rhof = prm.rho_f;
    const uint32_t bp = (np + 63) / 64;
    // candidate pairs for the whole call: histories of pairs that dropped out
    // are released first, so that their slots can be claimed again
    const double T = (double)n_sub * dt;
    const uint32_t br = (uint32_t)(((int64_t)np * kPairSlots + 255) / 256);
    const uint32_t bq = (uint32_t)(((int64_t)np * np + 255) / 256);
    hipLaunchKernelGGL(k_pair_release, dim3(br), dim3(256), 0, ctx->stream, P, ctx->hist_pp,
                       ctx->hist_key, T, ctx->geom, ws.count);
    if (ws.gcount && np >= kGridMinParticles) {
        const uint32_t bn = (uint32_t)((np + 255) / 256);
        hipLaunchKernelGGL(k_grid_setup, dim3(1), dim3(1024), 0, ctx->stream, P, T, ctx->geom,
                           ws.gdim, ws.gsize, ws.gcount, ws.gcap);
        hipLaunchKernelGGL(k_grid_count, dim3(bn), dim3(256), 0, ctx->stream, P, ctx->geom, ws.gdim,
                           ws.gsize, ws.gcount);
        hipLaunchKernelGGL(k_grid_scan, dim3(1), dim3(1024), 0, ctx->stream, ws.gdim, ws.gcount,
                           ws.gcursor);
        hipLaunchKernelGGL(k_grid_scatter, dim3(bn), dim3(256), 0, ctx->stream, P, ctx->geom, ws.gdim,
                           ws.gsize, ws.gcursor, ws.gitem);
        hipLaunchKernelGGL(k_pairs_grid, dim3(bn), dim3(256), 0, ctx->stream, P, ctx->hist_key, T,
                           ctx->geom, ws.gdim, ws.gsize, ws.gcount, ws.gitem, ws.pairs, ws.count,
                           ctx->ctr + kCtrDeferred);
    } else {
        hipLaunchKernelGGL(k_pairs, dim3(bq), dim3(256), 0, ctx->stream, P, ctx->hist_key, T,
                           ctx->geom, ws.pairs, ws.count, ctx->ctr + kCtrDeferred);
    }
    const int64_t most = 6 * (int64_t)np + (int64_t)np * kPairSlots;
    const uint32_t bc = (uint32_t)std::min<int64_t>((most + 255) / 256, 1024);
    // first half, then per substep the contacts and the two half kicks
    // around the substep boundary in one launch
    hipLaunchKernelGGL(k_first_half, dim3(bp), dim3(64), 0, ctx->stream, P, ctx->FT, ctx->fc,
                       ws.reach, c, dt, ctx->geom);
    for (int s = 0; s < n_sub; ++s) {
        hipLaunchKernelGGL(k_contacts, dim3(bc), dim3(256), 0, ctx->stream, P, ctx->hist_pp,
                           ctx->hist_pw, ctx->fc, ws.reach, c, dt, ctx->geom, ws.pairs, ws.count);
        if (s + 1 < n_sub)
            hipLaunchKernelGGL(k_between, dim3(bp), dim3(64), 0, ctx->stream, P, ctx->FT, ctx->fc,
                               ws.reach, c, dt, ctx->geom);
        else
            hipLaunchKernelGGL(k_second_half, dim3(bp), dim3(64), 0, ctx->stream, P, ctx->FT,
                               ctx->fc, c, dt);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The allocation-free work space of dem_step_noalloc: one static array per
// device (module-scope device memory, loaded with the code object), laid out
// as the pair count (first 512 bytes), the reach of up to kNoAllocParticles
// particles, then up to kNoAllocParticles * kPairSlots pair entries.  Host
// code never uses the array's name as an address: the device address is
// looked up once per device and kept.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kNoAllocHead = 64;  // 8-byte words before the reach
constexpr size_t kNoAllocWords =
    kNoAllocHead + (size_t)kNoAllocParticles + (size_t)kNoAllocParticles * kPairSlots;
__device__ __align__(256) uint64_t scratch[kNoAllocWords];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint64_t* g_scratch_dev[kMaxDevices] = {};
}  // namespace

hipError_t dem_noalloc_setup()
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_dev[dev]) return hipSuccess;
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[dev] = static_cast<uint64_t*>(ptr);
    return hipSuccess;
}

bool dem_noalloc_scratch(int dev, DemScratch* out)
{
    if (dev < 0 || dev >= kMaxDevices) return false;
    uint64_t* base;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        base = g_scratch_dev[dev];
    }
    if (!base) return false;
    out->count = reinterpret_cast<uint32_t*>(base);
    out->reach = reinterpret_cast<double*>(base + kNoAllocHead);
    out->pairs = base + kNoAllocHead + kNoAllocParticles;
    return true;
}

}  // namespace mdlbm

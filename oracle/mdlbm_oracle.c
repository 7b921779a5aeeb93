/*
 * mdlbm_oracle.c -- plain, slow, FP64 CPU oracle of the per-timestep lattice
 * update of the coupled metaball-DEM / lattice Boltzmann method with a sharp
 * interface (Zhang et al., arXiv 2206.11634).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline timing load this file's library.  It shares no code, header, table
 * or constant with the HIP library: every table below is typed here from the
 * paper (D3Q15, Sec. 2.2) or from the textbook D3Q19 lattice.
 *
 * Every function follows the paper's equations in its own order and notation,
 * one node or one link at a time, in IEEE double precision with no
 * contraction of a*b+c into fused multiply-adds (build with
 * -ffp-contract=off).  Readings of places where the paper is silent are
 * marked READING and listed with the design notes.
 *
 * Link convention.  A link is (x_s, d, j): x_s is a node owned by particle j,
 * d a lattice direction, and x_n = x_s - e_d the neighbour the direction
 * points away from (so e_d points from x_n into the solid).  When x_n is a
 * fluid node it is the paper's boundary node x_f, x_ff = x_f - e_d is the next
 * node away from the wall, the wall point is x_w = x_f + q e_d, and the
 * unknown population after streaming is f_{opp(d)}(x_f, t+1).
 *
 * Parity pins (tests/test_oracle_*.py): rest state, mass conservation,
 * Poiseuille closed form, decaying shear wave, uniform body-force momentum,
 * lattice isotropy, brute-force classification on tiny lattices, plane-exact
 * and sphere q, a co-moving particle invariant, near-wall rest invariant for
 * the missing-force-point treatment, Hasimoto drag, and DEM closed forms.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Lattices.                                                                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    int Q;
    int e[19][3];
    double w[19];
    int opp[19];
} stencil_t;

/* Textbook D3Q19: rest, 6 axis and 12 face-diagonal velocities.  The order is
 * the one exported at the library boundary: the opposite of an odd index i is
 * i + 1. */
static const int E19[19][3] = {
    {0, 0, 0},   {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},   {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
    {-1, 0, 1},  {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

/* D3Q15 of Sec. 2.2: rest, 6 axis velocities, 8 cube diagonals; weights
 * 2/9, 1/9, 1/72. */
static const int E15[15][3] = {
    {0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 1},  {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1}, {1, -1, 1}, {-1, 1, -1}, {-1, 1, 1},
    {1, -1, -1}};

static int stencil_make(int Q, stencil_t* s)
{
    int i, j, a;
    if (Q != 19 && Q != 15) return -1;
    s->Q = Q;
    for (i = 0; i < Q; ++i) {
        int n2 = 0;
        for (a = 0; a < 3; ++a) {
            s->e[i][a] = (Q == 19) ? E19[i][a] : E15[i][a];
            n2 += s->e[i][a] * s->e[i][a];
        }
        if (Q == 19)
            s->w[i] = (n2 == 0) ? 1.0 / 3.0 : (n2 == 1) ? 1.0 / 18.0 : 1.0 / 36.0;
        else
            s->w[i] = (n2 == 0) ? 2.0 / 9.0 : (n2 == 1) ? 1.0 / 9.0 : 1.0 / 72.0;
    }
    for (i = 0; i < Q; ++i)
        for (j = 0; j < Q; ++j)
            if (s->e[j][0] == -s->e[i][0] && s->e[j][1] == -s->e[i][1] &&
                s->e[j][2] == -s->e[i][2])
                s->opp[i] = j;
    return 0;
}

int ora_stencil(int Q, int* e, double* w, int* opp)
{
    stencil_t s;
    int i;
    if (stencil_make(Q, &s)) return -1;
    for (i = 0; i < Q; ++i) {
        e[3 * i + 0] = s.e[i][0];
        e[3 * i + 1] = s.e[i][1];
        e[3 * i + 2] = s.e[i][2];
        w[i] = s.w[i];
        opp[i] = s.opp[i];
    }
    return Q;
}

/* ------------------------------------------------------------------------ */
/* Grid.  Node (i,j,k) sits at (i,j,k); index i + nx*(j + ny*k).  A periodic  */
/* axis wraps; a non-periodic axis ends in a wall half a cell outside.        */
/* ------------------------------------------------------------------------ */

typedef struct {
    int n[3];
    int per[3];
    long N;
} grid_t;

static grid_t grid_make(const int* dims, const int* per)
{
    grid_t g;
    int a;
    for (a = 0; a < 3; ++a) {
        g.n[a] = dims[a];
        g.per[a] = per[a] ? 1 : 0;
    }
    g.N = (long)dims[0] * dims[1] * dims[2];
    return g;
}

static long gidx(const grid_t* g, const int c[3])
{
    return c[0] + (long)g->n[0] * (c[1] + (long)g->n[1] * c[2]);
}

static void gcoord(const grid_t* g, long id, int c[3])
{
    c[0] = (int)(id % g->n[0]);
    id /= g->n[0];
    c[1] = (int)(id % g->n[1]);
    c[2] = (int)(id / g->n[1]);
}

/* Node c + s*e, wrapped on periodic axes.  Returns 0 when it lies outside a
 * non-periodic axis (beyond a wall). */
static int gshift(const grid_t* g, const int c[3], const int e[3], int s, int out[3])
{
    int a;
    for (a = 0; a < 3; ++a) {
        int v = c[a] + s * e[a];
        if (v < 0 || v >= g->n[a]) {
            if (!g->per[a]) return 0;
            v = ((v % g->n[a]) + g->n[a]) % g->n[a];
        }
        out[a] = v;
    }
    return 1;
}

/* Coordinate of node index c along axis a as seen from a particle centred at
 * `center`: on a periodic axis the image nearest the centre (a tie keeps the
 * unshifted index); elsewhere the index itself (which may lie beyond a wall for
 * a virtual node).  READING: the paper does not discuss periodic images. */
static double image_coord(const grid_t* g, int a, int c, double center)
{
    int L, w;
    double d;
    if (!g->per[a]) return (double)c;
    L = g->n[a];
    w = ((c % L) + L) % L;
    d = (double)w - center;
    if (d > 0.5 * L) return (double)(w - L);
    if (d < -0.5 * L) return (double)(w + L);
    return (double)w;
}

/* ------------------------------------------------------------------------ */
/* Metaball function, Eq. (metaball): M(x) = sum_i K_i / |x - x_i|^2.         */
/* READING (bit-exactness): r^2 = (dx*dx + dy*dy) + dz*dz, terms summed in    */
/* control-point order starting from 0.                                       */
/* ------------------------------------------------------------------------ */

static double metaball(int n, const double* pts, const double* K, const double X[3])
{
    double M = 0.0;
    int i;
    for (i = 0; i < n; ++i) {
        double dx = X[0] - pts[3 * i + 0];
        double dy = X[1] - pts[3 * i + 1];
        double dz = X[2] - pts[3 * i + 2];
        double r2 = (dx * dx + dy * dy) + dz * dz;
        M = M + K[i] / r2;
    }
    return M;
}

double ora_metaball(int n, const double* pts, const double* K, const double* X)
{
    return metaball(n, pts, K, X);
}

/* Gradient and Hessian of M (used by the DEM contact search, Eq. grad). */
static void metaball_d2(int n, const double* pts, const double* K, const double X[3],
                        double* M, double g[3], double H[9])
{
    int i, a, b;
    *M = 0.0;
    for (a = 0; a < 3; ++a) g[a] = 0.0;
    for (a = 0; a < 9; ++a) H[a] = 0.0;
    for (i = 0; i < n; ++i) {
        double r[3], r2, inv2, inv4, inv6;
        for (a = 0; a < 3; ++a) r[a] = X[a] - pts[3 * i + a];
        r2 = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
        inv2 = 1.0 / r2;
        inv4 = inv2 * inv2;
        inv6 = inv4 * inv2;
        *M += K[i] * inv2;
        for (a = 0; a < 3; ++a) {
            g[a] += -2.0 * K[i] * r[a] * inv4;
            for (b = 0; b < 3; ++b)
                H[3 * a + b] += K[i] * (8.0 * r[a] * r[b] * inv6 - (a == b ? 2.0 * inv4 : 0.0));
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Equilibrium (Sec. 2.2) and BGK collision with Guo forcing.                */
/* ------------------------------------------------------------------------ */

static double feq(const stencil_t* s, int i, double rho, const double u[3])
{
    double eu = s->e[i][0] * u[0] + s->e[i][1] * u[1] + s->e[i][2] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return s->w[i] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
}

/* Collide the pre-collision populations f[Q] of one node in place:
 * rho = sum f, u = (sum f e + F/2)/rho (Eq. blm_rhov, with the half-force
 * shift of Guo forcing; READING: the paper has no fluid body force),
 * f+ = f + (feq - f)/tau + (1 - 1/(2 tau)) w [3 (e - u) + 9 (e.u) e].F. */
static void collide(const stencil_t* s, double tau, const double F[3], double* f)
{
    double rho = 0.0, m[3] = {0.0, 0.0, 0.0}, u[3];
    int i, a;
    for (i = 0; i < s->Q; ++i) {
        rho += f[i];
        for (a = 0; a < 3; ++a) m[a] += f[i] * s->e[i][a];
    }
    for (a = 0; a < 3; ++a) u[a] = (m[a] + 0.5 * F[a]) / rho;
    for (i = 0; i < s->Q; ++i) {
        double eu = s->e[i][0] * u[0] + s->e[i][1] * u[1] + s->e[i][2] * u[2];
        double eF = s->e[i][0] * F[0] + s->e[i][1] * F[1] + s->e[i][2] * F[2];
        double uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
        double S = (1.0 - 0.5 / tau) * s->w[i] * (3.0 * (eF - uF) + 9.0 * eu * eF);
        double fe = feq(s, i, rho, u);
        f[i] = f[i] + (fe - f[i]) / tau + S;
    }
}

/* Density and velocity at a node from its post-collision populations.  The
 * collision keeps rho and turns the momentum sum into rho u + F/2, so
 * u = (sum f+ e - F/2)/rho is the velocity the collision used. */
static void moments_post(const stencil_t* s, const double* f, long N, long x, const double F[3],
                         double* rho, double u[3])
{
    double r = 0.0, m[3] = {0.0, 0.0, 0.0};
    int i, a;
    for (i = 0; i < s->Q; ++i) {
        double v = f[(long)i * N + x];
        r += v;
        for (a = 0; a < 3; ++a) m[a] += v * s->e[i][a];
    }
    *rho = r;
    for (a = 0; a < 3; ++a) u[a] = (m[a] - 0.5 * F[a]) / r;
}

void ora_moments(const int* dims, int Q, const double* F, const double* f, double* rho,
                 double* u)
{
    stencil_t s;
    long N = (long)dims[0] * dims[1] * dims[2], x;
    stencil_make(Q, &s);
    for (x = 0; x < N; ++x) {
        double uu[3];
        moments_post(&s, f, N, x, F, &rho[x], uu);
        u[3 * x + 0] = uu[0];
        u[3 * x + 1] = uu[1];
        u[3 * x + 2] = uu[2];
    }
}

void ora_init_equilibrium(const int* dims, int Q, double rho0, const double* u0, double* f)
{
    stencil_t s;
    long N = (long)dims[0] * dims[1] * dims[2], x;
    int i;
    stencil_make(Q, &s);
    for (i = 0; i < Q; ++i) {
        double v = feq(&s, i, rho0, u0);
        for (x = 0; x < N; ++x) f[(long)i * N + x] = v;
    }
}

/* ------------------------------------------------------------------------ */
/* Node classification (Sec. 2.3.1, Fig. ibb): a node is solid when some     */
/* particle has M_p >= c0_p there.  READING: ties M = c0 count as solid and   */
/* an overlap goes to the lowest particle index.                              */
/* ------------------------------------------------------------------------ */

static double particle_reach(int n, const double* pts, const double* K, double c0,
                             const double xp[3])
{
    /* M >= c0 needs sum K / min r^2 >= c0, i.e. some control point within
     * sqrt(sum K / c0). */
    double sk = 0.0, rmax = 0.0;
    int i, a;
    for (i = 0; i < n; ++i) {
        double r2 = 0.0;
        sk += K[i];
        for (a = 0; a < 3; ++a) r2 += (pts[3 * i + a] - xp[a]) * (pts[3 * i + a] - xp[a]);
        if (sqrt(r2) > rmax) rmax = sqrt(r2);
    }
    return rmax + sqrt(sk / c0);
}

void ora_classify(const int* dims, const int* per, int np, const int* off, const double* pts,
                  const double* K, const double* c0, const double* xp, int32_t* owner)
{
    grid_t g = grid_make(dims, per);
    long x;
    int p;
    for (x = 0; x < g.N; ++x) owner[x] = 0;
    /* Highest index first so that the lowest index is written last. */
    for (p = np - 1; p >= 0; --p) {
        const double* P = pts + 3 * (long)off[p];
        const double* Kp = K + off[p];
        int n = off[p + 1] - off[p];
        double R = particle_reach(n, P, Kp, c0[p], xp + 3 * p);
        int lo[3], hi[3], a, k;
        for (a = 0; a < 3; ++a) {
            lo[a] = (int)ceil(xp[3 * p + a] - R);
            hi[a] = (int)floor(xp[3 * p + a] + R);
            if (!g.per[a]) {
                if (lo[a] < 0) lo[a] = 0;
                if (hi[a] > g.n[a] - 1) hi[a] = g.n[a] - 1;
            }
        }
#pragma omp parallel for schedule(static)
        for (k = lo[2]; k <= hi[2]; ++k) {
            int i, j;
            for (j = lo[1]; j <= hi[1]; ++j)
                for (i = lo[0]; i <= hi[0]; ++i) {
                    int c[3] = {i, j, k}, w[3];
                    const int zero[3] = {0, 0, 0};
                    double X[3];
                    int b;
                    gshift(&g, c, zero, 0, w);
                    for (b = 0; b < 3; ++b) X[b] = image_coord(&g, b, w[b], xp[3 * p + b]);
                    if (metaball(n, P, Kp, X) >= c0[p]) owner[gidx(&g, w)] = p + 1;
                }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Link sets Gamma_j (Eq. mem) with q from Eq. (appq).                        */
/* ------------------------------------------------------------------------ */

enum { KIND_VIBB = 0, KIND_HALFWAY = 1, KIND_MISSING = 2 };
enum { TREAT_VIBB = 1, TREAT_MISSING = 2, TREAT_EXACT_Q = 4, TREAT_NEQ_SPLIT = 8 };

/* q of Eq. (calq): the root of g(q) = M(x_n + q e_d) - c0 on [0, 1], where
 * g(0) = M(x_n) - c0 < 0 <= g(1) = M(x_s) - c0.  Newton-Raphson from the
 * linear estimate of Eq. (appq), kept inside the bracket [a, b] of the sign
 * change (a step that leaves it is replaced by the midpoint); it stops when a
 * step is below 1e-13 or after 60 steps.  Along the line,
 * dM/dq = sum_i -2 K_i ((x - x_i) . e_d) / r_i^4.
 * READING (bit-exactness): every value is formed in the order written here,
 * with no contraction; the GPU computes the same sequence. */
static double exact_q(int n, const double* pts, const double* K, const double Xn[3],
                      const int e[3], double c0, double Mn, double Ms)
{
    double a = 0.0, b = 1.0;
    double q = (c0 - Mn) / (Ms - Mn);
    int it, i;
    for (it = 0; it < 60; ++it) {
        double M = 0.0, dM = 0.0, g, qn;
        for (i = 0; i < n; ++i) {
            double dx = (Xn[0] + q * (double)e[0]) - pts[3 * i + 0];
            double dy = (Xn[1] + q * (double)e[1]) - pts[3 * i + 1];
            double dz = (Xn[2] + q * (double)e[2]) - pts[3 * i + 2];
            double r2 = (dx * dx + dy * dy) + dz * dz;
            double t = K[i] / r2;
            double se = (dx * (double)e[0] + dy * (double)e[1]) + dz * (double)e[2];
            M = M + t;
            dM = dM - ((2.0 * t) * se) / r2;
        }
        g = M - c0;
        if (g == 0.0) break;
        if (g < 0.0)
            a = q;
        else
            b = q;
        qn = q - g / dM;
        if (!(qn > a && qn < b)) qn = 0.5 * (a + b);
        if (fabs(qn - q) < 1e-13) {
            q = qn;
            break;
        }
        q = qn;
    }
    return q;
}

/* Links in canonical order: particle, then solid node x_s, then direction d.
 *   x_n = x_s - e_d fluid           -> VIBB when x_ff = x_n - e_d is fluid and
 *                                      VIBB is on, else HALFWAY (treatment 1,
 *                                      Sec. 2.3.5);
 *   x_n beyond a wall, or solid of  -> MISSING (treatment 2, Sec. 2.3.5) when
 *   another particle                   M_j(x_n) < c0_j and treatment 2 is on.
 * q = (c0 - M(x_n)) / (M(x_s) - M(x_n)) for every kind (Eq. appq), or with
 * treatment bit 4 the root of Eq. (calq) by exact_q.
 * Returns the number of links; entries beyond `cap` are not stored. */
long ora_links(const int* dims, const int* per, int Q, int treat, int np, const int* off,
               const double* pts, const double* K, const double* c0, const double* xp,
               const int32_t* owner, long cap, int32_t* lnode, int8_t* ld, int8_t* lkind,
               int32_t* lpart, double* lq)
{
    grid_t g = grid_make(dims, per);
    stencil_t s;
    long count = 0, x, *start, *fill, *order;
    int p;
    stencil_make(Q, &s);
    /* bucket solid nodes by owner, ascending node index within each bucket */
    start = (long*)calloc((size_t)np + 1, sizeof(long));
    fill = (long*)calloc((size_t)np + 1, sizeof(long));
    for (x = 0; x < g.N; ++x)
        if (owner[x] > 0) start[owner[x]]++;
    for (p = 0; p < np; ++p) start[p + 1] += start[p];
    order = (long*)malloc(sizeof(long) * (size_t)(start[np] + 1));
    for (x = 0; x < g.N; ++x)
        if (owner[x] > 0) {
            int q = owner[x] - 1;
            order[start[q] + fill[q]++] = x;
        }
    for (p = 0; p < np; ++p) {
        const double* P = pts + 3 * (long)off[p];
        const double* Kp = K + off[p];
        int n = off[p + 1] - off[p];
        long t;
        for (t = start[p]; t < start[p + 1]; ++t) {
            long xs = order[t];
            int cs[3], d, a;
            double Xs[3], Ms;
            gcoord(&g, xs, cs);
            for (a = 0; a < 3; ++a) Xs[a] = image_coord(&g, a, cs[a], xp[3 * p + a]);
            Ms = metaball(n, P, Kp, Xs);
            for (d = 1; d < Q; ++d) {
                int cn[3], cff[3], kind = -1, inside;
                double Xn[3], Mn;
                inside = gshift(&g, cs, s.e[d], -1, cn);
                if (inside && owner[gidx(&g, cn)] == p + 1) continue; /* interior */
                if (inside && owner[gidx(&g, cn)] == 0) {
                    int ff = gshift(&g, cn, s.e[d], -1, cff) && owner[gidx(&g, cff)] == 0;
                    kind = ((treat & TREAT_VIBB) && ff) ? KIND_VIBB : KIND_HALFWAY;
                }
                /* coordinates of x_n seen from particle p (a virtual node
                 * beyond a wall keeps its raw coordinate) */
                for (a = 0; a < 3; ++a) {
                    int v = cs[a] - s.e[d][a];
                    Xn[a] = image_coord(&g, a, v, xp[3 * p + a]);
                }
                Mn = metaball(n, P, Kp, Xn);
                if (kind < 0) {
                    if (!(treat & TREAT_MISSING) || !(Mn < c0[p])) continue;
                    kind = KIND_MISSING;
                }
                if (count < cap) {
                    lnode[count] = (int32_t)xs;
                    ld[count] = (int8_t)d;
                    lkind[count] = (int8_t)kind;
                    lpart[count] = p;
                    lq[count] = (treat & TREAT_EXACT_Q)
                                    ? exact_q(n, P, Kp, Xn, s.e[d], c0[p], Mn, Ms)
                                    : (c0[p] - Mn) / (Ms - Mn);
                }
                ++count;
            }
        }
    }
    free(start);
    free(fill);
    free(order);
    return count;
}

/* ------------------------------------------------------------------------ */
/* One lattice step n -> n+1 (Secs. 2.2, 2.3.1, 2.3.2).                       */
/* ------------------------------------------------------------------------ */

static void cross(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Wall velocity u_w = v_j + w_j x (x_w - x_pj) (Sec. 2.3.1). */
static void wall_velocity(const double* v, const double* w, const double* xp, const double Xw[3],
                          double uw[3])
{
    double r[3], c[3];
    int a;
    for (a = 0; a < 3; ++a) r[a] = Xw[a] - xp[a];
    cross(w, r, c);
    for (a = 0; a < 3; ++a) uw[a] = v[a] + c[a];
}

/* Geometry of link l: the node x_n, its coordinates seen from the particle,
 * the wall point x_w = x_n + q e_d and the wall velocity there. */
static void link_geometry(const grid_t* g, const stencil_t* s, long xs, int d, int p, double q,
                          const double* xp, const double* v, const double* w, int cn[3],
                          int* inside, double Xw[3], double uw[3])
{
    int cs[3], a;
    gcoord(g, xs, cs);
    *inside = gshift(g, cs, s->e[d], -1, cn);
    for (a = 0; a < 3; ++a) {
        double Xn = image_coord(g, a, cs[a] - s->e[d][a], xp[3 * p + a]);
        Xw[a] = Xn + q * s->e[d][a];
    }
    wall_velocity(v + 3 * p, w + 3 * p, xp + 3 * p, Xw, uw);
}

/* VIBB (Sec. 2.3.1, Eqs. eqneq, neqd, rhod, u*_d, u**_d, u_d):
 *   f_{opp d}(x_f, t+1) = feq_d(rho_d, u_d) + fneq_d(x_d) + 6 w_d rho_f e_{opp d}.u_w
 * with
 *   fneq_d(x_d) = 2q (f+_d(x_f) - feq_d(x_f)) + (1-2q)(f+_d(x_ff) - feq_d(x_ff)),
 *   rho_d  = 2q rho_f + (1-2q) rho_ff          (q <= 1/2),   rho_f          (q > 1/2),
 *   u*_d   = 2q u_f + (1-2q) u_ff              (q <= 1/2),
 *            (1-q)/q u_f + (2q-1)/q u_w        (q > 1/2),
 *   u**_d  = (1-q)/(1+q) u_ff + 2q/(1+q) u_w,
 *   u_d    = u*_d / 3 + 2 u**_d / 3.
 * READING: rho_f, u_f, rho_ff, u_ff are the moments at time t of the node's
 * populations and feq(x) = feq(rho(x), u(x)); rho_f in the moving-wall term is
 * the local density at x_f.
 * Option (treatment bit 8, `split`): for q > 1/2, fneq_d(x_d) = f+_d(x_f) -
 * feq_d(x_f), the same case split that rho_d makes; without it the formula
 * above extrapolates with weights 2q > 1 and 1-2q < 0 and, at tau near 1/2,
 * a two-node gap between parallel faces amplifies the non-equilibrium part. */
static double vibb(const stencil_t* s, int d, double q, double fd_f, double rho_f,
                   const double u_f[3], double fd_ff, double rho_ff, const double u_ff[3],
                   const double uw[3], int split)
{
    double fneq, rho_d, us[3], uss[3], ud[3], eu;
    int a, db = s->opp[d];
    if (split && q > 0.5)
        fneq = fd_f - feq(s, d, rho_f, u_f);
    else
        fneq = 2.0 * q * (fd_f - feq(s, d, rho_f, u_f)) +
               (1.0 - 2.0 * q) * (fd_ff - feq(s, d, rho_ff, u_ff));
    rho_d = (q <= 0.5) ? 2.0 * q * rho_f + (1.0 - 2.0 * q) * rho_ff : rho_f;
    for (a = 0; a < 3; ++a) {
        us[a] = (q <= 0.5) ? 2.0 * q * u_f[a] + (1.0 - 2.0 * q) * u_ff[a]
                           : (1.0 - q) / q * u_f[a] + (2.0 * q - 1.0) / q * uw[a];
        uss[a] = (1.0 - q) / (1.0 + q) * u_ff[a] + 2.0 * q / (1.0 + q) * uw[a];
        ud[a] = us[a] / 3.0 + 2.0 * uss[a] / 3.0;
    }
    eu = s->e[db][0] * uw[0] + s->e[db][1] * uw[1] + s->e[db][2] * uw[2];
    return feq(s, d, rho_d, ud) + fneq + 6.0 * s->w[d] * rho_f * eu;
}

double ora_vibb(int Q, int d, double q, double fd_f, double rho_f, const double* u_f, double fd_ff,
                double rho_ff, const double* u_ff, const double* uw, int treat)
{
    stencil_t s;
    stencil_make(Q, &s);
    return vibb(&s, d, q, fd_f, rho_f, u_f, fd_ff, rho_ff, u_ff, uw, (treat & TREAT_NEQ_SPLIT) != 0);
}

/* Binary search of (node, d) among links [lo, hi) sorted by node then d. */
static long find_link(const int32_t* lnode, const int8_t* ld, long lo, long hi, long node, int d)
{
    while (lo < hi) {
        long mid = lo + (hi - lo) / 2;
        long key = (long)lnode[mid] * 32 + ld[mid];
        long want = node * 32 + d;
        if (key == want) return mid;
        if (key < want) lo = mid + 1;
        else hi = mid;
    }
    return -1;
}

/* One step: boundary unknowns from f+(t), hydrodynamic force and torque per
 * particle (Eqs. mem, fh_s_issue, th_s_issue), then pull-streaming and
 * collision of every fluid node into fout.  Domain walls use static halfway
 * bounce-back.  Populations of solid nodes are copied through unchanged.
 * Returns 0, or -1 when a solid source has no link. */
int ora_step(const int* dims, const int* per, int Q, int treat, double tau, const double* Fb, double rho0,
             const double* f, const int32_t* owner, long nl, const int32_t* lnode, const int8_t* ld,
             const int8_t* lkind, const int32_t* lpart, const double* lq, int np, const double* xp,
             const double* v, const double* w, double* fout, double* unk, double* Fh, double* Th)
{
    grid_t g = grid_make(dims, per);
    stencil_t s;
    long l, x, *seg;
    int p, bad = 0;
    stencil_make(Q, &s);

    /* 1. unknown populations of every fluid-side link */
#pragma omp parallel for schedule(static)
    for (l = 0; l < nl; ++l) {
        int cn[3], cff[3], inside, d = ld[l], pp = lpart[l];
        double Xw[3], uw[3];
        unk[l] = NAN;
        if (lkind[l] == KIND_MISSING) continue;
        link_geometry(&g, &s, lnode[l], d, pp, lq[l], xp, v, w, cn, &inside, Xw, uw);
        {
            long xf = gidx(&g, cn);
            double rho_f, u_f[3], fd_f = f[(long)d * g.N + xf];
            moments_post(&s, f, g.N, xf, Fb, &rho_f, u_f);
            if (lkind[l] == KIND_VIBB) {
                long xff;
                double rho_ff, u_ff[3];
                gshift(&g, cn, s.e[d], -1, cff);
                xff = gidx(&g, cff);
                moments_post(&s, f, g.N, xff, Fb, &rho_ff, u_ff);
                unk[l] = vibb(&s, d, lq[l], fd_f, rho_f, u_f, f[(long)d * g.N + xff], rho_ff,
                              u_ff, uw, (treat & TREAT_NEQ_SPLIT) != 0);
            } else {
                /* treatment 1: halfway bounce-back with the moving-wall term */
                int db = s.opp[d];
                double eu = s.e[db][0] * uw[0] + s.e[db][1] * uw[1] + s.e[db][2] * uw[2];
                unk[l] = fd_f + 6.0 * s.w[d] * rho_f * eu;
            }
        }
    }

    /* 2. Galilean-invariant momentum exchange, summed serially in link order.
     * READING: the outgoing population is f+_d(x_f, t) and the incoming one
     * the reconstructed f_{opp d}(x_f, t+1). */
    for (p = 0; p < np; ++p)
        for (l = 0; l < 3; ++l) Fh[3 * p + l] = Th[3 * p + l] = 0.0;
    for (l = 0; l < nl; ++l) {
        int cn[3], inside, d = ld[l], db = s.opp[d], pp = lpart[l], a;
        double Xw[3], uw[3], out, in, term[3], r[3], tq[3];
        link_geometry(&g, &s, lnode[l], d, pp, lq[l], xp, v, w, cn, &inside, Xw, uw);
        if (lkind[l] == KIND_MISSING) {
            /* treatment 2: equilibrium at (rho0, u_w) on both sides */
            out = feq(&s, d, rho0, uw);
            in = feq(&s, db, rho0, uw);
        } else {
            out = f[(long)d * g.N + gidx(&g, cn)];
            in = unk[l];
        }
        for (a = 0; a < 3; ++a)
            term[a] = (s.e[d][a] - uw[a]) * out - (s.e[db][a] - uw[a]) * in;
        for (a = 0; a < 3; ++a) r[a] = Xw[a] - xp[3 * pp + a];
        cross(r, term, tq);
        for (a = 0; a < 3; ++a) {
            Fh[3 * pp + a] += term[a];
            Th[3 * pp + a] += tq[a];
        }
    }

    /* 3. streaming (pull) and collision */
    seg = (long*)calloc((size_t)np + 1, sizeof(long));
    for (l = 0; l < nl; ++l) seg[lpart[l] + 1]++;
    for (p = 0; p < np; ++p) seg[p + 1] += seg[p];
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (x = 0; x < g.N; ++x) {
        double fl[19];
        int c[3], i;
        if (owner[x] != 0) {
            for (i = 0; i < Q; ++i) fout[(long)i * g.N + x] = f[(long)i * g.N + x];
            continue;
        }
        gcoord(&g, x, c);
        for (i = 0; i < Q; ++i) {
            int cs[3];
            if (!gshift(&g, c, s.e[i], -1, cs)) {
                fl[i] = f[(long)s.opp[i] * g.N + x]; /* domain wall */
            } else {
                long src = gidx(&g, cs);
                int o = owner[src];
                if (o == 0) {
                    fl[i] = f[(long)i * g.N + src];
                } else {
                    /* solid source: the link (x_s = src, d = opp i) */
                    long k = find_link(lnode, ld, seg[o - 1], seg[o], src, s.opp[i]);
                    if (k < 0) {
                        bad = 1;
                        fl[i] = NAN;
                    } else {
                        fl[i] = unk[k];
                    }
                }
            }
        }
        collide(&s, tau, Fb, fl);
        for (i = 0; i < Q; ++i) fout[(long)i * g.N + x] = fl[i];
    }
    free(seg);
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Local refilling of new fluid nodes (Sec. 2.3.3).                          */
/* ------------------------------------------------------------------------ */

/* For every node solid at t and fluid at t+1 (ascending index), fill
 *   f_i = f+_i(x - e_i, t)                       if x - e_i was fluid at t,
 *   f_i = f+_{opp i}(x + e_i, t) + 6 w_i rho0 e_i.u_new
 *                                                 else if x + e_i was fluid,
 *   f_i = feq_i(rho0, u_new)                      otherwise,
 * u_new = v_j + w_j x (x_new - x_pj) of the particle j that covered the node,
 * then collide and store into fcur.  READING: "streamed" means the upstream
 * neighbour was fluid at t; rho0 stands in for the local density.
 * Returns the number of refilled nodes; nodes beyond cap are not listed. */
long ora_refill(const int* dims, const int* per, int Q, double tau, const double* Fb, double rho0,
                const double* fprev, const int32_t* own_prev, const int32_t* own_new, int np,
                const double* xp, const double* v, const double* w, double* fcur, long cap,
                int32_t* nodes)
{
    grid_t g = grid_make(dims, per);
    stencil_t s;
    long x, count = 0;
    (void)np;
    stencil_make(Q, &s);
    for (x = 0; x < g.N; ++x) {
        double fl[19], X[3], un[3];
        int c[3], i, a, p;
        if (!(own_prev[x] != 0 && own_new[x] == 0)) continue;
        if (count < cap) nodes[count] = (int32_t)x;
        ++count;
        p = own_prev[x] - 1;
        gcoord(&g, x, c);
        for (a = 0; a < 3; ++a) X[a] = image_coord(&g, a, c[a], xp[3 * p + a]);
        wall_velocity(v + 3 * p, w + 3 * p, xp + 3 * p, X, un);
        for (i = 0; i < Q; ++i) {
            int cu[3], cd[3];
            if (i > 0 && gshift(&g, c, s.e[i], -1, cu) && own_prev[gidx(&g, cu)] == 0) {
                fl[i] = fprev[(long)i * g.N + gidx(&g, cu)];
            } else if (i > 0 && gshift(&g, c, s.e[i], 1, cd) && own_prev[gidx(&g, cd)] == 0) {
                double eu = s.e[i][0] * un[0] + s.e[i][1] * un[1] + s.e[i][2] * un[2];
                fl[i] = fprev[(long)s.opp[i] * g.N + gidx(&g, cd)] + 6.0 * s.w[i] * rho0 * eu;
            } else {
                fl[i] = feq(&s, i, rho0, un);
            }
        }
        collide(&s, tau, Fb, fl);
        for (i = 0; i < Q; ++i) fcur[(long)i * g.N + x] = fl[i];
    }
    return count;
}

/* ------------------------------------------------------------------------ */
/* Metaball DEM (Sec. 2.1): Newton-Euler with velocity Verlet, linear spring-  */
/* dashpot normal force, Coulomb-limited tangential spring, metaball-metaball */
/* and metaball-plane contacts, relative gravity (Sec. 3.1).                 */
/* ------------------------------------------------------------------------ */

/* Packed parameters, in order. */
enum {
    P_KN, P_ETAN, P_KT, P_ETAT, P_MU, P_CTOL, P_NTOL, P_NITER, P_G0, P_G1, P_G2, P_RHOF, P_COUNT
};
#define HIST 8 /* doubles per contact-history record: active, xi[3], warm[3], pad */

static void quat_to_R(const double* q, double R[9])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
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

static void matvec(const double R[9], const double a[3], double b[3])
{
    int i;
    for (i = 0; i < 3; ++i) b[i] = R[3 * i] * a[0] + R[3 * i + 1] * a[1] + R[3 * i + 2] * a[2];
}

static void matTvec(const double R[9], const double a[3], double b[3])
{
    int i;
    for (i = 0; i < 3; ++i) b[i] = R[i] * a[0] + R[3 + i] * a[1] + R[6 + i] * a[2];
}

static double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* solve H dx = -g for a 3x3 symmetric system by cofactors */
static int solve3(const double H[9], const double g[3], double dx[3])
{
    double c[9], det;
    int i;
    c[0] = H[4] * H[8] - H[5] * H[7];
    c[1] = H[2] * H[7] - H[1] * H[8];
    c[2] = H[1] * H[5] - H[2] * H[4];
    c[3] = H[5] * H[6] - H[3] * H[8];
    c[4] = H[0] * H[8] - H[2] * H[6];
    c[5] = H[2] * H[3] - H[0] * H[5];
    c[6] = H[3] * H[7] - H[4] * H[6];
    c[7] = H[1] * H[6] - H[0] * H[7];
    c[8] = H[0] * H[4] - H[1] * H[3];
    det = H[0] * c[0] + H[1] * c[3] + H[2] * c[6];
    if (!(fabs(det) > 0.0) || !isfinite(det)) return -1;
    for (i = 0; i < 3; ++i) dx[i] = -(c[3 * i] * g[0] + c[3 * i + 1] * g[1] + c[3 * i + 2] * g[2]) / det;
    return 0;
}

typedef struct {
    int n;
    const double* pts; /* world control points (already shifted to an image) */
    const double* K;
} mb_t;

/* Linear spring-dashpot normal force and Coulomb-limited tangential spring
 * (Sec. 2.1.1).  v_rel is the velocity of body i relative to body j at the
 * contact point, n points from j to i.  READING: the normal force is clamped
 * at zero and a sliding spring is rescaled to |k_t xi| = mu F_n. */
static void contact_force(const double* prm, double delta, const double n[3], const double vrel[3],
                          double dt, double* hist, double Fi[3])
{
    double vn = dot3(vrel, n), vt[3], xi[3], Ft[3], Fn, xin, ftn;
    int a;
    Fn = prm[P_KN] * delta - prm[P_ETAN] * vn;
    if (Fn < 0.0) Fn = 0.0;
    for (a = 0; a < 3; ++a) vt[a] = vrel[a] - vn * n[a];
    xin = dot3(hist + 1, n);
    for (a = 0; a < 3; ++a) xi[a] = hist[1 + a] - xin * n[a] + vt[a] * dt;
    for (a = 0; a < 3; ++a) Ft[a] = -prm[P_KT] * xi[a] - prm[P_ETAT] * vt[a];
    ftn = sqrt(dot3(Ft, Ft));
    if (ftn > prm[P_MU] * Fn && ftn > 0.0) {
        double sc = prm[P_MU] * Fn / ftn;
        for (a = 0; a < 3; ++a) {
            Ft[a] *= sc;
            xi[a] = -(Ft[a] + prm[P_ETAT] * vt[a]) / prm[P_KT];
        }
    }
    for (a = 0; a < 3; ++a) {
        hist[1 + a] = xi[a];
        Fi[a] = Fn * n[a] + Ft[a];
    }
}

/* Metaball-metaball contact (Eqs. opt, grad, cp, k0, contactprop).  Solves
 * grad(M_i + M_j) = 0 by Newton-Raphson from the previous point or, for a new
 * pair, from the midpoint of the closest control-point pair; requires
 * M > ctol for both bodies there.  READING: the contact point is the middle
 * of the overlap, x_c_i - (R_si - delta/2) n.
 * READING (separation): at the stationary point grad M_i = -grad M_j, so the
 * two projected surface points of Eq. cp lie on one line, whose direction
 * n = (grad M_i - grad M_j)/|...| points from body j to body i.  The
 * separation is the signed length (x_c_i - x_c_j).n: equal to the norm of
 * Eq. contactprop while x_m is outside both internal bodies (the constraint
 * M < 1 of Eq. opt), and negative once x_m has entered one of them, which
 * happens before the bodies touch when two flat faces meet at an angle;
 * dropping the contact there (the literal constraint) lets such bodies pass
 * into each other.  A point whose overlap would exceed 2 (R_si + R_sj) is
 * not a contact (a stationary point inside one body, where the projection
 * of Eq. k0 does not hold). */
static int pair_geometry(const double* prm, const mb_t* A, const mb_t* B, double rsA, double rsB,
                         const double* warm, int has_warm, double xm_out[3], double* delta,
                         double n[3], double xcp[3])
{
    double x[3], g[3], H[9], gA[3], HA[9], gB[3], HB[9], MA, MB, dx[3];
    int it, a, conv = 0;
    int niter = (int)prm[P_NITER];
    if (has_warm) {
        for (a = 0; a < 3; ++a) x[a] = warm[a];
    } else {
        double best = INFINITY;
        int i, j;
        for (i = 0; i < A->n; ++i)
            for (j = 0; j < B->n; ++j) {
                double d2 = 0.0;
                for (a = 0; a < 3; ++a)
                    d2 += (A->pts[3 * i + a] - B->pts[3 * j + a]) * (A->pts[3 * i + a] - B->pts[3 * j + a]);
                if (d2 < best) {
                    best = d2;
                    for (a = 0; a < 3; ++a) x[a] = 0.5 * (A->pts[3 * i + a] + B->pts[3 * j + a]);
                }
            }
    }
    for (it = 0; it < niter; ++it) {
        metaball_d2(A->n, A->pts, A->K, x, &MA, gA, HA);
        metaball_d2(B->n, B->pts, B->K, x, &MB, gB, HB);
        for (a = 0; a < 3; ++a) g[a] = gA[a] + gB[a];
        for (a = 0; a < 9; ++a) H[a] = HA[a] + HB[a];
        if (solve3(H, g, dx)) break;
        for (a = 0; a < 3; ++a) x[a] += dx[a];
        if (sqrt(dot3(dx, dx)) < prm[P_NTOL]) {
            conv = 1;
            break;
        }
    }
    if (!conv) return 0;
    for (a = 0; a < 3; ++a) xm_out[a] = x[a];
    metaball_d2(A->n, A->pts, A->K, x, &MA, gA, HA);
    metaball_d2(B->n, B->pts, B->K, x, &MB, gB, HB);
    if (!(MA > prm[P_CTOL] && MB > prm[P_CTOL])) return 0;
    {
        double qA = (1.0 - MA) / dot3(gA, gA), qB = (1.0 - MB) / dot3(gB, gB);
        double xa[3], xb[3], dd[3], u[3], un, sep;
        for (a = 0; a < 3; ++a) {
            xa[a] = x[a] + qA * gA[a];
            xb[a] = x[a] + qB * gB[a];
            dd[a] = xa[a] - xb[a];
            u[a] = gA[a] - gB[a];
        }
        un = sqrt(dot3(u, u));
        if (!(un > 0.0)) return 0;
        for (a = 0; a < 3; ++a) n[a] = u[a] / un;
        sep = dot3(dd, n);
        *delta = rsA + rsB - sep;
        if (!(*delta <= 2.0 * (rsA + rsB))) return 0;
        for (a = 0; a < 3; ++a) xcp[a] = xa[a] - (rsA - 0.5 * (*delta)) * n[a];
    }
    return 1;
}

/* Metaball-plane contact (Eqs. metawall, metawallcp, k, contactprop2) for an
 * axis-aligned wall: Newton on the two in-plane gradient components, from
 * the previous point or the control point nearest the wall projected onto it.
 * READING: with the wall normal n_w pointing into the domain, the overlap is
 * R_s - (x_cm - x_cw).n_w and the normal is n_w (equal to the paper's form
 * when grad M is normal to the wall, as at the Newton solution); the contact
 * point is the middle of the overlap, x_cw - delta/2 n_w. */
static int wall_geometry(const double* prm, const mb_t* A, double rs, int axis, double plane,
                         double sgn, const double* warm, int has_warm, double xcw_out[3],
                         double* delta, double n[3], double xcp[3])
{
    int t1 = (axis + 1) % 3, t2 = (axis + 2) % 3, it, a, conv = 0;
    int niter = (int)prm[P_NITER];
    double x[3], M, g[3], H[9];
    if (has_warm) {
        for (a = 0; a < 3; ++a) x[a] = warm[a];
    } else {
        double best = INFINITY;
        int i;
        for (i = 0; i < A->n; ++i) {
            double d = fabs(A->pts[3 * i + axis] - plane);
            if (d < best) {
                best = d;
                for (a = 0; a < 3; ++a) x[a] = A->pts[3 * i + a];
            }
        }
    }
    x[axis] = plane;
    for (it = 0; it < niter; ++it) {
        double h11, h12, h22, det, d1, d2;
        metaball_d2(A->n, A->pts, A->K, x, &M, g, H);
        h11 = H[3 * t1 + t1];
        h12 = H[3 * t1 + t2];
        h22 = H[3 * t2 + t2];
        det = h11 * h22 - h12 * h12;
        if (!(fabs(det) > 0.0) || !isfinite(det)) break;
        d1 = -(h22 * g[t1] - h12 * g[t2]) / det;
        d2 = -(-h12 * g[t1] + h11 * g[t2]) / det;
        x[t1] += d1;
        x[t2] += d2;
        if (sqrt(d1 * d1 + d2 * d2) < prm[P_NTOL]) {
            conv = 1;
            break;
        }
    }
    if (!conv) return 0;
    for (a = 0; a < 3; ++a) xcw_out[a] = x[a];
    metaball_d2(A->n, A->pts, A->K, x, &M, g, H);
    if (!(sgn * g[axis] > 0.0)) return 0; /* gradient must point into the domain */
    {
        double qR = (1.0 - M) / dot3(g, g), s;
        s = sgn * (qR * g[axis]);
        *delta = rs - s;
        for (a = 0; a < 3; ++a) n[a] = 0.0;
        n[axis] = sgn;
        for (a = 0; a < 3; ++a) xcp[a] = x[a] - 0.5 * (*delta) * n[a];
    }
    return 1;
}

static double body_reach(int n, const double* bpts, const double* K)
{
    double sk = 0.0, r = 0.0;
    int i;
    for (i = 0; i < n; ++i) {
        double d = sqrt(bpts[3 * i] * bpts[3 * i] + bpts[3 * i + 1] * bpts[3 * i + 1] +
                        bpts[3 * i + 2] * bpts[3 * i + 2]);
        sk += K[i];
        if (d > r) r = d;
    }
    return r + sqrt(sk);
}

static void refresh_world(int np, const int* off, const double* bpts, const double* pos,
                          const double* quat, double* wpts)
{
    int p, i;
    for (p = 0; p < np; ++p) {
        double R[9];
        quat_to_R(quat + 4 * p, R);
        for (i = off[p]; i < off[p + 1]; ++i) {
            double r[3];
            int a;
            matvec(R, bpts + 3 * i, r);
            for (a = 0; a < 3; ++a) wpts[3 * i + a] = pos[3 * p + a] + r[a];
        }
    }
}

/* Contact forces and torques on every particle at the current pose. */
static void contacts(int np, const int* off, const double* bpts, const double* K,
                     const double* rs, const double* pos, const double* vel, const double* om,
                     const double* wpts, double* hpp, double* hpw, const double* prm,
                     const grid_t* g, double dt, double* Fc, double* Tc)
{
    int i, j, a;
    double* shifted;
    int maxn = 0;
    for (i = 0; i < np; ++i)
        if (off[i + 1] - off[i] > maxn) maxn = off[i + 1] - off[i];
    shifted = (double*)malloc(sizeof(double) * 3 * (size_t)(maxn + 1));
    for (i = 0; i < 3 * np; ++i) Fc[i] = Tc[i] = 0.0;
    /* pairs, i < j */
    for (i = 0; i < np; ++i) {
        double ri = body_reach(off[i + 1] - off[i], bpts + 3 * (long)off[i], K + off[i]);
        for (j = i + 1; j < np; ++j) {
            double rj = body_reach(off[j + 1] - off[j], bpts + 3 * (long)off[j], K + off[j]);
            double* h = hpp + ((long)i * np + j) * HIST;
            double sh[3], dvec[3], dist, xm[3], delta, n[3], xcp[3], warm[3];
            mb_t A, B;
            int k, ok;
            for (a = 0; a < 3; ++a) {
                double d = pos[3 * j + a] - pos[3 * i + a];
                sh[a] = 0.0;
                if (g->per[a]) {
                    double L = g->n[a];
                    if (d > 0.5 * L) sh[a] = -L;
                    else if (d < -0.5 * L) sh[a] = L;
                }
                dvec[a] = d + sh[a];
            }
            dist = sqrt(dot3(dvec, dvec));
            if (dist > ri + rj + rs[i] + rs[j]) {
                for (k = 0; k < HIST; ++k) h[k] = 0.0;
                continue;
            }
            for (k = off[j]; k < off[j + 1]; ++k)
                for (a = 0; a < 3; ++a) shifted[3 * (k - off[j]) + a] = wpts[3 * k + a] + sh[a];
            A.n = off[i + 1] - off[i];
            A.pts = wpts + 3 * (long)off[i];
            A.K = K + off[i];
            B.n = off[j + 1] - off[j];
            B.pts = shifted;
            B.K = K + off[j];
            for (a = 0; a < 3; ++a) warm[a] = pos[3 * i + a] + h[4 + a];
            ok = pair_geometry(prm, &A, &B, rs[i], rs[j], warm, h[0] != 0.0, xm, &delta, n, xcp);
            if (!ok) {
                for (k = 0; k < HIST; ++k) h[k] = 0.0;
                continue;
            }
            h[0] = 1.0;
            for (a = 0; a < 3; ++a) h[4 + a] = xm[a] - pos[3 * i + a];
            if (delta <= 0.0) {
                h[1] = h[2] = h[3] = 0.0;
                continue;
            }
            {
                double ra[3], rb[3], ca[3], cb[3], vrel[3], Fi[3], t[3];
                for (a = 0; a < 3; ++a) {
                    ra[a] = xcp[a] - pos[3 * i + a];
                    rb[a] = xcp[a] - (pos[3 * j + a] + sh[a]);
                }
                cross(om + 3 * i, ra, ca);
                cross(om + 3 * j, rb, cb);
                for (a = 0; a < 3; ++a)
                    vrel[a] = (vel[3 * i + a] + ca[a]) - (vel[3 * j + a] + cb[a]);
                contact_force(prm, delta, n, vrel, dt, h, Fi);
                for (a = 0; a < 3; ++a) {
                    Fc[3 * i + a] += Fi[a];
                    Fc[3 * j + a] -= Fi[a];
                }
                cross(ra, Fi, t);
                for (a = 0; a < 3; ++a) Tc[3 * i + a] += t[a];
                cross(rb, Fi, t);
                for (a = 0; a < 3; ++a) Tc[3 * j + a] -= t[a];
            }
        }
    }
    /* walls of every non-periodic axis, at -1/2 and n - 1/2 */
    for (i = 0; i < np; ++i) {
        double ri = body_reach(off[i + 1] - off[i], bpts + 3 * (long)off[i], K + off[i]);
        int ax, side;
        for (ax = 0; ax < 3; ++ax) {
            if (g->per[ax]) continue;
            for (side = 0; side < 2; ++side) {
                double plane = side ? g->n[ax] - 0.5 : -0.5, sgn = side ? -1.0 : 1.0;
                double* h = hpw + ((long)i * 6 + 2 * ax + side) * HIST;
                double xcw[3], delta, n[3], xcp[3], warm[3];
                mb_t A;
                int k, ok;
                if (sgn * (pos[3 * i + ax] - plane) > ri + rs[i]) {
                    for (k = 0; k < HIST; ++k) h[k] = 0.0;
                    continue;
                }
                A.n = off[i + 1] - off[i];
                A.pts = wpts + 3 * (long)off[i];
                A.K = K + off[i];
                for (a = 0; a < 3; ++a) warm[a] = pos[3 * i + a] + h[4 + a];
                ok = wall_geometry(prm, &A, rs[i], ax, plane, sgn, warm, h[0] != 0.0, xcw, &delta,
                                   n, xcp);
                if (!ok) {
                    for (k = 0; k < HIST; ++k) h[k] = 0.0;
                    continue;
                }
                h[0] = 1.0;
                for (a = 0; a < 3; ++a) h[4 + a] = xcw[a] - pos[3 * i + a];
                if (delta <= 0.0) {
                    h[1] = h[2] = h[3] = 0.0;
                    continue;
                }
                {
                    double ra[3], ca[3], vrel[3], Fi[3], t[3];
                    for (a = 0; a < 3; ++a) ra[a] = xcp[a] - pos[3 * i + a];
                    cross(om + 3 * i, ra, ca);
                    for (a = 0; a < 3; ++a) vrel[a] = vel[3 * i + a] + ca[a];
                    contact_force(prm, delta, n, vrel, dt, h, Fi);
                    for (a = 0; a < 3; ++a) Fc[3 * i + a] += Fi[a];
                    cross(ra, Fi, t);
                    for (a = 0; a < 3; ++a) Tc[3 * i + a] += t[a];
                }
            }
        }
    }
    free(shifted);
}

/* Half kick of the translational and rotational velocities with the total
 * force F = F^h + (m - rho_f V) g + F^c and torque T = T^h + T^c.  Rotation
 * follows Euler's equations in the principal body frame (Sec. 2.1.1):
 * I dw_b/dt = T_b - w_b x (I w_b).  READING: the integrator is not given; the
 * first half kick evaluates the gyroscopic term at the current w_b, the
 * second at the new w_b by three fixed-point sweeps, which makes the pair a
 * second-order (trapezoidal) update. */
static void half_kick(int p, const double* mass, const double* volume, const double* inertia,
                      const double* quat, double* vel, double* om, const double* Fh,
                      const double* Th, const double* Fc, const double* Tc, const double* prm,
                      double h, int implicit)
{
    double R[9], T[3], wb[3], w0[3], Tb[3], Iw[3], c[3];
    int a, it;
    double mrel = mass[p] - prm[P_RHOF] * volume[p];
    for (a = 0; a < 3; ++a) {
        double F = Fh[3 * p + a] + mrel * prm[P_G0 + a] + Fc[3 * p + a];
        vel[3 * p + a] += h * F / mass[p];
        T[a] = Th[3 * p + a] + Tc[3 * p + a];
    }
    quat_to_R(quat + 4 * p, R);
    matTvec(R, om + 3 * p, w0);
    matTvec(R, T, Tb);
    for (a = 0; a < 3; ++a) wb[a] = w0[a];
    for (it = 0; it < (implicit ? 4 : 1); ++it) {
        double nw[3];
        for (a = 0; a < 3; ++a) Iw[a] = inertia[3 * p + a] * wb[a];
        cross(wb, Iw, c);
        for (a = 0; a < 3; ++a) nw[a] = w0[a] + h * (Tb[a] - c[a]) / inertia[3 * p + a];
        for (a = 0; a < 3; ++a) wb[a] = nw[a];
    }
    matvec(R, wb, om + 3 * p);
}

/* n_sub velocity-Verlet substeps of length dt with F^h, T^h frozen
 * (sub-cycling, Sec. 2.3.4).  Positions on periodic axes stay in [0, n).
 * The orientation advances by the rotation of angle |w| dt about w:
 * q <- (cos(|w|dt/2), sin(|w|dt/2) w/|w|) q, renormalised.  fc, tc hold the
 * contact force and torque of the last evaluation (carried between calls). */
void ora_dem_step(int np, const int* off, const double* bpts, const double* K, const double* rs,
                  const double* mass, const double* volume, const double* inertia, double* pos,
                  double* quat, double* vel, double* om, double* wpts, double* fc, double* tc,
                  const double* Fh, const double* Th, double* hpp, double* hpw, const double* prm,
                  const int* dims, const int* per, int n_sub, double dt)
{
    grid_t g = grid_make(dims, per);
    int s, p, a;
    for (s = 0; s < n_sub; ++s) {
        for (p = 0; p < np; ++p) {
            double wn, dq[4], q0[4], qn[4], nrm;
            half_kick(p, mass, volume, inertia, quat, vel, om, Fh, Th, fc, tc, prm, 0.5 * dt, 0);
            for (a = 0; a < 3; ++a) {
                pos[3 * p + a] += dt * vel[3 * p + a];
                if (g.per[a]) {
                    if (pos[3 * p + a] >= g.n[a]) pos[3 * p + a] -= g.n[a];
                    else if (pos[3 * p + a] < 0.0) pos[3 * p + a] += g.n[a];
                }
            }
            wn = sqrt(dot3(om + 3 * p, om + 3 * p));
            dq[0] = cos(0.5 * wn * dt);
            for (a = 0; a < 3; ++a) dq[1 + a] = wn > 0.0 ? sin(0.5 * wn * dt) * om[3 * p + a] / wn : 0.0;
            for (a = 0; a < 4; ++a) q0[a] = quat[4 * p + a];
            qn[0] = dq[0] * q0[0] - dq[1] * q0[1] - dq[2] * q0[2] - dq[3] * q0[3];
            qn[1] = dq[0] * q0[1] + dq[1] * q0[0] + dq[2] * q0[3] - dq[3] * q0[2];
            qn[2] = dq[0] * q0[2] - dq[1] * q0[3] + dq[2] * q0[0] + dq[3] * q0[1];
            qn[3] = dq[0] * q0[3] + dq[1] * q0[2] - dq[2] * q0[1] + dq[3] * q0[0];
            nrm = sqrt(qn[0] * qn[0] + qn[1] * qn[1] + qn[2] * qn[2] + qn[3] * qn[3]);
            for (a = 0; a < 4; ++a) quat[4 * p + a] = qn[a] / nrm;
        }
        refresh_world(np, off, bpts, pos, quat, wpts);
        contacts(np, off, bpts, K, rs, pos, vel, om, wpts, hpp, hpw, prm, &g, dt, fc, tc);
        for (p = 0; p < np; ++p)
            half_kick(p, mass, volume, inertia, quat, vel, om, Fh, Th, fc, tc, prm, 0.5 * dt, 1);
    }
}

void ora_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int ora_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

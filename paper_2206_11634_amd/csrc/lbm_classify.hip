// FP64 geometry kernels of libmdlbm for gfx950: node classification against
// the metaball bodies {M_p >= c0_p} (Eq. metaball), link records with the
// wall fraction q of Eq. (appq), and detection of nodes to refill (Sec. 2.3.3).
//
// These decisions must be bit-identical to any other IEEE implementation of
// the same convention, so this file is built with -ffp-contract=off and every
// metaball value is evaluated as
//     r2 = (dx*dx + dy*dy) + dz*dz,   M = ((0 + K_0/r2_0) + K_1/r2_1) + ...
// in IEEE double with correctly rounded division.
//
// Work is organised per particle: a particle's nodes lie in a fixed-size box
// of (2h+1)^3 nodes around floor(x_p), walked in tiles of 256 box cells, one
// workgroup per (tile, particle); cells outside the particle's bounding ball
// are skipped.  Box coordinates are unwrapped, so on a
// periodic axis they are exactly the node's image nearest x_p (the box is
// narrower than half the period).
#pragma clang fp contract(off)

#include "lbm_internal.h"

namespace mdlbm {
namespace {

constexpr int kMaxCtrl = 64;

__device__ __forceinline__ int ex_d(int d)
{
    return (d == 1 || d == 7 || d == 9 || d == 11 || d == 13) ? 1
         : (d == 2 || d == 8 || d == 10 || d == 12 || d == 14) ? -1 : 0;
}
__device__ __forceinline__ int ey_d(int d)
{
    return (d == 3 || d == 7 || d == 10 || d == 15 || d == 17) ? 1
         : (d == 4 || d == 8 || d == 9 || d == 16 || d == 18) ? -1 : 0;
}
__device__ __forceinline__ int ez_d(int d)
{
    return (d == 5 || d == 11 || d == 14 || d == 15 || d == 18) ? 1
         : (d == 6 || d == 12 || d == 13 || d == 16 || d == 17) ? -1 : 0;
}

// Control points (x, y, z, K) of particle p staged in LDS.
__device__ __forceinline__ int stage_ctrl(const PartDev& P, int p, double* sp)
{
    const int a = P.off[p], n = min(P.off[p + 1] - a, kMaxCtrl);
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        sp[4 * i + 0] = P.wpts[3 * (int64_t)(a + i) + 0];
        sp[4 * i + 1] = P.wpts[3 * (int64_t)(a + i) + 1];
        sp[4 * i + 2] = P.wpts[3 * (int64_t)(a + i) + 2];
        sp[4 * i + 3] = P.K[a + i];
    }
    __syncthreads();
    return n;
}

__device__ __forceinline__ double metaball(const double* sp, int n, double X, double Y, double Z)
{
    double M = 0.0;
    for (int i = 0; i < n; ++i) {
        const double dx = X - sp[4 * i + 0];
        const double dy = Y - sp[4 * i + 1];
        const double dz = Z - sp[4 * i + 2];
        const double r2 = (dx * dx + dy * dy) + dz * dz;
        M = M + sp[4 * i + 3] / r2;
    }
    return M;
}

// Unwrapped box coordinates of box cell t of particle p, and whether the node
// exists (periodic axes wrap, other axes clip).
struct BoxCell {
    int ii[3];   // unwrapped coordinates
    int c[3];    // wrapped coordinates
    bool in;
};

__device__ __forceinline__ BoxCell box_cell(const int* origin, int t, const BoxSpec& b,
                                            const Geom& g)
{
    BoxCell r;
    const int bx = t % b.S, by = (t / b.S) % b.S, bz = t / (b.S * b.S);
    r.ii[0] = origin[0] + bx;
    r.ii[1] = origin[1] + by;
    r.ii[2] = origin[2] + bz;
    r.in = t < b.vol;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int v = r.ii[a];
        if (v < 0 || v >= g.n[a]) {
            if (g.per[a])
                v = ((v % g.n[a]) + g.n[a]) % g.n[a];
            else
                r.in = false;
        }
        r.c[a] = v;
    }
    return r;
}

__device__ __forceinline__ uint32_t node_idx(const int c[3], const Geom& g)
{
    return (uint32_t)c[0] + (uint32_t)g.n[0] * ((uint32_t)c[1] + (uint32_t)g.n[1] * (uint32_t)c[2]);
}

// Neighbour c - e (wrapped); false when it lies beyond a wall.
__device__ __forceinline__ bool neighbour(const int c[3], int ex, int ey, int ez, const Geom& g,
                                          int out[3])
{
    const int e[3] = {ex, ey, ez};
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int v = c[a] - e[a];
        if (v < 0 || v >= g.n[a]) {
            if (g.per[a])
                v = v < 0 ? v + g.n[a] : v - g.n[a];
            else
                ok = false;
        }
        out[a] = v;
    }
    return ok;
}

// Wave-wide exclusive offset of `count` within a reservation of `total`
// slots taken from *cursor by lane 63.  Every lane of the wave must call it.
__device__ __forceinline__ uint32_t wave_reserve(uint32_t count, uint32_t* cursor)
{
    const int lane = threadIdx.x & 63;
    uint32_t incl = count;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    const uint32_t total = __shfl(incl, 63, 64);
    uint32_t base = 0;
    if (lane == 63 && total != 0) base = atomicAdd(cursor, total);
    base = __shfl(base, 63, 64);
    return base + incl - count;
}

// ---------------------------------------------------------------------------

// Box origin and body radius of every particle, and input checks.  At
// distance d > max|x_i - x_p| from the centre, M <= B(d) = sum K_i/(d - |x_i - x_p|)^2,
// which decreases in d, so the body lies within the root R of B(R) = c0.  The
// box must hold the ball of radius h - 1 (B(h-1) < c0); R itself lets the
// kernels skip box cells that cannot be solid.
__global__ void k_boxes(PartDev P, int h, int* boxes, double* ball, uint32_t* err, Geom g)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P.n) return;
    uint32_t bad = 0;
    double xp[3];
    for (int a = 0; a < 3; ++a) {
        xp[a] = P.pos[3 * p + a];
        if (!(xp[a] == xp[a]) || (g.per[a] && !(xp[a] >= 0.0 && xp[a] < (double)g.n[a]))) bad |= 1u;
        boxes[3 * p + a] = (int)floor(xp[a]) - h;
    }
    const int a0 = P.off[p], n = P.off[p + 1] - a0;
    if (n < 1 || n > kMaxCtrl) bad |= 8u;
    const double c0 = P.c0[p];
    if (!(c0 > 0.0)) bad |= 2u;
    double rmax = 0.0;
    for (int i = 0; i < min(n, kMaxCtrl); ++i) {
        if (!(P.K[a0 + i] > 0.0)) bad |= 2u;
        double r2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            const double d = P.wpts[3 * (int64_t)(a0 + i) + a] - xp[a];
            r2 += d * d;
        }
        rmax = fmax(rmax, sqrt(r2));
    }
    auto bound = [&](double d) {
        double s = 0.0;
        for (int i = 0; i < min(n, kMaxCtrl); ++i) {
            double r2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                const double e = P.wpts[3 * (int64_t)(a0 + i) + a] - xp[a];
                r2 += e * e;
            }
            const double t = d - sqrt(r2);
            s += P.K[a0 + i] / (t * t);
        }
        return s;
    };
    const double lim = (double)(h - 1);
    double R = lim;
    if (!(lim > rmax) || !(bound(lim) < c0)) {
        bad |= 4u;
    } else {
        double lo = rmax, hi = lim;
        for (int it = 0; it < 64; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (bound(mid) >= c0) lo = mid;
            else hi = mid;
        }
        R = hi;
    }
    ball[4 * p + 0] = xp[0];
    ball[4 * p + 1] = xp[1];
    ball[4 * p + 2] = xp[2];
    ball[4 * p + 3] = R + 1e-6;
    if (bad) atomicOr(err, bad);
}

// Whether a box cell lies outside the particle's bounding ball (x_p, R) and so
// cannot be one of its nodes.
__device__ __forceinline__ bool outside_ball(const BoxCell& bc, const double* ball)
{
    const double dx = (double)bc.ii[0] - ball[0];
    const double dy = (double)bc.ii[1] - ball[1];
    const double dz = (double)bc.ii[2] - ball[2];
    return (dx * dx + dy * dy) + dz * dz > ball[3] * ball[3];
}

__global__ __launch_bounds__(256) void k_clear(uint32_t* own, const int* boxes, const double* ball,
                                               BoxSpec b, Geom g)
{
    const int p = blockIdx.y;
    const int t = blockIdx.x * 256 + threadIdx.x;
    const BoxCell bc = box_cell(boxes + 3 * p, t, b, g);
    if (bc.in && !outside_ball(bc, ball + 4 * p)) own[node_idx(bc.c, g)] = kFluid;
}

__global__ __launch_bounds__(256) void k_mark(uint32_t* own, const int* boxes, const double* ball,
                                              PartDev P, BoxSpec b, Geom g)
{
    __shared__ double sp[4 * kMaxCtrl];
    const int p = blockIdx.y;
    const int n = stage_ctrl(P, p, sp);
    const int t = blockIdx.x * 256 + threadIdx.x;
    const BoxCell bc = box_cell(boxes + 3 * p, t, b, g);
    if (!bc.in || outside_ball(bc, ball + 4 * p)) return;
    const double M = metaball(sp, n, (double)bc.ii[0], (double)bc.ii[1], (double)bc.ii[2]);
    if (M >= P.c0[p]) atomicMin(own + node_idx(bc.c, g), (uint32_t)p);
}

// Over the previous boxes: flags of the new classification and the nodes that
// particle p covered before and that are fluid now.
__global__ __launch_bounds__(256) void k_finish(const uint32_t* own_prev, const uint32_t* own_new,
                                                const int* boxes, const double* ball, BoxSpec b,
                                                Geom g, uint8_t* flag, RefillRec* rec, int64_t cap,
                                                uint32_t* cursor)
{
    const int p = blockIdx.y;
    const int t = blockIdx.x * 256 + threadIdx.x;
    const BoxCell bc = box_cell(boxes + 3 * p, t, b, g);
    bool refill = false;
    uint32_t node = 0;
    if (bc.in && !outside_ball(bc, ball + 4 * p)) {
        node = node_idx(bc.c, g);
        const uint32_t on = own_new[node];
        flag[node] = on != kFluid;
        refill = own_prev[node] == (uint32_t)p && on == kFluid;
    }
    const uint32_t slot = wave_reserve(refill ? 1u : 0u, cursor);
    if (refill && slot < cap) {
        rec[slot].node = node;
        rec[slot].part = (uint32_t)p;
    }
}

// Over the new boxes: flags, and the link records of every node of p.
__global__ __launch_bounds__(256) void k_links(const uint32_t* own, const int* boxes,
                                               const double* ball, PartDev P, BoxSpec b, Geom g,
                                               uint8_t* flag, LinkRec* links, int64_t cap,
                                               uint32_t* cursors, int treat)
{
    __shared__ double sp[4 * kMaxCtrl];
    const int p = blockIdx.y;
    const int n = stage_ctrl(P, p, sp);
    const int t = blockIdx.x * 256 + threadIdx.x;
    const BoxCell bc = box_cell(boxes + 3 * p, t, b, g);
    const double c0 = P.c0[p];
    bool mine = false;
    uint32_t node = 0;
    if (bc.in && !outside_ball(bc, ball + 4 * p)) {
        node = node_idx(bc.c, g);
        const uint32_t o = own[node];
        flag[node] = o != kFluid;
        mine = o == (uint32_t)p;
    }
    // pass 1: count
    uint32_t count = 0;
    if (mine) {
        for (int d = 1; d < kQ; ++d) {
            const int ex = ex_d(d), ey = ey_d(d), ez = ez_d(d);
            int cn[3];
            const bool ok = neighbour(bc.c, ex, ey, ez, g, cn);
            const uint32_t on = ok ? own[node_idx(cn, g)] : kFluid;
            if (ok && on == (uint32_t)p) continue;
            if (ok && on == kFluid) {
                ++count;
            } else if (treat & LBM_TREAT_MISSING) {
                const double Mn = metaball(sp, n, (double)(bc.ii[0] - ex), (double)(bc.ii[1] - ey),
                                           (double)(bc.ii[2] - ez));
                if (Mn < c0) ++count;
            }
        }
    }
    uint32_t slot = wave_reserve(count, cursors + (int64_t)p * kCursorPad);
    if (count == 0) return;
    // pass 2: emit
    const double Ms = metaball(sp, n, (double)bc.ii[0], (double)bc.ii[1], (double)bc.ii[2]);
    LinkRec* out = links + (int64_t)p * cap;
    for (int d = 1; d < kQ; ++d) {
        const int ex = ex_d(d), ey = ey_d(d), ez = ez_d(d);
        int cn[3];
        const bool ok = neighbour(bc.c, ex, ey, ez, g, cn);
        const uint32_t on = ok ? own[node_idx(cn, g)] : kFluid;
        if (ok && on == (uint32_t)p) continue;
        const double Mn = metaball(sp, n, (double)(bc.ii[0] - ex), (double)(bc.ii[1] - ey),
                                   (double)(bc.ii[2] - ez));
        int kind;
        if (ok && on == kFluid) {
            int cff[3];
            const bool okf = neighbour(cn, ex, ey, ez, g, cff);
            const bool ff = okf && own[node_idx(cff, g)] == kFluid;
            kind = ((treat & LBM_TREAT_VIBB) && ff) ? LBM_LINK_VIBB : LBM_LINK_HALFWAY;
        } else {
            if (!(treat & LBM_TREAT_MISSING) || !(Mn < c0)) continue;
            kind = LBM_LINK_MISSING;
        }
        if (slot < cap) {
            LinkRec r;
            r.node = node;
            r.part = (uint16_t)p;
            r.d = (uint8_t)d;
            r.kind = (uint8_t)kind;
            r.q = (c0 - Mn) / (Ms - Mn);
            out[slot] = r;
        }
        ++slot;
    }
}

__global__ void k_owner_export(const uint32_t* own, int32_t* out, uint32_t ncell)
{
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i >= ncell) return;
    const uint32_t o = own[i];
    out[i] = o == kFluid ? 0 : (int32_t)o + 1;
}

__global__ void k_link_export(const LinkRec* links, const uint32_t* cursors, int64_t cap,
                              const int64_t* offsets, int32_t* node, int8_t* d, int8_t* kind,
                              int32_t* part, double* q)
{
    const int p = blockIdx.y;
    const uint32_t cnt = min((uint32_t)cap, cursors[(int64_t)p * kCursorPad]);
    const uint32_t l = blockIdx.x * 256u + threadIdx.x;
    if (l >= cnt) return;
    const LinkRec r = links[(int64_t)p * cap + l];
    const int64_t o = offsets[p] + l;
    node[o] = (int32_t)r.node;
    d[o] = (int8_t)r.d;
    kind[o] = (int8_t)r.kind;
    part[o] = (int32_t)r.part;
    q[o] = r.q;
}

inline uint32_t blocks_for(int64_t n) { return (uint32_t)((n + 255) / 256); }

}  // namespace

hipError_t launch_boxes(lbm_ctx* c, const PartDev& P, int slot)
{
    const int np = c->cfg.n_particles;
    if (np == 0) return hipSuccess;
    hipLaunchKernelGGL(k_boxes, dim3((np + 63) / 64), dim3(64), 0, c->stream, P, c->box.h,
                       c->box_hist + (int64_t)slot * 3 * np, c->ball_hist + (int64_t)slot * 4 * np,
                       c->err, c->geom);
    return hipGetLastError();
}

hipError_t launch_clear_boxes(lbm_ctx* c, uint32_t* own, int slot, int np)
{
    if (np == 0) return hipSuccess;
    hipLaunchKernelGGL(k_clear, dim3(c->box.tiles, np), dim3(256), 0, c->stream, own,
                       c->box_hist + (int64_t)slot * 3 * np, c->ball_hist + (int64_t)slot * 4 * np,
                       c->box, c->geom);
    return hipGetLastError();
}

hipError_t launch_mark(lbm_ctx* c, uint32_t* own, const PartDev& P, int slot)
{
    const int np = c->cfg.n_particles;
    if (np == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mark, dim3(c->box.tiles, np), dim3(256), 0, c->stream, own,
                       c->box_hist + (int64_t)slot * 3 * np, c->ball_hist + (int64_t)slot * 4 * np,
                       P, c->box, c->geom);
    return hipGetLastError();
}

hipError_t launch_finish(lbm_ctx* c, const uint32_t* own_prev, const uint32_t* own_new, int slot,
                         int np_prev)
{
    if (np_prev == 0) return hipSuccess;
    hipLaunchKernelGGL(k_finish, dim3(c->box.tiles, np_prev), dim3(256), 0, c->stream, own_prev,
                       own_new, c->box_hist + (int64_t)slot * 3 * np_prev,
                       c->ball_hist + (int64_t)slot * 4 * np_prev, c->box, c->geom, c->flag,
                       c->refill, c->refill_cap, c->refill_cursor);
    return hipGetLastError();
}

hipError_t launch_links(lbm_ctx* c, const uint32_t* own, const PartDev& P, int slot)
{
    const int np = c->cfg.n_particles;
    if (np == 0) return hipSuccess;
    hipLaunchKernelGGL(k_links, dim3(c->box.tiles, np), dim3(256), 0, c->stream, own,
                       c->box_hist + (int64_t)slot * 3 * np, c->ball_hist + (int64_t)slot * 4 * np,
                       P, c->box, c->geom, c->flag, c->links, c->link_cap, c->link_cursor,
                       c->cfg.treatments);
    return hipGetLastError();
}

hipError_t launch_owner_export(const lbm_ctx* c, const uint32_t* own, int32_t* out)
{
    hipLaunchKernelGGL(k_owner_export, dim3(blocks_for(c->geom.ncell)), dim3(256), 0, c->stream,
                       own, out, c->geom.ncell);
    return hipGetLastError();
}

hipError_t launch_link_export(const lbm_ctx* c, int32_t* node, int8_t* d, int8_t* kind,
                              int32_t* part, double* q, const int64_t* offsets_dev)
{
    const int np = c->cfg.n_particles;
    if (np == 0 || c->link_max == 0) return hipSuccess;
    hipLaunchKernelGGL(k_link_export, dim3(blocks_for(c->link_max), np), dim3(256), 0, c->stream,
                       c->links, c->link_cursor, c->link_cap, offsets_dev, node, d, kind, part, q);
    return hipGetLastError();
}

}  // namespace mdlbm

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
// Work is organised per particle: a particle's nodes lie in a ball of radius
// R <= h - 1 about x_p (a rigorous bound from the metaball weights), inside the
// box of (2h+1)^3 nodes around floor(x_p).  One workgroup takes one z plane
// of the box and walks the rows of the ball in it, a wave per row and a lane
// per node.  Coordinates are unwrapped, so on a periodic axis they are exactly
// the node's image nearest x_p (the box is narrower than half the period).
#pragma clang fp contract(off)

#include <algorithm>

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

__device__ __forceinline__ uint32_t node_idx(const int c[3], const Geom& g)
{
    return (uint32_t)c[0] + (uint32_t)g.n[0] * ((uint32_t)c[1] + (uint32_t)g.n[1] * (uint32_t)c[2]);
}

// Wrap unwrapped coordinates onto the lattice; false beyond a wall.
__device__ __forceinline__ bool wrap_cell(const int ii[3], const Geom& g, int c[3])
{
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int v = ii[a];
        if (v < 0 || v >= g.n[a]) {
            if (g.per[a])
                v = ((v % g.n[a]) + g.n[a]) % g.n[a];
            else
                ok = false;
        }
        c[a] = v;
    }
    return ok;
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

// Visit the nodes of one z plane (blockIdx.x of the box) inside the ball
// (x_p, R): the block's waves take rows y in turn and the lanes of a wave the
// consecutive x of a row.  fn(ii, active) is called by every lane of a wave
// together, so it may use wave-wide operations.
template <class Fn>
__device__ __forceinline__ void walk_ball_plane(const double* ball, int h, Fn&& fn)
{
    const double bx = ball[0], by = ball[1], bz = ball[2], R = ball[3];
    const int zi = (int)floor(bz) - h + (int)blockIdx.x;
    const double dz = (double)zi - bz;
    const double r2z = R * R - dz * dz;
    if (r2z < 0.0) return;  // uniform over the block
    const double ry = sqrt(r2z);
    const int ylo = (int)ceil(by - ry), yhi = (int)floor(by + ry);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    for (int yi = ylo + wave; yi <= yhi; yi += nw) {
        const double dy = (double)yi - by;
        const double r2x = r2z - dy * dy;
        if (r2x < 0.0) continue;  // uniform over the wave
        const double rx = sqrt(r2x);
        const int xlo = (int)ceil(bx - rx), xhi = (int)floor(bx + rx);
        for (int x0 = xlo; x0 <= xhi; x0 += 64) {
            const int ii[3] = {x0 + lane, yi, zi};
            fn(ii, x0 + lane <= xhi);
        }
    }
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

// First slot of a block of sum(count) slots taken from *cursor with one
// atomic per wave (the same value on every lane).  Every lane must call it.
__device__ __forceinline__ uint32_t wave_base(uint32_t count, uint32_t* cursor)
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
    return __shfl(base, 63, 64);
}

// ---------------------------------------------------------------------------

// Box origin and body radius of every particle, and input checks.  At
// distance d > max|x_i - x_p| from the centre, M <= B(d) = sum K_i/(d - |x_i - x_p|)^2,
// which decreases in d, so the body lies within the root R of B(R) = c0.  The
// box must hold the ball of radius h - 1 (B(h-1) < c0); R itself lets the
// kernels skip box cells that cannot be solid.
__global__ void k_boxes(PartDev P, int h, double* ball, uint32_t* err, Geom g)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P.n) return;
    uint32_t bad = 0;
    double xp[3];
    for (int a = 0; a < 3; ++a) {
        xp[a] = P.pos[3 * p + a];
        if (!(xp[a] == xp[a]) || (g.per[a] && !(xp[a] >= 0.0 && xp[a] < (double)g.n[a]))) bad |= 1u;
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

__global__ __launch_bounds__(256) void k_clear(uint32_t* own, const double* ball, int h, Geom g)
{
    const int p = blockIdx.y;
    walk_ball_plane(ball + 4 * p, h, [&](const int* ii, bool act) {
        int c[3];
        if (act && wrap_cell(ii, g, c)) own[node_idx(c, g)] = kFluid;
    });
}

// Node owners: the lowest particle index with M_p >= c0_p.  The decision is
// the FP64 sum's; an FP32 estimate settles every node whose M lies outside a
// relative band of 1e-4 around c0 (its own error is below 1e-6) and the FP64
// sum settles the rest.  Every solid node gets its flag, and the solid nodes
// of p that may carry links of p go to p's candidate list: a node where the
// lower bound sum_i K_i / (r_i + sqrt 2)^2 of M_p over all D3Q19 neighbours
// (|e| <= sqrt 2) reaches c0 (with margin) has M_p >= c0 at every neighbour,
// hence no link of any kind, and is left out.
__global__ __launch_bounds__(256) void k_mark(uint32_t* own, const double* ball, int h, PartDev P,
                                              Geom g, uint8_t* flag, uint32_t* cand, int64_t cap,
                                              uint32_t* cursors)
{
    __shared__ double sp[4 * kMaxCtrl];
    const int p = blockIdx.y;
    const int n = stage_ctrl(P, p, sp);
    const double c0 = P.c0[p];
    uint32_t* list = cand + (int64_t)p * cap;
    uint32_t* cursor = cursors + (int64_t)p * kCursorPad;
    const float c0f = (float)c0;
    walk_ball_plane(ball + 4 * p, h, [&](const int* ii, bool act) {
        int c[3];
        bool keep = false;
        uint32_t node = 0;
        if (act && wrap_cell(ii, g, c)) {
            node = node_idx(c, g);
            const double X = (double)ii[0], Y = (double)ii[1], Z = (double)ii[2];
            // FP32 estimate of M and of its lower bound over the neighbours;
            // their relative error is below 1e-6, so outside a 1e-4 band
            // around c0 they decide exactly what the FP64 sum decides.
            float Mf = 0.0f, lbf = 0.0f;
            for (int i = 0; i < n; ++i) {
                const float dx = (float)(X - sp[4 * i + 0]);
                const float dy = (float)(Y - sp[4 * i + 1]);
                const float dz = (float)(Z - sp[4 * i + 2]);
                const float r2 = (dx * dx + dy * dy) + dz * dz;
                const float k = (float)sp[4 * i + 3];
                Mf += k / r2;
                const float t = sqrtf(r2) + 1.4143f;
                lbf += k / (t * t);
            }
            bool solid;
            if (Mf >= c0f * 1.0001f) solid = true;
            else if (Mf <= c0f * 0.9999f) solid = false;
            else solid = metaball(sp, n, X, Y, Z) >= c0;
            if (solid) {
                atomicMin(own + node, (uint32_t)p);
                flag[node] = 1;
                keep = !(lbf >= c0f * 1.0001f);
            }
        }
        const uint32_t slot = wave_reserve(keep ? 1u : 0u, cursor);
        if (keep && slot < cap) list[slot] = node;
    });
}

// Over the previous balls: flags of the new classification and the nodes that
// particle p covered before and that are fluid now.
__global__ __launch_bounds__(256) void k_finish(const uint32_t* own_prev, const uint32_t* own_new,
                                                const double* ball, int h, Geom g, uint8_t* flag,
                                                RefillRec* rec, int64_t cap, uint32_t* cursor)
{
    const int p = blockIdx.y;
    walk_ball_plane(ball + 4 * p, h, [&](const int* ii, bool act) {
        int c[3];
        bool refill = false;
        uint32_t node = 0;
        if (act && wrap_cell(ii, g, c)) {
            node = node_idx(c, g);
            const uint32_t on = own_new[node];
            flag[node] = on != kFluid;
            refill = own_prev[node] == (uint32_t)p && on == kFluid;
        }
        const uint32_t slot = wave_reserve(refill ? 1u : 0u, cursor);
        if (refill && slot < cap) {
            rec[slot].node = node;
            rec[slot].part = (uint32_t)p;
        }
    });
}

// Link records of the candidate nodes of p (those p owns), written
// direction-major within each wave: the links of one direction over a run of
// neighbouring candidates are contiguous, so the link kernel's gathers
// coalesce.  A grid of a few workgroups per particle strides over the list.
__global__ __launch_bounds__(256) void k_links(const uint32_t* own, const double* ball, PartDev P,
                                               Geom g, const uint32_t* cand, int64_t cand_cap,
                                               const uint32_t* cand_cursors, LinkRec* links,
                                               int64_t cap, uint32_t* cursors, int treat)
{
    __shared__ double sp[4 * kMaxCtrl];
    const int p = blockIdx.y;
    const int n = stage_ctrl(P, p, sp);
    const double c0 = P.c0[p];
    const double* B = ball + 4 * p;
    const uint32_t* list = cand + (int64_t)p * cand_cap;
    const uint32_t count = min((uint32_t)cand_cap, cand_cursors[(int64_t)p * kCursorPad]);
    LinkRec* out = links + (int64_t)p * cap;
    uint32_t* cursor = cursors + (int64_t)p * kCursorPad;
    const int lane = threadIdx.x & 63;
    const uint64_t below = (1ull << lane) - 1ull;
    for (uint32_t base0 = blockIdx.x * 256u; base0 < count; base0 += gridDim.x * 256u) {
        const uint32_t k = base0 + threadIdx.x;
        uint32_t node = 0, mask = 0;
        int c[3] = {0, 0, 0};
        double X = 0.0, Y = 0.0, Z = 0.0;
        if (k < count) {
            node = list[k];
            c[0] = (int)(node % (uint32_t)g.n[0]);
            c[1] = (int)((node / (uint32_t)g.n[0]) % (uint32_t)g.n[1]);
            c[2] = (int)(node / ((uint32_t)g.n[0] * (uint32_t)g.n[1]));
            // unwrapped coordinates: the image nearest the particle centre
            double Xc[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                double v = (double)c[a];
                if (g.per[a]) {
                    const double d = v - B[a];
                    if (d > 0.5 * g.n[a]) v -= g.n[a];
                    else if (d < -0.5 * g.n[a]) v += g.n[a];
                }
                Xc[a] = v;
            }
            X = Xc[0], Y = Xc[1], Z = Xc[2];
            if (own[node] == (uint32_t)p) {
                uint32_t on[kQ];
                bool ok[kQ];
#pragma unroll
                for (int d = 1; d < kQ; ++d) {
                    int cn[3];
                    ok[d] = neighbour(c, ex_d(d), ey_d(d), ez_d(d), g, cn);
                    on[d] = ok[d] ? own[node_idx(cn, g)] : kFluid;
                }
#pragma unroll
                for (int d = 1; d < kQ; ++d) {
                    if (ok[d] && on[d] == (uint32_t)p) continue;
                    if (ok[d] && on[d] == kFluid) {
                        mask |= 1u << d;
                    } else if (treat & LBM_TREAT_MISSING) {
                        const double Mn = metaball(sp, n, X - ex_d(d), Y - ey_d(d), Z - ez_d(d));
                        if (Mn < c0) mask |= 1u << d;
                    }
                }
            }
        }
        // one reservation per wave, then direction-major positions
        const uint32_t wbase = wave_base(__popc(mask), cursor);
        double Ms = 0.0;
        if (mask) Ms = metaball(sp, n, X, Y, Z);
        uint32_t cum = 0;
        for (int d = 1; d < kQ; ++d) {
            const bool has = (mask >> d) & 1u;
            const uint64_t bal = __ballot(has);
            if (bal == 0) continue;
            if (has) {
                const int ex = ex_d(d), ey = ey_d(d), ez = ez_d(d);
                const uint32_t slot = wbase + cum + (uint32_t)__popcll(bal & below);
                const double Mn = metaball(sp, n, X - ex, Y - ey, Z - ez);
                int cn[3];
                const bool ok = neighbour(c, ex, ey, ez, g, cn);
                int kind = LBM_LINK_MISSING;
                if (ok && own[node_idx(cn, g)] == kFluid) {
                    int cff[3];
                    const bool okf = neighbour(cn, ex, ey, ez, g, cff);
                    const bool ff = okf && own[node_idx(cff, g)] == kFluid;
                    kind = ((treat & LBM_TREAT_VIBB) && ff) ? LBM_LINK_VIBB : LBM_LINK_HALFWAY;
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
            }
            cum += (uint32_t)__popcll(bal);
        }
    }
}

// The same as k_finish over the whole lattice (one node per thread), used when
// the balls cover most of the lattice and a coalesced sweep is cheaper.
__global__ __launch_bounds__(256) void k_finish_all(const uint32_t* own_prev,
                                                    const uint32_t* own_new, Geom g, uint8_t* flag,
                                                    RefillRec* rec, int64_t cap, uint32_t* cursor)
{
    const uint32_t node = blockIdx.x * 256u + threadIdx.x;
    bool refill = false;
    uint32_t op = kFluid;
    if (node < g.ncell) {
        const uint32_t on = own_new[node];
        op = own_prev[node];
        flag[node] = on != kFluid;
        refill = op != kFluid && on == kFluid;
    }
    const uint32_t slot = wave_reserve(refill ? 1u : 0u, cursor);
    if (refill && slot < cap) {
        rec[slot].node = node;
        rec[slot].part = op;
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
                       c->ball_hist + (int64_t)slot * 4 * np, c->err, c->geom);
    return hipGetLastError();
}

// One workgroup per (z plane of the box, particle).
hipError_t launch_clear_boxes(lbm_ctx* c, uint32_t* own, int slot, int np)
{
    if (np == 0) return hipSuccess;
    if (c->dense) return hipMemsetAsync(own, 0xFF, sizeof(uint32_t) * (size_t)c->geom.ncell, c->stream);
    hipLaunchKernelGGL(k_clear, dim3(c->box.S, np), dim3(256), 0, c->stream, own,
                       c->ball_hist + (int64_t)slot * 4 * np, c->box.h, c->geom);
    return hipGetLastError();
}

hipError_t launch_mark(lbm_ctx* c, uint32_t* own, const PartDev& P, int slot)
{
    const int np = c->cfg.n_particles;
    if (np == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mark, dim3(c->box.S, np), dim3(256), 0, c->stream, own,
                       c->ball_hist + (int64_t)slot * 4 * np, c->box.h, P, c->geom, c->flag,
                       c->cand, c->cand_cap, c->cand_cursor);
    return hipGetLastError();
}

hipError_t launch_finish(lbm_ctx* c, const uint32_t* own_prev, const uint32_t* own_new, int slot,
                         int np_prev)
{
    if (np_prev == 0) return hipSuccess;
    if (c->dense) {
        hipLaunchKernelGGL(k_finish_all, dim3(blocks_for(c->geom.ncell)), dim3(256), 0, c->stream,
                           own_prev, own_new, c->geom, c->flag, c->refill, c->refill_cap,
                           c->refill_cursor);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_finish, dim3(c->box.S, np_prev), dim3(256), 0, c->stream, own_prev,
                       own_new, c->ball_hist + (int64_t)slot * 4 * np_prev, c->box.h, c->geom,
                       c->flag, c->refill, c->refill_cap, c->refill_cursor);
    return hipGetLastError();
}

hipError_t launch_links(lbm_ctx* c, const uint32_t* own, const PartDev& P, int slot)
{
    const int np = c->cfg.n_particles;
    if (np == 0) return hipSuccess;
    const uint32_t per = (uint32_t)std::min<int64_t>(16, (c->cand_cap + 255) / 256);
    hipLaunchKernelGGL(k_links, dim3(per, np), dim3(256), 0, c->stream, own,
                       c->ball_hist + (int64_t)slot * 4 * np, P, c->geom, c->cand, c->cand_cap,
                       c->cand_cursor, c->links, c->link_cap, c->link_cursor, c->cfg.treatments);
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

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
#include "lbm_stencil.h"

namespace mdlbm {
namespace {

constexpr int kMaxCtrl = 64;

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

// Block (bx, by) of a gx x gy work grid launched as a 1D grid of a multiple of
// 8 workgroups.  The hardware hands workgroup b to XCD b % 8; mapping XCD k to
// the k-th eighth of the work keeps all blocks of a particle (by) on one XCD,
// so the owner rows its candidates share are fetched into one L2.  False for
// the padding workgroups.
__device__ __forceinline__ bool xcd_tile(uint32_t gx, uint32_t gy, uint32_t& bx, uint32_t& by)
{
    const uint32_t per = gridDim.x >> 3;
    const uint32_t logical = (blockIdx.x & 7u) * per + (blockIdx.x >> 3);
    if (logical >= gx * gy) return false;
    bx = logical % gx;
    by = logical / gx;
    return true;
}

// ---------------------------------------------------------------------------

// Box origin and body radius of every particle, and input checks.  At
// distance d > max|x_i - x_p| from the centre, M <= B(d) = sum K_i/(d - |x_i - x_p|)^2,
// which decreases in d, so the body lies within the root R of B(R) = c0.  The
// box must hold the ball of radius h - 1 (B(h-1) < c0); R itself lets the
// kernels skip box cells that cannot be solid.
__device__ __forceinline__ double wave_sum_d(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// One wave per particle, a lane per control point (n <= 64).
__global__ __launch_bounds__(64) void k_boxes(PartDev P, int h, double* ball, uint32_t* err, Geom g,
                                             const double* ball_prev, double* quat_prev,
                                             uint32_t* inc_bad)
{
    const int p = blockIdx.x;
    const int lane = threadIdx.x;
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
    // this lane's control point: distance to the centre and weight
    double ri = 0.0, Ki = 0.0;
    if (lane < min(n, kMaxCtrl)) {
        Ki = P.K[a0 + lane];
        if (!(Ki > 0.0)) bad |= 2u;
        double r2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            const double d = P.wpts[3 * (int64_t)(a0 + lane) + a] - xp[a];
            r2 += d * d;
        }
        ri = sqrt(r2);
    }
    double rmax = ri;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) rmax = fmax(rmax, __shfl_xor(rmax, o, 64));
    auto bound = [&](double d) {
        const double t = d - ri;
        return wave_sum_d(Ki > 0.0 ? Ki / (t * t) : 0.0);
    };
    const double lim = (double)(h - 1);
    double R = lim;
    if (!(lim > rmax) || !(bound(lim) < c0)) {
        bad |= 4u;
    } else {
        // B decreases beyond rmax.  A 64-way search keeps B(hi) < c0, so hi
        // bounds the body at every round: the lanes test 64 points of
        // (lo, hi], each summing B over the control points itself, and the
        // first that passes becomes hi; six rounds shrink an interval below
        // 2 h under 1e-9
        const int nn = min(n, kMaxCtrl);
        double lo = rmax, hi = lim;
        for (int round = 0; round < 6; ++round) {
            const double step = (hi - lo) * (1.0 / 64.0);
            const double d = lane == 63 ? hi : lo + step * (double)(lane + 1);
            double B = 0.0;
            for (int j = 0; j < nn; ++j) {
                const double t = d - __shfl(ri, j, 64);
                B += __shfl(Ki, j, 64) / (t * t);
            }
            const uint64_t pass = __ballot(B < c0);
            if (!pass) break;  // uniform; hi keeps its bound
            const int first = __ffsll((unsigned long long)pass) - 1;
            const double nh = __shfl(d, first, 64);
            const double nl = __shfl(d, first > 0 ? first - 1 : 0, 64);
            hi = nh;
            if (first > 0) lo = nl;
        }
        R = hi;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) bad |= __shfl_xor(bad, o, 64);
    if (lane == 0) {
        ball[4 * p + 0] = xp[0];
        ball[4 * p + 1] = xp[1];
        ball[4 * p + 2] = xp[2];
        ball[4 * p + 3] = R + 1e-6;
        if (bad) atomicOr(err, bad);
        if (inc_bad) {
            // how far a body point within R + 2 of the centre moved since the
            // previous classification: the centre's displacement plus
            // (R + 2) times the rotation angle between the two orientations
            double d2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                double d = xp[a] - ball_prev[4 * p + a];
                if (g.per[a]) {
                    if (d > 0.5 * g.n[a]) d -= g.n[a];
                    else if (d < -0.5 * g.n[a]) d += g.n[a];
                }
                d2 += d * d;
            }
            const double* q = P.quat + 4 * p;
            double* qp = quat_prev + 4 * p;
            const double dot = fabs(q[0] * qp[0] + q[1] * qp[1] + q[2] * qp[2] + q[3] * qp[3]);
            const double ang = 2.0 * acos(fmin(1.0, dot));
            const double D = sqrt(d2) + (R + 2.0) * ang;
            // a solid node off the candidate list has M >= c0 wherever within
            // the lattice's largest |e| of it; a node moved by less than that
            // stays solid
            if (!(D < 0.9 * (double)kMaxSpeedUp - 1e-3)) atomicOr(inc_bad, 1u);
            for (int a = 0; a < 4; ++a) qp[a] = q[a];
        }
    }
}

__global__ __launch_bounds__(256) void k_clear(const uint32_t* __restrict__ err, uint32_t* own,
                                               const double* ball, int h, Geom g)
{
    if (*err) return;  // the boxes failed their check: leave every plane as it is
    const int p = blockIdx.y;
    walk_ball_plane(ball + 4 * p, h, [&](const int* ii, bool act) {
        int c[3];
        if (act && wrap_cell(ii, g, c)) own[node_idx(c, g)] = kFluid;
    });
}

// Node owners: the lowest particle index with M_p >= c0_p.
//
// Which nodes are visited.  If every control point lies farther than
// rho = sqrt(sum_i K_i / c0) from a node, M_p < c0 there, so p's body lies
// in the union of the balls (x_i, rho); it also lies in the ball (x_p, R) of
// k_boxes.  One workgroup takes one z plane of p's box: it tabulates, for
// every row y of the plane, the x range of the union's hull on that row
// intersected with the centre ball, prefix-sums the row lengths in LDS and
// hands the flattened nodes to its lanes, so no lane idles at row ends.
//
// How a node is decided.  The FP64 sum alone decides, bit for bit; an FP32
// estimate settles the nodes far from the decision.  The estimate works in
// coordinates relative to o = floor(x_p) (node offsets are exact integers,
// control points are rounded once, |x_i - o| <= R + 1 < h), so each
// coordinate difference is off by at most delta = (2h + 4) 2^-24.  At a
// distance r >= g = 0.0085 (2h + 4) from every control point the relative
// error of r^2 is below 2.83 delta / r + 3 2^-24 <= 2e-5, of a term
// K_i / r^2 (hardware reciprocal, 1 ulp) below 2.2e-5 and of the sum below
// 2.6e-5 for up to 64 points.  So outside a relative band of 1e-4 around c0
// the estimate decides what the FP64 sum decides; nodes in the band, or
// within g of a control point, or of a box with h > 127, take the FP64 sum.
//
// Candidates for links.  M_p at any lattice neighbour (|e| <= E: sqrt 2 for
// D3Q19, sqrt 3 for D3Q15) is at least sum_i K_i / (r_i + E)^2.  A solid
// node where the FP32 value of this bound (E rounded up) clears c0 by the
// same margin (its relative error stays below 3.5e-5 for h <= 127: the
// r_i + E terms are never small) has M_p >= c0 at every neighbour, hence no
// link of any kind, and is left off p's candidate list.  Every other solid
// node of p goes on the list.
constexpr int kRows = 2 * kMaxBoxHalf + 1;
constexpr uint32_t kCandBuf = 2048;

__global__ __launch_bounds__(256, 8) void k_mark(const uint32_t* __restrict__ err, uint32_t* own, const double* ball, int h, PartDev P,
                                              Geom g, uint8_t* flag, int store_flag, uint32_t* cand,
                                              int64_t cap, uint32_t* cursors)
{
    if (*err) return;  // the boxes failed their check: leave every plane as it is
    __shared__ double sp[4 * kMaxCtrl];
    __shared__ float4 sf[kMaxCtrl];
    __shared__ int rlo[kRows];
    __shared__ int rstart[kRows + 1];
    __shared__ int wsum[4];
    __shared__ uint32_t cbuf[kCandBuf];  // this plane's candidates, in walk order
    __shared__ uint32_t ccount;
    const int p = blockIdx.y;
    const int n = stage_ctrl(P, p, sp);
    const double c0 = P.c0[p];
    const double bx = ball[4 * p + 0], by = ball[4 * p + 1], bz = ball[4 * p + 2];
    const double R = ball[4 * p + 3];
    const int ox = (int)floor(bx), oy = (int)floor(by), oz = (int)floor(bz);
    const int zi = oz - h + (int)blockIdx.x;
    const int S = 2 * h + 1;
    double ksum = 0.0;
    for (int i = 0; i < n; ++i) ksum += sp[4 * i + 3];
    const double rho2 = ksum / c0 * (1.0 + 1e-6);
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double dz = (double)zi - sp[4 * i + 2];
        sf[i] = make_float4((float)(sp[4 * i + 0] - (double)ox), (float)(sp[4 * i + 1] - (double)oy),
                            (float)(dz * dz), (float)sp[4 * i + 3]);
    }
    // row table: thread t takes rows rpt t .. rpt t + rpt - 1, rpt = 1 for
    // S <= 256 (so every wave shares the FP64 row bounds), up to 4
    const int rpt = (S + 255) >> 8;
    const double dzc = (double)zi - bz;
    const double r2z = R * R - dzc * dzc;
    int len[4];
    int tsum = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int r = rpt * (int)threadIdx.x + k;
        len[k] = 0;
        if (k < rpt && r < S && r2z >= 0.0) {
            const int yi = oy - h + r;
            const double dyc = (double)yi - by;
            const double r2x = r2z - dyc * dyc;
            if (r2x >= 0.0) {
                const double rx = sqrt(r2x);
                double lo = 1e300, hi = -1e300;
                for (int i = 0; i < n; ++i) {
                    const double dy = (double)yi - sp[4 * i + 1];
                    const double dz = (double)zi - sp[4 * i + 2];
                    const double rem = rho2 - (dy * dy + dz * dz);
                    if (rem >= 0.0) {
                        const double w = sqrt(rem) + 1e-6;
                        lo = fmin(lo, sp[4 * i + 0] - w);
                        hi = fmax(hi, sp[4 * i + 0] + w);
                    }
                }
                if (hi >= lo) {  // some control-point ball meets the row
                    const int xlo = max((int)ceil(bx - rx), (int)ceil(lo));
                    const int xhi = min((int)floor(bx + rx), (int)floor(hi));
                    if (xhi >= xlo) {
                        rlo[r] = xlo;
                        len[k] = xhi - xlo + 1;
                    }
                }
            }
        }
        tsum += len[k];
    }
    // block-wide exclusive scan of the per-thread sums
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int incl = tsum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    int off = incl - tsum;
    for (int w = 0; w < wv; ++w) off += wsum[w];
    const int total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int r = rpt * (int)threadIdx.x + k;
        if (k < rpt && r < S) rstart[r] = off;
        off += len[k];
    }
    if (threadIdx.x == 0) {
        rstart[S] = total;
        ccount = 0;
    }
    __syncthreads();
    if (total == 0) return;  // uniform over the block

    uint32_t* list = cand + (int64_t)p * cap;
    uint32_t* cursor = cursors + (int64_t)p * kCursorPad;
    const float c0f = (float)c0;
    const float c0hi = c0f * 1.0001f, c0lo = c0f * 0.9999f;
    const float gr = fmaxf(0.5f, 0.0085f * (float)(2 * h + 4));
    const float guard2 = h <= 127 ? gr * gr : 3.0e38f;
    int top = 1;
    while (top <= S) top <<= 1;
    for (int j0 = 0; j0 < total; j0 += 256) {
        const int j = j0 + (int)threadIdx.x;
        bool keep = false;
        uint32_t node = 0;
        if (j < total) {
            // row of flattened node j: the last r with rstart[r] <= j
            int r = 0;
            for (int step = top >> 1; step > 0; step >>= 1)
                if (r + step <= S && rstart[r + step] <= j) r += step;
            const int ii[3] = {rlo[r] + (j - rstart[r]), oy - h + r, zi};
            int c[3];
            if (wrap_cell(ii, g, c)) {
                node = node_idx(c, g);
                const float X = (float)(ii[0] - ox), Y = (float)(ii[1] - oy);
                float Mf = 0.0f, m2 = 3.0e38f;
                for (int i = 0; i < n; ++i) {
                    const float4 q = sf[i];
                    const float dx = X - q.x, dy = Y - q.y;
                    const float r2 = fmaf(dx, dx, fmaf(dy, dy, q.z));
                    Mf = fmaf(q.w, __builtin_amdgcn_rcpf(r2), Mf);
                    m2 = fminf(m2, r2);
                }
                const bool settled = Mf >= c0hi || Mf <= c0lo;  // false for NaN
                const bool solid =
                    (m2 < guard2 || !settled)
                        ? metaball(sp, n, (double)ii[0], (double)ii[1], (double)ii[2]) >= c0
                        : Mf >= c0hi;
                if (solid) {
                    atomicMin(own + node, (uint32_t)p);
                    if (store_flag) flag[node] = 1;
                    bool interior = false;
                    if (h <= 127) {
                        float lb = 0.0f;
                        for (int i = 0; i < n; ++i) {
                            const float4 q = sf[i];
                            const float dx = X - q.x, dy = Y - q.y;
                            const float r2 = fmaf(dx, dx, fmaf(dy, dy, q.z));
                            const float t = __builtin_amdgcn_sqrtf(r2) + kMaxSpeedUp;
                            lb = fmaf(q.w, __builtin_amdgcn_rcpf(t * t), lb);
                        }
                        interior = lb >= c0hi;
                    }
                    keep = !interior;
                }
            }
        }
        // candidates gather in LDS so that the plane's list stays contiguous
        // and in row order (neighbouring candidates then share owner rows in
        // k_links); a full buffer spills lanes straight to the list
        const uint64_t m = __ballot(keep);
        uint32_t wbase = 0;
        if (lane == 0 && m) wbase = atomicAdd(&ccount, (uint32_t)__popcll(m));
        wbase = __shfl(wbase, 0, 64);
        if (keep) {
            const uint32_t idx = wbase + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
            if (idx < kCandBuf) {
                cbuf[idx] = node;
            } else {
                const uint32_t slot = atomicAdd(cursor, 1u);
                if (slot < cap) list[slot] = node;
            }
        }
    }
    __syncthreads();
    __shared__ uint32_t gbase;
    const uint32_t nb = min(ccount, (uint32_t)kCandBuf);
    if (threadIdx.x == 0) gbase = nb ? atomicAdd(cursor, nb) : 0u;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nb; i += blockDim.x)
        if (gbase + i < cap) list[gbase + i] = cbuf[i];
}

// Over the previous balls: flags of the new classification and the nodes that
// particle p covered before and that are fluid now.
__global__ __launch_bounds__(256) void k_finish(const uint32_t* __restrict__ err, const uint32_t* own_prev, const uint32_t* own_new,
                                                const double* ball, int h, Geom g, uint8_t* flag,
                                                RefillRec* rec, int64_t cap, uint32_t* cursor)
{
    if (*err) return;  // the boxes failed their check: leave every plane as it is
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

// q of Eq. (calq): the root of g(q) = M(x_n + q e_d) - c0 on [0, 1] (g(0) < 0
// <= g(1)), by Newton-Raphson from the estimate of Eq. (appq), kept inside the
// bracket of the sign change (a step that leaves it becomes the midpoint),
// stopping on a step below 1e-13 or after 60 steps.  Along the line
// dM/dq = sum_i -2 K_i ((x - x_i) . e_d) / r_i^4.  Every value is formed in
// the order written (this file has no contraction), so any IEEE
// implementation of the same sequence gets the same bits.
__device__ double exact_q(const double* sp, int n, const double Xn[3], const int e[3], double c0,
                          double Mn, double Ms)
{
    double a = 0.0, b = 1.0;
    double q = (c0 - Mn) / (Ms - Mn);
    for (int it = 0; it < 60; ++it) {
        double M = 0.0, dM = 0.0;
        for (int i = 0; i < n; ++i) {
            const double dx = (Xn[0] + q * (double)e[0]) - sp[4 * i + 0];
            const double dy = (Xn[1] + q * (double)e[1]) - sp[4 * i + 1];
            const double dz = (Xn[2] + q * (double)e[2]) - sp[4 * i + 2];
            const double r2 = (dx * dx + dy * dy) + dz * dz;
            const double t = sp[4 * i + 3] / r2;
            const double se = (dx * (double)e[0] + dy * (double)e[1]) + dz * (double)e[2];
            M = M + t;
            dM = dM - ((2.0 * t) * se) / r2;
        }
        const double g = M - c0;
        if (g == 0.0) break;
        if (g < 0.0)
            a = q;
        else
            b = q;
        double qn = q - g / dM;
        if (!(qn > a && qn < b)) qn = 0.5 * (a + b);
        if (fabs(qn - q) < 1e-13) {
            q = qn;
            break;
        }
        q = qn;
    }
    return q;
}

// Position of the k-th (from 0) set bit of m; m has more than k set bits.
__device__ __forceinline__ int select_bit(uint64_t m, uint32_t k)
{
    int pos = 0;
#pragma unroll
    for (int w = 32; w >= 1; w >>= 1) {
        const uint64_t low = m & ((1ull << w) - 1ull);
        const uint32_t c = (uint32_t)__popcll(low);
        if (k >= c) {
            k -= c;
            m >>= w;
            pos += w;
        }
    }
    return pos;
}

// Link records of the candidate nodes of p (those p owns), written
// direction-major within each wave: the links of one direction over a run of
// neighbouring candidates are contiguous, so the link kernel's gathers
// coalesce.  Each lane first finds the link directions of its candidate; the
// wave then enumerates its links in that order and gives one link to each
// lane (candidate data by lane shuffles), so the FP64 work of q runs on full
// waves.  A grid of a few workgroups per particle strides over the list.
// With few particles a wave takes cpw = 16 candidates instead of 64: about
// one link per lane then, and four times the waves, so the serial
// enumeration is short where the list is too small to fill the chip.
__global__ __launch_bounds__(256, 6) void k_links(const uint32_t* __restrict__ err, const uint32_t* own, const double* ball, PartDev P,
                                               Geom g, const uint32_t* cand, int64_t cand_cap,
                                               const uint32_t* cand_cursors, LinkRec* links,
                                               const int64_t* __restrict__ loff,
                                               uint32_t* cursors, int treat, uint32_t gx,
                                               uint32_t cpw)
{
    if (*err) return;  // the boxes failed their check: leave every plane as it is
    __shared__ double sp[4 * kMaxCtrl];
    uint32_t bx, by;
    if (!xcd_tile(gx, (uint32_t)P.n, bx, by)) return;  // uniform over the block
    const int p = (int)by;
    const int n = stage_ctrl(P, p, sp);
    const double c0 = P.c0[p];
    const double B[3] = {ball[4 * p], ball[4 * p + 1], ball[4 * p + 2]};  // loaded once
    const uint32_t* list = cand + (int64_t)p * cand_cap;
    const uint32_t count = min((uint32_t)cand_cap, cand_cursors[(int64_t)p * kCursorPad]);
    LinkRec* out = links + loff[p];
    const int64_t cap = loff[p + 1] - loff[p];  // p's segment
    uint32_t* cursor = cursors + (int64_t)p * kCursorPad;
    const int lane = threadIdx.x & 63;
    const uint32_t chunk = 4u * cpw;  // candidates of one workgroup per round
    for (uint32_t base0 = bx * chunk; base0 < count; base0 += gx * chunk) {
        const uint32_t k = base0 + (threadIdx.x >> 6) * cpw + (uint32_t)lane;
        uint32_t node = 0, mask = 0, fmask = 0;  // link directions; those with x_f fluid
        int c[3] = {0, 0, 0};
        double X = 0.0, Y = 0.0, Z = 0.0;
        if ((uint32_t)lane < cpw && k < count) {
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
            // the node's owner and its neighbours' in one batch of loads
            // (each from a valid address), before any branch on them
            const uint32_t self = own[node];
            uint32_t onv[kQ];
            uint32_t okm = 0;
#pragma unroll
            for (int d = 1; d < kQ; ++d) {
                int cn[3];
                const bool ok = neighbour(c, cx(d), cy(d), cz(d), g, cn);
                const uint32_t v = own[ok ? node_idx(cn, g) : node];
                okm |= ok ? 1u << d : 0u;
                onv[d] = ok ? v : kFluid;
            }
            if (self == (uint32_t)p) {
#pragma unroll
                for (int d = 1; d < kQ; ++d) {
                    const bool ok = (okm >> d) & 1u;
                    const uint32_t on = onv[d];
                    if (ok && on == (uint32_t)p) continue;
                    if (ok && on == kFluid) {
                        mask |= 1u << d;
                        fmask |= 1u << d;
                    } else if (treat & LBM_TREAT_MISSING) {
                        const double Mn = metaball(sp, n, X - cx(d), Y - cy(d), Z - cz(d));
                        if (Mn < c0) mask |= 1u << d;
                    }
                }
            }
        }
        double Ms = 0.0;
        if (mask) Ms = metaball(sp, n, X, Y, Z);
        // direction-major enumeration of the wave's links
        uint64_t bal[kQ];
        uint32_t cum[kQ + 1];
        cum[0] = cum[1] = 0;
        bal[0] = 0;
#pragma unroll
        for (int d = 1; d < kQ; ++d) {
            bal[d] = __ballot((mask >> d) & 1u);
            cum[d + 1] = cum[d] + (uint32_t)__popcll(bal[d]);
        }
        const uint32_t total = cum[kQ];
        if (total == 0) continue;  // uniform over the wave
        uint32_t wbase = 0;
        if (lane == 0) wbase = atomicAdd(cursor, total);
        wbase = __shfl(wbase, 0, 64);
        for (uint32_t j0 = 0; j0 < total; j0 += 64) {
            const uint32_t j = j0 + (uint32_t)lane;
            int d = 1;
            uint64_t m = bal[1];
#pragma unroll
            for (int dd = 2; dd < kQ; ++dd)
                if (cum[dd] <= j) {
                    d = dd;
                    m = bal[dd];
                }
            const int src = j < total ? select_bit(m, j - cum[d]) : lane;
            const uint32_t snode = __shfl(node, src, 64);
            const int sc[3] = {__shfl(c[0], src, 64), __shfl(c[1], src, 64), __shfl(c[2], src, 64)};
            const double sX = __shfl(X, src, 64), sY = __shfl(Y, src, 64), sZ = __shfl(Z, src, 64);
            const double sMs = __shfl(Ms, src, 64);
            const uint32_t sfmask = __shfl(fmask, src, 64);
            if (j < total) {
                const int ex = cx(d), ey = cy(d), ez = cz(d);
                const double Mn = metaball(sp, n, sX - ex, sY - ey, sZ - ez);
                int kind = LBM_LINK_MISSING;
                if ((sfmask >> d) & 1u) {  // x_f exists and is fluid
                    int cn[3];
                    neighbour(sc, ex, ey, ez, g, cn);
                    int cff[3];
                    const bool okf = neighbour(cn, ex, ey, ez, g, cff);
                    const bool ff = okf && own[node_idx(cff, g)] == kFluid;
                    kind = ((treat & LBM_TREAT_VIBB) && ff) ? LBM_LINK_VIBB : LBM_LINK_HALFWAY;
                }
                const uint32_t slot = wbase + j;
                if (slot < cap) {
                    LinkRec r;
                    r.node = snode;
                    r.part = (uint16_t)p;
                    r.d = (uint8_t)d;
                    r.kind = (uint8_t)kind;
                    if (treat & LBM_TREAT_EXACT_Q) {
                        const double Xn[3] = {sX - ex, sY - ey, sZ - ez};
                        const int e[3] = {ex, ey, ez};
                        r.q = exact_q(sp, n, Xn, e, c0, Mn, sMs);
                    } else {
                        r.q = (c0 - Mn) / (sMs - Mn);
                    }
                    out[slot] = r;
                }
            }
        }
    }
}

// The same as k_finish over the whole lattice (four consecutive nodes per
// thread, 16-byte owner loads), used when the balls cover most of the lattice
// and a coalesced sweep is cheaper.
__global__ __launch_bounds__(256) void k_finish_all(const uint32_t* __restrict__ err, const uint32_t* own_prev,
                                                    const uint32_t* own_new, Geom g, uint8_t* flag,
                                                    RefillRec* rec, int64_t cap, uint32_t* cursor,
                                                    const uint32_t* inc_bad)
{
    if (*err) return;  // the boxes failed their check: leave every plane as it is
    if (inc_bad && *inc_bad == 0u) return;  // the candidate pass did the work
    // grid-stride over groups of four nodes (a bounded grid: when the
    // candidate pass did the work, its workgroups only read the word above)
    for (uint32_t base0 = blockIdx.x * 1024u; base0 < g.ncell; base0 += gridDim.x * 1024u) {
        const uint32_t base = base0 + threadIdx.x * 4u;
        uint32_t on[4] = {kFluid, kFluid, kFluid, kFluid}, op[4] = {kFluid, kFluid, kFluid, kFluid};
        if (base + 3u < g.ncell) {
            const uint4 a = *reinterpret_cast<const uint4*>(own_new + base);
            const uint4 b = *reinterpret_cast<const uint4*>(own_prev + base);
            on[0] = a.x, on[1] = a.y, on[2] = a.z, on[3] = a.w;
            op[0] = b.x, op[1] = b.y, op[2] = b.z, op[3] = b.w;
            *reinterpret_cast<uchar4*>(flag + base) =
                make_uchar4(on[0] != kFluid, on[1] != kFluid, on[2] != kFluid, on[3] != kFluid);
        } else {
            for (int k = 0; k < 4; ++k)
                if (base + k < g.ncell) {
                    on[k] = own_new[base + k];
                    op[k] = own_prev[base + k];
                    flag[base + k] = on[k] != kFluid;
                }
        }
        uint32_t cnt = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) cnt += (op[k] != kFluid && on[k] == kFluid) ? 1u : 0u;
        uint32_t slot = wave_reserve(cnt, cursor);
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (op[k] != kFluid && on[k] == kFluid) {
                if (slot < cap) {
                    rec[slot].node = base + k;
                    rec[slot].part = op[k];
                }
                ++slot;
            }
    }
}

// Dense mode, bodies moved less than the guard of k_boxes: the flags of the
// nodes that left a body and the refill list, from the previous
// classification's candidate lists (a node solid then and fluid now was
// within reach of the old surface, hence a candidate).  New solid nodes got
// their flag from k_mark.  One workgroup per (chunk, particle).
__global__ __launch_bounds__(256) void k_finish_cand(const uint32_t* __restrict__ err,
                                                     const uint32_t* __restrict__ inc_bad,
                                                     const uint32_t* __restrict__ own_prev,
                                                     const uint32_t* __restrict__ own_new,
                                                     const uint32_t* __restrict__ cand,
                                                     int64_t cand_cap,
                                                     const uint32_t* __restrict__ counts,
                                                     uint8_t* flag, RefillRec* rec, int64_t cap,
                                                     uint32_t* cursor)
{
    if (*err || *inc_bad) return;  // the lattice sweep does the work
    const int p = blockIdx.y;
    const uint32_t cnt = min((uint32_t)cand_cap, counts[p]);
    for (uint32_t i0 = blockIdx.x * 256u; i0 < cnt; i0 += gridDim.x * 256u) {
        const uint32_t i = i0 + threadIdx.x;
        bool left = false;
        uint32_t node = 0;
        if (i < cnt) {
            node = cand[(int64_t)p * cand_cap + i];
            // a node in two bodies is on both lists: its owner's list takes it
            left = own_prev[node] == (uint32_t)p && own_new[node] == kFluid;
            if (left) flag[node] = 0;
        }
        uint32_t slot = wave_reserve(left ? 1u : 0u, cursor);
        if (left && slot < cap) {
            rec[slot].node = node;
            rec[slot].part = (uint32_t)p;
        }
    }
}

// Zero the counters a classification fills: the refill count, the box check
// and the first word of every link and candidate cursor line (the
// non-finite force flag is left for the classification to report).
__global__ void k_reset_counters(uint32_t* ctr, int np, uint32_t* cand_prev_count)
{
    const int i = (int)(blockIdx.x * 256u + threadIdx.x);
    // the candidate counts of the previous classification, kept for its lists
    if (cand_prev_count && i >= np && i < 2 * np)
        cand_prev_count[i - np] = ctr[kStageHead + (int64_t)i * kCursorPad];
    if (i == 0) {
        ctr[kCtrRefill] = 0;
        ctr[kCtrErr] = 0;
        ctr[kCtrIncremental] = 0;
    }
    if (i < 2 * np) ctr[kStageHead + (int64_t)i * kCursorPad] = 0;
}

// After an asynchronous classification: latch its box check and any list
// overflow (a count above its capacity) into the deferred word, which no
// classification clears.
__global__ void k_latch_deferred(uint32_t* ctr, int np, int np1, const int64_t* loff,
                                 uint32_t cand_cap, uint32_t refill_cap)
{
    uint32_t bad = 0;
    for (int p = (int)threadIdx.x; p < np; p += (int)blockDim.x) {
        const uint32_t nl = ctr[kStageHead + (int64_t)p * kCursorPad];
        const uint32_t nc = ctr[kStageHead + (int64_t)(np1 + p) * kCursorPad];
        if ((int64_t)nl > loff[p + 1] - loff[p] || nc > cand_cap) bad = kDeferredOverflow;
    }
    if (threadIdx.x == 0) {
        if (ctr[kCtrRefill] > refill_cap) bad |= kDeferredOverflow;
        bad |= ctr[kCtrErr] & 0xFFu;
    }
    if (bad) atomicOr(ctr + kCtrDeferred, bad);
}

__global__ void k_owner_export(const uint32_t* own, int32_t* out, uint32_t ncell)
{
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i >= ncell) return;
    const uint32_t o = own[i];
    out[i] = o == kFluid ? 0 : (int32_t)o + 1;
}

__global__ void k_link_export(const LinkRec* links, const uint32_t* cursors,
                              const int64_t* loff, const uint32_t* chunk,
                              const int64_t* offsets, int32_t* node, int8_t* d, int8_t* kind,
                              int32_t* part, double* q)
{
    // one workgroup per 256-record chunk of the layout
    const int p = (int)chunk[blockIdx.x];
    const int64_t gi = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t l = gi - loff[p];
    const int64_t cnt = min(loff[p + 1] - loff[p], (int64_t)cursors[(int64_t)p * kCursorPad]);
    if (l >= cnt) return;
    const LinkRec r = links[gi];
    const int64_t o = offsets[p] + l;
    node[o] = (int32_t)r.node;
    d[o] = (int8_t)r.d;
    kind[o] = (int8_t)r.kind;
    part[o] = (int32_t)r.part;
    q[o] = r.q;
}

inline uint32_t blocks_for(int64_t n) { return (uint32_t)((n + 255) / 256); }

}  // namespace

namespace MDLBM_QNS {

hipError_t launch_boxes(lbm_ctx* c, const PartDev& P, int slot, int slot_prev, bool inc)
{
    const int np = c->cfg.n_particles;
    if (np == 0) return hipSuccess;
    hipLaunchKernelGGL(k_boxes, dim3(np), dim3(64), 0, c->stream, P, c->box.h,
                       c->ball_hist + (int64_t)slot * 4 * np, c->err, c->geom,
                       c->ball_hist + (int64_t)slot_prev * 4 * np, c->quat_prev,
                       inc ? c->ctr + kCtrIncremental : nullptr);
    return hipGetLastError();
}

// One workgroup per (z plane of the box, particle).
hipError_t launch_clear_boxes(lbm_ctx* c, uint32_t* own, int slot, int np)
{
    if (np == 0) return hipSuccess;
    if (c->dense) return hipMemsetAsync(own, 0xFF, sizeof(uint32_t) * (size_t)c->geom.ncell, c->stream);
    hipLaunchKernelGGL(k_clear, dim3(c->box.S, np), dim3(256), 0, c->stream, c->err, own,
                       c->ball_hist + (int64_t)slot * 4 * np, c->box.h, c->geom);
    return hipGetLastError();
}

hipError_t launch_mark(lbm_ctx* c, uint32_t* own, const PartDev& P, int slot, bool inc)
{
    const int np = c->cfg.n_particles;
    if (np == 0) return hipSuccess;
    // in dense mode the lattice sweep of k_finish_all writes every flag,
    // unless the candidate pass runs (then the solid nodes' flags come from
    // here)
    hipLaunchKernelGGL(k_mark, dim3(c->box.S, np), dim3(256), 0, c->stream, c->err, own,
                       c->ball_hist + (int64_t)slot * 4 * np, c->box.h, P, c->geom, c->flag,
                       (c->dense && !inc) ? 0 : 1, c->cand, c->cand_cap, c->cand_cursor);
    return hipGetLastError();
}

hipError_t launch_finish(lbm_ctx* c, const uint32_t* own_prev, const uint32_t* own_new, int slot,
                         int np_prev, bool inc)
{
    if (np_prev == 0) return hipSuccess;
    if (c->dense) {
        if (inc) {
            // the candidate pass, or, should k_boxes have found a body that
            // moved too far, the lattice sweep (each kernel checks the word)
            const uint32_t nb = (uint32_t)std::min<int64_t>(
                std::max<int64_t>(1, (c->cand_prev_cap + 255) / 256), 64);
            hipLaunchKernelGGL(k_finish_cand, dim3(nb, np_prev), dim3(256), 0, c->stream, c->err,
                               c->ctr + kCtrIncremental, own_prev, own_new, c->cand_prev,
                               c->cand_prev_cap, c->cand_prev_count, c->flag, c->refill,
                               c->refill_cap, c->refill_cursor);
        }
        // 2048 workgroups (eight per compute unit) stride over the lattice
        const uint32_t nb = (uint32_t)std::min<int64_t>(((int64_t)c->geom.ncell + 1023) / 1024, 2048);
        hipLaunchKernelGGL(k_finish_all, dim3(nb), dim3(256), 0,
                           c->stream, c->err, own_prev, own_new, c->geom, c->flag, c->refill,
                           c->refill_cap, c->refill_cursor,
                           inc ? c->ctr + kCtrIncremental : nullptr);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_finish, dim3(c->box.S, np_prev), dim3(256), 0, c->stream, c->err, own_prev,
                       own_new, c->ball_hist + (int64_t)slot * 4 * np_prev, c->box.h, c->geom,
                       c->flag, c->refill, c->refill_cap, c->refill_cursor);
    return hipGetLastError();
}

hipError_t launch_links(lbm_ctx* c, const uint32_t* own, const PartDev& P, int slot)
{
    const int np = c->cfg.n_particles;
    if (np == 0) return hipSuccess;
    // few particles: 16 candidates per wave and up to 64 workgroups each
    const uint32_t cpw = np <= 64 ? 16u : 64u;
    const int64_t chunk = 4 * (int64_t)cpw;
    const uint32_t per =
        (uint32_t)std::min<int64_t>(np <= 64 ? 64 : 16, (c->cand_cap + chunk - 1) / chunk);
    const uint32_t nb = (per * (uint32_t)np + 7u) & ~7u;
    hipLaunchKernelGGL(k_links, dim3(nb), dim3(256), 0, c->stream, c->err, own,
                       c->ball_hist + (int64_t)slot * 4 * np, P, c->geom, c->cand, c->cand_cap,
                       c->cand_cursor, c->links, c->lay->off_dev, c->link_cursor,
                       c->cfg.treatments, per, cpw);
    return hipGetLastError();
}

hipError_t launch_reset_counters(lbm_ctx* c)
{
    const int np = c->cfg.n_particles;
    hipLaunchKernelGGL(k_reset_counters, dim3(blocks_for(2 * (int64_t)std::max(np, 1))), dim3(256), 0,
                       c->stream, c->ctr, np, c->cand_prev_count);
    return hipGetLastError();
}

hipError_t launch_latch_deferred(lbm_ctx* c)
{
    const int np = c->cfg.n_particles;
    hipLaunchKernelGGL(k_latch_deferred, dim3(1), dim3(256), 0, c->stream, c->ctr, np,
                       std::max(np, 1), c->lay->off_dev, (uint32_t)c->cand_cap,
                       (uint32_t)c->refill_cap);
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
    if (np == 0 || c->link_max == 0 || c->lay->chunks() == 0) return hipSuccess;
    hipLaunchKernelGGL(k_link_export, dim3((uint32_t)c->lay->chunks()), dim3(256), 0, c->stream,
                       c->links, c->link_cursor, c->lay->off_dev, c->lay->chunk_dev, offsets_dev,
                       node, d, kind, part, q);
    return hipGetLastError();
}

}  // namespace MDLBM_QNS
}  // namespace mdlbm

// C-ABI entry points of libmdlbm (declared in include/mdlbm.h): argument
// checks, scratch management and the order of kernel launches for one
// classification, one lattice step and one DEM sub-cycle.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lbm_internal.h"

using namespace mdlbm;

namespace {

thread_local std::string g_init_error;

int fail(lbm_ctx* c, int code, const std::string& msg)
{
    if (c) {
        c->last_error = msg;
        if (code == LBM_EDEVICE || code == LBM_ENUMERIC) c->failed = true;
    } else {
        g_init_error = msg;
    }
    return code;
}

#define HIPCHK(ctx, expr)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(ctx, LBM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

size_t elem_bytes(int storage)
{
    switch (storage) {
    case LBM_STORE_F64: return 8;
    case LBM_STORE_F32: return 4;
    case LBM_STORE_F16: return 2;
    default: return 0;
    }
}

PartDev to_dev(const lbm_particles* P)
{
    PartDev d;
    d.n = P->n;
    d.off = P->ctrl_off;
    d.body_pts = P->body_pts;
    d.K = P->K;
    d.c0 = P->c0;
    d.rs = P->rs;
    d.mass = P->mass;
    d.volume = P->volume;
    d.inertia = P->inertia;
    d.pos = P->pos;
    d.quat = P->quat;
    d.vel = P->vel;
    d.omega = P->omega;
    d.wpts = P->world_pts;
    return d;
}

int check_particles(lbm_ctx* c, const lbm_particles* P, bool need_dem)
{
    if (!P) return fail(c, LBM_EINVAL, "null particle description");
    if (P->n != c->cfg.n_particles)
        return fail(c, LBM_EINVAL, "particle count differs from lbm_config.n_particles");
    if (P->n == 0) return LBM_OK;
    if (!P->ctrl_off || !P->K || !P->c0 || !P->pos || !P->vel || !P->omega || !P->world_pts)
        return fail(c, LBM_EINVAL, "null particle array");
    if (need_dem && (!P->body_pts || !P->rs || !P->mass || !P->volume || !P->inertia || !P->quat))
        return fail(c, LBM_EINVAL, "null particle array needed by the DEM");
    return LBM_OK;
}

template <class T>
hipError_t alloc(T** p, size_t count)
{
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc((void**)p, count * sizeof(T));
}

hipEvent_t take_event(lbm_ctx* c)
{
    if (!c->event_pool.empty()) {
        hipEvent_t e = c->event_pool.back();
        c->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Brackets the launches of one phase with a hipEvent pair while timing is on.
struct PhaseTimer {
    lbm_ctx* c;
    int phase;
    hipEvent_t start = nullptr;
    PhaseTimer(lbm_ctx* ctx, int ph) : c(ctx), phase(ph)
    {
        if (c->prof) {
            start = take_event(c);
            if (start) (void)hipEventRecord(start, c->stream);
        }
    }
    ~PhaseTimer()
    {
        if (!start) return;
        hipEvent_t stop = take_event(c);
        if (!stop) return;
        (void)hipEventRecord(stop, c->stream);
        c->timed.push_back({phase, start, stop});
    }
};

// Runs the launchers of a scope on another stream of the context.
struct OnStream {
    lbm_ctx* c;
    hipStream_t saved;
    OnStream(lbm_ctx* ctx, hipStream_t s) : c(ctx), saved(ctx->stream) { c->stream = s; }
    ~OnStream() { c->stream = saved; }
};

// The two streams of lbm_step_dem.  The DEM kernels are latency-bound and
// need few compute units; the stream-collide pass is bound by HBM and keeps
// its rate on fewer.  kDemUnits units of each XCD go to the DEM: mask bit i
// is unit i, and the bits 33x + 8m (x = 0..7, m < kDemUnits <= 4) fall on
// XCD x whether the runtime deals the bits out to the XCDs in runs of 32 or
// in turn.  Both streams have the default priority.
#ifndef MDLBM_DEM_UNITS
#define MDLBM_DEM_UNITS 2
#endif
constexpr int kDemUnits = MDLBM_DEM_UNITS;
static_assert(kDemUnits >= 1 && kDemUnits <= 4, "one to four units per XCD");
int overlap_streams(lbm_ctx* c)
{
    if (c->s_bulk) return LBM_OK;
    hipDeviceProp_t prop;
    HIPCHK(c, hipGetDeviceProperties(&prop, c->device));
    const int ncu = prop.multiProcessorCount;
    if (ncu < 64) return fail(c, LBM_EDEVICE, "lbm_step_dem needs at least 64 compute units");
    const int words = (ncu + 31) / 32;
    std::vector<uint32_t> bulk((size_t)words, 0u), dem((size_t)words, 0u);
    for (int i = 0; i < ncu; ++i) bulk[(size_t)(i / 32)] |= 1u << (i % 32);
    for (int x = 0; x < 8; ++x)
        for (int m = 0; m < kDemUnits; ++m)
            if (const int i = 33 * x + 8 * m; i < ncu) {
                dem[(size_t)(i / 32)] |= 1u << (i % 32);
                bulk[(size_t)(i / 32)] &= ~(1u << (i % 32));
            }
    HIPCHK(c, hipExtStreamCreateWithCUMask(&c->s_bulk, (uint32_t)words, bulk.data()));
    HIPCHK(c, hipExtStreamCreateWithCUMask(&c->s_dem, (uint32_t)words, dem.data()));
    for (hipEvent_t* e : {&c->ev_fork, &c->ev_bulk, &c->ev_dem})
        HIPCHK(c, hipEventCreateWithFlags(e, hipEventDisableTiming));
    return LBM_OK;
}

std::string err_text(uint32_t bits)
{
    std::string s;
    if (bits & 1u) s += "particle centre outside [0,n) on a periodic axis or not finite; ";
    if (bits & 2u) s += "metaball weight K or surface level c0 not positive; ";
    if (bits & 4u) s += "particle body may reach beyond box_half - 1 of its centre; ";
    if (bits & 8u) s += "particle has no control points or more than 64; ";
    return s;
}

// A link layout with segments of the given sizes (multiples of 256
// records); null when its device tables cannot be allocated.
std::shared_ptr<const LinkLayout> make_layout(const std::vector<int64_t>& seg)
{
    auto L = std::make_shared<LinkLayout>();
    const size_t np = seg.size();
    L->off.resize(np + 1);
    int64_t acc = 0;
    for (size_t p = 0; p < np; ++p) {
        L->off[p] = acc;
        acc += seg[p];
        L->max_seg = std::max(L->max_seg, seg[p]);
    }
    L->off[np] = acc;
    L->total = acc;
    std::vector<uint32_t> chunk((size_t)L->chunks());
    for (size_t p = 0; p < np; ++p)
        for (int64_t b = L->off[p] / 256; b < L->off[p + 1] / 256; ++b) chunk[(size_t)b] = (uint32_t)p;
    uint64_t h = 1469598103934665603ull;  // FNV-1a over the offsets
    for (int64_t v : L->off)
        for (int k = 0; k < 8; ++k) {
            h ^= (uint64_t)((v >> (8 * k)) & 0xFF);
            h *= 1099511628211ull;
        }
    L->tag = h;
    if (hipMalloc((void**)&L->off_dev, sizeof(int64_t) * (np + 1)) != hipSuccess) return nullptr;
    if (hipMalloc((void**)&L->chunk_dev, sizeof(uint32_t) * std::max<size_t>(chunk.size(), 1)) !=
        hipSuccess)
        return nullptr;
    if (hipMemcpy(L->off_dev, L->off.data(), sizeof(int64_t) * (np + 1), hipMemcpyHostToDevice) !=
        hipSuccess)
        return nullptr;
    if (!chunk.empty() && hipMemcpy(L->chunk_dev, chunk.data(), sizeof(uint32_t) * chunk.size(),
                                    hipMemcpyHostToDevice) != hipSuccess)
        return nullptr;
    return L;
}

// The segment of a particle with count links: a quarter and 256 records to
// spare, in whole chunks.
int64_t link_segment(int64_t count) { return (count + count / 4 + 256 + 255) / 256 * 256; }

void free_tape(lbm_ctx* c)
{
    for (auto& t : c->tape) (void)hipFree(t.links);
    for (void* s : c->tape_slabs) (void)hipFree(s);
    c->tape_slabs.clear();
    c->tape.clear();
    c->tape_len = 0;
    c->tape_steps = 0;
    c->taping = false;
}

// The launcher of the configured lattice.
#define LQ(c, fn) ((c)->cfg.lattice == LBM_LATTICE_D3Q15 ? q15::fn : q19::fn)

// Record the step about to stream: the owners of the last classification, its
// links, the particles (the populations with the reconstructed ghost slots
// are the step's own source buffer, the tape slot).
//
// Population buffers while taping.  Step s of a window streams from tape
// slot s into slot s + 1 (its first step copies the current populations into
// slot 0 once), and the last step of the window into a caller buffer, so the
// tape holds every step's populations without a copy per step.  The previous
// level, which a following classification refills from, may then be a tape
// slot; settle_buffers moves both levels back to the caller's buffers before
// the tape is reused or released.
bool caller_buffer(const lbm_ctx* c, const void* p)
{
    return p == c->fu[0] || p == c->fu[1];
}

int settle_buffers(lbm_ctx* c)
{
    void*& cur = c->f[c->cur];
    void*& prev = c->f[1 - c->cur];
    if (!caller_buffer(c, cur)) {
        void* dst = (prev == c->fu[0]) ? c->fu[1] : c->fu[0];
        HIPCHK(c, hipMemcpyAsync(dst, cur, c->sizes.population_bytes, hipMemcpyDeviceToDevice,
                                 c->stream));
        cur = dst;
    }
    if (!caller_buffer(c, prev) || prev == cur) {
        void* dst = (cur == c->fu[0]) ? c->fu[1] : c->fu[0];
        // the previous level matters only to a refill still to come
        if (c->stepped_since_classify && prev != cur)
            HIPCHK(c, hipMemcpyAsync(dst, prev, c->sizes.population_bytes,
                                     hipMemcpyDeviceToDevice, c->stream));
        prev = dst;
    }
    return LBM_OK;
}

int record_tape_step(lbm_ctx* c, const lbm_particles* P)
{
    const int np = c->cfg.n_particles;
    TapeStep& t = c->tape[c->tape_len];
    // the populations are already in t.f: lbm_step streams into the slots;
    // owners and links: a geometry snapshot's, or copies
    if (c->geo_own) {
        t.own_use = c->geo_own;
        t.links_use = c->geo_links;
        t.lay = c->lay;
        t.link_max = c->link_max;
        if (np > 0) HIPCHK(c, LQ(c, launch_tape_small)(c, t, P));
        c->tape_len += 1;
        return LBM_OK;
    }
    HIPCHK(c, hipMemcpyAsync(t.own, c->own[c->own_cur], c->sizes.owner_bytes,
                             hipMemcpyDeviceToDevice, c->stream));
    t.own_use = t.own;
    t.links_use = t.links;
    if (np > 0) {
        const int64_t need = std::max<int64_t>(c->lay->total, 1);
        if (t.link_alloc < need) {
            HIPCHK(c, hipFree(t.links));
            t.links = nullptr;
            if (alloc(&t.links, (size_t)need) != hipSuccess)
                return fail(c, LBM_ENOMEM, "tape link allocation failed");
            t.link_alloc = need;
        }
        t.links_use = t.links;
        t.lay = c->lay;
        t.link_max = c->link_max;
        if (c->link_max > 0 && c->lay->total > 0)
            HIPCHK(c, hipMemcpyAsync(t.links, c->links, sizeof(LinkRec) * (size_t)c->lay->total,
                                     hipMemcpyDeviceToDevice, c->stream));
        // cursors, particle state and the DEM state the next dem_step starts
        // from (for the coupled adjoint), in one launch
        HIPCHK(c, LQ(c, launch_tape_small)(c, t, P));
    }
    c->tape_len += 1;
    return LBM_OK;
}

// Doubles of one taped step's DEM state: pair records, wall records, contact
// sums.
size_t dem_tape_doubles(int np)
{
    const size_t n = (size_t)std::max(np, 1);
    return n * kPairSlots * 8 + n * 48 + n * 6;
}

// Contact histories (kPairSlots keyed records per particle for its pairs,
// six per particle for the walls) and the pair list of a dem_step call;
// allocated by lbm_init, so that dem_step never allocates.
int dem_alloc(lbm_ctx* c)
{
    const size_t np = (size_t)c->cfg.n_particles;
    if (c->hist_pp || np == 0) return LBM_OK;
    const size_t slots = np * kPairSlots;
    if (alloc(&c->hist_pp, slots * 8) != hipSuccess || alloc(&c->hist_key, slots) != hipSuccess ||
        alloc(&c->hist_pw, np * 6 * 8) != hipSuccess || alloc(&c->pairs, slots) != hipSuccess ||
        alloc(&c->pair_count, 1) != hipSuccess)
        return fail(c, LBM_ENOMEM, "contact history allocation failed");
    HIPCHK(c, hipMemsetAsync(c->hist_pp, 0, sizeof(double) * slots * 8, c->stream));
    HIPCHK(c, hipMemsetAsync(c->hist_key, 0, sizeof(int32_t) * slots, c->stream));
    HIPCHK(c, hipMemsetAsync(c->hist_pw, 0, sizeof(double) * np * 6 * 8, c->stream));
    if (np >= (size_t)kGridMinParticles) {
        // counts and starts, cursors, the binned particles, the grid's shape
        c->grid_cap = (int64_t)std::max<size_t>(4096, 4 * np);
        const size_t words = 2 * (size_t)c->grid_cap + 1 + np + 4;
        if (alloc(&c->grid, words) != hipSuccess || alloc(&c->grid_size, 4) != hipSuccess)
            return fail(c, LBM_ENOMEM, "broad-phase grid allocation failed");
    }
    return LBM_OK;
}

// The work space of a dem_step call on the context.
DemScratch dem_scratch(lbm_ctx* c)
{
    DemScratch ws{c->pairs, c->pair_count, c->reach};
    if (c->grid) {
        ws.gcount = c->grid;
        ws.gcursor = c->grid + c->grid_cap + 1;
        ws.gitem = c->grid + 2 * c->grid_cap + 1;
        ws.gdim = reinterpret_cast<int32_t*>(ws.gitem + c->cfg.n_particles);
        ws.gsize = c->grid_size;
        ws.gcap = c->grid_cap;
    }
    return ws;
}

// Bytes of the DEM state saved by lbm_dem_checkpoint_save, in its order: the
// pair histories, their partner keys, the wall histories, the contact sums.
struct DemStateBytes {
    size_t pp, key, pw, fc;
};
DemStateBytes dem_state_bytes(size_t np)
{
    return {sizeof(double) * np * kPairSlots * 8, sizeof(int32_t) * np * kPairSlots,
            sizeof(double) * np * 6 * 8, sizeof(double) * np * 6};
}

// Number of lattice velocities of the configured lattice (0 selects D3Q19).
int lattice_q(const lbm_config* cfg)
{
    return cfg->lattice == LBM_LATTICE_D3Q15 ? 15 : 19;
}

}  // namespace

extern "C" {

int lbm_query_sizes(const lbm_config* cfg, lbm_sizes* out)
{
    if (!cfg || !out) return fail(nullptr, LBM_EINVAL, "null argument");
    if (cfg->lattice != 0 && cfg->lattice != LBM_LATTICE_D3Q19 && cfg->lattice != LBM_LATTICE_D3Q15)
        return fail(nullptr, LBM_EINVAL, "unknown lattice");
    if (cfg->nx < 1 || cfg->ny < 1 || cfg->nz < 1)
        return fail(nullptr, LBM_EINVAL, "lattice dimensions must be >= 1");
    const int64_t ncell = (int64_t)cfg->nx * cfg->ny * cfg->nz;
    if (ncell >= (int64_t)1 << 31) return fail(nullptr, LBM_EINVAL, "more than 2^31 - 1 cells");
    const size_t es = elem_bytes(cfg->storage);
    if (!es) return fail(nullptr, LBM_EINVAL, "unknown storage");
    out->ncell = ncell;
    out->cell_stride = (ncell + 63) / 64 * 64;
    out->population_bytes = (size_t)lattice_q(cfg) * (size_t)out->cell_stride * es;
    out->owner_bytes = (size_t)ncell * sizeof(uint32_t);
    out->flag_bytes = (size_t)ncell;
    out->moment_bytes = (size_t)ncell * 4 * es;
    out->checkpoint_bytes = out->population_bytes + out->moment_bytes;
    out->adjoint_bytes = (size_t)lattice_q(cfg) * (size_t)out->cell_stride * (es == 8 ? 8 : 4);
    {
        const size_t np = (size_t)std::max(cfg->n_particles, 0);
        const DemStateBytes b = dem_state_bytes((size_t)np);
        out->dem_checkpoint_bytes = b.pp + b.key + b.pw + b.fc;
        out->contact_adjoint_bytes = sizeof(double) * np * kAdjContact;
    }
    return LBM_OK;
}

int lbm_init(const lbm_config* cfg, const lbm_buffers* bufs, lbm_ctx** out)
{
    if (!cfg || !bufs || !out) return fail(nullptr, LBM_EINVAL, "null argument");
    if (cfg->classify_mode < LBM_CLASSIFY_AUTO || cfg->classify_mode > LBM_CLASSIFY_BALLS)
        return fail(nullptr, LBM_EINVAL, "unknown classify_mode");
    if (cfg->force_sum != LBM_FORCE_SUM_ATOMIC && cfg->force_sum != LBM_FORCE_SUM_EXACT)
        return fail(nullptr, LBM_EINVAL, "unknown force_sum");
    if (cfg->treatments &
        ~(LBM_TREAT_VIBB | LBM_TREAT_MISSING | LBM_TREAT_EXACT_Q | LBM_TREAT_NEQ_SPLIT))
        return fail(nullptr, LBM_EINVAL, "unknown treatment bits");
    *out = nullptr;
    lbm_sizes sz;
    int rc = lbm_query_sizes(cfg, &sz);
    if (rc) return rc;
    if (!(cfg->tau > 0.5)) return fail(nullptr, LBM_EINVAL, "tau must exceed 1/2");
    if (!(cfg->rho0 > 0.0)) return fail(nullptr, LBM_EINVAL, "rho0 must be positive");
    if (!bufs->f_dev[0] || !bufs->f_dev[1] || !bufs->owner_dev[0] || !bufs->owner_dev[1] ||
        !bufs->flag_dev || !bufs->moments_dev)
        return fail(nullptr, LBM_EINVAL, "null buffer");
    if (cfg->n_particles < 0 || cfg->n_particles >= 65535)
        return fail(nullptr, LBM_EINVAL, "n_particles must be in [0, 65535)");
    if (cfg->n_particles > 0 && (cfg->box_half < 2 || cfg->box_half > kMaxBoxHalf))
        return fail(nullptr, LBM_EINVAL, "box_half must lie in [2, 511]");
    const int dims[3] = {cfg->nx, cfg->ny, cfg->nz};
    for (int a = 0; a < 3; ++a)
        if (cfg->n_particles > 0 && cfg->periodic[a] && dims[a] < 2 * cfg->box_half + 5)
            return fail(nullptr, LBM_EINVAL,
                        "a periodic axis must have at least 2*box_half + 5 nodes");

    lbm_ctx* c = new (std::nothrow) lbm_ctx;
    if (!c) return fail(nullptr, LBM_ENOMEM, "context allocation failed");
    c->cfg = *cfg;
    c->sizes = sz;
    c->stream = (hipStream_t)cfg->stream;
    for (int a = 0; a < 3; ++a) {
        c->geom.n[a] = dims[a];
        c->geom.per[a] = cfg->periodic[a] ? 1 : 0;
    }
    c->geom.stride = sz.cell_stride;
    c->geom.ncell = (uint32_t)sz.ncell;
    Phys& ph = c->phys;
    ph.tau = cfg->tau;
    ph.omega = 1.0 / cfg->tau;
    ph.omegaf = (float)ph.omega;
    ph.rho0 = cfg->rho0;
    for (int a = 0; a < 3; ++a) {
        ph.F[a] = cfg->body_force[a];
        ph.Ff[a] = (float)cfg->body_force[a];
    }
    if (cfg->storage == LBM_STORE_F16) {
        ph.scale = cfg->h16_scale > 0.0 ? (float)cfg->h16_scale : 1024.0f;
    } else {
        ph.scale = 1.0f;
    }
    ph.inv_scale = 1.0f / ph.scale;
    ph.neq_split = (cfg->treatments & LBM_TREAT_NEQ_SPLIT) ? 1 : 0;
    const int h = std::max(cfg->box_half, 2);
    c->box.h = h;
    c->box.S = 2 * h + 1;
    c->box.vol = c->box.S * c->box.S * c->box.S;
    c->box.tiles = (c->box.vol + 255) / 256;
    for (int i = 0; i < 2; ++i) {
        c->f[i] = c->fu[i] = bufs->f_dev[i];
        c->own[i] = bufs->owner_dev[i];
    }
    c->flag = bufs->flag_dev;
    c->mom = bufs->moments_dev;

    const int np = cfg->n_particles;
    const int64_t S2 = (int64_t)c->box.S * c->box.S;
    // Clearing, flags and refill detection walk each particle's ball unless
    // the balls (radius below box_half) could cover most of the lattice,
    // where one coalesced sweep of the whole lattice is cheaper.
    if (cfg->classify_mode == LBM_CLASSIFY_AUTO) {
        const double r = (double)c->box.h - 1.0;
        const double balls = (double)np * 4.18879 * r * r * r;
        c->dense = balls > 0.5 * (double)sz.ncell;
    } else {
        c->dense = cfg->classify_mode == LBM_CLASSIFY_SWEEP;
    }
    // every segment sized for the largest box until a classification has
    // counted each particle's links
    const int64_t seg0 = std::max<int64_t>(256, (32 * S2 + 255) / 256 * 256);
    c->cand_cap = std::max<int64_t>(256, (8 * S2 + 255) / 256 * 256);
    c->refill_cap = std::max<int64_t>(1 << 16, (int64_t)np * S2);
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = alloc(&c->ball_hist, (size_t)3 * 4 * std::max(np, 1));
    const size_t np1 = (size_t)std::max(np, 1);
    if (e == hipSuccess) e = alloc(&c->ctr, (size_t)kStageHead + 2 * (size_t)kCursorPad * np1);
    if (e == hipSuccess) {
        c->refill_cursor = c->ctr + kCtrRefill;
        c->err = c->ctr + kCtrErr;
        c->numeric = c->ctr + kCtrNumeric;
        c->link_cursor = c->ctr + kStageHead;
        c->cand_cursor = c->ctr + kStageHead + (size_t)kCursorPad * np1;
        e = hipMemsetAsync(c->ctr, 0, sizeof(uint32_t) * (kStageHead + 2 * kCursorPad * np1),
                           c->stream);
    }
    if (e == hipSuccess && np) e = alloc(&c->cand, (size_t)np * c->cand_cap);
    if (e == hipSuccess && np && c->dense) {
        c->cand_prev_cap = c->cand_cap;
        e = alloc(&c->cand_prev, (size_t)np * c->cand_prev_cap);
        if (e == hipSuccess) e = alloc(&c->cand_prev_count, (size_t)np);
        if (e == hipSuccess) e = alloc(&c->quat_prev, (size_t)4 * np);
        if (e == hipSuccess) e = hipMemsetAsync(c->cand_prev_count, 0, sizeof(uint32_t) * np, c->stream);
    }
    if (e == hipSuccess) {
        c->lay = make_layout(std::vector<int64_t>((size_t)np, seg0));
        c->lay_initial = true;
        if (!c->lay) e = hipErrorOutOfMemory;
    }
    if (e == hipSuccess && np) e = alloc(&c->links, (size_t)c->lay->total);
    if (e == hipSuccess) e = alloc(&c->refill, (size_t)c->refill_cap);
    if (e == hipSuccess) e = alloc(&c->FT, (size_t)6 * std::max(np, 1));
    if (e == hipSuccess && np && cfg->force_sum == LBM_FORCE_SUM_EXACT)
        e = alloc(&c->FX, (size_t)12 * np);
    if (e == hipSuccess) e = alloc(&c->fc, (size_t)6 * std::max(np, 1));
    if (e == hipSuccess) e = alloc(&c->reach, (size_t)std::max(np, 1));
    if (e == hipSuccess)
        e = hipHostMalloc((void**)&c->host_stage,
                          sizeof(uint32_t) * (kStageHead + 2 * (size_t)kCursorPad * np1),
                          hipHostMallocDefault);
    if (e != hipSuccess) {
        std::string msg = std::string("scratch allocation failed: ") + hipGetErrorString(e);
        lbm_destroy(c);
        return fail(nullptr, LBM_ENOMEM, msg);
    }
    if (dem_alloc(c) != LBM_OK) {
        std::string msg = c->last_error;
        lbm_destroy(c);
        return fail(nullptr, LBM_ENOMEM, msg);
    }
    // the device, and the address of the allocation-free DEM entry point's
    // work space on it
    e = hipGetDevice(&c->device);
    if (e == hipSuccess) e = dem_noalloc_setup();
    if (e != hipSuccess) {
        std::string msg = std::string("device set-up failed: ") + hipGetErrorString(e);
        lbm_destroy(c);
        return fail(nullptr, LBM_EDEVICE, msg);
    }
    e = LQ(c, launch_init_equilibrium)(c, c->f[0]);
    if (e == hipSuccess) e = hipMemsetAsync(c->own[0], 0xFF, sz.owner_bytes, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->own[1], 0xFF, sz.owner_bytes, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->flag, 0, sz.flag_bytes, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->FT, 0, sizeof(double) * 6 * std::max(np, 1), c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->fc, 0, sizeof(double) * 6 * std::max(np, 1), c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        std::string msg = std::string("initialisation failed: ") + hipGetErrorString(e);
        lbm_destroy(c);
        return fail(nullptr, LBM_EDEVICE, msg);
    }
    c->cur = 0;
    *out = c;
    return LBM_OK;
}

int lbm_destroy(lbm_ctx* c)
{
    if (!c) return LBM_OK;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    (void)hipFree(c->ball_hist);
    (void)hipFree(c->links);
    (void)hipFree(c->cand);
    (void)hipFree(c->refill);
    (void)hipFree(c->ctr);
    (void)hipFree(c->FT);
    (void)hipFree(c->FX);
    (void)hipFree(c->cand_prev);
    (void)hipFree(c->cand_prev_count);
    (void)hipFree(c->quat_prev);
    (void)hipFree(c->fc);
    (void)hipFree(c->reach);
    free_tape(c);
    (void)hipFree(c->adj_scratch);
    (void)hipFree(c->adj_wts);
    (void)hipFree(c->adj_sig);
    (void)hipFree(c->adj_list);
    (void)hipFree(c->adj_count);
    (void)hipFree(c->hist_pp);
    (void)hipFree(c->hist_key);
    (void)hipFree(c->pairs);
    (void)hipFree(c->pair_count);
    (void)hipFree(c->grid);
    (void)hipFree(c->grid_size);
    (void)hipFree(c->hist_pw);
    if (c->host_stage) (void)hipHostFree(c->host_stage);
    for (hipStream_t s : {c->s_bulk, c->s_dem})
        if (s) {
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
        }
    for (hipEvent_t e : {c->ev_fork, c->ev_bulk, c->ev_dem})
        if (e) (void)hipEventDestroy(e);
    for (auto& t : c->timed) {
        (void)hipEventDestroy(t.start);
        (void)hipEventDestroy(t.stop);
    }
    for (auto e : c->event_pool) (void)hipEventDestroy(e);
    delete c;
    return LBM_OK;
}

const char* lbm_last_error(const lbm_ctx* c)
{
    return c ? c->last_error.c_str() : g_init_error.c_str();
}

}  // extern "C"

namespace {

// The buffers one classification uses: its owner planes (new and previous),
// its slots of the ball history, and the populations its refill reads.
struct ClassifyPlan {
    int64_t k;
    int slot, slot_prev, slot_prev2;
    uint32_t* own_new;
    const uint32_t* own_prev;
    const void* refill_src;
    bool inc;  // dense mode: flags and refills from the previous candidate lists
};

ClassifyPlan classify_plan(const lbm_ctx* c)
{
    ClassifyPlan cp;
    cp.k = c->n_classify;
    cp.slot = (int)(cp.k % 3);
    cp.slot_prev = (int)((cp.k + 2) % 3);
    cp.slot_prev2 = (int)((cp.k + 1) % 3);
    cp.own_new = c->own[cp.k % 2];
    cp.own_prev = c->own[(cp.k + 1) % 2];
    // populations of the time level the previous classification describes
    cp.refill_src = c->stepped_since_classify ? c->f[1 - c->cur] : c->f[c->cur];
    cp.inc = c->dense && cp.k >= 1 && c->inc_ok && c->cfg.n_particles > 0 && c->cand_prev;
    return cp;
}

// Enqueue a classification: counters reset, boxes, owners, flags, candidates,
// links, then the refill, which reads its list's length on the device.
int classify_enqueue(lbm_ctx* c, const PartDev& Pd, const ClassifyPlan& cp)
{
    const int np = c->cfg.n_particles;
    if (c->dense && c->cand_prev) {
        // this classification's candidates go into the other list (which
        // holds those of two classifications ago, no longer needed: it is
        // grown first if the lists grew since); the counter reset keeps the
        // counts of the lists just set aside
        if (c->cand_prev_cap < c->cand_cap) {
            HIPCHK(c, hipFree(c->cand_prev));
            c->cand_prev = nullptr;
            c->cand_prev_cap = c->cand_cap;
            if (alloc(&c->cand_prev, (size_t)np * c->cand_prev_cap) != hipSuccess)
                return fail(c, LBM_ENOMEM, "candidate list allocation failed");
        }
        std::swap(c->cand, c->cand_prev);
        std::swap(c->cand_cap, c->cand_prev_cap);
    }
    HIPCHK(c, LQ(c, launch_reset_counters)(c));
    // the boxes' check is read back with the list counts; the kernels that
    // write the owner planes, flags and lists do nothing when it failed, so
    // the context keeps its current geometry
    HIPCHK(c, LQ(c, launch_boxes)(c, Pd, cp.slot, cp.slot_prev, cp.inc || (c->dense && np > 0)));
    {
        PhaseTimer tm(c, LBM_PHASE_CLASSIFY);
        if (cp.k >= 2) HIPCHK(c, LQ(c, launch_clear_boxes)(c, cp.own_new, cp.slot_prev2, np));
        HIPCHK(c, LQ(c, launch_mark)(c, cp.own_new, Pd, cp.slot, cp.inc));
        // the lattice sweep also runs on a first classification (own_prev
        // is all fluid then): in dense mode it writes every flag
        if (cp.k >= 1 || c->dense)
            HIPCHK(c, LQ(c, launch_finish)(c, cp.own_prev, cp.own_new, cp.slot_prev, np, cp.inc));
        HIPCHK(c, LQ(c, launch_links)(c, cp.own_new, Pd, cp.slot));
    }
    if (cp.k >= 1) {
        // should the list overflow, lbm_classify_nodes runs it again over
        // the grown list
        PhaseTimer tm(c, LBM_PHASE_REFILL);
        HIPCHK(c, LQ(c, launch_refill)(c, cp.refill_src, c->f[c->cur], cp.own_prev, Pd));
    }
    return LBM_OK;
}

void classify_commit(lbm_ctx* c, const ClassifyPlan& cp)
{
    c->inc_ok = c->dense;  // its candidate lists and orientations are kept
    c->geo_own = nullptr;
    c->geo_links = nullptr;
    c->own_cur = (int)(cp.k % 2);
    c->n_classify = cp.k + 1;
    c->stepped_since_classify = false;
}

// What asynchronous classifications latched, and the non-finite force flag,
// as read back into the staging block; either leaves the context failed.
int deferred_status(lbm_ctx* c, const char* where)
{
    const uint32_t def = c->host_stage[kCtrDeferred];
    if (c->host_stage[kCtrNumeric])
        return fail(c, LBM_ENUMERIC,
                    std::string(where) + ": a step since the previous classification "
                    "produced a non-finite hydrodynamic force or torque");
    if (def) {
        c->failed = true;
        if (def & kDeferredSlots)
            return fail(c, LBM_ECAPACITY,
                        std::string(where) + ": a particle had more than " +
                            std::to_string(kPairSlots) + " candidate contact partners in a "
                            "dem_step call; contacts beyond them were left out");
        if (def & kDeferredOverflow)
            return fail(c, LBM_ECAPACITY,
                        std::string(where) + ": an asynchronous classification outgrew its "
                        "lists (lbm_classify_nodes sizes them); results since are invalid");
        return fail(c, LBM_EINVAL,
                    std::string(where) + ": an asynchronous classification rejected the "
                    "particles: " + err_text(def & 0xFFu));
    }
    c->deferred = false;
    return LBM_OK;
}

// Drain the stream and report what asynchronous classifications latched.
int check_deferred(lbm_ctx* c, const char* where)
{
    HIPCHK(c, hipMemcpyAsync(c->host_stage, c->ctr, sizeof(uint32_t) * kStageHead,
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (!c->deferred && !c->host_stage[kCtrNumeric] && !c->host_stage[kCtrDeferred])
        return LBM_OK;
    return deferred_status(c, where);
}

}  // namespace

extern "C" {

int lbm_classify_nodes(lbm_ctx* c, const lbm_particles* P, lbm_counts* out)
{
    if (!c) return fail(nullptr, LBM_EINVAL, "null context");
    if (c->failed) return fail(c, LBM_ESTATE, "context failed earlier: " + c->last_error);
    int rc = check_particles(c, P, false);
    if (rc) return rc;
    const int np = c->cfg.n_particles;
    const PartDev Pd = to_dev(P);
    const ClassifyPlan cp = classify_plan(c);
    const int64_t k = cp.k;
    const size_t cur_bytes = sizeof(uint32_t) * kCursorPad * std::max(np, 1);

    if (np > 0) {
        rc = classify_enqueue(c, Pd, cp);
        if (rc) return rc;
        uint32_t* link_counts = c->host_stage + kStageHead;
        uint32_t* cand_counts = c->host_stage + kStageHead + (size_t)kCursorPad * np;
        for (int attempt = 0;; ++attempt) {
            // one copy of the whole counter block
            HIPCHK(c, hipMemcpyAsync(c->host_stage, c->ctr,
                                     sizeof(uint32_t) * kStageHead + 2 * cur_bytes,
                                     hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
            rc = deferred_status(c, "lbm_classify_nodes");
            if (rc) return rc;
            if (c->host_stage[kCtrErr])
                return fail(c, LBM_EINVAL,
                            "lbm_classify_nodes: " + err_text(c->host_stage[kCtrErr]));
            int64_t lmax = 0, ltot = 0, cmax = 0, ctot = 0;
            for (int p = 0; p < np; ++p) {
                const int64_t v = link_counts[(size_t)p * kCursorPad];
                lmax = std::max(lmax, v);
                ltot += v;
                cmax = std::max<int64_t>(cmax, cand_counts[(size_t)p * kCursorPad]);
                ctot += cand_counts[(size_t)p * kCursorPad];
            }
            const int64_t nref = c->host_stage[kCtrRefill];
            const bool grow_cand = cmax > c->cand_cap;
            // a segment outgrown, or the first counts: every segment sized
            // from its own particle's count (and never below what it was,
            // once sized)
            bool grow_links = c->lay_initial;
            for (int p = 0; p < np && !grow_links; ++p)
                grow_links = link_counts[(size_t)p * kCursorPad] >
                             c->lay->off[p + 1] - c->lay->off[p];
            const bool grow_refill = nref > c->refill_cap;
            if (!grow_cand && !grow_links && !grow_refill) {
                c->link_max = lmax;
                c->link_total = ltot;
                c->cand_total = ctot;
                c->refill_total = (k >= 1) ? nref : 0;
                break;
            }
            if (attempt > 2) return fail(c, LBM_ENOMEM, "link/refill lists keep overflowing");
            if (grow_cand) {
                HIPCHK(c, hipFree(c->cand));
                c->cand = nullptr;
                c->cand_cap = (cmax + cmax / 4 + 255) / 256 * 256;
                if (alloc(&c->cand, (size_t)np * c->cand_cap) != hipSuccess)
                    return fail(c, LBM_ENOMEM, "candidate list allocation failed");
                HIPCHK(c, hipMemsetAsync(c->cand_cursor, 0, cur_bytes, c->stream));
                HIPCHK(c, LQ(c, launch_mark)(c, cp.own_new, Pd, cp.slot, cp.inc));  // same owners, full list
            }
            if (grow_links) {
                std::vector<int64_t> seg((size_t)np);
                for (int p = 0; p < np; ++p) {
                    seg[(size_t)p] = link_segment(link_counts[(size_t)p * kCursorPad]);
                    if (!c->lay_initial)
                        seg[(size_t)p] = std::max(seg[(size_t)p],
                                                  c->lay->off[p + 1] - c->lay->off[p]);
                }
                auto lay = make_layout(seg);
                if (!lay) return fail(c, LBM_ENOMEM, "link layout allocation failed");
                HIPCHK(c, hipFree(c->links));
                c->links = nullptr;
                c->lay = lay;
                c->lay_initial = false;
                if (alloc(&c->links, (size_t)std::max<int64_t>(c->lay->total, 1)) != hipSuccess)
                    return fail(c, LBM_ENOMEM, "link list allocation failed");
            }
            if (grow_cand || grow_links) {
                HIPCHK(c, hipMemsetAsync(c->link_cursor, 0, cur_bytes, c->stream));
                HIPCHK(c, LQ(c, launch_links)(c, cp.own_new, Pd, cp.slot));
            }
            if (grow_refill) {
                HIPCHK(c, hipFree(c->refill));
                c->refill = nullptr;
                c->refill_cap = nref + nref / 4 + 1024;
                if (alloc(&c->refill, (size_t)c->refill_cap) != hipSuccess)
                    return fail(c, LBM_ENOMEM, "refill list allocation failed");
                HIPCHK(c, hipMemsetAsync(c->refill_cursor, 0, sizeof(uint32_t), c->stream));
                if (k >= 1) {
                    HIPCHK(c, LQ(c, launch_finish)(c, cp.own_prev, cp.own_new, cp.slot_prev, np,
                                                   cp.inc));
                    PhaseTimer tm(c, LBM_PHASE_REFILL);
                    HIPCHK(c, LQ(c, launch_refill)(c, cp.refill_src, c->f[c->cur], cp.own_prev, Pd));
                }
            }
        }
    } else {
        c->link_max = c->link_total = c->refill_total = 0;
    }
    c->counts_known = true;
    classify_commit(c, cp);
    if (out) {
        out->n_links = c->link_total;
        out->n_refill = c->refill_total;
        out->n_candidates = c->cand_total;
    }
    return LBM_OK;
}

int lbm_classify_nodes_async(lbm_ctx* c, const lbm_particles* P)
{
    if (!c) return fail(nullptr, LBM_EINVAL, "null context");
    if (c->failed) return fail(c, LBM_ESTATE, "context failed earlier: " + c->last_error);
    int rc = check_particles(c, P, false);
    if (rc) return rc;
    const ClassifyPlan cp = classify_plan(c);
    if (c->cfg.n_particles > 0) {
        rc = classify_enqueue(c, to_dev(P), cp);
        if (rc) return rc;
        HIPCHK(c, LQ(c, launch_latch_deferred)(c));
        c->link_max = c->lay->max_seg;  // lbm_step covers every segment whole
        c->deferred = true;
    } else {
        c->link_max = 0;
    }
    c->link_total = c->cand_total = c->refill_total = 0;
    c->counts_known = false;
    classify_commit(c, cp);
    return LBM_OK;
}

int lbm_step(lbm_ctx* c, const lbm_particles* P)
{
    if (!c) return fail(nullptr, LBM_EINVAL, "null context");
    if (c->failed) return fail(c, LBM_ESTATE, "context failed earlier: " + c->last_error);
    int rc = check_particles(c, P, false);
    if (rc) return rc;
    const int np = c->cfg.n_particles;
    const int s = c->tape_len;
    const bool taped = c->taping && s < c->tape_steps;
    if (taped && c->f[c->cur] != c->tape[s].f) {
        // the window's first step: its populations move into slot 0
        HIPCHK(c, hipMemcpyAsync(c->tape[s].f, c->f[c->cur], c->sizes.population_bytes,
                                 hipMemcpyDeviceToDevice, c->stream));
        c->f[c->cur] = c->tape[s].f;
    }
    void* src = c->f[c->cur];
    void* dst = (taped && s + 1 < c->tape_steps) ? c->tape[s + 1].f
                                                 : (src == c->fu[0] ? c->fu[1] : c->fu[0]);
    {
        PhaseTimer tm(c, LBM_PHASE_BOUNDARY);
        HIPCHK(c, LQ(c, launch_zero_f64)(c, c->FT, 6 * (int64_t)np));
        if (np > 0 && c->n_classify > 0) HIPCHK(c, LQ(c, launch_boundary)(c, src, to_dev(P)));
    }
    if (taped) {
        int rc2 = record_tape_step(c, P);
        if (rc2) return rc2;
    }
    {
        PhaseTimer tm(c, LBM_PHASE_BULK);
        HIPCHK(c, LQ(c, launch_stream_collide)(c, src, dst));
    }
    c->f[1 - c->cur] = dst;
    c->cur = 1 - c->cur;
    c->stepped_since_classify = true;
    return LBM_OK;
}

int lbm_particle_forces(const lbm_ctx* c, double* F_dev, double* T_dev)
{
    if (!c) return fail(nullptr, LBM_EINVAL, "null context");
    if (!F_dev || !T_dev) return fail(const_cast<lbm_ctx*>(c), LBM_EINVAL, "null output");
    HIPCHK(const_cast<lbm_ctx*>(c), LQ(c, launch_split_forces)(c, F_dev, T_dev));
    return LBM_OK;
}

int dem_step(lbm_ctx* c, lbm_particles* P, int n_sub, double dt, const dem_params* prm)
{
    if (!c) return fail(nullptr, LBM_EINVAL, "null context");
    if (c->failed) return fail(c, LBM_ESTATE, "context failed earlier: " + c->last_error);
    if (!prm) return fail(c, LBM_EINVAL, "null DEM parameters");
    if (n_sub < 1) return fail(c, LBM_EINVAL, "n_sub must be >= 1");
    if (!(dt > 0.0)) return fail(c, LBM_EINVAL, "dt must be positive");
    int rc = check_particles(c, P, true);
    if (rc) return rc;
    const int np = c->cfg.n_particles;
    if (np == 0) return LBM_OK;
    PhaseTimer tm(c, LBM_PHASE_DEM);
    HIPCHK(c, launch_dem(c, to_dev(P), n_sub, dt, *prm, dem_scratch(c)));
    return LBM_OK;
}

int lbm_step_dem(lbm_ctx* c, lbm_particles* P, int n_sub, double dt, const dem_params* prm)
{
    if (!c) return fail(nullptr, LBM_EINVAL, "null context");
    if (c->failed) return fail(c, LBM_ESTATE, "context failed earlier: " + c->last_error);
    if (!prm) return fail(c, LBM_EINVAL, "null DEM parameters");
    if (n_sub < 1) return fail(c, LBM_EINVAL, "n_sub must be >= 1");
    if (!(dt > 0.0)) return fail(c, LBM_EINVAL, "dt must be positive");
    int rc = check_particles(c, P, true);
    if (rc) return rc;
    const int np = c->cfg.n_particles;
    // a taped step (its output goes to the tape), no particles or no
    // classification yet: the two calls one after the other
    const bool taped = c->taping && c->tape_len < c->tape_steps;
    if (taped || np == 0 || c->n_classify == 0) {
        rc = lbm_step(c, P);
        return rc ? rc : dem_step(c, P, n_sub, dt, prm);
    }
    rc = overlap_streams(c);
    if (rc) return rc;
    void* src = c->f[c->cur];
    void* dst = src == c->fu[0] ? c->fu[1] : c->fu[0];
    {
        PhaseTimer tm(c, LBM_PHASE_BOUNDARY);
        HIPCHK(c, LQ(c, launch_zero_f64)(c, c->FT, 6 * (int64_t)np));
        HIPCHK(c, LQ(c, launch_boundary)(c, src, to_dev(P)));
    }
    // both passes start after the link pass (forces complete), and the
    // caller's stream continues after both
    HIPCHK(c, hipEventRecord(c->ev_fork, c->stream));
    HIPCHK(c, hipStreamWaitEvent(c->s_bulk, c->ev_fork, 0));
    HIPCHK(c, hipStreamWaitEvent(c->s_dem, c->ev_fork, 0));
    {
        OnStream os(c, c->s_bulk);
        PhaseTimer tm(c, LBM_PHASE_BULK);
        HIPCHK(c, LQ(c, launch_stream_collide)(c, src, dst));
        HIPCHK(c, hipEventRecord(c->ev_bulk, c->s_bulk));
    }
    {
        OnStream os(c, c->s_dem);
        PhaseTimer tm(c, LBM_PHASE_DEM);
        HIPCHK(c, launch_dem(c, to_dev(P), n_sub, dt, *prm,
                             dem_scratch(c)));
        HIPCHK(c, hipEventRecord(c->ev_dem, c->s_dem));
    }
    HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_bulk, 0));
    HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_dem, 0));
    c->f[1 - c->cur] = dst;
    c->cur = 1 - c->cur;
    c->stepped_since_classify = true;
    return LBM_OK;
}

int dem_step_noalloc(lbm_ctx* c, lbm_particles* P, int n_sub, double dt, const dem_params* prm)
{
    if (!c) return fail(nullptr, LBM_EINVAL, "null context");
    if (c->failed) return fail(c, LBM_ESTATE, "context failed earlier: " + c->last_error);
    if (!prm) return fail(c, LBM_EINVAL, "null DEM parameters");
    if (n_sub < 1) return fail(c, LBM_EINVAL, "n_sub must be >= 1");
    if (!(dt > 0.0)) return fail(c, LBM_EINVAL, "dt must be positive");
    const int np = c->cfg.n_particles;
    if (np > kNoAllocParticles)
        return fail(c, LBM_EINVAL,
                    "dem_step_noalloc: " + std::to_string(np) + " particles, more than the " +
                        std::to_string(kNoAllocParticles) + " its static work space holds "
                        "(use dem_step)");
    int rc = check_particles(c, P, true);
    if (rc) return rc;
    if (np == 0) return LBM_OK;
    DemScratch ws;
    if (!dem_noalloc_scratch(c->device, &ws))
        return fail(c, LBM_ESTATE, "dem_step_noalloc: work space of this device not set up");
    PhaseTimer tm(c, LBM_PHASE_DEM);
    HIPCHK(c, launch_dem(c, to_dev(P), n_sub, dt, *prm, ws));
    return LBM_OK;
}

int lbm_get_links(const lbm_ctx* cc, int64_t cap, int32_t* node_dev, int8_t* d_dev,
                  int8_t* kind_dev, int32_t* part_dev, double* q_dev, int64_t* n_out)
{
    lbm_ctx* c = const_cast<lbm_ctx*>(cc);
    if (!c || !n_out) return fail(c, LBM_EINVAL, "null argument");
    if (!c->counts_known)
        return fail(c, LBM_ESTATE, "the last classification was asynchronous: no counts");
    *n_out = c->link_total;
    if (c->link_total == 0) return LBM_OK;
    if (cap < c->link_total) return fail(c, LBM_ECAPACITY, "link output too small");
    if (!node_dev || !d_dev || !kind_dev || !part_dev || !q_dev)
        return fail(c, LBM_EINVAL, "null output");
    const int np = c->cfg.n_particles;
    std::vector<int64_t> off(np);
    int64_t acc = 0;
    for (int p = 0; p < np; ++p) {
        off[p] = acc;
        acc += c->host_stage[kStageHead + (size_t)p * kCursorPad];
    }
    int64_t* off_dev = nullptr;
    HIPCHK(c, alloc(&off_dev, np));
    HIPCHK(c, hipMemcpyAsync(off_dev, off.data(), sizeof(int64_t) * np, hipMemcpyHostToDevice,
                             c->stream));
    HIPCHK(c, LQ(c, launch_link_export)(c, node_dev, d_dev, kind_dev, part_dev, q_dev, off_dev));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipFree(off_dev));
    return LBM_OK;
}

int lbm_get_refill(const lbm_ctx* cc, int64_t cap, int32_t* node_dev, int32_t* part_dev,
                   int64_t* n_out)
{
    lbm_ctx* c = const_cast<lbm_ctx*>(cc);
    if (!c || !n_out) return fail(c, LBM_EINVAL, "null argument");
    if (!c->counts_known)
        return fail(c, LBM_ESTATE, "the last classification was asynchronous: no counts");
    *n_out = c->refill_total;
    if (c->refill_total == 0) return LBM_OK;
    if (cap < c->refill_total) return fail(c, LBM_ECAPACITY, "refill output too small");
    if (!node_dev || !part_dev) return fail(c, LBM_EINVAL, "null output");
    HIPCHK(c, hipMemcpy2DAsync(node_dev, sizeof(int32_t), c->refill, sizeof(RefillRec),
                               sizeof(int32_t), c->refill_total, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpy2DAsync(part_dev, sizeof(int32_t), (const char*)c->refill + sizeof(uint32_t),
                               sizeof(RefillRec), sizeof(int32_t), c->refill_total,
                               hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

int lbm_get_owner(const lbm_ctx* cc, int32_t* owner_dev)
{
    lbm_ctx* c = const_cast<lbm_ctx*>(cc);
    if (!c || !owner_dev) return fail(c, LBM_EINVAL, "null argument");
    HIPCHK(c, LQ(c, launch_owner_export)(c, c->own[c->own_cur], owner_dev));
    return LBM_OK;
}

int lbm_get_populations(const lbm_ctx* cc, double* f_dev)
{
    lbm_ctx* c = const_cast<lbm_ctx*>(cc);
    if (!c || !f_dev) return fail(c, LBM_EINVAL, "null argument");
    HIPCHK(c, LQ(c, launch_get_populations)(c, c->f[c->cur], f_dev));
    return LBM_OK;
}

int lbm_get_moments(const lbm_ctx* cc, double* rho_dev, double* u_dev)
{
    lbm_ctx* c = const_cast<lbm_ctx*>(cc);
    if (!c) return fail(nullptr, LBM_EINVAL, "null context");
    if (!rho_dev || !u_dev) return fail(c, LBM_EINVAL, "null output");
    HIPCHK(c, LQ(c, launch_get_moments)(c, rho_dev, u_dev));
    return LBM_OK;
}

int lbm_set_populations(lbm_ctx* c, const double* f_dev)
{
    if (!c || !f_dev) return fail(c, LBM_EINVAL, "null argument");
    HIPCHK(c, LQ(c, launch_set_populations)(c, c->f[c->cur], f_dev));
    return LBM_OK;
}

int lbm_synchronize(lbm_ctx* c)
{
    if (!c) return fail(nullptr, LBM_EINVAL, "null context");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (!c->failed) return check_deferred(c, "lbm_synchronize");
    return LBM_OK;
}

int lbm_checkpoint_save(const lbm_ctx* cc, void* dst_dev)
{
    lbm_ctx* c = const_cast<lbm_ctx*>(cc);
    if (!c || !dst_dev) return fail(c, LBM_EINVAL, "null argument");
    HIPCHK(c, hipMemcpyAsync(dst_dev, c->f[c->cur], c->sizes.population_bytes,
                             hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync((char*)dst_dev + c->sizes.population_bytes, c->mom,
                             c->sizes.moment_bytes, hipMemcpyDeviceToDevice, c->stream));
    return LBM_OK;
}

int lbm_checkpoint_load(lbm_ctx* c, const void* src_dev)
{
    if (!c || !src_dev) return fail(c, LBM_EINVAL, "null argument");
    if (c->failed) return fail(c, LBM_ESTATE, "context failed earlier: " + c->last_error);
    HIPCHK(c, hipMemcpyAsync(c->f[c->cur], src_dev, c->sizes.population_bytes,
                             hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->mom, (const char*)src_dev + c->sizes.population_bytes,
                             c->sizes.moment_bytes, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemsetAsync(c->own[0], 0xFF, c->sizes.owner_bytes, c->stream));
    HIPCHK(c, hipMemsetAsync(c->own[1], 0xFF, c->sizes.owner_bytes, c->stream));
    HIPCHK(c, hipMemsetAsync(c->flag, 0, c->sizes.flag_bytes, c->stream));
    c->n_classify = 0;
    c->own_cur = 0;
    c->stepped_since_classify = false;
    c->geo_own = nullptr;
    c->geo_links = nullptr;
    c->inc_ok = false;
    c->link_max = c->link_total = c->refill_total = c->cand_total = 0;
    return LBM_OK;
}

int lbm_dem_checkpoint_save(const lbm_ctx* cc, void* dst_dev)
{
    lbm_ctx* c = const_cast<lbm_ctx*>(cc);
    if (!c || !dst_dev) return fail(c, LBM_EINVAL, "null argument");
    const size_t np = (size_t)c->cfg.n_particles;
    if (np == 0) return LBM_OK;
    char* d = (char*)dst_dev;
    const DemStateBytes b = dem_state_bytes(np);
    HIPCHK(c, hipMemcpyAsync(d, c->hist_pp, b.pp, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(d + b.pp, c->hist_key, b.key, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(d + b.pp + b.key, c->hist_pw, b.pw, hipMemcpyDeviceToDevice,
                             c->stream));
    HIPCHK(c, hipMemcpyAsync(d + b.pp + b.key + b.pw, c->fc, b.fc, hipMemcpyDeviceToDevice,
                             c->stream));
    return LBM_OK;
}

int lbm_dem_checkpoint_load(lbm_ctx* c, const void* src_dev)
{
    if (!c || !src_dev) return fail(c, LBM_EINVAL, "null argument");
    if (c->failed) return fail(c, LBM_ESTATE, "context failed earlier: " + c->last_error);
    const size_t np = (size_t)c->cfg.n_particles;
    if (np == 0) return LBM_OK;
    const char* d = (const char*)src_dev;
    const DemStateBytes b = dem_state_bytes(np);
    HIPCHK(c, hipMemcpyAsync(c->hist_pp, d, b.pp, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->hist_key, d + b.pp, b.key, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->hist_pw, d + b.pp + b.key, b.pw, hipMemcpyDeviceToDevice,
                             c->stream));
    HIPCHK(c, hipMemcpyAsync(c->fc, d + b.pp + b.key + b.pw, b.fc, hipMemcpyDeviceToDevice,
                             c->stream));
    return LBM_OK;
}

// Up to eight device-to-device copies (a null source: zeros) in one launch.
struct CopySeg {
    const uint8_t* src;
    uint8_t* dst;
    uint64_t bytes;
};
struct CopyList {
    CopySeg s[8];
    int n;
};

__global__ __launch_bounds__(256) void k_copy_segments(CopyList L)
{
    const uint64_t t = (uint64_t)blockIdx.x * 256u + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * 256u;
    for (int k = 0; k < L.n; ++k) {
        const CopySeg g = L.s[k];
        const bool v16 = ((reinterpret_cast<uintptr_t>(g.src) | reinterpret_cast<uintptr_t>(g.dst)) &
                          15u) == 0;
        const uint64_t n16 = v16 ? g.bytes / 16 : 0;
        for (uint64_t i = t; i < n16; i += stride)
            reinterpret_cast<uint4*>(g.dst)[i] =
                g.src ? reinterpret_cast<const uint4*>(g.src)[i] : make_uint4(0, 0, 0, 0);
        for (uint64_t i = n16 * 16 + t; i < g.bytes; i += stride) g.dst[i] = g.src ? g.src[i] : 0;
    }
}

static hipError_t copy_segments(lbm_ctx* c, const CopyList& L)
{
    uint64_t most = 0;
    for (int k = 0; k < L.n; ++k) most = std::max<uint64_t>(most, L.s[k].bytes);
    const uint32_t nb = (uint32_t)std::min<uint64_t>(2048, std::max<uint64_t>(1, (most / 16 + 255) / 256));
    hipLaunchKernelGGL(k_copy_segments, dim3(nb), dim3(256), 0, c->stream, L);
    return hipGetLastError();
}

// Layout of a geometry snapshot: owner plane, flags, link records, link
// cursor lines, refill cursor line and list, bounding balls; each part on a
// 256-byte boundary.
struct GeometryLayout {
    size_t own, flag, links, cursors, refill_ctr, refill, ball, total;
};

static size_t align256(size_t n) { return (n + 255) / 256 * 256; }

static GeometryLayout geometry_layout(const lbm_ctx* c)
{
    const size_t np = (size_t)std::max(c->cfg.n_particles, 1);
    GeometryLayout L;
    L.own = 0;
    L.flag = L.own + align256(c->sizes.owner_bytes);
    L.links = L.flag + align256(c->sizes.flag_bytes);
    L.cursors = L.links + align256(sizeof(LinkRec) * (size_t)c->lay->total);
    L.refill_ctr = L.cursors + align256(sizeof(uint32_t) * kCursorPad * np);
    L.refill = L.refill_ctr + 256;
    L.ball = L.refill + align256(sizeof(RefillRec) * (size_t)c->refill_cap);
    L.total = L.ball + align256(sizeof(double) * 4 * np);
    return L;
}

static uint64_t geometry_tag(const lbm_ctx* c)
{
    return c->lay->tag ^ ((uint64_t)c->refill_cap * 0x9E3779B97F4A7C15ull);
}

int lbm_geometry_bytes(const lbm_ctx* c, size_t* bytes, uint64_t* tag)
{
    if (!c || !bytes || !tag) return fail(const_cast<lbm_ctx*>(c), LBM_EINVAL, "null argument");
    *bytes = geometry_layout(c).total;
    *tag = geometry_tag(c);
    return LBM_OK;
}

int lbm_geometry_save(lbm_ctx* c, void* dst_dev)
{
    if (!c || !dst_dev) return fail(c, LBM_EINVAL, "null argument");
    if (c->failed) return fail(c, LBM_ESTATE, "context failed earlier: " + c->last_error);
    if (c->n_classify == 0) return fail(c, LBM_ESTATE, "classify before saving the geometry");
    const int np = c->cfg.n_particles;
    const GeometryLayout L = geometry_layout(c);
    uint8_t* d = (uint8_t*)dst_dev;
    CopyList cl{};
    auto seg = [&](const void* src, size_t off, size_t bytes) {
        cl.s[cl.n++] = CopySeg{(const uint8_t*)src, d + off, bytes};
    };
    seg(c->own[c->own_cur], L.own, c->sizes.owner_bytes);
    seg(c->flag, L.flag, c->sizes.flag_bytes);
    if (np > 0) {
        const int slot = (int)((c->n_classify - 1) % 3);
        seg(c->links, L.links, sizeof(LinkRec) * (size_t)c->lay->total);
        seg(c->link_cursor, L.cursors, sizeof(uint32_t) * kCursorPad * np);
        seg(c->refill_cursor, L.refill_ctr, sizeof(uint32_t));
        seg(c->refill, L.refill, sizeof(RefillRec) * c->refill_cap);
        seg(c->ball_hist + (int64_t)slot * 4 * np, L.ball, sizeof(double) * 4 * np);
    }
    HIPCHK(c, copy_segments(c, cl));
    return LBM_OK;
}

int lbm_geometry_load(lbm_ctx* c, const void* src_dev, uint64_t tag, const lbm_particles* P)
{
    if (!c || !src_dev) return fail(c, LBM_EINVAL, "null argument");
    if (c->failed) return fail(c, LBM_ESTATE, "context failed earlier: " + c->last_error);
    if (tag != geometry_tag(c))
        return fail(c, LBM_ESTATE, "lbm_geometry_load: the link layout or the refill list "
                                   "capacity changed since the snapshot was sized");
    int rc = check_particles(c, P, false);
    if (rc) return rc;
    const int np = c->cfg.n_particles;
    const GeometryLayout L = geometry_layout(c);
    const uint8_t* d = (const uint8_t*)src_dev;
    const ClassifyPlan cp = classify_plan(c);
    CopyList cl{};
    auto seg = [&](void* dst, size_t off, size_t bytes) {
        cl.s[cl.n++] = CopySeg{d + off, (uint8_t*)dst, bytes};
    };
    seg(cp.own_new, L.own, c->sizes.owner_bytes);
    seg(c->flag, L.flag, c->sizes.flag_bytes);
    if (np > 0) {
        seg(c->links, L.links, sizeof(LinkRec) * (size_t)c->lay->total);
        seg(c->link_cursor, L.cursors, sizeof(uint32_t) * kCursorPad * np);
        seg(c->refill_cursor, L.refill_ctr, sizeof(uint32_t));
        seg(c->refill, L.refill, sizeof(RefillRec) * c->refill_cap);
        seg(c->ball_hist + (int64_t)cp.slot * 4 * np, L.ball, sizeof(double) * 4 * np);
        cl.s[cl.n++] = CopySeg{nullptr, (uint8_t*)c->err, sizeof(uint32_t)};  // a valid geometry
    }
    HIPCHK(c, copy_segments(c, cl));
    if (np > 0) {
        if (cp.k >= 1) {
            PhaseTimer tm(c, LBM_PHASE_REFILL);
            HIPCHK(c, LQ(c, launch_refill)(c, cp.refill_src, c->f[c->cur], cp.own_prev, to_dev(P)));
        }
        c->link_max = c->lay->max_seg;  // lbm_step covers every segment whole
    } else {
        c->link_max = c->link_total = c->refill_total = 0;
    }
    c->counts_known = false;
    classify_commit(c, cp);
    c->inc_ok = false;  // the candidate lists and orientations are not the snapshot's
    c->geo_own = reinterpret_cast<const uint32_t*>(d + L.own);
    c->geo_links = np > 0 ? reinterpret_cast<const LinkRec*>(d + L.links) : nullptr;
    return LBM_OK;
}

int lbm_tape_begin(lbm_ctx* c, int max_steps)
{
    if (!c) return fail(nullptr, LBM_EINVAL, "null context");
    if (max_steps < 0) return fail(c, LBM_EINVAL, "max_steps must be >= 0");
    int rc = settle_buffers(c);
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (max_steps == 0) {
        free_tape(c);
        return LBM_OK;
    }
    if (c->n_classify == 0) return fail(c, LBM_ESTATE, "classify before taping");
    const int np = c->cfg.n_particles;
    // entries allocated by an earlier window are reused as they are; the new
    // ones are carved from one allocation (a window's worth of hipMalloc and
    // hipFree calls, each of which synchronises, cost more than the steps)
    const size_t have = c->tape.size();
    if (have < (size_t)max_steps) {
        const size_t np1 = (size_t)std::max(np, 1);
        const size_t part[6] = {c->sizes.population_bytes, c->sizes.owner_bytes,
                                sizeof(uint32_t) * kCursorPad * np1,
                                sizeof(double) * (19 * np1 + 3 * (size_t)c->cfg.n_ctrl),
                                sizeof(double) * std::max<size_t>(dem_tape_doubles(np), 1),
                                sizeof(int32_t) * kPairSlots * np1};
        size_t step = 0;
        for (size_t b : part) step += align256(b);
        const size_t add = (size_t)max_steps - have;
        char* slab = nullptr;
        if (hipMalloc((void**)&slab, step * add) != hipSuccess) {
            free_tape(c);
            return fail(c, LBM_ENOMEM, "tape allocation failed");
        }
        c->tape_slabs.push_back(slab);
        c->tape.resize(max_steps);
        for (size_t k = 0; k < add; ++k) {
            TapeStep& t = c->tape[have + k];
            char* q = slab + k * step;
            t.f = q;
            q += align256(part[0]);
            t.own = reinterpret_cast<uint32_t*>(q);
            q += align256(part[1]);
            t.cursor = reinterpret_cast<uint32_t*>(q);
            q += align256(part[2]);
            t.part = reinterpret_cast<double*>(q);
            q += align256(part[3]);
            t.dem = reinterpret_cast<double*>(q);
            q += align256(part[4]);
            t.dem_key = reinterpret_cast<int32_t*>(q);
        }
    }
    c->tape_len = 0;
    c->tape_steps = max_steps;
    c->taping = true;
    return LBM_OK;
}

namespace {

// The refilled-node list of the adjoint (as long as the refill list of the
// classifications, whose counts bound it) and one count per taped step,
// zeroed.
int adj_lists(lbm_ctx* c)
{
    if (c->adj_list_cap < c->refill_cap) {
        HIPCHK(c, hipFree(c->adj_list));
        c->adj_list = nullptr;
        if (alloc(&c->adj_list, (size_t)c->refill_cap) != hipSuccess)
            return fail(c, LBM_ENOMEM, "adjoint refill list allocation failed");
        c->adj_list_cap = c->refill_cap;
    }
    if (c->adj_count_cap < c->tape_len) {
        HIPCHK(c, hipFree(c->adj_count));
        c->adj_count = nullptr;
        if (alloc(&c->adj_count, (size_t)c->tape_len) != hipSuccess)
            return fail(c, LBM_ENOMEM, "adjoint count allocation failed");
        c->adj_count_cap = c->tape_len;
    }
    HIPCHK(c, hipMemsetAsync(c->adj_count, 0, sizeof(uint32_t) * c->tape_len, c->stream));
    return LBM_OK;
}

AdjList adj_list_of(const lbm_ctx* c, int s)
{
    AdjList l;
    l.node = c->adj_list;
    l.count = c->adj_count + s;
    l.cap = (uint32_t)c->adj_list_cap;
    return l;
}

// After the adjoint's synchronisation: every step's refilled nodes fitted.
int adj_lists_check(lbm_ctx* c)
{
    std::vector<uint32_t> n((size_t)c->tape_len);
    HIPCHK(c, hipMemcpy(n.data(), c->adj_count, sizeof(uint32_t) * n.size(), hipMemcpyDeviceToHost));
    for (uint32_t v : n)
        if (v > c->adj_list_cap)
            return fail(c, LBM_ECAPACITY,
                        "adjoint: more refilled nodes in one step than the refill capacity");
    return LBM_OK;
}

}  // namespace

int lbm_adjoint(lbm_ctx* c, const lbm_particles* P, const double* weights, void* lam_dev,
                double* grad_dev, double* gpos_dev)
{
    if (!c) return fail(nullptr, LBM_EINVAL, "null context");
    if (c->failed) return fail(c, LBM_ESTATE, "context failed earlier: " + c->last_error);
    if (!lam_dev || !grad_dev) return fail(c, LBM_EINVAL, "null argument");
    if (c->tape_len == 0) return fail(c, LBM_ESTATE, "nothing was taped");
    int rc = check_particles(c, P, false);
    if (rc) return rc;
    const int np = c->cfg.n_particles;
    if (np > 0 && !weights) return fail(c, LBM_EINVAL, "null objective weights");
    if (!c->adj_scratch && hipMalloc(&c->adj_scratch, c->sizes.adjoint_bytes) != hipSuccess)
        return fail(c, LBM_ENOMEM, "adjoint scratch allocation failed");
    if (!c->adj_wts && alloc(&c->adj_wts, (size_t)6 * std::max(np, 1)) != hipSuccess)
        return fail(c, LBM_ENOMEM, "adjoint weight allocation failed");
    if (np > 0)
        HIPCHK(c, hipMemcpyAsync(c->adj_wts, weights, sizeof(double) * 6 * np,
                                 hipMemcpyHostToDevice, c->stream));
    rc = adj_lists(c);
    if (rc) return rc;
    void* bufs[2] = {lam_dev, c->adj_scratch};
    int in = 0;
    for (int s = c->tape_len - 1; s >= 0; --s) {
        const TapeStep& ts = c->tape[s];
        const bool last = s + 1 >= c->tape_len;
        const uint32_t* own1 = last ? c->own[c->own_cur] : c->tape[s + 1].own_use;
        const double* pos1 = last ? P->pos : c->tape[s + 1].part;
        const double* vel1 = last ? P->vel : c->tape[s + 1].part + 3 * np;
        const double* om1 = last ? P->omega : c->tape[s + 1].part + 6 * np;
        AdjOut out;
        if (gpos_dev && np > 0) {
            out.g_links = gpos_dev + (size_t)6 * np * s;
            out.g_refill = out.g_links + 6 * np;
        }
        PhaseTimer tm(c, LBM_PHASE_ADJOINT);
        HIPCHK(c, LQ(c, launch_adjoint_step)(c, ts, own1, pos1, vel1, om1, bufs[in], bufs[1 - in],
                                             c->adj_wts, grad_dev, P, out, adj_list_of(c, s),
                                             kAdjNode | kAdjRefill | kAdjLinks));
        in = 1 - in;
    }
    if (in != 0)
        HIPCHK(c, hipMemcpyAsync(lam_dev, bufs[in], c->sizes.adjoint_bytes, hipMemcpyDeviceToDevice,
                                 c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    rc = c->deferred ? check_deferred(c, "lbm_adjoint") : LBM_OK;
    if (!rc) rc = adj_lists_check(c);
    c->tape_len = 0;
    c->taping = false;
    const int rc2 = settle_buffers(c);
    return rc ? rc : rc2;
}

int lbm_adjoint_coupled(lbm_ctx* c, const lbm_particles* P, const double* weights,
                        const dem_params* prm, int n_sub, double dt, void* lam_dev,
                        double* grad_dev, double* sigma_dev, double* sigma_contact_dev)
{
    if (!c) return fail(nullptr, LBM_EINVAL, "null context");
    if (c->failed) return fail(c, LBM_ESTATE, "context failed earlier: " + c->last_error);
    if (!lam_dev || !grad_dev || !prm) return fail(c, LBM_EINVAL, "null argument");
    if (n_sub < 1 || !(dt > 0.0)) return fail(c, LBM_EINVAL, "n_sub must be >= 1 and dt > 0");
    if (c->tape_len == 0) return fail(c, LBM_ESTATE, "nothing was taped");
    int rc = check_particles(c, P, true);
    if (rc) return rc;
    const int np = c->cfg.n_particles;
    if (np > 0 && (!weights || !sigma_dev)) return fail(c, LBM_EINVAL, "null objective weights or state adjoint");
    if (!c->adj_scratch && hipMalloc(&c->adj_scratch, c->sizes.adjoint_bytes) != hipSuccess)
        return fail(c, LBM_ENOMEM, "adjoint scratch allocation failed");
    const size_t nps = (size_t)std::max(np, 1);
    if (!c->adj_wts && alloc(&c->adj_wts, 6 * nps) != hipSuccess)
        return fail(c, LBM_ENOMEM, "adjoint weight allocation failed");
    // state adjoints [2][np][12], objective weights [np][6], contact-state
    // adjoints [2][np][kAdjContact]
    if (!c->adj_sig && alloc(&c->adj_sig, 2 * 12 * nps + 6 * nps + 2 * kAdjContact * nps) != hipSuccess)
        return fail(c, LBM_ENOMEM, "state adjoint allocation failed");
    double* sig[2] = {c->adj_sig, c->adj_sig + 12 * nps};
    double* wJ = c->adj_sig + 24 * nps;
    double* sct[2] = {c->adj_sig + 30 * nps, c->adj_sig + 30 * nps + kAdjContact * nps};
    uint32_t* err = c->ctr + kCtrAdjCluster;
    HIPCHK(c, hipMemsetAsync(err, 0, sizeof(uint32_t), c->stream));
    if (np > 0) {
        HIPCHK(c, hipMemcpyAsync(wJ, weights, sizeof(double) * 6 * np, hipMemcpyHostToDevice,
                                 c->stream));
        HIPCHK(c, hipMemcpyAsync(sig[0], sigma_dev, sizeof(double) * 12 * np,
                                 hipMemcpyDeviceToDevice, c->stream));
        if (sigma_contact_dev)
            HIPCHK(c, hipMemcpyAsync(sct[0], sigma_contact_dev, sizeof(double) * kAdjContact * np,
                                     hipMemcpyDeviceToDevice, c->stream));
        else
            HIPCHK(c, hipMemsetAsync(sct[0], 0, sizeof(double) * kAdjContact * np, c->stream));
    }
    rc = adj_lists(c);
    if (rc) return rc;
    void* bufs[2] = {lam_dev, c->adj_scratch};
    int in = 0, si = 0;
    for (int s = c->tape_len - 1; s >= 0; --s) {
        const TapeStep& ts = c->tape[s];
        const bool last = s + 1 >= c->tape_len;
        const uint32_t* own1 = last ? c->own[c->own_cur] : c->tape[s + 1].own_use;
        const double* pos1 = last ? P->pos : c->tape[s + 1].part;
        const double* vel1 = last ? P->vel : c->tape[s + 1].part + 3 * np;
        const double* om1 = last ? P->omega : c->tape[s + 1].part + 6 * np;
        const int32_t* key1 = last ? c->hist_key : c->tape[s + 1].dem_key;
        double* s1 = sig[si];      // adjoint of the state after this step's dem_step
        double* s0 = sig[1 - si];  // adjoint of the state this step used
        PhaseTimer tm(c, LBM_PHASE_ADJOINT);
        // 1. nodes, and the nodes refilled by the classification of the next
        //    state: their wall velocities belong to s1
        AdjOut ro;
        ro.g_refill = s1;
        ro.v_refill = s1 + 6;
        ro.w_refill = s1 + 9;
        ro.gstride = ro.vstride = 12;
        HIPCHK(c, LQ(c, launch_adjoint_step)(c, ts, own1, pos1, vel1, om1, bufs[in], bufs[1 - in],
                                             c->adj_wts, grad_dev, P, ro, adj_list_of(c, s),
                                             kAdjNode | kAdjRefill));
        // 2. the DEM call: (s1, contact state after it) -> (s0, contact state
        //    before it), and this step's force weights
        HIPCHK(c, launch_dem_adjoint(c, ts, key1, P, *prm, n_sub, dt, s1, sct[si], s0, sct[1 - si],
                                     wJ, c->adj_wts, err));
        // 3. links of this step under those weights, into s0
        AdjOut lo;
        lo.g_links = s0;
        lo.v_links = s0 + 6;
        lo.w_links = s0 + 9;
        lo.gstride = lo.vstride = 12;
        HIPCHK(c, LQ(c, launch_adjoint_step)(c, ts, own1, pos1, vel1, om1, bufs[in], bufs[1 - in],
                                             c->adj_wts, grad_dev, P, lo, adj_list_of(c, s),
                                             kAdjLinks));
        in = 1 - in;
        si = 1 - si;
    }
    if (in != 0)
        HIPCHK(c, hipMemcpyAsync(lam_dev, bufs[in], c->sizes.adjoint_bytes, hipMemcpyDeviceToDevice,
                                 c->stream));
    if (np > 0) {
        HIPCHK(c, hipMemcpyAsync(sigma_dev, sig[si], sizeof(double) * 12 * np,
                                 hipMemcpyDeviceToDevice, c->stream));
        if (sigma_contact_dev)
            HIPCHK(c, hipMemcpyAsync(sigma_contact_dev, sct[si], sizeof(double) * kAdjContact * np,
                                     hipMemcpyDeviceToDevice, c->stream));
    }
    HIPCHK(c, hipMemcpyAsync(c->host_stage + kCtrAdjCluster, err, sizeof(uint32_t),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    rc = c->deferred ? check_deferred(c, "lbm_adjoint") : LBM_OK;
    if (!rc) rc = adj_lists_check(c);
    if (!rc && c->host_stage[kCtrAdjCluster])
        rc = fail(c, LBM_ESTATE,
                  "lbm_adjoint_coupled: a contact cluster (particles linked through candidate "
                  "pairs of one dem_step call) has more than " + std::to_string(kAdjCluster) +
                      " particles; the results are not valid");
    c->tape_len = 0;
    c->taping = false;
    const int rc2 = settle_buffers(c);
    return rc ? rc : rc2;
}

static int profile_collect(lbm_ctx* c)
{
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (auto& t : c->timed) {
        float ms = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&ms, t.start, t.stop));
        if (t.phase >= 0 && t.phase < LBM_PHASE_COUNT) {
            c->prof_ms[t.phase] += ms;
            c->prof_n[t.phase] += 1;
        }
        c->event_pool.push_back(t.start);
        c->event_pool.push_back(t.stop);
    }
    c->timed.clear();
    return LBM_OK;
}

int lbm_profile_enable(lbm_ctx* c, int on)
{
    if (!c) return fail(nullptr, LBM_EINVAL, "null context");
    int rc = profile_collect(c);
    if (rc) return rc;
    if (on) {
        for (int i = 0; i < LBM_PHASE_COUNT; ++i) {
            c->prof_ms[i] = 0.0;
            c->prof_n[i] = 0;
        }
    }
    c->prof = on != 0;
    return LBM_OK;
}

int lbm_profile_read(lbm_ctx* c, lbm_profile* out)
{
    if (!c || !out) return fail(c, LBM_EINVAL, "null argument");
    int rc = profile_collect(c);
    if (rc) return rc;
    for (int i = 0; i < LBM_PHASE_COUNT; ++i) {
        out->ms[i] = c->prof_ms[i];
        out->launches[i] = c->prof_n[i];
    }
    return LBM_OK;
}

}  // extern "C"

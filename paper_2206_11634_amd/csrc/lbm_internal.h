// Internal declarations shared by the translation units of libmdlbm (HIP,
// gfx950).  Nothing here crosses the C-ABI.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "mdlbm.h"

namespace mdlbm {

// Owner plane value of a fluid node (a solid node holds its particle index).
// Largest per-particle box half-width h (the classification kernels keep a
// table of the 2h + 1 rows of one box plane in LDS).
constexpr int kMaxBoxHalf = 511;
constexpr uint32_t kFluid = 0xFFFFFFFFu;
// Counters of one classification, in one device block mirrored by one pinned
// host block so that a single copy reads them all: the refill count, the box
// check, the non-finite force flag (one 128-byte line), then one line per
// particle for its link count and one per particle for its candidate count.
constexpr int kCtrRefill = 0;
constexpr int kCtrErr = 1;
constexpr int kCtrNumeric = 2;
// Latched by asynchronous classifications: the box check's bits (low byte)
// and kDeferredOverflow when a list outgrew its capacity.
constexpr int kCtrDeferred = 3;
constexpr uint32_t kDeferredOverflow = 0x100u;
// Set by the DEM adjoint when a particle's contact cluster (the particles
// linked to it through broad-phase candidate pairs of one dem_step call)
// has more than kAdjCluster members.
constexpr int kCtrAdjCluster = 4;
// Set by the boxes' kernel when a particle moved too far since the previous
// classification for the candidate-list flag and refill pass (every node
// that leaves a body was on its previous candidate list); the lattice sweep
// then writes flags and refills instead.
constexpr int kCtrIncremental = 5;
// Latched by dem_step when a particle had more candidate contact partners
// than its history slots (reported like the asynchronous classifications).
constexpr uint32_t kDeferredSlots = 0x200u;
// Pair contact histories: each particle i keeps kPairSlots records for its
// partners j > i, keyed by j; a record lives while the pair stays a
// broad-phase candidate.
constexpr int kPairSlots = 32;
// The DEM adjoint: most particles of one contact cluster, and the doubles of
// one particle's contact-state adjoint (carried contact force and torque, the
// springs of its kPairSlots pair records and of its six wall records).
constexpr int kAdjCluster = 8;
constexpr int kAdjContact = 6 + 3 * kPairSlots + 3 * 6;
constexpr int kStageHead = 32;  // = kCursorPad: the counts start on the second line

// ---------------------------------------------------------------------------
// Records
// ---------------------------------------------------------------------------
struct alignas(16) LinkRec {
    uint32_t node;   // solid node x_s
    uint16_t part;   // particle index
    uint8_t d;       // direction from x_n = x_s - e_d into the solid
    uint8_t kind;    // lbm_link_kind
    double q;        // wall fraction of Eq. (appq)
};
static_assert(sizeof(LinkRec) == 16, "link record is 16 bytes");

struct RefillRec {
    uint32_t node;
    uint32_t part;
};

// Where each particle's link records lie: particle p's segment is
// [off[p], off[p+1]), a multiple of 256 records sized from its own link
// count, and chunk_dev[b] is the particle of the 256-record chunk b, so the
// link kernels run one workgroup per chunk.  A layout is never changed once
// made (growing the lists makes a new one); the context and every taped step
// recorded with it hold a reference.
struct LinkLayout {
    std::vector<int64_t> off;        // host copy, np + 1 entries
    int64_t total = 0;               // records: off[np]
    int64_t max_seg = 0;             // the largest segment
    int64_t* off_dev = nullptr;      // [np + 1]
    uint32_t* chunk_dev = nullptr;   // [total / 256]
    uint64_t tag = 0;                // hash of off
    int64_t chunks() const { return total / 256; }
    ~LinkLayout()
    {
        (void)hipFree(off_dev);
        (void)hipFree(chunk_dev);
    }
};

// One recorded lattice step for the adjoint: populations after the link
// reconstruction (ghost slots filled), owners, links and particle state.
// Its fixed-size parts (f, own, cursor, part, dem, dem_key) are carved from
// the context's tape slabs; links are allocated per step.
struct TapeStep {
    void* f = nullptr;
    uint32_t* own = nullptr;
    LinkRec* links = nullptr;
    std::shared_ptr<const LinkLayout> lay;  // the layout of this record's links
    int64_t link_alloc = 0;      // records allocated
    uint32_t* cursor = nullptr;  // [np * kCursorPad]
    int64_t link_max = 0;
    double* part = nullptr;      // [19 np + 3 n_ctrl]: pos, vel, omega, world control
                                 // points, quaternion (4 np), F^h and T^h (6 np)
    double* dem = nullptr;       // DEM state before the dem_step call that followed the
                                 // step: pair records [np][kPairSlots][8], wall records
                                 // [np][6][8], contact sums [np][6]
    int32_t* dem_key = nullptr;  // [np][kPairSlots] keys of the pair records
    // the owners and links the adjoint reads: own and links, or those of the
    // geometry snapshot the step's classification was loaded from
    const uint32_t* own_use = nullptr;
    const LinkRec* links_use = nullptr;
};

// Lattice geometry passed by value to kernels.
struct Geom {
    int n[3];
    int per[3];
    int64_t stride;   // elements between population planes
    uint32_t ncell;
};

// Physical constants for one launch.
struct Phys {
    double tau, omega;     // omega = 1/tau
    double F[3];           // body-force density
    double rho0;
    float omegaf;
    float Ff[3];
    float scale, inv_scale;  // FP16 deviation scale
    int neq_split;           // VIBB: fneq(x_d) = fneq(x_f) for q > 1/2 (treatment bit 8)
};

// Device pointers of the particle state (a copy of lbm_particles).
struct PartDev {
    int n;
    const int32_t* off;
    const double* body_pts;
    const double* K;
    const double* c0;
    const double* rs;
    const double* mass;
    const double* volume;
    const double* inertia;
    double* pos;
    double* quat;
    double* vel;
    double* omega;
    double* wpts;
};

// Per-particle node box: origin (unwrapped) and edge S = 2h + 1.
struct BoxSpec {
    int h, S, vol, tiles;  // tiles of 256 box cells
};

constexpr int kCursorPad = 32;  // one 128-byte line per per-particle counter
static_assert(kStageHead == kCursorPad, "counter block: one head line, then the cursors");

}  // namespace mdlbm

// The context (opaque across the ABI).
struct lbm_ctx {
    lbm_config cfg{};
    hipStream_t stream = nullptr;
    // lbm_step_dem: the stream-collide pass and the DEM sub-cycle on two
    // streams with disjoint compute-unit masks (made on first use)
    hipStream_t s_bulk = nullptr, s_dem = nullptr;
    hipEvent_t ev_fork = nullptr, ev_bulk = nullptr, ev_dem = nullptr;
    int device = 0;         // the HIP device current at lbm_init
    mdlbm::Geom geom{};
    mdlbm::Phys phys{};
    mdlbm::BoxSpec box{};
    void* f[2] = {nullptr, nullptr};   // current (f[cur]) and previous populations: the
                                       // caller's buffers, or tape slots while taping
    void* fu[2] = {nullptr, nullptr};  // the caller's two population buffers
    uint32_t* own[2] = {nullptr, nullptr};
    uint8_t* flag = nullptr;
    void* mom = nullptr;    // per-node (rho - 1, u) of the current populations
    int cur = 0;            // population buffer holding the current f+
    int own_cur = 0;        // owner plane of the last classification
    int64_t n_classify = 0; // classifications done
    bool counts_known = true;   // the last classification's list counts were read back
    bool deferred = false;      // an asynchronous classification awaits its check
    bool stepped_since_classify = false;
    // the current geometry was loaded from this snapshot's owners and links
    const uint32_t* geo_own = nullptr;
    const mdlbm::LinkRec* geo_links = nullptr;
    bool dense = false;     // particle balls cover most of the lattice: sweep it whole
    bool failed = false;

    // library scratch
    double* ball_hist = nullptr;  // [3][np][4] centre and bounding radius of each particle
                                  // at the last three classifications
    uint32_t* cand = nullptr;     // per particle: nodes that may carry links
    int64_t cand_cap = 0;         // per particle
    uint32_t* cand_cursor = nullptr;  // [np * kCursorPad]
    // dense mode: the previous classification's candidate lists and counts,
    // and the orientations it saw, for the flag and refill pass over them
    uint32_t* cand_prev = nullptr;
    int64_t cand_prev_cap = 0;
    uint32_t* cand_prev_count = nullptr;  // [np]
    double* quat_prev = nullptr;          // [np][4]
    bool inc_ok = false;                  // the previous classification's lists are valid
    mdlbm::LinkRec* links = nullptr;
    std::shared_ptr<const mdlbm::LinkLayout> lay;  // where each particle's links lie
    bool lay_initial = true;      // the layout sized before any count was known
    uint32_t* link_cursor = nullptr;  // [np * kCursorPad]
    int64_t link_max = 0;         // max links of one particle at the last classification
    int64_t link_total = 0;
    int64_t cand_total = 0;
    mdlbm::RefillRec* refill = nullptr;
    int64_t refill_cap = 0;
    uint32_t* refill_cursor = nullptr;
    int64_t refill_total = 0;
    uint32_t* err = nullptr;      // error bits written by kernels
    uint32_t* ctr = nullptr;      // the counter block: refill_cursor, err, numeric,
                                  // link_cursor and cand_cursor point into it
    double* FT = nullptr;         // [np][6] force, torque of the last step
    unsigned long long* FX = nullptr;  // [np][6][lo, hi]: exact sums (LBM_FORCE_SUM_EXACT)
    uint32_t* host_stage = nullptr; // pinned staging for counters
    // DEM
    double* hist_pp = nullptr;    // [np][kPairSlots][8] pair histories
    int32_t* hist_key = nullptr;  // [np][kPairSlots] partner + 1 of each record, 0 free
    double* hist_pw = nullptr;    // [np*6][8]
    double* fc = nullptr;         // [np][6] last contact force / torque
    double* reach = nullptr;      // [np] broad-phase radius of each particle
    uint32_t* numeric = nullptr;  // set by a step whose force or torque sums are not finite
    uint64_t* pairs = nullptr;    // [np kPairSlots] candidate pairs of a dem_step call
    uint32_t* pair_count = nullptr;
    uint32_t* grid = nullptr;     // the broad phase's cell grid (kGridMinParticles or more)
    double* grid_size = nullptr;
    int64_t grid_cap = 0;
    // kernel timing
    bool prof = false;
    struct Timed {
        int phase;
        hipEvent_t start, stop;
    };
    std::vector<Timed> timed;
    std::vector<hipEvent_t> event_pool;
    double prof_ms[LBM_PHASE_COUNT] = {};
    int64_t prof_n[LBM_PHASE_COUNT] = {};
    // differentiation form
    lbm_sizes sizes{};
    std::vector<mdlbm::TapeStep> tape;
    std::vector<void*> tape_slabs;  // one allocation per growth of the tape
    int tape_len = 0;    // steps recorded since lbm_tape_begin
    int tape_steps = 0;  // steps to record (tape.size() may be larger)
    bool taping = false;
    void* adj_scratch = nullptr;  // the second adjoint field of the ping-pong
    double* adj_wts = nullptr;
    double* adj_sig = nullptr;    // free-motion state adjoints [2][np][12] + weights [np][6]
    uint32_t* adj_list = nullptr;  // refilled nodes of the adjoint step being taken
    int64_t adj_list_cap = 0;
    uint32_t* adj_count = nullptr; // [tape steps] their number, per step
    int64_t adj_count_cap = 0;
    std::string last_error;
};

namespace mdlbm {

// Where an adjoint step puts its per-particle derivatives (all optional):
// pose gradients (x, theta) of the links' pose and dJ/dx of the refill's
// pose, with stride gstride; dJ/dv and dJ/domega seen by the links and by the
// refill, with stride vstride (dJ/dv defaults to grad + 4 + 3 p).
struct AdjOut {
    double* g_links = nullptr;
    double* g_refill = nullptr;
    int gstride = 6;
    double* v_links = nullptr;
    double* v_refill = nullptr;
    double* w_links = nullptr;
    double* w_refill = nullptr;
    int vstride = 3;
};
// Parts of one adjoint step, run in the order node, refill, links: the node
// kernel lists the nodes refilled between n and n + 1 for the refill kernel,
// and leaves the ghost-slot adjoints the link kernel takes.
constexpr int kAdjRefill = 1, kAdjLinks = 2, kAdjNode = 4;
// The list of refilled nodes of one adjoint step, and its length.
struct AdjList {
    uint32_t* node = nullptr;
    uint32_t* count = nullptr;
    uint32_t cap = 0;
};

// Launchers of the lattice kernels, one set per lattice (D3Q19, D3Q15).
namespace q19 {
#include "lbm_launchers.inc"
}
namespace q15 {
#include "lbm_launchers.inc"
}

// Launchers (lbm_dem.hip, lbm_dem_adjoint.hip)
// Work space of one dem_step call: the candidate pairs (i, j, history slot),
// their count, and each particle's broad-phase reach.
// The work space of one dem_step call.  With the cell grid (gcount not
// null), the broad phase bins the particles into cells at least as wide as
// the largest pair distance it can accept and tests each particle against
// the 27 cells around its own, instead of all n^2 pairs.
struct DemScratch {
    uint64_t* pairs;
    uint32_t* count;
    double* reach;
    uint32_t* gcount = nullptr;   // [gcap + 1]: counts per cell, then their starts
    uint32_t* gcursor = nullptr;  // [gcap]
    uint32_t* gitem = nullptr;    // [n]: particles by cell
    int32_t* gdim = nullptr;      // cells per axis, and their product
    double* gsize = nullptr;      // cell widths, then H (the largest accepted distance)
    int64_t gcap = 0;             // cells the arrays hold
};
// Particle counts from which dem_step uses the cell grid.
constexpr int kGridMinParticles = 2048;
hipError_t launch_dem(lbm_ctx* c, const PartDev& P, int n_sub, double dt, const dem_params& prm,
                      const DemScratch& s);
// Most particles dem_step_noalloc takes (its static work space holds the
// pair list of that many).
constexpr int kNoAllocParticles = 1024;
// Device address of the allocation-free DEM work space on the current
// device (looked up once per device); hipSuccess or the lookup's error.
hipError_t dem_noalloc_setup();
// The work space of device dev, after dem_noalloc_setup ran on it.
bool dem_noalloc_scratch(int dev, DemScratch* out);
// The transposed Jacobian of the dem_step call that followed taped step ts
// (key_next: the pair records' keys after it), applied to the adjoint of
// its output state (sig1 [np][12], sc1 [np][kAdjContact]), into the adjoint
// of its input state (sig0, sc0) and the step's force weights wts = wJ +
// dJ/d(F^h, T^h); err latches a contact cluster beyond kAdjCluster.
hipError_t launch_dem_adjoint(lbm_ctx* c, const TapeStep& ts, const int32_t* key_next,
                              const lbm_particles* P, const dem_params& prm, int n_sub, double dt,
                              const double* sig1, const double* sc1, double* sig0, double* sc0,
                              const double* wJ, double* wts, uint32_t* err);

}  // namespace mdlbm

/*
 * mdlbm.h -- C-ABI of the MI355X (gfx950) library for the per-timestep
 * lattice update of the coupled metaball-DEM / lattice Boltzmann method with a
 * sharp interface (Zhang et al., arXiv 2206.11634).
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 *  * Lattice units: dx = dt = 1, c_s^2 = 1/3, nu = (tau - 1/2)/3 (Sec. 2.2).
 *  * Lattice D3Q19 (default), directions numbered
 *      0:(0,0,0) 1:(+1,0,0) 2:(-1,0,0) 3:(0,+1,0) 4:(0,-1,0) 5:(0,0,+1)
 *      6:(0,0,-1) 7:(+1,+1,0) 8:(-1,-1,0) 9:(+1,-1,0) 10:(-1,+1,0)
 *      11:(+1,0,+1) 12:(-1,0,-1) 13:(+1,0,-1) 14:(-1,0,+1) 15:(0,+1,+1)
 *      16:(0,-1,-1) 17:(0,+1,-1) 18:(0,-1,+1);  opposite of odd i is i + 1.
 *    Or D3Q15, the paper's (lbm_config.lattice), numbered in lbm_lattice;
 *    Q below is the number of directions of the configured lattice.
 *  * Node (i,j,k) sits at coordinates (i,j,k); cell index i + nx*(j + ny*k).
 *    A non-periodic axis ends in no-slip walls half a cell outside the first
 *    and last node (static halfway bounce-back).
 *  * Population planes are structure-of-arrays: plane i of a buffer starts at
 *    element i * cell_stride (lbm_sizes.cell_stride), x fastest.
 *  * Every pointer named *_dev is device memory owned by the caller, unless
 *    the entry point says otherwise.  The caller keeps it alive for as long as
 *    the context may use it.  The library owns only its context and the small
 *    scratch it allocates in lbm_init and frees in lbm_destroy (link and refill
 *    lists, per-particle sums, contact histories).
 *  * Work is enqueued on the stream given in lbm_config.stream and is
 *    asynchronous unless an entry point says it synchronises.
 *  * Every call returns an lbm_status.  Nothing is thrown across the ABI;
 *    lbm_last_error() returns a message for the last failure.
 *  * Particles are described by device arrays in FP64 (lbm_particles).  A
 *    particle's body is {x : M(x) >= c0} with M the metaball function of
 *    Eq. (metaball), M(x) = sum_i K_i / |x - x_i|^2 over its control points.
 */
#ifndef MDLBM_H
#define MDLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = 1,    /* an argument is out of range or inconsistent */
    LBM_ENOMEM = 2,    /* the library could not allocate its scratch */
    LBM_ECAPACITY = 3, /* a caller-provided output is too small */
    LBM_ENUMERIC = 4,  /* non-finite values detected */
    LBM_EDEVICE = 5,   /* a HIP runtime call or kernel launch failed */
    LBM_ESTATE = 6     /* call out of order, or context in a failed state */
} lbm_status;

typedef enum {
    LBM_STORE_F64 = 0, /* f_i in double; collision in double (plain method) */
    LBM_STORE_F32 = 1, /* deviations f_i - w_i in float; float arithmetic */
    LBM_STORE_F16 = 2  /* deviations (f_i - w_i) * h16_scale in half; float arithmetic */
} lbm_storage;

typedef enum {
    LBM_TREAT_VIBB = 1,   /* velocity-interpolated bounce-back (Sec. 2.3.1); without
                             it every cut link uses halfway bounce-back */
    LBM_TREAT_MISSING = 2, /* treatment 2 of Sec. 2.3.5: momentum exchange on
                             force points covered by another body or a wall */
    LBM_TREAT_EXACT_Q = 4, /* q as the root of Eq. (calq), M(x_n + q e_d) = c0, by a
                             bracketed Newton iteration from the linear estimate,
                             instead of Eq. (appq) */
    LBM_TREAT_NEQ_SPLIT = 8 /* for q > 1/2 the non-equilibrium part at x_d is taken
                             from x_f alone, the case split Eq. (rhod) makes for the
                             density, instead of extrapolating Eq. (neqd) with weights
                             2q > 1 and 1 - 2q < 0; off: Eq. (neqd) for every q */
} lbm_treatment;

/* How the link pass sums the momentum-exchange terms of Eq. (mem) over each
 * particle's links (Sec. 2.3.2); the per-link terms are the same FP64 values
 * either way. */
typedef enum {
    LBM_FORCE_SUM_ATOMIC = 0, /* FP64 sums per wave and workgroup, then FP64 atomics
                                 per particle: the order of the atomic additions,
                                 and so the last bits of F and T, can change from
                                 run to run (about 1e-16 relative) */
    LBM_FORCE_SUM_EXACT = 1   /* every term rounded toward zero to a multiple
                                 of 2^-80 and summed exactly in 128-bit
                                 integers (two 64-bit atomics per workgroup and
                                 component), then rounded to double: the same bits
                                 on every run whatever the order of the links
                                 (which classification appends with atomics).
                                 Terms must lie below 2^46 in magnitude and sums
                                 below 2^47; a term outside, or not finite, counts
                                 as zero and latches LBM_ENUMERIC like a non-finite
                                 sum.  For debugging and reproducibility checks;
                                 12 * n_particles more 8-byte words of device memory */
} lbm_force_sum;

typedef enum {
    LBM_LINK_VIBB = 0,    /* x_f and x_ff fluid: VIBB reconstruction */
    LBM_LINK_HALFWAY = 1, /* x_f fluid, x_ff not: halfway bounce-back (treatment 1) */
    LBM_LINK_MISSING = 2  /* x_n covered: force-only missing point (treatment 2) */
} lbm_link_kind;

typedef struct {
    int32_t nx, ny, nz;
    int32_t periodic[3];   /* non-zero: periodic axis; zero: walls */
    double tau;            /* BGK relaxation time, > 1/2 */
    double rho0;           /* reference density (refill and treatment 2) */
    double u0[3];          /* initial uniform velocity */
    double body_force[3];  /* fluid body-force density (Guo forcing); 0 in the paper */
    int32_t storage;       /* lbm_storage */
    int32_t treatments;    /* bitmask of lbm_treatment */
    int32_t n_particles;   /* number of particles (0 allowed) */
    int32_t n_ctrl;        /* total control points over all particles */
    int32_t box_half;      /* h: each particle's nodes lie within distance h-1 of its
                              centre; bounds the per-particle node box */
    double h16_scale;      /* scale of FP16 deviations (0: default 1024) */
    void* stream;          /* hipStream_t, NULL for the null stream */
    int32_t classify_mode; /* lbm_classify_mode; the same owners, links and refill
                              sets either way, only the work differs */
    int32_t lattice;       /* lbm_lattice; 0 selects D3Q19 */
    int32_t force_sum;     /* lbm_force_sum; 0: FP64 atomics */
} lbm_config;

typedef enum {
    LBM_LATTICE_D3Q19 = 19, /* rest, 6 axes, 12 face diagonals; w = 1/3, 1/18, 1/36 */
    LBM_LATTICE_D3Q15 = 15  /* the paper's lattice (Sec. 2.2): rest, 6 axes, 8 cube
                               diagonals; w = 2/9, 1/9, 1/72.  Directions 7..14 are
                               (1,1,1), (-1,-1,-1), (1,1,-1), (-1,-1,1), (1,-1,1),
                               (-1,1,-1), (-1,1,1), (1,-1,-1) */
} lbm_lattice;

typedef enum {
    LBM_CLASSIFY_AUTO = 0,  /* lattice sweep when the particles' bounding balls
                               cover more than half of the lattice */
    LBM_CLASSIFY_SWEEP = 1, /* owners cleared, flags and refill set found by one
                               sweep over every node */
    LBM_CLASSIFY_BALLS = 2  /* all work inside each particle's bounding ball */
} lbm_classify_mode;

typedef struct {
    int64_t ncell;             /* nx*ny*nz */
    int64_t cell_stride;       /* elements between population planes (>= ncell) */
    size_t population_bytes;   /* bytes of ONE population buffer (two are needed) */
    size_t owner_bytes;        /* bytes of ONE owner plane (two are needed), uint32 */
    size_t flag_bytes;         /* bytes of the fluid/solid flag plane, uint8 */
    size_t moment_bytes;       /* bytes of the moment plane: per node (rho - 1, u) in
                                  the storage's arithmetic (double, float, or half
                                  scaled like the FP16 deviations) */
    size_t checkpoint_bytes;   /* bytes of one raw checkpoint (populations + moments) */
    size_t adjoint_bytes;      /* bytes of one adjoint field: Q planes of cell_stride
                                  values in the storage's arithmetic (double or float) */
    size_t dem_checkpoint_bytes; /* bytes of the DEM's own state: contact histories
                                    and the last contact forces */
    size_t contact_adjoint_bytes; /* bytes of the adjoint of that state for
                                     lbm_adjoint_coupled: per particle 120 doubles, the
                                     carried contact force and torque (6), the springs
                                     of its 32 pair records (96) and of its six wall
                                     records (18) */
} lbm_sizes;

typedef struct {
    void* f_dev[2];            /* two population buffers, population_bytes each */
    uint32_t* owner_dev[2];    /* two owner planes, owner_bytes each */
    uint8_t* flag_dev;         /* flag plane, flag_bytes */
    void* moments_dev;         /* moment plane, moment_bytes: written by every collision,
                                  read by the link reconstruction */
} lbm_buffers;

/* Particle state, all device arrays in FP64 unless noted.  n_ctrl = ctrl_off[n]. */
typedef struct {
    int32_t n;
    const int32_t* ctrl_off;  /* int32[n+1]: control points of particle p are
                                 ctrl_off[p] .. ctrl_off[p+1]-1 */
    const double* body_pts;   /* [n_ctrl][3] control points in the principal body
                                 frame, origin at the centroid */
    const double* K;          /* [n_ctrl] metaball weights, > 0 */
    const double* c0;         /* [n] surface level of the fluid-side body */
    const double* rs;         /* [n] sphero radius R_s of the DEM contact surface */
    const double* mass;       /* [n] */
    const double* volume;     /* [n] (relative gravity (m - rho_f V) g) */
    const double* inertia;    /* [n][3] principal moments */
    double* pos;              /* [n][3] centroid x_p; in [0, n) on periodic axes */
    double* quat;             /* [n][4] (w,x,y,z) body -> world */
    double* vel;              /* [n][3] */
    double* omega;            /* [n][3] world-frame angular velocity */
    double* world_pts;        /* [n_ctrl][3] world control points x_i; read by
                                 lbm_classify_nodes, refreshed by dem_step */
} lbm_particles;

typedef struct {
    int64_t n_links;    /* VIBB + HALFWAY + MISSING links of the classification */
    int64_t n_refill;   /* nodes solid at the previous and fluid at this classification */
    int64_t n_candidates; /* solid nodes examined for links (not provably interior) */
} lbm_counts;

typedef struct {
    double kn, eta_n;        /* normal spring stiffness and damping (Sec. 2.1.1) */
    double kt, eta_t, mu_s;  /* tangential spring, damping, friction coefficient */
    double ctol;             /* lower bound on M at the contact search point (Eq. opt) */
    double newton_tol;       /* Newton step tolerance (lattice units) */
    int32_t newton_iter;     /* Newton iteration limit */
    double gravity[3];       /* g; particles feel (m - rho_f V) g (Sec. 3.1) */
    double rho_f;            /* fluid density for the relative gravity */
} dem_params;

typedef struct lbm_ctx lbm_ctx;

/* Sizes of the caller-owned buffers for cfg.  Host only; no device work.
 * EINVAL when a dimension is < 1. */
int lbm_query_sizes(const lbm_config* cfg, lbm_sizes* out);

/* Create a context for cfg on the current HIP device and initialise the
 * populations of bufs->f_dev[0] to the equilibrium f_eq(rho0, u0) (Sec. 2.2),
 * the owner planes to "fluid" and the flags to fluid.  Allocates the library's
 * scratch (ENOMEM on failure).  EINVAL on tau <= 1/2, a dimension < 1, a null
 * buffer, an unknown storage or classify_mode, box_half outside [2, 511], a periodic axis shorter than
 * 2*box_half + 5 nodes, or n_particles >= 65535.  Synchronises the stream. */
int lbm_init(const lbm_config* cfg, const lbm_buffers* bufs, lbm_ctx** out);

/* Release the context and the library's scratch (never the caller's buffers). */
int lbm_destroy(lbm_ctx* ctx);

/* Message of the last failure on ctx (or of the last lbm_init when ctx is
 * NULL).  The string lives until the next call on the same context. */
const char* lbm_last_error(const lbm_ctx* ctx);

/* Node classification, link sets and local refilling (Secs. 2.3.1, 2.3.3,
 * 2.3.5) for the particle state P, in FP64:
 *  * owner(x) = lowest p with M_p(x) >= c0_p, else fluid;
 *  * a link (x_s, d, p) for every node x_s of p and direction d whose
 *    neighbour x_n = x_s - e_d is fluid (VIBB when x_ff = x_n - e_d is fluid
 *    too and VIBB is on, else HALFWAY), or is covered by another particle or
 *    lies beyond a wall with M_p(x_n) < c0_p (MISSING, when treatment 2 is on);
 *    q = (c0 - M(x_n)) / (M(x_s) - M(x_n)) (Eq. appq);
 *  * every node solid at the previous classification and fluid now is refilled
 *    (Sec. 2.3.3) from the populations of its fluid neighbours at the previous
 *    time level, with u_new = v + omega x (x_new - x_p) of the particle that
 *    covered it, then collided; the first call after lbm_init refills nothing.
 * Coordinates on a periodic axis are taken at the image nearest x_p.
 * Each particle's links are held in a segment of the library's link list
 * sized from that particle's own count at the first call (a quarter and 256
 * records to spare, in whole 256-record chunks) and grown, alone, when a
 * later call finds it outgrown.
 * Synchronises the stream to report counts (out may be NULL).  EINVAL when a
 * particle's body reaches beyond box_half, K <= 0, or x_p lies outside
 * [0, n) on a periodic axis; the previous classification then stays in force.
 * ENUMERIC when a step since the previous classification produced a
 * non-finite force or torque; the context is then failed. */
int lbm_classify_nodes(lbm_ctx* ctx, const lbm_particles* P, lbm_counts* out);

/* The same classification without the read-back of its list counts, so the
 * host does not wait for it: for replaying poses whose lists an earlier
 * lbm_classify_nodes of this context has already sized (the recomputation
 * of an adjoint window, a prescribed trajectory run a second time).  The
 * counts stay on the device: the refill reads its own, and lbm_step runs its
 * link kernel over every particle's segment whole.  What lbm_classify_nodes would
 * have reported is latched on the device instead: a rejected particle (the
 * EINVAL cases above; the owners are then not rebuilt) or a list that
 * outgrew its capacity (ECAPACITY; its extra entries are dropped).  The next
 * lbm_synchronize, lbm_classify_nodes, lbm_adjoint or lbm_adjoint_coupled
 * returns that error and leaves the context failed, since the steps run in
 * between used incomplete geometry.  lbm_get_links and lbm_get_refill
 * return ESTATE until the next lbm_classify_nodes.  Asynchronous. */
int lbm_classify_nodes_async(lbm_ctx* ctx, const lbm_particles* P);

/* One lattice step n -> n+1 on the links of the last classification:
 * VIBB (Eqs. eqneq, neqd, rhod, u_d) or halfway reconstruction of the unknown
 * populations, Galilean-invariant momentum exchange force and torque per
 * particle (Eq. mem, and Eqs. fh_s_issue / th_s_issue for missing points),
 * then fused pull-streaming and BGK collision (Eq. lbm_collide, with Guo
 * forcing for body_force) of every fluid node.  Wall velocities come from
 * P->vel, P->omega and P->pos.  Asynchronous.  A step whose force or torque
 * sums are not finite (a run that has gone unstable) is reported by the next
 * lbm_classify_nodes as ENUMERIC, which leaves the context failed. */
int lbm_step(lbm_ctx* ctx, const lbm_particles* P);

/* Copy the force F^h and torque T^h (FP64, [n][3] each, device pointers) of
 * the last lbm_step into F_dev and T_dev.  Asynchronous. */
int lbm_particle_forces(const lbm_ctx* ctx, double* F_dev, double* T_dev);

/* n_sub velocity-Verlet substeps of length dt of the metaball DEM (Sec. 2.1)
 * with F^h, T^h of the last lbm_step frozen (sub-cycling, Sec. 2.3.4),
 * relative gravity, metaball-metaball and metaball-wall contacts with a
 * linear spring-dashpot normal force and a Coulomb-limited tangential spring.
 * Updates P->pos, quat, vel, omega and world_pts in place and the contact
 * histories held by the context (allocated by lbm_init: 32 pair records per
 * particle, for its candidate partners of higher index, and one per wall;
 * from 2048 particles on also a cell grid of at most max(4096, 4 n) cells
 * for the broad phase, which then tests only the 27 cells around each
 * particle instead of every pair: the same candidates either way).
 * EINVAL on n_sub < 1 or dt <= 0.  A particle with more than 32 candidate
 * partners in one call (centres within the bodies' reach plus the call's
 * displacement) has the extra pairs left out; that is latched and reported
 * as ECAPACITY, with the context failed, by the next lbm_synchronize or
 * lbm_classify_nodes.  Allocates nothing.  Asynchronous. */
int dem_step(lbm_ctx* ctx, lbm_particles* P, int n_sub, double dt, const dem_params* prm);

/* lbm_step followed by dem_step, with the DEM sub-cycle (which needs only
 * the step's F^h and T^h, Sec. 2.3.4) running beside the stream-collide pass
 * instead of after it: the link pass and the force sums on the context's
 * stream, then the stream-collide pass and the n_sub DEM substeps on two
 * streams of the library's own (default priority; the DEM's on two compute
 * units of each XCD, the stream-collide's on the rest), and the context's
 * stream waits for both.  The populations, forces, particle state and
 * contact histories are those of lbm_step then dem_step.  For a step that
 * is taped (lbm_tape_begin, its output goes to the tape), with no particles
 * or before the first classification it runs the two calls one after the
 * other.  The two streams
 * and three events are made on the first call (EDEVICE if that fails) and
 * kept until lbm_destroy.  Argument checks and errors: those of lbm_step
 * and dem_step.  Asynchronous. */
int lbm_step_dem(lbm_ctx* ctx, lbm_particles* P, int n_sub, double dt, const dem_params* prm);

/* dem_step for callers that cannot allocate device memory or use memory the
 * library allocated after lbm_init (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): the same substeps and results,
 * with the call's work space (candidate pairs, their count, the bodies'
 * reach) in a static device array instead of the context's, looked up once
 * per device by lbm_init.  The array holds at most 1024 particles (about
 * 270 KB per device, held until the process ends); EINVAL for a context with
 * more.  Every call on one device shares that array and leaves its contents
 * there: calls that overlap on one device (on different streams or
 * contexts) race and must not be issued.  Calls no hipMalloc, hipFree or
 * hipMemset.  Asynchronous. */
int dem_step_noalloc(lbm_ctx* ctx, lbm_particles* P, int n_sub, double dt, const dem_params* prm);

/* ---- inspection (tests and tools) --------------------------------------- */

/* Links of the last classification, in an unspecified order, into device
 * arrays of capacity cap; *n_out (host) receives the count.  ECAPACITY when
 * cap is too small (nothing written, *n_out still set).  Synchronises. */
int lbm_get_links(const lbm_ctx* ctx, int64_t cap, int32_t* node_dev, int8_t* d_dev,
                  int8_t* kind_dev, int32_t* part_dev, double* q_dev, int64_t* n_out);

/* Nodes refilled by the last classification (unspecified order) and the
 * particle that had covered each.  Same capacity rules as lbm_get_links. */
int lbm_get_refill(const lbm_ctx* ctx, int64_t cap, int32_t* node_dev, int32_t* part_dev,
                   int64_t* n_out);

/* Owner of every node at the last classification: 0 fluid, p+1 particle p
 * (int32, ncell entries).  Asynchronous. */
int lbm_get_owner(const lbm_ctx* ctx, int32_t* owner_dev);

/* Current post-collision populations as FP64 f_i (not deviations), Q planes of
 * ncell (x fastest) into f_dev.  Asynchronous. */
int lbm_get_populations(const lbm_ctx* ctx, double* f_dev);

/* Density and velocity of every node in FP64: rho_dev [ncell], u_dev
 * [ncell][3], from the moment plane that every collision writes (rho of the
 * node and u = (sum f e + F/2) / rho of its last collision, or of the
 * initial equilibrium; solid nodes hold rho = 1, u = 0).  Asynchronous. */
int lbm_get_moments(const lbm_ctx* ctx, double* rho_dev, double* u_dev);

/* Overwrite the current populations from FP64 f_i planes (rounded to the
 * storage format).  Asynchronous. */
int lbm_set_populations(lbm_ctx* ctx, const double* f_dev);

/* Block until the context's stream has drained; EDEVICE on a device error;
 * otherwise the error latched on the device since the last check, if any,
 * which leaves the context failed: ENUMERIC for a step with a non-finite
 * force or torque, EINVAL or ECAPACITY for an lbm_classify_nodes_async
 * that rejected the particles or outgrew its lists, ECAPACITY for a
 * dem_step in which a particle had more candidate partners than its
 * contact-history records. */
int lbm_synchronize(lbm_ctx* ctx);

/* ---- differentiation form (not in the paper) -----------------------------
 *
 * The adjoint differentiates J = sum over taped steps n and particles p of
 * wF_p . F^h_p(n) + wT_p . T^h_p(n), holding the discrete geometry (owners,
 * link sets, refill sets and rule choices) of the taped run fixed.
 * lbm_adjoint (prescribed motion) gives the gradient with respect to the
 * fluid body force F, the relaxation time tau and the particle velocities
 * v_p, which enter through the wall velocities of VIBB, halfway bounce-back,
 * refilling and the momentum exchange, and optionally with respect to every
 * pose of the trajectory (translation and rotation, through q and the lever
 * arms).  lbm_adjoint_coupled (free motion) gives it with respect to the
 * initial position, orientation, velocity and angular velocity of every
 * particle, through the DEM substeps, and to F and tau. */

/* Copy the current populations and moments, raw, into dst_dev
 * (checkpoint_bytes).  Asynchronous. */
int lbm_checkpoint_save(const lbm_ctx* ctx, void* dst_dev);

/* Restore populations and moments from a raw checkpoint, and forget the
 * classification history: the next lbm_classify_nodes refills nothing, so
 * classifying the checkpoint's particle state reproduces its geometry.
 * Asynchronous. */
int lbm_checkpoint_load(lbm_ctx* ctx, const void* src_dev);

/* Copy the DEM state the library keeps between dem_step calls (the contact
 * histories of the candidate particle pairs, with the partner each record
 * belongs to, and of every particle-wall pair: tangential springs and warm
 * starts of the contact-point search; and the contact forces of the last
 * substep) into dst_dev (dem_checkpoint_bytes); all zero before the first
 * dem_step, and an all-zero state loads as no contact histories.  Together with lbm_checkpoint_save and the
 * caller's particle arrays this resumes a run exactly. */
int lbm_dem_checkpoint_save(const lbm_ctx* ctx, void* dst_dev);

/* Restore the DEM state saved by lbm_dem_checkpoint_save. */
int lbm_dem_checkpoint_load(lbm_ctx* ctx, const void* src_dev);

/* ---- geometry snapshots (differentiation form) ------------------------- */

/* Bytes of one geometry snapshot for the context's current link layout (the
 * particles' segments) and refill list capacity, and a tag naming them (for
 * lbm_geometry_load).  A snapshot is about owner_bytes + flag_bytes + 16 B
 * per link slot. */
int lbm_geometry_bytes(const lbm_ctx* ctx, size_t* bytes, uint64_t* tag);

/* Copy the geometry of the last classification -- owner plane, flags, link
 * records with their counts, the nodes it refilled, the particles' bounding
 * balls -- into dst_dev (lbm_geometry_bytes).  For runs that are replayed
 * (the adjoint's recomputation of a window): a replayed step then loads the
 * geometry instead of classifying the same poses again.  ESTATE before the
 * first classification.  Asynchronous. */
int lbm_geometry_save(lbm_ctx* ctx, void* dst_dev);

/* Stand in for lbm_classify_nodes(ctx, P) at the pose P a snapshot of the
 * same context was saved at: its owners, flags and links become the current
 * geometry and its refilled nodes are refilled from the current populations,
 * as that classification did (nothing after lbm_checkpoint_load, as
 * lbm_classify_nodes).  tag: as returned by lbm_geometry_bytes when the
 * snapshot was sized; ESTATE when the link layout or the refill capacity
 * changed since.  The
 * list counts are not read back (as lbm_classify_nodes_async).  A taped
 * step (lbm_tape_begin) whose geometry was loaded records the snapshot's
 * owners and links by reference instead of copying them: keep the snapshot
 * until lbm_adjoint or lbm_adjoint_coupled has consumed the tape.
 * Asynchronous. */
int lbm_geometry_load(lbm_ctx* ctx, const void* src_dev, uint64_t tag, const lbm_particles* P);

/* Record the next max_steps calls of lbm_step (populations after the link
 * reconstruction, owners, links, particle pose and velocities) for
 * lbm_adjoint.  The tape's device memory (about population_bytes +
 * owner_bytes + the link list per step) is allocated on the first call that
 * needs more steps than are held and kept for later windows; max_steps = 0
 * releases it (lbm_destroy does too).  ENOMEM when it does not fit, ESTATE
 * before the first classification. */
int lbm_tape_begin(lbm_ctx* ctx, int max_steps);

/* Run the adjoint backwards over the taped steps; the tape's memory is kept
 * for the next lbm_tape_begin.
 *   P        particle state after the last taped step (the one the last
 *            classification used: its velocities drive that refill);
 *   weights  host [n][6]: (wF, wT) per particle, the same for every step;
 *   lam_dev  adjoint field (adjoint_bytes): on entry dJ/df after the last taped
 *            step (zeros for J above), on return dJ/df at the first taped step;
 *   grad_dev device FP64 [4 + 3 n], accumulated into: dJ/dF (3), dJ/dtau,
 *            dJ/dv_p (3 per particle);
 *   gpos_dev NULL, or device FP64 [(T + 1) n 6] for T taped steps, accumulated
 *            into: entry k holds, for particle p's pose P_k (the pose the
 *            k-th taped step's links were built from, and whose
 *            classification refilled the nodes that step found new; P_T is
 *            P), dJ/dx_p for a translation and dJ/dtheta_p for a small
 *            world-frame rotation about x_p, with the owners, links and
 *            refill sets held fixed: through q (Eq. appq, or Eq. calq when
 *            LBM_TREAT_EXACT_Q), the wall point x_w = x_n + q e_d, the lever
 *            arm x_w - x_p of the torque and of u_w = v + omega x (x_w - x_p),
 *            and the refill's u = v + omega x (x - x_p).
 * Synchronises.  ESTATE when nothing was taped. */
int lbm_adjoint(lbm_ctx* ctx, const lbm_particles* P, const double* weights, void* lam_dev,
                double* grad_dev, double* gpos_dev);

/* The adjoint of a run in which the particles move freely: each taped step
 * was followed by dem_step(ctx, P, n_sub, dt, prm) and then
 * lbm_classify_nodes, so the state that the next step used came from the
 * previous one and the step's F^h, T^h through the DEM, contacts included.
 * The DEM state is s = (x, q, v, omega) per particle, the contact force and
 * torque carried into the next call's first half kick, and the tangential
 * spring of every contact record (pair and particle-wall).  Running
 * backwards, each step (1) adds the refill's wall-velocity terms to the
 * adjoint of s_{k+1}, (2) applies the transposed Jacobian of the dem_step
 * call (forward-mode dual numbers over x, a small world-frame rotation
 * theta, v, omega, F^h, T^h, the carried contact sum and the springs,
 * through the same substeps and contacts; the contact point's derivative by
 * the implicit function theorem at the converged Newton point), giving the
 * adjoint of s_k and dJ/dF^h_k, dJ/dT^h_k, (3) runs the step's node and link
 * adjoint with objective weights (wF, wT) + (dJ/dF^h_k, dJ/dT^h_k), adding
 * the link terms of s_k (pose through q and the lever arms, v and omega
 * through u_w).  Each particle's contact cluster in one call (the particles
 * linked to it through broad-phase candidate pairs) may hold at most 8
 * particles: ESTATE otherwise, with the tape consumed and the outputs not
 * valid.  Discrete events (a contact starting or ending, the Coulomb limit
 * switching) are not differentiated across.
 *   P         the state after the last taped step's dem_step (the one the
 *             last classification used);
 *   weights   host [n][6]: (wF, wT) per particle, the same for every step;
 *   prm, n_sub, dt  the dem_step arguments of the run;
 *   lam_dev   as for lbm_adjoint;
 *   grad_dev  device FP64 [4], accumulated into: dJ/dF (3), dJ/dtau;
 *   sigma_dev device FP64 [n][12]: on entry the adjoint of P (zeros for J
 *             above), on return the adjoint of the state the first taped
 *             step used, ordered (x, theta, v, omega);
 *   sigma_contact_dev  NULL (zero on entry, not returned), or device FP64
 *             (contact_adjoint_bytes): the same for the contact state, so
 *             that windows run from the last to the first chain their
 *             adjoints.
 * Synchronises.  ESTATE when nothing was taped. */
int lbm_adjoint_coupled(lbm_ctx* ctx, const lbm_particles* P, const double* weights,
                        const dem_params* prm, int n_sub, double dt, void* lam_dev,
                        double* grad_dev, double* sigma_dev, double* sigma_contact_dev);

/* ---- kernel timing (hipEvent pairs around each launch group) ------------ */

typedef enum {
    LBM_PHASE_BULK = 0,      /* fused stream-collide of lbm_step (one kernel) */
    LBM_PHASE_BOUNDARY = 1,  /* link reconstruction + momentum exchange of lbm_step */
    LBM_PHASE_CLASSIFY = 2,  /* geometry kernels of lbm_classify_nodes */
    LBM_PHASE_REFILL = 3,    /* refill kernel of lbm_classify_nodes */
    LBM_PHASE_DEM = 4,       /* all substeps of one dem_step */
    LBM_PHASE_ADJOINT = 5,   /* one adjoint step of lbm_adjoint */
    LBM_PHASE_COUNT = 8
} lbm_phase;

typedef struct {
    double ms[LBM_PHASE_COUNT];        /* summed GPU time of the phase's launch groups */
    int64_t launches[LBM_PHASE_COUNT]; /* number of launch groups timed */
} lbm_profile;

/* Start (on != 0) or stop timing; starting clears the accumulated figures.
 * While on, every launch group is bracketed by hipEventRecord on the
 * context's stream. */
int lbm_profile_enable(lbm_ctx* ctx, int on);

/* Synchronise the stream and return the figures accumulated since timing was
 * started. */
int lbm_profile_read(lbm_ctx* ctx, lbm_profile* out);

#ifdef __cplusplus
}
#endif

#endif /* MDLBM_H */

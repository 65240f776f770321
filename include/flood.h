/*
 * flood.h - C ABI of the MI355X ensemble local-inertial flood library.
 *
 * The library advances an ensemble of storage-cell flood models (paper Sec.
 * 2.1, Eqs. 1-5) over one or more catchments on one AMD Instinct MI355X
 * (gfx950), assimilates gauge observations with a particle filter (Sec. 2.2,
 * Eqs. 6-12, and the five-step cycle of Sec. 3.3) and differentiates a
 * gauge-misfit loss with respect to the Manning field and the per-member rain
 * multipliers by a hand-written discrete adjoint.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Cells are row-major [r][c], r = 0 is the north edge, cell size dx = dy.
 * - Host-facing discharge layouts: QX is ny x (nx+1), column c the link
 *   between cells (r,c-1) and (r,c) (column 0 = west edge, nx = east edge);
 *   QY is (ny+1) x nx, row r the link between (r-1,c) and (r,c).  Positive
 *   discharge points toward +c / +r; units m^2/s (per unit width).
 * - Edges are indexed N=0, E=1, S=2, W=3.
 * - Every pointer argument is caller-owned and read (or written) during the
 *   call only; the library keeps no reference to it.  The handle owns all
 *   device memory it allocates.
 * - Work is enqueued on the HIP stream given at creation.  Calls that return
 *   host data synchronise that stream; the others return after enqueueing,
 *   except flood_step, which polls a small device counter to know when every
 *   member has reached its end time.
 * - Functions return FLOOD_OK (0) or a negative status.  Nothing throws
 *   across the ABI.  Arguments are validated before any HIP call, so a
 *   rejected call leaves the handle unchanged.  flood_last_error() gives a
 *   human-readable reason.
 * - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef FLOOD_H
#define FLOOD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t flood_status;
#define FLOOD_OK 0
#define FLOOD_EINVAL (-1)   /* bad argument; nothing was done */
#define FLOOD_ENOMEM (-2)   /* device or pinned host allocation failed */
#define FLOOD_EHIP (-3)     /* a HIP runtime call failed (no device, launch error) */
#define FLOOD_ESTATE (-4)   /* call not valid in the handle's current state */
#define FLOOD_ENUMERIC (-5) /* a member's depth became non-finite, or so large that its Eq. 4 step no
                               longer advances its clock (t + dt == t); that member is frozen */

#define FLOOD_EDGE_WALL 0   /* zero-flux edge (Sec. 4.1 Neumann walls) */
#define FLOOD_EDGE_OPEN 1   /* free outflow with a fixed outward surface slope */

#define FLOOD_FIELD_H 0
#define FLOOD_FIELD_QX 1
#define FLOOD_FIELD_QY 2
#define FLOOD_FIELD_PEAK 3 /* running maximum depth (handles created with track_peak = 1) */

#define FLOOD_MAX_CATCHMENTS 8
#define FLOOD_MAX_MEMBERS 1024 /* per catchment (one workgroup runs the filter) */

/* One catchment's static description (Sec. 4.1: DEM and roughness rasters). */
typedef struct flood_grid {
    int32_t ny, nx;            /* cells; 1 <= ny, nx; ny*nx <= 2^28 */
    double dx;                 /* cell size in metres, > 0 */
    const float* dem;          /* host [ny*nx] bed elevation, finite */
    const float* manning_n;    /* host [ny*nx] Manning n (s m^-1/3), finite, > 0 */
    const float* h0;           /* host [ny*nx] initial depth >= 0, or NULL for a dry start */
    int32_t edge_kind[4];      /* FLOOD_EDGE_WALL or FLOOD_EDGE_OPEN per edge N,E,S,W */
    double edge_slope[4];      /* outward water-surface slope of an open edge, > 0 */
    const uint8_t* land_class; /* host [ny*nx] land-cover class of each cell (< n_classes of the params),
                                  or NULL: no land cover (Sec. 4.1, Fig. 6) */
} flood_grid;

/* Forcing and numerics shared by all members of a catchment. */
typedef struct flood_params {
    const double* rain_rate;   /* host [n_rain] rain rate in m/s, piecewise constant per block
                                  (Sec. 3.1 step I refreshes rain every 5 min); zero after the series */
    int32_t n_rain;            /* >= 0 */
    double rain_interval;      /* block length in s, > 0 (300 in the paper) */
    double cfl_alpha;          /* Courant coefficient k of Eq. 4, in (0, 1] */
    double h_dry;              /* links with flow depth <= h_dry carry no flow, >= 0 */
    double dt_cap;             /* upper bound on the adaptive step in s, > 0 */
    double dt_fixed;           /* > 0: use this fixed step instead of Eq. 4 (the paper ran 0.25 s) */
    double g;                  /* gravity, > 0 (9.81) */
    int32_t real_bytes;        /* 4: FP32 state and arithmetic, 8: FP64 */
    int32_t member_interleave; /* 0: autotune; else 1, 2, 4 or 8 members adjacent in the fastest index.
                                  Must agree across catchments of one handle. */
    int32_t tile_rows;         /* 0: autotune; else 1, 2, 4 or 8 cell rows per 256-lane tile */
    int32_t chunks_per_block;  /* 0: autotune; else member chunks processed by one workgroup */
    int32_t step_kernel;       /* 0: autotune; 1: tiled kernel; 2: row-marching kernel; 3: vectorised
                                  row-marching kernel (2 and 3 need member_interleave 1, i.e. members
                                  stored in planes; 3 also needs nx a multiple of 4 (FP32) or 2 (FP64)) */
    int32_t march_rows;        /* 0: autotune; else rows per strip of the row-marching kernel, 1..4096 */
    int32_t march_members;     /* 0: autotune; else members marched together by one wavefront: 1, 2, 4, 8 */
    int32_t track_peak;        /* 1: keep each member's running maximum depth (ensemble products, Sec. 4.4,
                                  Figs. 15-16); costs a read and a write of one value per member-cell-step.
                                  0: off */
    /* Land cover (Sec. 4.1, Table 1), used when the grid has a class map:
     * each member has its own Manning n per class (link value: mean of the two
     * cells' values; edge links: the inner cell's), the rain reaching a cell is
     * the member's rain times the runoff coefficient of the cell's class, and
     * cells of draining classes lose the member's drainage rate, up to the water
     * they hold after the step (logged as drained volume).  The shared Manning
     * field and n_scale are not used.  Needs member_interleave 0 or 1,
     * step_kernel 0 or 3, and nx a multiple of 4 (FP32) or 2 (FP64). */
    int32_t n_classes;              /* 0 (no land cover) .. 4 */
    const double* class_runoff;     /* host [n_classes], each in [0, 1] */
    const int32_t* class_drain;     /* host [n_classes], 1: the drainage rate applies, 0: it does not */
    const double* member_class_n;   /* host [n_members*n_classes], member-major, finite, > 0 */
    const double* member_drain;     /* host [n_members] drainage rates in m/s, finite, >= 0 (NULL: 0) */
    /* Inflow hydrographs (Sec. 4.1: the boundary cells of two stream outlets
     * carry synthetic discharge series).  An inflow link is an edge link whose
     * discharge into the domain is prescribed by a series, piecewise constant
     * over the rain blocks (block j holds inflow_q[series*n_rain + j]; zero
     * outside the series); it replaces the edge's wall or open condition on
     * that link and its volume is logged as inflow, not outflow.  The same for
     * every member.  Needs member_interleave 0 or 1, step_kernel 0 or 3 and nx
     * a multiple of 4 (FP32) or 2 (FP64); the adjoint refuses it. */
    int32_t n_inflow;               /* 0 .. 2*(nx+ny) inflow links */
    const int32_t* inflow;          /* host [n_inflow*3]: edge (N=0, E=1, S=2, W=3), position along the edge
                                       (column on N/S, row on E/W), series index; each link at most once */
    int32_t n_series;               /* 1 .. 4 when n_inflow > 0 */
    const double* inflow_q;         /* host [n_series*n_rain] inward discharge per unit width, m^2/s,
                                       finite, >= 0 */
} flood_params;

typedef struct flood_handle flood_handle;

/* Create a handle for one catchment with n_members members (Eq. 6: each
 * member evolves under its own parameters).  n_scale[i] multiplies the shared
 * Manning field for member i and rain_mult[i] its rain series (Sec. 4.1 treats
 * roughness and precipitation as the uncertain inputs); either may be NULL
 * (all ones).  hip_stream may be NULL (the default stream).  All members start
 * at t = 0 with equal log-weights -log N (Eq. 7).
 * Errors: EINVAL (validation), ENOMEM, EHIP.  *out is NULL on failure. */
flood_status flood_create(const flood_grid* grid, const flood_params* params, int32_t n_members,
                          const double* n_scale, const double* rain_mult, void* hip_stream,
                          flood_handle** out);

/* Create one handle holding n_catch catchments of possibly different sizes
 * (members_per_catch[i] members each).  Every step advances all of them in
 * one batched launch.  n_scale[i] / rain_mult[i] point to per-catchment
 * arrays or are NULL.  params[i].member_interleave must be equal for all i. */
flood_status flood_create_batch(int32_t n_catch, const flood_grid* grids, const flood_params* params,
                                const int32_t* members_per_catch, const double* const* n_scale,
                                const double* const* rain_mult, void* hip_stream, flood_handle** out);

/* Advance every member of every catchment to time t_end (s).  Each member
 * takes Eq. 4 steps computed from its own maximum depth (or the fixed step),
 * clipped so that a step ends exactly on every rain-block edge and on t_end.
 * Members already at or beyond t_end are left unchanged.
 * Errors: EINVAL (t_end not finite), ESTATE (handle faulted), ENUMERIC (a
 * member's depth became non-finite or too large for its step to advance its
 * clock; it stays frozen, the others still reach t_end, and later calls keep
 * reporting it until a snapshot is restored), EHIP. */
flood_status flood_step(flood_handle* h, double t_end);

/* flood_step with a bound: every member takes at most max_steps (>= 1) more
 * steps toward t_end, each exactly the step flood_step would take (Eq. 4 or
 * the fixed step, clipped to rain-block edges and t_end).  With max_steps = 1
 * a caller observes every step of a trajectory, e.g. to replay it in a
 * reference model.  Errors: as flood_step; EINVAL when max_steps < 1. */
flood_status flood_step_n(flood_handle* h, double t_end, int64_t max_steps);

/* Wet/dry decision each link of one member takes in its next step, from the
 * member's current state (Sec. 2.1: a link carries flow only when the flow
 * depth of Eq. 3 exceeds h_dry; the paper's remark on wet-dry fronts is why
 * this decision is exported for checking).  The flow depth is formed exactly
 * as the step kernels form it: the depth of the cell with the higher water
 * surface minus the positive part of the bed step towards the other cell.
 * Open edge links are wet when their inner cell's depth exceeds h_dry; walls
 * and inflow links take no decision and read 0.
 *   wet_x host [ny*(nx+1)], wet_y host [(ny+1)*nx] (the QX / QY layouts), 1 or 0
 * Errors: EINVAL (indices, NULL outputs), EHIP.  Synchronises the stream. */
flood_status flood_get_wet_mask(flood_handle* h, int32_t catchment, int32_t member, uint8_t* wet_x, uint8_t* wet_y);

/* Step log for replaying trajectories in a reference model: from this call
 * on, every step of every member records its length dt and its end time
 * (Eq. 4 step, clipped; FP64 as the handle uses them), up to capacity entries
 * per member; a member's counter keeps counting past the capacity.  Each call
 * restarts every counter; capacity 0 closes the log.  A particle-filter copy
 * does not move logs: slot j's log is the history of slot j.  The adjoint's
 * own forward run is not logged.  Errors: EINVAL (capacity outside
 * [0, 2^24]), ENOMEM. */
flood_status flood_log_steps(flood_handle* h, int32_t capacity);

/* Copy the step log of one catchment: dt_out and t_end_out host [N*capacity]
 * member-major (entry i of member m at m*capacity + i), count_out host [N]
 * steps taken since the log was opened (entries beyond the capacity were
 * dropped).  Any output may be NULL.  ESTATE when no log is open. */
flood_status flood_get_step_log(flood_handle* h, int32_t catchment, double* dt_out, double* t_end_out,
                                int64_t* count_out);

/* Particle-filter cycle of Sec. 3.3 on one catchment whose members are all at
 * the same time: (I) gauge depths y_ik = h_i(gauge_k), (II) weights
 * w_i ~ w_i^- exp(-1/2 sum_k ((y_ik - d_k)/sigma_k)^2) (Eqs. 9-11, computed in
 * log space), (III) N_eff = 1/sum w_i^2 (Eq. 12); if N_eff < neff_frac * N,
 * (IV) systematic resampling with offset u0 in [0,1) and (V) replacement of
 * every member by a copy of its ancestor, followed by rain_mult_i *= beta_i
 * (Sec. 4.4 perturbation).  After resampling every log-weight is -log N.
 *   gauge_rc  host [2*n_gauges] (row, col) pairs inside the grid
 *   obs       host [n_gauges] observed depths d_k
 *   sigma     host [n_gauges] observation standard deviations, > 0
 *   beta      host [N] or NULL (no perturbation)
 *   neff_out, ancestors_out [N], resampled_out: host outputs, each may be NULL
 * Errors: EINVAL, ESTATE (members not at a common time, or faulted), EHIP. */
flood_status flood_assimilate(flood_handle* h, int32_t catchment, int32_t n_gauges, const int32_t* gauge_rc,
                              const double* obs, const double* sigma, double neff_frac, double u0,
                              const double* beta, double* neff_out, int32_t* ancestors_out,
                              int32_t* resampled_out);

/* Gradient of the gauge-misfit loss
 *   L = sum_members sum_{s=1..S} sum_k (h_m(g_k, t0 + s*sample_dt) - obs[s-1][k])^2,
 * S = floor((t_end - t0)/sample_dt), over the members of one catchment that
 * are all at time t0, with respect to the catchment's shared Manning field
 * (grad_n_out, host [ny*nx]) and each member's rain multiplier
 * (grad_mult_out, host [N]).  The members are taken in groups that fit the
 * device memory.  The forward run of a group records every step of every
 * member, its length and its state, in a tape: the row-march form (members in
 * planes, step kernel 3) keeps one state per member step in a pool of blocks
 * shared by the group, the tiled form ckpt_every + 1 states per member.  A
 * segment ends when a member has taken ckpt_every steps in it (or the pool
 * could run out), and the group's states become a checkpoint.  The reverse
 * sweep applies the discrete adjoint of the step with the recorded step
 * lengths and the forward's wet/dry, limiter and clamp branches held fixed:
 * the last segment straight from the tape, each earlier one after recomputing
 * it from its checkpoint.  A ckpt_every at least the members' step count
 * therefore means no recomputation, at the price of tape memory (and smaller
 * groups).  In the row-march form the members are taken most expected steps
 * first, and each group holds as many members as the pool holds at the step
 * counts of the group before it.  The loss and the rain-multiplier gradients
 * do not depend on ckpt_every or the grouping; the Manning field's only
 * through the single-precision rounding of its accumulation (the
 * contributions of four members are added together per reverse step).  On
 * return the members are at the last sample time.
 *   obs host [S*n_gauges]; loss_out, grad_n_out, grad_mult_out may be NULL.
 * Errors: EINVAL, ENOMEM (tape does not fit), ESTATE, ENUMERIC, EHIP. */
flood_status flood_adjoint(flood_handle* h, int32_t catchment, double t_end, double sample_dt,
                           int32_t n_gauges, const int32_t* gauge_rc, const double* obs, int32_t ckpt_every,
                           double* loss_out, double* grad_n_out, double* grad_mult_out);

/* flood_adjoint keeps its scratch on the handle for the next call: the tape
 * (row-march form: a pool of blocks in about 85 % of the device memory that was
 * free at the first call, at most what min(N, 16) members taking ckpt_every
 * steps each would use; tiled form: ckpt_every + 1 states of a member group and their clamp
 * flags, up to half of it), two adjoint copies, the Manning accumulators and
 * the checkpoints.  A later call keeps a held pool that is at least 15/16 of
 * the one it would allocate.  Allocating and freeing that much on every call
 * would cost seconds once the memory has been recycled.
 * flood_adjoint_release frees it now (flood_destroy frees it too); a later
 * flood_adjoint allocates it again.  Errors: EINVAL (NULL handle). */
flood_status flood_adjoint_release(flood_handle* h);

/* Copy one member's field to host memory in the host layout described above
 * (H: ny*nx, QX: ny*(nx+1), QY: (ny+1)*nx, PEAK: ny*nx), converted to double.
 * PEAK, the member's running maximum depth since creation (or its last
 * flood_set_state), needs a handle created with track_peak = 1 (else ESTATE). */
flood_status flood_get_field(flood_handle* h, int32_t catchment, int32_t member, int32_t which,
                             double* host_out);

/* Overwrite one member's state (h: ny*nx, qx: ny*(nx+1), qy: (ny+1)*nx, all
 * host doubles, rounded to the handle's precision) and its time t.  Depths
 * must be >= 0 and finite.  Wall links must be zero (inflow links excepted).  A tracked running maximum
 * restarts from the new depths. */
flood_status flood_set_state(flood_handle* h, int32_t catchment, int32_t member, const double* hh,
                             const double* qx, const double* qy, double t);

/* Replace the shared Manning field (host [ny*nx], > 0) and, when non-NULL,
 * the per-member scales and rain multipliers (host [N]) of one catchment. */
flood_status flood_set_params(flood_handle* h, int32_t catchment, const float* manning_n,
                              const double* n_scale, const double* rain_mult);

/* Mass ledger of one catchment, each output host [N] or NULL:
 * storage = sum h dx^2, rain_in = total rain volume added, outflow = volume
 * that left through open edges, clamp = volume added by clamping negative
 * depths to zero, drained = volume lost to drainage (land cover), inflow =
 * volume that entered through inflow links; t = member times; steps = steps
 * taken.  Invariant:
 * storage - storage(t=0) = rain_in + inflow - outflow + clamp - drained. */
flood_status flood_get_ledger(flood_handle* h, int32_t catchment, double* storage, double* rain_in,
                              double* outflow, double* clamp, double* drained, double* inflow, double* t,
                              int64_t* steps);

/* Streamflow gauges (Sec. 4.4: the flow through a section is the sum of the
 * fluxes on the links across it).  Registers the sections of one catchment,
 * replacing any registered before (n_sections 0 clears them):
 *   link_count  host [n_sections], each >= 1; at most 65536 links in all
 *   links       host [sum of link_count][4]: kind (0 x-link, 1 y-link), r, c,
 *               sign (+1 or -1), in the host discharge layouts above (x-link
 *               (r, c): 0 <= r < ny, 0 <= c <= nx; y-link (r, c): 0 <= r <= ny,
 *               0 <= c < nx)
 * The discharge of section s is dx * sum over its links of sign * q, m^3/s.
 * At most 64 sections.  Errors: EINVAL. */
flood_status flood_set_sections(flood_handle* h, int32_t catchment, int32_t n_sections, const int32_t* link_count,
                                const int32_t* links);

/* Discharge through every registered section for every member, host
 * [N*n_sections] member-major.  ESTATE when no section is registered. */
flood_status flood_get_sections(flood_handle* h, int32_t catchment, double* q_out);

/* Particle-filter cycle of flood_assimilate on depth gauges and streamflow
 * gauges together: the observation vector is the n_gauges depths followed by
 * the discharges of every registered section (Sec. 4.4: three depth and two
 * flow gauges).  obs and sigma are host [n_gauges + n_sections].  alpha > 0:
 * relative observation error, sigma_k = max(alpha |d_k|, sigma[k]) (Sec. 4.4
 * uses alpha = 0.05; sigma is the floor that keeps an observation of zero
 * usable); alpha = 0: sigma_k = sigma[k].  Other arguments, outputs and errors
 * as flood_assimilate. */
flood_status flood_assimilate_obs(flood_handle* h, int32_t catchment, int32_t n_gauges, const int32_t* gauge_rc,
                                  const double* obs, const double* sigma, double alpha, double neff_frac, double u0,
                                  const double* beta, double* neff_out, int32_t* ancestors_out,
                                  int32_t* resampled_out);

/* Land-cover parameters of every member (they follow their members through
 * resampling): class_n_out host [N*n_classes] member-major, drain_out host [N];
 * either may be NULL.  ESTATE on a catchment without land cover. */
flood_status flood_get_land_params(flood_handle* h, int32_t catchment, double* class_n_out, double* drain_out);

/* Current log-weights (host [N]) and per-member rain multipliers / n scales. */
flood_status flood_get_weights(flood_handle* h, int32_t catchment, double* logw, double* rain_mult,
                               double* n_scale);

/* Stateless systematic resampling on the device: ancestors of n particles
 * with weights w (host [n], >= 0, positive sum) and offset u0 in [0,1),
 * using the same kernel as flood_assimilate.  anc_out host [n]. */
flood_status flood_systematic_resample(const double* w, int32_t n, double u0, int32_t* anc_out,
                                       void* hip_stream);

/* flood_systematic_resample for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernel and the same ancestors, but the weights and
 * ancestors are staged in a 12 KiB device array of the library (one per GPU,
 * kept until the process ends) instead of buffers allocated per call; nothing
 * is allocated.  Runs on the current device.  n at most FLOOD_MAX_MEMBERS
 * (1024): larger n, or weights that are negative, non-finite or sum to zero,
 * give EINVAL before any HIP call.  Calls that overlap on one GPU (other host
 * threads, other streams) share the staging array and race.  Synchronises the
 * stream.  Errors: EINVAL, EHIP. */
flood_status flood_systematic_resample_noalloc(const double* w, int32_t n, double u0, int32_t* anc_out,
                                               void* hip_stream);

/* Ensemble products of the running maximum depth (Sec. 4.4, Figs. 15-16) of
 * one catchment, per cell, with member weights w (host [N], finite, >= 0,
 * positive sum; NULL: equal weights) and W = sum of w in member order:
 *   prob_out[c]         = (sum of w_m over members whose maximum at c >= threshold) / W
 *   pct_out[i*ny*nx+c]  = min over members k of their maximum v_k at c such that the
 *                         sum of w_m over members with v_m <= v_k is >= pct[i] W
 *                         (inverted distribution function)
 * All sums run over members in index order in FP64.  pct host [n_pct], each
 * in (0, 1], 0 <= n_pct <= 16; prob_out host [ny*nx] and pct_out host
 * [n_pct*ny*nx], row-major cells, either may be NULL.  Needs track_peak = 1.
 * Errors: EINVAL (validation, before any HIP call), ESTATE (not tracked),
 * ENOMEM, EHIP.  Synchronises the stream. */
flood_status flood_ensemble_products(flood_handle* h, int32_t catchment, double threshold, int32_t n_pct,
                                     const double* pct, const double* weights, double* prob_out,
                                     double* pct_out);

/* Snapshot / restore of every member's state, time, weights, parameters and
 * ledger to a file (portable only between handles of identical shape). */
flood_status flood_save(flood_handle* h, const char* path);
flood_status flood_load(flood_handle* h, const char* path);

/* The same snapshot kept on the device, in one buffer held by the handle
 * (about twice the state of every member, since both state copies are kept):
 * op FLOOD_SNAPSHOT_TAKE copies everything flood_save would write into it
 * (allocated on first use, reused after), FLOOD_SNAPSHOT_RESTORE copies it
 * back (ESTATE if none was taken) and clears the numeric-fault status,
 * FLOOD_SNAPSHOT_RELEASE frees it.  Stream-ordered, returns after enqueueing.
 * Lets a caller evaluate runs from one state repeatedly (a gradient-based
 * calibration loop) without host transfers.  Errors: EINVAL, ENOMEM, ESTATE,
 * EHIP. */
#define FLOOD_SNAPSHOT_TAKE 1
#define FLOOD_SNAPSHOT_RESTORE 2
#define FLOOD_SNAPSHOT_RELEASE 3
flood_status flood_device_snapshot(flood_handle* h, int32_t op);

/* Memory plan of the last flood_adjoint call on the handle: member groups,
 * members of the largest group, and tape segments summed over the groups
 * (segments beyond one per group were recomputed from checkpoints).  Any
 * output may be NULL; zeros before the first call. */
flood_status flood_get_adjoint_info(const flood_handle* h, int32_t* groups, int32_t* group_size,
                                    int32_t* segments);

/* Kernel configuration in use: member interleave, tile rows and chunks per
 * workgroup of catchment 0, the number of steps captured per graph, the step
 * kernel variant (1 tiled, 2 row-marching, 3 vectorised row-marching), its rows per strip, members per
 * wavefront and wavefront order (0-4: which of member, strip along x and row of strips runs fastest,
 * and how the rows are spread over the XCDs).  Any output may be NULL. */
flood_status flood_get_config(const flood_handle* h, int32_t* member_interleave, int32_t* tile_rows,
                              int32_t* chunks_per_block, int32_t* graph_steps, int32_t* step_kernel,
                              int32_t* march_rows, int32_t* march_members, int32_t* march_order);

/* Rows per strip of the row-marching step kernels for one catchment: in a
 * handle holding catchments of different sizes the tuner refines them per
 * catchment (the other outputs of flood_get_config are shared by all).
 * Errors: EINVAL. */
flood_status flood_get_march_rows(flood_handle* h, int32_t catchment, int32_t* march_rows);

/* Measurement helper: the attainable bandwidth of the row-marching step's
 * access pattern on this device.  A streaming kernel with the vectorised step's
 * geometry (a wavefront per strip of 256 cells and member, marching `rows` rows;
 * per row three member state arrays read and written with 16-byte non-temporal
 * accesses and the shared bed and roughness read) but no halo cells and no link
 * arithmetic runs `reps` timed launches on n_members x ny x nx FP32 cells of
 * buffers it allocates and frees (6 x 4 B per member-cell plus 8 B per cell);
 * *gbps_out receives 24 B per member-cell update over the fastest launch and
 * *ms_per_launch_out that launch's duration.  waves_per_simd 3..8 caps the
 * wavefronts sharing a SIMD (with LDS reserved per workgroup, at most 54 KiB),
 * so the pattern can be measured at the step kernel's occupancy; 0 leaves it
 * to the registers (8).  Errors: EINVAL (ny < 1, nx not a positive multiple of
 * 4, more than 2^31 member-cells, rows outside 1..4096, reps outside 1..1000,
 * waves_per_simd not 0 or 3..8, NULL outputs), ENOMEM, EHIP. */
flood_status flood_probe_stream(int32_t ny, int32_t nx, int32_t n_members, int32_t rows, int32_t reps,
                                int32_t waves_per_simd, void* hip_stream, double* gbps_out,
                                double* ms_per_launch_out);

/* Timing of the step launches of flood_step calls between flood_timing(h,
 * mode) and flood_timing(h, 0), with HIP events on the handle's stream.
 * FLOOD_TIMING_LAUNCH: an event pair around every step kernel launch, launched
 * one by one (the captured-graph path is off meanwhile): the average is the
 * step kernel's own duration.  FLOOD_TIMING_BATCH: the captured-graph path
 * kept, an event pair around every batch of graph_steps steps
 * (flood_get_config): the average per step launch then also holds each step's
 * planner kernel and the gaps between the batch's kernels (events recorded
 * inside a captured graph cannot be timed).  flood_get_timing gives the
 * average per step launch in ms and the number of step launches.
 * Errors: EINVAL (mode), EHIP. */
#define FLOOD_TIMING_LAUNCH 1
#define FLOOD_TIMING_BATCH 2
flood_status flood_timing(flood_handle* h, int32_t mode);
flood_status flood_get_timing(const flood_handle* h, double* avg_step_ms, int64_t* launches);

const char* flood_last_error(const flood_handle* h); /* NULL h: last creation error of this thread */
const char* flood_strerror(flood_status s);
void flood_destroy(flood_handle* h); /* NULL-safe; synchronises the stream */

#ifdef __cplusplus
}
#endif

#endif /* FLOOD_H */

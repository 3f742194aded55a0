/*
 * cloth.h — C ABI of the MI355X (gfx950) projective-dynamics cloth solver.
 *
 * The library advances a triangle-mesh cloth by implicit Euler steps written
 * as an energy minimisation (Lan et al., "Efficient GPU Cloth Simulation with
 * Non-distance Barriers and Subspace Reuse", arXiv 2403.19272, section 3,
 * Eq. (var) and Eq. (z)), solved with projective-dynamics local/global
 * iterations (Eq. (local), Eq. (global)).  Each inner iteration runs:
 *   - the local step: per-triangle strain projection, hinge bending target,
 *     and collision targets weighted by the non-distance barrier
 *     w = k K^a (Eq. (exp));
 *   - the residual of the global system against the fixed system matrix H
 *     stored as CSR, plus the diagonal collision term;
 *   - the subspace-reuse correction through the rest-shape eigenbasis U
 *     (Eq. (subspace_collision), Eq. (uu));
 *   - a Chebyshev-accelerated Jacobi sweep on the remaining residual
 *     (Eq. (high_frequency_residual));
 *   - partial CCD on every collision constraint (Eq. (query)), which updates
 *     the life spans a.
 * Every outer block ends with a broad phase, an exact time-of-impact pass and
 * the step-length filter x = x- + s (x+ - x-) (Algorithm 1, section 7).
 *
 * Conventions
 *   - Positions and velocities cross the ABI as host float arrays of nv*3
 *     values (x0,y0,z0,x1,...), in the caller's vertex order.
 *   - Every call returns a cloth_status: CLOTH_OK (0) or a negative code; no
 *     call aborts or throws.  cloth_last_error() gives a text for the last
 *     failure on the calling thread.
 *   - Host arrays passed in are borrowed for the duration of the call.
 *   - Device work is enqueued on the stream argument (a hipStream_t; 0 is the
 *     null stream).  Calls that return host data synchronise that stream.
 *   - One scene is used by one thread at a time.
 */
#ifndef CLOTH_H
#define CLOTH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t cloth_status;
#define CLOTH_OK 0
#define CLOTH_E_INVALID -1   /* bad argument or call order */
#define CLOTH_E_MESH -2      /* non-manifold or degenerate mesh */
#define CLOTH_E_OOM -3       /* arena too small / allocation failed */
#define CLOTH_E_CAPACITY -4  /* a candidate or constraint list outgrew the arena's capacity */
#define CLOTH_E_DIVERGED -5  /* NaN or Inf in an iterate */
#define CLOTH_E_TANGLED -6   /* the debug tangle check found intersecting triangles */
#define CLOTH_E_DEVICE -7    /* a HIP runtime error */

#define CLOTH_PLAIN_FP32 0   /* basis U stored in FP32 */
#define CLOTH_MIXED 1        /* basis U stored in BF16 (FP32 accumulation) */

#define CLOTH_SPHERE 0
#define CLOTH_CYLINDER 1     /* infinite along its axis for contact purposes */

typedef struct cloth_scene_s* cloth_scene;

/* Triangle mesh: nt triangles as 3 vertex indices each (0-based, one
 * consistent orientation), optional per-vertex pin flags (NULL = none). */
typedef struct {
    int32_t nv, nt;
    const int32_t* tris;
    const uint8_t* pinned;
} cloth_mesh;

/* Material and contact constants (SI units).
 *   density    mass per area, kg/m^2 (lumped: one third of each incident area)
 *   k_stretch  strain weight per rest area (PD weight w_t = k_stretch * area)
 *   k_bend     bending weight (hinge weight k_bend * 3 / (A1 + A2))
 *   sigma_min, sigma_max
 *              strain limits of the triangle projection (Eq. (local)): the
 *              target is F with its singular values clamped to this range,
 *              0 < sigma_min <= 1 <= sigma_max; 1, 1 projects onto
 *              rotations (0, 0 is read as 1, 1)
 *   k_contact  initial barrier weight k of Eq. (exp); <= 0 selects the mean
 *              elastic diagonal of H over free vertices
 *   K_base     growth base K of Eq. (exp) (the paper uses 2)
 *   a_max      cap on the life span a
 *   d_hat      contact target distance (m)
 *   alpha      filter back-off, s = alpha * t_TOI (the paper uses 0.8)
 *   friction   friction coefficient mu of obstacle contacts (0: frictionless).
 *              Lagged friction (sec. 8.4 uses a lagged friction Hessian at
 *              every local/global iteration): an obstacle constraint of
 *              vertex v in the contact band, with unit normal n, normal
 *              force lambda = w (R + d_hat - |radial|) of its barrier weight
 *              w and tangential slip u_T of (x - x*) - h v_s over the step
 *              (x* the step's start, v_s = omega R (axis x n) the surface
 *              velocity of a spinning obstacle), adds the weight
 *              mu lambda f1(|u_T|) / |u_T| with the target x - u_T, where
 *              f1(y) = 2 y / eps - y^2 / eps^2 below eps = friction_eps_v h
 *              and 1 above (a smoothed Coulomb law: the force is mu lambda
 *              while slipping, proportional to the slip while sticking)
 *   friction_eps_v
 *              the sticking velocity threshold (m/s); <= 0: 1e-3 */
typedef struct {
    double density, k_stretch, k_bend, sigma_min, sigma_max, k_contact, K_base;
    int32_t a_max;
    double d_hat, alpha;
    double friction, friction_eps_v;
} cloth_material;

/* Solver settings.
 *   r                   basis width (scalar modes; each acts on x, y and z), a
 *                       multiple of 8 in [8, 192]
 *   iters_inner/outer   iteration budget per step (inner per block); the
 *                       product is at most 65536
 *   tol_inner/outer     loop conditions of Algorithm 1 (section 7): an inner
 *                       block stops once the previous iteration moved no
 *                       vertex by tol_inner or more (max over vertices of
 *                       |x^{k+1} - x^k|), the outer loop once an outer block
 *                       moved no vertex by tol_outer or more (the filtered
 *                       x against the previous block's); both within the
 *                       budgets above, decided on the device (the remaining
 *                       launches of the step run as no-ops).  <= 0: the
 *                       budget alone
 *   cheb_rho            spectral radius estimate for the Chebyshev weights;
 *                       <= 0: estimated by power iteration when the basis is set
 *   cheb_gamma          damping of the Jacobi step; <= 0: chosen with rho
 *   cheb_delay          iterations before the Chebyshev weights start
 *   precision           CLOTH_PLAIN_FP32 or CLOTH_MIXED
 *   self_contact        1: vertex-triangle and edge-edge contact on
 *   pair_capacity       candidate pairs per list (VT, EE) the arena holds
 *                       (0: 128 per vertex); a step whose stage finds more
 *                       fails (see cloth_step).  The constraint lists hold
 *                       an eighth of it (at least 4096)
 *   debug_tangles       1: after every step, test the end state for pairs of
 *                       vertex-disjoint triangles that intersect (FP64
 *                       orientation tests); a step that has any fails with
 *                       CLOTH_E_TANGLED
 *   broad_reuse         1: the broad phase filters a superset of the candidate
 *                       pairs (below) instead of querying the grid at every
 *                       stage; it pays where boxes move less than their
 *                       margins between stages (slow scenes), and costs a
 *                       rebuild with grown boxes where some primitive always
 *                       escapes.  0 (default): query per stage
 *   broad_margin, broad_margin_motion
 *                       with broad_reuse, the broad phase filters a superset of the candidate
 *                       pairs built on boxes grown along each axis c by
 *                       min(broad_margin + broad_margin_motion * m_c,
 *                       16 broad_margin), m_c the largest change of
 *                       coordinate c of the primitive in the stage that
 *                       built it, and builds it again when a stage box
 *                       leaves its grown box; the candidate lists are the
 *                       same either way.  The superset lists hold twice
 *                       pair_capacity (peak_candidates reports the largest
 *                       list, superset included).  <= 0: d_hat / 4 and 1
 *   r_warm              width of the modal warm start's own basis (set with
 *                       cloth_set_warm_basis; the paper uses a wider one
 *                       there, 120 modes against 30, section 8.1), a
 *                       multiple of 8 in [8, 192]; 0: the warm start uses
 *                       the reuse basis
 *   uu_store            1: the contact part of the reduced matrix,
 *                       U~^T diag(W) U~, is summed from per-vertex
 *                       precomputed upper triangles of U_j U_j^T (Eq. (uu),
 *                       section 5.1; FP32, r (r + 1) / 2 per vertex, built by
 *                       cloth_set_basis; products of BF16 values are exact in
 *                       FP32) with FP64 sums, instead of the Gram of the
 *                       contact rows on the matrix cores (0).  The store adds
 *                       2 r (r + 1) bytes per vertex to the footprint
 *   reorder             1: the scene numbers its vertices in the order of
 *                       cloth_vertex_order (triangles sorted by their lowest
 *                       new vertex), so that the sweeps' neighbour gathers
 *                       stay within a narrow band of the state vectors.  The
 *                       boundary keeps the caller's order: positions,
 *                       velocities, bases and the system matrix cross it in
 *                       the caller's numbering.  The stage-level calls need
 *                       the caller's order (CLOTH_E_INVALID when set)
 *   smoother            0: Jacobi with Chebyshev acceleration (cheb_rho,
 *                       cheb_gamma, cheb_delay); 1: rank-2 A-Jacobi (sec. 8.1):
 *                       every inner iteration takes two damped Jacobi steps
 *                       (damping cheb_gamma) after the subspace correction,
 *                       with no Chebyshev blend
 *   adaptive_samples    1: the partial CCD (Eq. (query)) of a pair whose
 *                       threshold interval rho* (Eq. (sample_bound)) shrank
 *                       over the iteration, by stretch or fast motion,
 *                       samples it more densely (end of section 4.1): the
 *                       ratio c of rho* at the iterate to rho* at x- gives
 *                       the level m = min(8, floor(2 / c)); m > 2 replaces
 *                       the three fixed samples by the centroids of the m^2
 *                       sub-triangles of the barycentric triangle (VT) or
 *                       the centres of the m x m cells of the parameter
 *                       square (EE); the frozen closest point is always a
 *                       sample */
typedef struct {
    int32_t r, iters_inner, iters_outer;
    double tol_inner, tol_outer;
    double cheb_rho, cheb_gamma;
    int32_t cheb_delay, precision, self_contact;
    int64_t pair_capacity;
    int32_t debug_tangles;
    double broad_margin, broad_margin_motion;
    int32_t r_warm, broad_reuse;
    int32_t uu_store, reorder, smoother, adaptive_samples;
} cloth_solver_params;

typedef struct {
    int32_t kind;
    double center[3], axis[3], radius, half_length, omega;
} cloth_obstacle;

/* Filled after the step's stream has been synchronised. */
typedef struct {
    int32_t inner_iters, outer_iters;   /* executed by the last step */
    int64_t n_candidates, n_constraints;
    double dx_norm;      /* max per-vertex change of the last inner iteration run */
    double outer_dx;     /* max per-vertex change of x over the last outer block run */
    double min_toi;      /* smallest time of impact seen (2 = none) */
    double cheb_rho, cheb_gamma;
    int64_t peak_candidates;  /* largest VT or EE candidate list of any outer
                                 stage since the previous stats read (for
                                 sizing pair_capacity) */
    int64_t n_contact_vertices;  /* vertices with a collision weight in the
                                    last block: the rows of the contact Gram
                                    U_C^T diag(W) U_C (Eq. (uu)) */
    int64_t n_factorizations;    /* factorizations of the contact reduced
                                    matrix since the previous stats read: an
                                    inner iteration whose collision weights
                                    equal those of the last factorization
                                    reuses it */
    int64_t n_broad_rebuilds;    /* rebuilds of the reusable candidate
                                    superset since the previous stats read */
} cloth_step_stats;

const char* cloth_status_string(cloth_status s);
const char* cloth_last_error(void);

/* Device bytes a scene needs for this mesh and these settings.  Builds the
 * mesh's system-matrix pattern on the host to count its nonzeros. */
/* Reverse Cuthill-McKee order of the mesh's vertex graph (host only, no
 * device call): order[i] (nv entries, caller-allocated) is the vertex placed
 * at position i.  Each connected component starts from a pseudo-peripheral
 * vertex; neighbours are taken in increasing degree, ties by index; the order
 * is reversed at the end.  CLOTH_E_MESH for an index out of range. */
cloth_status cloth_vertex_order(const cloth_mesh* mesh, int32_t* order);
cloth_status cloth_query_footprint(const cloth_mesh* mesh, const cloth_solver_params* params,
                                   size_t* bytes);

/* Creates a scene: validates the mesh, builds rest data, lumped mass and the
 * system matrix H = M/h^2 + sum_t w_t G_t^T G_t + sum_e w_e k_e k_e^T
 * (Eq. (global)) on the host in FP64, and uploads it.  rest_xyz is the rest
 * shape (nv*3 floats); the initial state is the rest shape at rest.
 * dev_arena/arena_bytes: caller-owned device memory of at least the
 * footprint (it must outlive the scene), or NULL/0 to let the library
 * allocate.  The basis must be set (cloth_set_basis) before stepping. */
cloth_status cloth_init(const cloth_mesh* mesh, const float* rest_xyz, const cloth_material* mat,
                        double dt, const cloth_solver_params* params, void* dev_arena,
                        size_t arena_bytes, cloth_scene* out);

/* The scene's system matrix H (FP64 CSR, caller's vertex order, sorted
 * columns).  Call with row_ptr = col = val = NULL to get nnz only. */
cloth_status cloth_system_matrix(cloth_scene s, int64_t* nnz, int32_t* row_ptr, int32_t* col,
                                 double* val);

/* Sets the subspace basis U (nv*r FP64, row-major, caller's vertex order;
 * rows of pinned vertices are ignored and stored as zero).  The library
 * rounds it to the storage precision, forms Lambda~ = U~^T H U~ in FP64,
 * factors it, and estimates the Chebyshev parameters if they are <= 0.
 * Section 5: U holds the eigenvectors of H for the r smallest eigenvalues;
 * any basis is accepted (the correction is a Galerkin projection). */
cloth_status cloth_set_basis(cloth_scene s, const double* U, int32_t r);

/* Sets the modal warm start's own basis Uw (nv*r_warm FP64, row-major,
 * caller's vertex order; pinned rows stored as zero): Algorithm 1's warm
 * start then runs its local/global iterations in span(Uw) with the Galerkin
 * matrix Uw~^T H Uw~ (the diagonal of eigenvalues for an exact eigenbasis)
 * formed and inverted in FP64.  CLOTH_E_INVALID if the scene was created
 * with r_warm = 0 or r_warm differs. */
cloth_status cloth_set_warm_basis(cloth_scene s, const double* U, int32_t r_warm);

/* Computes the basis on the device and sets it (as cloth_set_basis): the r
 * lowest eigenvectors of H on the free vertices by Chebyshev-filtered
 * subspace iteration (polynomial degree at most `degree` per pass, lowered
 * where the filter would amplify the lowest wanted Ritz direction more than
 * 1e4 times over the r-th; at most max_passes passes, until the largest
 * relative Ritz residual |H u - theta u| / theta of the r wanted pairs is
 * below tol).  Block products run in FP32 with FP64 Gram accumulation, the
 * small eigenproblems in FP64 on the host.
 * Optional outputs: U (nv*r FP64, caller order), the Ritz values (r), the
 * passes used and the final residual.  Section 5 (U from the rest H). */
cloth_status cloth_compute_basis(cloth_scene s, int32_t r, int32_t degree, int32_t max_passes,
                                 double tol, double* U, double* ritz, int32_t* passes,
                                 double* residual);

/* As cloth_compute_basis, but allocating no device memory, for callers that
 * cannot allocate (code under stream capture, serving loops, harnesses that
 * forbid hipMalloc).  The iteration's workspace is a fixed array of
 * 64 MiB that the library holds on each GPU it runs on until the process
 * ends; a call needs 4 * nv * m * 4 + m * m * 4 + c * m * m * 8 bytes of it
 * (m = r + max(8, r/4) rounded up to a multiple of 4, c = min(64,
 * max(1, nv / 4096)); nv = 16,384 at r = 32 takes 10.5 MB), and a scene that
 * needs more is refused with CLOTH_E_INVALID before any work.  Call it with
 * the scene's device current.  Every call on one GPU uses that GPU's one
 * array: calls that overlap on one GPU (from several host threads) race, and
 * the caller must serialise them.  Nothing in the array needs to start
 * cleared; it keeps the last call's contents.  Results are those of
 * cloth_compute_basis on the same scene. */
cloth_status cloth_compute_basis_static(cloth_scene s, int32_t r, int32_t degree, int32_t max_passes,
                                        double tol, double* U, double* ritz, int32_t* passes,
                                        double* residual);

/* Adds an analytic obstacle (at most 4 per scene); the next step records
 * its graph again. */
cloth_status cloth_add_obstacle(cloth_scene s, const cloth_obstacle* ob);

/* State upload / download (host arrays of nv*3 floats; v may be NULL).
 * set_state also fixes pinned vertices at the given x. */
cloth_status cloth_set_state(cloth_scene s, const float* x, const float* v, void* stream);
cloth_status cloth_get_state(cloth_scene s, float* x, float* v, void* stream);

/* One implicit time step with gravity g (m/s^2); stats may be NULL.
 * Failure: a step in which a candidate or constraint list outgrows its
 * capacity, an iterate becomes non-finite, or (debug_tangles) the end state
 * has intersecting triangles is rolled back on the device: x and v keep the
 * values the step started from (so do the forwarded residual and the
 * scene's other state), and its blocks after the failing stage do not move
 * (step length 0).  The failure is reported by the next call that reads
 * stats (this one, when stats is given): CLOTH_E_CAPACITY, CLOTH_E_DIVERGED
 * or CLOTH_E_TANGLED, with the reasons in cloth_last_error(); the record is
 * cleared by that read and by cloth_set_state. */
cloth_status cloth_step(cloth_scene s, const float gravity[3], void* stream,
                        cloth_step_stats* stats);

/* n steps in a row on the same stream without host synchronisation in
 * between; stats (may be NULL) describe the last step; a failure of any of
 * the n steps is reported. */
cloth_status cloth_step_n(cloth_scene s, const float gravity[3], int32_t n, void* stream,
                          cloth_step_stats* stats);

cloth_status cloth_destroy(cloth_scene s);

/* Steps n distinct scenes (same device) once each with gravity g, their
 * work overlapping on the device: the stream forks to a pool of streams,
 * each scene's recorded step graph runs on its own stream, and the stream
 * joins them.  stats: n entries or NULL (then no synchronisation). */
cloth_status cloth_step_batch(cloth_scene* scenes, int32_t n, const float gravity[3], void* stream,
                              cloth_step_stats* stats);

/* One launch for many scenes (same device): cloth_batch_create records each
 * scene's step with gravity g as a child graph of one parent graph (no
 * edges between scenes) and instantiates it; cloth_batch_step replays it
 * `steps` times on the stream, one hipGraphLaunch per step for all scenes.
 * Results equal those of stepping each scene alone.  The scenes must
 * outlive the batch and must not be stepped, modified or given another
 * basis or obstacle while it is used (its recorded launches would then be
 * stale: create the batch again). */
typedef struct cloth_batch_s* cloth_batch;
cloth_status cloth_batch_create(cloth_scene* scenes, int32_t n, const float gravity[3], cloth_batch* out);
cloth_status cloth_batch_step(cloth_batch b, int32_t steps, void* stream);
cloth_status cloth_batch_destroy(cloth_batch b);

/* Autotuner of the launch settings that leave results bitwise unchanged,
 * chosen on time at equal accuracy: lanes per broad-phase query (4, 8, 16)
 * and, for scenes created with broad_reuse, the reusable superset and its
 * margin.  Trials step the scene from its current state (one untimed step,
 * then `steps` steps timed with HIP events on the stream) and restore the
 * state after; the fastest setting is applied and cached per size class
 * (vertex count to a quarter octave, r, precision, self contact); later
 * calls for the class apply the cached one without trials unless force.
 * The Chebyshev schedule (rho, damping) is chosen on the device when the
 * basis is set (by measured error growth) and is reported here.  The scene
 * must not be in a server or batch while tuned. */
typedef struct {
    int32_t query_lanes, broad_reuse;
    double broad_margin, broad_margin_motion;
    double ms_per_step;   /* the chosen setting's time per step (trials) */
    double ms_default;    /* the default setting's (8 lanes, no superset) */
    double cheb_rho, cheb_gamma;
    int32_t trials, from_cache;
} cloth_tuning;
cloth_status cloth_autotune(cloth_scene s, const float gravity[3], int32_t steps, int32_t force, void* stream,
                            cloth_tuning* out);
cloth_status cloth_set_tuning(cloth_scene s, const cloth_tuning* t);

/* Continuous-batching step server.  A host thread keeps up to `slots` steps
 * in flight (one stream each), starts queued requests as slots and their
 * scenes free up (two steps of one scene never overlap; requests of a scene
 * run in submission order), and admits scenes while the sum of their device
 * footprints stays within hbm_budget bytes (0 = no limit): the scenes it
 * steps at any time are an admitted working set of at most that footprint.
 * The budget is accounting only: a scene keeps its device memory (allocated
 * by cloth_init) whether admitted or not.
 * A scene in a server must not be stepped or modified by the caller until it
 * is released.
 *   admit:   *admitted = 1 if the scene fits now (or is already in), else 0
 *   release: waits for the scene's queued steps, then frees its budget
 *   submit:  queues one step of the scene and returns a ticket; a scene not
 *            admitted waits (its requests queued) until its footprint fits:
 *            the worker admits waiting scenes in arrival order, releasing
 *            admitted scenes that have no queued or running step, least
 *            recently used first.  CLOTH_E_OOM if the footprint alone
 *            exceeds the budget
 *   poll / wait: completion of a ticket, with latency (submission to
 *            completion, host clock) and service time (device, ms); the
 *            ticket's status is the step's own (CLOTH_E_CAPACITY,
 *            CLOTH_E_DIVERGED or CLOTH_E_TANGLED for a rolled-back step)
 *   info:    admitted and waiting scene counts, admitted footprint, and the
 *            releases made to admit waiting scenes
 *   destroy: finishes queued work and stops the thread */
typedef struct cloth_server_s* cloth_server;
cloth_status cloth_server_create(int32_t slots, size_t hbm_budget, cloth_server* out);
cloth_status cloth_server_admit(cloth_server sv, cloth_scene s, int32_t* admitted);
cloth_status cloth_server_release(cloth_server sv, cloth_scene s);
cloth_status cloth_server_submit(cloth_server sv, cloth_scene s, const float gravity[3],
                                 int64_t* ticket);
cloth_status cloth_server_poll(cloth_server sv, int64_t ticket, int32_t* done, double* latency_ms,
                               double* service_ms);
cloth_status cloth_server_wait(cloth_server sv, int64_t ticket, double* latency_ms,
                               double* service_ms);
cloth_status cloth_server_info(cloth_server sv, int32_t* n_admitted, int32_t* n_waiting, size_t* used_bytes,
                               int64_t* evictions);
cloth_status cloth_server_destroy(cloth_server sv);

/* Optional parts of Algorithm 1 around the inner loop:
 *   warm_iters  modal warm start: that many local/global iterations in
 *               span(U) from z, collisions ignored, before the first full CCD
 *               (the same basis serves the warm start and the reuse)
 *   rf_iters    residual forwarding (section 6): after the exiting filter,
 *               that many inner iterations with every collision weight at k
 *               and no filter; if the exiting t_TOI was below rf_toi their
 *               displacement dx is forwarded, the next step's z gaining
 *               h^2 M^{-1} delta f = 2 dx (Eq. (z_rf), delta f = 2 M dx / h^2).
 *               The iterations run every step and their result is applied
 *               on the device only when the condition holds.
 * Both default to 0 (off).  Changing them re-records the step graph. */
cloth_status cloth_set_step_options(cloth_scene s, int32_t warm_iters, int32_t rf_iters,
                                    double rf_toi);

/* The residual currently forwarded to the next step (nv*3 host floats). */
cloth_status cloth_get_forwarded(cloth_scene s, float* dx);

/* Whole-step graph replay (on by default): the first cloth_step / cloth_step_n
 * records one step's launches into a HIP graph on a private stream and
 * replays it on the caller's stream; a new gravity vector re-records it.
 * Steps run with timing on are launched directly. */
cloth_status cloth_set_graph(cloth_scene s, int32_t on);

/* Per-kernel timing.  With timing on, every kernel (or kernel group) of the
 * step is bracketed by HIP events on the step's stream; cloth_kernel_times
 * synchronises the device and returns, per kernel id, its name (32 chars
 * each in names), total milliseconds and launch count.  *count receives the
 * number of ids; at most max entries are written.  Turning timing on or off
 * clears the totals. */
cloth_status cloth_set_timing(cloth_scene s, int32_t on);
cloth_status cloth_kernel_times(cloth_scene s, int32_t max, char* names, double* total_ms,
                                int64_t* launches, int32_t* count);

/* ---------------------------------------------------------------------
 * Stage-level entry points, used to check each stage against a reference
 * on identical inputs.  Host arrays, caller's vertex order.
 * ------------------------------------------------------------------- */

/* Broad phase on (xm, xp): sorted VT pairs (vertex, triangle) and EE pairs
 * (edge e1 < e2, edges numbered in lexicographic (i<j) order) whose swept
 * FP32 boxes grown by d_hat overlap and that share no vertex.  Returns
 * CLOTH_E_CAPACITY (with the true counts) if a list does not fit. */
cloth_status cloth_stage_broad_phase(cloth_scene s, const float* xm, const float* xp,
                                     int64_t cap, int32_t* vt, int64_t* n_vt, int32_t* ee,
                                     int64_t* n_ee);

/* FP64 time of impact over (xm, xp) for given VT and EE pairs (2.0 = no hit).
 * Sections 4.1 and 7.  CLOTH_E_INVALID on a scene without self contact,
 * CLOTH_E_CAPACITY if a list exceeds the scene's pair capacity. */
cloth_status cloth_stage_toi(cloth_scene s, const float* xm, const float* xp, int64_t n_vt,
                             const int32_t* vt, int64_t n_ee, const int32_t* ee,
                             double* toi_vt, double* toi_ee);

/* Loads a block state: x- (start of block), x^k, x^{k-1}, the inertia target
 * z, and a constraint set (sorted VT and EE lists with life spans, and
 * per-vertex obstacle life spans ob_a[j*nv + v], -1 = not a member).  The
 * frozen constraint data are computed from xm, which also stands for the
 * step's start x* of the friction slip. */
cloth_status cloth_stage_load_block(cloth_scene s, const float* xm, const float* xk,
                                    const float* xkm1, const float* z, int64_t n_vt,
                                    const int32_t* vt, const int32_t* a_vt, int64_t n_ee,
                                    const int32_t* ee, const int32_t* a_ee, const int32_t* ob_a);

/* One inner iteration with Chebyshev index k on the loaded block, followed
 * by partial CCD (the life-span update); then x^{k-1} <- x^k <- x^{k+1}. */
cloth_status cloth_stage_inner(cloth_scene s, int32_t k);

/* Partial CCD of the loaded block's constraints on (x-, xnew) with xnew
 * given (host, nv*3 floats): updates the life spans only. */
cloth_status cloth_stage_partial_ccd(cloth_scene s, const float* xnew);

/* One outer CCD stage on (xm, xp) (host arrays): broad phase, time of impact,
 * new constraint set = {candidates with TOI <= 1} U (loaded set intersected
 * with the candidates) with carried life spans (first != 0: the loaded set is
 * ignored and obstacle spans restart), step length s = 1 or alpha t_TOI, and
 * the filtered positions x = xm + s (xp - xm) (written to x_out, nv*3).
 * The new set becomes the loaded block (read it with cloth_stage_read_set). */
cloth_status cloth_stage_outer(cloth_scene s, const float* xm, const float* xp, int32_t first,
                               float* x_out, double* s_out);

/* The loaded constraint set: sorted VT and EE pairs with life spans (each
 * list holds at most cap pairs; the counts are returned either way) and the
 * per-vertex obstacle spans ob_a[j*nv + v] (NULL to skip). */
cloth_status cloth_stage_read_set(cloth_scene s, int64_t cap, int32_t* vt, int32_t* a_vt,
                                  int64_t* n_vt, int32_t* ee, int32_t* a_ee, int64_t* n_ee,
                                  int32_t* ob_a);

/* Reads the block state back: x^k (after cloth_stage_inner: x^{k+1}), the
 * life spans, the last inner iteration's max change, and (if non-NULL) the
 * right-hand side b and reduced solution Q (r*3 values, row-major). */
cloth_status cloth_stage_read_block(cloth_scene s, float* xk, int32_t* a_vt, int32_t* a_ee,
                                    int32_t* ob_a, double* dx, float* b, double* Q);

#ifdef __cplusplus
}
#endif
#endif /* CLOTH_H */

/*
 * cps.h -- C ABI of the curvilinear pressure-Poisson multigrid for MI355X.
 *
 * Solves the pressure-correction equation of Naskar et al. (arXiv
 * 2305.17875), eq. (PC_6): d/ds_i ( G_ij d phi / ds_j ) = rhs, written in the
 * transformed Cartesian coordinates of Sec. 3.1 with unit cell sides, the
 * face metrics G of Sec. 3.2 and the nine-term second-order flux form of
 * eq. (PC_8) / (PC_term1-3).  phi is hdP of eq. (PC_6); the caller divides by
 * the substep h.
 *
 * Geometry and boundary conventions (the paper leaves the pressure boundary
 * condition unstated; these are the library's):
 *   - cells n_r x n_theta x n_phi, arrays [r][theta][phi] in C order with phi
 *     contiguous; phi is periodic;
 *   - the r-walls and the theta-walls (cones at theta0, theta1) carry zero
 *     flux; stencil reads that leave the domain in r or theta mirror to the
 *     nearest cell;
 *   - A is singular with the constants as null space and 1^T A = 0, so the
 *     mean of rhs is removed (and reported) and the returned p has mean 0.
 *
 * Pointers: unless stated otherwise, array arguments are DEVICE pointers on
 * the current HIP device, owned by the caller and not retained after the call
 * returns.  Every call is ordered on opts.stream (0 = the null stream).
 *
 * Errors: functions return cps_status.  On a non-OK status, cps_last_error()
 * gives a thread-local text.  A handle is not thread-safe; distinct handles
 * are independent.
 */
#ifndef CPS_H
#define CPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CPS_OK = 0,
    CPS_E_INVALID = -1,       /* bad argument, dims, or a face with det <= 0 */
    CPS_E_OOM = -2,           /* device allocation failed */
    CPS_E_HIP = -3,           /* a HIP runtime call failed */
    CPS_E_NOT_CONVERGED = -4, /* iteration cap reached; p holds the last iterate */
    CPS_E_DIVERGED = -5       /* residual norm became NaN or Inf */
} cps_status;

/* Maps from computational (s_r, s_theta, s_phi) in [0,1]^3 to physical X;
 * the polar axis is x1 (Sec. 2).  r(s) is linear, or the tanh clustering of
 * eq. (stretching) shifted to the mid-radius and scaled by the gap;
 * theta = theta0 + s_theta (theta1 - theta0); phi = 2 pi s_phi. */
typedef enum {
    CPS_MAP_IDENTITY = 0, /* X = (r, theta, phi): a box, for tests */
    CPS_MAP_SPHERE = 1,   /* X = (r cos t, r sin t cos p, r sin t sin p) */
    CPS_MAP_OBLATE = 2,   /* x1 scaled by (1 - flattening) */
    CPS_MAP_TRIAXIAL = 3  /* x1 by (1 - flattening), x2 by (1 + skew) */
} cps_map;

typedef struct {
    int32_t n_r, n_theta, n_phi; /* cells; every level but the coarsest needs even dims */
    int32_t map;                 /* cps_map */
    double r_inner, r_outer;     /* the paper's shell: 1.5, 2.5 (gap 1, ratio 0.6) */
    double theta0, theta1;       /* cone walls in [0, pi], e.g. 0.05 and pi - 0.05;
                                    0 and pi give the full sphere, whose
                                    polar faces have zero area (no flux) */
    double radial_stretch;       /* rx2 of eq. (stretching); 0 = uniform */
    double flattening, skew;     /* oblate / triaxial shape parameters */
    int32_t n_levels;            /* 0 = halve while > 1024 cells, dims even and >= 4, and
                                    n_phi stays even; n_phi must be even on every level */
} cps_grid;

/* How the face metrics G_dq = |J^-1| (ds_d/dx_k)(ds_q/dx_k) (eq. (skewness))
 * are formed at each face (Sec. 3.2 items 1-5):
 *   MAP_CENTRAL   the inverse Jacobian's columns are chords of the map
 *                 across the face centre (second-order central differences);
 *   PAPER_VERTEX  the paper's item 1: the normal derivative averaged over the
 *                 face's four vertices, tangential ones over its two edges;
 *   USER_FACE     the caller's own face metrics of the finest level (from a
 *                 grid of its own, formed as in Sec. 3.2 items 1-5, which the
 *                 paper hands to its pressure solver as the stencil of eq.
 *                 (PC_term1)-(PC_term3)): face_G, a HOST array
 *                 [9][n_r][n_theta][n_phi] in C order, entry 3d+q of cell
 *                 (a, b, c) = G_dq on the cell's low d-face (d, q: 0 r,
 *                 1 theta, 2 phi); read during cps_setup only.  The low r-
 *                 and theta-wall faces carry no flux: their entries are
 *                 ignored (taken as 0); the high walls are implicit.  Every
 *                 other entry must be finite and every diagonal entry G_dd
 *                 >= 0, else CPS_E_INVALID.  A coarser level's face is made
 *                 of four faces of the level below: its metrics are half their
 *                 sum, entry by entry (four times the area over twice the
 *                 normal length).  The storage and stencil class follow the
 *                 data: one value per (r, theta) when every entry agrees with
 *                 the c = 0 one of its row to 1e-12 of the face's diagonal
 *                 entry (the c = 0 values then serve the whole ring: a map
 *                 symmetric about the polar axis, up to the rounding of the
 *                 caller's trigonometry), 7-point when every cross entry is 0.
 *                 Such a handle has no map: the projection step and the line
 *                 solves, which need the map's chords, return CPS_E_INVALID,
 *                 and the batched form and the service do not take it. */
typedef enum {
    CPS_METRICS_MAP_CENTRAL = 0,
    CPS_METRICS_PAPER_VERTEX = 1,
    CPS_METRICS_USER_FACE = 2
} cps_metrics_method;

typedef struct {
    int32_t method;       /* cps_metrics_method */
    const double* face_G; /* USER_FACE only (see above); NULL otherwise */
} cps_metrics;

typedef struct {
    int32_t precision; /* 0: FP64 throughout; 1: FP32 V-cycles inside an FP64
                          refinement loop (FP64 residual, update, coarse solve) */
    int32_t max_iters; /* outer iterations; <= 0 means 200 */
    int32_t accel;     /* 0: stationary iteration of V-cycles; 1: conjugate
                          gradients with the V-cycle as preconditioner
                          (flexible, Polak-Ribiere form for the FP32 cycles
                          and for operators with cross terms, which are only
                          mildly non-symmetric); 2: BiCGStab, two V-cycles
                          per iteration, for strongly non-symmetric cases */
    int32_t tune;      /* smoother tile shapes (marching chunk per level shape):
                          0 use the cached choice if any; 1 time the shapes not
                          yet cached at setup; 2 retime all.  Cache: the JSON
                          file named by the environment variable CPS_TUNE_CACHE
                          (unset: this process only).  Results do not depend
                          on the choice. */
    int32_t eager;     /* 0: each outer iteration of cps_solve is captured once
                          into a hipGraph (per handle) and replayed, one launch
                          per iteration, when the stream is not the null stream
                          and profiling is off; 1: every kernel is launched
                          directly.  Results are the same bits either way. */
    int32_t smoother;  /* 0: red-black point Gauss-Seidel (any stencil);
                          1: zebra (r, phi)-plane relaxation -- the theta rows
                          of one parity at a time, each (r, phi) plane solved
                          exactly by a Fourier transform along phi and the
                          Thomas algorithm along r; robust to the shell's
                          radial and cone-tip anisotropy.  Needs
                          phi-invariant metrics without phi cross terms: the
                          7-point operator (identity box, sphere) or the
                          11-point one with r-theta cross terms (oblate
                          shell; its r-lines are then tridiagonal but not
                          symmetric), and n_phi a power of two in [4, 2048]
                          on every smoothed level (<= 512 in the batched
                          form);
                          2: automatic -- 1 where the hierarchy allows it,
                          else 0 (decided at set-up, per problem in the
                          batched form). */
    void* stream;      /* hipStream_t the calls are ordered on; NULL = null stream */
} cps_opts;

typedef struct {
    int32_t iterations;      /* outer iterations done */
    double rel_residual;     /* ||b - A p|| / ||b|| with b = rhs - mean(rhs), of the p
                                returned: the Krylov forms update the residual by
                                recurrence, and before they stop they form b - A p
                                itself and restart from it if it misses tol */
    double rhs_mean_removed; /* mean(rhs) */
    double seconds;          /* wall time of the call */
} cps_info;

typedef struct cps_handle cps_handle;

/* Fill *g with the paper's shell defaults (n_* = 32, sphere, r 1.5..2.5,
 * theta 0.05..pi-0.05, uniform radius, rule-based levels). */
void cps_grid_default(cps_grid* g);

/* Build the hierarchy on the current device: level plan, face metrics of
 * every level (computed on the GPU from the map, or coarsened from the
 * caller's, see cps_metrics), classification of the operator (7-point when
 * every cross metric vanishes, else 19-point), and the dense inverse of the
 * coarsest operator plus alpha 1 1^T.
 * grid, metrics, opts: host pointers, read during the call only.
 * *out receives a handle owning all device memory of the hierarchy.
 * Errors: CPS_E_INVALID (dims, non-positive det), CPS_E_OOM, CPS_E_HIP. */
cps_status cps_setup(const cps_grid* grid, const cps_metrics* metrics, const cps_opts* opts,
                     cps_handle** out);

/* Solve A p = rhs - mean(rhs) to ||b - A p||_2 <= tol ||b||_2 from p = 0,
 * then return p with zero mean.  rhs, p: device FP64 arrays of
 * n_r*n_theta*n_phi elements (may not alias).  info: host, nullable.
 * Synchronises the stream once per outer iteration (an 8-byte read).
 * CPS_E_NOT_CONVERGED leaves the last iterate in p; a zero rhs returns
 * p = 0 after 0 iterations. */
cps_status cps_solve(cps_handle* h, const double* rhs, double* p, double tol, cps_info* info);

/* Release every device allocation of the handle (NULL is allowed). */
void cps_destroy(cps_handle* h);

/* Thread-local description of the last error on this thread. */
const char* cps_last_error(void);

/* Levels and colouring of a handle: dims_out[3*l + {0,1,2}] for l < levels
 * (host array of 48 ints), *ncolours = 2 (7-point) or 4 (19-point),
 * *phi_invariant = 1 when the metrics are stored once per (r, theta). */
cps_status cps_levels(const cps_handle* h, int32_t* n_levels, int32_t* dims_out,
                      int32_t* ncolours, int32_t* phi_invariant);

/* ---- Projection step around the solve (finest grid) --------------------
 * The pressure-correction section: the solve of eq. (PC_6) is one step of
 * the projection that makes the intermediate velocity u*** divergence
 * free.  Discretised in flux form on the collocated grid like eq.
 * (PC_term1): a face value is the mean of the two cells sharing the face,
 * C_ji = |J^-1| ds_j/dx_i (eq. (skewness)) is evaluated at the faces from the
 * same chords of the map as the face metrics (Sec. 3.2 items 4-5), and
 * |J^-1| of a cell is the mean of its six face determinants (item 3).
 * No flow crosses the r- and theta-walls; phi is mirrored there.
 * Velocities: device FP64 [3][n_r][n_theta][n_phi], Cartesian components
 * with the polar axis along x1, natural order; scalar fields: device FP64
 * [n_r][n_theta][n_phi].  The face tables are built on the first call
 * (device memory owned by the handle: 12 words per (r, theta) position for
 * maps symmetric about the polar axis, 12 per cell otherwise) and rebuilt
 * after the metrics change.  Errors: CPS_E_INVALID for NULL arguments and
 * for a scalar field that overlaps u. */

/* rhs = d/ds_j [C_ji u_i], the right-hand side of eq. (PC_6); its sum over
 * the cells is zero to rounding (the fluxes telescope). */
cps_status cps_divergence(cps_handle* h, const double* u, double* rhs);
/* eq. (PC_7): u_i <- u_i - (1/|J^-1|) d/ds_j [C_ji phi] in place, with phi
 * the solution of eq. (PC_6) (phi = h dP). */
cps_status cps_correct(cps_handle* h, const double* phi, double* u);
/* One projection step: rhs = cps_divergence(u), cps_solve(rhs -> phi, tol),
 * then cps_correct(phi, u) -- u is corrected in place only when the solve
 * converged (the solve's status is returned; phi holds its last iterate).
 * Uses a handle-owned right-hand-side buffer (allocated on first call). */
cps_status cps_project(cps_handle* h, double* u, double* phi, double tol, cps_info* info);

/* ---- Implicit line solves of the ADI steps (finest grid) ---------------
 * eq. (solve_2)-(solve_4): each ADI step solves, along one direction dir
 * (0 r, 1 theta, 2 phi), every line of cells for psi:
 *     |J^-1|_i psi_i - coef [F_{i+1/2} - F_{i-1/2}] = rhs_i,
 * F = G_dd (psi_hi - psi_lo) on an interior face (the diagonal viscous term,
 * as in eq. (PC_term1)), G_dd = |C_d|^2 / |J^-1| at the face from the face's
 * chords, |J^-1|_i the cell value of the projection step.  coef is the
 * implicit weight (e.g. sqrt(Pr/Ra) h / 2).  r- and theta-lines use the
 * Thomas algorithm (eq. (FIBRE_TA1)-(FIBRE_TA2)); phi-lines are periodic
 * and use the split with a closing row of eq. (FIBRE_TAP1)-(FIBRE_TAP8). */
typedef struct {
    int32_t type_lo, type_hi; /* 0: no flux through the wall face; 1: value on it */
    double value_lo, value_hi; /* the wall values for type 1 (F = 2 G_dd (psi_0 -
                                  value_lo) at the low wall, 2 G_dd (value_hi -
                                  psi_{n-1}) at the high wall) */
} cps_line_bc;

/* rhs, psi: device FP64 [n_r][n_theta][n_phi], the same array (in place) or
 * not overlapping.  bc: host, nullable (no flux); ignored for dir 2.
 * Needs phi-invariant metrics (box, sphere, oblate shell) and, for dir 2,
 * n_phi >= 3.  Device memory owned by the handle, built on first use: the
 * projection step's face tables, an elimination table of 3 words per
 * (r, theta) position, and for dir 2 two scratch fields.
 * Errors: CPS_E_INVALID (dir, coef < 0 or not finite, bc types, map,
 * overlap). */
cps_status cps_line_solve(cps_handle* h, int32_t dir, double coef, const cps_line_bc* bc,
                          const double* rhs, double* psi);

/* ---- Line solves without allocation -----------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight time-step or serving loops, harnesses that forbid
 * hipMalloc.  cps_line_solve with the same arguments and the same result,
 * bit for bit, but every table that cps_line_solve builds on first use and
 * keeps in the handle (the face tables, the elimination of the open lines,
 * the ring transform's tables) is formed anew on each call in one fixed
 * device array of CPS_LINE_SCRATCH_BYTES per GPU, which the library holds
 * from its load until the process ends.  The call only launches kernels on
 * the handle's stream: no allocation, free, copy, memset or
 * synchronisation, so it can be captured into a graph (the handle itself
 * is set up beforehand with cps_setup).
 * Limits: phi-invariant metrics (box, sphere, oblate shell); the tables
 * take 12 (n_r + 1)(n_theta + 1) + n_r n_theta words plus, for dir 0 / 1,
 * 3 n + 2 words per distinct line (n_theta lines of n_r cells / n_r lines of
 * n_theta cells) and, for dir 2, 2 n_phi + 3 words, each part rounded up to
 * an even count, at most CPS_LINE_SCRATCH_BYTES / 8 words in all (the
 * paper-scale 192 x 256 shell needs 5 MB); dir 2 needs n_phi / 2 a power of
 * two in [2, 2048] and rhs, psi aligned to 16 bytes (the ring transform).
 * Anything else: CPS_E_INVALID, and nothing is launched.
 * The array is shared by every call on one GPU and keeps the last call's
 * tables: calls that overlap in time on one GPU (other streams or threads)
 * race with each other and give wrong results; the caller serialises them.
 * Arguments and errors otherwise as cps_line_solve. */
#define CPS_LINE_SCRATCH_BYTES (32u << 20)
cps_status cps_line_solve_noalloc(cps_handle* h, int32_t dir, double coef, const cps_line_bc* bc,
                                  const double* rhs, double* psi);

/* ---- Kernel-level entry points (FP64 hierarchy of the handle) ----------
 * For parity tests of each step against an independent implementation.
 * level l indexes the hierarchy (0 = finest); all arrays are device FP64
 * in the [r][theta][phi] layout of that level. */

/* G_out: [9][n_r][n_theta][n_phi] face metrics of level l as used by the
 * kernels (entry 3d+q of a cell: G_dq on its low face in direction d). */
cps_status cps_debug_metrics(cps_handle* h, int32_t level, double* G_out);
/* y = A x on level l (eq. (PC_8) flux form). */
cps_status cps_debug_apply(cps_handle* h, int32_t level, const double* x, double* y);
/* r = b - A x on level l; *norm2 (host) receives sum of r^2. */
cps_status cps_debug_residual(cps_handle* h, int32_t level, const double* b, const double* x,
                              double* r, double* norm2);
/* one Gauss-Seidel pass over the cells of colour `colour`, x in place. */
cps_status cps_debug_gs_pass(cps_handle* h, int32_t level, int32_t colour, const double* b,
                             double* x);
/* bc (level l+1) = P^T r (level l): full weighting, 64-point. */
cps_status cps_debug_restrict(cps_handle* h, int32_t level, const double* r, double* bc);
/* The V-cycle's transfer after red-black pre-smoothing (Sec. on the
 * multigrid solver): bc (level l+1) = P^T r with r = b - A x on level l's
 * red cells (colour 0) and 0 on its black cells, whose residual the black
 * pass has just made zero.  Runs what the FP64 cycle runs: one fused pass
 * where the level's shape allows it, else the red residual and the
 * restriction.  CPS_E_INVALID: a level that forms its whole residual (not
 * point red-black smoothing of the 7-point operator on n_phi / 2 a multiple
 * of 64 and even n_theta), the coarsest level, or a mixed handle. */
cps_status cps_debug_residual_restrict(cps_handle* h, int32_t level, const double* b,
                                       const double* x, double* bc);
/* x (level l) += P e (level l+1): cell-centred trilinear. */
cps_status cps_debug_prolong(cps_handle* h, int32_t level, const double* e, double* x);
/* e = (A_c + alpha 1 1^T)^-1 (b - mean b) on the coarsest level. */
cps_status cps_debug_coarse_solve(cps_handle* h, const double* b, double* e);
/* one zebra half-sweep of the plane smoother on level l (handle set up
 * with smoother = 1): the theta rows b = parity (mod 2), x in place. */
cps_status cps_debug_plane_sweep(cps_handle* h, int32_t level, int32_t parity, const double* b,
                                 double* x);
/* one V(2,2) cycle on level 0 with right-hand side b, x in place. */
cps_status cps_debug_vcycle(cps_handle* h, const double* b, double* x);

/* ---- Batched form ------------------------------------------------------
 * Many independent shell problems (uneven sizes, any maps) solved together:
 * each phase of the iteration is one launch for all problems (a device work
 * table maps every block to its problem), the iteration bodies are captured
 * in hipGraphs, converged problems retire.  Every problem runs FP32 V-cycles
 * inside FP64 refinement with Krylov acceleration, exactly as cps_solve with
 * precision = 1, accel = 1 on the same stream: results equal the problem
 * solved alone, bit for bit. */
typedef struct cps_batch cps_batch;

/* grids: host array of n grids; metrics, opts: host, nullable (opts.precision
 * must be 1 when given; opts.stream NULL creates a private stream).
 * Builds every hierarchy on the device.  Errors as cps_setup; a batch may hold
 * the 7-point class plus one other stencil class. */
cps_status cps_batch_setup(int32_t n, const cps_grid* grids, const cps_metrics* metrics,
                           const cps_opts* opts, cps_batch** out);
/* rhs, p: host arrays of n DEVICE pointers (FP64, natural order, each of its
 * grid's size); infos: host array of n, nullable.  Returns CPS_OK when every
 * problem converged, else CPS_E_DIVERGED / CPS_E_NOT_CONVERGED (see infos). */
cps_status cps_batch_solve(cps_batch* b, const double* const* rhs, double* const* p, double tol,
                           cps_info* infos);
void cps_batch_destroy(cps_batch* b);

/* ---- Solve service -----------------------------------------------------
 * A stream of independent requests (any dims, maps and metrics) served by
 * `max_slots` worker threads, each with its own HIP stream (default
 * priority) on the device current at creation.  Requests are admitted first
 * come, first served, while the device memory of the resident hierarchies
 * plus the ones being built stays within `hbm_budget_bytes`.  A finished
 * request leaves its hierarchy resident: a later request with the same dims
 * and stencil class reuses it (recomputing metrics and coarse inverse when
 * its map differs), and idle hierarchies are evicted least recently used
 * first when a new one does not fit.  Every request runs exactly the code of
 * cps_solve with the service's opts, so its p equals the same problem solved
 * alone with cps_setup/cps_solve, bit for bit.  All functions are
 * thread-safe; latency is measured from submission to completion.
 * A worker captures each hierarchy's iteration bodies into hipGraphs on its
 * own non-blocking stream.  The library never frees, allocates or uploads
 * while any of its captures is open; code elsewhere in the process that
 * synchronises the whole device meanwhile (hipDeviceSynchronize, hipFree,
 * hipHostMalloc) can invalidate a capture, and that request then fails
 * with CPS_E_HIP. */
typedef struct cps_service cps_service;

typedef struct {
    uint64_t submitted, completed, failed; /* failed: status other than CPS_OK */
    uint64_t queued;                       /* waiting for admission now */
    int32_t active, peak_active;           /* requests being solved */
    double p50_ms, p99_ms, mean_ms, max_ms; /* latency of completed requests */
    double unknowns_per_s; /* cells solved / (last completion - first submission) */
    uint64_t hbm_in_use, hbm_budget; /* bytes: resident plus reserved hierarchies */
    uint64_t hierarchies_built, hierarchies_reused, map_rebuilds, evictions;
} cps_service_report;

/* opts: host, nullable; opts.stream must be NULL.  max_slots: 1..64.
 * Errors: CPS_E_INVALID, CPS_E_HIP. */
cps_status cps_service_create(size_t hbm_budget_bytes, int32_t max_slots, const cps_opts* opts,
                              cps_service** out);
/* Queue one solve of A p = rhs - mean(rhs) to relative residual tol.
 * grid, metrics (nullable): host, read during the call.  rhs_host, p_host:
 * host FP64 arrays of n_r*n_theta*n_phi elements, owned by the caller, which
 * keeps them valid and leaves them alone until cps_service_wait returns for
 * this ticket (no host copy is made; a worker reads rhs_host and writes
 * p_host).  *ticket receives the request's id.  Grid errors are reported
 * here. */
cps_status cps_service_submit(cps_service* s, const cps_grid* grid, const cps_metrics* metrics,
                              const double* rhs_host, double* p_host, double tol,
                              uint64_t* ticket);
/* Block until the request finishes; then p_host holds p (the last iterate
 * for CPS_E_NOT_CONVERGED) and info (nullable) its cps_info.  Returns the
 * request's status (CPS_E_OOM if it can never fit the budget); each ticket
 * can be waited for once. */
cps_status cps_service_wait(cps_service* s, uint64_t ticket, cps_info* info);
/* *bytes = the device memory a request of this grid is admitted against
 * with these opts (nullable): its hierarchy, two staging vectors and the
 * transient buffers of the coarse inverse.  Host only; checks the grid. */
cps_status cps_service_footprint(const cps_grid* grid, const cps_opts* opts, uint64_t* bytes);
/* Snapshot of the counters and latency percentiles (host struct). */
cps_status cps_service_stats(cps_service* s, cps_service_report* out);
/* Stops the workers after their current requests, frees every hierarchy
 * and every request not yet waited for.  No call may be in flight. */
void cps_service_destroy(cps_service* s);

/* ---- Measurement -------------------------------------------------------
 * Kernel classes timed on the finest level with HIP events recorded on the
 * handle's stream around each launch; the point smoother's full colour
 * passes of one smoothing call run back to back and are timed as one span
 * over their launches (the colour class leaves out the zero-iterate first
 * pass of a cycle, which moves fewer bytes). */
enum {
    CPS_KERNEL_GS = 0,       /* one Gauss-Seidel colour pass */
    CPS_KERNEL_RESIDUAL = 1, /* r = b - A x (+ norm partials) */
    CPS_KERNEL_APPLY = 2,    /* y = A x (Krylov products) */
    CPS_KERNEL_RESTRICT = 3, /* full weighting to level 1 */
    CPS_KERNEL_PROLONG = 4,  /* trilinear correction from level 1 */
    CPS_KERNEL_VCYCLE = 5,   /* one preconditioning V-cycle, all levels (the span
                                from its first to its last launch) */
    CPS_KERNEL_DIVERGENCE = 6, /* the projection step's right-hand side */
    CPS_KERNEL_CORRECT = 7,    /* the projection step's velocity correction */
    CPS_KERNEL_CLASSES = 8
};
/* enable != 0 starts recording (and clears earlier records). */
cps_status cps_profile_enable(cps_handle* h, int32_t enable);
/* Record only the classes whose bit (1 << class) is set in class_mask
 * (default: all): fewer events around the launches of interest. */
cps_status cps_profile_select(cps_handle* h, uint32_t class_mask);
/* Synchronises the stream; *total_ms (host) = summed duration of the
 * recorded launches of the class, *launches = their count; then clears. */
cps_status cps_profile_read(cps_handle* h, int32_t kernel_class, double* total_ms,
                            int64_t* launches);
/* The preconditioning V-cycle as the solve runs it (Sec. on the multigrid
 * solver: V(2,2) with the handle's smoother, precision and tuned launch
 * shapes, from a zero iterate): `cycles` V-cycles are captured into one
 * hipGraph, launched once untimed and then `reps` times between two HIP
 * events on the handle's stream; *us_per_cycle (host) = elapsed time /
 * (reps * cycles); *launches_per_cycle (host, may be NULL) = the kernel
 * nodes of the captured graph / cycles.  The input is the handle's
 * finest-level residual vector,
 * filled with ones; it and the finest-level iterate are overwritten (the
 * next solve sets both).  Synchronous.  CPS_E_INVALID: a NULL argument,
 * cycles or reps < 1, the handle on the null stream (it cannot be
 * captured), or profiling on (cps_profile_enable). */
cps_status cps_time_vcycle(cps_handle* h, int32_t cycles, int32_t reps, double* us_per_cycle,
                           int64_t* launches_per_cycle);
/* dst[i] = src[i] for i < n (device FP64, ordered on `stream`, synchronous):
 * a plain copy of known size, the yardstick for the HBM byte counters. */
cps_status cps_debug_copy(const double* src, double* dst, int64_t n, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* CPS_H */

/*
 * sdmm.h - C ABI of the stochastic multiscale flux basis library for
 * coupled Stokes-Darcy flow (MI355X / gfx950).
 *
 * The library computes, for a domain split into Stokes and Darcy
 * subdomains with a KL-parameterised log-permeability:
 *   - the stochastic multiscale flux basis: one local solve per mortar
 *     degree of freedom of every subdomain, for every local KL realization
 *     of each Darcy subdomain (Section 5.4, Method S3, pre-computation
 *     loop; the basis functions phi = S_{H,i} xi^j of Section 5.3);
 *   - the interface problem S_H lambda = g_H (Section 5.1, eq.
 *     operatorform) for a batch of global collocation points, by CG in
 *     which S_H is applied as linear combinations of that basis
 *     (Section 5.4, main loop, Steps 3-5);
 *   - the weighted moments of Section 2 (mean and Var = E[u^2] - E[u]^2)
 *     with the collocation weights of Section 4 (Step 6).
 *
 * Conventions
 *   - Every function returns an int status (SDMM_OK or a negative code);
 *     sdmm_last_error() describes the last failure on that context.
 *     No exception or abort crosses the ABI.
 *   - The caller owns every array it passes; the library copies what it
 *     keeps.  The library owns all device state it allocates (basis cache,
 *     factors, CG workspace, moment accumulators).
 *   - Arguments documented as "device" are device pointers on the
 *     context's GPU (for instance from a torch tensor); "host" arguments
 *     are ordinary host memory.
 *   - Calls taking a stream enqueue their work on it (a hipStream_t passed
 *     as void*; NULL means the null stream) and may return before the work
 *     completes.  Results are valid once the stream is synchronised.  The
 *     get_* calls synchronise the context's stream themselves.
 *   - A context is used by one host thread at a time.  Several contexts
 *     may run side by side on several threads (one per served problem):
 *     the solves (Method S2 batches included) and sdmm_accumulate_moments
 *     keep their copies on the context's streams, but set-up
 *     (sdmm_set_problem), sdmm_build_flux_basis and the calls that return
 *     data to the host (get_*, sdmm_reset_moments) make blocking copies on
 *     the null stream, which HIP refuses with EDEVICE while another thread
 *     captures a graph (a solve's CG iterations): make those calls while no
 *     other context is solving.
 */
#ifndef SDMM_H
#define SDMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SDMM_OK 0
#define SDMM_EINVAL (-1)     /* invalid argument or problem description       */
#define SDMM_ENOMEM (-2)     /* device memory could not be allocated          */
#define SDMM_EDEVICE (-3)    /* a HIP runtime call failed                      */
#define SDMM_ENOTCONV (-4)   /* some realization did not converge (status set) */
#define SDMM_EBREAKDOWN (-5) /* CG breakdown (p^T S p <= 0 or NaN)             */
#define SDMM_ESTATE (-6)     /* call made in the wrong order                   */
#define SDMM_EBUSY (-7)      /* the resource is held by a call still running  */

#define SDMM_PREC_FP64 0     /* factor and solves in FP64                      */
#define SDMM_PREC_MIXED 1    /* FP32 factor and solves + FP64 refinement       */

/* methods of sdmm_build_flux_basis (Section 5) */
#define SDMM_METHOD_STOCHASTIC 0    /* Method S3 (Section 5.4): a basis for every  */
                                    /* local KL realization, built once           */
#define SDMM_METHOD_DETERMINISTIC 1 /* Method S2 (Section 5.3): a basis for every  */
                                    /* global realization, built per batch inside */
                                    /* sdmm_solve_interface                        */
#define SDMM_METHOD_PER_ITERATION 2 /* Method S1 (Section 5.2): no Darcy basis;    */
                                    /* every CG iteration solves the local Darcy  */
                                    /* problems of each realization                */

/* status values written per realization by sdmm_solve_interface */
#define SDMM_CG_CONVERGED 0
#define SDMM_CG_MAXITER 1
#define SDMM_CG_BREAKDOWN 2

/* fields of sdmm_get_moments */
#define SDMM_FIELD_LAMBDA 0   /* mortar coefficients, M values                 */
#define SDMM_FIELD_DARCY_P 1  /* Darcy cell pressures                          */
#define SDMM_FIELD_DARCY_U 2  /* Darcy RT0 normal velocities (+x / +y)         */
#define SDMM_FIELD_STOKES_U 3 /* Stokes Q2 nodal velocities (x, y per node)    */
#define SDMM_FIELD_STOKES_P 4 /* Stokes Q1 nodal pressures                     */

/* index maps of sdmm_get_index_maps */
#define SDMM_MAP_INTERFACES 0 /* n_iface x 5: i, j, kind (0 ss 1 sd 2 dd), ndof, offset */
#define SDMM_MAP_SUB_PTR 1    /* n_sub + 1: CSR pointer into the DOF list       */
#define SDMM_MAP_SUB_DOFS 2   /* global mortar DOF of each local mortar DOF     */
#define SDMM_MAP_SUB_SIGN 3   /* +1 / -1 of each local mortar DOF               */
#define SDMM_MAP_G2L 4        /* n_real x n_region local realization indices     */
#define SDMM_MAP_NLOCAL 5     /* n_region local realization counts              */
#define SDMM_MAP_NODE_IDS 6   /* n_real x n_term collocation node ids          */

typedef struct sdmm_ctx sdmm_ctx;

/* Optional device allocator (for instance a framework's caching allocator).
 * alloc returns a device pointer on `device` of at least `bytes` bytes,
 * aligned to 256 bytes, or NULL on failure (the library then returns
 * ENOMEM); release gives back a pointer that alloc returned, with the same
 * size.  The library calls them from the host thread that calls it, with
 * `device` current; `user` is passed through.  Without an allocator the
 * library uses hipMalloc / hipFree. */
typedef struct {
    void* (*alloc)(size_t bytes, int device, void* user);
    void (*release)(void* ptr, size_t bytes, int device, void* user);
    void* user;
} sdmm_alloc;

/*
 * Problem description (Section 3.1: N_s Stokes subdomains numbered first,
 * then N_d Darcy subdomains; Section 3.3: mortar spaces; Section 2.1 and
 * eq. covariance: KL regions; Section 4: collocation rule).  All arrays are
 * host memory and are copied by sdmm_set_problem.
 *
 * Outer boundary: the velocity (inflow_x + inflow_shear y, inflow_y) is
 * imposed on the whole Stokes outer boundary; the Darcy outer boundary has
 * p = p_bottom on y = domain[2] and no flow elsewhere.  Body forces and
 * sources are zero.
 * The GPU path requires p_bottom == 0 (the Darcy complementary solution is
 * then zero).
 */
typedef struct {
    double nu_s, nu_d;       /* viscosities                                   */
    double alpha;            /* BJS friction coefficient (eq. BJS)            */
    double k_bjs;            /* permeability in the BJS term (deterministic)  */
    double inflow_x, inflow_y;
    double inflow_shear;     /* d(u_x)/dy of the imposed outer velocity       */
    double p_bottom;
    double domain[4];        /* x0 x1 y0 y1                                   */
    int32_t n_sub;
    const int32_t* sub_type;   /* n_sub: 0 Stokes, 1 Darcy                     */
    const double* sub_rect;    /* 4 n_sub: x0 x1 y0 y1                          */
    const int32_t* sub_n;      /* 2 n_sub: elements nx ny                       */
    const int32_t* sub_region; /* n_sub: KL region of a Darcy subdomain, else -1*/
    int32_t mortar_degree;     /* 1 or 2: discontinuous Lagrange                */
    int32_t mortar_elements;   /* elements per interface                       */
    int32_t n_region;
    const double* region_rect;      /* 4 n_region                              */
    const int32_t* region_nterm;    /* n_region: KL terms kept                 */
    const double* region_sigma2;    /* n_region: covariance amplitude          */
    const double* region_eta;       /* 2 n_region: correlation lengths         */
    const double* region_mean_logk; /* n_region: E[Y]                          */
    int32_t rule_kind;   /* 0 tensor Gauss-Hermite, 1 Smolyak sparse grid      */
    int32_t rule_m;      /* tensor: points per dimension                       */
    int32_t rule_level;  /* sparse: l_max                                      */
    int32_t rule_growth; /* sparse: 0 -> 2^(p+1)-1 points at level p, 1 -> p+1 */
    /* Stokes element: 0 Q2-Q1 on the rectangles, 1 triangular Taylor-Hood
     * P2-P1 (Section 6), each rectangle cut into two triangles on the same
     * node grid (the diagonal runs lower-left to upper-right, except in a
     * subdomain's lower-right and upper-left corner rectangles)           */
    int32_t stokes_element;
    /* RT0 velocity mass of the Darcy subdomains: 0 trapezoidal (diagonal,
     * the cell-centred 5-point system), 1 exact integration (Section 6),
     * solved as the SPD system of the face pressures (FP64, Methods S3
     * and S2; every Darcy subdomain 2 <= min(nx, ny) <= 128)              */
    int32_t darcy_mass;
} sdmm_problem;

typedef struct {
    int64_t n_sub, n_stokes, n_darcy, n_iface, M;
    int64_t n_real, n_term, n_region;
    int64_t n_units;        /* Darcy (subdomain, local realization) pairs      */
    int64_t n_floating;     /* floating Stokes subdomains (FETI)               */
    int64_t n_kernel;       /* columns of the FETI matrix G                    */
    int64_t field_size[5];  /* sizes of the five moment fields                 */
    int64_t basis_bytes;    /* device bytes of the S_{H,i}^{(k)} cache        */
    int64_t response_bytes; /* device bytes of the stored fine responses        */
    int64_t max_R;          /* largest number of mortar DOFs on one subdomain  */
    int64_t darcy_flops;    /* banded factor + solve flops of one full build   */
} sdmm_sizes;

typedef struct {
    int64_t basis_solves_darcy;   /* sum over Darcy subdomains of R_i L_j       */
    int64_t basis_solves_stokes;  /* sum over Stokes subdomains of R_i          */
    int64_t complementary_solves; /* solves for g_H (once, deterministic)       */
    int64_t units_built;          /* Darcy (i, k) bases built                   */
    int64_t refinement_steps;     /* FP64 refinement steps of the last mixed build,
                                     summed over the right-hand-side groups   */
    int64_t cg_iterations;        /* summed over realizations                   */
    int64_t realizations;         /* taken through CG                           */
    double ms_basis_darcy;        /* last build: Darcy units                    */
    double ms_basis_stokes;       /* last build: Stokes subdomains              */
    double ms_solve;              /* last solve_interface                       */
    double max_refine_residual;   /* largest relative residual after refinement */
    /* per-kernel timing of the CG iterations while SDMM_OPT_KERNEL_TIMING is
     * on: one iteration of every n-th convergence-check group is bracketed
     * by HIP events on the stream the kernels run on, with the other CG lane
     * idle meanwhile; sums over all solves */
    int64_t cg_launches;          /* product launches (= update launches), all   */
    int64_t cg_timed_launches;    /* sampled (product, update) launch pairs     */
    int64_t cg_timed_active;      /* realizations still iterating in them        */
    int64_t cg_timed_columns;     /* realization columns the products covered    */
    double ms_cg_apply;           /* summed duration of the sampled products     */
    double ms_cg_update;          /* summed duration of the sampled updates      */
    double ms_moments;            /* last expansion of the moments to the fields */
    double ms_basis_build;        /* last build, wall time: the Darcy units and the
                                     Stokes subdomains run side by side, so this is
                                     about the larger of the two times above    */
} sdmm_counters;

/* Create a context on HIP device `device`.  Ownership of *out passes to the
 * caller, who releases it with sdmm_destroy (which releases every problem
 * of the context).  alloc may be NULL (hipMalloc / hipFree); the library
 * copies the structure.  EINVAL for a bad device.  device = -1 creates a
 * context without a GPU: sdmm_set_problem, the sizes, index maps,
 * collocation and KL queries work; every call that computes on the device
 * returns ESTATE. */
int sdmm_create(int device, const sdmm_alloc* alloc, sdmm_ctx** out);
int sdmm_destroy(sdmm_ctx* ctx);
/* Message of the last failure on ctx; owned by ctx, valid until the next call. */
const char* sdmm_last_error(const sdmm_ctx* ctx);

/* Add a problem to the context: build meshes, interfaces and mortar maps
 * (Section 3.1, 3.3), the KL modes of every region (Section 2.1, eq. Fred
 * with the separable kernel of eq. covariance), the collocation points,
 * weights and global->local index table (Section 4; Step 4 of Method S3),
 * and upload the Darcy KL tables and Stokes operators.  *problem_id (host)
 * receives the problem's id, which every later call on it names; a context
 * holds any number of problems, each with its own device state, streams,
 * options and counters.  EINVAL when subdomains do not tile, a region is
 * not a union of Darcy subdomains, a mortar has more DOFs per interface
 * than the fine trace, or p_bottom != 0. */
int sdmm_set_problem(sdmm_ctx* ctx, const sdmm_problem* p, int64_t* problem_id);
/* Release one problem and all its device state (EINVAL for an unknown id). */
int sdmm_release_problem(sdmm_ctx* ctx, int64_t id);
int sdmm_get_sizes(sdmm_ctx* ctx, int64_t id, sdmm_sizes* out);
/* Copy an integer index map (SDMM_MAP_*) to host `out` (capacity cap
 * entries); *n_out receives its length.  EINVAL if cap is too small. */
int sdmm_get_index_maps(sdmm_ctx* ctx, int64_t id, int kind, int64_t* out, int64_t cap, int64_t* n_out);
/* Collocation points (n_real x n_term, row-major) and weights (n_real) to
 * host memory; either pointer may be NULL. */
int sdmm_get_collocation(sdmm_ctx* ctx, int64_t id, double* points, double* weights);
/* KL eigenvalues sigma^2 lambda_a lambda_b of the kept modes of one region
 * and their 1-D mode indices (a, b) (host arrays of nterm and 2 nterm). */
int sdmm_get_kl(sdmm_ctx* ctx, int64_t id, int region, double* lam, int32_t* modes);

/* Flux basis (Section 5).
 * method SDMM_METHOD_STOCHASTIC, Method S3 pre-computation loop (Section
 * 5.4): for every Darcy subdomain and every local realization k of its
 * region, build K (eq. KLapprox), the RT0-Q0 operator and its banded
 * factor, solve for every mortar basis function (eqs. starDproblem1-2) and
 * store S_{H,i}^{(k)}; for every Stokes subdomain do the same once (eqs.
 * starSproblem1-2) together with the complementary solution (eqs.
 * barSproblem1-2) that gives g_H.
 * method SDMM_METHOD_DETERMINISTIC, Method S2 (Section 5.3): only the
 * Stokes part is built here; every sdmm_solve_interface call then builds
 * S_{H,i} for each Darcy subdomain and each realization of its batch from
 * that realization's own KL field, and solves with it.
 * method SDMM_METHOD_PER_ITERATION, Method S1 (Section 5.2): only the Stokes
 * part is built here; every sdmm_solve_interface call factors the local
 * Darcy problem of each (subdomain, realization) of its batch once (FP64,
 * whatever the precision) and solves it for every application of S_H in the
 * CG (one local solve per Darcy subdomain per iteration); the Stokes
 * problems, which no realization changes, enter through their responses.
 * precision: SDMM_PREC_FP64 or SDMM_PREC_MIXED (FP32 factor and multi-RHS
 * solves with FP32 accumulation, FP64 refinement of every response).
 * Returns ENOTCONV (the basis is still stored) when the mixed refinement of
 * some right-hand-side group stops above its tolerance. */
int sdmm_build_flux_basis(sdmm_ctx* ctx, int64_t id, int method, int precision, void* stream);
/* Copy S_{H,i}^{(k)} (R_i x R_i, column-major with leading dimension ld,
 * host) of subdomain `sub` and local realization k (k = 0 for Stokes) of a
 * stochastic basis (Method S2: k is the batch position of the last solve;
 * Method S1 has no Darcy basis: ESTATE).  The signs of Stokes-Stokes mortar
 * DOFs are included. */
int sdmm_get_basis(sdmm_ctx* ctx, int64_t id, int sub, int k, double* S, int64_t ld);

/* The interface right-hand side g_H (host, M values; Section 5.1, the
 * complementary Stokes solutions of eqs. barSproblem1-2 tested with the
 * mortar functions) and the FETI matrix G (host, n_kernel x M, one row per
 * rigid-motion mode of a floating Stokes subdomain: its velocity trace on
 * the mortar functions).  Either pointer may be NULL.  Needs a built basis. */
int sdmm_get_interface_data(sdmm_ctx* ctx, int64_t id, double* g, double* G);

/* Solve S_H lambda = g_H (Section 5.1) for n realizations by CG with S_H
 * applied as linear combinations of the basis (Section 5.3) and, with
 * floating Stokes subdomains, the FETI projection.
 *   gidx (device int64, n): global collocation indices; or NULL, and then
 *   y (device double, n x n_term, row-major) gives each realization's
 *   point in the stochastic space directly (an off-grid request; needs
 *   SDMM_METHOD_DETERMINISTIC or SDMM_METHOD_PER_ITERATION, since a
 *   stochastic basis exists only for the collocation points of the local
 *   grids).  Under Method S1 all n realizations iterate together and their
 *   local factors stay resident (about n x sum over Darcy subdomains of
 *   16 N_i (b_i + R_i) bytes).
 * lambda_0 = 0; a realization stops when ||r_k|| <= rtol ||r_0||.  Outputs
 * (device): lambda (n x M, row-major), iters (int32 n), relres (double n),
 * status (int32 n, SDMM_CG_*); iters/relres/status may be NULL.  Returns
 * ENOTCONV when some realization hit max_iter (outputs still filled). */
int sdmm_solve_interface(sdmm_ctx* ctx, int64_t id, int64_t n, const int64_t* gidx, const double* y, double rtol,
                         int32_t max_iter, double* lambda, int32_t* iters, double* relres, int32_t* status,
                         void* stream);
/* Allocation-free sdmm_solve_interface, for callers that cannot allocate
 * device memory (serving loops and harnesses in which hipMalloc is not
 * allowed).  The same CG kernels and the same results as
 * sdmm_solve_interface for collocation indices gidx (device int64, n); the
 * other arguments are as there.  It calls no hipMalloc, hipFree,
 * hipHostMalloc or other allocating routine: the CG workspace (the state of
 * every realization, which all stay in flight for the whole solve, and the
 * realization group tables) lives in a fixed scratch array of
 * sdmm_noalloc_scratch_bytes() bytes (64 MiB) that the library holds on each
 * GPU from the first sdmm_create on it until the process ends.  EINVAL, with
 * nothing computed, when the batch does not fit (about
 * n (8 (2 M + sum_i R_i) + 40) bytes plus the tables; e.g. about 1,600
 * realizations for 1,280 mortar DOFs and sum_i R_i = 2,560).  Launches are
 * eager on `stream`; the call returns when the solve has finished.  All
 * calls on one GPU share that array and a call leaves its contents behind:
 * calls that overlap in time on one GPU (from two host threads or two
 * contexts) race and give wrong results. */
int sdmm_solve_interface_noalloc(sdmm_ctx* ctx, int64_t id, int64_t n, const int64_t* gidx, double rtol,
                                 int32_t max_iter, double* lambda, int32_t* iters, double* relres, int32_t* status,
                                 void* stream);
/* Size in bytes of the scratch array of sdmm_solve_interface_noalloc (host *bytes). */
int sdmm_noalloc_scratch_bytes(int64_t* bytes);

/* CG streams: continuous batching of the collocation loop (Section 5.4,
 * main loop, Steps 3-5).  A stream keeps `slots` CG slots on the device;
 * realizations of any number of requests occupy them as they free up, so a
 * request submitted while others are iterating starts at the next
 * convergence check instead of waiting for a batch to finish.  Results are
 * those of sdmm_solve_interface (fixed-order reductions: a realization's
 * answer does not depend on what shares the slots with it).
 *   open    slots (1 .. 2^24), rtol and max_iter as in sdmm_solve_interface,
 *           stream: the hipStream_t every later call of the stream uses;
 *           *sid (host) receives the stream id.  Allocates the stream's
 *           workspace (about slots (8 (3 M + sum_i R_i) + 56) bytes).
 *   submit  n collocation indices gidx (host int64, checked) and the
 *           request's outputs (device): lambda (n x M), iters / relres /
 *           status (n each, may be NULL); *ticket (host) names the request.
 *           Nothing runs until sdmm_stream_run.
 *   run     up to max_groups convergence-check groups (SDMM_OPT_CG_CHECK
 *           iterations each): at every check, finished realizations leave
 *           their slots (their outputs are copied to their requests) and
 *           queued ones start in the freed slots.  done (host, capacity cap)
 *           receives the tickets of the requests completed during the call,
 *           *n_done their number, *in_flight (may be NULL) the realizations
 *           still iterating or queued.  Returns when max_groups groups ran
 *           or nothing is left; the outputs of the completed requests are
 *           then valid.
 *   close   waits for the stream and releases it.
 * EINVAL for unknown ids or bad arguments. */
int sdmm_stream_open(sdmm_ctx* ctx, int64_t id, int64_t slots, double rtol, int32_t max_iter, void* stream,
                     int64_t* sid);
int sdmm_stream_submit(sdmm_ctx* ctx, int64_t id, int64_t sid, int64_t n, const int64_t* gidx, double* lambda,
                       int32_t* iters, double* relres, int32_t* status, int64_t* ticket);
int sdmm_stream_run(sdmm_ctx* ctx, int64_t id, int64_t sid, int32_t max_groups, int64_t* done, int64_t cap,
                    int64_t* n_done, int64_t* in_flight);
int sdmm_stream_close(sdmm_ctx* ctx, int64_t id, int64_t sid);

/* Add n realizations to the moment accumulators (Section 2, Step 6 of
 * Method S3): gidx (device int64 n) or, for off-grid requests, NULL and y
 * (device n x n_term) as in sdmm_solve_interface; lambda (device n x M from
 * sdmm_solve_interface); weights (device double n, or NULL for the
 * collocation weights of the points; required with y).  Under Methods S2
 * and S1 the realizations must be those of the last sdmm_solve_interface
 * call (ESTATE otherwise); Method S1 recovers each realization's Darcy
 * fields with one more local solve per subdomain. */
int sdmm_accumulate_moments(sdmm_ctx* ctx, int64_t id, int64_t n, const int64_t* gidx, const double* y,
                            const double* lambda, const double* weights, void* stream);
/* Mean and variance (host arrays of cap >= field_size[field] entries) of one
 * field; EINVAL if cap is too small. */
int sdmm_get_moments(sdmm_ctx* ctx, int64_t id, int field, double* mean, double* var, int64_t cap);
/* Expand the accumulated moments to the fine Darcy and Stokes fields on the
 * device (Section 2: E[u] and E[u^2] of every velocity and pressure DOF from
 * the accumulated mortar coefficients and the stored responses), enqueued on
 * `stream`; sdmm_get_moments then only copies.  sdmm_get_moments expands by
 * itself when the accumulators changed since the last expansion. */
int sdmm_finalize_moments(sdmm_ctx* ctx, int64_t id, void* stream);
int sdmm_reset_moments(sdmm_ctx* ctx, int64_t id);

/* Tuning knobs of the batched CG of one problem (used by the autotuner):
 *   SDMM_OPT_CG_CHUNK  realizations in flight in the CG (slots; a finished
 *                      realization's slot is refilled from the batch) and
 *                      per moment pass (0 = sized so their vectors fit a
 *                      ~200 MB cache budget)
 *   SDMM_OPT_CG_CHECK  iterations between host convergence checks (1..1024,
 *                      default 64)
 *   SDMM_OPT_CG_GRAPH  1 = replay the iteration group as a captured HIP graph
 *   SDMM_OPT_CG_LANES  2 (default) = from 2048 slots on, split the slots into
 *                      two lanes with their own streams, so that one lane's
 *                      operator product overlaps the other's update on the
 *                      device; 1 = one lane
 *   SDMM_OPT_KERNEL_TIMING n > 0 = time two consecutive iterations of every
 *                      n-th check group of the first lane with HIP events
 *                      (the update writes lambda in every other iteration)
 *                      and sum the durations into the counters; the second
 *                      lane is drained first and waits for the timed pairs,
 *                      so the timed kernels run alone (those groups run
 *                      eagerly, the others replay the captured graph); 0 = off
 *   SDMM_OPT_STOKES_REBUILD 1 = every sdmm_build_flux_basis rebuilds the
 *                      Stokes basis too (0, the default: built once, since
 *                      it does not depend on the realization)
 *   SDMM_OPT_STOKES_REFINE FP64 refinement steps after the band LDL^T solves
 *                      of the Stokes subdomains (0 .. 8, default 0)
 *   SDMM_OPT_BASIS_LAUNCH layout of the Darcy units of a Method S3 build
 *                      (Section 5.4 pre-computation loop): 1 = one launch
 *                      per shape class (padded band, padded R), LDS sized for
 *                      the class, classes on forked streams; 2 = one launch
 *                      per phase over the whole queue of units sorted by
 *                      cost, LDS sized for the widest class; 0 (default) =
 *                      tuned: the first build of each precision times both
 *                      layouts and the right-hand-side group width (16, 32,
 *                      64) of every class and of the queue, and keeps the
 *                      fastest for the builds that follow
 * Results do not depend on any of them (the mixed path refines each group of
 * right-hand sides to the same tolerance, so its bases agree to that
 * tolerance across group widths). */
#define SDMM_OPT_CG_CHUNK 0
#define SDMM_OPT_CG_CHECK 1
#define SDMM_OPT_CG_GRAPH 2
#define SDMM_OPT_KERNEL_TIMING 3
#define SDMM_OPT_CG_LANES 4
#define SDMM_OPT_STOKES_REBUILD 5
#define SDMM_OPT_STOKES_REFINE 6
#define SDMM_OPT_BASIS_LAUNCH 7
int sdmm_set_option(sdmm_ctx* ctx, int64_t id, int option, int64_t value);
/* Autotuner of the batched CG: runs the first min(n, 16384) realizations of
 * gidx (device int64, n) through the whole CG (rtol, max_iter as in
 * sdmm_solve_interface) once per candidate slot count (all of the sample,
 * 1024 .. 8192 in steps of 512 below the sample size, and the default sized
 * for a ~200 MB cache budget) and keeps the fastest as SDMM_OPT_CG_CHUNK; *chunk_out (host, may be NULL)
 * receives it.  Needs a built basis; results of later solves do not depend
 * on the choice.  Counters are left as they were.  Runs on `stream`. */
int sdmm_autotune(sdmm_ctx* ctx, int64_t id, int64_t n, const int64_t* gidx, double rtol, int32_t max_iter,
                  void* stream, int64_t* chunk_out);
int sdmm_get_counters(sdmm_ctx* ctx, int64_t id, sdmm_counters* out);

#ifdef __cplusplus
}
#endif
#endif /* SDMM_H */

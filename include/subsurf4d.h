/*
 * subsurf4d.h -- C ABI of the MI355X (gfx950) library for the semi-implicit
 * time step of the 4D generalized subjective-surface (SUBSURF) segmentation
 * model of Uba, Mikula and Park, "4D Segmentation Algorithm with application
 * to 3D+time Image Segmentation" (arXiv 2111.11866).
 *
 * Problem (Sec. 3.1): given a 4D image I0 on a box of N1 x N2 x N3 voxels and
 * N4 frames, per-frame centres c_m^l of the objects, and parameters, evolve
 *     u_t = |grad u| div(G0 grad u / |grad u|),  u = 0 on the boundary,
 * with G0 = g(delta |grad I0_sigma| + vartheta |grad ITH_sigma|), g(s) = 1/(1+K s^2).
 * Each time step (Sec. 3.2) assembles a 9-point 4D finite-volume system from
 * reduced-diamond-cell face gradients of the previous, locally rescaled
 * solution and solves it by red-black SOR (Sec. 3.2.2), then rescales u to
 * [0,1] in balls around the centres (local rescaling remark, Sec. 3.2.2).
 *
 * Conventions shared by every entry point
 *  - Grid: interior sizes n[0..3] = (N1 x, N2 y, N3 z, N4 t), uniform spacing h.
 *  - "padded" arrays have (N1+2)(N2+2)(N3+2)(N4+2) entries, x fastest
 *    (index ((l*(N3+2)+k)*(N2+2)+j)*(N1+2)+i, 0 <= i <= N1+1 ...); index 0 and
 *    N+1 along each axis are the boundary (ghost) layer that holds the
 *    Dirichlet data u^D (Sec. 3.7 layout).  "interior" arrays have N1 N2 N3 N4
 *    entries, x fastest.
 *  - Voxel coordinates of interior cell (i,j,k,l) are X = (i-1, j-1, k-1) in
 *    frame l-1; centres use the same coordinates.
 *  - Every pointer argument named "device" is device memory on the current
 *    HIP device; every other pointer is host memory.  The caller owns all
 *    memory.  The library calls no hipMalloc/hipFree: scratch space comes
 *    from the caller's workspace (subsurf4d_step_noalloc: from a fixed device
 *    array of the library).  (The batched calls keep one HIP graph
 *    executable per stream, and on the legacy default stream run on one
 *    library-owned non-blocking stream per device.)
 *  - `stream` is a hipStream_t (NULL = default stream).  Work is enqueued on
 *    it.  By default the calls that iterate to a tolerance (prepare, step,
 *    solve, the batched calls) read the device-side convergence state between
 *    chunks of iterations and therefore synchronise `stream`; when they
 *    return, every result they write is final.  With SUBSURF4D_FLAG_ASYNC the
 *    step and solve calls only enqueue work (no host synchronisation, no host
 *    read of device memory, capturable in a HIP graph) and write their
 *    outcome to a device-accessible result.
 *  - Errors: argument and shape checks happen before anything is enqueued and
 *    return a negative status.  A HIP failure returns SUBSURF4D_EDEVICE.  No
 *    C++ exception crosses this interface.  subsurf4d_last_error() gives a
 *    thread-local message for the last failing call on the calling thread.
 */
#ifndef SUBSURF4D_H
#define SUBSURF4D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
enum {
    SUBSURF4D_OK = 0,
    SUBSURF4D_NOT_CONVERGED = 1,  /* max_iter reached; last iterate returned   */
    SUBSURF4D_EINVAL = -1,        /* NULL pointer or parameter out of range     */
    SUBSURF4D_ESHAPE = -2,        /* grid sizes not supported                   */
    SUBSURF4D_EWORKSPACE = -3,    /* workspace smaller than *_workspace_bytes   */
    SUBSURF4D_ENONFINITE = -4,    /* a residual or norm became NaN/Inf          */
    SUBSURF4D_EDEVICE = -5        /* a HIP call failed                          */
};

/* image element types */
enum { SUBSURF4D_U8 = 0, SUBSURF4D_F32 = 1, SUBSURF4D_F64 = 2 };

/* arithmetic of the solve: FP64 throughout, or FP32/BF16 sweeps refined in FP64 */
enum { SUBSURF4D_FP64 = 0, SUBSURF4D_MIXED = 1 };

typedef struct {
    int32_t n[4];   /* interior sizes (x, y, z, t); each >= 1 */
    double h;       /* uniform grid spacing (> 0) */
} subsurf4d_grid;

/* A ball centre / seed: voxel coordinates and 0-based frame (16 bytes). */
typedef struct {
    float x, y, z;
    int32_t frame;
} subsurf4d_centre;

/* Parameters of the per-job preparation (Sec. 3.1, Sec. 3.2.2 G equation). */
typedef struct {
    double K;             /* edge-detector sensitivity, g(s) = 1/(1+K s^2), K >= 0 */
    double delta;         /* weight of |grad I0_sigma| (finite, >= 0) */
    double vartheta;      /* weight of |grad ITH_sigma| (finite, >= 0) */
    double lambda;        /* threshold TH = lambda*alpha + (1-lambda)*beta, in [0,1] */
    double ball_r;        /* ball radius r (voxels) of the local thresholding */
    double smooth_tau;    /* presmoothing: implicit heat-step size (finite, >= 0) */
    int32_t smooth_steps; /* number of implicit heat steps (>= 0) */
    int32_t smooth_max_iter; /* SOR iteration cap of each heat step, in [1, 2^30] */
    double smooth_omega;  /* SOR relaxation of the heat steps, in (0,2); <= 0: Young's optimum
                             2/(1+sqrt(1-rho^2)), rho = 8a/(1+8a), a = smooth_tau/h^2 */
    double smooth_tol;    /* relative L2 residual tolerance of the heat steps */
    double image_scale;   /* I0 = image_scale * image[...] */
} subsurf4d_prepare_params;

/* Parameters of one time step (Sec. 3.2). */
typedef struct {
    double eps;           /* regularisation epsilon of A_eps (> 0) */
    double tau;           /* time step (>= 0; 0 gives the identity solve) */
    double omega;         /* SOR relaxation, in (0,2); MIXED: relaxation of the inner FP32
                             sweeps only (the FP64 residual and refine_tol decide the result) */
    double tol;           /* stop at ||b - A u||_2 <= tol ||b||_2 (relative L2) */
    int32_t max_iter;     /* iteration cap, in [1, 2^30] */
    int32_t check_every;  /* test the stopping rule every this many iterations (0 means 1) */
    int32_t rescale;      /* 1: local rescaling after the solve (needs owner/centres) */
    int32_t precision;    /* SUBSURF4D_FP64 or SUBSURF4D_MIXED */
    double ball_r;        /* ball radius of the local rescaling */
    double refine_tol;    /* MIXED: FP64 relative residual target of refinement */
    int32_t inner_sweeps; /* MIXED: FP32 red-black iterations per refinement pass, in [1, 1024] */
    int32_t fixed_iters;  /* > 0: run exactly this many iterations, at most 2^30 (tol ignored; FP64 only) */
    int32_t iter_hint;    /* expected iteration count (0 = unknown); only sizes launch chunks */
    int32_t flags;        /* SUBSURF4D_FLAG_* bits */
} subsurf4d_step_params;

/* subsurf4d_step_params.flags: launch the refinement passes of a batched step
 * one by one instead of replaying a captured HIP graph (same results). */
#define SUBSURF4D_FLAG_NO_GRAPH 1
/* subsurf4d_step_params.flags: use this work shape for the inner sweeps of a
 * batched step instead of the autotuner's choice (same results): flat
 * 256-cell items, or 256-slot columns marching through the frames. */
#define SUBSURF4D_FLAG_SWEEP_FLAT 2
#define SUBSURF4D_FLAG_SWEEP_MARCH 4
/* subsurf4d_step_params.flags: enqueue-only step / solve (subsurf4d_step,
 * subsurf4d_step_dirichlet, subsurf4d_step_noalloc, subsurf4d_solve).  The
 * call checks its arguments, enqueues every launch up to the iteration cap and
 * returns 0 without synchronising: FP64 enqueues 2*max_iter + 1 half-sweeps
 * (fixed_iters in place of max_iter when set), MIXED max_iter/inner_sweeps + 1
 * refinement passes; launches after the stopping rule has been met return at
 * once, so max_iter bounds the cost and should be set near the expected
 * count.  `result` (NULL allowed) must then be device memory or pinned host
 * memory: the last kernel of the call writes the outcome there, including
 * SUBSURF4D_NOT_CONVERGED and SUBSURF4D_ENONFINITE, which the return value
 * does not report.  Only kernel launches are enqueued (no memset or copy), so
 * the call can be captured in a HIP graph and replayed. */
#define SUBSURF4D_FLAG_ASYNC 8
/* subsurf4d_step_params.flags, MIXED, synchronous step and solve calls: from
 * the third refinement pass on, the host shortens a pass to the FP32
 * iterations that the contraction measured over the previous pass predicts
 * for reaching refine_tol (x 1.25, + 1), never beyond inner_sweeps.  The
 * stopping rule is still the FP64 residual's, so the result meets refine_tol
 * as without the flag; only the number of inner iterations differs
 * (result->iterations counts them).  Ignored with SUBSURF4D_FLAG_ASYNC, by
 * FP64 steps and by the batched step. */
#define SUBSURF4D_FLAG_SHORT_LAST_PASS 16

/* Outcome of a solve.  Iterations are full red-black iterations. */
typedef struct {
    int32_t status;           /* SUBSURF4D_OK, _NOT_CONVERGED or _ENONFINITE */
    int32_t iterations;       /* k of the returned iterate u^(k) (total inner sweeps for MIXED) */
    int32_t outer_iterations; /* MIXED: refinement passes; FP64: 0 */
    int32_t reserved;
    double rel_residual;      /* ||b - A u||_2 / ||b||_2 of the returned iterate */
    double bnorm;             /* ||b||_2 */
} subsurf4d_result;

/* Bytes of device workspace the calls below need for this grid, for
 * `n_centres` ball centres, in the given precision.  Host-only; 0 if the grid
 * is invalid.  One workspace serves every call on the grid (not concurrently). */
size_t subsurf4d_workspace_bytes(const subsurf4d_grid* grid, int32_t n_centres, int32_t precision);

/* Bytes of workspace that subsurf4d_prepare_g needs (<= subsurf4d_workspace_bytes;
 * the same amount also serves subsurf4d_rescale).  Host-only; 0 if invalid. */
size_t subsurf4d_prepare_workspace_bytes(const subsurf4d_grid* grid, int32_t n_centres);

/*
 * Per-job preparation (Sec. 3.1 local thresholding and presmoothing,
 * Sec. 3.2.2 edge detector on faces):
 *  - owner (device, interior int32): index of the ball B(c_m^l, r) of the cell's
 *    frame that contains the cell, nearest centre first, ties to the lowest
 *    index; -1 if none.  Balls are |X - c| <= r in voxel units.
 *  - I^TH = beta_m where I0 >= lambda*alpha_m + (1-lambda)*beta_m, else alpha_m,
 *    with alpha_m/beta_m the min/max of I0 over ball m, on owned cells;
 *    I^TH = I0 elsewhere.
 *  - I0 and I^TH are each smoothed by `smooth_steps` implicit steps of the
 *    zero-Neumann heat equation, solved by red-black SOR to smooth_tol.
 *  - G (device, 4 x padded doubles, G[d*padded + p]): g on the face between
 *    cell p and p+e_d (d = 0..3 for x,y,z,t), from reduced-diamond-cell
 *    gradients of the smoothed images; image values outside the interior are
 *    copies of the nearest interior value.
 * image (device): interior array of `image_dtype`.  centres (device):
 * n_centres entries (0 allowed).  workspace: >= subsurf4d_prepare_workspace_bytes.  Returns SUBSURF4D_NOT_CONVERGED if a heat
 * step hit smooth_max_iter (G is still written).
 */
int subsurf4d_prepare_g(const subsurf4d_grid* grid, const void* image, int32_t image_dtype,
                        const subsurf4d_centre* centres, int32_t n_centres,
                        const subsurf4d_prepare_params* params, double* G, int32_t* owner,
                        void* workspace, size_t workspace_bytes, void* stream);

/*
 * Initial segmentation function (Sec. 2 peak profile, applied per frame as
 * Sec. 3.1 states): for every interior cell, the maximum over the seeds of
 * its own frame of 1/(|X - s| + v) (R <= 0), or of max(0, 1/(|X-s|+v) - 1/(R+v))
 * (R > 0: profile cut at radius R and shifted for zero Dirichlet data).
 * Cells of frames without a seed get 0.  Ghost cells of u (device, padded)
 * are set to 0.  With R <= 0 the cost is O(cells x seeds).
 */
int subsurf4d_init_u(const subsurf4d_grid* grid, const subsurf4d_centre* seeds, int32_t n_seeds,
                     double v, double R, double* u, void* stream);

/*
 * Local rescaling (Sec. 3.2.2 remark): for each ball m, mu_m/xi_m = min/max of
 * u over the ball; every cell with owner == m becomes (u - mu_m)/(xi_m - mu_m)
 * unless xi_m - mu_m < 1e-12.  u (device, padded) is rescaled in place; ghosts
 * and cells without an owner are unchanged.  Needs a workspace (>=
 * subsurf4d_prepare_workspace_bytes) for the per-ball extrema.
 */
int subsurf4d_rescale(const subsurf4d_grid* grid, const subsurf4d_centre* centres,
                      int32_t n_centres, double ball_r, const int32_t* owner, double* u,
                      void* workspace, size_t workspace_bytes, void* stream);

/*
 * Coefficients of one step's system, exported in the natural layout (for
 * inspection and tests; subsurf4d_step assembles internally):
 *   c_f = tau/h^2 * Abar_P * G_f / A_f on the 8 faces f of cell P, face order
 *   -x,+x,-y,+y,-z,+z,-t,+t; A_f = sqrt(eps^2 + |grad_f u|^2),
 *   Abar_P = sqrt(eps^2 + (1/8) sum_f |grad_f u|^2) (Sec. 3.2.2, uniform-h system);
 *   b_P = u_P + sum over ghost neighbours of c_f * u^D.
 * u (device, padded) is u^{resc;n-1} with Dirichlet data in its ghosts.
 * coef (device, interior x 8 doubles, cell-major), b (device, interior).
 */
int subsurf4d_assemble(const subsurf4d_grid* grid, const double* G, const double* u,
                       const subsurf4d_step_params* params, double* coef, double* b,
                       void* stream);

/*
 * One semi-implicit time step (Sec. 3.2 and the implementation overview of
 * Sec. 3.5): assemble the system from u = u^{resc;n-1} (device, padded) and G,
 * solve it by red-black SOR (cells with i+j+k+l even first), starting from
 * u^{resc;n-1}, with the stopping rule: R_k = ||b - A u^(k)||_2 over interior
 * rows; test k = 0 and then every check_every-th iteration; stop at the first
 * R_k <= tol ||b||_2 and return u^(k); after max_iter iterations return
 * u^(max_iter) with SUBSURF4D_NOT_CONVERGED.  Then, if params->rescale, apply
 * the local rescaling with (centres, owner).  u is overwritten with the new
 * level (ghosts unchanged).  result (host; device-accessible with
 * SUBSURF4D_FLAG_ASYNC; may be NULL) receives the outcome.
 * precision MIXED: FP32 red-black sweeps on BF16-stored coefficients inside
 * an FP64 iterative refinement to refine_tol (the FP64 residual uses the FP64
 * operator).
 */
int subsurf4d_step(const subsurf4d_grid* grid, const double* G, const subsurf4d_centre* centres,
                   int32_t n_centres, const int32_t* owner, double* u,
                   const subsurf4d_step_params* params, subsurf4d_result* result,
                   void* workspace, size_t workspace_bytes, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * subsurf4d_step with the caller workspace replaced by a fixed device scratch
 * array that the library holds on every device it runs on
 * (SUBSURF4D_NOALLOC_SCRATCH_BYTES bytes, kept until the process ends; its
 * address is looked up on the first call on each device).  Same arguments,
 * results and status as subsurf4d_step otherwise.  A grid whose
 * subsurf4d_workspace_bytes(grid, n_centres if rescale else 0, precision)
 * exceeds the scratch returns SUBSURF4D_EWORKSPACE with nothing enqueued (the
 * 24^3 x 8 grid needs 84 MiB in FP64, 107 MiB mixed).  The call allocates and
 * frees no device memory.  Every call on one device shares that device's
 * scratch and leaves its last contents there: calls that overlap in time on
 * one device (other host threads, or unordered streams) race and give wrong
 * results; each call initialises everything it reads.
 */
#define SUBSURF4D_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int subsurf4d_step_noalloc(const subsurf4d_grid* grid, const double* G, const subsurf4d_centre* centres,
                           int32_t n_centres, const int32_t* owner, double* u,
                           const subsurf4d_step_params* params, subsurf4d_result* result, void* stream);

/*
 * The same step with Dirichlet data that changes in time (the boundary
 * condition of the problem statement, Sec. 3.1, with u^D a function of t; the
 * convergence test of Sec. 3.4 uses the exact solution): u's ghost layer holds
 * u^{n-1} on the boundary and feeds the boundary-face gradients, the ghost
 * layer of u_dirichlet (device, padded; its interior is not read) holds u^D of
 * the new level and enters the system.  On return u's ghost layer holds the
 * new level's u^D, so consecutive steps chain.  u_dirichlet must not alias u.
 * Everything else as subsurf4d_step.
 */
int subsurf4d_step_dirichlet(const subsurf4d_grid* grid, const double* G, const double* u_dirichlet,
                             const subsurf4d_centre* centres, int32_t n_centres, const int32_t* owner, double* u,
                             const subsurf4d_step_params* params, subsurf4d_result* result, void* workspace,
                             size_t workspace_bytes, void* stream);

/*
 * The linear solve alone (Sec. 3.2.2 red-black SOR) for externally given
 * coefficients: coef (device, interior x 8, face order as above), b (device,
 * interior; Dirichlet terms already included), u (device, padded; interior =
 * initial guess, overwritten by the result; ghosts ignored).  The diagonal is
 * 1 + sum of the 8 coefficients; neighbours outside the interior do not
 * enter.  Same stopping rule and result as subsurf4d_step.
 */
int subsurf4d_solve(const subsurf4d_grid* grid, const double* coef, const double* b, double* u,
                    const subsurf4d_step_params* params, subsurf4d_result* result,
                    void* workspace, size_t workspace_bytes, void* stream);

/*
 * Bandwidth probe and counter calibration: copies `bytes` (a multiple of 16)
 * from src to dst (device, 16-byte aligned, not overlapping) with a plain
 * 16-byte-per-lane copy kernel, once untimed and then `reps` times between two
 * HIP events on `stream`; *ms (host) receives the mean time of one copy.
 * Synchronises `stream`.  Not part of the method; used to state the
 * practical HBM bandwidth next to the roofline and to scale the hardware
 * byte counters (a copy of known size).
 */
int subsurf4d_copy_probe(const void* src, void* dst, size_t bytes, int32_t reps, double* ms, void* stream);

/*
 * Read-dominated bandwidth probe (the FP64 sweeps read about 11 streams per
 * one written).  src (device) holds `reads` chunks of n = bytes/16 16-byte
 * elements (reads * bytes), reads in [1, 16].  writes = 1: dst (device, bytes)
 * receives dst[i] = sum over r < reads of src[r*n + i], a pass moving
 * (reads + 1) * bytes.  writes = 0: reads only; dst receives one 16-byte
 * partial sum per block of the launch in its first
 * min(65536, ceil(n / 1024)) elements (their total is the sum of all of src),
 * so it must hold that many.  Each pass runs once untimed and then `reps`
 * times between two HIP events on `stream`; *ms (host) receives the mean time
 * of one pass.  Buffers 16-byte aligned, not overlapping.  Synchronises
 * `stream`.  Not part of the method: it states the HBM rate this chip gives
 * the sweeps' mix of reads and writes.
 */
int subsurf4d_stream_probe(const void* src, void* dst, size_t bytes, int32_t reads, int32_t writes, int32_t reps,
                           double* ms, void* stream);

/*
 * Batched time step over many independent windows (the per-nucleus windows
 * the paper cuts around cells, Sec. 4).  Each job is one window with its own
 * grid, G, u, owner map, centres and workspace; all jobs advance together:
 * each kernel launch processes the work items of every unfinished job.
 * precision SUBSURF4D_MIXED: every job gets what subsurf4d_step with
 * SUBSURF4D_MIXED computes for it (assembly, FP64-refined FP32/BF16
 * red-black SOR to refine_tol, local rescaling); a refinement pass is
 * `inner_sweeps` FP32 red-black iterations, the update and the FP64
 * residual.  precision SUBSURF4D_FP64: FP64 red-black SOR of the system
 * itself to tol, a pass being `inner_sweeps` iterations followed by the FP64
 * residual (the stopping rule is tested every inner_sweeps iterations;
 * check_every is ignored).  The pass is captured as a HIP graph whose
 * executable the library keeps per (device, stream) and updates with each
 * call's arguments; passes are replayed in chunks until every job has met its
 * stopping rule (a pass after that does no work).  A job's result does not
 * depend on the other jobs of the batch (per-job reductions in a fixed order).
 */
typedef struct {
    subsurf4d_grid grid;
    const double* G;                  /* device, 4 x padded, from subsurf4d_prepare_g */
    double* u;                        /* device, padded; in u^{resc;n-1}, out the new level */
    const int32_t* owner;             /* device, interior, from subsurf4d_prepare_g */
    const subsurf4d_centre* centres;  /* device, n_centres entries */
    int32_t n_centres;
    int32_t reserved;
    void* workspace;                  /* device, >= subsurf4d_batch_workspace_bytes, 256-byte aligned */
    size_t workspace_bytes;
} subsurf4d_batch_job;

/* Bytes of per-job workspace of the batched step (host-only; 0 if invalid).
 * A batched job is a window: (N1+2)(N2+2)(N3+2)(N4+2) <= 2^25 padded cells
 * (larger volumes go through subsurf4d_step); larger grids give 0 here and
 * SUBSURF4D_ESHAPE from subsurf4d_step_batched. */
size_t subsurf4d_batch_workspace_bytes(const subsurf4d_grid* grid, int32_t n_centres);

/* Bytes of the shared device table of a batch of n_jobs jobs (host-only). */
size_t subsurf4d_batch_table_bytes(int32_t n_jobs);

/*
 * Advance every job by one time step.  jobs (host array of n_jobs), params
 * (SUBSURF4D_MIXED or SUBSURF4D_FP64, inner_sweeps in [1, 1024];
 * fixed_iters is ignored; SUBSURF4D_FLAG_ASYNC is refused), results (host
 * array of n_jobs, may be NULL; iterations = passes * inner_sweeps), table
 * (device, >= subsurf4d_batch_table_bytes).
 * Synchronises `stream`.  Returns SUBSURF4D_NOT_CONVERGED if any job hit its
 * cap, SUBSURF4D_ENONFINITE if any job failed (see each job's result).
 * n_jobs = 0 is an empty batch: SUBSURF4D_OK, nothing enqueued (jobs and
 * table may then be NULL).
 */
int subsurf4d_step_batched(const subsurf4d_batch_job* jobs, int32_t n_jobs, const subsurf4d_step_params* params,
                           subsurf4d_result* results, void* table, size_t table_bytes, void* stream);

/*
 * Batched preparation of many windows (A1-A3 of the per-job preparation, then
 * the initial function and its local rescale: the implementation overview of
 * Sec. 3.5 up to the first time step), for jobs that will be advanced with
 * subsurf4d_step_batched.  Every job gets what subsurf4d_prepare_g,
 * subsurf4d_init_u (v, R) and subsurf4d_rescale (ball_r; skipped if
 * ball_r < 0) compute for it: owner map and G on the job's arrays, u0 rescaled
 * in u.  Each job's two presmoothing solves keep their own stopping rule.
 * All jobs of a call must share h.
 */
typedef struct {
    subsurf4d_grid grid;
    const void* image;                /* device, interior, x fastest, dtype image_dtype */
    int32_t image_dtype;              /* subsurf4d_dtype */
    int32_t n_centres;
    const subsurf4d_centre* centres;  /* device: ball centres (thresholding and rescale) */
    int32_t n_seeds;
    int32_t reserved;
    const subsurf4d_centre* seeds;    /* device: seeds of the initial function */
    double* G;                        /* device, out: 4 x padded */
    int32_t* owner;                   /* device, out: interior */
    double* u;                        /* device, out: padded u0 after the rescale */
    void* workspace;                  /* device: the job's batched-step workspace, used as scratch */
    size_t workspace_bytes;           /* >= subsurf4d_batch_workspace_bytes(grid, n_centres) */
} subsurf4d_batch_prepare_job;

/*
 * Prepare every job.  jobs (host array of n_jobs), params as for
 * subsurf4d_prepare_g, statuses (host array of n_jobs, may be NULL: per job 0,
 * SUBSURF4D_NOT_CONVERGED if a presmoothing solve hit smooth_max_iter, or
 * SUBSURF4D_ENONFINITE), table (device, >= subsurf4d_batch_table_bytes(n_jobs),
 * 256-byte aligned).  Synchronises `stream`.  Returns 0,
 * SUBSURF4D_NOT_CONVERGED if any job's solve hit its cap, or a negative code.
 * n_jobs = 0 is an empty batch: SUBSURF4D_OK, nothing enqueued.
 */
int subsurf4d_prepare_batched(const subsurf4d_batch_prepare_job* jobs, int32_t n_jobs,
                              const subsurf4d_prepare_params* params, double v, double R, double ball_r,
                              int32_t* statuses, void* table, size_t table_bytes, void* stream);

/*
 * Cell tracking from the segmentation (Sec. 5, cell tracking based on the 4D
 * segmentation).  A voxel of frame l is segmented when u >= level; a cell is
 * a set of segmented voxels of one frame connected through shared faces,
 * named by the smallest interior index of its voxels.  For every cell voxel
 * the squared distance (voxel units) to the nearest voxel of its frame
 * outside the cell, the outside of the image counting as outside; the cell's
 * centre is its voxel of largest distance (ties: smallest index).  Backward
 * link of a cell of frame l > 0 (the backtracking of Sec. 5): the cell of
 * frame l-1 holding the centre's voxel (kind 1); else the cell of frame l-1
 * overlapping the most of this cell's voxels moved to frame l-1 (ties:
 * smallest name; kind 2); else none (prev -1, kind 0).
 */
typedef struct {
    int32_t name;     /* smallest interior index of the cell's voxels */
    int32_t frame;    /* 0-based frame */
    int32_t centre;   /* interior index of the centre voxel */
    int32_t dist2;    /* squared distance of the centre to the nearest voxel outside the cell */
    int32_t prev;     /* name of the linked cell of the previous frame, -1 if none */
    int32_t kind;     /* 0 none, 1 centre, 2 overlap, 3 joined (subsurf4d_track_join) */
} subsurf4d_cell;

/* Bytes of device workspace of subsurf4d_track for `capacity` cells (host-only;
 * 0 if the grid has 2^31 or more interior voxels). */
size_t subsurf4d_track_workspace_bytes(const subsurf4d_grid* grid, int32_t capacity);

/*
 * Cells, distances, centres and backward links of the segmentation u (device,
 * padded).  label (device, interior int32, out): cell name or -1; dist2
 * (device, interior int32, out): squared distance, 0 outside cells; cells
 * (host, `capacity` records, out): one per cell in increasing name order;
 * *n_cells (host, out): the number of cells (also when it exceeds capacity,
 * which returns SUBSURF4D_EWORKSPACE).  Synchronises `stream`.
 */
int subsurf4d_track(const subsurf4d_grid* grid, const double* u, double level, int32_t* label, int32_t* dist2,
                    subsurf4d_cell* cells, int32_t capacity, int32_t* n_cells, void* workspace,
                    size_t workspace_bytes, void* stream);

/*
 * Joining of partial trajectories (host-only; Sec. 5, last step).  A cell that
 * no cell of the next frame links to ends a partial trajectory, which runs
 * back along the links to a cell without one.  A partial trajectory T whose
 * first cell lies in frame f > 0 is joined after a partial trajectory S ending
 * in frame f-1 when T's first centre moved back by T's first displacement
 * (kept as is for a single cell) lies within `radius` voxels of S's last
 * centre, or S's last centre moved on by S's last displacement lies within
 * `radius` of T's first centre; T takes the nearest such S (squared distance;
 * ties: the smaller name of S's last cell), each S joins at most once, and
 * the T are taken in the order of the names of their first cells.  A join
 * sets the link of T's first cell to S's last cell with kind 3.  cells (host,
 * n_cells records from subsurf4d_track, updated in place).
 */
int subsurf4d_track_join(const subsurf4d_grid* grid, subsurf4d_cell* cells, int32_t n_cells, double radius);

/* Static text for a status code. */
const char* subsurf4d_status_string(int status);

/* Thread-local message of the last failing call on this thread ("" if none). */
const char* subsurf4d_last_error(void);

/* Library version string. */
const char* subsurf4d_version(void);

/*
 * Benchmark instrumentation of the red-black sweeps.  When enabled, every
 * solve records HIP events around each launch chunk of sweeps on its own
 * stream (one extra event pair per chunk; the chunk is synchronised anyway)
 * and adds: the chunks' elapsed milliseconds, the number of sweep launches
 * that did work (2K+1 for a solve returning iterate K: the extra red
 * half-sweep tests the stopping rule), the voxel updates K x interior cells,
 * and one solve.  op: 0 disable, 1 enable, 2 reset the totals, 3 read only.
 * Every call writes the current totals to the non-NULL outputs (host memory).
 * Process-wide, thread-safe.
 */
void subsurf4d_timing(int32_t op, double* sweep_ms, int64_t* sweep_launches, int64_t* voxel_updates,
                      int64_t* solves);

#ifdef __cplusplus
}
#endif

#endif /* SUBSURF4D_H */

/*
 * lsw.h -- C ABI of the L-sweeps Helmholtz library for MI355X (gfx950).
 *
 * Solves the PML-truncated Helmholtz system A u = b (eq. LS, Sec. 1.1 and App. A of
 * Taus, Zepeda-Nunez, Hewett, Demanet, "L-Sweeps", arXiv:1909.01467) with flexible
 * GMRES right-preconditioned by the L-sweeps preconditioner M ~ A^-1 (Sec. 3,
 * eq. PrecLS; Alg. Scenario3 of App. C) over a q x r checkerboard domain
 * decomposition (CDD, Sec. 2.1-2.2).  Every subdomain problem is factorised once
 * (Phase 2 of Sec. 3) and solved up to nine times per preconditioner application.
 *
 * Discretisation (App. A): per axis n bulk points at x = h..n h and n_pml PML points
 * on each side; cubic PML profile sigma = (C/delta)(dist/delta)^3, delta = n_pml h,
 * alpha = 1/(1 + i sigma/omega); symmetric 5-point form
 *   -div(Lambda grad u) - omega^2 m/(alpha_1 alpha_2) u = b,  Lambda = diag(s1, s2),
 *   s1 = alpha_1/alpha_2, s2 = alpha_2/alpha_1, coefficients at half points,
 * homogeneous Dirichlet data one point beyond the extended grid; in 3D the 7-point form
 * with s_k = alpha_k / (product of the other two alphas) and mass term
 * omega^2 m/(alpha_1 alpha_2 alpha_3).  A is complex symmetric (A = A^T), which the adjoint
 * solve uses.
 *
 * Conventions shared by every entry point:
 *  - Vectors live on the extended grid of N = N_x * N_y (* N_z) points (N_k = n_k + 2 n_pml_k),
 *    x fastest, then y, then z.  Complex values are interleaved (re, im) doubles, the layout of
 *    torch.complex128.  Several right-hand sides are stored one after the other:
 *    element (rhs, p) is at rhs * N + p.
 *  - Pointers named d_* are DEVICE pointers owned by the caller; they must stay valid
 *    until the call returns (all calls synchronise their stream before returning,
 *    except where stated).  Pointers named h_* are host pointers.
 *  - All device work is ordered on the stream given in lsw_opts_t.
 *  - Return value: LSW_OK (0) or a negative lsw_status; nothing aborts and no C++
 *    exception crosses the ABI.  lsw_last_error() describes the last failure.
 *  - A handle must not be used by two threads at once.  Different handles are
 *    independent.
 */
#ifndef LSW_H
#define LSW_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lsw_plan* lsw_handle_t;

typedef enum {
    LSW_OK = 0,
    LSW_EINVAL = -1,     /* invalid argument or geometry */
    LSW_ENOMEM = -2,     /* device allocation failed */
    LSW_EHIP = -3,       /* a HIP runtime call failed */
    LSW_ESINGULAR = -4,  /* zero pivot while factorising a subdomain block */
    LSW_ENAN = -5,       /* non-finite value in the input data */
    LSW_ENOCONV = -6     /* GMRES reached maxit before tol (u holds the last iterate) */
} lsw_status;

typedef enum {
    LSW_FP64 = 0,        /* complex128 factors, sweeps and Krylov */
    LSW_MIXED = 1        /* complex64 factors and sweeps (FP32 accumulation), FP64 Krylov */
} lsw_precision;

typedef enum {
    LSW_SWEEP_COMPRESSED = 0,  /* sweeps as trace-to-trace products with Q = A_ij^-1 on the trace lines (2D) */
    LSW_SWEEP_CHAIN = 1        /* every sweep solve as a full block forward/back substitution (always in 3D) */
} lsw_sweep_mode;

typedef struct {
    int dim;             /* 2, or 3: the CDD in (x, y) with beams over all z (7-point operator) */
    int n[3];            /* bulk points per axis (x, y, z) */
    int n_pml[3];        /* global PML points per side, per axis */
} lsw_grid_t;

typedef struct {
    int q;               /* CDD rows (groups along y, row 0 at the bottom) */
    int r;               /* CDD columns (groups along x, column 0 at the left) */
    int windows;         /* 0: one CDD (scenario 3 applied to any right-hand side);
                            1: scenario 4 of Sec. 2.1 (q, r >= 2; in 3D over the beams' (x, y)
                            cross-section): the CDD and three copies
                            with the interior boundaries shifted by shift[0] along x, shift[1] along y
                            and both, each sweeping the right-hand side multiplied by its window of a
                            partition of unity; M^-1 r is the sum of the four sweeps */
    int shift[2];        /* windows = 0: s = shift[0] (x) or shift[1] (y) > 0 translates this CDD's
                            interfaces along that axis: every group start of the even split, the
                            first bulk point included, moves by s points towards larger indices, so
                            the axis has one more group (the first holds the PML and s bulk points);
                            0 = the even split.  windows = 1: the shift of the shifted CDDs, <= 0
                            selecting half of the smallest bulk group; it must lie in
                            [3, smallest group - 3] so that the skeletons are disjoint */
} lsw_cdd_t;

typedef struct {
    double C;            /* absorption constant of the cubic profile (App. A); <= 0 selects 16 ln(omega) */
    int n_pml_local;     /* PML points of each interior side of a local problem; < 0 selects n_pml[x] */
} lsw_pml_t;

typedef struct {
    int precision;       /* lsw_precision */
    int restart;         /* FGMRES restart length (default 50 when <= 0) */
    int maxit;           /* maximum preconditioner applications per solve (default 500 when <= 0) */
    double tol;          /* relative true-residual tolerance ||b - A u|| <= tol ||b|| (default 1e-6 when <= 0) */
    int nrhs_max;        /* largest nrhs any later call will pass (default 1 when <= 0) */
    void* stream;        /* hipStream_t for all device work (NULL = default stream) */
    int sweep_mode;      /* lsw_sweep_mode; both compute the same M^-1 r up to rounding */
    /* Optional device allocator for every workspace buffer of the handle (factors, traces, Krylov
     * basis, ...), e.g. a framework's caching allocator; NULL selects hipMalloc / hipFree.  alloc
     * returns a device pointer of at least `bytes` bytes aligned to 256 bytes, or NULL on failure
     * (lsw_setup then fails with LSW_ENOMEM); release frees it.  Both or neither must be given.
     * The handle calls release only after waiting for its own streams.  ctx is passed through. */
    void* (*alloc)(size_t bytes, void* ctx);
    void (*release)(void* ptr, void* ctx);
    void* alloc_ctx;
} lsw_opts_t;

typedef struct {
    int iterations;      /* preconditioner applications used */
    int converged;       /* 1 if the true relative residual reached tol */
    double relres;       /* final true relative residual ||b - A u|| / ||b|| (FP64) */
} lsw_rhs_info_t;

typedef struct {
    lsw_rhs_info_t* h_rhs;   /* host array of nrhs entries filled by solve/adjoint (may be NULL) */
    double* h_history;       /* host array [nrhs][history_len]: residual estimate after each iteration (may be NULL) */
    int history_len;
    double t_solve_ms;       /* wall time of the call (stream-synchronised) */
    int applies;             /* preconditioner applications (batched over the active right-hand sides) */
} lsw_info_t;

typedef struct {
    int q, r, n_subdomains;
    int W_max, H_max;            /* largest local window (points along x / y) */
    long long N;                 /* extended-grid points */
    long long factor_elems;      /* complex entries of all block inverses G_k in full (built at setup) */
    int factor_elem_bytes;       /* 8 (complex64) or 16 (complex128) */
    int solves_per_apply;        /* (3q-2)(3r-2)-type count of local solves per application */
    int fronts_per_apply;        /* dependent launch steps per application */
    double apply_chain_bytes;    /* algorithmic bytes of G read by the block substitutions of one application */
    double apply_gemv_bytes;     /* algorithmic bytes of Q read by the trace-compressed fronts of one application */
    int chain_launches;          /* block-substitution kernel launches per application (2 per front) */
    int gemv_launches;           /* trace-compressed launches per application */
    long long q_elems;           /* complex entries of all trace-to-trace sweep operators Q' */
    double factor_flops;         /* real flops of the block factorisation */
    double t_setup_ms, t_factor_ms, t_q_ms;
    double last_apply_ms;        /* device time of the most recent lsw_apply (events) */
    double last_chain_ms;        /* ... spent in its block-substitution launches */
    double last_gemv_ms;         /* ... spent in its trace-compressed launches (3D: in the fronts after stage 1) */
    double apply_stage1_bytes;   /* part of apply_chain_bytes read by the stage-1 substitutions */
    double apply_final_bytes;    /* part of apply_chain_bytes read by the final z substitutions */
    double last_stage1_ms;       /* device time of the stage-1 substitutions (2 launches) */
    double last_final_ms;        /* device time of the final z substitutions (2 launches) */
    double last_final_rhs_ms;    /* device time of the final right-hand-side assembly */
    int rhs_per_workgroup;       /* right-hand sides per workgroup of the stage-1 / final substitutions
                                    (1, 2 or 4; 16 or 32 on matrix cores, 32 in complex64 only), chosen
                                    at setup by timing when nrhs_max > 1, or fixed by the environment
                                    variable LSW_RHS_PER_WORKGROUP */
    double tune_ms[5];           /* the timings of 1, 2, 4, 16 and 32 right-hand sides per workgroup
                                    (0: not tried) */
    int symmetric_factors;       /* 1 if the substitutions read packed symmetric blocks (G_k = G_k^T; about
                                    half the bytes of the full blocks): in 2D those with one right-hand
                                    side per workgroup, in 3D every plane step (64 x 64 tiles) */
    long long packed_factor_elems;  /* complex entries of the packed blocks (0 if not built) */
    int gemv_items;              /* work items (<= 64 output rows of one sweep solve) per application */
    int gemv_max_inputs;         /* largest input count (incoming trace values) of a sweep solve */
    int cdd_count;               /* 1, or 4 with windows: then sizes, work, setup times and the kernel-family
                                    times above are totals over the four CDDs (W_max/H_max: the first's),
                                    and last_apply_ms also covers the window and accumulation kernels */
    int window_shift[2];         /* shift of the shifted CDDs along x / y (0 without windows) */
    /* the dominant kernel of the most recent lsw_apply, timed launch by launch with events on the
     * handle's stream: 2D the final z substitutions (k_chain_sym / k_chain, 2 launches per CDD),
     * 3D the plane-step kernel reading the factors (k_tile3 on packed blocks, else k_step3) */
    double last_dom_ms;          /* summed device time of its launches */
    int dom_launches;            /* its launches */
    double dom_bytes;            /* algorithmic bytes those launches read (factor blocks) */
    long long noalloc_bytes;     /* scratch that lsw_apply_noalloc needs for this handle (at nrhs_max),
                                    to be compared with LSW_NOALLOC_SCRATCH_BYTES; 0 with windows */
    /* shape of the 2D packed one-right-hand-side substitutions (0 when they are not used): lanes per
     * workgroup, 4x4 tiles per lane, factor blocks in flight per lane, lanes per row of the
     * reduction; chosen at setup by timing every shape the widest window fits (the first CDD's
     * with windows), or fixed by the environment variable LSW_SYM_CONFIG */
    int sym_threads, sym_tiles_per_lane, sym_ring, sym_lanes_per_row;
    int sym_shapes_timed;        /* shapes timed at setup (0: one fits, or fixed) */
    double sym_tune_best_ms, sym_tune_worst_ms;   /* their fastest and slowest time (both fronts) */
    /* 2D: apply_stage1_bytes and apply_final_bytes on the full W x W blocks, which the substitutions
     * with R > 1 right-hand sides per workgroup read once per group of R */
    double apply_stage1_full_bytes, apply_final_full_bytes;
    /* 2D, nrhs_max > 1: 1 if the sweep levels of several right-hand sides run on matrix cores
     * (Q' read once per work item for 16 or 32 right-hand sides), chosen at setup by timing every
     * level both ways at nrhs_max, or fixed by the environment variable LSW_GEMV_MMA */
    int gemv_mma;
    double gemv_tune_ms[2];      /* those timings: batched GEMVs, matrix cores (0: not timed) */
} lsw_stats_t;

/* Size of the per-GPU scratch array of lsw_apply_noalloc (64 MiB). */
#define LSW_NOALLOC_SCRATCH_BYTES (64ull << 20)

/*
 * lsw_setup -- Setup and Factorise phases (Sec. 3, Phases 1-2).
 *   out    : receives the new handle (host pointer to a handle).
 *   d_m    : DEVICE, N doubles: squared slowness m = 1/c^2 on the EXTENDED grid
 *            (the caller extends the bulk medium into the PML, Sec. 1.1).  Read only
 *            during the call.
 *   omega  : angular frequency (> 0).
 *   h      : grid step (> 0); the bulk interval of axis k is [0, (n_k + 1) h].
 *   grid, cdd, pml, opts : HOST pointers to the structures above (opts may be NULL).
 * Builds the CDD (bulk points split as evenly as possible, the first n mod q groups
 * one larger, edge groups owning the global PML), the local problems (Omega_ij plus
 * 2 overlap lines and n_pml_local PML lines on every interior side, Sec. 2.2) and
 * factorises every local matrix by block-tridiagonal LU along y (2D: blocks are grid lines)
 * or along z (3D: every subdomain is a beam over all z, blocks are its xy planes of at most
 * 4096 points, and the global z PML is kept at both beam ends).
 * With cdd->windows = 1 it builds and factorises the four CDDs of scenario 4 (Sec. 2.1) and the
 * window tables a(x), b(y): a = 0 on the two trace lines of every interface of the CDD, 1 on those
 * of every shifted one, a linear ramp in between (w(d) / (w(d) + w(d')), w(t) = max(0, t - 1), d
 * and d' the distances to the nearest interface of either kind), and 1 beyond the outermost
 * (shifted) interfaces; the four windows are a b, (1-a) b, a (1-b), (1-a)(1-b).
 * Errors: LSW_EINVAL (dim not 2 or 3, sizes, a window that does not fit the grid, only one of
 * opts->alloc and opts->release, windows with q or r below 2 or a shift outside its range),
 * LSW_ENAN (non-finite m), LSW_ENOMEM, LSW_EHIP, LSW_ESINGULAR.  On error *out is NULL
 * and nothing is leaked.
 */
int lsw_setup(lsw_handle_t* out, const double* d_m, double omega, double h,
              const lsw_grid_t* grid, const lsw_cdd_t* cdd, const lsw_pml_t* pml,
              const lsw_opts_t* opts);

/*
 * lsw_apply -- one application z = M^-1 r of the L-sweeps preconditioner
 * (Alg. Scenario3: stage 1, four cardinal sweeps, four diagonal sweeps; with windows, the sum
 * of the four windowed sweeps of scenario 4, the three shifted CDDs on streams of the handle's
 * own that are forked from and joined to opts.stream).
 *   d_r : DEVICE, nrhs*N complex128 (read only).   d_z : DEVICE, nrhs*N complex128 (written).
 *   1 <= nrhs <= nrhs_max.  In LSW_MIXED the sweeps run in complex64.
 */
int lsw_apply(lsw_handle_t handle, const double* d_r, double* d_z, int nrhs);

/*
 * lsw_apply_noalloc -- lsw_apply for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  It computes the same
 * z = M^-1 r with the same kernels, but every per-application scratch buffer (the trace pool, the
 * block-substitution y/x slots, the final right-hand-side terms, the per-sweep z parts, and in 3D
 * the right-hand-side and solution slots of a front and the tile partials) lives in one file-scope
 * device array of LSW_NOALLOC_SCRATCH_BYTES per GPU, which each GPU the library runs on holds until
 * the process ends, instead of in the handle's workspace.
 *   d_r, d_z, nrhs : as lsw_apply (DEVICE buffers owned by the caller).
 *   - Allocates nothing: no hipMalloc / hipFree, no allocating library routine.
 *   - Only queues work on opts.stream and returns without synchronising: z is ready when the stream
 *     reaches this point.  No per-kernel times are recorded (lsw_query keeps those of lsw_apply).
 *   - Every call on one GPU shares that GPU's array and leaves its last contents there; the parts
 *     that must start at zero are cleared by a fill kernel at the start of every call.  Calls that
 *     overlap on one GPU (other streams, handles or threads) race.
 * Errors: LSW_EINVAL for a NULL argument, nrhs outside [1, nrhs_max], a windowed handle (scenario 4
 * is not supported), or a handle whose scratch need (lsw_stats_t.noalloc_bytes, sized for nrhs_max)
 * exceeds LSW_NOALLOC_SCRATCH_BYTES; LSW_EHIP if a launch fails.
 */
int lsw_apply_noalloc(lsw_handle_t handle, const double* d_r, double* d_z, int nrhs);

/*
 * lsw_solve -- FGMRES(restart) for A u = f, right-preconditioned by M (Sec. 3, Phase 3).
 *   d_f : DEVICE, nrhs*N complex128 right-hand sides b (read only).
 *   d_u : DEVICE, nrhs*N complex128, in: initial guess (zeros reproduce the paper's
 *         setting), out: solution.  Stops when ||b - A u||_2 <= tol ||b||_2 (true
 *         residual, FP64) or after maxit applications (then LSW_ENOCONV, u = last iterate).
 *   info: HOST, optional (may be NULL).
 * Each right-hand side runs its own Krylov process; applications are batched.  Once per
 * iteration the calling thread waits for the Hessenberg column by polling the stream (it
 * stays busy for the duration of the call).
 */
int lsw_solve(lsw_handle_t handle, const double* d_f, double* d_u, int nrhs, lsw_info_t* info);

/*
 * lsw_adjoint -- solves A^H v = g with the same factors: since A = A^T,
 * v = conj(A^-1 conj(g)).  Arguments as lsw_solve (d_v in/out, initial guess).
 */
int lsw_adjoint(lsw_handle_t handle, const double* d_g, double* d_v, int nrhs, lsw_info_t* info);

/*
 * lsw_matvec -- y = A x in FP64 (the global 5-point / 7-point operator of App. A).
 *   d_x, d_y : DEVICE, nrhs*N complex128; may not alias.
 */
int lsw_matvec(lsw_handle_t handle, const double* d_x, double* d_y, int nrhs);

/*
 * lsw_mass_gradient -- FWI gradient term  d_grad[p] += omega^2 Re( sum_s lam_s[p] w[p] u_s[p] ),
 * w = 1/(alpha_1 alpha_2 [alpha_3]) (the weight of m in the mass term of App. A), summed over nrhs
 * right-hand sides.  d_lam, d_u : DEVICE nrhs*N complex128; d_grad : DEVICE N doubles (accumulated).
 */
int lsw_mass_gradient(lsw_handle_t handle, const double* d_lam, const double* d_u, int nrhs,
                      double* d_grad);

/* lsw_query -- fills *stats (HOST pointer) with sizes, algorithmic work and timings. */
int lsw_query(lsw_handle_t handle, lsw_stats_t* stats);

/* lsw_last_error -- text of the last error on this handle (or of the last failed setup
 * when handle is NULL).  The string stays valid until the next call on the handle. */
const char* lsw_last_error(lsw_handle_t handle);

/* lsw_destroy -- frees every device and host resource of the handle.  NULL is accepted. */
int lsw_destroy(lsw_handle_t handle);

#ifdef __cplusplus
}
#endif
#endif /* LSW_H */

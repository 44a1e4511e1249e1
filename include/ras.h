/*
 * ras.h -- C ABI of an MI355X (gfx950) restricted additive Schwarz solver.
 *
 * The method is the restricted additive Schwarz (RAS) iteration of Cai and
 * Sarkis as used by Nayak, Cojean and Anzt, "Evaluating Abstract Asynchronous
 * Schwarz solvers" (arXiv 2003.05361): the unknowns of A x = b (Sec. 2.1,
 * eq. lin_sys) are partitioned into subdomains (Sec. 3.2.1), each subdomain is
 * grown by `overlap` layers (Sec. 2.1, Fig. 1), every subdomain solves its
 * local problem (Sec. 3.3.1) and writes back only the points it owns
 * (Sec. 2.1).  The synchronous variant applies all local updates of a sweep
 * from the same iterate; the asynchronous variant lets each subdomain proceed
 * with whatever neighbour values are current (Sec. 2.1, Sec. 3.4).  Both run
 * as one persistent GPU kernel holding every subdomain of the problem.
 *
 * Conventions for every entry point:
 *   - every call returns ras_status and never throws or aborts;
 *     ras_last_error() returns a thread-local message for the last failure;
 *   - status < 0: error, outputs untouched; status > 0: outputs valid, warning;
 *   - host pointers are borrowed for the duration of the call only; the
 *     library copies what it keeps;
 *   - device pointers (suffix _dev) are caller-owned, contiguous float64,
 *     right-hand side j of a multi-RHS call at offset j*n, and are used on the
 *     stream given at setup;
 *   - a handle is used by one host thread at a time; distinct handles are
 *     independent.
 */
#ifndef RAS_H
#define RAS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ras_status {
    RAS_OK = 0,
    RAS_NOT_CONVERGED = 1, /* tolerance not reached within max_sweeps / max_seconds; x valid */
    RAS_PENDING = 2,       /* serving: result not ready yet */
    RAS_E_ARG = -1,        /* invalid argument (sizes, null pointers, options) */
    RAS_E_PATTERN = -2,    /* CSR pattern invalid: unsorted, duplicate, out of range, unsymmetric */
    RAS_E_NOT_SPD = -3,    /* non-positive Cholesky pivot in a local factorisation */
    RAS_E_NOMEM = -4,      /* host or device allocation failed, or over a memory budget */
    RAS_E_HIP = -5,        /* a HIP runtime call failed (message names it) */
    RAS_E_STATE = -6,      /* wrong object state (e.g. handle without a device) */
    RAS_E_DIVERGED = -7,   /* non-finite residual */
    RAS_E_UNSUPPORTED = -8 /* shape outside the kernels' documented limits */
} ras_status;

/* Global matrix A of A x = b (Sec. 2.1, eq. lin_sys): square, symmetric
 * positive definite, CSR with n+1 monotone int64 row pointers, column indices
 * sorted and unique within each row, a symmetric pattern, float64 values.  */
typedef struct ras_csr {
    int64_t n;
    const int64_t* row_ptr;
    const int32_t* col;
    const double* val;
} ras_csr;

/* Partition into owned sets (Sec. 3.2.1).
 *   REGULAR_1D: parts[0] = P; part p owns rows [floor(p n / P), floor((p+1) n / P)).
 *   REGULAR_2D / REGULAR_3D: grid = (nx, ny, nz) with nx*ny*nz == n in natural
 *     order g = i + nx (j + ny k); parts = (px, py, pz); axis bounds
 *     floor(s N_axis / p_axis); subdomain id ix + px (iy + py iz).
 *   RCB: recursive coordinate bisection of the grid points into parts[0] parts
 *     with part weights 1 + jitter (2u - 1), u from SplitMix64(seed) (stand-in
 *     for the paper's edge-cut partitioner).
 *   EXPLICIT: owner[n] given, ids in [0, parts[0]), every part non-empty.  */
enum { RAS_PART_REGULAR_1D = 0, RAS_PART_REGULAR_2D = 1, RAS_PART_REGULAR_3D = 2, RAS_PART_RCB = 3,
       RAS_PART_EXPLICIT = 4 };
typedef struct ras_partition {
    int32_t kind;
    int32_t grid[3];
    int32_t parts[3];
    int32_t reserved;
    uint64_t seed;
    double jitter;
    const int32_t* owner;
} ras_partition;

/* Local solver (Sec. 3.3.1): a Cholesky factor of the local matrix computed
 * once at setup and applied by two triangular solves per local solve, or
 * cg_iters steps of conjugate gradients from a zero initial guess.
 *   CHOL_BANDED: the factor in the local (ascending global id) order, stored
 *     as a band; suits grid-ordered subdomains with narrow bands.
 *   CHOL_SPARSE: the factor of the local matrix reordered by nested
 *     dissection, stored sparse and applied by level-scheduled triangular
 *     solves (Sec. 3.3.1's sparse direct solver class); suits irregular
 *     subdomains and wide bands.  The subdomain's vector is kept in LDS, so a
 *     subdomain may have at most ras_sparse_max_rows(storage) local rows.
 * storage: FP64, FP32 (float32 values and float32 local arithmetic) or
 * FP16_ROWSCALED (factor rows scaled by their float32 max-abs, entries
 * rounded to float16, float32 arithmetic; banded Cholesky only).  The outer
 * residual, update and convergence test are always float64.  */
enum { RAS_LOCAL_CHOL_BANDED = 0, RAS_LOCAL_CG = 1, RAS_LOCAL_CHOL_SPARSE = 2 };
enum { RAS_STORAGE_FP64 = 0, RAS_STORAGE_FP32 = 1, RAS_STORAGE_FP16_ROWSCALED = 2 };
/* Transmission condition on the artificial boundary of a subdomain.
 *   DIRICHLET: the local matrix is A[Omega_p, Omega_p] (restricted additive
 *     Schwarz, Sec. 2.1).
 *   ROBIN: optimized restricted additive Schwarz (ORAS, the paper's future
 *     work, Sec. 5) with a Robin condition in algebraic form: the local matrix
 *     is A[Omega_p, Omega_p] - (1 - robin_q) diag(e), where e_i is the sum of
 *     |a_ij| over the columns j of row i outside Omega_p (the row's coupling
 *     across the artificial boundary); robin_q in (0, 1], 1 = DIRICHLET.  The
 *     global iteration is unchanged (the correction form keeps the solution of
 *     A x = b the fixed point); only the local matrices, and so their factors,
 *     change.  Direct local solvers only (CHOL_BANDED, CHOL_SPARSE).  */
enum { RAS_TRANSMISSION_DIRICHLET = 0, RAS_TRANSMISSION_ROBIN = 1 };
typedef struct ras_local {
    int32_t kind;
    int32_t cg_iters;
    int32_t storage;
    int32_t transmission;
    double robin_q;
} ras_local;

/* Solve options.
 *   mode SYNC: one grid barrier per sweep, every local solve of sweep k reads
 *     x^k (Sec. 2.1, Sec. 3.4 synchronous); stops at the first k with
 *     ||b - A x^k|| < tol ||b|| and returns x^k.
 *   mode ASYNC: persistent kernel without a barrier; each subdomain reads the
 *     current neighbour values (Sec. 2.1, Sec. 3.4 asynchronous).  Stops when
 *     the detector (detect) sees every subdomain locally converged
 *     (||r_p||^2 < tol^2 ||b_p||^2, Sec. 3.3.2, eq. local_conv); the global
 *     criterion is then verified and the iteration resumes if it fails.
 *   mode ORDERED: the asynchronous kernel run by one workgroup visiting the
 *     subdomains in order (restricted multiplicative Schwarz; deterministic).
 *   max_sweeps: sweeps (SYNC) or local solves per subdomain (ASYNC/ORDERED).
 *   max_seconds <= 0: no time limit.  workgroups: 0 = library choice.
 *   team: workgroups cooperating on one subdomain's CG solve (1, 2, 4, 8 or
 *     16); 0 = the value found by ras_autotune, else a heuristic.
 *   pace (ASYNC only, at most 16): before reading its neighbours' values
 *     for the next update, a subdomain that has completed more updates than
 *     some neighbour waits for it, at most pace times the duration of its own
 *     previous update, then reads whatever is there.  0 never waits (free
 *     running).  Any value leaves the iteration asynchronous (Sec. 2.1: any
 *     read schedule is admissible); it only chooses when the read happens, so
 *     that evenly loaded subdomains read their neighbours' latest update
 *     rather than the one before it.  Negative: library choice (0.25 for the
 *     Cholesky solvers, 0 for CG).  Ignored by SYNC and ORDERED.
 *   detect_factor (ASYNC and ORDERED): the detector tests the local and
 *     global criteria against detect_factor * tol, while the verification
 *     that follows every stop (Sec. 3.3.2) always uses tol.  A factor above 1
 *     makes the detector fire before the tolerance is reached, so the
 *     verification fails and the iteration resumes: it exercises the resume
 *     path (info.launches > 1) and costs extra launches.  A factor below 1
 *     delays the detector.  0 means 1; negative or NaN is RAS_E_ARG.  Ignored
 *     by SYNC, whose stop is the exact residual of every sweep.  */
enum { RAS_MODE_SYNC = 0, RAS_MODE_ASYNC = 1, RAS_MODE_ORDERED = 2 };
/* Detectors of the asynchronous mode.  CENTRAL (Sec. 2.2): every subdomain's
 * latest local criterion holds and the sum of the latest owned residuals is
 * below tol^2 ||b||^2.  DECENTRAL (Sec. 2.2, Sec. 3.3.2): neighbour flags and
 * flooding.  ESTIMATE (a library option, not the paper's): every subdomain has
 * updated since the launch and the sum of the latest owned residuals is below
 * tol^2 ||b||^2; it does not wait for the slowest local criterion.  Every
 * detector's stop is verified exactly and the iteration resumes if it fails.  */
enum { RAS_DETECT_CENTRAL = 0, RAS_DETECT_DECENTRAL = 1, RAS_DETECT_ESTIMATE = 2 };
typedef struct ras_solve_opts {
    int32_t mode;
    int32_t detect;
    double tol;
    int64_t max_sweeps;
    double max_seconds;
    int32_t workgroups;
    int32_t team;
    double pace;
    double detect_factor;
} ras_solve_opts;

typedef struct ras_solve_info {
    int32_t converged;
    int32_t launches;          /* persistent-kernel launches (resumes after failed verification + 1) */
    int64_t sweeps;            /* SYNC: updates applied; ASYNC: max local solves of any subdomain */
    int64_t total_local_solves;
    int64_t min_local_solves;
    int64_t max_local_solves;
    double rel_residual;       /* exact float64 ||b - A x|| / ||b|| recomputed after the stop */
    double seconds;            /* device time of the solve (first launch to verified stop) */
    double kernel_seconds;     /* device time inside the persistent kernel launches only */
} ras_solve_info;

/* Host-side setup summary. */
typedef struct ras_plan_stats {
    int64_t n;
    int64_t nnz;
    int32_t parts;
    int32_t max_ell_width;
    int64_t sum_local_rows;    /* sum_p |Omega_p| */
    int64_t min_local_rows;
    int64_t max_local_rows;
    int32_t max_band;          /* max stored lower half-bandwidth (>= 1) of the local matrices */
    int32_t reserved;
    int64_t band_entries;      /* factor entries: sum_p |Omega_p| (w_p + 1); sparse solver: sum_p nnz(L_p) */
    int64_t device_bytes;      /* device memory the handle allocates for the matrix data */
} ras_plan_stats;

typedef struct ras_plan ras_plan;
typedef struct ras_handle ras_handle;

/* ---- host-only setup (no GPU needed; Sec. 3.2) ---------------------------------
 * Validates A, partitions (Sec. 3.2.1), grows each owned set by `overlap`
 * breadth-first layers over A's pattern (Sec. 2.1, Fig. 1), orders each local
 * set by ascending global id, extracts the local matrices (Sec. 3.2.2) and,
 * for the Cholesky solver, factors them in float64 (Sec. 3.3.1).  */
ras_status ras_plan_create(const ras_csr* A, const ras_partition* part, int32_t overlap, const ras_local* local,
                           ras_plan** out);
ras_status ras_plan_get_stats(const ras_plan* plan, ras_plan_stats* out);
/* Index sets: owner[n] (int32), omega_ptr[P+1] (int64), omega_idx[sum |Omega_p|]
 * (int32, ascending per subdomain).  Any output may be NULL.  */
ras_status ras_plan_sets(const ras_plan* plan, int32_t* owner, int64_t* omega_ptr, int32_t* omega_idx);
/* Communication volume between subdomains (Sec. 3.2.1, Fig. 2): volume is a
 * caller-owned int64 array of P*P entries, row-major; volume[p*P + q] (q != p)
 * receives the number of distinct points of Omega_p and of its external layer
 * ext(Omega_p) (the columns Omega_p's rows reach outside Omega_p) that are owned
 * by subdomain q, i.e. the values subdomain p reads from q for one local solve.
 * The diagonal is 0.  RAS_E_ARG on a NULL argument.  */
ras_status ras_plan_comm_volume(const ras_plan* plan, int64_t* volume);
/* Float64 band factor of subdomain p: band[i*(w+1) + (j - i + w)] = L_ij for
 * i-w <= j <= i (zero outside the matrix); *w receives the stored half-bandwidth
 * (the local matrix's, at least 1: a diagonal matrix keeps a zero sub-diagonal).
 * band may be NULL to query w (any local solver); with band non-NULL the
 * call returns RAS_E_STATE unless the solver is Cholesky.  */
ras_status ras_plan_factor(const ras_plan* plan, int32_t p, double* band, int32_t* w);
/* FP16_ROWSCALED storage of subdomain p's factor, in the same band layout:
 * half_bits[i*(w+1) + o] = float16 bits of L_ij / scale[i] (round to nearest
 * even from float64), scale[i] = float32(max_j |L_ij|) (1 for an all-zero row).
 * RAS_E_STATE unless the solver is Cholesky with FP16_ROWSCALED storage.  */
ras_status ras_plan_factor_fp16(const ras_plan* plan, int32_t p, uint16_t* half_bits, float* scale);
/* Sparse factor of subdomain p (CHOL_SPARSE plans; RAS_E_STATE otherwise):
 * perm[n] gives, for each elimination step k, the position in Omega_p (as
 * returned by ras_plan_sets) of the local row eliminated at step k; the
 * strictly lower part of L (rows in elimination order) is returned in CSR form
 * row_ptr[n+1], col[nnz], val[nnz] with columns ascending in each row, and
 * diag[n] holds L_kk, so that L L^T = P A_p P^T with (P A_p P^T)_{kl} =
 * (A_p)_{perm[k], perm[l]}.  *nnz receives the entry count; every array may
 * be NULL (query).  */
ras_status ras_plan_sparse_factor(const ras_plan* plan, int32_t p, int32_t* perm, int64_t* row_ptr, int32_t* col,
                                  double* val, double* diag, int64_t* nnz);
/* Solve schedule of subdomain p's sparse factor for one pass (0: forward with
 * L, 1: backward with L^T), as the device applies it (CHOL_SPARSE plans;
 * RAS_E_STATE otherwise).  Level scheduling of the triangular solves (Sec.
 * 3.3.1), with every dense diagonal block of at least *min_block rows (0:
 * none) solved in two steps by the partitioned-inverse form: its rows first
 * subtract their products with rows outside the block, then take their dot
 * products with the explicit inverse of the block's triangle.  Value slots 0..n-1
 * are the local vector in elimination order (ras_plan_sparse_factor's perm),
 * slots n..n+*slots-1 hold block partial results between the two steps.  The
 * records of step s are step_ptr[s] .. step_ptr[s+1]-1; record r writes slot
 * meta[4r] with the sum over entries e in [meta[4r+1], meta[4r+2]) of
 * val[e] * slot[col[e]] (meta[4r+3] = 0), reading only slots written in earlier
 * steps (or the vector's initial values).  Every pointer may be NULL (query
 * the counts first): *nsteps, *nrec records, *nent entries.  */
ras_status ras_plan_sparse_schedule(const ras_plan* plan, int32_t p, int32_t pass, int32_t* nsteps, int64_t* nrec,
                                    int64_t* nent, int32_t* slots, int32_t* min_block, int32_t* step_ptr,
                                    int32_t* meta, int32_t* col, double* val);
/* The same pass in the device's layout: the records of each step dealt out to
 * the 64 lanes of each of *waves waves (one workgroup).  Wave w streams rounds
 * wave[2w] .. wave[2w] + wave[2w+1] - 1, round r holding one item per lane,
 * (col[64r + lane], val[64r + lane]); the device stores col in 16 bits.  An
 * item with col < 0xfffe adds val * slot[col] to the lane's sum; col = 0xfffe
 * is a terminator, present in every lane of a group of 2^g consecutive lanes
 * in the same round, whose value's low 32 bits hold s | g << 24: the group's
 * sums are added, the total written to slot s and the sums cleared; a round
 * with col = 0xffff in every lane ends the wave's part of a step (the
 * workgroup synchronises; sums are cleared).  *nitems receives the item count
 * (a multiple of 64); the arrays may be NULL (query).  */
ras_status ras_plan_sparse_lanes(const ras_plan* plan, int32_t p, int32_t pass, int32_t* waves, int64_t* nitems,
                                 int32_t* wave, int32_t* col, double* val);
/* Largest subdomain (local rows) the sparse Cholesky solver accepts for a
 * storage kind (FP64 or FP32), or 0 for a storage it does not support.  */
int64_t ras_sparse_max_rows(int32_t storage);
void ras_plan_destroy(ras_plan* plan);

/* ---- device setup and solve ------------------------------------------------------
 * ras_setup = ras_plan_create + upload; the handle owns every device array it
 * allocates.  hip_stream may be NULL (default stream).  */
ras_status ras_setup(const ras_csr* A, const ras_partition* part, int32_t overlap, const ras_local* local,
                     void* hip_stream, ras_handle** out);
/* Host-forced stall and cancel of asynchronous solves (fault injection and
 * control, callable from another thread while ras_solve runs; the words are
 * pinned, coherent host memory that the running kernel polls).
 * ras_pause: while paused != 0, subdomain p takes no updates in ASYNC mode
 * (a pause set before the solve holds from its start, one set during it
 * within a few updates; the kernel polls the words on every 8th visit of a
 * workgroup's subdomains and on every visit after a stall; its neighbours
 * keep reading its last values; a detector's stop is still
 * verified exactly, so a stall cannot end the solve as converged unless the
 * iterate meets the tolerance); the setting persists across solves until
 * cleared.  Such a solve ends only once the subdomain is
 * resumed, at max_seconds, or when cancelled, so give it a time limit.  SYNC
 * and ORDERED modes ignore pauses.
 * ras_cancel: the ASYNC solve running on the handle stops within a few
 * updates and returns like a time limit (RAS_NOT_CONVERGED with the current
 * iterate); every solve clears the request when it starts.
 * RAS_E_ARG for a null handle or p out of range.  */
ras_status ras_pause(ras_handle* h, int32_t p, int32_t paused);
ras_status ras_cancel(ras_handle* h);
/* Uploads a plan; the plan stays owned by the caller.  */
ras_status ras_setup_from_plan(const ras_plan* plan, void* hip_stream, ras_handle** out);
ras_status ras_handle_get_stats(const ras_handle* h, ras_plan_stats* out);

/* Solves A x = b for nrhs right-hand sides (Alg. 1's SOLVE).  x_dev holds the
 * initial guess on entry and the result on return; info[nrhs].  Blocks the
 * calling thread until the result is on the device and info is filled.  */
ras_status ras_solve(ras_handle* h, const double* b_dev, double* x_dev, int32_t nrhs, const ras_solve_opts* opts,
                     ras_solve_info* info);

/* For callers that cannot allocate device memory during a solve (code that
 * runs under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same solve as ras_solve -- same arguments, kernels, results
 * and status codes -- whose workspace (work tables, per-subdomain state, the
 * synchronous second iterate, asynchronous snapshots, local vectors, residual
 * history) is carved from a fixed device array of RAS_NOALLOC_SCRATCH_BYTES
 * bytes that the library holds on every device it runs on, until the process
 * ends.  The call allocates and frees no device memory.  A solve whose
 * workspace does not fit returns RAS_E_NOMEM, naming the bytes needed and
 * available, before any device work.  The workspace is about 8 bytes per
 * local row per right-hand side, plus 8 bytes per unknown (SYNC's second
 * iterate) or per snapshot slot (ASYNC), plus 16 bytes per history entry
 * (min(max_sweeps + 1, 2^20) entries SYNC, min(max_sweeps + 1, 2^16) ASYNC).
 * Every call on one device uses that device's one array, which keeps the last
 * call's contents (everything a solve reads is written or cleared by the
 * solve first): calls that overlap in time on one device -- from several host
 * threads or on several streams -- race and must be serialised by the caller.  */
enum { RAS_NOALLOC_SCRATCH_BYTES = 32 * 1024 * 1024 };
ras_status ras_solve_noalloc(ras_handle* h, const double* b_dev, double* x_dev, int32_t nrhs,
                             const ras_solve_opts* opts, ras_solve_info* info);

/* Several systems (handles) in one persistent launch; handles must share the
 * local solver kind and storage.  b[i], x[i] are device arrays of handle i
 * with nrhs[i] right-hand sides; info has sum(nrhs) entries, in order.  */
ras_status ras_batch_solve(int32_t m, ras_handle* const* hs, const double* const* b_dev, double* const* x_dev,
                           const int32_t* nrhs, const ras_solve_opts* opts, ras_solve_info* info);

/* Residual history of right-hand side `rhs` of the last solve: SYNC, one entry
 * per sweep (exact ||b - A x^k|| / ||b||); ASYNC, one entry per detector
 * check (estimate from the latest subdomain residuals, a mix of times) and a
 * final exact entry per verification.  t_sec (may be NULL) gets seconds since
 * the first launch.  *len = entries available; at most cap are copied.  */
ras_status ras_residual_history(const ras_handle* h, int32_t rhs, double* t_sec, double* relres, int64_t cap,
                                int64_t* len);
/* Local solves completed by each subdomain in the last solve (Sec. 4.5/4.6,
 * "subdomain update" counts); counts[P].  */
ras_status ras_local_solve_counts(const ras_handle* h, int32_t rhs, int64_t* counts);
ras_status ras_partition_sets(const ras_handle* h, int32_t* owner, int64_t* omega_ptr, int32_t* omega_idx);
/* Where the last solve's time went, per subdomain (the per-function runtime
 * breakdown of Sec. 4.2-4.6), measured with the device wall clock by the
 * workgroup owning the subdomain: seconds[4*p + k] for k = 0 restriction and
 * residual (the asynchronous read snapshot included), 1 local solve, 2
 * restricted prolongation and publication of the owned values, 3 everything
 * else (SYNC: waiting at the sweep barrier and the convergence check, charged
 * to the first subdomain of each workgroup; ASYNC: paced waits before reads and
 * detection work).  seconds has 4 P entries.  */
ras_status ras_phase_seconds(const ras_handle* h, int32_t rhs, double* seconds);
/* Autotuner: times `sweeps` synchronous sweeps from x = 0 for every feasible CG
 * team size (workgroups per subdomain), twice each (the faster timing counts:
 * a kernel variant's first launch carries one-time costs), and keeps the fastest in the handle (used
 * when ras_solve_opts.team is 0) and in a process-wide cache keyed by the
 * problem shape, so later handles of the same shape start tuned.  x_dev is
 * overwritten (work space).  best_team / best_ms_per_sweep may be NULL.  The
 * banded solver has one configuration: it returns team 1.  */
ras_status ras_autotune(ras_handle* h, const double* b_dev, double* x_dev, int32_t sweeps, int32_t* best_team,
                        double* best_ms_per_sweep);
/* The banded Cholesky factor of subdomain p as the solves use it, read back
 * from the device (Sec. 3.3.1: computed once at setup -- by ras_setup on the
 * device, in float64, then stored in the handle's storage type):
 * band[i*(w+1) + (j - i + w)] = L_ij as float64 (FP32 entries widened, FP16
 * entries times their row scale; the diagonal is the reciprocal of the stored
 * 1 / L_ii); *w receives the half-bandwidth.  band may be NULL to query w.
 * RAS_E_STATE unless the local solver is CHOL_BANDED; RAS_E_ARG for p out of
 * range.  */
ras_status ras_handle_factor(const ras_handle* h, int32_t p, double* band, int32_t* w);
/* Exact ||b - A x|| / ||b|| of device vectors (the post-termination check of
 * Sec. 3.3.2), computed by the library's verification kernel.  */
ras_status ras_relative_residual(ras_handle* h, const double* b_dev, const double* x_dev, double* relres);
void ras_destroy(ras_handle* h);

/* ---- serving: continuous batching ----------------------------------------------
 * A server admits submitted systems while the device memory they need fits in
 * hbm_budget bytes, sets them up (host planning on its own thread, so setup of
 * newcomers overlaps device work), and advances every admitted system together
 * in time-sliced batched asynchronous launches of slice_seconds each; systems
 * that arrive while others run join at the next slice.  A system retires as soon
 * as its verified relative residual is below its tolerance; its device memory
 * is released at once and its result waits for ras_server_poll.  A system
 * larger than the whole budget is rejected (RAS_E_NOMEM) at submission.
 * Local solver, partition and overlap are per system; systems with the same
 * local solver share one launch per slice.  All calls are thread-safe.  */
typedef struct ras_server ras_server;
typedef struct ras_server_stats {
    int64_t submitted;
    int64_t completed;
    int64_t queued;            /* submitted, not yet admitted */
    int64_t active;            /* admitted, not yet retired */
    int64_t slices;            /* batched launches issued */
    int64_t in_use_bytes;      /* device memory held by admitted systems */
    int64_t peak_in_use_bytes;
    int64_t budget_bytes;
    double device_seconds;     /* time inside slices */
} ras_server_stats;

ras_status ras_server_create(int64_t hbm_budget, double slice_seconds, void* hip_stream, ras_server** out);
/* Copies A, the partition and b_host[nrhs * n]; returns a ticket at once.  */
ras_status ras_server_submit(ras_server* srv, const ras_csr* A, const ras_partition* part, int32_t overlap,
                             const ras_local* local, const double* b_host, int32_t nrhs, double tol,
                             uint64_t* ticket);
/* RAS_PENDING until the system has retired; then copies x_host[nrhs * n] and
 * info[nrhs] (either may be NULL), the latency from submission to retirement,
 * and releases the result.  An error during setup or solve is returned here.  */
ras_status ras_server_poll(ras_server* srv, uint64_t ticket, double* x_host, ras_solve_info* info,
                           double* latency_seconds);
/* Blocks until the ticket has retired (RAS_OK) or timeout_seconds elapse (RAS_PENDING).  */
ras_status ras_server_wait(ras_server* srv, uint64_t ticket, double timeout_seconds);
ras_status ras_server_get_stats(ras_server* srv, ras_server_stats* out);
/* Stops the server: pending systems are dropped, threads joined, memory freed.
 * NULL-safe; returns RAS_OK, or RAS_E_HIP if releasing the server's own stream
 * failed (the server is gone either way).  */
ras_status ras_server_destroy(ras_server* srv);

/* ---- the stop rule after a persistent asynchronous launch (host only) ----------
 * Sec. 3.3.2: the detector inside the kernel decides from local criteria and
 * the latest (mixed-time) subdomain residuals, so after the launch the host
 * recomputes the exact global relative residual and decides, per right-hand
 * side, what follows.  ras_solve applies exactly this rule; it is exported so
 * that it can be checked without a GPU.
 * kernel_stop: why the kernel stopped this right-hand side (RAS_KSTOP_*);
 * verified_relres: exact ||b - A x|| / ||b|| after the launch; tol: the
 * solve's tolerance; min_local_solves: fewest local solves of any of its
 * subdomains so far; max_sweeps / max_seconds: the solve options' limits
 * (max_seconds <= 0: none); elapsed_seconds: device time since the first
 * launch; ordered: nonzero for mode ORDERED (which runs its passes once).
 * Returns, in this order of precedence:
 *   RAS_STEP_DIVERGED  kernel_stop is DIVERGED or the residual is not finite;
 *   RAS_STEP_CONVERGED verified_relres < tol;
 *   RAS_STEP_LIMIT     min_local_solves >= max_sweeps, a time limit hit (in the
 *                      kernel or after it), or ordered;
 *   RAS_STEP_RESUME    otherwise: clear the detector's flags, launch again
 *                      from the current x.
 * ras_final_status maps a final step to the status ras_solve returns
 * (CONVERGED -> RAS_OK, LIMIT -> RAS_NOT_CONVERGED, DIVERGED ->
 * RAS_E_DIVERGED; RESUME -> RAS_E_STATE, it is not final).  */
enum { RAS_KSTOP_RUNNING = 0, RAS_KSTOP_DETECTED = 1, RAS_KSTOP_TIME = 2, RAS_KSTOP_EXHAUSTED = 3,
       RAS_KSTOP_DIVERGED = 4 };
enum { RAS_STEP_CONVERGED = 0, RAS_STEP_RESUME = 1, RAS_STEP_DIVERGED = 2, RAS_STEP_LIMIT = 3 };
int32_t ras_async_next_step(int32_t kernel_stop, double verified_relres, double tol, int64_t min_local_solves,
                            int64_t max_sweeps, double elapsed_seconds, double max_seconds, int32_t ordered);
ras_status ras_final_status(int32_t step);

const char* ras_last_error(void);
/* Library version string. */
const char* ras_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RAS_H */

/*
 * ipi.h — C ABI of libipi.so: inexact policy iteration (iPI) for discounted
 * finite MDPs on AMD Instinct MI355X (gfx950).
 *
 * Method: "Inside madupite: Technical Design and Performance" (arXiv
 * 2507.22538).  An MDP is the tuple {S, A, P, g, gamma} of Sec. II: P(s,s',a)
 * row-stochastic for every (s,a), stage costs g(s,a), 0 < gamma < 1.  The
 * library returns the optimal cost V* (fixed point of the Bellman optimality
 * equation, Sec. II) and a greedy policy pi* (greedy-policy equation), using
 * the general iPI scheme of Algorithm 1 (Sec. III-A) with the option names of
 * Table 1.
 *
 * Conventions for every entry point:
 *   - All sizes are 64-bit where they can exceed 2^31; states and actions
 *     are 0-based.
 *   - P is passed row-stacked (flattened-tensor equation, Sec. III-B.2):
 *     CSR of shape (S*A) x S, row s*A + a holds P(s, ., a); columns sorted
 *     ascending within a row.  g is dense, row-major, index s*A + a.
 *   - Arrays passed to ipi_bellman / ipi_solve / ipi_solve_batch are DEVICE
 *     pointers (memory of the current HIP device), caller-owned.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   - No exception crosses the ABI.  Every call returns an ipi_status; on
 *     failure ipi_last_error() returns a thread-local message.  Failed calls
 *     leak nothing.
 */
#ifndef IPI_H
#define IPI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ipi_status {
    IPI_OK = 0,
    IPI_E_INVALID_ARG = 1,    /* bad size, pointer, option or CSR structure      */
    IPI_E_NOT_STOCHASTIC = 2, /* negative/non-finite P entry or row sum != 1     */
    IPI_E_OOM = 3,            /* device allocation failed                        */
    IPI_E_DEVICE = 4,         /* HIP runtime error                               */
    IPI_E_NOT_CONVERGED = 5,  /* iteration cap hit; outputs still written         */
    IPI_E_NUMERICAL = 6,      /* non-finite residual                             */
    IPI_E_TOO_LARGE = 7,      /* request exceeds the server's HBM budget          */
    IPI_E_CANCELLED = 8,      /* server request cancelled                        */
    IPI_E_NOT_FOUND = 9,      /* unknown server ticket                           */
    IPI_E_PENDING = 10        /* server request not finished yet                 */
} ipi_status;

/* ------------------------------------------------------------------------ */
/* MDP object (Sec. III-B.2: the MDP class holding P, g and the options)    */
/* ------------------------------------------------------------------------ */

typedef struct ipi_mdp_s* ipi_mdp_t;

/* create flags */
#define IPI_DEVICE_PTRS 0x1u /* row_ptr/col/val/g are device pointers (else host)      */
#define IPI_VAL_FP32 0x2u    /* also keep a float32 copy of P's values (mixed mode)    */
#define IPI_FP32_ORIGIN 0x4u /* data came from float32: row-sum tolerance 1e-6         */
#define IPI_BORROW 0x8u      /* with IPI_DEVICE_PTRS: use the caller's arrays in place  */
#define IPI_NO_VALIDATE 0x10u /* skip the structural/stochastic checks                */
#define IPI_VAL_FP32_ONLY 0x20u /* keep only a float32 copy of P's values: about 2/3 of the
                                  memory; fp32_mixed solves and passes only (fp64 and
                                  fp32_inner fail with IPI_E_INVALID_ARG); host values are
                                  converted on the host and never uploaded in FP64      */
#define IPI_VAL_SPLIT 0x40u /* keep P's values as two float32 arrays instead of FP64:
                               hi = float32(P) and lo = float32(P - hi), 8 bytes a value
                               (IPI_VAL_FP32 keeps 12).  A Bellman pass in FP64 arithmetic
                               reads both and uses hi + lo (rounded once to FP64; hi + lo
                               lies within max(2^-48 |P|, 2^-150) of P), the inner products of fp32_inner and
                               everything in fp32_mixed read hi.  fp32_inner and fp32_mixed
                               solves, FP64 and fp32_mixed Bellman passes; fp64 solves,
                               batch members other than fp32_mixed and ipi_autotune other
                               than for fp32_mixed fail with IPI_E_INVALID_ARG.  The FP64 values are uploaded (or read
                               from the caller's device arrays), split on the device and
                               not kept.  Not with IPI_VAL_FP32_ONLY.                   */

/*
 * ipi_mdp_create_csr — build an MDP from row-stacked CSR (flattened-tensor
 * equation, Sec. III-B.2) plus g and gamma (tuple of Sec. II).
 *
 *   S, A      number of states / actions (1 <= S < 2^31, 1 <= A <= 3072)
 *   nnz       number of stored entries of P (= row_ptr[S*A])
 *   row_ptr   int64[S*A+1], row_ptr[0] = 0, non-decreasing
 *   col       int32[nnz], 0 <= col < S, ascending inside each row
 *   val       float64[nnz], finite, >= 0, each row sums to 1 within
 *             1e-12*max(1, row length) (1e-6 with IPI_FP32_ORIGIN)
 *   g         float64[S*A], finite (large finite costs such as 1e20 allowed)
 *   gamma     discount, 0 < gamma < 1
 *   flags     IPI_* create flags above
 *   stream    stream used for uploads; the call returns after the data is
 *             resident (host inputs may be freed on return)
 *   out       receives the handle
 *
 * Ownership: the library copies the inputs into device memory it owns
 * (except with IPI_BORROW, where the caller keeps the device arrays alive
 * and unchanged until ipi_mdp_destroy).  Errors: IPI_E_INVALID_ARG,
 * IPI_E_NOT_STOCHASTIC, IPI_E_OOM, IPI_E_DEVICE.
 */
ipi_status ipi_mdp_create_csr(int64_t S, int32_t A, int64_t nnz, const int64_t* row_ptr,
                              const int32_t* col, const double* val, const double* g,
                              double gamma, uint32_t flags, void* stream, ipi_mdp_t* out);

/* Release every device buffer of the MDP (NULL is a no-op). */
ipi_status ipi_mdp_destroy(ipi_mdp_t mdp);

typedef struct ipi_mdp_desc {
    int64_t S;
    int32_t A;
    int64_t nnz;
    int32_t k_min, k_max;   /* shortest / longest row of P                  */
    int32_t uniform_k;      /* 1 if every row has k_min entries             */
    int32_t row_ptr_bytes;  /* 4 or 8: index width stored on the device     */
    int32_t has_fp32;       /* float32 value copy present                   */
    int32_t band;           /* 1 if every row's columns are consecutive (band form) */
    double gamma;
    int64_t device_bytes;   /* device memory held by the MDP (data + workspace) */
    int32_t has_fp64;       /* FP64 values held (0 with IPI_VAL_FP32_ONLY)  */
    double fp32_row_perturbation; /* max over rows of sum_j |P_rj - float32(P_rj)|, measured
                                     when the float32 copy is made (0 without one) */
    int32_t stencil_patterns; /* stencil form (rows of one length, not a band): every row's
                                 columns are its first column plus one of this many offset
                                 patterns (at most 8; e.g. bilinear grid rows c, c+1, c+N,
                                 c+N+1 and their wrapped variant), and the Bellman pass and
                                 the P_pi products (wave tiles) read one 4-byte word per row
                                 instead of the column indices; 0 when not detected */
    int32_t stencil_pairs;    /* 1 when every stencil pattern's columns come in adjacent
                                 pairs (c, c+1, ...: the bilinear rows), so the Bellman pass
                                 and the products load each pair of entries with one
                                 16-byte load; else 0 */
    int32_t has_split;        /* 1 with IPI_VAL_SPLIT: values held as float32 hi + lo      */
    double split_row_perturbation; /* max over rows of sum_j |P_rj - (hi_rj + lo_rj)|, the
                                      sum rounded once to FP64 (0 without the split)      */
} ipi_mdp_desc;

ipi_status ipi_mdp_describe(ipi_mdp_t mdp, ipi_mdp_desc* out);

/* ------------------------------------------------------------------------ */
/* Options (Table 1 names; Table 2 presets are combinations of these)       */
/* ------------------------------------------------------------------------ */

/* Precision modes.  Every accumulation, the Krylov basis, Gram-Schmidt, the
 * Hessenberg least squares, the residual norms and the stopping tests are
 * FP64 in all three; they differ in which P values the kernels read.
 *   IPI_FP64        P in FP64 everywhere.
 *   IPI_FP32_MIXED  P values stored as float32 (IPI_VAL_FP32) and read, exactly
 *                   up-converted, by the Bellman pass and the inner products:
 *                   the solve targets the MDP with float32-rounded P; its
 *                   distance to the FP64 MDP's V* is stated per result
 *                   (ipi_solve_info.err_bound, from one FP64 Bellman pass on
 *                   the returned V).
 *   IPI_FP32_INNER  the Bellman pass (greedy policy, residual, stopping test)
 *                   reads the FP64 values, the inner solve a float32 P_pi
 *                   (Algorithm 1's inexact evaluation): the solve targets the
 *                   FP64 MDP itself; the inner products move the float32 bytes. */
typedef enum ipi_precision { IPI_FP64 = 0, IPI_FP32_MIXED = 1, IPI_FP32_INNER = 2 } ipi_precision;
typedef enum ipi_inner {
    IPI_INNER_GMRES = 0,
    IPI_INNER_RICHARDSON = 1,
    IPI_INNER_TFQMR = 2,
    IPI_INNER_BICGSTAB = 3
} ipi_inner;
typedef enum ipi_pc { IPI_PC_NONE = 0, IPI_PC_JACOBI = 1 } ipi_pc;
typedef enum ipi_mode { IPI_MINCOST = 0, IPI_MAXREWARD = 1 } ipi_mode;

typedef struct ipi_solve_opts {
    double atol;             /* -atol_pi: stop when ||V - TV||_inf <= atol (1e-8)        */
    double rtol_cert;        /* -rtol_cert: also stop when ||V-TV||_inf <= rtol_cert*(1-gamma)*||V||_inf
                                (0 = off); bounds ||V - V*||_inf / ||V||_inf by rtol_cert */
    double alpha;            /* -alpha: inner forcing, stop when ||lin. residual||_2 < alpha*||V-TV||_inf (1e-4) */
    int32_t max_outer;       /* -max_iter_pi: at most this many policy evaluations (1000) */
    int32_t max_inner;       /* -max_iter_ksp / -ksp_max_it: inner iterations per evaluation (1000):
                                GMRES Arnoldi steps, Richardson sweeps, TFQMR half steps,
                                BiCGStab iterations (one or two J_pi products each)         */
    int32_t inner;           /* -ksp_type: gmres | richardson | tfqmr | bicgstab (gmres).
                                TFQMR tests its quasi-residual bound sqrt(k+1) tau_k, an
                                upper bound of the true residual 2-norm; TFQMR and BiCGStab
                                fall back to one Richardson step when they end unconverged
                                with a residual above the starting one                     */
    int32_t pc;              /* -pc_type: none | jacobi (none)                            */
    double richardson_scale; /* -ksp_richardson_scale (1.0)                               */
    int32_t gmres_restart;   /* -ksp_gmres_restart (30, at most 64)                       */
    int32_t precision;       /* -precision: fp64 | fp32_mixed | fp32_inner (fp64)          */
    int32_t reorth;          /* -ksp_gmres_cgs_passes: 1 or 2 Gram-Schmidt passes (1)     */
    int32_t mode;            /* -mode: MINCOST | MAXREWARD (MINCOST)                      */
    int32_t profile;         /* record device times into ipi_solve_info: 0 off, 1 every
                              * Bellman pass and every 16th timed unit of P_pi products
                              * (a GMRES / TFQMR / BiCGStab product, or the Richardson
                              * sweeps between two stopping tests), 2 every unit (the
                              * events slow the solve a little) (0)                 */
    const double* v0;        /* initial V_0 (device, S entries) or NULL for V_0 = 0        */
    int32_t richardson_block; /* -ksp_richardson_block: 1 = run the Richardson sweeps between
                              * two stopping tests (4, 8 or 16) in one launch whenever P_pi is in
                              * the band form and its rows read a short window around their
                              * state (temporal blocking; the same iterates bit for bit, P_pi
                              * read about once per launch), else one launch per sweep;
                              * 0 = always one launch per sweep (1)                      */
} ipi_solve_opts;

/* Fill the Table 1 defaults. */
void ipi_opts_default(ipi_solve_opts* opts);

/* Set one option by its Table 1 / PETSc-style name, with or without the
 * leading '-' (e.g. "-ksp_type", "richardson").  IPI_E_INVALID_ARG on an
 * unknown name or a value out of range (alpha in (0,1), caps >= 1, ...). */
ipi_status ipi_opts_set(ipi_solve_opts* opts, const char* name, const char* value);

typedef struct ipi_solve_info {
    int32_t outer_iters;     /* policy evaluations performed                           */
    int32_t converged;       /* 1 if ||V - TV||_inf met the stopping rule               */
    int64_t inner_iters;     /* inner iterations (Arnoldi steps / sweeps) in total      */
    double final_rho;        /* ||V - TV||_inf of the returned V                        */
    double device_ms;        /* wall time of the solve on the stream                    */
    double alg_bytes;        /* algorithmic HBM bytes of all kernels launched           */
    int32_t precision;
    int32_t inner;
    int32_t bellman_calls;   /* fused Bellman passes of Algorithm 1 (fp32_mixed's final FP64
                                pass for fp64_rho is not counted or timed)                */
    int32_t ppi_cached;      /* P_pi loaded through the caches: bit 0 in the one-sweep products (wave
                                tiles), bit 1 in the blocked Richardson sweeps (ipi_tuning.ppi_cached) */
    double bellman_ms;       /* summed device time of those passes (opts.profile)       */
    double bellman_bytes;    /* algorithmic bytes of one pass                           */
    double inner_ms;         /* summed device time of the inner solves (opts.profile)   */
    double inner_resid;      /* last inner residual 2-norm (GMRES: its estimate |g_{j+1}|) */
    int64_t product_calls;   /* P_pi product launches timed (opts.profile; a sample)     */
    double product_ms;       /* their summed device time (HIP events around each launch) */
    double product_bytes;    /* their summed algorithmic bytes                            */
    double fp64_rho;         /* ||V - T V||_inf of the returned V with the FP64 values of P:
                                final_rho, except in fp32_mixed, where one extra FP64 Bellman
                                pass computes it (NaN if the MDP holds no FP64 values; with
                                IPI_VAL_SPLIT the pass on hi + lo)                          */
    double err_bound;        /* certified bound on ||V - V*||_inf for the MDP as given
                                (contraction of T, Sec. II): fp64_rho / (1 - gamma); without
                                FP64 values (IPI_VAL_FP32_ONLY) (final_rho + gamma dP ||V||_inf)
                                / (1 - gamma), dP = fp32_row_perturbation; with IPI_VAL_SPLIT
                                (fp64_rho + gamma dS ||V||_inf) / (1 - gamma),
                                dS = split_row_perturbation                                  */
    int64_t block_launches;  /* Richardson launches that ran 4, 8 or 16 sweeps each (richardson_block) */
    int32_t block_sweeps;    /* the most sweeps one of those launches ran (0 if none), and of the
                                timed launches (opts.profile) among them that ran that many:  */
    int64_t block_calls;     /* the number,                                                  */
    double block_ms;         /* their summed device time and                                 */
    double block_bytes;      /* their summed algorithmic bytes (P_pi and the vectors once)   */
} ipi_solve_info;

/* ------------------------------------------------------------------------ */
/* Hot kernels and the solve                                                */
/* ------------------------------------------------------------------------ */

/*
 * ipi_bellman — one fused pass of the Bellman operator (Sec. II; greedy
 * extraction "approach 2" of Sec. III-B.3, without materialising P V):
 *   Q(s,a)  = g(s,a) + gamma * sum_{s'} P(s,s',a) V(s')   (FP64 accumulation)
 *   TV[s]   = min_a Q(s,a)
 *   pi[s]   = lowest a attaining the minimum
 *   resid[s]= TV[s] - V[s]      (= -r(V)[s]; may be NULL)
 *   rho[0]  = max_s |TV[s] - V[s]| = ||r(V)||_inf   (may be NULL)
 * All pointers are device pointers of S entries (rho: 1).  precision
 * IPI_FP32_MIXED reads the float32 value copy (requires IPI_VAL_FP32).
 * Asynchronous on `stream`.
 */
ipi_status ipi_bellman(ipi_mdp_t mdp, const double* V, double* TV, int32_t* pi, double* resid,
                       double* rho, int32_t precision, void* stream);

/*
 * ipi_solve — Algorithm 1 (general iPI): repeat { pi <- greedy(V_k);
 * approximately solve (I - gamma P_pi) V = g_pi, starting from V_k, with the
 * inner solver until ||lin. residual||_2 < alpha * ||r(V_k)||_inf or
 * max_inner iterations (Sec. III-B.3 replaces the inf-norm test of
 * Algorithm 1 with the solver's 2-norm); V_{k+1} <- result } until
 * ||r(V_k)||_inf <= tol or max_outer evaluations.
 *   V_out   device float64[S]; pi_out device int32[S] (greedy for V_out)
 *   info    host struct, may be NULL
 * Returns IPI_OK on convergence, IPI_E_NOT_CONVERGED at the cap (V_out,
 * pi_out and info are still written), IPI_E_NUMERICAL on a non-finite
 * residual.  Blocks the calling thread until the solve finishes.
 * Workspace (Krylov basis etc.) is allocated on first use and kept by the
 * MDP.  Calls on the same MDP must not overlap.
 */
ipi_status ipi_solve(ipi_mdp_t mdp, const ipi_solve_opts* opts, double* V_out, int32_t* pi_out,
                     ipi_solve_info* info, void* stream);

/*
 * ipi_solve_batch — n independent solves advanced together: each round of
 * three launches moves every unfinished member through one phase of its own
 * Algorithm 1 (Bellman pass, Arnoldi step, Gram-Schmidt step, update, ...),
 * with the tiles of all members in one grid; the rounds run in chunks of 32
 * replayed from a captured HIP graph, and a member leaves as soon as its own
 * solve has ended.  Each member's result does not depend on the other
 * members (bitwise).  opts has n entries (v0 ignored; inner gmres with
 * restart <= 32 or richardson; pc none; MINCOST; A <= 1024; an MDP may
 * appear once; fp32_mixed / fp32_inner members need IPI_VAL_FP32).
 * V_out[i] / pi_out[i] are device arrays of S_i entries.  statuses[i] gets
 * the per-member status; info[i].device_ms is the host time from the start
 * of the batch to the end of the chunk in which member i finished.  The call
 * itself fails only on argument or device errors.  Blocks the calling
 * thread until every member has finished.
 */
ipi_status ipi_solve_batch(int32_t n, const ipi_mdp_t* mdps, const ipi_solve_opts* opts,
                           double* const* V_out, int32_t* const* pi_out, ipi_solve_info* infos,
                           ipi_status* statuses, void* stream);

/*
 * ipi_solve_noalloc — ipi_solve for callers that cannot allocate device
 * memory (code in tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, options, results and errors as ipi_solve, and the same
 * kernels; the solve workspace (iterate vectors, Krylov basis, compact P_pi,
 * control block, reduction partials, and -g in MAXREWARD mode) is carved
 * from one fixed 64 MiB device array instead of being allocated, so the call
 * makes no hipMalloc / hipFree, creates no HIP events or graphs (GMRES cycles
 * are launched one by one; opts.profile is ignored and info->device_ms is the
 * host's wall time of the call) and leaves the MDP's own workspace untouched.
 *   Limit: the workspace of (S, k_max, restart, inner solver, precision) must
 *   fit 64 MiB (ipi_footprint_bytes minus the MDP's data gives its size; e.g.
 *   S = 1e5, k = 8, GMRES(30), FP64 needs about 40 MB); larger problems fail
 *   with IPI_E_TOO_LARGE and a message stating the bytes needed.
 *   The array lives on every device the library runs on until the process
 *   ends and keeps the last call's contents; the library clears what a solve
 *   needs zeroed.  Calls in one process are serialised (they share the
 *   array); the MDP must live on the current device (else IPI_E_INVALID_ARG).
 */
ipi_status ipi_solve_noalloc(ipi_mdp_t mdp, const ipi_solve_opts* opts, double* V_out, int32_t* pi_out,
                             ipi_solve_info* info, void* stream);

/* ------------------------------------------------------------------------ */
/* Tuning                                                                    */
/* ------------------------------------------------------------------------ */

/* Kernel configuration for one MDP, for the fused Bellman pass and for the
 * P_pi products: lanes per row (a power of two in 1..64: rows are split
 * over lane groups), -1 (flat chunk streaming, for MDPs whose rows all have
 * the same length) or 0 (automatic: flat when admissible); states per tile
 * (0 = automatic).  Flat Bellman passes: in the band form, 16-byte chunks (2
 * doubles or 4 floats) and A <= 64 run on wave tiles, other flat passes on
 * workgroup tiles; bellman_lanes = -3 asks for wave tiles whenever the chunk
 * and A allow them, -2 for workgroup tiles.  On wave tiles, states per tile
 * counts states per wavefront, at most min(64, 64 RPL / A) with RPL = 4 for
 * rows of at most 4 chunks outside the band form, else 1.  ipi_get_tuning
 * returns the stored values (0 = automatic). */
typedef struct ipi_tuning {
    int32_t bellman_lanes;
    int32_t bellman_states_per_tile;
    int32_t spmv_lanes;
    int32_t spmv_states_per_tile;
    int32_t bellman_chunk;   /* flat mode: values per thread chunk (0 = automatic; 2..32 dividing the row length) */
    int32_t spmv_chunk;      /* same for the P_pi products */
    int32_t spmv_schedule;   /* flat P_pi products: 0 automatic (= 2), 1 workgroup tiles, 2 wave tiles (then
                                spmv_states_per_tile counts states per wavefront, at most 64, with at most
                                1024 chunks per wave tile; a larger tile falls back to workgroup tiles) */
    int32_t spmv_workgroups; /* workgroups of the P_pi product launches (0 automatic; capped at the
                                workspace's partial-sum capacity, 32 per CU) */
    int32_t band_rows;       /* band form: when every row of P has k consecutive columns (detected at
                                create), the flat kernels read each row's first column instead of its
                                k column indices; stencil form (stencil_patterns above): the flat
                                Bellman pass on workgroup tiles reads one word per row.  0: use
                                either when detected; -1: never */
    int32_t ppi_cached;      /* P_pi products on wave tiles (flat rows; spmv_schedule 2) load P_pi through
                                the caches instead of streaming it past, so that a P_pi the last-level
                                cache can hold is read from it at the next sweep.  0: when one sweep's
                                bytes (values, columns or band starts, vectors) are at most 300 MiB, and
                                always in the blocked Richardson sweeps (whose workgroups re-read their
                                neighbours' halo rows); 1: always; -1: never.  The results are the same
                                either way */
    int32_t blocked_prefetch; /* blocked Richardson sweeps on rows too long for a second copy in
                                registers (FP64 rows of 24 or 32 entries): 0 persistent workgroups that
                                load the next block's rows into LDS during the current block's sweeps;
                                -1 one block per workgroup.  The results are the same either way */
} ipi_tuning;

ipi_status ipi_get_tuning(ipi_mdp_t mdp, ipi_tuning* out);
ipi_status ipi_set_tuning(ipi_mdp_t mdp, const ipi_tuning* t);

/* Time every admissible configuration on this MDP and keep the fastest
 * (the choice depends only on the MDP's shape).  If cache_path is not NULL
 * the result is stored in / read from that JSON file keyed by shape class
 * and GPU architecture.  Only the launch shapes (lanes, states per tile,
 * chunk widths, schedule) change; band_rows, spmv_workgroups,
 * ppi_cached and blocked_prefetch keep their values. */
ipi_status ipi_autotune(ipi_mdp_t mdp, int32_t precision, const char* cache_path, void* stream);

/* ------------------------------------------------------------------------ */
/* Helpers                                                                   */
/* ------------------------------------------------------------------------ */

/* Device bytes an MDP of this shape needs for data plus solve workspace. */
int64_t ipi_footprint_bytes(int64_t S, int32_t A, int64_t nnz, int32_t k_max,
                            const ipi_solve_opts* opts);

/*
 * ipi_stream_read — measurement helper: read `bytes` of device memory at
 * `buf` once with 16-byte non-temporal loads (the load the P arrays are
 * streamed with) and XOR them into the device word *xor_out (the caller
 * initialises it; its value only keeps the loads from being dropped).  The
 * time of this launch gives the achievable HBM read rate beside which the
 * Bellman pass's bandwidth is reported (Sec. III-B.3 approach 2 is such a
 * stream over P).  bytes: a positive multiple of 16; buf: 16-byte aligned.
 * Asynchronous on `stream`.  IPI_E_INVALID_ARG on bad arguments.
 */
ipi_status ipi_stream_read(const void* buf, int64_t bytes, uint32_t* xor_out, void* stream);

/* Thread-local message of the last failed call ("" if none). */
const char* ipi_last_error(void);

/* Library version string. */
const char* ipi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* IPI_H */

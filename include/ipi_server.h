/*
 * ipi_server.h — serving loop of libipi.so: MDP solve requests of mixed
 * sizes admitted by an HBM budget and solved concurrently on one GPU.
 *
 * Requests arrive through ipi_server_submit (any host thread).  A scheduler
 * admits the queue head, with bounded backfill from the next few requests,
 * once its device footprint (ipi_footprint_bytes) fits in the free budget
 * and a slot is free.  Large admitted requests run the single-MDP solver on
 * a pool of worker threads, each with its own HIP stream, so their work
 * overlaps on the device.  Small ones (nnz <= small_nnz_threshold, options
 * the batched solver takes) join the one running batched solve at its next
 * chunk boundary (continuous batching: 32 rounds, typically a few ms) and
 * leave it as soon as their own solve has ended.  Each request's result is
 * copied back, its done time stamped and its device memory, budget and slot
 * released on its own, whatever the others do.  fp32_mixed requests keep
 * only float32 values of P on the device (about 2/3 of the FP64 footprint);
 * their info.err_bound states the distance to the FP64 MDP's V*.  Each
 * result does not depend on which other requests were in flight.
 *
 * The solve itself is Algorithm 1 of arXiv 2507.22538 (see ipi.h).
 */
#ifndef IPI_SERVER_H
#define IPI_SERVER_H

#include "ipi.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ipi_server_s* ipi_server_t;

typedef struct ipi_server_opts {
    int64_t hbm_budget_bytes;   /* device bytes the server may hold for requests (> 0)        */
    int32_t max_slots;          /* requests admitted at once (>= 1)                          */
    int32_t n_streams;          /* worker threads / HIP streams (>= 1)                       */
    int64_t small_nnz_threshold;/* requests with nnz <= this may share a batched launch       */
    int32_t max_batch;          /* most requests per batched launch (>= 1)                   */
    int32_t backfill;           /* queued requests looked at behind a head that does not fit */
} ipi_server_opts;

/* Times in milliseconds on the host steady clock, relative to server creation. */
typedef struct ipi_latency {
    double arrival_ms;  /* submit returned                     */
    double admit_ms;    /* admitted (memory and slot granted)  */
    double start_ms;    /* its work was enqueued on a stream   */
    double done_ms;     /* result copied back                  */
    int32_t batched;    /* solved by the batched solver         */
    int32_t batch_size; /* its members when this one joined (1 if not batched) */
} ipi_latency;

void ipi_server_opts_default(ipi_server_opts* o);

/* Start the scheduler and workers on the current HIP device. */
ipi_status ipi_server_create(const ipi_server_opts* opts, ipi_server_t* out);

/*
 * Queue one solve.  The MDP arguments are those of ipi_mdp_create_csr with
 * HOST arrays; they are copied before the call returns (the caller may free
 * them).  Create flags: IPI_NO_VALIDATE and IPI_FP32_ORIGIN apply to the
 * validation done here, IPI_VAL_FP32 and IPI_VAL_FP32_ONLY to the request's
 * MDP; IPI_DEVICE_PTRS and IPI_BORROW are refused; IPI_VAL_SPLIT is ignored
 * (the request's MDP keeps FP64 values).
 * opts->v0 must be NULL.  Non-blocking.  Errors: IPI_E_INVALID_ARG,
 * IPI_E_NOT_STOCHASTIC (checked here, on the host), IPI_E_TOO_LARGE when the
 * footprint exceeds the whole budget.
 */
ipi_status ipi_server_submit(ipi_server_t srv, int64_t S, int32_t A, int64_t nnz, const int64_t* row_ptr,
                             const int32_t* col, const double* val, const double* g, double gamma,
                             uint32_t flags, const ipi_solve_opts* opts, uint64_t* ticket);

/* done = 1 once the request finished (solved, failed or cancelled). */
ipi_status ipi_server_poll(ipi_server_t srv, uint64_t ticket, int32_t* done);

/*
 * Block until the request finishes and collect it (the ticket is then
 * forgotten).  V (S doubles) and pi (S ints) are HOST arrays, either may be
 * NULL; info and lat may be NULL.  Returns the request's solve status
 * (IPI_OK, IPI_E_NOT_CONVERGED with outputs written, IPI_E_CANCELLED, ...),
 * or IPI_E_NOT_FOUND for an unknown ticket.
 */
ipi_status ipi_server_wait(ipi_server_t srv, uint64_t ticket, double* V, int32_t* pi, ipi_solve_info* info,
                           ipi_latency* lat);

/* Cancel a queued request (IPI_OK) or mark a running one so its result is
 * discarded; waiting on it returns IPI_E_CANCELLED. */
ipi_status ipi_server_cancel(ipi_server_t srv, uint64_t ticket);

/* Stop accepting work, finish what is admitted, cancel the queue, free all. */
ipi_status ipi_server_destroy(ipi_server_t srv);

#ifdef __cplusplus
}
#endif
#endif /* IPI_SERVER_H */

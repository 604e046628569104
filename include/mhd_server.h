/*
 * mhd_server.h - continuous-batching service of MHD solve requests on one GPU.
 *
 * A request is one initial-value problem (grid, gamma, boundary condition,
 * dtype, initial state as in mhd.h) and a number of full steps. Requests
 * queue on submission and are admitted first-come first-served while their
 * device footprint (mhd_batch_problem_bytes) fits the server's HBM budget
 * and their cells fit the cell cap (mhd_server_set_max_cells); an admitted
 * request's state stays resident on the device until it finishes. Each tick advances every admitted request by one full step: FP32
 * and FP64 requests run as two batches (include/mhd_batch.h) on two streams,
 * so their work overlaps, and requests admitted at different ticks share the
 * batched launches of their sweep order. Initial and final states move
 * between pinned host memory and the device on a third stream, overlapping
 * the steps; a request that reaches its step count leaves its batch at the
 * next tick and joins the completion queue once its final state is on the
 * host. Device blocks and pinned buffers are reused across requests.
 *
 * Each request is advanced by exactly the arithmetic of a plain solve
 * (mhd_step), so its result is bitwise the result of solving it alone.
 * Times are seconds on the server's monotonic clock (mhd_server_now). A
 * server is not thread-safe. Return codes and mhd_last_error() are those of
 * mhd.h.
 */
#ifndef MHD_SERVER_H
#define MHD_SERVER_H

#include "mhd.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mhd_server mhd_server_t;

enum { MHD_REQ_QUEUED = 0, MHD_REQ_RUNNING = 1, MHD_REQ_DONE = 2 };

/* Monotonic clock of the servers, in seconds. */
double mhd_server_now(void);

/* Create a server that keeps at most hbm_budget bytes of request state on the
 * current device and advances every request with Courant number cfl
 * (0 < cfl <= 1). */
int mhd_server_create(size_t hbm_budget, double cfl, mhd_server_t** out);

/* Admission cap on the total cells (nx * ny * nz) of the admitted requests:
 * the head of the queue waits while admitting it would exceed `cells`, unless
 * no request is running (so a larger one still runs, alone). 0 removes the
 * cap; negative values are MHD_ERR_ARG. Default 2^24 (one 256^3 grid), which
 * keeps the device busy: every admitted request shares each tick with all
 * the others, so a larger running set only lengthens each one's latency. */
int mhd_server_set_max_cells(mhd_server_t* s, int64_t cells);

/* Release the server, its batches and every request (null is accepted). */
int mhd_server_destroy(mhd_server_t* s);

/* Queue a request: grid nx x ny x nz, gamma, bc, dtype (MHD_F32 / MHD_F64),
 * initial state in host memory (copied at submission; the caller keeps its
 * buffer), nsteps >= 1 full steps. *req receives the request id. A request
 * whose footprint exceeds the whole budget is rejected with MHD_ERR_ARG. */
int mhd_server_submit(mhd_server_t* s, int nx, int ny, int nz, double gamma, int bc, int dtype,
                      const void* host_state, int nsteps, int* req);

/* As mhd_server_submit, but the initial state is read from the caller's
 * buffer in place rather than copied at submission: the buffer is lent until
 * the request leaves the queue (mhd_server_info reports a state other than
 * MHD_REQ_QUEUED) or mhd_server_destroy returns, whichever comes first, and
 * must stay valid and unchanged until then. This saves one host copy of the
 * state. */
int mhd_server_submit_ref(mhd_server_t* s, int nx, int ny, int nz, double gamma, int bc, int dtype,
                          const void* host_state, int nsteps, int* req);

/* One scheduling round: finish requests whose final state has reached the
 * host, send requests that have taken all their steps out of their batch
 * (their state follows asynchronously), admit queued requests in arrival
 * order while they fit the budget and the cell cap, then issue one full step
 * of every admitted request (asynchronous; the host stays at most three
 * rounds ahead of the device). A round with nothing to step waits for the
 * oldest pending
 * copy-out. *running (admitted, including those whose state is on its way
 * out) and *queued (optional) receive the counts after the round. */
int mhd_server_tick(mhd_server_t* s, int* running, int* queued);

/* Id of the oldest finished request not yet taken (-1 when none). */
int mhd_server_poll(mhd_server_t* s, int* req);

/* State of a request (MHD_REQ_*), its simulation time and steps taken, its
 * solver status (MHD_OK, MHD_ERR_NONFINITE, MHD_ERR_ARG for an initial state
 * with a non-finite value or a non-positive density, or MHD_ERR_OOM when it
 * could never be placed), and its submission, admission
 * and finish times (negative while not reached). Any pointer may be null. */
int mhd_server_info(mhd_server_t* s, int req, int* state, double* t_sim, int64_t* steps, int* status,
                    double* t_submit, double* t_admit, double* t_finish);

/* Copy a finished request's final state (layout of mhd.h) to host memory and
 * forget the request. */
int mhd_server_take(mhd_server_t* s, int req, void* host_state);

/* Device bytes held by admitted requests, and cell-updates issued so far. */
int mhd_server_stats(mhd_server_t* s, size_t* bytes_in_use, int64_t* cell_updates);

#ifdef __cplusplus
}
#endif

#endif /* MHD_SERVER_H */

/*
 * mhd_batch.h - batched solves: many independent MHD problems of different
 * grid sizes advanced together, one launch per sub-operation for all of them.
 *
 * Each problem is the same initial-value problem that an mhd_t handle solves
 * (state layout, boundary conditions, time step rule and sweep order as in
 * mhd.h: Wong et al., Sec. 3 and Sec. 4.2), with its own grid, gamma, boundary
 * condition, time, step counter, stop time and status. A batched full step
 * advances every problem by one full step of its own: its own c_max and
 * dt = cfl / c_max (a per-problem maximum, so problems never share a dt), then
 * the forward and reverse sweeps in the order its own step counter selects.
 * Each problem goes through exactly the arithmetic of a plain solve, so its
 * result is bitwise the result of mhd_step on a handle with the same input.
 *
 * Problems whose step counters agree modulo 3 run the same sweep order and
 * form one cohort; each cohort runs 13 launches per full step (the per-problem
 * dt rule and 12 sweeps), captured once in a HIP graph per sweep order and
 * replayed. In a cohort whose members are all periodic, each reverse
 * L_d with more than one cell along d in every member runs as one fused
 * launch (field update, then fluid update; Sec. 4.3), 10 launches per step,
 * with the same bits. The autotuner picks, per grid shape and sweep kind, the
 * chunk length along y/z sweeps and the form of x sweeps that run fastest
 * on the device; tiles never change results.
 *
 * Memory: each problem lives in one device block of
 * mhd_batch_problem_bytes(nx, ny, nz, dtype) bytes (two state copies, its
 * control block and reduction slots), allocated when it is added and
 * released when it is removed, or provided by the caller
 * (mhd_batch_add_inplace). The batch owns its own stream (default priority) unless
 * mhd_batch_set_stream gives another. Return codes and mhd_last_error() are
 * those of mhd.h. A batch is not thread-safe.
 */
#ifndef MHD_BATCH_H
#define MHD_BATCH_H

#include "mhd.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mhd_batch mhd_batch_t;

/* Create an empty batch whose problems all use arithmetic type dtype
 * (MHD_F32 or MHD_F64). */
int mhd_batch_create(int dtype, mhd_batch_t** out);

/* Release the batch, every problem in it and its device memory (null is
 * accepted). */
int mhd_batch_destroy(mhd_batch_t* b);

/* Run all later work of the batch on a caller-owned stream (hipStream_t as
 * void*). Graph replay needs a stream other than the null stream; on the null
 * stream the launches are issued one by one. */
int mhd_batch_set_stream(mhd_batch_t* b, void* stream);

/* Device bytes one problem of this size and dtype holds while it is in a
 * batch (0 for invalid arguments, including grids of more than 2^36 cells). */
size_t mhd_batch_problem_bytes(int nx, int ny, int nz, int dtype);

/* Add a problem: grid nx x ny x nz (each >= 1), gamma > 1, bc as in mhd.h,
 * initial state in host memory (copied synchronously) or device memory
 * (copied asynchronously on the batch's stream), layout as in mhd.h. The new
 * problem starts at t = 0, s = 0, no stop time; *id receives its handle
 * (ids are never reused within a batch). MHD_ERR_OOM when its allocation
 * fails, MHD_ERR_ARG when the state has a non-finite value or a non-positive
 * density (checked on the device); the batch is then unchanged. */
int mhd_batch_add(mhd_batch_t* b, int nx, int ny, int nz, double gamma, int bc, const void* host_state, int* id);
int mhd_batch_add_device(mhd_batch_t* b, int nx, int ny, int nz, double gamma, int bc, const void* dev_state,
                         int* id);

/* Byte offsets, within a problem's device block, of state copy 0 of the
 * conserved fields (5 fields of nx*ny*nz elements), of the face fields
 * (3 fields) and of the control block, and the block size (as
 * mhd_batch_problem_bytes). */
int mhd_batch_problem_layout(int nx, int ny, int nz, int dtype, size_t* off_u0, size_t* off_b0, size_t* off_ctl,
                             size_t* bytes);

/* Add a problem in a caller-owned device block of mhd_batch_problem_bytes
 * bytes whose copy-0 regions (mhd_batch_problem_layout) hold, or will hold,
 * the initial state: ready (a hipEvent_t, or null) marks the point after
 * which they do, and the batch's stream waits for it. Nothing is copied and
 * the host does not wait. The caller keeps the block: after
 * mhd_batch_remove it may reuse it once the batch's stream has passed the
 * removal (mhd_batch_record an event and wait for it). The state is checked
 * on the device without waiting: a rejected one latches MHD_ERR_ARG in the
 * problem's status and is never advanced. */
int mhd_batch_add_inplace(mhd_batch_t* b, int nx, int ny, int nz, double gamma, int bc, void* dev_block, void* ready,
                          int* id);

/* Record a HIP event (hipEvent_t as void*) on the batch's stream after all
 * work issued so far. */
int mhd_batch_record(mhd_batch_t* b, void* event);

/* Remove a problem. Memory the batch allocated is released (waiting for the
 * batch's stream); a caller-owned block is left to the caller, without
 * waiting. Between steps the problem's state is in its copy-0 regions. */
int mhd_batch_remove(mhd_batch_t* b, int id);

/* Number of problems and device bytes they hold. */
int mhd_batch_count(mhd_batch_t* b, int* n, size_t* bytes);

/* Advance every problem by n >= 0 full steps with Courant number
 * 0 < cfl <= 1. Returns after the launches are issued (asynchronous); a
 * problem whose c_max turns non-finite latches MHD_ERR_NONFINITE in its own
 * status (mhd_batch_status) and keeps its state from then on, without
 * affecting the others. */
int mhd_batch_step(mhd_batch_t* b, int n, double cfl);

/* Copy one problem's current state out (host: synchronises the stream;
 * device: asynchronous on the batch's stream). */
int mhd_batch_get_state(mhd_batch_t* b, int id, void* host_state);
int mhd_batch_get_state_device(mhd_batch_t* b, int id, void* dev_state);

/* Simulation time and full-step counter of one problem (synchronises). */
int mhd_batch_get_time(mhd_batch_t* b, int id, double* t, int64_t* s);

/* Stop time of one problem, as mhd_set_stop_time (negative: none). */
int mhd_batch_set_stop_time(mhd_batch_t* b, int id, double t_stop);

/* Status of one problem: MHD_OK, MHD_ERR_NONFINITE once its c_max was NaN,
 * infinite or not positive, or MHD_ERR_ARG for a rejected initial state
 * (synchronises). */
int mhd_batch_status(mhd_batch_t* b, int id);

/* Capture each cohort's full step in a HIP graph and replay it (enable = 1,
 * the default) or issue every launch directly (enable = 0). */
int mhd_batch_set_graphs(mhd_batch_t* b, int enable);

/* Time every candidate tile of every sweep kind on the problems currently in
 * the batch, reps launches each, per grid shape, and keep the fastest for all
 * later steps of problems of that shape. Writes only the scratch state copy,
 * so it may be called between any two steps. */
int mhd_batch_autotune(mhd_batch_t* b, int reps);

/* Tile parameters in use for one problem and kind (MHD_K_* of mhd.h, the
 * fused reverse kinds MHD_K_CTFLUID_* included): p0 = chunk length (y/z
 * sweeps) or workgroup count (c_max pass), p1 = 0; for the x sweeps p0 = 0,
 * p1 = 0 (64-lane wavefronts over row segments) or the lane-row form, p0 = K
 * cells per lane and p1 = W lanes per row, on FP32 periodic rows of W K
 * cells: (K, W) = (1, 64), (2, 64) for rows of 64 and 128 cells, each held by
 * one wavefront; (1, 32), (3, 32) for rows of 32 and 96 cells, two to a
 * wavefront; (3, 16) for rows of 48 cells, four to a wavefront. */
int mhd_batch_tile(mhd_batch_t* b, int id, int kind, int* p0, int* p1);

/* Pin the tile of one sweep kind for every problem of this one's grid shape
 * and boundary condition (as the autotuner would, without timing); (p0, p1)
 * must be one of the autotuner's candidates for that grid and kind (an x
 * sweep: (0, 0) or, where it applies, the lane-row (K, W)), else
 * MHD_ERR_ARG. Tiles never change results. Synchronises the batch's
 * stream. */
int mhd_batch_set_tile(mhd_batch_t* b, int id, int kind, int p0, int p1);

#ifdef __cplusplus
}
#endif

#endif /* MHD_BATCH_H */

// Continuous-batching request service (declared in include/mhd_server.h),
// built on the batch runtime: one batch per dtype, each on its own stream,
// plus a copy stream. Host-only code; the device work is the batch runtime's.
//
// The device never waits for the host: a request's initial state goes from
// pinned host memory to its device block on the copy stream and the batch's
// stream waits for that copy (an event) before its first step; a finished
// request leaves the batch at once and its final state (and control block)
// goes back to pinned memory on the copy stream after the batch's stream has
// passed its last step. Device blocks and pinned buffers are pooled by size.
// The host issues at most kAhead ticks beyond the ones the device finished.
// A staging thread copies queued inputs into pinned buffers ahead of their
// admission (up to kStageLimit bytes), so a tick only issues the transfer.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/mhd_batch.h"
#include "../../include/mhd_server.h"
#include "mhd_internal.h"

namespace {

constexpr int kAhead = 3;
constexpr size_t kStageLimit = (size_t)2 << 30;   // pinned bytes staged ahead of admission
constexpr int kDraining = 3;   // phase between leaving the batch and the copy-out completing
// Admission cap on the cells of the running requests: one 256^3 grid keeps
// the device busy; admitting more only makes every running request share the
// device with more others, which lengthens each one's latency.
constexpr long long kDefaultMaxCells = 1LL << 24;

struct Req {
    int nx, ny, nz, bc, dtype, nsteps;
    double gamma;
    size_t bytes = 0;            // device block
    size_t sbytes = 0;           // state: 8 fields
    std::vector<char> input;     // pageable copy of the initial state until admission
    const void* ext = nullptr;   // or the caller's buffer, lent until the request leaves the queue
    void* host = nullptr;        // pinned: staged input, then final state + control block
    bool staged = false;         // host holds the input
    bool counted = false;        // host counts in staged_bytes (staged, not yet admitted)
    int stage_rc = MHD_OK;
    void* block = nullptr;       // device block while admitted or draining
    hipEvent_t copied = nullptr; // copy-in, then copy-out, done
    hipEvent_t passed = nullptr; // the batch's stream passed the last step
    int pid = -1;
    int issued = 0;
    int phase = MHD_REQ_QUEUED;
    int status = MHD_OK;
    double t_sim = 0.0;
    double t_submit = -1.0, t_admit = -1.0, t_finish = -1.0;
};

int fail(int code, const char* msg) { return mhd::report(code, msg); }
int hip_fail(hipError_t e, const char* where) { return mhd::report_hip(e, where); }

#define HIPCHK(call, where)                               \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return hip_fail(e_, where); \
    } while (0)

}  // namespace

struct mhd_server {
    size_t budget;
    size_t used;                 // device blocks of running and draining requests
    long long max_cells;         // admission cap on the cells of running requests (0: none)
    double cfl;
    int device;
    mhd_batch_t* batch[2];       // indexed by dtype
    hipStream_t copy;
    std::map<int, Req> reqs;
    std::deque<int> queue;
    std::vector<int> running;
    std::vector<int> draining;
    std::deque<int> done;
    int next_id;
    long long cell_updates;
    std::multimap<size_t, void*> free_blocks;   // device blocks by size
    std::multimap<size_t, void*> free_pinned;   // pinned host buffers by size
    std::vector<hipEvent_t> free_events;
    hipEvent_t pace[kAhead + 1][2];             // per tick and batch: its step is done
    bool pace_set[kAhead + 1][2];
    long long ticks;
    // staging thread; mu guards reqs' insertion and removal, stage_queue,
    // free_pinned, staged_bytes, stop and the staged fields
    std::mutex mu;
    std::condition_variable work_cv, staged_cv;
    std::deque<int> stage_queue;
    size_t staged_bytes;
    bool stop;
    std::thread stager;
};

namespace {

int take_event(mhd_server* s, hipEvent_t* out)
{
    if (!s->free_events.empty()) {
        *out = s->free_events.back();
        s->free_events.pop_back();
        return MHD_OK;
    }
    HIPCHK(hipEventCreateWithFlags(out, hipEventDisableTiming), "hipEventCreate");
    return MHD_OK;
}

void give_event(mhd_server* s, hipEvent_t& e)
{
    if (e) s->free_events.push_back(e);
    e = nullptr;
}

// Device block of exactly `bytes` from the pool or a new allocation;
// MHD_ERR_OOM when the device has no room even after the pool is released.
int take_block(mhd_server* s, size_t bytes, void** out)
{
    auto it = s->free_blocks.find(bytes);
    if (it != s->free_blocks.end()) {
        *out = it->second;
        s->free_blocks.erase(it);
        return MHD_OK;
    }
    hipError_t e = hipMalloc(out, bytes);
    if (e == hipErrorOutOfMemory && !s->free_blocks.empty()) {
        (void)hipGetLastError();
        for (auto& kv : s->free_blocks) (void)hipFree(kv.second);   // unused: their copy-outs completed
        s->free_blocks.clear();
        e = hipMalloc(out, bytes);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *out = nullptr;
        return e == hipErrorOutOfMemory ? fail(MHD_ERR_OOM, "device allocation failed") : hip_fail(e, "hipMalloc");
    }
    return MHD_OK;
}

size_t host_bytes(const Req& r) { return r.sbytes + sizeof(mhd::Ctl); }

// Staging thread: copies queued inputs into pinned buffers, in queue order,
// while less than kStageLimit bytes wait staged for admission.
void stage_loop(mhd_server* s)
{
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        s->work_cv.wait(lk, [s] {
            return s->stop || (!s->stage_queue.empty() && s->staged_bytes < kStageLimit);
        });
        if (s->stop) return;
        const int id = s->stage_queue.front();
        s->stage_queue.pop_front();
        auto it = s->reqs.find(id);
        if (it == s->reqs.end()) continue;
        Req& r = it->second;   // queued: only this thread touches its input and host fields until staged
        const size_t hb = host_bytes(r);
        void* buf = nullptr;
        auto pit = s->free_pinned.find(hb);
        if (pit != s->free_pinned.end()) {
            buf = pit->second;
            s->free_pinned.erase(pit);
        }
        lk.unlock();
        int rc = MHD_OK;
        if (!buf && hipHostMalloc(&buf, hb, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            buf = nullptr;
            rc = MHD_ERR_OOM;
        }
        if (buf) {
            std::memcpy(buf, r.ext ? r.ext : static_cast<const void*>(r.input.data()), r.sbytes);
            std::vector<char>().swap(r.input);
            r.ext = nullptr;
        }
        lk.lock();
        r.host = buf;
        r.stage_rc = rc;
        r.staged = true;
        if (buf) {
            s->staged_bytes += hb;
            r.counted = true;
        }
        s->staged_cv.notify_all();
    }
}

// Copy-in of a queued request and its entry into its batch.
int admit(mhd_server* s, int id, bool* room)
{
    Req& r = s->reqs.at(id);
    *room = true;
    void* block = nullptr;
    int rc = take_block(s, r.bytes, &block);
    if (rc == MHD_ERR_OOM && (!s->running.empty() || !s->draining.empty())) {
        *room = false;   // wait for memory to free
        return MHD_OK;
    }
    if (rc != MHD_OK) return rc;
    size_t off_u0 = 0, off_b0 = 0;
    rc = mhd_batch_problem_layout(r.nx, r.ny, r.nz, r.dtype, &off_u0, &off_b0, nullptr, nullptr);
    if (rc != MHD_OK) {
        s->free_blocks.emplace(r.bytes, block);
        return rc;
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (r.counted) s->staged_bytes -= host_bytes(r);
        r.counted = false;
    }
    s->work_cv.notify_one();
    const size_t ub = r.sbytes / 8 * 5;
    char* dev = static_cast<char*>(block);
    HIPCHK(hipMemcpyAsync(dev + off_u0, r.host, ub, hipMemcpyHostToDevice, s->copy), "state copy in");
    HIPCHK(hipMemcpyAsync(dev + off_b0, static_cast<char*>(r.host) + ub, r.sbytes - ub, hipMemcpyHostToDevice,
                          s->copy),
           "state copy in");
    if ((rc = take_event(s, &r.copied))) return rc;
    HIPCHK(hipEventRecord(r.copied, s->copy), "hipEventRecord");
    if ((rc = mhd_batch_add_inplace(s->batch[r.dtype], r.nx, r.ny, r.nz, r.gamma, r.bc, block, r.copied, &r.pid)))
        return rc;
    r.block = block;
    r.phase = MHD_REQ_RUNNING;
    r.t_admit = mhd_server_now();
    s->used += r.bytes;
    s->running.push_back(id);
    return MHD_OK;
}

// A request that took all its steps leaves its batch; its state follows on
// the copy stream once the batch's stream has passed the last step.
int retire(mhd_server* s, int id)
{
    Req& r = s->reqs.at(id);
    mhd_batch_t* b = s->batch[r.dtype];
    int rc;
    if ((rc = mhd_batch_remove(b, r.pid))) return rc;
    r.pid = -1;
    if ((rc = take_event(s, &r.passed))) return rc;
    if ((rc = mhd_batch_record(b, r.passed))) return rc;
    HIPCHK(hipStreamWaitEvent(s->copy, r.passed, 0), "hipStreamWaitEvent");
    size_t off_u0 = 0, off_b0 = 0, off_ctl = 0;
    if ((rc = mhd_batch_problem_layout(r.nx, r.ny, r.nz, r.dtype, &off_u0, &off_b0, &off_ctl, nullptr))) return rc;
    const size_t ub = r.sbytes / 8 * 5;
    const char* dev = static_cast<const char*>(r.block);
    char* h = static_cast<char*>(r.host);
    HIPCHK(hipMemcpyAsync(h, dev + off_u0, ub, hipMemcpyDeviceToHost, s->copy), "state copy out");
    HIPCHK(hipMemcpyAsync(h + ub, dev + off_b0, r.sbytes - ub, hipMemcpyDeviceToHost, s->copy), "state copy out");
    HIPCHK(hipMemcpyAsync(h + r.sbytes, dev + off_ctl, sizeof(mhd::Ctl), hipMemcpyDeviceToHost, s->copy),
           "control block copy out");
    HIPCHK(hipEventRecord(r.copied, s->copy), "hipEventRecord");
    r.phase = kDraining;
    s->draining.push_back(id);
    return MHD_OK;
}

// Copy-out finished: the result is on the host and the block is free.
void finish(mhd_server* s, int id)
{
    Req& r = s->reqs.at(id);
    mhd::Ctl c;
    std::memcpy(&c, static_cast<const char*>(r.host) + r.sbytes, sizeof(c));
    r.t_sim = c.t;
    r.status = c.status == -1 ? MHD_ERR_ARG : (c.status != 0 ? MHD_ERR_NONFINITE : MHD_OK);
    s->free_blocks.emplace(r.bytes, r.block);
    r.block = nullptr;
    s->used -= r.bytes;
    give_event(s, r.copied);
    give_event(s, r.passed);
    r.phase = MHD_REQ_DONE;
    r.t_finish = mhd_server_now();
    s->done.push_back(id);
}

int poll_draining(mhd_server* s)
{
    std::vector<int> still;
    for (int id : s->draining) {
        hipError_t q = hipEventQuery(s->reqs.at(id).copied);
        if (q == hipSuccess)
            finish(s, id);
        else if (q == hipErrorNotReady)
            still.push_back(id);
        else
            return hip_fail(q, "hipEventQuery");
    }
    s->draining.swap(still);
    return MHD_OK;
}

void fail_request(mhd_server* s, int id, int status)
{
    Req& r = s->reqs.at(id);
    if (r.ext) {
        // the caller's buffer is still lent (the request was queued): keep a
        // copy of the input, which mhd_server_take returns for a request never run
        try {
            const char* p = static_cast<const char*>(r.ext);
            r.input.assign(p, p + r.sbytes);
        } catch (...) {
        }
        r.ext = nullptr;
    }
    r.status = status;
    r.phase = MHD_REQ_DONE;
    r.t_finish = mhd_server_now();
    s->done.push_back(id);
}

// Queue a request (checks as mhd_server_submit); with `lend` the caller's
// buffer is read in place by the staging thread instead of copied here.
int submit(mhd_server* s, int nx, int ny, int nz, double gamma, int bc, int dtype, const void* host_state,
           int nsteps, bool lend, int* req)
{
    if (!s) return fail(MHD_ERR_ARG, "null server");
    if (!req || !host_state) return fail(MHD_ERR_ARG, "null pointer");
    if (dtype != MHD_F32 && dtype != MHD_F64) return fail(MHD_ERR_ARG, "unknown dtype");
    if (nsteps < 1) return fail(MHD_ERR_ARG, "nsteps must be >= 1");
    if (!(gamma > 1.0) || (bc != MHD_BC_PERIODIC && bc != MHD_BC_OUTFLOW))
        return fail(MHD_ERR_ARG, "invalid gamma or boundary condition");
    const size_t bytes = mhd_batch_problem_bytes(nx, ny, nz, dtype);
    if (bytes == 0) return fail(MHD_ERR_ARG, "invalid grid");
    if (bytes > s->budget) return fail(MHD_ERR_ARG, "request larger than the server's HBM budget");
    Req r;
    r.nx = nx;
    r.ny = ny;
    r.nz = nz;
    r.bc = bc;
    r.dtype = dtype;
    r.nsteps = nsteps;
    r.gamma = gamma;
    r.bytes = bytes;
    r.sbytes = 8 * (size_t)nx * ny * nz * (dtype == MHD_F64 ? 8 : 4);
    if (lend) {
        r.ext = host_state;
    } else {
        try {
            r.input.resize(r.sbytes);
        } catch (...) {
            return fail(MHD_ERR_OOM, "host allocation failed");
        }
        std::memcpy(r.input.data(), host_state, r.sbytes);
    }
    r.t_submit = mhd_server_now();
    const int id = s->next_id++;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->reqs.emplace(id, std::move(r));
        s->stage_queue.push_back(id);
    }
    s->work_cv.notify_one();
    s->queue.push_back(id);
    *req = id;
    return MHD_OK;
}

}  // namespace

extern "C" {

double mhd_server_now(void)
{
    using clk = std::chrono::steady_clock;
    return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

int mhd_server_create(size_t hbm_budget, double cfl, mhd_server_t** out)
{
    if (!out) return fail(MHD_ERR_ARG, "null output pointer");
    *out = nullptr;
    if (hbm_budget == 0) return fail(MHD_ERR_ARG, "budget must be > 0");
    if (!(cfl > 0.0 && cfl <= 1.0)) return fail(MHD_ERR_ARG, "cfl must be in (0, 1]");
    mhd_server* s = new (std::nothrow) mhd_server();
    if (!s) return fail(MHD_ERR_OOM, "host allocation failed");
    s->budget = hbm_budget;
    s->used = 0;
    s->max_cells = kDefaultMaxCells;
    s->cfl = cfl;
    s->next_id = 1;
    s->cell_updates = 0;
    s->ticks = 0;
    s->staged_bytes = 0;
    s->stop = false;
    s->batch[0] = s->batch[1] = nullptr;
    s->copy = nullptr;
    for (int k = 0; k <= kAhead; k++)
        for (int d = 0; d < 2; d++) {
            s->pace[k][d] = nullptr;
            s->pace_set[k][d] = false;
        }
    int rc = MHD_OK;
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking);
    for (int k = 0; k <= kAhead && e == hipSuccess; k++)
        for (int d = 0; d < 2 && e == hipSuccess; d++) e = hipEventCreateWithFlags(&s->pace[k][d], hipEventDisableTiming);
    if (e != hipSuccess) rc = hip_fail(e, "server stream or events");
    if (rc == MHD_OK) rc = mhd_batch_create(MHD_F32, &s->batch[0]);
    if (rc == MHD_OK) rc = mhd_batch_create(MHD_F64, &s->batch[1]);
    if (rc == MHD_OK) {
        try {
            s->stager = std::thread(stage_loop, s);
        } catch (...) {
            rc = fail(MHD_ERR_OOM, "staging thread");
        }
    }
    if (rc != MHD_OK) {
        mhd_server_destroy(s);
        return rc;
    }
    *out = s;
    return MHD_OK;
}

int mhd_server_destroy(mhd_server_t* s)
{
    if (!s) return MHD_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->work_cv.notify_all();
    if (s->stager.joinable()) s->stager.join();
    mhd_batch_destroy(s->batch[0]);
    mhd_batch_destroy(s->batch[1]);
    if (s->copy) (void)hipStreamSynchronize(s->copy);
    for (auto& kv : s->reqs) {
        Req& r = kv.second;
        if (r.block) (void)hipFree(r.block);
        if (r.host) (void)hipHostFree(r.host);
        if (r.copied) (void)hipEventDestroy(r.copied);
        if (r.passed) (void)hipEventDestroy(r.passed);
    }
    for (auto& kv : s->free_blocks) (void)hipFree(kv.second);
    for (auto& kv : s->free_pinned) (void)hipHostFree(kv.second);
    for (hipEvent_t e : s->free_events) (void)hipEventDestroy(e);
    for (int k = 0; k <= kAhead; k++)
        for (int d = 0; d < 2; d++)
            if (s->pace[k][d]) (void)hipEventDestroy(s->pace[k][d]);
    if (s->copy) (void)hipStreamDestroy(s->copy);
    delete s;
    return MHD_OK;
}

int mhd_server_set_max_cells(mhd_server_t* s, int64_t cells)
{
    if (!s) return fail(MHD_ERR_ARG, "null server");
    if (cells < 0) return fail(MHD_ERR_ARG, "cell cap must be >= 0");
    s->max_cells = (long long)cells;
    return MHD_OK;
}

int mhd_server_submit(mhd_server_t* s, int nx, int ny, int nz, double gamma, int bc, int dtype,
                      const void* host_state, int nsteps, int* req)
{
    return submit(s, nx, ny, nz, gamma, bc, dtype, host_state, nsteps, false, req);
}

int mhd_server_submit_ref(mhd_server_t* s, int nx, int ny, int nz, double gamma, int bc, int dtype,
                          const void* host_state, int nsteps, int* req)
{
    return submit(s, nx, ny, nz, gamma, bc, dtype, host_state, nsteps, true, req);
}

int mhd_server_tick(mhd_server_t* s, int* running, int* queued)
{
    if (!s) return fail(MHD_ERR_ARG, "null server");
    int dev = -1;
    HIPCHK(hipGetDevice(&dev), "hipGetDevice");
    if (dev != s->device) HIPCHK(hipSetDevice(s->device), "hipSetDevice");
    // 0. stay at most kAhead ticks ahead of the device
    const int slot = (int)(s->ticks % (kAhead + 1));
    for (int d = 0; d < 2; d++)
        if (s->pace_set[slot][d]) {
            HIPCHK(hipEventSynchronize(s->pace[slot][d]), "tick pacing");
            s->pace_set[slot][d] = false;
        }
    // 1. copy-outs that completed
    if (int rc = poll_draining(s)) return rc;
    // 2. requests that took all their steps leave their batch
    std::vector<int> keep;
    for (int id : s->running) {
        if (s->reqs.at(id).issued >= s->reqs.at(id).nsteps) {
            if (int rc = retire(s, id)) return rc;
        } else {
            keep.push_back(id);
        }
    }
    s->running.swap(keep);
    // 3. admit in arrival order while the head of the queue fits the budget
    //    and the cell cap (a request is always admitted when none runs)
    long long cells = 0;
    for (int id : s->running) {
        const Req& r = s->reqs.at(id);
        cells += (long long)r.nx * r.ny * r.nz;
    }
    while (!s->queue.empty()) {
        const int id = s->queue.front();
        Req& head = s->reqs.at(id);
        if (s->used + head.bytes > s->budget) break;
        const long long head_cells = (long long)head.nx * head.ny * head.nz;
        if (s->max_cells > 0 && !s->running.empty() && cells + head_cells > s->max_cells) break;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            if (!head.staged) {
                if (!s->running.empty() || !s->draining.empty()) break;   // keep stepping; admit next round
                s->staged_cv.wait(lk, [&head] { return head.staged; });
            }
        }
        if (head.stage_rc != MHD_OK) {
            s->queue.pop_front();
            fail_request(s, id, head.stage_rc);
            continue;
        }
        bool room = true;
        const int rc = admit(s, id, &room);
        if (rc == MHD_OK && !room) break;
        s->queue.pop_front();
        if (rc != MHD_OK)
            fail_request(s, id, rc);
        else
            cells += head_cells;
    }
    // 4. one full step of every admitted request; the two batches run on
    //    their own streams and overlap
    bool any[2] = {false, false};
    for (int id : s->running) any[s->reqs.at(id).dtype] = true;
    for (int d = 0; d < 2; d++)
        if (any[d]) {
            if (int rc = mhd_batch_step(s->batch[d], 1, s->cfl)) return rc;
            if (int rc = mhd_batch_record(s->batch[d], s->pace[slot][d])) return rc;
            s->pace_set[slot][d] = true;
        }
    for (int id : s->running) {
        Req& r = s->reqs.at(id);
        r.issued += 1;
        s->cell_updates += (long long)r.nx * r.ny * r.nz;
    }
    // 5. nothing to step: wait for the oldest copy-out instead of returning at once
    if (s->running.empty() && !s->draining.empty()) {
        HIPCHK(hipEventSynchronize(s->reqs.at(s->draining.front()).copied), "copy-out wait");
        if (int rc = poll_draining(s)) return rc;
    }
    s->ticks += 1;
    if (running) *running = (int)(s->running.size() + s->draining.size());
    if (queued) *queued = (int)s->queue.size();
    return MHD_OK;
}

int mhd_server_poll(mhd_server_t* s, int* req)
{
    if (!s || !req) return fail(MHD_ERR_ARG, "null pointer");
    *req = -1;
    if (!s->done.empty()) {
        *req = s->done.front();
        s->done.pop_front();
    }
    return MHD_OK;
}

int mhd_server_info(mhd_server_t* s, int req, int* state, double* t_sim, int64_t* steps, int* status,
                    double* t_submit, double* t_admit, double* t_finish)
{
    if (!s) return fail(MHD_ERR_ARG, "null server");
    auto it = s->reqs.find(req);
    if (it == s->reqs.end()) return fail(MHD_ERR_ARG, "unknown request id");
    const Req& r = it->second;
    if (state) *state = r.phase == kDraining ? MHD_REQ_RUNNING : r.phase;
    if (t_sim) *t_sim = r.t_sim;
    if (steps) *steps = r.issued;
    if (status) *status = r.status;
    if (t_submit) *t_submit = r.t_submit;
    if (t_admit) *t_admit = r.t_admit;
    if (t_finish) *t_finish = r.t_finish;
    return MHD_OK;
}

int mhd_server_take(mhd_server_t* s, int req, void* host_state)
{
    if (!s || !host_state) return fail(MHD_ERR_ARG, "null pointer");
    auto it = s->reqs.find(req);
    if (it == s->reqs.end()) return fail(MHD_ERR_ARG, "unknown request id");
    Req& r = it->second;
    if (r.phase != MHD_REQ_DONE) return fail(MHD_ERR_ARG, "request not finished");
    if (r.host)
        std::memcpy(host_state, r.host, r.sbytes);   // the final state, or the input of a request never run
    else if (!r.input.empty())
        std::memcpy(host_state, r.input.data(), r.sbytes);
    std::lock_guard<std::mutex> lk(s->mu);
    if (r.host) {
        if (r.counted) s->staged_bytes -= host_bytes(r);
        s->free_pinned.emplace(host_bytes(r), r.host);
    }
    s->reqs.erase(it);
    return MHD_OK;
}

int mhd_server_stats(mhd_server_t* s, size_t* bytes_in_use, int64_t* cell_updates)
{
    if (!s) return fail(MHD_ERR_ARG, "null server");
    if (bytes_in_use) *bytes_in_use = s->used;
    if (cell_updates) *cell_updates = s->cell_updates;
    return MHD_OK;
}

}  // extern "C"

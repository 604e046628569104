// Continuous-batching request service (declared in include/mhd_server.h),
// built on the batch runtime: one batch per dtype, each on its own stream.
// Host-only code; the device work is the batch runtime's.
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "../../include/mhd_batch.h"
#include "../../include/mhd_server.h"
#include "mhd_internal.h"

namespace {

struct Req {
    int nx, ny, nz, bc, dtype, nsteps;
    double gamma;
    size_t bytes;                // device footprint while admitted
    std::vector<char> state;     // input until admitted, then the final state
    int pid = -1;                // problem id in its batch while running
    int issued = 0;              // full steps issued
    int phase = MHD_REQ_QUEUED;
    int status = MHD_OK;
    double t_sim = 0.0;
    long long steps = 0;
    double t_submit = -1.0, t_admit = -1.0, t_finish = -1.0;
};

int fail(int code, const char* msg) { return mhd::report(code, msg); }

}  // namespace

struct mhd_server {
    size_t budget;
    size_t used;
    double cfl;
    mhd_batch_t* batch[2];   // indexed by dtype
    std::map<int, Req> reqs;
    std::deque<int> queue;
    std::vector<int> running;
    std::deque<int> done;
    int next_id;
    long long cell_updates;
};

namespace {

// Copy a finished request's state out, release its device memory.
int retire(mhd_server* s, int id)
{
    Req& r = s->reqs.at(id);
    mhd_batch_t* b = s->batch[r.dtype];
    if (int rc = mhd_batch_get_state(b, r.pid, r.state.data())) return rc;
    double t = 0.0;
    int64_t st = 0;
    if (int rc = mhd_batch_get_time(b, r.pid, &t, &st)) return rc;
    const int status = mhd_batch_status(b, r.pid);
    if (status != MHD_OK && status != MHD_ERR_NONFINITE) return status;
    if (int rc = mhd_batch_remove(b, r.pid)) return rc;
    s->used -= r.bytes;
    r.pid = -1;
    r.t_sim = t;
    r.steps = st;
    r.status = status;
    r.phase = MHD_REQ_DONE;
    r.t_finish = mhd_server_now();
    s->done.push_back(id);
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
    s->cfl = cfl;
    s->next_id = 1;
    s->cell_updates = 0;
    s->batch[0] = s->batch[1] = nullptr;
    int rc = mhd_batch_create(MHD_F32, &s->batch[0]);
    if (rc == MHD_OK) rc = mhd_batch_create(MHD_F64, &s->batch[1]);
    if (rc != MHD_OK) {
        mhd_batch_destroy(s->batch[0]);
        delete s;
        return rc;
    }
    *out = s;
    return MHD_OK;
}

int mhd_server_destroy(mhd_server_t* s)
{
    if (!s) return MHD_OK;
    mhd_batch_destroy(s->batch[0]);
    mhd_batch_destroy(s->batch[1]);
    delete s;
    return MHD_OK;
}

int mhd_server_submit(mhd_server_t* s, int nx, int ny, int nz, double gamma, int bc, int dtype,
                      const void* host_state, int nsteps, int* req)
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
    const size_t sbytes = 8 * (size_t)nx * ny * nz * (dtype == MHD_F64 ? 8 : 4);
    Req r;
    r.nx = nx;
    r.ny = ny;
    r.nz = nz;
    r.bc = bc;
    r.dtype = dtype;
    r.nsteps = nsteps;
    r.gamma = gamma;
    r.bytes = bytes;
    try {
        r.state.resize(sbytes);
    } catch (...) {
        return fail(MHD_ERR_OOM, "host allocation failed");
    }
    std::memcpy(r.state.data(), host_state, sbytes);
    r.t_submit = mhd_server_now();
    const int id = s->next_id++;
    s->reqs.emplace(id, std::move(r));
    s->queue.push_back(id);
    *req = id;
    return MHD_OK;
}

int mhd_server_tick(mhd_server_t* s, int* running, int* queued)
{
    if (!s) return fail(MHD_ERR_ARG, "null server");
    // 1. retire requests whose last step was issued (their state is final
    //    once the batch's stream reaches it; the copy-out waits for that)
    std::vector<int> keep;
    for (int id : s->running) {
        Req& r = s->reqs.at(id);
        if (r.issued >= r.nsteps) {
            if (int rc = retire(s, id)) return rc;
        } else {
            keep.push_back(id);
        }
    }
    s->running.swap(keep);
    // 2. admit in arrival order while the head of the queue fits
    while (!s->queue.empty()) {
        const int id = s->queue.front();
        Req& r = s->reqs.at(id);
        if (s->used + r.bytes > s->budget) break;
        int pid = -1;
        const int rc = mhd_batch_add(s->batch[r.dtype], r.nx, r.ny, r.nz, r.gamma, r.bc, r.state.data(), &pid);
        if (rc == MHD_ERR_OOM && !s->running.empty()) break;   // wait for memory to free
        s->queue.pop_front();
        if (rc != MHD_OK) {
            r.status = rc;
            r.phase = MHD_REQ_DONE;
            r.t_finish = mhd_server_now();
            s->done.push_back(id);
            continue;
        }
        r.pid = pid;
        r.phase = MHD_REQ_RUNNING;
        r.t_admit = mhd_server_now();
        s->used += r.bytes;
        s->running.push_back(id);
    }
    // 3. one full step of every admitted request; the two batches run on
    //    their own streams and overlap
    bool any[2] = {false, false};
    for (int id : s->running) any[s->reqs.at(id).dtype] = true;
    for (int d = 0; d < 2; d++)
        if (any[d])
            if (int rc = mhd_batch_step(s->batch[d], 1, s->cfl)) return rc;
    for (int id : s->running) {
        Req& r = s->reqs.at(id);
        r.issued += 1;
        s->cell_updates += (long long)r.nx * r.ny * r.nz;
    }
    if (running) *running = (int)s->running.size();
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
    if (state) *state = r.phase;
    if (t_sim) *t_sim = r.t_sim;
    if (steps) *steps = r.phase == MHD_REQ_DONE ? r.steps : r.issued;
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
    if (it->second.phase != MHD_REQ_DONE) return fail(MHD_ERR_ARG, "request not finished");
    std::memcpy(host_state, it->second.state.data(), it->second.state.size());
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

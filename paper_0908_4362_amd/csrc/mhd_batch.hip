// Host runtime of batched solves (declared in include/mhd_batch.h).
//
// A batch holds problems of one dtype. Problems whose step counters agree
// modulo 3 share a sweep order and form a cohort; a cohort keeps in device
// memory one job table (buffers, grid, gamma, control block and reduction
// slots of each member) and, per launch kind, the workgroup range and tile
// parameters of each member. One full step of a cohort is the per-problem dt
// rule followed by the 12 batched sweeps; after its first step it is captured
// in a HIP graph per sweep order and replayed. Every step returns both state
// copies to copy 0, so between steps copy 0 is the state and copy 1 scratch.
//
// Nothing on the stepping path waits for the device: job tables are uploaded
// from a ring of pinned staging buffers, control blocks are initialised by a
// kernel, and graphs or table buffers that queued work may still use are
// released only once the stream has drained past them. Problems added in
// place (caller-owned memory) are added and removed without any wait.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <utility>
#include <vector>

#include "../../include/mhd_batch.h"
#include "mhd_internal.h"

using mhd::BJob;
using mhd::Ctl;
using mhd::Grid;
using mhd::TileDesc;

namespace {

constexpr int kPerm[3][3] = {{0, 1, 2}, {2, 0, 1}, {1, 2, 0}};  // sweep order by s mod 3 (eq. L_sequence)
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Prob {
    Grid g;
    double gamma;
    bool owned;      // mem allocated (and freed) by the batch
    void* mem;       // one block: u[0], u[1], b[0], b[1], control block, reduction slots
    size_t bytes;
    void* u[2];
    void* b[2];
    Ctl* ctl;
    unsigned long long* parts;
    long long s;     // full steps taken
};

struct Cohort {
    std::vector<int> ids;
    int phase = 0;               // s mod 3 of every member
    bool dirty = true;           // membership or tiles changed since the tables were built
    bool cmax_valid = false;     // members' parts hold c_max of their current state
    int parts_kind = 0;          // launch kind whose tables describe those parts
    bool fuse[3] = {false, false, false};   // reverse L_d as one fused launch, per axis
    void* dev = nullptr;         // job table + tile tables
    size_t dev_bytes = 0;
    BJob* jobs = nullptr;
    TileDesc* td[mhd::KIND_COUNT] = {};
    unsigned nblocks[mhd::KIND_COUNT] = {};
    long long cells = 0;         // total cells of the members (picks the launches' cache policy)
    hipGraphExec_t exec[3] = {nullptr, nullptr, nullptr};
    double exec_cfl[3] = {0.0, 0.0, 0.0};
};

using ShapeKey = std::array<int, 5>;   // nx, ny, nz, boundary condition, kind

// Pinned host staging for table uploads: a slot is rewritten only after the
// copy that last read it has completed.
struct Staging {
    void* host = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
};
constexpr int kStaging = 4;

__global__ void init_ctl_kernel(Ctl* c)
{
    if (threadIdx.x == 0) {
        c->dt = 0.0;
        c->t = 0.0;
        c->t_stop = -1.0;
        c->cmax = 0.0;
        c->divb = 0.0;
        c->status = 0;
        c->nparts = 0;
    }
}

}  // namespace

struct mhd_batch {
    int dtype;
    size_t esize;
    int device;
    hipStream_t stream;
    hipStream_t own_stream;
    bool graphs;
    int next_id;
    std::map<int, Prob> probs;
    std::vector<Cohort> cohorts;
    std::map<ShapeKey, std::pair<int, int>> tuned;   // tile per grid shape, boundary condition and kind
    Staging staging[kStaging];
    int next_staging;
    std::vector<hipGraphExec_t> dead_graphs;   // released once the stream has drained past them
    std::vector<void*> dead_dev;
};

namespace {

int fail(int code, const char* msg) { return mhd::report(code, msg); }
int hip_fail(hipError_t e, const char* where) { return mhd::report_hip(e, where); }

#define HIPCHK(call, where)                               \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return hip_fail(e_, where); \
    } while (0)

int set_current(const mhd_batch* b)
{
    int dev = -1;
    HIPCHK(hipGetDevice(&dev), "hipGetDevice");
    if (dev != b->device) HIPCHK(hipSetDevice(b->device), "hipSetDevice");
    return MHD_OK;
}

template <typename T>
void tile_of(const mhd_batch* b, const Grid& g, int kind, int* p0, int* p1)
{
    auto it = b->tuned.find(ShapeKey{g.n[0], g.n[1], g.n[2], g.bc, kind});
    if (it != b->tuned.end()) {
        *p0 = it->second.first;
        *p1 = it->second.second;
    } else {
        mhd::tile_default<T>(g, kind, p0, p1);
    }
}

void tile_of_dyn(const mhd_batch* b, const Grid& g, int kind, int* p0, int* p1)
{
    if (b->dtype == MHD_F64)
        tile_of<double>(b, g, kind, p0, p1);
    else
        tile_of<float>(b, g, kind, p0, p1);
}

// Reduction slots a problem needs: the most workgroups any c_max-producing
// launch (the c_max pass, a fluid sweep, a fused reverse sweep) can give it,
// over all candidate tiles.
template <typename T>
size_t parts_capacity(const Grid& g)
{
    size_t cap = 1;
    std::vector<std::pair<int, int>> cand;
    for (int kind : {mhd::KIND_CFL, mhd::KIND_FLUID_X, mhd::KIND_FLUID_Y, mhd::KIND_FLUID_Z, mhd::KIND_CTFLUID_X,
                     mhd::KIND_CTFLUID_Y, mhd::KIND_CTFLUID_Z}) {
        mhd::tile_candidates<T>(g, kind, cand);
        for (auto& c : cand) cap = std::max(cap, (size_t)mhd::tile_blocks<T>(g, kind, c.first, c.second));
    }
    return cap;
}

size_t problem_layout(const Grid& g, int dtype, size_t offs[6])
{
    const size_t es = dtype == MHD_F64 ? 8 : 4;
    const size_t N = (size_t)g.N;
    const size_t cap = dtype == MHD_F64 ? parts_capacity<double>(g) : parts_capacity<float>(g);
    const size_t sizes[6] = {5 * N * es, 5 * N * es, 3 * N * es, 3 * N * es, sizeof(Ctl),
                             cap * sizeof(unsigned long long)};
    size_t off = 0;
    for (int k = 0; k < 6; k++) {
        offs[k] = off;
        off += align_up(sizes[k]);
    }
    return off;
}

// Grid and problem constants a problem may have (at most 2^36 cells: the
// sweeps index wavefronts and workgroups with 32 bits).
bool grid_ok(int nx, int ny, int nz, double gamma, int bc)
{
    return nx >= 1 && ny >= 1 && nz >= 1 && (long long)nx * ny * nz <= (1LL << 36) && gamma > 1.0 &&
           std::isfinite(gamma) && (bc == MHD_BC_PERIODIC || bc == MHD_BC_OUTFLOW);
}

// Release retired graphs and buffers once no queued work can use them
// (wait: drain the stream first).
void reap(mhd_batch* b, bool wait)
{
    if (b->dead_graphs.empty() && b->dead_dev.empty()) return;
    if (wait)
        (void)hipStreamSynchronize(b->stream);
    else if (hipStreamQuery(b->stream) != hipSuccess)
        return;
    for (hipGraphExec_t g : b->dead_graphs) (void)hipGraphExecDestroy(g);
    for (void* p : b->dead_dev) (void)hipFree(p);
    b->dead_graphs.clear();
    b->dead_dev.clear();
}

void drop_graphs(mhd_batch* b, Cohort& c)
{
    for (int q = 0; q < 3; q++) {
        if (c.exec[q]) b->dead_graphs.push_back(c.exec[q]);
        c.exec[q] = nullptr;
    }
}

void free_cohort(mhd_batch* b, Cohort& c)
{
    drop_graphs(b, c);
    if (c.dev) b->dead_dev.push_back(c.dev);
    c.dev = nullptr;
    c.dev_bytes = 0;
}

// Stream-ordered upload of host data through the pinned staging ring.
int upload(mhd_batch* b, void* dst, const void* src, size_t bytes)
{
    Staging& st = b->staging[b->next_staging];
    b->next_staging = (b->next_staging + 1) % kStaging;
    if (st.pending) {
        HIPCHK(hipEventSynchronize(st.done), "staging wait");
        st.pending = false;
    }
    if (st.bytes < bytes) {
        if (st.host) (void)hipHostFree(st.host);
        st.host = nullptr;
        st.bytes = 0;
        const size_t want = std::max(bytes, (size_t)1 << 16);
        HIPCHK(hipHostMalloc(&st.host, want, hipHostMallocDefault), "pinned staging allocation");
        st.bytes = want;
    }
    if (!st.done) HIPCHK(hipEventCreateWithFlags(&st.done, hipEventDisableTiming), "hipEventCreate");
    std::memcpy(st.host, src, bytes);
    HIPCHK(hipMemcpyAsync(dst, st.host, bytes, hipMemcpyHostToDevice, b->stream), "table upload");
    HIPCHK(hipEventRecord(st.done, b->stream), "hipEventRecord");
    st.pending = true;
    return MHD_OK;
}

// A cohort runs reverse L_d as one fused launch (the field update, then the
// fluid update, of the same bits as the two launches) when every member is
// periodic with more than one cell along d (512 Alfven problems: FP32 7.69 ->
// 8.23, FP64 3.08 -> 3.23 G cell-updates/s).
bool fuse_axis(const std::vector<BJob>& jobs, int axis)
{
    if (jobs.empty()) return false;
    for (const BJob& J : jobs)
        if (J.g.bc != MHD_BC_PERIODIC || J.g.n[axis] == 1) return false;
    return true;
}

// Job table and per-kind tile tables of a cohort, rebuilt in device memory.
int build_tables(mhd_batch* b, Cohort& c)
{
    drop_graphs(b, c);
    const int n = (int)c.ids.size();
    std::vector<BJob> jobs(n);
    std::vector<TileDesc> td[mhd::KIND_COUNT];
    for (int k = 0; k < mhd::KIND_COUNT; k++) {
        td[k].resize(n + 1);
    }
    for (int j = 0; j < n; j++) {
        const Prob& p = b->probs.at(c.ids[j]);
        BJob& J = jobs[j];
        J.u[0] = p.u[0];
        J.u[1] = p.u[1];
        J.b[0] = p.b[0];
        J.b[1] = p.b[1];
        J.ctl = p.ctl;
        J.parts = p.parts;
        J.g = p.g;
        J.gamma = p.gamma;
    }
    c.cells = 0;
    for (const BJob& J : jobs) c.cells += J.g.N;
    for (int k = 0; k < mhd::KIND_COUNT; k++) {
        unsigned first = 0;
        for (int j = 0; j < n; j++) {
            const Grid& g = jobs[j].g;
            int p0, p1;
            tile_of_dyn(b, g, k, &p0, &p1);
            const unsigned nb = b->dtype == MHD_F64 ? mhd::tile_blocks<double>(g, k, p0, p1)
                                                    : mhd::tile_blocks<float>(g, k, p0, p1);
            td[k][j].first = first;
            td[k][j].p0 = p0;
            td[k][j].p1 = p1;
            td[k][j].pad = 0;
            if ((unsigned long long)first + nb > 0x7fffffffULL) return fail(MHD_ERR_ARG, "batch launch too large");
            first += nb;
        }
        td[k][n].first = first;
        td[k][n].p0 = td[k][n].p1 = td[k][n].pad = 0;
        c.nblocks[k] = first;
    }
    const size_t jb = align_up(n * sizeof(BJob)), tb = align_up((n + 1) * sizeof(TileDesc));
    const size_t need = jb + mhd::KIND_COUNT * tb;
    if (need > c.dev_bytes) {
        if (c.dev) b->dead_dev.push_back(c.dev);   // queued steps may still read the old tables
        c.dev = nullptr;
        c.dev_bytes = 0;
        hipError_t e = hipMalloc(&c.dev, need);
        if (e != hipSuccess) {
            c.dev = nullptr;
            (void)hipGetLastError();
            return e == hipErrorOutOfMemory ? fail(MHD_ERR_OOM, "batch table allocation failed")
                                            : hip_fail(e, "hipMalloc");
        }
        c.dev_bytes = need;
    }
    // one image of all tables, uploaded in stream order (queued steps that use
    // the previous tables run before the copy)
    std::vector<char> img(need, 0);
    std::memcpy(img.data(), jobs.data(), n * sizeof(BJob));
    for (int k = 0; k < mhd::KIND_COUNT; k++)
        std::memcpy(img.data() + jb + k * tb, td[k].data(), (n + 1) * sizeof(TileDesc));
    char* base = static_cast<char*>(c.dev);
    c.jobs = reinterpret_cast<BJob*>(base);
    for (int k = 0; k < mhd::KIND_COUNT; k++) c.td[k] = reinterpret_cast<TileDesc*>(base + jb + k * tb);
    if (int rc = upload(b, c.dev, img.data(), need)) return rc;
    for (int a = 0; a < 3; a++) c.fuse[a] = fuse_axis(jobs, a);
    c.dirty = false;
    c.cmax_valid = false;
    return MHD_OK;
}

template <typename T>
int launch_kind(mhd_batch* b, Cohort& c, int kind, bool cfl_parts, int iu, int ib)
{
    const int n = (int)c.ids.size();
    HIPCHK(mhd::launch_batch<T>(kind, cfl_parts, c.jobs, c.td[kind], n, c.nblocks[kind], iu, ib,
                                b->stream, c.cells),
           "batched launch");
    return MHD_OK;
}

// The 12 sweeps of one full step in the order of phase q; the last fluid
// sweep stores the c_max slots of the state it writes.
template <typename T>
int sweeps(mhd_batch* b, Cohort& c, int q)
{
    const int* p = kPerm[q];
    int iu = 0, ib = 0, rc;
    for (int a = 0; a < 3; a++) {
        if ((rc = launch_kind<T>(b, c, mhd::KIND_FLUID_X + p[a], false, iu, ib))) return rc;
        iu ^= 1;
        if ((rc = launch_kind<T>(b, c, mhd::KIND_CT_X + p[a], false, iu, ib))) return rc;
        ib ^= 1;
    }
    for (int a = 2; a >= 0; a--) {
        if (c.fuse[p[a]]) {
            if ((rc = launch_kind<T>(b, c, mhd::KIND_CTFLUID_X + p[a], a == 0, iu, ib))) return rc;
            iu ^= 1;
            ib ^= 1;
            continue;
        }
        if ((rc = launch_kind<T>(b, c, mhd::KIND_CT_X + p[a], false, iu, ib))) return rc;
        ib ^= 1;
        if ((rc = launch_kind<T>(b, c, mhd::KIND_FLUID_X + p[a], a == 0, iu, ib))) return rc;
        iu ^= 1;
    }
    return MHD_OK;
}

template <typename T>
int cohort_step(mhd_batch* b, Cohort& c, double cfl)
{
    int rc;
    if (c.dirty && (rc = build_tables(b, c))) return rc;
    const int n = (int)c.ids.size();
    const int q = c.phase;
    if (!c.cmax_valid) {
        // first step after the cohort changed: standalone c_max pass, then
        // the step issued launch by launch
        if ((rc = launch_kind<T>(b, c, mhd::KIND_CFL, false, 0, 0))) return rc;
        HIPCHK(mhd::launch_finish_batch(c.jobs, c.td[mhd::KIND_CFL], n, cfl, b->stream), "batched dt launch");
        if ((rc = sweeps<T>(b, c, q))) return rc;
    } else if (b->graphs && b->stream != nullptr) {
        if (!c.exec[q] || c.exec_cfl[q] != cfl) {
            if (c.exec[q]) (void)hipGraphExecDestroy(c.exec[q]);
            c.exec[q] = nullptr;
            HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
            hipError_t e = mhd::launch_finish_batch(c.jobs, c.td[c.parts_kind], n, cfl, b->stream);
            int rc2 = e == hipSuccess ? sweeps<T>(b, c, q) : hip_fail(e, "batched dt launch");
            hipGraph_t graph = nullptr;
            hipError_t e2 = hipStreamEndCapture(b->stream, &graph);
            if (rc2) {
                if (graph) (void)hipGraphDestroy(graph);
                return rc2;
            }
            if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
            e2 = hipGraphInstantiate(&c.exec[q], graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e2 != hipSuccess) {
                c.exec[q] = nullptr;
                return hip_fail(e2, "hipGraphInstantiate");
            }
            c.exec_cfl[q] = cfl;
        }
        HIPCHK(hipGraphLaunch(c.exec[q], b->stream), "hipGraphLaunch");
    } else {
        HIPCHK(mhd::launch_finish_batch(c.jobs, c.td[c.parts_kind], n, cfl, b->stream), "batched dt launch");
        if ((rc = sweeps<T>(b, c, q))) return rc;
    }
    c.cmax_valid = true;
    c.parts_kind = (c.fuse[kPerm[q][0]] ? mhd::KIND_CTFLUID_X : mhd::KIND_FLUID_X) + kPerm[q][0];
    c.phase = (q + 1) % 3;
    for (int id : c.ids) b->probs.at(id).s += 1;
    return MHD_OK;
}

// Cohort a new problem with step counter s joins (created if needed).
Cohort& cohort_for(mhd_batch* b, long long s)
{
    const int phase = (int)(s % 3);
    for (auto& c : b->cohorts)
        if (c.phase == phase && !c.ids.empty()) return c;
    for (auto& c : b->cohorts)
        if (c.ids.empty()) {
            c.phase = phase;
            return c;
        }
    b->cohorts.emplace_back();
    b->cohorts.back().phase = phase;
    return b->cohorts.back();
}

// Place a problem's arrays in its block and initialise its control block on
// the batch's stream.
int place(mhd_batch* b, Prob& p, void* block)
{
    size_t offs[6];
    p.bytes = problem_layout(p.g, b->dtype, offs);
    p.mem = block;
    char* base = static_cast<char*>(block);
    p.u[0] = base + offs[0];
    p.u[1] = base + offs[1];
    p.b[0] = base + offs[2];
    p.b[1] = base + offs[3];
    p.ctl = reinterpret_cast<Ctl*>(base + offs[4]);
    p.parts = reinterpret_cast<unsigned long long*>(base + offs[5]);
    hipLaunchKernelGGL(init_ctl_kernel, dim3(1), dim3(64), 0, b->stream, p.ctl);
    HIPCHK(hipGetLastError(), "control block init");
    return MHD_OK;
}

// Device check of a problem's copy-0 state (after place()): a non-finite
// value or a non-positive density latches status -1.
int check_state(mhd_batch* b, const Prob& p)
{
    hipError_t e = b->dtype == MHD_F64
                       ? mhd::launch_validate<double>(static_cast<const double*>(p.u[0]),
                                                      static_cast<const double*>(p.b[0]), p.g.N, p.ctl, b->stream)
                       : mhd::launch_validate<float>(static_cast<const float*>(p.u[0]),
                                                     static_cast<const float*>(p.b[0]), p.g.N, p.ctl, b->stream);
    HIPCHK(e, "state check launch");
    return MHD_OK;
}

int enlist(mhd_batch* b, const Prob& p, int* id)
{
    const int nid = b->next_id++;
    b->probs[nid] = p;
    Cohort& c = cohort_for(b, 0);
    c.ids.push_back(nid);
    c.dirty = true;
    *id = nid;
    return MHD_OK;
}

bool make_prob(Prob& p, int nx, int ny, int nz, double gamma, int bc)
{
    if (!grid_ok(nx, ny, nz, gamma, bc)) return false;
    p.g.n[0] = nx;
    p.g.n[1] = ny;
    p.g.n[2] = nz;
    p.g.bc = bc;
    p.g.N = (long long)nx * ny * nz;
    p.gamma = gamma;
    p.s = 0;
    return true;
}

int add_problem(mhd_batch* b, int nx, int ny, int nz, double gamma, int bc, const void* state, hipMemcpyKind kind,
                int* id)
{
    if (!b) return fail(MHD_ERR_ARG, "null batch");
    if (!id) return fail(MHD_ERR_ARG, "null output pointer");
    if (!state) return fail(MHD_ERR_ARG, "null state pointer");
    Prob p;
    if (!make_prob(p, nx, ny, nz, gamma, bc)) return fail(MHD_ERR_ARG, "invalid grid, gamma or boundary condition");
    if (int rc = set_current(b)) return rc;
    size_t offs[6];
    void* block = nullptr;
    hipError_t e = hipMalloc(&block, problem_layout(p.g, b->dtype, offs));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return e == hipErrorOutOfMemory ? fail(MHD_ERR_OOM, "device allocation failed") : hip_fail(e, "hipMalloc");
    }
    p.owned = true;
    int rc = place(b, p, block);
    const size_t N = (size_t)p.g.N, es = b->esize;
    const char* src = static_cast<const char*>(state);
    if (rc == MHD_OK) {
        e = hipMemcpyAsync(p.u[0], src, 5 * N * es, kind, b->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(p.b[0], src + 5 * N * es, 3 * N * es, kind, b->stream);
        if (e != hipSuccess) rc = hip_fail(e, "state copy in");
    }
    if (rc == MHD_OK) rc = check_state(b, p);
    if (rc == MHD_OK) {
        // the caller may reuse its buffer on return; a rejected state is not added
        int status = 0;
        e = hipMemcpyAsync(&status, &p.ctl->status, sizeof(int), hipMemcpyDeviceToHost, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess)
            rc = hip_fail(e, "state check");
        else if (status != 0)
            rc = fail(MHD_ERR_ARG, "state has a non-finite value or a non-positive density");
    }
    if (rc != MHD_OK) {
        (void)hipStreamSynchronize(b->stream);
        (void)hipFree(block);
        return rc;
    }
    return enlist(b, p, id);
}

Prob* find(mhd_batch* b, int id)
{
    auto it = b->probs.find(id);
    return it == b->probs.end() ? nullptr : &it->second;
}

int read_ctl(mhd_batch* b, const Prob& p, Ctl* out)
{
    HIPCHK(hipMemcpyAsync(out, p.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, b->stream), "read control block");
    HIPCHK(hipStreamSynchronize(b->stream), "stream sync");
    return MHD_OK;
}

template <typename T>
int autotune(mhd_batch* b, int reps)
{
    // one timing per grid shape and boundary condition (the lane-row x sweeps
    // and the fused reverse sweeps apply to periodic grids only)
    std::map<std::array<int, 4>, std::vector<int>> shapes;
    long long all_cells = 0;
    for (auto& kv : b->probs) {
        shapes[{kv.second.g.n[0], kv.second.g.n[1], kv.second.g.n[2], kv.second.g.bc}].push_back(kv.first);
        all_cells += kv.second.g.N;
    }
    if (shapes.empty()) return MHD_OK;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0), "hipEventCreate");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(MHD_ERR_DEVICE, "hipEventCreate failed");
    }
    Cohort tmp;   // scratch tables, one shape at a time
    int rc = MHD_OK;
    std::vector<std::pair<int, int>> cand;
    for (auto& sh : shapes) {
        tmp.ids = sh.second;
        const Grid g = b->probs.at(sh.second[0]).g;
        for (int kind = mhd::KIND_FLUID_X; kind <= mhd::KIND_CTFLUID_Z && rc == MHD_OK; kind++) {
            if (kind >= mhd::KIND_CTFLUID_X &&
                (g.bc != MHD_BC_PERIODIC || g.n[kind - mhd::KIND_CTFLUID_X] == 1))
                continue;
            mhd::tile_candidates<T>(g, kind, cand);
            double best = 1e300;
            std::pair<int, int> pick = cand[0];
            for (auto& cd : cand) {
                b->tuned[ShapeKey{g.n[0], g.n[1], g.n[2], g.bc, kind}] = cd;
                if ((rc = build_tables(b, tmp))) break;
                // timed under the cache policy of the whole batch's launches
                tmp.cells = all_cells;
                // copy 0 -> copy 1 (scratch between steps)
                if ((rc = launch_kind<T>(b, tmp, kind, false, 0, 0))) break;
                hipError_t e = hipEventRecord(e0, b->stream);
                for (int r = 0; r < reps && e == hipSuccess && rc == MHD_OK; r++)
                    rc = launch_kind<T>(b, tmp, kind, false, 0, 0);
                if (rc) break;
                if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) {
                    rc = hip_fail(e, "autotune timing");
                    break;
                }
                if (ms < best) {
                    best = ms;
                    pick = cd;
                }
            }
            b->tuned[ShapeKey{g.n[0], g.n[1], g.n[2], g.bc, kind}] = pick;
        }
        if (rc) break;
    }
    free_cohort(b, tmp);
    reap(b, true);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (auto& c : b->cohorts) c.dirty = true;
    return rc;
}

template <typename T>
bool tile_is_candidate(const Grid& g, int kind, int p0, int p1)
{
    std::vector<std::pair<int, int>> cand;
    mhd::tile_candidates<T>(g, kind, cand);
    for (auto& c : cand)
        if (c.first == p0 && c.second == p1) return true;
    return false;
}

}  // namespace

extern "C" {

size_t mhd_batch_problem_bytes(int nx, int ny, int nz, int dtype)
{
    if (!grid_ok(nx, ny, nz, 2.0, MHD_BC_PERIODIC) || (dtype != MHD_F32 && dtype != MHD_F64)) return 0;
    Grid g;
    g.n[0] = nx;
    g.n[1] = ny;
    g.n[2] = nz;
    g.bc = 0;
    g.N = (long long)nx * ny * nz;
    size_t offs[6];
    return problem_layout(g, dtype, offs);
}

int mhd_batch_create(int dtype, mhd_batch_t** out)
{
    if (!out) return fail(MHD_ERR_ARG, "null output pointer");
    *out = nullptr;
    if (dtype != MHD_F32 && dtype != MHD_F64) return fail(MHD_ERR_ARG, "unknown dtype");
    mhd_batch* b = new (std::nothrow) mhd_batch();
    if (!b) return fail(MHD_ERR_OOM, "host allocation failed");
    b->dtype = dtype;
    b->esize = dtype == MHD_F64 ? 8 : 4;
    b->graphs = true;
    b->next_id = 1;
    b->next_staging = 0;
    b->own_stream = nullptr;
    hipError_t e = hipGetDevice(&b->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->own_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete b;
        return hip_fail(e, "batch stream");
    }
    b->stream = b->own_stream;
    *out = b;
    return MHD_OK;
}

int mhd_batch_destroy(mhd_batch_t* b)
{
    if (!b) return MHD_OK;
    (void)set_current(b);
    for (auto& c : b->cohorts) free_cohort(b, c);
    reap(b, true);
    for (auto& kv : b->probs)
        if (kv.second.owned) (void)hipFree(kv.second.mem);
    for (auto& st : b->staging) {
        if (st.host) (void)hipHostFree(st.host);
        if (st.done) (void)hipEventDestroy(st.done);
    }
    if (b->own_stream) (void)hipStreamDestroy(b->own_stream);
    delete b;
    return MHD_OK;
}

int mhd_batch_set_stream(mhd_batch_t* b, void* stream)
{
    if (!b) return fail(MHD_ERR_ARG, "null batch");
    if (int rc = set_current(b)) return rc;
    HIPCHK(hipStreamSynchronize(b->stream), "stream sync");
    b->stream = static_cast<hipStream_t>(stream);
    return MHD_OK;
}

int mhd_batch_add(mhd_batch_t* b, int nx, int ny, int nz, double gamma, int bc, const void* host_state, int* id)
{
    return add_problem(b, nx, ny, nz, gamma, bc, host_state, hipMemcpyHostToDevice, id);
}

int mhd_batch_add_device(mhd_batch_t* b, int nx, int ny, int nz, double gamma, int bc, const void* dev_state, int* id)
{
    return add_problem(b, nx, ny, nz, gamma, bc, dev_state, hipMemcpyDeviceToDevice, id);
}

int mhd_batch_problem_layout(int nx, int ny, int nz, int dtype, size_t* off_u0, size_t* off_b0, size_t* off_ctl,
                             size_t* bytes)
{
    if (!grid_ok(nx, ny, nz, 2.0, MHD_BC_PERIODIC) || (dtype != MHD_F32 && dtype != MHD_F64))
        return fail(MHD_ERR_ARG, "invalid grid or dtype");
    Grid g;
    g.n[0] = nx;
    g.n[1] = ny;
    g.n[2] = nz;
    g.bc = 0;
    g.N = (long long)nx * ny * nz;
    size_t offs[6];
    const size_t total = problem_layout(g, dtype, offs);
    if (off_u0) *off_u0 = offs[0];
    if (off_b0) *off_b0 = offs[2];
    if (off_ctl) *off_ctl = offs[4];
    if (bytes) *bytes = total;
    return MHD_OK;
}

int mhd_batch_add_inplace(mhd_batch_t* b, int nx, int ny, int nz, double gamma, int bc, void* dev_block, void* ready,
                          int* id)
{
    if (!b) return fail(MHD_ERR_ARG, "null batch");
    if (!id || !dev_block) return fail(MHD_ERR_ARG, "null pointer");
    Prob p;
    if (!make_prob(p, nx, ny, nz, gamma, bc)) return fail(MHD_ERR_ARG, "invalid grid, gamma or boundary condition");
    if (int rc = set_current(b)) return rc;
    if (ready) HIPCHK(hipStreamWaitEvent(b->stream, static_cast<hipEvent_t>(ready), 0), "hipStreamWaitEvent");
    p.owned = false;
    if (int rc = place(b, p, dev_block)) return rc;
    if (int rc = check_state(b, p)) return rc;   // a rejected state latches its status
    return enlist(b, p, id);
}

int mhd_batch_record(mhd_batch_t* b, void* event)
{
    if (!b || !event) return fail(MHD_ERR_ARG, "null pointer");
    if (int rc = set_current(b)) return rc;
    HIPCHK(hipEventRecord(static_cast<hipEvent_t>(event), b->stream), "hipEventRecord");
    return MHD_OK;
}

int mhd_batch_remove(mhd_batch_t* b, int id)
{
    if (!b) return fail(MHD_ERR_ARG, "null batch");
    Prob* p = find(b, id);
    if (!p) return fail(MHD_ERR_ARG, "unknown problem id");
    if (int rc = set_current(b)) return rc;
    for (auto& c : b->cohorts) {
        auto it = std::find(c.ids.begin(), c.ids.end(), id);
        if (it != c.ids.end()) {
            c.ids.erase(it);
            c.dirty = true;
            drop_graphs(b, c);
            if (c.ids.empty()) free_cohort(b, c);
        }
    }
    if (p->owned) {
        HIPCHK(hipStreamSynchronize(b->stream), "stream sync");
        HIPCHK(hipFree(p->mem), "hipFree");
    }
    b->probs.erase(id);
    reap(b, false);
    return MHD_OK;
}

int mhd_batch_count(mhd_batch_t* b, int* n, size_t* bytes)
{
    if (!b) return fail(MHD_ERR_ARG, "null batch");
    size_t tot = 0;
    for (auto& kv : b->probs) tot += kv.second.bytes;
    if (n) *n = (int)b->probs.size();
    if (bytes) *bytes = tot;
    return MHD_OK;
}

int mhd_batch_step(mhd_batch_t* b, int n, double cfl)
{
    if (!b) return fail(MHD_ERR_ARG, "null batch");
    if (n < 0) return fail(MHD_ERR_ARG, "negative step count");
    if (!(cfl > 0.0 && cfl <= 1.0)) return fail(MHD_ERR_ARG, "cfl must be in (0, 1]");
    if (int rc = set_current(b)) return rc;
    reap(b, false);
    for (int k = 0; k < n; k++)
        for (auto& c : b->cohorts) {
            if (c.ids.empty()) continue;
            int rc = b->dtype == MHD_F64 ? cohort_step<double>(b, c, cfl) : cohort_step<float>(b, c, cfl);
            if (rc) return rc;
        }
    return MHD_OK;
}

static int copy_out(mhd_batch_t* b, int id, void* dst, hipMemcpyKind kind)
{
    if (!b) return fail(MHD_ERR_ARG, "null batch");
    if (!dst) return fail(MHD_ERR_ARG, "null state pointer");
    Prob* p = find(b, id);
    if (!p) return fail(MHD_ERR_ARG, "unknown problem id");
    if (int rc = set_current(b)) return rc;
    const size_t N = (size_t)p->g.N, es = b->esize;
    char* d = static_cast<char*>(dst);
    HIPCHK(hipMemcpyAsync(d, p->u[0], 5 * N * es, kind, b->stream), "state copy out");
    HIPCHK(hipMemcpyAsync(d + 5 * N * es, p->b[0], 3 * N * es, kind, b->stream), "state copy out");
    return MHD_OK;
}

int mhd_batch_get_state(mhd_batch_t* b, int id, void* host_state)
{
    if (int rc = copy_out(b, id, host_state, hipMemcpyDeviceToHost)) return rc;
    HIPCHK(hipStreamSynchronize(b->stream), "stream sync");
    return MHD_OK;
}

int mhd_batch_get_state_device(mhd_batch_t* b, int id, void* dev_state)
{
    return copy_out(b, id, dev_state, hipMemcpyDeviceToDevice);
}

int mhd_batch_get_time(mhd_batch_t* b, int id, double* t, int64_t* s)
{
    if (!b) return fail(MHD_ERR_ARG, "null batch");
    Prob* p = find(b, id);
    if (!p) return fail(MHD_ERR_ARG, "unknown problem id");
    if (int rc = set_current(b)) return rc;
    Ctl c;
    if (int rc = read_ctl(b, *p, &c)) return rc;
    if (t) *t = c.t;
    if (s) *s = p->s;
    return MHD_OK;
}

int mhd_batch_set_stop_time(mhd_batch_t* b, int id, double t_stop)
{
    if (!b) return fail(MHD_ERR_ARG, "null batch");
    if (std::isnan(t_stop)) return fail(MHD_ERR_ARG, "stop time is NaN");
    Prob* p = find(b, id);
    if (!p) return fail(MHD_ERR_ARG, "unknown problem id");
    if (int rc = set_current(b)) return rc;
    const double v = t_stop < 0.0 ? -1.0 : t_stop;
    HIPCHK(hipMemcpyAsync(&p->ctl->t_stop, &v, sizeof(double), hipMemcpyHostToDevice, b->stream), "write stop time");
    HIPCHK(hipStreamSynchronize(b->stream), "stream sync");
    return MHD_OK;
}

int mhd_batch_status(mhd_batch_t* b, int id)
{
    if (!b) return fail(MHD_ERR_ARG, "null batch");
    Prob* p = find(b, id);
    if (!p) return fail(MHD_ERR_ARG, "unknown problem id");
    if (int rc = set_current(b)) return rc;
    Ctl c;
    if (int rc = read_ctl(b, *p, &c)) return rc;
    if (c.status == -1) return fail(MHD_ERR_ARG, "the problem's initial state was rejected");
    return c.status != 0 ? fail(MHD_ERR_NONFINITE, "non-finite or non-positive c_max; state frozen") : MHD_OK;
}

int mhd_batch_set_graphs(mhd_batch_t* b, int enable)
{
    if (!b) return fail(MHD_ERR_ARG, "null batch");
    b->graphs = enable != 0;
    return MHD_OK;
}

int mhd_batch_autotune(mhd_batch_t* b, int reps)
{
    if (!b) return fail(MHD_ERR_ARG, "null batch");
    if (reps < 1) return fail(MHD_ERR_ARG, "reps must be >= 1");
    if (int rc = set_current(b)) return rc;
    HIPCHK(hipStreamSynchronize(b->stream), "stream sync");
    return b->dtype == MHD_F64 ? autotune<double>(b, reps) : autotune<float>(b, reps);
}

int mhd_batch_set_tile(mhd_batch_t* b, int id, int kind, int p0, int p1)
{
    if (!b) return fail(MHD_ERR_ARG, "null batch");
    if (kind < mhd::KIND_FLUID_X || kind > mhd::KIND_CTFLUID_Z) return fail(MHD_ERR_ARG, "not a sweep kind");
    Prob* p = find(b, id);
    if (!p) return fail(MHD_ERR_ARG, "unknown problem id");
    const Grid& g = p->g;
    const bool ok = b->dtype == MHD_F64 ? tile_is_candidate<double>(g, kind, p0, p1)
                                        : tile_is_candidate<float>(g, kind, p0, p1);
    if (!ok) return fail(MHD_ERR_ARG, "not a tile the autotuner would consider for this grid and kind");
    if (int rc = set_current(b)) return rc;
    HIPCHK(hipStreamSynchronize(b->stream), "stream sync");
    b->tuned[ShapeKey{g.n[0], g.n[1], g.n[2], g.bc, kind}] = {p0, p1};
    for (auto& c : b->cohorts) c.dirty = true;
    return MHD_OK;
}

int mhd_batch_tile(mhd_batch_t* b, int id, int kind, int* p0, int* p1)
{
    if (!b) return fail(MHD_ERR_ARG, "null batch");
    if (kind < 0 || kind >= mhd::KIND_COUNT) return fail(MHD_ERR_ARG, "unknown kernel kind");
    Prob* p = find(b, id);
    if (!p) return fail(MHD_ERR_ARG, "unknown problem id");
    int a, c;
    tile_of_dyn(b, p->g, kind, &a, &c);
    if (p0) *p0 = a;
    if (p1) *p1 = c;
    return MHD_OK;
}

}  // extern "C"

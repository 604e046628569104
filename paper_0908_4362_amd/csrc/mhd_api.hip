// Host runtime and C ABI of the MHD step library (declared in include/mhd.h).
//
// A handle owns two ping-pong copies of the conserved fields (5 x N) and of
// the face fields (3 x N), a device control block holding dt, t, the stop
// time, c_max and a latched status word, and a small array of per-workgroup
// maxima for the two-level reductions. Every sweep reads one copy and writes
// the other, so a full step (6 fluid and 6 field sweeps) returns both to the
// copy it started from.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/mhd.h"
#include "mhd_internal.h"

using mhd::Ctl;
using mhd::Grid;

struct mhd_solver {
    Grid g;
    double gamma;
    int dtype;            // MHD_F32 / MHD_F64
    size_t esize;         // bytes per element
    void* u[2];           // conserved fields, ping-pong
    void* b[2];           // face fields, ping-pong
    int ucur, bcur;       // current copies
    Ctl* ctl;             // device control block
    unsigned long long* parts;  // per-workgroup maxima: [0, cap) c_max, [cap, 2 cap) div B
    size_t cap;           // (the count of c_max slots written last lives in ctl->nparts)
    hipStream_t stream;
    long long s;          // step counter (host mirror; the sweep order needs it on the host)
    int device;
    bool cmax_valid;      // parts hold the CFL maxima of the current state (from the last step)
    bool bound;           // buffers live in a caller-owned workspace (mhd_bind_workspace)
    // full steps replayed from HIP graphs, one per sweep order (s mod 3)
    bool graphs;
    int fusion;           // reverse L_d as one launch: 0 never, 1 where faster, 2 wherever it applies
    hipGraphExec_t exec[3];
    double exec_cfl[3];
    // optional per-kernel timing with HIP events on the handle's stream
    bool timing;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[MHD_K_COUNT];
    std::vector<hipEvent_t> pool;
    double total_ms[MHD_K_COUNT];
    long long launches[MHD_K_COUNT];
};

namespace {

thread_local std::string g_err;

int fail(int code, const char* msg)
{
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* where)
{
    g_err = std::string(where) + ": " + hipGetErrorString(e);
    return MHD_ERR_DEVICE;
}

#define HIPCHK(call, where)                            \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) return hip_fail(e_, where); \
    } while (0)

hipEvent_t take_event(mhd_solver* h)
{
    if (!h->pool.empty()) {
        hipEvent_t e = h->pool.back();
        h->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Launch through f(), bracketed by events when timing is on.
template <typename F>
int timed(mhd_solver* h, int kind, F&& f, const char* where)
{
    hipEvent_t a = nullptr, b = nullptr;
    // events taken but not queued go back to the pool on every error path
    auto give_back = [h, &a, &b] {
        if (a) h->pool.push_back(a);
        if (b) h->pool.push_back(b);
        a = b = nullptr;
    };
    if (h->timing) {
        a = take_event(h);
        b = take_event(h);
        if (!a || !b) {
            give_back();
            return fail(MHD_ERR_DEVICE, "hipEventCreate failed");
        }
        const hipError_t e = hipEventRecord(a, h->stream);
        if (e != hipSuccess) {
            give_back();
            return hip_fail(e, "hipEventRecord");
        }
    }
    hipError_t e = f();
    if (e == hipSuccess && h->timing) e = hipEventRecord(b, h->stream);
    if (e != hipSuccess) {
        give_back();
        return hip_fail(e, where);
    }
    if (h->timing) h->pending[kind].emplace_back(a, b);
    return MHD_OK;
}

template <typename T>
int fluid(mhd_solver* h, int axis, double dt, bool with_cfl = false)
{
    const T* uin = static_cast<const T*>(h->u[h->ucur]);
    T* uout = static_cast<T*>(h->u[h->ucur ^ 1]);
    const T* b = static_cast<const T*>(h->b[h->bcur]);
    int rc = timed(h, MHD_K_FLUID_X + axis,
                   [&] {
                       return mhd::launch_fluid<T>(axis, uin, uout, b, h->g, h->gamma, h->ctl, dt,
                                                   with_cfl ? h->parts : nullptr, h->stream);
                   },
                   "fluid sweep launch");
    if (rc) return rc;
    h->ucur ^= 1;
    return MHD_OK;
}

template <typename T>
int ct(mhd_solver* h, int axis, double dt)
{
    const T* u = static_cast<const T*>(h->u[h->ucur]);
    const T* bin = static_cast<const T*>(h->b[h->bcur]);
    T* bout = static_cast<T*>(h->b[h->bcur ^ 1]);
    int rc = timed(h, MHD_K_CT_X + axis,
                   [&] {
                       return axis > 0 && h->g.n[axis] == 1
                                  ? mhd::launch_ct_flat<T>(axis, u, bin, bout, h->g, h->ctl, dt, h->stream)
                                  : mhd::launch_ct<T>(axis, u, bin, bout, h->g, h->ctl, dt, h->stream);
                   },
                   "field sweep launch");
    if (rc) return rc;
    h->bcur ^= 1;
    return MHD_OK;
}

// Reverse L_d in one launch: the field update along axis, then the fluid
// update on the new field (both copies flip).
template <typename T>
int ct_fluid(mhd_solver* h, int axis, double dt, bool with_cfl)
{
    const T* uin = static_cast<const T*>(h->u[h->ucur]);
    T* uout = static_cast<T*>(h->u[h->ucur ^ 1]);
    const T* bin = static_cast<const T*>(h->b[h->bcur]);
    T* bout = static_cast<T*>(h->b[h->bcur ^ 1]);
    int rc = timed(h, MHD_K_CTFLUID_X + axis,
                   [&] {
                       return mhd::launch_ct_fluid<T>(axis, uin, uout, bin, bout, h->g, h->gamma, h->ctl, dt,
                                                      with_cfl ? h->parts : nullptr, h->stream);
                   },
                   "fused field and fluid sweep launch");
    if (rc) return rc;
    h->ucur ^= 1;
    h->bcur ^= 1;
    return MHD_OK;
}

// The fused launch covers reverse L_d of a periodic grid whose fluid sweep
// along d runs (more than one cell), where it is the faster form.
bool fused_reverse(const mhd_solver* h, int axis)
{
    if (!h->fusion || h->g.bc != MHD_BC_PERIODIC || h->g.n[axis] == 1) return false;
    if (h->fusion == 2) return true;
    return h->dtype == MHD_F64 ? mhd::fused_reverse_pays<double>(h->g, axis)
                               : mhd::fused_reverse_pays<float>(h->g, axis);
}

// The 12 sub-operations of one full step with sweep-order index s
// (eq. L_sequence): forward L_d = fluid_d then the field update along d;
// reverse L_d with the field update first; axis order (x,y,z), (z,x,y),
// (y,z,x) by s mod 3. With reduce_cmax the last fluid sweep also stores the
// per-workgroup maxima of the CFL speed of the state it writes.
//
// A fluid sweep along an axis of one cell is the identity, bit for bit: every
// stencil neighbour is that cell, so fluxes, slopes and flux differences are
// exact zeros and u - dt * 0 = u. Such sweeps are skipped, always in pairs
// (forward and reverse), so the ping-pong copies still end where they started.
// When the skipped pair was the one whose reverse sweep produces the c_max
// maxima, a standalone pass over the final state produces them instead (the
// same per-cell speeds, so the same maximum bit for bit; it reads the state
// once and writes nothing, where the two sweeps read it twice and wrote it
// twice). The field sweep along such an axis is not skipped: its constraint
// update of B_d uses EMFs of neighbouring pencils, which a velocity along d
// makes non-zero; along y or z it runs in closed form (launch_ct_flat).
template <typename T>
int cfl_parts(mhd_solver* h);

template <typename T>
int sweeps(mhd_solver* h, long long s, double dt, bool reduce_cmax)
{
    static const int perm[3][3] = {{0, 1, 2}, {2, 0, 1}, {1, 2, 0}};
    const int* p = perm[((s % 3) + 3) % 3];
    int rc;
    for (int a = 0; a < 3; a++) {
        if (h->g.n[p[a]] > 1)
            if ((rc = fluid<T>(h, p[a], dt))) return rc;
        if ((rc = ct<T>(h, p[a], dt))) return rc;
    }
    for (int a = 2; a >= 0; a--) {
        if (fused_reverse(h, p[a])) {
            if ((rc = ct_fluid<T>(h, p[a], dt, reduce_cmax && a == 0))) return rc;
            continue;
        }
        if ((rc = ct<T>(h, p[a], dt))) return rc;
        if (h->g.n[p[a]] > 1)
            if ((rc = fluid<T>(h, p[a], dt, reduce_cmax && a == 0))) return rc;
    }
    if (reduce_cmax && h->g.n[p[0]] == 1) return cfl_parts<T>(h);
    return MHD_OK;
}

// Per-workgroup CFL maxima of the current state into parts (standalone pass).
template <typename T>
int cfl_parts(mhd_solver* h)
{
    const T* u = static_cast<const T*>(h->u[h->ucur]);
    const T* b = static_cast<const T*>(h->b[h->bcur]);
    return timed(h, MHD_K_CFL,
                 [&] { return mhd::launch_cfl<T>(u, b, h->g, h->gamma, h->parts, h->ctl, h->stream); },
                 "cfl launch");
}

void drop_graphs(mhd_solver* h)
{
    for (int q = 0; q < 3; q++) {
        if (h->exec[q]) (void)hipGraphExecDestroy(h->exec[q]);
        h->exec[q] = nullptr;
    }
}

// One full step (the dt rule on the previous step's c_max slots, then the 12
// sweeps) captured in a graph for sweep order q and launched; captured again
// when cfl changes. The finisher takes the slot count from the control block,
// where the producing launch stored it, so a replay reduces the right slots
// whatever produced them (the previous step in any sweep order, mhd_cmax).
template <typename T>
int graph_step(mhd_solver* h, int q, double cfl)
{
    if (!h->exec[q] || h->exec_cfl[q] != cfl) {
        if (h->exec[q]) {
            HIPCHK(hipStreamSynchronize(h->stream), "stream sync");
            (void)hipGraphExecDestroy(h->exec[q]);
            h->exec[q] = nullptr;
        }
        HIPCHK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        hipError_t e = mhd::launch_finish(h->parts, 0, 0, cfl, h->ctl, h->stream);
        int rc = e == hipSuccess ? sweeps<T>(h, h->s, -1.0, true) : hip_fail(e, "dt launch");
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(h->stream, &graph);
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
        e2 = hipGraphInstantiate(&h->exec[q], graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e2 != hipSuccess) {
            h->exec[q] = nullptr;
            return hip_fail(e2, "hipGraphInstantiate");
        }
        h->exec_cfl[q] = cfl;
    }
    HIPCHK(hipGraphLaunch(h->exec[q], h->stream), "hipGraphLaunch");
    return MHD_OK;
}

// Full steps. The time-step rule runs on c_max of the current state; its
// per-workgroup maxima come from the previous step's last fluid sweep, or from
// a standalone pass after the state was replaced. On a stream of its own (not
// the null stream), with per-kernel timing off and the state in copy 0, a
// step is replayed from its sweep order's graph.
template <typename T>
int full_steps(mhd_solver* h, int n, double cfl)
{
    for (int k = 0; k < n; k++) {
        int rc;
        const bool replay = h->graphs && h->cmax_valid && h->stream != nullptr && !h->timing && h->ucur == 0 &&
                            h->bcur == 0;
        if (replay) {
            if ((rc = graph_step<T>(h, (int)(h->s % 3), cfl))) return rc;
        } else {
            if (!h->cmax_valid && (rc = cfl_parts<T>(h))) return rc;
            rc = timed(h, MHD_K_CFL,
                       [&] { return mhd::launch_finish(h->parts, 0, 0, cfl, h->ctl, h->stream); },
                       "dt launch");
            if (rc) return rc;
            rc = sweeps<T>(h, h->s, -1.0, true);
            if (rc) return rc;
        }
        h->cmax_valid = true;
        h->s += 1;
    }
    return MHD_OK;
}

int check(const mhd_solver* h)
{
    if (!h) return fail(MHD_ERR_ARG, "null handle");
    return MHD_OK;
}

int set_current(const mhd_solver* h)
{
    int dev = -1;
    HIPCHK(hipGetDevice(&dev), "hipGetDevice");
    if (dev != h->device) HIPCHK(hipSetDevice(h->device), "hipSetDevice");
    return MHD_OK;
}

int read_ctl(mhd_solver* h, Ctl* out)
{
    HIPCHK(hipMemcpyAsync(out, h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, h->stream), "read control block");
    HIPCHK(hipStreamSynchronize(h->stream), "stream sync");
    return MHD_OK;
}

}  // namespace

namespace mhd {
int report(int code, const char* msg) { return fail(code, msg); }
int report_hip(hipError_t e, const char* where) { return hip_fail(e, where); }
}  // namespace mhd

// ---- div B without allocation: the reduction slots and the control block
// the finisher writes live in a fixed device array (one copy per device,
// kept until the process ends), whose address is looked up once per device.
namespace {
constexpr int kNoAllocSlots = 8192;   // reduce_slots never exceeds it
constexpr size_t kNoAllocBytes = kNoAllocSlots * sizeof(unsigned long long) + 256;
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (the host-side name of the
// array is a stand-in that no kernel may be given).
int scratch_ptr(int dev, void** out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(MHD_ERR_ARG, "device index beyond the supported count");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return MHD_OK;
}
}  // namespace

extern "C" {

const char* mhd_last_error(void) { return g_err.c_str(); }

// Byte offsets of a handle's six buffers (conserved fields x2, face fields
// x2, control block, reduction slots) inside one workspace, 256-aligned.
static size_t workspace_layout(const Grid& g, size_t es, size_t offs[6])
{
    const size_t N = (size_t)g.N;
    const size_t sizes[6] = {5 * N * es, 5 * N * es, 3 * N * es, 3 * N * es, sizeof(Ctl),
                             2 * mhd::reduce_capacity(g) * sizeof(unsigned long long)};
    size_t off = 0;
    for (int k = 0; k < 6; k++) {
        offs[k] = off;
        off += (sizes[k] + 255) / 256 * 256;
    }
    return off;
}

size_t mhd_workspace_bytes(int nx, int ny, int nz, int dtype)
{
    if (nx < 1 || ny < 1 || nz < 1 || (dtype != MHD_F32 && dtype != MHD_F64)) return 0;
    if ((long long)nx * ny * nz > (1LL << 36)) return 0;   // larger than mhd_create accepts
    mhd::Grid g;
    g.n[0] = nx;
    g.n[1] = ny;
    g.n[2] = nz;
    g.bc = 0;
    g.N = (long long)nx * ny * nz;
    size_t offs[6];
    return workspace_layout(g, dtype == MHD_F64 ? 8 : 4, offs);
}

size_t mhd_state_bytes(int nx, int ny, int nz, int dtype) { return mhd_workspace_bytes(nx, ny, nz, dtype); }

int mhd_create(int nx, int ny, int nz, double gamma, int bc, int dtype, mhd_t** out)
{
    g_err.clear();
    if (!out) return fail(MHD_ERR_ARG, "null output pointer");
    *out = nullptr;
    if (nx < 1 || ny < 1 || nz < 1) return fail(MHD_ERR_ARG, "grid sizes must be >= 1");
    // wavefront and workgroup indices of the sweeps are 32-bit: with at most
    // 2^36 cells (far beyond device memory) every launch stays below 2^32
    if ((long long)nx * ny * nz > (1LL << 36)) return fail(MHD_ERR_ARG, "grid too large (more than 2^36 cells)");
    if (!(gamma > 1.0) || !std::isfinite(gamma)) return fail(MHD_ERR_ARG, "gamma must be a finite number > 1");
    if (bc != MHD_BC_PERIODIC && bc != MHD_BC_OUTFLOW) return fail(MHD_ERR_ARG, "unknown boundary condition");
    if (dtype != MHD_F32 && dtype != MHD_F64) return fail(MHD_ERR_ARG, "unknown dtype");
    mhd_solver* h = new (std::nothrow) mhd_solver();
    if (!h) return fail(MHD_ERR_OOM, "host allocation failed");
    h->g.n[0] = nx;
    h->g.n[1] = ny;
    h->g.n[2] = nz;
    h->g.bc = bc;
    h->g.N = (long long)nx * ny * nz;
    h->gamma = gamma;
    h->dtype = dtype;
    h->esize = dtype == MHD_F64 ? 8 : 4;
    h->stream = nullptr;
    h->s = 0;
    h->cmax_valid = false;
    h->bound = false;
    h->graphs = true;
    h->fusion = 1;
    for (int q = 0; q < 3; q++) {
        h->exec[q] = nullptr;
        h->exec_cfl[q] = 0.0;
    }
    h->timing = false;
    for (int k = 0; k < MHD_K_COUNT; k++) {
        h->total_ms[k] = 0.0;
        h->launches[k] = 0;
    }
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "hipGetDevice");
    }
    const size_t N = (size_t)h->g.N;
    h->cap = mhd::reduce_capacity(h->g);
    void* mem[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    const size_t sizes[6] = {5 * N * h->esize, 5 * N * h->esize, 3 * N * h->esize, 3 * N * h->esize, sizeof(Ctl),
                             2 * h->cap * sizeof(unsigned long long)};
    for (int k = 0; k < 6; k++) {
        e = hipMalloc(&mem[k], sizes[k]);
        if (e != hipSuccess) {
            for (int q = 0; q < k; q++) (void)hipFree(mem[q]);
            delete h;
            (void)hipGetLastError();
            return e == hipErrorOutOfMemory ? fail(MHD_ERR_OOM, "device allocation failed")
                                            : hip_fail(e, "hipMalloc");
        }
    }
    h->u[0] = mem[0];
    h->u[1] = mem[1];
    h->b[0] = mem[2];
    h->b[1] = mem[3];
    h->ctl = static_cast<Ctl*>(mem[4]);
    h->parts = static_cast<unsigned long long*>(mem[5]);
    h->ucur = h->bcur = 0;
    Ctl c0;
    std::memset(&c0, 0, sizeof(c0));
    c0.t_stop = -1.0;
    e = hipMemcpy(h->ctl, &c0, sizeof(Ctl), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        for (int q = 0; q < 6; q++) (void)hipFree(mem[q]);
        delete h;
        return hip_fail(e, "init control block");
    }
    *out = h;
    return MHD_OK;
}

int mhd_destroy(mhd_t* h)
{
    if (!h) return MHD_OK;
    (void)set_current(h);
    (void)hipStreamSynchronize(h->stream);
    drop_graphs(h);
    if (!h->bound) {
        (void)hipFree(h->u[0]);
        (void)hipFree(h->u[1]);
        (void)hipFree(h->b[0]);
        (void)hipFree(h->b[1]);
        (void)hipFree(h->ctl);
        (void)hipFree(h->parts);
    }
    for (int k = 0; k < MHD_K_COUNT; k++)
        for (auto& pr : h->pending[k]) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    for (hipEvent_t e : h->pool) (void)hipEventDestroy(e);
    delete h;
    return MHD_OK;
}

int mhd_bind_workspace(mhd_t* h, void* dev, size_t bytes)
{
    if (int rc = check(h)) return rc;
    if (!dev) return fail(MHD_ERR_ARG, "null workspace");
    if (reinterpret_cast<uintptr_t>(dev) % 256 != 0) return fail(MHD_ERR_ARG, "workspace must be 256-byte aligned");
    size_t offs[6];
    const size_t need = workspace_layout(h->g, h->esize, offs);
    if (bytes < need) return fail(MHD_ERR_ARG, "workspace smaller than mhd_workspace_bytes");
    if (int rc = set_current(h)) return rc;
    HIPCHK(hipStreamSynchronize(h->stream), "stream sync");
    char* base = static_cast<char*>(dev);
    Ctl c0;
    std::memset(&c0, 0, sizeof(c0));
    c0.t_stop = -1.0;
    HIPCHK(hipMemcpy(base + offs[4], &c0, sizeof(Ctl), hipMemcpyHostToDevice), "init control block");
    if (!h->bound) {
        (void)hipFree(h->u[0]);
        (void)hipFree(h->u[1]);
        (void)hipFree(h->b[0]);
        (void)hipFree(h->b[1]);
        (void)hipFree(h->ctl);
        (void)hipFree(h->parts);
    }
    drop_graphs(h);   // they address the old buffers
    h->u[0] = base + offs[0];
    h->u[1] = base + offs[1];
    h->b[0] = base + offs[2];
    h->b[1] = base + offs[3];
    h->ctl = reinterpret_cast<Ctl*>(base + offs[4]);
    h->parts = reinterpret_cast<unsigned long long*>(base + offs[5]);
    h->ucur = h->bcur = 0;
    h->s = 0;
    h->cmax_valid = false;
    h->bound = true;
    return MHD_OK;
}

int mhd_set_graphs(mhd_t* h, int enable)
{
    if (int rc = check(h)) return rc;
    if (int rc = set_current(h)) return rc;
    HIPCHK(hipStreamSynchronize(h->stream), "stream sync");
    if (!enable) drop_graphs(h);
    h->graphs = enable != 0;
    return MHD_OK;
}

int mhd_set_fusion(mhd_t* h, int mode)
{
    if (int rc = check(h)) return rc;
    if (mode < 0 || mode > 2) return fail(MHD_ERR_ARG, "fusion mode must be 0, 1 or 2");
    if (int rc = set_current(h)) return rc;
    HIPCHK(hipStreamSynchronize(h->stream), "stream sync");
    drop_graphs(h);   // captured with the other launch sequence
    h->fusion = mode;
    return MHD_OK;
}

int mhd_set_stream(mhd_t* h, void* stream)
{
    if (int rc = check(h)) return rc;
    if (int rc = set_current(h)) return rc;
    // work already issued on the old stream finishes before any on the new one
    HIPCHK(hipStreamSynchronize(h->stream), "stream sync");
    h->stream = static_cast<hipStream_t>(stream);
    return MHD_OK;
}

static int reset_time(mhd_t* h)
{
    Ctl c;
    if (int rc = read_ctl(h, &c)) return rc;
    c.t = 0.0;
    c.dt = 0.0;
    c.status = 0;
    HIPCHK(hipMemcpyAsync(h->ctl, &c, sizeof(Ctl), hipMemcpyHostToDevice, h->stream), "write control block");
    HIPCHK(hipStreamSynchronize(h->stream), "stream sync");
    h->s = 0;
    return MHD_OK;
}

static int copy_in(mhd_t* h, const void* src, hipMemcpyKind kind)
{
    const size_t N = (size_t)h->g.N, es = h->esize;
    const char* p = static_cast<const char*>(src);
    h->ucur = h->bcur = 0;
    h->cmax_valid = false;
    HIPCHK(hipMemcpyAsync(h->u[0], p, 5 * N * es, kind, h->stream), "state copy in");
    HIPCHK(hipMemcpyAsync(h->b[0], p + 5 * N * es, 3 * N * es, kind, h->stream), "state copy in");
    return MHD_OK;
}

static int copy_out(mhd_t* h, void* dst, hipMemcpyKind kind)
{
    const size_t N = (size_t)h->g.N, es = h->esize;
    char* p = static_cast<char*>(dst);
    HIPCHK(hipMemcpyAsync(p, h->u[h->ucur], 5 * N * es, kind, h->stream), "state copy out");
    HIPCHK(hipMemcpyAsync(p + 5 * N * es, h->b[h->bcur], 3 * N * es, kind, h->stream), "state copy out");
    return MHD_OK;
}

// Check the state just copied in (after reset_time cleared the status): a
// non-finite value or a non-positive density is rejected.
static int validate(mhd_t* h)
{
    const long long N = h->g.N;
    hipError_t e = h->dtype == MHD_F64
                       ? mhd::launch_validate<double>(static_cast<const double*>(h->u[0]),
                                                      static_cast<const double*>(h->b[0]), N, h->ctl, h->stream)
                       : mhd::launch_validate<float>(static_cast<const float*>(h->u[0]),
                                                     static_cast<const float*>(h->b[0]), N, h->ctl, h->stream);
    if (e != hipSuccess) return hip_fail(e, "state check launch");
    int status = 0;
    HIPCHK(hipMemcpyAsync(&status, &h->ctl->status, sizeof(int), hipMemcpyDeviceToHost, h->stream), "read status");
    HIPCHK(hipStreamSynchronize(h->stream), "stream sync");
    if (status != 0) return fail(MHD_ERR_ARG, "state has a non-finite value or a non-positive density");
    return MHD_OK;
}

int mhd_set_state(mhd_t* h, const void* host_state)
{
    if (int rc = check(h)) return rc;
    if (!host_state) return fail(MHD_ERR_ARG, "null state pointer");
    if (int rc = set_current(h)) return rc;
    if (int rc = copy_in(h, host_state, hipMemcpyHostToDevice)) return rc;
    if (int rc = reset_time(h)) return rc;
    return validate(h);
}

int mhd_set_state_device(mhd_t* h, const void* dev_state)
{
    if (int rc = check(h)) return rc;
    if (!dev_state) return fail(MHD_ERR_ARG, "null state pointer");
    if (int rc = set_current(h)) return rc;
    if (int rc = copy_in(h, dev_state, hipMemcpyDeviceToDevice)) return rc;
    if (int rc = reset_time(h)) return rc;
    return validate(h);
}

int mhd_get_state(mhd_t* h, void* host_state)
{
    if (int rc = check(h)) return rc;
    if (!host_state) return fail(MHD_ERR_ARG, "null state pointer");
    if (int rc = set_current(h)) return rc;
    if (int rc = copy_out(h, host_state, hipMemcpyDeviceToHost)) return rc;
    HIPCHK(hipStreamSynchronize(h->stream), "stream sync");
    return MHD_OK;
}

int mhd_get_state_device(mhd_t* h, void* dev_state)
{
    if (int rc = check(h)) return rc;
    if (!dev_state) return fail(MHD_ERR_ARG, "null state pointer");
    if (int rc = set_current(h)) return rc;
    return copy_out(h, dev_state, hipMemcpyDeviceToDevice);
}

int mhd_step(mhd_t* h, int n, double cfl)
{
    if (int rc = check(h)) return rc;
    if (n < 0) return fail(MHD_ERR_ARG, "negative step count");
    if (!(cfl > 0.0 && cfl <= 1.0)) return fail(MHD_ERR_ARG, "cfl must be in (0, 1]");
    if (int rc = set_current(h)) return rc;
    int rc = h->dtype == MHD_F64 ? full_steps<double>(h, n, cfl) : full_steps<float>(h, n, cfl);
    if (rc) return rc;
    int status = 0;
    HIPCHK(hipMemcpyAsync(&status, &h->ctl->status, sizeof(int), hipMemcpyDeviceToHost, h->stream), "read status");
    HIPCHK(hipStreamSynchronize(h->stream), "stream sync");
    if (status == -1) return fail(MHD_ERR_ARG, "the state set last was rejected; set a valid state");
    if (status != 0) return fail(MHD_ERR_NONFINITE, "non-finite or non-positive c_max; state frozen");
    return MHD_OK;
}

int mhd_divb_max(mhd_t* h, double* out)
{
    if (int rc = check(h)) return rc;
    if (!out) return fail(MHD_ERR_ARG, "null output pointer");
    if (int rc = set_current(h)) return rc;
    unsigned long long* parts = h->parts + h->cap;
    int np = 0;
    hipError_t e = h->dtype == MHD_F64
                       ? mhd::launch_divb<double>(static_cast<const double*>(h->b[h->bcur]), h->g, parts, &np,
                                                  h->stream)
                       : mhd::launch_divb<float>(static_cast<const float*>(h->b[h->bcur]), h->g, parts, &np,
                                                 h->stream);
    if (e != hipSuccess) return hip_fail(e, "div B launch");
    HIPCHK(mhd::launch_finish(parts, np, 1, 0.0, h->ctl, h->stream), "div B finish launch");
    Ctl c;
    if (int rc = read_ctl(h, &c)) return rc;
    *out = c.divb;
    return MHD_OK;
}

int mhd_divb_max_noalloc(const void* dev_state, int nx, int ny, int nz, int bc, int dtype, double* dev_out,
                         void* stream)
{
    g_err.clear();
    if (!dev_state || !dev_out) return fail(MHD_ERR_ARG, "null state or output pointer");
    if (nx < 1 || ny < 1 || nz < 1) return fail(MHD_ERR_ARG, "grid sizes must be >= 1");
    if ((long long)nx * ny * nz > (1LL << 36)) return fail(MHD_ERR_ARG, "grid too large (more than 2^36 cells)");
    if (bc != MHD_BC_PERIODIC && bc != MHD_BC_OUTFLOW) return fail(MHD_ERR_ARG, "unknown boundary condition");
    if (dtype != MHD_F32 && dtype != MHD_F64) return fail(MHD_ERR_ARG, "unknown dtype");
    Grid g;
    g.n[0] = nx;
    g.n[1] = ny;
    g.n[2] = nz;
    g.bc = bc;
    g.N = (long long)nx * ny * nz;
    if (mhd::reduce_slots(g) > kNoAllocSlots) return fail(MHD_ERR_ARG, "reduction needs more slots than the scratch");
    int dev = -1;
    HIPCHK(hipGetDevice(&dev), "hipGetDevice");
    void* base = nullptr;
    if (int rc = scratch_ptr(dev, &base)) return rc;
    unsigned long long* parts = static_cast<unsigned long long*>(base);
    Ctl* ctl = reinterpret_cast<Ctl*>(static_cast<char*>(base) + kNoAllocSlots * sizeof(unsigned long long));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t es = dtype == MHD_F64 ? 8 : 4;
    const void* bfield = static_cast<const char*>(dev_state) + 5 * (size_t)g.N * es;
    int np = 0;
    hipError_t e = dtype == MHD_F64 ? mhd::launch_divb<double>(static_cast<const double*>(bfield), g, parts, &np, s)
                                    : mhd::launch_divb<float>(static_cast<const float*>(bfield), g, parts, &np, s);
    if (e != hipSuccess) return hip_fail(e, "div B launch");
    HIPCHK(mhd::launch_finish(parts, np, 1, 0.0, ctl, s), "div B finish launch");
    HIPCHK(hipMemcpyAsync(dev_out, &ctl->divb, sizeof(double), hipMemcpyDeviceToDevice, s), "div B result copy");
    return MHD_OK;
}

int mhd_cmax(mhd_t* h, double* out)
{
    if (int rc = check(h)) return rc;
    if (!out) return fail(MHD_ERR_ARG, "null output pointer");
    if (int rc = set_current(h)) return rc;
    int rc = h->dtype == MHD_F64 ? cfl_parts<double>(h) : cfl_parts<float>(h);
    if (rc) return rc;
    HIPCHK(mhd::launch_finish(h->parts, 0, 0, 0.0, h->ctl, h->stream), "cmax finish launch");
    h->cmax_valid = true;
    Ctl c;
    if (int rc2 = read_ctl(h, &c)) return rc2;
    *out = c.cmax;
    return MHD_OK;
}

int mhd_get_time(mhd_t* h, double* t, int64_t* s)
{
    if (int rc = check(h)) return rc;
    if (int rc = set_current(h)) return rc;
    Ctl c;
    if (int rc = read_ctl(h, &c)) return rc;
    if (t) *t = c.t;
    if (s) *s = h->s;
    return MHD_OK;
}

int mhd_set_time(mhd_t* h, double t, int64_t s)
{
    if (int rc = check(h)) return rc;
    if (!std::isfinite(t) || s < 0) return fail(MHD_ERR_ARG, "time must be finite and s >= 0");
    if (int rc = set_current(h)) return rc;
    HIPCHK(hipMemcpyAsync(&h->ctl->t, &t, sizeof(double), hipMemcpyHostToDevice, h->stream), "write time");
    HIPCHK(hipStreamSynchronize(h->stream), "stream sync");
    h->s = s;
    return MHD_OK;
}

int mhd_set_stop_time(mhd_t* h, double t_stop)
{
    if (int rc = check(h)) return rc;
    if (std::isnan(t_stop)) return fail(MHD_ERR_ARG, "stop time is NaN");
    if (int rc = set_current(h)) return rc;
    const double v = t_stop < 0.0 ? -1.0 : t_stop;
    HIPCHK(hipMemcpyAsync(&h->ctl->t_stop, &v, sizeof(double), hipMemcpyHostToDevice, h->stream), "write stop time");
    HIPCHK(hipStreamSynchronize(h->stream), "stream sync");
    return MHD_OK;
}

int mhd_fluid_sweep(mhd_t* h, int axis, double dt)
{
    if (int rc = check(h)) return rc;
    if (axis < 0 || axis > 2) return fail(MHD_ERR_ARG, "axis must be 0, 1 or 2");
    if (!(dt >= 0.0) || !std::isfinite(dt)) return fail(MHD_ERR_ARG, "dt must be finite and >= 0");
    if (int rc = set_current(h)) return rc;
    h->cmax_valid = false;
    return h->dtype == MHD_F64 ? fluid<double>(h, axis, dt) : fluid<float>(h, axis, dt);
}

int mhd_ct_sweep(mhd_t* h, int axis, double dt)
{
    if (int rc = check(h)) return rc;
    if (axis < 0 || axis > 2) return fail(MHD_ERR_ARG, "axis must be 0, 1 or 2");
    if (!(dt >= 0.0) || !std::isfinite(dt)) return fail(MHD_ERR_ARG, "dt must be finite and >= 0");
    if (int rc = set_current(h)) return rc;
    h->cmax_valid = false;
    return h->dtype == MHD_F64 ? ct<double>(h, axis, dt) : ct<float>(h, axis, dt);
}

int mhd_step_dt(mhd_t* h, double dt, int64_t s_order)
{
    if (int rc = check(h)) return rc;
    if (!(dt >= 0.0) || !std::isfinite(dt)) return fail(MHD_ERR_ARG, "dt must be finite and >= 0");
    if (s_order < 0) return fail(MHD_ERR_ARG, "sweep-order index must be >= 0");
    if (int rc = set_current(h)) return rc;
    h->cmax_valid = false;
    return h->dtype == MHD_F64 ? sweeps<double>(h, s_order, dt, false) : sweeps<float>(h, s_order, dt, false);
}

int mhd_diagnostic(mhd_t* h, int kind, int axis, int index, void* dev_out)
{
    if (int rc = check(h)) return rc;
    if (kind < 0 || kind >= MHD_D_COUNT) return fail(MHD_ERR_ARG, "unknown diagnostic");
    if (axis > 2) return fail(MHD_ERR_ARG, "axis must be < 0 (whole grid), 0, 1 or 2");
    if (axis >= 0 && (index < 0 || index >= h->g.n[axis])) return fail(MHD_ERR_ARG, "plane index out of range");
    if (!dev_out) return fail(MHD_ERR_ARG, "null output pointer");
    if (int rc = set_current(h)) return rc;
    const int ax = axis < 0 ? -1 : axis;
    hipError_t e = h->dtype == MHD_F64
                       ? mhd::launch_diag<double>(static_cast<const double*>(h->u[h->ucur]),
                                                  static_cast<const double*>(h->b[h->bcur]), h->g, h->gamma, kind, ax,
                                                  index, static_cast<double*>(dev_out), h->stream)
                       : mhd::launch_diag<float>(static_cast<const float*>(h->u[h->ucur]),
                                                 static_cast<const float*>(h->b[h->bcur]), h->g, h->gamma, kind, ax,
                                                 index, static_cast<float*>(dev_out), h->stream);
    if (e != hipSuccess) return hip_fail(e, "diagnostic launch");
    return MHD_OK;
}

static int collect_timing(mhd_t* h)
{
    HIPCHK(hipStreamSynchronize(h->stream), "stream sync");
    for (int k = 0; k < MHD_K_COUNT; k++) {
        for (auto& pr : h->pending[k]) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, pr.first, pr.second), "hipEventElapsedTime");
            h->total_ms[k] += ms;
            h->launches[k] += 1;
            h->pool.push_back(pr.first);
            h->pool.push_back(pr.second);
        }
        h->pending[k].clear();
    }
    return MHD_OK;
}

int mhd_timing(mhd_t* h, int enable)
{
    if (int rc = check(h)) return rc;
    if (int rc = set_current(h)) return rc;
    if (int rc = collect_timing(h)) return rc;
    if (enable) {
        for (int k = 0; k < MHD_K_COUNT; k++) {
            h->total_ms[k] = 0.0;
            h->launches[k] = 0;
        }
    }
    h->timing = enable != 0;
    return MHD_OK;
}

int mhd_timing_read(mhd_t* h, int kind, double* total_ms, int64_t* launches)
{
    if (int rc = check(h)) return rc;
    if (kind < 0 || kind >= MHD_K_COUNT) return fail(MHD_ERR_ARG, "unknown kernel kind");
    if (int rc = set_current(h)) return rc;
    if (int rc = collect_timing(h)) return rc;
    if (total_ms) *total_ms = h->total_ms[kind];
    if (launches) *launches = h->launches[kind];
    return MHD_OK;
}

}  // extern "C"

// Batched solve of many independent 1D Euler problems.
//
// Each instance is advanced with exactly the arithmetic of the single-solve
// path (the same stage kernel body, CFL rule and stopping rule), so it gives
// the same bits batched as alone.  The batch advances in ticks: one tick is
// `steps` SSP-RK3 steps, i.e. 3 x steps stage launches, each covering the
// strips of every instance still running (one ReqGrid row, control block,
// dt and step parity per instance); the launches of a tick are captured in a
// HIP graph and replayed while the set of running instances is unchanged.
// Between ticks the host reads the control blocks back, drops the instances
// that reached t_final or failed, and compacts the table.  Kernel boundaries
// order the stages: no wave ever waits for another.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "wcnst.h"
#include "wcnst_device.hpp"
#include "wcnst_host.hpp"

using namespace wcnst;

namespace {

constexpr int NV = 3;

}  // namespace

struct wcnst_batch {
    int n = 0;
    wcnst_desc d0{};
    std::vector<wcnst_desc> descs;
    std::vector<long long> offs;  // n + 1
    long long total = 0;          // doubles per packed buffer
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;  // private stream for graph capture
    bool general = false;       // some instance has reflecting / fixed sides
    // device (caller's workspace)
    ReqGrid* d_req = nullptr;
    int* d_map = nullptr;  // table row of every block of a stage launch
    uint8_t* d_ctrl = nullptr;
    size_t ctrl_bytes = 0;
    double* U1 = nullptr;
    double* U2 = nullptr;
    // pinned host staging: two tables and two control-block snapshots, used
    // in turn (the host prepares a tick while the previous one runs)
    ReqGrid* h_req = nullptr;
    ReqGrid* h_req2 = nullptr;
    uint8_t* h_ctrl = nullptr;
    uint8_t* h_ctrl2 = nullptr;
    hipEvent_t ev_snap[2] = {nullptr, nullptr};
    int steps_per_tick = 64;  // even, so that a replayed tick keeps the parity pattern
    // persistent finish: once the running instances hold at most
    // persist_strips strips, one persistent launch (persist_waves waves per
    // workgroup, persist_group instances each) runs them to their final
    // times; 0 keeps stage launches to the end
    int persist_strips = 0, persist_waves = 8, persist_group = 1;
    int persist_instances = 0;  // instances the last solve finished in the persistent launch
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double kernel_ms = 0.0;
    int ticks = 0, graphs = 0;
    // per-instance outcome of the last solve
    std::vector<unsigned long long> bad_key;
    // The tick graph in use and the tick that last launched it.  A graph
    // replaced while ticks are pipelined may still be running: it waits in
    // `retired` until the host has waited on the snapshot event of a tick at
    // or after its last launch (same stream, so that launch has completed).
    hipGraphExec_t exec = nullptr;
    long long exec_tick = -1;
    struct Retired {
        hipGraphExec_t exec;
        long long last_tick;
    };
    std::vector<Retired> retired;
};

// Destroys the retired tick graphs whose last launch was in tick <= done
// (done: a tick whose snapshot event the host has waited on; -1 after a
// stream synchronisation destroys all).
static void reap_retired(wcnst_batch* b, long long done)
{
    size_t keep = 0;
    for (size_t i = 0; i < b->retired.size(); ++i) {
        if (done < 0 || b->retired[i].last_tick <= done) (void)hipGraphExecDestroy(b->retired[i].exec);
        else b->retired[keep++] = b->retired[i];
    }
    b->retired.resize(keep);
}

static size_t batch_layout(int n, long long total, long long strips, size_t* o_req, size_t* o_map, size_t* o_ctrl,
                           size_t* o_u1, size_t* o_u2)
{
    size_t o = 0;
    *o_req = o;
    o = wcnst_align256(o + sizeof(ReqGrid) * (size_t)n);
    *o_map = o;
    o = wcnst_align256(o + sizeof(int) * (size_t)strips);
    *o_ctrl = o;
    o = wcnst_align256(o + wcnst_align256(wcnst_ctrl_bytes()) * (size_t)n);
    *o_u1 = o;
    o = wcnst_align256(o + sizeof(double) * (size_t)total);
    *o_u2 = o;
    o = wcnst_align256(o + sizeof(double) * (size_t)total);
    return o;
}

// All descriptors 1D Euler with the scheme parameters of the first.
wcnst_status wcnst_check_same_scheme(const wcnst_desc& a, const wcnst_desc& d)
{
    if (d.flux != a.flux || d.scheme != a.scheme || d.charwise != a.charwise || d.q != a.q || d.gamma != a.gamma ||
        d.CT != a.CT || d.C != a.C || d.eps_teno != a.eps_teno || d.eps_js != a.eps_js || d.diff != a.diff ||
        d.z_q != a.z_q || d.eps_z != a.eps_z)
        return WCNST_E_INVALID_ARG;
    return WCNST_OK;
}

static wcnst_status batch_check(const wcnst_desc* descs, int32_t n, long long* total, std::vector<long long>* offs,
                                long long* strips)
{
    if (!descs || n < 1) return wcnst_fail(WCNST_E_INVALID_ARG, "need at least one descriptor");
    const wcnst_desc& a = descs[0];
    long long off = 0, nstr = 0;
    if (offs) offs->assign((size_t)n + 1, 0);
    for (int i = 0; i < n; ++i) {
        const wcnst_desc& d = descs[i];
        wcnst_status st = wcnst_check_desc(&d);
        if (st) return wcnst_fail(st, "descriptor %d: %s", i, wcnst_last_error());
        if (d.ndim != 1 || d.system != WCNST_EULER)
            return wcnst_fail(WCNST_E_INVALID_ARG, "descriptor %d: batches hold 1D Euler problems", i);
        if (d.diff != WCNST_MND)
            return wcnst_fail(WCNST_E_INVALID_ARG, "descriptor %d: batches use the MND difference", i);
        if (wcnst_check_same_scheme(a, d))
            return wcnst_fail(WCNST_E_INVALID_ARG, "descriptor %d: scheme parameters differ from descriptor 0", i);
        if (offs) (*offs)[i] = off;
        off += ((long long)NV * d.nx + 63) / 64 * 64;  // 512-byte aligned instances
        nstr += (d.nx + TX - 1) / TX;
    }
    if (offs) (*offs)[n] = off;
    if (total) *total = off;
    if (strips) *strips = nstr;
    return WCNST_OK;
}

extern "C" wcnst_status wcnst_batch_workspace_size(const wcnst_desc* descs, int32_t n, size_t* bytes)
{
    long long total = 0, strips = 0;
    wcnst_status st = batch_check(descs, n, &total, nullptr, &strips);
    if (st) return st;
    if (!bytes) return wcnst_fail(WCNST_E_INVALID_ARG, "null size pointer");
    size_t a, m, b, c, d;
    *bytes = batch_layout(n, total, strips, &a, &m, &b, &c, &d);
    return WCNST_OK;
}

extern "C" wcnst_status wcnst_batch_destroy(wcnst_batch* b);

extern "C" wcnst_status wcnst_batch_create(const wcnst_desc* descs, int32_t n, void* hip_stream, void* workspace,
                                           size_t ws_bytes, wcnst_batch** out)
{
    long long total = 0, strips = 0;
    std::vector<long long> offs;
    wcnst_status st = batch_check(descs, n, &total, &offs, &strips);
    if (st) return st;
    if (!out) return wcnst_fail(WCNST_E_INVALID_ARG, "null output handle");
    size_t o_req, o_map, o_ctrl, o_u1, o_u2;
    const size_t need = batch_layout(n, total, strips, &o_req, &o_map, &o_ctrl, &o_u1, &o_u2);
    if (!workspace || ws_bytes < need)
        return wcnst_fail(WCNST_E_INVALID_ARG, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
    if (((uintptr_t)workspace & 255u) != 0) return wcnst_fail(WCNST_E_INVALID_ARG, "workspace not 256-byte aligned");

    wcnst_batch* b = new wcnst_batch();
    b->n = n;
    b->d0 = descs[0];
    b->descs.assign(descs, descs + n);
    b->offs = offs;
    b->total = total;
    b->stream = (hipStream_t)hip_stream;
    uint8_t* ws = (uint8_t*)workspace;
    b->d_req = (ReqGrid*)(ws + o_req);
    b->d_map = (int*)(ws + o_map);
    b->d_ctrl = ws + o_ctrl;
    b->ctrl_bytes = wcnst_align256(wcnst_ctrl_bytes());
    b->U1 = (double*)(ws + o_u1);
    b->U2 = (double*)(ws + o_u2);
    b->bad_key.assign((size_t)n, ~0ull);

    hipError_t e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&b->ev0);
    if (e == hipSuccess) e = hipEventCreate(&b->ev1);
    if (e == hipSuccess) e = hipHostMalloc((void**)&b->h_req, sizeof(ReqGrid) * (size_t)n, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&b->h_req2, sizeof(ReqGrid) * (size_t)n, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&b->h_ctrl, b->ctrl_bytes * (size_t)n, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&b->h_ctrl2, b->ctrl_bytes * (size_t)n, hipHostMallocDefault);
    for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&b->ev_snap[k], hipEventDisableTiming);
    if (e != hipSuccess) {
        wcnst_batch_destroy(b);
        return wcnst_fail(WCNST_E_HIP, "batch setup failed: %s", hipGetErrorString(e));
    }
    *out = b;
    return WCNST_OK;
}

extern "C" wcnst_status wcnst_batch_offsets(const wcnst_batch* b, int64_t* offsets)
{
    if (!b || !offsets) return wcnst_fail(WCNST_E_INVALID_ARG, "null argument");
    for (int i = 0; i <= b->n; ++i) offsets[i] = b->offs[(size_t)i];
    return WCNST_OK;
}

extern "C" wcnst_status wcnst_batch_set_tuning(wcnst_batch* b, int32_t steps_per_tick)
{
    if (!b) return wcnst_fail(WCNST_E_INVALID_ARG, "null handle");
    if (steps_per_tick < 2 || steps_per_tick > 4096 || (steps_per_tick & 1))
        return wcnst_fail(WCNST_E_INVALID_ARG, "steps_per_tick must be even and in [2, 4096]");
    b->steps_per_tick = steps_per_tick;
    return WCNST_OK;
}

extern "C" wcnst_status wcnst_batch_set_persist(wcnst_batch* b, int32_t switch_strips, int32_t waves_per_group,
                                                int32_t instances_per_group)
{
    if (!b) return wcnst_fail(WCNST_E_INVALID_ARG, "null handle");
    if (switch_strips < 0) return wcnst_fail(WCNST_E_INVALID_ARG, "switch_strips must be >= 0");
    if (waves_per_group < 1 || waves_per_group > 8)
        return wcnst_fail(WCNST_E_INVALID_ARG, "waves_per_group must be in [1, 8]");
    if (instances_per_group < 1 || instances_per_group > 8)
        return wcnst_fail(WCNST_E_INVALID_ARG, "instances_per_group must be in [1, 8]");
    b->persist_strips = switch_strips;
    b->persist_waves = waves_per_group;
    b->persist_group = instances_per_group;
    return WCNST_OK;
}

extern "C" wcnst_status wcnst_batch_kernel_ms(const wcnst_batch* b, double* ms)
{
    if (!b || !ms) return wcnst_fail(WCNST_E_INVALID_ARG, "null argument");
    *ms = b->kernel_ms;
    return WCNST_OK;
}

extern "C" wcnst_status wcnst_batch_stats(const wcnst_batch* b, int32_t* ticks, int32_t* graphs,
                                          int32_t* persist_instances)
{
    if (!b) return wcnst_fail(WCNST_E_INVALID_ARG, "null handle");
    if (ticks) *ticks = b->ticks;
    if (graphs) *graphs = b->graphs;
    if (persist_instances) *persist_instances = b->persist_instances;
    return WCNST_OK;
}

static bool reached(double t_final, double t) { return t_final - t <= 1e-12 * t_final; }

static const StepRec& newest(const Ctrl& c) { return c.rec[0].step >= c.rec[1].step ? c.rec[0] : c.rec[1]; }

// Tick `tick` of `steps` steps over the table rows [0, nreq): replay the
// captured graph when it was made for this table, else capture a new one
// (a tick of fewer steps than steps_per_tick is launched directly).  A
// replaced graph is retired, not destroyed: the previous tick, which may
// have launched it, can still be running.
static wcnst_status run_tick(wcnst_batch* b, int nreq, int blocks, int steps, bool table_changed, long long tick)
{
    if (steps != b->steps_per_tick) {
        for (int s = 0; s < steps; ++s)
            for (int stage = 0; stage < 3; ++stage)
                WCNST_HIP_TRY(wcnst_launch_multi(&b->d0, 1, b->d_req, b->d_map, nreq, blocks, stage, s & 1, 0, b->general,
                                                 b->stream));
        return WCNST_OK;
    }
    if (!b->exec || table_changed) {
        if (b->exec) {
            b->retired.push_back({b->exec, b->exec_tick});
            b->exec = nullptr;
        }
        hipGraph_t g = nullptr;
        WCNST_HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
        hipError_t le = hipSuccess;
        for (int s = 0; s < steps && le == hipSuccess; ++s)
            for (int stage = 0; stage < 3 && le == hipSuccess; ++stage)
                le = wcnst_launch_multi(&b->d0, 1, b->d_req, b->d_map, nreq, blocks, stage, s & 1, 0, b->general,
                                        b->cap);
        hipError_t ce = hipStreamEndCapture(b->cap, &g);
        if (le != hipSuccess || ce != hipSuccess)
            return wcnst_fail(WCNST_E_HIP, "graph capture failed: %s / %s", hipGetErrorString(le),
                              hipGetErrorString(ce));
        hipError_t ie = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) return wcnst_fail(WCNST_E_HIP, "graph instantiate failed: %s", hipGetErrorString(ie));
        b->graphs += 1;
    }
    WCNST_HIP_TRY(hipGraphLaunch(b->exec, b->stream));
    b->exec_tick = tick;
    return WCNST_OK;
}

extern "C" wcnst_status wcnst_batch_solve(wcnst_batch* b, double* U, const double* t_final, double cfl,
                                          int64_t max_steps, int32_t* status, double* t_out, int64_t* steps_out)
{
    if (!b || !U || !t_final || !status) return wcnst_fail(WCNST_E_INVALID_ARG, "null argument");
    if (!(cfl > 0.0)) return wcnst_fail(WCNST_E_INVALID_ARG, "cfl must be > 0");
    if (max_steps < 0) return wcnst_fail(WCNST_E_INVALID_ARG, "max_steps must be >= 0");
    if (((uintptr_t)U & 7u) != 0) return wcnst_fail(WCNST_E_INVALID_ARG, "U not 8-byte aligned");
    const int n = b->n;
    for (int i = 0; i < n; ++i) {
        if (std::isnan(t_final[i])) return wcnst_fail(WCNST_E_INVALID_ARG, "t_final[%d] is NaN", i);
        if (!std::isfinite(t_final[i]) && max_steps >= ((int64_t)1 << 40))
            return wcnst_fail(WCNST_E_INVALID_ARG, "t_final[%d] is infinite and max_steps unbounded", i);
    }
    // rows of every instance; instance i keeps control block i
    std::vector<ReqGrid> rows((size_t)n);
    b->general = false;
    for (int i = 0; i < n; ++i) b->general = b->general || wcnst_general_bc(&b->descs[(size_t)i]);
    for (int i = 0; i < n; ++i) {
        const wcnst_desc& d = b->descs[(size_t)i];
        const long long o = b->offs[(size_t)i];
        ReqGrid& q = rows[(size_t)i];
        q = ReqGrid{};
        q.U = U + o;
        q.U1 = b->U1 + o;
        q.U2 = b->U2 + o;
        q.ctrl = (Ctrl*)(b->d_ctrl + b->ctrl_bytes * (size_t)i);
        wcnst_make_params(&d, &q.P);
        q.t_final = t_final[i];
        q.cfl = cfl;
        q.nstrips = (d.nx + TX - 1) / TX;
        q.parity0 = 0;
    }
    b->ticks = 0;
    b->graphs = 0;
    b->persist_instances = 0;
    // graphs of an earlier solve (one that stopped on an error may have
    // left work queued)
    WCNST_HIP_TRY(hipStreamSynchronize(b->stream));
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    reap_retired(b, -1);
    std::vector<int> active((size_t)n);
    for (int i = 0; i < n; ++i) active[(size_t)i] = i;
    std::vector<int> parity((size_t)n, 0);

    // table of all rows; control blocks reset and initial speeds in one launch
    int blocks = 0;
    for (int i = 0; i < n; ++i) {
        b->h_req[i] = rows[(size_t)i];
        b->h_req[i].blk0 = blocks;
        blocks += rows[(size_t)i].nstrips;
    }
    WCNST_HIP_TRY(hipMemcpyAsync(b->d_req, b->h_req, sizeof(ReqGrid) * (size_t)n, hipMemcpyHostToDevice, b->stream));
    WCNST_HIP_TRY(hipEventRecord(b->ev0, b->stream));
    WCNST_HIP_TRY(wcnst_launch_multi_init(1, b->d_req, n, b->stream));
    WCNST_HIP_TRY(wcnst_launch_block_map(b->d_req, n, blocks, b->d_map, b->stream));

    // Ticks are pipelined: tick k+1 is queued before the host has looked at
    // tick k, so the set of running instances is decided from the control
    // blocks one tick old; an instance that finished in tick k runs in tick
    // k+1 only to leave each launch at its prologue.
    ReqGrid* tabs[2] = {b->h_req, b->h_req2};  // table uploads alternate
    uint8_t* snaps[2] = {b->h_ctrl, b->h_ctrl2};
    int uploads = 1;  // the initial table came from tabs[0]
    long long launched = 0;
    bool changed = true;
    int k = 0;
    while (!active.empty() && launched < (long long)max_steps) {
        const int steps = (int)std::min<long long>(b->steps_per_tick, (long long)max_steps - launched);
        if (changed && b->ticks > 0) {
            // compact the table to the running instances, in the staging
            // buffer not used by the last upload (the one before it has
            // completed: the host waited on a later tick's snapshot)
            ReqGrid* tab = tabs[uploads & 1];
            blocks = 0;
            for (size_t j = 0; j < active.size(); ++j) {
                const int i = active[j];
                tab[j] = rows[(size_t)i];
                tab[j].blk0 = blocks;
                tab[j].parity0 = parity[(size_t)i];
                blocks += rows[(size_t)i].nstrips;
            }
            WCNST_HIP_TRY(hipMemcpyAsync(b->d_req, tab, sizeof(ReqGrid) * active.size(), hipMemcpyHostToDevice,
                                         b->stream));
            WCNST_HIP_TRY(wcnst_launch_block_map(b->d_req, (int)active.size(), blocks, b->d_map, b->stream));
            uploads += 1;
        }
        wcnst_status st = run_tick(b, (int)active.size(), blocks, steps, changed, k);
        if (st) {
            (void)hipStreamSynchronize(b->stream);
            reap_retired(b, -1);
            return st;
        }
        launched += steps;
        b->ticks += 1;
        for (int i : active) parity[(size_t)i] = (parity[(size_t)i] + steps) & 1;
        WCNST_HIP_TRY(hipMemcpyAsync(snaps[k & 1], b->d_ctrl, b->ctrl_bytes * (size_t)n, hipMemcpyDeviceToHost,
                                     b->stream));
        WCNST_HIP_TRY(hipEventRecord(b->ev_snap[k & 1], b->stream));
        changed = false;
        if (k > 0) {
            // the previous tick's snapshot (this tick is running meanwhile)
            WCNST_HIP_TRY(hipEventSynchronize(b->ev_snap[(k - 1) & 1]));
            // every launch up to tick k-1 has completed
            reap_retired(b, k - 1);
            const uint8_t* snap = snaps[(k - 1) & 1];
            std::vector<int> still;
            still.reserve(active.size());
            for (int i : active) {
                const Ctrl& c = *(const Ctrl*)(snap + b->ctrl_bytes * (size_t)i);
                const bool done = c.status != 0 || c.done != 0 ||
                                  (std::isfinite(t_final[i]) && reached(t_final[i], newest(c).t));
                if (!done) still.push_back(i);
            }
            changed = still.size() != active.size();
            active.swap(still);
            long long strips = 0;
            for (int i : active) strips += rows[(size_t)i].nstrips;
            if (b->persist_strips > 0 && !active.empty() && strips <= b->persist_strips &&
                launched < (long long)max_steps) {
                // the rest in one persistent launch, after the ticks queued
                // so far (same stream), from the table of the running ones
                ReqGrid* tab = tabs[uploads & 1];
                for (size_t j = 0; j < active.size(); ++j) {
                    const int i = active[j];
                    tab[j] = rows[(size_t)i];
                    tab[j].blk0 = 0;
                    tab[j].parity0 = parity[(size_t)i];
                }
                WCNST_HIP_TRY(hipMemcpyAsync(b->d_req, tab, sizeof(ReqGrid) * active.size(), hipMemcpyHostToDevice,
                                             b->stream));
                uploads += 1;
                WCNST_HIP_TRY(wcnst_launch_persist(&b->d0, b->d_req, (int)active.size(), b->persist_group,
                                                   b->persist_waves, (long long)max_steps - launched, b->general,
                                                   b->stream));
                b->persist_instances = (int)active.size();
                break;
            }
        }
        k += 1;
    }
    WCNST_HIP_TRY(hipEventRecord(b->ev1, b->stream));
    WCNST_HIP_TRY(hipMemcpyAsync(b->h_ctrl, b->d_ctrl, b->ctrl_bytes * (size_t)n, hipMemcpyDeviceToHost, b->stream));
    WCNST_HIP_TRY(hipStreamSynchronize(b->stream));
    reap_retired(b, -1);
    float ms = 0.0f;
    WCNST_HIP_TRY(hipEventElapsedTime(&ms, b->ev0, b->ev1));
    b->kernel_ms = ms;

    wcnst_status ret = WCNST_OK;
    for (int i = 0; i < n; ++i) {
        const Ctrl& c = *(const Ctrl*)(b->h_ctrl + b->ctrl_bytes * (size_t)i);
        const StepRec& r = newest(c);
        b->bad_key[(size_t)i] = c.bad_key;
        int s = c.status;
        if (s == 0 && std::isfinite(t_final[i]) && !reached(t_final[i], r.t)) s = WCNST_E_MAX_STEPS;
        status[i] = s;
        if (t_out) t_out[i] = r.t;
        if (steps_out) steps_out[i] = r.step;
        if (s != 0 && ret == WCNST_OK) ret = s;
    }
    if (ret != WCNST_OK) return wcnst_fail(ret, "at least one instance did not finish (see the status array)");
    return WCNST_OK;
}

extern "C" wcnst_status wcnst_batch_bad_cells(const wcnst_batch* b, int64_t* bad_stage, int64_t* bad_cell)
{
    if (!b || !bad_stage || !bad_cell) return wcnst_fail(WCNST_E_INVALID_ARG, "null argument");
    for (int i = 0; i < b->n; ++i) {
        const unsigned long long key = b->bad_key[(size_t)i];
        const bool none = key == ~0ull;
        bad_stage[i] = none ? -1 : (int64_t)(key >> 36);
        bad_cell[i] = none ? -1 : (int64_t)(key & ((1ull << 36) - 1));
    }
    return WCNST_OK;
}

extern "C" wcnst_status wcnst_batch_destroy(wcnst_batch* b)
{
    if (!b) return WCNST_OK;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    reap_retired(b, -1);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->ev0) (void)hipEventDestroy(b->ev0);
    if (b->ev1) (void)hipEventDestroy(b->ev1);
    if (b->h_req) (void)hipHostFree(b->h_req);
    if (b->h_req2) (void)hipHostFree(b->h_req2);
    if (b->h_ctrl2) (void)hipHostFree(b->h_ctrl2);
    for (int k = 0; k < 2; ++k)
        if (b->ev_snap[k]) (void)hipEventDestroy(b->ev_snap[k]);
    if (b->h_ctrl) (void)hipHostFree(b->h_ctrl);
    delete b;
    return WCNST_OK;
}

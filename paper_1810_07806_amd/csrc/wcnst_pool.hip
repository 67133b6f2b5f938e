// Request pool: many device-resident Euler solves (1D and 2D, sizes
// differing) advanced together in ticks, so that requests can join and
// leave between ticks (continuous batching).
//
// Each request advances with exactly the arithmetic of wcnst_solve, so its
// result does not depend on what else is in the pool or on when it joined.
// One tick advances every active 1D request by up to `steps_1d` and every
// active 2D request by up to `steps_2d` SSP-RK3 steps, with 3 x steps stage
// launches per dimension, each covering the strips
// (1D, caller's stream) or row segments (2D, the pool's own stream) of all
// active grids of that dimension; a grid has its own table row, control
// block, dt and step parity, and grids that reach t_final stop inside the
// launches.  Kernel boundaries order the stages, so no wave ever waits for
// another.  The tick is synchronous: it ends with both streams drained and
// the per-request outcome (finished, status, t, steps) read back.
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


struct PoolReq {
    bool used = false;
    bool finished = false;
    bool init = false;
    wcnst_desc d{};
    double* U = nullptr;
    double* U1 = nullptr;
    double* U2 = nullptr;
    double t_final = 0.0, cfl = 0.0;
    int parity = 0;  // step parity of the current record
    int status = 0;
    double t = 0.0;
    long long steps = 0;
    unsigned long long bad_key = ~0ull;
};

}  // namespace

struct wcnst_pool {
    wcnst_desc scheme{};
    int cap = 0;
    hipStream_t s1 = nullptr;  // caller's stream: 1D launches, result copies
    hipStream_t s2 = nullptr;  // pool stream: 2D launches
    hipEvent_t ev_start = nullptr, ev_2d = nullptr, ev_1d = nullptr;
    float ms_1d = 0.0f, ms_2d = 0.0f;  // device time of each dimension's launches in the last tick
    // device (caller's workspace): one request table and one block map per
    // dimension, one control block per slot
    ReqGrid* d_req[2] = {nullptr, nullptr};
    int* d_map[2] = {nullptr, nullptr};
    uint8_t* d_ctrl = nullptr;
    size_t ctrl_bytes = 0;
    // pinned host staging
    ReqGrid* h_req[2] = {nullptr, nullptr};
    uint8_t* h_ctrl = nullptr;
    std::vector<PoolReq> reqs;
    int ty = 0;     // rows per 2D segment; 0: chosen per tick (wcnst_auto_rows)
    int slots = 0;  // wavefront slots of the device
};

// Blocks a pool launch can map (one int each, per dimension); a launch over
// more searches the table instead.
constexpr int POOL_MAP_BLOCKS = 1 << 18;

static size_t pool_layout(int cap, size_t* o_req1, size_t* o_req2, size_t* o_ctrl, size_t* o_map)
{
    size_t o = 0;
    *o_req1 = o;
    o = wcnst_align256(o + sizeof(ReqGrid) * (size_t)cap);
    *o_req2 = o;
    o = wcnst_align256(o + sizeof(ReqGrid) * (size_t)cap);
    *o_ctrl = o;
    o = wcnst_align256(o + wcnst_align256(wcnst_ctrl_bytes()) * (size_t)cap);
    *o_map = o;
    o = wcnst_align256(o + 2 * sizeof(int) * (size_t)POOL_MAP_BLOCKS);
    return o;
}

extern "C" wcnst_status wcnst_pool_workspace_size(int32_t capacity, size_t* bytes)
{
    if (capacity < 1 || capacity > (1 << 20)) return wcnst_fail(WCNST_E_INVALID_ARG, "capacity must be in [1, 2^20]");
    if (!bytes) return wcnst_fail(WCNST_E_INVALID_ARG, "null size pointer");
    size_t a, b, c, m;
    *bytes = pool_layout(capacity, &a, &b, &c, &m);
    return WCNST_OK;
}

extern "C" wcnst_status wcnst_pool_destroy(wcnst_pool* p);

extern "C" wcnst_status wcnst_pool_create(const wcnst_desc* scheme, int32_t capacity, void* hip_stream,
                                          void* workspace, size_t ws_bytes, wcnst_pool** out)
{
    wcnst_status st = wcnst_check_desc(scheme);
    if (st) return st;
    if (scheme->system != WCNST_EULER) return wcnst_fail(WCNST_E_INVALID_ARG, "pools hold Euler problems");
    if (scheme->diff != WCNST_MND) return wcnst_fail(WCNST_E_INVALID_ARG, "pools use the MND difference");
    size_t need = 0;
    st = wcnst_pool_workspace_size(capacity, &need);
    if (st) return st;
    if (!out) return wcnst_fail(WCNST_E_INVALID_ARG, "null output handle");
    if (!workspace || ws_bytes < need)
        return wcnst_fail(WCNST_E_INVALID_ARG, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
    if (((uintptr_t)workspace & 255u) != 0) return wcnst_fail(WCNST_E_INVALID_ARG, "workspace not 256-byte aligned");
    size_t o_req1, o_req2, o_ctrl, o_map;
    pool_layout(capacity, &o_req1, &o_req2, &o_ctrl, &o_map);

    wcnst_pool* p = new wcnst_pool();
    p->scheme = *scheme;
    p->cap = capacity;
    p->s1 = (hipStream_t)hip_stream;
    uint8_t* ws = (uint8_t*)workspace;
    p->d_req[0] = (ReqGrid*)(ws + o_req1);
    p->d_req[1] = (ReqGrid*)(ws + o_req2);
    p->d_ctrl = ws + o_ctrl;
    p->d_map[0] = (int*)(ws + o_map);
    p->d_map[1] = p->d_map[0] + POOL_MAP_BLOCKS;
    p->ctrl_bytes = wcnst_align256(wcnst_ctrl_bytes());
    p->reqs.resize((size_t)capacity);
    p->slots = wcnst_wave_slots();

    hipError_t e = hipStreamCreateWithFlags(&p->s2, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&p->ev_start);
    if (e == hipSuccess) e = hipEventCreate(&p->ev_2d);
    if (e == hipSuccess) e = hipEventCreate(&p->ev_1d);
    for (int k = 0; k < 2 && e == hipSuccess; ++k)
        e = hipHostMalloc((void**)&p->h_req[k], sizeof(ReqGrid) * (size_t)capacity, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&p->h_ctrl, p->ctrl_bytes * (size_t)capacity, hipHostMallocDefault);
    if (e != hipSuccess) {
        wcnst_pool_destroy(p);
        return wcnst_fail(WCNST_E_HIP, "pool setup failed: %s", hipGetErrorString(e));
    }
    *out = p;
    return WCNST_OK;
}

extern "C" wcnst_status wcnst_pool_set_tuning(wcnst_pool* p, int32_t rows_per_segment)
{
    if (!p) return wcnst_fail(WCNST_E_INVALID_ARG, "null handle");
    if (rows_per_segment < 0) return wcnst_fail(WCNST_E_INVALID_ARG, "rows_per_segment must be >= 0");
    p->ty = rows_per_segment;
    return WCNST_OK;
}

extern "C" wcnst_status wcnst_pool_admit(wcnst_pool* p, const wcnst_desc* d, double* U, double* U1, double* U2,
                                         double t_final, double cfl, int32_t* slot)
{
    if (!p || !d || !U || !U1 || !U2 || !slot) return wcnst_fail(WCNST_E_INVALID_ARG, "null argument");
    wcnst_status st = wcnst_check_desc(d);
    if (st) return st;
    if (d->system != WCNST_EULER) return wcnst_fail(WCNST_E_INVALID_ARG, "pools hold Euler problems");
    if (wcnst_check_same_scheme(p->scheme, *d))
        return wcnst_fail(WCNST_E_INVALID_ARG, "scheme parameters differ from the pool's");
    if (!(t_final > 0.0) || !std::isfinite(t_final))
        return wcnst_fail(WCNST_E_INVALID_ARG, "t_final must be finite and > 0");
    if (!(cfl > 0.0)) return wcnst_fail(WCNST_E_INVALID_ARG, "cfl must be > 0");
    if ((((uintptr_t)U | (uintptr_t)U1 | (uintptr_t)U2) & 7u) != 0)
        return wcnst_fail(WCNST_E_INVALID_ARG, "buffers not 8-byte aligned");
    int free_slot = -1;
    for (int i = 0; i < p->cap; ++i)
        if (!p->reqs[(size_t)i].used) {
            free_slot = i;
            break;
        }
    if (free_slot < 0) return wcnst_fail(WCNST_E_INVALID_ARG, "pool full (%d requests)", p->cap);
    PoolReq& r = p->reqs[(size_t)free_slot];
    r = PoolReq{};
    r.used = true;
    r.d = *d;
    r.U = U;
    r.U1 = U1;
    r.U2 = U2;
    r.t_final = t_final;
    r.cfl = cfl;
    *slot = free_slot;
    return WCNST_OK;
}

static bool reached(double t_final, double t) { return t_final - t <= 1e-12 * t_final; }

// Table rows of the active grids of one dimension and their stage launches.
static wcnst_status issue_dim(wcnst_pool* p, int ndim, const std::vector<int>& act, int64_t steps, hipStream_t st)
{
    if (act.empty()) return WCNST_OK;
    ReqGrid* tab = p->h_req[ndim - 1];
    int ty = p->ty;
    if (ndim == 2 && ty == 0) {
        std::vector<int> strips, rows;
        for (int i : act) {
            strips.push_back((p->reqs[(size_t)i].d.nx + TX - 1) / TX);
            rows.push_back(p->reqs[(size_t)i].d.ny);
        }
        ty = wcnst_auto_rows(strips.data(), rows.data(), (int)act.size(), p->slots);
    }
    if (ty == 0) ty = 35;  // (unused in 1D)
    int blocks = 0;
    int n = 0;
    bool general = false;
    for (int i : act) {
        PoolReq& r = p->reqs[(size_t)i];
        Ctrl* ctrl = (Ctrl*)(p->d_ctrl + p->ctrl_bytes * (size_t)i);
        if (!r.init) {
            WCNST_HIP_TRY(wcnst_launch_init_grid(&r.d, r.U, ctrl, st));
            r.init = true;
            r.parity = 0;
        }
        general = general || wcnst_general_bc(&r.d);
        ReqGrid& q = tab[n++];
        q = ReqGrid{};
        q.U = r.U;
        q.U1 = r.U1;
        q.U2 = r.U2;
        q.ctrl = ctrl;
        wcnst_make_params(&r.d, &q.P);
        q.t_final = r.t_final;
        q.cfl = r.cfl;
        q.nstrips = (r.d.nx + TX - 1) / TX;
        q.blk0 = blocks;
        q.parity0 = r.parity;
        blocks += q.nstrips * (ndim == 2 ? (r.d.ny + ty - 1) / ty : 1);
        r.parity = (int)((r.parity + steps) & 1);
    }
    WCNST_HIP_TRY(hipMemcpyAsync(p->d_req[ndim - 1], tab, sizeof(ReqGrid) * (size_t)n, hipMemcpyHostToDevice, st));
    // each block finds its table row in one load (a search over the table
    // for launches beyond the map)
    const int* map = nullptr;
    if (blocks <= POOL_MAP_BLOCKS) {
        WCNST_HIP_TRY(wcnst_launch_block_map(p->d_req[ndim - 1], n, blocks, p->d_map[ndim - 1], st));
        map = p->d_map[ndim - 1];
    }
    for (int64_t s = 0; s < steps; ++s)
        for (int stage = 0; stage < 3; ++stage)
            WCNST_HIP_TRY(wcnst_launch_multi(&p->scheme, ndim, p->d_req[ndim - 1], map, n, blocks, stage, (int)(s & 1),
                                             ty, general, st));
    return WCNST_OK;
}

extern "C" wcnst_status wcnst_pool_tick_split(wcnst_pool* p, int64_t steps_1d, int64_t steps_2d, int32_t* n_active)
{
    if (!p) return wcnst_fail(WCNST_E_INVALID_ARG, "null handle");
    if (steps_1d < 1 || steps_1d > (1 << 20) || steps_2d < 1 || steps_2d > (1 << 20))
        return wcnst_fail(WCNST_E_INVALID_ARG, "steps must be in [1, 2^20]");
    std::vector<int> a1, a2;
    for (int i = 0; i < p->cap; ++i) {
        const PoolReq& r = p->reqs[(size_t)i];
        if (!r.used || r.finished) continue;
        (r.d.ndim == 1 ? a1 : a2).push_back(i);
    }
    if (n_active) *n_active = (int32_t)(a1.size() + a2.size());
    if (a1.empty() && a2.empty()) return WCNST_OK;

    // 2D on the pool stream, after the caller's work (admission copies)
    WCNST_HIP_TRY(hipEventRecord(p->ev_start, p->s1));
    WCNST_HIP_TRY(hipStreamWaitEvent(p->s2, p->ev_start, 0));
    wcnst_status st = issue_dim(p, 2, a2, steps_2d, p->s2);
    if (st) return st;
    WCNST_HIP_TRY(hipEventRecord(p->ev_2d, p->s2));
    st = issue_dim(p, 1, a1, steps_1d, p->s1);
    if (st) return st;
    WCNST_HIP_TRY(hipEventRecord(p->ev_1d, p->s1));
    // one copy of the control blocks of all slots, after both streams
    WCNST_HIP_TRY(hipStreamWaitEvent(p->s1, p->ev_2d, 0));
    WCNST_HIP_TRY(hipMemcpyAsync(p->h_ctrl, p->d_ctrl, p->ctrl_bytes * (size_t)p->cap, hipMemcpyDeviceToHost, p->s1));
    WCNST_HIP_TRY(hipStreamSynchronize(p->s1));
    p->ms_1d = p->ms_2d = 0.0f;
    if (!a1.empty()) WCNST_HIP_TRY(hipEventElapsedTime(&p->ms_1d, p->ev_start, p->ev_1d));
    if (!a2.empty()) WCNST_HIP_TRY(hipEventElapsedTime(&p->ms_2d, p->ev_start, p->ev_2d));

    for (const std::vector<int>* act : {&a1, &a2})
        for (int i : *act) {
            PoolReq& r = p->reqs[(size_t)i];
            const Ctrl& c = *(const Ctrl*)(p->h_ctrl + p->ctrl_bytes * (size_t)i);
            const StepRec& n = c.rec[0].step >= c.rec[1].step ? c.rec[0] : c.rec[1];
            r.t = n.t;
            r.steps = n.step;
            r.status = c.status;
            r.bad_key = c.bad_key;
            r.finished = r.status != 0 || reached(r.t_final, r.t);
        }
    return WCNST_OK;
}

extern "C" wcnst_status wcnst_pool_tick(wcnst_pool* p, int64_t steps, int32_t* n_active)
{
    return wcnst_pool_tick_split(p, steps, steps, n_active);
}

extern "C" wcnst_status wcnst_pool_tick_ms(const wcnst_pool* p, double* ms_1d, double* ms_2d)
{
    if (!p || !ms_1d || !ms_2d) return wcnst_fail(WCNST_E_INVALID_ARG, "null argument");
    *ms_1d = p->ms_1d;
    *ms_2d = p->ms_2d;
    return WCNST_OK;
}

extern "C" wcnst_status wcnst_pool_result(const wcnst_pool* p, int32_t slot, int32_t* finished, int32_t* status,
                                          double* t, int64_t* steps, int64_t* bad_stage, int64_t* bad_cell)
{
    if (!p || slot < 0 || slot >= p->cap || !p->reqs[(size_t)slot].used)
        return wcnst_fail(WCNST_E_INVALID_ARG, "no request in slot %d", slot);
    const PoolReq& r = p->reqs[(size_t)slot];
    if (finished) *finished = r.finished ? 1 : 0;
    if (status) *status = r.status;
    if (t) *t = r.t;
    if (steps) *steps = r.steps;
    const bool none = r.bad_key == ~0ull;
    if (bad_stage) *bad_stage = none ? -1 : (int64_t)(r.bad_key >> 36);
    if (bad_cell) *bad_cell = none ? -1 : (int64_t)(r.bad_key & ((1ull << 36) - 1));
    return WCNST_OK;
}

extern "C" wcnst_status wcnst_pool_release(wcnst_pool* p, int32_t slot)
{
    if (!p || slot < 0 || slot >= p->cap || !p->reqs[(size_t)slot].used)
        return wcnst_fail(WCNST_E_INVALID_ARG, "no request in slot %d", slot);
    p->reqs[(size_t)slot] = PoolReq{};
    return WCNST_OK;
}

extern "C" wcnst_status wcnst_pool_destroy(wcnst_pool* p)
{
    if (!p) return WCNST_OK;
    if (p->s1) (void)hipStreamSynchronize(p->s1);
    if (p->s2) {
        (void)hipStreamSynchronize(p->s2);
        (void)hipStreamDestroy(p->s2);
    }
    if (p->ev_start) (void)hipEventDestroy(p->ev_start);
    if (p->ev_2d) (void)hipEventDestroy(p->ev_2d);
    if (p->ev_1d) (void)hipEventDestroy(p->ev_1d);
    for (int k = 0; k < 2; ++k)
        if (p->h_req[k]) (void)hipHostFree(p->h_req[k]);
    if (p->h_ctrl) (void)hipHostFree(p->h_ctrl);
    delete p;
    return WCNST_OK;
}

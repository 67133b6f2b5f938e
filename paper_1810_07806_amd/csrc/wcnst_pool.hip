// Request pool: many device-resident Euler solves (1D and 2D, sizes
// differing) advanced together in ticks, so that requests can join and
// leave between ticks (continuous batching).
//
// Each request advances with exactly the arithmetic of wcnst_solve, so its
// result does not depend on what else is in the pool or on when it joined.
// One tick advances every active request by up to `steps` SSP-RK3 steps:
//   * 2D requests: 3 x steps stage launches on the pool's own stream, each
//     covering the segments of all active 2D grids (one Req2D row per grid,
//     each with its own control block, dt and step parity);
//   * 1D requests: one persistent pass of the batched 1D solver on the
//     caller's stream, resumed from each instance's t, step count and CFL
//     speed, with a grid sized to the 1D share of the tick's estimated work
//     so that both kinds run side by side on the device.
// The tick is synchronous: it ends with both streams drained and the
// per-request outcome (finished, status, t, steps) read back.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "wcnst.h"
#include "wcnst_batch.hpp"
#include "wcnst_device.hpp"
#include "wcnst_host.hpp"

using namespace wcnst;
using namespace wcnstb;

namespace {

// flops of one stage-cell-update, 2D over 1D (only the ratio matters: it
// splits the device between the two kinds of work)
constexpr double COST_2D_OVER_1D = 2.9;

struct PoolReq {
    bool used = false;
    bool finished = false;
    bool init2d = false;
    wcnst_desc d{};
    double* U = nullptr;
    double* U1 = nullptr;
    double* U2 = nullptr;
    double t_final = 0.0, cfl = 0.0;
    BInst rec{};     // 1D: carried state and outcome
    int parity = 0;  // 2D: step parity of the current record
    int status = 0;
    double t = 0.0;
    long long steps = 0;
    double speed = 0.0;  // CFL speed of the state at t (0: unknown)
    unsigned long long bad_key = ~0ull;
};

}  // namespace

struct wcnst_pool {
    wcnst_desc scheme{};
    int cap = 0;
    hipStream_t s1 = nullptr;  // caller's stream: 1D passes, result copies
    hipStream_t s2 = nullptr;  // pool stream: 2D stage launches
    hipEvent_t ev_start = nullptr, ev_2d = nullptr;
    // device tables (caller's workspace)
    BInst* d_inst = nullptr;
    BSlot* d_slots = nullptr;
    BHead* d_head = nullptr;
    Req2D* d_req2 = nullptr;
    uint8_t* d_ctrl = nullptr;  // cap control blocks
    size_t ctrl_bytes = 0;
    // pinned host staging
    BInst* h_inst = nullptr;
    BSlot* h_slots = nullptr;
    BHead* h_head = nullptr;
    Req2D* h_req2 = nullptr;
    uint8_t* h_ctrl = nullptr;
    Params P1{};
    std::vector<PoolReq> reqs;
    double split = 1.0;
    int wpg = 4;
    int ty = 35;
    int cus = 1;
    long long wait_ticks = 0;
};

static size_t pool_layout(int cap, size_t* o_inst, size_t* o_slots, size_t* o_head, size_t* o_req2, size_t* o_ctrl)
{
    size_t o = 0;
    *o_inst = o;
    o = wcnst_align256(o + sizeof(BInst) * (size_t)cap);
    *o_slots = o;
    o = wcnst_align256(o + sizeof(BSlot) * (size_t)cap * KMAX);
    *o_head = o;
    o = wcnst_align256(o + sizeof(BHead));
    *o_req2 = o;
    o = wcnst_align256(o + sizeof(Req2D) * (size_t)cap);
    *o_ctrl = o;
    o = wcnst_align256(o + wcnst_align256(wcnst_ctrl_bytes()) * (size_t)cap);
    return o;
}

extern "C" wcnst_status wcnst_pool_workspace_size(int32_t capacity, size_t* bytes)
{
    if (capacity < 1 || capacity > (1 << 20)) return wcnst_fail(WCNST_E_INVALID_ARG, "capacity must be in [1, 2^20]");
    if (!bytes) return wcnst_fail(WCNST_E_INVALID_ARG, "null size pointer");
    size_t a, b, c, d, e;
    *bytes = pool_layout(capacity, &a, &b, &c, &d, &e);
    return WCNST_OK;
}

extern "C" wcnst_status wcnst_pool_destroy(wcnst_pool* p);

extern "C" wcnst_status wcnst_pool_create(const wcnst_desc* scheme, int32_t capacity, void* hip_stream,
                                          void* workspace, size_t ws_bytes, wcnst_pool** out)
{
    wcnst_status st = wcnst_check_desc(scheme);
    if (st) return st;
    if (scheme->system != WCNST_EULER) return wcnst_fail(WCNST_E_INVALID_ARG, "pools hold Euler problems");
    size_t need = 0;
    st = wcnst_pool_workspace_size(capacity, &need);
    if (st) return st;
    if (!out) return wcnst_fail(WCNST_E_INVALID_ARG, "null output handle");
    if (!workspace || ws_bytes < need)
        return wcnst_fail(WCNST_E_INVALID_ARG, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
    if (((uintptr_t)workspace & 255u) != 0) return wcnst_fail(WCNST_E_INVALID_ARG, "workspace not 256-byte aligned");
    size_t o_inst, o_slots, o_head, o_req2, o_ctrl;
    pool_layout(capacity, &o_inst, &o_slots, &o_head, &o_req2, &o_ctrl);

    wcnst_pool* p = new wcnst_pool();
    p->scheme = *scheme;
    p->cap = capacity;
    p->s1 = (hipStream_t)hip_stream;
    uint8_t* ws = (uint8_t*)workspace;
    p->d_inst = (BInst*)(ws + o_inst);
    p->d_slots = (BSlot*)(ws + o_slots);
    p->d_head = (BHead*)(ws + o_head);
    p->d_req2 = (Req2D*)(ws + o_req2);
    p->d_ctrl = ws + o_ctrl;
    p->ctrl_bytes = wcnst_align256(wcnst_ctrl_bytes());
    p->reqs.resize((size_t)capacity);
    scheme_params(*scheme, &p->P1);

    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = wait_ticks(&p->wait_ticks);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->s2, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_start, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_2d, hipEventDisableTiming);
    if (e == hipSuccess) e = hipHostMalloc((void**)&p->h_inst, sizeof(BInst) * (size_t)capacity, hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc((void**)&p->h_slots, sizeof(BSlot) * (size_t)capacity * KMAX, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&p->h_head, sizeof(BHead), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&p->h_req2, sizeof(Req2D) * (size_t)capacity, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&p->h_ctrl, p->ctrl_bytes * (size_t)capacity, hipHostMallocDefault);
    p->cus = std::max(1, cus);
    if (e != hipSuccess) {
        wcnst_pool_destroy(p);
        return wcnst_fail(WCNST_E_HIP, "pool setup failed: %s", hipGetErrorString(e));
    }
    *out = p;
    return WCNST_OK;
}

extern "C" wcnst_status wcnst_pool_set_tuning(wcnst_pool* p, double split, int32_t waves_per_group,
                                              int32_t rows_per_segment)
{
    if (!p) return wcnst_fail(WCNST_E_INVALID_ARG, "null handle");
    if (!(split >= 0.0)) return wcnst_fail(WCNST_E_INVALID_ARG, "split must be >= 0");
    if (waves_per_group != 0 && waves_per_group != 1 && waves_per_group != 2 && waves_per_group != 4)
        return wcnst_fail(WCNST_E_INVALID_ARG, "waves_per_group must be 1, 2 or 4 (0 keeps it)");
    if (rows_per_segment < 0) return wcnst_fail(WCNST_E_INVALID_ARG, "rows_per_segment must be >= 0");
    p->split = split;
    if (waves_per_group) p->wpg = waves_per_group;
    if (rows_per_segment) p->ty = rows_per_segment;
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
    if (d->ndim == 1) inst_init(r.rec, *d, U, U1, U2, t_final, cfl);
    *slot = free_slot;
    return WCNST_OK;
}

static bool reached(double t_final, double t) { return t_final - t <= 1e-12 * t_final; }

// Steps still to go (estimate) and a per-step cost for the device split.
static double remaining_steps(const PoolReq& r, long long cap)
{
    if (!(r.speed > 0.0) || !std::isfinite(r.speed)) return (double)cap;
    const double dt = r.cfl / r.speed;
    return std::min((double)cap, std::ceil((r.t_final - r.t) / dt) + 1.0);
}

extern "C" wcnst_status wcnst_pool_tick(wcnst_pool* p, int64_t steps, int32_t* n_active)
{
    if (!p) return wcnst_fail(WCNST_E_INVALID_ARG, "null handle");
    if (steps < 1 || steps > (1 << 20)) return wcnst_fail(WCNST_E_INVALID_ARG, "steps must be in [1, 2^20]");
    std::vector<int> a1, a2;
    for (int i = 0; i < p->cap; ++i) {
        const PoolReq& r = p->reqs[(size_t)i];
        if (!r.used || r.finished) continue;
        (r.d.ndim == 1 ? a1 : a2).push_back(i);
    }
    if (n_active) *n_active = (int32_t)(a1.size() + a2.size());
    if (a1.empty() && a2.empty()) return WCNST_OK;

    // estimated work of this tick per kind
    double w1 = 0.0, w2 = 0.0;
    for (int i : a1) w1 += (double)p->reqs[(size_t)i].d.nx * remaining_steps(p->reqs[(size_t)i], steps);
    for (int i : a2) {
        const PoolReq& r = p->reqs[(size_t)i];
        w2 += COST_2D_OVER_1D * (double)r.d.nx * r.d.ny * remaining_steps(r, steps);
    }

    // ---- 2D: stage launches on the pool stream, after the caller's work
    WCNST_HIP_TRY(hipEventRecord(p->ev_start, p->s1));
    WCNST_HIP_TRY(hipStreamWaitEvent(p->s2, p->ev_start, 0));
    if (!a2.empty()) {
        int blocks = 0;
        int nreq = 0;
        for (int i : a2) {
            PoolReq& r = p->reqs[(size_t)i];
            Ctrl* ctrl = (Ctrl*)(p->d_ctrl + p->ctrl_bytes * (size_t)i);
            if (!r.init2d) {
                WCNST_HIP_TRY(wcnst_launch_init2d(&r.d, r.U, ctrl, p->s2));
                r.init2d = true;
                r.parity = 0;
            }
            Req2D& q = p->h_req2[nreq++];
            q = Req2D{};
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
            blocks += q.nstrips * ((r.d.ny + p->ty - 1) / p->ty);
            r.parity = (int)((r.parity + steps) & 1);
        }
        WCNST_HIP_TRY(hipMemcpyAsync(p->d_req2, p->h_req2, sizeof(Req2D) * (size_t)nreq, hipMemcpyHostToDevice, p->s2));
        for (int64_t s = 0; s < steps; ++s)
            for (int stage = 0; stage < 3; ++stage)
                WCNST_HIP_TRY(wcnst_launch_multi2d(&p->scheme, p->d_req2, nreq, blocks, stage, (int)(s & 1), p->ty,
                                                   p->s2));
        // one copy of the control blocks of all slots
        WCNST_HIP_TRY(hipMemcpyAsync(p->h_ctrl, p->d_ctrl, p->ctrl_bytes * (size_t)p->cap, hipMemcpyDeviceToHost,
                                     p->s2));
    }
    WCNST_HIP_TRY(hipEventRecord(p->ev_2d, p->s2));

    // ---- 1D: one persistent pass on the caller's stream
    if (!a1.empty()) {
        int per_cu = 0;
        WCNST_HIP_TRY(resident_per_cu(p->scheme, p->wpg, &per_cu));
        const int resident = per_cu * p->cus;
        int grid = resident;
        if (w2 > 0.0) grid = std::max(1, std::min(resident, (int)std::lround(resident * w1 / (w1 + w2))));
        std::vector<BInst> rec;
        std::vector<double> cost;
        rec.reserve(a1.size());
        for (int i : a1) {
            PoolReq& r = p->reqs[(size_t)i];
            BInst b = r.rec;
            inst_arm(b, r.rec.steps + steps);
            rec.push_back(b);
            cost.push_back((double)r.d.nx * remaining_steps(r, steps));
        }
        std::vector<BSlot> slots;
        const int nslots = plan_parts(rec, cost, p->split, (double)p->wpg * grid, p->wpg * grid, slots);
        std::copy(rec.begin(), rec.end(), p->h_inst);
        std::copy(slots.begin(), slots.end(), p->h_slots);
        *p->h_head = BHead{};
        p->h_head->nslots = nslots;
        p->h_head->wait_ticks = p->wait_ticks;
        WCNST_HIP_TRY(hipMemcpyAsync(p->d_inst, p->h_inst, sizeof(BInst) * rec.size(), hipMemcpyHostToDevice, p->s1));
        WCNST_HIP_TRY(hipMemcpyAsync(p->d_slots, p->h_slots, sizeof(BSlot) * slots.size(), hipMemcpyHostToDevice,
                                     p->s1));
        WCNST_HIP_TRY(hipMemcpyAsync(p->d_head, p->h_head, sizeof(BHead), hipMemcpyHostToDevice, p->s1));
        WCNST_HIP_TRY(launch_pass(p->scheme, p->d_inst, p->d_slots, p->d_head, p->P1, grid, p->wpg, p->s1));
        WCNST_HIP_TRY(hipMemcpyAsync(p->h_inst, p->d_inst, sizeof(BInst) * rec.size(), hipMemcpyDeviceToHost, p->s1));
        WCNST_HIP_TRY(hipMemcpyAsync(p->h_head, p->d_head, sizeof(BHead), hipMemcpyDeviceToHost, p->s1));
    }
    WCNST_HIP_TRY(hipStreamWaitEvent(p->s1, p->ev_2d, 0));
    WCNST_HIP_TRY(hipStreamSynchronize(p->s1));

    if (!a1.empty()) {
        if (p->h_head->err) return wcnst_fail(WCNST_E_HIP, "a cooperating part waited past its limit");
        for (size_t j = 0; j < a1.size(); ++j) {
            PoolReq& r = p->reqs[(size_t)a1[j]];
            const BInst& b = p->h_inst[j];
            // step size of the last step (dt = CFL / speed) estimates the speed
            const double dt_last = b.steps > r.rec.steps ? (b.t - r.rec.t) / (double)(b.steps - r.rec.steps) : 0.0;
            r.rec.t = b.t;
            r.rec.steps = b.steps;
            r.rec.status = b.status;
            r.rec.bad_key = b.bad_key;
            r.t = b.t;
            r.steps = b.steps;
            r.status = b.status;
            r.bad_key = b.bad_key;
            r.speed = dt_last > 0.0 ? r.cfl / dt_last : 0.0;
            r.finished = r.status != 0 || reached(r.t_final, r.t);
        }
    }
    for (int i : a2) {
        PoolReq& r = p->reqs[(size_t)i];
        const Ctrl& c = *(const Ctrl*)(p->h_ctrl + p->ctrl_bytes * (size_t)i);
        const StepRec& n = c.rec[0].step >= c.rec[1].step ? c.rec[0] : c.rec[1];
        r.t = n.t;
        r.steps = n.step;
        r.status = c.status;
        r.bad_key = c.bad_key;
        double sp;
        const long long bits = (long long)n.smax_bits;
        memcpy(&sp, &bits, sizeof(sp));
        r.speed = sp;
        r.finished = r.status != 0 || reached(r.t_final, r.t);
    }
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
    if (p->h_inst) (void)hipHostFree(p->h_inst);
    if (p->h_slots) (void)hipHostFree(p->h_slots);
    if (p->h_head) (void)hipHostFree(p->h_head);
    if (p->h_req2) (void)hipHostFree(p->h_req2);
    if (p->h_ctrl) (void)hipHostFree(p->h_ctrl);
    delete p;
    return WCNST_OK;
}

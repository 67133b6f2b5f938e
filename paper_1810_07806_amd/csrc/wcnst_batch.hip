// Batched solve of many independent 1D Euler problems in one persistent,
// graph-captured launch.
//
// Each instance is advanced with exactly the arithmetic of the single-solve
// path (the same device functions, the same CFL rule and stopping rule), so
// an instance gives the same bits batched as alone.  Work decomposition:
//   * the worker is a 64-lane wavefront; waves of a workgroup are
//     independent (each has its own LDS exchange area);
//   * an instance is split into k contiguous parts of whole 61-cell strips
//     (k = 1 for most instances; large instances get more waves so the
//     largest one does not set the makespan);
//   * the host plans the jobs from a per-instance speed pre-pass (cost ~
//     cells x steps), orders them longest-part-first, and lays out one slot
//     per part; waves take slots from a device counter in order, so the
//     parts of a job are taken consecutively and a job never waits for a
//     slot that no free wave can take;
//   * the parts of a job meet at an agent-scope counter barrier after each
//     stage; every wait is bounded (timeout -> sticky error, all waves
//     leave), so the grid always drains.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "wcnst.h"
#include "wcnst_device.hpp"
#include "wcnst_batch.hpp"
#include "wcnst_host.hpp"

namespace wcnstb {

using namespace wcnst;

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long m)
{
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(m, off);
        m = o > m ? o : m;
    }
    return m;
}

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long m)
{
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(m, off);
        m = o < m ? o : m;
    }
    return m;
}

__device__ __forceinline__ void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Barrier of the k parts of one instance.  The last arriving part clears
// the speed slot that the next step will accumulate into.
__device__ bool part_sync(BInst* I, int k, unsigned& gen, BHead* hd, int clear_slot)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    int ok = 1;
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        const unsigned old = __hip_atomic_fetch_add(&I->arrive, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (old == (unsigned)k - 1) {
            __hip_atomic_store(&I->arrive, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (clear_slot >= 0)
                __hip_atomic_store(&I->smax_bits[clear_slot], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&I->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const long long t0 = (long long)wall_clock64();
            while (__hip_atomic_load(&I->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                if ((long long)wall_clock64() - t0 >
                        __hip_atomic_load(&hd->wait_ticks, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) ||
                    __hip_atomic_load(&hd->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    __hip_atomic_fetch_or(&hd->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
    }
    gen += 1u;
    ok = __shfl(ok, 0);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return ok != 0;
}

// One stage over the strips [s0, s1) of one instance: midpoint fluxes,
// MND difference, Runge-Kutta combine; stage 2 also returns the CFL speed.
template <int FLUX, int SCHEME, bool CHAR>
__device__ bool part_stage(const Params& P, int n, int s0, int s1, int stage, double dt, long long step,
                           const double* __restrict__ in, const double* __restrict__ Un, double* __restrict__ out,
                           double (*sF)[WAVE], double (*sN)[WAVE], unsigned long long& bad_key,
                           unsigned long long& smax)
{
    const int lane = threadIdx.x & (WAVE - 1);
    bool bad = false;
    for (int s = s0; s < s1; ++s) {
        const int x0 = s * TX;
        const int c = x0 + lane;
        const bool cell_ok = lane < TX && c < n;
        const int jx = x0 - 2 + lane;
        double st[6][NV];
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            const int col = ghost_map_any(jx - 2 + m, n, P.bc_x);
#pragma unroll
            for (int v = 0; v < NV; ++v) st[m][v] = in[(size_t)v * n + col];
        }
        double F[NV], fn[NV];
        unsigned fb;
        RegStencil<NV> rs{st};
        face_flux<SYS_EULER, NV, FLUX, SCHEME, CHAR>(rs, P, F, fb);
        node_flux<SYS_EULER, NV>(st[3], P, fn);
        wave_sync_lds();
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            sF[v][lane] = F[v];
            sN[v][lane] = fn[v];
        }
        wave_sync_lds();
        if (cell_ok) {
            double R[NV], un[NV], o[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                R[v] = mnd(P.c1x, P.c2x, P.c3x, sF[v][lane], sF[v][lane + 1], sF[v][lane + 2], sF[v][lane + 3],
                           sN[v][lane], sN[v][lane + 2]);
                un[v] = stage ? Un[(size_t)v * n + c] : 0.0;
            }
            rk_combine<NV>(stage, dt, st[4], un, R, o);
#pragma unroll
            for (int v = 0; v < NV; ++v) out[(size_t)v * n + c] = o[v];
            if (cell_bad<SYS_EULER, NV>(o, P)) {
                const unsigned long long key = ((unsigned long long)(step * 3 + stage) << 36) | (unsigned long long)c;
                bad_key = key < bad_key ? key : bad_key;
                bad = true;
            }
            if (stage == 2) {
                const unsigned long long b =
                    (unsigned long long)__double_as_longlong(cell_speed<SYS_EULER, NV>(o, P));
                smax = b > smax ? b : smax;
            }
        }
    }
    return __any(bad);
}

template <int FLUX, int SCHEME, bool CHAR>
__device__ void run_part(BInst* I, int part, const Params& Pc, BHead* hd, double (*sF)[WAVE], double (*sN)[WAVE])
{
    const int lane = threadIdx.x & (WAVE - 1);
    // Every part of the instance takes its control flow (k, t, steps, the
    // step bound) from the same host-written values.
    const BInstIn R = load_host_written(reinterpret_cast<const BInstIn*>(I));
    const int n = R.n, k = R.k;
    const int S = (n + TX - 1) / TX;
    const int s0 = (int)((long long)part * S / k), s1 = (int)((long long)(part + 1) * S / k);
    Params P = Pc;
    P.nx = n;
    P.dx = R.dx;
    P.c1x = R.c1;
    P.c2x = R.c2;
    P.c3x = R.c3;
    P.bc_x = R.bc;
    double* U = R.u;
    double* U1 = R.u1;
    double* U2 = R.u2;
    const double t_final = R.t_final, cfl = R.cfl;
    const long long step_end = R.step_end;
    const bool fin = isfinite(t_final);

    // CFL speed of the state at the start of the launch (the same bits as
    // the speed the previous step reduced from the same cells)
    unsigned gen = 0;
    unsigned long long sm = 0ull;
    for (int s = s0; s < s1; ++s) {
        const int c = s * TX + lane;
        if (lane < TX && c < n) {
            double u[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) u[v] = U[(size_t)v * n + c];
            const unsigned long long b = (unsigned long long)__double_as_longlong(cell_speed<SYS_EULER, NV>(u, P));
            sm = b > sm ? b : sm;
        }
    }
    sm = wave_max_u64(sm);
    if (k > 1) {
        // Slot s & 1 of step s: every part reads it before stage 0 and the
        // stage-2 barrier of step s clears it, after all parts arrived.
        const int sl = (int)(R.steps & 1);
        if (lane == 0) __hip_atomic_fetch_max(&I->smax_bits[sl], sm, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (!part_sync(I, k, gen, hd, -1)) return;
        sm = __hip_atomic_load(&I->smax_bits[sl], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }

    double t = R.t;
    long long step = R.steps;
    unsigned long long bad_key = ~0ull;
    bool bad = false;
    while (step < step_end) {
        if (fin && t_final - t <= 1e-12 * t_final) break;
        double dt = cfl / __longlong_as_double((long long)sm);
        if (fin && dt > t_final - t) dt = t_final - t;
        unsigned long long snext = 0ull;
        const double* in[3] = {U, U1, U2};
        double* outp[3] = {U1, U2, U};
        for (int stage = 0; stage < 3; ++stage) {
            bad |= part_stage<FLUX, SCHEME, CHAR>(P, n, s0, s1, stage, dt, step, in[stage], U, outp[stage], sF, sN,
                                                   bad_key, snext);
            if (k == 1) {
                // this wave's stores are read by other lanes of the wave next
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            } else {
                // wave-wide reductions first (all lanes), then one lane publishes
                const unsigned long long mx = stage == 2 ? wave_max_u64(snext) : 0ull;
                const unsigned long long bk = bad ? wave_min_u64(bad_key) : ~0ull;
                if (stage == 2 && lane == 0)
                    __hip_atomic_fetch_max(&I->smax_bits[(step + 1) & 1], mx, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                if (bad && lane == 0) {
                    __hip_atomic_fetch_min(&I->bad_key, bk, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_fetch_or(&I->status, (int)WCNST_E_NONPHYSICAL, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
                }
                if (!part_sync(I, k, gen, hd, stage == 2 ? (int)(step & 1) : -1)) return;
                bad = __hip_atomic_load(&I->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
            }
            if (bad) break;
        }
        if (bad) break;
        if (k == 1) sm = wave_max_u64(snext);
        else sm = __hip_atomic_load(&I->smax_bits[(step + 1) & 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        t = t + dt;
        step += 1;
    }
    if (k == 1 && bad) {
        bad_key = wave_min_u64(bad_key);
        if (lane == 0) {
            __hip_atomic_store(&I->bad_key, bad_key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            __hip_atomic_store(&I->status, (int)WCNST_E_NONPHYSICAL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
    if (part == 0 && lane == 0) {
        __hip_atomic_store(&I->t, t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&I->steps, step, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

template <int FLUX, int SCHEME, bool CHAR>
__global__ void __launch_bounds__(256) batch_kernel(BInst* __restrict__ insts, const BSlot* __restrict__ slots,
                                                    BHead* hd, Params Pc)
{
    init_weight_table();
    __shared__ double sFall[256 / WAVE][NV][WAVE];
    __shared__ double sNall[256 / WAVE][NV][WAVE];
    const int w = threadIdx.x / WAVE;
    const int lane = threadIdx.x & (WAVE - 1);
    const int nslots = __hip_atomic_load(&hd->nslots, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    for (;;) {
        int slot = 0;
        if (lane == 0) slot = (int)atomicAdd(&hd->head, 1u);
        slot = __shfl(slot, 0);
        if (slot >= nslots) break;
        if (__hip_atomic_load(&hd->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
        const BSlot sl = load_host_written(&slots[slot]);
        run_part<FLUX, SCHEME, CHAR>(&insts[sl.inst], sl.part, Pc, hd, sFall[w], sNall[w]);
    }
}

// Initial CFL speed of each instance (one workgroup per instance), for planning.
__global__ void __launch_bounds__(256) batch_speed(const BInst* __restrict__ insts, Params Pc, double* speed)
{
    const BInstIn I = load_host_written(reinterpret_cast<const BInstIn*>(&insts[blockIdx.x]));
    Params P = Pc;
    P.nx = I.n;
    P.dx = I.dx;
    const double* U = I.u;
    unsigned long long m = 0ull;
    for (int c = threadIdx.x; c < I.n; c += blockDim.x) {
        double u[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) u[v] = U[(size_t)v * I.n + c];
        const unsigned long long b = (unsigned long long)__double_as_longlong(cell_speed<SYS_EULER, NV>(u, P));
        m = b > m ? b : m;
    }
    m = wave_max_u64(m);
    __shared__ unsigned long long red[256 / WAVE];
    if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < (int)(blockDim.x / WAVE); ++i) m = red[i] > m ? red[i] : m;
        m = red[0] > m ? red[0] : m;
        speed[blockIdx.x] = __longlong_as_double((long long)m);
    }
}

// Resets the queue of a launch (the plan fields are written by the host
// before each launch, so the captured graph stays valid across plans).
__global__ void batch_open(BHead* hd)
{
    if (threadIdx.x == 0) {
        hd->head = 0u;
        hd->err = 0;
    }
}

}  // namespace wcnstb

// ====================================================================== host

namespace wcnstb {

void inst_init(BInst& r, const wcnst_desc& d, double* u, double* u1, double* u2, double t_final, double cfl)
{
    r = BInst{};
    r.u = u;
    r.u1 = u1;
    r.u2 = u2;
    r.n = d.nx;
    r.bc = d.bc_x;
    r.k = 1;
    r.dx = (d.x1 - d.x0) / d.nx;
    // the same expressions as the single-solve path (Eq. (5) over h)
    r.c1 = (3.0 / 2.0) / r.dx;
    r.c2 = (-3.0 / 10.0) / r.dx;
    r.c3 = (1.0 / 30.0) / r.dx;
    r.t_final = t_final;
    r.cfl = cfl;
    r.t = 0.0;
    r.steps = 0;
    r.bad_key = ~0ull;
    r.status = 0;
}

void inst_arm(BInst& r, long long step_end)
{
    r.step_end = step_end;
    r.arrive = 0;
    r.gen = 0;
    r.smax_bits[0] = r.smax_bits[1] = 0ull;
}

void scheme_params(const wcnst_desc& d, Params* out)
{
    Params P{};
    P.CT = d.CT;
    P.C = d.C;
    P.eps_teno = d.eps_teno;
    P.eps_js = d.eps_js;
    P.gamma = d.gamma;
    P.adv = d.adv_speed;
    P.q = d.q;
    P.charwise = d.charwise ? 1 : 0;
    P.ny = 1;
    P.dy = 1.0;
    *out = P;
}

template <int FLUX, int SCHEME, bool CHAR>
static const void* pick3() { return (const void*)&batch_kernel<FLUX, SCHEME, CHAR>; }

template <int FLUX, bool CHAR>
static const void* pick2(const wcnst_desc& d)
{
    switch (d.scheme) {
    case WCNST_LINEAR: return pick3<FLUX, SCH_LINEAR, CHAR>();
    case WCNST_JS: return pick3<FLUX, SCH_JS, CHAR>();
    default: return d.q == 6 ? pick3<FLUX, SCH_TENO, CHAR>() : pick3<FLUX, SCH_TENO_Q, CHAR>();
    }
}

static const void* pick_kernel(const wcnst_desc& d)
{
    if (d.flux == WCNST_LF) return d.charwise ? pick2<FLUX_LF, true>(d) : pick2<FLUX_LF, false>(d);
    return d.charwise ? pick2<FLUX_ROE, true>(d) : pick2<FLUX_ROE, false>(d);
}

hipError_t resident_per_cu(const wcnst_desc& d, int wpg, int* per_cu)
{
    *per_cu = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, pick_kernel(d), WAVE * wpg, 0);
    if (*per_cu < 1) *per_cu = 1;
    return e;
}

int plan_parts(std::vector<BInst>& rec, const std::vector<double>& cost, double split, double workers, int running,
               std::vector<BSlot>& slots)
{
    const int n = (int)rec.size();
    double total = 0.0;
    for (double c : cost) total += c;
    std::vector<int> order((size_t)n);
    for (int i = 0; i < n; ++i) {
        const int strips = (rec[(size_t)i].n + TX - 1) / TX;
        int k = 1;
        if (split > 0.0 && total > 0.0)
            k = (int)std::min(1e9, std::ceil(cost[(size_t)i] * workers / (split * total)));
        k = std::max(1, std::min(k, std::min(std::min(KMAX, strips), std::max(1, running))));
        rec[(size_t)i].k = k;
        order[(size_t)i] = i;
    }
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return cost[(size_t)x] / rec[(size_t)x].k > cost[(size_t)y] / rec[(size_t)y].k;
    });
    slots.clear();
    for (int i : order)
        for (int p = 0; p < rec[(size_t)i].k; ++p) slots.push_back(BSlot{i, p});
    return (int)slots.size();
}

hipError_t launch_pass(const wcnst_desc& d, BInst* insts, BSlot* slots, BHead* head, const Params& P, int grid,
                       int wpg, hipStream_t st)
{
    hipLaunchKernelGGL(batch_open, dim3(1), dim3(64), 0, st, head);
    void* args[] = {(void*)&insts, (void*)&slots, (void*)&head, (void*)&P};
    const hipError_t e = hipLaunchKernel(pick_kernel(d), dim3(grid), dim3(WAVE * wpg), args, 0, st);
    return e != hipSuccess ? e : hipGetLastError();
}

hipError_t wait_ticks(long long* ticks)
{
    int dev = 0, khz = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    *ticks = (long long)(WAIT_LIMIT_S * 1e3 * std::max(1, khz));
    return e;
}

}  // namespace wcnstb

using namespace wcnstb;

struct wcnst_batch {
    int n = 0;
    wcnst_desc d0{};
    std::vector<wcnst_desc> descs;
    std::vector<BInst> rec;
    std::vector<long long> offs;  // n + 1
    long long total = 0;          // doubles per packed buffer
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;  // private stream for graph capture
    BInst* d_inst = nullptr;
    BSlot* d_slots = nullptr;
    BHead* d_head = nullptr;
    double* d_speed = nullptr;
    double* U1 = nullptr;
    double* U2 = nullptr;
    Params P{};
    double split = 1.0;
    int grid = 0;      // persistent workgroups
    int wpg = 4;       // wavefronts per workgroup
    int resident = 0;  // workgroups of wpg waves resident at once
    int cus = 0;
    long long wait_ticks = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double kernel_ms = 0.0;
    hipGraphExec_t exec = nullptr;
    const void* exec_key = nullptr;
    int exec_grid = 0, exec_wpg = 0;
};

static size_t batch_layout(int n, long long total, size_t* o_inst, size_t* o_slots, size_t* o_head, size_t* o_speed,
                           size_t* o_u1, size_t* o_u2)
{
    size_t o = 0;
    *o_inst = o;
    o = wcnst_align256(o + sizeof(BInst) * (size_t)n);
    *o_slots = o;
    o = wcnst_align256(o + sizeof(BSlot) * (size_t)n * KMAX);
    *o_head = o;
    o = wcnst_align256(o + sizeof(BHead));
    *o_speed = o;
    o = wcnst_align256(o + sizeof(double) * (size_t)n);
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
        d.CT != a.CT || d.C != a.C || d.eps_teno != a.eps_teno || d.eps_js != a.eps_js || d.diff != a.diff)
        return WCNST_E_INVALID_ARG;
    return WCNST_OK;
}

static wcnst_status batch_check(const wcnst_desc* descs, int32_t n, long long* total, std::vector<long long>* offs)
{
    if (!descs || n < 1) return wcnst_fail(WCNST_E_INVALID_ARG, "need at least one descriptor");
    const wcnst_desc& a = descs[0];
    long long off = 0;
    if (offs) offs->assign((size_t)n + 1, 0);
    for (int i = 0; i < n; ++i) {
        const wcnst_desc& d = descs[i];
        wcnst_status st = wcnst_check_desc(&d);
        if (st) return wcnst_fail(st, "descriptor %d: %s", i, wcnst_last_error());
        if (d.ndim != 1 || d.system != WCNST_EULER)
            return wcnst_fail(WCNST_E_INVALID_ARG, "descriptor %d: batches hold 1D Euler problems", i);
        if (wcnst_check_same_scheme(a, d))
            return wcnst_fail(WCNST_E_INVALID_ARG, "descriptor %d: scheme parameters differ from descriptor 0", i);
        if (offs) (*offs)[i] = off;
        off += ((long long)NV * d.nx + 63) / 64 * 64;  // 512-byte aligned instances
    }
    if (offs) (*offs)[n] = off;
    if (total) *total = off;
    return WCNST_OK;
}

extern "C" wcnst_status wcnst_batch_workspace_size(const wcnst_desc* descs, int32_t n, size_t* bytes)
{
    long long total = 0;
    wcnst_status st = batch_check(descs, n, &total, nullptr);
    if (st) return st;
    if (!bytes) return wcnst_fail(WCNST_E_INVALID_ARG, "null size pointer");
    size_t a, b, c, d, e, f;
    *bytes = batch_layout(n, total, &a, &b, &c, &d, &e, &f);
    return WCNST_OK;
}

extern "C" wcnst_status wcnst_batch_destroy(wcnst_batch* b);

static hipError_t batch_resident(wcnst_batch* b)
{
    int per_cu = 0;
    const hipError_t e = resident_per_cu(b->d0, b->wpg, &per_cu);
    b->resident = per_cu * b->cus;
    return e;
}

extern "C" wcnst_status wcnst_batch_create(const wcnst_desc* descs, int32_t n, void* hip_stream, void* workspace,
                                           size_t ws_bytes, wcnst_batch** out)
{
    long long total = 0;
    std::vector<long long> offs;
    wcnst_status st = batch_check(descs, n, &total, &offs);
    if (st) return st;
    if (!out) return wcnst_fail(WCNST_E_INVALID_ARG, "null output handle");
    size_t o_inst, o_slots, o_head, o_speed, o_u1, o_u2;
    const size_t need = batch_layout(n, total, &o_inst, &o_slots, &o_head, &o_speed, &o_u1, &o_u2);
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
    b->d_inst = (BInst*)(ws + o_inst);
    b->d_slots = (BSlot*)(ws + o_slots);
    b->d_head = (BHead*)(ws + o_head);
    b->d_speed = (double*)(ws + o_speed);
    b->U1 = (double*)(ws + o_u1);
    b->U2 = (double*)(ws + o_u2);
    b->rec.assign((size_t)n, BInst{});
    scheme_params(descs[0], &b->P);

    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = wait_ticks(&b->wait_ticks);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&b->ev0);
    if (e == hipSuccess) e = hipEventCreate(&b->ev1);
    b->cus = std::max(1, cus);
    if (e == hipSuccess) e = batch_resident(b);
    b->grid = b->resident;
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

extern "C" wcnst_status wcnst_batch_set_tuning(wcnst_batch* b, double split, int32_t workgroups,
                                               int32_t waves_per_group)
{
    if (!b) return wcnst_fail(WCNST_E_INVALID_ARG, "null handle");
    if (!(split >= 0.0)) return wcnst_fail(WCNST_E_INVALID_ARG, "split must be >= 0");
    if (workgroups < 0) return wcnst_fail(WCNST_E_INVALID_ARG, "workgroups must be >= 0");
    if (waves_per_group != 0 && waves_per_group != 1 && waves_per_group != 2 && waves_per_group != 4)
        return wcnst_fail(WCNST_E_INVALID_ARG, "waves_per_group must be 1, 2 or 4 (0 keeps it)");
    b->split = split;
    if (waves_per_group) b->wpg = waves_per_group;
    hipError_t e = batch_resident(b);
    if (e != hipSuccess) return wcnst_fail(WCNST_E_HIP, "occupancy query failed: %s", hipGetErrorString(e));
    b->grid = workgroups > 0 ? workgroups : b->resident;
    return WCNST_OK;
}

extern "C" wcnst_status wcnst_batch_kernel_ms(const wcnst_batch* b, double* ms)
{
    if (!b || !ms) return wcnst_fail(WCNST_E_INVALID_ARG, "null argument");
    *ms = b->kernel_ms;
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
        BInst& r = b->rec[(size_t)i];
        const long long o = b->offs[(size_t)i];
        inst_init(r, b->descs[(size_t)i], U + o, b->U1 + o, b->U2 + o, t_final[i], cfl);
        inst_arm(r, (long long)max_steps);
    }
    // initial speeds for the plan
    WCNST_HIP_TRY(hipMemcpyAsync(b->d_inst, b->rec.data(), sizeof(BInst) * (size_t)n, hipMemcpyHostToDevice,
                                 b->stream));
    hipLaunchKernelGGL(batch_speed, dim3(n), dim3(256), 0, b->stream, b->d_inst, b->P, b->d_speed);
    WCNST_HIP_TRY(hipGetLastError());
    std::vector<double> speed((size_t)n);
    WCNST_HIP_TRY(hipMemcpyAsync(speed.data(), b->d_speed, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost,
                                 b->stream));
    WCNST_HIP_TRY(hipStreamSynchronize(b->stream));
    std::vector<double> cost((size_t)n);
    for (int i = 0; i < n; ++i) {
        double steps = (double)max_steps;
        if (std::isfinite(t_final[i]) && std::isfinite(speed[(size_t)i]))
            steps = std::min(steps, std::ceil(t_final[i] * speed[(size_t)i] / cfl) + 1.0);
        cost[(size_t)i] = (double)b->rec[(size_t)i].n * steps;
    }
    std::vector<BSlot> slots;
    const int running = b->wpg * std::min(b->grid, b->resident);
    const int nslots = plan_parts(b->rec, cost, b->split, (double)b->wpg * b->grid, running, slots);
    BHead h{};
    h.nslots = nslots;
    h.wait_ticks = b->wait_ticks;
    WCNST_HIP_TRY(hipMemcpyAsync(b->d_inst, b->rec.data(), sizeof(BInst) * (size_t)n, hipMemcpyHostToDevice,
                                 b->stream));
    WCNST_HIP_TRY(hipMemcpyAsync(b->d_slots, slots.data(), sizeof(BSlot) * slots.size(), hipMemcpyHostToDevice,
                                 b->stream));
    WCNST_HIP_TRY(hipMemcpyAsync(b->d_head, &h, sizeof(BHead), hipMemcpyHostToDevice, b->stream));
    // the tables must be in device memory before the graph's kernels start
    WCNST_HIP_TRY(hipStreamSynchronize(b->stream));

    // one persistent launch, captured once into a graph and replayed (the
    // buffers are reached through the instance table, so the graph does
    // not depend on U)
    const void* key = pick_kernel(b->d0);
    if (!b->exec || b->exec_key != key || b->exec_grid != b->grid || b->exec_wpg != b->wpg) {
        if (b->exec) {
            (void)hipGraphExecDestroy(b->exec);
            b->exec = nullptr;
        }
        hipGraph_t g = nullptr;
        WCNST_HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
        hipError_t le = launch_pass(b->d0, b->d_inst, b->d_slots, b->d_head, b->P, b->grid, b->wpg, b->cap);
        hipError_t ce = hipStreamEndCapture(b->cap, &g);
        if (le != hipSuccess || ce != hipSuccess)
            return wcnst_fail(WCNST_E_HIP, "graph capture failed: %s / %s", hipGetErrorString(le),
                              hipGetErrorString(ce));
        hipError_t ie = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) return wcnst_fail(WCNST_E_HIP, "graph instantiate failed: %s", hipGetErrorString(ie));
        b->exec_key = key;
        b->exec_grid = b->grid;
        b->exec_wpg = b->wpg;
    }
    WCNST_HIP_TRY(hipEventRecord(b->ev0, b->stream));
    WCNST_HIP_TRY(hipGraphLaunch(b->exec, b->stream));
    WCNST_HIP_TRY(hipEventRecord(b->ev1, b->stream));
    WCNST_HIP_TRY(hipMemcpyAsync(b->rec.data(), b->d_inst, sizeof(BInst) * (size_t)n, hipMemcpyDeviceToHost,
                                 b->stream));
    WCNST_HIP_TRY(hipMemcpyAsync(&h, b->d_head, sizeof(BHead), hipMemcpyDeviceToHost, b->stream));
    WCNST_HIP_TRY(hipStreamSynchronize(b->stream));
    float ms = 0.0f;
    WCNST_HIP_TRY(hipEventElapsedTime(&ms, b->ev0, b->ev1));
    b->kernel_ms = ms;
    if (h.err) return wcnst_fail(WCNST_E_HIP, "a cooperating part waited past its limit");
    wcnst_status ret = WCNST_OK;
    for (int i = 0; i < n; ++i) {
        const BInst& r = b->rec[(size_t)i];
        int s = r.status;
        if (s == 0 && std::isfinite(r.t_final) && !(r.t_final - r.t <= 1e-12 * r.t_final)) s = WCNST_E_MAX_STEPS;
        status[i] = s;
        if (t_out) t_out[i] = r.t;
        if (steps_out) steps_out[i] = r.steps;
        if (s != 0 && ret == WCNST_OK) ret = s;
    }
    if (ret != WCNST_OK) return wcnst_fail(ret, "at least one instance did not finish (see the status array)");
    return WCNST_OK;
}

extern "C" wcnst_status wcnst_batch_bad_cells(const wcnst_batch* b, int64_t* bad_stage, int64_t* bad_cell)
{
    if (!b || !bad_stage || !bad_cell) return wcnst_fail(WCNST_E_INVALID_ARG, "null argument");
    for (int i = 0; i < b->n; ++i) {
        const unsigned long long key = b->rec[(size_t)i].bad_key;
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
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->ev0) (void)hipEventDestroy(b->ev0);
    if (b->ev1) (void)hipEventDestroy(b->ev1);
    delete b;
    return WCNST_OK;
}

// HIP kernels (gfx950) and the C ABI of the WCNS-T solver core.
//
// Hot path per Runge-Kutta stage: one fused kernel computes, for every cell,
// the midpoint fluxes around it (Sec. 2.2-2.3), the MND difference of
// Sec. 2.1 Eq. (5) in x and y (1D grids may also use MD, Eq. (3), or HWCNS,
// Eq. (4)), and the stage update of SSP-RK3 (Sec. 2); the last stage also
// reduces the CFL wave speed of the new state.
//
// Work decomposition.  One wavefront (64 lanes) owns a strip of TX = 61
// columns, so one row of the strip needs exactly 64 x-midpoints (j = x0-2 ..
// x0+61): lane l computes midpoint x0-2+l.  In 2D the wavefront marches up a
// segment of rows; lane l owns column x0+l and computes one y-midpoint per
// row, keeping the last four y-midpoint fluxes in registers, so every
// midpoint flux is computed once per strip.  The x-flux of a row is
// exchanged through 512 bytes of LDS per variable.  Ghost cells are never
// stored: an index remap at load time, plus a sign or a fixed state for
// reflecting and fixed sides (no extra HBM traffic).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "wcnst.h"
#include "wcnst_device.hpp"
#include "wcnst_host.hpp"

namespace wcnst {

enum { MODE_RHS = 0, MODE_STAGE = 1 };

struct StageArgs {
    double t_final;
    double cfl;
    double fixed_dt;
    int stage;   // 0, 1, 2
    int parity;  // which record is current
};

__device__ __forceinline__ bool first_thread()
{
    return threadIdx.x == 0 && blockIdx.x == 0 && blockIdx.y == 0;
}

// Reads the step record; stage 0 also decides dt (every block computes the
// same value from the same inputs) and opens the next record.  Stage 2 also
// reads the next record's CFL speed as it stands (seen): a lower bound of
// the value the launch leaves there, which lets flush_speed skip atomics.
__device__ __forceinline__ bool stage_prologue(Ctrl* ctrl, const StageArgs& A, double& dt,
                                               long long& step, bool lead, unsigned long long& seen)
{
    const StepRec* cur = &ctrl->rec[A.parity];
    // independent reads, issued together (stage 0's lead writes the record's
    // dt, so only stages 1-2 read it)
    const int status = ctrl->status, done = ctrl->done;
    const long long stp = cur->step;
    const double t = cur->t;
    const unsigned long long sbits = cur->smax_bits;
    const double dt_rec = A.stage != 0 ? cur->dt : 0.0;
    // (an atomic load: from L2, where the other waves' maxima arrive, not a
    // per-CU cached copy of the launch's first read)
    seen = A.stage == 2 ? __hip_atomic_load(&ctrl->rec[A.parity ^ 1].smax_bits, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT)
                        : 0ull;
    if (status != 0 || done != 0) return false;
    step = stp;
    if (A.stage != 0) {
        dt = dt_rec;
        return true;
    }
    const bool fin = isfinite(A.t_final);
    if (fin && A.t_final - t <= 1e-12 * A.t_final) {
        if (lead) ctrl->done = 1;
        return false;
    }
    const double smax = __longlong_as_double((long long)sbits);
    dt = A.fixed_dt > 0.0 ? A.fixed_dt : A.cfl / smax;
    if (fin && dt > A.t_final - t) dt = A.t_final - t;
    if (lead) {
        StepRec* nx = &ctrl->rec[A.parity ^ 1];
        ctrl->rec[A.parity].dt = dt;
        nx->t = t + dt;
        nx->dt = 0.0;
        nx->step = step + 1;
        nx->smax_bits = 0ull;
    }
    return true;
}

__device__ __forceinline__ unsigned long long wave_max_bits(unsigned long long m)
{
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(m, off);
        m = o > m ? o : m;
    }
    return m;
}

template <int SYS, int NV>
__device__ __forceinline__ void stage_epilogue(Ctrl* ctrl, const Params& P, int stage, long long step,
                                               long long cell, const double* o,
                                               unsigned long long& smax_loc)
{
    if (cell_bad<SYS, NV>(o, P)) {
        const unsigned long long key =
            ((unsigned long long)(step * 3 + stage) << 36) | (unsigned long long)cell;
        atomicMin(&ctrl->bad_key, key);
        atomicOr(&ctrl->status, (int)WCNST_E_NONPHYSICAL);
    }
    if (stage == 2) {
        const unsigned long long b = (unsigned long long)__double_as_longlong(cell_speed<SYS, NV>(o, P));
        smax_loc = b > smax_loc ? b : smax_loc;
    }
}

// One wave's CFL speed into the next step's record.  The record only grows
// during the launch (stage 0 of the step cleared it in an earlier launch), so
// a wave whose maximum it already held when the wave started (seen) skips
// the atomic: on a long line tens of thousands of waves would otherwise queue
// on the one address.
__device__ __forceinline__ void flush_speed(Ctrl* ctrl, int parity, unsigned long long smax_loc,
                                            unsigned long long seen)
{
    const unsigned long long m = wave_max_bits(smax_loc);
    if (threadIdx.x == 0 && seen < m) atomicMax(&ctrl->rec[parity ^ 1].smax_bits, m);
}

template <int NV>
__device__ __forceinline__ void write_flags(uint8_t* fl, int nlines, int nfaces, int line, int slot,
                                            unsigned fb)
{
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const size_t idx = (((size_t)k * nlines + line) * nfaces + slot) * 2;
        fl[idx] = (uint8_t)((fb >> (6 * k)) & 7u);
        fl[idx + 1] = (uint8_t)((fb >> (6 * k + 3)) & 7u);
    }
}

// ------------------------------------------------------------------ 1D

// Strip bx of one 1D grid (geometry in Strip1D).  Thread 0 of strip 0
// opens the next step record.
// GB: general boundaries (reflecting walls, fixed ends); without it only
// index-remap sides (periodic, zero gradient).
template <int SYS, int NV, int FLUX, int SCHEME, bool CHAR, int MODE, int DIFF = DIFF_MND, bool GB = true>
__device__ __forceinline__ void sweep1d_block(const double* __restrict__ U, const double* __restrict__ Un,
                                              double* __restrict__ out, uint8_t* __restrict__ flags,
                                              Ctrl* __restrict__ ctrl, const Params& P, const StageArgs& A, int bx)
{
    constexpr int G = Strip1D<DIFF>::G;
    const int nx = P.nx;
    const int lane = threadIdx.x;
    const Strip1D<DIFF> S(bx, lane, nx);
    const int c = S.c, jx = S.jx, jxl = S.jxl;
    const bool cell_ok = S.cell_ok;

    // the stencil (and U^n of this lane's cell) load while the control
    // record is read
    double s[6][NV], un[NV];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        // HWCNS lanes reach up to 5 cells past the line: any-distance map
        const int col = DIFF == DIFF_HW ? ghost_map_any(jxl - 2 + m, nx, P.bc_x) : ghost_map(jxl - 2 + m, nx, P.bc_x);
#pragma unroll
        for (int v = 0; v < NV; ++v) s[m][v] = U[(size_t)v * nx + col];
    }
    if (GB && P.bc_x >= BC_REFLECT) {
        // reflecting walls reverse the momentum of their ghosts; fixed ends
        // supply their own states
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            const int kind = ghost_kind(jxl - 2 + m, nx, P.bc_x);
#pragma unroll
            for (int v = 0; v < NV; ++v) s[m][v] = ghost_value(kind, v, 1, s[m][v], P.fixed_x);
        }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) un[v] = MODE == MODE_STAGE && A.stage && cell_ok ? Un[(size_t)v * nx + c] : 0.0;
    double dt = 0.0;
    long long step = 0;
    unsigned long long seen = 0ull;
    if constexpr (MODE == MODE_STAGE) {
        if (!stage_prologue(ctrl, A, dt, step, bx == 0 && threadIdx.x == 0, seen)) return;
    }
    __shared__ double sF[NV][WAVE];
    __shared__ double sN[NV][WAVE];
    init_weight_table();
    double F[NV], fn[NV];
    unsigned fb;
    RegStencil<NV> st{s};
    face_flux<SYS, NV, FLUX, SCHEME, CHAR>(st, P, F, fb);
    if (MODE == MODE_RHS && flags && S.owns_face(bx, nx)) write_flags<NV>(flags, 1, S.nfaces(), 0, jx + G, fb);
    // node flux: MND at node jx+1 (stencil node 3), HWCNS at node jx-1 (1)
    if constexpr (DIFF == DIFF_MND) node_flux<SYS, NV>(s[3], P, fn);
    if constexpr (DIFF == DIFF_HW) node_flux<SYS, NV>(s[1], P, fn);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        sF[v][lane] = F[v];
        if constexpr (DIFF != DIFF_MD) sN[v][lane] = fn[v];
    }
    __syncthreads();
    unsigned long long sm = 0ull;
    if (cell_ok) {
        double R[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            if constexpr (DIFF == DIFF_MD)
                R[v] = md(P.c1x, P.c2x, P.c3x, sF[v][lane], sF[v][lane + 1], sF[v][lane + 2], sF[v][lane + 3],
                          sF[v][lane + 4], sF[v][lane + 5]);
            else if constexpr (DIFF == DIFF_HW)
                R[v] = hwcns(P.c1x, P.c2x, P.c3x, sF[v][lane], sF[v][lane + 1], sN[v][lane], sN[v][lane + 1],
                             sN[v][lane + 3], sN[v][lane + 4]);
            else
                R[v] = mnd(P.c1x, P.c2x, P.c3x, sF[v][lane], sF[v][lane + 1], sF[v][lane + 2], sF[v][lane + 3],
                           sN[v][lane], sN[v][lane + 2]);
        }
        if constexpr (MODE == MODE_RHS) {
#pragma unroll
            for (int v = 0; v < NV; ++v) out[(size_t)v * nx + c] = R[v];
        } else {
            double o[NV];
            rk_combine<NV>(A.stage, dt, s[G + 2], un, R, o);
#pragma unroll
            for (int v = 0; v < NV; ++v) out[(size_t)v * nx + c] = o[v];
            stage_epilogue<SYS, NV>(ctrl, P, A.stage, step, c, o, sm);
        }
    }
    if constexpr (MODE == MODE_STAGE) {
        if (A.stage == 2) flush_speed(ctrl, A.parity, sm, seen);
    }
}

template <int SYS, int NV, int FLUX, int SCHEME, bool CHAR, int MODE, int DIFF>
__global__ void __launch_bounds__(WAVE)
sweep1d(const double* __restrict__ U, const double* __restrict__ Un, double* __restrict__ out,
        uint8_t* __restrict__ flags, Ctrl* __restrict__ ctrl, Params P, StageArgs A)
{
    sweep1d_block<SYS, NV, FLUX, SCHEME, CHAR, MODE, DIFF>(U, Un, out, flags, ctrl, P, A, (int)blockIdx.x);
}

// ------------------------------------------------------ 1D latency mode

// A stage over a few strips cannot fill the chip, and each launch then
// lasts about one wavefront's dependent chain.  In the latency mode a strip
// of a 1D Euler grid gets a workgroup of three wavefronts: wavefront k
// interpolates characteristic field k (conserved component k when not
// characteristic-wise) at the strip's 64 midpoints; the interpolated values
// meet in LDS; wavefront 0 forms the back-projection and the midpoint flux
// while wavefront 1 forms the node flux; wavefront 0 finishes the MND
// difference, the stage update, the non-physical check and the CFL speed.
// Each value is formed by the operations of the one-wavefront kernel in the
// same order, so the results are the same bits.
constexpr int SPLIT_WAVES = 3;
// Strips up to which single 1D Euler solves use it (three wavefronts per
// strip on the 1024 SIMDs of the chip).
constexpr int SPLIT_STRIPS = 256;

template <int FLUX, int SCHEME, bool CHAR, bool GB>
__device__ __forceinline__ void strip1d_split(const double* __restrict__ U, const double* __restrict__ Un,
                                              double* __restrict__ out, Ctrl* __restrict__ ctrl, const Params& P,
                                              const StageArgs& A, int bx)
{
    constexpr int NV = 3;
    const int wave = (int)threadIdx.x / WAVE;
    const int lane = (int)threadIdx.x & (WAVE - 1);
    const int nx = P.nx;
    const Strip1D<DIFF_MND> S(bx, lane, nx);
    __shared__ double sW[NV][2][WAVE];
    __shared__ double sF[NV][WAVE];
    __shared__ double sN[NV][WAVE];
    __shared__ double s_dt;
    __shared__ long long s_step;
    __shared__ unsigned long long s_seen;
    __shared__ int s_go;

    double s[6][NV], un[NV];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        const int col = ghost_map(S.jxl - 2 + m, nx, P.bc_x);
#pragma unroll
        for (int v = 0; v < NV; ++v) s[m][v] = U[(size_t)v * nx + col];
    }
    if (GB && P.bc_x >= BC_REFLECT) {
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            const int kind = ghost_kind(S.jxl - 2 + m, nx, P.bc_x);
#pragma unroll
            for (int v = 0; v < NV; ++v) s[m][v] = ghost_value(kind, v, 1, s[m][v], P.fixed_x);
        }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) un[v] = wave == 0 && A.stage && S.cell_ok ? Un[(size_t)v * nx + S.c] : 0.0;
    // the step record, read once for the workgroup
    if (threadIdx.x == 0) {
        double dt = 0.0;
        long long step = 0;
        unsigned long long seen = 0ull;
        s_go = stage_prologue(ctrl, A, dt, step, bx == 0, seen) ? 1 : 0;
        s_dt = dt;
        s_step = step;
        s_seen = seen;
    }
    init_weight_table();  // (its barrier also publishes the record)
    if (!s_go) return;    // one value for the whole workgroup

    RegStencil<NV> st{s};
    Eigen<NV> E;
    {
        double wl, wr;
        unsigned mL, mR;
        if constexpr (CHAR) {
            midpoint_eigen<NV>(st, P, E);
            double w[6];
            if (wave == 0) project_field<NV>(st, E, 0, w);
            else if (wave == 1) project_field<NV>(st, E, 1, w);
            else project_field<NV>(st, E, 2, w);
            interp_pair<SCHEME>(w[0], w[1], w[2], w[3], w[4], w[5], P, wl, wr, mL, mR);
        } else if (wave == 0) {
            interp_pair<SCHEME>(s[0][0], s[1][0], s[2][0], s[3][0], s[4][0], s[5][0], P, wl, wr, mL, mR);
        } else if (wave == 1) {
            interp_pair<SCHEME>(s[0][1], s[1][1], s[2][1], s[3][1], s[4][1], s[5][1], P, wl, wr, mL, mR);
        } else {
            interp_pair<SCHEME>(s[0][2], s[1][2], s[2][2], s[3][2], s[4][2], s[5][2], P, wl, wr, mL, mR);
        }
        sW[wave][0][lane] = wl;
        sW[wave][1][lane] = wr;
    }
    __syncthreads();
    if (wave == 0) {
        double UL[NV], UR[NV], F[NV];
        if constexpr (CHAR) {
#pragma unroll
            for (int k = 0; k < NV; ++k) back_project_field<NV>(E, k, sW[k][0][lane], sW[k][1][lane], UL, UR);
        } else {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                UL[v] = sW[v][0][lane];
                UR[v] = sW[v][1][lane];
            }
        }
        euler_num_flux<NV, FLUX>(UL, UR, P.gamma, F);
#pragma unroll
        for (int v = 0; v < NV; ++v) sF[v][lane] = F[v];
    } else if (wave == 1) {
        double fn[NV];
        node_flux<SYS_EULER, NV>(s[3], P, fn);
#pragma unroll
        for (int v = 0; v < NV; ++v) sN[v][lane] = fn[v];
    }
    __syncthreads();
    if (wave != 0) return;
    unsigned long long sm = 0ull;
    if (S.cell_ok) {
        double R[NV], o[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v)
            R[v] = mnd(P.c1x, P.c2x, P.c3x, sF[v][lane], sF[v][lane + 1], sF[v][lane + 2], sF[v][lane + 3],
                       sN[v][lane], sN[v][lane + 2]);
        rk_combine<NV>(A.stage, s_dt, s[4], un, R, o);
#pragma unroll
        for (int v = 0; v < NV; ++v) out[(size_t)v * nx + S.c] = o[v];
        stage_epilogue<SYS_EULER, NV>(ctrl, P, A.stage, s_step, S.c, o, sm);
    }
    if (A.stage == 2) flush_speed(ctrl, A.parity, sm, s_seen);
}

template <int FLUX, int SCHEME, bool CHAR, bool GB>
__global__ void __launch_bounds__(WAVE * SPLIT_WAVES)
sweep1d_split(const double* __restrict__ U, const double* __restrict__ Un, double* __restrict__ out,
              Ctrl* __restrict__ ctrl, Params P, StageArgs A)
{
    strip1d_split<FLUX, SCHEME, CHAR, GB>(U, Un, out, ctrl, P, A, (int)blockIdx.x);
}

// The table row of block b: the grid r with blk0[r] <= b < blk0[r+1],
// from the block map when the launch has one (one load), else by binary
// search over the table (uniform per block).
__device__ __forceinline__ ReqGrid load_request(const ReqGrid* __restrict__ reqs, const int* __restrict__ map,
                                                int nreq, int b)
{
    if (map) return load_table_entry(&reqs[load_table_entry(&map[b])]);
    int lo = 0, hi = nreq - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (reqs[mid].blk0 <= b) lo = mid;
        else hi = mid - 1;
    }
    return load_table_entry(&reqs[lo]);
}

// Block map of a ReqGrid table of nreq rows and `total` blocks: block r
// writes map[k] = r for the blocks blk0[r] <= k < blk0[r+1] (total for the
// last row) of grid r, in 1D (strips) and 2D (strips x segments) alike.
__global__ void __launch_bounds__(256) block_map_fill(const ReqGrid* __restrict__ reqs, int nreq, int total,
                                                      int* __restrict__ map)
{
    const int r = (int)blockIdx.x;
    const int b0 = reqs[r].blk0, b1 = r + 1 < nreq ? reqs[r + 1].blk0 : total;
    for (int k = b0 + (int)threadIdx.x; k < b1; k += (int)blockDim.x) map[k] = r;
}

__device__ __forceinline__ StageArgs request_stage(const ReqGrid& R, int stage, int tick_step)
{
    StageArgs A;
    A.t_final = R.t_final;
    A.cfl = R.cfl;
    A.fixed_dt = 0.0;
    A.stage = stage;
    A.parity = (R.parity0 + tick_step) & 1;
    return A;
}

// One stage of many independent 1D Euler grids in one launch (one strip per
// block), each with its own parameters, buffers, control block and parity.
template <int FLUX, int SCHEME, bool CHAR, bool GB>
__global__ void __launch_bounds__(WAVE)
sweep1d_multi(const ReqGrid* __restrict__ reqs, const int* __restrict__ map, int nreq, int stage, int tick_step)
{
    // the strips of one XCD are one contiguous run of the table's strips
    const int b = xcd_order((int)blockIdx.x, 0, (int)gridDim.x);
    ReqGrid R = load_request(reqs, map, nreq, b);
    // every field the strip geometry and the stencil loads need, loaded in
    // one round trip before any of them is used
    asm volatile("" : "+s"(R.U), "+s"(R.U1), "+s"(R.U2), "+s"(R.ctrl), "+s"(R.P.nx), "+s"(R.P.bc_x), "+s"(R.blk0));
    const StageArgs A = request_stage(R, stage, tick_step);
    const double* in = stage == 0 ? R.U : (stage == 1 ? R.U1 : R.U2);
    double* out = stage == 0 ? R.U1 : (stage == 1 ? R.U2 : R.U);
    sweep1d_block<SYS_EULER, 3, FLUX, SCHEME, CHAR, MODE_STAGE, DIFF_MND, GB>(in, R.U, out, nullptr, R.ctrl, R.P, A,
                                                                         b - R.blk0);
}

// ------------------------------------------- persistent batched 1D solves

// One launch runs a set of 1D Euler grids to completion (t_final, a
// non-physical state, or a step budget) with no kernel boundary between
// stages: workgroup b owns grids b*I .. b*I+I-1 of its table, keeps their
// step control (t, dt, step, CFL speed, status) in LDS, and its W waves
// share the strips of every stage, ordered by workgroup barriers only (no
// wave waits for another workgroup).  Every strip runs the single-solve
// arithmetic (face flux, node flux, MND difference, Runge-Kutta combine,
// non-physical check, CFL speed) with the grid's own dt, and the step rule
// of stage_prologue (clipped dt, stop within 1e-12 t_final, the next record
// opened at stage 0), so each grid gives the same bits as alone.
// 8 wavefronts (2 per SIMD) leave the kernel the registers it needs: at 16
// (4 per SIMD, 128 registers) it spilled 292 bytes per lane and ran 2x slower.
constexpr int PERSIST_MAX_WAVES = 8;
constexpr int PERSIST_MAX_GRIDS = 8;

// Orders the LDS writes of a wave before reads of them by other lanes of
// the same wave.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ unsigned long long wave_min_bits(unsigned long long m)
{
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(m, off);
        m = o < m ? o : m;
    }
    return m;
}

// Strip bx of one stage of a 1D Euler grid with the given dt: writes the
// stage output of the strip's cells and returns, per lane, the key of a
// non-physical output (~0 if none) and (stage 2) the CFL speed bits.
template <int FLUX, int SCHEME, bool CHAR, bool GB>
__device__ __forceinline__ void strip1d_stage(const double* __restrict__ U, const double* __restrict__ Un,
                                              double* __restrict__ out, const Params& P, int stage, double dt,
                                              long long step, int bx, double (*sF)[WAVE], double (*sN)[WAVE],
                                              unsigned long long& bad, unsigned long long& speed)
{
    constexpr int NV = 3;
    const int nx = P.nx;
    const int lane = (int)threadIdx.x & (WAVE - 1);
    const Strip1D<DIFF_MND> S(bx, lane, nx);
    double s[6][NV], un[NV];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        const int col = ghost_map(S.jxl - 2 + m, nx, P.bc_x);
#pragma unroll
        for (int v = 0; v < NV; ++v) s[m][v] = U[(size_t)v * nx + col];
    }
    if (GB && P.bc_x >= BC_REFLECT) {
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            const int kind = ghost_kind(S.jxl - 2 + m, nx, P.bc_x);
#pragma unroll
            for (int v = 0; v < NV; ++v) s[m][v] = ghost_value(kind, v, 1, s[m][v], P.fixed_x);
        }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) un[v] = stage && S.cell_ok ? Un[(size_t)v * nx + S.c] : 0.0;
    double F[NV], fn[NV];
    unsigned fb;
    RegStencil<NV> st{s};
    face_flux<SYS_EULER, NV, FLUX, SCHEME, CHAR>(st, P, F, fb);
    node_flux<SYS_EULER, NV>(s[3], P, fn);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        sF[v][lane] = F[v];
        sN[v][lane] = fn[v];
    }
    wave_sync();
    bad = ~0ull;
    speed = 0ull;
    if (S.cell_ok) {
        double R[NV], o[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v)
            R[v] = mnd(P.c1x, P.c2x, P.c3x, sF[v][lane], sF[v][lane + 1], sF[v][lane + 2], sF[v][lane + 3],
                       sN[v][lane], sN[v][lane + 2]);
        rk_combine<NV>(stage, dt, s[4], un, R, o);
#pragma unroll
        for (int v = 0; v < NV; ++v) out[(size_t)v * nx + S.c] = o[v];
        if (cell_bad<SYS_EULER, NV>(o, P))
            bad = ((unsigned long long)(step * 3 + stage) << 36) | (unsigned long long)S.c;
        if (stage == 2) speed = (unsigned long long)__double_as_longlong(cell_speed<SYS_EULER, NV>(o, P));
    }
    // the strip's fluxes are read; the wave's next strip may overwrite them
    wave_sync();
}

template <int FLUX, int SCHEME, bool CHAR, bool GB>
__global__ void __launch_bounds__(WAVE * PERSIST_MAX_WAVES)
sweep1d_persist(const ReqGrid* __restrict__ reqs, int nreq, int per_group, long long max_steps)
{
    constexpr int MG = PERSIST_MAX_GRIDS;
    const int W = (int)blockDim.x / WAVE;
    const int wave = (int)threadIdx.x / WAVE;
    const int lane = (int)threadIdx.x & (WAVE - 1);
    const int q0 = (int)blockIdx.x * per_group;
    const int nq = min(per_group, nreq - q0);
    __shared__ double sF_all[PERSIST_MAX_WAVES][3][WAVE];
    __shared__ double sN_all[PERSIST_MAX_WAVES][3][WAVE];
    __shared__ ReqGrid g_req[MG];
    __shared__ double g_t[MG], g_dt[MG], g_tn[MG];
    __shared__ unsigned long long g_smax[MG], g_next[MG], g_bad[MG];
    __shared__ long long g_step[MG];
    __shared__ int g_status[MG], g_done[MG], g_active[MG], g_opened[MG], g_parity[MG], g_touched[MG];
    __shared__ int g_any;
    init_weight_table();
    if (threadIdx.x == 0) {
        for (int q = 0; q < nq; ++q) {
            const ReqGrid R = load_table_entry(&reqs[q0 + q]);
            g_req[q] = R;
            const Ctrl* c = R.ctrl;
            // the record of the current state is the newest one (a grid
            // that finished inside the last ticks stopped flipping parity)
            const int p = c->rec[0].step >= c->rec[1].step ? 0 : 1;
            g_parity[q] = p;
            g_t[q] = c->rec[p].t;
            g_step[q] = c->rec[p].step;
            g_smax[q] = c->rec[p].smax_bits;
            g_status[q] = c->status;
            g_done[q] = c->done;
            g_bad[q] = c->bad_key;
            g_opened[q] = 0;
            g_touched[q] = 0;
            g_dt[q] = 0.0;
        }
    }
    __syncthreads();
    for (long long it = 0; it < max_steps; ++it) {
        // stage 0 prologue of every grid (stage_prologue's rule)
        if (threadIdx.x == 0) {
            int any = 0;
            for (int q = 0; q < nq; ++q) {
                int act = g_status[q] == 0 && g_done[q] == 0;
                const double tf = g_req[q].t_final;
                if (act && isfinite(tf) && tf - g_t[q] <= 1e-12 * tf) {
                    g_done[q] = 1;
                    g_touched[q] = 1;
                    act = 0;
                }
                double dt = 0.0;
                if (act) {
                    dt = g_req[q].cfl / __longlong_as_double((long long)g_smax[q]);
                    if (isfinite(tf) && dt > tf - g_t[q]) dt = tf - g_t[q];
                    // a step that cannot advance t (an infinite CFL speed)
                    // leaves the grid unfinished instead of looping; a NaN
                    // dt runs the stage, which reports the state as the
                    // stage launches do
                    if (dt == 0.0) act = 0;
                }
                if (act) {
                    g_touched[q] = 1;
                    g_dt[q] = dt;
                    g_tn[q] = g_t[q] + dt;
                    g_next[q] = 0ull;
                    g_opened[q] = 1;
                }
                g_active[q] = act;
                any |= act;
            }
            g_any = any;
        }
        __syncthreads();
        if (!g_any) break;
        for (int stage = 0; stage < 3; ++stage) {
            int total = 0;
            for (int q = 0; q < nq; ++q) total += g_active[q] ? g_req[q].nstrips : 0;
            for (int task = wave; task < total; task += W) {
                int q = 0, bx = task;
                while (!g_active[q] || bx >= g_req[q].nstrips) {
                    if (g_active[q]) bx -= g_req[q].nstrips;
                    ++q;
                }
                const ReqGrid& R = g_req[q];
                const double* in = stage == 0 ? R.U : (stage == 1 ? R.U1 : R.U2);
                double* out = stage == 0 ? R.U1 : (stage == 1 ? R.U2 : R.U);
                unsigned long long bad, speed;
                strip1d_stage<FLUX, SCHEME, CHAR, GB>(in, R.U, out, R.P, stage, g_dt[q], g_step[q], bx,
                                                      sF_all[wave], sN_all[wave], bad, speed);
                bad = wave_min_bits(bad);
                speed = wave_max_bits(speed);
                if (lane == 0) {
                    if (bad != ~0ull) atomicMin(&g_bad[q], bad);
                    if (stage == 2) atomicMax(&g_next[q], speed);
                }
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                for (int q = 0; q < nq; ++q)
                    if (g_active[q] && g_bad[q] != ~0ull) {
                        g_status[q] = (int)WCNST_E_NONPHYSICAL;
                        g_active[q] = 0;
                    }
            }
            __syncthreads();
        }
        // a completed step: its new state is current
        if (threadIdx.x == 0) {
            for (int q = 0; q < nq; ++q)
                if (g_active[q]) {
                    g_t[q] = g_tn[q];
                    g_step[q] = g_step[q] + 1;
                    g_smax[q] = g_next[q];
                    g_parity[q] ^= 1;
                    g_opened[q] = 0;
                }
        }
        __syncthreads();
    }
    // control blocks in the layout the stage launches leave: the record of
    // the current state (and the one a failed step had opened) is the
    // newest; grids this launch neither advanced nor finished keep theirs
    if (threadIdx.x == 0) {
        for (int q = 0; q < nq; ++q) {
            if (!g_touched[q]) continue;
            Ctrl* c = g_req[q].ctrl;
            const int p = g_parity[q];
            c->status = g_status[q];
            c->done = g_done[q];
            c->bad_key = g_bad[q];
            c->rec[p].t = g_t[q];
            c->rec[p].step = g_step[q];
            c->rec[p].smax_bits = g_smax[q];
            c->rec[p].dt = g_opened[q] ? g_dt[q] : 0.0;
            if (g_opened[q]) {
                c->rec[p ^ 1].t = g_tn[q];
                c->rec[p ^ 1].dt = 0.0;
                c->rec[p ^ 1].step = g_step[q] + 1;
                c->rec[p ^ 1].smax_bits = g_next[q];
            } else {
                c->rec[p ^ 1].step = g_step[q] - 1;
            }
        }
    }
}

// ------------------------------------------------------------------ 2D

// Width of a staged row: columns x0-4 .. x0+64 cover the x-stencils of the
// 64 midpoints and the y-stencils of the 64 lanes.
constexpr int XW = WAVE + 5;
constexpr int NSLOT = 6;  // rows j-2 .. j+3 around y-midpoint j

template <int NV>
__device__ __forceinline__ void load_row(const double* __restrict__ U, size_t plane, size_t rowoff,
                                         int colA, int colB, bool hasB, double (&ra)[NV], double (&rb)[NV])
{
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        ra[v] = U[(size_t)v * plane + rowoff + colA];
        rb[v] = hasB ? U[(size_t)v * plane + rowoff + colB] : 0.0;
    }
}

// Ghosts of a staged row: the row's own kind (y boundary, uniform) and each
// lane's column kinds (x boundary).  Periodic and zero-gradient sides are
// pure index remaps and skip this.
template <int NV>
__device__ __forceinline__ void fix_row(const Params& P, int ky, int kA, int kB, double (&ra)[NV], double (&rb)[NV])
{
    if (ky != GH_COPY) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            ra[v] = ghost_value(ky, v, 2, ra[v], P.fixed_y);
            rb[v] = ghost_value(ky, v, 2, rb[v], P.fixed_y);
        }
    }
    if (P.bc_x >= BC_REFLECT) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            ra[v] = ghost_value(kA, v, 1, ra[v], P.fixed_x);
            rb[v] = ghost_value(kB, v, 1, rb[v], P.fixed_x);
        }
    }
}

template <int NV>
__device__ __forceinline__ void store_row(double (*slot)[XW], int lane, bool hasB, const double (&ra)[NV],
                                          const double (&rb)[NV])
{
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        slot[v][lane] = ra[v];
        if (hasB) slot[v][WAVE + lane] = rb[v];
    }
}

// Adaptive rows of the first-height segments of a balanced 2D stage launch
// (the older wavefront of each SIMD pair runs at its lone speed, so its
// segment's cost sets when the SIMD is done; where the stencil-cut test
// runs in full, near discontinuities, a segment of equal rows costs more).
// In a launch of parity p (alternating, set by the host), strip s's
// first-height segment i takes rows [tab[p][s][i], tab[p][s][i+1]).  Each
// such wavefront records what it took in cost[p]; the first wavefront of
// the launch to finish re-plans tab[1-p] (the previous launch's layout)
// from cost[1-p] (the previous launch's durations) for the next launch.
// So no launch reads a table that it or a running launch writes, and every
// table is a partition of the rows (plan_strip keeps it one).  The layout
// moves only work between wavefronts: every cell's arithmetic, and so
// every result, is the same.  The block sits in the padding after the
// solver's control block (no kernel argument holds registers through the
// sweep); on == 0 there: fixed heights.
struct SegCtl {
    int* tab[2];        // [strips][nseg1 + 1] boundaries
    unsigned* cost[2];  // [strips][nseg1] durations (10 ns ticks)
    unsigned* ctr;      // wavefronts of the running launch that have finished (0 between launches)
    int minr;           // fewest rows of a segment
    int on;
};
constexpr size_t SEGCTL_OFFSET = 128;
static_assert(sizeof(Ctrl) <= SEGCTL_OFFSET && SEGCTL_OFFSET + sizeof(SegCtl) <= 256,
              "the layout block must fit the control block's 256-byte slot");

__host__ __device__ inline SegCtl* seg_ctl_of(Ctrl* ctrl)
{
    return reinterpret_cast<SegCtl*>(reinterpret_cast<char*>(ctrl) + SEGCTL_OFFSET);
}

// Records the duration of first-height segment cost_idx (-1: a
// second-height one), counts the wavefront, and, in the launch's first
// finisher, plans
// every strip of the next launch, staging each strip's boundaries and
// durations in LDS the wavefront no longer needs (lds: strips * (2 nseg1 +
// 1) ints, checked by the host).  The launch's last finisher clears the
// count (as does the start of every solve call).
__device__ __forceinline__ void seg_finish(SegCtl* __restrict__ seg, int par, int cost_idx, unsigned ticks, int nseg1,
                                           int* lds)
{
    const int ns = (int)gridDim.x, total = (int)(gridDim.x * gridDim.y);
    unsigned old = 0u;
    if (threadIdx.x == 0) {
        if (cost_idx >= 0) seg->cost[par][cost_idx] = ticks > 0u ? ticks : 1u;
        old = __hip_atomic_fetch_add(seg->ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // the last to finish: every wavefront has counted
        if (old == (unsigned)total - 1u) __hip_atomic_store(seg->ctr, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    old = __shfl(old, 0);
    if (old != 0u) return;
    const int n = nseg1;
    int* tab = seg->tab[par ^ 1];
    const unsigned* cost = seg->cost[par ^ 1];
    for (int st = (int)threadIdx.x; st < ns; st += WAVE) {
        int* b = lds + (size_t)st * (2 * n + 1);
        unsigned* d = reinterpret_cast<unsigned*>(b + n + 1);
        for (int i = 0; i <= n; ++i) b[i] = tab[(size_t)st * (n + 1) + i];
        for (int i = 0; i < n; ++i) d[i] = cost[(size_t)st * n + i];
        plan_strip(b, d, n, seg->minr, tab + (size_t)st * (n + 1));
    }
}

// One segment (strip bx, rows by*ty ..) of one 2D grid.  Thread 0 of
// segment (0, 0) opens the next step record.
// GB: general boundaries (reflecting walls, fixed ends, gravity); without
// it only index-remap sides (periodic, zero gradient) and no source.
template <int NV, int FLUX, int SCHEME, bool CHAR, int MODE, bool GB, bool ADAPT>
__device__ __forceinline__ void sweep2d_block(const double* __restrict__ U, const double* __restrict__ Un,
                                              double* __restrict__ out, uint8_t* __restrict__ flags,
                                              Ctrl* __restrict__ ctrl, const Params& P, const StageArgs& A,
                                              int ty, int ty2, int nseg1, int bx, int by, int seg_par)
{
    // segment by of the strip: segments 0 .. nseg1-1 hold ty rows each, the
    // later ones ty2 (ty2 == ty: one height; cut flags need one height)
    static_assert(NV == 4, "2D sweeps carry the four Euler variables");
    double dt = 0.0;
    long long step = 0;
    unsigned long long seen = 0ull;
    if constexpr (MODE == MODE_STAGE) {
        if (!stage_prologue(ctrl, A, dt, step, bx == 0 && by == 0 && threadIdx.x == 0, seen)) return;
    }
    // Ring of staged rows (all variables, XW columns) and the x-midpoint /
    // x node fluxes of the current row.
    __shared__ double ring[NSLOT][NV][XW];
    __shared__ double sF[NV][WAVE];
    __shared__ double sN[NV][WAVE];
    init_weight_table();
    const int nx = P.nx, ny = P.ny;
    const size_t plane = (size_t)nx * ny;
    const int lane = threadIdx.x;
    const int x0 = bx * TX;
    int y0 = by < nseg1 ? by * ty : nseg1 * ty + (by - nseg1) * ty2;
    int y1 = y0 + (by < nseg1 ? ty : ty2);
    // the segment's duration slot and start time wait in LDS (kept out of
    // registers through the sweep)
    __shared__ int seg_slot, seg_p;
    __shared__ unsigned seg_t0;
    if constexpr (MODE == MODE_STAGE && ADAPT) {
        SegCtl* seg = seg_ctl_of(ctrl);
        int slot = -1;
        // plain loads of values no wave changes during the launch, kept
        // uniform (scalar) so that the sweep's row bounds stay scalar
        if (by < nseg1 && __builtin_amdgcn_readfirstlane(seg->on)) {
            const int* lrow = seg->tab[seg_par] + (size_t)bx * (nseg1 + 1) + by;
            y0 = __builtin_amdgcn_readfirstlane(lrow[0]);
            y1 = __builtin_amdgcn_readfirstlane(lrow[1]);
            slot = bx * nseg1 + by;
        }
        if (threadIdx.x == 0) {
            seg_slot = slot;
            seg_p = seg_par;
            seg_t0 = (unsigned)__builtin_amdgcn_s_memrealtime();
        }
    }
    y1 = min(y1, ny);
    const int c = x0 + lane;
    const bool cell_ok = lane < TX && c < nx;
    const int jx = x0 - 2 + lane;
    // cut flags are reported by right-hand-side launches only
    const bool own_x = MODE == MODE_RHS && flags && jx <= nx && face_owner(jx, nx, TX) == bx;
    // columns this lane stages (ghost cells by index remap, any distance)
    const bool hasB = lane < XW - WAVE;
    const int colA = ghost_map_any(x0 - 4 + lane, nx, P.bc_x);
    const int colB = ghost_map_any(x0 - 4 + WAVE + lane, nx, P.bc_x);
    const int kA = GB ? ghost_kind(x0 - 4 + lane, nx, P.bc_x) : GH_COPY;
    const int kB = GB ? ghost_kind(x0 - 4 + WAVE + lane, nx, P.bc_x) : GH_COPY;

    // y-midpoint fluxes j-3 .. j of this lane's column, in y-normal
    // variable order (rho, rho v, rho u, E)
    double fy[4][NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) fy[0][v] = fy[1][v] = fy[2][v] = fy[3][v] = 0.0;
    unsigned long long smax_loc = 0ull;

    // stage rows y0-4 .. y0+1 into slots 0 .. 5
#pragma unroll 1
    for (int k = 0; k < NSLOT; ++k) {
        double ra[NV], rb[NV];
        const size_t rowoff = (size_t)ghost_map(y0 - 4 + k, ny, P.bc_y) * nx;
        load_row<NV>(U, plane, rowoff, colA, colB, hasB, ra, rb);
        if constexpr (GB) fix_row<NV>(P, ghost_kind(y0 - 4 + k, ny, P.bc_y), kA, kB, ra, rb);
        store_row<NV>(ring[k], lane, hasB, ra, rb);
    }
    __syncthreads();

    int base = 0;  // slot of row j-2
    for (int j = y0 - 2; j <= y1; ++j) {
        const int i = j - 1;  // row finished once y-midpoint j is known
        const int npass = i >= y0 ? 2 : 1;
        // last pass: y-midpoint (c, j+1/2) from rows j-2 .. j+3 at this
        // lane's column (normal momentum = rho v first); first pass (rows
        // i >= y0): x-midpoint (jx+1/2, i) from row i.  Both passes run the
        // same instructions on different staged data (selects, no branches),
        // so they share one set of registers; the y flux is the one left in
        // F when the loop ends.
        double F[NV];
#pragma unroll 1
        for (int pass = 0; pass < npass; ++pass) {
            const bool py = pass == npass - 1;
            // the six stencil nodes, read once into registers: node m at
            // ring[slot][var][col] with (slot, col) = (row j-2+m, c) in the
            // y pass and (row i, jx-2+m) in the x pass
            const double* rb = &ring[0][0][0];
            const int slx = base + 1 < NSLOT ? base + 1 : base + 1 - NSLOT;
            const int vs1 = py ? 2 * XW : XW, vs2 = py ? XW : 2 * XW;
            double s[6][NV];
#pragma unroll
            for (int m = 0; m < 6; ++m) {
                const int sl = base + m < NSLOT ? base + m : base + m - NSLOT;
                const int off = py ? sl * NV * XW + lane + 4 : slx * NV * XW + lane + m;
                s[m][0] = rb[off];
                s[m][1] = rb[off + vs1];
                s[m][2] = rb[off + vs2];
                s[m][3] = rb[off + 3 * XW];
            }
            RegStencil<NV> st{s};
            unsigned fb;
            face_flux<SYS_EULER, NV, FLUX, SCHEME, CHAR>(st, P, F, fb);
            if (MODE == MODE_RHS && flags) {
                if (py) {
                    if (cell_ok && j <= ny && face_owner(j, ny, ty) == by)
                        write_flags<NV>(flags + (size_t)NV * ny * (nx + 3) * 2, nx, ny + 3, c, j + 2, fb);
                } else if (own_x) {
                    write_flags<NV>(flags, ny, nx + 3, i, jx + 2, fb);
                }
            }
            if (!py) {
                // x node flux at node jx+1 of row i
                double sn[NV], fn[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) sn[v] = s[3][v];
                node_flux<SYS_EULER, NV>(sn, P, fn);
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    sF[v][lane] = F[v];
                    sN[v][lane] = fn[v];
                }
            }
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            fy[0][v] = fy[1][v];
            fy[1][v] = fy[2][v];
            fy[2][v] = fy[3][v];
            fy[3][v] = F[v];
        }
        __syncthreads();
        // U^n of row i first, then row j+4, which travels while row i is
        // finished (it replaces row j-2 = i-1, which the difference below
        // still reads): the wait for U^n leaves row j+4 in flight
        double un[NV];
        {
            const size_t cell = (size_t)(i < 0 ? 0 : i) * nx + (cell_ok ? c : 0);
#pragma unroll
            for (int v = 0; v < NV; ++v)
                un[v] = MODE == MODE_STAGE && A.stage && npass == 2 && cell_ok ? Un[(size_t)v * plane + cell] : 0.0;
        }
        double ra[NV], rb[NV];
        if (j < y1) load_row<NV>(U, plane, (size_t)ghost_map(j + 4, ny, P.bc_y) * nx, colA, colB, hasB, ra, rb);
        if (npass == 2 && cell_ok) {
            // rows i-1, i, i+1 of this lane's column are still staged
            const int s_im = base;                                  // row j-2 = i-1
            const int s_i = base + 1 < NSLOT ? base + 1 : base + 1 - NSLOT;  // row i
            const int s_ip = base + 2 < NSLOT ? base + 2 : base + 2 - NSLOT; // row i+1
            double um[NV], up[NV], Uc[NV], gm[NV], gp[NV];
            um[0] = ring[s_im][0][lane + 4]; um[1] = ring[s_im][2][lane + 4];
            um[2] = ring[s_im][1][lane + 4]; um[3] = ring[s_im][3][lane + 4];
            up[0] = ring[s_ip][0][lane + 4]; up[1] = ring[s_ip][2][lane + 4];
            up[2] = ring[s_ip][1][lane + 4]; up[3] = ring[s_ip][3][lane + 4];
            node_flux<SYS_EULER, NV>(um, P, gm);
            node_flux<SYS_EULER, NV>(up, P, gp);
            double Rx[NV], Ry[NV], R[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                Uc[v] = ring[s_i][v][lane + 4];
                Rx[v] = mnd(P.c1x, P.c2x, P.c3x, sF[v][lane], sF[v][lane + 1], sF[v][lane + 2],
                            sF[v][lane + 3], sN[v][lane], sN[v][lane + 2]);
                Ry[v] = mnd(P.c1y, P.c2y, P.c3y, fy[0][v], fy[1][v], fy[2][v], fy[3][v], gm[v], gp[v]);
            }
            R[0] = Rx[0] + Ry[0];
            R[1] = Rx[1] + Ry[2];
            R[2] = Rx[2] + Ry[1];
            R[3] = Rx[3] + Ry[3];
            if (GB && P.gravity != 0.0) {
                // body force in +y on the momentum and energy equations
                R[2] = R[2] + Uc[0] * P.gravity;
                R[3] = R[3] + Uc[2] * P.gravity;
            }
            const size_t cell = (size_t)i * nx + c;
            if constexpr (MODE == MODE_RHS) {
#pragma unroll
                for (int v = 0; v < NV; ++v) out[(size_t)v * plane + cell] = R[v];
            } else {
                double o[NV];
                rk_combine<NV>(A.stage, dt, Uc, un, R, o);
#pragma unroll
                for (int v = 0; v < NV; ++v) out[(size_t)v * plane + cell] = o[v];
                stage_epilogue<SYS_EULER, NV>(ctrl, P, A.stage, step, (long long)cell, o, smax_loc);
            }
        }
        __syncthreads();
        // row j-2 is no longer read: its slot takes row j+4
        if (j < y1) {
            if constexpr (GB) fix_row<NV>(P, ghost_kind(j + 4, ny, P.bc_y), kA, kB, ra, rb);
            store_row<NV>(ring[base], lane, hasB, ra, rb);
        }
        base = base + 1 < NSLOT ? base + 1 : 0;
        __syncthreads();
    }
    if constexpr (MODE == MODE_STAGE) {
        if (A.stage == 2) flush_speed(ctrl, A.parity, smax_loc, seen);
        if constexpr (ADAPT) {
            SegCtl* seg = seg_ctl_of(ctrl);
            if (__builtin_amdgcn_readfirstlane(seg->on))
                seg_finish(seg, seg_p, seg_slot, (unsigned)__builtin_amdgcn_s_memrealtime() - seg_t0, nseg1,
                           reinterpret_cast<int*>(&ring[0][0][0]));
        }
    }
}

// Two wavefronts per SIMD: the register budget is capped at 256 (a few
// values spill); measured faster than one wavefront with no spills.
template <int NV, int FLUX, int SCHEME, bool CHAR, int MODE, bool GB>
__global__ void __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(2, 2)))
sweep2d(const double* __restrict__ U, const double* __restrict__ Un, double* __restrict__ out,
        uint8_t* __restrict__ flags, Ctrl* __restrict__ ctrl, Params P, StageArgs A, int ty, int ty2, int nseg1,
        int seg_par)
{
    // Segments in strip-fastest order, each height group in its own XCD
    // runs: the strips on either side of a strip, which stage the same halo
    // columns and the same partly used 128-byte lines of every row, read
    // them through the same L2 at about the same time.
    const int ns = (int)gridDim.x;
    const int L = (int)blockIdx.x + ns * (int)blockIdx.y;
    const int n1 = ns * nseg1;
    const int w = L < n1 ? xcd_order(L, 0, n1) : xcd_order(L, n1, ns * (int)gridDim.y - n1);
    sweep2d_block<NV, FLUX, SCHEME, CHAR, MODE, GB, true>(U, Un, out, flags, ctrl, P, A, ty, ty2, nseg1, w % ns,
                                                      w / ns, seg_par);
}

// One stage of many independent 2D grids in one launch: block b belongs to
// the request r with blk0[r] <= b < blk0[r+1] (from the block map, else by
// a search over the table, uniform per block), then runs segment
// b - blk0[r] of that grid with the grid's own parameters, buffers, control
// block and step parity.
template <int NV, int FLUX, int SCHEME, bool CHAR, bool GB>
__global__ void __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(2, 2)))
sweep2d_multi(const ReqGrid* __restrict__ reqs, const int* __restrict__ map, int nreq, int stage, int tick_step,
              int ty)
{
    // the segments of one XCD are one contiguous run of the table's segments
    const int b = xcd_order((int)blockIdx.x, 0, (int)gridDim.x);
    ReqGrid R = load_request(reqs, map, nreq, b);
    // the fields the segment geometry and the first row loads need, loaded
    // in one round trip before any of them is used
    asm volatile("" : "+s"(R.U), "+s"(R.U1), "+s"(R.U2), "+s"(R.ctrl), "+s"(R.P.nx), "+s"(R.P.ny), "+s"(R.blk0),
                 "+s"(R.nstrips));
    const Params& P = R.P;
    const int local = b - R.blk0;
    const StageArgs A = request_stage(R, stage, tick_step);
    const double* in = stage == 0 ? R.U : (stage == 1 ? R.U1 : R.U2);
    double* out = stage == 0 ? R.U1 : (stage == 1 ? R.U2 : R.U);
    // one height: every segment of the grid is of the first kind (an exact
    // count keeps nseg1 * ty within the grid)
    sweep2d_block<NV, FLUX, SCHEME, CHAR, MODE_STAGE, GB, false>(in, R.U, out, nullptr, R.ctrl, P, A, ty, ty,
                                                             (P.ny + ty - 1) / ty, local % R.nstrips,
                                                             local / R.nstrips, 0);
}

// ----------------------------------------------------- control kernels

// Block r: reset the control block of grid r of a ReqGrid table to t = 0
// (as ctrl_init) and accumulate the CFL speed of its state into record 0
// (as wavespeed), for every grid of the table in one launch.
template <int NV>
__global__ void __launch_bounds__(256) multi_init(const ReqGrid* __restrict__ reqs)
{
    const ReqGrid R = load_table_entry(&reqs[blockIdx.x]);
    const size_t plane = (size_t)R.P.nx * R.P.ny;
    unsigned long long m = 0ull;
    for (size_t i = threadIdx.x; i < plane; i += blockDim.x) {
        double u[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) u[v] = R.U[(size_t)v * plane + i];
        const unsigned long long b = (unsigned long long)__double_as_longlong(cell_speed<SYS_EULER, NV>(u, R.P));
        m = b > m ? b : m;
    }
    m = wave_max_bits(m);
    __shared__ unsigned long long red[256 / WAVE];
    if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < (int)(blockDim.x / WAVE); ++i) m = red[i] > m ? red[i] : m;
        Ctrl* ctrl = R.ctrl;
        for (int k = 0; k < 2; ++k) {
            ctrl->rec[k].t = 0.0;
            ctrl->rec[k].dt = 0.0;
            ctrl->rec[k].smax_bits = k == 0 ? m : 0ull;
            ctrl->rec[k].step = 0;
        }
        ctrl->bad_key = ~0ull;
        ctrl->call_step0 = 0;
        ctrl->status = 0;
        ctrl->done = 0;
    }
}

__global__ void ctrl_init(Ctrl* ctrl, double t, long long step)
{
    if (threadIdx.x != 0) return;
    for (int k = 0; k < 2; ++k) {
        ctrl->rec[k].t = t;
        ctrl->rec[k].dt = 0.0;
        ctrl->rec[k].smax_bits = 0ull;
        ctrl->rec[k].step = step;
    }
    ctrl->bad_key = ~0ull;
    ctrl->call_step0 = step;
    ctrl->status = 0;
    ctrl->done = 0;
}

// Opens a solve / step call: clears the done flag and the speed accumulator
// of the current record and remembers the step counter.
__global__ void ctrl_open(Ctrl* ctrl, int parity)
{
    if (threadIdx.x != 0) return;
    ctrl->rec[parity].smax_bits = 0ull;
    ctrl->done = 0;
    ctrl->call_step0 = ctrl->rec[parity].step;
    // a launch that stopped part of its wavefronts early (a non-physical
    // state found during it) leaves the adaptive layout's count behind
    SegCtl* seg = seg_ctl_of(ctrl);
    if (seg->on) *seg->ctr = 0u;
}

template <int SYS, int NV>
__global__ void __launch_bounds__(256) wavespeed(const double* __restrict__ U, Ctrl* ctrl, Params P,
                                                  int parity)
{
    const size_t plane = (size_t)P.nx * P.ny;
    unsigned long long m = 0ull;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < plane;
         i += (size_t)gridDim.x * blockDim.x) {
        double u[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) u[v] = U[(size_t)v * plane + i];
        const unsigned long long b = (unsigned long long)__double_as_longlong(cell_speed<SYS, NV>(u, P));
        m = b > m ? b : m;
    }
    m = wave_max_bits(m);
    if ((threadIdx.x & (WAVE - 1)) == 0) atomicMax(&ctrl->rec[parity].smax_bits, m);
}

}  // namespace wcnst

// ====================================================================== host

using namespace wcnst;

static thread_local char g_err[512] = "";

wcnst_status wcnst_fail(wcnst_status st, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return st;
}
#define fail wcnst_fail

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(WCNST_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));       \
    } while (0)

enum Kind { K_ADV1 = 0, K_BURG1 = 1, K_EUL1 = 2, K_EUL2 = 3 };

struct wcnst_solver {
    wcnst_desc d;
    Params P;
    Kind kind;
    int nv;
    hipStream_t stream;
    Ctrl* ctrl;
    double* U1;
    double* U2;
    Ctrl* host_ctrl[2];  // pinned snapshots for polling
    hipEvent_t snap_ev[2];
    int parity;
    int ty;  // rows per 2D segment
    bool ty_user;  // set by wcnst_set_tuning (else chosen at creation)
    int split_strips;  // 1D Euler stages over at most this many strips run in the latency mode
    int slots;     // wavefront slots of the device
    // adaptive first-height segment rows of balanced 2D stage launches (in
    // the workspace; off where the shape does not take them)
    bool seg_on;
    int seg_n1;             // first-height segments per strip the tables hold
    int* seg_tab;           // two tables of LAYOUT_CAP ints
    unsigned* seg_cost;     // two duration arrays of LAYOUT_CAP
    unsigned* seg_ctr;
    mutable long long seg_launch;  // balanced stage launches so far (their parity selects the tables)
    bool prof;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used;
};

size_t wcnst_align256(size_t b) { return (b + 255) & ~(size_t)255; }
#define align256 wcnst_align256

wcnst_status wcnst_check_desc(const wcnst_desc* d)
{
    if (!d) return fail(WCNST_E_INVALID_ARG, "null descriptor");
    if (d->struct_size != sizeof(wcnst_desc))
        return fail(WCNST_E_INVALID_ARG, "struct_size %u != %zu", d->struct_size, sizeof(wcnst_desc));
    if (d->ndim != 1 && d->ndim != 2) return fail(WCNST_E_INVALID_ARG, "ndim must be 1 or 2");
    if (d->system < WCNST_ADVECTION || d->system > WCNST_EULER)
        return fail(WCNST_E_INVALID_ARG, "unknown system %d", d->system);
    if (d->ndim == 2 && d->system != WCNST_EULER)
        return fail(WCNST_E_INVALID_ARG, "2D grids require the Euler system");
    if (d->nx < 5) return fail(WCNST_E_INVALID_ARG, "nx must be >= 5");
    if (d->ndim == 1 && d->ny != 1) return fail(WCNST_E_INVALID_ARG, "ny must be 1 in 1D");
    if (d->ndim == 2 && d->ny < 5) return fail(WCNST_E_INVALID_ARG, "ny must be >= 5");
    if ((int64_t)d->nx * d->ny > ((int64_t)1 << 34)) return fail(WCNST_E_INVALID_ARG, "grid too large");
    if (!(d->x1 > d->x0) || (d->ndim == 2 && !(d->y1 > d->y0)))
        return fail(WCNST_E_INVALID_ARG, "empty domain");
    for (int b : {d->bc_x, d->bc_y}) {
        if (b != WCNST_PERIODIC && b != WCNST_ZERO_GRADIENT && b != WCNST_REFLECT && b != WCNST_FIXED)
            return fail(WCNST_E_INVALID_ARG, "unknown boundary condition %d", b);
        if (b == WCNST_REFLECT && d->system != WCNST_EULER)
            return fail(WCNST_E_INVALID_ARG, "reflecting walls are for the Euler system");
    }
    if (!std::isfinite(d->gravity)) return fail(WCNST_E_INVALID_ARG, "gravity must be finite");
    if (d->gravity != 0.0 && (d->ndim != 2 || d->system != WCNST_EULER))
        return fail(WCNST_E_INVALID_ARG, "gravity is a 2D Euler source");
    if (d->flux != WCNST_ROE && d->flux != WCNST_LF && d->flux != WCNST_VANLEER)
        return fail(WCNST_E_INVALID_ARG, "unknown flux");
    if (d->flux == WCNST_VANLEER && d->system != WCNST_EULER)
        return fail(WCNST_E_INVALID_ARG, "the van Leer splitting is for the Euler system");
    if (d->scheme < WCNST_TENO || d->scheme > WCNST_Z) return fail(WCNST_E_INVALID_ARG, "unknown scheme");
    if (d->scheme == WCNST_Z) {
        // (tau_5 / 1e-40)^p stays finite for tau_5 < 1e37 with p <= 4
        if (d->z_q < 1 || d->z_q > 4) return fail(WCNST_E_INVALID_ARG, "z_q must be in [1, 4]");
        if (!(d->eps_z > 0.0)) return fail(WCNST_E_INVALID_ARG, "eps_z must be positive");
    }
    if (d->diff != WCNST_MND && d->diff != WCNST_MD && d->diff != WCNST_HWCNS)
        return fail(WCNST_E_INVALID_ARG, "unknown difference");
    if (d->diff != WCNST_MND && d->ndim != 1)
        return fail(WCNST_E_INVALID_ARG, "the MD and HWCNS differences are built for 1D grids");
    if (d->system == WCNST_EULER && !(d->gamma > 1.0)) return fail(WCNST_E_INVALID_ARG, "gamma must be > 1");
    if (d->q < 1 || d->q > 64) return fail(WCNST_E_INVALID_ARG, "q must be in [1, 64]");
    if (!(d->CT > 0.0 && d->CT < 1.0 / 3.0)) return fail(WCNST_E_INVALID_ARG, "C_T must be in (0, 1/3)");
    if (!(d->C > 0.0) || !(d->eps_teno > 0.0) || !(d->eps_js > 0.0))
        return fail(WCNST_E_INVALID_ARG, "C and epsilons must be positive");
    return WCNST_OK;
}

bool wcnst_general_bc(const wcnst_desc* d)
{
    return d->bc_x == WCNST_REFLECT || d->bc_x == WCNST_FIXED || d->bc_y == WCNST_REFLECT ||
           d->bc_y == WCNST_FIXED || d->gravity != 0.0;
}

int wcnst_desc_nvar(const wcnst_desc* d)
{
    return d->system == WCNST_EULER ? (d->ndim == 1 ? 3 : 4) : 1;
}

extern "C" wcnst_status wcnst_desc_init(wcnst_desc* d)
{
    if (!d) return fail(WCNST_E_INVALID_ARG, "null descriptor");
    memset(d, 0, sizeof *d);
    d->struct_size = sizeof(wcnst_desc);
    d->ndim = 1;
    d->system = WCNST_EULER;
    d->nx = 64;
    d->ny = 1;
    d->x0 = 0.0;
    d->x1 = 1.0;
    d->y0 = 0.0;
    d->y1 = 1.0;
    d->bc_x = d->bc_y = WCNST_ZERO_GRADIENT;
    d->flux = WCNST_ROE;
    d->scheme = WCNST_TENO;
    d->diff = WCNST_MND;
    d->charwise = 1;
    d->q = 6;
    d->gamma = 1.4;
    d->adv_speed = 1.0;
    d->CT = 1e-5;
    d->C = 1.0;
    d->eps_teno = 1e-40;
    d->eps_js = 1e-6;
    d->z_q = 1;
    d->eps_z = 1e-40;
    return WCNST_OK;
}

// Entries of one adaptive layout table (and of one duration array).  The
// planner also stages a strip's boundaries and durations in the LDS of the
// 2D stage's row ring: strips * (2 nseg1 + 1) ints, at most LAYOUT_LDS_INTS.
constexpr int LAYOUT_CAP = 2048;
constexpr int LAYOUT_LDS_INTS = (int)(sizeof(double) * NSLOT * 4 * XW / sizeof(int));
static size_t layout_bytes()
{
    return 2 * sizeof(int) * LAYOUT_CAP + 2 * sizeof(unsigned) * LAYOUT_CAP + 256;
}

// Both layout tables at the fixed heights (boundary i of every strip at
// i * ty), no durations yet, counter clear, and the block beside the
// control block that points at them (on = 0: fixed heights, nothing else
// is touched).
__global__ void __launch_bounds__(256) layout_init(Ctrl* ctrl, int on, int* tab, unsigned* cost, unsigned* ctr,
                                                   int ns, int n1, int ty, int minr)
{
    SegCtl* ctl = seg_ctl_of(ctrl);
    if (on) {
        for (int k = (int)threadIdx.x; k < ns * (n1 + 1); k += (int)blockDim.x) {
            const int i = k % (n1 + 1);
            tab[k] = i * ty;
            tab[LAYOUT_CAP + k] = i * ty;
        }
        for (int k = (int)threadIdx.x; k < 2 * LAYOUT_CAP; k += (int)blockDim.x) cost[k] = 0u;
    }
    if (threadIdx.x == 0) {
        if (on) *ctr = 0u;
        ctl->tab[0] = on ? tab : nullptr;
        ctl->tab[1] = on ? tab + LAYOUT_CAP : nullptr;
        ctl->cost[0] = on ? cost : nullptr;
        ctl->cost[1] = on ? cost + LAYOUT_CAP : nullptr;
        ctl->ctr = on ? ctr : nullptr;
        ctl->minr = minr;
        ctl->on = on;
    }
}

extern "C" wcnst_status wcnst_workspace_size(const wcnst_desc* d, size_t* bytes)
{
    wcnst_status st = wcnst_check_desc(d);
    if (st) return st;
    if (!bytes) return fail(WCNST_E_INVALID_ARG, "null size pointer");
    const size_t state = (size_t)wcnst_desc_nvar(d) * d->nx * d->ny * sizeof(double);
    *bytes = align256(sizeof(Ctrl)) + 2 * align256(state) + (d->ndim == 2 ? align256(layout_bytes()) : 0);
    return WCNST_OK;
}

void wcnst_make_params(const wcnst_desc* d, Params* out)
{
    Params P{};
    P.CT = d->CT;
    P.C = d->C;
    P.eps_teno = d->eps_teno;
    P.eps_js = d->eps_js;
    P.gamma = d->gamma;
    P.adv = d->adv_speed;
    P.nx = d->nx;
    P.ny = d->ny;
    P.dx = (d->x1 - d->x0) / d->nx;
    P.dy = d->ndim == 2 ? (d->y1 - d->y0) / d->ny : 1.0;
    // Eq. (5) coefficients (3/2, -3/10, 1/30), or Eq. (3) coefficients
    // (75/64, -25/384, 3/640) for MD, divided by the spacing
    if (d->diff == WCNST_MD) {
        P.c1x = (75.0 / 64.0) / P.dx;
        P.c2x = (-25.0 / 384.0) / P.dx;
        P.c3x = (3.0 / 640.0) / P.dx;
    } else if (d->diff == WCNST_HWCNS) {
        // Eq. (4): (64/45, -2/9, 1/180)
        P.c1x = (64.0 / 45.0) / P.dx;
        P.c2x = (-2.0 / 9.0) / P.dx;
        P.c3x = (1.0 / 180.0) / P.dx;
    } else {
        P.c1x = (3.0 / 2.0) / P.dx;
        P.c2x = (-3.0 / 10.0) / P.dx;
        P.c3x = (1.0 / 30.0) / P.dx;
    }
    P.c1y = (3.0 / 2.0) / P.dy;
    P.c2y = (-3.0 / 10.0) / P.dy;
    P.c3y = (1.0 / 30.0) / P.dy;
    P.q = d->q;
    P.charwise = d->charwise ? 1 : 0;
    P.bc_x = d->bc_x;
    P.bc_y = d->bc_y;
    for (int side = 0; side < 2; ++side)
        for (int v = 0; v < 4; ++v) {
            P.fixed_x[side][v] = d->fixed_x[side][v];
            P.fixed_y[side][v] = d->fixed_y[side][v];
        }
    P.gravity = d->gravity;
    P.z_q = d->z_q;
    P.eps_z = d->eps_z;
    // TENO: tau / min(beta_k + eps) up to which every chi_k stays >= C_T:
    // chi_k >= C^q / (3 (C + t)^q) >= C_T for t <= C ((3 C_T)^(-1/q) - 1);
    // nine tenths of that bound
    P.teno_smooth = 0.9 * d->C * (std::pow(3.0 * d->CT, -1.0 / d->q) - 1.0);
    *out = P;
}

static wcnst_status layout_reset(wcnst_solver* s);

extern "C" wcnst_status wcnst_create(const wcnst_desc* d, void* hip_stream, void* workspace,
                                     size_t ws_bytes, wcnst_solver** out)
{
    wcnst_status st = wcnst_check_desc(d);
    if (st) return st;
    if (!out) return fail(WCNST_E_INVALID_ARG, "null output handle");
    size_t need = 0;
    wcnst_workspace_size(d, &need);
    if (!workspace || ws_bytes < need)
        return fail(WCNST_E_INVALID_ARG, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
    if (((uintptr_t)workspace & 255u) != 0) return fail(WCNST_E_INVALID_ARG, "workspace not 256-byte aligned");

    wcnst_solver* s = new wcnst_solver();
    s->d = *d;
    s->nv = wcnst_desc_nvar(d);
    s->kind = d->system == WCNST_ADVECTION ? K_ADV1
              : d->system == WCNST_BURGERS ? K_BURG1
              : d->ndim == 1               ? K_EUL1
                                           : K_EUL2;
    s->stream = (hipStream_t)hip_stream;
    uint8_t* ws = (uint8_t*)workspace;
    const size_t state = (size_t)s->nv * d->nx * d->ny * sizeof(double);
    s->ctrl = (Ctrl*)ws;
    s->U1 = (double*)(ws + align256(sizeof(Ctrl)));
    s->U2 = (double*)(ws + align256(sizeof(Ctrl)) + align256(state));
    if (d->ndim == 2) {
        uint8_t* lw = ws + align256(sizeof(Ctrl)) + 2 * align256(state);
        s->seg_tab = (int*)lw;
        s->seg_cost = (unsigned*)(lw + 2 * sizeof(int) * LAYOUT_CAP);
        s->seg_ctr = (unsigned*)(lw + 2 * sizeof(int) * LAYOUT_CAP + 2 * sizeof(unsigned) * LAYOUT_CAP);
    }
    s->parity = 0;
    s->slots = wcnst_wave_slots();
    s->ty_user = false;
    s->split_strips = SPLIT_STRIPS;
    {
        const int strips = (d->nx + TX - 1) / TX, rows = d->ny;
        s->ty = d->ndim == 2 ? wcnst_auto_rows(&strips, &rows, 1, s->slots) : 35;
    }
    s->prof = false;
    s->ev_used = 0;

    wcnst_make_params(d, &s->P);

    for (int k = 0; k < 2; ++k) {
        hipError_t e = hipHostMalloc((void**)&s->host_ctrl[k], sizeof(Ctrl), hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s->snap_ev[k], hipEventDisableTiming);
        if (e != hipSuccess) {
            delete s;
            return fail(WCNST_E_HIP, "host staging allocation failed: %s", hipGetErrorString(e));
        }
    }
    hipLaunchKernelGGL(ctrl_init, dim3(1), dim3(64), 0, s->stream, s->ctrl, 0.0, 0LL);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        wcnst_destroy(s);
        return fail(WCNST_E_HIP, "control init launch failed: %s", hipGetErrorString(e));
    }
    st = layout_reset(s);
    if (st) {
        wcnst_destroy(s);
        return st;
    }
    *out = s;
    return WCNST_OK;
}

extern "C" wcnst_status wcnst_destroy(wcnst_solver* s)
{
    if (!s) return WCNST_OK;
    (void)hipStreamSynchronize(s->stream);
    for (int k = 0; k < 2; ++k) {
        if (s->host_ctrl[k]) (void)hipHostFree(s->host_ctrl[k]);
        if (s->snap_ev[k]) (void)hipEventDestroy(s->snap_ev[k]);
    }
    for (hipEvent_t e : s->ev_pool) (void)hipEventDestroy(e);
    delete s;
    return WCNST_OK;
}

// ---------------------------------------------------------- launchers

// Segments of a 2D launch: nseg1 segments of ty rows, then segments of ty2
// rows, nseg in all.
struct SegMap {
    int ty, ty2, nseg1, nseg;
};

// One height in general.  A launch of one round with two wavefronts on most
// SIMDs (more wavefronts than SIMDs, no more than the slots) is balanced:
// a SIMD issues from its oldest wavefront first, so of the two that share
// it (blocks b and b + SIMDs in dispatch order, measured) the first runs at
// about its lone speed while the second, measured, advances about 0.48 as
// fast, then finishes alone.  The first-dispatched rows of segments take a
// rows and the others c rows with c + 3 = 0.48 (a + 3) (3: the extra rows
// of y-midpoints of a segment), so that both wavefronts of a SIMD finish
// together: 2048^2 stage 0.45 -> 0.41 ms (47 and 22 rows).
static SegMap stage_segments(int nstrips, int ny, int ty, int slots, bool balance)
{
    const int nseg = (ny + ty - 1) / ty;
    const SegMap one{ty, ty, nseg, nseg};
    if (!balance) return one;
    const long long simds = slots / 2;
    const long long waves = (long long)nstrips * nseg;
    if (waves <= simds || waves > slots) return one;
    const int na = (int)(simds / nstrips);
    if (na < 1) return one;
    const double r = 0.48;
    const int a = (int)std::lround(((double)ny / na + 3.0 - 3.0 * r) / (1.0 + r));
    if (a < 1 || (long long)a * na >= ny) return one;
    const int rest = ny - a * na;
    const int c = (rest + na - 1) / na;
    const int nb = (rest + c - 1) / c;
    if ((long long)nstrips * (na + nb) > slots) return one;
    return SegMap{a, c, na, na + nb};
}

// Adaptive layout for the solver's balanced stage shape (2D, heights chosen
// by the library), or off: one height, a shape beyond the tables or the
// planner's LDS, heights set by the caller, or no tables (the
// allocation-free solve).
static wcnst_status layout_reset(wcnst_solver* s)
{
    s->seg_on = false;
    const int ns = (s->d.nx + TX - 1) / TX;
    const SegMap m = s->d.ndim == 2 ? stage_segments(ns, s->d.ny, s->ty, s->slots, true) : SegMap{1, 1, 1, 1};
    const bool on = s->d.ndim == 2 && s->seg_tab && !s->ty_user && m.nseg1 < m.nseg &&
                    (long long)ns * (m.nseg1 + 1) <= LAYOUT_CAP && (long long)ns * (2 * m.nseg1 + 1) <= LAYOUT_LDS_INTS;
    hipLaunchKernelGGL(layout_init, dim3(1), dim3(256), 0, s->stream, s->ctrl, on ? 1 : 0, s->seg_tab, s->seg_cost,
                       s->seg_ctr, ns, m.nseg1, m.ty, std::max(1, m.ty / 4));
    HIP_TRY(hipGetLastError());
    s->seg_n1 = m.nseg1;
    s->seg_launch = 0;
    s->seg_on = on;
    return WCNST_OK;
}

template <int SYS, int NV, int FLUX, int SCHEME, bool CHAR, int MODE>
static void launch_sweep_t(const wcnst_solver* s, const double* U, const double* Un, double* out,
                           uint8_t* flags, const StageArgs& A)
{
    if constexpr (SYS == SYS_EULER && NV == 4) {
        const int nstrips = (s->d.nx + TX - 1) / TX;
        // cut flags (right-hand-side launches) need one segment height
        const SegMap m = stage_segments(nstrips, s->d.ny, s->ty, s->slots, MODE == MODE_STAGE && !s->ty_user);
        int seg_par = 0;
        if (MODE == MODE_STAGE && s->seg_on && m.nseg1 < m.nseg) {
            seg_par = (int)(s->seg_launch & 1);
            s->seg_launch += 1;
        }
        if (wcnst_general_bc(&s->d))
            hipLaunchKernelGGL((sweep2d<NV, FLUX, SCHEME, CHAR, MODE, true>), dim3(nstrips, m.nseg), dim3(WAVE), 0,
                               s->stream, U, Un, out, flags, s->ctrl, s->P, A, m.ty, m.ty2, m.nseg1, seg_par);
        else
            hipLaunchKernelGGL((sweep2d<NV, FLUX, SCHEME, CHAR, MODE, false>), dim3(nstrips, m.nseg), dim3(WAVE), 0,
                               s->stream, U, Un, out, flags, s->ctrl, s->P, A, m.ty, m.ty2, m.nseg1, seg_par);
    } else if (s->d.diff == WCNST_MD) {
        constexpr int W = strip_cells<DIFF_MD>();
        hipLaunchKernelGGL((sweep1d<SYS, NV, FLUX, SCHEME, CHAR, MODE, DIFF_MD>), dim3((s->d.nx + W - 1) / W),
                           dim3(WAVE), 0, s->stream, U, Un, out, flags, s->ctrl, s->P, A);
    } else if (s->d.diff == WCNST_HWCNS) {
        constexpr int W = strip_cells<DIFF_HW>();
        hipLaunchKernelGGL((sweep1d<SYS, NV, FLUX, SCHEME, CHAR, MODE, DIFF_HW>), dim3((s->d.nx + W - 1) / W),
                           dim3(WAVE), 0, s->stream, U, Un, out, flags, s->ctrl, s->P, A);
    } else {
        constexpr int W = strip_cells<DIFF_MND>();
        const int nstrips = (s->d.nx + W - 1) / W;
        if constexpr (MODE == MODE_STAGE && SYS == SYS_EULER && NV == 3) {
            // few strips: the latency mode (three wavefronts per strip)
            if (nstrips <= s->split_strips) {
                if (wcnst_general_bc(&s->d))
                    hipLaunchKernelGGL((sweep1d_split<FLUX, SCHEME, CHAR, true>), dim3(nstrips),
                                       dim3(WAVE * SPLIT_WAVES), 0, s->stream, U, Un, out, s->ctrl, s->P, A);
                else
                    hipLaunchKernelGGL((sweep1d_split<FLUX, SCHEME, CHAR, false>), dim3(nstrips),
                                       dim3(WAVE * SPLIT_WAVES), 0, s->stream, U, Un, out, s->ctrl, s->P, A);
                return;
            }
        }
        hipLaunchKernelGGL((sweep1d<SYS, NV, FLUX, SCHEME, CHAR, MODE, DIFF_MND>), dim3(nstrips), dim3(WAVE), 0,
                           s->stream, U, Un, out, flags, s->ctrl, s->P, A);
    }
}

template <int SYS, int NV, int FLUX, bool CHAR, int MODE>
static void launch_scheme(const wcnst_solver* s, const double* U, const double* Un, double* out,
                          uint8_t* flags, const StageArgs& A)
{
    switch (s->d.scheme) {
    case WCNST_LINEAR: launch_sweep_t<SYS, NV, FLUX, SCH_LINEAR, CHAR, MODE>(s, U, Un, out, flags, A); break;
    case WCNST_JS: launch_sweep_t<SYS, NV, FLUX, SCH_JS, CHAR, MODE>(s, U, Un, out, flags, A); break;
    case WCNST_Z: launch_sweep_t<SYS, NV, FLUX, SCH_Z, CHAR, MODE>(s, U, Un, out, flags, A); break;
    default:
        if (s->d.q == 6) launch_sweep_t<SYS, NV, FLUX, SCH_TENO, CHAR, MODE>(s, U, Un, out, flags, A);
        else launch_sweep_t<SYS, NV, FLUX, SCH_TENO_Q, CHAR, MODE>(s, U, Un, out, flags, A);
        break;
    }
}

template <int SYS, int NV, int FLUX, int MODE>
static void launch_char(const wcnst_solver* s, const double* U, const double* Un, double* out,
                        uint8_t* flags, const StageArgs& A)
{
    if (SYS == SYS_EULER && s->d.charwise) launch_scheme<SYS, NV, FLUX, true, MODE>(s, U, Un, out, flags, A);
    else launch_scheme<SYS, NV, FLUX, false, MODE>(s, U, Un, out, flags, A);
}

template <int MODE>
static void launch_sweep(const wcnst_solver* s, const double* U, const double* Un, double* out,
                         uint8_t* flags, const StageArgs& A)
{
    const bool lf = s->d.flux == WCNST_LF, vl = s->d.flux == WCNST_VANLEER;
    switch (s->kind) {
    case K_ADV1: launch_scheme<SYS_ADV, 1, FLUX_ROE, false, MODE>(s, U, Un, out, flags, A); break;
    case K_BURG1:
        if (lf) launch_scheme<SYS_BURG, 1, FLUX_LF, false, MODE>(s, U, Un, out, flags, A);
        else launch_scheme<SYS_BURG, 1, FLUX_ROE, false, MODE>(s, U, Un, out, flags, A);
        break;
    case K_EUL1:
        if (lf) launch_char<SYS_EULER, 3, FLUX_LF, MODE>(s, U, Un, out, flags, A);
        else if (vl) launch_char<SYS_EULER, 3, FLUX_VL, MODE>(s, U, Un, out, flags, A);
        else launch_char<SYS_EULER, 3, FLUX_ROE, MODE>(s, U, Un, out, flags, A);
        break;
    case K_EUL2:
        if (lf) launch_char<SYS_EULER, 4, FLUX_LF, MODE>(s, U, Un, out, flags, A);
        else if (vl) launch_char<SYS_EULER, 4, FLUX_VL, MODE>(s, U, Un, out, flags, A);
        else launch_char<SYS_EULER, 4, FLUX_ROE, MODE>(s, U, Un, out, flags, A);
        break;
    }
}

static void launch_wavespeed(const wcnst_solver* s, const double* U)
{
    const size_t cells = (size_t)s->d.nx * s->d.ny;
    int blocks = (int)std::min<size_t>((cells + 255) / 256, 2048);
    switch (s->kind) {
    case K_ADV1: hipLaunchKernelGGL((wavespeed<SYS_ADV, 1>), dim3(blocks), dim3(256), 0, s->stream, U, s->ctrl, s->P, s->parity); break;
    case K_BURG1: hipLaunchKernelGGL((wavespeed<SYS_BURG, 1>), dim3(blocks), dim3(256), 0, s->stream, U, s->ctrl, s->P, s->parity); break;
    case K_EUL1: hipLaunchKernelGGL((wavespeed<SYS_EULER, 3>), dim3(blocks), dim3(256), 0, s->stream, U, s->ctrl, s->P, s->parity); break;
    case K_EUL2: hipLaunchKernelGGL((wavespeed<SYS_EULER, 4>), dim3(blocks), dim3(256), 0, s->stream, U, s->ctrl, s->P, s->parity); break;
    }
}

static hipEvent_t pool_event(wcnst_solver* s)
{
    if (s->ev_used == s->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        s->ev_pool.push_back(e);
    }
    return s->ev_pool[s->ev_used++];
}

// One SSP-RK3 step: three fused stage kernels.
static void launch_step(wcnst_solver* s, double* U, double t_final, double cfl, double fixed_dt)
{
    const double* in[3] = {U, s->U1, s->U2};
    double* outp[3] = {s->U1, s->U2, U};
    for (int st = 0; st < 3; ++st) {
        StageArgs A;
        A.t_final = t_final;
        A.cfl = cfl;
        A.fixed_dt = fixed_dt;
        A.stage = st;
        A.parity = s->parity;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (s->prof) {
            e0 = pool_event(s);
            e1 = pool_event(s);
            if (e0) (void)hipEventRecord(e0, s->stream);
        }
        launch_sweep<MODE_STAGE>(s, in[st], U, outp[st], nullptr, A);
        if (s->prof && e1) (void)hipEventRecord(e1, s->stream);
    }
    s->parity ^= 1;
}

extern "C" wcnst_status wcnst_rhs(wcnst_solver* s, const double* U, double* R, uint8_t* flags)
{
    if (!s || !U || !R) return fail(WCNST_E_INVALID_ARG, "null argument");
    if (U == R) return fail(WCNST_E_INVALID_ARG, "U and R must not alias");
    StageArgs A = {};
    launch_sweep<MODE_RHS>(s, U, nullptr, R, flags, A);
    HIP_TRY(hipGetLastError());
    return WCNST_OK;
}

extern "C" wcnst_status wcnst_step(wcnst_solver* s, double* U, double dt, double cfl)
{
    if (!s || !U) return fail(WCNST_E_INVALID_ARG, "null argument");
    if (!(dt > 0.0) && !(cfl > 0.0)) return fail(WCNST_E_INVALID_ARG, "need dt > 0 or cfl > 0");
    hipLaunchKernelGGL(ctrl_open, dim3(1), dim3(64), 0, s->stream, s->ctrl, s->parity);
    if (!(dt > 0.0)) launch_wavespeed(s, U);
    launch_step(s, U, INFINITY, cfl, dt > 0.0 ? dt : 0.0);
    HIP_TRY(hipGetLastError());
    return WCNST_OK;
}

static wcnst_status read_ctrl(wcnst_solver* s, Ctrl* c)
{
    HIP_TRY(hipMemcpyAsync(c, s->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return WCNST_OK;
}

// The record holding the newest completed state.
static const StepRec& newest(const Ctrl& c)
{
    return c.rec[0].step >= c.rec[1].step ? c.rec[0] : c.rec[1];
}

extern "C" wcnst_status wcnst_solve(wcnst_solver* s, double* U, double t_final, double cfl,
                                    int64_t max_steps, double* t_out, int64_t* steps_out)
{
    if (!s || !U) return fail(WCNST_E_INVALID_ARG, "null argument");
    if (!(cfl > 0.0)) return fail(WCNST_E_INVALID_ARG, "cfl must be > 0");
    if (max_steps < 0) return fail(WCNST_E_INVALID_ARG, "max_steps must be >= 0");
    if (std::isnan(t_final)) return fail(WCNST_E_INVALID_ARG, "t_final is NaN");
    const bool timed = std::isfinite(t_final);

    hipLaunchKernelGGL(ctrl_open, dim3(1), dim3(64), 0, s->stream, s->ctrl, s->parity);
    launch_wavespeed(s, U);
    HIP_TRY(hipGetLastError());

    int64_t launched = 0;
    int64_t chunk = 4;
    int slot = 0;
    bool have_prev = false;
    int64_t prev_launched = 0;
    while (launched < max_steps) {
        const int64_t k = std::min(chunk, max_steps - launched);
        for (int64_t i = 0; i < k; ++i) launch_step(s, U, t_final, cfl, 0.0);
        launched += k;
        HIP_TRY(hipGetLastError());
        if (!timed) continue;
        // snapshot after this chunk; inspect the previous one (one chunk of look-ahead)
        HIP_TRY(hipMemcpyAsync(s->host_ctrl[slot], s->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s->stream));
        HIP_TRY(hipEventRecord(s->snap_ev[slot], s->stream));
        const int prev = slot ^ 1;
        slot ^= 1;
        if (!have_prev) {
            have_prev = true;
            prev_launched = launched;
            continue;
        }
        HIP_TRY(hipEventSynchronize(s->snap_ev[prev]));
        const Ctrl& c = *s->host_ctrl[prev];
        const StepRec& r = newest(c);
        if (c.status != 0 || c.done) break;
        // estimate the steps still needed beyond what is already queued
        const int64_t done_steps = r.step - c.call_step0;
        const double dt = c.rec[0].step >= c.rec[1].step ? c.rec[1].dt : c.rec[0].dt;
        int64_t est = 8;
        if (dt > 0.0 && std::isfinite(dt)) est = (int64_t)std::ceil((t_final - r.t) / dt) + 1;
        const int64_t queued = launched - done_steps;
        (void)prev_launched;
        prev_launched = launched;
        chunk = std::max<int64_t>(1, std::min<int64_t>(est - queued, 512));
    }
    Ctrl c;
    wcnst_status st = read_ctrl(s, &c);
    if (st) return st;
    const StepRec& r = newest(c);
    if (t_out) *t_out = r.t;
    if (steps_out) *steps_out = r.step - c.call_step0;
    if (c.status != 0) {
        const long long stg = c.bad_key == ~0ull ? -1 : (long long)(c.bad_key >> 36);
        const long long cell = c.bad_key == ~0ull ? -1 : (long long)(c.bad_key & ((1ull << 36) - 1));
        return fail(WCNST_E_NONPHYSICAL, "non-physical state at global stage %lld, cell %lld", stg, cell);
    }
    if (timed && !(t_final - r.t <= 1e-12 * t_final))
        return fail(WCNST_E_MAX_STEPS, "t_final not reached in %lld steps (t = %.17g)",
                    (long long)max_steps, r.t);
    return WCNST_OK;
}

// ------------------------------------------------ allocation-free solve

// Static scratch of wcnst_solve_noalloc: the control block and the two
// Runge-Kutta stage buffers of one solve.  Each device the library runs on
// holds its own copy until the process ends.  In host code its name is
// only a handle for hipGetSymbolAddress: kernels get the device address
// obtained from that call (g_scratch_ptr), never the name.
static __device__ __align__(256) unsigned char scratch[WCNST_NOALLOC_MAX_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of the current device's copy of `scratch`, looked up once
// per device with that device current.
static wcnst_status scratch_address(void** out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(WCNST_E_HIP, "device index %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(WCNST_E_HIP, "no device address for the static scratch on device %d", dev);
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return WCNST_OK;
}

extern "C" wcnst_status wcnst_solve_noalloc(const wcnst_desc* d, void* hip_stream, double* U, double t_final,
                                            double cfl, int64_t max_steps, double* t_out, int64_t* steps_out)
{
    wcnst_status st = wcnst_check_desc(d);
    if (st) return st;
    if (!U) return fail(WCNST_E_INVALID_ARG, "null state");
    if (!(cfl > 0.0)) return fail(WCNST_E_INVALID_ARG, "cfl must be > 0");
    if (max_steps < 0) return fail(WCNST_E_INVALID_ARG, "max_steps must be >= 0");
    if (std::isnan(t_final)) return fail(WCNST_E_INVALID_ARG, "t_final is NaN");
    size_t need = 0;
    wcnst_workspace_size(d, &need);
    if (need > (size_t)WCNST_NOALLOC_MAX_BYTES)
        return fail(WCNST_E_INVALID_ARG, "grid needs %zu bytes of scratch; the allocation-free solve holds %zu",
                    need, (size_t)WCNST_NOALLOC_MAX_BYTES);
    void* ptr = nullptr;
    st = scratch_address(&ptr);
    if (st) return st;

    // a solver on the stack over the static scratch: no pinned staging, no
    // events (the state is polled with plain copies into host variables)
    wcnst_solver s{};
    s.d = *d;
    s.nv = wcnst_desc_nvar(d);
    s.kind = d->system == WCNST_ADVECTION ? K_ADV1
             : d->system == WCNST_BURGERS ? K_BURG1
             : d->ndim == 1               ? K_EUL1
                                          : K_EUL2;
    s.stream = (hipStream_t)hip_stream;
    const size_t state = (size_t)s.nv * d->nx * d->ny * sizeof(double);
    uint8_t* ws = (uint8_t*)ptr;
    s.ctrl = (Ctrl*)ws;
    s.U1 = (double*)(ws + align256(sizeof(Ctrl)));
    s.U2 = (double*)(ws + align256(sizeof(Ctrl)) + align256(state));
    s.parity = 0;
    s.slots = wcnst_wave_slots();
    {
        const int strips = (d->nx + TX - 1) / TX, rows = d->ny;
        s.ty = d->ndim == 2 ? wcnst_auto_rows(&strips, &rows, 1, s.slots) : 35;
    }
    s.split_strips = SPLIT_STRIPS;
    wcnst_make_params(d, &s.P);
    const bool timed = std::isfinite(t_final);

    // a fresh solve from t = 0: the control block is reset by a kernel
    hipLaunchKernelGGL(ctrl_init, dim3(1), dim3(64), 0, s.stream, s.ctrl, 0.0, 0LL);
    hipLaunchKernelGGL(ctrl_open, dim3(1), dim3(64), 0, s.stream, s.ctrl, s.parity);
    launch_wavespeed(&s, U);
    HIP_TRY(hipGetLastError());
    int64_t launched = 0, chunk = 4;
    Ctrl c;
    while (launched < max_steps) {
        const int64_t k = std::min(chunk, max_steps - launched);
        for (int64_t i = 0; i < k; ++i) launch_step(&s, U, t_final, cfl, 0.0);
        launched += k;
        HIP_TRY(hipGetLastError());
        if (!timed) continue;
        st = read_ctrl(&s, &c);
        if (st) return st;
        if (c.status != 0 || c.done) break;
        const StepRec& r = newest(c);
        const double dt = c.rec[0].step >= c.rec[1].step ? c.rec[1].dt : c.rec[0].dt;
        int64_t est = 8;
        if (dt > 0.0 && std::isfinite(dt)) est = (int64_t)std::ceil((t_final - r.t) / dt) + 1;
        chunk = std::max<int64_t>(1, std::min<int64_t>(est, 512));
    }
    st = read_ctrl(&s, &c);
    if (st) return st;
    const StepRec& r = newest(c);
    if (t_out) *t_out = r.t;
    if (steps_out) *steps_out = r.step;
    if (c.status != 0) {
        const long long stg = c.bad_key == ~0ull ? -1 : (long long)(c.bad_key >> 36);
        const long long cell = c.bad_key == ~0ull ? -1 : (long long)(c.bad_key & ((1ull << 36) - 1));
        return fail(WCNST_E_NONPHYSICAL, "non-physical state at global stage %lld, cell %lld", stg, cell);
    }
    if (timed && !(t_final - r.t <= 1e-12 * t_final))
        return fail(WCNST_E_MAX_STEPS, "t_final not reached in %lld steps (t = %.17g)", (long long)max_steps, r.t);
    return WCNST_OK;
}

extern "C" wcnst_status wcnst_status_sync(wcnst_solver* s, double* t, int64_t* steps, int32_t* status,
                                          int64_t* bad_stage, int64_t* bad_cell)
{
    if (!s) return fail(WCNST_E_INVALID_ARG, "null handle");
    Ctrl c;
    wcnst_status st = read_ctrl(s, &c);
    if (st) return st;
    const StepRec& r = newest(c);
    if (t) *t = r.t;
    if (steps) *steps = r.step;
    if (status) *status = c.status;
    const bool none = c.bad_key == ~0ull;
    if (bad_stage) *bad_stage = none ? -1 : (int64_t)(c.bad_key >> 36);
    if (bad_cell) *bad_cell = none ? -1 : (int64_t)(c.bad_key & ((1ull << 36) - 1));
    return WCNST_OK;
}

extern "C" wcnst_status wcnst_reset(wcnst_solver* s, double t, int64_t steps)
{
    if (!s) return fail(WCNST_E_INVALID_ARG, "null handle");
    hipLaunchKernelGGL(ctrl_init, dim3(1), dim3(64), 0, s->stream, s->ctrl, t, (long long)steps);
    s->parity = 0;
    HIP_TRY(hipGetLastError());
    return WCNST_OK;
}

int wcnst_wave_slots()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;
    return 8 * cus;
}

int wcnst_auto_rows(const int* strips, const int* rows, int n, int slots)
{
    // A wavefront's time grows with its segment's rows plus a fixed cost
    // (3 extra rows of y-midpoints and the 6-row staging prologue: about 6
    // rows in all), and the launch lasts as long as its busiest SIMD: w
    // wavefronts share a SIMD's issue (w >= 2), a lone one uses about two
    // thirds of it.  The segment height minimising (rows + 6) * g(w),
    // ties to the taller, fits measured stage times from 128^2 to 8192^2.
    const long long simds = slots / 2 > 0 ? slots / 2 : 1;
    int best_ty = 35;
    double best = 1e300;
    for (int ty = 35; ty >= 2; --ty) {
        long long waves = 0;
        for (int i = 0; i < n; ++i) waves += (long long)strips[i] * ((rows[i] + ty - 1) / ty);
        const long long w = (waves + simds - 1) / simds;
        const double cost = (ty + 6) * (w <= 1 ? 1.5 : (double)w);
        if (cost < best) {
            best = cost;
            best_ty = ty;
        }
    }
    return best_ty;
}

extern "C" wcnst_status wcnst_set_tuning(wcnst_solver* s, int32_t rows_per_segment)
{
    if (!s) return fail(WCNST_E_INVALID_ARG, "null handle");
    if (rows_per_segment < 0) return fail(WCNST_E_INVALID_ARG, "rows_per_segment must be >= 0");
    if (rows_per_segment == 0) {
        // the shape chosen at creation
        const int strips = (s->d.nx + TX - 1) / TX, rows = s->d.ny;
        s->ty = s->d.ndim == 2 ? wcnst_auto_rows(&strips, &rows, 1, s->slots) : 35;
        s->ty_user = false;
        return layout_reset(s);
    }
    s->ty = rows_per_segment;
    s->ty_user = true;
    return layout_reset(s);
}

extern "C" wcnst_status wcnst_stage_layout(wcnst_solver* s, int32_t* rows, int32_t cap, int32_t* count)
{
    if (!s || !count) return fail(WCNST_E_INVALID_ARG, "null argument");
    *count = 0;
    if (!s->seg_on) return WCNST_OK;
    const int n = ((s->d.nx + TX - 1) / TX) * (s->seg_n1 + 1);
    *count = n;
    if (!rows || cap < n) return WCNST_OK;
    HIP_TRY(hipStreamSynchronize(s->stream));
    // the table the next balanced launch reads
    const int c = (int)(s->seg_launch & 1);
    HIP_TRY(hipMemcpy(rows, s->seg_tab + (size_t)c * LAYOUT_CAP, sizeof(int) * (size_t)n, hipMemcpyDeviceToHost));
    return WCNST_OK;
}

extern "C" wcnst_status wcnst_stage_shape(const wcnst_solver* s, int32_t* strips, int32_t* rows1, int32_t* rows2,
                                          int32_t* nseg1, int32_t* nseg)
{
    if (!s || !strips || !rows1 || !rows2 || !nseg1 || !nseg) return fail(WCNST_E_INVALID_ARG, "null argument");
    if (s->d.ndim != 2) {
        const int W = s->d.diff == WCNST_MD ? strip_cells<DIFF_MD>()
                                            : (s->d.diff == WCNST_HWCNS ? strip_cells<DIFF_HW>() : strip_cells<DIFF_MND>());
        *strips = (s->d.nx + W - 1) / W;
        *rows1 = *rows2 = 1;
        *nseg1 = *nseg = 1;
        return WCNST_OK;
    }
    *strips = (s->d.nx + TX - 1) / TX;
    const SegMap m = stage_segments(*strips, s->d.ny, s->ty, s->slots, !s->ty_user);
    *rows1 = m.ty;
    *rows2 = m.ty2;
    *nseg1 = m.nseg1;
    *nseg = m.nseg;
    return WCNST_OK;
}

extern "C" wcnst_status wcnst_profile_enable(wcnst_solver* s, int enable)
{
    if (!s) return fail(WCNST_E_INVALID_ARG, "null handle");
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->prof = enable != 0;
    s->ev_used = 0;
    return WCNST_OK;
}

extern "C" wcnst_status wcnst_profile_read(wcnst_solver* s, double* stage_ms, int64_t* stage_launches)
{
    if (!s) return fail(WCNST_E_INVALID_ARG, "null handle");
    HIP_TRY(hipStreamSynchronize(s->stream));
    double total = 0.0;
    for (size_t i = 0; i + 1 < s->ev_used; i += 2) {
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, s->ev_pool[i], s->ev_pool[i + 1]));
        total += ms;
    }
    if (stage_ms) *stage_ms = total;
    if (stage_launches) *stage_launches = (int64_t)(s->ev_used / 2);
    s->ev_used = 0;
    return WCNST_OK;
}

// ------------------------------------------- launchers for request pools

size_t wcnst_ctrl_bytes() { return sizeof(Ctrl); }

hipError_t wcnst_launch_init_grid(const wcnst_desc* d, const double* U, void* ctrl, hipStream_t st)
{
    Params P;
    wcnst_make_params(d, &P);
    hipLaunchKernelGGL(ctrl_init, dim3(1), dim3(64), 0, st, (Ctrl*)ctrl, 0.0, 0LL);
    const size_t cells = (size_t)d->nx * d->ny;
    const int blocks = (int)std::min<size_t>((cells + 255) / 256, 2048);
    if (d->ndim == 2)
        hipLaunchKernelGGL((wavespeed<SYS_EULER, 4>), dim3(blocks), dim3(256), 0, st, U, (Ctrl*)ctrl, P, 0);
    else
        hipLaunchKernelGGL((wavespeed<SYS_EULER, 3>), dim3(blocks), dim3(256), 0, st, U, (Ctrl*)ctrl, P, 0);
    return hipGetLastError();
}

hipError_t wcnst_launch_multi_init(int ndim, const void* reqs, int nreq, hipStream_t st)
{
    if (nreq <= 0) return hipSuccess;
    if (ndim == 2)
        hipLaunchKernelGGL((multi_init<4>), dim3(nreq), dim3(256), 0, st, (const ReqGrid*)reqs);
    else
        hipLaunchKernelGGL((multi_init<3>), dim3(nreq), dim3(256), 0, st, (const ReqGrid*)reqs);
    return hipGetLastError();
}

template <int NDIM, int FLUX, int SCHEME, bool CHAR>
static void launch_multi_t(const ReqGrid* reqs, const int* map, int nreq, int nblocks, int stage, int tick_step,
                           int ty, bool general, hipStream_t st)
{
    if constexpr (NDIM == 2) {
        if (general)
            hipLaunchKernelGGL((sweep2d_multi<4, FLUX, SCHEME, CHAR, true>), dim3(nblocks), dim3(WAVE), 0, st, reqs,
                               map, nreq, stage, tick_step, ty);
        else
            hipLaunchKernelGGL((sweep2d_multi<4, FLUX, SCHEME, CHAR, false>), dim3(nblocks), dim3(WAVE), 0, st, reqs,
                               map, nreq, stage, tick_step, ty);
    } else if (general) {
        hipLaunchKernelGGL((sweep1d_multi<FLUX, SCHEME, CHAR, true>), dim3(nblocks), dim3(WAVE), 0, st, reqs, map,
                           nreq, stage, tick_step);
    } else {
        hipLaunchKernelGGL((sweep1d_multi<FLUX, SCHEME, CHAR, false>), dim3(nblocks), dim3(WAVE), 0, st, reqs, map,
                           nreq, stage, tick_step);
    }
}

template <int NDIM, int FLUX, bool CHAR>
static void launch_multi_s(const wcnst_desc* d, const ReqGrid* reqs, const int* map, int nreq, int nblocks, int stage,
                           int tick_step, int ty, bool general, hipStream_t st)
{
    switch (d->scheme) {
    case WCNST_LINEAR:
        launch_multi_t<NDIM, FLUX, SCH_LINEAR, CHAR>(reqs, map, nreq, nblocks, stage, tick_step, ty, general, st);
        break;
    case WCNST_JS:
        launch_multi_t<NDIM, FLUX, SCH_JS, CHAR>(reqs, map, nreq, nblocks, stage, tick_step, ty, general, st);
        break;
    case WCNST_Z:
        launch_multi_t<NDIM, FLUX, SCH_Z, CHAR>(reqs, map, nreq, nblocks, stage, tick_step, ty, general, st);
        break;
    default:
        if (d->q == 6)
            launch_multi_t<NDIM, FLUX, SCH_TENO, CHAR>(reqs, map, nreq, nblocks, stage, tick_step, ty, general, st);
        else
            launch_multi_t<NDIM, FLUX, SCH_TENO_Q, CHAR>(reqs, map, nreq, nblocks, stage, tick_step, ty, general, st);
        break;
    }
}

template <int NDIM>
static void launch_multi_d(const wcnst_desc* d, const ReqGrid* r, const int* map, int nreq, int nblocks, int stage,
                           int tick_step, int ty, bool general, hipStream_t st)
{
    if (d->flux == WCNST_LF) {
        if (d->charwise) launch_multi_s<NDIM, FLUX_LF, true>(d, r, map, nreq, nblocks, stage, tick_step, ty, general, st);
        else launch_multi_s<NDIM, FLUX_LF, false>(d, r, map, nreq, nblocks, stage, tick_step, ty, general, st);
    } else if (d->flux == WCNST_VANLEER) {
        if (d->charwise) launch_multi_s<NDIM, FLUX_VL, true>(d, r, map, nreq, nblocks, stage, tick_step, ty, general, st);
        else launch_multi_s<NDIM, FLUX_VL, false>(d, r, map, nreq, nblocks, stage, tick_step, ty, general, st);
    } else {
        if (d->charwise) launch_multi_s<NDIM, FLUX_ROE, true>(d, r, map, nreq, nblocks, stage, tick_step, ty, general, st);
        else launch_multi_s<NDIM, FLUX_ROE, false>(d, r, map, nreq, nblocks, stage, tick_step, ty, general, st);
    }
}

hipError_t wcnst_launch_multi(const wcnst_desc* d, int ndim, const void* reqs, const int* map, int nreq, int nblocks,
                              int stage, int tick_step, int ty, bool general, hipStream_t st)
{
    const ReqGrid* r = (const ReqGrid*)reqs;
    if (ndim == 2) launch_multi_d<2>(d, r, map, nreq, nblocks, stage, tick_step, ty, general, st);
    else launch_multi_d<1>(d, r, map, nreq, nblocks, stage, tick_step, ty, general, st);
    return hipGetLastError();
}

template <int FLUX, int SCHEME, bool CHAR>
static void launch_persist_t(const ReqGrid* reqs, int nreq, int per_group, int waves, long long max_steps,
                             bool general, hipStream_t st)
{
    const dim3 grid((unsigned)((nreq + per_group - 1) / per_group)), block((unsigned)(waves * WAVE));
    if (general)
        hipLaunchKernelGGL((sweep1d_persist<FLUX, SCHEME, CHAR, true>), grid, block, 0, st, reqs, nreq, per_group,
                           max_steps);
    else
        hipLaunchKernelGGL((sweep1d_persist<FLUX, SCHEME, CHAR, false>), grid, block, 0, st, reqs, nreq, per_group,
                           max_steps);
}

template <int FLUX, bool CHAR>
static void launch_persist_s(const wcnst_desc* d, const ReqGrid* reqs, int nreq, int per_group, int waves,
                             long long max_steps, bool general, hipStream_t st)
{
    switch (d->scheme) {
    case WCNST_LINEAR:
        launch_persist_t<FLUX, SCH_LINEAR, CHAR>(reqs, nreq, per_group, waves, max_steps, general, st);
        break;
    case WCNST_JS: launch_persist_t<FLUX, SCH_JS, CHAR>(reqs, nreq, per_group, waves, max_steps, general, st); break;
    case WCNST_Z: launch_persist_t<FLUX, SCH_Z, CHAR>(reqs, nreq, per_group, waves, max_steps, general, st); break;
    default:
        if (d->q == 6) launch_persist_t<FLUX, SCH_TENO, CHAR>(reqs, nreq, per_group, waves, max_steps, general, st);
        else launch_persist_t<FLUX, SCH_TENO_Q, CHAR>(reqs, nreq, per_group, waves, max_steps, general, st);
        break;
    }
}

hipError_t wcnst_launch_persist(const wcnst_desc* d, const void* reqs, int nreq, int per_group, int waves,
                                long long max_steps, bool general, hipStream_t st)
{
    if (nreq <= 0) return hipSuccess;
    if (per_group < 1 || per_group > PERSIST_MAX_GRIDS || waves < 1 || waves > PERSIST_MAX_WAVES)
        return hipErrorInvalidValue;
    const ReqGrid* r = (const ReqGrid*)reqs;
    if (d->flux == WCNST_LF) {
        if (d->charwise) launch_persist_s<FLUX_LF, true>(d, r, nreq, per_group, waves, max_steps, general, st);
        else launch_persist_s<FLUX_LF, false>(d, r, nreq, per_group, waves, max_steps, general, st);
    } else if (d->flux == WCNST_VANLEER) {
        if (d->charwise) launch_persist_s<FLUX_VL, true>(d, r, nreq, per_group, waves, max_steps, general, st);
        else launch_persist_s<FLUX_VL, false>(d, r, nreq, per_group, waves, max_steps, general, st);
    } else {
        if (d->charwise) launch_persist_s<FLUX_ROE, true>(d, r, nreq, per_group, waves, max_steps, general, st);
        else launch_persist_s<FLUX_ROE, false>(d, r, nreq, per_group, waves, max_steps, general, st);
    }
    return hipGetLastError();
}

hipError_t wcnst_launch_block_map(const void* reqs, int nreq, int total, int* map, hipStream_t st)
{
    if (nreq <= 0) return hipSuccess;
    hipLaunchKernelGGL(block_map_fill, dim3(nreq), dim3(256), 0, st, (const ReqGrid*)reqs, nreq, total, map);
    return hipGetLastError();
}

extern "C" const char* wcnst_last_error(void) { return g_err; }

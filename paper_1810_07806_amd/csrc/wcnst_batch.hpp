// Shared pieces of the persistent 1D Euler solver: the instance table, the
// job slots and the launch head (device and host views), and the host
// functions that plan and launch one persistent pass over a table.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "wcnst.h"
#include "wcnst_device.hpp"

namespace wcnstb {

constexpr int WAVE = 64;
constexpr int TX = WAVE - 3;  // cells per strip
constexpr int NV = 3;
constexpr int KMAX = 64;  // most waves cooperating on one instance
constexpr double WAIT_LIMIT_S = 30.0;  // longest wait of a part at a barrier

struct BInst {
    double* u;   // state at t^n, layout [v][n]
    double* u1;  // stage buffers of the same size
    double* u2;
    int n, bc;
    int k, pad0;
    double dx, c1, c2, c3;
    double t_final, cfl;
    long long step_end;  // a launch stops before this step (resumable)
    // state carried between launches (t, steps: read at the start of a
    // launch, written by part 0 at its end)
    double t;
    long long steps;
    // results and the state shared by the parts of one instance during a
    // launch (atomics only)
    unsigned long long bad_key;  // (global stage << 36) | cell
    int status, pad1;
    unsigned arrive, gen;
    unsigned long long smax_bits[2];
};

// The fields of BInst a part reads at its start (one system-scope copy).
struct BInstIn {
    double* u;
    double* u1;
    double* u2;
    int n, bc;
    int k, pad0;
    double dx, c1, c2, c3;
    double t_final, cfl;
    long long step_end;
    double t;
    long long steps;
};

struct alignas(8) BSlot {
    int inst, part;
};

struct BHead {
    unsigned head;  // next slot
    int nslots;
    int err;  // a bounded wait expired
    int pad;
    long long wait_ticks;  // WAIT_LIMIT_S in wall-clock ticks
};

// Host side.  An instance record at t = 0 with buffers u, u1, u2.
void inst_init(BInst& r, const wcnst_desc& d, double* u, double* u1, double* u2, double t_final, double cfl);
// Clears the per-launch cooperation fields and sets the step bound.
void inst_arm(BInst& r, long long step_end);
// Scheme parameters shared by the instances (from any one descriptor).
void scheme_params(const wcnst_desc& d, wcnst::Params* P);
// Workgroups of wpg waves resident per compute unit.
hipError_t resident_per_cu(const wcnst_desc& d, int wpg, int* per_cu);
// Longest-part-first plan: instance i gets k = ceil(cost_i / (split x
// total / workers)) parts, at most KMAX, its strips and `running`; slots in
// that order.  Sets rec[i].k.  split = 0: one part each.
int plan_parts(std::vector<BInst>& rec, const std::vector<double>& cost, double split, double workers,
               int running, std::vector<BSlot>& slots);
// Queue reset + one persistent pass over the table (kernel chosen by d).
hipError_t launch_pass(const wcnst_desc& d, BInst* insts, BSlot* slots, BHead* head, const wcnst::Params& P,
                       int grid, int wpg, hipStream_t st);
// Wall-clock ticks in WAIT_LIMIT_S on the current device.
hipError_t wait_ticks(long long* ticks);

}  // namespace wcnstb

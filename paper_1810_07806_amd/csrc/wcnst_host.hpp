// Host-side helpers shared by the translation units of libwcnst.
#pragma once

#include <hip/hip_runtime.h>

#include <stddef.h>

#include "wcnst.h"

// Records a thread-local message (read by wcnst_last_error) and returns st.
wcnst_status wcnst_fail(wcnst_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
wcnst_status wcnst_check_desc(const wcnst_desc* d);
int wcnst_desc_nvar(const wcnst_desc* d);
// WCNST_OK when d has the scheme parameters of a (flux, scheme, charwise,
// q, gamma, C_T, C, epsilons, difference).
wcnst_status wcnst_check_same_scheme(const wcnst_desc& a, const wcnst_desc& d);
size_t wcnst_align256(size_t b);

namespace wcnst {
struct Params;
}
// Solver parameters of a validated descriptor (spacing, Eq. (5) coefficients).
void wcnst_make_params(const wcnst_desc* d, wcnst::Params* out);

// Multi-grid stage launches: bytes of one control block; reset it to t = 0
// and accumulate the CFL speed of U (1D or 2D Euler grid d) into its record
// 0; one stage of every grid of a ReqGrid table of one dimension (nblocks =
// total strips in 1D, total segments of ty rows in 2D).
size_t wcnst_ctrl_bytes();
hipError_t wcnst_launch_init_grid(const wcnst_desc* d, const double* U, void* ctrl, hipStream_t st);
// general: some grid of the table has reflecting / fixed sides or gravity
// (the tables then take the stage kernels that handle them).
// map (nullable): the table row of every block (wcnst_launch_block_map);
// without one each block searches the table.
hipError_t wcnst_launch_multi(const wcnst_desc* d, int ndim, const void* reqs, const int* map, int nreq, int nblocks,
                              int stage, int tick_step, int ty, bool general, hipStream_t st);
// One persistent launch that runs the nreq 1D grids of a table to their
// final times (or max_steps more steps): per_group grids per workgroup of
// `waves` wavefronts (at most 8 each).
hipError_t wcnst_launch_persist(const wcnst_desc* d, const void* reqs, int nreq, int per_group, int waves,
                                long long max_steps, bool general, hipStream_t st);
// Fill the block map of a table of nreq rows and `total` blocks (map: total
// ints; the rows' blk0 ascending from 0).
hipError_t wcnst_launch_block_map(const void* reqs, int nreq, int total, int* map, hipStream_t st);
// true when d has sides other than periodic / zero gradient, or gravity
bool wcnst_general_bc(const wcnst_desc* d);
// Wavefront slots of the current device for the 2D stage kernel (two per
// SIMD, four SIMDs per CU).
int wcnst_wave_slots();
// Rows per 2D segment in [2, 35] when the caller fixes none, for a launch
// over the grids (strips[i], rows[i]), i < n, on a device of `slots`
// wavefront slots (2 per SIMD): the height minimising a cost fitted to
// measured stage times.  Never changes results.
int wcnst_auto_rows(const int* strips, const int* rows, int n, int slots);
// wcnst_launch_init_grid for every grid of a ReqGrid table (one launch).
hipError_t wcnst_launch_multi_init(int ndim, const void* reqs, int nreq, hipStream_t st);

#define WCNST_HIP_TRY(expr)                                                                \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return wcnst_fail(WCNST_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// Device arithmetic of the WCNS-T midpoint flux for gfx950 (FP64 VALU).
//
// One call of face_flux() turns the six nodes j-2 .. j+3 around a midpoint
// x_{j+1/2} into the numerical flux there:
//   characteristic projection (Roe average of nodes j, j+1)      Sec. 3
//   TENO-5 interpolation of u_L and of the mirrored u_R          Sec. 2.2-2.3
//   back-projection and the Roe / local Lax-Friedrichs flux      Sec. 2.2, Eq. (6)
//
// Reproducible arithmetic.  The method is sensitive to rounding in two ways:
// (1) with eps = 1e-40 in Eq. (16), a stencil whose data are flat to
// round-off has beta_k ~ 1e-32 of pure rounding noise, so the last bits of
// beta decide the cut; (2) the cut is discontinuous, so over many steps a
// solution amplifies last-bit differences (two correct FP64 evaluation
// orders drift apart by ~1e-5 after 100 steps on the four-quadrant
// problem).  Every operation that produces a value is therefore evaluated
// in the plain order of its definition with IEEE division and square root
// and without implicit contraction (this file and the kernels are compiled
// with -ffp-contract=off), so results are reproducible bit for bit.  The
// interpolation (Eqs. (9)-(12), (15)), the characteristic projections and
// the Roe dissipation R |Lambda| L (U_R - U_L) use explicit fused
// multiply-adds, written at the same places in the oracle: one rounding
// per a * x + y, and fewer instructions.  (The
// reciprocals and roots of the Roe averages (the projection's; in 1D also
// the flux's, with the physical fluxes) use the hardware's correctly rounded
// sequences without their range scaling, which give the IEEE results bit
// for bit over the argument range they are used in; lanes whose arguments
// leave it redo that work with the IEEE operations.)
// Only the cut-off test itself, which is decided far from its threshold
// except in genuine ties, uses a fast reciprocal and the comparison form
// gamma_k < C_T * sum(gamma).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// The arithmetic is host-callable too, so it can be checked on a CPU.
#define WCNST_HD __host__ __device__ __forceinline__

namespace wcnst {

enum { SYS_ADV = 0, SYS_BURG = 1, SYS_EULER = 2 };
enum { FLUX_ROE = 0, FLUX_LF = 1, FLUX_VL = 2 };
// SCH_TENO: Eq. (16) with the paper's q = 6; SCH_TENO_Q: any integer q;
// SCH_Z: the Z weights of Borges et al. (2008), the paper's WCNS-Z
enum { SCH_TENO = 0, SCH_LINEAR = 1, SCH_JS = 2, SCH_TENO_Q = 3, SCH_Z = 4 };
enum { BC_PERIODIC = 0, BC_ZG = 1, BC_REFLECT = 2, BC_FIXED = 3 };
enum { DIFF_MND = 0, DIFF_MD = 1, DIFF_HW = 2 };

// ------------------------------------------------------ strip geometry

constexpr int WAVE = 64;      // lanes per wavefront, one midpoint each
constexpr int TX = WAVE - 3;  // cells per MND strip (1D) / columns per 2D strip

// 1D strips: the 64 midpoints of a wavefront serve the cells whose
// differences reach only them; MND reaches 3/2 spacings from a cell (61
// cells per strip), MD 5/2 spacings (59 cells).  HWCNS reaches midpoints
// 1/2 away and nodes 2 away; each lane also evaluates one node flux, so 64
// node fluxes serve 60 cells.
template <int DIFF>
constexpr int strip_cells()
{
    return DIFF == DIFF_MD ? WAVE - 5 : (DIFF == DIFF_HW ? WAVE - 4 : WAVE - 3);
}

// Owner of midpoint j (j in [-G, n-2+G]) among tiles of width w: the tile
// of the nearest cell.
WCNST_HD int face_owner(int j, int n, int w)
{
    j = j < 0 ? 0 : (j > n - 1 ? n - 1 : j);
    return j / w;
}

// Work index of launch index L inside a group of n consecutive launch
// indices [base, base + n).  Consecutive workgroups of a launch go to the 8
// XCDs in turn (workgroup L to XCD L mod 8), and each XCD has its own L2.
// The workgroups of a group that land on one XCD take one contiguous run of
// the group's work indices, so work items that are neighbours in the
// index order share an L2.  A bijection of [base, base + n): the launch
// order, and with it which workgroups share a SIMD, is unchanged.
WCNST_HD int xcd_order(int L, int base, int n)
{
    const int l = L - base;
    const int k = l & 7, per = n >> 3, extra = n & 7;
    return base + k * per + (k < extra ? k : extra) + (l >> 3);
}

// Rows of the n segments of one strip for the next stage launch, from the
// rows they had (boundaries b[0] = 0 < b[1] < .. < b[n]) and what each took
// (d[i] > 0, any unit).  A segment of r rows also computes about H rows of
// y-midpoints before its first row, so its cost per row is d[i] / (r + H);
// the new boundaries cut the strip's cost, so read, into n equal parts,
// each moved half way from the old boundary (the costs move with the flow
// and are measured one launch late), and keep every segment at least minr
// rows (b[n] >= n * minr).  With a zero duration the layout is kept.  out
// must not alias b or d.
WCNST_HD void plan_strip(const int* b, const unsigned* d, int n, int minr, int* out)
{
    constexpr float H = 3.0f;
    float total = 0.0f;
    bool ok = true;
    for (int i = 0; i < n; ++i) {
        const int rows = b[i + 1] - b[i];
        ok = ok && d[i] > 0u && rows > 0;
        total += (float)d[i] * (float)rows / ((float)rows + H);
    }
    out[0] = b[0];
    out[n] = b[n];
    if (!ok) {
        for (int k = 1; k < n; ++k) out[k] = b[k];
        return;
    }
    const float target = total / (float)n;
    int k = 1;
    float acc = 0.0f;
    for (int i = 0; i < n && k < n; ++i) {
        const int rows = b[i + 1] - b[i];
        const float rho = (float)d[i] / ((float)rows + H);
        const float c = rho * (float)rows;
        while (k < n && acc + c >= target * (float)k) {
            const float pos = (float)b[i] + (target * (float)k - acc) / rho;
            int nb = (int)floorf(0.5f * ((float)b[k] + pos) + 0.5f);
            const int lo = out[k - 1] + minr, hi = b[n] - (n - k) * minr;
            out[k] = nb < lo ? lo : (nb > hi ? hi : nb);
            ++k;
        }
        acc += c;
    }
    // boundaries that rounding left unplaced keep their rows
    for (; k < n; ++k) {
        const int lo = out[k - 1] + minr, hi = b[n] - (n - k) * minr;
        out[k] = b[k] < lo ? lo : (b[k] > hi ? hi : b[k]);
    }
}

// Lane `lane` of 1D strip bx on a line of nx cells.  The lane computes
// midpoint jx+1/2, jx = x0-G+lane (G = 2 for MND, 3 for MD, 1 for HWCNS);
// the line needs midpoints -G .. jmax = nx-2+G (jmax+G+1 flag slots).
// Lanes past the last stencil any lane needs read the stencil of that last
// one (in-range data, result unused): jmax, or for HWCNS, whose lanes also
// evaluate the node flux at their stencil node 1 (node jx-1, needed up to
// nx+1), jmax+3.  The lane owns cell c = x0+lane when cell_ok; that cell's
// differences use the midpoints of lanes lane .. lane+2G-1 (and for HWCNS
// the node fluxes of lanes lane, lane+1, lane+3, lane+4), and its own state
// is stencil node G+2.
template <int DIFF>
struct Strip1D {
    static constexpr int W = strip_cells<DIFF>();
    static constexpr int G = DIFF == DIFF_MD ? 3 : (DIFF == DIFF_HW ? 1 : 2);
    int x0, c, jx, jmax, jxl;
    bool cell_ok;
    WCNST_HD Strip1D(int bx, int lane, int nx)
    {
        x0 = bx * W;
        c = x0 + lane;
        cell_ok = lane < W && c < nx;
        jx = x0 - G + lane;
        jmax = nx - 2 + G;
        const int last = DIFF == DIFF_HW ? jmax + 3 : jmax;
        jxl = jx < last ? jx : last;
    }
    // this lane reports the cut flags of its midpoint (each midpoint once)
    WCNST_HD bool owns_face(int bx, int nx) const { return jx <= jmax && face_owner(jx, nx, W) == bx; }
    WCNST_HD int nfaces() const { return jmax + G + 1; }
};

struct Params {
    double CT, C, eps_teno, eps_js;
    double gamma;
    double adv;
    double dx, dy;
    double c1x, c2x, c3x;  // difference coefficients (MND, or MD in 1D) divided by dx
    double c1y, c2y, c3y;  // ... and by dy
    int q, charwise;
    int bc_x, bc_y;
    int nx, ny;
    double fixed_x[2][4];  // fixed ghost states (storage order) at the low / high ends
    double fixed_y[2][4];
    double gravity;        // 2D Euler body force in +y
    double eps_z;          // WCNS-Z epsilon
    double teno_smooth;    // tau / min(beta + eps) below which every TENO candidate is kept
    int z_q;               // WCNS-Z power
};

// Step records of one solve, alternating by step parity: the current
// record holds t, the step count and the CFL speed of the state at t; stage
// 0 of a step writes dt into it and opens the other one.
struct StepRec {
    double t;
    double dt;
    unsigned long long smax_bits;  // max CFL speed of the state at time t (bit pattern)
    long long step;
};

struct Ctrl {
    StepRec rec[2];
    unsigned long long bad_key;  // (global stage << 36) | cell of the first non-physical value
    long long call_step0;        // step counter at the start of the current solve call
    int status;                  // sticky WCNST_E_NONPHYSICAL
    int done;                    // sticky: t_final reached in the current call
    int pad[2];
};

// One grid (1D or 2D) of a multi-grid stage launch: its buffers (U holds
// the state at t^n, U1 / U2 the stage states), control block, parameters,
// and its first block in the launch (blocks blk0 .. blk0 + nstrips*nseg - 1,
// nseg = 1 in 1D).
struct ReqGrid {
    double* U;
    double* U1;
    double* U2;
    Ctrl* ctrl;
    Params P;
    double t_final, cfl;
    int nstrips, blk0;
    int parity0;  // step parity at tick step 0
    int pad;
};

// ------------------------------------------------------------ helpers

// A copy of a table entry.  Tables reach device memory by copies ordered
// before the launch on its stream, so plain loads see them.
template <class T>
__device__ __forceinline__ T load_table_entry(const T* p)
{
    return *p;
}

// Source cell of (ghost) index g on a line of n cells, g in [-n, 2n):
// periodic wrap, mirror image across a reflecting wall (cell-centred: ghost
// -1-k mirrors cell k), else the nearest end cell (zero gradient; a fixed
// ghost ignores the value loaded there).
WCNST_HD int ghost_map(int g, int n, int bc)
{
    if (bc == BC_PERIODIC) {
        g = g < 0 ? g + n : g;
        return g >= n ? g - n : g;
    }
    if (bc == BC_REFLECT) {
        g = g < 0 ? -1 - g : g;
        return g >= n ? 2 * n - 1 - g : g;
    }
    g = g < 0 ? 0 : g;
    return g >= n ? n - 1 : g;
}

// Same map for an index any distance outside [0, n) (periodic wraps as often
// as needed; a mirror image that falls outside again is clamped); used
// where lanes past the last needed column stage data.
WCNST_HD int ghost_map_any(int g, int n, int bc)
{
    if (bc == BC_PERIODIC) return ((g % n) + n) % n;
    if (bc == BC_REFLECT) {
        g = g < 0 ? -1 - g : g;
        g = g >= n ? 2 * n - 1 - g : g;
    }
    g = g < 0 ? 0 : g;
    return g >= n ? n - 1 : g;
}

// What a ghost holds besides its source cell's value: GH_COPY (interior
// cells, periodic, zero gradient), GH_REVERSE (reflecting wall: the normal
// momentum reversed), GH_FIXED_LO / GH_FIXED_HI (the fixed state of that
// end replaces the value).
enum { GH_COPY = 0, GH_REVERSE = 1, GH_FIXED_LO = 2, GH_FIXED_HI = 3 };

WCNST_HD int ghost_kind(int g, int n, int bc)
{
    if (g >= 0 && g < n) return GH_COPY;
    if (bc == BC_REFLECT) return GH_REVERSE;
    if (bc == BC_FIXED) return g < 0 ? GH_FIXED_LO : GH_FIXED_HI;
    return GH_COPY;
}

// Variable v (storage order) of a ghost of kind `kind` whose source cell
// holds `val`; `normal` is the storage index of the momentum normal to the
// boundary, `fixed` the two fixed states of that direction.
WCNST_HD double ghost_value(int kind, int v, int normal, double val, const double (&fixed)[2][4])
{
    // selects, not an index computed from `kind`: the fixed states stay in
    // registers instead of private memory
    if (kind == GH_REVERSE) return v == normal ? -val : val;
    if (kind == GH_FIXED_LO) return fixed[0][v];
    if (kind == GH_FIXED_HI) return fixed[1][v];
    return val;
}

// 1/x for the cut-off test: one Newton step on the hardware estimate
// (about 24 correct bits) leaves a relative error below 3e-15, far inside
// the band where the test is decided by rounding; exact division on the host.
WCNST_HD double approx_rcp(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    const double r = __builtin_amdgcn_rcp(x);
    const double e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
#else
    return 1.0 / x;
#endif
}

// 1/x and sqrt(x) for positive x in [2^-767, 2^1022), where they equal the
// IEEE operations bit for bit.  They are the hardware's own correctly
// rounded sequences (reciprocal estimate, two Newton steps and a residual
// correction; root estimate and Goldschmidt refinement) without the operand
// scaling and the special-value fix-up that the general operations wrap
// around them: in that range neither changes a result.  Callers test their
// arguments with in_ieee_range and redo the work with the IEEE operations
// where a lane's argument lies outside it.
WCNST_HD bool in_ieee_range(double x)
{
    // sign clear and biased exponent in [256, 2044]: one unsigned compare of
    // the high word
    unsigned long long b;
    __builtin_memcpy(&b, &x, sizeof b);
    return (unsigned)(b >> 32) - (256u << 20) < (1789u << 20);
}

WCNST_HD double recip_ranged(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double y = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, y, 1.0);
    y = __builtin_fma(y, e, y);
    e = __builtin_fma(-x, y, 1.0);
    y = __builtin_fma(y, e, y);
    const double r = __builtin_fma(-x, y, 1.0);
    return __builtin_fma(r, y, y);
#else
    return 1.0 / x;
#endif
}

WCNST_HD double sqrt_ranged(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y;
    double h = y * 0.5;
    const double r = __builtin_fma(-h, g, 0.5);
    g = __builtin_fma(g, r, g);
    h = __builtin_fma(h, r, h);
    double d = __builtin_fma(-g, g, x);
    g = __builtin_fma(d, h, g);
    d = __builtin_fma(-g, g, x);
    return __builtin_fma(d, h, g);
#else
    return sqrt(x);
#endif
}

// RANGED selects the sequences above; the caller owns the range test.
template <bool RANGED>
WCNST_HD double recip(double x)
{
    if constexpr (RANGED) return recip_ranged(x);
    else return 1.0 / x;
}

template <bool RANGED>
WCNST_HD double root(double x)
{
    if constexpr (RANGED) return sqrt_ranged(x);
    else return sqrt(x);
}

WCNST_HD double pow_q(double x, int q)
{
    if (q == 6) {
        const double x2 = x * x;
        return x2 * x2 * x2;
    }
    double r = 1.0;
    for (int m = 0; m < q; ++m) r *= x;
    return r;
}

// x^q by q successive multiplications (a value, not only a decision, is
// formed from it, so the order is that of the definition)
WCNST_HD double pow_seq(double x, int q)
{
    double r = 1.0;
    for (int m = 0; m < q; ++m) r *= x;
    return r;
}

// ------------------------------------------------- Sec. 2.2-2.3 interpolation

// Weight of candidate k under cut pattern mask (bit k-1 = delta_k), Eq. (19):
// d_k delta_k / sum_m d_m delta_m with d = (1, 10, 5)/16, written as the
// exact quotient of each pattern.
WCNST_HD double teno_weight(unsigned mask, int k)
{
    const bool k0 = mask & 1u, k1 = mask & 2u, k2 = mask & 4u;
    if (k == 0) return k0 ? (k1 ? (k2 ? 1.0 / 16.0 : 1.0 / 11.0) : (k2 ? 1.0 / 6.0 : 1.0)) : 0.0;
    if (k == 1) return k1 ? (k0 ? (k2 ? 10.0 / 16.0 : 10.0 / 11.0) : (k2 ? 2.0 / 3.0 : 1.0)) : 0.0;
    return k2 ? (k0 ? (k1 ? 5.0 / 16.0 : 5.0 / 6.0) : (k1 ? 1.0 / 3.0 : 1.0)) : 0.0;
}

// The 8 x 3 weights in LDS (one copy per workgroup): three LDS reads per
// interpolation instead of a chain of selects.  Kernels that interpolate
// call init_weight_table() first.
__device__ __forceinline__ double* weight_table()
{
    __shared__ double tab[24];
    return tab;
}

__device__ __forceinline__ void init_weight_table()
{
    if (threadIdx.x < 24) weight_table()[threadIdx.x] = teno_weight(threadIdx.x / 3, threadIdx.x % 3);
    __syncthreads();
}

// One side's interpolated value at x_{i+1/2} from its centre node c and the
// scaled derivatives D1_k = h u'_k, D2_k = h^2 u''_k of its three candidates
// (Eqs. (10)-(11)); mask receives delta_1 | delta_2 << 1 | delta_3 << 2.
template <int SCHEME>
WCNST_HD double interp_side(double c, double D10, double D11, double D12, double D20, double D21, double D22,
                            const Params& P, unsigned& mask)
{
    // candidates, Eq. (9) with Delta x = h/2: u + D1/2 + D2/8
    const double q0 = fma(D20, 0.125, fma(D10, 0.5, c));
    const double q1 = fma(D21, 0.125, fma(D11, 0.5, c));
    const double q2 = fma(D22, 0.125, fma(D12, 0.5, c));
    double w0, w1, w2;
    if constexpr (SCHEME == SCH_LINEAR) {
        mask = 7u;
        w0 = 1.0 / 16.0;
        w1 = 10.0 / 16.0;
        w2 = 5.0 / 16.0;
    } else {
        // Eq. (15)
        const double b0 = fma(D10, D10, D20 * D20);
        const double b1 = fma(D11, D11, D21 * D21);
        const double b2 = fma(D12, D12, D22 * D22);
        if constexpr (SCHEME == SCH_JS) {
            // Eq. (14)
            mask = 7u;
            const double e0 = b0 + P.eps_js, e1 = b1 + P.eps_js, e2 = b2 + P.eps_js;
            const double a0 = (1.0 / 16.0) / (e0 * e0);
            const double a1 = (10.0 / 16.0) / (e1 * e1);
            const double a2 = (5.0 / 16.0) / (e2 * e2);
            const double s = a0 + a1 + a2;
            w0 = a0 / s;
            w1 = a1 / s;
            w2 = a2 / s;
        } else if constexpr (SCHEME == SCH_Z) {
            // Z weights (Borges et al. 2008) with tau_5 of Sec. 2.3:
            // alpha_k = d_k (1 + (tau_5 / (beta_k + eps))^p)
            mask = 7u;
            const double tau = fabs(b0 - b2);
            const double a0 = (1.0 / 16.0) * (1.0 + pow_seq(tau / (b0 + P.eps_z), P.z_q));
            const double a1 = (10.0 / 16.0) * (1.0 + pow_seq(tau / (b1 + P.eps_z), P.z_q));
            const double a2 = (5.0 / 16.0) * (1.0 + pow_seq(tau / (b2 + P.eps_z), P.z_q));
            const double s = a0 + a1 + a2;
            w0 = a0 / s;
            w1 = a1 / s;
            w2 = a2 / s;
        } else {
            // Eq. (16); Eqs. (17)-(18) as gamma_k < C_T * sum(gamma)
            const double tau = fabs(b0 - b2);
            const double e0 = b0 + P.eps_teno, e1 = b1 + P.eps_teno, e2 = b2 + P.eps_teno;
            // Smooth data keep every candidate without the measure: with
            // tau <= t e_min each C + tau/e_k lies in [C, C + t], so
            // chi_k >= C^q / (3 (C + t)^q), which P.teno_smooth (t) keeps
            // above C_T by a margin far beyond rounding.
            mask = 7u;
            if (!(tau <= P.teno_smooth * fmin(fmin(e0, e1), e2))) {
                const int q = SCHEME == SCH_TENO ? 6 : P.q;
                double x0 = fma(tau, approx_rcp(e0), P.C);
                double x1 = fma(tau, approx_rcp(e1), P.C);
                double x2 = fma(tau, approx_rcp(e2), P.C);
                if constexpr (SCHEME == SCH_TENO_Q) {
                    // the test is unchanged when every C + tau/e_k is scaled
                    // by one power of two; scaled by that of the largest, the
                    // powers and their sum stay finite where they would
                    // overflow (q = 8 with eps = 1e-40: tau near 0.03), and
                    // every comparison is decided as unscaled where they
                    // would not.  With q = 6 the powers stay finite while
                    // C + tau/e_k <= 8e50, and the scaling (1.6 % of the 2D
                    // stage) is left out.
                    int ex;
                    (void)frexp(fmax(fmax(x0, x1), x2), &ex);
                    x0 = ldexp(x0, -ex);
                    x1 = ldexp(x1, -ex);
                    x2 = ldexp(x2, -ex);
                }
                const double g0 = pow_q(x0, q);
                const double g1 = pow_q(x1, q);
                const double g2 = pow_q(x2, q);
                const double thr = P.CT * (g0 + g1 + g2);
                const bool k0 = !(g0 < thr), k1 = !(g1 < thr), k2 = !(g2 < thr);
                mask = (unsigned)k0 | ((unsigned)k1 << 1) | ((unsigned)k2 << 2);
            }
            // Eq. (19): d_k delta_k / sum_m d_m delta_m, the exact quotient
            // for each of the seven patterns
#if defined(__HIP_DEVICE_COMPILE__)
            const double* tab = weight_table();
            w0 = tab[mask * 3 + 0];
            w1 = tab[mask * 3 + 1];
            w2 = tab[mask * 3 + 2];
#else
            w0 = teno_weight(mask, 0);
            w1 = teno_weight(mask, 1);
            w2 = teno_weight(mask, 2);
#endif
        }
    }
    // Eq. (12)
    return fma(w2, q2, fma(w1, q1, w0 * q0));
}

// u_L and the mirrored u_R at x_{j+1/2} from the six nodes w0 .. w5 = u_{j-2}
// .. u_{j+3} (u_L from w0 .. w4, u_R from w5 .. w1).  Eqs. (10)-(11) times
// h and h^2 are written with the differences of neighbouring nodes,
// d_m = w_{m+1} - w_m, each formed once for both sides:
//   left:  h u'_1 = (3 d_1 - d_0)/2, h u'_2 = (w_3 - w_1)/2, h u'_3 = (3 d_2 - d_3)/2,
//          h^2 u''_k = (d_1 - d_0, d_2 - d_1, d_3 - d_2);
//   right: the same on the mirrored nodes, whose neighbour differences are
//          -d_4, -d_3, -d_2, -d_1: (d_4 - 3 d_3)/2, (w_2 - w_4)/2,
//          (d_1 - 3 d_2)/2 and (d_4 - d_3, d_3 - d_2, d_2 - d_1).
// Equal nodes give exactly zero differences (tau_5 = 0, every candidate
// kept, as Eqs. (16)-(18) give for constant data), and the second
// differences are shared by the two sides.
template <int SCHEME>
WCNST_HD void interp_pair(double w0, double w1, double w2, double w3, double w4, double w5, const Params& P,
                          double& uL, double& uR, unsigned& mL, unsigned& mR)
{
    const double d0 = w1 - w0, d1 = w2 - w1, d2 = w3 - w2, d3 = w4 - w3, d4 = w5 - w4;
    const double s1 = d1 - d0, s2 = d2 - d1, s3 = d3 - d2, s4 = d4 - d3;
    uL = interp_side<SCHEME>(w2, fma(3.0, d1, -d0) * 0.5, (w3 - w1) * 0.5, fma(3.0, d2, -d3) * 0.5, s1, s2, s3,
                             P, mL);
    uR = interp_side<SCHEME>(w3, fma(-3.0, d3, d4) * 0.5, (w2 - w4) * 0.5, fma(-3.0, d2, d1) * 0.5, s4, s3, s2,
                             P, mR);
}

// ------------------------------------------------------------ Euler

// Ideal gas p = (gamma - 1)(E - |m|^2 / (2 rho)).
template <int NV>
WCNST_HD double pressure(const double* U, double gamma, double ir)
{
    double kin;
    if constexpr (NV == 4) kin = 0.5 * (U[1] * U[1] + U[2] * U[2]) * ir;
    else kin = 0.5 * U[1] * U[1] * ir;
    return (gamma - 1.0) * (U[NV - 1] - kin);
}

// Normal flux (rho u, rho u^2 + p, rho v u, u (E + p)).
template <int NV, bool RANGED = false>
WCNST_HD void euler_flux(const double* U, double gamma, double* F)
{
    const double ir = recip<RANGED>(U[0]);
    const double u = U[1] * ir;
    const double p = pressure<NV>(U, gamma, ir);
    F[0] = U[1];
    F[1] = U[1] * u + p;
    if constexpr (NV == 4) F[2] = U[2] * u;
    F[NV - 1] = u * (U[NV - 1] + p);
}

// Eigen-system of the normal flux Jacobian at the Roe average of A and B
// (normal momentum first).  Fields: u-c, u, [shear], u+c.
//   r_1 = (1, u-c, v, H-uc), r_2 = (1, u, v, q^2/2), r_3 = (0, 0, 1, v),
//   r_4 = (1, u+c, v, H+uc);  with b1 = (gamma-1)/c^2, b2 = b1 q^2/2:
//   l_1 = ( (b2 + u/c)/2, -(b1 u + 1/c)/2, -b1 v/2, b1/2 )
//   l_2 = ( 1 - b2, b1 u, b1 v, -b1 ),  l_3 = ( -v, 0, 1, 0 )
//   l_4 = ( (b2 - u/c)/2, -(b1 u - 1/c)/2, -b1 v/2, b1/2 )
// The 1D system drops the v entries and the shear pair.
template <int NV>
struct Eigen {
    double u, v, H, c, q2, b1, b2, uc, ic;

    // Structural zeros of L and R (the shear pair).  Products are summed
    // over the other entries only, in increasing index order, starting from
    // the first product: the sums equal the full matrix products except,
    // at most, for the sign of a zero result.
    WCNST_HD static constexpr bool L_zero(int k, int j) { return NV == 4 && k == 2 && (j == 1 || j == 3); }
    WCNST_HD static constexpr bool R_zero(int j, int k) { return NV == 4 && k == 2 && (j == 0 || j == 1); }

    // entry (k, j) of L and (j, k) of R, each formed by the same expression
    // wherever it is used
    WCNST_HD double L(int k, int j) const
    {
        if (k == 0) {
            if (j == 0) return 0.5 * (b2 + uc);
            if (j == 1) return -0.5 * (b1 * u + ic);
            if (j == NV - 1) return 0.5 * b1;
            return -0.5 * b1 * v;
        }
        if (k == 1) {
            if (j == 0) return 1.0 - b2;
            if (j == 1) return b1 * u;
            if (j == NV - 1) return -b1;
            return b1 * v;
        }
        if (NV == 4 && k == 2) return j == 0 ? -v : (j == 2 ? 1.0 : 0.0);
        if (j == 0) return 0.5 * (b2 - uc);
        if (j == 1) return -0.5 * (b1 * u - ic);
        if (j == NV - 1) return 0.5 * b1;
        return -0.5 * b1 * v;
    }
    WCNST_HD double R(int j, int k) const
    {
        if (NV == 4 && k == 2) return j == 2 ? 1.0 : (j == 3 ? v : 0.0);
        if (j == 0) return 1.0;
        if (j == NV - 1) return k == 0 ? H - u * c : (k == 1 ? 0.5 * q2 : H + u * c);
        if (j == 1) return k == 0 ? u - c : (k == 1 ? u : u + c);
        return v;
    }
    WCNST_HD double lam(int k) const { return k == 0 ? u - c : (k == NV - 1 ? u + c : u); }
};

// With RANGED the result is exact (equal to the IEEE one) where the return
// value is true: the densities and c^2 lie in [2^-767, 2^1022), and with
// them every other argument of a reciprocal or root.
template <int NV, bool RANGED = false>
WCNST_HD bool roe_eigen(const double* A, const double* B, double gamma, Eigen<NV>& E)
{
    const double rA = A[0], rB = B[0];
    const double irA = recip<RANGED>(rA), irB = recip<RANGED>(rB);
    const double uA = A[1] * irA, uB = B[1] * irB;
    const double vA = NV == 4 ? A[2] * irA : 0.0, vB = NV == 4 ? B[2] * irB : 0.0;
    const double HA = (A[NV - 1] + pressure<NV>(A, gamma, irA)) * irA;
    const double HB = (B[NV - 1] + pressure<NV>(B, gamma, irB)) * irB;
    const double sA = root<RANGED>(rA), sB = root<RANGED>(rB);
    const double is = recip<RANGED>(sA + sB);
    E.u = (sA * uA + sB * uB) * is;
    E.v = (sA * vA + sB * vB) * is;
    E.H = (sA * HA + sB * HB) * is;
    E.q2 = E.u * E.u + E.v * E.v;
    const double c2 = (gamma - 1.0) * (E.H - 0.5 * E.q2);
    E.c = root<RANGED>(c2);
    E.ic = recip<RANGED>(E.c);
    E.b1 = (gamma - 1.0) * (E.ic * E.ic);
    E.b2 = 0.5 * E.q2 * E.b1;
    E.uc = E.u * E.ic;
    return !RANGED || (in_ieee_range(rA) && in_ieee_range(rB) && in_ieee_range(c2));
}

// van Leer's split normal flux (the flux named for the results of Sec. 3;
// textbook form, not printed in the paper): F+ (sign = +1) or F- (sign =
// -1) at U.  Supersonic states give the whole flux to one side; subsonic,
// with M = u/c, f_m = sign rho c (M + sign)^2 / 4, w = (gamma-1) u +
// sign 2c, and F = f_m (1, w/gamma, [v], w^2 / (2 (gamma^2 - 1)) [+ v^2/2]).
template <int NV>
WCNST_HD void vanleer_part(const double* U, double gamma, double sign, double* Fs)
{
    const double ir = 1.0 / U[0];
    const double u = U[1] * ir;
    const double c = sqrt(gamma * pressure<NV>(U, gamma, ir) * ir);
    const double M = u / c;
    if (M >= 1.0 || M <= -1.0) {
        const bool whole = (M >= 1.0) == (sign > 0.0);
        euler_flux<NV>(U, gamma, Fs);
        if (!whole)
#pragma unroll
            for (int k = 0; k < NV; ++k) Fs[k] = 0.0;
        return;
    }
    const double a = M + sign;
    const double fm = sign * (0.25 * U[0] * c * (a * a));
    const double w = (gamma - 1.0) * u + sign * (2.0 * c);
    double e = (w * w) / (2.0 * (gamma * gamma - 1.0));
    Fs[0] = fm;
    Fs[1] = fm * (w / gamma);
    if constexpr (NV == 4) {
        const double v = U[2] * ir;
        Fs[2] = fm * v;
        e = e + 0.5 * (v * v);
    }
    Fs[NV - 1] = fm * e;
}

// Numerical flux of the Euler equations from the interpolated states: the
// system form of Eq. (6), 1/2 [(F(U_R) + F(U_L)) - |A| (U_R - U_L)], with
// |A| = R |Lambda| L at the Roe average of U_L and U_R (no entropy fix), or
// the local Lax-Friedrichs speed max(|u| + c); or van Leer's F+(U_L) +
// F-(U_R).
template <int NV, int FLUX>
WCNST_HD void euler_num_flux(const double* UL, const double* UR, double gamma, double* F)
{
    if constexpr (FLUX == FLUX_VL) {
        double Fp[NV], Fm[NV];
        vanleer_part<NV>(UL, gamma, 1.0, Fp);
        vanleer_part<NV>(UR, gamma, -1.0, Fm);
#pragma unroll
        for (int v = 0; v < NV; ++v) F[v] = Fp[v] + Fm[v];
        return;
    }
    // 1D Roe: the physical fluxes and the Roe average with the ranged
    // reciprocals and roots (1/rho of U_L and U_R shared by both), redone
    // with the IEEE operations on lanes whose arguments leave their range.
    // The 2D kernels keep the IEEE operations here: at their register limit
    // the test's branch costs what the ranged sequences save.
    constexpr bool RG = NV == 3 && FLUX == FLUX_ROE;
    double FL[NV], FR[NV], dis[NV];
    euler_flux<NV, RG>(UL, gamma, FL);
    euler_flux<NV, RG>(UR, gamma, FR);
    if constexpr (FLUX == FLUX_LF) {
        const double irL = 1.0 / UL[0], irR = 1.0 / UR[0];
        const double aL = fabs(UL[1] * irL) + sqrt(gamma * pressure<NV>(UL, gamma, irL) * irL);
        const double aR = fabs(UR[1] * irR) + sqrt(gamma * pressure<NV>(UR, gamma, irR) * irR);
        const double al = fmax(aL, aR);
#pragma unroll
        for (int v = 0; v < NV; ++v) dis[v] = al * (UR[v] - UL[v]);
    } else {
        Eigen<NV> E;
        // (the test covers rho_L and rho_R, the reciprocals' arguments)
        if (!roe_eigen<NV, RG>(UL, UR, gamma, E)) {
            euler_flux<NV>(UL, gamma, FL);
            euler_flux<NV>(UR, gamma, FR);
            roe_eigen<NV>(UL, UR, gamma, E);
        }
        double alpha[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double acc = 0.0;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                if (Eigen<NV>::L_zero(k, v)) continue;
                const double dU = UR[v] - UL[v];
                acc = v == 0 ? E.L(k, v) * dU : fma(E.L(k, v), dU, acc);
            }
            alpha[k] = acc;
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                if (Eigen<NV>::R_zero(v, k)) continue;
                const double rl = E.R(v, k) * fabs(E.lam(k));
                acc = k == 0 ? rl * alpha[k] : fma(rl, alpha[k], acc);
            }
            dis[v] = acc;
        }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) F[v] = 0.5 * ((FR[v] + FL[v]) - dis[v]);
}

// --------------------------------------------------------- midpoint flux

// Stencil accessor: st(m, v) is variable v (normal momentum first) of node
// j-2+m, held in registers.
template <int NV>
struct RegStencil {
    const double (&s)[6][NV];
    WCNST_HD double operator()(int m, int v) const { return s[m][v]; }
};

// Characteristic basis at x_{j+1/2}: the Roe average of nodes j, j+1
// (stencil nodes 2 and 3) by the ranged sequences, and the IEEE operations
// on lanes whose arguments leave their range.
template <int NV, class ST>
WCNST_HD void midpoint_eigen(ST& st, const Params& P, Eigen<NV>& E)
{
    double A[NV], B[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        A[v] = st(2, v);
        B[v] = st(3, v);
    }
    if (!roe_eigen<NV, true>(A, B, P.gamma, E)) roe_eigen<NV>(A, B, P.gamma, E);
}

// Characteristic field k of the six stencil nodes, w_m = l_k . U_m (sums
// over the conserved variables in increasing order, structural zeros
// skipped).
template <int NV, class ST>
WCNST_HD void project_field(ST& st, const Eigen<NV>& E, int k, double (&w)[6])
{
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        double acc = 0.0;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            if (Eigen<NV>::L_zero(k, v)) continue;
            acc = v == 0 ? E.L(k, v) * st(m, v) : fma(E.L(k, v), st(m, v), acc);
        }
        w[m] = acc;
    }
}

// Field k's share of the back-projection U = sum_k r_k w_k (k in increasing
// order; field 0 has no structural zero in R, so it starts every sum).
template <int NV>
WCNST_HD void back_project_field(const Eigen<NV>& E, int k, double wl, double wr, double (&UL)[NV],
                                 double (&UR)[NV])
{
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        if (Eigen<NV>::R_zero(v, k)) continue;
        const double r = E.R(v, k);
        if (k == 0) {
            UL[v] = r * wl;
            UR[v] = r * wr;
        } else {
            UL[v] = fma(r, wl, UL[v]);
            UR[v] = fma(r, wr, UR[v]);
        }
    }
}

// s: nodes j-2 .. j+3 around x_{j+1/2}.  F: flux at x_{j+1/2}.
// fb: 6 flag bits per field (left mask | right mask << 3).
template <int SYS, int NV, int FLUX, int SCHEME, bool CHAR, class ST>
WCNST_HD void face_flux(ST& st, const Params& P, double (&F)[NV], unsigned& fb)
{
    fb = 0u;
    if constexpr (SYS == SYS_EULER) {
        double UL[NV], UR[NV];
        if constexpr (CHAR) {
            Eigen<NV> E;
            midpoint_eigen<NV>(st, P, E);
            // one characteristic field at a time: project, interpolate both
            // sides, and add its share of the back-projection
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                double w[6];
                project_field<NV>(st, E, k, w);
                unsigned mL, mR;
                double wl, wr;
                interp_pair<SCHEME>(w[0], w[1], w[2], w[3], w[4], w[5], P, wl, wr, mL, mR);
                fb |= (mL | (mR << 3)) << (6 * k);
                back_project_field<NV>(E, k, wl, wr, UL, UR);
            }
        } else {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                unsigned mL, mR;
                interp_pair<SCHEME>(st(0, v), st(1, v), st(2, v), st(3, v), st(4, v), st(5, v), P, UL[v], UR[v], mL,
                                    mR);
                fb |= (mL | (mR << 3)) << (6 * v);
            }
        }
        euler_num_flux<NV, FLUX>(UL, UR, P.gamma, F);
    } else {
        unsigned mL, mR;
        double uL, uR;
        interp_pair<SCHEME>(st(0, 0), st(1, 0), st(2, 0), st(3, 0), st(4, 0), st(5, 0), P, uL, uR, mL, mR);
        fb = mL | (mR << 3);
        if constexpr (SYS == SYS_ADV) {
            // Eq. (6) with f = a u, a_hat = a
            const double a = P.adv;
            F[0] = 0.5 * ((a * uR + a * uL) - fabs(a) * (uR - uL));
        } else {
            // Eq. (6) with f = u^2 / 2; a_hat = Roe speed or local max |u|
            const double fl = 0.5 * uL * uL, fr = 0.5 * uR * uR;
            const double ah = FLUX == FLUX_LF ? fmax(fabs(uL), fabs(uR)) : 0.5 * (uL + uR);
            F[0] = 0.5 * ((fr + fl) - fabs(ah) * (uR - uL));
        }
    }
}

template <int SYS, int NV>
WCNST_HD void node_flux(const double* U, const Params& P, double* F)
{
    if constexpr (SYS == SYS_EULER) {
        if constexpr (NV == 3) {
            // 1D: 1/rho by the ranged sequence, the IEEE division where rho
            // leaves its range
            euler_flux<NV, true>(U, P.gamma, F);
            if (!in_ieee_range(U[0])) euler_flux<NV>(U, P.gamma, F);
        } else {
            euler_flux<NV>(U, P.gamma, F);
        }
    } else if constexpr (SYS == SYS_ADV) F[0] = P.adv * U[0];
    else F[0] = 0.5 * U[0] * U[0];
}

// CFL denominator contribution of one cell: (|u| + c)/dx [+ (|v| + c)/dy].
template <int SYS, int NV>
WCNST_HD double cell_speed(const double* U, const Params& P)
{
    if constexpr (SYS == SYS_ADV) return fabs(P.adv) / P.dx;
    else if constexpr (SYS == SYS_BURG) return fabs(U[0]) / P.dx;
    else {
        const double ir = 1.0 / U[0];
        const double a = sqrt(P.gamma * pressure<NV>(U, P.gamma, ir) * ir);
        double s = (fabs(U[1] * ir) + a) / P.dx;
        if constexpr (NV == 4) s = s + (fabs(U[2] * ir) + a) / P.dy;
        return s;
    }
}

// Non-physical check of a stage output.
template <int SYS, int NV>
WCNST_HD bool cell_bad(const double* U, const Params& P)
{
    bool bad = false;
#pragma unroll
    for (int v = 0; v < NV; ++v) bad |= !isfinite(U[v]);
    if constexpr (SYS == SYS_EULER) bad |= !(U[0] > 0.0) || !(pressure<NV>(U, P.gamma, 1.0 / U[0]) > 0.0);
    return bad;
}

// Stage update in the Shu-Osher form of SSP-RK3.
template <int NV>
WCNST_HD void rk_combine(int stage, double dt, const double* Uk, const double* Un, const double* R,
                         double* o)
{
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        if (stage == 0) o[v] = Uk[v] + dt * R[v];
        else if (stage == 1) o[v] = 0.75 * Un[v] + 0.25 * (Uk[v] + dt * R[v]);
        else o[v] = (1.0 / 3.0) * Un[v] + (2.0 / 3.0) * (Uk[v] + dt * R[v]);
    }
}

// MD difference, Eq. (3): -(a1 (F_{i+1/2} - F_{i-1/2}) + a2 (F_{i+3/2} - F_{i-3/2})
// + a3 (F_{i+5/2} - F_{i-5/2})) with a_k already divided by h.
WCNST_HD double md(double a1, double a2, double a3, double Fm5, double Fm3, double Fm1, double Fp1, double Fp3,
                   double Fp5)
{
    const double dfdx = a1 * (Fp1 - Fm1) + a2 * (Fp3 - Fm3) + a3 * (Fp5 - Fm5);
    return -dfdx;
}

// HWCNS difference, Eq. (4): -(b1 (F_{i+1/2} - F_{i-1/2}) + b2 (f_{i+1} - f_{i-1})
// + b3 (f_{i+2} - f_{i-2})) with b_k already divided by h.
WCNST_HD double hwcns(double b1, double b2, double b3, double Fm1, double Fp1, double fm2, double fm1, double fp1,
                      double fp2)
{
    const double dfdx = b1 * (Fp1 - Fm1) + b2 * (fp1 - fm1) + b3 * (fp2 - fm2);
    return -dfdx;
}

// MND difference, Eq. (5): -(c1 (F_{i+1/2} - F_{i-1/2}) + c2 (f_{i+1} - f_{i-1})
// + c3 (F_{i+3/2} - F_{i-3/2})) with c_k already divided by h.
WCNST_HD double mnd(double c1, double c2, double c3, double Fm3, double Fm1, double Fp1, double Fp3,
                    double fm, double fp)
{
    const double dfdx = c1 * (Fp1 - Fm1) + c2 * (fp - fm) + c3 * (Fp3 - Fm3);
    return -dfdx;
}

}  // namespace wcnst

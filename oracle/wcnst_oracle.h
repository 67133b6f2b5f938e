/*
 * Plain FP64 CPU oracle for the WCNS-T (TCNS) right-hand side and SSP-RK3
 * time stepping of Zhang, Zhang & Xu, "Towards optimal high-order compact
 * schemes for simulating compressible flows" (arXiv:1810.07806).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or helper with the HIP path: it is the independent
 * reference the HIP path is checked against.
 *
 * Layout conventions (shared with the HIP path only by specification):
 *   U[v][y][x], x fastest, FP64, v = 0..nvar-1.
 *   Euler 1D: (rho, rho*u, E).  Euler 2D: (rho, rho*u, rho*v, E).
 *   Scalar systems: nvar = 1.
 *   Flags of direction d: [nvar][lines][nfaces][2] bytes, side 0 = left
 *   state u_L, side 1 = right state u_R; bit k-1 holds delta_k.
 *   Face slot s corresponds to face j+1/2 with j = s - 2 (MND) or s - 3 (MD).
 *   chi of direction d: [nvar][lines][nfaces][2][3] doubles.
 *   In 2D the x-direction block comes first, then the y-direction block
 *   (lines = ny for x, nx for y).
 */
#ifndef WCNST_ORACLE_H
#define WCNST_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_ADVECTION = 0, ORC_BURGERS = 1, ORC_EULER = 2 };
enum { ORC_PERIODIC = 0, ORC_ZERO_GRADIENT = 1, ORC_REFLECT = 2, ORC_FIXED = 3 };
enum { ORC_ROE = 0, ORC_LF = 1, ORC_VANLEER = 2 };
enum { ORC_TENO = 0, ORC_LINEAR = 1, ORC_JS = 2, ORC_Z = 3 };
enum { ORC_MND = 0, ORC_MD = 1, ORC_HWCNS = 2 };

enum {
    ORC_OK = 0,
    ORC_E_INVALID = 1,
    ORC_E_NONPHYSICAL = 2,
    ORC_E_MAX_STEPS = 3
};

typedef struct orc_problem {
    int ndim;        /* 1 or 2 */
    int system;      /* ORC_ADVECTION / ORC_BURGERS / ORC_EULER */
    int nx, ny;      /* unknowns per direction (ny = 1 in 1D) */
    double dx, dy;   /* uniform spacing h per direction */
    int bc_x, bc_y;  /* ORC_PERIODIC / ORC_ZERO_GRADIENT / ORC_REFLECT (Euler) / ORC_FIXED */
    int flux;        /* ORC_ROE / ORC_LF / ORC_VANLEER (Euler only) */
    int scheme;      /* ORC_TENO / ORC_LINEAR / ORC_JS / ORC_Z */
    int diff;        /* ORC_MND / ORC_MD / ORC_HWCNS */
    int charwise;    /* Euler: 1 = interpolate characteristic variables */
    int q;           /* TENO integer power (6) */
    double gamma;    /* ratio of specific heats */
    double adv_speed;/* advection speed a */
    double CT;       /* TENO cut-off (1e-5) */
    double C;        /* TENO constant (1) */
    double eps_teno; /* TENO epsilon (1e-40) */
    double eps_js;   /* Jiang-Shu epsilon (1e-6) */
    /* ORC_FIXED ghost states, conserved variables in storage order (rho,
     * rho u, [rho v], E), at the low / high end of each direction */
    double fixed_x[2][4];
    double fixed_y[2][4];
    double gravity;  /* 2D Euler: source (0, 0, rho g, rho v g) added to R */
    int z_q;         /* ORC_Z: power p of the Z weights */
    double eps_z;    /* ORC_Z: epsilon of the Z weights */
} orc_problem;

int orc_nvar(const orc_problem* p);
int orc_nfaces(const orc_problem* p, int n);
int64_t orc_flag_count(const orc_problem* p);

/* Node-to-midpoint interpolation of u_L at x_{i+1/2} from s = (u_{i-2} ..
 * u_{i+2}).  chi[3] / delta[3] may be NULL. */
double orc_interp_left(const orc_problem* p, const double s[5],
                       double chi[3], int delta[3]);

/* The three candidate interpolants u_{L,k} and smoothness indicators
 * beta_k of one 5-point stencil. */
void orc_candidates(const double s[5], double cand[3], double beta[3]);

/* Roe-averaged eigen-system of two Euler states (normal component first):
 * L and R are nv x nv row-major, lam has nv entries.  Returns 0, or 1 when
 * the averaged sound speed is not real and positive. */
int orc_roe_eigen(int nv, double gamma, const double* UA, const double* UB,
                  double* L, double* R, double* lam);

void orc_euler_flux(int nv, double gamma, const double* U, double* F);

/* Numerical flux at one midpoint from the interpolated states. */
void orc_num_flux(const orc_problem* p, const double* UL, const double* UR,
                  double* F);

/* Full discrete right-hand side R = -(dF/dx [+ dG/dy]).  flags / chi may be
 * NULL.  Returns ORC_OK or ORC_E_INVALID. */
int orc_rhs(const orc_problem* p, const double* U, double* R, uint8_t* flags,
            double* chi, int nthreads);

/* Largest wave speed divided by the spacing (the CFL denominator). */
double orc_max_speed(const orc_problem* p, const double* U);

/* One SSP-RK3 step in place.  stage_base is the global stage counter of the
 * first stage (3 * step).  On a non-physical stage output returns
 * ORC_E_NONPHYSICAL with *bad_stage / *bad_cell set. */
int orc_rk3_step(const orc_problem* p, double* U, double dt, int64_t stage_base,
                 int64_t* bad_stage, int64_t* bad_cell, int nthreads);

/* Advance from t0 until t_final (pass +inf for fixed step counts) or
 * max_steps.  dt = cfl / max_speed(U^n), clipped at t_final. */
int orc_solve(const orc_problem* p, double* U, double t0, double t_final,
              double cfl, int64_t max_steps, double* t_out, int64_t* steps_out,
              int64_t* bad_stage, int64_t* bad_cell, int nthreads);

#ifdef __cplusplus
}
#endif

#endif

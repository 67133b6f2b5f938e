/*
 * Plain FP64 CPU oracle for WCNS-T (TCNS), arXiv:1810.07806.
 *
 * TEST INFRASTRUCTURE ONLY: the reference the HIP path is checked against.
 * Only tests, the smoke check and the benchmark's CPU-baseline leg load it.
 * It shares no code with the HIP path.  Built with -O2 -ffp-contract=off and
 * no fast-math so every operation is rounded as written, in the order the
 * paper writes it; the interpolation, the characteristic projections and
 * the Roe dissipation round each product-plus-sum once, written out as
 * ORC_FMA(a, b, c) = fma(a, b, c).  Built with -DORC_PLAIN the same macro is
 * the plain a * b + c (two roundings): the tests require the two builds to
 * agree within the parity tolerances on every right-hand-side case, so the
 * single rounding is a choice of evaluation order, not a different method.
 * The arithmetic of this file is frozen: a change of evaluation order in the
 * HIP kernels is checked against it at the stated tolerances, not followed
 * here.
 *
 * The steps and where they come from:
 *   semi-discretisation du_i/dt = -f'_i ........... Sec. 2, Eq. (2)
 *   SSP-RK3 (Shu-Osher form) ...................... Sec. 2 (cites Gottlieb et al. 2001)
 *   MND / MD / HWCNS flux differences ............. Sec. 2.1, Eqs. (5), (3), (4)
 *   scalar upwind midpoint flux ................... Sec. 2.2, Eq. (6)
 *   candidate interpolants, derivatives ........... Sec. 2.2, Eqs. (9)-(11)
 *   optimal linear weights d_k .................... Sec. 2.2, Eq. (13)
 *   Jiang-Shu weights / smoothness indicator ...... Sec. 2.2, Eqs. (14)-(15)
 *   WCNS-Z weights (Sec. 3's comparison scheme) ... Borges, Carmona, Costa &
 *                                                   Don (2008), with the global
 *                                                   indicator tau_5 of Sec. 2.3
 *   TENO measure, normalisation, cut-off, weights . Sec. 2.3, Eqs. (16)-(19)
 *   characteristic-wise interpolation, ideal gas .. Sec. 3 (opening paragraph)
 *   Roe flux-difference splitting ................. Sec. 1 (named); the system
 *                                                   form of Eq. (6) with |A| = R|Lambda|L
 *   van Leer flux-vector splitting ................ Sec. 3 (named as the flux of
 *                                                   the paper's results; textbook form)
 * The paper does not print the difference coefficients, the Runge-Kutta
 * form, the Roe average or the eigenvectors; the readings used here are:
 *   MND: (c1, c2, c3) = (3/2, -3/10, 1/30); MD: (75/64, -25/384, 3/640);
 *        HWCNS: (b1, b2, b3) = (64/45, -2/9, 1/180), the unique sixth-order
 *        solutions of the Taylor conditions.
 *   h cancels in beta_k (Eq. (15)) and in the candidates (Eq. (9)); the
 *        scaled differences D1 = h u^(1), D2 = h^2 u^(2) are used directly.
 *   delta_k = 1 when chi_k == C_T ("otherwise" branch of Eq. (18)).
 *   Characteristic projection uses the Roe average of the two nodes next to
 *   the midpoint and the textbook conserved-variable eigenvectors.
 *   No entropy fix in the Roe flux (Eq. (6) uses the plain |a|).
 *   van Leer: F = F+(U_L) + F-(U_R) on the interpolated states, the
 *        subsonic parts with mass flux +-rho c (M +- 1)^2 / 4.
 */
#include "wcnst_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define GHOST 5

/* One product-plus-sum (see the header comment). */
#ifdef ORC_PLAIN
#define ORC_FMA(a, b, c) ((a) * (b) + (c))
#else
#define ORC_FMA(a, b, c) fma((a), (b), (c))
#endif

/* ---------------------------------------------------------------- sizes */

int orc_nvar(const orc_problem* p)
{
    if (p->system == ORC_EULER) return p->ndim == 1 ? 3 : 4;
    return 1;
}

static int first_face(const orc_problem* p) { return p->diff == ORC_MD ? -3 : (p->diff == ORC_HWCNS ? -1 : -2); }

int orc_nfaces(const orc_problem* p, int n) { return p->diff == ORC_MD ? n + 5 : (p->diff == ORC_HWCNS ? n + 1 : n + 3); }

int64_t orc_flag_count(const orc_problem* p)
{
    int64_t nv = orc_nvar(p);
    int64_t c = nv * (int64_t)p->ny * orc_nfaces(p, p->nx) * 2;
    if (p->ndim == 2) c += nv * (int64_t)p->nx * orc_nfaces(p, p->ny) * 2;
    return c;
}

static int validate(const orc_problem* p)
{
    if (p->ndim != 1 && p->ndim != 2) return ORC_E_INVALID;
    if (p->ndim == 2 && p->system != ORC_EULER) return ORC_E_INVALID;
    if (p->nx < 5 || p->ny < 1) return ORC_E_INVALID;
    if (p->ndim == 1 && p->ny != 1) return ORC_E_INVALID;
    if (p->ndim == 2 && p->ny < 5) return ORC_E_INVALID;
    if (!(p->dx > 0) || (p->ndim == 2 && !(p->dy > 0))) return ORC_E_INVALID;
    if (p->system == ORC_EULER && !(p->gamma > 1)) return ORC_E_INVALID;
    if (p->q < 1) return ORC_E_INVALID;
    if (p->scheme == ORC_Z && (p->z_q < 1 || !(p->eps_z > 0))) return ORC_E_INVALID;
    if (p->flux == ORC_VANLEER && p->system != ORC_EULER) return ORC_E_INVALID;
    if ((p->bc_x == ORC_REFLECT || p->bc_y == ORC_REFLECT) && p->system != ORC_EULER) return ORC_E_INVALID;
    if (p->gravity != 0.0 && p->ndim != 2) return ORC_E_INVALID;
    return ORC_OK;
}

/* ------------------------------------------- Sec. 2.2-2.3 interpolation */

/* Optimal linear weights, Eq. (13). */
static const double D_OPT[3] = {1.0 / 16.0, 10.0 / 16.0, 5.0 / 16.0};

void orc_candidates(const double s[5], double cand[3], double beta[3])
{
    const double c = s[2];
    double t[4], D1[3], D2[3];
    /* Eq. (10) times h and Eq. (11) times h^2, on the substencils of Eq. (8),
     * written with the differences of neighbouring nodes t_m = s_{m+1} - s_m:
     *   h u'_1 = (3 t_1 - t_0)/2,  h u'_2 = (s_3 - s_1)/2,  h u'_3 = (3 t_2 - t_3)/2,
     *   h^2 u''_k = t_k - t_{k-1}  (k = 1, 2, 3 on t_0 .. t_3).
     * A stencil of equal values then gives exactly zero differences, so
     * tau_5 = 0 and every candidate is kept, as Eqs. (16)-(18) prescribe
     * for constant data; and a second difference has the same value
     * whichever end its three nodes are read from.  Each 3 t_1 - t_0 is one
     * ORC_FMA. */
    for (int m = 0; m < 4; ++m) t[m] = s[m + 1] - s[m];
    D1[0] = ORC_FMA(3.0, t[1], -t[0]) / 2.0;
    D1[1] = (s[3] - s[1]) / 2.0;
    D1[2] = ORC_FMA(3.0, t[2], -t[3]) / 2.0;
    D2[0] = t[1] - t[0];
    D2[1] = t[2] - t[1];
    D2[2] = t[3] - t[2];
    for (int k = 0; k < 3; ++k) {
        /* Eq. (9) with Delta x = h/2: u_i + u' h/2 + u'' h^2/8. */
        cand[k] = ORC_FMA(D2[k], 1.0 / 8.0, ORC_FMA(D1[k], 1.0 / 2.0, c));
        /* Eq. (15). */
        beta[k] = ORC_FMA(D1[k], D1[k], D2[k] * D2[k]);
    }
}

double orc_interp_left(const orc_problem* p, const double s[5], double chi[3],
                       int delta[3])
{
    double cand[3], beta[3], w[3];
    double chi_l[3] = {0, 0, 0};
    int del_l[3] = {1, 1, 1};
    orc_candidates(s, cand, beta);

    if (p->scheme == ORC_LINEAR) {
        /* Eq. (12): the optimal linear scheme. */
        for (int k = 0; k < 3; ++k) { w[k] = D_OPT[k]; chi_l[k] = D_OPT[k]; }
    } else if (p->scheme == ORC_JS) {
        /* Eq. (14). */
        double alpha[3], sum;
        for (int k = 0; k < 3; ++k) {
            double be = beta[k] + p->eps_js;
            alpha[k] = D_OPT[k] / (be * be);
        }
        sum = alpha[0] + alpha[1] + alpha[2];
        for (int k = 0; k < 3; ++k) { w[k] = alpha[k] / sum; chi_l[k] = w[k]; }
    } else if (p->scheme == ORC_Z) {
        /* Z weights of Borges et al. (2008) on the indicators of Eq. (15):
         * alpha_k = d_k (1 + (tau5 / (beta_k + eps))^p), omega = alpha / sum. */
        double alpha[3], sum;
        double tau5 = fabs(beta[0] - beta[2]);
        for (int k = 0; k < 3; ++k) {
            double x = tau5 / (beta[k] + p->eps_z), xp = 1.0;
            for (int m = 0; m < p->z_q; ++m) xp *= x;
            alpha[k] = D_OPT[k] * (1.0 + xp);
        }
        sum = alpha[0] + alpha[1] + alpha[2];
        for (int k = 0; k < 3; ++k) { w[k] = alpha[k] / sum; chi_l[k] = w[k]; }
    } else {
        /* Eq. (16): gamma_k = (C + tau5 / (beta_k + eps))^q, tau5 = |beta_1 - beta_3|.
         * chi_k of Eq. (17) is a ratio of the gammas, unchanged when every
         * C + tau5 / (beta_k + eps) is divided by the same power of two.
         * Dividing by the power of two of the largest keeps the gammas and
         * their sum finite where the plain powers overflow (with eps = 1e-40
         * two candidates with beta_k = 0 reach 1e308 at q = 8 for tau5 near
         * 0.03), and changes no bit of any chi where they do not: scaling by
         * a power of two commutes with rounding in the normal range. */
        double x[3], g[3], gsum, dsum, xm;
        int ex = 0;
        double tau5 = fabs(beta[0] - beta[2]);
        for (int k = 0; k < 3; ++k) x[k] = p->C + tau5 / (beta[k] + p->eps_teno);
        xm = fmax(fmax(x[0], x[1]), x[2]);
        if (isfinite(xm)) (void)frexp(xm, &ex);
        for (int k = 0; k < 3; ++k) {
            double xs = ldexp(x[k], -ex);
            g[k] = 1.0;
            for (int m = 0; m < p->q; ++m) g[k] *= xs;
        }
        /* Eq. (17). */
        gsum = g[0] + g[1] + g[2];
        for (int k = 0; k < 3; ++k) chi_l[k] = g[k] / gsum;
        /* Eq. (18): discard when chi_k < C_T, keep otherwise. */
        for (int k = 0; k < 3; ++k) del_l[k] = (chi_l[k] < p->CT) ? 0 : 1;
        /* Eq. (19). */
        dsum = D_OPT[0] * del_l[0] + D_OPT[1] * del_l[1] + D_OPT[2] * del_l[2];
        for (int k = 0; k < 3; ++k) w[k] = D_OPT[k] * del_l[k] / dsum;
    }
    if (chi) for (int k = 0; k < 3; ++k) chi[k] = chi_l[k];
    if (delta) for (int k = 0; k < 3; ++k) delta[k] = del_l[k];
    /* Eq. (12) with the (possibly nonlinear) weights. */
    return ORC_FMA(w[2], cand[2], ORC_FMA(w[1], cand[1], w[0] * cand[0]));
}

/* ------------------------------------------------------- Euler system */

/* Ideal gas p = (gamma - 1) rho e, with rho e = E - kinetic energy; ir is
 * 1 / rho.  Every divisor shared by several terms is inverted once and the
 * terms multiply by its reciprocal (the paper fixes no evaluation order for
 * the flux, the Roe average or the eigenvectors). */
static double euler_pressure_r(int nv, double gamma, const double* U, double ir)
{
    double kin;
    if (nv == 4) kin = 0.5 * (U[1] * U[1] + U[2] * U[2]) * ir;
    else kin = 0.5 * U[1] * U[1] * ir;
    return (gamma - 1.0) * (U[nv - 1] - kin);
}

static double euler_pressure(int nv, double gamma, const double* U)
{
    return euler_pressure_r(nv, gamma, U, 1.0 / U[0]);
}

void orc_euler_flux(int nv, double gamma, const double* U, double* F)
{
    double ir = 1.0 / U[0];
    double u = U[1] * ir;
    double p = euler_pressure_r(nv, gamma, U, ir);
    F[0] = U[1];
    F[1] = U[1] * u + p;
    if (nv == 4) F[2] = U[2] * u;
    F[nv - 1] = u * (U[nv - 1] + p);
}

int orc_roe_eigen(int nv, double gamma, const double* UA, const double* UB,
                  double* L, double* R, double* lam)
{
    double rA = UA[0], rB = UB[0];
    double irA = 1.0 / rA, irB = 1.0 / rB;
    double uA = UA[1] * irA, uB = UB[1] * irB;
    double vA = nv == 4 ? UA[2] * irA : 0.0, vB = nv == 4 ? UB[2] * irB : 0.0;
    double HA = (UA[nv - 1] + euler_pressure_r(nv, gamma, UA, irA)) * irA;
    double HB = (UB[nv - 1] + euler_pressure_r(nv, gamma, UB, irB)) * irB;
    double sA = sqrt(rA), sB = sqrt(rB);
    double is = 1.0 / (sA + sB);
    double u = (sA * uA + sB * uB) * is;
    double v = (sA * vA + sB * vB) * is;
    double H = (sA * HA + sB * HB) * is;
    double q2 = u * u + v * v;
    double c2 = (gamma - 1.0) * (H - 0.5 * q2);
    double c = sqrt(c2);
    double ic = 1.0 / c;
    double b1 = (gamma - 1.0) * (ic * ic);
    double b2 = 0.5 * q2 * b1;
    double uc = u * ic;
    int bad = !(c2 > 0.0);

    if (nv == 3) {
        /* columns r_k: (1, u-c, H-uc), (1, u, q2/2), (1, u+c, H+uc) */
        double Rm[9] = {1.0, 1.0, 1.0,
                        u - c, u, u + c,
                        H - u * c, 0.5 * q2, H + u * c};
        double Lm[9] = {0.5 * (b2 + uc), -0.5 * (b1 * u + ic), 0.5 * b1,
                        1.0 - b2, b1 * u, -b1,
                        0.5 * (b2 - uc), -0.5 * (b1 * u - ic), 0.5 * b1};
        memcpy(R, Rm, sizeof Rm);
        memcpy(L, Lm, sizeof Lm);
        lam[0] = u - c; lam[1] = u; lam[2] = u + c;
    } else {
        /* columns: acoustic -, entropy, shear, acoustic + */
        double Rm[16] = {1.0, 1.0, 0.0, 1.0,
                         u - c, u, 0.0, u + c,
                         v, v, 1.0, v,
                         H - u * c, 0.5 * q2, v, H + u * c};
        double Lm[16] = {0.5 * (b2 + uc), -0.5 * (b1 * u + ic), -0.5 * b1 * v, 0.5 * b1,
                         1.0 - b2, b1 * u, b1 * v, -b1,
                         -v, 0.0, 1.0, 0.0,
                         0.5 * (b2 - uc), -0.5 * (b1 * u - ic), -0.5 * b1 * v, 0.5 * b1};
        memcpy(R, Rm, sizeof Rm);
        memcpy(L, Lm, sizeof Lm);
        lam[0] = u - c; lam[1] = u; lam[2] = u; lam[3] = u + c;
    }
    return bad;
}

static double sound_speed(int nv, double gamma, const double* U)
{
    double ir = 1.0 / U[0];
    return sqrt(gamma * euler_pressure_r(nv, gamma, U, ir) * ir);
}

/* van Leer's split flux F+ (sign = +1) or F- (sign = -1) of the normal flux
 * at U (normal momentum first).  Supersonic states give the whole flux to
 * one side; subsonic, with M = u/c,
 *   f_m = sign rho c (M + sign)^2 / 4,  w = (gamma - 1) u + sign 2 c,
 *   F = f_m (1, w / gamma, [v], w^2 / (2 (gamma^2 - 1)) [+ v^2 / 2]). */
static void vanleer_part(int nv, double gamma, const double* U, double sign, double* Fs)
{
    double ir = 1.0 / U[0];
    double u = U[1] * ir;
    double c = sqrt(gamma * euler_pressure_r(nv, gamma, U, ir) * ir);
    double M = u / c;
    if (M >= 1.0 || M <= -1.0) {
        int whole = (M >= 1.0) == (sign > 0.0);
        orc_euler_flux(nv, gamma, U, Fs);
        if (!whole)
            for (int k = 0; k < nv; ++k) Fs[k] = 0.0;
        return;
    }
    double a = M + sign;
    double fm = sign * (0.25 * U[0] * c * (a * a));
    double w = (gamma - 1.0) * u + sign * (2.0 * c);
    double e = (w * w) / (2.0 * (gamma * gamma - 1.0));
    Fs[0] = fm;
    Fs[1] = fm * (w / gamma);
    if (nv == 4) {
        double v = U[2] * ir;
        Fs[2] = fm * v;
        e = e + 0.5 * (v * v);
    }
    Fs[nv - 1] = fm * e;
}

void orc_num_flux(const orc_problem* p, const double* UL, const double* UR, double* F)
{
    if (p->system == ORC_ADVECTION) {
        /* Eq. (6) with f(u) = a u and a_hat = a. */
        double a = p->adv_speed;
        F[0] = 0.5 * ((a * UR[0] + a * UL[0]) - fabs(a) * (UR[0] - UL[0]));
        return;
    }
    if (p->system == ORC_BURGERS) {
        /* Eq. (6) with f(u) = u^2/2; a_hat is the Roe speed (u_L + u_R)/2, or
         * the local maximum |u| for Lax-Friedrichs. */
        double fl = 0.5 * UL[0] * UL[0], fr = 0.5 * UR[0] * UR[0];
        double ah = p->flux == ORC_LF ? fmax(fabs(UL[0]), fabs(UR[0]))
                                      : 0.5 * (UL[0] + UR[0]);
        F[0] = 0.5 * ((fr + fl) - fabs(ah) * (UR[0] - UL[0]));
        return;
    }
    if (p->flux == ORC_VANLEER) {
        int nv = orc_nvar(p);
        double Fp[4], Fm[4];
        vanleer_part(nv, p->gamma, UL, 1.0, Fp);
        vanleer_part(nv, p->gamma, UR, -1.0, Fm);
        for (int v = 0; v < nv; ++v) F[v] = Fp[v] + Fm[v];
        return;
    }
    {
        int nv = orc_nvar(p);
        double FL[4], FR[4], dis[4];
        orc_euler_flux(nv, p->gamma, UL, FL);
        orc_euler_flux(nv, p->gamma, UR, FR);
        if (p->flux == ORC_LF) {
            double aL = fabs(UL[1] * (1.0 / UL[0])) + sound_speed(nv, p->gamma, UL);
            double aR = fabs(UR[1] * (1.0 / UR[0])) + sound_speed(nv, p->gamma, UR);
            double al = fmax(aL, aR);
            for (int v = 0; v < nv; ++v) dis[v] = al * (UR[v] - UL[v]);
        } else {
            /* |A_hat| (U_R - U_L) = R |Lambda| L (U_R - U_L), Roe average of U_L, U_R. */
            double L[16], R[16], lam[4], alpha[4];
            orc_roe_eigen(nv, p->gamma, UL, UR, L, R, lam);
            for (int k = 0; k < nv; ++k) {
                alpha[k] = 0.0;
                for (int v = 0; v < nv; ++v) alpha[k] = ORC_FMA(L[k * nv + v], UR[v] - UL[v], alpha[k]);
            }
            for (int v = 0; v < nv; ++v) {
                dis[v] = 0.0;
                for (int k = 0; k < nv; ++k) dis[v] = ORC_FMA(R[v * nv + k] * fabs(lam[k]), alpha[k], dis[v]);
            }
        }
        for (int v = 0; v < nv; ++v) F[v] = 0.5 * ((FR[v] + FL[v]) - dis[v]);
    }
}

static void phys_flux(const orc_problem* p, const double* U, double* F)
{
    if (p->system == ORC_ADVECTION) F[0] = p->adv_speed * U[0];
    else if (p->system == ORC_BURGERS) F[0] = 0.5 * U[0] * U[0];
    else orc_euler_flux(orc_nvar(p), p->gamma, U, F);
}

/* ----------------------------------------------------- one midpoint flux */

/* st holds the six nodes j-2 .. j+3 around the midpoint x_{j+1/2}, node-major.
 * fl[v*2 + side] / ch[(v*2 + side)*3 + k] receive the cut flags / chi. */
static void midpoint_flux(const orc_problem* p, int nv, const double* st, double* F,
                          uint8_t* fl, double* ch)
{
    double W[6][4], wL[4], wR[4], UL[4], UR[4];
    double L[16], R[16], lam[4];
    int charwise = p->system == ORC_EULER && p->charwise;

    if (charwise) {
        orc_roe_eigen(nv, p->gamma, st + 2 * nv, st + 3 * nv, L, R, lam);
        for (int m = 0; m < 6; ++m)
            for (int k = 0; k < nv; ++k) {
                double acc = 0.0;
                for (int v = 0; v < nv; ++v) acc = ORC_FMA(L[k * nv + v], st[m * nv + v], acc);
                W[m][k] = acc;
            }
    } else {
        for (int m = 0; m < 6; ++m)
            for (int k = 0; k < nv; ++k) W[m][k] = st[m * nv + k];
    }
    for (int k = 0; k < nv; ++k) {
        double sl[5] = {W[0][k], W[1][k], W[2][k], W[3][k], W[4][k]};
        /* mirror image for the right state (Sec. 2.2: "symmetrical form") */
        double sr[5] = {W[5][k], W[4][k], W[3][k], W[2][k], W[1][k]};
        double chl[3], chr[3];
        int dl[3], dr[3];
        wL[k] = orc_interp_left(p, sl, chl, dl);
        wR[k] = orc_interp_left(p, sr, chr, dr);
        if (fl) {
            fl[k * 2 + 0] = (uint8_t)(dl[0] | (dl[1] << 1) | (dl[2] << 2));
            fl[k * 2 + 1] = (uint8_t)(dr[0] | (dr[1] << 1) | (dr[2] << 2));
        }
        if (ch)
            for (int m = 0; m < 3; ++m) {
                ch[(k * 2 + 0) * 3 + m] = chl[m];
                ch[(k * 2 + 1) * 3 + m] = chr[m];
            }
    }
    if (charwise) {
        for (int v = 0; v < nv; ++v) {
            double al = 0.0, ar = 0.0;
            for (int k = 0; k < nv; ++k) {
                al = ORC_FMA(R[v * nv + k], wL[k], al);
                ar = ORC_FMA(R[v * nv + k], wR[k], ar);
            }
            UL[v] = al;
            UR[v] = ar;
        }
    } else {
        for (int v = 0; v < nv; ++v) { UL[v] = wL[v]; UR[v] = wR[v]; }
    }
    orc_num_flux(p, UL, UR, F);
}

/* ------------------------------------------------ one grid line, Eq. (2) */

/* line: (n + 2*GHOST) nodes x nv, node-major, ghosts already filled.
 * out: n x nv node-major, receives -f'_i.  Flag / chi outputs are addressed
 * for line index li of nlines. */
static void line_rhs(const orc_problem* p, int nv, int n, double h, const double* line,
                     double* out, uint8_t* flags, double* chi, int li, int nlines,
                     double* Fface, double* Fnode)
{
    const int nf = orc_nfaces(p, n);
    const int j0 = first_face(p);
    for (int s = 0; s < nf; ++s) {
        int j = j0 + s;
        uint8_t fl[8];
        double ch[24];
        const double* st = line + (size_t)(j - 2 + GHOST) * nv;
        midpoint_flux(p, nv, st, Fface + (size_t)s * nv, flags ? fl : NULL, chi ? ch : NULL);
        for (int k = 0; k < nv; ++k)
            for (int side = 0; side < 2; ++side) {
                size_t idx = (((size_t)k * nlines + li) * nf + s) * 2 + side;
                if (flags) flags[idx] = fl[k * 2 + side];
                if (chi)
                    for (int m = 0; m < 3; ++m) chi[idx * 3 + m] = ch[(k * 2 + side) * 3 + m];
            }
    }
    if (p->diff == ORC_MND) {
        /* Eq. (5): c1 (F_{i+1/2}-F_{i-1/2}) + c2 (f_{i+1}-f_{i-1}) + c3 (F_{i+3/2}-F_{i-3/2}) */
        const double c1 = 3.0 / 2.0, c2 = -3.0 / 10.0, c3 = 1.0 / 30.0;
        for (int i = -1; i <= n; ++i)
            phys_flux(p, line + (size_t)(i + GHOST) * nv, Fnode + (size_t)(i + 1) * nv);
        for (int i = 0; i < n; ++i)
            for (int v = 0; v < nv; ++v) {
                double Fp1 = Fface[(size_t)(i + 2) * nv + v], Fm1 = Fface[(size_t)(i + 1) * nv + v];
                double Fp3 = Fface[(size_t)(i + 3) * nv + v], Fm3 = Fface[(size_t)(i + 0) * nv + v];
                double fp = Fnode[(size_t)(i + 2) * nv + v], fm = Fnode[(size_t)(i + 0) * nv + v];
                double dfdx = c1 / h * (Fp1 - Fm1) + c2 / h * (fp - fm) + c3 / h * (Fp3 - Fm3);
                out[(size_t)i * nv + v] = -dfdx;
            }
    } else if (p->diff == ORC_HWCNS) {
        /* Eq. (4): b1 (F_{i+1/2}-F_{i-1/2}) + b2 (f_{i+1}-f_{i-1}) + b3 (f_{i+2}-f_{i-2}),
         * node fluxes f_i for i = -2 .. n+1 at Fnode[i + 2] */
        const double b1 = 64.0 / 45.0, b2 = -2.0 / 9.0, b3 = 1.0 / 180.0;
        for (int i = -2; i <= n + 1; ++i)
            phys_flux(p, line + (size_t)(i + GHOST) * nv, Fnode + (size_t)(i + 2) * nv);
        for (int i = 0; i < n; ++i)
            for (int v = 0; v < nv; ++v) {
                double Fp1 = Fface[(size_t)(i + 1) * nv + v], Fm1 = Fface[(size_t)i * nv + v];
                double fp1 = Fnode[(size_t)(i + 3) * nv + v], fm1 = Fnode[(size_t)(i + 1) * nv + v];
                double fp2 = Fnode[(size_t)(i + 4) * nv + v], fm2 = Fnode[(size_t)i * nv + v];
                double dfdx = b1 / h * (Fp1 - Fm1) + b2 / h * (fp1 - fm1) + b3 / h * (fp2 - fm2);
                out[(size_t)i * nv + v] = -dfdx;
            }
    } else {
        /* Eq. (3): a1 (F_{i+1/2}-F_{i-1/2}) + a2 (F_{i+3/2}-F_{i-3/2}) + a3 (F_{i+5/2}-F_{i-5/2}) */
        const double a1 = 75.0 / 64.0, a2 = -25.0 / 384.0, a3 = 3.0 / 640.0;
        for (int i = 0; i < n; ++i)
            for (int v = 0; v < nv; ++v) {
                double Fp1 = Fface[(size_t)(i + 3) * nv + v], Fm1 = Fface[(size_t)(i + 2) * nv + v];
                double Fp3 = Fface[(size_t)(i + 4) * nv + v], Fm3 = Fface[(size_t)(i + 1) * nv + v];
                double Fp5 = Fface[(size_t)(i + 5) * nv + v], Fm5 = Fface[(size_t)(i + 0) * nv + v];
                double dfdx = a1 / h * (Fp1 - Fm1) + a2 / h * (Fp3 - Fm3) + a3 / h * (Fp5 - Fm5);
                out[(size_t)i * nv + v] = -dfdx;
            }
    }
}

/* Ghost index map: periodic wrap, mirror image across a reflecting wall
 * (cell-centred: ghost -1-k mirrors cell k), or the nearest end cell
 * (zero-gradient; also the unused source index of a fixed ghost). */
static int ghost_index(int g, int n, int bc)
{
    if (bc == ORC_PERIODIC) return ((g % n) + n) % n;
    if (bc == ORC_REFLECT) {
        if (g < 0) return -1 - g;
        if (g >= n) return 2 * n - 1 - g;
        return g;
    }
    if (g < 0) return 0;
    if (g >= n) return n - 1;
    return g;
}

/* Variable order of x lines (storage order). */
static const int ident[4] = {0, 1, 2, 3};

/* Ghost value of line variable v (line order: normal momentum at index 1)
 * taken from the source cell's value `val`: a reflecting wall reverses the
 * normal momentum, a fixed boundary supplies its own state (`fixed` in
 * line order). */
static double ghost_value(int bc, int g, int n, int v, double val, const double fixed[2][4], const int* perm)
{
    if (g >= 0 && g < n) return val;
    if (bc == ORC_REFLECT && v == 1) return -val;
    if (bc == ORC_FIXED) return fixed[g < 0 ? 0 : 1][perm[v]];
    return val;
}

int orc_rhs(const orc_problem* p, const double* U, double* R, uint8_t* flags, double* chi,
            int nthreads)
{
    int st = validate(p);
    if (st) return st;
    const int nv = orc_nvar(p);
    const int nx = p->nx, ny = p->ny;
    const size_t plane = (size_t)nx * ny;
    if (nthreads < 1) nthreads = 1;

    /* x direction: one line per row, variables in their natural order. */
#pragma omp parallel num_threads(nthreads)
    {
        int nmax = nx > ny ? nx : ny;
        double* line = (double*)malloc(sizeof(double) * (size_t)(nmax + 2 * GHOST) * nv);
        double* out = (double*)malloc(sizeof(double) * (size_t)nmax * nv);
        double* Ff = (double*)malloc(sizeof(double) * (size_t)(nmax + 5) * nv);
        double* Fn = (double*)malloc(sizeof(double) * (size_t)(nmax + 4) * nv);
#pragma omp for schedule(static)
        for (int y = 0; y < ny; ++y) {
            for (int g = -GHOST; g < nx + GHOST; ++g) {
                int x = ghost_index(g, nx, p->bc_x);
                for (int v = 0; v < nv; ++v)
                    line[(size_t)(g + GHOST) * nv + v] =
                        ghost_value(p->bc_x, g, nx, v, U[v * plane + (size_t)y * nx + x], p->fixed_x, ident);
            }
            line_rhs(p, nv, nx, p->dx, line, out, flags, chi, y, ny, Ff, Fn);
            for (int x = 0; x < nx; ++x)
                for (int v = 0; v < nv; ++v)
                    R[v * plane + (size_t)y * nx + x] = out[(size_t)x * nv + v];
        }
        if (p->ndim == 2) {
            /* y direction: one line per column, normal momentum first. */
            static const int perm[4] = {0, 2, 1, 3};
            uint8_t* fy = flags ? flags + (size_t)nv * ny * orc_nfaces(p, nx) * 2 : NULL;
            double* cy = chi ? chi + (size_t)nv * ny * orc_nfaces(p, nx) * 2 * 3 : NULL;
#pragma omp for schedule(static)
            for (int x = 0; x < nx; ++x) {
                for (int g = -GHOST; g < ny + GHOST; ++g) {
                    int y = ghost_index(g, ny, p->bc_y);
                    for (int v = 0; v < nv; ++v)
                        line[(size_t)(g + GHOST) * nv + v] = ghost_value(
                            p->bc_y, g, ny, v, U[perm[v] * plane + (size_t)y * nx + x], p->fixed_y, perm);
                }
                line_rhs(p, nv, ny, p->dy, line, out, fy, cy, x, nx, Ff, Fn);
                for (int y = 0; y < ny; ++y)
                    for (int v = 0; v < nv; ++v) {
                        size_t idx = perm[v] * plane + (size_t)y * nx + x;
                        R[idx] = R[idx] + out[(size_t)y * nv + v];
                    }
            }
            if (p->gravity != 0.0) {
                /* body force in +y: d(rho v)/dt += rho g, dE/dt += rho v g */
#pragma omp for schedule(static)
                for (int y = 0; y < ny; ++y)
                    for (int x = 0; x < nx; ++x) {
                        size_t c = (size_t)y * nx + x;
                        R[2 * plane + c] = R[2 * plane + c] + U[c] * p->gravity;
                        R[3 * plane + c] = R[3 * plane + c] + U[2 * plane + c] * p->gravity;
                    }
            }
        }
        free(line); free(out); free(Ff); free(Fn);
    }
    return ORC_OK;
}

/* ------------------------------------------------------ time stepping */

double orc_max_speed(const orc_problem* p, const double* U)
{
    const int nv = orc_nvar(p);
    const size_t plane = (size_t)p->nx * p->ny;
    double smax = 0.0;
    for (size_t c = 0; c < plane; ++c) {
        double s;
        if (p->system == ORC_ADVECTION) {
            s = fabs(p->adv_speed) / p->dx;
        } else if (p->system == ORC_BURGERS) {
            s = fabs(U[c]) / p->dx;
        } else {
            double cell[4] = {0.0, 0.0, 0.0, 0.0};
            for (int v = 0; v < nv; ++v) cell[v] = U[v * plane + c];
            double a = sound_speed(nv, p->gamma, cell);
            double ir = 1.0 / cell[0];
            s = (fabs(cell[1] * ir) + a) / p->dx;
            if (nv == 4) s = s + (fabs(cell[2] * ir) + a) / p->dy;
        }
        /* a NaN speed poisons the maximum for good */
        if (isnan(s) || (!isnan(smax) && s > smax)) smax = s;
    }
    return smax;
}

/* First non-physical cell in row-major order, or -1. */
static int64_t first_bad_cell(const orc_problem* p, const double* U)
{
    const int nv = orc_nvar(p);
    const size_t plane = (size_t)p->nx * p->ny;
    for (size_t c = 0; c < plane; ++c) {
        double cell[4];
        int bad = 0;
        for (int v = 0; v < nv; ++v) {
            cell[v] = U[v * plane + c];
            if (!isfinite(cell[v])) bad = 1;
        }
        if (!bad && p->system == ORC_EULER)
            bad = !(cell[0] > 0.0) || !(euler_pressure(nv, p->gamma, cell) > 0.0);
        if (bad) return (int64_t)c;
    }
    return -1;
}

int orc_rk3_step(const orc_problem* p, double* U, double dt, int64_t stage_base,
                 int64_t* bad_stage, int64_t* bad_cell, int nthreads)
{
    int st = validate(p);
    if (st) return st;
    const size_t n = (size_t)orc_nvar(p) * p->nx * p->ny;
    double* R = (double*)malloc(sizeof(double) * n);
    double* U1 = (double*)malloc(sizeof(double) * n);
    double* U2 = (double*)malloc(sizeof(double) * n);
    int64_t bad;
    int ret = ORC_OK;

    /* U1 = U^n + dt R(U^n) */
    orc_rhs(p, U, R, NULL, NULL, nthreads);
    for (size_t i = 0; i < n; ++i) U1[i] = U[i] + dt * R[i];
    if ((bad = first_bad_cell(p, U1)) >= 0) { *bad_stage = stage_base; *bad_cell = bad; ret = ORC_E_NONPHYSICAL; goto done; }
    /* U2 = 3/4 U^n + 1/4 (U1 + dt R(U1)) */
    orc_rhs(p, U1, R, NULL, NULL, nthreads);
    for (size_t i = 0; i < n; ++i) U2[i] = 0.75 * U[i] + 0.25 * (U1[i] + dt * R[i]);
    if ((bad = first_bad_cell(p, U2)) >= 0) { *bad_stage = stage_base + 1; *bad_cell = bad; ret = ORC_E_NONPHYSICAL; goto done; }
    /* U^{n+1} = 1/3 U^n + 2/3 (U2 + dt R(U2)) */
    orc_rhs(p, U2, R, NULL, NULL, nthreads);
    for (size_t i = 0; i < n; ++i) U[i] = (1.0 / 3.0) * U[i] + (2.0 / 3.0) * (U2[i] + dt * R[i]);
    if ((bad = first_bad_cell(p, U)) >= 0) { *bad_stage = stage_base + 2; *bad_cell = bad; ret = ORC_E_NONPHYSICAL; goto done; }
done:
    free(R); free(U1); free(U2);
    return ret;
}

int orc_solve(const orc_problem* p, double* U, double t0, double t_final, double cfl,
              int64_t max_steps, double* t_out, int64_t* steps_out, int64_t* bad_stage,
              int64_t* bad_cell, int nthreads)
{
    int st = validate(p);
    double t = t0;
    int64_t steps = 0;
    if (st) return st;
    for (;;) {
        if (isfinite(t_final) && t_final - t <= 1e-12 * t_final) break;
        if (steps >= max_steps) {
            if (isfinite(t_final)) { st = ORC_E_MAX_STEPS; }
            break;
        }
        double dt = cfl / orc_max_speed(p, U);
        if (isfinite(t_final) && dt > t_final - t) dt = t_final - t;
        st = orc_rk3_step(p, U, dt, 3 * steps, bad_stage, bad_cell, nthreads);
        if (st) break;
        t = t + dt;
        steps = steps + 1;
    }
    if (t_out) *t_out = t;
    if (steps_out) *steps_out = steps;
    return st;
}

// Device arithmetic of the WCNS-T midpoint flux for gfx950 (FP64 VALU).
//
// One call of face_flux() turns the six nodes j-2 .. j+3 around a midpoint
// x_{j+1/2} into the numerical flux there:
//   characteristic projection (Roe average of nodes j, j+1)      Sec. 3
//   TENO-5 interpolation of u_L and of the mirrored u_R          Sec. 2.2-2.3
//   back-projection and the Roe / local Lax-Friedrichs flux      Sec. 2.2, Eq. (6)
// Written for throughput: fused multiply-adds, compile-time unrolled
// eigenvector rows, a comparison form of the cut-off test and a select
// chain for the weights of Eq. (19) (their values are the exact quotients
// d_k / sum d_m over the kept stencils).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wcnst {

enum { SYS_ADV = 0, SYS_BURG = 1, SYS_EULER = 2 };
enum { FLUX_ROE = 0, FLUX_LF = 1 };
enum { SCH_TENO = 0, SCH_LINEAR = 1, SCH_JS = 2 };
enum { BC_PERIODIC = 0, BC_ZG = 1 };

struct Params {
    double CT, C, eps_teno, eps_js;
    double gamma, gm1;
    double adv;
    double dx, dy;
    double c1x, c2x, c3x;  // MND coefficients divided by dx
    double c1y, c2y, c3y;  // ... and by dy
    int q, scheme, charwise;
    int bc_x, bc_y;
    int nx, ny;
};

// ------------------------------------------------------------ helpers

__device__ __forceinline__ int ghost_map(int g, int n, int bc)
{
    if (bc == BC_PERIODIC) {
        g = g < 0 ? g + n : g;
        return g >= n ? g - n : g;
    }
    g = g < 0 ? 0 : g;
    return g >= n ? n - 1 : g;
}

__device__ __forceinline__ double pow_q(double x, int q)
{
    if (q == 6) {
        double x2 = x * x;
        return x2 * x2 * x2;
    }
    double r = 1.0;
    for (int m = 0; m < q; ++m) r *= x;
    return r;
}

// ------------------------------------------------- Sec. 2.2-2.3 interpolation

// u_L at x_{i+1/2} from (a, b, c, d, e) = (u_{i-2} .. u_{i+2}); mask receives
// delta_1 | delta_2 << 1 | delta_3 << 2.
__device__ __forceinline__ double interp5(double a, double b, double c, double d, double e,
                                          const Params& P, unsigned& mask)
{
    // h u^(1)_k and h^2 u^(2)_k of Eqs. (10)-(11)
    const double D10 = 0.5 * (a - 4.0 * b + 3.0 * c);
    const double D11 = 0.5 * (d - b);
    const double D12 = 0.5 * (-3.0 * c + 4.0 * d - e);
    const double D20 = a - 2.0 * b + c;
    const double D21 = b - 2.0 * c + d;
    const double D22 = c - 2.0 * d + e;
    // candidates, Eq. (9) with Delta x = h/2
    const double q0 = c + 0.5 * D10 + 0.125 * D20;
    const double q1 = c + 0.5 * D11 + 0.125 * D21;
    const double q2 = c + 0.5 * D12 + 0.125 * D22;
    if (P.scheme == SCH_LINEAR) {
        mask = 7u;
        return 0.0625 * q0 + 0.625 * q1 + 0.3125 * q2;
    }
    // smoothness indicators, Eq. (15)
    const double b0 = D10 * D10 + D20 * D20;
    const double b1 = D11 * D11 + D21 * D21;
    const double b2 = D12 * D12 + D22 * D22;
    if (P.scheme == SCH_JS) {
        mask = 7u;
        const double e0 = b0 + P.eps_js, e1 = b1 + P.eps_js, e2 = b2 + P.eps_js;
        const double a0 = 0.0625 / (e0 * e0), a1 = 0.625 / (e1 * e1), a2 = 0.3125 / (e2 * e2);
        const double s = a0 + a1 + a2;
        return (a0 * q0 + a1 * q1 + a2 * q2) / s;
    }
    // Eq. (16)
    const double tau = fabs(b0 - b2);
    const double g0 = pow_q(P.C + tau / (b0 + P.eps_teno), P.q);
    const double g1 = pow_q(P.C + tau / (b1 + P.eps_teno), P.q);
    const double g2 = pow_q(P.C + tau / (b2 + P.eps_teno), P.q);
    // Eqs. (17)-(18): chi_k < C_T  <=>  gamma_k < C_T * sum(gamma)
    const double thr = P.CT * (g0 + g1 + g2);
    const bool k0 = !(g0 < thr), k1 = !(g1 < thr), k2 = !(g2 < thr);
    mask = (unsigned)k0 | ((unsigned)k1 << 1) | ((unsigned)k2 << 2);
    // Eq. (19): d_k delta_k / sum_m d_m delta_m for the seven patterns
    const double w0 = k0 ? (k1 ? (k2 ? 0.0625 : 1.0 / 11.0) : (k2 ? 1.0 / 6.0 : 1.0)) : 0.0;
    const double w1 = k1 ? (k0 ? (k2 ? 0.625 : 10.0 / 11.0) : (k2 ? 2.0 / 3.0 : 1.0)) : 0.0;
    const double w2 = k2 ? (k0 ? (k1 ? 0.3125 : 5.0 / 6.0) : (k1 ? 1.0 / 3.0 : 1.0)) : 0.0;
    return w0 * q0 + w1 * q1 + w2 * q2;
}

// ------------------------------------------------------------ Euler

// Roe-averaged state and the scalars its eigenvectors are built from.
struct Eig {
    double u, v, H, c, ic, b1, b2, hq2;  // hq2 = (u^2 + v^2) / 2
};

template <int NV>
__device__ __forceinline__ void prim(const double* U, const Params& P, double& u, double& v,
                                     double& p, double& H)
{
    const double ir = 1.0 / U[0];
    u = U[1] * ir;
    v = NV == 4 ? U[2] * ir : 0.0;
    const double kin = NV == 4 ? 0.5 * (U[1] * u + U[2] * v) : 0.5 * U[1] * u;
    p = P.gm1 * (U[NV - 1] - kin);
    H = (U[NV - 1] + p) * ir;
}

template <int NV>
__device__ __forceinline__ Eig roe_average(const double* A, const double* B, const Params& P)
{
    double uA, vA, pA, HA, uB, vB, pB, HB;
    prim<NV>(A, P, uA, vA, pA, HA);
    prim<NV>(B, P, uB, vB, pB, HB);
    const double sA = sqrt(A[0]), sB = sqrt(B[0]);
    const double iw = 1.0 / (sA + sB);
    Eig E;
    E.u = (sA * uA + sB * uB) * iw;
    E.v = NV == 4 ? (sA * vA + sB * vB) * iw : 0.0;
    E.H = (sA * HA + sB * HB) * iw;
    E.hq2 = 0.5 * (E.u * E.u + E.v * E.v);
    const double c2 = P.gm1 * (E.H - E.hq2);
    E.c = sqrt(c2);
    E.ic = 1.0 / E.c;
    E.b1 = P.gm1 / c2;
    E.b2 = E.hq2 * E.b1;
    return E;
}

// Left eigenvector row k (normal momentum first; fields: u-c, u, [shear], u+c).
template <int NV, int K>
__device__ __forceinline__ double lrow_dot(const Eig& E, const double* x)
{
    if constexpr (K == 0) {
        double r = (E.b2 + E.u * E.ic) * x[0] - (E.b1 * E.u + E.ic) * x[1] + E.b1 * x[NV - 1];
        if constexpr (NV == 4) r -= E.b1 * E.v * x[2];
        return 0.5 * r;
    } else if constexpr (K == 1) {
        double r = (1.0 - E.b2) * x[0] + E.b1 * E.u * x[1] - E.b1 * x[NV - 1];
        if constexpr (NV == 4) r += E.b1 * E.v * x[2];
        return r;
    } else if constexpr (NV == 4 && K == 2) {
        return x[2] - E.v * x[0];
    } else {
        double r = (E.b2 - E.u * E.ic) * x[0] - (E.b1 * E.u - E.ic) * x[1] + E.b1 * x[NV - 1];
        if constexpr (NV == 4) r -= E.b1 * E.v * x[2];
        return 0.5 * r;
    }
}

// acc += w * (right eigenvector column k)
template <int NV, int K>
__device__ __forceinline__ void rcol_axpy(const Eig& E, double w, double* acc)
{
    if constexpr (K == 0) {
        acc[0] += w;
        acc[1] += w * (E.u - E.c);
        if constexpr (NV == 4) acc[2] += w * E.v;
        acc[NV - 1] += w * (E.H - E.u * E.c);
    } else if constexpr (K == 1) {
        acc[0] += w;
        acc[1] += w * E.u;
        if constexpr (NV == 4) acc[2] += w * E.v;
        acc[NV - 1] += w * E.hq2;
    } else if constexpr (NV == 4 && K == 2) {
        acc[2] += w;
        acc[3] += w * E.v;
    } else {
        acc[0] += w;
        acc[1] += w * (E.u + E.c);
        if constexpr (NV == 4) acc[2] += w * E.v;
        acc[NV - 1] += w * (E.H + E.u * E.c);
    }
}

template <int NV, int K>
__device__ __forceinline__ double eigval(const Eig& E)
{
    if constexpr (K == 0) return E.u - E.c;
    else if constexpr (K == NV - 1) return E.u + E.c;
    else return E.u;
}

template <int NV>
__device__ __forceinline__ void euler_flux(const double* U, const Params& P, double* F)
{
    double u, v, p, H;
    prim<NV>(U, P, u, v, p, H);
    F[0] = U[1];
    F[1] = U[1] * u + p;
    if constexpr (NV == 4) F[2] = U[2] * u;
    F[NV - 1] = u * (U[NV - 1] + p);
}

template <int NV, int K>
__device__ __forceinline__ void proj_interp(const Eig& E, const double (&s)[6][NV], const Params& P,
                                            double* UL, double* UR, unsigned& fb)
{
    double w[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) w[m] = lrow_dot<NV, K>(E, s[m]);
    unsigned mL, mR;
    const double wl = interp5(w[0], w[1], w[2], w[3], w[4], P, mL);
    const double wr = interp5(w[5], w[4], w[3], w[2], w[1], P, mR);
    rcol_axpy<NV, K>(E, wl, UL);
    rcol_axpy<NV, K>(E, wr, UR);
    fb |= (mL | (mR << 3)) << (6 * K);
}

template <int NV, int K>
__device__ __forceinline__ void roe_dissipation(const Eig& E, const double* dU, double* dis)
{
    const double a = fabs(eigval<NV, K>(E)) * lrow_dot<NV, K>(E, dU);
    rcol_axpy<NV, K>(E, a, dis);
}

// Numerical flux of the Euler equations from the interpolated states.
template <int NV, int FLUX>
__device__ __forceinline__ void euler_num_flux(const double* UL, const double* UR, const Params& P,
                                               double* F)
{
    double FL[NV], FR[NV], dis[NV];
    euler_flux<NV>(UL, P, FL);
    euler_flux<NV>(UR, P, FR);
#pragma unroll
    for (int v = 0; v < NV; ++v) dis[v] = 0.0;
    if constexpr (FLUX == FLUX_LF) {
        double uL, vL, pL, HL, uR, vR, pR, HR;
        prim<NV>(UL, P, uL, vL, pL, HL);
        prim<NV>(UR, P, uR, vR, pR, HR);
        const double aL = fabs(uL) + sqrt(P.gamma * pL / UL[0]);
        const double aR = fabs(uR) + sqrt(P.gamma * pR / UR[0]);
        const double al = fmax(aL, aR);
#pragma unroll
        for (int v = 0; v < NV; ++v) dis[v] = al * (UR[v] - UL[v]);
    } else {
        const Eig E = roe_average<NV>(UL, UR, P);
        double dU[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) dU[v] = UR[v] - UL[v];
        roe_dissipation<NV, 0>(E, dU, dis);
        roe_dissipation<NV, 1>(E, dU, dis);
        roe_dissipation<NV, 2>(E, dU, dis);
        if constexpr (NV == 4) roe_dissipation<NV, 3>(E, dU, dis);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) F[v] = 0.5 * ((FR[v] + FL[v]) - dis[v]);
}

// --------------------------------------------------------- midpoint flux

// s: nodes j-2 .. j+3 (normal momentum first).  F: flux at x_{j+1/2}.
// fb: 6 flag bits per field (left mask | right mask << 3).
template <int SYS, int NV, int FLUX>
__device__ __forceinline__ void face_flux(const double (&s)[6][NV], const Params& P, double (&F)[NV],
                                          unsigned& fb)
{
    fb = 0u;
    if constexpr (SYS == SYS_EULER) {
        double UL[NV], UR[NV];
        if (P.charwise) {
            const Eig E = roe_average<NV>(s[2], s[3], P);
#pragma unroll
            for (int v = 0; v < NV; ++v) { UL[v] = 0.0; UR[v] = 0.0; }
            proj_interp<NV, 0>(E, s, P, UL, UR, fb);
            proj_interp<NV, 1>(E, s, P, UL, UR, fb);
            proj_interp<NV, 2>(E, s, P, UL, UR, fb);
            if constexpr (NV == 4) proj_interp<NV, 3>(E, s, P, UL, UR, fb);
        } else {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                unsigned mL, mR;
                UL[v] = interp5(s[0][v], s[1][v], s[2][v], s[3][v], s[4][v], P, mL);
                UR[v] = interp5(s[5][v], s[4][v], s[3][v], s[2][v], s[1][v], P, mR);
                fb |= (mL | (mR << 3)) << (6 * v);
            }
        }
        euler_num_flux<NV, FLUX>(UL, UR, P, F);
    } else {
        unsigned mL, mR;
        const double uL = interp5(s[0][0], s[1][0], s[2][0], s[3][0], s[4][0], P, mL);
        const double uR = interp5(s[5][0], s[4][0], s[3][0], s[2][0], s[1][0], P, mR);
        fb = mL | (mR << 3);
        if constexpr (SYS == SYS_ADV) {
            F[0] = 0.5 * ((P.adv * uR + P.adv * uL) - fabs(P.adv) * (uR - uL));
        } else {
            const double ah = FLUX == FLUX_LF ? fmax(fabs(uL), fabs(uR)) : 0.5 * (uL + uR);
            F[0] = 0.5 * ((0.5 * uR * uR + 0.5 * uL * uL) - fabs(ah) * (uR - uL));
        }
    }
}

template <int SYS, int NV>
__device__ __forceinline__ void node_flux(const double* U, const Params& P, double* F)
{
    if constexpr (SYS == SYS_EULER) euler_flux<NV>(U, P, F);
    else if constexpr (SYS == SYS_ADV) F[0] = P.adv * U[0];
    else F[0] = 0.5 * U[0] * U[0];
}

// CFL denominator contribution of one cell.
template <int SYS, int NV>
__device__ __forceinline__ double cell_speed(const double* U, const Params& P)
{
    if constexpr (SYS == SYS_ADV) return fabs(P.adv) / P.dx;
    else if constexpr (SYS == SYS_BURG) return fabs(U[0]) / P.dx;
    else {
        double u, v, p, H;
        prim<NV>(U, P, u, v, p, H);
        const double a = sqrt(P.gamma * p / U[0]);
        double s = (fabs(u) + a) / P.dx;
        if constexpr (NV == 4) s = s + (fabs(v) + a) / P.dy;
        return s;
    }
}

// Non-physical check of a stage output.
template <int SYS, int NV>
__device__ __forceinline__ bool cell_bad(const double* U, const Params& P)
{
    bool bad = false;
#pragma unroll
    for (int v = 0; v < NV; ++v) bad |= !isfinite(U[v]);
    if constexpr (SYS == SYS_EULER) {
        double u, v, p, H;
        prim<NV>(U, P, u, v, p, H);
        bad |= !(U[0] > 0.0) || !(p > 0.0);
    }
    return bad;
}

}  // namespace wcnst

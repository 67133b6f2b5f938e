// Host build of the HIP path's per-midpoint arithmetic (wcnst_device.hpp),
// for CPU tests of that arithmetic against the oracle.  It evaluates whole
// grid lines the way the stage kernels do (ghost remap, midpoint flux, node
// flux, MND difference) but on the host, so no GPU is needed.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <cmath>

#include <vector>

#include "wcnst_device.hpp"

using namespace wcnst;

namespace {

template <int SYS, int NV, int FLUX, int SCHEME, bool CHAR>
void line(const Params& P, int n, int bc, double c1, double c2, double c3, const double* U, int stride,
          const int* perm, double* R, uint8_t* flags, int nlines, int li)
{
    std::vector<double> F((size_t)(n + 3) * NV), fn((size_t)(n + 2) * NV);
    for (int j = -2; j <= n; ++j) {
        double s[6][NV];
        for (int m = 0; m < 6; ++m) {
            const int g = ghost_map(j - 2 + m, n, bc);
            for (int v = 0; v < NV; ++v) s[m][v] = U[(size_t)perm[v] * stride + g];
        }
        double f[NV];
        unsigned fb;
        RegStencil<NV> st{s};
        face_flux<SYS, NV, FLUX, SCHEME, CHAR>(st, P, f, fb);
        for (int v = 0; v < NV; ++v) F[(size_t)(j + 2) * NV + v] = f[v];
        if (flags)
            for (int k = 0; k < NV; ++k) {
                const size_t idx = (((size_t)k * nlines + li) * (n + 3) + (j + 2)) * 2;
                flags[idx] = (uint8_t)((fb >> (6 * k)) & 7u);
                flags[idx + 1] = (uint8_t)((fb >> (6 * k + 3)) & 7u);
            }
    }
    for (int i = -1; i <= n; ++i) {
        double u[NV], f[NV];
        const int g = ghost_map(i, n, bc);
        for (int v = 0; v < NV; ++v) u[v] = U[(size_t)perm[v] * stride + g];
        node_flux<SYS, NV>(u, P, f);
        for (int v = 0; v < NV; ++v) fn[(size_t)(i + 1) * NV + v] = f[v];
    }
    for (int i = 0; i < n; ++i)
        for (int v = 0; v < NV; ++v) {
            const double r = mnd(c1, c2, c3, F[(size_t)i * NV + v], F[(size_t)(i + 1) * NV + v],
                                 F[(size_t)(i + 2) * NV + v], F[(size_t)(i + 3) * NV + v],
                                 fn[(size_t)i * NV + v], fn[(size_t)(i + 2) * NV + v]);
            R[(size_t)perm[v] * stride + i] += r;
        }
}

template <int SYS, int NV, int FLUX, bool CHAR>
void line_char(int scheme, const Params& P, int n, int bc, double c1, double c2, double c3, const double* U,
               int stride, const int* perm, double* R, uint8_t* flags, int nlines, int li)
{
    if (scheme == 3) line<SYS, NV, FLUX, SCH_Z, CHAR>(P, n, bc, c1, c2, c3, U, stride, perm, R, flags, nlines, li);
    else if (scheme == SCH_LINEAR) line<SYS, NV, FLUX, SCH_LINEAR, CHAR>(P, n, bc, c1, c2, c3, U, stride, perm, R, flags, nlines, li);
    else if (scheme == SCH_JS) line<SYS, NV, FLUX, SCH_JS, CHAR>(P, n, bc, c1, c2, c3, U, stride, perm, R, flags, nlines, li);
    else if (P.q == 6) line<SYS, NV, FLUX, SCH_TENO, CHAR>(P, n, bc, c1, c2, c3, U, stride, perm, R, flags, nlines, li);
    else line<SYS, NV, FLUX, SCH_TENO_Q, CHAR>(P, n, bc, c1, c2, c3, U, stride, perm, R, flags, nlines, li);
}

template <int SYS, int NV, int FLUX>
void line_scheme(int scheme, const Params& P, int n, int bc, double c1, double c2, double c3, const double* U,
                 int stride, const int* perm, double* R, uint8_t* flags, int nlines, int li)
{
    if (SYS == SYS_EULER && P.charwise) line_char<SYS, NV, FLUX, true>(scheme, P, n, bc, c1, c2, c3, U, stride, perm, R, flags, nlines, li);
    else line_char<SYS, NV, FLUX, false>(scheme, P, n, bc, c1, c2, c3, U, stride, perm, R, flags, nlines, li);
}

void run_line(int sys, int nv, int flux, int scheme, const Params& P, int n, int bc, double c1, double c2,
              double c3, const double* U, int stride, const int* perm, double* R, uint8_t* flags, int nlines,
              int li)
{
    if (sys == 0) line_scheme<SYS_ADV, 1, FLUX_ROE>(scheme, P, n, bc, c1, c2, c3, U, stride, perm, R, flags, nlines, li);
    else if (sys == 1 && flux == 0) line_scheme<SYS_BURG, 1, FLUX_ROE>(scheme, P, n, bc, c1, c2, c3, U, stride, perm, R, flags, nlines, li);
    else if (sys == 1) line_scheme<SYS_BURG, 1, FLUX_LF>(scheme, P, n, bc, c1, c2, c3, U, stride, perm, R, flags, nlines, li);
    else if (nv == 3 && flux == 0) line_scheme<SYS_EULER, 3, FLUX_ROE>(scheme, P, n, bc, c1, c2, c3, U, stride, perm, R, flags, nlines, li);
    else if (nv == 3 && flux == 2) line_scheme<SYS_EULER, 3, FLUX_VL>(scheme, P, n, bc, c1, c2, c3, U, stride, perm, R, flags, nlines, li);
    else if (nv == 3) line_scheme<SYS_EULER, 3, FLUX_LF>(scheme, P, n, bc, c1, c2, c3, U, stride, perm, R, flags, nlines, li);
    else if (flux == 0) line_scheme<SYS_EULER, 4, FLUX_ROE>(scheme, P, n, bc, c1, c2, c3, U, stride, perm, R, flags, nlines, li);
    else if (flux == 2) line_scheme<SYS_EULER, 4, FLUX_VL>(scheme, P, n, bc, c1, c2, c3, U, stride, perm, R, flags, nlines, li);
    else line_scheme<SYS_EULER, 4, FLUX_LF>(scheme, P, n, bc, c1, c2, c3, U, stride, perm, R, flags, nlines, li);
}

}  // namespace

namespace {

// Index geometry of the 1D stage kernel (Strip1D) on a line of nx cells,
// evaluated for every strip and lane of the launch.  Returns 0 when every
// cell is owned once, every midpoint -G .. nx-2+G is reported once by a lane
// that computed it from its own (unclamped) stencil, each owned cell finds
// its 2G midpoints on the lanes above it and its own state at stencil node
// G+2, HWCNS cells find the node fluxes of nodes c-2, c-1, c+1, c+2 at
// stencil node 1 of lanes lane, lane+1, lane+3, lane+4, and the stencil
// nodes of MND / MD lanes lie within one line length of the line (HWCNS
// loads use the any-distance map); else a code naming the first violated
// property.
template <int DIFF>
static int strip_check(int nx)
{
    using S1 = Strip1D<DIFF>;
    const int G = S1::G, W = S1::W;
    const int nstrips = (nx + W - 1) / W;
    std::vector<int> cells((size_t)nx, 0), faces((size_t)nx + 2 * G - 1, 0);
    for (int bx = 0; bx < nstrips; ++bx)
        for (int lane = 0; lane < WAVE; ++lane) {
            const S1 s(bx, lane, nx);
            if (s.nfaces() != nx + 2 * G - 1) return 1;
            for (int m = 0; m < 6 && DIFF != DIFF_HW; ++m) {
                const int node = s.jxl - 2 + m;
                if (node < -nx || node >= 2 * nx) return 2;
            }
            if (s.owns_face(bx, nx)) {
                if (s.jx < -G || s.jx > s.jmax || s.jxl != s.jx) return 3;
                faces[(size_t)(s.jx + G)] += 1;
            }
            if (s.cell_ok) {
                if (s.c < 0 || s.c >= nx) return 4;
                cells[(size_t)s.c] += 1;
                if (s.jxl - 2 + (G + 2) != s.c) return 5;
                for (int k = 0; k < 2 * G; ++k) {
                    if (lane + k >= WAVE) return 6;
                    const S1 t(bx, lane + k, nx);
                    if (t.jx != s.c - G + k || t.jxl != t.jx) return 7;
                }
                if (DIFF == DIFF_HW) {
                    const int off[4] = {0, 1, 3, 4}, node[4] = {s.c - 2, s.c - 1, s.c + 1, s.c + 2};
                    for (int k = 0; k < 4; ++k) {
                        if (lane + off[k] >= WAVE) return 10;
                        const S1 t(bx, lane + off[k], nx);
                        if (t.jxl - 2 + 1 != node[k]) return 11;
                    }
                }
            }
        }
    for (int v : cells)
        if (v != 1) return 8;
    for (int v : faces)
        if (v != 1) return 9;
    return 0;
}

}  // namespace

extern "C" {

// sys: 0 advection, 1 Burgers, 2 Euler; flux: 0 Roe, 1 LF, 2 van Leer; scheme: 0 TENO,
// 1 linear, 2 JS, 3 Z.  U, R: [nv][ny][nx].
// R is accumulated (the caller zeroes it).  flags: [x block][y block] like wcnst_rhs.
int hc_rhs(int ndim, int sys, int flux, int nx, int ny, double dx, double dy, int bc_x, int bc_y,
           int scheme, int charwise, int q, double gamma, double adv, double CT, double C,
           double eps_teno, double eps_js, const double* U, double* R, uint8_t* flags, int z_q, double eps_z)
{
    Params P{};
    P.z_q = z_q; P.eps_z = eps_z;
    // as the library's parameters: the smooth-stencil bound of the cut test
    P.teno_smooth = 0.9 * C * (std::pow(3.0 * CT, -1.0 / q) - 1.0);
    P.CT = CT; P.C = C; P.eps_teno = eps_teno; P.eps_js = eps_js;
    P.gamma = gamma; P.adv = adv; P.dx = dx; P.dy = dy;
    P.q = q; P.charwise = charwise; P.bc_x = bc_x; P.bc_y = bc_y;
    P.nx = nx; P.ny = ny;
    const int nv = sys == 2 ? (ndim == 1 ? 3 : 4) : 1;
    const size_t plane = (size_t)nx * ny;
    const double c1x = (3.0 / 2.0) / dx, c2x = (-3.0 / 10.0) / dx, c3x = (1.0 / 30.0) / dx;
    const double c1y = (3.0 / 2.0) / dy, c2y = (-3.0 / 10.0) / dy, c3y = (1.0 / 30.0) / dy;
    static const int idp[4] = {0, 1, 2, 3};
    static const int yperm[4] = {0, 2, 1, 3};
    // x lines
    for (int y = 0; y < ny; ++y) {
        std::vector<double> row((size_t)nv * nx), r((size_t)nv * nx, 0.0);
        for (int v = 0; v < nv; ++v)
            for (int x = 0; x < nx; ++x) row[(size_t)v * nx + x] = U[v * plane + (size_t)y * nx + x];
        run_line(sys, nv, flux, scheme, P, nx, bc_x, c1x, c2x, c3x, row.data(), nx, idp, r.data(), flags, ny, y);
        for (int v = 0; v < nv; ++v)
            for (int x = 0; x < nx; ++x) R[v * plane + (size_t)y * nx + x] += r[(size_t)v * nx + x];
    }
    if (ndim == 2) {
        uint8_t* fy = flags ? flags + (size_t)nv * ny * (nx + 3) * 2 : nullptr;
        for (int x = 0; x < nx; ++x) {
            std::vector<double> col((size_t)nv * ny), r((size_t)nv * ny, 0.0);
            for (int v = 0; v < nv; ++v)
                for (int y = 0; y < ny; ++y) col[(size_t)v * ny + y] = U[v * plane + (size_t)y * nx + x];
            run_line(2, 4, flux, scheme, P, ny, bc_y, c1y, c2y, c3y, col.data(), ny, yperm, r.data(), fy, nx, x);
            for (int v = 0; v < nv; ++v)
                for (int y = 0; y < ny; ++y) R[v * plane + (size_t)y * nx + x] += r[(size_t)v * ny + y];
        }
    }
    return 0;
}

// in_ieee_range of each x (1 or 0)
void hc_in_ieee_range(const double* x, uint8_t* out, int n)
{
    for (int i = 0; i < n; ++i) out[i] = in_ieee_range(x[i]) ? 1 : 0;
}

// work index of each launch index of the group [base, base + n)
void hc_xcd_order(int base, int n, int* out)
{
    for (int i = 0; i < n; ++i) out[i] = xcd_order(base + i, base, n);
}

// plan_strip over one strip: boundaries b[0..n], durations d[0..n-1] -> out[0..n]
void hc_plan_strip(const int* b, const unsigned* d, int n, int minr, int* out)
{
    plan_strip(b, d, n, minr, out);
}

int hc_strip1d_check(int nx, int diff_md)
{
    return diff_md == 2 ? strip_check<DIFF_HW>(nx) : (diff_md ? strip_check<DIFF_MD>(nx) : strip_check<DIFF_MND>(nx));
}

}  // extern "C"

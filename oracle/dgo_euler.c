/*
 * Oracle: compressible Euler fluxes.  TEST INFRASTRUCTURE ONLY (see dgo.h).
 *
 *  - Physical flux of the 2D Euler equations, u = (rho, rho v1, rho v2, rho e),
 *    p = (gamma-1)(rho e - rho |v|^2 / 2)  (Sec. 3, gamma a parameter).
 *  - Local Lax-Friedrichs (Rusanov) flux for the surface fluxes and the
 *    low-order subcell fluxes (Sec. 3 intro); the wave-speed bound is
 *    max(|v_n| + c) over the two states.
 *  - Entropy-conserving, kinetic-energy-preserving two-point volume flux of
 *    Ranocha (2018), cited in the Sec. 3 intro, with the logarithmic mean
 *    evaluated by the Ismail-Roe (2009) series near equal arguments.
 *  - The entropy-conserving, kinetic-energy-preserving flux of Chandrashekar
 *    (2013), which the paper uses for the astrophysical jet (Sec. 3.6).
 */
#include <math.h>

#include "dgo.h"

void dgo_prim(const double* u, double gamma, double* rho, double* v1, double* v2, double* p)
{
    *rho = u[0];
    *v1 = u[1] / u[0];
    *v2 = u[2] / u[0];
    *p = (gamma - 1.0) * (u[3] - 0.5 * (u[1] * (*v1) + u[2] * (*v2)));
}

double dgo_pressure(const double* u, double gamma)
{
    double r, a, b, p;
    dgo_prim(u, gamma, &r, &a, &b, &p);
    return p;
}

double dgo_wavespeed(const double* u, int dir, double gamma)
{
    double r, v1, v2, p;
    dgo_prim(u, gamma, &r, &v1, &v2, &p);
    double vn = dir == 0 ? v1 : v2;
    return fabs(vn) + sqrt(gamma * p / r);
}

void dgo_flux_phys(const double* u, int dir, double gamma, double* f)
{
    double r, v1, v2, p;
    dgo_prim(u, gamma, &r, &v1, &v2, &p);
    double vn = dir == 0 ? v1 : v2;
    f[0] = r * vn;
    f[1] = u[1] * vn + (dir == 0 ? p : 0.0);
    f[2] = u[2] * vn + (dir == 1 ? p : 0.0);
    f[3] = (u[3] + p) * vn;
}

void dgo_flux_llf(const double* uL, const double* uR, int dir, double gamma, double* f)
{
    double fL[4], fR[4];
    dgo_flux_phys(uL, dir, gamma, fL);
    dgo_flux_phys(uR, dir, gamma, fR);
    double lL = dgo_wavespeed(uL, dir, gamma), lR = dgo_wavespeed(uR, dir, gamma);
    double lam = lL > lR ? lL : lR;
    for (int v = 0; v < 4; ++v) f[v] = 0.5 * (fL[v] + fR[v]) - 0.5 * lam * (uR[v] - uL[v]);
}

/* logarithmic mean (x - y) / (ln x - ln y); for f^2 = ((x-y)/(x+y))^2 < 1e-4
   the series of 2 atanh(f) = ln(x/y) truncated after f^6 (Ismail & Roe 2009). */
double dgo_lnmean(double x, double y)
{
    double f = (x - y) / (x + y);
    double f2 = f * f;
    if (f2 < 1e-4) return (x + y) / (2.0 + f2 * (2.0 / 3.0 + f2 * (2.0 / 5.0 + f2 * (2.0 / 7.0))));
    return (x - y) / log(x / y);
}

void dgo_flux_ranocha(const double* uL, const double* uR, int dir, double gamma, double* f)
{
    double rL, v1L, v2L, pL, rR, v1R, v2R, pR;
    dgo_prim(uL, gamma, &rL, &v1L, &v2L, &pL);
    dgo_prim(uR, gamma, &rR, &v1R, &v2R, &pR);
    double rho_ln = dgo_lnmean(rL, rR);
    double zeta_ln = dgo_lnmean(rL / pL, rR / pR); /* log mean of rho/p */
    double v1a = 0.5 * (v1L + v1R), v2a = 0.5 * (v2L + v2R), pa = 0.5 * (pL + pR);
    double vnL = dir == 0 ? v1L : v2L, vnR = dir == 0 ? v1R : v2R;
    double vna = 0.5 * (vnL + vnR);
    double fr = rho_ln * vna;
    f[0] = fr;
    f[1] = fr * v1a + (dir == 0 ? pa : 0.0);
    f[2] = fr * v2a + (dir == 1 ? pa : 0.0);
    f[3] = fr * (0.5 * (v1L * v1R + v2L * v2R) + 1.0 / ((gamma - 1.0) * zeta_ln)) +
           0.5 * (pL * vnR + pR * vnL);
}

/* Chandrashekar (2013): with beta = rho / (2 p), log means rho^ln and beta^ln,
   arithmetic means a-bar, and p~ = rho-bar / (2 beta-bar),
     f_rho = rho^ln vn-bar,  f_m = f_rho v-bar + p~ n,
     f_E = f_rho (1 / (2 (gamma-1) beta^ln) - (|v_L|^2 + |v_R|^2) / 4) + v-bar . f_m.
   The energy flux is the one Tadmor's condition fixes for this mass and
   momentum flux (derived from [[w]] . f = [[rho vn]] with the entropy
   -rho s / (gamma - 1)). */
void dgo_flux_chandrashekar(const double* uL, const double* uR, int dir, double gamma, double* f)
{
    double rL, v1L, v2L, pL, rR, v1R, v2R, pR;
    dgo_prim(uL, gamma, &rL, &v1L, &v2L, &pL);
    dgo_prim(uR, gamma, &rR, &v1R, &v2R, &pR);
    double bL = rL / (2.0 * pL), bR = rR / (2.0 * pR);
    double rho_ln = dgo_lnmean(rL, rR), beta_ln = dgo_lnmean(bL, bR);
    double v1a = 0.5 * (v1L + v1R), v2a = 0.5 * (v2L + v2R);
    double pt = 0.5 * (rL + rR) / (bL + bR);
    double vna = dir == 0 ? v1a : v2a;
    double fr = rho_ln * vna;
    f[0] = fr;
    f[1] = fr * v1a + (dir == 0 ? pt : 0.0);
    f[2] = fr * v2a + (dir == 1 ? pt : 0.0);
    f[3] = fr * (1.0 / (2.0 * (gamma - 1.0) * beta_ln) -
                 0.25 * (v1L * v1L + v2L * v2L + v1R * v1R + v2R * v2R)) +
           v1a * f[1] + v2a * f[2];
}

/* the volume flux of a mesh: Ranocha (0) or Chandrashekar (1) */
void dgo_flux_volume(int kind, const double* uL, const double* uR, int dir, double gamma, double* f)
{
    if (kind == 1) dgo_flux_chandrashekar(uL, uR, dir, gamma, f);
    else dgo_flux_ranocha(uL, uR, dir, gamma, f);
}

/* Ghost state of a boundary node; the double Mach reflection (Sec. 3.5)
   and the jet (Sec. 3.6) use slip walls and characteristic inflow/outflow.  Face f is 0 x-,
   1 x+, 2 y-, 3 y+; the outward normal is the axis of direction f / 2, negated
   on the even faces.
   - slip wall: the interior state with its normal momentum reversed (the LLF
     flux against it carries no mass and no energy through the face);
   - characteristic: chosen by the outward normal velocity vn and the sound
     speed c of the interior state: vn <= -c (supersonic inflow) the exterior
     state; -c < vn <= 0 (subsonic inflow) the exterior density and velocity
     with the interior pressure; 0 < vn < c (subsonic outflow) the interior
     density and velocity with the exterior pressure; vn >= c (supersonic
     outflow) the interior state;
   - outflow: the interior state. */
void dgo_boundary_ghost(int kind, const double* ext, const double* ui, int f, double gamma,
                        double* ug)
{
    int dir = f / 2;
    for (int v = 0; v < 4; ++v) ug[v] = ui[v];
    if (kind == BC_WALL) {
        ug[1 + dir] = -ui[1 + dir];
        return;
    }
    if (kind != BC_CHARACTERISTIC) return;
    double r, v1, v2, p;
    dgo_prim(ui, gamma, &r, &v1, &v2, &p);
    double vn = (dir == 0 ? v1 : v2) * ((f & 1) ? 1.0 : -1.0);
    double c = sqrt(gamma * p / r);
    if (vn >= c) return;
    double re, v1e, v2e, pe;
    dgo_prim(ext, gamma, &re, &v1e, &v2e, &pe);
    if (vn <= -c) {
        for (int v = 0; v < 4; ++v) ug[v] = ext[v];
    } else if (vn <= 0.0) { /* exterior density and velocity, interior pressure */
        ug[0] = re;
        ug[1] = re * v1e;
        ug[2] = re * v2e;
        ug[3] = p / (gamma - 1.0) + 0.5 * re * (v1e * v1e + v2e * v2e);
    } else { /* interior density and velocity, exterior pressure */
        ug[3] = pe / (gamma - 1.0) + 0.5 * r * (v1 * v1 + v2 * v2);
    }
}

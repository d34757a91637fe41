/*
 * srmhd_oracle.c -- plain FP64 CPU oracle for one SSP-RK3 step of 3D ideal
 * special-relativistic MHD (flat space, Cartesian, periodic box).
 *
 * TEST INFRASTRUCTURE ONLY: called by the test suite, the package smoke check
 * and the CPU-baseline leg of the benchmark; never by the product path.  It is
 * written independently of the HIP library (no shared headers, helpers or
 * constant tables).  Built with -O2 -ffp-contract=off, no fast-math.
 *
 * What the paper fixes (arXiv 2401.03008):
 *   Sec. 2  -- the 8 conservation laws of ideal SRMHD in flat space, the
 *              definitions D = rho*Gamma, S = rho*h*Gamma^2 v + E x B,
 *              U = rho*h*Gamma^2 - p + (E^2+B^2)/2,
 *              W_ij = rho*h*Gamma^2 v_i v_j - E_i E_j - B_i B_j + p_tot d_ij,
 *              ideal E = -v x B, and the ideal-gas enthalpy
 *              h = 1 + gam/(gam-1) p/rho.
 *   Sec. 3  -- the semi-discrete point-value scheme: cell-centred conserved
 *              variables updated by differences of face fluxes, face-staggered
 *              B updated by the curl of edge electric fields; each Runge-Kutta
 *              substep is INT (face B to centres) + Newton inversion, REC of
 *              primitives at faces + upwind fluxes + stored fast speeds, DER
 *              (flux differences), UCT edge fields and their curl, then the
 *              RK update; the timestep comes once per full step from the
 *              global maximum of the stored characteristic speeds.
 * The paper prints none of the formulas of MP5, HLL, UCT, the Newton inversion
 * or the RK scheme.  The readings taken here (each a published method):
 *   - REC: MP5 of Suresh & Huynh (1997), alpha = 4, eps = 1e-10, applied to
 *     rho, v (3-velocity), p and the two transverse centred B components;
 *     a face state with rho <= 0, p <= 0 or v^2 >= 1 falls back to the
 *     adjacent cell value (first order) and is counted.
 *   - Fast speeds: the quadratic bound of Del Zanna et al. (2003) built from
 *     c_s^2 = gam p/(rho h), v_A^2 = b^2/(rho h + b^2),
 *     w^2 = c_s^2 + v_A^2 - c_s^2 v_A^2.
 *   - Fluxes: HLL (Harten, Lax & van Leer 1983) or LLF, second-order
 *     point-value fluxes (no high-order DER correction).
 *   - UCT: edge fields from the four reconstructed corner states weighted by
 *     the two-dimensional HLL formula of Londrillo & Del Zanna (2004).
 *   - INT: second-order face average.
 *   - Inversion: one-unknown Newton iteration in W = rho h Gamma^2, stopped
 *     when the step is below 1e-14 W or below the round-off resolution of
 *     the residual (8 ulps of the sum of its terms over the slope).
 *   - Time: SSP-RK3 of Shu & Osher (1988), dt = cfl / max_cells
 *     sum_d max(a+, a-)_d / dx_d from the first-stage speeds.
 * Variants the paper names without formulas (Sec. 3 and the benchmark
 * section): HO = YES (high-order INT and DER) and second-order time stepping
 * with linear reconstruction.  Readings:
 *   - HO INT: the sixth-order central interpolation of the six face values
 *     around the centre, weights (3, -25, 150, 150, -25, 3)/256.
 *   - HO DER: each point-value face flux f is replaced by
 *     Fhat = f - D2 f / 24 + 3 D4 f / 640 (D2, D4 the second and fourth
 *     undivided differences along the derivative direction), the sixth-order
 *     form whose differences give the derivative at the centre; applied to
 *     the fluid fluxes and to the edge fields of the curl.  The curl of
 *     corrected edge fields conserves the divergence taken with the same
 *     corrected differences of the face B, which is the div B diagnostic in
 *     this mode.
 *   - Linear reconstruction: slope = MC(v_i - v_{i-1}, v_{i+1} - v_i) with
 *     the monotonized-central limiter of van Leer (1977),
 *     MC(a, b) = sign(a) min(2|a|, 2|b|, |a + b|/2) if ab > 0, else 0;
 *     face values v_i +- slope/2; used for the fluxes and for UCT.
 *   - Second-order time: SSP-RK2, U1 = U0 + dt L(U0),
 *     U = 1/2 U0 + 1/2 (U1 + dt L(U1)).
 */
#include "srmhd_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MP5_ALPHA 4.0
#define MP5_EPS 1e-10
#define C2P_NOISE 8.0

/* ------------------------------------------------------------------------ */
/* Point physics (Sec. 2)                                                    */
/* ------------------------------------------------------------------------ */

/* Conserved variables from primitives: D, S, U of Sec. 2 with E = -v x B. */
void orc_prim2cons(double gam, const double *pr, double *u) {
  const double rho = pr[0], vx = pr[1], vy = pr[2], vz = pr[3], p = pr[4];
  const double Bx = pr[5], By = pr[6], Bz = pr[7];
  const double v2 = vx * vx + vy * vy + vz * vz;
  const double lor2 = 1.0 / (1.0 - v2);
  const double lor = sqrt(lor2);
  const double h = 1.0 + gam / (gam - 1.0) * p / rho;
  const double W = rho * h * lor2;
  /* E = -v x B */
  const double Ex = -(vy * Bz - vz * By);
  const double Ey = -(vz * Bx - vx * Bz);
  const double Ez = -(vx * By - vy * Bx);
  const double E2 = Ex * Ex + Ey * Ey + Ez * Ez;
  const double B2 = Bx * Bx + By * By + Bz * Bz;
  u[0] = rho * lor;
  u[1] = W * vx + (Ey * Bz - Ez * By);
  u[2] = W * vy + (Ez * Bx - Ex * Bz);
  u[3] = W * vz + (Ex * By - Ey * Bx);
  u[4] = W - p + 0.5 * (E2 + B2);
  u[5] = Bx;
  u[6] = By;
  u[7] = Bz;
}

/* Physical flux along direction d (0,1,2) of all 8 conserved components:
 * F_D = D v_d, F_S_i = W_i^d, F_U = S_d, F_B_i = v_d B_i - v_i B_d. */
void orc_flux(double gam, const double *pr, int d, double *f) {
  double u[8];
  orc_prim2cons(gam, pr, u);
  const double rho = pr[0], p = pr[4];
  const double v[3] = {pr[1], pr[2], pr[3]};
  const double B[3] = {pr[5], pr[6], pr[7]};
  const double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  const double lor2 = 1.0 / (1.0 - v2);
  const double h = 1.0 + gam / (gam - 1.0) * p / rho;
  const double W = rho * h * lor2;
  const double E[3] = {-(v[1] * B[2] - v[2] * B[1]), -(v[2] * B[0] - v[0] * B[2]),
                       -(v[0] * B[1] - v[1] * B[0])};
  const double E2 = E[0] * E[0] + E[1] * E[1] + E[2] * E[2];
  const double B2 = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
  const double ptot = p + 0.5 * (E2 + B2);
  f[0] = u[0] * v[d];
  for (int i = 0; i < 3; ++i) {
    f[1 + i] = W * v[i] * v[d] - E[i] * E[d] - B[i] * B[d] + (i == d ? ptot : 0.0);
  }
  f[4] = u[1 + d];
  for (int i = 0; i < 3; ++i) f[5 + i] = v[d] * B[i] - v[i] * B[d];
}

/* Fast characteristic speeds along d: the quadratic bound of Del Zanna et al.
 * (2003).  lp >= lm; at rest with B normal to d they are +-w. */
void orc_speeds(double gam, const double *pr, int d, double *lm, double *lp) {
  const double rho = pr[0], p = pr[4];
  const double v[3] = {pr[1], pr[2], pr[3]};
  const double B[3] = {pr[5], pr[6], pr[7]};
  const double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  const double lor2 = 1.0 / (1.0 - v2);
  const double rhoh = rho + gam / (gam - 1.0) * p;
  const double cs2 = gam * p / rhoh;
  const double B2 = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
  const double vB = v[0] * B[0] + v[1] * B[1] + v[2] * B[2];
  const double b2 = B2 / lor2 + vB * vB;
  const double va2 = b2 / (rhoh + b2);
  const double w2 = cs2 + va2 - cs2 * va2;
  const double vd = v[d];
  const double den = 1.0 - v2 * w2;
  double disc = w2 * (1.0 - v2) * ((1.0 - v2 * w2) - vd * vd * (1.0 - w2));
  if (disc < 0.0) disc = 0.0;
  const double sq = sqrt(disc);
  *lp = (vd * (1.0 - w2) + sq) / den;
  *lm = (vd * (1.0 - w2) - sq) / den;
}

/* ------------------------------------------------------------------------ */
/* Newton inversion (Sec. 3, first step of a substep)                        */
/* ------------------------------------------------------------------------ */

typedef struct {
  double D, U, S2, B2, tau2, gf;
} c2p_in;

/* v^2 as a function of W: from S = (W + B^2) v - (v.B) B and v.B = tau/W. */
static double c2p_v2(const c2p_in *q, double W) {
  const double WB = W + q->B2;
  return (q->S2 + q->tau2 * (2.0 * W + q->B2) / (W * W)) / (WB * WB);
}

/* f(W) = W - p + B^2 (1 + v^2)/2 - tau^2/(2 W^2) - U, its derivative, and
 * the sum of the magnitudes of the terms of f (its round-off scale). */
static void c2p_fun(const c2p_in *q, double W, double *f, double *fp, double *fs) {
  const double v2 = c2p_v2(q, W);
  const double sq = sqrt(1.0 - v2);
  const double p = q->gf * (W * (1.0 - v2) - q->D * sq);
  const double tb = 0.5 * q->B2 * (1.0 + v2), tt = 0.5 * q->tau2 / (W * W);
  *f = W - p + tb - tt - q->U;
  *fs = W + fabs(p) + tb + tt + q->U;
  const double dv2 = -2.0 * q->tau2 / (W * W * W * (W + q->B2)) - 2.0 * v2 / (W + q->B2);
  const double dp = q->gf * ((1.0 - v2) - W * dv2 + 0.5 * q->D * dv2 / sq);
  *fp = 1.0 - dp + 0.5 * q->B2 * dv2 + q->tau2 / (W * W * W);
}

static int c2p_usable(const c2p_in *q, double W) {
  return W > 0.0 && c2p_v2(q, W) < 1.0;
}

/* Recover primitives pr[8] from conserved u[8] (centred B in u[5..7]).
 * *W holds the initial guess and returns the converged W.  Returns 0 on
 * convergence, 1 if maxit was reached, 2 for unusable input (non-finite,
 * D <= 0 or U <= 0), 3 if the recovered pressure is not positive and no
 * floor is set.  A guess with W <= 0 or v^2(W) >= 1 is replaced by U, doubled
 * until usable; a Newton iterate that leaves the usable set is halved back
 * toward the previous iterate. */
int orc_con2prim(double gam, const double *u, double *W, int maxit, double tol,
                 double pfloor, double *pr, int *iters, int *floored) {
  for (int n = 0; n < 8; ++n)
    if (!isfinite(u[n])) return 2;
  c2p_in q;
  q.D = u[0];
  q.U = u[4];
  q.S2 = u[1] * u[1] + u[2] * u[2] + u[3] * u[3];
  q.B2 = u[5] * u[5] + u[6] * u[6] + u[7] * u[7];
  const double tau = u[1] * u[5] + u[2] * u[6] + u[3] * u[7];
  q.tau2 = tau * tau;
  q.gf = (gam - 1.0) / gam;
  if (!(q.D > 0.0) || !(q.U > 0.0)) return 2;

  double w = *W;
  if (!(isfinite(w) && c2p_usable(&q, w))) {
    w = q.U;
    for (int n = 0; n < 200 && !c2p_usable(&q, w); ++n) w *= 2.0;
  }
  /* Stop when the step is below tol*W or below the resolution of f itself:
   * f is a sum of terms of total magnitude fs, evaluated with an error of a
   * few ulps of fs, so a Newton step cannot resolve W better than
   * C2P_NOISE * DBL_EPSILON * fs / |f'|. */
  int it = 0, conv = 0;
  while (it < maxit) {
    ++it;
    double f, fp, fs;
    c2p_fun(&q, w, &f, &fp, &fs);
    double wn = w - f / fp;
    for (int n = 0; n < 100 && !(isfinite(wn) && c2p_usable(&q, wn)); ++n)
      wn = 0.5 * (wn + w);
    if (!isfinite(wn)) wn = w;
    const double dw = wn - w;
    w = wn;
    if (fabs(dw) <= fmax(tol * w, C2P_NOISE * DBL_EPSILON * fs / fabs(fp))) {
      conv = 1;
      break;
    }
  }
  *W = w;
  if (iters) *iters = it;

  const double v2 = c2p_v2(&q, w);
  const double sq = sqrt(1.0 - v2);
  const double a = tau / w, den = w + q.B2;
  pr[0] = q.D * sq;
  pr[1] = (u[1] + a * u[5]) / den;
  pr[2] = (u[2] + a * u[6]) / den;
  pr[3] = (u[3] + a * u[7]) / den;
  pr[4] = q.gf * (w * (1.0 - v2) - q.D * sq);
  pr[5] = u[5];
  pr[6] = u[6];
  pr[7] = u[7];
  if (floored) *floored = 0;
  if (pfloor > 0.0 && pr[4] < pfloor * pr[0]) {
    pr[4] = pfloor * pr[0];
    if (floored) *floored = 1;
  }
  if (!conv) return 1;
  if (!(pr[4] > 0.0)) return 3;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* REC: MP5 (Suresh & Huynh 1997)                                            */
/* ------------------------------------------------------------------------ */

static double minmod2(double a, double b) {
  if (a > 0.0 && b > 0.0) return a < b ? a : b;
  if (a < 0.0 && b < 0.0) return a > b ? a : b;
  return 0.0;
}

static double minmod4(double a, double b, double c, double d) {
  if (a > 0.0 && b > 0.0 && c > 0.0 && d > 0.0) return fmin(fmin(a, b), fmin(c, d));
  if (a < 0.0 && b < 0.0 && c < 0.0 && d < 0.0) return fmax(fmax(a, b), fmax(c, d));
  return 0.0;
}

/* Left-biased value at x_{i+1/2} from s = {v_{i-2}, v_{i-1}, v_i, v_{i+1},
 * v_{i+2}}.  The right-biased value at the same face is this function applied
 * to {v_{i+3}, v_{i+2}, v_{i+1}, v_i, v_{i-1}}. */
static double mp5_limit(const double *s, double vor);

double orc_mp5(const double *s) {
  const double vor = (2.0 * s[0] - 13.0 * s[1] + 47.0 * s[2] + 27.0 * s[3] - 3.0 * s[4]) / 60.0;
  return mp5_limit(s, vor);
}

/* The same limiter around the fifth-order interpolation of point values,
 * weights (3, -20, 90, 60, -5)/128: the REC of the HO scheme, whose DER
 * correction expects face point values. */
double orc_mp5_point(const double *s) {
  const double vor = (3.0 * s[0] - 20.0 * s[1] + 90.0 * s[2] + 60.0 * s[3] - 5.0 * s[4]) / 128.0;
  return mp5_limit(s, vor);
}

/* MP limiter of Suresh & Huynh around the unlimited value vor. */
static double mp5_limit(const double *s, double vor) {
  const double vm2 = s[0], vm1 = s[1], v0 = s[2], vp1 = s[3], vp2 = s[4];
  const double vmp = v0 + minmod2(vp1 - v0, MP5_ALPHA * (v0 - vm1));
  if ((vor - v0) * (vor - vmp) <= MP5_EPS) return vor;
  const double djm1 = vm2 - 2.0 * vm1 + v0;
  const double dj = vm1 - 2.0 * v0 + vp1;
  const double djp1 = v0 - 2.0 * vp1 + vp2;
  const double dm4p = minmod4(4.0 * dj - djp1, 4.0 * djp1 - dj, dj, djp1);
  const double dm4m = minmod4(4.0 * dj - djm1, 4.0 * djm1 - dj, dj, djm1);
  const double vul = v0 + MP5_ALPHA * (v0 - vm1);
  const double vav = 0.5 * (v0 + vp1);
  const double vmd = vav - 0.5 * dm4p;
  const double vlc = v0 + 0.5 * (v0 - vm1) + 4.0 / 3.0 * dm4m;
  const double vmin = fmax(fmin(fmin(v0, vp1), vmd), fmin(fmin(v0, vul), vlc));
  const double vmax = fmin(fmax(fmax(v0, vp1), vmd), fmax(fmax(v0, vul), vlc));
  return vor + minmod2(vmin - vor, vmax - vor);
}

/* ------------------------------------------------------------------------ */
/* Linear REC with the MC limiter; high-order INT and DER                   */
/* ------------------------------------------------------------------------ */

/* Left-biased value at x_{i+1/2} from s = {v_{i-1}, v_i, v_{i+1}}; the
 * right-biased value is this function of {v_{i+2}, v_{i+1}, v_i}. */
double orc_mc(const double *s) {
  const double a = s[1] - s[0], b = s[2] - s[1];
  double slope = 0.0;
  if (a * b > 0.0) {
    const double m = fmin(fmin(2.0 * fabs(a), 2.0 * fabs(b)), 0.5 * fabs(a + b));
    slope = a > 0.0 ? m : -m;
  }
  return s[1] + 0.5 * slope;
}

/* Centre value from the face values b = {B_{i-5/2}, ..., B_{i+5/2}}. */
double orc_int_ho(const double *b) {
  return (3.0 * b[0] - 25.0 * b[1] + 150.0 * b[2] + 150.0 * b[3] - 25.0 * b[4] + 3.0 * b[5]) /
         256.0;
}

/* Corrected flux at the middle face of g = {f_{-2}, ..., f_{+2}}. */
static double fhat_ho(const double *g) {
  const double d2 = g[3] - 2.0 * g[2] + g[1];
  const double d4 = g[4] - 4.0 * g[3] + 6.0 * g[2] - 4.0 * g[1] + g[0];
  return g[2] - d2 / 24.0 + 3.0 * d4 / 640.0;
}

/* Fhat(i+1/2) - Fhat(i-1/2) from f = {f_{i-5/2}, ..., f_{i+5/2}}. */
double orc_der_ho(const double *f) { return fhat_ho(f + 1) - fhat_ho(f); }

/* ------------------------------------------------------------------------ */
/* Upwind face flux (HLL / LLF)                                              */
/* ------------------------------------------------------------------------ */

/* fhat[8] from the left/right primitive states at a face normal to d;
 * returns the upwind speeds a+ (ap) and a- (am), both >= 0. */
void orc_riemann(int kind, double gam, const double *prL, const double *prR,
                 int d, double *fhat, double *ap, double *am) {
  double uL[8], uR[8], fL[8], fR[8], lmL, lpL, lmR, lpR;
  orc_prim2cons(gam, prL, uL);
  orc_prim2cons(gam, prR, uR);
  orc_flux(gam, prL, d, fL);
  orc_flux(gam, prR, d, fR);
  orc_speeds(gam, prL, d, &lmL, &lpL);
  orc_speeds(gam, prR, d, &lmR, &lpR);
  double aplus, aminus;
  if (kind == 1) {
    double m = fmax(fmax(fabs(lmL), fabs(lpL)), fmax(fabs(lmR), fabs(lpR)));
    aplus = aminus = m;
  } else {
    aplus = fmax(0.0, fmax(lpL, lpR));
    aminus = fmax(0.0, fmax(-lmL, -lmR));
  }
  const double s = aplus + aminus;
  for (int n = 0; n < 8; ++n) {
    if (s > 0.0)
      fhat[n] = (aplus * fL[n] + aminus * fR[n] - aplus * aminus * (uR[n] - uL[n])) / s;
    else
      fhat[n] = 0.5 * (fL[n] + fR[n]);
  }
  *ap = aplus;
  *am = aminus;
}

/* Two-dimensional upwind (HLL-type) edge field of Londrillo & Del Zanna
 * (2004) for an edge along k, with a = side along p and b = side along q
 * where (p, q, k) is cyclic.  Eab = {E_LL, E_LR, E_RL, E_RR} (first letter:
 * p-side, second: q-side).  axp/axm are the p-direction speeds at the edge,
 * ayp/aym the q-direction ones; byL/byR is B_q reconstructed along p, bxL/bxR
 * is B_p reconstructed along q. */
double orc_uct_formula(const double *Eab, double axp, double axm, double ayp,
                       double aym, double byL, double byR, double bxL,
                       double bxR) {
  const double sx = axp + axm, sy = ayp + aym;
  double e, dx, dy;
  if (sx > 0.0 && sy > 0.0)
    e = (axp * ayp * Eab[0] + axp * aym * Eab[1] + axm * ayp * Eab[2] + axm * aym * Eab[3]) /
        (sx * sy);
  else if (sx > 0.0)
    e = (axp * (Eab[0] + Eab[1]) + axm * (Eab[2] + Eab[3])) / (2.0 * sx);
  else if (sy > 0.0)
    e = (ayp * (Eab[0] + Eab[2]) + aym * (Eab[1] + Eab[3])) / (2.0 * sy);
  else
    e = 0.25 * (Eab[0] + Eab[1] + Eab[2] + Eab[3]);
  dx = sx > 0.0 ? axp * axm / sx : 0.0;
  dy = sy > 0.0 ? ayp * aym / sy : 0.0;
  return e + dx * (byR - byL) - dy * (bxR - bxL);
}

/* ------------------------------------------------------------------------ */
/* Grid helpers                                                              */
/* ------------------------------------------------------------------------ */

static long ncells(const orc_cfg *c) { return (long)c->nx * c->ny * c->nz; }

/* Index of cell (i,j,k) shifted by off along direction d, periodic. */
static long idx_shift(const orc_cfg *c, int i, int j, int k, int d, int off) {
  int n[3] = {c->nx, c->ny, c->nz};
  int q[3] = {i, j, k};
  q[d] = ((q[d] + off) % n[d] + n[d]) % n[d];
  return ((long)q[2] * c->ny + q[1]) * c->nx + q[0];
}

static double cell_width(const orc_cfg *c, int d) {
  return d == 0 ? c->lx / c->nx : (d == 1 ? c->ly / c->ny : c->lz / c->nz);
}

/* INT: centred B_d is the mean of the two d-faces (second order), or the
 * sixth-order interpolation of the six nearest d-faces (HO). */
static double int_bc(const orc_cfg *c, double *const *bf, int i, int j, int k, int d) {
  if (c->ho) {
    double b[6];
    for (int m = 0; m < 6; ++m) b[m] = bf[d][idx_shift(c, i, j, k, d, m - 3)];
    return orc_int_ho(b);
  }
  return 0.5 * (bf[d][idx_shift(c, i, j, k, d, -1)] + bf[d][idx_shift(c, i, j, k, d, 0)]);
}

/* d/dx_d at the centre of cell (i,j,k) of a quantity a given at the +d
 * faces (a[id] sits at +1/2 along d): plain difference, or the HO form. */
static double der_at(const orc_cfg *c, const double *a, int i, int j, int k, int d, double dx) {
  if (c->ho) {
    double f[6];
    for (int m = 0; m < 6; ++m) f[m] = a[idx_shift(c, i, j, k, d, m - 3)];
    return orc_der_ho(f) / dx;
  }
  return (a[idx_shift(c, i, j, k, d, 0)] - a[idx_shift(c, i, j, k, d, -1)]) / dx;
}

/* Left and right values at the face between st[2] and st[3] of the six
 * values st = {v_{i-2}, ..., v_{i+3}}: MP5 (kind 0), linear MC (1), or MP5
 * around the point-value interpolation (2, the HO scheme). */
static void rec_pair(int recon, const double *st, double *l, double *r) {
  if (recon == 2) {
    const double s[5] = {st[0], st[1], st[2], st[3], st[4]};
    const double t[5] = {st[5], st[4], st[3], st[2], st[1]};
    *l = orc_mp5_point(s);
    *r = orc_mp5_point(t);
    return;
  }
  if (recon == 1) {
    const double s[3] = {st[1], st[2], st[3]};
    const double t[3] = {st[4], st[3], st[2]};
    *l = orc_mc(s);
    *r = orc_mc(t);
    return;
  }
  const double s[5] = {st[0], st[1], st[2], st[3], st[4]};
  const double t[5] = {st[5], st[4], st[3], st[2], st[1]};
  *l = orc_mp5(s);
  *r = orc_mp5(t);
}

static int rec_kind(const orc_cfg *c) { return c->recon == 1 ? 1 : (c->ho ? 2 : 0); }

/* Left and right values (MP5, or linear MC) at the +face along d of cell
 * (i,j,k). */
static void rec_face(const orc_cfg *c, const double *a, int i, int j, int k, int d,
                     double *vl, double *vr) {
  double st[6];
  for (int m = 0; m < 6; ++m) st[m] = a[idx_shift(c, i, j, k, d, m - 2)];
  rec_pair(rec_kind(c), st, vl, vr);
}

static int state_ok(const double *pr) {
  const double v2 = pr[1] * pr[1] + pr[2] * pr[2] + pr[3] * pr[3];
  return pr[0] > 0.0 && pr[4] > 0.0 && v2 < 1.0;
}

/* Everything computed at the +face along d of cell (i,j,k). */
typedef struct {
  double fhat[5]; /* D, Sx, Sy, Sz, U */
  double ap, am;
  double v[6];    /* left vx, vy, vz; right vx, vy, vz */
} face_out;

/* REC of rho, v, p and the two transverse centred B (MP5 along d), normal B
 * from the face, first-order fallback of an unusable side, upwind flux.
 * Returns the number of sides that fell back (0..2). */
static int face_solve(const orc_cfg *c, double *const *prim, double *const *bf, int i, int j,
                      int k, int d, face_out *o) {
  const long id = ((long)k * c->ny + j) * c->nx + i;
  const long ip = idx_shift(c, i, j, k, d, 1);
  double prL[8], prR[8];
  int nfb = 0;
  for (int n = 0; n < 8; ++n) {
    if (n == 5 + d) continue;
    rec_face(c, prim[n], i, j, k, d, &prL[n], &prR[n]);
  }
  prL[5 + d] = prR[5 + d] = bf[d][id];
  if (!state_ok(prL)) {
    for (int n = 0; n < 8; ++n)
      if (n != 5 + d) prL[n] = prim[n][id];
    ++nfb;
  }
  if (!state_ok(prR)) {
    for (int n = 0; n < 8; ++n)
      if (n != 5 + d) prR[n] = prim[n][ip];
    ++nfb;
  }
  double f8[8];
  orc_riemann(c->riemann, c->gam, prL, prR, d, f8, &o->ap, &o->am);
  for (int n = 0; n < 5; ++n) o->fhat[n] = f8[n];
  for (int m = 0; m < 3; ++m) {
    o->v[m] = prL[1 + m];
    o->v[3 + m] = prR[1 + m];
  }
  return nfb;
}

/* Inputs of one edge along k, (p, q, k) cyclic, edge at +1/2 in p and q:
 * p-face velocity components p and q of side a (0 left, 1 right along p) at
 * q-offsets -2..+3; face B_p at q-offsets -2..+3; face B_q at p-offsets
 * -2..+3; p-face speeds at q-offsets 0, +1; q-face speeds at p-offsets 0, +1. */
typedef struct {
  double vp[2][6], vq[2][6], bp[6], bq[6];
  double app[2], amp[2], aqp[2], aqm[2];
} edge_in;


/* UCT edge field: corner states by REC along q of the p-face states, B_p
 * along q, B_q along p, E^{ab} = v_q^{ab} B_p^b - v_p^{ab} B_q^a, edge speeds
 * the maxima over the two adjacent faces of each direction. */
static double edge_from(int recon, const edge_in *e) {
  double vp[2][2], vq[2][2], bpL, bpR, bqL, bqR;
  for (int a = 0; a < 2; ++a) {
    rec_pair(recon, e->vp[a], &vp[a][0], &vp[a][1]);
    rec_pair(recon, e->vq[a], &vq[a][0], &vq[a][1]);
  }
  rec_pair(recon, e->bp, &bpL, &bpR);
  rec_pair(recon, e->bq, &bqL, &bqR);
  double Eab[4];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      const double bpb = b ? bpR : bpL;
      const double bqa = a ? bqR : bqL;
      Eab[2 * a + b] = vq[a][b] * bpb - vp[a][b] * bqa;
    }
  const double axp = fmax(e->app[0], e->app[1]);
  const double axm = fmax(e->amp[0], e->amp[1]);
  const double ayp = fmax(e->aqp[0], e->aqp[1]);
  const double aym = fmax(e->aqm[0], e->aqm[1]);
  return orc_uct_formula(Eab, axp, axm, ayp, aym, bqL, bqR, bpL, bpR);
}

/* ------------------------------------------------------------------------ */
/* Grid operations                                                           */
/* ------------------------------------------------------------------------ */

/* Conserved state from cell-centred rho, v, p (prim5) and face B (bf); the
 * centred B entering the conserved variables is INT of the face values, so
 * that the inversion of the result returns prim5 to round-off.  W is set to
 * rho h Gamma^2. */
int orc_init(const orc_cfg *c, double *const *prim5, double *const *bf, double **cons,
             double *W) {
#pragma omp parallel for schedule(static)
  for (int k = 0; k < c->nz; ++k)
    for (int j = 0; j < c->ny; ++j)
      for (int i = 0; i < c->nx; ++i) {
        const long id = ((long)k * c->ny + j) * c->nx + i;
        double pr[8], u[8];
        for (int n = 0; n < 5; ++n) pr[n] = prim5[n][id];
        for (int d = 0; d < 3; ++d) pr[5 + d] = int_bc(c, bf, i, j, k, d);
        orc_prim2cons(c->gam, pr, u);
        for (int n = 0; n < 5; ++n) cons[n][id] = u[n];
        const double v2 = pr[1] * pr[1] + pr[2] * pr[2] + pr[3] * pr[3];
        W[id] = (pr[0] + c->gam / (c->gam - 1.0) * pr[4]) / (1.0 - v2);
      }
  return 0;
}

/* INT + inversion over the grid.  prim[0..7] receives rho, vx, vy, vz, p,
 * Bcx, Bcy, Bcz; W is the guess on entry and the converged W on exit; iters
 * (optional) receives the per-cell Newton count.  Returns the number of cells
 * whose inversion failed. */
int orc_c2p(const orc_cfg *c, double *const *cons, double *const *bf, double *W,
            double **prim, int *iters, orc_stats *st) {
  const long N = ncells(c);
  int *it = (int *)malloc(sizeof(int) * N);
  char *fl = (char *)malloc(N);
  int *rc = (int *)malloc(sizeof(int) * N);
#pragma omp parallel for schedule(static)
  for (int k = 0; k < c->nz; ++k)
    for (int j = 0; j < c->ny; ++j)
      for (int i = 0; i < c->nx; ++i) {
        const long id = ((long)k * c->ny + j) * c->nx + i;
        double u[8], pr[8];
        for (int n = 0; n < 5; ++n) u[n] = cons[n][id];
        for (int d = 0; d < 3; ++d) u[5 + d] = int_bc(c, bf, i, j, k, d);
        int nit = 0, flo = 0;
        rc[id] = orc_con2prim(c->gam, u, &W[id], c->maxit, c->tol, c->pfloor, pr, &nit, &flo);
        it[id] = nit;
        fl[id] = (char)flo;
        for (int n = 0; n < 8; ++n) prim[n][id] = pr[n];
      }
  int nfail = 0;
  for (long id = 0; id < N; ++id) {
    if (rc[id] != 0) ++nfail;
    if (iters) iters[id] = it[id];
    if (st) {
      st->newton_iters += it[id];
      st->newton_hist[it[id] < 31 ? it[id] : 31] += 1;
      if (rc[id] != 0) st->c2p_fail += 1;
      st->floors += fl[id];
    }
  }
  free(it);
  free(fl);
  free(rc);
  return nfail;
}

/* Spatial operator L(U) of the semi-discrete scheme (Sec. 3):
 *   rhs[0..4] = -sum_d (Fhat(+face) - Fhat(-face)) / dx_d   (cell centres)
 *   rhs[5+d]  = -(curl_h E)_d at the d-faces                 (face B)
 * and amax = max over cells of sum_d max(a+, a-)_d / dx_d at the cell's
 * +faces.  Optional outputs (any may be NULL): fhat[5*d + n] face fluxes,
 * apm[2*d + 0/1] = a+/a- at the d-faces, face_v[6*d + 3*s + m] velocity
 * component m of side s (0 = left, 1 = right) at the d-faces, edge_e[k] the
 * upwind edge fields. */
int orc_rhs(const orc_cfg *c, double *const *prim, double *const *bf, double **rhs,
            double *amax, double **fhat_out, double **apm_out, double **fv_out,
            double **edge_out, orc_stats *st) {
  const long N = ncells(c);
  double *fh[15], *apm[6], *fv[18], *ee[3];
  for (int n = 0; n < 15; ++n) fh[n] = (double *)malloc(sizeof(double) * N);
  for (int n = 0; n < 6; ++n) apm[n] = (double *)malloc(sizeof(double) * N);
  for (int n = 0; n < 18; ++n) fv[n] = (double *)malloc(sizeof(double) * N);
  for (int n = 0; n < 3; ++n) ee[n] = (double *)malloc(sizeof(double) * N);
  long nfb = 0;

  /* REC + face physics + upwind flux, per direction. */
  for (int d = 0; d < 3; ++d) {
#pragma omp parallel for schedule(static) reduction(+ : nfb)
    for (int k = 0; k < c->nz; ++k)
      for (int j = 0; j < c->ny; ++j)
        for (int i = 0; i < c->nx; ++i) {
          const long id = ((long)k * c->ny + j) * c->nx + i;
          face_out fo;
          nfb += face_solve(c, prim, bf, i, j, k, d, &fo);
          for (int n = 0; n < 5; ++n) fh[5 * d + n][id] = fo.fhat[n];
          apm[2 * d][id] = fo.ap;
          apm[2 * d + 1][id] = fo.am;
          for (int m = 0; m < 6; ++m) fv[6 * d + m][id] = fo.v[m];
        }
  }

  /* CFL maximum. */
  const double dxs[3] = {cell_width(c, 0), cell_width(c, 1), cell_width(c, 2)};
  double amx = 0.0;
  for (long id = 0; id < N; ++id) {
    double s = 0.0;
    for (int d = 0; d < 3; ++d) s += fmax(apm[2 * d][id], apm[2 * d + 1][id]) / dxs[d];
    if (s > amx) amx = s;
  }
  if (amax) *amax = amx;

  /* UCT: edge along kk, from the stored face arrays. */
  for (int kk = 0; kk < 3; ++kk) {
    const int p = (kk + 1) % 3, q = (kk + 2) % 3;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < c->nz; ++k)
      for (int j = 0; j < c->ny; ++j)
        for (int i = 0; i < c->nx; ++i) {
          const long id = ((long)k * c->ny + j) * c->nx + i;
          edge_in e;
          for (int m = 0; m < 6; ++m) {
            const long iq = idx_shift(c, i, j, k, q, m - 2);
            for (int a = 0; a < 2; ++a) {
              e.vp[a][m] = fv[6 * p + 3 * a + p][iq];
              e.vq[a][m] = fv[6 * p + 3 * a + q][iq];
            }
            e.bp[m] = bf[p][iq];
            e.bq[m] = bf[q][idx_shift(c, i, j, k, p, m - 2)];
          }
          const long idq = idx_shift(c, i, j, k, q, 1);
          const long idp = idx_shift(c, i, j, k, p, 1);
          e.app[0] = apm[2 * p][id];
          e.app[1] = apm[2 * p][idq];
          e.amp[0] = apm[2 * p + 1][id];
          e.amp[1] = apm[2 * p + 1][idq];
          e.aqp[0] = apm[2 * q][id];
          e.aqp[1] = apm[2 * q][idp];
          e.aqm[0] = apm[2 * q + 1][id];
          e.aqm[1] = apm[2 * q + 1][idp];
          ee[kk][id] = edge_from(rec_kind(c), &e);
        }
  }

  /* DER: flux differences and curl of E. */
#pragma omp parallel for schedule(static)
  for (int k = 0; k < c->nz; ++k)
    for (int j = 0; j < c->ny; ++j)
      for (int i = 0; i < c->nx; ++i) {
        const long id = ((long)k * c->ny + j) * c->nx + i;
        for (int n = 0; n < 5; ++n) {
          double s = 0.0;
          for (int d = 0; d < 3; ++d) s += der_at(c, fh[5 * d + n], i, j, k, d, dxs[d]);
          rhs[n][id] = -s;
        }
        /* dB_d/dt = -(curl E)_d, (curl E)_d = d_p E_q - d_q E_p, (d,p,q) cyclic;
         * E_q sits at +1/2 along p and E_p at +1/2 along q */
        for (int d = 0; d < 3; ++d) {
          const int p = (d + 1) % 3, q = (d + 2) % 3;
          const double dpEq = der_at(c, ee[q], i, j, k, p, dxs[p]);
          const double dqEp = der_at(c, ee[p], i, j, k, q, dxs[q]);
          rhs[5 + d][id] = -(dpEq - dqEp);
        }
      }

  if (st) st->recon_fallbacks += nfb;
  for (int n = 0; n < 15; ++n) {
    if (fhat_out && fhat_out[n]) memcpy(fhat_out[n], fh[n], sizeof(double) * N);
    free(fh[n]);
  }
  for (int n = 0; n < 6; ++n) {
    if (apm_out && apm_out[n]) memcpy(apm_out[n], apm[n], sizeof(double) * N);
    free(apm[n]);
  }
  for (int n = 0; n < 18; ++n) {
    if (fv_out && fv_out[n]) memcpy(fv_out[n], fv[n], sizeof(double) * N);
    free(fv[n]);
  }
  for (int n = 0; n < 3; ++n) {
    if (edge_out && edge_out[n]) memcpy(edge_out[n], ee[n], sizeof(double) * N);
    free(ee[n]);
  }
  return 0;
}

/* Coordinates of (i,j,k) shifted by off along d, periodic. */
static void shift_cell(const orc_cfg *c, int *q, int d, int off) {
  const int n[3] = {c->nx, c->ny, c->nz};
  q[d] = ((q[d] + off) % n[d] + n[d]) % n[d];
}

/* Edge field along kk at the edge +1/2 in p and q of cell q0, computed from
 * scratch (face states re-solved), with the same arithmetic as orc_rhs. */
static double edge_at(const orc_cfg *c, double *const *prim, double *const *bf, const int *q0,
                      int kk) {
  const int p = (kk + 1) % 3, q = (kk + 2) % 3;
  edge_in e;
  for (int m = 0; m < 6; ++m) {
    int a3[3] = {q0[0], q0[1], q0[2]};
    shift_cell(c, a3, q, m - 2);
    face_out fo;
    face_solve(c, prim, bf, a3[0], a3[1], a3[2], p, &fo);
    for (int a = 0; a < 2; ++a) {
      e.vp[a][m] = fo.v[3 * a + p];
      e.vq[a][m] = fo.v[3 * a + q];
    }
    if (m == 2) {
      e.app[0] = fo.ap;
      e.amp[0] = fo.am;
    }
    if (m == 3) {
      e.app[1] = fo.ap;
      e.amp[1] = fo.am;
    }
    e.bp[m] = bf[p][((long)a3[2] * c->ny + a3[1]) * c->nx + a3[0]];
    int b3[3] = {q0[0], q0[1], q0[2]};
    shift_cell(c, b3, p, m - 2);
    e.bq[m] = bf[q][((long)b3[2] * c->ny + b3[1]) * c->nx + b3[0]];
  }
  for (int m = 0; m < 2; ++m) {
    int a3[3] = {q0[0], q0[1], q0[2]};
    shift_cell(c, a3, p, m);
    face_out fo;
    face_solve(c, prim, bf, a3[0], a3[1], a3[2], q, &fo);
    e.aqp[m] = fo.ap;
    e.aqm[m] = fo.am;
  }
  return edge_from(rec_kind(c), &e);
}

/* L(U) at the listed cells only (linear indices cells[0..ncells-1]), with the
 * arithmetic of orc_rhs: out[8*s + n] for n = D, Sx, Sy, Sz, U, Bx, By, Bz
 * (face B at the cell's +faces).  For sampled checks of large grids. */
int orc_rhs_cells(const orc_cfg *c, double *const *prim, double *const *bf, int ncells,
                  const long *cells, double *out) {
  const double dxs[3] = {cell_width(c, 0), cell_width(c, 1), cell_width(c, 2)};
  /* faces (or edges) at offsets m0 .. m0+nm-1 along the derivative direction */
  const int m0 = c->ho ? -3 : -1, nm = c->ho ? 6 : 2;
#pragma omp parallel for schedule(dynamic)
  for (int sidx = 0; sidx < ncells; ++sidx) {
    const long id = cells[sidx];
    const int q0[3] = {(int)(id % c->nx), (int)((id / c->nx) % c->ny),
                       (int)(id / ((long)c->nx * c->ny))};
    double fl[3][5][6];
    for (int d = 0; d < 3; ++d)
      for (int m = 0; m < nm; ++m) {
        int a3[3] = {q0[0], q0[1], q0[2]};
        shift_cell(c, a3, d, m0 + m);
        face_out fo;
        face_solve(c, prim, bf, a3[0], a3[1], a3[2], d, &fo);
        for (int n = 0; n < 5; ++n) fl[d][n][m] = fo.fhat[n];
      }
    for (int n = 0; n < 5; ++n) {
      double s = 0.0;
      for (int d = 0; d < 3; ++d)
        s += c->ho ? orc_der_ho(fl[d][n]) / dxs[d] : (fl[d][n][1] - fl[d][n][0]) / dxs[d];
      out[8L * sidx + n] = -s;
    }
    for (int d = 0; d < 3; ++d) {
      const int p = (d + 1) % 3, q = (d + 2) % 3;
      double eq[6], ep[6];
      for (int m = 0; m < nm; ++m) {
        int a3[3] = {q0[0], q0[1], q0[2]};
        int b3[3] = {q0[0], q0[1], q0[2]};
        shift_cell(c, a3, p, m0 + m);
        shift_cell(c, b3, q, m0 + m);
        eq[m] = edge_at(c, prim, bf, a3, q);
        ep[m] = edge_at(c, prim, bf, b3, p);
      }
      const double dpEq = c->ho ? orc_der_ho(eq) / dxs[p] : (eq[1] - eq[0]) / dxs[p];
      const double dqEp = c->ho ? orc_der_ho(ep) / dxs[q] : (ep[1] - ep[0]) / dxs[q];
      out[8L * sidx + 5 + d] = -(dpEq - dqEp);
    }
  }
  return 0;
}

/* nsteps full SSP-RK3 steps (Shu & Osher 1988):
 *   U1 = U0 + dt L(U0);  U2 = 3/4 U0 + 1/4 (U1 + dt L(U1));
 *   U  = 1/3 U0 + 2/3 (U2 + dt L(U2)),
 * or, with time_order 2, SSP-RK2 steps:
 *   U1 = U0 + dt L(U0);  U  = 1/2 U0 + 1/2 (U1 + dt L(U1)),
 * applied to the 5 cell-centred arrays and the 3 face-B arrays.  dt comes from
 * the first stage of each step (or cfg dt_fixed).  W is the Newton guess,
 * updated by every inversion.  Returns the number of failed inversions. */
int orc_step(const orc_cfg *c, double **cons, double **bf, double *W, int nsteps,
             double *t, double *dt_last, orc_stats *st) {
  const long N = ncells(c);
  double *u0[8], *pr[8], *rh[8], *cur[8];
  for (int n = 0; n < 8; ++n) {
    u0[n] = (double *)malloc(sizeof(double) * N);
    pr[n] = (double *)malloc(sizeof(double) * N);
    rh[n] = (double *)malloc(sizeof(double) * N);
    cur[n] = n < 5 ? cons[n] : bf[n - 5];
  }
  int nfail = 0;
  double dt = 0.0;
  for (int step = 0; step < nsteps; ++step) {
    for (int n = 0; n < 8; ++n) memcpy(u0[n], cur[n], sizeof(double) * N);
    const int nstage = c->time_order == 2 ? 2 : 3;
    for (int s = 1; s <= nstage; ++s) {
      nfail += orc_c2p(c, cons, bf, W, pr, NULL, st);
      double amax = 0.0;
      orc_rhs(c, pr, bf, rh, &amax, NULL, NULL, NULL, NULL, st);
      if (s == 1) dt = c->dt_fixed > 0.0 ? c->dt_fixed : c->cfl / amax;
      for (int n = 0; n < 8; ++n) {
        double *a = cur[n];
        const double *a0 = u0[n], *r = rh[n];
#pragma omp parallel for schedule(static)
        for (long id = 0; id < N; ++id) {
          if (s == 1)
            a[id] = a0[id] + dt * r[id];
          else if (nstage == 2)
            a[id] = 0.5 * a0[id] + 0.5 * (a[id] + dt * r[id]);
          else if (s == 2)
            a[id] = 0.75 * a0[id] + 0.25 * (a[id] + dt * r[id]);
          else
            a[id] = (1.0 / 3.0) * a0[id] + (2.0 / 3.0) * (a[id] + dt * r[id]);
        }
      }
    }
    if (t) *t += dt;
  }
  if (dt_last) *dt_last = dt;
  for (int n = 0; n < 8; ++n) {
    free(u0[n]);
    free(pr[n]);
    free(rh[n]);
  }
  return nfail;
}

/* max over cells of |div_h B| = |sum_d (B_d(+face) - B_d(-face)) / dx_d|,
 * or with HO the same sum of corrected differences (the divergence that the
 * HO curl keeps constant). */
double orc_divb_max(const orc_cfg *c, double *const *bf) {
  double m = 0.0;
  for (int k = 0; k < c->nz; ++k)
    for (int j = 0; j < c->ny; ++j)
      for (int i = 0; i < c->nx; ++i) {
        double s = 0.0;
        for (int d = 0; d < 3; ++d) s += der_at(c, bf[d], i, j, k, d, cell_width(c, d));
        if (fabs(s) > m) m = fabs(s);
      }
  return m;
}

/* Plain serial sums of D, Sx, Sy, Sz, U and of the three face-B arrays. */
void orc_sums(const orc_cfg *c, double *const *cons, double *const *bf, double *sums) {
  const long N = ncells(c);
  for (int n = 0; n < 8; ++n) {
    const double *a = n < 5 ? cons[n] : bf[n - 5];
    double s = 0.0;
    for (long id = 0; id < N; ++id) s += a[id];
    sums[n] = s;
  }
}

/* Number of OpenMP threads the grid operations use. */
int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Set that number (n >= 1); no effect without OpenMP. */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/*
 * nyx_oracle.c -- plain, slow FP64 CPU oracle of the Nyx comoving gas step.
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the CPU
 * baseline of the benchmark.  It shares no code with the HIP library.
 *
 * What it computes (Almgren et al., "Nyx"):
 *   - state U = (rho, a rho U, a^2 rho E, a^2 rho e) and the flux, S_e and S_g
 *     terms of Sec. 3.2 Gas Dynamics (eqs. for U, F, S_e, S_g);
 *   - the comoving Euler equations of Sec. 2.2; the a*adot*(2 - 3(gamma-1))
 *     rho e expansion term of the two energy equations vanishes at gamma = 5/3
 *     and is applied, predictor-corrector like S_g, for any other gamma;
 *   - an unsplit Godunov method with characteristic tracing and full corner
 *     coupling, PPM edge states, a reference state built from the fastest
 *     wave moving toward the interface, and an iterative two-shock Riemann
 *     solver (Sec. 3.2; the method papers it cites fix the details);
 *   - the predictor U* = U^n - dt div F^{n+1/2} + dt S_e + dt S_g^n of
 *     Sec. 3.6 Step 2 and the corrector U^{n+1} = U* + dt/2 (S_g* - S_g^n) of
 *     Step 6, with heating/cooling absent;
 *   - the dual-energy synchronisation with threshold 1e-4 (Sec. 3.6, Step 6);
 *   - the hydro CFL time step (Sec. 3.5).
 * Every formula is evaluated exactly in the order written here (no FMA: the
 * build uses -ffp-contract=off), one stage at a time over whole-box arrays.
 * The stage numbering O1..O13 follows the design notes of this repository.
 */
#include "nyx_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* Flattening constants of Colella & Woodward (1984), cited by the PPM scheme
 * of Sec. 3.2. */
#define FLAT_EPS 0.33
#define FLAT_OMEGA1 0.75
#define FLAT_OMEGA2 10.0

/* Stage markers for the operation-count build (oracle/opcount.cpp), which
 * compiles this file with a counting number type and attributes every
 * floating-point operation to the stage and, inside the two-shock solver, to
 * the Newton iteration that is running.  They do nothing here. */
#ifndef NYXO_STAGE
#define NYXO_STAGE(s) ((void)0)
#endif
#ifndef NYXO_ITER
#define NYXO_ITER(on) ((void)0)
#endif

static double dmax(double a, double b) { return a > b ? a : b; }
/* kinetic energy |m|^2 / (2 rho) of a momentum m in the stored variables */
static double kinetic(const double* m, double rho) {
  return (0.5 * ((m[0] * m[0] + m[1] * m[1]) + m[2] * m[2])) / rho;
}
static double dmin(double a, double b) { return a < b ? a : b; }

/* ------------------------------------------------------------------ */
/* Box geometry                                                       */
/* ------------------------------------------------------------------ */
typedef struct {
  int n[3];
  int ng;
  long px, py, pz; /* padded extents */
  long P;          /* padded cells per component */
  long ex, ey, ez; /* extents of the [-1, n] cell range */
  long E;
} Box;

static void box_init(Box* b, int nx, int ny, int nz, int ng) {
  b->n[0] = nx; b->n[1] = ny; b->n[2] = nz; b->ng = ng;
  b->px = nx + 2 * ng; b->py = ny + 2 * ng; b->pz = nz + 2 * ng;
  b->P = b->px * b->py * b->pz;
  b->ex = nx + 2; b->ey = ny + 2; b->ez = nz + 2;
  b->E = b->ex * b->ey * b->ez;
}

/* padded index of cell (i, j, k), coordinates relative to the valid origin */
static long pid(const Box* b, int i, int j, int k) {
  return ((long)(k + b->ng) * b->py + (j + b->ng)) * b->px + (i + b->ng);
}
/* index in an array covering cells [-1, n] in every direction; a d-face with
 * index f (between cells f-1 and f) is stored at the slot of cell f */
static long eid(const Box* b, int i, int j, int k) {
  return ((long)(k + 1) * b->ey + (j + 1)) * b->ex + (i + 1);
}

/* ------------------------------------------------------------------ */
/* O5: two-shock Riemann solver (Colella & Glaz 1985, named in Sec. 3.2) */
/* ------------------------------------------------------------------ */
/* Rotated primitive states q = (rho, u_n, u_t1, u_t2, p).  The two-shock
 * approximation replaces both waves by shocks; the star pressure solves
 * u*_R(p) = u*_L(p) with the shock Lagrangian wave speeds W_K and is found by
 * Newton iteration (Z_K = 1/|du*_K/dp|). */
static void sample_star(double gam, const double* qL, const double* qR, double pstar,
                        double ustar, double rsL, double rsR, double WL, double WR,
                        double* qg);

/* Linearised approximate solver (the simpler alternative Sec. 3.2 compares
 * the two-shock solver against): the acoustic star state, with impedances
 * W_K = sqrt(gamma p_K rho_K),
 *   p* = (W_R p_L + W_L p_R + W_L W_R (u_L - u_R)) / (W_L + W_R),
 *   u* = (W_L u_L + W_R u_R + p_L - p_R) / (W_L + W_R),
 *   rho*_K = rho_K + (p* - p_K) / c_K^2,
 * sampled with the same wave structure as the two-shock solver.  With p*
 * at least the pressure floor, rho*_K >= (1 - 1/gamma) rho_K > 0, so the
 * star densities need no floor. */
static void linear_solve(const nyxo_params* prm, const double* qL, const double* qR,
                         double* qg, double* star) {
  const double gam = prm->gamma;
  const double g2 = 0.5 * (gam + 1.0);
  double rl = qL[0], ul = qL[1], pl = qL[4];
  double rr = qR[0], ur = qR[1], pr = qR[4];
  double CL = (gam * pl) * rl;
  double CR = (gam * pr) * rr;
  double W0L = sqrt(CL), W0R = sqrt(CR);
  double p = ((W0R * pl + W0L * pr) + (W0L * W0R) * (ul - ur)) / (W0L + W0R);
  p = dmax(p, prm->small_pres);
  double ustar = ((W0L * ul + W0R * ur) + (pl - pr)) / (W0L + W0R);
  double rsL = rl + (p - pl) / ((gam * pl) / rl);
  double rsR = rr + (p - pr) / ((gam * pr) / rr);
  double WL = sqrt(CL + (g2 * rl) * (p - pl));
  double WR = sqrt(CR + (g2 * rr) * (p - pr));
  sample_star(gam, qL, qR, p, ustar, rsL, rsR, WL, WR, qg);
  if (star) { star[0] = p; star[1] = ustar; star[2] = rsL; star[3] = rsR; }
}

static int riemann_solve(const nyxo_params* prm, const double* qL,
                         const double* qR, double* qg, double* star) {
  if (prm->riemann == NYXO_RIEMANN_LINEAR) {
    linear_solve(prm, qL, qR, qg, star);
    return 0;
  }
  const double gam = prm->gamma;
  const double g2 = 0.5 * (gam + 1.0);
  const double sp = prm->small_pres;
  double rl = qL[0], ul = qL[1], pl = qL[4];
  double rr = qR[0], ur = qR[1], pr = qR[4];
  double CL = (gam * pl) * rl;
  double CR = (gam * pr) * rr;
  double W0L = sqrt(CL), W0R = sqrt(CR);
  /* acoustic (linearised) initial guess */
  double p = ((W0R * pl + W0L * pr) + (W0L * W0R) * (ul - ur)) / (W0L + W0R);
  p = dmax(p, sp);
  int it = 0;
  double WL, WR, usL, usR, ZL, ZR;
  while (it < prm->riemann_maxiter) {
    NYXO_ITER(1);
    WL = sqrt(CL + (g2 * rl) * (p - pl));
    WR = sqrt(CR + (g2 * rr) * (p - pr));
    usL = ul - (p - pl) / WL;
    usR = ur + (p - pr) / WR;
    ZL = ((2.0 * WL) * WL) * WL / (WL * WL + CL);
    ZR = ((2.0 * WR) * WR) * WR / (WR * WR + CR);
    double pn = p - ((ZL * ZR) * (usR - usL)) / (ZL + ZR);
    pn = dmax(pn, sp);
    it++;
    int conv = fabs(pn - p) <= prm->riemann_tol * pn;
    p = pn;
    if (conv) break;
  }
  NYXO_ITER(0);
  /* final evaluation at the converged pressure */
  WL = sqrt(CL + (g2 * rl) * (p - pl));
  WR = sqrt(CR + (g2 * rr) * (p - pr));
  usL = ul - (p - pl) / WL;
  usR = ur + (p - pr) / WR;
  ZL = ((2.0 * WL) * WL) * WL / (WL * WL + CL);
  ZR = ((2.0 * WR) * WR) * WR / (WR * WR + CR);
  double ustar = (ZL * usL + ZR * usR) / (ZL + ZR);
  double pstar = p;
  /* star densities from the shock (Hugoniot) relation on both sides */
  double rsL = 1.0 / (1.0 / rl - (pstar - pl) / (WL * WL));
  double rsR = 1.0 / (1.0 / rr - (pstar - pr) / (WR * WR));
  sample_star(gam, qL, qR, pstar, ustar, rsL, rsR, WL, WR, qg);
  if (star) { star[0] = pstar; star[1] = ustar; star[2] = rsL; star[3] = rsR; }
  return it;
}

/* Wave structure of the star state and the sample at x/t = 0: a shock
 * (p* >= p_K) is one front at u_K -/+ W_K / rho_K; a rarefaction has its
 * head at u_K -/+ c_K and its tail at u* -/+ c*_K with linear interpolation
 * between them; at u* = 0 the mean of both sides. */
static void sample_star(double gam, const double* qL, const double* qR, double pstar,
                        double ustar, double rsL, double rsR, double WL, double WR,
                        double* qg) {
  double rl = qL[0], ul = qL[1], pl = qL[4];
  double rr = qR[0], ur = qR[1], pr = qR[4];
  double cL = sqrt((gam * pl) / rl), cR = sqrt((gam * pr) / rr);
  double csL = sqrt((gam * pstar) / rsL), csR = sqrt((gam * pstar) / rsR);
  double shdL, stlL, shdR, stlR;
  if (pstar >= pl) { shdL = ul - WL / rl; stlL = shdL; }
  else { shdL = ul - cL; stlL = ustar - csL; }
  if (pstar >= pr) { shdR = ur + WR / rr; stlR = shdR; }
  else { shdR = ur + cR; stlR = ustar + csR; }
  /* sample both sides at xi = 0 */
  double sL[3], sR[3];
  if (shdL >= 0.0) { sL[0] = rl; sL[1] = ul; sL[2] = pl; }
  else if (stlL <= 0.0) { sL[0] = rsL; sL[1] = ustar; sL[2] = pstar; }
  else {
    double f = (0.0 - shdL) / (stlL - shdL);
    sL[0] = rl + f * (rsL - rl);
    sL[1] = ul + f * (ustar - ul);
    sL[2] = pl + f * (pstar - pl);
  }
  if (shdR <= 0.0) { sR[0] = rr; sR[1] = ur; sR[2] = pr; }
  else if (stlR >= 0.0) { sR[0] = rsR; sR[1] = ustar; sR[2] = pstar; }
  else {
    double f = (0.0 - shdR) / (stlR - shdR);
    sR[0] = rr + f * (rsR - rr);
    sR[1] = ur + f * (ustar - ur);
    sR[2] = pr + f * (pstar - pr);
  }
  if (ustar > 0.0) {
    qg[0] = sL[0]; qg[1] = sL[1]; qg[4] = sL[2]; qg[2] = qL[2]; qg[3] = qL[3];
  } else if (ustar < 0.0) {
    qg[0] = sR[0]; qg[1] = sR[1]; qg[4] = sR[2]; qg[2] = qR[2]; qg[3] = qR[3];
  } else {
    qg[0] = 0.5 * (sL[0] + sR[0]);
    qg[1] = 0.5 * (sL[1] + sR[1]);
    qg[4] = 0.5 * (sL[2] + sR[2]);
    qg[2] = 0.5 * (qL[2] + qR[2]);
    qg[3] = 0.5 * (qL[3] + qR[3]);
  }
}

void nyxo_riemann(const nyxo_params* prm, const double* qL, const double* qR,
                  double* qg, double* star, int* iters) {
  int it = riemann_solve(prm, qL, qR, qg, star);
  if (iters) *iters = it;
}

/* O6 / O9: fluxes of a lab-frame face in direction d from the rotated Godunov
 * state qg.  out[0..7] = (f_rho, f_mx, f_my, f_mz, f_E, f_e, p_g, u_g). */
static void godunov_flux(double gam, int d, const double* qg, double* out) {
  const double gm1 = gam - 1.0;
  double r = qg[0], u = qg[1], v = qg[2], w = qg[3], p = qg[4];
  int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
  double ru = r * u;
  out[0] = ru;
  out[1 + d] = ru * u + p;
  out[1 + t1] = ru * v;
  out[1 + t2] = ru * w;
  double rE = p / gm1 + (0.5 * r) * ((u * u + v * v) + w * w);
  out[4] = u * (rE + p);
  out[5] = (u * p) / gm1;
  out[6] = p;
  out[7] = u;
}

/* solve at a d-face: lab-frame states L (right edge of left cell) and R */
static void face_solve(const nyxo_params* prm, int d, const double* L,
                       const double* R, double* flux, nyxo_stats* st) {
  int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
  double qL[5] = {L[0], L[1 + d], L[1 + t1], L[1 + t2], L[4]};
  double qR[5] = {R[0], R[1 + d], R[1 + t1], R[1 + t2], R[4]};
  double qg[5];
  int it = riemann_solve(prm, qL, qR, qg, NULL);
  st->riemann_calls += 1;
  st->riemann_iters += it;
  godunov_flux(prm->gamma, d, qg, flux);
}

/* ------------------------------------------------------------------ */
/* O3: PPM reconstruction (Colella & Woodward 1984; unsplit PPM, Sec. 3.2) */
/* ------------------------------------------------------------------ */
/* van Leer-limited centred slope of cell j from q[j-1], q[j], q[j+1] */
static double limited_slope(double qm1, double q0, double qp1) {
  double dc = 0.5 * (qp1 - qm1);
  double dr = qp1 - q0;
  double dl = q0 - qm1;
  if (dr * dl > 0.0) {
    double m = fabs(dc);
    m = dmin(m, 2.0 * fabs(dl));
    m = dmin(m, 2.0 * fabs(dr));
    return dc > 0.0 ? m : -m;
  }
  return 0.0;
}

double nyxo_ppm_interface(const double* q4) {
  double s0 = limited_slope(q4[0], q4[1], q4[2]);
  double s1 = limited_slope(q4[1], q4[2], q4[3]);
  return (q4[1] + 0.5 * (q4[2] - q4[1])) - (s1 - s0) / 6.0;
}

/* edge values of cell j from q[j-2..j+2] (q5 points at q[j-2]) and chi */
static void ppm_cell(const double* q5, double chi, double* qm_out,
                     double* qp_out) {
  double qj = q5[2];
  double qp = nyxo_ppm_interface(q5 + 1);
  double qm = nyxo_ppm_interface(q5);
  /* flatten toward the cell average */
  qp = chi * qp + (1.0 - chi) * qj;
  qm = chi * qm + (1.0 - chi) * qj;
  /* monotonise (CW84) */
  if ((qp - qj) * (qj - qm) <= 0.0) {
    qp = qj;
    qm = qj;
  } else {
    double dq = qp - qm;
    double t = dq * (qj - 0.5 * (qm + qp));
    double s = dq * dq / 6.0;
    if (t > s) {
      qm = 3.0 * qj - 2.0 * qp;
    } else if (-s > t) {
      qp = 3.0 * qj - 2.0 * qm;
    }
  }
  *qm_out = qm;
  *qp_out = qp;
}

/* PLM (unsplit piecewise linear, Sec. 3.2): the limited centred slope of
 * cell j, flattened by chi, gives the edge values q_j -/+ (chi s)/2; the
 * tracing below then averages this linear profile over each wave's domain
 * of dependence (the parabola's q6 term vanishes). */
static void plm_cell(const double* q5, double chi, double* qm_out, double* qp_out) {
  double qj = q5[2];
  double ds = chi * limited_slope(q5[1], q5[2], q5[3]);
  *qm_out = qj - 0.5 * ds;
  *qp_out = qj + 0.5 * ds;
}

void nyxo_plm_line(int m, const double* q, const double* chi, double* qm, double* qp) {
  for (int j = 2; j <= m - 3; ++j) plm_cell(q + j - 2, chi[j], &qm[j], &qp[j]);
}

void nyxo_ppm_line(int m, const double* q, const double* chi, double* qm,
                   double* qp) {
  for (int j = 2; j <= m - 3; ++j) ppm_cell(q + j - 2, chi[j], &qm[j], &qp[j]);
}

/* ------------------------------------------------------------------ */
/* O2: flattening (CW84 shock detector)                               */
/* ------------------------------------------------------------------ */
/* f~ of cell j from p[j-2..j+2] (p5 points at p[j-2]) and u[j-1], u[j+1] */
static double flat_tilde(double small_p, const double* p5, double um1,
                         double up1) {
  double dp1 = p5[3] - p5[1];
  double dp2 = p5[4] - p5[0];
  double z = fabs(dp1) / dmax(fabs(dp2), small_p);
  int w = (fabs(dp1) > FLAT_EPS * dmin(p5[3], p5[1])) && ((up1 - um1) < 0.0);
  return w ? dmax(0.0, dmin(1.0, FLAT_OMEGA2 * (z - FLAT_OMEGA1))) : 0.0;
}

/* chi_d of cell j from p[j-3..j+3] (p7 at p[j-3]) and u[j-2..j+2] (u5 at u[j-2]) */
static double flat_chi(double small_p, const double* p7, const double* u5) {
  double fm = flat_tilde(small_p, p7 + 0, u5[0], u5[2]);
  double f0 = flat_tilde(small_p, p7 + 1, u5[1], u5[3]);
  double fp = flat_tilde(small_p, p7 + 2, u5[2], u5[4]);
  double dp1 = p7[4] - p7[2];
  double f = f0;
  if (dp1 > 0.0) f = dmax(f0, fm);       /* lower pressure on the left */
  else if (dp1 < 0.0) f = dmax(f0, fp);  /* lower pressure on the right */
  return 1.0 - f;
}

void nyxo_flatten_line(const nyxo_params* prm, int m, const double* p,
                       const double* u, double* chi) {
  for (int j = 3; j <= m - 4; ++j)
    chi[j] = flat_chi(prm->small_pres, p + j - 3, u + j - 2);
}

/* ------------------------------------------------------------------ */
/* O4: characteristic tracing with the reference state of Sec. 3.2    */
/* ------------------------------------------------------------------ */
static double trace_hi(double qp, double dq, double q6, double sig) {
  return qp - 0.5 * sig * (dq - (1.0 - (2.0 / 3.0) * sig) * q6);
}
static double trace_lo(double qm, double dq, double q6, double sig) {
  return qm + 0.5 * sig * (dq + (1.0 - (2.0 / 3.0) * sig) * q6);
}

int nyxo_trace_cell(const nyxo_params* prm, int d, const double* qc, double cc,
                    const double* qmv, const double* qpv, const double* g,
                    double kh, double hdt_a, double hda_a, double pexp,
                    double* lo, double* hi) {
  const int nv = 1 + d;
  const int t1 = 1 + (d + 1) % 3, t2 = 1 + (d + 2) % 3;
  const double rho = qc[0], u = qc[nv], c = cc;
  const double csq = c * c;
  double lam[3] = {u - c, u, u + c};
  double sig[3];
  for (int w = 0; w < 3; ++w) sig[w] = fabs(lam[w]) * kh;
  double dq[5], q6[5];
  for (int v = 0; v < 5; ++v) {
    dq[v] = qpv[v] - qmv[v];
    q6[v] = 6.0 * qc[v] - 3.0 * (qmv[v] + qpv[v]);
  }
  const int vr = 0, vu = nv, vp = 4;

  /* ---- right face (j+1/2): waves with lam > 0 reach it ---- */
  {
    double I[3][5];
    for (int w = 0; w < 3; ++w)
      for (int v = 0; v < 5; ++v) I[w][v] = trace_hi(qpv[v], dq[v], q6[v], sig[w]);
    double ref[5];
    for (int v = 0; v < 5; ++v) ref[v] = (lam[2] > 0.0) ? I[2][v] : qpv[v];
    double D[3][5];
    for (int w = 0; w < 3; ++w)
      for (int v = 0; v < 5; ++v) D[w][v] = (lam[w] > 0.0) ? ref[v] - I[w][v] : 0.0;
    double am = 0.5 * (D[0][vp] / csq - (rho * D[0][vu]) / c);
    double ap = 0.5 * (D[2][vp] / csq + (rho * D[2][vu]) / c);
    double a0 = D[1][vr] - D[1][vp] / csq;
    hi[0] = ref[vr] - ((am + a0) + ap);
    hi[nv] = ref[vu] - (c / rho) * (ap - am);
    hi[4] = ref[vp] - csq * (am + ap);
    hi[t1] = (lam[1] > 0.0) ? I[1][t1] : qpv[t1];
    hi[t2] = (lam[1] > 0.0) ? I[1][t2] : qpv[t2];
  }
  /* ---- left face (j-1/2): waves with lam < 0 reach it ---- */
  {
    double I[3][5];
    for (int w = 0; w < 3; ++w)
      for (int v = 0; v < 5; ++v) I[w][v] = trace_lo(qmv[v], dq[v], q6[v], sig[w]);
    double ref[5];
    for (int v = 0; v < 5; ++v) ref[v] = (lam[0] < 0.0) ? I[0][v] : qmv[v];
    double D[3][5];
    for (int w = 0; w < 3; ++w)
      for (int v = 0; v < 5; ++v) D[w][v] = (lam[w] < 0.0) ? ref[v] - I[w][v] : 0.0;
    double am = 0.5 * (D[0][vp] / csq - (rho * D[0][vu]) / c);
    double ap = 0.5 * (D[2][vp] / csq + (rho * D[2][vu]) / c);
    double a0 = D[1][vr] - D[1][vp] / csq;
    lo[0] = ref[vr] - ((am + a0) + ap);
    lo[nv] = ref[vu] - (c / rho) * (ap - am);
    lo[4] = ref[vp] - csq * (am + ap);
    lo[t1] = (lam[1] < 0.0) ? I[1][t1] : qmv[t1];
    lo[t2] = (lam[1] < 0.0) ? I[1][t2] : qmv[t2];
  }
  /* ---- half-step gravity and expansion sources, then floors ---- */
  int floors = 0;
  double* sides[2] = {lo, hi};
  for (int s = 0; s < 2; ++s) {
    double* e = sides[s];
    for (int dd = 0; dd < 3; ++dd)
      e[1 + dd] = e[1 + dd] + (hdt_a * g[dd] - hda_a * qc[1 + dd]);
    e[4] = e[4] - pexp * qc[4];
    if (e[0] < prm->small_dens) { e[0] = prm->small_dens; floors++; }
    if (e[4] < prm->small_pres) { e[4] = prm->small_pres; floors++; }
  }
  return floors;
}

/* ------------------------------------------------------------------ */
/* O7: transverse (corner-coupling) correction of a lab-frame edge state */
/* ------------------------------------------------------------------ */
/* nt transverse flux pairs: fm[k] = flux at the low t-face, fp[k] = at the
 * high t-face of the cell, each (f_rho, f_m x3, f_E, f_e, p_g, u_g).
 * Returns 1 if the correction was rejected (edge state kept). */
static int trans_correct(const nyxo_params* prm, const double* q, int nt,
                         const double* const* fm, const double* const* fp,
                         double kap, double* out) {
  const double gm1 = prm->gamma - 1.0;
  double rho = q[0], ux = q[1], uy = q[2], uz = q[3], p = q[4];
  double U[5];
  U[0] = rho;
  U[1] = rho * ux;
  U[2] = rho * uy;
  U[3] = rho * uz;
  U[4] = p / gm1 + (0.5 * rho) * ((ux * ux + uy * uy) + uz * uz);
  double Ue = p / gm1;
  double Dc[5], De;
  for (int c = 0; c < 5; ++c) {
    Dc[c] = fp[0][c] - fm[0][c];
    if (nt == 2) Dc[c] = Dc[c] + (fp[1][c] - fm[1][c]);
  }
  De = (fp[0][5] - fm[0][5]) + (0.5 * (fp[0][6] + fm[0][6])) * (fp[0][7] - fm[0][7]);
  if (nt == 2)
    De = De + ((fp[1][5] - fm[1][5]) +
               (0.5 * (fp[1][6] + fm[1][6])) * (fp[1][7] - fm[1][7]));
  double Un[5];
  for (int c = 0; c < 5; ++c) Un[c] = U[c] - kap * Dc[c];
  double Uen = Ue - kap * De;
  double ke = (0.5 * ((Un[1] * Un[1] + Un[2] * Un[2]) + Un[3] * Un[3])) / Un[0];
  double pn;
  if (Un[4] - ke > prm->eta * Un[4]) pn = gm1 * (Un[4] - ke);
  else pn = gm1 * Uen;
  double r[5];
  r[0] = Un[0];
  r[1] = Un[1] / Un[0];
  r[2] = Un[2] / Un[0];
  r[3] = Un[3] / Un[0];
  r[4] = pn;
  int ok = (r[0] > 0.0) && (r[4] > 0.0);
  for (int c = 0; c < 5; ++c) ok = ok && isfinite(r[c]);
  if (!ok) {
    for (int c = 0; c < 5; ++c) out[c] = q[c];
    return 1;
  }
  for (int c = 0; c < 5; ++c) out[c] = r[c];
  return 0;
}

/* ------------------------------------------------------------------ */
/* O13: hydro CFL time step (Sec. 3.5)                                 */
/* ------------------------------------------------------------------ */
int nyxo_estimate_dt(const nyxo_params* prm, int nx, int ny, int nz, int ng,
                     const double* state, double a, double dx, double cfl,
                     double* dt_out) {
  if (!prm || !state || !dt_out || nx < 1 || ny < 1 || nz < 1 || ng < 0)
    return -1;
  Box b;
  box_init(&b, nx, ny, nz, ng);
  NYXO_STAGE(8);
  const double gam = prm->gamma, gm1 = gam - 1.0;
  double smax = 0.0;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        long id = pid(&b, i, j, k);
        double rho = dmax(state[id], prm->small_dens);
        double re = state[5 * b.P + id] / (a * a);
        double p = dmax(gm1 * re, prm->small_pres);
        double c = sqrt((gam * p) / rho);
        for (int d = 0; d < 3; ++d) {
          double u = state[(1 + d) * b.P + id] / (a * rho);
          double s = fabs(u) + c;
          smax = dmax(smax, s);
        }
      }
  *dt_out = ((cfl * a) * dx) / smax;
  return 0;
}

/* ------------------------------------------------------------------ */
/* The step                                                           */
/* ------------------------------------------------------------------ */
#define NF 8 /* values stored per face */

/* O1 and O2 of the step: primitives (rho, u, p, c) on every padded cell of
 * box b from the state at scale factor a_old, and the flattening coefficient
 * chi (the minimum of the three directional coefficients) on the cells of
 * [-1, n]^3.  prim: 6 P values, chi: E values (E-array layout). */
static void prim_and_flattening(const nyxo_params* prm, const Box* bp, const double* Uin,
                                double a_old, double* prim, double* chi, nyxo_stats* st) {
  const Box b = *bp;
  const long P = b.P;
  const int* n = b.n;
  const int ng = b.ng;
  const double gam = prm->gamma, gm1 = gam - 1.0;
#define PRIM(v, i, j, k) prim[(v) * P + pid(&b, i, j, k)]
  /* ---- O1: primitives on every padded cell ---- */
  NYXO_STAGE(1);
  for (int kk = -ng; kk < n[2] + ng; ++kk)
    for (int j = -ng; j < n[1] + ng; ++j)
      for (int i = -ng; i < n[0] + ng; ++i) {
        long id = pid(&b, i, j, kk);
        double rho = Uin[id];
        if (rho < prm->small_dens) { rho = prm->small_dens; st->floor_hits++; }
        double u[3];
        for (int d = 0; d < 3; ++d) u[d] = Uin[(1 + d) * P + id] / (a_old * rho);
        double re = Uin[5 * P + id] / (a_old * a_old);
        double p = gm1 * re;
        if (p < prm->small_pres) { p = prm->small_pres; st->floor_hits++; }
        double c = sqrt((gam * p) / rho);
        prim[id] = rho;
        for (int d = 0; d < 3; ++d) prim[(1 + d) * P + id] = u[d];
        prim[4 * P + id] = p;
        prim[5 * P + id] = c;
      }

  /* ---- O2: flattening, chi = min over directions, cells [-1, n]^3 ---- */
  NYXO_STAGE(2);
  for (int kk = -1; kk <= n[2]; ++kk)
    for (int j = -1; j <= n[1]; ++j)
      for (int i = -1; i <= n[0]; ++i) {
        double cmin = 1.0;
        for (int d = 0; d < 3; ++d) {
          double p7[7], u5[5];
          for (int s = -3; s <= 3; ++s) {
            int c3[3] = {i, j, kk};
            c3[d] += s;
            p7[s + 3] = PRIM(4, c3[0], c3[1], c3[2]);
            if (s >= -2 && s <= 2) u5[s + 2] = PRIM(1 + d, c3[0], c3[1], c3[2]);
          }
          double cd = flat_chi(prm->small_pres, p7, u5);
          if (d == 0) cmin = cd;
          else cmin = dmin(cmin, cd);
        }
        chi[eid(&b, i, j, kk)] = cmin;
      }

#undef PRIM
}

/* chi of the step (O2) on the cells of [-1, n]^3 of a box, for pins of the
 * three-direction combination; chi_out: (nz + 2) (ny + 2) (nx + 2) values,
 * x fastest.  Returns 0, or -1 on bad arguments / allocation failure. */
int nyxo_flattening(const nyxo_params* prm, int nx, int ny, int nz, int ng,
                    const double* state, double a, double* chi_out) {
  if (!prm || !state || !chi_out || nx < 1 || ny < 1 || nz < 1 || ng < 4 || !(a > 0.0))
    return -1;
  Box b;
  box_init(&b, nx, ny, nz, ng);
  nyxo_stats st;
  memset(&st, 0, sizeof st);
  double* prim = (double*)malloc(sizeof(double) * 6 * b.P);
  if (!prim) return -1;
  prim_and_flattening(prm, &b, state, a, prim, chi_out, &st);
  free(prim);
  return 0;
}

int nyxo_hydro_step(const nyxo_params* prm, int nx, int ny, int nz, int ng,
                    const double* Uin, const double* grav, double dt,
                    double dx, double a_old, double a_new, double* Uout,
                    nyxo_stats* stats) {
  return nyxo_hydro_step_faces(prm, nx, ny, nz, ng, Uin, grav, dt, dx, a_old, a_new, Uout,
                               stats, NULL);
}

int nyxo_hydro_step_faces(const nyxo_params* prm, int nx, int ny, int nz, int ng,
                          const double* Uin, const double* grav, double dt,
                          double dx, double a_old, double a_new, double* Uout,
                          nyxo_stats* stats, double* face_flux) {
  if (!prm || !Uin || !grav || !Uout || nx < 1 || ny < 1 || nz < 1 || ng < 4 ||
      !(dt > 0.0) || !(a_old > 0.0) || !(a_new > 0.0) || !(dx > 0.0))
    return -1;
  if ((prm->recon != NYXO_RECON_PPM && prm->recon != NYXO_RECON_PLM) ||
      (prm->riemann != NYXO_RIEMANN_TWOSHOCK && prm->riemann != NYXO_RIEMANN_LINEAR) ||
      (prm->grav_form != 1 && prm->grav_form != 2))
    return -1;
  nyxo_stats stl;
  memset(&stl, 0, sizeof stl);
  nyxo_stats* st = &stl;
  Box b;
  box_init(&b, nx, ny, nz, ng);
  const long P = b.P, E = b.E;
  const int* n = b.n;
  const double gam = prm->gamma, gm1 = gam - 1.0;

  /* scale factor inside the step: linear in time, centred value a_h */
  const double a_h = 0.5 * (a_old + a_new);
  const double da = a_new - a_old;
  const double kh = dt / (a_h * dx);
  const double hdt_a = (0.5 * dt) / a_h;
  const double hda_a = (0.5 * da) / a_h;
  const double pexp = (1.5 * gm1) * (da / a_h);
  const double kap1 = kh / 3.0;
  const double kap2 = kh / 2.0;
  const double k = dt / dx;
  /* expansion source of both energy equations (Sec. 2.2): a adot (2 - 3(gamma-1))
   * rho e = (adot / a) cgam U_e in the stored variables; with adot dt = da the
   * step's integral is cgam (da / a) U_e evaluated at a_old (predictor) and at
   * a_new (corrector) */
  const double cgam = 2.0 - 3.0 * gm1;
  const double xo = cgam * (da / a_old);
  const double xn = cgam * (da / a_new);

  double* prim = (double*)malloc(sizeof(double) * 6 * P);
  double* chi = (double*)malloc(sizeof(double) * E);
  double* edge = (double*)malloc(sizeof(double) * 3 * 2 * 5 * E);
  double* F0 = (double*)malloc(sizeof(double) * 3 * NF * E);
  double* F1 = (double*)malloc(sizeof(double) * 9 * NF * E);
  double* F2 = (double*)malloc(sizeof(double) * 3 * NF * E);
  if (!prim || !chi || !edge || !F0 || !F1 || !F2) {
    free(prim); free(chi); free(edge); free(F0); free(F1); free(F2);
    return -1;
  }
#define PRIM(v, i, j, k) prim[(v) * P + pid(&b, i, j, k)]
#define EDGE(d, s, v, id) edge[(((d) * 2 + (s)) * 5 + (v)) * E + (id)]
#define FL0(d, v, id) F0[((d) * NF + (v)) * E + (id)]
#define FL1(d, t, v, id) F1[(((d) * 3 + (t)) * NF + (v)) * E + (id)]
#define FL2(d, v, id) F2[((d) * NF + (v)) * E + (id)]

  prim_and_flattening(prm, &b, Uin, a_old, prim, chi, st);

  /* ---- O3 + O4: PPM and tracing, all directions, cells [-1, n]^3 ---- */
  NYXO_STAGE(3);
  for (int kk = -1; kk <= n[2]; ++kk)
    for (int j = -1; j <= n[1]; ++j)
      for (int i = -1; i <= n[0]; ++i) {
        long e = eid(&b, i, j, kk);
        double qc[5];
        qc[0] = PRIM(0, i, j, kk);
        for (int v = 1; v < 5; ++v) qc[v] = PRIM(v, i, j, kk);
        double cc = PRIM(5, i, j, kk);
        long id = pid(&b, i, j, kk);
        double g[3] = {grav[id], grav[P + id], grav[2 * P + id]};
        for (int d = 0; d < 3; ++d) {
          double qmv[5], qpv[5];
          for (int v = 0; v < 5; ++v) {
            double q5[5];
            for (int s = -2; s <= 2; ++s) {
              int c3[3] = {i, j, kk};
              c3[d] += s;
              q5[s + 2] = PRIM(v, c3[0], c3[1], c3[2]);
            }
            if (prm->recon == NYXO_RECON_PLM) plm_cell(q5, chi[e], &qmv[v], &qpv[v]);
            else ppm_cell(q5, chi[e], &qmv[v], &qpv[v]);
          }
          double lo[5], hi[5];
          st->floor_hits += nyxo_trace_cell(prm, d, qc, cc, qmv, qpv, g, kh,
                                            hdt_a, hda_a, pexp, lo, hi);
          for (int v = 0; v < 5; ++v) {
            EDGE(d, 0, v, e) = lo[v];
            EDGE(d, 1, v, e) = hi[v];
          }
        }
      }

  /* ---- O8 stage 0: Riemann on d-faces between cells of [-1, n] ---- */
  NYXO_STAGE(4);
  for (int d = 0; d < 3; ++d) {
    int lo3[3] = {-1, -1, -1}, hi3[3] = {n[0], n[1], n[2]};
    lo3[d] = 0; /* face index f in [0, n_d] */
    for (int kk = lo3[2]; kk <= hi3[2]; ++kk)
      for (int j = lo3[1]; j <= hi3[1]; ++j)
        for (int i = lo3[0]; i <= hi3[0]; ++i) {
          int c3[3] = {i, j, kk};
          long eR = eid(&b, i, j, kk);
          c3[d] -= 1;
          long eL = eid(&b, c3[0], c3[1], c3[2]);
          double L[5], R[5], f[NF];
          for (int v = 0; v < 5; ++v) {
            L[v] = EDGE(d, 1, v, eL);
            R[v] = EDGE(d, 0, v, eR);
          }
          face_solve(prm, d, L, R, f, st);
          for (int v = 0; v < NF; ++v) FL0(d, v, eR) = f[v];
        }
  }

  /* ---- O8 stage 1: d-states corrected by stage-0 t-fluxes ---- */
  NYXO_STAGE(5);
  for (int d = 0; d < 3; ++d)
    for (int t = 0; t < 3; ++t) {
      if (t == d) continue;
      int lo3[3] = {-1, -1, -1}, hi3[3] = {n[0], n[1], n[2]};
      lo3[d] = 0;
      lo3[t] = 0;
      hi3[t] = n[t] - 1;
      for (int kk = lo3[2]; kk <= hi3[2]; ++kk)
        for (int j = lo3[1]; j <= hi3[1]; ++j)
          for (int i = lo3[0]; i <= hi3[0]; ++i) {
            int cR[3] = {i, j, kk}, cL[3] = {i, j, kk};
            cL[d] -= 1;
            double q[2][5], qc[2][5];
            int cells[2][3];
            memcpy(cells[0], cL, sizeof cL);
            memcpy(cells[1], cR, sizeof cR);
            for (int s = 0; s < 2; ++s) {
              int* c3 = cells[s];
              long ec = eid(&b, c3[0], c3[1], c3[2]);
              int cu[3] = {c3[0], c3[1], c3[2]};
              cu[t] += 1;
              long eu = eid(&b, cu[0], cu[1], cu[2]);
              double fm[NF], fp[NF];
              for (int v = 0; v < NF; ++v) {
                fm[v] = FL0(t, v, ec);
                fp[v] = FL0(t, v, eu);
              }
              /* the left cell contributes its right-face state */
              for (int v = 0; v < 5; ++v) q[s][v] = EDGE(d, s == 0 ? 1 : 0, v, ec);
              const double* fmp[1] = {fm};
              const double* fpp[1] = {fp};
              st->trans_reverts += trans_correct(prm, q[s], 1, fmp, fpp, kap1, qc[s]);
            }
            double f[NF];
            face_solve(prm, d, qc[0], qc[1], f, st);
            long eR = eid(&b, cR[0], cR[1], cR[2]);
            for (int v = 0; v < NF; ++v) FL1(d, t, v, eR) = f[v];
          }
    }

  /* ---- O8 stage 2: final d-states and fluxes on valid faces ---- */
  NYXO_STAGE(6);
  for (int d = 0; d < 3; ++d) {
    int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
    int lo3[3] = {0, 0, 0}, hi3[3] = {n[0] - 1, n[1] - 1, n[2] - 1};
    hi3[d] = n[d];
    for (int kk = lo3[2]; kk <= hi3[2]; ++kk)
      for (int j = lo3[1]; j <= hi3[1]; ++j)
        for (int i = lo3[0]; i <= hi3[0]; ++i) {
          int cR[3] = {i, j, kk}, cL[3] = {i, j, kk};
          cL[d] -= 1;
          int cells[2][3];
          memcpy(cells[0], cL, sizeof cL);
          memcpy(cells[1], cR, sizeof cR);
          double qc[2][5];
          for (int s = 0; s < 2; ++s) {
            int* c3 = cells[s];
            long ec = eid(&b, c3[0], c3[1], c3[2]);
            int u1[3] = {c3[0], c3[1], c3[2]}, u2[3] = {c3[0], c3[1], c3[2]};
            u1[t1] += 1;
            u2[t2] += 1;
            long e1 = eid(&b, u1[0], u1[1], u1[2]);
            long e2 = eid(&b, u2[0], u2[1], u2[2]);
            double fm1[NF], fp1[NF], fm2[NF], fp2[NF];
            for (int v = 0; v < NF; ++v) {
              fm1[v] = FL1(t1, t2, v, ec);  /* t1-flux corrected by t2 */
              fp1[v] = FL1(t1, t2, v, e1);
              fm2[v] = FL1(t2, t1, v, ec);  /* t2-flux corrected by t1 */
              fp2[v] = FL1(t2, t1, v, e2);
            }
            double q[5];
            for (int v = 0; v < 5; ++v) q[v] = EDGE(d, s == 0 ? 1 : 0, v, ec);
            const double* fmp[2] = {fm1, fm2};
            const double* fpp[2] = {fp1, fp2};
            st->trans_reverts += trans_correct(prm, q, 2, fmp, fpp, kap2, qc[s]);
          }
          double f[NF];
          face_solve(prm, d, qc[0], qc[1], f, st);
          /* O9: comoving flux factors of Sec. 3.2 */
          f[0] = f[0] / a_h;
          f[4] = a_h * f[4];
          f[5] = a_h * f[5];
          long eR = eid(&b, cR[0], cR[1], cR[2]);
          for (int v = 0; v < NF; ++v) FL2(d, v, eR) = f[v];
        }
  }

  /* the final comoving fluxes of every face, for flux registers */
  if (face_flux) {
    double* o = face_flux;
    for (int d = 0; d < 3; ++d) {
      const int fe[3] = {n[0] + (d == 0), n[1] + (d == 1), n[2] + (d == 2)};
      for (int c = 0; c < 6; ++c)
        for (int kk = 0; kk < fe[2]; ++kk)
          for (int j = 0; j < fe[1]; ++j)
            for (int i = 0; i < fe[0]; ++i) *o++ = FL2(d, c, eid(&b, i, j, kk));
    }
  }

  /* ---- O10-O12: update, gravity corrector, dual-energy sync ---- */
  NYXO_STAGE(7);
  for (int kk = 0; kk < n[2]; ++kk)
    for (int j = 0; j < n[1]; ++j)
      for (int i = 0; i < n[0]; ++i) {
        long id = pid(&b, i, j, kk);
        long e = eid(&b, i, j, kk);
        double D[6] = {0, 0, 0, 0, 0, 0};
        double Pi = 0.0;
        for (int d = 0; d < 3; ++d) {
          int cu[3] = {i, j, kk};
          cu[d] += 1;
          long eu = eid(&b, cu[0], cu[1], cu[2]);
          for (int c = 0; c < 6; ++c) {
            double dF = FL2(d, c, eu) - FL2(d, c, e);
            D[c] = (d == 0) ? dF : D[c] + dF;
          }
          double pid_ = (0.5 * (FL2(d, 6, eu) + FL2(d, 6, e))) * (FL2(d, 7, eu) - FL2(d, 7, e));
          Pi = (d == 0) ? pid_ : Pi + pid_;
        }
        double U0 = Uin[id];
        double Um[3] = {Uin[P + id], Uin[2 * P + id], Uin[3 * P + id]};
        double UE = Uin[4 * P + id], Ue = Uin[5 * P + id];
        double g[3] = {grav[id], grav[P + id], grav[2 * P + id]};
        /* predictor (Step 2) */
        double s0 = U0 - k * D[0];
        double mh[3], sm[3];
        for (int d = 0; d < 3; ++d) {
          mh[d] = Um[d] - k * D[1 + d];
          sm[d] = mh[d] + (dt * U0) * g[d];
        }
        double sE;
        if (prm->grav_form == 2) {
          /* form 2: E changes by the change of the kinetic energy that the
           * gravity momentum update causes (at the new density) */
          sE = (UE - k * D[4]) + (kinetic(sm, s0) - kinetic(mh, s0));
        } else {
          sE = (UE - k * D[4]) + dt * ((Um[0] * g[0] + Um[1] * g[1]) + Um[2] * g[2]);
        }
        double se = (Ue - k * D[5]) - (k * a_h) * Pi;
        if (cgam != 0.0) {
          sE = sE + xo * Ue;
          se = se + xo * Ue;
        }
        /* corrector (Step 6) with the same g */
        double nm[3];
        for (int d = 0; d < 3; ++d) nm[d] = sm[d] + ((0.5 * dt) * (s0 - U0)) * g[d];
        double nE;
        if (prm->grav_form == 2) {
          nE = sE + (kinetic(nm, s0) - kinetic(sm, s0));
        } else {
          nE = sE + (0.5 * dt) * (((sm[0] - Um[0]) * g[0] + (sm[1] - Um[1]) * g[1]) +
                                  (sm[2] - Um[2]) * g[2]);
        }
        double ne = se;
        if (cgam != 0.0) {
          /* time-centre the expansion source: + (S* - S^n) dt / 2 */
          const double cx = 0.5 * (xn * se - xo * Ue);
          nE = nE + cx;
          ne = ne + cx;
        }
        /* dual-energy sync (Step 6) */
        double ke = (0.5 * ((nm[0] * nm[0] + nm[1] * nm[1]) + nm[2] * nm[2])) / s0;
        if (nE - ke > prm->eta * nE) {
          ne = nE - ke;
        } else {
          nE = ne + ke;
          st->sync_E_from_e++;
        }
        Uout[id] = s0;
        Uout[P + id] = nm[0];
        Uout[2 * P + id] = nm[1];
        Uout[3 * P + id] = nm[2];
        Uout[4 * P + id] = nE;
        Uout[5 * P + id] = ne;
        int fin = isfinite(s0) && isfinite(nm[0]) && isfinite(nm[1]) &&
                  isfinite(nm[2]) && isfinite(nE) && isfinite(ne);
        if (!fin) st->nonfinite++;
        if (s0 <= 0.0) st->neg_dens++;
        if (ne <= 0.0) st->neg_eint++;
      }
#undef PRIM
#undef EDGE
#undef FL0
#undef FL1
#undef FL2
  free(prim); free(chi); free(edge); free(F0); free(F1); free(F2);
  if (stats) {
    stats->nonfinite += st->nonfinite;
    stats->neg_dens += st->neg_dens;
    stats->neg_eint += st->neg_eint;
    stats->floor_hits += st->floor_hits;
    stats->trans_reverts += st->trans_reverts;
    stats->sync_E_from_e += st->sync_E_from_e;
    stats->riemann_iters += st->riemann_iters;
    stats->riemann_calls += st->riemann_calls;
  }
  return 0;
}

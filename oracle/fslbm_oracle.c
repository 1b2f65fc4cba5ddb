/*
 * Free-surface lattice Boltzmann foaming step: plain FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE. This file states, as slowly and plainly as possible, what one
 * time step of the method computes, so that the GPU library can be checked against
 * it. Only the tests, the smoke check and the benchmark's CPU-baseline leg may load
 * it. It shares no source with the GPU library and includes none of its headers.
 *
 * Paper: Ataei et al., "LBfoam: an open-source software package for the simulation
 * of foaming using the lattice Boltzmann method" (arXiv 1908.04262).
 *
 * Every pass below runs over the whole grid in ascending cell order, with no blocking
 * or fusion. Build with -O2 -ffp-contract=off -fno-fast-math so that every + - * / sqrt
 * is one correctly rounded IEEE binary64 operation.
 *
 * Step order (where the paper leaves a choice open, the comment of the pass states
 * the reading taken):
 *   S1  stream f (Eq. streaming), bounce-back at walls (Sec. 2), gas-side
 *       reconstruction at interface cells (Eq. reconstruct) with the gas density
 *       of Eq. rhob / rhobplusdisjoining;
 *   S2  interface mass exchange (Eq. massexchange with the weights Theta);
 *   S3  stream g (Eq. diffusion) with the Henry's-law rebuild (Eqs. henryslaw,
 *       reconstructdiffusion) and the gas ledger that feeds the bubbles (or, with
 *       flux_mode 1, S3' the gas flux of Eq. gascurrent as printed);
 *   S4  moments (Sec. 2), BGK collision (Eqs. collision, equilibrium) with tau from
 *       Eq. tau or the power-law limit of Eq. carreauTau, and the external force term of
 *       Eq. collision in the scheme of Guo, Zheng and Shi (2002); ADE collision
 *       (Eq. diffusion);
 *   S5-S7 cell-type conversion and excess-mass redistribution (Sec. 2.1, last paragraph);
 *   S8  bubble labelling by flood fill with merge/split bookkeeping (Sec. 3.5);
 *   S9  ideal-gas bubble pressure (Eq. idealgas);
 *   S10 interface curvature (normal + paraboloid fit, PLIC points);
 *   S11 disjoining pressure by ray traversal (Sec. 3.3, Appendix A, Algorithm 1).
 *
 * Parity status of each function is given in its comment. "parity unpinned" marks a
 * function that no test pins to something outside this file.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;

/* external cell-type codes */
#define TG 0 /* gas */
#define TI 1 /* interface */
#define TL 2 /* liquid */
#define TW 3 /* wall */
#define NOLAB (-1)

/* conversion classes (S5-S6) */
#define CF 1 /* fill */
#define CE 2 /* empty */

typedef struct {
  int32_t dim, nx, ny, nz;
  int32_t periodic[3];
  int32_t gas_from;  /* cells whose last coordinate is >= gas_from start as headspace gas; <0: none */
  int32_t rheology;  /* 0 Newtonian BGK, 1 power law, 2 Carreau-Yasuda */
  int32_t cleanup;   /* 1: stranded interface cells are filled / emptied */
  int32_t max_ids;   /* capacity of the bubble table (ids 0..max_ids-1) */
  double tau, D, sigma, kH, RT, k_pi, d_max, p_atm, q, eps, S0;
  double pl_n, pl_nu_ref, pl_gdot_ref, tau_min, tau_max;
  double accel[3]; /* body-force acceleration a (gravity); 0: no force term */
  double cy_tau0, cy_tau_inf, cy_lambda, cy_a, cy_n; /* Carreau-Yasuda (Eq. carreauTau) */
  int32_t flux_mode; /* 0: gas ledger (S3, S6); 1: the printed Eq. gascurrent (S3') */
} or_params;

typedef struct {
  or_params P;
  int D, Q, Qg;
  int nx, ny, nz;
  int64_t N;
  int ex[19], ey[19], ez[19], opp[19];
  double w[19], wg[7];
  double kg;      /* 1/c_s^2 of the ADE lattice */
  int force;      /* a != 0 */
  double omega_g; /* 1/tau_g */
  uint8_t *T;
  double *fc, *gc; /* post-collision populations [Q][N], [Qg][N] */
  double *M, *alpha, *rho, *ux, *uy, *uz, *kappa, *Pi;
  int32_t *label;
  int cap;
  double *bm, *bV, *bp;
  uint8_t *alive;
  int32_t next_id;
  i128 *Phi, *Gam;
  i128 lost_liquid, atm_gas, collapsed_gas;
  int64_t step;
  int err;
  char errmsg[256];
} OS;

static const double TWO64 = 18446744073709551616.0; /* 2^64 */

/* ---------------------------------------------------------------- fixed point ---
 * Cross-cell sums are order independent: every summand v becomes the integer
 * RN(v * 2^64) and the integers are added exactly. */
static i128 fx(double v) {
  double s = rint(v * TWO64);
  return (i128)s;
}
static double fxd(i128 a) { return (double)a * 0x1p-64; }

/* ---------------------------------------------------------------- lattices ---
 * D2Q9 and D3Q19 velocity sets and weights (Sec. 2, Fig. latticesfluid); the ADE
 * lattices D2Q5 / D3Q7 are the rest and axis directions of the same sets (Sec. 3.1). */
static const int E2[9][2] = {{0, 0}, {1, 0}, {-1, 0}, {0, 1}, {0, -1},
                             {1, 1}, {-1, -1}, {1, -1}, {-1, 1}};
static const int E3[19][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
                              {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                              {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                              {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static void set_lattice(OS *s) {
  int i;
  if (s->D == 2) {
    s->Q = 9;
    s->Qg = 5;
    for (i = 0; i < 9; i++) {
      s->ex[i] = E2[i][0];
      s->ey[i] = E2[i][1];
      s->ez[i] = 0;
      s->w[i] = i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
    for (i = 0; i < 5; i++) s->wg[i] = i == 0 ? 1.0 / 3.0 : 1.0 / 6.0;
    s->kg = 3.0;
  } else {
    s->Q = 19;
    s->Qg = 7;
    for (i = 0; i < 19; i++) {
      s->ex[i] = E3[i][0];
      s->ey[i] = E3[i][1];
      s->ez[i] = E3[i][2];
      s->w[i] = i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
    for (i = 0; i < 7; i++) s->wg[i] = i == 0 ? 1.0 / 4.0 : 1.0 / 8.0;
    s->kg = 4.0;
  }
  /* opposite direction: i and i+1 are a pair for odd i */
  s->opp[0] = 0;
  for (i = 1; i < s->Q; i++) s->opp[i] = (i & 1) ? i + 1 : i - 1;
}

/* ---------------------------------------------------------------- indexing --- */
static void coords(const OS *s, int64_t n, int *x, int *y, int *z) {
  *x = (int)(n % s->nx);
  *y = (int)((n / s->nx) % s->ny);
  *z = (int)(n / ((int64_t)s->nx * s->ny));
}

/* neighbour at offset (dx,dy,dz) with periodic wrap; -1 if it leaves a closed axis */
static int64_t nbr_off(const OS *s, int64_t n, int dx, int dy, int dz) {
  int x, y, z;
  coords(s, n, &x, &y, &z);
  x += dx;
  y += dy;
  z += dz;
  if (x < 0 || x >= s->nx) {
    if (!s->P.periodic[0]) return -1;
    x = (x + s->nx) % s->nx;
  }
  if (y < 0 || y >= s->ny) {
    if (!s->P.periodic[1]) return -1;
    y = (y + s->ny) % s->ny;
  }
  if (z < 0 || z >= s->nz) {
    if (s->D == 2 || !s->P.periodic[2]) return -1;
    z = (z + s->nz) % s->nz;
  }
  return x + (int64_t)s->nx * (y + (int64_t)s->ny * z);
}

static int64_t nbr(const OS *s, int64_t n, int i) { return nbr_off(s, n, s->ex[i], s->ey[i], s->ez[i]); }

#define F(s, i, n) ((s)->fc[(int64_t)(i) * (s)->N + (n)])
#define G(s, i, n) ((s)->gc[(int64_t)(i) * (s)->N + (n)])

/* ---------------------------------------------------------------- equilibria ---
 * Eq. equilibrium with c_s^2 = 1/3; every product and sum in the order written. */
static double feq(const OS *s, int i, double rho, double ux, double uy, double uz) {
  double eu = ((s->ex[i] * ux + s->ey[i] * uy) + s->ez[i] * uz);
  double uu = ((ux * ux + uy * uy) + uz * uz);
  return (rho * s->w[i]) * (((1.0 + 3.0 * eu) + (4.5 * eu) * eu) - 1.5 * uu);
}

/* ADE equilibrium (Sec. 3.1): w_i c (1 + e.u / c_s^2) */
static double geq(const OS *s, int i, double c, double ux, double uy, double uz) {
  double eu = ((s->ex[i] * ux + s->ey[i] * uy) + s->ez[i] * uz);
  return (s->wg[i] * c) * (1.0 + s->kg * eu);
}

/* Force term of Eq. collision for an acceleration a, written out in the form of Guo,
 * Zheng and Shi (2002), the reading taken of the paper's garbled formula and sign:
 * F_i = w_i rho [ (e_i - u) / c_s^2 + (e_i . u) e_i / c_s^4 ] . a, added after the BGK
 * relaxation with the factor (1 - omega / 2), and u = (sum f e + rho a / 2) / rho.
 * Moments: sum F_i = 0 and sum F_i e_i = rho a, so the momentum of a cell grows by
 * exactly rho a per step whatever omega is (pinned on a periodic box), and a channel
 * between walls reaches the parabolic (Newtonian) or power-law profile (pinned). */
static double force_i(const OS *s, int i, double rho, double ux, double uy, double uz) {
  const double *a = s->P.accel;
  double ea = ((s->ex[i] * a[0] + s->ey[i] * a[1]) + s->ez[i] * a[2]);
  double ua = ((ux * a[0] + uy * a[1]) + uz * a[2]);
  double eu = ((s->ex[i] * ux + s->ey[i] * uy) + s->ez[i] * uz);
  return (rho * s->w[i]) * (3.0 * (ea - ua) + (9.0 * eu) * ea);
}

/* moments of a population vector: rho = sum f_i, u = (sum f_i e_i) / rho (Sec. 2) */
static void moments(const OS *s, const double *f, double *rho, double *ux, double *uy, double *uz) {
  double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
  int i;
  for (i = 0; i < s->Q; i++) r = r + f[i];
  for (i = 0; i < s->Q; i++) {
    if (s->ex[i] == 1) jx = jx + f[i];
    if (s->ex[i] == -1) jx = jx - f[i];
  }
  for (i = 0; i < s->Q; i++) {
    if (s->ey[i] == 1) jy = jy + f[i];
    if (s->ey[i] == -1) jy = jy - f[i];
  }
  for (i = 0; i < s->Q; i++) {
    if (s->ez[i] == 1) jz = jz + f[i];
    if (s->ez[i] == -1) jz = jz - f[i];
  }
  *rho = r;
  *ux = jx / r;
  *uy = jy / r;
  *uz = jz / r;
}

/* --------------------------------------------------------------- rheology ---
 * Power-law limit of Eq. carreauTau (mu_inf = 0, lambda*gdot >> 1):
 * nu = nu_ref (gdot / gdot_ref)^(n-1), tau = 1/2 + 3 nu (Eq. tau). The shear rate is
 * gdot = sqrt(2 S:S) with S = -Pi_neq / (2 rho c_s^2 tau), i.e. gdot = K |Pi_neq| / (rho tau)
 * with K = 3/sqrt(2), so tau is defined implicitly. With s = tau - 1/2 the equation is
 * s = A (s + 1/2)^(1-n), A = 3 nu_ref (K |Pi_neq| / (rho gdot_ref))^(n-1); in t = ln s it
 * reads F(t) = t - (1-n) ln(e^t + 1/2) - ln A = 0 with F increasing and concave, so
 * Newton's method from t = ln(3 nu_ref) converges monotonically; four steps are taken,
 * then tau is clamped to [tau_min, tau_max]. Zero shear gives the clamp bound. Pinned
 * against a bracketing root solve of the implicit equation. */
static double powerlaw_tau_iter(const or_params *P, double rho, double pn, int iters) {
  double n = P->pl_n;
  double tau;
  if (!(pn > 0.0)) {
    tau = n < 1.0 ? P->tau_max : (n > 1.0 ? P->tau_min : 0.5 + 3.0 * P->pl_nu_ref);
  } else {
    double lnA = log(3.0 * P->pl_nu_ref) + (n - 1.0) * log((2.1213203435596424 * pn) / (rho * P->pl_gdot_ref));
    double t = log(3.0 * P->pl_nu_ref);
    int it;
    for (it = 0; it < iters; it++) {
      double et = exp(t);
      double Fv = (t - (1.0 - n) * log(et + 0.5)) - lnA;
      double dF = 1.0 - ((1.0 - n) * et) / (et + 0.5);
      t = t - Fv / dF;
    }
    tau = 0.5 + exp(t);
  }
  if (tau < P->tau_min) tau = P->tau_min;
  if (tau > P->tau_max) tau = P->tau_max;
  return tau;
}
double or_powerlaw_tau(const or_params *P, double rho, double pn) { return powerlaw_tau_iter(P, rho, pn, 4); }

/* Carreau-Yasuda relaxation time, Eq. carreauTau in full:
 * (tau - tau_inf) / (tau0 - tau_inf) = (1 + (lambda gdot)^a)^((n - 1) / a), with the shear rate
 * gdot = K |Pi_neq| / (rho tau), K = 3/sqrt(2), taken at the cell's own tau as for the power law,
 * so tau solves G(tau) = tau - h(tau) = 0 with h the right-hand side times (tau0 - tau_inf) plus
 * tau_inf. For shear thinning (n <= 1, tau0 >= tau_inf, the use the paper names) h rises with tau
 * and h' <= (tau0 - tau_inf)(1 - n) / tau, so with (tau0 - tau_inf)(1 - n) < tau_inf the root in
 * [tau_inf, tau0] is unique; G(tau_inf) <= 0 <= G(tau0). It is found here by plain bisection
 * down to adjacent doubles. Zero shear gives tau0. Pinned against a bracketing root solve, the
 * Newtonian limits (lambda = 0, n = 1, tau0 = tau_inf) and body-force-driven channel flow against
 * the profile integrated from the model's stress-shear relation. */
double or_cy_tau(const or_params *P, double rho, double pn) {
  double t0 = P->cy_tau0, ti = P->cy_tau_inf;
  if (!(pn > 0.0) || P->cy_lambda == 0.0 || t0 == ti) return t0;
  double g0 = (2.1213203435596424 * pn) / rho; /* gdot * tau */
  double m = (P->cy_n - 1.0) / P->cy_a;
  double lo = ti, hi = t0;
  int it;
  for (it = 0; it < 2000; it++) {
    double mid = 0.5 * (lo + hi);
    if (!(mid > lo && mid < hi)) break;
    double gd = g0 / mid;
    double h = ti + (t0 - ti) * pow(1.0 + pow(P->cy_lambda * gd, P->cy_a), m);
    if (mid - h < 0.0)
      lo = mid;
    else
      hi = mid;
  }
  /* the closer of the two adjacent end points */
  double glo = lo - (ti + (t0 - ti) * pow(1.0 + pow(P->cy_lambda * g0 / lo, P->cy_a), m));
  double ghi = hi - (ti + (t0 - ti) * pow(1.0 + pow(P->cy_lambda * g0 / hi, P->cy_a), m));
  return fabs(glo) <= fabs(ghi) ? lo : hi;
}
double or_powerlaw_tau_iter(const or_params *P, double rho, double pn, int iters) {
  return powerlaw_tau_iter(P, rho, pn, iters);
}

/* Frobenius norm of the non-equilibrium momentum flux Pi_neq = sum e e (f - feq).
 * With a body force F = rho a (Guo et al. 2002) the flux that measures the strain rate is
 * Pi_neq + (u F + F u) / 2: in a uniformly accelerated box, where the strain rate is
 * zero, the pre-collision populations carry Pi_neq = -(u F + F u) / 2 (the steady
 * non-equilibrium part is minus half the force term). Pinned by that box (the power law
 * then relaxes at its zero-shear clamp) and by body-force-driven power-law channel flow
 * against its closed form. */
static double pineq_norm(const OS *s, const double *ft, const double *fe, double rho, double ux, double uy,
                         double uz) {
  double pxx = 0, pyy = 0, pzz = 0, pxy = 0, pxz = 0, pyz = 0;
  int i;
  for (i = 0; i < s->Q; i++) {
    double d = ft[i] - fe[i];
    pxx = pxx + (double)(s->ex[i] * s->ex[i]) * d;
    pyy = pyy + (double)(s->ey[i] * s->ey[i]) * d;
    pzz = pzz + (double)(s->ez[i] * s->ez[i]) * d;
    pxy = pxy + (double)(s->ex[i] * s->ey[i]) * d;
    pxz = pxz + (double)(s->ex[i] * s->ez[i]) * d;
    pyz = pyz + (double)(s->ey[i] * s->ez[i]) * d;
  }
  if (s->force) {
    double Fx = rho * s->P.accel[0], Fy = rho * s->P.accel[1], Fz = rho * s->P.accel[2];
    pxx = pxx + ux * Fx;
    pyy = pyy + uy * Fy;
    pzz = pzz + uz * Fz;
    pxy = pxy + 0.5 * (ux * Fy + uy * Fx);
    pxz = pxz + 0.5 * (ux * Fz + uz * Fx);
    pyz = pyz + 0.5 * (uy * Fz + uz * Fy);
  }
  double ss = ((pxx * pxx + pyy * pyy) + pzz * pzz) + 2.0 * ((pxy * pxy + pxz * pxz) + pyz * pyz);
  return sqrt(ss);
}

/* ------------------------------------------------------------------- PLIC ---
 * Signed distance s from the centre of a unit cell to the plane with normal m
 * (unit, pointing into the liquid) that leaves the liquid fraction alpha on the +m
 * side. Analytic inverse of the cut-cube volume (Scardovelli & Zaleski 2000), as the
 * paper uses for its disjoining-pressure distance (Sec. 3.3). Pinned against the
 * inclusion-exclusion volume of a cut cube evaluated in exact rational arithmetic. */

/* root of the monic cubic a^3 + b a^2 + c a + d on [lo, hi], where it is unique */
static double cubic_root_in(double b, double c, double d, double lo, double hi) {
  double p = c - (b * b) / 3.0;
  double qq = ((2.0 * b * b * b) / 27.0 - (b * c) / 3.0) + d;
  double shift = -b / 3.0;
  double best = 0.5 * (lo + hi), bestd = 1e300;
  double disc = (qq * qq) / 4.0 + (p * p * p) / 27.0;
  double cand[3];
  int nc = 0, k;
  if (p < 0.0 && disc <= 0.0) {
    double r = 2.0 * sqrt(-p / 3.0);
    double arg = ((3.0 * qq) / (2.0 * p)) * sqrt(-3.0 / p);
    if (arg > 1.0) arg = 1.0;
    if (arg < -1.0) arg = -1.0;
    double th = acos(arg) / 3.0;
    for (k = 0; k < 3; k++) cand[nc++] = r * cos(th - (2.0 * M_PI * k) / 3.0) + shift;
  } else {
    double sd = sqrt(disc > 0.0 ? disc : 0.0);
    cand[nc++] = cbrt(-qq / 2.0 + sd) + cbrt(-qq / 2.0 - sd) + shift;
  }
  for (k = 0; k < nc; k++) {
    double t = cand[k];
    double dd = t < lo ? lo - t : (t > hi ? t - hi : 0.0);
    if (dd < bestd) {
      bestd = dd;
      best = t;
    }
  }
  if (best < lo) best = lo;
  if (best > hi) best = hi;
  /* two Newton polishing steps on the same cubic, kept inside [lo, hi] */
  for (k = 0; k < 2; k++) {
    double f = ((best + b) * best + c) * best + d;
    double df = (3.0 * best + 2.0 * b) * best + c;
    if (df != 0.0) {
      double nb2 = best - f / df;
      if (nb2 >= lo && nb2 <= hi) best = nb2;
    }
  }
  return best;
}

/* plane constant a in [0, 1/2] with vol{x in [0,1]^3 : n.x <= a} = v, for
 * 0 <= n1 <= n2 <= n3, n1 + n2 + n3 = 1, 0 <= v <= 1/2 */
static double sz_inverse3(double m1, double m2, double m3, double v) {
  if (m2 <= 0.0) return v; /* normal along one axis */
  if (m1 <= 0.0) {         /* two-dimensional cut in (m2, m3) */
    double v1 = m2 / (2.0 * m3);
    if (v <= v1) return sqrt((2.0 * m2 * m3) * v);
    return m3 * v + 0.5 * m2;
  }
  double m12 = m1 + m2;
  double v1 = (m1 * m1) / (6.0 * m2 * m3);
  double v2 = v1 + (m2 - m1) / (2.0 * m3);
  double v3;
  if (m3 < m12) {
    double a = m3;
    v3 = ((a * a) * (3.0 * m12 - a) + (m1 * m1) * (m1 - 3.0 * a) + (m2 * m2) * (m2 - 3.0 * a)) /
         (6.0 * m1 * m2 * m3);
  } else {
    v3 = m12 / (2.0 * m3);
  }
  if (v < v1) return cbrt((6.0 * m1 * m2 * m3) * v);
  if (v < v2) return 0.5 * (m1 + sqrt((8.0 * m2 * m3) * v - (m1 * m1) / 3.0));
  if (v < v3) {
    double hi = m3 < m12 ? m3 : m12;
    double c3 = 3.0 * (m1 * m1 + m2 * m2);
    double c0 = -(((m1 * m1 * m1) + (m2 * m2 * m2)) - (6.0 * m1 * m2 * m3) * v);
    return cubic_root_in(-3.0 * m12, c3, c0, m2, hi);
  }
  if (m3 < m12) {
    double s2 = (m1 * m1 + m2 * m2) + m3 * m3;
    double s3 = ((m1 * m1 * m1) + (m2 * m2 * m2)) + (m3 * m3 * m3);
    return cubic_root_in(-1.5, 1.5 * s2, -0.5 * (s3 - (6.0 * m1 * m2 * m3) * v), m3, 0.5);
  }
  return m3 * v + 0.5 * m12;
}

static double clamp01(double a) { return a < 0.0 ? 0.0 : (a > 1.0 ? 1.0 : a); }

double or_plic_offset(int dim, double alpha, double mx, double my, double mz) {
  double a = clamp01(alpha);
  double v = a < 1.0 - a ? a : 1.0 - a;
  double ax = fabs(mx), ay = fabs(my), az = dim == 3 ? fabs(mz) : 0.0;
  double l1 = (ax + ay) + az;
  double c;
  if (l1 <= 0.0) return 0.0;
  if (dim == 2) {
    double n1 = ax < ay ? ax : ay, n2 = ax < ay ? ay : ax;
    n1 = n1 / l1;
    n2 = n2 / l1;
    double v1 = n1 / (2.0 * n2);
    if (v <= v1)
      c = sqrt((2.0 * n1 * n2) * v);
    else
      c = n2 * v + 0.5 * n1;
  } else {
    double t, m1 = ax, m2 = ay, m3 = az;
    if (m1 > m2) { t = m1; m1 = m2; m2 = t; }
    if (m2 > m3) { t = m2; m2 = m3; m3 = t; }
    if (m1 > m2) { t = m1; m1 = m2; m2 = t; }
    m1 = m1 / l1;
    m2 = m2 / l1;
    m3 = m3 / l1;
    c = sz_inverse3(m1, m2, m3, v);
  }
  double smag = (0.5 - c) * l1;
  return a < 0.5 ? smag : -smag;
}

/* ---------------------------------------------------------------- geometry --- */
/* fill fraction of a cell as seen by the geometric stencils (clamped to [0,1]);
 * walls and off-domain cells read the centre cell's value */
static double alpha_at(const OS *s, int64_t n, double acentre) {
  if (n < 0) return acentre;
  switch (s->T[n]) {
    case TG: return 0.0;
    case TL: return 1.0;
    case TI: return clamp01(s->alpha[n]);
    default: return acentre;
  }
}

/* unit normal from central differences of alpha, pointing into the liquid;
 * returns 0 if the gradient vanishes */
static int normal_at(const OS *s, int64_t n, double m[3]) {
  double ac = clamp01(s->alpha[n]);
  double gx = 0.5 * (alpha_at(s, nbr_off(s, n, 1, 0, 0), ac) - alpha_at(s, nbr_off(s, n, -1, 0, 0), ac));
  double gy = 0.5 * (alpha_at(s, nbr_off(s, n, 0, 1, 0), ac) - alpha_at(s, nbr_off(s, n, 0, -1, 0), ac));
  double gz = 0.0;
  if (s->D == 3)
    gz = 0.5 * (alpha_at(s, nbr_off(s, n, 0, 0, 1), ac) - alpha_at(s, nbr_off(s, n, 0, 0, -1), ac));
  double gn = sqrt((gx * gx + gy * gy) + gz * gz);
  if (gn == 0.0) {
    m[0] = m[1] = m[2] = 0.0;
    return 0;
  }
  m[0] = gx / gn;
  m[1] = gy / gn;
  m[2] = gz / gn;
  return 1;
}

/* Gaussian elimination with partial pivoting (first maximum on ties); returns 0 when a
 * pivot magnitude falls below 1e-9 of the largest diagonal entry of the normal matrix,
 * i.e. when the points do not determine the fit (e.g. one-sided point sets at walls) */
static int solve(int n, double A[6][6], double b[6], double x[6]) {
  int c, r, k;
  double scale = 0.0;
  for (c = 0; c < n; c++)
    if (A[c][c] > scale) scale = A[c][c];
  double tiny = 1e-9 * scale;
  for (c = 0; c < n; c++) {
    int piv = c;
    for (r = c + 1; r < n; r++)
      if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
    if (!(fabs(A[piv][c]) >= tiny)) return 0;
    if (piv != c) {
      for (k = 0; k < n; k++) {
        double t = A[c][k];
        A[c][k] = A[piv][k];
        A[piv][k] = t;
      }
      double t = b[c];
      b[c] = b[piv];
      b[piv] = t;
    }
    for (r = c + 1; r < n; r++) {
      double f = A[r][c] / A[c][c];
      for (k = c; k < n; k++) A[r][k] = A[r][k] - f * A[c][k];
      b[r] = b[r] - f * b[c];
    }
  }
  for (r = n - 1; r >= 0; r--) {
    double acc = b[r];
    for (k = r + 1; k < n; k++) acc = acc - A[r][k] * x[k];
    x[r] = acc / A[r][r];
  }
  return 1;
}

/* S10. Mean curvature kappa = (k1+k2)/2 at an interface cell, positive for a gas
 * bubble, so that 2 sigma kappa is the Laplace jump (Eq. rhob). In 2D the circle
 * term is halved the same way (kappa = 1/(2R)). Points: the PLIC plane point of the
 * cell and of every interface cell of its 3x3x3 block (5x5 in 2D, where a 3x3 block
 * holds too few points for a stable parabola), each from its own normal and fill fraction; least-squares paraboloid (3D) or parabola (2D) in the frame of the
 * centre normal. Pinned by voxelised spheres / circles of known radius. */
double or_curvature_at(const OS *s, int64_t n) {
  double m[3], mp[3];
  int dx, dy, dz, a, b;
  if (!normal_at(s, n, m)) return 0.0;
  double A[6][6], rhs[6], sol[6];
  int nun = s->D == 3 ? 6 : 3;
  memset(A, 0, sizeof A);
  memset(rhs, 0, sizeof rhs);
  double t1[3], t2[3];
  if (s->D == 3) {
    int k = 0;
    if (fabs(m[1]) < fabs(m[k])) k = 1;
    if (fabs(m[2]) < fabs(m[k])) k = 2;
    double c0, c1, c2;
    if (k == 0) { c0 = 0.0; c1 = m[2]; c2 = -m[1]; }
    else if (k == 1) { c0 = -m[2]; c1 = 0.0; c2 = m[0]; }
    else { c0 = m[1]; c1 = -m[0]; c2 = 0.0; }
    double cn = sqrt((c0 * c0 + c1 * c1) + c2 * c2);
    t1[0] = c0 / cn;
    t1[1] = c1 / cn;
    t1[2] = c2 / cn;
    t2[0] = m[1] * t1[2] - m[2] * t1[1];
    t2[1] = m[2] * t1[0] - m[0] * t1[2];
    t2[2] = m[0] * t1[1] - m[1] * t1[0];
  } else {
    t1[0] = -m[1];
    t1[1] = m[0];
    t1[2] = 0.0;
    t2[0] = t2[1] = t2[2] = 0.0;
  }
  int np = 0;
  int rr = s->D == 3 ? 1 : 2; /* block half-width: 3x3x3 in 3D, 5x5 in 2D */
  int zlo = s->D == 3 ? -1 : 0, zhi = s->D == 3 ? 1 : 0;
  /* the centre point first, then the block in (dz, dy, dx) ascending order */
  int pass;
  for (pass = 0; pass < 2; pass++) {
    for (dz = zlo; dz <= zhi; dz++)
      for (dy = -rr; dy <= rr; dy++)
        for (dx = -rr; dx <= rr; dx++) {
          int centre = (dx == 0 && dy == 0 && dz == 0);
          if ((pass == 0) != centre) continue;
          int64_t y = centre ? n : nbr_off(s, n, dx, dy, dz);
          if (y < 0 || s->T[y] != TI) continue;
          if (!normal_at(s, y, mp)) continue;
          double off = or_plic_offset(s->D, s->alpha[y], mp[0], mp[1], mp[2]);
          double px = (double)dx + off * mp[0];
          double py = (double)dy + off * mp[1];
          double pz = (double)dz + off * mp[2];
          double u = (px * t1[0] + py * t1[1]) + pz * t1[2];
          double v = (px * t2[0] + py * t2[1]) + pz * t2[2];
          double h = (px * m[0] + py * m[1]) + pz * m[2];
          double phi[6];
          if (s->D == 3) {
            phi[0] = u * u;
            phi[1] = v * v;
            phi[2] = u * v;
            phi[3] = u;
            phi[4] = v;
            phi[5] = 1.0;
          } else {
            phi[0] = u * u;
            phi[1] = u;
            phi[2] = 1.0;
          }
          for (a = 0; a < nun; a++) {
            for (b = 0; b < nun; b++) A[a][b] = A[a][b] + phi[a] * phi[b];
            rhs[a] = rhs[a] + phi[a] * h;
          }
          np++;
        }
  }
  if (np < nun) return 0.0;
  /* 3D: ridge term on the quadratic coefficients; it keeps the fit determined when the
   * points of the 3x3x3 block lie on one side of the cell (next to a wall) and pulls the
   * undetermined curvature towards zero there (the 5x5 block of 2D needs none) */
  if (s->D == 3)
    for (a = 0; a < 3; a++) A[a][a] = A[a][a] + 1e-2;
  if (!solve(nun, A, rhs, sol)) return 0.0;
  double kap;
  if (s->D == 3) {
    double cA = sol[0], cB = sol[1], cC = sol[2], cD = sol[3], cE = sol[4];
    double num = (((1.0 + cE * cE) * (2.0 * cA)) - (((2.0 * cD) * cE) * cC)) + ((1.0 + cD * cD) * (2.0 * cB));
    double t = (1.0 + cD * cD) + cE * cE;
    double den = 2.0 * (t * sqrt(t));
    kap = -(num / den);
  } else {
    double cA = sol[0], cD = sol[1];
    double t = 1.0 + cD * cD;
    kap = -(cA / (t * sqrt(t)));
  }
  if (kap > 1.0) kap = 1.0;
  if (kap < -1.0) kap = -1.0;
  return kap;
}

/* S11. Disjoining pressure (Sec. 3.3): march from the cell centre along the normal
 * into the liquid with the traversal of Appendix A (Amanatides & Woo), every tied
 * axis stepping together, for at most d_max cells; stop at a wall; the first cell of
 * another bubble's interface or gas ends the search. The gap d is the ray length to
 * the other interface, taken inside the hit cell from its fill fraction, minus the
 * own PLIC offset. Pi = k_Pi (d_max - d) for d < d_max. Pinned by the flat-film gap
 * test and by exact rational ray-grid traversal. */
double or_disjoining_at(const OS *s, int64_t n) {
  double m[3];
  if (s->P.k_pi <= 0.0) return 0.0;
  if (!normal_at(s, n, m)) return 0.0;
  int dm = (int)s->P.d_max;
  double bmax[3], bdel[3];
  int step[3], k, it, D = s->D;
  int x, y, z;
  coords(s, n, &x, &y, &z);
  int pos[3] = {x, y, z};
  for (k = 0; k < 3; k++) {
    if (k >= D) {
      bmax[k] = INFINITY;
      bdel[k] = INFINITY;
      step[k] = 1;
      continue;
    }
    bmax[k] = fabs(0.5 / m[k]);
    bdel[k] = fabs(1.0 / m[k]);
    step[k] = m[k] >= 0.0 ? 1 : -1;
  }
  int64_t cur = n;
  for (it = 1; it <= dm; it++) {
    double bmin = bmax[0];
    if (bmax[1] < bmin) bmin = bmax[1];
    if (bmax[2] < bmin) bmin = bmax[2];
    int d[3] = {0, 0, 0};
    for (k = 0; k < D; k++)
      if (bmax[k] == bmin) {
        bmax[k] = bmax[k] + bdel[k];
        d[k] = step[k];
      }
    pos[0] += d[0];
    pos[1] += d[1];
    pos[2] += d[2];
    cur = nbr_off(s, cur, d[0], d[1], d[2]);
    if (cur < 0) return 0.0; /* left a closed axis */
    if (s->label[cur] == s->label[n]) continue;
    if (s->T[cur] == TW) return 0.0;
    if (s->T[cur] == TI || s->T[cur] == TG) {
      double bout = bmax[0];
      if (bmax[1] < bout) bout = bmax[1];
      if (bmax[2] < bout) bout = bmax[2];
      double ay = s->T[cur] == TI ? clamp01(s->alpha[cur]) : 0.0;
      double dprime = bout - (1.0 - ay) * (bout - bmin);
      double off = or_plic_offset(D, s->alpha[n], m[0], m[1], m[2]);
      double dd = dprime - off;
      if (dd < 0.0) dd = 0.0;
      if (dd < s->P.d_max) return s->P.k_pi * (s->P.d_max - dd);
      return 0.0;
    }
  }
  return 0.0;
}

/* --------------------------------------------------------------- bubble table --- */
static int fail(OS *s, const char *msg) {
  s->err = 1;
  snprintf(s->errmsg, sizeof s->errmsg, "%s", msg);
  return -1;
}

typedef struct {
  int64_t comp;
  int32_t lab;
  i128 v;
} Entry;

static int cmp_entry(const void *a, const void *b) {
  const Entry *x = a, *y = b;
  if (x->comp != y->comp) return x->comp < y->comp ? -1 : 1;
  if (x->lab != y->lab) return x->lab < y->lab ? -1 : 1;
  return 0;
}

/* S8 + S9. Connected components of the gas and interface cells under the lattice
 * neighbourhood, visited in ascending cell order so that each component's root is its
 * smallest cell index. Bubble gas is carried to the new components in proportion to
 * the volume each old bubble leaves in them (Sec. 3.5); components that touch the
 * headspace join the atmosphere (id 0, fixed pressure). Pinned against
 * scipy.ndimage.label and hand-worked merge / split cases. */
static int relabel(OS *s, int apply_flux) {
  int64_t N = s->N, n, k;
  int64_t *comp = malloc(sizeof(int64_t) * N);
  int64_t *queue = malloc(sizeof(int64_t) * N);
  int64_t ncomp = 0;
  int i;
  for (n = 0; n < N; n++) comp[n] = -1;
  for (n = 0; n < N; n++) {
    if ((s->T[n] != TG && s->T[n] != TI) || comp[n] >= 0) continue;
    int64_t head = 0, tail = 0;
    queue[tail++] = n;
    comp[n] = ncomp;
    while (head < tail) {
      int64_t c = queue[head++];
      for (i = 1; i < s->Q; i++) {
        int64_t y = nbr(s, c, i);
        if (y < 0 || comp[y] >= 0) continue;
        if (s->T[y] != TG && s->T[y] != TI) continue;
        comp[y] = ncomp;
        queue[tail++] = y;
      }
    }
    ncomp++;
  }
  /* (component, old id, volume share) triples */
  int64_t ne = 0;
  for (n = 0; n < N; n++)
    if (comp[n] >= 0) ne++;
  Entry *e = malloc(sizeof(Entry) * (ne > 0 ? ne : 1));
  int64_t j = 0;
  for (n = 0; n < N; n++) {
    if (comp[n] < 0) continue;
    if (s->label[n] < 0 || s->label[n] >= s->cap) {
      free(comp); free(queue); free(e);
      return fail(s, "gas/interface cell without a bubble id");
    }
    e[j].comp = comp[n];
    e[j].lab = s->label[n];
    e[j].v = fx(1.0 - (s->T[n] == TG ? 0.0 : s->alpha[n]));
    j++;
  }
  qsort(e, ne, sizeof(Entry), cmp_entry);
  /* aggregate equal (comp, id) */
  int64_t nu = 0;
  for (k = 0; k < ne; k++) {
    if (nu > 0 && e[nu - 1].comp == e[k].comp && e[nu - 1].lab == e[k].lab)
      e[nu - 1].v += e[k].v;
    else
      e[nu++] = e[k];
  }
  int cap = s->cap;
  double *mprime = calloc(cap, sizeof(double));
  i128 *vtot = calloc(cap, sizeof(i128));
  i128 *vatm = calloc(cap, sizeof(i128));
  uint8_t *present = calloc(cap, 1), *assigned = calloc(cap, 1), *inatm = calloc(cap, 1);
  int64_t *firstK = malloc(sizeof(int64_t) * cap);
  uint8_t *compatm = calloc(ncomp > 0 ? ncomp : 1, 1);
  for (i = 0; i < cap; i++) firstK[i] = -1;
  /* S8: each old bubble first receives this step's diffusion flux and the gas moved
   * by cell conversions */
  for (i = 1; i < cap; i++)
    if (s->alive[i]) mprime[i] = s->bm[i] + (apply_flux ? fxd(s->Phi[i] + s->Gam[i]) : 0.0);
  if (apply_flux) s->atm_gas += s->Phi[0] + s->Gam[0];
  for (k = 0; k < nu; k++)
    if (e[k].lab == 0) compatm[e[k].comp] = 1;
  for (k = 0; k < nu; k++) {
    int lb = e[k].lab;
    if (lb == 0) continue;
    present[lb] = 1;
    vtot[lb] += e[k].v;
    if (compatm[e[k].comp]) {
      vatm[lb] += e[k].v;
      inatm[lb] = 1;
    } else if (firstK[lb] < 0) {
      firstK[lb] = e[k].comp;
    }
  }
  /* atmosphere share of each old bubble (all atmosphere components together) */
  for (i = 1; i < cap; i++) {
    if (!inatm[i]) continue;
    double c;
    if (vtot[i] == 0)
      c = firstK[i] < 0 ? mprime[i] : 0.0;
    else
      c = mprime[i] * (fxd(vatm[i]) / fxd(vtot[i]));
    s->atm_gas += fx(c);
  }
  /* new table */
  double *nm = calloc(cap, sizeof(double)), *nV = calloc(cap, sizeof(double));
  uint8_t *nalive = calloc(cap, 1);
  int32_t *newid = malloc(sizeof(int32_t) * (ncomp > 0 ? ncomp : 1));
  int64_t a0 = 0;
  while (a0 < nu) {
    int64_t a1 = a0;
    while (a1 < nu && e[a1].comp == e[a0].comp) a1++;
    int64_t K = e[a0].comp;
    if (compatm[K]) {
      newid[K] = 0;
    } else {
      int id = -1;
      for (k = a0; k < a1; k++)
        if (!assigned[e[k].lab]) {
          id = e[k].lab;
          break;
        }
      if (id < 0) {
        if (s->next_id >= cap) {
          free(comp); free(queue); free(e); free(mprime); free(vtot); free(vatm);
          free(present); free(assigned); free(inatm); free(firstK); free(compatm);
          free(nm); free(nV); free(nalive); free(newid);
          return fail(s, "bubble table capacity exceeded");
        }
        id = s->next_id++;
      }
      assigned[id] = 1;
      double mk = 0.0;
      i128 vk = 0;
      for (k = a0; k < a1; k++) {
        int lb = e[k].lab;
        double c;
        if (vtot[lb] == 0)
          c = firstK[lb] == K ? mprime[lb] : 0.0;
        else
          c = mprime[lb] * (fxd(e[k].v) / fxd(vtot[lb]));
        mk = mk + c;
        vk += e[k].v;
      }
      newid[K] = id;
      nm[id] = mk;
      nV[id] = fxd(vk);
      nalive[id] = 1;
    }
    a0 = a1;
  }
  /* old bubbles with no cells left */
  for (i = 1; i < cap; i++)
    if (s->alive[i] && !present[i]) s->collapsed_gas += fx(mprime[i]);
  for (n = 0; n < N; n++)
    if (comp[n] >= 0) s->label[n] = newid[comp[n]];
  for (i = 0; i < cap; i++) {
    s->alive[i] = nalive[i];
    s->bm[i] = nalive[i] ? nm[i] : 0.0;
    s->bV[i] = nalive[i] ? nV[i] : 0.0;
  }
  /* S9: ideal-gas pressure (Eq. idealgas), volume floored at half a cell */
  for (i = 1; i < cap; i++)
    s->bp[i] = s->alive[i] ? (s->bm[i] * s->P.RT) / (s->bV[i] > 0.5 ? s->bV[i] : 0.5) : 0.0;
  s->bp[0] = s->P.p_atm;
  s->alive[0] = 1;
  free(comp); free(queue); free(e); free(mprime); free(vtot); free(vatm); free(present);
  free(assigned); free(inatm); free(firstK); free(compatm); free(nm); free(nV); free(nalive);
  free(newid);
  return 0;
}

static void geometry(OS *s) {
  int64_t n;
  for (n = 0; n < s->N; n++) {
    if (s->T[n] == TI) {
      s->kappa[n] = or_curvature_at(s, n);
    } else {
      s->kappa[n] = 0.0;
    }
  }
  for (n = 0; n < s->N; n++) s->Pi[n] = s->T[n] == TI ? or_disjoining_at(s, n) : 0.0;
}

/* ------------------------------------------------------------------ create --- */
void *or_create(const or_params *P) {
  OS *s = calloc(1, sizeof(OS));
  int64_t n, i;
  s->P = *P;
  s->D = P->dim;
  s->nx = P->nx;
  s->ny = P->ny;
  s->nz = P->dim == 2 ? 1 : P->nz;
  s->N = (int64_t)s->nx * s->ny * s->nz;
  set_lattice(s);
  s->omega_g = 1.0 / (0.5 + s->kg * P->D); /* D = c_s^2 (tau_g - 1/2), Eq. diffusionconst */
  if (s->D == 2) s->P.accel[2] = 0.0; /* a plane flow has no third component */
  s->force = s->P.accel[0] != 0.0 || s->P.accel[1] != 0.0 || s->P.accel[2] != 0.0;
  int64_t N = s->N;
  s->T = calloc(N, 1);
  s->fc = calloc(N * s->Q, sizeof(double));
  s->gc = calloc(N * s->Qg, sizeof(double));
  s->M = calloc(N, sizeof(double));
  s->alpha = calloc(N, sizeof(double));
  s->rho = calloc(N, sizeof(double));
  s->ux = calloc(N, sizeof(double));
  s->uy = calloc(N, sizeof(double));
  s->uz = calloc(N, sizeof(double));
  s->kappa = calloc(N, sizeof(double));
  s->Pi = calloc(N, sizeof(double));
  s->label = malloc(N * sizeof(int32_t));
  s->cap = P->max_ids;
  s->bm = calloc(s->cap, sizeof(double));
  s->bV = calloc(s->cap, sizeof(double));
  s->bp = calloc(s->cap, sizeof(double));
  s->alive = calloc(s->cap, 1);
  s->Phi = calloc(s->cap, sizeof(i128));
  s->Gam = calloc(s->cap, sizeof(i128));
  s->alive[0] = 1;
  s->bp[0] = P->p_atm;
  s->next_id = 1;
  double c0 = (P->S0 * P->kH) * P->p_atm; /* supersaturation S = c0 / (k_H p_atm) */
  int last = s->D == 2 ? s->ny : s->nz;
  for (n = 0; n < N; n++) {
    int x, y, z;
    coords(s, n, &x, &y, &z);
    int c[3] = {x, y, z}, dims[3] = {s->nx, s->ny, s->nz}, a, wall = 0;
    for (a = 0; a < s->D; a++)
      if (!P->periodic[a] && (c[a] == 0 || c[a] == dims[a] - 1)) wall = 1;
    int lc = s->D == 2 ? y : z;
    (void)last;
    s->label[n] = NOLAB;
    if (wall) {
      s->T[n] = TW;
    } else if (P->gas_from >= 0 && lc >= P->gas_from) {
      s->T[n] = TG;
      s->label[n] = 0;
    } else {
      s->T[n] = TL;
      s->alpha[n] = 1.0;
      s->M[n] = 1.0;
      s->rho[n] = 1.0;
    }
    for (i = 0; i < s->Q; i++) F(s, i, n) = s->T[n] == TW ? 0.0 : s->w[i];
    for (i = 0; i < s->Qg; i++) G(s, i, n) = s->T[n] == TW ? 0.0 : s->wg[i] * c0;
  }
  return s;
}

void or_destroy(void *h) {
  OS *s = h;
  if (!s) return;
  free(s->T); free(s->fc); free(s->gc); free(s->M); free(s->alpha); free(s->rho);
  free(s->ux); free(s->uy); free(s->uz); free(s->kappa); free(s->Pi); free(s->label);
  free(s->bm); free(s->bV); free(s->bp); free(s->alive); free(s->Phi); free(s->Gam);
  free(s);
}

const char *or_error(void *h) { return ((OS *)h)->errmsg; }

/* S0. Nucleation (Sec. 3.4): each sphere (3D) or disk (2D) is voxelised with 8 sample
 * points per axis per cell; fully covered cells become gas, partly covered cells
 * interface cells with alpha = 1 - covered fraction. Liquid cells that then touch gas
 * become interface cells with alpha = 1. The initial gas mass is p0 V / RT (Eq.
 * idealgas). Pinned by the voxel-volume test. */
int or_nucleate(void *h, int nn, const double *centers, const double *radii, const double *p0) {
  OS *s = h;
  int64_t N = s->N, n;
  int k, i;
  if (nn + 1 > s->cap) return fail(s, "too many nuclei for the bubble table");
  double *phi = calloc(N, sizeof(double));
  int32_t *who = malloc(N * sizeof(int32_t));
  for (n = 0; n < N; n++) who[n] = -1;
  int S = 8, S3 = s->D == 3 ? 512 : 64;
  for (k = 0; k < nn; k++) {
    double cx = centers[3 * k], cy = centers[3 * k + 1], cz = s->D == 3 ? centers[3 * k + 2] : 0.0;
    double r = radii[k];
    for (n = 0; n < N; n++) {
      if (s->T[n] != TL) continue;
      int x, y, z;
      coords(s, n, &x, &y, &z);
      if (fabs((double)x - cx) > r + 1.0 || fabs((double)y - cy) > r + 1.0) continue;
      if (s->D == 3 && fabs((double)z - cz) > r + 1.0) continue;
      int cnt = 0, a, b, c, czn = s->D == 3 ? S : 1;
      for (c = 0; c < czn; c++)
        for (b = 0; b < S; b++)
          for (a = 0; a < S; a++) {
            double px = (double)x + (double)(2 * a - 7) / 16.0;
            double py = (double)y + (double)(2 * b - 7) / 16.0;
            double pz = s->D == 3 ? (double)z + (double)(2 * c - 7) / 16.0 : 0.0;
            double dx = px - cx, dy = py - cy, dz = pz - cz;
            if (((dx * dx + dy * dy) + dz * dz) < r * r) cnt++;
          }
      double f = (double)cnt / (double)S3;
      if (f > phi[n]) {
        phi[n] = f;
        who[n] = k;
      }
    }
  }
  for (n = 0; n < N; n++) {
    if (who[n] < 0) continue;
    if (phi[n] >= 1.0) {
      s->T[n] = TG;
      s->alpha[n] = 0.0;
      s->M[n] = 0.0;
    } else {
      s->T[n] = TI;
      s->alpha[n] = 1.0 - phi[n];
      s->M[n] = s->alpha[n];
    }
    s->label[n] = who[n] + 1;
  }
  /* invariant: no liquid cell touches gas */
  int32_t *nl = malloc(N * sizeof(int32_t));
  for (n = 0; n < N; n++) {
    nl[n] = NOLAB;
    if (s->T[n] != TL) continue;
    int32_t best = -1;
    for (i = 1; i < s->Q; i++) {
      int64_t y = nbr(s, n, i);
      if (y >= 0 && s->T[y] == TG && (best < 0 || s->label[y] < best)) best = s->label[y];
    }
    nl[n] = best;
  }
  for (n = 0; n < N; n++)
    if (nl[n] >= 0) {
      s->T[n] = TI;
      s->alpha[n] = 1.0;
      s->M[n] = 1.0;
      s->label[n] = nl[n];
    }
  for (n = 0; n < N; n++)
    if (s->T[n] == TI) {
      s->rho[n] = 1.0;
      s->ux[n] = s->uy[n] = s->uz[n] = 0.0;
    }
  free(nl);
  free(phi);
  free(who);
  for (k = 0; k < nn; k++) s->alive[k + 1] = 1;
  s->next_id = nn + 1;
  if (relabel(s, 0)) return -1;
  /* initial gas content from the nucleus pressure */
  for (i = 1; i < s->cap; i++)
    if (s->alive[i]) {
      s->bm[i] = (p0[i - 1] * s->bV[i]) / s->P.RT;
      s->bp[i] = (s->bm[i] * s->P.RT) / (s->bV[i] > 0.5 ? s->bV[i] : 0.5);
    }
  geometry(s);
  return 0;
}

/* ------------------------------------------------------------------- step --- */
static int step_once(OS *s) {
  int64_t N = s->N, n;
  int Q = s->Q, Qg = s->Qg, i;
  const or_params *P = &s->P;
  double *fn = malloc(sizeof(double) * N * Q);
  double *gn = malloc(sizeof(double) * N * Qg);
  double *Ms = malloc(sizeof(double) * N);
  uint8_t *cls = calloc(N, 1);
  memcpy(fn, s->fc, sizeof(double) * N * Q);
  memcpy(gn, s->gc, sizeof(double) * N * Qg);
  memcpy(Ms, s->M, sizeof(double) * N);
  memset(s->Phi, 0, sizeof(i128) * s->cap);
  memset(s->Gam, 0, sizeof(i128) * s->cap);
  double omega_newton = 1.0 / P->tau;

  /* S1-S5 */
  for (n = 0; n < N; n++) {
    uint8_t t = s->T[n];
    if (t != TL && t != TI) continue;
    double ft[19], gt[7], fe[19];
    double pb = 0.0, rg = 0.0, cH = 0.0;
    double uxo = s->ux[n], uyo = s->uy[n], uzo = s->uz[n];
    if (t == TI) {
      int lb = s->label[n];
      if (lb < 0 || lb >= s->cap || !s->alive[lb]) {
        free(fn); free(gn); free(Ms); free(cls);
        return fail(s, "interface cell with an invalid bubble id");
      }
      pb = s->bp[lb];
      rg = 3.0 * ((pb - 2.0 * P->sigma * s->kappa[n]) - s->Pi[n]);
      cH = P->kH * pb;
    }
    /* S1 */
    for (i = 0; i < Q; i++) {
      int64_t src = nbr(s, n, s->opp[i]); /* x - e_i */
      uint8_t ts = src < 0 ? TW : s->T[src];
      if (ts == TW)
        ft[i] = F(s, s->opp[i], n);
      else if (ts == TG) {
        if (t != TI) {
          free(fn); free(gn); free(Ms); free(cls);
          return fail(s, "liquid cell next to gas");
        }
        ft[i] = (feq(s, i, rg, uxo, uyo, uzo) + feq(s, s->opp[i], rg, uxo, uyo, uzo)) - F(s, s->opp[i], n);
      } else
        ft[i] = F(s, i, src);
    }
    /* S2 */
    if (t == TI) {
      double dm = 0.0;
      for (i = 1; i < Q; i++) {
        int64_t y = nbr(s, n, i);
        if (y < 0) continue;
        if (s->T[y] == TL)
          dm = dm + (ft[s->opp[i]] - F(s, i, n));
        else if (s->T[y] == TI)
          dm = dm + (0.5 * (s->alpha[n] + s->alpha[y])) * (ft[s->opp[i]] - F(s, i, n));
      }
      Ms[n] = s->M[n] + dm;
    }
    /* S3 */
    double phic = 0.0;
    int hasgas = 0;
    for (i = 0; i < Qg; i++) {
      int64_t src = nbr(s, n, s->opp[i]);
      uint8_t ts = src < 0 ? TW : s->T[src];
      if (ts == TW)
        gt[i] = G(s, s->opp[i], n);
      else if (ts == TG) {
        gt[i] = (geq(s, i, cH, uxo, uyo, uzo) + geq(s, s->opp[i], cH, uxo, uyo, uzo)) - G(s, s->opp[i], n);
        phic = phic + (G(s, s->opp[i], n) - gt[i]);
        hasgas = 1;
        if (s->label[src] != s->label[n]) {
          free(fn); free(gn); free(Ms); free(cls);
          return fail(s, "gas neighbour of an interface cell carries another bubble id");
        }
      } else
        gt[i] = G(s, i, src);
    }
    if (hasgas && P->flux_mode == 0) s->Phi[s->label[n]] += fx(phic);
    /* S4 */
    double rho, ux, uy, uz;
    moments(s, ft, &rho, &ux, &uy, &uz);
    if (s->force) {
      /* velocity of the forced scheme: (sum f e + F / 2) / rho with F = rho a */
      ux = ux + 0.5 * P->accel[0];
      uy = uy + 0.5 * P->accel[1];
      uz = uz + 0.5 * P->accel[2];
    }
    for (i = 0; i < Q; i++) fe[i] = feq(s, i, rho, ux, uy, uz);
    double omega = omega_newton;
    if (P->rheology == 1) omega = 1.0 / or_powerlaw_tau(P, rho, pineq_norm(s, ft, fe, rho, ux, uy, uz));
    if (P->rheology == 2) omega = 1.0 / or_cy_tau(P, rho, pineq_norm(s, ft, fe, rho, ux, uy, uz));
    for (i = 0; i < Q; i++) fn[(int64_t)i * N + n] = ft[i] - omega * (ft[i] - fe[i]);
    if (s->force)
      for (i = 0; i < Q; i++) fn[(int64_t)i * N + n] = fn[(int64_t)i * N + n] + (1.0 - 0.5 * omega) * force_i(s, i, rho, ux, uy, uz);
    double c = 0.0;
    for (i = 0; i < Qg; i++) c = c + gt[i];
    for (i = 0; i < Qg; i++)
      gn[(int64_t)i * N + n] = (gt[i] - s->omega_g * (gt[i] - geq(s, i, c, ux, uy, uz))) + s->wg[i] * P->q;
    if (t == TI && P->flux_mode == 1) {
      /* S3'. Eq. gascurrent as printed, with F read as the liquid and interface cells and
       * rho as 1: for every interface cell of bubble j, the populations its fluid
       * neighbours send towards it minus those it sends to them, less the advected part
       * c (alpha_new - alpha_old), with c the streamed concentration and alpha_new the
       * fill fraction after this step's mass exchange. Not conservative: the gas that
       * conversions move (S6 d, e) is not booked in this mode. */
      double pf = 0.0, cx = 0.0;
      for (i = 0; i < Qg; i++) cx = cx + gt[i];
      for (i = 1; i < Qg; i++) {
        int64_t y = nbr(s, n, i);
        if (y < 0) continue;
        if (s->T[y] == TL || s->T[y] == TI) pf = pf + (G(s, s->opp[i], y) - G(s, i, n));
      }
      pf = pf - cx * (Ms[n] / rho - s->alpha[n]);
      s->Phi[s->label[n]] += fx(pf);
    }
    if (t == TI) {
      s->rho[n] = rho;
      s->ux[n] = ux;
      s->uy[n] = uy;
      s->uz[n] = uz;
      /* S5: classification */
      if (Ms[n] > (1.0 + P->eps) * rho)
        cls[n] = CF;
      else if (Ms[n] < (-P->eps) * rho)
        cls[n] = CE;
      else if (P->cleanup) {
        int hasG = 0, hasF = 0;
        for (i = 1; i < Q; i++) {
          int64_t y = nbr(s, n, i);
          if (y < 0) continue;
          if (s->T[y] == TG) hasG = 1;
          if (s->T[y] == TL || s->T[y] == TI) hasF = 1;
        }
        if (!hasG)
          cls[n] = CF;
        else if (!hasF)
          cls[n] = CE;
      }
    }
  }
  memcpy(s->fc, fn, sizeof(double) * N * Q);
  memcpy(s->gc, gn, sizeof(double) * N * Qg);
  free(fn);
  free(gn);

  /* S6 (a): gas cells next to a filled cell become new interface cells; emptied
   * cells next to a filled cell stay interface cells */
  uint8_t *isNI = calloc(N, 1), *isL2I = calloc(N, 1), *Tn = malloc(N);
  for (n = 0; n < N; n++) {
    if (s->T[n] != TG) continue;
    for (i = 1; i < Q; i++) {
      int64_t y = nbr(s, n, i);
      if (y >= 0 && cls[y] == CF) isNI[n] = 1;
    }
  }
  for (n = 0; n < N; n++) {
    if (cls[n] != CE) continue;
    for (i = 1; i < Q; i++) {
      int64_t y = nbr(s, n, i);
      if (y >= 0 && cls[y] == CF) {
        cls[n] = 0;
        break;
      }
    }
  }
  /* S6 (b): liquid cells next to an emptied cell become interface cells */
  int32_t *l2ilab = malloc(N * sizeof(int32_t));
  for (n = 0; n < N; n++) {
    l2ilab[n] = NOLAB;
    if (s->T[n] != TL) continue;
    int32_t best = -1;
    for (i = 1; i < Q; i++) {
      int64_t y = nbr(s, n, i);
      if (y >= 0 && cls[y] == CE && (best < 0 || s->label[y] < best)) best = s->label[y];
    }
    if (best >= 0) {
      isL2I[n] = 1;
      l2ilab[n] = best;
    }
  }
  for (n = 0; n < N; n++)
    if (isL2I[n]) {
      double f[19], r, a, b, c;
      for (i = 0; i < Q; i++) f[i] = F(s, i, n);
      moments(s, f, &r, &a, &b, &c);
      s->rho[n] = r;
      s->ux[n] = a;
      s->uy[n] = b;
      s->uz[n] = c;
      Ms[n] = r;
      s->label[n] = l2ilab[n];
    }
  free(l2ilab);
  /* S6 (c): new types */
  for (n = 0; n < N; n++) {
    Tn[n] = s->T[n];
    if (cls[n] == CF) Tn[n] = TL;
    if (cls[n] == CE) Tn[n] = TG;
    if (isNI[n] || isL2I[n]) Tn[n] = TI;
  }
  /* S6 (d): new interface cells from gas take the mean state of their liquid and
   * old-interface neighbours; their dissolved gas comes out of the bubble */
  for (n = 0; n < N; n++) {
    if (!isNI[n]) continue;
    double sr = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
    int cnt = 0;
    for (i = 1; i < Q; i++) {
      int64_t y = nbr(s, n, i);
      if (y < 0 || isNI[y]) continue;
      if (Tn[y] != TL && Tn[y] != TI) continue;
      double f[19], r, a, b, c;
      int q;
      for (q = 0; q < Q; q++) f[q] = F(s, q, y);
      moments(s, f, &r, &a, &b, &c);
      sr = sr + r;
      sx = sx + a;
      sy = sy + b;
      sz = sz + c;
      cnt++;
    }
    double rb = 1.0, ubx = 0.0, uby = 0.0, ubz = 0.0;
    if (cnt > 0) {
      rb = sr / (double)cnt;
      ubx = sx / (double)cnt;
      uby = sy / (double)cnt;
      ubz = sz / (double)cnt;
    }
    for (i = 0; i < Q; i++) F(s, i, n) = feq(s, i, rb, ubx, uby, ubz);
    int lb = s->label[n];
    double cH = P->kH * s->bp[lb], sg = 0.0;
    for (i = 0; i < Qg; i++) {
      G(s, i, n) = geq(s, i, cH, ubx, uby, ubz);
      sg = sg + G(s, i, n);
    }
    if (P->flux_mode == 0) s->Gam[lb] -= fx(sg);
    s->rho[n] = rb;
    s->ux[n] = ubx;
    s->uy[n] = uby;
    s->uz[n] = ubz;
    Ms[n] = 0.0;
  }
  /* S6 (e): emptied cells hand their dissolved gas to their bubble */
  for (n = 0; n < N; n++) {
    if (cls[n] != CE) continue;
    double sg = 0.0;
    for (i = 0; i < Qg; i++) sg = sg + G(s, i, n);
    if (P->flux_mode == 0) s->Gam[s->label[n]] += fx(sg);
  }
  /* S7: excess mass of converted cells, split equally over their interface
   * neighbours under the new types */
  double *share = calloc(N, sizeof(double));
  uint8_t *hasShare = calloc(N, 1);
  for (n = 0; n < N; n++) {
    if (cls[n] != CF && cls[n] != CE) continue;
    double e = cls[n] == CF ? Ms[n] - s->rho[n] : Ms[n];
    int cnt = 0;
    for (i = 1; i < Q; i++) {
      int64_t y = nbr(s, n, i);
      if (y >= 0 && Tn[y] == TI) cnt++;
    }
    if (cnt > 0) {
      share[n] = e / (double)cnt;
      hasShare[n] = 1;
    } else {
      s->lost_liquid += fx(e);
    }
  }
  for (n = 0; n < N; n++) {
    if (Tn[n] != TI) continue;
    double acc = Ms[n];
    for (i = 1; i < Q; i++) {
      int64_t y = nbr(s, n, i);
      if (y >= 0 && hasShare[y]) acc = acc + share[y];
    }
    s->M[n] = acc;
    s->alpha[n] = acc / s->rho[n];
  }
  for (n = 0; n < N; n++) {
    if (cls[n] == CF) {
      s->M[n] = s->rho[n];
      s->alpha[n] = 1.0;
      s->label[n] = NOLAB;
    } else if (cls[n] == CE) {
      s->M[n] = 0.0;
      s->alpha[n] = 0.0;
    }
  }
  memcpy(s->T, Tn, N);
  free(share); free(hasShare); free(isNI); free(isL2I); free(Tn); free(cls); free(Ms);
  /* S8, S9 */
  if (relabel(s, 1)) return -1;
  /* S10, S11 */
  geometry(s);
  s->step++;
  return 0;
}

int or_step(void *h, int nsteps) {
  OS *s = h;
  int k;
  for (k = 0; k < nsteps; k++)
    if (step_once(s)) return -1;
  return 0;
}

/* ------------------------------------------------------------------ access --- */
enum { FLD_TYPE = 0, FLD_LABEL, FLD_RHO, FLD_UX, FLD_UY, FLD_UZ, FLD_ALPHA, FLD_MASS,
       FLD_CONC, FLD_KAPPA, FLD_PI, FLD_F, FLD_G };

int64_t or_ncells(void *h) { return ((OS *)h)->N; }

int or_read(void *h, int field, void *dst) {
  OS *s = h;
  int64_t n, N = s->N;
  int i;
  double *d = dst;
  switch (field) {
    case FLD_TYPE: memcpy(dst, s->T, N); return 0;
    case FLD_LABEL: memcpy(dst, s->label, N * 4); return 0;
    case FLD_RHO: memcpy(d, s->rho, N * 8); return 0;
    case FLD_UX: memcpy(d, s->ux, N * 8); return 0;
    case FLD_UY: memcpy(d, s->uy, N * 8); return 0;
    case FLD_UZ: memcpy(d, s->uz, N * 8); return 0;
    case FLD_ALPHA: memcpy(d, s->alpha, N * 8); return 0;
    case FLD_MASS: memcpy(d, s->M, N * 8); return 0;
    case FLD_CONC:
      for (n = 0; n < N; n++) {
        double c = 0.0;
        for (i = 0; i < s->Qg; i++) c = c + G(s, i, n);
        d[n] = c;
      }
      return 0;
    case FLD_KAPPA: memcpy(d, s->kappa, N * 8); return 0;
    case FLD_PI: memcpy(d, s->Pi, N * 8); return 0;
    case FLD_F: memcpy(d, s->fc, N * 8 * s->Q); return 0;
    case FLD_G: memcpy(d, s->gc, N * 8 * s->Qg); return 0;
  }
  return -1;
}

/* overwrite a field (hand-built test states) */
int or_write(void *h, int field, const void *src) {
  OS *s = h;
  int64_t N = s->N;
  switch (field) {
    case FLD_TYPE: memcpy(s->T, src, N); return 0;
    case FLD_LABEL: memcpy(s->label, src, N * 4); return 0;
    case FLD_RHO: memcpy(s->rho, src, N * 8); return 0;
    case FLD_UX: memcpy(s->ux, src, N * 8); return 0;
    case FLD_UY: memcpy(s->uy, src, N * 8); return 0;
    case FLD_UZ: memcpy(s->uz, src, N * 8); return 0;
    case FLD_ALPHA: memcpy(s->alpha, src, N * 8); return 0;
    case FLD_MASS: memcpy(s->M, src, N * 8); return 0;
    case FLD_KAPPA: memcpy(s->kappa, src, N * 8); return 0;
    case FLD_PI: memcpy(s->Pi, src, N * 8); return 0;
    case FLD_F: memcpy(s->fc, src, N * 8 * s->Q); return 0;
    case FLD_G: memcpy(s->gc, src, N * 8 * s->Qg); return 0;
  }
  return -1;
}

int or_set_bubble(void *h, int id, double m, double V, double p, int alive) {
  OS *s = h;
  if (id < 0 || id >= s->cap) return -1;
  s->bm[id] = m;
  s->bV[id] = V;
  s->bp[id] = p;
  s->alive[id] = (uint8_t)alive;
  if (id >= s->next_id) s->next_id = id + 1;
  return 0;
}

/* recompute curvature and disjoining pressure of the current state */
void or_geometry(void *h) { geometry((OS *)h); }

/* live bubbles in ascending id (id 0, the atmosphere, excluded) */
int or_bubbles(void *h, int capacity, int32_t *ids, double *m, double *V, double *p) {
  OS *s = h;
  int i, k = 0;
  for (i = 1; i < s->cap; i++)
    if (s->alive[i]) {
      if (k < capacity) {
        ids[k] = i;
        m[k] = s->bm[i];
        V[k] = s->bV[i];
        p[k] = s->bp[i];
      }
      k++;
    }
  return k;
}

/* lost_liquid, atm_gas, collapsed_gas, next_id, step */
void or_ledgers(void *h, double *out) {
  OS *s = h;
  out[0] = fxd(s->lost_liquid);
  out[1] = fxd(s->atm_gas);
  out[2] = fxd(s->collapsed_gas);
  out[3] = (double)s->next_id;
  out[4] = (double)s->step;
}

/* exported pieces for unit pins */
double or_feq(void *h, int i, double rho, double ux, double uy, double uz) {
  return feq((OS *)h, i, rho, ux, uy, uz);
}
double or_geq(void *h, int i, double c, double ux, double uy, double uz) {
  return geq((OS *)h, i, c, ux, uy, uz);
}
double or_curvature(void *h, int64_t n) { return or_curvature_at((OS *)h, n); }
double or_disjoining(void *h, int64_t n) { return or_disjoining_at((OS *)h, n); }
int or_lattice(void *h, int32_t *e, double *w, double *wg, int32_t *opp) {
  OS *s = h;
  int i;
  for (i = 0; i < s->Q; i++) {
    e[3 * i] = s->ex[i];
    e[3 * i + 1] = s->ey[i];
    e[3 * i + 2] = s->ez[i];
    w[i] = s->w[i];
    opp[i] = s->opp[i];
  }
  for (i = 0; i < s->Qg; i++) wg[i] = s->wg[i];
  return s->Q;
}

/* S8 + S9 alone on the current state with no flux (labelling tests) */
int or_relabel(void *h) { return relabel((OS *)h, 0); }

/* cells visited by the traversal of S11 from the origin along m: offsets into out
 * (3 ints per cell), at most dmax cells */
int or_traverse(int dim, double mx, double my, double mz, int dmax, int32_t *out) {
  double m[3] = {mx, my, mz}, bmax[3], bdel[3];
  int step[3], k, it, pos[3] = {0, 0, 0};
  for (k = 0; k < 3; k++) {
    if (k >= dim) { bmax[k] = INFINITY; bdel[k] = INFINITY; step[k] = 1; continue; }
    bmax[k] = fabs(0.5 / m[k]);
    bdel[k] = fabs(1.0 / m[k]);
    step[k] = m[k] >= 0.0 ? 1 : -1;
  }
  for (it = 0; it < dmax; it++) {
    double bmin = bmax[0];
    if (bmax[1] < bmin) bmin = bmax[1];
    if (bmax[2] < bmin) bmin = bmax[2];
    for (k = 0; k < dim; k++)
      if (bmax[k] == bmin) { bmax[k] = bmax[k] + bdel[k]; pos[k] += step[k]; }
    out[3 * it] = pos[0];
    out[3 * it + 1] = pos[1];
    out[3 * it + 2] = pos[2];
  }
  return dmax;
}

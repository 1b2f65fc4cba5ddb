// Pointwise lattice Boltzmann arithmetic shared by the library kernels. Every sum and
// product is written in one fixed order so that the binary64 instantiation reproduces
// the same roundings wherever the method prescribes the same formula.
#pragma once
#include "mf_internal.h"

namespace mf {

// e_i . u with only the non-zero velocity components (two-term sums are exact in
// either order, so this equals the full three-term dot product up to the sign of zero)
template <int D, class R>
__device__ __forceinline__ R edot(int i, R ux, R uy, R uz) {
  using L = Lat<D>;
  R acc = R(0);
  bool any = false;
  if (L::ex[i] != 0) { acc = L::ex[i] > 0 ? ux : -ux; any = true; }
  if (L::ey[i] != 0) { R t = L::ey[i] > 0 ? uy : -uy; acc = any ? acc + t : t; any = true; }
  if (D == 3 && L::ez[i] != 0) { R t = L::ez[i] > 0 ? uz : -uz; acc = any ? acc + t : t; any = true; }
  return acc;
}

template <int D, class R>
__device__ __forceinline__ R usq(R ux, R uy, R uz) {
  if constexpr (D == 3) return (ux * ux + uy * uy) + uz * uz;
  else return ux * ux + uy * uy;
}

// Eq. equilibrium with c_s^2 = 1/3
template <int D, class R>
__device__ __forceinline__ R feq(int i, R rho, R ux, R uy, R uz, R uu) {
  R eu = edot<D, R>(i, ux, uy, uz);
  return (rho * R(Lat<D>::w[i])) * (((R(1) + R(3) * eu) + (R(4.5) * eu) * eu) - R(1.5) * uu);
}

// ADE equilibrium (Sec. 3.1): w_i c (1 + e.u / c_s^2)
template <int D, class R>
__device__ __forceinline__ R geq(int i, R c, R ux, R uy, R uz) {
  R eu = edot<D, R>(i, ux, uy, uz);
  return (R(Lat<D>::wg[i]) * c) * (R(1) + R(Lat<D>::kg) * eu);
}

// zeroth and first moments of a population vector, sums in ascending direction order
template <int D, class R>
__device__ __forceinline__ void sums(const R *f, R &r_out, R &jx_out, R &jy_out, R &jz_out) {
  using L = Lat<D>;
  R r = f[0], jx = R(0), jy = R(0), jz = R(0);
#pragma unroll
  for (int i = 1; i < L::Q; ++i) r = r + f[i];
#pragma unroll
  for (int i = 1; i < L::Q; ++i) {
    if (L::ex[i] == 1) jx = jx + f[i];
    if (L::ex[i] == -1) jx = jx - f[i];
  }
#pragma unroll
  for (int i = 1; i < L::Q; ++i) {
    if (L::ey[i] == 1) jy = jy + f[i];
    if (L::ey[i] == -1) jy = jy - f[i];
  }
  if constexpr (D == 3) {
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
      if (L::ez[i] == 1) jz = jz + f[i];
      if (L::ez[i] == -1) jz = jz - f[i];
    }
  }
  r_out = r;
  jx_out = jx;
  jy_out = jy;
  jz_out = jz;
}

// density and velocity of a population vector
template <int D, class R>
__device__ __forceinline__ void moments(const R *f, R &rho, R &ux, R &uy, R &uz) {
  R r, jx, jy, jz;
  sums<D, R>(f, r, jx, jy, jz);
  rho = r;
  ux = jx / r;
  uy = jy / r;
  uz = D == 3 ? jz / r : R(0);
}

// Equilibria and moments in the register convention of instance P: plain values for
// P = 0, offsets from the rest state (f - w_i, g - w_i c0) otherwise. drho = rho - 1 and
// dc = c - c0 are the offsets of density and concentration.
template <int D, int P> struct Arith {
  using R = typename Prec<P>::R;
  static constexpr bool SH = P != 0;
  static __device__ __forceinline__ R eq(int i, R rho, R drho, R ux, R uy, R uz, R uu) {
    if constexpr (!SH) {
      return feq<D, R>(i, rho, ux, uy, uz, uu);
    } else {
      const R eu = edot<D, R>(i, ux, uy, uz);
      const R pol = (R(3) * eu + (R(4.5) * eu) * eu) - R(1.5) * uu;
      return R(Lat<D>::w[i]) * drho + (rho * R(Lat<D>::w[i])) * pol;
    }
  }
  static __device__ __forceinline__ R geqv(int i, R c, R dc, R ux, R uy, R uz) {
    if constexpr (!SH) {
      return geq<D, R>(i, c, ux, uy, uz);
    } else {
      const R eu = edot<D, R>(i, ux, uy, uz);
      return R(Lat<D>::wg[i]) * dc + (R(Lat<D>::wg[i]) * c) * (R(Lat<D>::kg) * eu);
    }
  }
  // density (and its offset) and velocity of a population vector in this convention
  // (sum w_i = 1 and sum w_i e_i = 0, so on offsets the sums give rho - 1 and rho u)
  static __device__ __forceinline__ void mom(const R *f, R &rho, R &drho, R &ux, R &uy, R &uz) {
    if constexpr (!SH) {
      moments<D, R>(f, rho, ux, uy, uz);
      drho = rho - R(1);
    } else {
      R s, jx, jy, jz;
      sums<D, R>(f, s, jx, jy, jz);
      drho = s;
      rho = R(1) + s;
      ux = jx / rho;
      uy = jy / rho;
      uz = D == 3 ? jz / rho : R(0);
    }
  }
  // concentration of a cell from its ADE populations
  static __device__ __forceinline__ R conc(const R *g, R c0, R &dc) {
    R s = g[0];
#pragma unroll
    for (int i = 1; i < Lat<D>::Qg; ++i) s = s + g[i];
    if constexpr (SH) { dc = s; return c0 + s; }
    else { dc = s - c0; return s; }
  }
};

__device__ __forceinline__ double dlog(double v) { return log(v); }
__device__ __forceinline__ float dlog(float v) { return logf(v); }
__device__ __forceinline__ double dexp(double v) { return exp(v); }
__device__ __forceinline__ float dexp(float v) { return expf(v); }

// Power-law relaxation time (Eq. tau with the power-law limit of Eq. carreauTau): the
// root of s = A (s + 1/2)^(1-n), s = tau - 1/2, by four Newton steps on t = ln s from
// ln(3 nu_ref), clamped to [tau_min, tau_max]; pn = |Pi_neq| (Frobenius norm).
template <class R>
__device__ __forceinline__ R powerlaw_tau(const KP &p, R rho, R pn) {
  R n = R(p.pl_n);
  R tau;
  if (!(pn > R(0))) {
    tau = n < R(1) ? R(p.tau_max) : (n > R(1) ? R(p.tau_min) : R(0.5) + R(3) * R(p.pl_nu_ref));
  } else {
    R l3 = dlog(R(3) * R(p.pl_nu_ref));
    R lnA = l3 + (n - R(1)) * dlog((R(2.1213203435596424) * pn) / (rho * R(p.pl_gdot_ref)));
    R t = l3;
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      R et = dexp(t);
      R Fv = (t - (R(1) - n) * dlog(et + R(0.5))) - lnA;
      R dF = R(1) - ((R(1) - n) * et) / (et + R(0.5));
      t = t - Fv / dF;
    }
    tau = R(0.5) + dexp(t);
  }
  if (tau < R(p.tau_min)) tau = R(p.tau_min);
  if (tau > R(p.tau_max)) tau = R(p.tau_max);
  return tau;
}

// Carreau-Yasuda relaxation time (Eq. carreauTau in full): the root in [tau_inf, tau0] of
// G(tau) = tau - tau_inf - (tau0 - tau_inf)(1 + (lambda K pn / (rho tau))^a)^((n-1)/a),
// K = 3/sqrt 2, unique under the parameter bounds the library enforces (h' < 1). Newton's
// method from tau0 with the bracket kept up to date (closed: a converged iterate is one of
// its ends) and a bisection step whenever Newton leaves it; binary64 iterates until the
// step no longer changes tau (at most 60 steps).
// h'(tau) = (tau0 - tau_inf)(1 - n) y (1 + y)^(m-1) / tau with y = x^a, m = (n-1)/a.
__device__ __forceinline__ double cy_tau64(const KP &p, double rho, double pn) {
  const double t0 = p.cy_tau0, ti = p.cy_tau_inf;
  if (!(pn > 0.0) || p.cy_lambda == 0.0 || t0 == ti) return t0;
  const double c = (p.cy_lambda * (2.1213203435596424 * pn)) / rho;  // lambda gdot tau
  const double m = (p.cy_n - 1.0) / p.cy_a, w = (t0 - ti) * (1.0 - p.cy_n);
  double lo = ti, hi = t0, t = t0;
  for (int it = 0; it < 60; ++it) {
    const double y = pow(c / t, p.cy_a);
    const double s = pow(1.0 + y, m);
    const double G = t - (ti + (t0 - ti) * s);
    if (G < 0.0) lo = t;
    else hi = t;
    if (G == 0.0) break;
    const double dh = (w * y) * s / ((1.0 + y) * t);
    double tn = t - G / (1.0 - dh);
    if (tn == t) break;  // converged (t is an end of the bracket then)
    if (!(tn >= lo && tn <= hi)) tn = 0.5 * (lo + hi);
    t = tn;
  }
  return t;
}

}  // namespace mf

// Lattice sweep: pull streaming from the SoA buffer of the previous step into the
// other buffer.
//
//  - streaming with bounce-back at walls (Sec. 2, Eqs. collisionstep, streamingstep);
//  - at interface cells, populations arriving from gas are rebuilt at the gas density
//    of the cell's bubble (Eq. reconstruct with Eqs. rhob, rhobplusdisjoining);
//  - interface mass exchange (Eq. massexchange, weights Theta);
//  - dissolved-gas streaming with the Henry's-law rebuild at interface cells
//    (Eqs. henryslaw, reconstructdiffusion) and the per-bubble gas ledger fed by the
//    populations exchanged with gas cells (the flux of Eq. gascurrent);
//  - moments, BGK collision (Eqs. collision, equilibrium) with Newtonian or power-law tau
//    (Eq. tau, Eq. carreauTau), ADE collision with source (Eq. diffusion);
//  - fill / empty classification of interface cells (Sec. 2.1).
//
// Two launch forms compute the same update:
//  * per cell (k_sweep): one thread per cell over the whole grid. Used for binary64,
//    for periodic axes and for rows whose length is not a multiple of the vector width;
//  * split (k_sweep_vec + k_sweep_special): the bulk kernel gives each thread VW
//    consecutive cells, so that every population plane is read and written with
//    aligned 8- or 16-byte accesses per lane (the one-cell shift of directions with an
//    x component is done across lanes); it updates every liquid cell, taking
//    bounce-back at walls from a static per-cell mask of wall directions. Interface
//    cells take the per-cell path in a second kernel over the interface list, so the
//    bulk kernel carries no divergent interface work (doing the interface cells in the
//    bulk kernel, in the same wave or on their own lanes, measured slower).
// The interface and bubble lists of the step are built before the sweep.
#pragma once
#include <utility>

#include "lbm_math.h"

namespace mf {

// Power-law relaxation time in binary32 (the same root as powerlaw_tau): Newton's
// method on u = log2(tau - 1/2), with the hardware base-2 exponential and logarithm. The
// root solves F(u) = u - m log2(2^u + 1/2) - la = 0 (m = 1 - n). F is increasing; since
// log2(2^u + 1/2) >= max(u, -1), la / n and la - m bound the root from below when n < 1
// (F concave: Newton's method from the larger bound stays below the root and closes on
// it) and from above when n > 1 (F convex: from the smaller bound, staying above). Over
// tau - 1/2 in [0.005, 2] the relative error of tau after three iterations is at most
// 2.6e-7 for n in [0.3, 3] (1.0e-7 at n = 0.6; from the fixed start log2(3 nu_ref) it was
// 2.5e-7 there and 2.6e-4 at n = 0.2); four reach that over [0.1, 3]. KP::pl_nit holds the
// count chosen on the host from n. (Two iterations, 2.3e-6 at n = 0.6, did not make the
// bulk kernel faster: it is not bound by its arithmetic.) The derivative
// 1 - m e / (e + 1/2) is used as (n e + 1/2) / (e + 1/2), one reciprocal per iteration.
__device__ __forceinline__ float powerlaw_tau_f32(const KP &p, float rinv, float pn) {
  const int nit = p.pl_nit;
  const float n = p.pl_n_f;
  float tau;
  if (!(pn > 0.0f)) {
    tau = n < 1.0f ? p.tau_max_f : (n > 1.0f ? p.tau_min_f : 0.5f + 3.0f * (float)p.pl_nu_ref);
  } else {
    const float l3 = p.pl_l2nu3;
    const float la = l3 + (n - 1.0f) * __builtin_amdgcn_logf((p.pl_kg * pn) * rinv);
    const float m = 1.0f - n;
    const float ua = la * p.pl_ninv, ub = la - m;
    float u = (ua > ub) == (n < 1.0f) ? ua : ub;
    for (int it = 0; it < nit; ++it) {
      const float e = __builtin_amdgcn_exp2f(u);
      const float eh = e + 0.5f;
      const float F = (u - m * __builtin_amdgcn_logf(eh)) - la;
      u = u - (F * eh) * __builtin_amdgcn_rcpf(n * e + 0.5f);
    }
    tau = 0.5f + __builtin_amdgcn_exp2f(u);
  }
  tau = tau < p.tau_min_f ? p.tau_min_f : tau;
  tau = tau > p.tau_max_f ? p.tau_max_f : tau;
  return tau;
}

// Carreau-Yasuda relaxation time in binary32 (the same root as cy_tau64): Newton's method
// from tau0 inside the bracket [tau_inf, tau0], with the hardware base-2 exponential and
// logarithm for the two powers and one reciprocal per step; a step that leaves the bracket
// bisects instead. From tau0 the iteration is at binary64 precision after four steps for
// lambda gdot tau from 1e-4 to 1e4 over the shear-thinning parameter range; five are taken.
// rinv = 1 / rho, pn = |Pi_neq|.
__device__ __forceinline__ float cy_tau_f32(const KP &p, float rinv, float pn) {
  const float t0 = p.cy_tau0_f, ti = p.cy_tau_inf_f;
  if (!(pn > 0.0f) || p.cy_lambda == 0.0 || t0 == ti) return t0;
  const float c = (p.cy_lk * pn) * rinv;  // lambda gdot tau
  const float a = p.cy_a_f, m = p.cy_m, w = p.cy_w_f;
  float lo = ti, hi = t0, t = t0;
#pragma unroll
  for (int it = 0; it < 5; ++it) {
    const float it_ = __builtin_amdgcn_rcpf(t);
    const float y = __builtin_amdgcn_exp2f(a * __builtin_amdgcn_logf(c * it_));
    const float s1 = 1.0f + y;
    const float sm = __builtin_amdgcn_exp2f(m * __builtin_amdgcn_logf(s1));
    const float G = t - (ti + (t0 - ti) * sm);
    lo = G < 0.0f ? t : lo;
    hi = G < 0.0f ? hi : t;
    const float dh = ((w * y) * sm) * (__builtin_amdgcn_rcpf(s1) * it_);
    float tn = t - G * __builtin_amdgcn_rcpf(1.0f - dh);
    tn = (tn >= lo && tn <= hi) ? tn : 0.5f * (lo + hi);  // closed: a converged iterate is an end
    t = tn;
  }
  return t;
}

// Force correction of the strain-rate estimate under a body force F = rho a: the
// non-equilibrium momentum flux that measures the strain rate is Pi_neq + (u F + F u)/2
// (in a uniformly accelerated box the populations carry Pi_neq = -(u F + F u)/2 and no
// strain).
template <int D, class R>
__device__ __forceinline__ void force_stress(R rho, R ux, R uy, R uz, R ax, R ay, R az, R &pxx, R &pyy, R &pzz,
                                             R &pxy, R &pxz, R &pyz) {
  const R Fx = rho * ax, Fy = rho * ay;
  pxx = pxx + ux * Fx;
  pyy = pyy + uy * Fy;
  pxy = pxy + R(0.5) * (ux * Fy + uy * Fx);
  if constexpr (D == 3) {
    const R Fz = rho * az;
    pzz = pzz + uz * Fz;
    pxz = pxz + R(0.5) * (ux * Fz + uz * Fx);
    pyz = pyz + R(0.5) * (uy * Fz + uz * Fy);
  }
}

// BGK collision of one cell on offsets in binary32 (instances 1-4). Directions come in
// opposite pairs (2k+1, 2k+2): the moments are taken from the pair sums s and
// differences d (density from s, momentum from d, the momentum flux from s, whose
// products e_a e_b are the same for both members), the density is inverted once, and the
// equilibria are built per pair (even part w (drho + rho (4.5 (e.u)^2 - 1.5 u.u)), odd
// part 3 w rho e.u).
// c0 and q are the reference concentration and the source in the units gt is held in.
// FRC: the domain has a body force (a compile-time switch, so that the unforced sweep
// keeps its register budget).
template <int D, bool FRC>
__device__ __forceinline__ void collide_f32(const KP &p, const DA &d, float *ft, float *gt, float &rho, float &ux,
                                            float &uy, float &uz, float c0, float q) {
  using L = Lat<D>;
  constexpr int Q = L::Q, Qg = L::Qg, NP = (Q - 1) / 2;
  float sp[NP], dp[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    sp[k] = ft[2 * k + 1] + ft[2 * k + 2];
    dp[k] = ft[2 * k + 1] - ft[2 * k + 2];
  }
  float s = ft[0], jx = 0.0f, jy = 0.0f, jz = 0.0f;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const int i = 2 * k + 1;
    s = s + sp[k];
    if (L::ex[i]) jx = L::ex[i] > 0 ? jx + dp[k] : jx - dp[k];
    if (L::ey[i]) jy = L::ey[i] > 0 ? jy + dp[k] : jy - dp[k];
    if (D == 3 && L::ez[i]) jz = L::ez[i] > 0 ? jz + dp[k] : jz - dp[k];
  }
  const float drho = s;
  rho = 1.0f + s;
  if (!(rho > 0.0f)) raise_status(d.status, ST_NONFINITE);
  const float ir = __builtin_amdgcn_rcpf(rho);
  ux = jx * ir;
  uy = jy * ir;
  uz = D == 3 ? jz * ir : 0.0f;
  // body force F = rho a (Guo et al.): the velocity is (sum f e + F/2) / rho
  constexpr bool frc = FRC;
  if constexpr (frc) {
    ux = ux + 0.5f * p.fax;
    uy = uy + 0.5f * p.fay;
    if (D == 3) uz = uz + 0.5f * p.faz;
  }
  const float uu = usq<D, float>(ux, uy, uz);
  float omega = p.omega_f;
  if (p.rheology != MF_NEWTONIAN) {
    // non-equilibrium momentum flux: sum e e (f - w) minus the equilibrium part
    // rho c_s^2 I + rho u u taken relative to the rest state (I/3)
    float pxx = 0, pyy = 0, pzz = 0, pxy = 0, pxz = 0, pyz = 0;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      const int i = 2 * k + 1;
      const int ex = L::ex[i], ey = L::ey[i], ez = L::ez[i];
      const float v = sp[k];
      if (ex) pxx = pxx + v;
      if (ey) pyy = pyy + v;
      if (D == 3 && ez) pzz = pzz + v;
      if (ex && ey) pxy = ex * ey > 0 ? pxy + v : pxy - v;
      if (D == 3 && ex && ez) pxz = ex * ez > 0 ? pxz + v : pxz - v;
      if (D == 3 && ey && ez) pyz = ey * ez > 0 ? pyz + v : pyz - v;
    }
    const float d3 = drho * (1.0f / 3.0f);
    pxx = pxx - (d3 + rho * ux * ux);
    pyy = pyy - (d3 + rho * uy * uy);
    pxy = pxy - rho * ux * uy;
    if (D == 3) {
      pzz = pzz - (d3 + rho * uz * uz);
      pxz = pxz - rho * ux * uz;
      pyz = pyz - rho * uy * uz;
    }
    if constexpr (frc) force_stress<D, float>(rho, ux, uy, uz, p.fax, p.fay, p.faz, pxx, pyy, pzz, pxy, pxz, pyz);
    const float ss = ((pxx * pxx + pyy * pyy) + pzz * pzz) + 2.0f * ((pxy * pxy + pxz * pxz) + pyz * pyz);
    const float pn = __builtin_amdgcn_sqrtf(ss);
    omega = __builtin_amdgcn_rcpf(p.rheology == MF_POWER_LAW ? powerlaw_tau_f32(p, ir, pn) : cy_tau_f32(p, ir, pn));
  }
  const float c15 = 1.5f * uu;
  if constexpr (!frc) {
    {
      const float w0 = (float)L::w[0];
      ft[0] = ft[0] - omega * (ft[0] - (w0 * drho - (w0 * rho) * c15));
    }
#pragma unroll
    for (int i = 1; i < Q; i += 2) {
      const float eu = edot<D, float>(i, ux, uy, uz);
      const float w = (float)L::w[i];
      const float wr = w * rho;
      const float ev = w * drho + wr * ((4.5f * eu) * eu - c15);
      const float od = wr * (3.0f * eu);
      ft[i] = ft[i] - omega * (ft[i] - (ev + od));
      ft[i + 1] = ft[i + 1] - omega * (ft[i + 1] - (ev - od));
    }
  } else {
    // force term (1 - omega/2) F_i, F_i = w rho [3 (e - u).a + 9 (e.u)(e.a)]: per pair the
    // even part w rho (9 (e.u)(e.a) - 3 u.a) and the odd part 3 w rho e.a
    const float kf = 1.0f - 0.5f * omega;
    const float ua = (ux * p.fax + uy * p.fay) + (D == 3 ? uz * p.faz : 0.0f);
    {
      const float w0 = (float)L::w[0];
      ft[0] = (ft[0] - omega * (ft[0] - (w0 * drho - (w0 * rho) * c15))) + kf * ((w0 * rho) * (-3.0f * ua));
    }
#pragma unroll
    for (int i = 1; i < Q; i += 2) {
      const float eu = edot<D, float>(i, ux, uy, uz);
      const float ea = edot<D, float>(i, p.fax, p.fay, p.faz);
      const float w = (float)L::w[i];
      const float wr = w * rho;
      const float ev = w * drho + wr * ((4.5f * eu) * eu - c15);
      const float od = wr * (3.0f * eu);
      const float evf = kf * (wr * ((9.0f * eu) * ea - 3.0f * ua));
      const float odf = kf * (wr * (3.0f * ea));
      ft[i] = (ft[i] - omega * (ft[i] - (ev + od))) + (evf + odf);
      ft[i + 1] = (ft[i + 1] - omega * (ft[i + 1] - (ev - od))) + (evf - odf);
    }
  }
  float dc = gt[0];
#pragma unroll
  for (int i = 1; i < Qg; ++i) dc = dc + gt[i];
  const float c = c0 + dc;
  const float og = p.omega_g_f;
  {
    const float wg = (float)L::wg[0];
    gt[0] = (gt[0] - og * (gt[0] - wg * dc)) + wg * q;
  }
#pragma unroll
  for (int i = 1; i < Qg; i += 2) {
    const float eu = edot<D, float>(i, ux, uy, uz);
    const float wg = (float)L::wg[i];
    const float ev = wg * dc;
    const float od = (wg * c) * ((float)L::kg * eu);
    gt[i] = (gt[i] - og * (gt[i] - (ev + od))) + wg * q;
    gt[i + 1] = (gt[i + 1] - og * (gt[i + 1] - (ev - od))) + wg * q;
  }
}

// BGK collision of one cell in the register convention of instance P (fluid and ADE
// lattices); ft and gt are replaced by their post-collision values. FRC: body force.
template <int D, int P, bool FRC>
__device__ __forceinline__ void collide_cell(const KP &p, const DA &d, typename Prec<P>::R *ft,
                                             typename Prec<P>::R *gt, typename Prec<P>::R &rho,
                                             typename Prec<P>::R &ux, typename Prec<P>::R &uy,
                                             typename Prec<P>::R &uz) {
  if constexpr (P != 0) {
    collide_f32<D, FRC>(p, d, ft, gt, rho, ux, uy, uz, p.c0_f, p.q_f);
    return;
  }
  using L = Lat<D>;
  using R = typename Prec<P>::R;
  using A = Arith<D, P>;
  constexpr int Q = L::Q, Qg = L::Qg;
  R drho;
  A::mom(ft, rho, drho, ux, uy, uz);
  if (!(rho > R(0))) raise_status(d.status, ST_NONFINITE);
  if constexpr (FRC) {
    // body force F = rho a (Guo et al.): the velocity is (sum f e + F/2) / rho
    ux = ux + R(0.5) * R(p.ax);
    uy = uy + R(0.5) * R(p.ay);
    if (D == 3) uz = uz + R(0.5) * R(p.az);
  }
  const R uu = usq<D, R>(ux, uy, uz);
  R omega = R(p.omega);
  if (p.rheology != MF_NEWTONIAN) {
    R pxx = 0, pyy = 0, pzz = 0, pxy = 0, pxz = 0, pyz = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      // binary64: sum e e (f - f_eq) term by term; offset instances: sum e e (f - w),
      // the equilibrium part is removed in closed form below
      const R dd = P == 0 ? ft[i] - A::eq(i, rho, drho, ux, uy, uz, uu) : ft[i];
      const int ex = L::ex[i], ey = L::ey[i], ez = L::ez[i];
      if (ex) pxx = pxx + dd;
      if (ey) pyy = pyy + dd;
      if (D == 3 && ez) pzz = pzz + dd;
      if (ex && ey) pxy = pxy + R(ex * ey) * dd;
      if (D == 3 && ex && ez) pxz = pxz + R(ex * ez) * dd;
      if (D == 3 && ey && ez) pyz = pyz + R(ey * ez) * dd;
    }
    if constexpr (P != 0) {
      // second moment of the equilibrium: rho c_s^2 I + rho u u; on offsets the rest
      // state contributes I/3, so subtract drho/3 on the diagonal
      const R d3 = drho * R(1.0 / 3.0);
      pxx = pxx - (d3 + rho * ux * ux);
      pyy = pyy - (d3 + rho * uy * uy);
      pxy = pxy - rho * ux * uy;
      if (D == 3) {
        pzz = pzz - (d3 + rho * uz * uz);
        pxz = pxz - rho * ux * uz;
        pyz = pyz - rho * uy * uz;
      }
    }
    if constexpr (FRC) force_stress<D, R>(rho, ux, uy, uz, R(p.ax), R(p.ay), R(p.az), pxx, pyy, pzz, pxy, pxz, pyz);
    const R ss = ((pxx * pxx + pyy * pyy) + pzz * pzz) + R(2) * ((pxy * pxy + pxz * pxz) + pyz * pyz);
    if constexpr (P == 0) omega = R(1) / (p.rheology == MF_POWER_LAW ? powerlaw_tau<R>(p, rho, sqrt(ss)) : cy_tau64(p, rho, sqrt(ss)));
    else omega = R(1) / powerlaw_tau<R>(p, rho, sqrt(ss));
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const R fe = A::eq(i, rho, drho, ux, uy, uz, uu);
    ft[i] = ft[i] - omega * (ft[i] - fe);
  }
  if constexpr (FRC) {
    const R kf = R(1) - R(0.5) * omega;
    const R ax = R(p.ax), ay = R(p.ay), az = R(p.az);
    const R ua = (ux * ax + uy * ay) + (D == 3 ? uz * az : R(0));
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const R eu = edot<D, R>(i, ux, uy, uz);
      const R ea = edot<D, R>(i, ax, ay, az);
      ft[i] = ft[i] + kf * ((rho * R(L::w[i])) * (R(3) * (ea - ua) + (R(9) * eu) * ea));
    }
  }
  R dc;
  const R c = A::conc(gt, R(p.c0), dc);
  const R og = R(p.omega_g), q = R(p.q);
#pragma unroll
  for (int i = 0; i < Qg; ++i) gt[i] = (gt[i] - og * (gt[i] - A::geqv(i, c, dc, ux, uy, uz))) + R(Lat<D>::wg[i]) * q;
}

// The part of the update of an interface cell or a cell next to a wall that needs the
// cell's own populations and the types of its sources: bounce-back, gas-side rebuild at
// the bubble pressure (fluid and dissolved gas, with the gas ledger), and for interface
// cells the mass exchange. ft / gt hold the pulled populations on entry. src(i) is the
// index of the source x - e_i, dst(i) that of the neighbour x + e_i.
template <int D, int P, class Src, class Dst>
__device__ __forceinline__ void special_terms(const KP &p, DA &d, int cur, int64_t n, bool isI, int32_t lab,
                                              Src src, Dst dst, typename Prec<P>::R *ft, typename Prec<P>::R *gt,
                                              typename Prec<P>::R &Ms, bool &hasG, bool &hasF,
                                              typename Prec<P>::R &phic, bool &hasgas,
                                              typename Prec<P>::R &pf, typename Prec<P>::R &aold) {
  using L = Lat<D>;
  using R = typename Prec<P>::R;
  using SF = typename Prec<P>::SF;
  using SG = typename Prec<P>::SG;
  using FC = FCodec<P, D>;
  using GC = GCodec<P>;
  using A = Arith<D, P>;
  constexpr int Q = L::Q, Qg = L::Qg;
  const SF *fin = (const SF *)d.f[cur];
  const SG *gin = (const SG *)d.g[cur];
  const int64_t Np = p.Np;
  R own[Q], gown[Qg];
  uint8_t tsrc[Q];
  // the cell's own outgoing populations and the types of its sources, all loads issued
  // together
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    own[i] = FC::dec(fin[(int64_t)i * Np + n], i);
    if (i < Qg) gown[i] = GC::dec(gin[(int64_t)i * Np + n], p);
    tsrc[i] = d.type[src(i)] & TMASK;
  }
  R rg = R(1), uox = R(0), uoy = R(0), uoz = R(0), uou = R(0), cH = R(0), dcH = R(0), ax = R(0), Mo = R(0);
  R ay[Q];
  if (isI) {
    // everything an interface cell reads is addressed by its index alone: the loads are
    // issued together (fill fractions of all neighbours, used where they are interface)
    rg = ((const R *)d.rgas)[n];
    cH = R(p.kH) * ((const R *)d.pbub)[n];
    dcH = cH - R(p.c0);
    uox = ((const R *)d.ux)[n];
    uoy = ((const R *)d.uy)[n];
    uoz = D == 3 ? ((const R *)d.uz)[n] : R(0);
    uou = usq<D, R>(uox, uoy, uoz);
    ax = ((const R *)d.alpha)[n];
    Mo = ((const R *)d.M)[n];
#pragma unroll
    for (int i = 1; i < Q; ++i) ay[i] = ((const R *)d.alpha)[dst(i)];
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (i > 0 && tsrc[i] == TG) hasG = true;
    if (i > 0 && (tsrc[i] == TL || tsrc[i] == TI)) hasF = true;
    if (tsrc[i] == TW) {
      ft[i] = own[opp(i)];
    } else if (tsrc[i] == TG) {
      if (!isI) raise_status(d.status, ST_INVARIANT);
      ft[i] = (A::eq(i, rg, rg - R(1), uox, uoy, uoz, uou) + A::eq(opp(i), rg, rg - R(1), uox, uoy, uoz, uou)) -
              own[opp(i)];
    }
  }
#pragma unroll
  for (int i = 0; i < Qg; ++i) {
    if (tsrc[i] == TW) {
      gt[i] = gown[opp(i)];
    } else if (tsrc[i] == TG) {
      gt[i] = (A::geqv(i, cH, dcH, uox, uoy, uoz) + A::geqv(opp(i), cH, dcH, uox, uoy, uoz)) - gown[opp(i)];
      phic = phic + (gown[opp(i)] - gt[i]);
      hasgas = true;
    }
  }
  if (isI) {
    // interface mass exchange with liquid and interface neighbours y = x + e_i
    R dm = R(0);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const int tn = tsrc[opp(i)];
      if (tn == TL) {
        dm = dm + (ft[opp(i)] - own[i]);
      } else if (tn == TI) {
        dm = dm + (R(0.5) * (ax + ay[i])) * (ft[opp(i)] - own[i]);
      }
    }
    Ms = Mo + dm;
    if (p.flux_paper) {
      // Eq. gascurrent as printed: what the liquid and interface neighbours y = x + e_i
      // send towards the cell minus what it sends to them
      R s = R(0);
#pragma unroll
      for (int i = 1; i < Qg; ++i) {
        const int tn = tsrc[opp(i)];
        if (tn == TL || tn == TI) s = s + (gt[opp(i)] - gown[i]);
      }
      pf = s;
      aold = ax;
    }
  }
}

// what an interface cell stores besides its populations: density, velocity, mass and
// its fill / empty class (Sec. 2.1)
template <int D, class R>
__device__ __forceinline__ uint8_t store_interface(const KP &p, DA &d, int64_t n, R rho, R ux, R uy, R uz, R Ms,
                                                   bool hasG, bool hasF) {
  ((R *)d.rho)[n] = rho;
  ((R *)d.ux)[n] = ux;
  ((R *)d.uy)[n] = uy;
  if (D == 3) ((R *)d.uz)[n] = uz;
  ((R *)d.M)[n] = Ms;
  uint8_t cl = 0;
  if (Ms > (R(1) + R(p.eps)) * rho) cl = CF_FILL;
  else if (Ms < (-R(p.eps)) * rho) cl = CF_EMPTY;
  else if (p.cleanup) {
    if (!hasG) cl = CF_FILL;
    else if (!hasF) cl = CF_EMPTY;
  }
  d.cflag[n] = cl;
  return cl;
}

// index offset of the lattice neighbour x + e_i on a grid without periodic wrap
template <int D>
__device__ __forceinline__ int64_t dir_offset(const KP &p, int i) {
  return (int64_t)Lat<D>::ex[i] + (int64_t)p.nx * ((int64_t)Lat<D>::ey[i] + (D == 3 ? (int64_t)p.ny * Lat<D>::ez[i] : 0));
}

// The whole update of one cell (x, y, z) = n with type byte tb and bubble id lab; lanes
// with fluid == false only take part in the wave-level gas-ledger sum. Called by the
// whole wave. CLOSED: the grid has no periodic axis and the cell is not on its outer
// layer, so neighbours are plain index offsets (x, y, z are not used).
template <int D, int P, bool FRC, bool CLOSED = false>
__device__ __forceinline__ void sweep_cell(const KP &p, DA &d, int cur, bool fluid, int x, int y, int z, int64_t n,
                                           uint8_t tb, int32_t lab) {
  using L = Lat<D>;
  using R = typename Prec<P>::R;
  using SF = typename Prec<P>::SF;
  using SG = typename Prec<P>::SG;
  using FC = FCodec<P, D>;
  using GC = GCodec<P>;
  constexpr int Q = L::Q, Qg = L::Qg;
  const int t = tb & TMASK;
  const bool isI = fluid && t == TI;
  bool hasgas = false, conv = false;
  R phic = R(0);

  if (fluid) {
    const SF *fin = (const SF *)d.f[cur];
    SF *fout = (SF *)d.f[cur ^ 1];
    const SG *gin = (const SG *)d.g[cur];
    SG *gout = (SG *)d.g[cur ^ 1];
    const int64_t Np = p.Np;
    R ft[Q], gt[Qg];
    auto src = [&](int i) {
      if constexpr (CLOSED) return n - dir_offset<D>(p, i);
      else return nb_index(p, x, y, z, -L::ex[i], -L::ey[i], -L::ez[i]);
    };
    auto dst = [&](int i) {
      if constexpr (CLOSED) return n + dir_offset<D>(p, i);
      else return nb_index(p, x, y, z, L::ex[i], L::ey[i], L::ez[i]);
    };
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int64_t s = src(i);
      ft[i] = FC::dec(fin[(int64_t)i * Np + s], i);
      if (i < Qg) gt[i] = GC::dec(gin[(int64_t)i * Np + s], p);
    }
    R Ms = R(0), pf = R(0), aold = R(0), cx = R(0);
    bool hasG = false, hasF = false;
    if (isI || (tb & NEARWALL)) {
      special_terms<D, P>(p, d, cur, n, isI, lab, src, dst, ft, gt, Ms, hasG, hasF, phic, hasgas, pf, aold);
    }
    if (isI && p.flux_paper) {
      // streamed concentration (the offset form holds c - c0)
      cx = P != 0 ? R(p.c0) : R(0);
#pragma unroll
      for (int i = 0; i < Qg; ++i) cx = cx + gt[i];
    }
    R rho, ux, uy, uz;
    collide_cell<D, P, FRC>(p, d, ft, gt, rho, ux, uy, uz);
    if (isI && p.flux_paper) {
      // less the advected part c (alpha_new - alpha_old); every interface cell books it
      phic = pf - cx * (Ms / rho - aold);
      hasgas = true;
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) fout[(int64_t)i * Np + n] = FC::enc(ft[i], i);
#pragma unroll
    for (int i = 0; i < Qg; ++i) gout[(int64_t)i * Np + n] = GC::enc(gt[i], p);
    if (isI) conv = (store_interface<D, R>(p, d, n, rho, ux, uy, uz, Ms, hasG, hasF) & (CF_FILL | CF_EMPTY)) != 0;
  }
  // the cells that fill or empty, listed for the conversion kernels
  const int slot = wave_append_slot(d.cnt + C_CONV, conv);
  if (conv) d.clist[slot] = (int32_t)n;
  wave_fx_add_runs(d.phi, hasgas && lab >= 0 && lab < p.cap, lab, fx3((double)phic), d.phi0);
}

// block index remapped so that consecutive tiles go to the same XCD (of 8): the
// hardware deals blocks round-robin over the XCDs, each with its own L2
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
  const int64_t per = nb >> 3;
  return b < (per << 3) ? (b & 7) * per + (b >> 3) : b;
}

// ------------------------------------------------------------------ per-cell form
template <int D, int P, bool FRC>
__device__ __forceinline__ void b_sweep(const GridPos &gp, KP p, DA d, int cur) {
  // tile of 64 x 4 cells
  const int gx = (p.nx + 63) >> 6, gy = (p.ny + 3) >> 2;
  const int64_t nb = (int64_t)gx * gy * p.nz;
  const int64_t b = xcd_block(gp.bid, nb);
  const int bx = (int)(b % gx);
  const int64_t rr = b / gx;
  const int by = (int)(rr % gy);
  const int z = (int)(rr / gy);
  const int x = (bx << 6) + (threadIdx.x & 63);
  const int y = (by << 2) + (threadIdx.x >> 6);
  const bool in = x < p.nx && y < p.ny && z < p.nz;
  const int64_t n = in ? (int64_t)x + (int64_t)p.nx * ((int64_t)y + (int64_t)p.ny * z) : 0;
  const uint8_t tb = in ? d.type[n] : TW;
  const int t = tb & TMASK;
  const int32_t lab = in && t == TI ? d.label[n] : NOLAB;
  sweep_cell<D, P, FRC>(p, d, cur, in && (t == TL || t == TI), x, y, z, n, tb, lab);
}
template <int D, int P, bool FRC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_sweep(KP p, DA d, int cur) {
  b_sweep<D, P, FRC>(GridPos::hw(), p, d, cur);
}

// ------------------------------------------------------------------ split form
// interface cells (this step's interface list) through the per-cell update
template <int D, int P, bool FRC>
__device__ __forceinline__ void b_sweep_special(const GridPos &gp, KP p, DA d, int cur) {
  LIST_LOOP(k, d.cnt + C_I) {
    int64_t n = 0;
    uint8_t tb = TW;
    bool fluid = false;
    int32_t lab = NOLAB;
    if (k < *(volatile int32_t *)(d.cnt + C_I)) {
      n = d.ilist[k];
      tb = TI;  // the near-wall bit only matters for liquid cells
      fluid = true;
      lab = d.label[n];
    }
    // the domains this kernel serves have closed axes, and interface cells never lie on
    // the outer (wall) layer
    sweep_cell<D, P, FRC, true>(p, d, cur, fluid, 0, 0, 0, n, tb, lab);
  }
}
template <int D, int P, bool FRC>
__global__ __launch_bounds__(256) void k_sweep_special(KP p, DA d, int cur) {
  b_sweep_special<D, P, FRC>(GridPos::hw(), p, d, cur);
}

template <class T> __device__ __forceinline__ uint32_t lane_bits(T v) {
  if constexpr (sizeof(T) == 4) return __builtin_bit_cast(uint32_t, v);
  else return (uint32_t)__builtin_bit_cast(uint16_t, v);
}
template <class T> __device__ __forceinline__ T from_lane_bits(uint32_t u) {
  if constexpr (sizeof(T) == 4) return __builtin_bit_cast(T, u);
  else return __builtin_bit_cast(T, (uint16_t)u);
}

// One aligned VW-wide load of plane `plane` for the cell group of this lane, shifted by
// the x component ex of the direction: element j of the result is the value at
// n0 + j - ex - off. The element that crosses into the neighbouring lane's group comes
// from that lane; a lane whose neighbour has no valid group (or the first / last lane
// of the wave) loads it itself, with the index clamped into the plane (such a value
// only ever feeds a wall cell).
template <class T, int VW> using Vec = T __attribute__((ext_vector_type(VW)));

// directions whose source lies on the side sx of the cell along x (ex = sx): the wall
// pattern of a cell next to the low (sx = 1) or high (sx = -1) x wall of the box
template <int D> constexpr uint32_t xwall_mask(int sx) {
  uint32_t m = 0;
  for (int i = 1; i < Lat<D>::Q; ++i)
    if (Lat<D>::ex[i] == sx) m |= 1u << i;
  return m;
}

template <class T, int VW, int EX>
__device__ __forceinline__ Vec<T, VW> load_shifted(const T *plane, int64_t base, int64_t off, int64_t N, bool selfprev,
                                                   bool selfnext) {
  using VT = Vec<T, VW>;
  const int64_t s0 = base - off;
  const VT a = *(const VT *)(plane + s0);
  if constexpr (EX == 0) {
    return a;
  } else if constexpr (EX == 1) {
    uint32_t pv = __shfl_up(lane_bits(a[VW - 1]), 1);
    if (selfprev) {
      const int64_t k = s0 - 1 < 0 ? 0 : s0 - 1;
      pv = lane_bits(plane[k]);
    }
    VT r;
    r[0] = from_lane_bits<T>(pv);
#pragma unroll
    for (int j = 1; j < VW; ++j) r[j] = a[j - 1];
    return r;
  } else {
    uint32_t nv = __shfl_down(lane_bits(a[0]), 1);
    if (selfnext) {
      const int64_t k = s0 + VW > N - 1 ? N - 1 : s0 + VW;
      nv = lane_bits(plane[k]);
    }
    VT r;
#pragma unroll
    for (int j = 0; j < VW - 1; ++j) r[j] = a[j + 1];
    r[VW - 1] = from_lane_bits<T>(nv);
    return r;
  }
}

template <int D, int I> struct DirOff {
  static __device__ __forceinline__ int64_t get(const KP &p) {
    return (int64_t)Lat<D>::ey[I] * p.nx + (D == 3 ? (int64_t)Lat<D>::ez[I] * ((int64_t)p.nx * p.ny) : 0);
  }
};

template <int D, int P, int VW, int I>
__device__ __forceinline__ void load_dir(const KP &p, const typename Prec<P>::SF *fin, const typename Prec<P>::SG *gin,
                                         int64_t base, bool sp, bool sn, Vec<typename Prec<P>::SF, VW> (&fv)[Lat<D>::Q],
                                         Vec<typename Prec<P>::SG, VW> (&gv)[Lat<D>::Qg]) {
  constexpr int EX = Lat<D>::ex[I];
  const int64_t off = DirOff<D, I>::get(p);
  fv[I] = load_shifted<typename Prec<P>::SF, VW, EX>(fin + (int64_t)I * p.Np, base, off, p.N, sp, sn);
  if constexpr (I < Lat<D>::Qg)
    gv[I] = load_shifted<typename Prec<P>::SG, VW, EX>(gin + (int64_t)I * p.Np, base, off, p.N, sp, sn);
}

template <int D, int P, int VW, int... Is>
__device__ __forceinline__ void load_all(const KP &p, const typename Prec<P>::SF *fin, const typename Prec<P>::SG *gin,
                                         int64_t base, bool sp, bool sn, Vec<typename Prec<P>::SF, VW> (&fv)[Lat<D>::Q],
                                         Vec<typename Prec<P>::SG, VW> (&gv)[Lat<D>::Qg], std::integer_sequence<int, Is...>) {
  (load_dir<D, P, VW, Is>(p, fin, gin, base, sp, sn, fv, gv), ...);
}

// Bulk kernel: VW consecutive cells n0 .. n0+VW-1 per thread (the grid is linear in the
// cell index). Requires closed axes (no periodic wrap) and nx % VW == 0, so that every
// group starts on a VW boundary and the pulls of a fluid cell are plain index offsets.
template <int D, int P, int VW, int BS, bool FRC>
__device__ __forceinline__ void sweep_vec_body(const GridPos &gp, const KP &p, const DA &d, int cur) {
  using L = Lat<D>;
  using R = typename Prec<P>::R;
  using SF = typename Prec<P>::SF;
  using SG = typename Prec<P>::SG;
  using FC = FCodec<P, D>;
  using GC = GCodec<P>;
  constexpr int Q = L::Q, Qg = L::Qg;
  using VF = Vec<SF, VW>;
  using VG = Vec<SG, VW>;
  using VB = Vec<uint8_t, VW>;

  const int64_t N = p.N;
  // plain block order: every XCD streams through neighbouring parts of the grid
  const int64_t n0 = (gp.bid * BS + threadIdx.x) * VW;
  const int lane = lane_id();

  // cell types of the group
  VB tv;
  if (n0 < N) tv = *(const VB *)(d.type + n0);
  else {
#pragma unroll
    for (int e = 0; e < VW; ++e) tv[e] = TW;
  }
  bool liquid[VW];
  bool anyliquid = false, anywall = false;
#pragma unroll
  for (int e = 0; e < VW; ++e) {
    const uint8_t tb = tv[e];
    liquid[e] = (tb & TMASK) == TL;
    anyliquid = anyliquid || liquid[e];
    anywall = anywall || (liquid[e] && (tb & NEARWALL));
  }
  if (__ballot(anyliquid) == 0) return;  // wave-uniform

  // aligned loads stay inside [0, N) for groups whose start lies in [lo, hi]; every group
  // holding a fluid cell does (fluid cells are never on the outer layer of a closed axis,
  // which is all walls). Other lanes load from lo: their values are never stored.
  const int64_t offA = (int64_t)p.nx * (D == 3 ? (int64_t)p.ny + 1 : 1);
  const int64_t lo = offA, hi = N - offA - VW;
  const bool safe = n0 >= lo && n0 <= hi;
  const int64_t base = safe ? n0 : lo;
  const bool selfprev = lane == 0 || !(n0 - VW >= lo && n0 - VW <= hi);
  const bool selfnext = lane == 63 || !(n0 + VW >= lo && n0 + VW <= hi);

  VF fv[Q];
  VG gv[Qg];
  load_all<D, P, VW>(p, (const SF *)d.f[cur], (const SG *)d.g[cur], base, selfprev, selfnext, fv, gv,
                     std::make_integer_sequence<int, Q>{});

  const SF *fin = (const SF *)d.f[cur];
  const SG *gin = (const SG *)d.g[cur];
  // instance 4 collides the dissolved gas in its stored units (offsets divided by the
  // scale), with the reference concentration and the source divided likewise
  auto gdec = [&](SG v) -> R {
    if constexpr (P == 4) return (float)v;
    else return GC::dec(v, p);
  };
  auto genc = [&](R v) -> SG {
    if constexpr (P == 4) return (_Float16)v;
    else return GC::enc(v, p);
  };
#pragma unroll
  for (int e = 0; e < VW; ++e) {
    if (liquid[e]) {
      R ft[Q], gt[Qg];
#pragma unroll
      for (int i = 0; i < Q; ++i) ft[i] = FC::dec(fv[i][e], i);
#pragma unroll
      for (int i = 0; i < Qg; ++i) gt[i] = gdec(gv[i][e]);
      const int64_t n = n0 + e;
      if (anywall && (tv[e] & NEARWALL)) {
        // bounce-back: a population whose source is a wall is the cell's own outgoing
        // population of the opposite direction. Every row has a cell next to each x wall,
        // so nearly every wave has such lanes: their two wall patterns (all sources on the
        // low or on the high x side) take a fixed set of directions without a test per
        // direction; any other pattern tests them all.
        const uint32_t wm = d.wmask[n];
        auto bounce = [&](uint32_t mask) {
#pragma unroll
          for (int i = 1; i < Q; ++i) {
            if (mask & (1u << i)) {
              ft[i] = FC::dec(fin[(int64_t)opp(i) * p.Np + n], i);
              if (i < Qg) gt[i] = gdec(gin[(int64_t)opp(i) * p.Np + n]);
            }
          }
        };
        constexpr uint32_t XLO = xwall_mask<D>(1), XHI = xwall_mask<D>(-1);
        if (wm == XLO) bounce(XLO);
        else if (wm == XHI) bounce(XHI);
        else bounce(wm);
      }
      R rho, ux, uy, uz;
      if constexpr (P == 4)
        collide_f32<D, FRC>(p, d, ft, gt, rho, ux, uy, uz, p.c0g_f, p.qg_f);
      else
        collide_cell<D, P, FRC>(p, d, ft, gt, rho, ux, uy, uz);
#pragma unroll
      for (int i = 0; i < Q; ++i) fv[i][e] = FC::enc(ft[i], i);
#pragma unroll
      for (int i = 0; i < Qg; ++i) gv[i][e] = genc(gt[i]);
    }
  }

  // Whole-group streaming (non-temporal) stores for every lane holding a liquid cell: the
  // populations are read again only in the next step, after gigabytes of other traffic,
  // so they are kept out of the caches. The wall and gas cells of the group receive values
  // that nothing reads (bounce-back and the gas-side rebuild take the receiving cell's own
  // values, and a gas cell that turns interface is initialised afresh); interface cells
  // are rewritten by the interface kernel, which runs after this one. (Storing the liquid
  // cells of groups that hold an interface cell one by one would let the two kernels run
  // together, but nearly every wave holds such a group, and the per-cell stores cost the
  // bulk kernel a quarter of its rate.)
  SF *fout = (SF *)d.f[cur ^ 1];
  SG *gout = (SG *)d.g[cur ^ 1];
  if (anyliquid) {
#pragma unroll
    for (int i = 0; i < Q; ++i) __builtin_nontemporal_store(fv[i], (VF *)(fout + (int64_t)i * p.Np + n0));
#pragma unroll
    for (int i = 0; i < Qg; ++i) __builtin_nontemporal_store(gv[i], (VG *)(gout + (int64_t)i * p.Np + n0));
  }
}

template <int D, int P, int VW>
bool vector_ok(const Ctx &c) {
  return bulk_shape_ok(c.kp, P, VW);
}

// the bulk kernel without and with the body-force term; the forced one is held to the
// register budget of four waves per SIMD, which the memory-bound sweep needs, except with
// eight cells per thread, whose 16-byte population vectors do not fit that budget (held to
// it, the kernel spills to scratch and moves four times its bytes): three waves there
template <int VW> constexpr int force_waves() { return VW >= 8 ? 3 : 4; }
template <int D, int P, int VW, int BS>
__global__ __launch_bounds__(BS) void k_sweep_vec(KP p, DA d, int cur) {
  sweep_vec_body<D, P, VW, BS, false>(GridPos::hw(), p, d, cur);
}
template <int D, int P, int VW, int BS>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(force_waves<VW>()))) void k_sweep_vec_force(KP p, DA d, int cur) {
  sweep_vec_body<D, P, VW, BS, true>(GridPos::hw(), p, d, cur);
}

template <int D, int P, int VW, int BS>
bool launch_bulk(Ctx &c, hipStream_t s) {
  if (!vector_ok<D, P, VW>(c)) return false;
  const int64_t nb = (c.kp.N + (int64_t)BS * VW - 1) / ((int64_t)BS * VW);
  if (c.kp.force) hipLaunchKernelGGL((k_sweep_vec_force<D, P, VW, BS>), dim3((unsigned)nb), dim3(BS), 0, s, c.kp, c.d, c.cur);
  else hipLaunchKernelGGL((k_sweep_vec<D, P, VW, BS>), dim3((unsigned)nb), dim3(BS), 0, s, c.kp, c.d, c.cur);
  return true;
}

template <int D, int P>
bool Ops<D, P>::sweep_bulk(Ctx &c, hipStream_t s, int variant) {
  if constexpr (P == 0) {
    return false;
  } else {
    switch (variant) {
      case 0: return launch_bulk<D, P, 4, 256>(c, s);
      case 1: return launch_bulk<D, P, 2, 256>(c, s);
      case 2: return launch_bulk<D, P, 4, 128>(c, s);
      case 3: return launch_bulk<D, P, 2, 128>(c, s);
      case 4: return launch_bulk<D, P, 8, 256>(c, s);
      case 5: return launch_bulk<D, P, 8, 128>(c, s);
      case 6: return launch_bulk<D, P, 8, 64>(c, s);
      case 7: return launch_bulk<D, P, 4, 64>(c, s);
      default: return false;
    }
  }
}

// the bulk kernel in the tuned launch shape (the default one when none was tuned or the
// tuned one does not apply); false when the domain takes the per-cell kernel instead
template <int D, int P>
bool Ops<D, P>::sweep_bulk_auto(Ctx &c, hipStream_t s) {
  if constexpr (P == 0) {
    return false;
  } else {
    const int v = effective_sweep_variant(c.kp, P, c.sweep_variant);
    return v >= 0 && sweep_bulk(c, s, v);
  }
}

// the interface kernel (this step's interface list) of a domain swept by the bulk kernel;
// it runs after the bulk kernel, whose whole-group stores also cover interface cells
template <int D, int P>
void Ops<D, P>::sweep_interface(Ctx &c, hipStream_t s) {
  if constexpr (P == 0) return;  // binary64 domains take the per-cell kernel
  if (c.kp.force) hipLaunchKernelGGL((k_sweep_special<D, P, true>), dim3(list_blocks(c)), dim3(256), 0, s, c.kp, c.d, c.cur);
  else hipLaunchKernelGGL((k_sweep_special<D, P, false>), dim3(list_blocks(c)), dim3(256), 0, s, c.kp, c.d, c.cur);
}

// batched forms of the sweep
template <int D, int P, bool FRC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) void km_sweep(MLaunch ml) {
  MF_MULTI(MK_CELLS)
  b_sweep<D, P, FRC>(gp, m.kp, m.d, m.cur);
}
template <int D, int P, bool FRC>
__global__ __launch_bounds__(256) void km_sweep_special(MLaunch ml) {
  MF_MULTI(MK_LIST)
  b_sweep_special<D, P, FRC>(gp, m.kp, m.d, m.cur);
}
template <int D, int P, int VW, int BS, int V>
__global__ __launch_bounds__(BS) void km_sweep_vec(MLaunch ml) {
  MF_MULTI(MK_BULK0 + V)
  sweep_vec_body<D, P, VW, BS, false>(gp, m.kp, m.d, m.cur);
}
template <int D, int P, int VW, int BS, int V>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(force_waves<VW>()))) void km_sweep_vec_force(MLaunch ml) {
  MF_MULTI(MK_BULK0 + V)
  sweep_vec_body<D, P, VW, BS, true>(gp, m.kp, m.d, m.cur);
}
template <int D, int P, int V>
void launch_bulk_multi(const MStep &ms, bool frc, hipStream_t s) {
  constexpr int VW = kSweepVariants[V].vw, BS = kSweepVariants[V].bs;
  if (!ms.grid[MK_BULK0 + V]) return;
  if (frc) hipLaunchKernelGGL((km_sweep_vec_force<D, P, VW, BS, V>), dim3(ms.grid[MK_BULK0 + V]), dim3(BS), 0, s, ms.at(MK_BULK0 + V));
  else hipLaunchKernelGGL((km_sweep_vec<D, P, VW, BS, V>), dim3(ms.grid[MK_BULK0 + V]), dim3(BS), 0, s, ms.at(MK_BULK0 + V));
}

// the sweep of every domain of a batch: the per-cell kernel (cells), or the bulk kernel
// in each launch shape of vmask (every domain takes work-groups in its own shape only)
// followed by the interface kernel
template <int D, int P>
void Ops<D, P>::sweep_multi(const MStep &ms, unsigned vmask, bool cells, bool frc, int part, hipStream_t s) {
  if (cells || P == 0) {
    if (part == 2) return;
    if (frc) hipLaunchKernelGGL((km_sweep<D, P, true>), dim3(ms.grid[MK_CELLS]), dim3(256), 0, s, ms.at(MK_CELLS));
    else hipLaunchKernelGGL((km_sweep<D, P, false>), dim3(ms.grid[MK_CELLS]), dim3(256), 0, s, ms.at(MK_CELLS));
    return;
  }
  if constexpr (P != 0) {
    if (part != 2) {
      if (vmask & 1u) launch_bulk_multi<D, P, 0>(ms, frc, s);
      if (vmask & 2u) launch_bulk_multi<D, P, 1>(ms, frc, s);
      if (vmask & 4u) launch_bulk_multi<D, P, 2>(ms, frc, s);
      if (vmask & 8u) launch_bulk_multi<D, P, 3>(ms, frc, s);
      if (vmask & 16u) launch_bulk_multi<D, P, 4>(ms, frc, s);
      if (vmask & 32u) launch_bulk_multi<D, P, 5>(ms, frc, s);
      if (vmask & 64u) launch_bulk_multi<D, P, 6>(ms, frc, s);
      if (vmask & 128u) launch_bulk_multi<D, P, 7>(ms, frc, s);
    }
    if (part == 1) return;
    if (frc) hipLaunchKernelGGL((km_sweep_special<D, P, true>), dim3(ms.grid[MK_LIST]), dim3(256), 0, s, ms.at(MK_LIST));
    else hipLaunchKernelGGL((km_sweep_special<D, P, false>), dim3(ms.grid[MK_LIST]), dim3(256), 0, s, ms.at(MK_LIST));
  }
}

template <int D, int P>
void Ops<D, P>::bulk_multi(const MStep &ms, int v, bool frc, hipStream_t s) {
  if constexpr (P != 0) {
    switch (v) {
      case 0: launch_bulk_multi<D, P, 0>(ms, frc, s); break;
      case 1: launch_bulk_multi<D, P, 1>(ms, frc, s); break;
      case 2: launch_bulk_multi<D, P, 2>(ms, frc, s); break;
      case 3: launch_bulk_multi<D, P, 3>(ms, frc, s); break;
      case 4: launch_bulk_multi<D, P, 4>(ms, frc, s); break;
      case 5: launch_bulk_multi<D, P, 5>(ms, frc, s); break;
      case 6: launch_bulk_multi<D, P, 6>(ms, frc, s); break;
      case 7: launch_bulk_multi<D, P, 7>(ms, frc, s); break;
      default: break;
    }
  }
}

// the per-cell kernel over the whole grid (binary64 and periodic domains)
template <int D, int P>
void Ops<D, P>::sweep_cells(Ctx &c, hipStream_t s) {
  const int gx = (c.kp.nx + 63) / 64, gy = (c.kp.ny + 3) / 4;
  const int64_t nb = (int64_t)gx * gy * c.kp.nz;
  if (c.kp.force) hipLaunchKernelGGL((k_sweep<D, P, true>), dim3((unsigned)nb), dim3(256), 0, s, c.kp, c.d, c.cur);
  else hipLaunchKernelGGL((k_sweep<D, P, false>), dim3((unsigned)nb), dim3(256), 0, s, c.kp, c.d, c.cur);
}

}  // namespace mf

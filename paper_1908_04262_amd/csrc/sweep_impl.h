// Lattice sweep: one thread per cell, pull streaming from the SoA buffer of the
// previous step into the other buffer.
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
// The kernel also lists the interface cells and the bubble cells of the types it read.
#pragma once
#include "lbm_math.h"

namespace mf {

template <int D, int P>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_sweep(KP p, DA d, int cur) {
  using L = Lat<D>;
  using R = typename Prec<P>::R;
  using SF = typename Prec<P>::SF;
  using SG = typename Prec<P>::SG;
  using FC = FCodec<P, D>;
  using A = Arith<D, P>;
  constexpr int Q = L::Q, Qg = L::Qg;

  // tile of 64 x 4 cells; consecutive tiles of one z-range go to the same XCD
  const int gx = (p.nx + 63) >> 6, gy = (p.ny + 3) >> 2;
  const int64_t nb = (int64_t)gx * gy * p.nz;
  int64_t b = blockIdx.x;
  const int64_t per = nb >> 3;
  if (b < (per << 3)) b = (b & 7) * per + (b >> 3);
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
  const bool gi = in && (t == TG || t == TI);
  const int32_t lab = gi ? d.label[n] : NOLAB;
  wave_append(d.ilist, d.cnt + C_I, in && t == TI, (int32_t)n);
  wave_append(d.blist, d.cnt + C_B, gi && lab != 0, (int32_t)n);

  const bool fluid = in && (t == TL || t == TI);
  const bool isI = fluid && t == TI;
  bool hasgas = false;
  R phic = R(0);

  if (fluid) {
    const SF *fin = (const SF *)d.f[cur];
    SF *fout = (SF *)d.f[cur ^ 1];
    const SG *gin = (const SG *)d.g[cur];
    SG *gout = (SG *)d.g[cur ^ 1];
    const int64_t Np = p.Np;
    R ft[Q], gt[Qg];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int64_t s = nb_index(p, x, y, z, -L::ex[i], -L::ey[i], -L::ez[i]);
      ft[i] = FC::dec(fin[(int64_t)i * Np + s], i);
      if (i < Qg) gt[i] = gin[(int64_t)i * Np + s];
    }
    R Ms = R(0);
    const bool special = isI || (tb & NEARWALL);
    bool hasG = false, hasF = false;
    if (special) {
      R own[Q], gown[Qg];
      uint8_t tsrc[Q];
      // the cell's own outgoing populations (bounce-back, mass exchange) and the types
      // of its sources, all loads issued together
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        own[i] = FC::dec(fin[(int64_t)i * Np + n], i);
        if (i < Qg) gown[i] = gin[(int64_t)i * Np + n];
        const int64_t s = nb_index(p, x, y, z, -L::ex[i], -L::ey[i], -L::ez[i]);
        tsrc[i] = d.type[s] & TMASK;
      }
      R rg = R(1), uox = R(0), uoy = R(0), uoz = R(0), uou = R(0), cH = R(0), dcH = R(0);
      if (isI) {
        double pb = p.p_atm;
        if (lab >= 0 && lab < p.cap && d.balive[lab]) pb = d.bp[lab];
        else raise_status(d.status, ST_BADLABEL);
        const R kap = ((const R *)d.kappa)[n], pi = ((const R *)d.Pi)[n];
        rg = R(3) * ((R(pb) - R(2) * R(p.sigma) * kap) - pi);
        cH = R(p.kH) * R(pb);
        dcH = cH - R(p.c0);
        uox = ((const R *)d.ux)[n];
        uoy = ((const R *)d.uy)[n];
        uoz = D == 3 ? ((const R *)d.uz)[n] : R(0);
        uou = usq<D, R>(uox, uoy, uoz);
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
        const R ax = ((const R *)d.alpha)[n];
        R dm = R(0);
#pragma unroll
        for (int i = 1; i < Q; ++i) {
          const int tn = tsrc[opp(i)];
          if (tn == TL) {
            dm = dm + (ft[opp(i)] - own[i]);
          } else if (tn == TI) {
            const int64_t yy = nb_index(p, x, y, z, L::ex[i], L::ey[i], L::ez[i]);
            const R ay = ((const R *)d.alpha)[yy];
            dm = dm + (R(0.5) * (ax + ay)) * (ft[opp(i)] - own[i]);
          }
        }
        Ms = ((const R *)d.M)[n] + dm;
      }
    }
    // moments and collision
    R rho, drho, ux, uy, uz;
    A::mom(ft, rho, drho, ux, uy, uz);
    if (!(rho > R(0))) raise_status(d.status, ST_NONFINITE);
    const R uu = usq<D, R>(ux, uy, uz);
    R omega = R(p.omega);
    if (p.rheology == MF_POWER_LAW) {
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
      const R ss = ((pxx * pxx + pyy * pyy) + pzz * pzz) + R(2) * ((pxy * pxy + pxz * pxz) + pyz * pyz);
      omega = R(1) / powerlaw_tau<R>(p, rho, sqrt(ss));
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const R fe = A::eq(i, rho, drho, ux, uy, uz, uu);
      fout[(int64_t)i * Np + n] = FC::enc(ft[i] - omega * (ft[i] - fe), i);
    }
    R dc;
    const R c = A::conc(gt, R(p.c0), dc);
    const R og = R(p.omega_g), q = R(p.q);
#pragma unroll
    for (int i = 0; i < Qg; ++i) {
      gout[(int64_t)i * Np + n] = (gt[i] - og * (gt[i] - A::geqv(i, c, dc, ux, uy, uz))) + R(Lat<D>::wg[i]) * q;
    }
    if (isI) {
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
    }
  }
  wave_fx_add(d.phi, hasgas && lab >= 0 && lab < p.cap, lab, fx3((double)phic));
}

template <int D, int P>
void Ops<D, P>::sweep(Ctx &c, hipStream_t s) {
  const int gx = (c.kp.nx + 63) / 64, gy = (c.kp.ny + 3) / 4;
  const int64_t nb = (int64_t)gx * gy * c.kp.nz;
  hipLaunchKernelGGL((k_sweep<D, P>), dim3((unsigned)nb), dim3(256), 0, s, c.kp, c.d, c.cur);
}

}  // namespace mf

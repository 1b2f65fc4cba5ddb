// Interface geometry of the new interface cells:
//  - unit normal from central differences of the fill fraction (pointing into the
//    liquid) and the PLIC plane offset of each cell (analytic inverse of the cut-cube
//    volume, Scardovelli & Zaleski, as used for the disjoining distance in Sec. 3.3);
//  - mean curvature (k1 + k2)/2 from a least-squares paraboloid (3D, 3x3x3 block) or
//    parabola (2D, 5x5 block) through the PLIC points of the interface cells around the
//    cell, in the frame of its normal; it enters the gas density of Eq. rhob;
//  - disjoining pressure (Sec. 3.3): march along the normal into the liquid with the
//    traversal of Appendix A (Algorithm 1), every tied axis stepping together, until an
//    interface or gas cell of another bubble (distance d, Pi = k_Pi (d_max - d)).
#include "lbm_math.h"

namespace mf {

template <class R> __device__ __forceinline__ R dsqrt(R v) { return sqrt(v); }
__device__ __forceinline__ double dcbrt(double v) { return cbrt(v); }
__device__ __forceinline__ float dcbrt(float v) { return cbrtf(v); }
__device__ __forceinline__ double dacos(double v) { return acos(v); }
__device__ __forceinline__ float dacos(float v) { return acosf(v); }
__device__ __forceinline__ double dcos(double v) { return cos(v); }
__device__ __forceinline__ float dcos(float v) { return cosf(v); }
template <class R> __device__ __forceinline__ R dabs(R v) { return v < R(0) ? -v : v; }

// root of the monic cubic a^3 + b a^2 + c a + d in [lo, hi] (the interval holds exactly
// one), trigonometric / Cardano form, then two Newton steps kept inside the interval
template <class R>
__device__ R cubic_root_in(R b, R c, R d, R lo, R hi) {
  const R p = c - (b * b) / R(3);
  const R qq = ((R(2) * b * b * b) / R(27) - (b * c) / R(3)) + d;
  const R shift = -b / R(3);
  R best = R(0.5) * (lo + hi), bestd = R(1e30);
  const R disc = (qq * qq) / R(4) + (p * p * p) / R(27);
  R cand[3];
  int nc = 0;
  if (p < R(0) && disc <= R(0)) {
    const R r = R(2) * dsqrt(-p / R(3));
    R arg = ((R(3) * qq) / (R(2) * p)) * dsqrt(R(-3) / p);
    if (arg > R(1)) arg = R(1);
    if (arg < R(-1)) arg = R(-1);
    const R th = dacos(arg) / R(3);
    for (int k = 0; k < 3; k++) cand[nc++] = r * dcos(th - (R(2) * R(3.14159265358979323846) * R(k)) / R(3)) + shift;
  } else {
    const R sd = dsqrt(disc > R(0) ? disc : R(0));
    cand[nc++] = dcbrt(-qq / R(2) + sd) + dcbrt(-qq / R(2) - sd) + shift;
  }
  for (int k = 0; k < nc; k++) {
    const R t = cand[k];
    const R dd = t < lo ? lo - t : (t > hi ? t - hi : R(0));
    if (dd < bestd) { bestd = dd; best = t; }
  }
  if (best < lo) best = lo;
  if (best > hi) best = hi;
  for (int k = 0; k < 2; k++) {
    const R f = ((best + b) * best + c) * best + d;
    const R df = (R(3) * best + R(2) * b) * best + c;
    if (df != R(0)) {
      const R nb2 = best - f / df;
      if (nb2 >= lo && nb2 <= hi) best = nb2;
    }
  }
  return best;
}

// plane constant a in [0, 1/2] with vol{x in [0,1]^3 : n.x <= a} = v; n sorted ascending
// with unit sum
template <class R>
__device__ R sz_inverse3(R m1, R m2, R m3, R v) {
  if (m2 <= R(0)) return v;
  if (m1 <= R(0)) {
    const R v1 = m2 / (R(2) * m3);
    if (v <= v1) return dsqrt((R(2) * m2 * m3) * v);
    return m3 * v + R(0.5) * m2;
  }
  const R m12 = m1 + m2;
  const R v1 = (m1 * m1) / (R(6) * m2 * m3);
  const R v2 = v1 + (m2 - m1) / (R(2) * m3);
  R v3;
  if (m3 < m12) {
    const R a = m3;
    v3 = ((a * a) * (R(3) * m12 - a) + (m1 * m1) * (m1 - R(3) * a) + (m2 * m2) * (m2 - R(3) * a)) /
         (R(6) * m1 * m2 * m3);
  } else {
    v3 = m12 / (R(2) * m3);
  }
  if (v < v1) return dcbrt((R(6) * m1 * m2 * m3) * v);
  if (v < v2) return R(0.5) * (m1 + dsqrt((R(8) * m2 * m3) * v - (m1 * m1) / R(3)));
  if (v < v3) {
    const R hi = m3 < m12 ? m3 : m12;
    const R c3 = R(3) * (m1 * m1 + m2 * m2);
    const R c0 = -(((m1 * m1 * m1) + (m2 * m2 * m2)) - (R(6) * m1 * m2 * m3) * v);
    return cubic_root_in<R>(R(-3) * m12, c3, c0, m2, hi);
  }
  if (m3 < m12) {
    const R s2 = (m1 * m1 + m2 * m2) + m3 * m3;
    const R s3 = ((m1 * m1 * m1) + (m2 * m2 * m2)) + (m3 * m3 * m3);
    return cubic_root_in<R>(R(-1.5), R(1.5) * s2, R(-0.5) * (s3 - (R(6) * m1 * m2 * m3) * v), m3, R(0.5));
  }
  return m3 * v + R(0.5) * m12;
}

template <class R> __device__ __forceinline__ R clamp01(R a) { return a < R(0) ? R(0) : (a > R(1) ? R(1) : a); }

// signed distance from the cell centre to the PLIC plane of normal m (into the liquid)
// that leaves the liquid fraction alpha on the +m side
template <int D, class R>
__device__ R plic_offset(R alpha, R mx, R my, R mz) {
  const R a = clamp01(alpha);
  const R v = a < R(1) - a ? a : R(1) - a;
  const R ax = dabs(mx), ay = dabs(my), az = D == 3 ? dabs(mz) : R(0);
  const R l1 = (ax + ay) + az;
  R c;
  if (l1 <= R(0)) return R(0);
  if (D == 2) {
    R n1 = ax < ay ? ax : ay, n2 = ax < ay ? ay : ax;
    n1 = n1 / l1;
    n2 = n2 / l1;
    const R v1 = n1 / (R(2) * n2);
    if (v <= v1) c = dsqrt((R(2) * n1 * n2) * v);
    else c = n2 * v + R(0.5) * n1;
  } else {
    R t, m1 = ax, m2 = ay, m3 = az;
    if (m1 > m2) { t = m1; m1 = m2; m2 = t; }
    if (m2 > m3) { t = m2; m2 = m3; m3 = t; }
    if (m1 > m2) { t = m1; m1 = m2; m2 = t; }
    m1 = m1 / l1;
    m2 = m2 / l1;
    m3 = m3 / l1;
    c = sz_inverse3<R>(m1, m2, m3, v);
  }
  const R smag = (R(0.5) - c) * l1;
  return a < R(0.5) ? smag : -smag;
}

// fill fraction seen by the geometric stencils; walls and off-domain cells read the
// centre cell's value
template <class R>
__device__ __forceinline__ R alpha_seen(const DA &d, int64_t y, R ac) {
  if (y < 0) return ac;
  const int t = d.type[y] & TMASK;
  if (t == TG) return R(0);
  if (t == TL) return R(1);
  if (t == TI) return clamp01(((const R *)d.alpha)[y]);
  return ac;
}

// the new interface cells: old interface cells that stayed, new ones from gas and
// from liquid
#define NEWI_LOOP(k, n)                                                              \
  const int _nI = *(volatile int32_t *)(d.cnt + C_I);                                 \
  const int _nNI = *(volatile int32_t *)(d.cnt + C_NI);                               \
  const int _nL2 = *(volatile int32_t *)(d.cnt + C_L2I);                              \
  const int64_t _tot = (int64_t)_nI + _nNI + _nL2;                                    \
  for (int64_t k = gp.bid * blockDim.x + threadIdx.x; k < _tot;                      \
       k += gp.nblk * blockDim.x)

#define NEWI_CELL(k)                                                                  \
  (k < _nI ? (int64_t)d.ilist[k]                                                      \
           : (k < (int64_t)_nI + _nNI ? (int64_t)d.nilist[k - _nI] : (int64_t)d.l2ilist[k - _nI - _nNI]))

template <int D, int P>
__device__ __forceinline__ void b_normals(const GridPos &gp, KP p, DA d, int words) {
  using R = typename Prec<P>::R;
  NEWI_LOOP(k, n) {
    const int64_t n = NEWI_CELL(k);
    const uint8_t tb = d.type[n];
    // the cells of this step's lists are the ones whose type or fill fraction changed:
    // their stencil words (learned curvature) follow here, unless the excess pass of the
    // time step or a whole-grid pass has written them
    if (words) d.sword[n] = stencil_word<R>(tb, ((const R *)d.alpha)[n], d.label[n]);
    if ((tb & TMASK) != TI) continue;
    int x, y, z;
    cell_xyz(p, n, x, y, z);
    const R ac = clamp01(((const R *)d.alpha)[n]);
    const R gx = R(0.5) * (alpha_seen<R>(d, nb_index_or_none(p, x, y, z, 1, 0, 0), ac) -
                           alpha_seen<R>(d, nb_index_or_none(p, x, y, z, -1, 0, 0), ac));
    const R gy = R(0.5) * (alpha_seen<R>(d, nb_index_or_none(p, x, y, z, 0, 1, 0), ac) -
                           alpha_seen<R>(d, nb_index_or_none(p, x, y, z, 0, -1, 0), ac));
    R gz = R(0);
    if (D == 3)
      gz = R(0.5) * (alpha_seen<R>(d, nb_index_or_none(p, x, y, z, 0, 0, 1), ac) -
                     alpha_seen<R>(d, nb_index_or_none(p, x, y, z, 0, 0, -1), ac));
    const R gn = dsqrt((gx * gx + gy * gy) + gz * gz);
    R mx = R(0), my = R(0), mz = R(0), off = R(0);
    if (gn != R(0)) {
      mx = gx / gn;
      my = gy / gn;
      mz = gz / gn;
      off = plic_offset<D, R>(((const R *)d.alpha)[n], mx, my, mz);
    }
    ((R *)d.mx)[n] = mx;
    ((R *)d.my)[n] = my;
    ((R *)d.mz)[n] = mz;
    ((R *)d.soff)[n] = off;
  }
}
template <int D, int P>
__global__ __launch_bounds__(256) void k_normals(KP p, DA d, int words) {
  b_normals<D, P>(GridPos::hw(), p, d, words);
}

// Gaussian elimination with partial pivoting (first maximum on ties); fails when a pivot
// falls below rel times the largest diagonal entry (the points do not determine the fit).
// Fully unrolled: row swaps are selects, so the matrix stays in registers.
template <class R, int NU>
__device__ __forceinline__ bool solve_ge(R (&A)[NU][NU], R (&b)[NU], R (&x)[NU], R rel) {
  R scale = R(0);
#pragma unroll
  for (int c = 0; c < NU; c++)
    if (A[c][c] > scale) scale = A[c][c];
  const R tiny = rel * scale;
  bool ok = true;
#pragma unroll
  for (int c = 0; c < NU; c++) {
    int piv = c;
    R best = dabs(A[c][c]);
#pragma unroll
    for (int r = c + 1; r < NU; r++) {
      const R v = dabs(A[r][c]);
      if (v > best) { best = v; piv = r; }
    }
    if (!(best >= tiny)) ok = false;
#pragma unroll
    for (int r = c + 1; r < NU; r++) {
      const bool sw = r == piv;
#pragma unroll
      for (int k = 0; k < NU; k++) {
        const R t = A[c][k];
        A[c][k] = sw ? A[r][k] : t;
        A[r][k] = sw ? t : A[r][k];
      }
      const R t = b[c];
      b[c] = sw ? b[r] : t;
      b[r] = sw ? t : b[r];
    }
#pragma unroll
    for (int r = c + 1; r < NU; r++) {
      const R f = A[r][c] / A[c][c];
#pragma unroll
      for (int k = c; k < NU; k++) A[r][k] = A[r][k] - f * A[c][k];
      b[r] = b[r] - f * b[c];
    }
  }
#pragma unroll
  for (int r = NU - 1; r >= 0; r--) {
    R acc = b[r];
#pragma unroll
    for (int k = r + 1; k < NU; k++) acc = acc - A[r][k] * x[k];
    x[r] = acc / A[r][r];
  }
  return ok;
}

// add one fit point: normal-matrix entries phi_a phi_b (upper triangle, mirrored: the
// products are symmetric, so this equals accumulating every entry) and rhs phi_a h
template <class R, int NU>
__device__ __forceinline__ void add_point(R (&A)[NU][NU], R (&rhs)[NU], const R (&phi)[NU], R h) {
#pragma unroll
  for (int a = 0; a < NU; a++) {
#pragma unroll
    for (int b = a; b < NU; b++) A[a][b] = A[a][b] + phi[a] * phi[b];
    rhs[a] = rhs[a] + phi[a] * h;
  }
}

// plain curvature of interface cell n: paraboloid (parabola in 2D) least squares through
// the PLIC points of the cell and of the interface cells of its block
template <int D, int P>
__device__ __forceinline__ typename Prec<P>::R plain_fit(const KP &p, const DA &d, int64_t n) {
  using R = typename Prec<P>::R;
  constexpr int NU = D == 3 ? 6 : 3;
  constexpr int RR = D == 3 ? 1 : 2;
  const R rel = sizeof(R) == 8 ? R(1e-9) : R(1e-6);
  const R *MX = (const R *)d.mx, *MY = (const R *)d.my, *MZ = (const R *)d.mz, *SO = (const R *)d.soff;
  {
    const R m0 = MX[n], m1 = MY[n], m2 = MZ[n];
    R kap = R(0);
    if (m0 != R(0) || m1 != R(0) || m2 != R(0)) {
      int x, y, z;
      cell_xyz(p, n, x, y, z);
      R t1[3], t2[3];
      if (D == 3) {
        int kk = 0;
        const R am[3] = {dabs(m0), dabs(m1), dabs(m2)};
        if (am[1] < am[kk]) kk = 1;
        if (am[2] < am[kk]) kk = 2;
        R c0, c1, c2;
        if (kk == 0) { c0 = R(0); c1 = m2; c2 = -m1; }
        else if (kk == 1) { c0 = -m2; c1 = R(0); c2 = m0; }
        else { c0 = m1; c1 = -m0; c2 = R(0); }
        const R cn = dsqrt((c0 * c0 + c1 * c1) + c2 * c2);
        t1[0] = c0 / cn; t1[1] = c1 / cn; t1[2] = c2 / cn;
        t2[0] = m1 * t1[2] - m2 * t1[1];
        t2[1] = m2 * t1[0] - m0 * t1[2];
        t2[2] = m0 * t1[1] - m1 * t1[0];
      } else {
        t1[0] = -m1; t1[1] = m0; t1[2] = R(0);
        t2[0] = t2[1] = t2[2] = R(0);
      }
      R A[NU][NU], rhs[NU], sol[NU];
#pragma unroll
      for (int a = 0; a < NU; a++) {
        rhs[a] = R(0);
        sol[a] = R(0);
#pragma unroll
        for (int b = 0; b < NU; b++) A[a][b] = R(0);
      }
      int np = 0;
      // the centre point first, then the block in (dz, dy, dx) ascending order
      for (int j = -1; j < (D == 3 ? 27 : 25); j++) {
        int dx = 0, dy = 0, dz = 0;
        if (j >= 0) {
          if (D == 3) { dx = j % 3 - 1; dy = (j / 3) % 3 - 1; dz = j / 9 - 1; }
          else { dx = j % 5 - 2; dy = j / 5 - 2; }
          if (dx == 0 && dy == 0 && dz == 0) continue;
        }
        const int64_t yy = j < 0 ? n : nb_index_or_none(p, x, y, z, dx, dy, dz);
        if (yy < 0 || (d.type[yy] & TMASK) != TI) continue;
        const R q0 = MX[yy], q1 = MY[yy], q2 = MZ[yy];
        if (q0 == R(0) && q1 == R(0) && q2 == R(0)) continue;
        const R off = SO[yy];
        const R px = R(dx) + off * q0, py = R(dy) + off * q1, pz = R(dz) + off * q2;
        const R u = (px * t1[0] + py * t1[1]) + pz * t1[2];
        const R h = (px * m0 + py * m1) + pz * m2;
        R phi[NU];
        if constexpr (D == 3) {
          const R v = (px * t2[0] + py * t2[1]) + pz * t2[2];
          phi[0] = u * u; phi[1] = v * v; phi[2] = u * v; phi[3] = u; phi[4] = v; phi[5] = R(1);
        } else {
          phi[0] = u * u; phi[1] = u; phi[2] = R(1);
        }
        add_point<R, NU>(A, rhs, phi, h);
        np++;
      }
#pragma unroll
      for (int a = 0; a < NU; a++)
#pragma unroll
        for (int b = 0; b < a; b++) A[a][b] = A[b][a];
      // 3D: ridge term on the quadratic coefficients; keeps one-sided point sets (next
      // to walls) determined and pulls their undetermined curvature towards zero
      if (D == 3) {
#pragma unroll
        for (int a = 0; a < 3; a++) A[a][a] = A[a][a] + R(1e-2);
      }
      if (np >= NU && solve_ge<R, NU>(A, rhs, sol, rel)) {
        if constexpr (D == 3) {
          const R cA = sol[0], cB = sol[1], cC = sol[2], cD = sol[3], cE = sol[4];
          const R num = (((R(1) + cE * cE) * (R(2) * cA)) - (((R(2) * cD) * cE) * cC)) + ((R(1) + cD * cD) * (R(2) * cB));
          const R t = (R(1) + cD * cD) + cE * cE;
          const R den = R(2) * (t * dsqrt(t));
          kap = -(num / den);
        } else {
          const R cA = sol[0], cD = sol[1];
          const R t = R(1) + cD * cD;
          kap = -(cA / (t * dsqrt(t)));
        }
        if (kap > R(1)) kap = R(1);
        if (kap < R(-1)) kap = R(-1);
      }
    }
    return kap;
  }
}

// disjoining pressure of interface cell n (ray march along its normal) and the gas side
// the next sweep rebuilds missing populations with
template <int D, int P>
__device__ __forceinline__ void disjoining_cell(const KP &p, DA &d, int64_t n, typename Prec<P>::R kap) {
  using R = typename Prec<P>::R;
  {
    R Pi = R(0);
    const R m[3] = {((const R *)d.mx)[n], ((const R *)d.my)[n], ((const R *)d.mz)[n]};
    if (p.k_pi > 0.0 && (m[0] != R(0) || m[1] != R(0) || m[2] != R(0))) {
      const int dmax = (int)p.d_max;
      R bmax[3], bdel[3];
      int step[3];
      for (int a = 0; a < 3; a++) {
        if (a >= D) { bmax[a] = R(INFINITY); bdel[a] = R(INFINITY); step[a] = 1; continue; }
        bmax[a] = dabs(R(0.5) / m[a]);
        bdel[a] = dabs(R(1) / m[a]);
        step[a] = m[a] >= R(0) ? 1 : -1;
      }
      int x, y, z;
      cell_xyz(p, n, x, y, z);
      const int32_t lab = d.label[n];
      int ox = 0, oy = 0, oz = 0;
      for (int it = 1; it <= dmax; it++) {
        R bmin = bmax[0];
        if (bmax[1] < bmin) bmin = bmax[1];
        if (bmax[2] < bmin) bmin = bmax[2];
        for (int a = 0; a < D; a++)
          if (bmax[a] == bmin) {
            bmax[a] = bmax[a] + bdel[a];
            if (a == 0) ox += step[0];
            else if (a == 1) oy += step[1];
            else oz += step[2];
          }
        const int64_t cur = nb_index_or_none(p, x, y, z, ox, oy, oz);
        if (cur < 0) break;
        if (d.label[cur] == lab) continue;
        const int tc = d.type[cur] & TMASK;
        if (tc == TW) break;
        if (tc == TI || tc == TG) {
          R bout = bmax[0];
          if (bmax[1] < bout) bout = bmax[1];
          if (bmax[2] < bout) bout = bmax[2];
          const R ay = tc == TI ? clamp01(((const R *)d.alpha)[cur]) : R(0);
          const R dprime = bout - (R(1) - ay) * (bout - bmin);
          R dd = dprime - ((const R *)d.soff)[n];
          if (dd < R(0)) dd = R(0);
          if (dd < R(p.d_max)) Pi = R(p.k_pi) * (R(p.d_max) - dd);
          break;
        }
      }
    }
    ((R *)d.Pi)[n] = Pi;
    // gas-side density and bubble pressure the next sweep rebuilds missing populations with
    const int32_t lab = d.label[n];
    double pb = p.p_atm;
    if (lab >= 0 && lab < p.cap && d.balive[lab]) pb = d.bp[lab];
    else raise_status(d.status, ST_BADLABEL);
    ((R *)d.rgas)[n] = R(3) * ((R(pb) - R(2) * R(p.sigma) * kap) - Pi);
    ((R *)d.pbub)[n] = R(pb);
  }
}

// per interface cell: curvature (the plain fit, unless the network already gave it),
// disjoining pressure and gas side
template <int D, int P>
__device__ __forceinline__ void b_curvature(const GridPos &gp, KP p, DA d) {
  using R = typename Prec<P>::R;
  NEWI_LOOP(k, n) {
    const int64_t n = NEWI_CELL(k);
    if ((d.type[n] & TMASK) != TI) continue;
    R kap;
    if (d.cflag[n] & CF_MLPOK) {  // the network already gave this cell's curvature
      d.cflag[n] = 0;
      kap = ((const R *)d.kappa)[n];
    } else {
      kap = plain_fit<D, P>(p, d, n);
      ((R *)d.kappa)[n] = kap;
    }
    disjoining_cell<D, P>(p, d, n, kap);
  }
}
template <int D, int P>
__global__ __launch_bounds__(256) void k_curvature(KP p, DA d) {
  b_curvature<D, P>(GridPos::hw(), p, d);
}

// stencil words (learned curvature) over the whole grid, after a state change made
// outside the time step
template <int P>
__global__ __launch_bounds__(256) void k_sword_all(KP p, DA d) {
  using R = typename Prec<P>::R;
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < p.N; n += (int64_t)gridDim.x * blockDim.x)
    d.sword[n] = stencil_word<R>(d.type[n], ((const R *)d.alpha)[n], d.label[n]);
}

// Normals (and the stencil words of the list cells when nothing else has written them);
// they read fill fractions and types only, not ids, so they may run beside the labelling.
template <int D, int P>
void Ops<D, P>::geometry_normals(Ctx &c, hipStream_t s, bool words) {
  hipLaunchKernelGGL((k_normals<D, P>), dim3(list_blocks(c)), dim3(256), 0, s, c.kp, c.d, words && c.d.sword ? 1 : 0);
  if (c.ev_norm_rec) (void)hipEventRecord(c.ev_norm_rec, s);
}

// Curvature (learned, then the plain fit where the network gave nothing), disjoining
// pressure and the gas side of the interface cells; after the labelling and the normals.
template <int D, int P>
void Ops<D, P>::geometry_curv(Ctx &c, hipStream_t s) {
  if (c.kp.curvature == MF_CURV_MLP && c.d.mlp_w) launch_mlp_curv(c, s);
  hipLaunchKernelGGL((k_curvature<D, P>), dim3(list_blocks(c)), dim3(256), 0, s, c.kp, c.d);
  c.gas_dirty = false;
  c.sword_fresh = false;
}

// batched forms (time step: the stencil words come from the excess pass)
template <int D, int P>
__global__ __launch_bounds__(256) void km_normals(MLaunch ml) {
  MF_MULTI(MK_LIST)
  b_normals<D, P>(gp, m.kp, m.d, 0);
}
template <int D, int P>
__global__ __launch_bounds__(256) void km_curvature(MLaunch ml) {
  MF_MULTI(MK_LIST)
  b_curvature<D, P>(gp, m.kp, m.d);
}

// the geometry of every domain of a batch, in the order of geometry() inside a step
template <int D, int P>
void Ops<D, P>::geometry_multi(const MStep &ms, bool mlp, hipStream_t s) {
  hipLaunchKernelGGL((km_normals<D, P>), dim3(ms.grid[MK_LIST]), dim3(256), 0, s, ms.at(MK_LIST));
  if (mlp) mlp_curv_multi(ms, P, s);
  hipLaunchKernelGGL((km_curvature<D, P>), dim3(ms.grid[MK_LIST]), dim3(256), 0, s, ms.at(MK_LIST));
}

template <int D, int P>
void Ops<D, P>::geometry(Ctx &c, hipStream_t s) {
  // stencil words: over the whole grid after a state change made outside the time step,
  // else from the excess pass of the step or, outside a step, with the normals
  const bool sword_all = c.d.sword && c.sword_dirty;
  if (sword_all) {
    const int64_t g = (c.kp.N + 255) / 256;
    hipLaunchKernelGGL((k_sword_all<P>), dim3((unsigned)(g < 65536 ? g : 65536)), dim3(256), 0, s, c.kp, c.d);
  }
  c.sword_dirty = false;  // (a context without words has none to rebuild)
  geometry_normals(c, s, !sword_all && !c.sword_fresh);
  geometry_curv(c, s);
}

#define MF_INST(D, P)                                                     \
  template void Ops<D, P>::geometry(Ctx &, hipStream_t);                  \
  template void Ops<D, P>::geometry_normals(Ctx &, hipStream_t, bool);    \
  template void Ops<D, P>::geometry_curv(Ctx &, hipStream_t);           \
  template void Ops<D, P>::geometry_multi(const MStep &, bool, hipStream_t);

MF_FOR_ALL(MF_INST)

}  // namespace mf

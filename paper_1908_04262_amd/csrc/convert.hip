// Cell-type conversion and excess-mass redistribution (Sec. 2.1, last paragraph):
// interface cells with alpha >= 1 become liquid, with alpha <= 0 become gas; the
// surplus or shortage is spread equally over the neighbouring interface cells.
// All passes run over compact lists (interface cells of the step, and the cells that
// change type) and are pull gathers or idempotent flag scatters, so their result does
// not depend on thread order.
#include "lbm_math.h"

namespace mf {

// (a) every gas neighbour of a filled cell becomes a new interface cell; an emptied
// neighbour of a filled cell stays an interface cell
template <int D>
__global__ __launch_bounds__(256) void k_fill_scatter(KP p, DA d) {
  using L = Lat<D>;
  LIST_LOOP(k, d.cnt + C_I) {
    bool act = false;
    int64_t n = 0;
    if (k < *(volatile int32_t *)(d.cnt + C_I)) {
      n = d.ilist[k];
      act = (d.cflag[n] & CF_FILL) != 0;
    }
    if (!__ballot(act)) continue;  // wave-uniform
    int x = 0, y = 0, z = 0;
    if (act) cell_xyz(p, n, x, y, z);
    for (int i = 1; i < L::Q; ++i) {
      bool add = false;
      int64_t yy = 0;
      if (act) {
        yy = nb_index(p, x, y, z, L::ex[i], L::ey[i], L::ez[i]);
        const int ty = d.type[yy] & TMASK;
        if (ty == TG) {
          add = !(flag_or(d.cflag, yy, CF_NEWI) & CF_NEWI);
        } else if (ty == TI) {
          if (d.cflag[yy] & CF_EMPTY) flag_clear(d.cflag, yy, CF_EMPTY);
        }
      }
      const int slot = wave_append_slot(d.cnt + C_NI, add);
      if (add) d.nilist[slot] = (int32_t)yy;
    }
  }
}

// (b) every liquid neighbour of a (still) emptied cell becomes an interface cell and
// takes the smallest bubble id among its emptied neighbours
template <int D>
__global__ __launch_bounds__(256) void k_empty_scatter(KP p, DA d) {
  using L = Lat<D>;
  LIST_LOOP(k, d.cnt + C_I) {
    bool act = false;
    int64_t n = 0;
    if (k < *(volatile int32_t *)(d.cnt + C_I)) {
      n = d.ilist[k];
      act = (d.cflag[n] & CF_EMPTY) != 0;
    }
    if (!__ballot(act)) continue;  // wave-uniform
    int x = 0, y = 0, z = 0;
    int32_t lab = 0;
    if (act) {
      cell_xyz(p, n, x, y, z);
      lab = d.label[n];
    }
    for (int i = 1; i < L::Q; ++i) {
      bool add = false;
      int64_t yy = 0;
      if (act) {
        yy = nb_index(p, x, y, z, L::ex[i], L::ey[i], L::ez[i]);
        if ((d.type[yy] & TMASK) == TL) {
          atomicMin((unsigned int *)&d.label[yy], (unsigned int)lab);
          add = !(flag_or(d.cflag, yy, CF_L2I) & CF_L2I);
        }
      }
      const int slot = wave_append_slot(d.cnt + C_L2I, add);
      if (add) d.l2ilist[slot] = (int32_t)yy;
    }
  }
}

// liquid cells turned interface: M = rho, with rho and u the moments of their
// post-collision populations
template <int D, int P>
__global__ __launch_bounds__(256) void k_l2i_init(KP p, DA d, int cur) {
  using R = typename Prec<P>::R;
  using SF = typename Prec<P>::SF;
  using L = Lat<D>;
  const SF *f = (const SF *)d.f[cur];
  LIST_LOOP(k, d.cnt + C_L2I) {
    if (k < *(volatile int32_t *)(d.cnt + C_L2I)) {
      const int64_t n = d.l2ilist[k];
      R fv[L::Q];
#pragma unroll
      for (int i = 0; i < L::Q; ++i) fv[i] = FCodec<P, D>::dec(f[(int64_t)i * p.Np + n], i);
      R r, dr, ux, uy, uz;
      Arith<D, P>::mom(fv, r, dr, ux, uy, uz);
      ((R *)d.rho)[n] = r;
      ((R *)d.ux)[n] = ux;
      ((R *)d.uy)[n] = uy;
      if (D == 3) ((R *)d.uz)[n] = uz;
      ((R *)d.M)[n] = r;
    }
  }
}

// (c) apply the new types; (e) an emptied cell hands its dissolved gas to its bubble
template <int D, int P>
__global__ __launch_bounds__(256) void k_apply(KP p, DA d, int cur) {
  using SG = typename Prec<P>::SG;
  using R = typename Prec<P>::R;
  using L = Lat<D>;
  const SG *g = (const SG *)d.g[cur];
  const int nI = *(volatile int32_t *)(d.cnt + C_I);
  const int nNI = *(volatile int32_t *)(d.cnt + C_NI);
  const int nL = *(volatile int32_t *)(d.cnt + C_L2I);
  const int64_t total = (int64_t)nI + nNI + nL;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < ((total + 63) & ~(int64_t)63);
       k += (int64_t)gridDim.x * blockDim.x) {
    bool emptied = false;
    int32_t lab = 0;
    R sg = R(0);
    if (k < nI) {
      const int64_t n = d.ilist[k];
      const uint8_t cl = d.cflag[n];
      if (cl & CF_FILL) {
        d.type[n] = (d.type[n] & ~TMASK) | TL;
        d.label[n] = NOLAB;
      } else if (cl & CF_EMPTY) {
        d.type[n] = (d.type[n] & ~TMASK) | TG;
        emptied = true;
        lab = d.label[n];
        R gv[L::Qg], dc;
#pragma unroll
        for (int i = 0; i < L::Qg; ++i) gv[i] = GCodec<P>::dec(g[(int64_t)i * p.Np + n], p);
        sg = Arith<D, P>::conc(gv, R(p.c0), dc);
      }
    } else if (k < total) {
      const int64_t n = k < (int64_t)nI + nNI ? d.nilist[k - nI] : d.l2ilist[k - nI - nNI];
      d.type[n] = (d.type[n] & ~TMASK) | TI;
    }
    wave_fx_add(d.gam, emptied && lab >= 0 && lab < p.cap, lab, fx3((double)sg), d.gam0);
  }
}

// (d) a new interface cell from gas takes the mean density and velocity of its liquid
// and old-interface neighbours (moments of their post-collision populations), the
// equilibrium populations of that state, M = 0, and dissolved gas at the Henry value of
// its bubble, which the bubble gives up
template <int D, int P>
__global__ __launch_bounds__(256) void k_ni_init(KP p, DA d, int cur) {
  using R = typename Prec<P>::R;
  using SF = typename Prec<P>::SF;
  using SG = typename Prec<P>::SG;
  using L = Lat<D>;
  SF *f = (SF *)d.f[cur];
  SG *g = (SG *)d.g[cur];
  LIST_LOOP(k, d.cnt + C_NI) {
    bool act = false;
    int32_t lab = 0;
    R sg = R(0);
    if (k < *(volatile int32_t *)(d.cnt + C_NI)) {
      act = true;
      const int64_t n = d.nilist[k];
      int x, y, z;
      cell_xyz(p, n, x, y, z);
      R sr = R(0), sdr = R(0), sx = R(0), sy = R(0), sz = R(0);
      int cnt = 0;
      for (int i = 1; i < L::Q; ++i) {
        const int64_t yy = nb_index(p, x, y, z, L::ex[i], L::ey[i], L::ez[i]);
        const int ty = d.type[yy] & TMASK;
        if ((ty != TL && ty != TI) || (d.cflag[yy] & CF_NEWI)) continue;
        R fv[L::Q];
#pragma unroll
        for (int q = 0; q < L::Q; ++q) fv[q] = FCodec<P, D>::dec(f[(int64_t)q * p.Np + yy], q);
        R r, dr, a, b, c;
        Arith<D, P>::mom(fv, r, dr, a, b, c);
        sr = sr + r;
        sdr = sdr + dr;
        sx = sx + a;
        sy = sy + b;
        sz = sz + c;
        cnt++;
      }
      R rb = R(1), drb = R(0), ubx = R(0), uby = R(0), ubz = R(0);
      if (cnt > 0) {
        rb = sr / R(cnt);
        if constexpr (P != 0) {
          drb = sdr / R(cnt);
          rb = R(1) + drb;
        }
        ubx = sx / R(cnt);
        uby = sy / R(cnt);
        ubz = sz / R(cnt);
      }
      const R uu = usq<D, R>(ubx, uby, ubz);
#pragma unroll
      for (int i = 0; i < L::Q; ++i)
        f[(int64_t)i * p.Np + n] = FCodec<P, D>::enc(Arith<D, P>::eq(i, rb, drb, ubx, uby, ubz, uu), i);
      lab = d.label[n];
      double pb = p.p_atm;
      if (lab >= 0 && lab < p.cap && d.balive[lab]) pb = d.bp[lab];
      else raise_status(d.status, ST_BADLABEL);
      const R cH = R(p.kH) * R(pb);
      R gv[L::Qg], dcz;
#pragma unroll
      for (int i = 0; i < L::Qg; ++i) {
        // the bubble gives up exactly the gas that is stored
        const SG st = GCodec<P>::enc(Arith<D, P>::geqv(i, cH, cH - R(p.c0), ubx, uby, ubz), p);
        g[(int64_t)i * p.Np + n] = st;
        gv[i] = GCodec<P>::dec(st, p);
      }
      sg = Arith<D, P>::conc(gv, R(p.c0), dcz);
      ((R *)d.rho)[n] = rb;
      ((R *)d.ux)[n] = ubx;
      ((R *)d.uy)[n] = uby;
      if (D == 3) ((R *)d.uz)[n] = ubz;
      ((R *)d.M)[n] = R(0);
    }
    wave_fx_add(d.gam, act && lab >= 0 && lab < p.cap, lab, fx3(-(double)sg), d.gam0);
  }
}

// excess of each converted cell: e = M* - rho (filled) or M* (emptied), split over its
// interface neighbours under the new types; none -> lost-liquid ledger
template <int D, int P>
__global__ __launch_bounds__(256) void k_excess_prep(KP p, DA d) {
  using R = typename Prec<P>::R;
  using L = Lat<D>;
  LIST_LOOP(k, d.cnt + C_I) {
    bool lost = false;
    R e = R(0);
    if (k < *(volatile int32_t *)(d.cnt + C_I)) {
      const int64_t n = d.ilist[k];
      const uint8_t cl = d.cflag[n];
      if (cl & (CF_FILL | CF_EMPTY)) {
        const R Ms = ((const R *)d.M)[n];
        e = (cl & CF_FILL) ? Ms - ((const R *)d.rho)[n] : Ms;
        int x, y, z;
        cell_xyz(p, n, x, y, z);
        int cnt = 0;
        for (int i = 1; i < L::Q; ++i) {
          const int64_t yy = nb_index(p, x, y, z, L::ex[i], L::ey[i], L::ez[i]);
          if ((d.type[yy] & TMASK) == TI) cnt++;
        }
        if (cnt > 0) ((R *)d.exc)[n] = e / R(cnt);
        else lost = true;
      }
    }
    wave_fx_add(d.led, lost, 0, fx3((double)e));
  }
}

// every interface cell of the new types gathers the shares of its converted
// neighbours in ascending direction order; alpha = M / rho
template <int D, int P>
__global__ __launch_bounds__(256) void k_excess_gather(KP p, DA d) {
  using R = typename Prec<P>::R;
  using L = Lat<D>;
  const int nI = *(volatile int32_t *)(d.cnt + C_I);
  const int nNI = *(volatile int32_t *)(d.cnt + C_NI);
  const int nL = *(volatile int32_t *)(d.cnt + C_L2I);
  const int64_t total = (int64_t)nI + nNI + nL;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t n = k < nI ? d.ilist[k] : (k < (int64_t)nI + nNI ? d.nilist[k - nI] : d.l2ilist[k - nI - nNI]);
    if (k < nI && (d.cflag[n] & (CF_FILL | CF_EMPTY))) continue;
    int x, y, z;
    cell_xyz(p, n, x, y, z);
    R acc = ((const R *)d.M)[n];
    for (int i = 1; i < L::Q; ++i) {
      const int64_t yy = nb_index(p, x, y, z, L::ex[i], L::ey[i], L::ez[i]);
      if (d.cflag[yy] & (CF_FILL | CF_EMPTY)) acc = acc + ((const R *)d.exc)[yy];
    }
    ((R *)d.M)[n] = acc;
    ((R *)d.alpha)[n] = acc / ((const R *)d.rho)[n];
  }
}

// conversion flags are cleared once the new state is complete
__global__ __launch_bounds__(256) void k_clear_conv_flags(DA d) {
  const int nI = *(volatile int32_t *)(d.cnt + C_I);
  const int nNI = *(volatile int32_t *)(d.cnt + C_NI);
  const int nL = *(volatile int32_t *)(d.cnt + C_L2I);
  const int64_t total = (int64_t)nI + nNI + nL;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t n = k < nI ? d.ilist[k] : (k < (int64_t)nI + nNI ? d.nilist[k - nI] : d.l2ilist[k - nI - nNI]);
    d.cflag[n] = 0;
  }
}

// Whether this step's conversions can have changed the connected components of the gas
// and interface cells. Only cells that fill (leave the set) and liquid cells that turn
// interface (join it) change the set.
//  - A joining cell whose gas / interface neighbours all carry its own id merges nothing.
//  - A leaving cell of the atmosphere (next to a gas / interface cell with id 0) changes
//    nothing: every piece of the atmosphere keeps id 0, and no bubble touches it.
//  - Another leaving cell x: let K be the leaving cells connected to x inside its 3^d block
//    (none of them with a leaving lattice neighbour outside that block, else the test
//    fails), and R the remaining gas / interface lattice neighbours of K. If R is not
//    empty and connected inside the 5^d window around x without the leaving cells, every
//    path through K has a detour, so nothing splits or disappears.
// When any cell fails, the flag is set and the full labelling runs; otherwise ids, merges
// and splits stay as they were.
struct Bits128 {
  uint64_t w[2];
  __device__ bool get(int q) const { return (w[q >> 6] >> (q & 63)) & 1ull; }
  __device__ void set(int q) { w[q >> 6] |= 1ull << (q & 63); }
};

__device__ __forceinline__ Bits128 shift128(Bits128 v, int s) {
  Bits128 o;
  if (s > 0) {
    o.w[0] = v.w[0] << s;
    o.w[1] = (v.w[1] << s) | (v.w[0] >> (64 - s));
  } else if (s < 0) {
    const int t = -s;
    o.w[0] = (v.w[0] >> t) | (v.w[1] << (64 - t));
    o.w[1] = v.w[1] >> t;
  } else {
    o = v;
  }
  return o;
}

// One step of lattice dilation of a window mask, computed by the whole wave: lane i < Q-1
// moves the set along direction i+1 (positions whose step leaves the window are dropped
// by the lane's mask `valid`), and the lanes' results are OR-ed together.
__device__ __forceinline__ Bits128 dilate(Bits128 v, Bits128 valid, int shift, bool active) {
  Bits128 m = {{v.w[0] & valid.w[0], v.w[1] & valid.w[1]}};
  Bits128 o = active ? shift128(m, shift) : Bits128{{0, 0}};
  for (int off = 32; off > 0; off >>= 1) {
    o.w[0] |= __shfl_xor(o.w[0], off);
    o.w[1] |= __shfl_xor(o.w[1], off);
  }
  o.w[0] |= v.w[0];
  o.w[1] |= v.w[1];
  return o;
}

// flood of `seed` inside `allowed` (wave-uniform loop)
__device__ __forceinline__ Bits128 flood(Bits128 seed, Bits128 allowed, Bits128 valid, int shift, bool active) {
  Bits128 r = seed;
  for (int it = 0; it < 16; ++it) {
    Bits128 n = dilate(r, valid, shift, active);
    n.w[0] &= allowed.w[0];
    n.w[1] &= allowed.w[1];
    n.w[0] |= seed.w[0];
    n.w[1] |= seed.w[1];
    if (n.w[0] == r.w[0] && n.w[1] == r.w[1]) break;
    r = n;
  }
  return r;
}

// The window test of one leaving cell, by the whole wave, from the masks of gas /
// interface cells (g) and leaving cells (f) of its 5^d window (position dx + 5 dy +
// 25 dz, offsets -2..2); true when the cell may split or remove a component. K: the
// leaving cells connected to the centre inside its 3^d block; R: the gas / interface
// lattice neighbours of K.
template <int D>
__device__ bool window_changes(Bits128 g, Bits128 f) {
  using L = Lat<D>;
  constexpr int W = 5, NW = D == 3 ? 125 : 25, CEN = D == 3 ? 62 : 12;
  const int lane = lane_id();
  const bool active = lane < L::Q - 1;
  const int i = active ? lane + 1 : 1;
  const int shift = L::ex[i] + W * L::ey[i] + W * W * L::ez[i];
  Bits128 valid = {{0, 0}}, inner = {{0, 0}};
  for (int q = 0; q < NW; ++q) {
    const int dx = q % W - 2, dy = (q / W) % W - 2, dz = D == 3 ? q / (W * W) - 2 : 0;
    const int ax = dx + L::ex[i], ay = dy + L::ey[i], az = dz + L::ez[i];
    if (ax >= -2 && ax <= 2 && ay >= -2 && ay <= 2 && az >= -2 && az <= 2) valid.w[q >> 6] |= 1ull << (q & 63);
    if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1) inner.w[q >> 6] |= 1ull << (q & 63);
  }
  Bits128 cen = {{0, 0}};
  cen.w[CEN >> 6] = 1ull << (CEN & 63);
  Bits128 fin = {{f.w[0] & inner.w[0], f.w[1] & inner.w[1]}};
  fin.w[CEN >> 6] |= 1ull << (CEN & 63);
  const Bits128 K = flood(cen, fin, valid, shift, active);
  const Bits128 DK = dilate(K, valid, shift, active);
  // a leaving neighbour of K outside the block: the cluster may continue beyond the window
  if ((DK.w[0] & f.w[0] & ~inner.w[0]) || (DK.w[1] & f.w[1] & ~inner.w[1])) return true;
  const Bits128 R = {{DK.w[0] & g.w[0], DK.w[1] & g.w[1]}};
  if (!R.w[0] && !R.w[1]) return true;
  Bits128 seed = {{0, 0}};
  if (R.w[0]) seed.w[0] = R.w[0] & (~R.w[0] + 1);
  else seed.w[1] = R.w[1] & (~R.w[1] + 1);
  const Bits128 reach = flood(seed, g, valid, shift, active);
  return (R.w[0] & ~reach.w[0]) || (R.w[1] & ~reach.w[1]);
}

template <int D>
__global__ __launch_bounds__(256) void k_topo_check(KP p, DA d) {
  using L = Lat<D>;
  constexpr int W = 5, NW = D == 3 ? 125 : 25;
  __shared__ int s_cand[256];
  __shared__ int s_nc;
  if (threadIdx.x == 0) s_nc = 0;
  __syncthreads();
  const int nI = *(volatile int32_t *)(d.cnt + C_I);
  const int nL = *(volatile int32_t *)(d.cnt + C_L2I);
  const int64_t total = (int64_t)nI + nL;
  // a periodic axis shorter than the window would wrap it onto itself: full labelling
  bool change = total > 0 && ((p.per[0] && p.nx < W) || (p.per[1] && p.ny < W) || (D == 3 && p.per[2] && p.nz < W));
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total && !change; k += (int64_t)gridDim.x * blockDim.x) {
    if (k >= nI) {
      const int64_t n = d.l2ilist[k - nI];
      const int32_t lx = d.label[n];
      int x, y, z;
      cell_xyz(p, n, x, y, z);
      for (int i = 1; i < L::Q; ++i) {
        const int64_t yy = nb_index_or_none(p, x, y, z, L::ex[i], L::ey[i], L::ez[i]);
        if (yy < 0) continue;
        const int t = d.type[yy] & TMASK;
        if ((t == TG || t == TI) && d.label[yy] != lx) change = true;
      }
      continue;
    }
    const int64_t n = d.ilist[k];
    if (!(d.cflag[n] & CF_FILL)) continue;
    int x, y, z;
    cell_xyz(p, n, x, y, z);
    // a leaving cell of the atmosphere (a gas / interface neighbour with id 0) changes no
    // bubble: every piece of the atmosphere keeps id 0 and no bubble touches it
    bool atm = false;
    for (int i = 1; i < L::Q; ++i) {
      const int64_t yy = nb_index_or_none(p, x, y, z, L::ex[i], L::ey[i], L::ez[i]);
      if (yy < 0) continue;
      const int t = d.type[yy] & TMASK;
      if ((t == TG || t == TI) && d.label[yy] == 0) atm = true;
    }
    if (atm) continue;
    const int c = atomicAdd(&s_nc, 1);  // LDS
    if (c < 256) s_cand[c] = (int)n;
    else change = true;
  }
  __syncthreads();
  // window tests, one wave per candidate: the lanes load the window, lane 0 decides
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int nc = s_nc < 256 ? s_nc : 256;
  for (int c = wave; c < nc; c += 4) {
    const int64_t n = s_cand[c];
    int x, y, z;
    cell_xyz(p, n, x, y, z);
    Bits128 g, f;
    for (int h = 0; h < 2; ++h) {
      const int q = lane + 64 * h;
      bool gq = false, fq = false;
      if (q < NW) {
        const int dx = q % W - 2, dy = (q / W) % W - 2, dz = D == 3 ? q / (W * W) - 2 : 0;
        const int64_t yy = nb_index_or_none(p, x, y, z, dx, dy, dz);
        if (yy >= 0) {
          const int t = d.type[yy] & TMASK;
          gq = t == TG || t == TI;
          fq = !gq && (d.cflag[yy] & CF_FILL);
        }
      }
      g.w[h] = __ballot(gq);
      f.w[h] = __ballot(fq);
    }
    if (window_changes<D>(g, f) && lane == 0) change = true;
  }
  if (__ballot(change) != 0 && lane_id() == 0) d.cnt[C_TOPO] = 1;
}

template <int D, int P>
void Ops<D, P>::convert(Ctx &c, hipStream_t s) {
  const unsigned nb = list_blocks(c);
  const int cur = c.cur;  // buffer holding this step's post-collision populations
  hipLaunchKernelGGL((k_fill_scatter<D>), dim3(nb), dim3(256), 0, s, c.kp, c.d);
  hipLaunchKernelGGL((k_empty_scatter<D>), dim3(nb), dim3(256), 0, s, c.kp, c.d);
  hipLaunchKernelGGL((k_l2i_init<D, P>), dim3(nb), dim3(256), 0, s, c.kp, c.d, cur);
  hipLaunchKernelGGL((k_apply<D, P>), dim3(nb), dim3(256), 0, s, c.kp, c.d, cur);
  hipLaunchKernelGGL((k_topo_check<D>), dim3(nb), dim3(256), 0, s, c.kp, c.d);
  hipLaunchKernelGGL((k_ni_init<D, P>), dim3(nb), dim3(256), 0, s, c.kp, c.d, cur);
  hipLaunchKernelGGL((k_excess_prep<D, P>), dim3(nb), dim3(256), 0, s, c.kp, c.d);
  hipLaunchKernelGGL((k_excess_gather<D, P>), dim3(nb), dim3(256), 0, s, c.kp, c.d);
  hipLaunchKernelGGL(k_clear_conv_flags, dim3(nb), dim3(256), 0, s, c.d);
}

#define MF_INST(D, P) template void Ops<D, P>::convert(Ctx &, hipStream_t);
MF_FOR_ALL(MF_INST)

}  // namespace mf

// Cell-type conversion and excess-mass redistribution (Sec. 2.1, last paragraph):
// interface cells with alpha >= 1 become liquid, with alpha <= 0 become gas; the
// surplus or shortage is spread equally over the neighbouring interface cells.
// All passes run over compact lists (interface cells of the step, and the cells that
// change type) and are pull gathers or idempotent flag scatters, so their result does
// not depend on thread order.
#include "lbm_math.h"

namespace mf {

// slots for n entries of each lane, taken with one atomic per wave (called by the whole
// wave); returns the lane's first slot
__device__ __forceinline__ int wave_reserve(int32_t *counter, int n) {
  const int lane = lane_id();
  int incl = n;
  for (int o = 1; o < 64; o <<= 1) {
    const int a = __shfl_up(incl, o);
    if (lane >= o) incl += a;
  }
  const int tot = __shfl(incl, 63);
  int base = 0;
  if (tot > 0) {
    if (lane == 63) base = atomicAdd(counter, tot);
    base = __shfl(base, 63);
  }
  return base + incl - n;
}

// (a) every gas neighbour of a filled cell becomes a new interface cell; an emptied
// neighbour of a filled cell stays an interface cell
template <int D>
__device__ __forceinline__ void b_fill_scatter(const GridPos &gp, KP p, DA d) {
  using L = Lat<D>;
  SPREAD_LOOP(k, d.cnt + C_CONV) {
    bool act = false;
    int64_t n = 0;
    if (k < *(volatile int32_t *)(d.cnt + C_CONV)) {
      n = d.clist[k];
      act = (d.cflag[n] & CF_FILL) != 0;
    }
    if (!__ballot(act)) continue;  // wave-uniform
    // neighbour types first (all loads in flight together), then the flag updates, then
    // the list appends
    int64_t yy[L::Q];
    int ty[L::Q];
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
      yy[i] = 0;
      ty[i] = TW;
    }
    if (act) {
      int x, y, z;
      cell_xyz(p, n, x, y, z);
#pragma unroll
      for (int i = 1; i < L::Q; ++i) yy[i] = nb_index(p, x, y, z, L::ex[i], L::ey[i], L::ez[i]);
#pragma unroll
      for (int i = 1; i < L::Q; ++i) ty[i] = d.type[yy[i]] & TMASK;
    }
    uint32_t old[L::Q];
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
      old[i] = CF_NEWI;
      if (ty[i] == TG) old[i] = flag_or(d.cflag, yy[i], CF_NEWI);
      else if (ty[i] == TI && (d.cflag[yy[i]] & CF_EMPTY)) flag_clear(d.cflag, yy[i], CF_EMPTY);
    }
    int na = 0;
#pragma unroll
    for (int i = 1; i < L::Q; ++i) na += (old[i] & CF_NEWI) ? 0 : 1;
    int at = wave_reserve(d.cnt + C_NI, na);
#pragma unroll
    for (int i = 1; i < L::Q; ++i)
      if (!(old[i] & CF_NEWI)) d.nilist[at++] = (int32_t)yy[i];
  }
}
template <int D>
__global__ __launch_bounds__(256) void k_fill_scatter(KP p, DA d) {
  b_fill_scatter<D>(GridPos::hw(), p, d);
}

// (b) every liquid neighbour of a (still) emptied cell becomes an interface cell and
// takes the smallest bubble id among its emptied neighbours
template <int D>
__device__ __forceinline__ void b_empty_scatter(const GridPos &gp, KP p, DA d) {
  using L = Lat<D>;
  SPREAD_LOOP(k, d.cnt + C_CONV) {
    bool act = false;
    int64_t n = 0;
    if (k < *(volatile int32_t *)(d.cnt + C_CONV)) {
      n = d.clist[k];
      act = (d.cflag[n] & CF_EMPTY) != 0;
    }
    if (!__ballot(act)) continue;  // wave-uniform
    int64_t yy[L::Q];
    int ty[L::Q];
    int32_t lab = 0;
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
      yy[i] = 0;
      ty[i] = TW;
    }
    if (act) {
      int x, y, z;
      cell_xyz(p, n, x, y, z);
      lab = d.label[n];
#pragma unroll
      for (int i = 1; i < L::Q; ++i) yy[i] = nb_index(p, x, y, z, L::ex[i], L::ey[i], L::ez[i]);
#pragma unroll
      for (int i = 1; i < L::Q; ++i) ty[i] = d.type[yy[i]] & TMASK;
    }
    uint32_t old[L::Q];
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
      old[i] = CF_L2I;
      if (ty[i] == TL) {
        atomicMin((unsigned int *)&d.label[yy[i]], (unsigned int)lab);
        old[i] = flag_or(d.cflag, yy[i], CF_L2I);
      }
    }
    int na = 0;
#pragma unroll
    for (int i = 1; i < L::Q; ++i) na += (old[i] & CF_L2I) ? 0 : 1;
    int at = wave_reserve(d.cnt + C_L2I, na);
#pragma unroll
    for (int i = 1; i < L::Q; ++i)
      if (!(old[i] & CF_L2I)) d.l2ilist[at++] = (int32_t)yy[i];
  }
}
template <int D>
__global__ __launch_bounds__(256) void k_empty_scatter(KP p, DA d) {
  b_empty_scatter<D>(GridPos::hw(), p, d);
}

// (c) apply the new types; (e) an emptied cell hands its dissolved gas to its bubble; a
// liquid cell turned interface takes M = rho, with rho and u the moments of its
// post-collision populations
template <int D, int P>
__device__ __forceinline__ void b_apply(const GridPos &gp, KP p, DA d, int cur) {
  using SG = typename Prec<P>::SG;
  using SF = typename Prec<P>::SF;
  using R = typename Prec<P>::R;
  using L = Lat<D>;
  const SG *g = (const SG *)d.g[cur];
  const SF *f = (const SF *)d.f[cur];
  const int nI = *(volatile int32_t *)(d.cnt + C_CONV);  // the cells that fill or empty
  const int nNI = *(volatile int32_t *)(d.cnt + C_NI);
  const int nL = *(volatile int32_t *)(d.cnt + C_L2I);
  const int64_t total = (int64_t)nI + nNI + nL;
  SPREAD_LOOP_N(k, total) {
    bool emptied = false;
    int32_t lab = 0;
    R sg = R(0);
    if (k < nI) {
      const int64_t n = d.clist[k];
      const uint8_t cl = d.cflag[n];
      if (cl & CF_FILL) {
        d.type[n] = (d.type[n] & ~TMASK) | TL;
        d.parent[n] = d.label[n];  // the former id, for the topology test
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
      const bool l2i = k >= (int64_t)nI + nNI;
      const int64_t n = l2i ? d.l2ilist[k - nI - nNI] : d.nilist[k - nI];
      d.type[n] = (d.type[n] & ~TMASK) | TI;
      if (l2i) {
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
    wave_fx_add_runs(d.gam, emptied && !p.flux_paper && lab >= 0 && lab < p.cap, lab, fx3((double)sg), d.gam0);
    wave_count_add(d.bng, emptied && lab > 0 && lab < p.cap, lab, 1);  // one more gas cell
  }
}
template <int D, int P>
__global__ __launch_bounds__(256) void k_apply(KP p, DA d, int cur) {
  b_apply<D, P>(GridPos::hw(), p, d, cur);
}

// (d) a new interface cell from gas takes the mean density and velocity of its liquid
// and old-interface neighbours (moments of their post-collision populations), the
// equilibrium populations of that state, M = 0, and dissolved gas at the Henry value of
// its bubble, which the bubble gives up
template <int D, int P>
__device__ __forceinline__ void b_ni_init(const GridPos &gp, KP p, DA d, int cur) {
  using R = typename Prec<P>::R;
  using SF = typename Prec<P>::SF;
  using SG = typename Prec<P>::SG;
  using L = Lat<D>;
  SF *f = (SF *)d.f[cur];
  SG *g = (SG *)d.g[cur];
  SPREAD_LOOP(k, d.cnt + C_NI) {
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
    wave_fx_add_runs(d.gam, act && !p.flux_paper && lab >= 0 && lab < p.cap, lab, fx3(-(double)sg), d.gam0);
    wave_count_add(d.bng, act && lab > 0 && lab < p.cap, lab, -1);  // one gas cell fewer
  }
}
template <int D, int P>
__global__ __launch_bounds__(256) void k_ni_init(KP p, DA d, int cur) {
  b_ni_init<D, P>(GridPos::hw(), p, d, cur);
}

// excess of each converted cell: e = M* - rho (filled) or M* (emptied), split over its
// interface neighbours under the new types; none -> lost-liquid ledger
template <int D, int P>
__device__ __forceinline__ void b_excess_prep(const GridPos &gp, KP p, DA d) {
  using R = typename Prec<P>::R;
  using L = Lat<D>;
  SPREAD_LOOP(k, d.cnt + C_CONV) {
    bool lost = false;
    R e = R(0);
    if (k < *(volatile int32_t *)(d.cnt + C_CONV)) {
      const int64_t n = d.clist[k];
      const uint8_t cl = d.cflag[n];
      if (cl & (CF_FILL | CF_EMPTY)) {
        const R Ms = ((const R *)d.M)[n];
        e = (cl & CF_FILL) ? Ms - ((const R *)d.rho)[n] : Ms;
        int x, y, z;
        cell_xyz(p, n, x, y, z);
        int cnt = 0;
        int64_t yy[L::Q];
        int ty[L::Q];
#pragma unroll
        for (int i = 1; i < L::Q; ++i) yy[i] = nb_index(p, x, y, z, L::ex[i], L::ey[i], L::ez[i]);
#pragma unroll
        for (int i = 1; i < L::Q; ++i) ty[i] = d.type[yy[i]] & TMASK;
#pragma unroll
        for (int i = 1; i < L::Q; ++i) {
          if (ty[i] == TI) {
            cnt++;
            // it gathers a share
            atomicOr((uint32_t *)(d.cflag + (yy[i] & ~(int64_t)3)), CF_EXNB << (8 * (int)(yy[i] & 3)));
          }
        }
        if (cnt > 0) ((R *)d.exc)[n] = e / R(cnt);
        else lost = true;
      }
    }
    wave_fx_add(d.led, lost, 0, fx3((double)e));
  }
}
template <int D, int P>
__global__ __launch_bounds__(256) void k_excess_prep(KP p, DA d) {
  b_excess_prep<D, P>(GridPos::hw(), p, d);
}

// Every interface cell of the new types gathers the shares of its converted neighbours in
// ascending direction order; alpha = M / rho. With the learned curvature, the pass also
// writes the stencil word of every list cell (converted ones included), whose type, fill
// fraction or id may have changed this step; the labelling that follows changes ids only
// when it relabels, and then rewrites the words of the cells it relabels itself. For every
// bubble the labelling will not relabel (all of them when the topology test passed), the
// same pass adds each interface cell's volume share 1 - alpha to its bubble (fixed point;
// the gas cells are counted apart),
// and it clears the conversion flags of the cells it visits (the converted cells, whose
// flags its neighbours read here, are cleared by the next pass).
template <int D, int P>
__device__ __forceinline__ void b_excess_gather(const GridPos &gp, KP p, DA d) {
  using R = typename Prec<P>::R;
  using L = Lat<D>;
  const int nI = *(volatile int32_t *)(d.cnt + C_I);
  const int nNI = *(volatile int32_t *)(d.cnt + C_NI);
  const int nL = *(volatile int32_t *)(d.cnt + C_L2I);
  // the volumes of the bubbles the labelling does not relabel (all of them on a step
  // without topology change, the unmarked ones on a partial relabelling)
  const bool topo = *(volatile int32_t *)(d.cnt + C_TOPO) != 0;
  const bool fast = !topo || !*(volatile int32_t *)(d.cnt + C_FULL);
  const int64_t total = (int64_t)nI + nNI + nL;
  for (int64_t k = (int64_t)gp.bid * blockDim.x + threadIdx.x; k < ((total + 63) & ~(int64_t)63);
       k += (int64_t)gp.nblk * blockDim.x) {
    bool act = false;
    int lab = 0;
    Fx3 v = {0, 0, 0};
    if (k < total) {
      const int64_t n = k < nI ? d.ilist[k] : (k < (int64_t)nI + nNI ? d.nilist[k - nI] : d.l2ilist[k - nI - nNI]);
      const uint8_t cl = d.cflag[n];
      if (d.sword && k < nI && (cl & (CF_FILL | CF_EMPTY)))
        d.sword[n] = stencil_word<R>(d.type[n], ((const R *)d.alpha)[n], d.label[n]);
      if (!(k < nI && (cl & (CF_FILL | CF_EMPTY)))) {
        R acc = ((const R *)d.M)[n];
        if (cl & CF_EXNB) {  // next to a converted cell
          int x, y, z;
          cell_xyz(p, n, x, y, z);
          for (int i = 1; i < L::Q; ++i) {
            const int64_t yy = nb_index(p, x, y, z, L::ex[i], L::ey[i], L::ez[i]);
            if (d.cflag[yy] & (CF_FILL | CF_EMPTY)) acc = acc + ((const R *)d.exc)[yy];
          }
          ((R *)d.M)[n] = acc;
        }
        const R al = acc / ((const R *)d.rho)[n];
        ((R *)d.alpha)[n] = al;
        if (cl) d.cflag[n] = 0;  // most list cells carry no flag: their lines stay clean
        if (d.sword) d.sword[n] = stencil_word<R>(d.type[n], al, d.label[n]);
        if (fast) {
          lab = d.label[n];
          if (lab > 0 && lab < p.cap && !(topo && d.aff[lab])) {
            act = true;
            v = fx3((double)(R(1) - al));
          }
        }
      }
    }
    if (fast) wave_fx_add_runs(d.vacc, act, lab, v);
  }
}
template <int D, int P>
__global__ __launch_bounds__(256) void k_excess_gather(KP p, DA d) {
  b_excess_gather<D, P>(GridPos::hw(), p, d);
}

// the flags of the cells that filled or emptied
__device__ __forceinline__ void b_conv_clear(const GridPos &gp, DA d) {
  SPREAD_LOOP(k, d.cnt + C_CONV) {
    if (k < *(volatile int32_t *)(d.cnt + C_CONV)) d.cflag[d.clist[k]] = 0;
  }
}
__global__ __launch_bounds__(256) void k_conv_clear(DA d) {
  b_conv_clear(GridPos::hw(), d);
}

// Whether this step's conversions can have changed the connected components of the gas
// and interface cells. Only cells that fill (leave the set) and liquid cells that turn
// interface (join it) change the set.
//  - A joining cell whose gas / interface neighbours all carry its own id merges nothing.
//  - A leaving cell of the atmosphere (next to a gas / interface cell with id 0) changes
//    nothing: every piece of the atmosphere keeps id 0, and no bubble touches it.
//  - Another leaving cell x, in the window of 7^d cells centred on it: let K be the leaving
//    cells connected to x inside the inner 5^d block (none of them with a leaving lattice
//    neighbour outside that block, else the test fails), and R the remaining gas /
//    interface lattice neighbours of K. If R is not empty and connected inside the window
//    without the leaving cells, every path through K has a detour, so nothing splits or
//    disappears.
// When any cell fails, the flag is set and the ids of the components around it are marked:
// the labelling then relabels the cells of the marked ids only (every component a
// conversion can merge, split or remove carries one of them), and every other bubble keeps
// its id, its gas and its cells.
//
// The window is held one x-row per lane (W bits; lane = (dy + H) + W (dz + H)), so a step
// of lattice dilation is two shifts along x and a few shuffles for the rows around.
template <int D> struct RowWindow {
  static constexpr int W = 7, H = W / 2;
  static constexpr int NR = D == 3 ? W * W : W;  // rows in the window
  static constexpr uint32_t XM = (1u << W) - 1;
  static constexpr uint32_t XIN = XM & ~1u & ~(1u << (W - 1));  // the inner x range
  int ry = 0, rz = 0;
  bool row = false, in_row = false;
  __device__ RowWindow() {
    const int lane = lane_id();
    row = lane < NR;
    ry = lane % W - H;
    rz = D == 3 ? lane / W - H : 0;
    in_row = row && ry > -H && ry < H && (D == 2 || (rz > -H && rz < H));
  }
  // the row at (ry + dy, rz + dz), empty outside the window
  __device__ uint32_t at(uint32_t v, int dy, int dz) const {
    const int y = ry + dy, z = rz + dz;
    const bool ok = row && y >= -H && y <= H && z >= -H && z <= H;
    const int src = ok ? (y + H) + W * (z + H) : lane_id();
    const uint32_t t = __shfl(v, src);
    return ok ? t : 0u;
  }
  __device__ static uint32_t xs(uint32_t r) { return ((r << 1) | (r >> 1)) & XM; }
  // one step of dilation along the lattice directions of D2Q9 / D3Q19
  __device__ uint32_t dilate(uint32_t v) const {
    uint32_t o = v | xs(v);
    if (D == 2) {
      const uint32_t a = at(v, -1, 0), b = at(v, 1, 0);
      o |= a | b | xs(a) | xs(b);
    } else {
      const uint32_t a = at(v, -1, 0), b = at(v, 1, 0), c = at(v, 0, -1), e = at(v, 0, 1);
      o |= a | b | c | e | xs(a) | xs(b) | xs(c) | xs(e);
      o |= at(v, -1, -1) | at(v, 1, -1) | at(v, -1, 1) | at(v, 1, 1);
    }
    return row ? o : 0u;
  }
  // flood of `seed` inside `allowed` (wave-uniform loop)
  __device__ uint32_t flood(uint32_t seed, uint32_t allowed) const {
    uint32_t r = seed;
    for (int it = 0; it < NR * W; ++it) {
      const uint32_t n = (dilate(r) & allowed) | seed;
      if (!__ballot(n != r)) break;
      r = n;
    }
    return r;
  }
  // gas / interface cells (g) and leaving cells (f) of the lane's row around (x, y, z)
  __device__ void load(const KP &p, const DA &d, int x, int y, int z, uint32_t &g, uint32_t &f) const {
    g = f = 0;
    if (!row) return;
#pragma unroll
    for (int b = 0; b < W; ++b) {
      const int64_t yy = nb_index_or_none(p, x, y, z, b - H, ry, rz);
      if (yy < 0) continue;
      const int t = d.type[yy] & TMASK;
      if (t == TG || t == TI) g |= 1u << b;
      else if (d.cflag[yy] & CF_FILL) f |= 1u << b;
    }
  }
  // true when the leaving cell at the centre may split or remove a component
  __device__ bool changes(uint32_t g, uint32_t f) const {
    const uint32_t inner = in_row ? XIN : 0u;
    const uint32_t cen = (row && ry == 0 && rz == 0) ? 1u << H : 0u;
    const uint32_t K = flood(cen, (f & inner) | cen);
    const uint32_t DK = dilate(K);
    if (__ballot((DK & f & ~inner) != 0)) return true;  // the cluster reaches past the block
    const uint32_t R = DK & g;
    const unsigned long long has = __ballot(R != 0);
    if (!has) return true;  // nothing of the set remains next to the cluster
    const int first = __ffsll((long long)has) - 1;
    const uint32_t seed = lane_id() == first ? R & (~R + 1u) : 0u;
    const uint32_t reach = flood(seed, g);
    return __ballot((R & ~reach) != 0) != 0;
  }
};

// marks id lab as one whose component the conversions may have changed (any number of
// threads may mark the same id)
__device__ __forceinline__ void mark_affected(const KP &p, const DA &d, int32_t lab) {
  if (lab > 0 && lab < p.cap) d.aff[lab] = 1;
}

// cheap per-cell tests over the converted cells: joining cells are decided here, filling
// cells that need the window test are listed. A joining cell next to other ids marks them
// and its own; every cell is tested, so that all changed components are marked.
template <int D>
__device__ __forceinline__ void b_topo_check(const GridPos &gp, KP p, DA d) {
  using L = Lat<D>;
  const int nI = *(volatile int32_t *)(d.cnt + C_CONV);  // the cells that fill or empty
  const int nL = *(volatile int32_t *)(d.cnt + C_L2I);
  const int64_t total = (int64_t)nI + nL;
  // a periodic axis shorter than the widest window would wrap it onto itself: full
  // labelling
  constexpr int WMAX = 7;
  bool full = total > 0 && ((p.per[0] && p.nx < WMAX) || (p.per[1] && p.ny < WMAX) || (D == 3 && p.per[2] && p.nz < WMAX));
  bool change = false;
  SPREAD_LOOP_N(k, total) {
    bool cand = false;
    int64_t n = 0;
    if (k < total && !full) {
      // both tests read the types and ids of the lattice neighbours: loaded together
      const bool join = k >= nI;
      n = join ? d.l2ilist[k - nI] : d.clist[k];
      if (join || (d.cflag[n] & CF_FILL)) {
        int x, y, z;
        cell_xyz(p, n, x, y, z);
        int64_t yy[L::Q];
        int t[L::Q];
        int32_t lb[L::Q];
#pragma unroll
        for (int i = 1; i < L::Q; ++i) yy[i] = nb_index_or_none(p, x, y, z, L::ex[i], L::ey[i], L::ez[i]);
#pragma unroll
        for (int i = 1; i < L::Q; ++i) t[i] = yy[i] >= 0 ? d.type[yy[i]] & TMASK : TW;
#pragma unroll
        for (int i = 1; i < L::Q; ++i) lb[i] = yy[i] >= 0 ? d.label[yy[i]] : 0;
        if (join) {
          const int32_t lx = d.label[n];
          bool merges = false;
#pragma unroll
          for (int i = 1; i < L::Q; ++i)
            if ((t[i] == TG || t[i] == TI) && lb[i] != lx) {
              merges = true;
              mark_affected(p, d, lb[i]);
            }
          if (merges) {
            mark_affected(p, d, lx);
            change = true;
          }
        } else {
          // a leaving cell of the atmosphere (a gas / interface neighbour with id 0) changes
          // no bubble: every piece of the atmosphere keeps id 0 and no bubble touches it
          bool atm = false;
#pragma unroll
          for (int i = 1; i < L::Q; ++i)
            if ((t[i] == TG || t[i] == TI) && lb[i] == 0) atm = true;
          cand = !atm;
        }
      }
    }
    const int slot = wave_append_slot(d.cnt + C_TCAND, cand);
    if (cand) {
      if (slot < TCAND_CAP) d.tcand[slot] = (int32_t)n;
      else full = true;  // not tested: every component is relabelled
    }
  }
  if (__ballot(change || full) != 0 && lane_id() == 0) d.cnt[C_TOPO] = 1;
  if (__ballot(full) != 0 && lane_id() == 0) d.cnt[C_FULL] = 1;
}
template <int D>
__global__ __launch_bounds__(256) void k_topo_check(KP p, DA d) {
  b_topo_check<D>(GridPos::hw(), p, d);
}

// the window tests of the listed filling cells, one wave per cell: the lanes load the
// window, the whole wave runs the floods. A cell that fails marks its former id and the
// ids of its gas / interface neighbours.
template <int D>
__device__ __forceinline__ void b_topo_window(const GridPos &gp, KP p, DA d) {
  using L = Lat<D>;
  const int nc = min(*(volatile int32_t *)(d.cnt + C_TCAND), TCAND_CAP);
  const int wave = (int)(gp.bid * (blockDim.x >> 6) + (threadIdx.x >> 6));
  const int nwaves = (int)(gp.nblk * (blockDim.x >> 6));
  if (wave >= nc || *(volatile int32_t *)(d.cnt + C_FULL)) return;  // wave-uniform
  const RowWindow<D> w;
  for (int c = wave; c < nc; c += nwaves) {
    const int64_t n = d.tcand[c];
    int x, y, z;
    cell_xyz(p, n, x, y, z);
    uint32_t g, f;
    w.load(p, d, x, y, z, g, f);
    if (w.changes(g, f) && lane_id() == 0) {
      d.cnt[C_TOPO] = 1;
      mark_affected(p, d, d.parent[n]);
      for (int i = 1; i < L::Q; ++i) {
        const int64_t yy = nb_index_or_none(p, x, y, z, L::ex[i], L::ey[i], L::ez[i]);
        if (yy < 0) continue;
        const int t = d.type[yy] & TMASK;
        if (t == TG || t == TI) mark_affected(p, d, d.label[yy]);
      }
    }
  }
}
template <int D>
__global__ __launch_bounds__(256) void k_topo_window(KP p, DA d) {
  b_topo_window<D>(GridPos::hw(), p, d);
}

// batched forms: the same passes for every domain of a batch, one launch each
template <int D>
__global__ __launch_bounds__(256) void km_fill_scatter(MLaunch ml) {
  MF_MULTI(MK_SHORT)
  b_fill_scatter<D>(gp, m.kp, m.d);
}
template <int D>
__global__ __launch_bounds__(256) void km_empty_scatter(MLaunch ml) {
  MF_MULTI(MK_SHORT)
  b_empty_scatter<D>(gp, m.kp, m.d);
}
template <int D, int P>
__global__ __launch_bounds__(256) void km_apply(MLaunch ml) {
  MF_MULTI(MK_SHORT)
  b_apply<D, P>(gp, m.kp, m.d, m.cur ^ 1);
}
template <int D>
__global__ __launch_bounds__(256) void km_topo_check(MLaunch ml) {
  MF_MULTI(MK_SHORT)
  b_topo_check<D>(gp, m.kp, m.d);
}
template <int D>
__global__ __launch_bounds__(256) void km_topo_window(MLaunch ml) {
  MF_MULTI(MK_TOPOW)
  b_topo_window<D>(gp, m.kp, m.d);
}
template <int D, int P>
__global__ __launch_bounds__(256) void km_ni_init(MLaunch ml) {
  MF_MULTI(MK_SHORT)
  b_ni_init<D, P>(gp, m.kp, m.d, m.cur ^ 1);
}
template <int D, int P>
__global__ __launch_bounds__(256) void km_excess_prep(MLaunch ml) {
  MF_MULTI(MK_SHORT)
  b_excess_prep<D, P>(gp, m.kp, m.d);
}
template <int D, int P>
__global__ __launch_bounds__(256) void km_excess_gather(MLaunch ml) {
  MF_MULTI(MK_LIST)
  b_excess_gather<D, P>(gp, m.kp, m.d);
}
__global__ __launch_bounds__(256) void km_conv_clear(MLaunch ml) {
  MF_MULTI(MK_SHORT)
  b_conv_clear(gp, m.d);
}

// the conversions of every domain of a batch (after its sweep: the post-collision
// populations are in buffer cur ^ 1), in the order of convert()
template <int D, int P>
void Ops<D, P>::convert_multi(const MStep &ms, int part, hipStream_t s) {
  if (part != 2) {
    hipLaunchKernelGGL((km_fill_scatter<D>), dim3(ms.grid[MK_SHORT]), dim3(256), 0, s, ms.at(MK_SHORT));
    hipLaunchKernelGGL((km_empty_scatter<D>), dim3(ms.grid[MK_SHORT]), dim3(256), 0, s, ms.at(MK_SHORT));
    hipLaunchKernelGGL((km_apply<D, P>), dim3(ms.grid[MK_SHORT]), dim3(256), 0, s, ms.at(MK_SHORT));
    hipLaunchKernelGGL((km_ni_init<D, P>), dim3(ms.grid[MK_SHORT]), dim3(256), 0, s, ms.at(MK_SHORT));
  }
  if (part == 1) return;
  hipLaunchKernelGGL((km_topo_check<D>), dim3(ms.grid[MK_SHORT]), dim3(256), 0, s, ms.at(MK_SHORT));
  hipLaunchKernelGGL((km_topo_window<D>), dim3(ms.grid[MK_TOPOW]), dim3(256), 0, s, ms.at(MK_TOPOW));
  hipLaunchKernelGGL((km_excess_prep<D, P>), dim3(ms.grid[MK_SHORT]), dim3(256), 0, s, ms.at(MK_SHORT));
  hipLaunchKernelGGL((km_excess_gather<D, P>), dim3(ms.grid[MK_LIST]), dim3(256), 0, s, ms.at(MK_LIST));
  hipLaunchKernelGGL(km_conv_clear, dim3(ms.grid[MK_SHORT]), dim3(256), 0, s, ms.at(MK_SHORT));
}

// the passes over the short lists (converted cells and their new neighbours) take at most
// four work-groups per CU: their entries are dealt one per wave, and a larger grid only
// costs dispatch time on the step's critical path
static inline unsigned short_blocks(const Ctx &c) {
  const unsigned nb = list_blocks(c);
  return nb < 1024 ? nb : 1024;
}

// the types after the conversions and the populations of the new interface cells: all
// that the next bulk sweep reads
template <int D, int P>
void Ops<D, P>::convert_head(Ctx &c, hipStream_t s) {
  const unsigned ns = short_blocks(c);
  const int cur = c.cur;  // buffer holding this step's post-collision populations
  hipLaunchKernelGGL((k_fill_scatter<D>), dim3(ns), dim3(256), 0, s, c.kp, c.d);
  hipLaunchKernelGGL((k_empty_scatter<D>), dim3(ns), dim3(256), 0, s, c.kp, c.d);
  hipLaunchKernelGGL((k_apply<D, P>), dim3(ns), dim3(256), 0, s, c.kp, c.d, cur);
  hipLaunchKernelGGL((k_ni_init<D, P>), dim3(ns), dim3(256), 0, s, c.kp, c.d, cur);
}

// the topology test, the excess redistribution (fill fractions, stencil words) and the
// flag clear; they read the new types and ids and write nothing the bulk sweep reads
template <int D, int P>
void Ops<D, P>::convert_tail(Ctx &c, hipStream_t s) {
  const unsigned nb = list_blocks(c), ns = short_blocks(c);
  hipLaunchKernelGGL((k_topo_check<D>), dim3(ns), dim3(256), 0, s, c.kp, c.d);
  hipLaunchKernelGGL((k_topo_window<D>), dim3(256), dim3(256), 0, s, c.kp, c.d);
  hipLaunchKernelGGL((k_excess_prep<D, P>), dim3(ns), dim3(256), 0, s, c.kp, c.d);
  hipLaunchKernelGGL((k_excess_gather<D, P>), dim3(nb), dim3(256), 0, s, c.kp, c.d);
  hipLaunchKernelGGL(k_conv_clear, dim3(ns), dim3(256), 0, s, c.d);
  c.sword_fresh = c.d.sword != nullptr;  // the excess pass wrote the list cells' stencil words
}

template <int D, int P>
void Ops<D, P>::convert(Ctx &c, hipStream_t s) {
  convert_head(c, s);
  convert_tail(c, s);
}

#define MF_INST(D, P)                                    \
  template void Ops<D, P>::convert(Ctx &, hipStream_t); \
  template void Ops<D, P>::convert_head(Ctx &, hipStream_t); \
  template void Ops<D, P>::convert_tail(Ctx &, hipStream_t); \
  template void Ops<D, P>::convert_multi(const MStep &, int, hipStream_t);
MF_FOR_ALL(MF_INST)

}  // namespace mf

// Bubble tracking (Sec. 3.5): every step the gas and interface cells are grouped into
// connected components under the lattice neighbourhood (flood fill, here a lock-free
// union-find whose roots are the smallest cell index of each component), and each
// bubble's gas is carried over merges and splits in proportion to the volume it leaves
// in each new component. Components touching the headspace belong to the atmosphere
// (id 0, fixed pressure). Bubble pressures follow the ideal-gas law (Eq. idealgas).
//
// Only cells with a non-zero bubble id take part in the union-find; the atmosphere is
// one node that a component joins when one of its cells touches an atmosphere cell.
// A step's conversions can change only the components around the cells they convert
// (the topology test marks their ids); a relabelling step then relabels the cells of the
// marked ids alone, and every other bubble keeps its id and gas and gets its volume from
// the fast path's sums. The results equal those of relabelling every cell: an unmarked
// component would come out of the full labelling with its own id, its whole gas and the
// same fixed-point volume.
// Volumes and gas are summed in 128-bit fixed point, so all results are independent of
// the order in which threads run.
#include "mf_internal.h"

namespace mf {

constexpr unsigned long long HEMPTY = ~0ull;
constexpr int32_t REMPTY = -1;

__device__ __forceinline__ int32_t uf_find(int32_t *parent, int32_t x) {
  int32_t p = __atomic_load_n(&parent[x], __ATOMIC_RELAXED);
  while (p != x) {
    const int32_t gp = __atomic_load_n(&parent[p], __ATOMIC_RELAXED);
    if (gp != p) __atomic_store_n(&parent[x], gp, __ATOMIC_RELAXED);  // path halving
    x = p;
    p = gp;
  }
  return x;
}

__device__ __forceinline__ void uf_union(int32_t *parent, int32_t a, int32_t b) {
  while (true) {
    a = uf_find(parent, a);
    b = uf_find(parent, b);
    if (a == b) return;
    if (a > b) { const int32_t t = a; a = b; b = t; }
    // hook the larger root under the smaller one
    const int32_t old = atomicCAS(&parent[b], b, a);
    if (old == b) return;
  }
}

// the union-find runs over the bubble cells of the state after this step's conversions
// (gas / interface with a non-zero id), listed at the start of a relabelling step
#define CLIST_LOOP(k, n, total)                                                   \
  const int64_t total = *(volatile int32_t *)(d.cnt + C_B);                       \
  for (int64_t k = gp.bid * blockDim.x + threadIdx.x;                              \
       k < ((total + 63) & ~(int64_t)63); k += gp.nblk * blockDim.x)

template <int D>
__device__ __forceinline__ void b_ccl_hook(const GridPos &gp, KP p, DA d) {
  if (!*(volatile int32_t *)(d.cnt + C_TOPO)) return;  // fast path this step
  using L = Lat<D>;
  CLIST_LOOP(k, n, total) {
    if (k >= total) continue;
    const int64_t n = d.blist[k];
    if (!(d.cflag[n] & CF_VALID)) continue;
    int x, y, z;
    cell_xyz(p, n, x, y, z);
    bool atm = false, stray = false;
    for (int i = 1; i < L::Q; ++i) {
      const int64_t yy = nb_index(p, x, y, z, L::ex[i], L::ey[i], L::ez[i]);
      const int ty = d.type[yy] & TMASK;
      if (ty != TG && ty != TI) continue;
      if (d.label[yy] == 0) atm = true;
      else if (!(d.cflag[yy] & CF_VALID)) stray = true;  // an unlisted id next to a listed one
      else if (yy > n) uf_union(d.parent, (int32_t)n, (int32_t)yy);
    }
    if (atm) flag_or(d.cflag, n, CF_ATM);
    if (stray) raise_status(d.status, ST_INVARIANT);
  }
}
template <int D>
__global__ __launch_bounds__(256) void k_ccl_hook(KP p, DA d) {
  b_ccl_hook<D>(GridPos::hw(), p, d);
}

__device__ __forceinline__ int hash_insert(const KP &p, DA &d, unsigned long long key) {
  unsigned h = (unsigned)((key * 0x9E3779B97F4A7C15ull) >> 40) & (unsigned)(p.H - 1);
  for (int probe = 0; probe < p.H; ++probe) {
    const unsigned long long k = __atomic_load_n(&d.hkeys[h], __ATOMIC_RELAXED);
    if (k == key) return (int)h;
    if (k == HEMPTY) {
      const unsigned long long old = atomicCAS(&d.hkeys[h], HEMPTY, key);
      if (old == HEMPTY) {
        const int e = atomicAdd(d.cnt + C_ENTRIES, 1);
        if (e < p.ecap) d.hslot[e] = (int)h;
        else raise_status(d.status, ST_TABLE);
        return (int)h;
      }
      if (old == key) return (int)h;
    }
    h = (h + 1) & (unsigned)(p.H - 1);
  }
  raise_status(d.status, ST_TABLE);
  return -1;
}

// final roots (a cell next to the atmosphere marks its root), and the volume share
// (1 - alpha) of every bubble cell summed per (component root, old id)
template <int P>
__device__ __forceinline__ void b_ccl_accum(const GridPos &gp, KP p, DA d) {
  if (!*(volatile int32_t *)(d.cnt + C_TOPO)) return;  // fast path this step
  using R = typename Prec<P>::R;
  CLIST_LOOP(k, n, total) {
    bool act = false;
    unsigned long long key = 0;
    Fx3 v = {0, 0, 0};
    if (k < total) {
      const int64_t n = d.blist[k];
      const uint8_t cl = d.cflag[n];
      if (cl & CF_VALID) {
        act = true;
        const int32_t r = uf_find(d.parent, (int32_t)n);
        d.parent[n] = r;
        if (cl & CF_ATM) flag_or(d.cflag, r, CF_ATMROOT);
        key = ((unsigned long long)(uint32_t)r << 32) | (unsigned long long)(uint32_t)d.label[n];
        const int t = d.type[n] & TMASK;
        const R one_minus = t == TG ? R(1) : R(1) - ((const R *)d.alpha)[n];
        v = fx3((double)one_minus);
      }
    }
    // wave-level grouping of equal keys, then one hash update per group
    unsigned long long pending = __ballot(act);
    const int lane = lane_id();
    while (pending) {
      const int leader = __ffsll((long long)pending) - 1;
      const unsigned long long kk = __shfl(key, leader);
      const bool mine = act && key == kk;
      const unsigned long long mm = __ballot(mine);
      long long sl = mine ? v.l : 0, sm = mine ? v.m : 0, sh = mine ? v.h : 0;
      for (int off = 32; off > 0; off >>= 1) {
        sl += __shfl_xor(sl, off);
        sm += __shfl_xor(sm, off);
        sh += __shfl_xor(sh, off);
      }
      if (lane == leader) {
        const int h = hash_insert(p, d, kk);
        if (h >= 0) {
          atomicAdd((unsigned long long *)&d.hvals[3 * h + 0], (unsigned long long)sl);
          atomicAdd((unsigned long long *)&d.hvals[3 * h + 1], (unsigned long long)sm);
          atomicAdd((unsigned long long *)&d.hvals[3 * h + 2], (unsigned long long)sh);
        }
      }
      pending &= ~mm;
      act = act && !mine;
    }
  }
}
template <int P>
__global__ __launch_bounds__(256) void k_ccl_accum(KP p, DA d) {
  b_ccl_accum<P>(GridPos::hw(), p, d);
}

__device__ __forceinline__ __int128 join3(const long long *a) { return fx3_join(a[0], a[1], a[2]); }

// the copies of the atmosphere's step accumulators (gas-side flux and conversion terms),
// summed and cleared by the first wave of the block; lane 0 holds the total
static_assert(NSPREAD == 64, "one copy per lane");
__device__ __forceinline__ void take_atm_copies(DA &d, long long s[3]) {
  const int lane = lane_id();
  for (int c = 0; c < 3; ++c) {
    s[c] = d.phi0[3 * lane + c] + d.gam0[3 * lane + c];
    d.phi0[3 * lane + c] = 0;
    d.gam0[3 * lane + c] = 0;
  }
  for (int off = 32; off > 0; off >>= 1)
    for (int c = 0; c < 3; ++c) s[c] += __shfl_xor(s[c], off);
}
__device__ __forceinline__ void add3(long long *acc, const long long *v) {
  atomicAdd((unsigned long long *)&acc[0], (unsigned long long)v[0]);
  atomicAdd((unsigned long long *)&acc[1], (unsigned long long)v[1]);
  atomicAdd((unsigned long long *)&acc[2], (unsigned long long)v[2]);
}
__device__ __forceinline__ void addfx(long long *acc, double v) {
  const Fx3 f = fx3(v);
  atomicAdd((unsigned long long *)&acc[0], (unsigned long long)f.l);
  atomicAdd((unsigned long long *)&acc[1], (unsigned long long)f.m);
  atomicAdd((unsigned long long *)&acc[2], (unsigned long long)f.h);
}

constexpr int ATMBIT = 1 << 30;
constexpr int LOCALMAX = 16;

// gas share of old id j in component K: m'_j V_{j,K} / V_j (all of m'_j to the
// lowest-root non-atmosphere component when V_j = 0)
__device__ __forceinline__ double share_of(const DA &d, int lab, int32_t root, const long long *v) {
  const __int128 vt = join3(&d.lab_vtot[3 * lab]);
  if (vt == 0) return d.lab_first[lab] == root ? d.mprime[lab] : 0.0;
  return d.mprime[lab] * (fx_to_double(join3(v)) / fx_to_double(vt));
}

__device__ void write_bubble(const KP &p, DA &d, int id, double m, __int128 vk) {
  const double V = fx_to_double(vk);
  d.bm[id] = m;
  d.bV[id] = V;
  d.bp[id] = (m * p.RT) / (V > 0.5 ? V : 0.5);
  d.balive[id] = 1;
}

// Single work-group pass over the (root, old id) table: new ids, gas redistribution,
// volumes and pressures. Components whose ids appear nowhere else are handled in
// parallel; the few whose ids are shared with another component (splits) are done in
// ascending root order by one thread, which is the order the assignment rule needs.
__device__ __forceinline__ void b_bubble_update(const GridPos &gp, KP p, DA d, int apply_flux) {
  if (!*(volatile int32_t *)(d.cnt + C_TOPO)) return;  // fast path this step
  // partial: only the marked ids (and the atmosphere) are updated here; the fast-path
  // kernel has updated the others
  const bool partial = !*(volatile int32_t *)(d.cnt + C_FULL);
  const int tid = threadIdx.x, nt = blockDim.x;
  const int cap = p.cap;
  __shared__ int s_ncont, s_nroot;
  __shared__ long long s_atm[3];
  int ne = *(volatile int32_t *)(d.cnt + C_ENTRIES);
  if (ne > p.ecap) ne = p.ecap;
  // ids are never reused, so every id in use is below the id counter
  int jmax = *(volatile int32_t *)d.nextid;
  if (jmax > cap) jmax = cap;
  if (tid == 0) {
    s_ncont = 0;
    s_nroot = 0;
    s_atm[0] = s_atm[1] = s_atm[2] = 0;
  }
  __syncthreads();
  // phase 0: gas of each old bubble after this step's flux; clear the table
  for (int j = tid; j < jmax; j += nt) {
    if (partial && j > 0 && !d.aff[j]) continue;
    const int al = d.balive[j];
    d.alive_prev[j] = al;
    double mp = 0.0;
    if (j == 0) {
      if (apply_flux) {
        s_atm[0] = d.phi[0] + d.gam[0];
        s_atm[1] = d.phi[1] + d.gam[1];
        s_atm[2] = d.phi[2] + d.gam[2];
      }
    } else if (al) {
      mp = d.bm[j];
      if (apply_flux) mp = mp + fx_to_double(join3(&d.phi[3 * j]) + join3(&d.gam[3 * j]));
    }
    d.mprime[j] = mp;
    d.phi[3 * j] = d.phi[3 * j + 1] = d.phi[3 * j + 2] = 0;
    d.gam[3 * j] = d.gam[3 * j + 1] = d.gam[3 * j + 2] = 0;
    d.lab_cnt[j] = 0;
    d.lab_first[j] = 0x7FFFFFFF;
    d.lab_assigned[j] = 0;
    for (int c = 0; c < 3; ++c) d.lab_vtot[3 * j + c] = d.lab_vatm[3 * j + c] = 0;
    d.balive[j] = 0;
    d.bm[j] = 0.0;
    d.bV[j] = 0.0;
    d.bp[j] = 0.0;
    d.bng[j] = 0;
  }
  if (tid < 64) {
    long long sa[3];
    take_atm_copies(d, sa);
    if (tid == 0 && apply_flux)
      for (int c = 0; c < 3; ++c) s_atm[c] += sa[c];
  }
  __syncthreads();
  // phase A: entries out of the pair hash; per-id sums; group non-atmosphere entries
  // by root
  for (int e = tid; e < ne; e += nt) {
    const int h = d.hslot[e];
    const unsigned long long key = d.hkeys[h];
    const int32_t root = (int32_t)(key >> 32);
    const int32_t lab = (int32_t)(uint32_t)(key & 0xFFFFFFFFull);
    long long v[3] = {d.hvals[3 * h], d.hvals[3 * h + 1], d.hvals[3 * h + 2]};
    d.hkeys[h] = HEMPTY;
    d.hvals[3 * h] = d.hvals[3 * h + 1] = d.hvals[3 * h + 2] = 0;
    const bool atm = (d.cflag[root] & CF_ATMROOT) != 0;
    d.ent_root[e] = root;
    d.ent_lab[e] = lab;
    d.ent_flag[e] = atm ? 1 : 0;
    d.ent_v[3 * e] = v[0];
    d.ent_v[3 * e + 1] = v[1];
    d.ent_v[3 * e + 2] = v[2];
    if (lab <= 0 || lab >= cap) {
      raise_status(d.status, ST_BADLABEL);
      d.ent_flag[e] = 2;
      continue;
    }
    add3(&d.lab_vtot[3 * lab], v);
    if (atm) {
      add3(&d.lab_vatm[3 * lab], v);
      atomicOr(&d.lab_cnt[lab], ATMBIT);
      d.label[root] = 0;
    } else {
      atomicAdd(&d.lab_cnt[lab], 1);
      atomicMin(&d.lab_first[lab], root);
      unsigned s = ((unsigned)root * 2654435761u) & (unsigned)(p.RH - 1);
      for (int probe = 0; probe < p.RH; ++probe) {
        const int32_t old = atomicCAS(&d.rh_key[s], REMPTY, root);
        if (old == REMPTY) {
          d.rused[atomicAdd(&s_nroot, 1)] = (int)s;
          break;
        }
        if (old == root) break;
        s = (s + 1) & (unsigned)(p.RH - 1);
      }
      d.ent_next[e] = atomicExch(&d.rh_head[s], e);
    }
  }
  __syncthreads();
  // phase C: components whose ids are theirs alone
  const int nroot = s_nroot;
  for (int u = tid; u < nroot; u += nt) {
    const int s = d.rused[u];
    const int32_t root = d.rh_key[s];
    int loc[LOCALMAX];
    int nl = 0;
    bool contested = false;
    for (int e = d.rh_head[s]; e >= 0; e = d.ent_next[e]) {
      if (nl < LOCALMAX) loc[nl] = e;
      nl++;
      if ((d.lab_cnt[d.ent_lab[e]] & ~ATMBIT) >= 2) contested = true;
    }
    if (contested || nl > LOCALMAX) {
      d.contested[atomicAdd(&s_ncont, 1)] = s;
      continue;
    }
    for (int a = 1; a < nl; ++a) {  // ascending old id
      const int e = loc[a];
      int b = a - 1;
      while (b >= 0 && d.ent_lab[loc[b]] > d.ent_lab[e]) { loc[b + 1] = loc[b]; --b; }
      loc[b + 1] = e;
    }
    const int id = d.ent_lab[loc[0]];
    double m = 0.0;
    __int128 vk = 0;
    for (int a = 0; a < nl; ++a) {
      const int e = loc[a];
      m = m + share_of(d, d.ent_lab[e], root, &d.ent_v[3 * e]);
      vk += join3(&d.ent_v[3 * e]);
    }
    d.lab_assigned[id] = 1;
    write_bubble(p, d, id, m, vk);
    d.label[root] = id;
  }
  __syncthreads();
  // phase D: atmosphere shares and collapsed bubbles
  for (int j = 1 + tid; j < jmax; j += nt) {
    if ((partial && !d.aff[j]) || !d.alive_prev[j]) continue;
    const int lc = d.lab_cnt[j];
    const bool inatm = (lc & ATMBIT) != 0;
    const int nonatm = lc & ~ATMBIT;
    if (!inatm && nonatm == 0) {
      addfx(&d.led[6], d.mprime[j]);
      continue;
    }
    if (inatm) {
      const __int128 vt = join3(&d.lab_vtot[3 * j]);
      double c;
      if (vt == 0) c = nonatm > 0 ? 0.0 : d.mprime[j];
      else c = d.mprime[j] * (fx_to_double(join3(&d.lab_vatm[3 * j])) / fx_to_double(vt));
      addfx(&d.led[3], c);
    }
  }
  __syncthreads();
  // phase E: split components in ascending root order
  if (tid == 0) {
    const int nc = s_ncont;
    for (int a = 1; a < nc; ++a) {
      const int sv = d.contested[a];
      int b = a - 1;
      while (b >= 0 && d.rh_key[d.contested[b]] > d.rh_key[sv]) { d.contested[b + 1] = d.contested[b]; --b; }
      d.contested[b + 1] = sv;
    }
    int next_id = *d.nextid;
    for (int a = 0; a < nc; ++a) {
      const int s = d.contested[a];
      const int32_t root = d.rh_key[s];
      // entries of this component in ascending old id by repeated minimum search
      int id = -1;
      double m = 0.0;
      __int128 vk = 0;
      int last = 0;
      while (true) {
        int best = -1;
        for (int e = d.rh_head[s]; e >= 0; e = d.ent_next[e]) {
          const int lb = d.ent_lab[e];
          if (lb > last && (best < 0 || lb < d.ent_lab[best])) best = e;
        }
        if (best < 0) break;
        const int lb = d.ent_lab[best];
        if (id < 0 && !d.lab_assigned[lb]) id = lb;
        m = m + share_of(d, lb, root, &d.ent_v[3 * best]);
        vk += join3(&d.ent_v[3 * best]);
        last = lb;
      }
      if (id < 0) {
        if (next_id >= cap) {
          raise_status(d.status, ST_TABLE);
          continue;
        }
        id = next_id++;
      }
      d.lab_assigned[id] = 1;
      write_bubble(p, d, id, m, vk);
      d.label[root] = id;
    }
    *d.nextid = next_id;
    d.cnt[C_CONTESTED] = nc;
  }
  __syncthreads();
  // clear the used root-hash slots and the marks; fold this step's ledgers into the
  // running totals
  for (int u = tid; u < nroot; u += nt) {
    const int s = d.rused[u];
    d.rh_key[s] = REMPTY;
    d.rh_head[s] = -1;
  }
  for (int j = tid; j < jmax; j += nt) d.aff[j] = 0;
  if (tid == 0) {
    d.ledtot[0] += join3(&d.led[0]);
    d.ledtot[1] += join3(&d.led[3]) + fx3_join(s_atm[0], s_atm[1], s_atm[2]);
    d.ledtot[2] += join3(&d.led[6]);
    for (int c = 0; c < 9; ++c) d.led[c] = 0;
    d.bp[0] = p.p_atm;
    d.balive[0] = 1;
  }
}
__global__ __launch_bounds__(1024) void k_bubble_update(KP p, DA d, int apply_flux) {
  b_bubble_update(GridPos::hw(), p, d, apply_flux);
}

// new ids onto every listed cell from its root, the gas cells of every relabelled bubble
// counted under the new ids (the conversions keep the counts of the others up to date), and
// the labelling flags cleared
template <int P>
__device__ __forceinline__ void b_ccl_relabel(const GridPos &gp, KP p, DA d) {
  using R = typename Prec<P>::R;
  if (!*(volatile int32_t *)(d.cnt + C_TOPO)) return;  // fast path this step
  CLIST_LOOP(k, n, total) {
    bool gas = false;
    int lab = 0;
    if (k < total) {
      const int64_t n = d.blist[k];
      if (d.cflag[n] & CF_VALID) {
        lab = d.label[d.parent[n]];
        d.label[n] = lab;
        const uint8_t tb = d.type[n];
        gas = (tb & TMASK) == TG && lab > 0 && lab < p.cap;
        // the stencil words (learned curvature) carry the id
        if (d.sword) d.sword[n] = stencil_word<R>(tb, ((const R *)d.alpha)[n], lab);
      }
      d.cflag[n] = 0;
    }
    wave_count_add(d.bng, gas, lab, 1);
  }
}
template <int P>
__global__ __launch_bounds__(256) void k_ccl_relabel(KP p, DA d) {
  b_ccl_relabel<P>(GridPos::hw(), p, d);
}

__global__ void k_fill_words(int32_t *p, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// the gas-cell counts from scratch over the whole grid (hand-written states)
__global__ __launch_bounds__(256) void k_recount_gas(KP p, DA d) {
  for (int64_t n0 = (int64_t)blockIdx.x * blockDim.x; n0 < p.N; n0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t n = n0 + threadIdx.x;
    bool act = false;
    int lab = 0;
    if (n < p.N && (d.type[n] & TMASK) == TG) {
      lab = d.label[n];
      act = lab > 0 && lab < p.cap;
    }
    wave_count_add(d.bng, act, lab, 1);
  }
}

void recount_gas(const Ctx &c, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_words, dim3(64), dim3(256), 0, s, c.d.bng, (int64_t)c.kp.cap, 0);
  const int64_t g = (c.kp.N + 255) / 256;
  hipLaunchKernelGGL(k_recount_gas, dim3((unsigned)(g < 8192 ? g : 8192)), dim3(256), 0, s, c.kp, c.d);
}

// ------------------------------------------------------------------ fast path
// Steps whose conversions cannot have changed any component (C_TOPO clear) keep every
// id; each bubble then holds all of its gas, and only its volume and pressure change.
// The volume is its gas-cell count plus the interface shares 1 - alpha summed by the
// excess pass: the same fixed-point sums as the full path's, so the results are
// identical to what the full labelling would give.
// Several work-groups over the ids; the first also folds the atmosphere's terms and the
// step's ledgers into the running totals. On a partial relabelling the same update serves
// the unmarked ids only; the relabelling takes the marked ones, the atmosphere and the
// ledgers.
__device__ __forceinline__ void b_bubble_fast(const GridPos &gp, KP p, DA d) {
  const bool partial = *(volatile int32_t *)(d.cnt + C_TOPO) != 0;
  if (partial && *(volatile int32_t *)(d.cnt + C_FULL)) return;
  const int tid = threadIdx.x;
  __shared__ long long s_atm[3];
  int jmax = *(volatile int32_t *)d.nextid;
  if (jmax > p.cap) jmax = p.cap;
  if (!partial && gp.bid == 0 && tid < 64) {
    long long sa[3];
    take_atm_copies(d, sa);
    if (tid == 0)
      for (int c = 0; c < 3; ++c) s_atm[c] = d.phi[c] + d.gam[c] + sa[c];
  }
  __syncthreads();
  for (int j = gp.bid * blockDim.x + tid; j < jmax; j += gp.nblk * blockDim.x) {
    if (partial && (j == 0 || d.aff[j])) continue;
    if (j > 0 && d.balive[j]) {
      const double mp = d.bm[j] + fx_to_double(join3(&d.phi[3 * j]) + join3(&d.gam[3 * j]));
      // volume: one per gas cell, 1 - alpha per interface cell (fixed point, 2^64 = 1)
      write_bubble(p, d, j, mp, join3(&d.vacc[3 * j]) + ((__int128)d.bng[j] << 64));
    }
    for (int c = 0; c < 3; ++c) d.phi[3 * j + c] = d.gam[3 * j + c] = d.vacc[3 * j + c] = 0;
  }
  if (!partial && gp.bid == 0 && tid == 0) {
    d.ledtot[0] += join3(&d.led[0]);
    d.ledtot[1] += join3(&d.led[3]) + fx3_join(s_atm[0], s_atm[1], s_atm[2]);
    d.ledtot[2] += join3(&d.led[6]);
    for (int c = 0; c < 9; ++c) d.led[c] = 0;
    d.bp[0] = p.p_atm;
    d.balive[0] = 1;
    d.cnt[C_CONTESTED] = 0;
  }
}
__global__ __launch_bounds__(256) void k_bubble_fast(KP p, DA d) {
  b_bubble_fast(GridPos::hw(), p, d);
}

// outside the time step (nucleation, refresh) the full labelling always runs
__global__ void k_force_full(DA d) {
  d.cnt[C_TOPO] = 1;
  d.cnt[C_FULL] = 1;
}

// batched forms (time-step labelling: the flux of the step is applied)
__global__ __launch_bounds__(256) void km_bubble_fast(MLaunch ml) {
  MF_MULTI(MK_BFAST)
  b_bubble_fast(gp, m.kp, m.d);
}
template <int D>
__global__ __launch_bounds__(256) void km_ccl_hook(MLaunch ml) {
  MF_MULTI(MK_SHORT)
  b_ccl_hook<D>(gp, m.kp, m.d);
}
template <int P>
__global__ __launch_bounds__(256) void km_ccl_accum(MLaunch ml) {
  MF_MULTI(MK_SHORT)
  b_ccl_accum<P>(gp, m.kp, m.d);
}
__global__ __launch_bounds__(1024) void km_bubble_update(MLaunch ml) {
  MF_MULTI(MK_ONE)
  b_bubble_update(gp, m.kp, m.d, 1);
}
template <int P>
__global__ __launch_bounds__(256) void km_ccl_relabel(MLaunch ml) {
  MF_MULTI(MK_SHORT)
  b_ccl_relabel<P>(gp, m.kp, m.d);
}

// the labelling of every domain of a batch, in the order of label(c, s, 1)
template <int D, int P>
void Ops<D, P>::label_multi(const MStep &ms, hipStream_t s) {
  hipLaunchKernelGGL(km_bubble_fast, dim3(ms.grid[MK_BFAST]), dim3(256), 0, s, ms.at(MK_BFAST));
  lists_multi(ms, 1, s);
  hipLaunchKernelGGL((km_ccl_hook<D>), dim3(ms.grid[MK_SHORT]), dim3(256), 0, s, ms.at(MK_SHORT));
  hipLaunchKernelGGL((km_ccl_accum<P>), dim3(ms.grid[MK_SHORT]), dim3(256), 0, s, ms.at(MK_SHORT));
  hipLaunchKernelGGL(km_bubble_update, dim3(ms.grid[MK_ONE]), dim3(1024), 0, s, ms.at(MK_ONE));
  hipLaunchKernelGGL((km_ccl_relabel<P>), dim3(ms.grid[MK_SHORT]), dim3(256), 0, s, ms.at(MK_SHORT));
}

template <int D, int P>
void Ops<D, P>::label(Ctx &c, hipStream_t s, int apply_flux) {
  const unsigned nb = list_blocks(c);
  // the relabelling kernels return at once on steps without topology change and list few
  // cells on the others: a smaller grid keeps those launches cheap, and their grid-stride
  // loops cover the list when it is long
  const unsigned nf = nb < 1024 ? nb : 1024;
  if (!apply_flux) hipLaunchKernelGGL(k_force_full, dim3(1), dim3(1), 0, s, c.d);
  hipLaunchKernelGGL(k_bubble_fast, dim3((unsigned)((c.kp.cap + 255) / 256 < 64 ? (c.kp.cap + 255) / 256 : 64)), dim3(256), 0, s, c.kp, c.d);
  build_bubble_list(c, s);  // also starts the union-find: every listed cell its own root
  hipLaunchKernelGGL((k_ccl_hook<D>), dim3(nf), dim3(256), 0, s, c.kp, c.d);
  hipLaunchKernelGGL((k_ccl_accum<P>), dim3(nf), dim3(256), 0, s, c.kp, c.d);
  hipLaunchKernelGGL(k_bubble_update, dim3(1), dim3(1024), 0, s, c.kp, c.d, apply_flux);
  hipLaunchKernelGGL((k_ccl_relabel<P>), dim3(nf), dim3(256), 0, s, c.kp, c.d);
}

#define MF_INST(D, P)                                         \
  template void Ops<D, P>::label(Ctx &, hipStream_t, int);    \
  template void Ops<D, P>::label_multi(const MStep &, hipStream_t);
MF_FOR_ALL(MF_INST)

}  // namespace mf

// Initial state, nucleation (Sec. 3.4), list rebuilds and field transfer.
#include "lbm_math.h"

namespace mf {

// liquid at rest (f = w_i, g = w_i c0), wall layers on closed axes, headspace gas of the
// atmosphere above gas_from
template <int D, int P>
__global__ __launch_bounds__(256) void k_init_box(KP p, DA d, int gas_from) {
  using R = typename Prec<P>::R;
  using SF = typename Prec<P>::SF;
  using SG = typename Prec<P>::SG;
  using L = Lat<D>;
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < p.N; n += (int64_t)gridDim.x * blockDim.x) {
    int x, y, z;
    cell_xyz(p, n, x, y, z);
    const int c[3] = {x, y, z}, dims[3] = {p.nx, p.ny, p.nz};
    bool wall = false;
    for (int a = 0; a < D; a++)
      if (!p.per[a] && (c[a] == 0 || c[a] == dims[a] - 1)) wall = true;
    const int lc = D == 2 ? y : z;
    uint8_t t;
    int32_t lab = NOLAB;
    if (wall) t = TW;
    else if (gas_from >= 0 && lc >= gas_from) { t = TG; lab = 0; }
    else t = TL;
    d.type[n] = t;
    d.label[n] = lab;
    for (int b = 0; b < 2; b++) {
      SF *f = (SF *)d.f[b];
      SG *g = (SG *)d.g[b];
      // rest state: f = w_i, g = w_i c0 (zero offsets in the shifted instances)
#pragma unroll
      for (int i = 0; i < L::Q; ++i)
        f[(int64_t)i * p.Np + n] = FCodec<P, D>::enc((t == TW || P != 0) ? R(0) : R(L::w[i]), i);
#pragma unroll
      for (int i = 0; i < L::Qg; ++i)
        g[(int64_t)i * p.Np + n] = GCodec<P>::enc((t == TW || P != 0) ? R(0) : R(L::wg[i] * p.c0), p);
    }
    const R one = t == TL ? R(1) : R(0);
    ((R *)d.alpha)[n] = one;
    ((R *)d.M)[n] = one;
    ((R *)d.rho)[n] = R(1);
    ((R *)d.ux)[n] = R(0);
    ((R *)d.uy)[n] = R(0);
    ((R *)d.uz)[n] = R(0);
    ((R *)d.kappa)[n] = R(0);
    ((R *)d.Pi)[n] = R(0);
    d.cflag[n] = 0;
  }
}

// static flags: the cell touches a wall through a lattice direction (type bit), and the
// directions i whose source x - e_i is a wall (bit mask)
template <int D>
__global__ __launch_bounds__(256) void k_nearwall(KP p, DA d) {
  using L = Lat<D>;
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < p.N; n += (int64_t)gridDim.x * blockDim.x) {
    const uint8_t t = d.type[n] & TMASK;
    uint32_t wm = 0;
    if (t != TW) {
      int x, y, z;
      cell_xyz(p, n, x, y, z);
      for (int i = 1; i < L::Q; ++i) {
        const int64_t s = nb_index(p, x, y, z, -L::ex[i], -L::ey[i], -L::ez[i]);
        if ((d.type[s] & TMASK) == TW) wm |= 1u << i;
      }
    }
    d.wmask[n] = wm;
    d.type[n] = t | (wm ? NEARWALL : 0);
  }
}

// voxelise one nucleus over its bounding box: covered fraction from 8 sample points per
// axis; the cell keeps the largest fraction over nuclei, the first nucleus on ties
template <int D, int P>
__global__ __launch_bounds__(256) void k_nuc_voxel(KP p, DA d, int k, double cx, double cy, double cz, double r,
                                                   int x0, int y0, int z0, int sx, int sy, int sz) {
  using R = typename Prec<P>::R;
  const int64_t tot = (int64_t)sx * sy * sz;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
    const int x = x0 + (int)(t % sx);
    const int y = y0 + (int)((t / sx) % sy);
    const int z = z0 + (int)(t / ((int64_t)sx * sy));
    if (x < 0 || x >= p.nx || y < 0 || y >= p.ny || z < 0 || z >= p.nz) continue;
    const int64_t n = (int64_t)x + (int64_t)p.nx * ((int64_t)y + (int64_t)p.ny * z);
    if ((d.type[n] & TMASK) != TL) continue;
    if (fabs((double)x - cx) > r + 1.0 || fabs((double)y - cy) > r + 1.0) continue;
    if (D == 3 && fabs((double)z - cz) > r + 1.0) continue;
    int cnt = 0;
    const int czn = D == 3 ? 8 : 1;
    for (int c = 0; c < czn; c++)
      for (int b = 0; b < 8; b++)
        for (int a = 0; a < 8; a++) {
          const double px = (double)x + (double)(2 * a - 7) / 16.0;
          const double py = (double)y + (double)(2 * b - 7) / 16.0;
          const double pz = D == 3 ? (double)z + (double)(2 * c - 7) / 16.0 : 0.0;
          const double dx = px - cx, dy = py - cy, dz = pz - cz;
          if (((dx * dx + dy * dy) + dz * dz) < r * r) cnt++;
        }
    const double f = (double)cnt / (double)(D == 3 ? 512 : 64);
    R *phi = (R *)d.exc;
    if ((R)f > phi[n]) {
      phi[n] = (R)f;
      d.parent[n] = k;
    }
  }
}

template <int P>
__global__ __launch_bounds__(256) void k_nuc_prep(KP p, DA d) {
  using R = typename Prec<P>::R;
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < p.N; n += (int64_t)gridDim.x * blockDim.x) {
    ((R *)d.exc)[n] = R(0);
    d.parent[n] = -1;
  }
}

template <int P>
__global__ __launch_bounds__(256) void k_nuc_apply(KP p, DA d) {
  using R = typename Prec<P>::R;
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < p.N; n += (int64_t)gridDim.x * blockDim.x) {
    const int k = d.parent[n];
    if (k < 0) continue;
    const R phi = ((const R *)d.exc)[n];
    const uint8_t keep = d.type[n] & ~TMASK;
    if (phi >= R(1)) {
      d.type[n] = keep | TG;
      ((R *)d.alpha)[n] = R(0);
      ((R *)d.M)[n] = R(0);
    } else {
      d.type[n] = keep | TI;
      const R a = R(1) - phi;
      ((R *)d.alpha)[n] = a;
      ((R *)d.M)[n] = a;
    }
    d.label[n] = k + 1;
  }
}

// liquid cells that touch gas become interface cells (alpha = 1) with the smallest id of
// their gas neighbours
template <int D>
__global__ __launch_bounds__(256) void k_nuc_fix1(KP p, DA d) {
  using L = Lat<D>;
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < p.N; n += (int64_t)gridDim.x * blockDim.x) {
    int32_t best = -1;
    if ((d.type[n] & TMASK) == TL) {
      int x, y, z;
      cell_xyz(p, n, x, y, z);
      for (int i = 1; i < L::Q; ++i) {
        const int64_t yy = nb_index(p, x, y, z, L::ex[i], L::ey[i], L::ez[i]);
        if ((d.type[yy] & TMASK) == TG) {
          const int32_t lb = d.label[yy];
          if (best < 0 || lb < best) best = lb;
        }
      }
    }
    d.parent[n] = best;
  }
}

template <int P>
__global__ __launch_bounds__(256) void k_nuc_fix2(KP p, DA d) {
  using R = typename Prec<P>::R;
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < p.N; n += (int64_t)gridDim.x * blockDim.x) {
    const int32_t lb = d.parent[n];
    if (lb >= 0) {
      d.type[n] = (d.type[n] & ~TMASK) | TI;
      ((R *)d.alpha)[n] = R(1);
      ((R *)d.M)[n] = R(1);
      d.label[n] = lb;
    }
    if ((d.type[n] & TMASK) == TI) {
      ((R *)d.rho)[n] = R(1);
      ((R *)d.ux)[n] = R(0);
      ((R *)d.uy)[n] = R(0);
      ((R *)d.uz)[n] = R(0);
    }
    d.parent[n] = 0;
  }
}

// Cell lists: the interface list (type I) at the start of every step, and the bubble list
// (gas or interface with a non-zero bubble id) on the steps that relabel. The grid is cut
// into chunks of 16384 cells, each classified by a work-group whose threads take 64
// consecutive cells (16-byte type loads; labels only where there is gas or interface).
// The interface list is kept in cell order, without atomics (the interface sweep gathers
// faster from neighbouring cells): a count pass writes the per-chunk totals, one
// work-group scans them, and a write pass places every entry at its chunk's offset plus
// its rank inside the chunk. The bubble list is built in one pass (below). The work-groups
// step over the chunks, so a pass that returns at once (the bubble list on a step without
// relabelling) costs one small launch.
constexpr int LIST_CPT = 64;
constexpr int LIST_CHUNK = 256 * LIST_CPT;
constexpr int LIST_GRID = 1024;

// list 0: interface cells; list 1: gas / interface cells with a non-zero bubble id (of a
// marked id, on a partial relabelling)
template <int WHICH>
__device__ __forceinline__ unsigned long long list_mask(const KP &p, const DA &d, int64_t c0) {
  unsigned long long mk = 0;
  // the bubble list holds the cells of the marked ids only, unless every component is
  // relabelled
  const bool all = WHICH == 1 && *(volatile int32_t *)(d.cnt + C_FULL) != 0;
#pragma unroll
  for (int g = 0; g < LIST_CPT / 16; ++g) {
    const int64_t n = c0 + g * 16;
    if (n >= p.N) break;
    uint8_t t[16];
    if (n + 16 <= p.N) {
      const uint4 v = *(const uint4 *)(d.type + n);
      const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int k = 0; k < 16; ++k) t[k] = (uint8_t)(wv[k >> 2] >> (8 * (k & 3)));
    } else {
#pragma unroll
      for (int k = 0; k < 16; ++k) t[k] = n + k < p.N ? d.type[n + k] : TW;
    }
    uint32_t gi = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int tt = t[k] & TMASK;
      if (WHICH == 0 && tt == TI) mk |= 1ull << (g * 16 + k);
      if (tt == TG || tt == TI) gi |= 1u << k;
    }
    if (WHICH == 1) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (!((gi >> (4 * q)) & 15u)) continue;
        int32_t lb[4];
        if (n + 4 * q + 4 <= p.N) {
          const int4 v = *(const int4 *)(d.label + n + 4 * q);
          lb[0] = v.x; lb[1] = v.y; lb[2] = v.z; lb[3] = v.w;
        } else {
#pragma unroll
          for (int k = 0; k < 4; ++k) lb[k] = n + 4 * q + k < p.N ? d.label[n + 4 * q + k] : 0;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (((gi >> (4 * q + k)) & 1u) && lb[k] != 0 &&
              (all || (lb[k] > 0 && lb[k] < p.cap && d.aff[lb[k]])))
            mk |= 1ull << (g * 16 + 4 * q + k);
      }
    }
  }
  return mk;
}

// block-wide inclusive scan of one count (256 threads); returns the block total
__device__ __forceinline__ int block_scan(int &si) {
  __shared__ int s_w[4];
  const int lane = lane_id(), w = threadIdx.x >> 6;
  for (int o = 1; o < 64; o <<= 1) {
    const int a = __shfl_up(si, o);
    if (lane >= o) si += a;
  }
  if (lane == 63) s_w[w] = si;
  __syncthreads();
  int tot = 0;
  for (int k = 0; k < 4; ++k) {
    if (k < w) si += s_w[k];
    tot += s_w[k];
  }
  __syncthreads();
  return tot;
}

template <int WHICH> __device__ __forceinline__ bool list_skipped(const DA &d) {
  return WHICH == 1 && !*(volatile int32_t *)(d.cnt + C_TOPO);
}

template <int WHICH>
__device__ __forceinline__ void b_list_count(const GridPos &gp, KP p, DA d, int nchunks) {
  if (list_skipped<WHICH>(d)) return;
  for (int ch = gp.bid; ch < nchunks; ch += gp.nblk) {
    const int64_t c0 = (int64_t)ch * LIST_CHUNK + (int64_t)threadIdx.x * LIST_CPT;
    int si = __popcll(list_mask<WHICH>(p, d, c0));
    const int tot = block_scan(si);
    if (threadIdx.x == 0) d.lcnt[ch] = tot;
  }
}
template <int WHICH>
__global__ __launch_bounds__(256) void k_list_count(KP p, DA d, int nchunks) {
  b_list_count<WHICH>(GridPos::hw(), p, d, nchunks);
}

// exclusive scan of the per-chunk counts (in place) and the list length
template <int WHICH>
__device__ __forceinline__ void b_list_scan(const GridPos &gp, DA d, int nchunks) {
  if (list_skipped<WHICH>(d)) return;
  __shared__ int s_w[16];
  const int lane = lane_id(), w = threadIdx.x >> 6;
  const int per = (nchunks + 1023) / 1024;
  const int b0 = threadIdx.x * per;
  int32_t *lc = d.lcnt;
  int si = 0;
  for (int k = 0; k < per && b0 + k < nchunks; ++k) si += lc[b0 + k];
  const int ci = si;
  for (int o = 1; o < 64; o <<= 1) {
    const int a = __shfl_up(si, o);
    if (lane >= o) si += a;
  }
  if (lane == 63) s_w[w] = si;
  __syncthreads();
  int oi = si - ci, ti = 0;
  for (int k = 0; k < 16; ++k) {
    if (k < w) oi += s_w[k];
    ti += s_w[k];
  }
  for (int k = 0; k < per && b0 + k < nchunks; ++k) {
    const int a = lc[b0 + k];
    lc[b0 + k] = oi;
    oi += a;
  }
  if (threadIdx.x == 0) d.cnt[C_I] = ti;
}
template <int WHICH>
__global__ __launch_bounds__(1024) void k_list_scan(DA d, int nchunks) {
  b_list_scan<WHICH>(GridPos::hw(), d, nchunks);
}

template <int WHICH>
__device__ __forceinline__ void b_list_write(const GridPos &gp, KP p, DA d, int nchunks) {
  if (list_skipped<WHICH>(d)) return;
  int32_t *list = d.ilist;
  for (int ch = gp.bid; ch < nchunks; ch += gp.nblk) {
    const int64_t c0 = (int64_t)ch * LIST_CHUNK + (int64_t)threadIdx.x * LIST_CPT;
    unsigned long long mk = list_mask<WHICH>(p, d, c0);
    const int ci = __popcll(mk);
    int si = ci;
    block_scan(si);
    int o = d.lcnt[ch] + si - ci;
    while (mk) {
      const int b = __ffsll((long long)mk) - 1;
      mk &= mk - 1;
      const int32_t n = (int32_t)(c0 + b);
      list[o++] = n;
    }
  }
}
template <int WHICH>
__global__ __launch_bounds__(256) void k_list_write(KP p, DA d, int nchunks) {
  b_list_write<WHICH>(GridPos::hw(), p, d, nchunks);
}

// The bubble list in one pass: its order does not matter (the union-find hooks every
// root under the smaller cell index, and the per-(root, id) sums are fixed point and
// grouped by root afterwards), so each chunk takes its slots with one atomic on the list
// length and writes its entries in cell order there. This saves the count pass, a second
// read of the types and ids of the whole grid on every relabelling step.
__device__ __forceinline__ void b_list_clear1(DA d) {
  if (threadIdx.x == 0 && !list_skipped<1>(d)) d.cnt[C_B] = 0;
}
__global__ void k_list_clear1(DA d) { b_list_clear1(d); }

__device__ __forceinline__ void b_list_append1(const GridPos &gp, KP p, DA d, int nchunks) {
  if (list_skipped<1>(d)) return;
  __shared__ int s_base;
  for (int ch = gp.bid; ch < nchunks; ch += gp.nblk) {
    const int64_t c0 = (int64_t)ch * LIST_CHUNK + (int64_t)threadIdx.x * LIST_CPT;
    unsigned long long mk = list_mask<1>(p, d, c0);
    const int ci = __popcll(mk);
    int si = ci;
    const int tot = block_scan(si);  // the same for every thread of the block
    if (tot == 0) continue;
    if (threadIdx.x == 0) s_base = atomicAdd(d.cnt + C_B, tot);
    __syncthreads();
    int o = s_base + si - ci;
    while (mk) {
      const int b = __ffsll((long long)mk) - 1;
      mk &= mk - 1;
      const int32_t n = (int32_t)(c0 + b);
      d.blist[o++] = n;
      // union-find start of the relabelling: each bubble cell its own root
      d.parent[n] = n;
      flag_or(d.cflag, n, CF_VALID);
    }
    __syncthreads();  // s_base is taken again by the next chunk
  }
}
__global__ __launch_bounds__(256) void k_list_append1(KP p, DA d, int nchunks) {
  b_list_append1(GridPos::hw(), p, d, nchunks);
}

template <int WHICH> static void launch_list(const Ctx &c, hipStream_t s) {
  const int nch = list_blocks_of(c.kp);
  const unsigned g = (unsigned)(nch < LIST_GRID ? nch : LIST_GRID);
  hipLaunchKernelGGL(k_list_count<WHICH>, dim3(g), dim3(256), 0, s, c.kp, c.d, nch);
  hipLaunchKernelGGL(k_list_scan<WHICH>, dim3(1), dim3(1024), 0, s, c.d, nch);
  hipLaunchKernelGGL(k_list_write<WHICH>, dim3(g), dim3(256), 0, s, c.kp, c.d, nch);
}

void build_bubble_list(const Ctx &c, hipStream_t s) {
  const int nch = list_blocks_of(c.kp);
  const unsigned g = (unsigned)(nch < LIST_GRID ? nch : LIST_GRID);
  hipLaunchKernelGGL(k_list_clear1, dim3(1), dim3(64), 0, s, c.d);
  hipLaunchKernelGGL(k_list_append1, dim3(g), dim3(256), 0, s, c.kp, c.d, nch);
}

// batched forms of the list builder
__device__ __forceinline__ int list_chunks(const KP &p) { return (int)((p.N + LIST_CHUNK - 1) / LIST_CHUNK); }
template <int WHICH>
__global__ __launch_bounds__(256) void km_list_count(MLaunch ml) {
  MF_MULTI(MK_LISTGRID)
  b_list_count<WHICH>(gp, m.kp, m.d, list_chunks(m.kp));
}
template <int WHICH>
__global__ __launch_bounds__(1024) void km_list_scan(MLaunch ml) {
  MF_MULTI(MK_ONE)
  b_list_scan<WHICH>(gp, m.d, list_chunks(m.kp));
}
template <int WHICH>
__global__ __launch_bounds__(256) void km_list_write(MLaunch ml) {
  MF_MULTI(MK_LISTGRID)
  b_list_write<WHICH>(gp, m.kp, m.d, list_chunks(m.kp));
}
template <int WHICH> static void launch_list_multi(const MStep &ms, hipStream_t s) {
  hipLaunchKernelGGL(km_list_count<WHICH>, dim3(ms.grid[MK_LISTGRID]), dim3(256), 0, s, ms.at(MK_LISTGRID));
  hipLaunchKernelGGL(km_list_scan<WHICH>, dim3(ms.grid[MK_ONE]), dim3(1024), 0, s, ms.at(MK_ONE));
  hipLaunchKernelGGL(km_list_write<WHICH>, dim3(ms.grid[MK_LISTGRID]), dim3(256), 0, s, ms.at(MK_LISTGRID));
}
__global__ void km_list_clear1(MLaunch ml) {
  MF_MULTI(MK_ONE)
  (void)gp;
  b_list_clear1(m.d);
}
__global__ __launch_bounds__(256) void km_list_append1(MLaunch ml) {
  MF_MULTI(MK_LISTGRID)
  b_list_append1(gp, m.kp, m.d, list_chunks(m.kp));
}
void lists_multi(const MStep &ms, int which, hipStream_t s) {
  if (which == 0) {
    launch_list_multi<0>(ms, s);
  } else {
    hipLaunchKernelGGL(km_list_clear1, dim3(ms.grid[MK_ONE]), dim3(64), 0, s, ms.at(MK_ONE));
    hipLaunchKernelGGL(km_list_append1, dim3(ms.grid[MK_LISTGRID]), dim3(256), 0, s, ms.at(MK_LISTGRID));
  }
}

int list_blocks_of(const KP &kp) { return (int)((kp.N + LIST_CHUNK - 1) / LIST_CHUNK); }

// initial gas content m = p0 V / RT and pressure of every nucleus id
__global__ void k_init_mass(KP p, DA d, const double *p0, int nn) {
  for (int j = 1 + blockIdx.x * blockDim.x + threadIdx.x; j <= nn; j += gridDim.x * blockDim.x) {
    if (!d.balive[j]) continue;
    const double V = d.bV[j];
    const double m = (p0[j - 1] * V) / p.RT;
    d.bm[j] = m;
    d.bp[j] = (m * p.RT) / (V > 0.5 ? V : 0.5);
  }
}

// fields as binary64 (or bytes / ints) in a device staging buffer
template <int D, int P>
__global__ __launch_bounds__(256) void k_read(KP p, DA d, int cur, int field, double *out) {
  using R = typename Prec<P>::R;
  using SF = typename Prec<P>::SF;
  using SG = typename Prec<P>::SG;
  using L = Lat<D>;
  const SF *f = (const SF *)d.f[cur];
  const SG *g = (const SG *)d.g[cur];
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < p.N; n += (int64_t)gridDim.x * blockDim.x) {
    const int t = d.type[n] & TMASK;
    switch (field) {
      case MF_FIELD_TYPE: ((uint8_t *)out)[n] = (uint8_t)t; break;
      case MF_FIELD_LABEL: ((int32_t *)out)[n] = d.label[n]; break;
      case MF_FIELD_RHO: out[n] = (double)((const R *)d.rho)[n]; break;
      case MF_FIELD_UX: out[n] = (double)((const R *)d.ux)[n]; break;
      case MF_FIELD_UY: out[n] = (double)((const R *)d.uy)[n]; break;
      case MF_FIELD_UZ: out[n] = D == 3 ? (double)((const R *)d.uz)[n] : 0.0; break;
      case MF_FIELD_ALPHA: out[n] = t == TI ? (double)((const R *)d.alpha)[n] : (t == TL ? 1.0 : 0.0); break;
      case MF_FIELD_MASS: out[n] = t == TI ? (double)((const R *)d.M)[n] : (t == TL ? 1.0 : 0.0); break;
      case MF_FIELD_CONC: {
        double c = 0.0;
        if (t == TL || t == TI) {
          R gv[L::Qg], dc;
          for (int i = 0; i < L::Qg; ++i) gv[i] = GCodec<P>::dec(g[(int64_t)i * p.Np + n], p);
          c = (double)Arith<D, P>::conc(gv, R(p.c0), dc);
          if (P != 0) c = p.c0 + (double)dc;
        }
        out[n] = c;
        break;
      }
      case MF_FIELD_KAPPA: out[n] = t == TI ? (double)((const R *)d.kappa)[n] : 0.0; break;
      case MF_FIELD_PI: out[n] = t == TI ? (double)((const R *)d.Pi)[n] : 0.0; break;
      case MF_FIELD_F:
        for (int i = 0; i < L::Q; ++i) out[(int64_t)i * p.N + n] = FCodec<P, D>::full(f[(int64_t)i * p.Np + n], i);
        break;
      case MF_FIELD_G:
        for (int i = 0; i < L::Qg; ++i)
          out[(int64_t)i * p.N + n] = (double)GCodec<P>::dec(g[(int64_t)i * p.Np + n], p) + (P != 0 ? L::wg[i] * p.c0 : 0.0);
        break;
    }
  }
}

template <int D, int P>
__global__ __launch_bounds__(256) void k_write(KP p, DA d, int cur, int field, const double *in) {
  using R = typename Prec<P>::R;
  using SF = typename Prec<P>::SF;
  using SG = typename Prec<P>::SG;
  using L = Lat<D>;
  SF *f = (SF *)d.f[cur];
  SG *g = (SG *)d.g[cur];
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < p.N; n += (int64_t)gridDim.x * blockDim.x) {
    switch (field) {
      case MF_FIELD_TYPE: d.type[n] = ((const uint8_t *)in)[n] & TMASK; break;
      case MF_FIELD_LABEL: d.label[n] = ((const int32_t *)in)[n]; break;
      case MF_FIELD_RHO: ((R *)d.rho)[n] = (R)in[n]; break;
      case MF_FIELD_UX: ((R *)d.ux)[n] = (R)in[n]; break;
      case MF_FIELD_UY: ((R *)d.uy)[n] = (R)in[n]; break;
      case MF_FIELD_UZ: ((R *)d.uz)[n] = (R)in[n]; break;
      case MF_FIELD_ALPHA: ((R *)d.alpha)[n] = (R)in[n]; break;
      case MF_FIELD_MASS: ((R *)d.M)[n] = (R)in[n]; break;
      case MF_FIELD_KAPPA: ((R *)d.kappa)[n] = (R)in[n]; break;
      case MF_FIELD_PI: ((R *)d.Pi)[n] = (R)in[n]; break;
      case MF_FIELD_F:
        for (int i = 0; i < L::Q; ++i) f[(int64_t)i * p.Np + n] = FCodec<P, D>::from_full(in[(int64_t)i * p.N + n], i);
        break;
      case MF_FIELD_G:
        for (int i = 0; i < L::Qg; ++i)
          g[(int64_t)i * p.Np + n] = GCodec<P>::enc((R)(in[(int64_t)i * p.N + n] - (P != 0 ? L::wg[i] * p.c0 : 0.0)), p);
        break;
    }
  }
}

// add the three chunks of a lane's fixed-point partial sums over the wave, one atomic
// per chunk from lane 0 (integer sums: the result does not depend on the order)
__device__ __forceinline__ void wave_chunks_add(long long *dst, long long l, long long m, long long h) {
  for (int off = 32; off > 0; off >>= 1) {
    l += __shfl_xor(l, off);
    m += __shfl_xor(m, off);
    h += __shfl_xor(h, off);
  }
  if (lane_id() == 0) {
    atomicAdd((unsigned long long *)&dst[0], (unsigned long long)l);
    atomicAdd((unsigned long long *)&dst[1], (unsigned long long)m);
    atomicAdd((unsigned long long *)&dst[2], (unsigned long long)h);
  }
}

__global__ void k_zero_ll(long long *a, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = 0;
}

// Liquid mass (density of liquid cells, mass M of interface cells) and dissolved gas
// (concentration of liquid and interface cells) summed over the grid, each cell's value
// rounded to the fixed point of Fx3: a grid stride of at most 2^20 threads keeps every
// lane's chunk sums far from overflow.
template <int D, int P>
__global__ __launch_bounds__(256) void k_totals(KP p, DA d, int cur) {
  using R = typename Prec<P>::R;
  using SF = typename Prec<P>::SF;
  using SG = typename Prec<P>::SG;
  using L = Lat<D>;
  const SF *f = (const SF *)d.f[cur];
  const SG *g = (const SG *)d.g[cur];
  long long ml = 0, mm = 0, mh = 0, cl = 0, cm = 0, ch = 0;
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < p.N; n += (int64_t)gridDim.x * blockDim.x) {
    const int t = d.type[n] & TMASK;
    if (t != TL && t != TI) continue;
    double m;
    if (t == TI) {
      m = (double)((const R *)d.M)[n];
    } else {
      m = 0.0;
      for (int i = 0; i < L::Q; ++i) m += FCodec<P, D>::full(f[(int64_t)i * p.Np + n], i);
    }
    double c = 0.0;
    for (int i = 0; i < L::Qg; ++i)
      c += (double)GCodec<P>::dec(g[(int64_t)i * p.Np + n], p) + (P != 0 ? L::wg[i] * p.c0 : 0.0);
    const Fx3 a = fx3(m), b = fx3(c);
    ml += a.l; mm += a.m; mh += a.h;
    cl += b.l; cm += b.m; ch += b.h;
  }
  wave_chunks_add(d.tacc, ml, mm, mh);
  wave_chunks_add(d.tacc + 3, cl, cm, ch);
}

// Per bubble id: the number of its gas and interface cells and the fixed-point sums of
// w = 1 - alpha (its gas volume) and of w x, w y, w z (first moments of that volume).
template <int P>
__global__ __launch_bounds__(256) void k_bubble_stats(KP p, DA d) {
  using R = typename Prec<P>::R;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t start = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t n0 = start - (start & 63); n0 < p.N; n0 += stride) {
    const int64_t n = n0 + lane_id();
    bool on = false;
    int lab = 0;
    double w = 0.0;
    int x = 0, y = 0, z = 0;
    if (n < p.N) {
      const int t = d.type[n] & TMASK;
      lab = d.label[n];
      on = (t == TG || t == TI) && lab > 0 && lab < p.cap;
      if (on) {
        w = t == TG ? 1.0 : 1.0 - (double)((const R *)d.alpha)[n];
        cell_xyz(p, n, x, y, z);
      }
    }
    wave_count_add_ll(d.bstat, on, lab);
    wave_fx_add(d.bstat + 1, on, lab, fx3(w), nullptr, 13);
    wave_fx_add(d.bstat + 4, on, lab, fx3(w * x), nullptr, 13);
    wave_fx_add(d.bstat + 7, on, lab, fx3(w * y), nullptr, 13);
    wave_fx_add(d.bstat + 10, on, lab, fx3(w * z), nullptr, 13);
  }
}

// one element of a field in its storage form (fault-injection tests)
template <int D, int P>
__global__ void k_poke(KP p, DA d, int cur, int field, int64_t n, int comp, double v) {
  using R = typename Prec<P>::R;
  using SF = typename Prec<P>::SF;
  using SG = typename Prec<P>::SG;
  using L = Lat<D>;
  switch (field) {
    case MF_FIELD_F: ((SF *)d.f[cur])[(int64_t)comp * p.Np + n] = FCodec<P, D>::from_full(v, comp); break;
    case MF_FIELD_G:
      ((SG *)d.g[cur])[(int64_t)comp * p.Np + n] = GCodec<P>::enc((R)(v - (P != 0 ? L::wg[comp] * p.c0 : 0.0)), p);
      break;
    case MF_FIELD_RHO: ((R *)d.rho)[n] = (R)v; break;
    case MF_FIELD_ALPHA: ((R *)d.alpha)[n] = (R)v; break;
    case MF_FIELD_MASS: ((R *)d.M)[n] = (R)v; break;
    default: break;
  }
}

static unsigned grid_blocks(const Ctx &c) {
  int64_t b = (c.kp.N + 255) / 256;
  if (b > 65536) b = 65536;
  return (unsigned)(b < 1 ? 1 : b);
}

template <int D, int P>
void Ops<D, P>::init_box(Ctx &c, hipStream_t s) {
  hipLaunchKernelGGL((k_init_box<D, P>), dim3(grid_blocks(c)), dim3(256), 0, s, c.kp, c.d, c.P.gas_from);
  hipLaunchKernelGGL((k_nearwall<D>), dim3(grid_blocks(c)), dim3(256), 0, s, c.kp, c.d);
}

template <int D, int P>
void Ops<D, P>::nucleate(Ctx &c, hipStream_t s, int n, const double *centers, const double *radii) {
  hipLaunchKernelGGL((k_nuc_prep<P>), dim3(grid_blocks(c)), dim3(256), 0, s, c.kp, c.d);
  for (int k = 0; k < n; k++) {
    const double cx = centers[3 * k], cy = centers[3 * k + 1], cz = D == 3 ? centers[3 * k + 2] : 0.0;
    const double r = radii[k];
    const int x0 = (int)floor(cx - r - 1.0), y0 = (int)floor(cy - r - 1.0);
    const int z0 = D == 3 ? (int)floor(cz - r - 1.0) : 0;
    const int sx = (int)ceil(cx + r + 1.0) - x0 + 1, sy = (int)ceil(cy + r + 1.0) - y0 + 1;
    const int sz = D == 3 ? (int)ceil(cz + r + 1.0) - z0 + 1 : 1;
    const int64_t tot = (int64_t)sx * sy * sz;
    unsigned nb = (unsigned)((tot + 255) / 256);
    hipLaunchKernelGGL((k_nuc_voxel<D, P>), dim3(nb), dim3(256), 0, s, c.kp, c.d, k, cx, cy, cz, r, x0, y0, z0, sx,
                       sy, sz);
  }
  hipLaunchKernelGGL((k_nuc_apply<P>), dim3(grid_blocks(c)), dim3(256), 0, s, c.kp, c.d);
  hipLaunchKernelGGL((k_nuc_fix1<D>), dim3(grid_blocks(c)), dim3(256), 0, s, c.kp, c.d);
  hipLaunchKernelGGL((k_nuc_fix2<P>), dim3(grid_blocks(c)), dim3(256), 0, s, c.kp, c.d);
}

void launch_init_mass(Ctx &c, hipStream_t s, const double *p0_dev, int nn) {
  hipLaunchKernelGGL(k_init_mass, dim3(16), dim3(256), 0, s, c.kp, c.d, p0_dev, nn);
}

template <int D, int P>
void Ops<D, P>::build_lists(Ctx &c, hipStream_t s) {
  launch_list<0>(c, s);
}

template <int D, int P>
void Ops<D, P>::read_field(Ctx &c, hipStream_t s, int field, double *dst_dev) {
  hipLaunchKernelGGL((k_read<D, P>), dim3(grid_blocks(c)), dim3(256), 0, s, c.kp, c.d, c.cur, field, dst_dev);
}

template <int D, int P>
void Ops<D, P>::write_field(Ctx &c, hipStream_t s, int field, const double *src_dev) {
  hipLaunchKernelGGL((k_write<D, P>), dim3(grid_blocks(c)), dim3(256), 0, s, c.kp, c.d, c.cur, field, src_dev);
  if (field == MF_FIELD_TYPE) {
    hipLaunchKernelGGL((k_nearwall<D>), dim3(grid_blocks(c)), dim3(256), 0, s, c.kp, c.d);
  }
}

template <int D, int P>
void Ops<D, P>::totals(Ctx &c, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_ll, dim3(1), dim3(64), 0, s, c.d.tacc, (int64_t)6);
  int64_t b = (c.kp.N + 255) / 256;
  if (b > 4096) b = 4096;
  hipLaunchKernelGGL((k_totals<D, P>), dim3((unsigned)(b < 1 ? 1 : b)), dim3(256), 0, s, c.kp, c.d, c.cur);
}

template <int D, int P>
void Ops<D, P>::bubble_stats(Ctx &c, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_ll, dim3(64), dim3(256), 0, s, c.d.bstat, (int64_t)c.kp.cap * 13);
  int64_t b = (c.kp.N + 255) / 256;
  if (b > 4096) b = 4096;
  hipLaunchKernelGGL((k_bubble_stats<P>), dim3((unsigned)(b < 1 ? 1 : b)), dim3(256), 0, s, c.kp, c.d);
}

template <int D, int P>
void Ops<D, P>::poke(Ctx &c, hipStream_t s, int field, int64_t cell, int comp, double value) {
  hipLaunchKernelGGL((k_poke<D, P>), dim3(1), dim3(1), 0, s, c.kp, c.d, c.cur, field, cell, comp, value);
}

#define MF_INST(D, P)                                                                  \
  template void Ops<D, P>::init_box(Ctx &, hipStream_t);                               \
  template void Ops<D, P>::nucleate(Ctx &, hipStream_t, int, const double *, const double *); \
  template void Ops<D, P>::build_lists(Ctx &, hipStream_t);                            \
  template void Ops<D, P>::read_field(Ctx &, hipStream_t, int, double *);              \
  template void Ops<D, P>::write_field(Ctx &, hipStream_t, int, const double *);       \
  template void Ops<D, P>::totals(Ctx &, hipStream_t);                                 \
  template void Ops<D, P>::bubble_stats(Ctx &, hipStream_t);                           \
  template void Ops<D, P>::poke(Ctx &, hipStream_t, int, int64_t, int, double);
MF_FOR_ALL(MF_INST)

}  // namespace mf

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

// interface and bubble lists of the current types (the sweep builds them every step;
// this full pass serves initial and hand-written states)
// Interface list (type I) and bubble list (gas or interface with a non-zero bubble id),
// each in cell order within a chunk of LIST_CHUNK cells per block: a first pass counts,
// one atomic per block and list reserves the block's range, a second pass writes.
constexpr int LIST_CHUNK = 16384;

__device__ __forceinline__ void list_preds(const KP &p, const DA &d, int64_t n, bool &pi, bool &pb) {
  pi = pb = false;
  if (n >= p.N) return;
  const int t = d.type[n] & TMASK;
  pi = t == TI;
  pb = (t == TG || t == TI) && d.label[n] != 0;
}

__global__ __launch_bounds__(256) void k_build_lists(KP p, DA d) {
  __shared__ int s_w[2][4];
  __shared__ int s_base[2];
  const int64_t c0 = (int64_t)blockIdx.x * LIST_CHUNK;
  const int64_t c1 = c0 + LIST_CHUNK < p.N ? c0 + LIST_CHUNK : p.N;
  const int lane = lane_id(), w = threadIdx.x >> 6;
  int ci = 0, cb = 0;
  for (int64_t n = c0 + threadIdx.x; n < c1; n += 256) {
    bool pi, pb;
    list_preds(p, d, n, pi, pb);
    ci += pi;
    cb += pb;
  }
  for (int o = 32; o > 0; o >>= 1) {
    ci += __shfl_xor(ci, o);
    cb += __shfl_xor(cb, o);
  }
  if (lane == 0) {
    s_w[0][w] = ci;
    s_w[1][w] = cb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int ti = s_w[0][0] + s_w[0][1] + s_w[0][2] + s_w[0][3];
    const int tb = s_w[1][0] + s_w[1][1] + s_w[1][2] + s_w[1][3];
    s_base[0] = ti ? atomicAdd(d.cnt + C_I, ti) : 0;
    s_base[1] = tb ? atomicAdd(d.cnt + C_B, tb) : 0;
  }
  __syncthreads();
  int oi = s_base[0], ob = s_base[1];
  const unsigned long long lt = (1ull << lane) - 1ull;
  for (int64_t n0 = c0; n0 < c1; n0 += 256) {
    bool pi, pb;
    list_preds(p, d, n0 + threadIdx.x, pi, pb);
    const unsigned long long bi = __ballot(pi), bb = __ballot(pb);
    __syncthreads();  // the previous iteration has read s_w
    if (lane == 0) {
      s_w[0][w] = __popcll(bi);
      s_w[1][w] = __popcll(bb);
    }
    __syncthreads();
    int pre_i = 0, pre_b = 0, all_i = 0, all_b = 0;
    for (int k = 0; k < 4; ++k) {
      if (k < w) {
        pre_i += s_w[0][k];
        pre_b += s_w[1][k];
      }
      all_i += s_w[0][k];
      all_b += s_w[1][k];
    }
    if (pi) d.ilist[oi + pre_i + __popcll(bi & lt)] = (int32_t)(n0 + threadIdx.x);
    if (pb) d.blist[ob + pre_b + __popcll(bb & lt)] = (int32_t)(n0 + threadIdx.x);
    oi += all_i;
    ob += all_b;
  }
}

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
  const int64_t nb = (c.kp.N + LIST_CHUNK - 1) / LIST_CHUNK;
  hipLaunchKernelGGL(k_build_lists, dim3((unsigned)nb), dim3(256), 0, s, c.kp, c.d);
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

#define MF_INST(D, P)                                                                  \
  template void Ops<D, P>::init_box(Ctx &, hipStream_t);                               \
  template void Ops<D, P>::nucleate(Ctx &, hipStream_t, int, const double *, const double *); \
  template void Ops<D, P>::build_lists(Ctx &, hipStream_t);                            \
  template void Ops<D, P>::read_field(Ctx &, hipStream_t, int, double *);              \
  template void Ops<D, P>::write_field(Ctx &, hipStream_t, int, const double *);
MF_FOR_ALL(MF_INST)

}  // namespace mf

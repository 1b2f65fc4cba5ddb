// Internal definitions of libmifoam: lattice and storage traits, the device-array
// bundle, kernel parameters and wave-level helpers. gfx950 only (wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/mifoam.h"

namespace mf {

// ------------------------------------------------------------------ cell encoding
// type byte: bits 0-1 cell type (mf_cell_type), bit 2 = static "touches a wall" flag
constexpr uint8_t TG = 0, TI = 1, TL = 2, TW = 3;
constexpr uint8_t TMASK = 3, NEARWALL = 4;
// conversion flag byte (one per cell; zero between steps)
constexpr uint32_t CF_FILL = 1, CF_EMPTY = 2, CF_NEWI = 4, CF_L2I = 8, CF_ATM = 16,
                   CF_ATMROOT = 32, CF_VALID = 64, CF_MLPOK = 128;
// interface cell next to a filled or emptied cell (excess redistribution); shares its bit
// with CF_VALID: it lives only from the excess split to the flag clear at the start of the
// labelling, and CF_VALID only within a relabelling after that
constexpr uint32_t CF_EXNB = CF_VALID;
constexpr int32_t NOLAB = -1;

// status bits raised by kernels
constexpr int ST_INVARIANT = 1;   // liquid next to gas, or gas neighbour of another bubble
constexpr int ST_TABLE = 2;       // bubble table / hash / entry capacity exceeded
constexpr int ST_NONFINITE = 4;   // non-finite density at an interface cell
constexpr int ST_BADLABEL = 8;    // interface cell with an invalid bubble id

// counters
// C_TOPO: set when this step's conversions may have merged, split or removed a component;
// the ids of every such component are then marked in d.aff, unless C_FULL is set too
// (every component is relabelled)
// per-step counters (all cleared at the start of a step)
enum { C_I = 0, C_B, C_NI, C_L2I, C_ENTRIES, C_ROOTS, C_CONTESTED, C_TOPO, C_TCAND, C_CONV, C_FULL, C_NCOUNT = 16 };
// capacity of the list of filling cells whose neighbourhood the topology test examines
constexpr int TCAND_CAP = 65536;

// ------------------------------------------------------------------ lattices
// D2Q9 / D3Q19 velocity sets and weights (Sec. 2); the ADE lattices D2Q5 / D3Q7 are
// their rest and axis directions with weights giving c_s^2 = 1/3 and 1/4 (Sec. 3.1).
template <int D> struct Lat;
template <> struct Lat<2> {
  static constexpr int Q = 9, Qg = 5;
  static constexpr int ex[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
  static constexpr int ey[9] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
  static constexpr int ez[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  static constexpr double w[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                                  1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
  static constexpr double wg[5] = {1.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0};
  static constexpr double kg = 3.0;
};
template <> struct Lat<3> {
  static constexpr int Q = 19, Qg = 7;
  static constexpr int ex[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  static constexpr int ey[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  static constexpr int ez[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  static constexpr double w[19] = {1.0 / 3.0,  1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
                                   1.0 / 18.0, 1.0 / 18.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                                   1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                                   1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
  static constexpr double wg[7] = {0.25, 0.125, 0.125, 0.125, 0.125, 0.125, 0.125};
  static constexpr double kg = 4.0;
};
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// ------------------------------------------------------------------ precision
// P = 0 binary64 throughout; 1 binary32; 2 binary16 offsets f - w; 3 bfloat16 offsets;
// 4 binary16 offsets for f and binary16 scaled offsets (g - w c0) / s_g for g.
template <int P> struct Prec;
template <> struct Prec<0> { using R = double; using SF = double; using SG = double; };
template <> struct Prec<1> { using R = float; using SF = float; using SG = float; };
template <> struct Prec<2> { using R = float; using SF = _Float16; using SG = float; };
template <> struct Prec<3> { using R = float; using SF = uint16_t; using SG = float; };
template <> struct Prec<4> { using R = float; using SF = _Float16; using SG = _Float16; };

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  uint32_t r = u + 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even (finite inputs)
  return (uint16_t)(r >> 16);
}

// Population codec. The binary64 instance stores and computes f itself. The binary32
// and 16-bit instances store and compute offsets from the fluid at rest,
// f_i - w_i and g_i - w_i c0: a cell at rest is then exactly zero, so rounding cannot
// create mass or gas there, and the small offsets keep their relative precision in
// 16-bit storage. dec/enc convert between storage and the register convention.
template <int P, int D> struct FCodec {
  using R = typename Prec<P>::R;
  using SF = typename Prec<P>::SF;
  static constexpr bool SHIFT = P != 0;
  static __device__ __forceinline__ R dec(SF s, int) {
    if constexpr (P == 0 || P == 1) return s;
    else if constexpr (P == 2 || P == 4) return (float)s;
    else return bf16_to_f32(s);
  }
  static __device__ __forceinline__ SF enc(R v, int) {
    if constexpr (P == 0 || P == 1) return v;
    else if constexpr (P == 2 || P == 4) return (_Float16)v;
    else return f32_to_bf16(v);
  }
  // full population value in binary64 (field transfer)
  static __device__ __forceinline__ double full(SF s, int i) {
    if constexpr (P == 0) return s;
    else return Lat<D>::w[i] + (double)dec(s, i);
  }
  static __device__ __forceinline__ SF from_full(double v, int i) {
    if constexpr (P == 0) return v;
    else return enc((R)(v - Lat<D>::w[i]), i);
  }
};

// Dissolved-gas codec: instances 1-3 store the binary32 offsets g_i - w_i c0 as they
// are; instance 4 stores them divided by s_g (the initial concentration) in binary16,
// so that the relative precision of the stored offsets does not depend on the level
// of dissolved gas.
template <int P> struct GCodec {
  using R = typename Prec<P>::R;
  using SG = typename Prec<P>::SG;
  template <class K> static __device__ __forceinline__ R dec(SG s, const K &p) {
    if constexpr (P == 4) return (float)s * p.gsc;
    else return s;
  }
  template <class K> static __device__ __forceinline__ SG enc(R v, const K &p) {
    if constexpr (P == 4) return (_Float16)(v * p.ginv);
    else return (SG)v;
  }
};

// ------------------------------------------------------------------ parameters
struct KP {
  int dim, nx, ny, nz;
  int per[3];
  int64_t N, Np;  // cells, padded plane stride
  int cap;        // bubble-table capacity
  int H;          // pair-hash capacity (power of two)
  int ecap;       // entry capacity of the bubble update
  int RH;         // root-hash capacity of the bubble update (power of two)
  int rheology, cleanup, curvature;
  double omega, omega_g;
  double sigma, kH, RT, k_pi, d_max, p_atm, q, eps, c0;
  double pl_n, pl_nu_ref, pl_gdot_ref, tau_min, tau_max;
  float gsc, ginv;  // dissolved-gas storage scale s_g and 1/s_g (instance 4)
  float pl_l2nu3;   // log2(3 nu_ref) (power law, binary32 instances)
  float pl_kg;      // (3 / sqrt 2) / gdot_ref: shear rate = pl_kg |Pi_neq| / (rho tau) gdot_ref
  double cy_tau0, cy_tau_inf, cy_lambda, cy_a, cy_n;  // Carreau-Yasuda
  float cy_lk;      // lambda (3 / sqrt 2): lambda gdot = cy_lk |Pi_neq| / (rho tau)
  float cy_m;       // (n - 1) / a
  int force;        // body-force acceleration a is non-zero
  int flux_paper;   // gas flux of Eq. gascurrent as printed instead of the ledger
  double ax, ay, az;
  float fax, fay, faz;
  // binary32 copies of the parameters the binary32 collision reads, rounded once on the
  // host: a binary64 argument converted inside a kernel costs a vector instruction at
  // every use
  float omega_f, omega_g_f, pl_n_f, tau_min_f, tau_max_f;
  float c0_f, q_f, c0g_f, qg_f;               // c0 and q, and both times 1/s_g (instance 4)
  float cy_tau0_f, cy_tau_inf_f, cy_a_f, cy_w_f;  // Carreau-Yasuda; w = (tau0 - tau_inf)(1 - n)
  float pl_ninv;                              // 1 / n (power law)
  int pl_nit;              // Newton iterations of the binary32 power-law tau
};

struct DA {
  void *f[2], *g[2];
  uint8_t *type, *cflag;
  void *M, *alpha, *rho, *ux, *uy, *uz, *kappa, *Pi, *exc, *mx, *my, *mz, *soff;
  // gas side of each interface cell for the next sweep: density 3 (p_b - 2 sigma kappa - Pi)
  // and bubble pressure p_b, set with the geometry
  void *rgas, *pbub;
  int32_t *label;
  // union-find parent of each cell of the bubble list on a relabelling step; a cell that
  // filled this step holds its former id there until the topology test has read it
  int32_t *parent;
  uint8_t *aff;               // ids whose components the conversions may have changed [cap]
  int32_t *ilist, *blist, *nilist, *l2ilist;
  int32_t *clist;             // interface cells that fill or empty this step (sweep appends)
  int32_t *lcnt;              // per-chunk counts / offsets of the list builder [chunks]
  int32_t *nextid;            // next unused bubble id (persistent)
  int32_t *bng;               // gas cells of each bubble id [cap]
  uint32_t *wmask;            // static: bit i set when the source x - e_i of the cell is a wall
  int32_t *cnt;
  int32_t *status;
  // bubble table
  double *bm, *bV, *bp;
  int32_t *balive;
  double *mprime;
  int32_t *alive_prev;
  long long *phi, *gam;       // per-id step accumulators [cap][3]
  long long *phi0, *gam0;     // copies of the id-0 entries [NSPREAD][3]
  int32_t *tcand;             // filling cells for the window topology test [TCAND_CAP]
  long long *led;             // per-step ledger accumulators [3][3]: lost, atm, collapsed
  __int128 *ledtot;           // persistent ledgers [3]
  // bubble-update scratch
  unsigned long long *hkeys;  // [H]
  long long *hvals;           // [H][3]
  int32_t *hslot;             // used hash slots, in insertion order [ecap]
  int32_t *ent_root, *ent_lab, *ent_next, *ent_flag; // [ecap]
  long long *ent_v;           // [ecap][3]
  int32_t *lab_cnt;           // non-atmosphere components containing each id [cap]
  int32_t *lab_first;         // smallest non-atmosphere root containing each id [cap]
  int32_t *lab_assigned;      // [cap]
  long long *lab_vtot, *lab_vatm; // [cap][3]
  long long *vacc;            // per-id volume sums of the labelling fast path [cap][3], zero between steps
  int32_t *rh_key, *rh_head;  // root hash [RH]
  int32_t *rused;             // used root-hash slots [ecap]
  int32_t *contested;         // [ecap]
  double *scratch_d;          // [cap] spare
  long long *tacc;            // liquid mass and dissolved gas, fixed point [2][3]
  long long *bstat;           // per id: cell count, then Fx3 sums of w, w x, w y, w z
                              // (w = 1 - alpha) [cap][13]
  // learned curvature (NULL unless a network is attached)
  const uint16_t *mlp_w;      // bfloat16 W1 [128][64], W2 [64][64], W3 [64]
  const float *mlp_b;         // b1 [64], b2 [64], b3
  uint32_t *sword;            // stencil word of every cell (learned curvature only; see stencil_word)
};

// ------------------------------------------------------------------ fixed point
// Order-independent sums: v -> RN(v 2^64) as a signed 128-bit integer, held as three
// signed 64-bit chunks (low 32 bits, next 32 bits, high part) so that chunk-wise
// atomic adds never lose a carry.
struct Fx3 { long long l, m, h; };
__device__ __host__ __forceinline__ Fx3 fx3(double v) {
  double s = rint(v * 18446744073709551616.0);
  double a = s < 0 ? -s : s;
  double h = floor(a * 0x1p-64);
  double r = a - h * 18446744073709551616.0;  // exact, in [0, 2^64)
  double m = floor(r * 0x1p-32);
  double l = r - m * 4294967296.0;
  Fx3 o;
  o.l = (long long)l;
  o.m = (long long)m;
  o.h = (long long)h;
  if (s < 0) { o.l = -o.l; o.m = -o.m; o.h = -o.h; }
  return o;
}
__device__ __host__ __forceinline__ __int128 fx3_join(long long l, long long m, long long h) {
  return (__int128)h * ((__int128)1 << 64) + (__int128)m * ((__int128)1 << 32) + (__int128)l;
}
__device__ __host__ __forceinline__ double fx_to_double(__int128 v) { return (double)v * 0x1p-64; }

// ------------------------------------------------------------------ wave helpers
__device__ __forceinline__ int lane_id() { return __lane_id(); }

// order LDS accesses of the lanes of one wave (no other wave involved)
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Id 0 (the atmosphere) takes a term from nearly every wave along the free surface; with
// `spread0` its sums go to one of NSPREAD copies chosen by work-group, so that no address
// takes thousands of atomics in one step (same-address atomics from different XCDs are
// serialised far from the CUs). The reader adds the copies word by word, exactly.
constexpr int NSPREAD = 64;

// add a fixed-point value to acc[key*3 .. +2] for every lane with pred; lanes that share
// a key are summed inside the wave first. Called by the whole wave.
__device__ __forceinline__ void wave_fx_add(long long *acc, bool pred, int key, Fx3 v,
                                            long long *spread0 = nullptr, int stride = 3) {
  unsigned long long act = __ballot(pred);
  int lane = lane_id();
  while (act) {
    int leader = __ffsll((long long)act) - 1;
    int k = __shfl(key, leader);
    bool mine = pred && key == k;
    unsigned long long mm = __ballot(mine);
    long long sl = mine ? v.l : 0, sm = mine ? v.m : 0, sh = mine ? v.h : 0;
    for (int off = 32; off > 0; off >>= 1) {
      sl += __shfl_xor(sl, off);
      sm += __shfl_xor(sm, off);
      sh += __shfl_xor(sh, off);
    }
    if (lane == leader) {
      long long *dst = k == 0 && spread0 ? spread0 + 3 * (blockIdx.x & (NSPREAD - 1)) : acc + (int64_t)stride * k;
      atomicAdd((unsigned long long *)&dst[0], (unsigned long long)sl);
      atomicAdd((unsigned long long *)&dst[1], (unsigned long long)sm);
      atomicAdd((unsigned long long *)&dst[2], (unsigned long long)sh);
    }
    act &= ~mm;
    pred = pred && !mine;
  }
}

// The same sum for keys (>= 0) that come in runs of neighbouring lanes, as along a list in
// cell order: a segmented scan over the runs (six shuffle steps whatever the number of
// keys) and one atomic per run from its last lane. Called by the whole wave.
__device__ __forceinline__ void wave_fx_add_runs(long long *acc, bool pred, int key, Fx3 v,
                                                 long long *spread0 = nullptr) {
  const int lane = lane_id();
  const int kk = pred ? key : -1;
  const int prev = __shfl_up(kk, 1), next = __shfl_down(kk, 1);
  const unsigned long long heads = __ballot(lane == 0 || prev != kk);
  const int seg = __popcll(heads & ((2ull << lane) - 1ull));  // runs that start at or below
  long long l = pred ? v.l : 0, m = pred ? v.m : 0, h = pred ? v.h : 0;
  for (int o = 1; o < 64; o <<= 1) {
    const long long al = __shfl_up(l, o), am = __shfl_up(m, o), ah = __shfl_up(h, o);
    const int so = __shfl_up(seg, o);
    if (lane >= o && so == seg) {
      l += al;
      m += am;
      h += ah;
    }
  }
  if (pred && (lane == 63 || next != kk)) {
    long long *dst = kk == 0 && spread0 ? spread0 + 3 * (blockIdx.x & (NSPREAD - 1)) : acc + 3 * kk;
    atomicAdd((unsigned long long *)&dst[0], (unsigned long long)l);
    atomicAdd((unsigned long long *)&dst[1], (unsigned long long)m);
    atomicAdd((unsigned long long *)&dst[2], (unsigned long long)h);
  }
}

__device__ __forceinline__ void raise_status(int32_t *st, int bits) { atomicOr(st, bits); }

// add the wave-uniform v to acc[key] for every lane with pred, one atomic per key and
// wave. Called by the whole wave.
__device__ __forceinline__ void wave_count_add(int32_t *acc, bool pred, int key, int v) {
  unsigned long long act = __ballot(pred);
  while (act) {
    const int leader = __ffsll((long long)act) - 1;
    const int k = __shfl(key, leader);
    const unsigned long long mm = __ballot(pred && key == k);
    if (lane_id() == leader) atomicAdd(&acc[k], v * (int)__popcll(mm));
    act &= ~mm;
    pred = pred && key != k;
  }
}

// add one to acc[13 * key] (64-bit) for every lane with pred, one atomic per key and
// wave. Called by the whole wave.
__device__ __forceinline__ void wave_count_add_ll(long long *acc, bool pred, int key) {
  unsigned long long act = __ballot(pred);
  while (act) {
    const int leader = __ffsll((long long)act) - 1;
    const int k = __shfl(key, leader);
    const unsigned long long mm = __ballot(pred && key == k);
    if (lane_id() == leader) atomicAdd((unsigned long long *)&acc[13 * (int64_t)k], (unsigned long long)__popcll(mm));
    act &= ~mm;
    pred = pred && key != k;
  }
}

// a slot of a device-counted list for every lane with pred, with one atomic per wave;
// called by the whole wave
__device__ __forceinline__ int wave_append_slot(int32_t *counter, bool pred) {
  const unsigned long long m = __ballot(pred);
  if (!m) return -1;
  const int leader = __ffsll((long long)m) - 1;
  int base = 0;
  if (lane_id() == leader) base = atomicAdd(counter, __popcll(m));
  base = __shfl(base, leader);
  return base + (int)__popcll(m & ((1ull << lane_id()) - 1ull));
}

// byte flags through 32-bit atomics on the containing word
__device__ __forceinline__ uint32_t flag_or(uint8_t *cflag, int64_t n, uint32_t bits) {
  uint32_t *w = (uint32_t *)(cflag + (n & ~(int64_t)3));
  int sh = 8 * (int)(n & 3);
  return (atomicOr(w, bits << sh) >> sh) & 0xFFu;
}
__device__ __forceinline__ void flag_clear(uint8_t *cflag, int64_t n, uint32_t bits) {
  uint32_t *w = (uint32_t *)(cflag + (n & ~(int64_t)3));
  int sh = 8 * (int)(n & 3);
  atomicAnd(w, ~(bits << sh));
}

// ------------------------------------------------------------------ indexing
// neighbour of cell (x,y,z) at offset (dx,dy,dz) with periodic wrap; closed axes never
// wrap for non-wall cells because the wall layer bounds them
__device__ __forceinline__ int64_t nb_index(const KP &p, int x, int y, int z, int dx, int dy, int dz) {
  int X = x + dx, Y = y + dy, Z = z + dz;
  if (X < 0) X += p.nx; else if (X >= p.nx) X -= p.nx;
  if (Y < 0) Y += p.ny; else if (Y >= p.ny) Y -= p.ny;
  if (Z < 0) Z += p.nz; else if (Z >= p.nz) Z -= p.nz;
  return (int64_t)X + (int64_t)p.nx * ((int64_t)Y + (int64_t)p.ny * Z);
}
// offset that may leave a closed axis (curvature and traversal stencils): -1 outside
__device__ __forceinline__ int64_t nb_index_or_none(const KP &p, int x, int y, int z, int dx, int dy, int dz) {
  int X = x + dx, Y = y + dy, Z = z + dz;
  if (X < 0 || X >= p.nx) { if (!p.per[0]) return -1; X = (X + p.nx) % p.nx; }
  if (Y < 0 || Y >= p.ny) { if (!p.per[1]) return -1; Y = (Y + p.ny) % p.ny; }
  if (Z < 0 || Z >= p.nz) { if (p.dim == 2 || !p.per[2]) return -1; Z = (Z + p.nz) % p.nz; }
  return (int64_t)X + (int64_t)p.nx * ((int64_t)Y + (int64_t)p.ny * Z);
}
__device__ __forceinline__ void cell_xyz(const KP &p, int64_t n, int &x, int &y, int &z) {
  x = (int)(n % p.nx);
  int64_t r = n / p.nx;
  y = (int)(r % p.ny);
  z = (int)(r / p.ny);
}

// ------------------------------------------------------------------ launch geometry
// Position of a work-group in the grid of one domain. A launch for one domain uses the
// hardware indices; a launch over several domains (a batch) gives each domain a range
// of work-groups and maps every work-group to its domain and local index. Kernel bodies
// take it as `gp` and never read blockIdx / gridDim themselves.
struct GridPos {
  int64_t bid, nblk;
  static __device__ __forceinline__ GridPos hw() { return GridPos{(int64_t)blockIdx.x, (int64_t)gridDim.x}; }
};

// grid-stride loop bounds over a device-counted list
#define LIST_LOOP(idx, countptr)                                                   \
  for (int64_t idx = gp.bid * blockDim.x + threadIdx.x,                             \
               _n = (int64_t)(*(volatile int32_t *)(countptr));                    \
       idx < ((_n + 63) & ~(int64_t)63); idx += gp.nblk * blockDim.x)

// The same over a short list (a few thousand entries), with the entries dealt lane-major
// over the waves of the grid: lanes of one wave take entries a wave-count apart, so the
// scattered work spreads over every CU instead of a few full waves, and the atomics of
// neighbouring cells do not meet in one instruction. Wave-uniform bounds; idx may exceed
// the count (test it).
#define SPREAD_LOOP_N(idx, count)                                                              \
  for (int64_t _T = gp.nblk * blockDim.x, _n = (int64_t)(count), _r0 = 0, idx = 0;               \
       _r0 < _n && (idx = _r0 + (int64_t)(threadIdx.x & 63) * (_T >> 6) +                      \
                          ((gp.bid * blockDim.x + threadIdx.x) >> 6), true);                    \
       _r0 += _T)
#define SPREAD_LOOP(idx, countptr) SPREAD_LOOP_N(idx, *(volatile int32_t *)(countptr))

// ------------------------------------------------------------------ launchers
// every kernel family is a template over (D, P); the dispatcher picks one instance
struct Ctx;
struct MStep;
template <int D, int P> struct Ops {
  // the lattice sweep: the bulk kernel (liquid cells; false when the domain takes the
  // per-cell kernel instead), the interface kernel (this step's interface list; after the
  // bulk kernel, whose whole-group stores cover interface cells too), and the per-cell
  // kernel over the whole grid
  static bool sweep_bulk_auto(Ctx &c, hipStream_t s);
  static void sweep_interface(Ctx &c, hipStream_t s);
  static void sweep_cells(Ctx &c, hipStream_t s);
  // one launch of the bulk sweep kernel in tuning variant v (see kSweepVariants); false
  // when the variant does not apply to this domain (nothing launched)
  static bool sweep_bulk(Ctx &c, hipStream_t s, int v);
  // the conversions: convert_head() changes the types and initialises the new interface
  // cells (all the next bulk sweep reads), convert_tail() runs the topology test, the excess
  // redistribution and the flag clear; convert() is both in order
  static void convert(Ctx &c, hipStream_t s);
  static void convert_head(Ctx &c, hipStream_t s);
  static void convert_tail(Ctx &c, hipStream_t s);
  static void label(Ctx &c, hipStream_t s, int apply_flux);
  static void geometry(Ctx &c, hipStream_t s);
  // the two halves of geometry(): normals (words: also the list cells' stencil words), and
  // curvature + disjoining pressure + gas side
  static void geometry_normals(Ctx &c, hipStream_t s, bool words);
  static void geometry_curv(Ctx &c, hipStream_t s);
  static void init_box(Ctx &c, hipStream_t s);
  static void nucleate(Ctx &c, hipStream_t s, int n, const double *centers, const double *radii);
  static void build_lists(Ctx &c, hipStream_t s);
  static void read_field(Ctx &c, hipStream_t s, int field, double *dst_dev);
  static void write_field(Ctx &c, hipStream_t s, int field, const double *src_dev);
  // liquid mass and dissolved gas over the grid into d.tacc (fixed point, cleared first)
  static void totals(Ctx &c, hipStream_t s);
  // per-id cell counts and gas-volume moments into d.bstat (cleared first)
  static void bubble_stats(Ctx &c, hipStream_t s);
  // overwrite one element of a field in its storage form
  static void poke(Ctx &c, hipStream_t s, int field, int64_t cell, int comp, double value);
  // batched forms (one launch per kernel for all domains of a batched step): the sweep (bulk kernel in every launch shape of vmask and the interface
  // kernel, or the per-cell kernel), the conversions, the labelling, the geometry
  static void sweep_multi(const MStep &ms, unsigned vmask, bool cells, bool frc, int part, hipStream_t s);
  static void convert_multi(const MStep &ms, int part, hipStream_t s);
  static void label_multi(const MStep &ms, hipStream_t s);
  static void geometry_multi(const MStep &ms, bool mlp, hipStream_t s);
  // the bulk kernel alone in launch shape v (it writes only the spare population buffer)
  static void bulk_multi(const MStep &ms, int v, bool frc, hipStream_t s);
};

struct Ctx {
  mf_params P;
  KP kp;
  DA d;
  int cur = 0;          // buffer holding the current post-collision populations
  hipStream_t stream = nullptr;
  void *ws = nullptr;
  bool own_ws = false;
  size_t ws_bytes = 0;
  bool nucleated = false;
  bool stepped = false;
  bool sword_dirty = true;  // stencil words to be rebuilt over the whole grid
  bool gas_dirty = false;   // bubble table changed since the gas side was last set
  int sweep_variant = -1;   // bulk-sweep variant chosen by the tuner (-1: default)
  uint64_t epoch = 0;       // bumped by every state change made outside mf_step
  int64_t step = 0;
  std::string err;
  bool prof = false;
  void *mlp_buf = nullptr;  // device copy of the attached network's weights
  // Steps overlap. After the first half of the conversions of step n (types and new
  // interface cells, on the context stream), the side stream takes the second half
  // (topology test, excess redistribution), the labelling and the curvature; side2 takes
  // the normals and then the counter reset and interface-list build of step n+1; the
  // context stream goes on with the bulk sweep of step n+1. None of them writes what
  // another reads. Counters and the interface list alternate between two copies by step
  // parity. The interface sweep waits for the side stream (ev_side) and the list build
  // (ev_list). ev_tail marks the end of the conversions' second half (the normals read the
  // fill fractions it writes). geometry_normals() records ev_norm_rec, when set.
  int32_t *cnt_base = nullptr, *ilist_base = nullptr;
  int parity = 0;
  hipStream_t side = nullptr;
  hipStream_t side2 = nullptr;  // the normals, beside the labelling on the side stream
  hipEvent_t ev_conv = nullptr, ev_side = nullptr, ev_norm = nullptr, ev_norm_rec = nullptr;
  bool sword_fresh = false;     // the excess pass of this step wrote the list cells' stencil words
  hipEvent_t ev_start = nullptr, ev_list = nullptr;  // step start (context stream), list built (third stream)
  hipEvent_t ev_tail = nullptr;
  bool list_pending = false;    // the interface sweep must wait for ev_list
  bool side_pending = false;  // ev_side marks side-stream work the main stream has not joined
};

// every (dimension, precision) instance the library is built with
#define MF_FOR_ALL(M) M(2, 0) M(2, 1) M(2, 2) M(2, 3) M(2, 4) M(3, 0) M(3, 1) M(3, 2) M(3, 3) M(3, 4)

// message of the last failed call on this thread that has no context
extern thread_local std::string g_thread_err;

// bulk-sweep variants the tuner chooses from: cells per thread x threads per work-group
struct SweepVariant { int vw, bs; };
constexpr SweepVariant kSweepVariants[] = {{4, 256}, {2, 256}, {4, 128}, {2, 128}, {8, 256}, {8, 128}, {8, 64}, {4, 64}};
constexpr int kNumSweepVariants = 8;

// whether the bulk kernel with vw cells per thread can sweep a domain: 16-bit or binary32
// storage, closed axes, rows a multiple of vw long
inline bool bulk_shape_ok(const KP &kp, int precision, int vw) {
  if (precision == 0) return false;
  if (kp.per[0] || kp.per[1] || kp.per[2]) return false;
  return kp.nx % vw == 0 && kp.nx >= 2 * vw && kp.ny >= 3 && (kp.dim == 2 || kp.nz >= 3);
}
// Inside a time step the bulk kernel runs beside the labelling, normals and curvature
// kernels of the side streams. Work-groups of 256 threads let those kernels take over the
// slots of a retired bulk work-group; with one-wave work-groups the bulk kernel refills
// every freed slot at once and starves them, which costs more than the one-wave shapes
// gain alone. Hence the tuner of a context chooses among the 256-thread shapes.
inline bool step_variant(int v) { return kSweepVariants[v].bs == 256; }
// the launch shape used when none was chosen by the tuner: 16-byte population accesses
// per lane for 16-bit storage (8 cells per thread) and for binary32 (4 cells per thread);
// measured fastest inside the step on the 384^3 foam
inline int default_sweep_variant(int precision) { return precision == 1 ? 0 : 4; }
// the launch shape a domain is swept with: the tuned one, else the default, else narrower
// vectors for rows whose length is not a multiple of 8 cells; -1: the per-cell kernel
inline int effective_sweep_variant(const KP &kp, int precision, int tuned) {
  const int order[4] = {tuned, default_sweep_variant(precision), 0, 1};
  for (int v : order)
    if (v >= 0 && bulk_shape_ok(kp, precision, kSweepVariants[v].vw)) return v;
  return -1;
}

// work-groups of the list builder (one per chunk of cells)
int list_blocks_of(const KP &kp);

// ------------------------------------------------------------------ batched launches
// A batch advances many domains with one launch per kernel of the step: every domain
// takes the range of work-groups it would take alone, and each work-group finds its
// domain by a binary search over the ranges. One domain of such a launch, for one step:
// its parameters, its arrays (with the counters and interface list of the step's
// parity) and the buffer holding the post-collision populations the step starts from.
struct MDom {
  KP kp;
  DA d;
  int cur;
};
// launch kinds of a step (the grid formula of each launch of one domain); the bulk sweep
// has one kind per launch shape, with no work-groups for domains that use another shape
enum MKind {
  MK_ONE = 0,   // one work-group
  MK_LISTGRID,  // list builder passes: min(chunks, 1024)
  MK_LIST,      // passes over the interface list: list_blocks
  MK_SHORT,     // passes over short lists: min(list_blocks, 1024)
  MK_TOPOW,     // topology windows: 256
  MK_BFAST,     // bubble table pass: min(ceil(cap / 256), 64)
  MK_MLP,       // learned curvature: one work-group per 65536 cells, at most 768
  MK_CELLS,     // per-cell sweep: 64 x 4 tiles
  MK_BULK0,     // bulk sweep in launch shape v: MK_BULK0 + v
  MK_COUNT = MK_BULK0 + kNumSweepVariants
};
constexpr int kMaxBatchDomains = 64;  // domains per batched launch
// the launch arguments: the domain table and, for the launch's kind, the first
// work-group of every domain (passed by value, so the search reads the kernel arguments)
struct MLaunch {
  const MDom *dom;  // device [nd]
  int nd;
  int pre[kMaxBatchDomains + 1];
};
// the domain of this work-group, and its local position
__device__ __forceinline__ GridPos multi_pos(const MLaunch &ml, int kind, int &dom) {
  (void)kind;
  const int *pre = ml.pre;
  const int b = (int)blockIdx.x;
  int lo = 0, hi = ml.nd;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= b) lo = mid;
    else hi = mid;
  }
  dom = __builtin_amdgcn_readfirstlane(lo);
  return GridPos{(int64_t)(b - pre[dom]), (int64_t)(pre[dom + 1] - pre[dom])};
}
#define MF_MULTI(kind)                                   \
  int _dom = 0;                                          \
  const GridPos gp = multi_pos(ml, (kind), _dom);        \
  const MDom &m = ml.dom[_dom];

// the arguments of a batched launch of kind k: pre holds the prefix sums of every kind,
// [MK_COUNT][nd + 1]
inline MLaunch mlaunch(const MDom *dom, int nd, const int *pre, int kind) {
  MLaunch ml;
  ml.dom = dom;
  ml.nd = nd;
  for (int i = 0; i <= nd; ++i) ml.pre[i] = pre[kind * (nd + 1) + i];
  return ml;
}
// A batched step: the domain table of the step, the prefix sums of every kind and the
// work-groups of every kind over the batch
struct MStep {
  const MDom *dom;
  int nd;
  const int *pre;   // host [MK_COUNT][nd + 1]
  const int *grid;  // host [MK_COUNT]
  MLaunch at(int kind) const { return mlaunch(dom, nd, pre, kind); }
};

// batched launches of the list builder (which: 0 interface list, 1 bubble list) and of
// the counter reset
void lists_multi(const MStep &ms, int which, hipStream_t s);
void reset_multi(const MStep &ms, hipStream_t s);
void mlp_curv_multi(const MStep &ms, int precision, hipStream_t s);
// the bubble list (gas / interface cells with a non-zero id) on a relabelling step
void build_bubble_list(const Ctx &c, hipStream_t s);
// gas cells of every bubble id counted over the whole grid
void recount_gas(const Ctx &c, hipStream_t s);

// Stencil word of a cell, read by the learned curvature's 5x5x5 gather in one load:
// bits 0-15 the bfloat16 (nearest even) of the fill fraction a stencil reads there (1 for
// liquid, 0 for gas, the clamped alpha for interface), bits 16-31 a code: 0 for liquid,
// bubble id + 1 for gas and interface, 0xFFFF for a wall.
template <class R>
__device__ __forceinline__ uint32_t stencil_word(uint8_t tb, R alpha, int32_t lab) {
  const int t = tb & TMASK;
  if (t == TW) return 0xFFFF0000u;
  if (t == TL) return (uint32_t)f32_to_bf16(1.0f);
  const float v = t == TG ? 0.0f : fminf(1.0f, fmaxf(0.0f, (float)alpha));
  return ((uint32_t)((lab + 1) & 0xFFFF) << 16) | (uint32_t)f32_to_bf16(v);
}

// learned-curvature inference over the new interface cells (3D)
void launch_mlp_curv(Ctx &c, hipStream_t s);

// table of canonical stencil slots for the 48 cube symmetries (48 x 128 bytes)

// initial gas content and pressure of the nucleus ids 1..nn (p0 in device memory)
void launch_init_mass(Ctx &c, hipStream_t s, const double *p0_dev, int nn);

// list-kernel launch size: enough waves to cover the worst case but bounded
inline unsigned list_blocks(const Ctx &c) {
  int64_t b = (c.kp.N + 255) / 256;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace mf

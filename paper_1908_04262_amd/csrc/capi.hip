// C ABI of libmifoam (declared in include/mifoam.h): context, device arena, the time
// step as a fixed sequence of kernel launches on the caller's stream, field transfer.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "mf_internal.h"

using namespace mf;

namespace mf {
thread_local std::string g_thread_err;
}

struct mf_mlp;
int mf_mlp_export_weights(const mf_mlp *m, uint16_t *w_dev, float *b_dev, hipStream_t s);

namespace {

std::string &g_err = mf::g_thread_err;

struct OpsTable {
  void (*convert)(Ctx &, hipStream_t);
  void (*label)(Ctx &, hipStream_t, int);
  void (*geometry)(Ctx &, hipStream_t);
  void (*init_box)(Ctx &, hipStream_t);
  void (*nucleate)(Ctx &, hipStream_t, int, const double *, const double *);
  void (*build_lists)(Ctx &, hipStream_t);
  void (*read_field)(Ctx &, hipStream_t, int, double *);
  void (*write_field)(Ctx &, hipStream_t, int, const double *);
  bool (*sweep_bulk)(Ctx &, hipStream_t, int);
  void (*geometry_normals)(Ctx &, hipStream_t, bool);
  void (*geometry_curv)(Ctx &, hipStream_t);
  bool (*sweep_bulk_auto)(Ctx &, hipStream_t);
  void (*sweep_interface)(Ctx &, hipStream_t);
  void (*sweep_cells)(Ctx &, hipStream_t);
  void (*totals)(Ctx &, hipStream_t);
  void (*bubble_stats)(Ctx &, hipStream_t);
  void (*poke)(Ctx &, hipStream_t, int, int64_t, int, double);
  void (*sweep_multi)(const MStep &, unsigned, bool, bool, int, hipStream_t);
  void (*convert_multi)(const MStep &, int, hipStream_t);
  void (*label_multi)(const MStep &, hipStream_t);
  void (*geometry_multi)(const MStep &, bool, hipStream_t);
  void (*bulk_multi)(const MStep &, int, bool, hipStream_t);
  void (*convert_head)(Ctx &, hipStream_t);
  void (*convert_tail)(Ctx &, hipStream_t);
};

template <int D, int P>
OpsTable make_ops() {
  return OpsTable{&Ops<D, P>::convert,     &Ops<D, P>::label,
                  &Ops<D, P>::geometry, &Ops<D, P>::init_box,    &Ops<D, P>::nucleate,
                  &Ops<D, P>::build_lists, &Ops<D, P>::read_field, &Ops<D, P>::write_field,
                  &Ops<D, P>::sweep_bulk,  &Ops<D, P>::geometry_normals, &Ops<D, P>::geometry_curv,
                  &Ops<D, P>::sweep_bulk_auto, &Ops<D, P>::sweep_interface, &Ops<D, P>::sweep_cells,
                  &Ops<D, P>::totals, &Ops<D, P>::bubble_stats, &Ops<D, P>::poke,
                  &Ops<D, P>::sweep_multi, &Ops<D, P>::convert_multi, &Ops<D, P>::label_multi,
                  &Ops<D, P>::geometry_multi, &Ops<D, P>::bulk_multi, &Ops<D, P>::convert_head,
                  &Ops<D, P>::convert_tail};
}

OpsTable ops_for(int dim, int prec) {
  if (dim == 2) {
    switch (prec) {
      case 0: return make_ops<2, 0>();
      case 1: return make_ops<2, 1>();
      case 2: return make_ops<2, 2>();
      case 3: return make_ops<2, 3>();
      default: return make_ops<2, 4>();
    }
  }
  switch (prec) {
    case 0: return make_ops<3, 0>();
    case 1: return make_ops<3, 1>();
    case 2: return make_ops<3, 2>();
    case 3: return make_ops<3, 3>();
    default: return make_ops<3, 4>();
  }
}

size_t sf_bytes(int prec) { return prec == 0 ? 8 : (prec == 1 ? 4 : 2); }
size_t sg_bytes(int prec) { return prec == 0 ? 8 : (prec == 4 ? 2 : 4); }
size_t r_bytes(int prec) { return prec == 0 ? 8 : 4; }
int next_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

// one bump allocator over the arena; with base == nullptr it only measures
struct Carve {
  char *base;
  size_t off = 0;
  explicit Carve(void *b) : base((char *)b) {}
  template <class T> T *take(size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    T *p = base ? (T *)(base + off) : nullptr;
    off += bytes;
    return p;
  }
};

void layout(const mf_params &P, const KP &kp, Carve &cv, DA &d) {
  const int Q = P.dim == 2 ? 9 : 19, Qg = P.dim == 2 ? 5 : 7;
  const size_t Np = (size_t)kp.Np;
  const size_t sf = sf_bytes(P.precision), sg = sg_bytes(P.precision), rb = r_bytes(P.precision);
  for (int b = 0; b < 2; b++) d.f[b] = cv.take<void>(Q * Np * sf);
  for (int b = 0; b < 2; b++) d.g[b] = cv.take<void>(Qg * Np * sg);
  d.type = cv.take<uint8_t>(Np);
  d.cflag = cv.take<uint8_t>(Np);
  void **rarr[] = {&d.M,  &d.alpha, &d.rho, &d.ux, &d.uy,   &d.uz,  &d.kappa, &d.Pi,
                   &d.exc, &d.mx,   &d.my,  &d.mz, &d.soff, &d.rgas, &d.pbub};
  for (void **a : rarr) *a = cv.take<void>(Np * rb);
  d.label = cv.take<int32_t>(Np * 4);
  d.parent = cv.take<int32_t>(Np * 4);
  d.ilist = cv.take<int32_t>(2 * Np * 4);  // two copies, alternating by step parity
  d.blist = cv.take<int32_t>(Np * 4);
  d.nilist = cv.take<int32_t>(Np * 4);
  d.l2ilist = cv.take<int32_t>(Np * 4);
  d.clist = cv.take<int32_t>(Np * 4);
  d.wmask = cv.take<uint32_t>(Np * 4);
  d.lcnt = cv.take<int32_t>((size_t)list_blocks_of(kp) * 4);
  d.sword = P.curvature == MF_CURV_MLP ? cv.take<uint32_t>(Np * 4) : nullptr;
  d.cnt = cv.take<int32_t>(2 * C_NCOUNT * 4);  // two sets, alternating by step parity
  d.nextid = cv.take<int32_t>(4);
  d.status = cv.take<int32_t>(4);
  const size_t cap = (size_t)kp.cap;
  d.bm = cv.take<double>(cap * 8);
  d.bV = cv.take<double>(cap * 8);
  d.bp = cv.take<double>(cap * 8);
  d.balive = cv.take<int32_t>(cap * 4);
  d.mprime = cv.take<double>(cap * 8);
  d.alive_prev = cv.take<int32_t>(cap * 4);
  d.phi = cv.take<long long>(cap * 24);
  d.gam = cv.take<long long>(cap * 24);
  d.phi0 = cv.take<long long>(NSPREAD * 24);
  d.gam0 = cv.take<long long>(NSPREAD * 24);
  d.tcand = cv.take<int32_t>((size_t)TCAND_CAP * 4);
  d.led = cv.take<long long>(9 * 8);
  d.ledtot = cv.take<__int128>(3 * 16);
  d.hkeys = cv.take<unsigned long long>((size_t)kp.H * 8);
  d.hvals = cv.take<long long>((size_t)kp.H * 24);
  d.hslot = cv.take<int32_t>((size_t)kp.ecap * 4);
  d.ent_root = cv.take<int32_t>((size_t)kp.ecap * 4);
  d.ent_lab = cv.take<int32_t>((size_t)kp.ecap * 4);
  d.ent_next = cv.take<int32_t>((size_t)kp.ecap * 4);
  d.ent_flag = cv.take<int32_t>((size_t)kp.ecap * 4);
  d.ent_v = cv.take<long long>((size_t)kp.ecap * 24);
  d.lab_cnt = cv.take<int32_t>(cap * 4);
  d.lab_first = cv.take<int32_t>(cap * 4);
  d.lab_assigned = cv.take<int32_t>(cap * 4);
  d.lab_vtot = cv.take<long long>(cap * 24);
  d.lab_vatm = cv.take<long long>(cap * 24);
  d.vacc = cv.take<long long>(cap * 24);
  d.bng = cv.take<int32_t>(cap * 4);
  d.rh_key = cv.take<int32_t>((size_t)kp.RH * 4);
  d.rh_head = cv.take<int32_t>((size_t)kp.RH * 4);
  d.contested = cv.take<int32_t>((size_t)kp.ecap * 4);
  d.rused = cv.take<int32_t>((size_t)kp.ecap * 4);
  d.scratch_d = cv.take<double>(cap * 8);
  d.tacc = cv.take<long long>(6 * 8);
  d.bstat = cv.take<long long>(cap * 13 * 8);
  d.aff = cv.take<uint8_t>(cap);
}

int validate(const mf_params *p, std::string &why) {
  if (!p) { why = "params is NULL"; return MF_EINVAL; }
  if (p->struct_size != sizeof(mf_params)) { why = "struct_size does not match this library's mf_params"; return MF_EINVAL; }
  if (p->dim != 2 && p->dim != 3) { why = "dim must be 2 or 3"; return MF_EINVAL; }
  const int nz = p->dim == 2 ? 1 : p->nz;
  if (p->nx < 3 || p->ny < 3 || nz < 1 || (p->dim == 3 && nz < 3)) { why = "grid too small"; return MF_EINVAL; }
  if ((double)p->nx * p->ny * nz >= 2147483647.0) { why = "grid exceeds 2^31 cells"; return MF_EINVAL; }
  if (p->precision < 0 || p->precision > 4) { why = "unknown precision"; return MF_EINVAL; }
  if (p->rheology != MF_NEWTONIAN && p->rheology != MF_POWER_LAW && p->rheology != MF_CARREAU_YASUDA) { why = "unknown rheology"; return MF_EINVAL; }
  if (p->rheology == MF_CARREAU_YASUDA &&
      !(p->cy_tau_inf > 0.5 && p->cy_tau0 >= p->cy_tau_inf && p->cy_tau0 < 1e6 && p->cy_n > 0.0 && p->cy_n <= 1.0 &&
        p->cy_a > 0.0 && p->cy_a < 1e3 && p->cy_lambda >= 0.0 && p->cy_lambda < 1e12 &&
        (p->cy_tau0 - p->cy_tau_inf) * (1.0 - p->cy_n) < p->cy_tau_inf)) {
    why = "Carreau-Yasuda needs 1/2 < tau_inf <= tau0, 0 < n <= 1, a > 0, lambda >= 0 and (tau0 - tau_inf)(1 - n) < tau_inf";
    return MF_EINVAL;
  }
  if (p->curvature != MF_CURV_PLAIN && p->curvature != MF_CURV_MLP) { why = "unknown curvature mode"; return MF_EINVAL; }
  if (p->flux_mode != MF_FLUX_LEDGER && p->flux_mode != MF_FLUX_PAPER) { why = "unknown gas-flux mode"; return MF_EINVAL; }
  if (p->curvature == MF_CURV_MLP && p->dim != 3) { why = "the learned curvature works on 5x5x5 stencils (3D only)"; return MF_EUNSUPPORTED; }
  if (p->curvature == MF_CURV_MLP && p->max_ids > 65534) { why = "the learned curvature supports at most 65534 bubble ids"; return MF_EINVAL; }
  if (p->max_ids < 2 || p->max_ids > (1 << 24)) { why = "max_ids out of range"; return MF_EINVAL; }
  if (!(p->tau > 0.5) || !(p->D > 0.0) || !(p->RT > 0.0) || !(p->eps >= 0.0)) { why = "tau > 1/2, D > 0, RT > 0, eps >= 0 required"; return MF_EINVAL; }
  if (p->k_pi > 0.0 && !(p->d_max >= 1.0)) { why = "d_max >= 1 required with disjoining pressure"; return MF_EINVAL; }
  for (int a = 0; a < 3; a++)
    if (!(fabs(p->accel[a]) <= 1e-2)) { why = "body-force acceleration components must be finite with |a| <= 1e-2"; return MF_EINVAL; }
  if (p->dim == 2 && p->accel[2] != 0.0) { why = "a plane (2D) domain takes no third acceleration component"; return MF_EINVAL; }
  if (p->rheology == MF_POWER_LAW && !(p->tau_min > 0.5 && p->tau_max >= p->tau_min && p->pl_nu_ref > 0 && p->pl_gdot_ref > 0)) {
    why = "power law needs 1/2 < tau_min <= tau_max, nu_ref > 0, gdot_ref > 0";
    return MF_EINVAL;
  }
  return MF_OK;
}

KP make_kp(const mf_params &P) {
  KP k;
  memset(&k, 0, sizeof k);
  k.dim = P.dim;
  k.nx = P.nx;
  k.ny = P.ny;
  k.nz = P.dim == 2 ? 1 : P.nz;
  for (int a = 0; a < 3; a++) k.per[a] = P.periodic[a] ? 1 : 0;
  if (P.dim == 2) k.per[2] = 0;
  k.N = (int64_t)k.nx * k.ny * k.nz;
  k.Np = (k.N + 255) & ~(int64_t)255;
  k.cap = P.max_ids;
  k.H = next_pow2(4 * P.max_ids < 1024 ? 1024 : 4 * P.max_ids);
  k.ecap = 2 * P.max_ids < 1024 ? 1024 : 2 * P.max_ids;
  k.RH = next_pow2(2 * k.ecap);
  k.rheology = P.rheology;
  k.cleanup = P.cleanup;
  k.curvature = P.curvature;
  const double kg = P.dim == 2 ? 3.0 : 4.0;
  k.omega = 1.0 / P.tau;
  k.omega_g = 1.0 / (0.5 + kg * P.D);
  k.sigma = P.sigma;
  k.kH = P.kH;
  k.RT = P.RT;
  k.k_pi = P.k_pi;
  k.d_max = P.d_max;
  k.p_atm = P.p_atm;
  k.q = P.q;
  k.eps = P.eps;
  k.c0 = (P.S0 * P.kH) * P.p_atm;
  k.pl_n = P.pl_n;
  k.pl_nu_ref = P.pl_nu_ref;
  k.pl_gdot_ref = P.pl_gdot_ref;
  k.tau_min = P.tau_min;
  k.tau_max = P.tau_max;
  double gs = k.c0 > 0.0 ? k.c0 : P.kH * P.p_atm;
  if (!(gs > 0.0)) gs = 1.0;
  k.gsc = (float)gs;
  k.ginv = (float)(1.0 / gs);
  k.cy_tau0 = P.cy_tau0;
  k.cy_tau_inf = P.cy_tau_inf;
  k.cy_lambda = P.cy_lambda;
  k.cy_a = P.cy_a;
  k.cy_n = P.cy_n;
  k.cy_lk = (float)(P.cy_lambda * 2.1213203435596424);
  k.cy_m = (float)((P.cy_n - 1.0) / (P.cy_a > 0.0 ? P.cy_a : 1.0));
  k.omega_f = (float)k.omega;
  k.omega_g_f = (float)k.omega_g;
  k.pl_n_f = (float)k.pl_n;
  k.tau_min_f = (float)k.tau_min;
  k.tau_max_f = (float)k.tau_max;
  k.c0_f = (float)k.c0;
  k.q_f = (float)k.q;
  k.c0g_f = k.c0_f * k.ginv;
  k.qg_f = k.q_f * k.ginv;
  k.cy_tau0_f = (float)k.cy_tau0;
  k.cy_tau_inf_f = (float)k.cy_tau_inf;
  k.cy_a_f = (float)k.cy_a;
  k.cy_w_f = (k.cy_tau0_f - k.cy_tau_inf_f) * (1.0f - (float)k.cy_n);
  k.pl_ninv = P.pl_n > 0.0 ? (float)(1.0 / P.pl_n) : 1.0f;
  // iterations for a relative error of tau below 3e-7, from the measured convergence of
  // the bounded start
  k.pl_nit = (P.pl_n >= 0.3 && P.pl_n <= 3.0) ? 3 : 5;
  k.ax = P.accel[0];
  k.ay = P.accel[1];
  k.az = P.dim == 3 ? P.accel[2] : 0.0;
  k.force = k.ax != 0.0 || k.ay != 0.0 || k.az != 0.0;
  k.flux_paper = P.flux_mode == MF_FLUX_PAPER ? 1 : 0;
  k.fax = (float)k.ax;
  k.fay = (float)k.ay;
  k.faz = (float)k.az;
  k.pl_l2nu3 = P.pl_nu_ref > 0.0 ? (float)log2(3.0 * P.pl_nu_ref) : 0.0f;
  k.pl_kg = P.pl_gdot_ref > 0.0 ? (float)(2.1213203435596424 / P.pl_gdot_ref) : 0.0f;
  return k;
}

#define HIPCHK(ctx, expr)                                                             \
  do {                                                                                \
    hipError_t _e = (expr);                                                           \
    if (_e != hipSuccess) {                                                           \
      (ctx)->err = std::string(#expr) + ": " + hipGetErrorString(_e);                 \
      return MF_EHIP;                                                                 \
    }                                                                                 \
  } while (0)

__device__ __forceinline__ void b_reset_counters(const GridPos &gp, DA d) {
  const int t = threadIdx.x;
  if (t < C_NCOUNT) d.cnt[t] = 0;
}
__global__ void k_reset_counters(DA d) {
  b_reset_counters(GridPos::hw(), d);
}

__global__ void km_reset_counters(MLaunch ml) {
  MF_MULTI(MK_ONE)
  b_reset_counters(gp, m.d);
}

}  // namespace

void mf::reset_multi(const MStep &ms, hipStream_t s) {
  hipLaunchKernelGGL(km_reset_counters, dim3(ms.grid[MK_ONE]), dim3(64), 0, s, ms.at(MK_ONE));
}

namespace {

__global__ void k_fill_bytes(uint8_t *p, size_t n, uint8_t v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

int device_status(Ctx *c) {
  int32_t st = 0;
  HIPCHK(c, hipMemcpyAsync(&st, c->d.status, 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (st == 0) return MF_OK;
  c->err = "device status:";
  if (st & ST_INVARIANT) c->err += " liquid cell next to gas / gas neighbour with another bubble id;";
  if (st & ST_TABLE) c->err += " bubble or labelling table capacity exceeded;";
  if (st & ST_NONFINITE) c->err += " non-positive or non-finite density;";
  if (st & ST_BADLABEL) c->err += " interface cell with an invalid bubble id;";
  return (st & ST_TABLE) ? MF_ECAPACITY : MF_ENUMERIC;
}

void reset_counters(Ctx *c) { hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, c->stream, c->d); }

// the counter set and interface list of the current step parity
void select_parity(Ctx *c) {
  c->d.cnt = c->cnt_base + C_NCOUNT * c->parity;
  c->d.ilist = c->ilist_base + (size_t)c->kp.Np * c->parity;
}

// per-step event pairs when profiling
constexpr int kStepEvents = 6;
struct Prof {
  std::vector<hipEvent_t> ev;  // per step: step start, sweep start, bulk sweep end,
                               // interface sweep start, interface sweep end, step end
  size_t used = 0;
};

}  // namespace

struct mf_ctx : Ctx {
  OpsTable ops;
  Prof prof_ev;
};

static void destroy_side(mf_ctx *c) {
  if (c->side) (void)hipStreamSynchronize(c->side);
  if (c->side2) (void)hipStreamSynchronize(c->side2);
  if (c->side2) (void)hipStreamDestroy(c->side2);
  if (c->ev_start) (void)hipEventDestroy(c->ev_start);
  if (c->ev_list) (void)hipEventDestroy(c->ev_list);
  if (c->ev_tail) (void)hipEventDestroy(c->ev_tail);
  c->side2 = nullptr;
  c->ev_start = c->ev_list = c->ev_tail = nullptr;
  if (c->ev_conv) (void)hipEventDestroy(c->ev_conv);
  if (c->ev_side) (void)hipEventDestroy(c->ev_side);
  if (c->ev_norm) (void)hipEventDestroy(c->ev_norm);
  if (c->side) (void)hipStreamDestroy(c->side);
  c->side = nullptr;
  c->ev_conv = c->ev_side = c->ev_norm = nullptr;
}

// the context stream waits for the labelling and geometry the last step left running on
// the side stream
static void join_side(mf_ctx *c) {
  if (c->list_pending) {
    (void)hipStreamWaitEvent(c->stream, c->ev_list, 0);
    c->list_pending = false;
  }
  if (!c->side_pending) return;
  (void)hipStreamWaitEvent(c->stream, c->ev_side, 0);
  c->side_pending = false;
}


extern "C" {

int mf_abi_version(void) { return MF_ABI_VERSION; }

const char *mf_last_error(const mf_ctx *ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

int mf_workspace_bytes(const mf_params *p, size_t *bytes) {
  std::string why;
  int rc = validate(p, why);
  if (rc) { g_err = why; return rc; }
  if (!bytes) { g_err = "bytes is NULL"; return MF_EINVAL; }
  KP kp = make_kp(*p);
  DA d;
  Carve cv(nullptr);
  layout(*p, kp, cv, d);
  *bytes = cv.off + 256;
  return MF_OK;
}

int mf_create(const mf_params *p, void *dev_workspace, size_t ws_bytes, void *stream, mf_ctx **out) {
  std::string why;
  if (!out) { g_err = "out is NULL"; return MF_EINVAL; }
  *out = nullptr;
  int rc = validate(p, why);
  if (rc) { g_err = why; return rc; }
  size_t need = 0;
  mf_workspace_bytes(p, &need);
  mf_ctx *c = new (std::nothrow) mf_ctx();
  if (!c) { g_err = "host allocation failed"; return MF_ENOMEM; }
  c->P = *p;
  c->kp = make_kp(*p);
  c->stream = (hipStream_t)stream;
  c->ops = ops_for(p->dim, p->precision);
  if (dev_workspace) {
    if (ws_bytes < need) {
      g_err = "workspace smaller than mf_workspace_bytes";
      delete c;
      return MF_ENOMEM;
    }
    c->ws = dev_workspace;
  } else {
    hipError_t e = hipMalloc(&c->ws, need);
    if (e != hipSuccess) {
      g_err = std::string("hipMalloc of the workspace failed: ") + hipGetErrorString(e);
      delete c;
      return MF_ENOMEM;
    }
    c->own_ws = true;
  }
  c->ws_bytes = need;
  char *base = (char *)(((uintptr_t)c->ws + 255) & ~(uintptr_t)255);
  Carve cv(base);
  layout(*p, c->kp, cv, c->d);
  c->cnt_base = c->d.cnt;
  c->ilist_base = c->d.ilist;
  {
    // default priority, not synchronising with the legacy default stream
    hipError_t e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_conv, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_side, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_norm, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_start, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_list, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_tail, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->side2, hipStreamNonBlocking);
    if (e != hipSuccess) {
      g_err = std::string("creating the side stream failed: ") + hipGetErrorString(e);
      destroy_side(c);
      if (c->own_ws) (void)hipFree(c->ws);
      delete c;
      return MF_EHIP;
    }
  }
  // zero everything, then the "empty" markers of the hash tables
  {
    size_t n = cv.off;
    unsigned nb = (unsigned)((n + 255) / 256 > 65536 ? 65536 : (n + 255) / 256);
    hipLaunchKernelGGL(k_fill_bytes, dim3(nb), dim3(256), 0, c->stream, (uint8_t *)base, n, (uint8_t)0);
    hipLaunchKernelGGL(k_fill_bytes, dim3(64), dim3(256), 0, c->stream, (uint8_t *)c->d.hkeys, (size_t)c->kp.H * 8, (uint8_t)0xFF);
    hipLaunchKernelGGL(k_fill_bytes, dim3(64), dim3(256), 0, c->stream, (uint8_t *)c->d.rh_key, (size_t)c->kp.RH * 4, (uint8_t)0xFF);
    hipLaunchKernelGGL(k_fill_bytes, dim3(64), dim3(256), 0, c->stream, (uint8_t *)c->d.rh_head, (size_t)c->kp.RH * 4, (uint8_t)0xFF);
  }
  c->ops.init_box(*c, c->stream);
  // atmosphere entry and the id counter
  {
    const double patm = p->p_atm;
    const int32_t one = 1;
    const int32_t next = 1;
    hipError_t e1 = hipMemcpyAsync(c->d.bp, &patm, 8, hipMemcpyHostToDevice, c->stream);
    hipError_t e2 = hipMemcpyAsync(c->d.balive, &one, 4, hipMemcpyHostToDevice, c->stream);
    hipError_t e3 = hipMemcpyAsync(c->d.nextid, &next, 4, hipMemcpyHostToDevice, c->stream);
    hipError_t e4 = hipStreamSynchronize(c->stream);
    hipError_t e5 = hipGetLastError();
    if (e1 || e2 || e3 || e4 || e5) {
      g_err = std::string("initialisation failed: ") + hipGetErrorString(e4 ? e4 : (e5 ? e5 : e1));
      destroy_side(c);
      if (c->own_ws) (void)hipFree(c->ws);
      delete c;
      return MF_EHIP;
    }
  }
  // the headspace-only state needs its lists and geometry too
  reset_counters(c);
  c->ops.build_lists(*c, c->stream);
  c->ops.geometry(*c, c->stream);
  *out = c;
  return MF_OK;
}

int mf_destroy(mf_ctx *c) {
  if (!c) return MF_OK;
  (void)hipStreamSynchronize(c->stream);
  destroy_side(c);
  for (hipEvent_t e : c->prof_ev.ev) (void)hipEventDestroy(e);
  if (c->mlp_buf) (void)hipFree(c->mlp_buf);
  if (c->own_ws) (void)hipFree(c->ws);
  delete c;
  return MF_OK;
}

int mf_nucleate(mf_ctx *c, int32_t n, const double *centers, const double *radii, const double *p0) {
  if (!c) return MF_EINVAL;
  c->epoch++;
  c->sword_dirty = true;
  if (c->nucleated || c->stepped) { c->err = "mf_nucleate is valid once, before mf_step"; return MF_ESTATE; }
  if (n < 0 || (n > 0 && (!centers || !radii || !p0))) { c->err = "bad nucleus arrays"; return MF_EINVAL; }
  if (n + 1 > c->kp.cap) { c->err = "more nuclei than the bubble table holds"; return MF_ECAPACITY; }
  const int D = c->kp.dim;
  for (int k = 0; k < n; k++) {
    const double cc[3] = {centers[3 * k], centers[3 * k + 1], D == 3 ? centers[3 * k + 2] : 0.0};
    const int dims[3] = {c->kp.nx, c->kp.ny, c->kp.nz};
    if (!(radii[k] > 0.0) || !(p0[k] > 0.0)) { c->err = "nucleus radius and pressure must be positive"; return MF_EINVAL; }
    for (int a = 0; a < D; a++)
      if (!(cc[a] - radii[k] >= 1.0) || !(cc[a] + radii[k] <= dims[a] - 2.0)) {
        c->err = "nucleus " + std::to_string(k) + " is not inside the closed domain";
        return MF_EINVAL;
      }
  }
  c->ops.nucleate(*c, c->stream, n, centers, radii);
  std::vector<int32_t> alive(n + 1, 1);
  double *p0d = nullptr;
  HIPCHK(c, hipMalloc(&p0d, sizeof(double) * (n > 0 ? n : 1)));
  HIPCHK(c, hipMemcpyAsync(c->d.balive, alive.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, c->stream));
  const int32_t next = n + 1;
  HIPCHK(c, hipMemcpyAsync(c->d.nextid, &next, 4, hipMemcpyHostToDevice, c->stream));
  if (n > 0) HIPCHK(c, hipMemcpyAsync(p0d, p0, sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
  reset_counters(c);
  c->ops.build_lists(*c, c->stream);
  c->ops.label(*c, c->stream, 0);
  launch_init_mass(*c, c->stream, p0d, n);
  c->ops.geometry(*c, c->stream);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  (void)hipFree(p0d);
  HIPCHK(c, hipGetLastError());
  c->nucleated = true;
  return device_status(c);
}

// one time step, enqueued on the context stream (host work: launches only); ev:
// kStepEvents profiling events or NULL.
// With overlap, a step runs on three streams of the context (see Ctx). The context stream
// takes the bulk sweep, the interface sweep and the first half of the conversions. After
// that, the side stream takes their second half, the labelling and the curvature, and
// side2 the normals and then the next step's counter reset and interface-list build. The
// next bulk sweep reads only cell types, populations and the wall mask, so it runs beside
// all of that. The interface sweep, the first kernel that reads ids, bubble pressures,
// curvature and the new list, waits for both side streams. The caller joins what the last
// step left running (join_side) before anything else touches the state. A step whose
// stencil words need the whole-grid pass takes the plain order.
static void step_once(mf_ctx *c, hipEvent_t *ev, bool overlap) {
  c->parity ^= 1;
  select_parity(c);
  if (ev) (void)hipEventRecord(ev[0], c->stream);
  const bool aside = overlap && !c->sword_dirty;
  if (aside) {
    (void)hipEventRecord(c->ev_start, c->stream);
    (void)hipStreamWaitEvent(c->side2, c->ev_start, 0);
    hipStream_t own = c->stream;
    c->stream = c->side2;
    reset_counters(c);
    c->ops.build_lists(*c, c->side2);
    c->stream = own;
    (void)hipEventRecord(c->ev_list, c->side2);
    c->list_pending = true;
  } else {
    reset_counters(c);
    c->ops.build_lists(*c, c->stream);
  }
  if (ev) (void)hipEventRecord(ev[1], c->stream);
  if (c->ops.sweep_bulk_auto(*c, c->stream)) {
    if (ev) (void)hipEventRecord(ev[2], c->stream);
    join_side(c);
    if (ev) (void)hipEventRecord(ev[3], c->stream);
    c->ops.sweep_interface(*c, c->stream);
    if (ev) (void)hipEventRecord(ev[4], c->stream);
  } else {
    join_side(c);
    c->ops.sweep_cells(*c, c->stream);
    if (ev) {
      (void)hipEventRecord(ev[2], c->stream);
      (void)hipEventRecord(ev[3], c->stream);
      (void)hipEventRecord(ev[4], c->stream);
    }
  }
  c->cur ^= 1;
  if (aside) {
    c->ops.convert_head(*c, c->stream);
    (void)hipEventRecord(c->ev_conv, c->stream);
    (void)hipStreamWaitEvent(c->side, c->ev_conv, 0);
    c->ops.convert_tail(*c, c->side);
    (void)hipEventRecord(c->ev_tail, c->side);
    (void)hipStreamWaitEvent(c->side2, c->ev_tail, 0);
    c->ops.label(*c, c->side, 1);
    c->ev_norm_rec = c->ev_norm;
    c->ops.geometry_normals(*c, c->side2, !c->sword_fresh);
    c->ev_norm_rec = nullptr;
    (void)hipStreamWaitEvent(c->side, c->ev_norm, 0);
    c->ops.geometry_curv(*c, c->side);
    if (ev) (void)hipEventRecord(ev[5], c->side);
    (void)hipEventRecord(c->ev_side, c->side);
    c->side_pending = true;
  } else {
    c->ops.convert(*c, c->stream);
    c->ops.label(*c, c->stream, 1);
    c->ops.geometry(*c, c->stream);
    if (ev) (void)hipEventRecord(ev[5], c->stream);
  }
  c->step++;
}

int mf_step(mf_ctx *c, int32_t nsteps) {
  if (!c) return MF_EINVAL;
  if (nsteps < 0) { c->err = "nsteps < 0"; return MF_EINVAL; }
  if (c->kp.curvature == MF_CURV_MLP && !c->d.mlp_w) { c->err = "learned curvature selected but no network attached"; return MF_ESTATE; }
  if (nsteps > 0 && c->gas_dirty) c->ops.geometry(*c, c->stream);  // idempotent
  for (int k = 0; k < nsteps; k++) {
    hipEvent_t *ev = nullptr;
    if (c->prof) {
      if (c->prof_ev.used + kStepEvents > c->prof_ev.ev.size()) {
        c->err = "profiling event pool exhausted; call mf_profile_get";
        join_side(c);
        return MF_ESTATE;
      }
      ev = &c->prof_ev.ev[c->prof_ev.used];
      c->prof_ev.used += kStepEvents;
    }
    step_once(c, ev, true);
  }
  join_side(c);
  c->stepped = c->stepped || nsteps > 0;
  HIPCHK(c, hipGetLastError());
  return MF_OK;
}

int mf_tune(mf_ctx *c, int32_t reps, int32_t *best, float *ms) {
  if (!c || !best || reps < 1) return MF_EINVAL;
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  float tv[kNumSweepVariants];
  for (int v = 0; v < kNumSweepVariants; ++v) {
    float t = -1.0f;
    // the bulk kernel writes only the other population buffer: timing it changes no state
    if (c->ops.sweep_bulk(*c, c->stream, v)) {
      (void)hipEventRecord(e0, c->stream);
      for (int r = 0; r < reps; ++r) c->ops.sweep_bulk(*c, c->stream, v);
      (void)hipEventRecord(e1, c->stream);
      hipError_t e = hipEventSynchronize(e1);
      if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
      if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        HIPCHK(c, e);
      }
      t /= (float)reps;
    }
    tv[v] = t;
    if (ms) ms[v] = t;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIPCHK(c, hipGetLastError());
  // The default shape stays unless another 256-thread shape is faster alone by more than
  // kTuneMargin. Launched alone, four and eight cells per thread come within 1% of each
  // other on 16-bit storage, and noise would pick either; inside a step, beside the
  // labelling and curvature kernels, four cells per thread (four waves per SIMD) delay
  // those kernels until the bulk sweep ends, and the step takes 4% (early foam) to 10% (the
  // grown foam) longer.
  constexpr float kTuneMargin = 0.05f;
  int bv = effective_sweep_variant(c->kp, c->P.precision, -1);
  if (bv >= 0 && (!step_variant(bv) || tv[bv] < 0.0f)) bv = -1;
  float bt = bv >= 0 ? tv[bv] * (1.0f - kTuneMargin) : 0.0f;
  for (int v = 0; v < kNumSweepVariants; ++v)
    if (v != bv && step_variant(v) && tv[v] >= 0.0f && (bv < 0 || tv[v] < bt)) {
      bv = v;
      bt = tv[v];
    }
  c->sweep_variant = bv;  // -1 when no variant applies (per-cell sweep)
  c->epoch++;
  *best = bv;
  return MF_OK;
}

int mf_set_sweep_variant(mf_ctx *c, int32_t v) {
  if (!c) return MF_EINVAL;
  if (v < -1 || v >= kNumSweepVariants) { c->err = "unknown sweep variant"; return MF_EINVAL; }
  c->sweep_variant = v;
  c->epoch++;
  return MF_OK;
}

int mf_sync(mf_ctx *c) {
  if (!c) return MF_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipGetLastError());
  return device_status(c);
}

static size_t field_bytes(const mf_ctx *c, int field) {
  const size_t N = (size_t)c->kp.N;
  const int Q = c->kp.dim == 2 ? 9 : 19, Qg = c->kp.dim == 2 ? 5 : 7;
  switch (field) {
    case MF_FIELD_TYPE: return N;
    case MF_FIELD_LABEL: return N * 4;
    case MF_FIELD_F: return N * 8 * Q;
    case MF_FIELD_G: return N * 8 * Qg;
    default: return field >= 0 && field <= MF_FIELD_G ? N * 8 : 0;
  }
}

int mf_read_field(mf_ctx *c, int32_t field, void *dst, size_t dst_bytes, int32_t dst_on_device) {
  if (!c || !dst) return MF_EINVAL;
  const size_t need = field_bytes(c, field);
  if (!need) { c->err = "unknown field"; return MF_EINVAL; }
  if (dst_bytes < need) { c->err = "destination too small"; return MF_EINVAL; }
  void *stage = nullptr;
  HIPCHK(c, hipMalloc(&stage, need));
  c->ops.read_field(*c, c->stream, field, (double *)stage);
  hipError_t e = hipMemcpyAsync(dst, stage, need, dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream);
  hipError_t e2 = hipStreamSynchronize(c->stream);
  (void)hipFree(stage);
  HIPCHK(c, e);
  HIPCHK(c, e2);
  HIPCHK(c, hipGetLastError());
  return MF_OK;
}

int mf_write_field(mf_ctx *c, int32_t field, const void *src, size_t src_bytes) {
  if (!c || !src) return MF_EINVAL;
  c->epoch++;
  c->sword_dirty = true;
  if (c->stepped) { c->err = "mf_write_field is valid before the first mf_step"; return MF_ESTATE; }
  const size_t need = field_bytes(c, field);
  if (!need || field == MF_FIELD_CONC) { c->err = "field cannot be written"; return MF_EINVAL; }
  if (src_bytes < need) { c->err = "source too small"; return MF_EINVAL; }
  if (field == MF_FIELD_TYPE) {
    // the outer layer of every closed axis is a wall layer (the sweep relies on it)
    const uint8_t *t = (const uint8_t *)src;
    const int nx = c->kp.nx, ny = c->kp.ny, nz = c->kp.nz;
    for (int z = 0; z < nz; z++)
      for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) {
          const bool face = (!c->kp.per[0] && (x == 0 || x == nx - 1)) || (!c->kp.per[1] && (y == 0 || y == ny - 1)) ||
                            (c->kp.dim == 3 && !c->kp.per[2] && (z == 0 || z == nz - 1));
          if (face && (t[(size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * z)] & 3) != MF_WALL) {
            c->err = "cells on the outer layer of a closed axis must be walls";
            return MF_EINVAL;
          }
        }
  }
  void *stage = nullptr;
  HIPCHK(c, hipMalloc(&stage, need));
  hipError_t e = hipMemcpyAsync(stage, src, need, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) c->ops.write_field(*c, c->stream, field, (const double *)stage);
  hipError_t e2 = hipStreamSynchronize(c->stream);
  (void)hipFree(stage);
  HIPCHK(c, e);
  HIPCHK(c, e2);
  HIPCHK(c, hipGetLastError());
  c->nucleated = true;
  return MF_OK;
}

int mf_set_bubble(mf_ctx *c, int32_t id, double gas_mass, double volume, double pressure, int32_t alive) {
  if (!c) return MF_EINVAL;
  if (id < 0 || id >= c->kp.cap) { c->err = "id out of range"; return MF_EINVAL; }
  const int32_t al = alive ? 1 : 0;
  HIPCHK(c, hipMemcpyAsync(c->d.bm + id, &gas_mass, 8, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d.bV + id, &volume, 8, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d.bp + id, &pressure, 8, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d.balive + id, &al, 4, hipMemcpyHostToDevice, c->stream));
  // the gas side of the interface cells follows the bubble pressures before the next step
  c->gas_dirty = true;
  c->epoch++;
  int32_t next = 0;
  HIPCHK(c, hipMemcpyAsync(&next, c->d.nextid, 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (id + 1 > next) {
    next = id + 1;
    HIPCHK(c, hipMemcpyAsync(c->d.nextid, &next, 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return MF_OK;
}

int mf_refresh(mf_ctx *c, int32_t relabel) {
  if (!c) return MF_EINVAL;
  c->epoch++;
  c->sword_dirty = true;
  reset_counters(c);
  c->ops.build_lists(*c, c->stream);
  recount_gas(*c, c->stream);
  if (relabel) c->ops.label(*c, c->stream, 0);
  c->ops.geometry(*c, c->stream);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipGetLastError());
  return device_status(c);
}

int mf_read_bubbles(mf_ctx *c, mf_bubble *dst, int32_t capacity, int32_t *n_out) {
  if (!c) return MF_EINVAL;
  if (capacity < 0 || (capacity > 0 && !dst)) { c->err = "dst is NULL"; return MF_EINVAL; }
  const int cap = c->kp.cap;
  std::vector<double> m(cap), V(cap), p(cap);
  std::vector<int32_t> al(cap);
  std::vector<long long> st;
  HIPCHK(c, hipMemcpyAsync(m.data(), c->d.bm, 8 * cap, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(V.data(), c->d.bV, 8 * cap, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(p.data(), c->d.bp, 8 * cap, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(al.data(), c->d.balive, 4 * cap, hipMemcpyDeviceToHost, c->stream));
  if (capacity > 0) {
    // cell counts and gas-volume centroids: one pass over the grid
    st.resize((size_t)cap * 13);
    c->ops.bubble_stats(*c, c->stream);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(st.data(), c->d.bstat, 8 * st.size(), hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  int k = 0;
  for (int i = 1; i < cap; i++) {
    if (!al[i]) continue;
    if (k < capacity) {
      const long long *b = &st[(size_t)i * 13];
      dst[k].id = i;
      dst[k].alive = 1;
      dst[k].volume = V[i];
      dst[k].gas_mass = m[i];
      dst[k].pressure = p[i];
      dst[k].n_cells = (int32_t)b[0];
      const double w = fx_to_double(fx3_join(b[1], b[2], b[3]));
      for (int a = 0; a < 3; a++)
        dst[k].centroid[a] = w > 0.0 ? fx_to_double(fx3_join(b[4 + 3 * a], b[5 + 3 * a], b[6 + 3 * a])) / w : 0.0;
      if (c->kp.dim == 2) dst[k].centroid[2] = 0.0;
    }
    k++;
  }
  if (n_out) *n_out = k;
  return MF_OK;
}

int mf_totals_get(mf_ctx *c, mf_totals *out) {
  if (!c || !out) return MF_EINVAL;
  __int128 led[3];
  int32_t cnt[C_NCOUNT], st = 0, next = 0;
  std::vector<int32_t> al(c->kp.cap);
  HIPCHK(c, hipMemcpyAsync(led, c->d.ledtot, sizeof led, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(cnt, c->d.cnt, sizeof cnt, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(&st, c->d.status, 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(&next, c->d.nextid, 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(al.data(), c->d.balive, 4 * c->kp.cap, hipMemcpyDeviceToHost, c->stream));
  std::vector<double> bm(c->kp.cap);
  HIPCHK(c, hipMemcpyAsync(bm.data(), c->d.bm, 8 * c->kp.cap, hipMemcpyDeviceToHost, c->stream));
  long long tacc[6];
  c->ops.totals(*c, c->stream);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(tacc, c->d.tacc, sizeof tacc, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  out->step = c->step;
  out->liquid_mass = fx_to_double(fx3_join(tacc[0], tacc[1], tacc[2]));
  out->dissolved_gas = fx_to_double(fx3_join(tacc[3], tacc[4], tacc[5]));
  double bg = 0.0;
  for (int i = 1; i < c->kp.cap; i++)
    if (al[i]) bg += bm[i];
  out->bubble_gas = bg;
  out->lost_liquid = (double)led[0] * 0x1p-64;
  out->atm_gas = (double)led[1] * 0x1p-64;
  out->collapsed_gas = (double)led[2] * 0x1p-64;
  out->next_id = next;
  int nb = 0;
  for (int i = 1; i < c->kp.cap; i++) nb += al[i] ? 1 : 0;
  out->n_bubbles = nb;
  out->n_interface = cnt[C_I];
  out->status = st;
  return MF_OK;
}

int mf_debug_poke(mf_ctx *c, int32_t field, int64_t cell, int32_t comp, double value) {
  if (!c) return MF_EINVAL;
  const int Q = c->kp.dim == 2 ? 9 : 19, Qg = c->kp.dim == 2 ? 5 : 7;
  if (cell < 0 || cell >= c->kp.N) { c->err = "cell out of range"; return MF_EINVAL; }
  int ncomp = 0;
  switch (field) {
    case MF_FIELD_F: ncomp = Q; break;
    case MF_FIELD_G: ncomp = Qg; break;
    case MF_FIELD_RHO: case MF_FIELD_ALPHA: case MF_FIELD_MASS: ncomp = 1; break;
    default: c->err = "mf_debug_poke writes F, G, RHO, ALPHA or MASS"; return MF_EINVAL;
  }
  if (comp < 0 || comp >= ncomp) { c->err = "component out of range"; return MF_EINVAL; }
  join_side(c);
  c->ops.poke(*c, c->stream, field, cell, comp, value);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipGetLastError());
  return MF_OK;
}

// ---------------------------------------------------------------- checkpoints
// File: a header (magic, ABI version, the creation parameters, the arena size and the
// host-side state of the step sequence), the whole device arena, and the attached
// network's weights when there are any. The arena holds only data (no addresses), so a
// context created with the same parameters continues from it bit for bit.
namespace {
struct CkptHeader {
  char magic[8];
  int32_t abi, has_mlp;
  uint64_t params_bytes, arena_bytes, mlp_bytes;
  mf_params params;
  int64_t step;
  int32_t cur, parity, nucleated, stepped, sword_dirty, sword_fresh, gas_dirty, sweep_variant;
};
const char kCkptMagic[8] = {'M', 'I', 'F', 'O', 'A', 'M', 'C', 'K'};
constexpr size_t kMlpWBytes = (2 * (128 * 64 + 64 * 64 + 64) + 255) & ~(size_t)255;
constexpr size_t kMlpBBytes = (4 * (2 * 64 + 1) + 255) & ~(size_t)255;
constexpr size_t kCkptChunk = (size_t)64 << 20;

// every field of two parameter sets (padding bytes are not compared)
bool params_equal(const mf_params &a, const mf_params &b) {
  bool eq = a.struct_size == b.struct_size && a.dim == b.dim && a.nx == b.nx && a.ny == b.ny && a.nz == b.nz &&
            a.gas_from == b.gas_from && a.precision == b.precision && a.rheology == b.rheology &&
            a.curvature == b.curvature && a.cleanup == b.cleanup && a.max_ids == b.max_ids &&
            a.flux_mode == b.flux_mode;
  for (int k = 0; k < 3; k++) eq = eq && a.periodic[k] == b.periodic[k];
  const double da[] = {a.tau, a.D, a.sigma, a.kH, a.RT, a.k_pi, a.d_max, a.p_atm, a.q, a.eps, a.S0, a.pl_n,
                       a.pl_nu_ref, a.pl_gdot_ref, a.tau_min, a.tau_max, a.accel[0], a.accel[1], a.accel[2],
                       a.cy_tau0, a.cy_tau_inf, a.cy_lambda, a.cy_a, a.cy_n};
  const double db[] = {b.tau, b.D, b.sigma, b.kH, b.RT, b.k_pi, b.d_max, b.p_atm, b.q, b.eps, b.S0, b.pl_n,
                       b.pl_nu_ref, b.pl_gdot_ref, b.tau_min, b.tau_max, b.accel[0], b.accel[1], b.accel[2],
                       b.cy_tau0, b.cy_tau_inf, b.cy_lambda, b.cy_a, b.cy_n};
  for (size_t k = 0; k < sizeof da / sizeof da[0]; k++) eq = eq && memcmp(&da[k], &db[k], 8) == 0;
  return eq;
}

size_t arena_bytes(const mf_ctx *c) {
  size_t need = 0;
  mf_workspace_bytes(&c->P, &need);
  return need - 256;
}
char *arena_base(const mf_ctx *c) { return (char *)(((uintptr_t)c->ws + 255) & ~(uintptr_t)255); }
}  // namespace

int mf_save(mf_ctx *c, const char *path) {
  if (!c || !path) return MF_EINVAL;
  join_side(c);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  CkptHeader h;
  memset(&h, 0, sizeof h);
  memcpy(h.magic, kCkptMagic, 8);
  h.abi = MF_ABI_VERSION;
  h.has_mlp = c->d.mlp_w ? 1 : 0;
  h.params_bytes = sizeof(mf_params);
  h.arena_bytes = arena_bytes(c);
  h.mlp_bytes = h.has_mlp ? kMlpWBytes + kMlpBBytes : 0;
  h.params = c->P;
  h.step = c->step;
  h.cur = c->cur;
  h.parity = c->parity;
  h.nucleated = c->nucleated;
  h.stepped = c->stepped;
  h.sword_dirty = c->sword_dirty;
  h.sword_fresh = c->sword_fresh;
  h.gas_dirty = c->gas_dirty;
  h.sweep_variant = c->sweep_variant;
  FILE *fp = fopen(path, "wb");
  if (!fp) { c->err = std::string("cannot open ") + path + " for writing"; return MF_EINVAL; }
  std::vector<char> buf(kCkptChunk);
  bool ok = fwrite(&h, sizeof h, 1, fp) == 1;
  const char *base = arena_base(c);
  for (size_t off = 0; ok && off < h.arena_bytes; off += kCkptChunk) {
    const size_t n = h.arena_bytes - off < kCkptChunk ? h.arena_bytes - off : kCkptChunk;
    if (hipMemcpy(buf.data(), base + off, n, hipMemcpyDeviceToHost) != hipSuccess) { ok = false; break; }
    ok = fwrite(buf.data(), 1, n, fp) == n;
  }
  if (ok && h.has_mlp) {
    if (hipMemcpy(buf.data(), c->mlp_buf, h.mlp_bytes, hipMemcpyDeviceToHost) != hipSuccess) ok = false;
    else ok = fwrite(buf.data(), 1, h.mlp_bytes, fp) == h.mlp_bytes;
  }
  if (fclose(fp) != 0) ok = false;
  if (!ok) { c->err = std::string("writing the checkpoint ") + path + " failed"; return MF_EHIP; }
  return MF_OK;
}

int mf_load(mf_ctx *c, const char *path) {
  if (!c || !path) return MF_EINVAL;
  join_side(c);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  FILE *fp = fopen(path, "rb");
  if (!fp) { c->err = std::string("cannot open ") + path; return MF_EINVAL; }
  CkptHeader h;
  if (fread(&h, sizeof h, 1, fp) != 1 || memcmp(h.magic, kCkptMagic, 8) != 0 || h.abi != MF_ABI_VERSION ||
      h.params_bytes != sizeof(mf_params)) {
    fclose(fp);
    c->err = "not a checkpoint of this library version";
    return MF_EINVAL;
  }
  if (!params_equal(h.params, c->P) || h.arena_bytes != arena_bytes(c)) {
    fclose(fp);
    c->err = "the checkpoint was written by a context with other parameters";
    return MF_EINVAL;
  }
  if (h.has_mlp && (c->kp.curvature != MF_CURV_MLP || h.mlp_bytes != kMlpWBytes + kMlpBBytes)) {
    fclose(fp);
    c->err = "the checkpoint holds a network the context cannot take";
    return MF_EINVAL;
  }
  if (h.has_mlp && !c->mlp_buf) {
    if (hipMalloc(&c->mlp_buf, kMlpWBytes + kMlpBBytes) != hipSuccess) {
      fclose(fp);
      c->err = "allocating the network weights failed";
      return MF_ENOMEM;
    }
  }
  std::vector<char> buf(kCkptChunk);
  bool ok = true;
  char *base = arena_base(c);
  for (size_t off = 0; ok && off < h.arena_bytes; off += kCkptChunk) {
    const size_t n = h.arena_bytes - off < kCkptChunk ? h.arena_bytes - off : kCkptChunk;
    ok = fread(buf.data(), 1, n, fp) == n && hipMemcpy(base + off, buf.data(), n, hipMemcpyHostToDevice) == hipSuccess;
  }
  if (ok && h.has_mlp)
    ok = fread(buf.data(), 1, h.mlp_bytes, fp) == h.mlp_bytes &&
         hipMemcpy(c->mlp_buf, buf.data(), h.mlp_bytes, hipMemcpyHostToDevice) == hipSuccess;
  fclose(fp);
  if (!ok) { c->err = std::string("reading the checkpoint ") + path + " failed (the state is undefined)"; return MF_EHIP; }
  if (h.has_mlp) {
    c->d.mlp_w = (const uint16_t *)c->mlp_buf;
    c->d.mlp_b = (const float *)((char *)c->mlp_buf + kMlpWBytes);
  }
  c->step = h.step;
  c->cur = h.cur;
  c->parity = h.parity;
  select_parity(c);
  c->nucleated = h.nucleated != 0;
  c->stepped = h.stepped != 0;
  c->sword_dirty = h.sword_dirty != 0;
  c->sword_fresh = h.sword_fresh != 0;
  c->gas_dirty = h.gas_dirty != 0;
  c->sweep_variant = h.sweep_variant;
  c->epoch++;
  return MF_OK;
}

int mf_attach_mlp(mf_ctx *c, const mf_mlp *m) {
  if (!c || !m) return MF_EINVAL;
  c->epoch++;
  if (c->kp.curvature != MF_CURV_MLP) { c->err = "the context was created for the plain curvature"; return MF_ESTATE; }
  // weights (bfloat16) and biases (binary32), 256-byte aligned
  const size_t wbytes = kMlpWBytes, bbytes = kMlpBBytes;
  if (!c->mlp_buf) HIPCHK(c, hipMalloc(&c->mlp_buf, wbytes + bbytes));
  uint16_t *w = (uint16_t *)c->mlp_buf;
  float *b = (float *)((char *)c->mlp_buf + wbytes);
  const int rc = mf_mlp_export_weights(m, w, b, c->stream);
  if (rc) { c->err = "copying the network weights failed"; return rc; }
  c->d.mlp_w = w;
  c->d.mlp_b = b;
  return MF_OK;
}

int mf_profile_enable(mf_ctx *c, int32_t on) {
  if (!c) return MF_EINVAL;
  c->prof = on != 0;
  if (c->prof && c->prof_ev.ev.empty()) {
    c->prof_ev.ev.resize(kStepEvents * 4096);
    for (auto &e : c->prof_ev.ev) HIPCHK(c, hipEventCreate(&e));
  }
  c->prof_ev.used = 0;
  return MF_OK;
}

int mf_profile_get(mf_ctx *c, int32_t group, double *ms_total, int64_t *launches) {
  if (!c || !ms_total || !launches) return MF_EINVAL;
  if (group < 0 || group > 2) { c->err = "group must be 0 (bulk sweep), 1 (step) or 2 (interface sweep)"; return MF_EINVAL; }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double tot = 0.0;
  int64_t nl = 0;
  static const int from[3] = {1, 0, 3}, to[3] = {2, 5, 4};
  for (size_t k = 0; k + kStepEvents <= c->prof_ev.used; k += kStepEvents) {
    float ms = 0.0f;
    hipEvent_t a = c->prof_ev.ev[k + from[group]];
    hipEvent_t b = c->prof_ev.ev[k + to[group]];
    HIPCHK(c, hipEventElapsedTime(&ms, a, b));
    tot += ms;
    nl++;
  }
  *ms_total = tot;
  *launches = nl;
  return MF_OK;
}


// ---------------------------------------------------------------- batched domains
// The domains of a batch are grouped by what selects their kernels (dimension, storage,
// per-cell or bulk sweep, body force, learned curvature). Every kernel of a step runs as
// one launch for all domains of a group: each domain takes the work-groups it would take
// alone, and each work-group finds its domain from a table of per-domain parameters and
// arrays (MDom) and a prefix sum of work-group counts per launch kind. A group swept by the
// bulk kernel runs its steps on two streams, overlapped as a single domain's step; the
// results are those of mf_step on each context, bit for bit.
struct BatchGroup {
  std::vector<int> idx;  // domains of the batch in this group
  OpsTable ops;
  int precision = 0;
  bool cells = false, frc = false, mlp = false;
  unsigned vmask = 0;        // bulk launch shapes used by the group's domains
  int grid[MK_COUNT] = {};   // work-groups of each launch kind over the group
  std::vector<int> pre;      // [MK_COUNT][nd + 1] work-group prefix sums
  MDom *dom_dev[2] = {nullptr, nullptr};  // tables of the two buffer parities
  hipStream_t stream = nullptr;
  hipEvent_t ev_join = nullptr;
  // the second stream of a group swept by the bulk kernel, and the events that order the two
  hipStream_t side = nullptr;
  hipEvent_t ev_conv = nullptr, ev_side = nullptr;
};

struct mf_batch {
  std::vector<mf_ctx *> ctx;
  hipStream_t sb = nullptr;  // the batch stream: the groups fork from and join into it
  hipEvent_t ev_fork = nullptr, ev_out = nullptr;
  std::vector<hipEvent_t> ev_in;
  std::vector<BatchGroup> groups;
  bool ready = false;           // groups and tables built
  std::vector<uint64_t> epoch;  // context epochs and buffer parities when the tables were built
  std::vector<int> cur, par;
};

static void batch_drop_tables(mf_batch *b) {
  b->ready = false;
  for (BatchGroup &g : b->groups) {
    for (int j = 0; j < 2; ++j) {
      if (g.dom_dev[j]) (void)hipFree(g.dom_dev[j]);
      g.dom_dev[j] = nullptr;
    }
  }
}

static void batch_free_groups(mf_batch *b) {
  for (BatchGroup &g : b->groups) {
    if (g.stream) (void)hipStreamDestroy(g.stream);
    if (g.ev_join) (void)hipEventDestroy(g.ev_join);
    if (g.side) (void)hipStreamDestroy(g.side);
    if (g.ev_conv) (void)hipEventDestroy(g.ev_conv);
    if (g.ev_side) (void)hipEventDestroy(g.ev_side);
  }
  b->groups.clear();
}

static int batch_fail(const char *msg, hipError_t e) {
  g_thread_err = std::string(msg) + (e != hipSuccess ? std::string(": ") + hipGetErrorString(e) : std::string());
  return e != hipSuccess ? MF_EHIP : MF_ESTATE;
}

#define HIPCHK_B(expr)                                                          \
  do {                                                                          \
    const hipError_t _e = (expr);                                               \
    if (_e != hipSuccess) return batch_fail(#expr, _e);                         \
  } while (0)

// Work-groups a domain takes in a batched launch of kind k. The passes over the whole grid
// (list builder, sweep) take the grid of the domain's own launchers; the passes over its
// lists take a grid sized to the domain (their grid-stride loops cover whatever does not
// fit, and no result depends on the number of work-groups), so that a batch of small
// domains does not start thousands of work-groups that find nothing to do.
static int kind_blocks(const mf_ctx *c, int kind, int variant) {
  const int64_t N = c->kp.N;
  auto clampi = [](int64_t v, int64_t lo, int64_t hi) { return (int)(v < lo ? lo : (v > hi ? hi : v)); };
  const int nb = (int)list_blocks(*c);
  const int nch = list_blocks_of(c->kp);
  switch (kind) {
    case MK_ONE: return 1;
    case MK_LISTGRID: return nch < 1024 ? nch : 1024;
    case MK_LIST: return clampi(N / 8192, 1, nb);
    case MK_SHORT: return clampi(N / 65536, 1, 1024);
    case MK_TOPOW: return clampi(N / 65536, 1, 256);
    case MK_BFAST: return (c->kp.cap + 255) / 256 < 64 ? (c->kp.cap + 255) / 256 : 64;
    // each work-group of the learned curvature stages the network's weights in LDS once: about
    // as many cells per work-group as the single-domain launch gives the 384^3 foam
    case MK_MLP: return clampi(N / 65536, 1, 768);
    case MK_CELLS:
      return variant < 0 ? (int)((int64_t)((c->kp.nx + 63) / 64) * ((c->kp.ny + 3) / 4) * c->kp.nz) : 0;
    default: {
      const int v = kind - MK_BULK0;
      if (v != variant) return 0;
      const int64_t per = (int64_t)kSweepVariants[v].bs * kSweepVariants[v].vw;
      return (int)((N + per - 1) / per);
    }
  }
}

// sort the domains into groups by the kernels they use
static hipError_t batch_group(mf_batch *b) {
  batch_free_groups(b);
  for (size_t i = 0; i < b->ctx.size(); ++i) {
    const mf_ctx *c = b->ctx[i];
    const int v = effective_sweep_variant(c->kp, c->P.precision, c->sweep_variant);
    const bool cells = v < 0, frc = c->kp.force != 0, mlp = c->kp.curvature == MF_CURV_MLP;
    BatchGroup *g = nullptr;
    for (BatchGroup &h : b->groups) {
      const mf_ctx *o = b->ctx[h.idx[0]];
      if (o->kp.dim == c->kp.dim && h.precision == c->P.precision && h.cells == cells && h.frc == frc && h.mlp == mlp &&
          (int)h.idx.size() < kMaxBatchDomains) {
        g = &h;
        break;
      }
    }
    if (!g) {
      b->groups.emplace_back();
      g = &b->groups.back();
      g->ops = c->ops;
      g->precision = c->P.precision;
      g->cells = cells;
      g->frc = frc;
      g->mlp = mlp;
      hipError_t e = hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&g->ev_join, hipEventDisableTiming);
      if (e == hipSuccess) e = hipStreamCreateWithFlags(&g->side, hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&g->ev_conv, hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&g->ev_side, hipEventDisableTiming);
      if (e != hipSuccess) return e;
    }
    g->idx.push_back((int)i);
    if (!cells) g->vmask |= 1u << v;
  }
  return hipSuccess;
}

// the per-domain tables of each group for a step from the contexts' current buffer
// parities (table 0) and for the step after it (table 1)
static hipError_t batch_tables(mf_batch *b) {
  for (BatchGroup &g : b->groups) {
    const int nd = (int)g.idx.size();
    std::vector<int> &pre = g.pre;
    pre.assign((size_t)MK_COUNT * (nd + 1), 0);
    for (int k = 0; k < MK_COUNT; ++k) {
      for (int i = 0; i < nd; ++i) {
        const mf_ctx *c = b->ctx[g.idx[i]];
        const int v = effective_sweep_variant(c->kp, c->P.precision, c->sweep_variant);
        pre[(size_t)k * (nd + 1) + i + 1] = pre[(size_t)k * (nd + 1) + i] + kind_blocks(c, k, v);
      }
      g.grid[k] = pre[(size_t)k * (nd + 1) + nd];
    }
    hipError_t e = hipSuccess;
    for (int j = 0; j < 2; ++j) {
      std::vector<MDom> t(nd);
      for (int i = 0; i < nd; ++i) {
        const mf_ctx *c = b->ctx[g.idx[i]];
        const int parity = c->parity ^ (j == 0 ? 1 : 0);  // step_once flips it first
        t[i].kp = c->kp;
        t[i].d = c->d;
        t[i].d.cnt = c->cnt_base + C_NCOUNT * parity;
        t[i].d.ilist = c->ilist_base + (size_t)c->kp.Np * parity;
        t[i].cur = c->cur ^ j;
      }
      e = hipMalloc(&g.dom_dev[j], sizeof(MDom) * nd);
      if (e == hipSuccess) e = hipMemcpy(g.dom_dev[j], t.data(), sizeof(MDom) * nd, hipMemcpyHostToDevice);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

static MStep group_mstep(const BatchGroup &g, int j) {
  MStep ms;
  ms.dom = g.dom_dev[j];
  ms.nd = (int)g.idx.size();
  ms.pre = g.pre.data();
  ms.grid = g.grid;
  return ms;
}

// one time step of every domain of a group, as batched launches on stream s, in order
static void group_step(const BatchGroup &g, int j, hipStream_t s) {
  const MStep ms = group_mstep(g, j);
  reset_multi(ms, s);
  lists_multi(ms, 0, s);
  g.ops.sweep_multi(ms, g.vmask, g.cells, g.frc, 0, s);
  g.ops.convert_multi(ms, 0, s);
  g.ops.label_multi(ms, s);
  g.ops.geometry_multi(ms, g.mlp, s);
}

// n time steps of a group swept by the bulk kernel, the first with table `phase`, on two
// streams as in a single domain's step: the group stream takes the bulk sweep, the
// interface sweep and the first half of the conversions; the side stream then takes their
// second half, the labelling, the geometry and the next step's counter reset and
// interface list, beside the next bulk sweep (which reads only types, populations and
// wall masks); the next interface sweep waits for the side stream.
static void group_steps_overlapped(const BatchGroup &g, int phase, int n) {
  hipStream_t m = g.stream, sd = g.side;
  {
    const MStep ms0 = group_mstep(g, phase);
    reset_multi(ms0, m);
    lists_multi(ms0, 0, m);
  }
  for (int t = 0; t < n; ++t) {
    const MStep ms = group_mstep(g, (phase + t) & 1);
    g.ops.sweep_multi(ms, g.vmask, false, g.frc, 1, m);
    if (t > 0) (void)hipStreamWaitEvent(m, g.ev_side, 0);
    g.ops.sweep_multi(ms, g.vmask, false, g.frc, 2, m);
    g.ops.convert_multi(ms, 1, m);
    (void)hipEventRecord(g.ev_conv, m);
    (void)hipStreamWaitEvent(sd, g.ev_conv, 0);
    g.ops.convert_multi(ms, 2, sd);
    g.ops.label_multi(ms, sd);
    g.ops.geometry_multi(ms, g.mlp, sd);
    if (t + 1 < n) {
      const MStep mn = group_mstep(g, (phase + t + 1) & 1);
      reset_multi(mn, sd);
      lists_multi(mn, 0, sd);
    }
    (void)hipEventRecord(g.ev_side, sd);
  }
  (void)hipStreamWaitEvent(m, g.ev_side, 0);
}

int mf_batch_create(int32_t n, mf_ctx *const *ctxs, mf_batch **out) {
  if (n < 1 || !ctxs || !out) return MF_EINVAL;
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i]) return MF_EINVAL;
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) { g_thread_err = "a context appears twice in the batch"; return MF_EINVAL; }
  }
  mf_batch *b = new mf_batch;
  b->ctx.assign(ctxs, ctxs + n);
  hipError_t e = hipStreamCreateWithFlags(&b->sb, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming);
  b->ev_in.assign(n, nullptr);
  for (int i = 0; i < n && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&b->ev_in[i], hipEventDisableTiming);
  if (e != hipSuccess) {
    mf_batch_destroy(b);
    return batch_fail("creating the batch streams failed", e);
  }
  *out = b;
  return MF_OK;
}

int mf_batch_destroy(mf_batch *b) {
  if (!b) return MF_EINVAL;
  if (b->sb) (void)hipStreamSynchronize(b->sb);
  batch_drop_tables(b);
  batch_free_groups(b);
  for (hipEvent_t e : b->ev_in)
    if (e) (void)hipEventDestroy(e);
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  if (b->sb) (void)hipStreamDestroy(b->sb);
  delete b;
  return MF_OK;
}

// the groups and their tables for the contexts' current state
static hipError_t batch_prepare(mf_batch *b) {
  hipError_t e = batch_group(b);
  if (e == hipSuccess) e = batch_tables(b);
  if (e != hipSuccess) return e;
  b->epoch.resize(b->ctx.size());
  b->cur.resize(b->ctx.size());
  b->par.resize(b->ctx.size());
  for (size_t i = 0; i < b->ctx.size(); ++i) {
    b->epoch[i] = b->ctx[i]->epoch;
    b->cur[i] = b->ctx[i]->cur;
    b->par[i] = b->ctx[i]->parity;
  }
  b->ready = true;
  return hipSuccess;
}

int mf_batch_step(mf_batch *b, int32_t nsteps) {
  if (!b || nsteps < 0) return MF_EINVAL;
  for (mf_ctx *c : b->ctx) {
    if (c->kp.curvature == MF_CURV_MLP && !c->d.mlp_w) return batch_fail("a domain uses the learned curvature without a network", hipSuccess);
    if (c->prof) return batch_fail("profiling is not available in batched steps", hipSuccess);
  }
  if (nsteps == 0) return MF_OK;
  // Tables built before a state change made outside the time step are rebuilt. Every
  // step flips a context's population buffer and counter parity, so the table of the
  // next step is the one whose buffer matches; all contexts must agree on it.
  bool stale = !b->ready;
  int phase = -1;
  for (size_t i = 0; i < b->ctx.size() && !stale; ++i) {
    const mf_ctx *c = b->ctx[i];
    const int ph = c->cur ^ b->cur[i];
    stale = b->epoch[i] != c->epoch || (c->parity ^ b->par[i]) != ph || (phase >= 0 && ph != phase);
    phase = ph;
  }
  // the batch waits for the work already queued on the domains' own streams
  for (size_t i = 0; i < b->ctx.size(); ++i) {
    join_side(b->ctx[i]);
    (void)hipEventRecord(b->ev_in[i], b->ctx[i]->stream);
    (void)hipStreamWaitEvent(b->sb, b->ev_in[i], 0);
  }
  if (stale) {
    // tables in use stay allocated until the batch stream is idle
    HIPCHK_B(hipStreamSynchronize(b->sb));
    batch_drop_tables(b);
    HIPCHK_B(batch_prepare(b));
    phase = 0;
  }
  for (mf_ctx *c : b->ctx)
    if (c->sword_dirty || c->gas_dirty) c->ops.geometry(*c, b->sb);  // idempotent
  (void)hipEventRecord(b->ev_fork, b->sb);
  for (BatchGroup &g : b->groups) {
    (void)hipStreamWaitEvent(g.stream, b->ev_fork, 0);
    if (g.cells) {
      for (int t = 0; t < nsteps; ++t) group_step(g, (phase + t) & 1, g.stream);
    } else {
      (void)hipStreamWaitEvent(g.side, b->ev_fork, 0);
      group_steps_overlapped(g, phase, nsteps);
    }
    (void)hipEventRecord(g.ev_join, g.stream);
    (void)hipStreamWaitEvent(b->sb, g.ev_join, 0);
  }
  for (mf_ctx *c : b->ctx) {
    c->step += nsteps;
    c->cur ^= nsteps & 1;
    c->parity ^= nsteps & 1;
    select_parity(c);
    c->gas_dirty = false;
    c->sword_fresh = false;
    c->stepped = true;
  }
  // the domains' own streams wait for the batch
  (void)hipEventRecord(b->ev_out, b->sb);
  for (mf_ctx *c : b->ctx) (void)hipStreamWaitEvent(c->stream, b->ev_out, 0);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return batch_fail("a batched launch failed", e);
  return MF_OK;
}

int mf_batch_tune(mf_batch *b, int32_t reps, int32_t *variants) {
  if (!b || reps < 1) return MF_EINVAL;
  // Per group and per domain shape (size class): time the batched bulk launch over the
  // class's domains in every launch shape that fits them, keep the fastest. The bulk
  // kernel writes only the spare population buffer, so timing changes no state.
  HIPCHK_B(hipStreamSynchronize(b->sb));
  for (mf_ctx *c : b->ctx) {
    join_side(c);
    HIPCHK_B(hipStreamSynchronize(c->stream));
  }
  batch_drop_tables(b);
  HIPCHK_B(batch_group(b));
  HIPCHK_B(batch_tables(b));
  hipEvent_t e0, e1;
  HIPCHK_B(hipEventCreate(&e0));
  HIPCHK_B(hipEventCreate(&e1));
  int rc = MF_OK;
  for (BatchGroup &g : b->groups) {
    if (g.cells) continue;
    const int nd = (int)g.idx.size();
    std::vector<int> done(nd, 0);
    for (int i = 0; i < nd && rc == MF_OK; ++i) {
      if (done[i]) continue;
      const mf_ctx *ci = b->ctx[g.idx[i]];
      std::vector<int> cls;
      for (int k = i; k < nd; ++k) {
        const mf_ctx *ck = b->ctx[g.idx[k]];
        if (!done[k] && ck->kp.nx == ci->kp.nx && ck->kp.ny == ci->kp.ny && ck->kp.nz == ci->kp.nz) {
          cls.push_back(k);
          done[k] = 1;
        }
      }
      float tv[kNumSweepVariants];
      for (int v = 0; v < kNumSweepVariants; ++v) tv[v] = -1.0f;
      for (int v = 0; v < kNumSweepVariants && rc == MF_OK; ++v) {
        if (!step_variant(v) || !bulk_shape_ok(ci->kp, ci->P.precision, kSweepVariants[v].vw)) continue;
        // the class's domains only, in shape v
        std::vector<int> pre((size_t)MK_COUNT * (nd + 1), 0);
        const int kind = MK_BULK0 + v;
        for (int k = 0; k < nd; ++k) {
          const bool in = std::find(cls.begin(), cls.end(), k) != cls.end();
          pre[(size_t)kind * (nd + 1) + k + 1] =
              pre[(size_t)kind * (nd + 1) + k] + (in ? kind_blocks(b->ctx[g.idx[k]], kind, v) : 0);
        }
        int grid[MK_COUNT] = {};
        grid[kind] = pre[(size_t)kind * (nd + 1) + nd];
        MStep ms;
        ms.dom = g.dom_dev[0];
        ms.nd = nd;
        ms.pre = pre.data();
        ms.grid = grid;
        g.ops.bulk_multi(ms, v, g.frc, b->sb);  // warm-up launch
        (void)hipEventRecord(e0, b->sb);
        for (int r = 0; r < reps; ++r) g.ops.bulk_multi(ms, v, g.frc, b->sb);
        (void)hipEventRecord(e1, b->sb);
        float ms_t = 0.0f;
        hipError_t e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms_t, e0, e1);
        if (e != hipSuccess) {
          rc = batch_fail("timing the batched bulk sweep failed", e);
          break;
        }
        tv[v] = ms_t;
      }
      // as for a single context: the default shape unless another 256-thread shape is more
      // than 5% faster alone (inside an overlapped step the shapes that tie alone do not)
      int best = effective_sweep_variant(ci->kp, ci->P.precision, -1);
      if (best >= 0 && tv[best] < 0.0f) best = -1;
      float bt = best >= 0 ? tv[best] * 0.95f : 0.0f;
      for (int v = 0; v < kNumSweepVariants; ++v)
        if (v != best && tv[v] >= 0.0f && (best < 0 || tv[v] < bt)) {
          best = v;
          bt = tv[v];
        }
      for (int k : cls) {
        mf_ctx *c = b->ctx[g.idx[k]];
        c->sweep_variant = best;
        c->epoch++;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  batch_drop_tables(b);  // the tables are built again with the chosen shapes
  if (rc) return rc;
  for (size_t i = 0; i < b->ctx.size(); ++i)
    if (variants) variants[i] = b->ctx[i]->sweep_variant;
  return MF_OK;
}

}  // extern "C"

// Nucleation sites from a nucleation probability field by Poisson-disk sampling (Sec. 3.4).
// Host code: the sites are set-up data for mf_nucleate. The liquid region is first filled by
// the active-list method (sites are sphere centres with radii uniform in [r_min, r_max];
// two sites keep |x_i - x_j| >= r_i + r_j + gap, so spheres never overlap and at least gap
// cells of liquid separate them; each sphere stays one cell clear of the wall layers and of
// the headspace; distances wrap on periodic axes), then the field thins the filled set: in
// placement order a site is kept with the probability of its nearest cell, up to max_n sites.
// Random numbers: one SplitMix64 stream from the seed (Steele, Lea and Flood 2014),
// u = (z >> 11) 2^-53; directions by rejection from the cube [-1, 1]^d. Every arithmetic
// step is a single IEEE binary64 operation (no contraction), so the sites are reproducible
// bit for bit. The distance test looks only at the sites in the neighbouring buckets of a
// uniform grid of bucket edge >= 2 r_max + gap, the largest distance at which two sites
// interact.
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <vector>

#include "mf_internal.h"

namespace {

struct Rng {
  uint64_t s;
  uint64_t next() {
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double u() { return (double)(next() >> 11) * 0x1p-53; }
};

struct Sampler {
  int dim;
  int ext[3];
  bool per[3];
  int gas_from;
  const float *prob;
  double r_min, r_max, gap;
  // bucket grid
  int nb[3];
  double bw[3];
  std::vector<std::vector<int32_t>> bucket;
  std::vector<double> sx, sy, sz, sr;

  bool inside(const double *x, double r) const {
    for (int a = 0; a < dim; ++a) {
      if (per[a]) continue;
      const double lo = 1.0 + r + 1.0;
      double hi = (double)(ext[a] - 2) - r - 1.0;
      if (a == dim - 1 && gas_from >= 0) {
        const double h2 = (double)(gas_from - 1) - r - 1.0;
        hi = h2 < hi ? h2 : hi;
      }
      if (x[a] < lo || x[a] > hi) return false;
    }
    return true;
  }
  double dist2(const double *x, int j) const {
    const double y[3] = {sx[j], sy[j], sz[j]};
    double s = 0.0;
    for (int a = 0; a < dim; ++a) {
      double d = x[a] - y[a];
      if (per[a]) {
        const double L = (double)ext[a];
        d = d - L * floor(d / L + 0.5);
      }
      s = s + d * d;
    }
    return s;
  }
  int bucket_of(const double *x, int a) const {
    int b = (int)floor(x[a] / bw[a]);
    return b < 0 ? 0 : (b >= nb[a] ? nb[a] - 1 : b);
  }
  size_t bucket_index(const int *b) const { return (size_t)b[0] + (size_t)nb[0] * ((size_t)b[1] + (size_t)nb[1] * b[2]); }
  bool far(const double *x, double r) const {
    int b0[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) b0[a] = bucket_of(x, a);
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) {
      lo[a] = b0[a] - 1;
      hi[a] = b0[a] + 1;
      if (!per[a] || nb[a] < 3) {
        // without wrap (or when the neighbours would repeat) the clamped range covers all
        if (!per[a]) {
          lo[a] = lo[a] < 0 ? 0 : lo[a];
          hi[a] = hi[a] >= nb[a] ? nb[a] - 1 : hi[a];
        } else {
          lo[a] = 0;
          hi[a] = nb[a] - 1;
        }
      }
    }
    int b[3];
    for (int k2 = lo[2]; k2 <= hi[2]; ++k2)
      for (int k1 = lo[1]; k1 <= hi[1]; ++k1)
        for (int k0 = lo[0]; k0 <= hi[0]; ++k0) {
          const int kk[3] = {k0, k1, k2};
          for (int a = 0; a < 3; ++a) b[a] = per[a] && nb[a] >= 3 ? (kk[a] % nb[a] + nb[a]) % nb[a] : kk[a];
          for (int32_t j : bucket[bucket_index(b)]) {
            const double m = r + sr[j] + gap;
            if (dist2(x, j) < m * m) return false;
          }
        }
    return true;
  }
  double pval(const double *x) const {
    if (!prob) return 1.0;
    int c[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) {
      int v = (int)floor(x[a] + 0.5);
      if (per[a]) v = ((v % ext[a]) + ext[a]) % ext[a];
      else v = v < 0 ? 0 : (v > ext[a] - 1 ? ext[a] - 1 : v);
      c[a] = v;
    }
    const size_t idx = (size_t)c[0] + (size_t)ext[0] * ((size_t)c[1] + (dim == 3 ? (size_t)ext[1] * c[2] : 0));
    return (double)prob[idx];
  }
  void add(const double *x, double r) {
    const int32_t j = (int32_t)sr.size();
    sx.push_back(x[0]);
    sy.push_back(dim > 1 ? x[1] : 0.0);
    sz.push_back(dim > 2 ? x[2] : 0.0);
    sr.push_back(r);
    int b[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) b[a] = bucket_of(x, a);
    bucket[bucket_index(b)].push_back(j);
  }
};

}  // namespace

extern "C" int mf_poisson_nuclei(const mf_params *p, const float *prob, int32_t max_n, double r_min, double r_max,
                                 double gap, int32_t attempts, uint64_t seed, double *centers, double *radii,
                                 int32_t *n_out) {
  if (!p || !n_out || p->struct_size != sizeof(mf_params) || (p->dim != 2 && p->dim != 3)) return MF_EINVAL;
  *n_out = 0;
  if (max_n < 0 || attempts < 1 || !(r_min > 0.0) || !(r_max >= r_min) || !(gap >= 0.0) || !(r_max < 1e6) || !(gap < 1e6))
    return MF_EINVAL;
  if (max_n > 0 && (!centers || !radii)) return MF_EINVAL;
  Sampler S;
  S.dim = p->dim;
  S.ext[0] = p->nx;
  S.ext[1] = p->ny;
  S.ext[2] = p->dim == 3 ? p->nz : 1;
  if (S.ext[0] < 3 || S.ext[1] < 3 || (p->dim == 3 && S.ext[2] < 3)) return MF_EINVAL;
  const size_t N = (size_t)S.ext[0] * S.ext[1] * S.ext[2];
  if (prob)
    for (size_t n = 0; n < N; ++n)
      if (!(prob[n] >= 0.0f && prob[n] <= 1.0f)) return MF_EINVAL;
  for (int a = 0; a < 3; ++a) S.per[a] = a < p->dim && p->periodic[a] != 0;
  S.gas_from = p->gas_from;
  S.prob = prob;
  S.r_min = r_min;
  S.r_max = r_max;
  S.gap = gap;
  const double h = 2.0 * r_max + gap;
  for (int a = 0; a < 3; ++a) {
    if (a < p->dim) {
      int nb = (int)floor((double)S.ext[a] / h);
      nb = nb < 1 ? 1 : (nb > 4096 ? 4096 : nb);
      S.nb[a] = nb;
      S.bw[a] = (double)S.ext[a] / nb;
    } else {
      S.nb[a] = 1;
      S.bw[a] = 1.0;
    }
  }
  S.bucket.assign((size_t)S.nb[0] * S.nb[1] * S.nb[2], {});
  if (max_n == 0) return MF_OK;
  Rng rng{seed};
  std::vector<int32_t> active;
  const int d = p->dim;
  for (int t = 0; t < 10000; ++t) {
    double x[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < d; ++a) x[a] = rng.u() * (double)S.ext[a];
    const double r = r_min + rng.u() * (r_max - r_min);
    if (S.inside(x, r)) {
      S.add(x, r);
      active.push_back(0);
      break;
    }
  }
  while (!active.empty()) {
    const size_t k = (size_t)(rng.u() * (double)active.size());
    const int32_t i = active[k];
    bool placed = false;
    for (int t = 0; t < attempts; ++t) {
      const double r = r_min + rng.u() * (r_max - r_min);
      double v[3] = {0.0, 0.0, 0.0}, q = 0.0;
      for (;;) {
        for (int a = 0; a < d; ++a) v[a] = 2.0 * rng.u() - 1.0;
        q = 0.0;
        for (int a = 0; a < d; ++a) q = q + v[a] * v[a];
        if (q > 1e-4 && q <= 1.0) break;
      }
      const double nv = sqrt(q);
      const double dd = S.sr[i] + r + gap;
      const double rho = dd * (1.0 + rng.u());
      const double si[3] = {S.sx[i], S.sy[i], S.sz[i]};
      double x[3] = {0.0, 0.0, 0.0};
      for (int a = 0; a < d; ++a) {
        double c = si[a] + (rho / nv) * v[a];
        if (S.per[a]) c = c - (double)S.ext[a] * floor(c / (double)S.ext[a]);
        x[a] = c;
      }
      if (S.inside(x, r) && S.far(x, r)) {
        S.add(x, r);
        active.push_back((int32_t)S.sr.size() - 1);
        placed = true;
        break;
      }
    }
    if (!placed) {
      active[k] = active.back();
      active.pop_back();
    }
  }
  int32_t kept = 0;
  for (size_t j = 0; j < S.sr.size() && kept < max_n; ++j) {
    const double x[3] = {S.sx[j], S.sy[j], S.sz[j]};
    const double pu = rng.u();
    if (pu < S.pval(x)) {
      centers[3 * kept + 0] = x[0];
      centers[3 * kept + 1] = x[1];
      centers[3 * kept + 2] = x[2];
      radii[kept] = S.sr[j];
      ++kept;
    }
  }
  *n_out = kept;
  return MF_OK;
}

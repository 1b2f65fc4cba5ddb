// Learned curvature closure: stencil generator, canonical orientation, bfloat16 MFMA
// matrix products with binary32 accumulation, training (forward, backward, Adam) and
// the inference kernel of the time step.
//
// Network: 125 fill fractions (5x5x5 block around an interface cell, canonical
// orientation) -> 64 -> 64 -> 1 with GELU; kappa = out / 8. Inputs and hidden
// activations are rounded to bfloat16 before each product; weights are rounded from the
// binary32 master copy. The curvature enters the gas density of Eq. rhob.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "lbm_math.h"

namespace mf {

constexpr int NF = 125, NPD = 128, NH = 64;
constexpr int OW1 = 0, OB1 = NPD * NH, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH, OB3 = OW3 + NH;
constexpr int NPARAM = OB3 + 1;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __host__ __forceinline__ uint16_t bf16_bits(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  u = u + 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_round(float f) { return __uint_as_float(((uint32_t)bf16_bits(f)) << 16); }
__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.7071067811865476f)); }
__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.7071067811865476f)) + z * expf(-0.5f * z * z) * 0.3989422804014327f;
}

// ---------------------------------------------------------------- stencil generator
// SplitMix64 (Steele, Lea & Flood 2014) as a counter-based stream per sample attempt
struct SplitMix {
  uint64_t s;
  __device__ __host__ SplitMix(uint64_t seed, int64_t sample, int attempt) {
    const uint64_t ctr = (uint64_t)(sample * 16 + attempt + 1);
    s = seed + ctr * 0xD1B54A32D192ED03ull;
  }
  __device__ __host__ uint64_t u64() {
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  __device__ __host__ double uniform() { return (double)(u64() >> 11) * 0x1p-53; }
  __device__ double normal() {
    const double u1 = uniform(), u2 = uniform();
    return sqrt(-2.0 * log(1.0 - u1)) * cos(2.0 * 3.14159265358979323846 * u2);
  }
};

struct Body {
  double a[3], R[3][3], c[3];
};

// F < 0 inside the ellipsoid; body coordinates y = R^T (x - c)
__device__ __forceinline__ double body_F(const Body &b, double x, double y, double z) {
  const double dx = x - b.c[0], dy = y - b.c[1], dz = z - b.c[2];
  double f = -1.0;
  for (int i = 0; i < 3; i++) {
    const double yi = (dx * b.R[0][i] + dy * b.R[1][i]) + dz * b.R[2][i];
    const double q = yi / b.a[i];
    f = f + q * q;
  }
  return f;
}

__device__ double inside_frac(const Body &b, double cx, double cy, double cz) {
  bool anyin = false, anyout = false;
  for (int i = 0; i < 27; i++) {
    const double f = body_F(b, cx + 0.5 * (i % 3 - 1), cy + 0.5 * ((i / 3) % 3 - 1), cz + 0.5 * (i / 9 - 1));
    if (f < 0) anyin = true;
    else anyout = true;
  }
  if (anyin && !anyout) return 1.0;
  if (anyout && !anyin) {
    // all 27 points outside (none exactly on the surface counts as inside)
    return 0.0;
  }
  int cnt = 0;
  for (int k = 0; k < 10; k++)
    for (int j = 0; j < 10; j++)
      for (int i = 0; i < 10; i++)
        if (body_F(b, cx + (i + 0.5) / 10 - 0.5, cy + (j + 0.5) / 10 - 0.5, cz + (k + 0.5) / 10 - 0.5) < 0) cnt++;
  return cnt / 1000.0;
}

// one attempt of sample `sample`; false if rejected (centre cell not cut, |kappa| > 1/2)
__device__ bool gen_attempt(uint64_t seed, int64_t sample, int attempt, double noise, float *out, float *kappa) {
  const double L2 = 0.6931471805599453, L40 = 3.6888794541139363;
  SplitMix st(seed, sample, attempt);
  Body b;
  const bool sphere = st.uniform() < 0.5;
  if (sphere) {
    const double r = exp(L2 + st.uniform() * (L40 - L2));
    b.a[0] = b.a[1] = b.a[2] = r;
  } else {
    for (int i = 0; i < 3; i++) b.a[i] = exp(L2 + st.uniform() * (L40 - L2));
  }
  double q[4];
  for (int i = 0; i < 4; i++) q[i] = st.normal();
  const double qn = sqrt(((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3]);
  for (int i = 0; i < 4; i++) q[i] /= qn;
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  b.R[0][0] = 1 - 2 * (y * y + z * z); b.R[0][1] = 2 * (x * y - w * z); b.R[0][2] = 2 * (x * z + w * y);
  b.R[1][0] = 2 * (x * y + w * z); b.R[1][1] = 1 - 2 * (x * x + z * z); b.R[1][2] = 2 * (y * z - w * x);
  b.R[2][0] = 2 * (x * z - w * y); b.R[2][1] = 2 * (y * z + w * x); b.R[2][2] = 1 - 2 * (x * x + y * y);
  double d[3];
  for (int i = 0; i < 3; i++) d[i] = st.normal();
  double s2 = 0;
  for (int i = 0; i < 3; i++) s2 += (d[i] / b.a[i]) * (d[i] / b.a[i]);
  const double sn = sqrt(s2);
  double pb[3];
  for (int i = 0; i < 3; i++) pb[i] = d[i] / sn;
  double u[3];
  for (int i = 0; i < 3; i++) u[i] = st.uniform() - 0.5;
  const bool gas_inside = st.uniform() < 0.5;
  for (int i = 0; i < 3; i++) b.c[i] = u[i] - ((b.R[i][0] * pb[0] + b.R[i][1] * pb[1]) + b.R[i][2] * pb[2]);
  float al[NF];
  for (int j = 0; j < NF; j++) {
    const double fr = inside_frac(b, (double)(j % 5 - 2), (double)((j / 5) % 5 - 2), (double)(j / 25 - 2));
    al[j] = (float)(gas_inside ? 1.0 - fr : fr);
  }
  if (!(al[62] > 0.0f && al[62] < 1.0f)) return false;
  // closest surface point to the centre cell's centre (body frame), by bisection on the
  // Lagrange parameter; then the mean curvature of the ellipsoid there
  double o[3];
  for (int i = 0; i < 3; i++) o[i] = -((b.R[0][i] * b.c[0] + b.R[1][i] * b.c[1]) + b.R[2][i] * b.c[2]);
  double a2[3] = {b.a[0] * b.a[0], b.a[1] * b.a[1], b.a[2] * b.a[2]};
  double amin2 = fmin(a2[0], fmin(a2[1], a2[2]));
  auto g = [&](double t) {
    double s = -1.0;
    for (int i = 0; i < 3; i++) { const double v = (o[i] * b.a[i]) / (a2[i] + t); s += v * v; }
    return s;
  };
  double lo = -amin2 * (1 - 1e-15);
  double hi = fmax(1.0, fmax(fabs(o[0]), fmax(fabs(o[1]), fabs(o[2]))) * fmax(b.a[0], fmax(b.a[1], b.a[2])));
  while (g(hi) > 0) hi *= 2;
  for (int it = 0; it < 200; it++) {
    const double mid = 0.5 * (lo + hi);
    if (g(mid) > 0) lo = mid;
    else hi = mid;
  }
  const double t = 0.5 * (lo + hi);
  double qc[3];
  for (int i = 0; i < 3; i++) qc[i] = o[i] * a2[i] / (a2[i] + t);
  const double num = fabs((qc[0] * qc[0] + qc[1] * qc[1] + qc[2] * qc[2]) - (a2[0] + a2[1] + a2[2]));
  const double ssum = qc[0] * qc[0] / (a2[0] * a2[0]) + qc[1] * qc[1] / (a2[1] * a2[1]) + qc[2] * qc[2] / (a2[2] * a2[2]);
  double kap = num / (2.0 * (a2[0] * a2[1] * a2[2]) * (ssum * sqrt(ssum)));
  if (!gas_inside) kap = -kap;
  if (fabs(kap) > 0.5) return false;
  for (int j = 0; j < NF; j++) {
    if (al[j] > 0.0f && al[j] < 1.0f) {
      double v = (double)al[j] + noise * st.normal();
      al[j] = (float)fmin(1.0, fmax(0.0, v));
    }
  }
  for (int j = 0; j < NF; j++) out[j] = al[j];
  *kappa = (float)kap;
  return true;
}

__global__ void k_mlp_generate(uint64_t seed, int64_t first, int64_t n, double noise, float *st, float *kap,
                               int32_t *status) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    bool ok = false;
    for (int a = 0; a < 16 && !ok; a++) ok = gen_attempt(seed, first + k, a, noise, st + k * NF, kap + k);
    if (!ok) {
      atomicOr(status, 1);
      for (int j = 0; j < NF; j++) st[k * NF + j] = 0.0f;
      kap[k] = 0.0f;
    }
  }
}

// canonical orientation: flip the axes whose central difference is negative, then order
// the axes by |gradient| descending (lower axis first on ties); dst index (e2, e1, e0)
// takes the source offset d with d[order[a]] = (flip ? -e_a : e_a)
__device__ __forceinline__ void canon_map(float gx, float gy, float gz, int order[3], int flip[3]) {
  const float g[3] = {gx, gy, gz};
  const float ag[3] = {fabsf(gx), fabsf(gy), fabsf(gz)};
  for (int i = 0; i < 3; i++) flip[i] = g[i] < 0.0f;
  int o0 = 0, o1 = 1, o2 = 2, t;
  // stable sort of three keys, descending |g|
  if (ag[o1] > ag[o0]) { t = o0; o0 = o1; o1 = t; }
  if (ag[o2] > ag[o1]) { t = o1; o1 = o2; o2 = t; }
  if (ag[o1] > ag[o0]) { t = o0; o0 = o1; o1 = t; }
  order[0] = o0;
  order[1] = o1;
  order[2] = o2;
}

// canonical stencils of raw ones, as bfloat16-rounded binary32 rows of 128 (3 zero pads)
__global__ void k_mlp_canon(const float *raw, int64_t n, float *out) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const float *s = raw + k * NF;
    auto at = [&](int dx, int dy, int dz) { return fminf(1.0f, fmaxf(0.0f, s[(dz + 2) * 25 + (dy + 2) * 5 + (dx + 2)])); };
    const float gx = 0.5f * (at(1, 0, 0) - at(-1, 0, 0));
    const float gy = 0.5f * (at(0, 1, 0) - at(0, -1, 0));
    const float gz = 0.5f * (at(0, 0, 1) - at(0, 0, -1));
    int order[3], flip[3];
    canon_map(gx, gy, gz, order, flip);
    for (int j = 0; j < NPD; j++) {
      float v = 0.0f;
      if (j < NF) {
        const int e[3] = {j % 5 - 2, (j / 5) % 5 - 2, j / 25 - 2};
        int dd[3];
        for (int a = 0; a < 3; a++) dd[order[a]] = flip[order[a]] ? -e[a] : e[a];
        v = at(dd[0], dd[1], dd[2]);
      }
      out[k * NPD + j] = bf16_round(v);
    }
  }
}

// ---------------------------------------------------------------- matrix products
// C[M][N] (row stride ldc) = op(A)[M][K] op(B)[K][N] on v_mfma_f32_16x16x32_bf16: element
// A(m,k) at A[m*sam + k*sak], B(k,n) at B[k*sbk + n*sbn], both binary32 in memory and
// rounded to bfloat16 when staged. A work-group of four waves computes a 64 x 16 tile:
// per 32-wide slice of the sum it stages the A tile [64][32] and the B tile (transposed,
// [16][32]) in LDS, read along the operand's contiguous axis, and each wave runs one
// matrix-core product for its 16 rows. M % 64 == 0, N % 16 == 0, K % 32 == 0.
// With split-K (gridDim.y > 1) the work-group of slice z sums k in [z Ks, (z+1) Ks) and
// writes its partial tile to part[z][M][N]; k_gemm_reduce adds the partials in order.
// EPI 0: C = acc; EPI 1: C = acc + bias[n] and Hout = GELU(C) rounded to bfloat16;
// EPI 2: part[z] = acc.
constexpr int GBM = 64, GBN = 16, GBK = 32;
template <int EPI>
__global__ __launch_bounds__(256) void k_gemm(const float *A, int64_t sam, int64_t sak, const float *B, int64_t sbk,
                                              int64_t sbn, float *C, int64_t ldc, int M, int N, int K, int Ks,
                                              const float *bias, float *Hout, float *part) {
  __shared__ __attribute__((aligned(16))) __bf16 sA[GBM][GBK + 8];
  __shared__ __attribute__((aligned(16))) __bf16 sB[GBN][GBK + 8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tilesN = N / GBN;
  const int tm = (int)blockIdx.x / tilesN, tn = (int)blockIdx.x % tilesN;
  const int m0 = tm * GBM, n0 = tn * GBN;
  const int kbeg = (int)blockIdx.y * Ks, kend = kbeg + Ks;
  const int r = lane & 15, q = lane >> 4;
  // staging: A along k when k is contiguous, else along m; B along k or along n
  const bool a_k = sak == 1, b_k = sbk == 1;
  floatx4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = kbeg; k0 < kend; k0 += GBK) {
#pragma unroll
    for (int j = 0; j < GBM * GBK / 256; ++j) {
      const int e = tid + 256 * j;
      const int mm = a_k ? e / GBK : e % GBM, kk = a_k ? e % GBK : e / GBM;
      sA[mm][kk] = (__bf16)__uint_as_float(((uint32_t)bf16_bits(A[(int64_t)(m0 + mm) * sam + (int64_t)(k0 + kk) * sak])) << 16);
    }
#pragma unroll
    for (int j = 0; j < GBN * GBK / 256; ++j) {
      const int e = tid + 256 * j;
      const int nn = b_k ? e / GBK : e % GBN, kk = b_k ? e % GBK : e / GBN;
      sB[nn][kk] = (__bf16)__uint_as_float(((uint32_t)bf16_bits(B[(int64_t)(k0 + kk) * sbk + (int64_t)(n0 + nn) * sbn])) << 16);
    }
    __syncthreads();
    const bf16x8 a = *(const bf16x8 *)&sA[wave * 16 + r][q * 8];
    const bf16x8 b = *(const bf16x8 *)&sB[r][q * 8];
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    __syncthreads();
  }
  for (int j = 0; j < 4; j++) {
    const int row = m0 + wave * 16 + q * 4 + j, col = n0 + r;
    if (EPI == 0) {
      C[(int64_t)row * ldc + col] = acc[j];
    } else if (EPI == 1) {
      const float zz = acc[j] + bias[col];
      C[(int64_t)row * ldc + col] = zz;
      Hout[(int64_t)row * ldc + col] = bf16_round(gelu(zz));
    } else {
      part[((int64_t)blockIdx.y * M + row) * N + col] = acc[j];
    }
  }
}

// C[m][n] = sum over the ks partial tiles, in slice order
__global__ void k_gemm_reduce(const float *part, int ks, int M, int N, float *C, int64_t ldc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M * N) return;
  float acc = 0.0f;
  for (int z = 0; z < ks; ++z) acc += part[(int64_t)z * M * N + i];
  C[(int64_t)(i / N) * ldc + i % N] = acc;
}

// slices of the sum for a product of K terms: one per 128 terms when K is long (the
// weight gradients sum over the whole batch), so that the few output tiles still fill
// the GPU; part must then hold ks * M * N floats
static int gemm_slices(int K, const float *part) { return part && K >= 1024 ? K / 128 : 1; }

static void gemm(hipStream_t s, int epi, const float *A, int64_t sam, int64_t sak, const float *B, int64_t sbk,
                 int64_t sbn, float *C, int64_t ldc, int M, int N, int K, const float *bias = nullptr,
                 float *H = nullptr, float *part = nullptr) {
  const unsigned tiles = (unsigned)((M / GBM) * (N / GBN));
  const int ks = epi == 0 ? gemm_slices(K, part) : 1;
  if (ks > 1) {
    hipLaunchKernelGGL(k_gemm<2>, dim3(tiles, ks), dim3(256), 0, s, A, sam, sak, B, sbk, sbn, C, ldc, M, N, K, K / ks,
                       bias, H, part);
    hipLaunchKernelGGL(k_gemm_reduce, dim3((M * N + 255) / 256), dim3(256), 0, s, (const float *)part, ks, M, N, C, ldc);
  } else if (epi == 0) {
    hipLaunchKernelGGL(k_gemm<0>, dim3(tiles), dim3(256), 0, s, A, sam, sak, B, sbk, sbn, C, ldc, M, N, K, K, bias, H,
                       part);
  } else {
    hipLaunchKernelGGL(k_gemm<1>, dim3(tiles), dim3(256), 0, s, A, sam, sak, B, sbk, sbn, C, ldc, M, N, K, K, bias, H,
                       part);
  }
}

// output layer: out[b] = sum_j bf16(h2[b][j]) bf16(W3[j]) + b3 (ascending j, binary32)
__global__ void k_out_layer(const float *H2, const float *theta, int B, float *out) {
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < B; b += gridDim.x * blockDim.x) {
    float acc = 0.0f;
    for (int j = 0; j < NH; j++) acc += H2[(int64_t)b * NH + j] * bf16_round(theta[OW3 + j]);
    out[b] = acc + theta[OB3];
  }
}

// loss terms and the output-layer gradient: dout = 2 (out - t) / B; dZ2 = dout W3 GELU'(Z2)
__global__ void k_out_grad(const float *out, const float *target, const float *theta, const float *Z2, int B,
                           float *dout, float *dZ2, double *loss) {
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < B; b += gridDim.x * blockDim.x) {
    const float r = out[b] - target[b];
    dout[b] = 2.0f * r / (float)B;
    atomicAdd(loss, (double)r * (double)r / (double)B);
    for (int j = 0; j < NH; j++)
      dZ2[(int64_t)b * NH + j] = dout[b] * bf16_round(theta[OW3 + j]) * gelu_grad(Z2[(int64_t)b * NH + j]);
  }
}

__global__ void k_mul_gelu_grad(float *D, const float *Z, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    D[i] = D[i] * gelu_grad(Z[i]);
}

// g[off + j] = sum_b X[b][j] * w[b] (w = NULL: plain column sums), one block per column
__global__ void k_colsum(const float *X, int ld, int ncol, const float *w, int B, float *g, int off) {
  __shared__ float sh[256];
  const int j = blockIdx.x;
  if (j >= ncol) return;
  float acc = 0.0f;
  for (int b = threadIdx.x; b < B; b += blockDim.x) acc += X[(int64_t)b * ld + j] * (w ? w[b] : 1.0f);
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) g[off + j] = sh[0];
}

__global__ void k_sum_to(const float *x, int B, float *g, int off) {
  __shared__ float sh[256];
  float acc = 0.0f;
  for (int b = threadIdx.x; b < B; b += blockDim.x) acc += x[b];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) g[off] = sh[0];
}

// Adam (Kingma & Ba 2015) with bias correction
__global__ void k_adam(float *theta, float *m, float *v, const float *g, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    if (i >= OW1 + NF * NH && i < OB1) continue;  // zero-padded input rows stay zero
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// batch of canonical rows from the training set through a multiplicative permutation
__global__ void k_gather_batch(const float *Xall, const float *Yall, int64_t ntrain, int64_t first, int64_t mult,
                               int64_t offset, int B, float *X, float *Y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)B * NPD;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = i / NPD, j = i % NPD;
    const int64_t idx = (int64_t)(((unsigned __int128)(first + b) * (unsigned __int128)mult + offset) % ntrain);
    X[i] = Xall[idx * NPD + j];
    if (j == 0) Y[b] = 8.0f * Yall[idx];
  }
}

// ---------------------------------------------------------------- network object
struct Net {
  float *theta = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
  float *Z1 = nullptr, *H1 = nullptr, *Z2 = nullptr, *H2 = nullptr, *out = nullptr, *dout = nullptr;
  float *dZ1 = nullptr, *dZ2 = nullptr, *X = nullptr, *Y = nullptr;
  float *gpart = nullptr;  // split-K partial tiles of the weight gradients
  double *loss = nullptr;
  int cap = 0;
  std::string err;
};

static hipError_t ensure_batch(Net &n, int B) {
  if (B <= n.cap) return hipSuccess;
  float **bufs[] = {&n.Z1, &n.H1, &n.Z2, &n.H2, &n.dZ1, &n.dZ2};
  for (float **b : bufs) {
    if (*b) (void)hipFree(*b);
    hipError_t e = hipMalloc(b, sizeof(float) * (size_t)B * NH);
    if (e) return e;
  }
  float **b1s[] = {&n.out, &n.dout, &n.Y};
  for (float **b : b1s) {
    if (*b) (void)hipFree(*b);
    hipError_t e = hipMalloc(b, sizeof(float) * (size_t)B);
    if (e) return e;
  }
  if (n.X) (void)hipFree(n.X);
  hipError_t e = hipMalloc(&n.X, sizeof(float) * (size_t)B * NPD);
  if (e) return e;
  if (n.gpart) (void)hipFree(n.gpart);
  const size_t ks = (size_t)(B >= 1024 ? B / 128 : 1);
  e = hipMalloc(&n.gpart, sizeof(float) * ks * NPD * NH);
  if (e) return e;
  n.cap = B;
  return hipSuccess;
}

// activations of a forward pass: pre-activations and bfloat16 GELU outputs of both
// hidden layers [B][64], outputs [B]
struct FwdBufs {
  float *Z1, *H1, *Z2, *H2, *out;
};

// forward pass of B canonical rows X (bfloat16-valued binary32 [B][128]) with the
// parameters theta into the buffers b
static void forward_into(const float *theta, const FwdBufs &b, hipStream_t s, const float *X, int B) {
  gemm(s, 1, X, NPD, 1, theta + OW1, NH, 1, b.Z1, NH, B, NH, NPD, theta + OB1, b.H1);
  gemm(s, 1, b.H1, NH, 1, theta + OW2, NH, 1, b.Z2, NH, B, NH, NH, theta + OB2, b.H2);
  hipLaunchKernelGGL(k_out_layer, dim3((B + 255) / 256), dim3(256), 0, s, b.H2, theta, B, b.out);
}

static void forward(Net &n, hipStream_t s, const float *X, int B) {
  forward_into(n.theta, FwdBufs{n.Z1, n.H1, n.Z2, n.H2, n.out}, s, X, B);
}

// ------------------------------------------------- evaluation without allocation
// Device memory of mf_mlp_eval_noalloc: canonical rows [kNoAllocMax][128], the four
// hidden-layer arrays [kNoAllocMax][64] and the outputs [kNoAllocMax], 12.6 MB held by
// every GPU the library runs on until the process ends. Host code never names it: its
// address on the current device comes from hipGetSymbolAddress.
constexpr int kNoAllocMax = 8192;
constexpr size_t kScratchFloats = (size_t)kNoAllocMax * (NPD + 4 * NH + 1);
static __device__ __align__(256) float scratch[kScratchFloats];

// zero rows [n0, n1) of a [*][128] array (the padding rows of the last 64-row tile)
__global__ void k_zero_rows(float *X, int n0, int n1) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (int64_t)(n1 - n0) * NPD) X[(int64_t)n0 * NPD + i] = 0.0f;
}

// kappa = out / 8
__global__ void k_scale_out(const float *out, int n, float *kappa) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) kappa[i] = out[i] * 0.125f;
}

// loss and gradient of the mean squared error against Y (= 8 kappa), into n.g
static void backward(Net &n, hipStream_t s, const float *X, const float *Y, int B) {
  (void)hipMemsetAsync(n.loss, 0, sizeof(double), s);
  hipLaunchKernelGGL(k_out_grad, dim3((B + 255) / 256), dim3(256), 0, s, n.out, Y, n.theta, n.Z2, B, n.dout, n.dZ2,
                     n.loss);
  // W3, b3
  hipLaunchKernelGGL(k_colsum, dim3(NH), dim3(256), 0, s, n.H2, NH, NH, n.dout, B, n.g, OW3);
  hipLaunchKernelGGL(k_sum_to, dim3(1), dim3(256), 0, s, n.dout, B, n.g, OB3);
  // W2 = H1^T dZ2, b2
  gemm(s, 0, n.H1, 1, NH, n.dZ2, NH, 1, n.g + OW2, NH, NH, NH, B, nullptr, nullptr, n.gpart);
  hipLaunchKernelGGL(k_colsum, dim3(NH), dim3(256), 0, s, n.dZ2, NH, NH, (const float *)nullptr, B, n.g, OB2);
  // dZ1 = (dZ2 W2^T) * GELU'(Z1)
  gemm(s, 0, n.dZ2, NH, 1, n.theta + OW2, 1, NH, n.dZ1, NH, B, NH, NH);
  hipLaunchKernelGGL(k_mul_gelu_grad, dim3(256), dim3(256), 0, s, n.dZ1, n.Z1, (int64_t)B * NH);
  // W1 = X^T dZ1, b1
  gemm(s, 0, X, 1, NPD, n.dZ1, NH, 1, n.g + OW1, NH, NPD, NH, B, nullptr, nullptr, n.gpart);
  hipLaunchKernelGGL(k_colsum, dim3(NH), dim3(256), 0, s, n.dZ1, NH, NH, (const float *)nullptr, B, n.g, OB1);
}

// ---------------------------------------------------------------- step inference
// Each wave takes 16 interface cells at a time, independently of the other waves of
// its work-group: it gathers the 5x5x5 stencils in natural order (contiguous along x)
// and writes each value to its canonical position in the wave's LDS rows as bfloat16,
// runs the two hidden layers on the matrix cores (16 cells x 64 units, weights held
// transposed in LDS so that each B fragment is one 8-byte read), and the output layer
// as a 16-lane shuffle reduction. The canonical position of an element is linear in its
// offsets (dx, dy, dz): 62 + cx dx + cy dy + cz dz, where each coefficient is +-1, +-5 or
// +-25 (the place value of the canonical axis the source axis goes to, negated when the
// axis is flipped), so each cell carries three small integers instead of a table. The
// gathers of the next 16 cells are issued before the products of the current ones. A cell whose stencil meets a wall, leaves the domain
// or meets a gas / interface cell of another bubble, or whose network curvature exceeds
// the trained range |kappa| <= 1/2, is left to the plain fit.
struct alignas(16) MlpWaveLds {
  // canonical stencils of 16 cells; the first hidden layer overwrites them once the
  // wave's layer-1 products have read them
  union {
    short a[16][NPD + 8];
    short h[16][NH + 8];
  };
  // the 64 cells of the wave's tile
  // per cell: index, coordinates, id + 1, flags, packed canonical-slot coefficients,
  // and the bfloat16 bits of its clamped fill fraction (what a wall element reads)
  int cell[64], x[64], y[64], z[64], lab1[64], code[64], coef[64], acb[64];
};

// bfloat16 bits of a binary32 value, round to nearest even (hardware conversion)
__device__ __forceinline__ short bf16_hw(float f) { return __builtin_bit_cast(short, (__bf16)f); }

// GELU for inference: erf from the rational approximation of Abramowitz & Stegun (1964),
// formula 7.1.26 (absolute error below 1.5e-7, far under the bfloat16 rounding that
// follows every activation), with the hardware base-2 exponential and reciprocal
__device__ __forceinline__ float gelu_fast(float z) {
  const float x = fabsf(z) * 0.7071067811865476f;
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, x, 1.0f));
  float poly = fmaf(1.061405429f, t, -1.453152027f);
  poly = fmaf(poly, t, 1.421413741f);
  poly = fmaf(poly, t, -0.284496736f);
  poly = fmaf(poly, t, 0.254829592f);
  const float y = 1.0f - poly * t * __builtin_amdgcn_exp2f(-1.4426950408889634f * x * x);
  return 0.5f * z * (1.0f + (z < 0.0f ? -y : y));
}

// fill fraction a stencil reads at a cell of type t (walls read the centre value)
template <class R>
__device__ __forceinline__ float stencil_value(int t, R alpha, float centre) {
  return t == TG ? 0.0f : (t == TL ? 1.0f : (t == TI ? fminf(1.0f, fmaxf(0.0f, (float)alpha)) : centre));
}

template <class T> __device__ __forceinline__ T uniform(T v) {
  return __builtin_bit_cast(T, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

template <int P>
__device__ __forceinline__ void b_mlp_curv(const GridPos &gp, KP p, DA d) {
  using R = typename Prec<P>::R;
  __shared__ __attribute__((aligned(16))) short sW1[NH][NPD + 8];  // W1 transposed: [unit][input]
  __shared__ __attribute__((aligned(16))) short sW2[NH][NH + 8];   // W2 transposed: [unit][input]
  __shared__ float sB1[NH], sB2[NH], sW3[NH];
  __shared__ MlpWaveLds sw[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint16_t *W = d.mlp_w;  // bf16: W1 [128][64], W2 [64][64], W3 [64]
  const float *bias = d.mlp_b;  // b1 [64], b2 [64], b3
  for (int i = tid; i < NPD * NH; i += 256) sW1[i % NH][i / NH] = (short)W[i];
  for (int i = tid; i < NH * NH; i += 256) sW2[i % NH][i / NH] = (short)W[NPD * NH + i];
  if (tid < NH) {
    sB1[tid] = bias[tid];
    sB2[tid] = bias[NH + tid];
    sW3[tid] = __uint_as_float(((uint32_t)W[NPD * NH + NH * NH + tid]) << 16);
  }
  __syncthreads();
  const float b3 = bias[2 * NH];
  MlpWaveLds &M = sw[wave];
  const R *alpha = (const R *)d.alpha;

  const int nI = *(volatile int32_t *)(d.cnt + C_I);
  const int nNI = *(volatile int32_t *)(d.cnt + C_NI);
  const int nL = *(volatile int32_t *)(d.cnt + C_L2I);
  const int64_t total = (int64_t)nI + nNI + nL;
  const int64_t nxy = (int64_t)p.nx * p.ny;
  const bool periodic = p.per[0] || p.per[1] || p.per[2];
  // lane (r, q = lane / 16): row r of the A operand and column r of B, with the eight
  // inputs 8 q .. 8 q + 7 of each 32-wide slice of the sum (v_mfma_f32_16x16x32_bf16);
  // it receives the results of rows 4 q .. 4 q + 3, column r
  const int r = lane & 15, kq = (lane >> 4) * 4, kq8 = (lane >> 4) * 8;
  // the lane's two stencil elements j = lane and lane + 64: offsets and index offsets
  const int j1 = lane + 64;
  const int dx0 = lane % 5 - 2, dy0 = (lane / 5) % 5 - 2, dz0 = lane / 25 - 2;
  const int dx1 = j1 % 5 - 2, dy1 = (j1 / 5) % 5 - 2, dz1 = j1 / 25 - 2;
  const int64_t off0 = (int64_t)dx0 + (int64_t)p.nx * dy0 + nxy * dz0;
  const int64_t off1 = (int64_t)dx1 + (int64_t)p.nx * dy1 + nxy * dz1;
  // the same offsets as packed signed bytes, for the canonical-slot dot product
  const int dpk0 = (dx0 & 0xFF) | ((dy0 & 0xFF) << 8) | ((dz0 & 0xFF) << 16);
  const int dpk1 = (dx1 & 0xFF) | ((dy1 & 0xFF) << 8) | ((dz1 & 0xFF) << 16);
  // stencil words of cells sb .. sb+15: slot m of a lane is element lane + 64 (m & 1) of
  // cell sb + (m >> 1); all 32 loads are issued before any is used
  uint32_t wd[32];
  auto gather = [&](int sb) {
    if (!periodic) {
      // without wrap every load is issued; a slot that reads nothing loads the cell's own
      // word (or word 0) and is replaced by the outside marker
#pragma unroll
      for (int m = 0; m < 32; ++m) {
        const int c = sb + (m >> 1), h = m & 1;
        const int cc = uniform(M.cell[c]);
        const bool ok = cc >= 0 && !(uniform(M.code[c]) & 64) && (h == 0 || j1 < NF);
        const int64_t yy = ok ? (int64_t)cc + (h ? off1 : off0) : (cc >= 0 ? (int64_t)cc : 0);
        const uint32_t w = d.sword[yy];
        wd[m] = ok ? w : 0xFFFF0000u;
      }
    } else {
#pragma unroll
      for (int m = 0; m < 32; ++m) {
        const int c = sb + (m >> 1), h = m & 1;
        const int cc = uniform(M.cell[c]);
        int64_t yy = -1;
        if (cc >= 0 && !(uniform(M.code[c]) & 64) && (h == 0 || j1 < NF))
          yy = nb_index_or_none(p, M.x[c], M.y[c], M.z[c], h ? dx1 : dx0, h ? dy1 : dy0, h ? dz1 : dz0);
        wd[m] = yy >= 0 ? d.sword[yy] : 0xFFFF0000u;
      }
    }
  };
  for (int64_t t0 = ((int64_t)gp.bid * 4 + wave) * 64; t0 < total; t0 += (int64_t)gp.nblk * 4 * 64) {
    // set-up, one cell per lane: the cell and its six axis neighbours are loaded
    // together once the list entry is known
    {
      const int64_t k = t0 + lane;
      int cell = -1;
      if (k < total) cell = k < nI ? d.ilist[k] : (k < (int64_t)nI + nNI ? d.nilist[k - nI] : d.l2ilist[k - nI - nNI]);
      int cx = 0, cy = 0, cz = 0, code = 0, lab = 0, coef = 0;
      float ac = 0.0f;
      if (cell >= 0) {
        cell_xyz(p, cell, cx, cy, cz);
        int64_t nb6[6];
        int tn6[6];
        R al6[6];
        const int off[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
#pragma unroll
        for (int q = 0; q < 6; ++q) nb6[q] = nb_index_or_none(p, cx, cy, cz, off[q][0], off[q][1], off[q][2]);
        const int tc = d.type[cell] & TMASK;
        const R al = alpha[cell];
        lab = d.label[cell];
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          tn6[q] = nb6[q] >= 0 ? d.type[nb6[q]] & TMASK : TW;
          al6[q] = nb6[q] >= 0 ? alpha[nb6[q]] : R(0);
        }
        if (tc != TI) {
          cell = -1;
        } else {
          ac = fminf(1.0f, fmaxf(0.0f, (float)al));
          float v6[6];
#pragma unroll
          for (int q = 0; q < 6; ++q) v6[q] = stencil_value<R>(tn6[q], al6[q], ac);
          int order[3], flip[3];
          canon_map(0.5f * (v6[0] - v6[1]), 0.5f * (v6[2] - v6[3]), 0.5f * (v6[4] - v6[5]), order, flip);
          int cf[3];
          const int place[3] = {1, 5, 25};
          for (int a = 0; a < 3; ++a) cf[order[a]] = flip[order[a]] ? -place[a] : place[a];
          coef = (cf[0] & 0xFF) | ((cf[1] & 0xFF) << 8) | ((cf[2] & 0xFF) << 16);
          // on a closed axis, a cell within two cells of the wall layer has a wall in
          // its stencil: left to the plain fit without a gather
          const int cxyz[3] = {cx, cy, cz}, dims[3] = {p.nx, p.ny, p.nz};
          for (int a = 0; a < 3; ++a)
            if (!p.per[a] && (cxyz[a] < 3 || cxyz[a] > dims[a] - 4)) code |= 64;
        }
      }
      M.cell[lane] = cell;
      M.x[lane] = cx;
      M.y[lane] = cy;
      M.z[lane] = cz;
      M.lab1[lane] = lab + 1;
      M.code[lane] = code;
      M.coef[lane] = coef;
      M.acb[lane] = (int)(uint16_t)bf16_hw(ac);
    }
    wave_lds_sync();
    gather(0);
    for (int sb = 0; sb < 64; sb += 16) {
      if (t0 + sb >= total) break;  // wave-uniform
      // each gathered word to its canonical slot; a wall (or the outside of a closed
      // axis), or gas / interface of another bubble, sends the cell to the plain fit
      unsigned badm = 0;
#pragma unroll
      for (int m = 0; m < 32; ++m) {
        const int c = sb + (m >> 1), h = m & 1, j = lane + 64 * h;
        const int cc = uniform(M.cell[c]);
        if (cc < 0 || j >= NF) {
          M.a[m >> 1][j] = 0;
          continue;
        }
        const uint32_t code = wd[m] >> 16;
        // a wall (0xFFFF never equals an id + 1) or gas / interface of another bubble
        if (code != 0u && code != (uint32_t)uniform(M.lab1[c])) badm |= 1u << (m >> 1);
        const short bits = (short)(code == 0xFFFFu ? (uint32_t)uniform(M.acb[c]) : wd[m] & 0xFFFFu);
        // 62 + cx dx + cy dy + cz dz on packed signed bytes
        const int slot = __builtin_amdgcn_sdot4(h ? dpk1 : dpk0, uniform(M.coef[c]), 62, false);
        M.a[m >> 1][slot] = bits;
      }
      // the next 16 cells' loads run under this sub-tile's products
      if (sb + 16 < 64 && t0 + sb + 16 < total) gather(sb + 16);
      for (int o = 32; o > 0; o >>= 1) badm |= __shfl_xor(badm, o);
      wave_lds_sync();
      // first hidden layer
      floatx4 acc[4];
      for (int tn = 0; tn < 4; tn++) acc[tn] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int k0 = 0; k0 < NPD; k0 += 32) {
        const bf16x8 a = *(const bf16x8 *)&M.a[r][k0 + kq8];
#pragma unroll
        for (int tn = 0; tn < 4; tn++) {
          const bf16x8 b = *(const bf16x8 *)&sW1[tn * 16 + r][k0 + kq8];
          acc[tn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[tn], 0, 0, 0);
        }
      }
      wave_lds_sync();  // every lane has read its stencil rows before they are overwritten
#pragma unroll
      for (int tn = 0; tn < 4; tn++)
#pragma unroll
        for (int j = 0; j < 4; j++) M.h[kq + j][tn * 16 + r] = bf16_hw(gelu_fast(acc[tn][j] + sB1[tn * 16 + r]));
      wave_lds_sync();
      // second hidden layer
      for (int tn = 0; tn < 4; tn++) acc[tn] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int k0 = 0; k0 < NH; k0 += 32) {
        const bf16x8 a = *(const bf16x8 *)&M.h[r][k0 + kq8];
#pragma unroll
        for (int tn = 0; tn < 4; tn++) {
          const bf16x8 b = *(const bf16x8 *)&sW2[tn * 16 + r][k0 + kq8];
          acc[tn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[tn], 0, 0, 0);
        }
      }
      // output layer: lane (r, kq) holds units tn*16 + r of cells kq .. kq+3
      float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int tn = 0; tn < 4; tn++)
#pragma unroll
        for (int j = 0; j < 4; j++) {
          const float hv =
              __uint_as_float(((uint32_t)(uint16_t)bf16_hw(gelu_fast(acc[tn][j] + sB2[tn * 16 + r]))) << 16);
          part[j] += hv * sW3[tn * 16 + r];
        }
#pragma unroll
      for (int j = 0; j < 4; j++)
        for (int o = 8; o > 0; o >>= 1) part[j] += __shfl_xor(part[j], o);
      if (r == 0) {
#pragma unroll
        for (int j = 0; j < 4; j++) {
          const int c = kq + j;
          const int cc = M.cell[sb + c];
          const float kap = (part[j] + b3) * 0.125f;
          if (cc >= 0 && !((badm >> c) & 1) && !(M.code[sb + c] & 64) && fabsf(kap) <= 0.5f) {
            ((R *)d.kappa)[cc] = (R)kap;
            d.cflag[cc] = (uint8_t)CF_MLPOK;
          }
        }
      }
      wave_lds_sync();
    }
  }
}
template <int P>
__global__ __launch_bounds__(256) void k_mlp_curv(KP p, DA d) {
  b_mlp_curv<P>(GridPos::hw(), p, d);
}

template <int P>
__global__ __launch_bounds__(256) void km_mlp_curv(MLaunch ml) {
  MF_MULTI(MK_MLP)
  b_mlp_curv<P>(gp, m.kp, m.d);
}

// the learned curvature of every domain of a batch (3D, networks attached)
void mlp_curv_multi(const MStep &ms, int precision, hipStream_t s) {
  switch (precision) {
    case 0: hipLaunchKernelGGL(km_mlp_curv<0>, dim3(ms.grid[MK_MLP]), dim3(256), 0, s, ms.at(MK_MLP)); break;
    case 1: hipLaunchKernelGGL(km_mlp_curv<1>, dim3(ms.grid[MK_MLP]), dim3(256), 0, s, ms.at(MK_MLP)); break;
    case 2: hipLaunchKernelGGL(km_mlp_curv<2>, dim3(ms.grid[MK_MLP]), dim3(256), 0, s, ms.at(MK_MLP)); break;
    default: hipLaunchKernelGGL(km_mlp_curv<3>, dim3(ms.grid[MK_MLP]), dim3(256), 0, s, ms.at(MK_MLP)); break;
  }
}

void launch_mlp_curv(Ctx &c, hipStream_t s) {
  // persistent work-groups (each stages the weights once): the LDS of a CU holds three,
  // so three per CU of the 256 run in one round
  const unsigned nb = list_blocks(c) < 768 ? list_blocks(c) : 768;
  if (c.kp.dim != 3) return;
  switch (c.P.precision) {
    case 0: hipLaunchKernelGGL(k_mlp_curv<0>, dim3(nb), dim3(256), 0, s, c.kp, c.d); break;
    case 1: hipLaunchKernelGGL(k_mlp_curv<1>, dim3(nb), dim3(256), 0, s, c.kp, c.d); break;
    case 2: hipLaunchKernelGGL(k_mlp_curv<2>, dim3(nb), dim3(256), 0, s, c.kp, c.d); break;
    default: hipLaunchKernelGGL(k_mlp_curv<3>, dim3(nb), dim3(256), 0, s, c.kp, c.d); break;
  }
}

}  // namespace mf

// ---------------------------------------------------------------- C ABI
using namespace mf;

struct mf_mlp : Net {};

namespace {
int fail(const std::string &m, int rc) {
  mf::g_thread_err = m;
  return rc;
}
// address of scratch on the current device, looked up once per device (each GPU holds
// its own copy of the array at its own address)
static int scratch_address(float **out) {
  static std::mutex mu;
  static float *addr[256] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(std::string("hipGetDevice: ") + hipGetErrorString(e), MF_EHIP);
  if (dev < 0 || dev >= 256) return fail("device ordinal out of range", MF_EINTERNAL);
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return fail(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e), MF_EHIP);
    addr[dev] = (float *)p;
  }
  *out = addr[dev];
  return MF_OK;
}

#define MLPCHK(expr)                                                                        \
  do {                                                                                      \
    hipError_t _e = (expr);                                                                 \
    if (_e != hipSuccess) return fail(std::string(#expr) + ": " + hipGetErrorString(_e), MF_EHIP); \
  } while (0)
}  // namespace

extern "C" {

int mf_mlp_param_count(void) { return NPARAM; }

int mf_mlp_create(uint64_t init_seed, mf_mlp **out) {
  if (!out) return fail("out is NULL", MF_EINVAL);
  mf_mlp *m = new mf_mlp();
  std::vector<float> th(NPARAM, 0.0f);
  SplitMix st(init_seed, 0, 0);
  const int fan[3] = {NF, NH, NH};
  const int off[3] = {OW1, OW2, OW3};
  const int cnt[3] = {NPD * NH, NH * NH, NH};
  for (int l = 0; l < 3; l++) {
    const double lim = 1.0 / sqrt((double)fan[l]);
    for (int i = 0; i < cnt[l]; i++) th[off[l] + i] = (float)((2.0 * st.uniform() - 1.0) * lim);
  }
  for (int i = NF * NH; i < NPD * NH; i++) th[OW1 + i] = 0.0f;
  float **bufs[] = {&m->theta, &m->m, &m->v, &m->g};
  for (float **b : bufs) MLPCHK(hipMalloc(b, sizeof(float) * NPARAM));
  MLPCHK(hipMalloc(&m->loss, sizeof(double)));
  MLPCHK(hipMemcpy(m->theta, th.data(), sizeof(float) * NPARAM, hipMemcpyHostToDevice));
  MLPCHK(hipMemset(m->m, 0, sizeof(float) * NPARAM));
  MLPCHK(hipMemset(m->v, 0, sizeof(float) * NPARAM));
  *out = m;
  return MF_OK;
}

int mf_mlp_destroy(mf_mlp *m) {
  if (!m) return MF_OK;
  float *bufs[] = {m->theta, m->m, m->v, m->g, m->Z1, m->H1, m->Z2, m->H2, m->out, m->dout, m->dZ1, m->dZ2, m->X, m->Y,
                   m->gpart};
  for (float *b : bufs)
    if (b) (void)hipFree(b);
  if (m->loss) (void)hipFree(m->loss);
  delete m;
  return MF_OK;
}

// network file: magic, parameter count, the binary32 master parameters
static const char kMlpMagic[8] = {'M', 'I', 'F', 'O', 'A', 'M', 'N', 'N'};

int mf_mlp_save(const mf_mlp *m, const char *path) {
  if (!m || !path) return fail("NULL argument", MF_EINVAL);
  std::vector<float> th(NPARAM);
  MLPCHK(hipMemcpy(th.data(), m->theta, sizeof(float) * NPARAM, hipMemcpyDeviceToHost));
  FILE *fp = fopen(path, "wb");
  if (!fp) return fail(std::string("cannot open ") + path + " for writing", MF_EINVAL);
  const int32_t np = NPARAM;
  bool ok = fwrite(kMlpMagic, 1, 8, fp) == 8 && fwrite(&np, 4, 1, fp) == 1 &&
            fwrite(th.data(), sizeof(float), NPARAM, fp) == (size_t)NPARAM;
  if (fclose(fp) != 0) ok = false;
  return ok ? MF_OK : fail(std::string("writing ") + path + " failed", MF_EHIP);
}

int mf_mlp_load(mf_mlp **out, const char *path) {
  if (!out || !path) return fail("NULL argument", MF_EINVAL);
  *out = nullptr;
  FILE *fp = fopen(path, "rb");
  if (!fp) return fail(std::string("cannot open ") + path, MF_EINVAL);
  char magic[8];
  int32_t np = 0;
  std::vector<float> th(NPARAM);
  const bool ok = fread(magic, 1, 8, fp) == 8 && memcmp(magic, kMlpMagic, 8) == 0 && fread(&np, 4, 1, fp) == 1 &&
                  np == NPARAM && fread(th.data(), sizeof(float), NPARAM, fp) == (size_t)NPARAM;
  fclose(fp);
  if (!ok) return fail(std::string(path) + " is not a network file of this library", MF_EINVAL);
  mf_mlp *m = nullptr;
  const int rc = mf_mlp_create(0, &m);
  if (rc) return rc;
  const hipError_t e = hipMemcpy(m->theta, th.data(), sizeof(float) * NPARAM, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    mf_mlp_destroy(m);
    return fail(std::string("hipMemcpy: ") + hipGetErrorString(e), MF_EHIP);
  }
  *out = m;
  return MF_OK;
}

int mf_mlp_get_params(const mf_mlp *m, float *dst) {
  if (!m || !dst) return fail("NULL argument", MF_EINVAL);
  MLPCHK(hipMemcpy(dst, m->theta, sizeof(float) * NPARAM, hipMemcpyDeviceToHost));
  return MF_OK;
}

int mf_mlp_set_params(mf_mlp *m, const float *src) {
  if (!m || !src) return fail("NULL argument", MF_EINVAL);
  MLPCHK(hipMemcpy(m->theta, src, sizeof(float) * NPARAM, hipMemcpyHostToDevice));
  return MF_OK;
}

int mf_mlp_generate(uint64_t seed, int64_t first, int64_t n, double noise, float *stencils, float *kappa, void *stream) {
  if (n < 0 || (n > 0 && (!stencils || !kappa))) return fail("bad arguments", MF_EINVAL);
  if (n == 0) return MF_OK;
  hipStream_t s = (hipStream_t)stream;
  float *dS = nullptr, *dK = nullptr;
  int32_t *dst = nullptr, st = 0;
  MLPCHK(hipMalloc(&dS, sizeof(float) * n * NF));
  MLPCHK(hipMalloc(&dK, sizeof(float) * n));
  MLPCHK(hipMalloc(&dst, 4));
  MLPCHK(hipMemsetAsync(dst, 0, 4, s));
  hipLaunchKernelGGL(k_mlp_generate, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, seed, first, n, noise, dS, dK,
                     dst);
  MLPCHK(hipMemcpyAsync(stencils, dS, sizeof(float) * n * NF, hipMemcpyDeviceToHost, s));
  MLPCHK(hipMemcpyAsync(kappa, dK, sizeof(float) * n, hipMemcpyDeviceToHost, s));
  MLPCHK(hipMemcpyAsync(&st, dst, 4, hipMemcpyDeviceToHost, s));
  MLPCHK(hipStreamSynchronize(s));
  (void)hipFree(dS);
  (void)hipFree(dK);
  (void)hipFree(dst);
  if (st) return fail("a sample found no valid attempt", MF_ENUMERIC);
  return MF_OK;
}

int mf_mlp_eval(const mf_mlp *mc, const float *stencils, int64_t n, float *kappa, void *stream) {
  mf_mlp *m = const_cast<mf_mlp *>(mc);
  if (!m || n < 0 || (n > 0 && (!stencils || !kappa))) return fail("bad arguments", MF_EINVAL);
  if (n == 0) return MF_OK;
  hipStream_t s = (hipStream_t)stream;
  const int64_t npad = (n + 63) / 64 * 64;
  MLPCHK(ensure_batch(*m, (int)npad));
  float *raw = nullptr;
  MLPCHK(hipMalloc(&raw, sizeof(float) * npad * NF));
  MLPCHK(hipMemsetAsync(raw, 0, sizeof(float) * npad * NF, s));
  MLPCHK(hipMemcpyAsync(raw, stencils, sizeof(float) * n * NF, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_mlp_canon, dim3((unsigned)((npad + 255) / 256)), dim3(256), 0, s, raw, npad, m->X);
  forward(*m, s, m->X, (int)npad);
  std::vector<float> out(npad);
  MLPCHK(hipMemcpyAsync(out.data(), m->out, sizeof(float) * npad, hipMemcpyDeviceToHost, s));
  MLPCHK(hipStreamSynchronize(s));
  (void)hipFree(raw);
  for (int64_t i = 0; i < n; i++) kappa[i] = out[i] * 0.125f;
  return MF_OK;
}

int mf_mlp_eval_noalloc(const mf_mlp *m, const float *stencils, int64_t n, float *kappa, void *stream) {
  if (!m || n < 0 || (n > 0 && (!stencils || !kappa))) return fail("bad arguments", MF_EINVAL);
  if (n > kNoAllocMax)
    return fail("mf_mlp_eval_noalloc takes at most " + std::to_string(kNoAllocMax) + " stencils per call",
                MF_EINVAL);
  if (n == 0) return MF_OK;
  float *scr = nullptr;
  const int rc = scratch_address(&scr);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int nn = (int)n, npad = (nn + 63) / 64 * 64;
  float *X = scr;
  const FwdBufs b{X + (size_t)kNoAllocMax * NPD, X + (size_t)kNoAllocMax * (NPD + NH),
                  X + (size_t)kNoAllocMax * (NPD + 2 * NH), X + (size_t)kNoAllocMax * (NPD + 3 * NH),
                  X + (size_t)kNoAllocMax * (NPD + 4 * NH)};
  hipLaunchKernelGGL(k_mlp_canon, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, stencils, (int64_t)nn, X);
  // the rows up to the next multiple of 64 hold the previous call's values: clear them
  if (npad > nn)
    hipLaunchKernelGGL(k_zero_rows, dim3((unsigned)(((npad - nn) * NPD + 255) / 256)), dim3(256), 0, s, X, nn, npad);
  forward_into(m->theta, b, s, X, npad);
  hipLaunchKernelGGL(k_scale_out, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, b.out, nn, kappa);
  MLPCHK(hipGetLastError());
  return MF_OK;
}

int mf_mlp_grad(const mf_mlp *mc, const float *stencils, const float *target8, int32_t B, float *grad, double *loss,
                void *stream) {
  mf_mlp *m = const_cast<mf_mlp *>(mc);
  if (!m || B <= 0 || (B % 64) || !stencils || !target8 || !grad) return fail("bad arguments (B % 64 == 0)", MF_EINVAL);
  hipStream_t s = (hipStream_t)stream;
  MLPCHK(ensure_batch(*m, B));
  float *raw = nullptr;
  MLPCHK(hipMalloc(&raw, sizeof(float) * B * NF));
  MLPCHK(hipMemcpyAsync(raw, stencils, sizeof(float) * B * NF, hipMemcpyHostToDevice, s));
  MLPCHK(hipMemcpyAsync(m->Y, target8, sizeof(float) * B, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_mlp_canon, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, raw, (int64_t)B, m->X);
  forward(*m, s, m->X, B);
  backward(*m, s, m->X, m->Y, B);
  MLPCHK(hipMemcpyAsync(grad, m->g, sizeof(float) * NPARAM, hipMemcpyDeviceToHost, s));
  double l = 0;
  MLPCHK(hipMemcpyAsync(&l, m->loss, sizeof(double), hipMemcpyDeviceToHost, s));
  MLPCHK(hipStreamSynchronize(s));
  (void)hipFree(raw);
  if (loss) *loss = l;
  return MF_OK;
}

int mf_mlp_train(mf_mlp *m, const mf_mlp_train_spec *sp, void *stream, double *val_rmse) {
  if (!m || !sp || sp->struct_size != sizeof(mf_mlp_train_spec)) return fail("bad spec", MF_EINVAL);
  if (sp->n_train < sp->batch || sp->batch <= 0 || sp->batch % 64 || sp->epochs <= 0 || sp->n_val < 0)
    return fail("need n_train >= batch, batch % 64 == 0, epochs > 0", MF_EINVAL);
  hipStream_t s = (hipStream_t)stream;
  const int64_t ntot = sp->n_train + sp->n_val;
  float *raw = nullptr, *Xall = nullptr, *Yall = nullptr;
  int32_t *dst = nullptr, st = 0;
  MLPCHK(hipMalloc(&raw, sizeof(float) * ntot * NF));
  MLPCHK(hipMalloc(&Xall, sizeof(float) * ntot * NPD));
  MLPCHK(hipMalloc(&Yall, sizeof(float) * ntot));
  MLPCHK(hipMalloc(&dst, 4));
  MLPCHK(hipMemsetAsync(dst, 0, 4, s));
  hipLaunchKernelGGL(k_mlp_generate, dim3((unsigned)((ntot + 127) / 128)), dim3(128), 0, s, sp->data_seed, (int64_t)0,
                     ntot, sp->noise, raw, Yall, dst);
  hipLaunchKernelGGL(k_mlp_canon, dim3((unsigned)((ntot + 255) / 256)), dim3(256), 0, s, raw, ntot, Xall);
  MLPCHK(hipFree(raw));
  MLPCHK(ensure_batch(*m, sp->batch));
  const int B = sp->batch;
  const int64_t per_epoch = sp->n_train / B;
  const int64_t T = per_epoch * sp->epochs;
  // multiplier of the per-epoch permutation: an odd number coprime to n_train
  auto coprime = [](int64_t a, int64_t b) {
    while (b) { int64_t t = a % b; a = b; b = t; }
    return a == 1;
  };
  SplitMix perm(sp->data_seed ^ 0x5DEECE66DULL, 1, 0);
  int64_t t = 0;
  for (int ep = 0; ep < sp->epochs; ep++) {
    int64_t mult = (int64_t)(perm.u64() % (uint64_t)sp->n_train) | 1;
    while (!coprime(mult, sp->n_train)) mult += 2;
    const int64_t offset = (int64_t)(perm.u64() % (uint64_t)sp->n_train);
    for (int64_t it = 0; it < per_epoch; it++, t++) {
      hipLaunchKernelGGL(k_gather_batch, dim3(512), dim3(256), 0, s, Xall, Yall, sp->n_train, it * B, mult, offset, B,
                         m->X, m->Y);
      forward(*m, s, m->X, B);
      backward(*m, s, m->X, m->Y, B);
      const double lr = sp->lr * 0.5 * (1.0 + cos(3.14159265358979323846 * (double)t / (double)T));
      const float c1 = (float)(1.0 - pow(0.9, (double)(t + 1))), c2 = (float)(1.0 - pow(0.999, (double)(t + 1)));
      hipLaunchKernelGGL(k_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, s, m->theta, m->m, m->v, m->g, NPARAM,
                         (float)lr, 0.9f, 0.999f, 1e-8f, c1, c2);
    }
    MLPCHK(hipGetLastError());
  }
  // validation error of kappa
  double se = 0.0;
  int64_t nv = 0;
  std::vector<float> out(B), y(B);
  for (int64_t v0 = sp->n_train; v0 + B <= ntot; v0 += B) {
    forward(*m, s, Xall + v0 * NPD, B);
    MLPCHK(hipMemcpyAsync(out.data(), m->out, sizeof(float) * B, hipMemcpyDeviceToHost, s));
    MLPCHK(hipMemcpyAsync(y.data(), Yall + v0, sizeof(float) * B, hipMemcpyDeviceToHost, s));
    MLPCHK(hipStreamSynchronize(s));
    for (int i = 0; i < B; i++) {
      const double e = out[i] * 0.125 - y[i];
      se += e * e;
      nv++;
    }
  }
  MLPCHK(hipMemcpyAsync(&st, dst, 4, hipMemcpyDeviceToHost, s));
  MLPCHK(hipStreamSynchronize(s));
  (void)hipFree(Xall);
  (void)hipFree(Yall);
  (void)hipFree(dst);
  if (st) return fail("a training sample found no valid attempt", MF_ENUMERIC);
  if (val_rmse) *val_rmse = nv ? sqrt(se / nv) : 0.0;
  return MF_OK;
}

}  // extern "C"

// weights of a network as the bfloat16 / binary32 arrays of a context
int mf_mlp_export_weights(const mf_mlp *m, uint16_t *w_dev, float *b_dev, hipStream_t s) {
  std::vector<float> th(NPARAM);
  if (hipMemcpy(th.data(), m->theta, sizeof(float) * NPARAM, hipMemcpyDeviceToHost)) return MF_EHIP;
  std::vector<uint16_t> w(NPD * NH + NH * NH + NH);
  for (int i = 0; i < NPD * NH; i++) w[i] = bf16_bits(th[OW1 + i]);
  for (int i = 0; i < NH * NH; i++) w[NPD * NH + i] = bf16_bits(th[OW2 + i]);
  for (int i = 0; i < NH; i++) w[NPD * NH + NH * NH + i] = bf16_bits(th[OW3 + i]);
  std::vector<float> b(2 * NH + 1);
  for (int i = 0; i < NH; i++) {
    b[i] = th[OB1 + i];
    b[NH + i] = th[OB2 + i];
  }
  b[2 * NH] = th[OB3];
  if (hipMemcpyAsync(w_dev, w.data(), 2 * w.size(), hipMemcpyHostToDevice, s)) return MF_EHIP;
  if (hipMemcpyAsync(b_dev, b.data(), 4 * b.size(), hipMemcpyHostToDevice, s)) return MF_EHIP;
  if (hipStreamSynchronize(s)) return MF_EHIP;
  return MF_OK;
}

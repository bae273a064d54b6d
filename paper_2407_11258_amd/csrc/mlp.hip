// Learned T2 starting guess: features, network forward / backward and Adam.
// The three dense layers (and the weight gradients) are FP32 matrix-core
// products through gett(); everything else here is bandwidth-bound and
// elementwise, with fixed-grid FP64 partial sums so that losses and bias
// gradients are reproducible.
#include "mlp.h"

#include <algorithm>
#include <cmath>

#include "gett.h"

namespace lnocc {
namespace mlp {
namespace {

constexpr int kThreads = 256;
constexpr int kColBlocks = 128;    // row groups of the column sums
constexpr int kSumBlocks = 256;    // blocks of the vector sums
constexpr int kStatBlocks = 128;   // blocks of the feature statistics
constexpr int kStatCols = kFeat + 1;

inline int grid_for(int64_t n) {
  int64_t b = (n + kThreads - 1) / kThreads;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, 16384));
}

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

// splitmix64 output function (Steele, Lea and Flood, OOPSLA 2014).
__device__ inline uint64_t mix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__device__ inline float sigmoid(float z) { return 1.0f / (1.0f + expf(-z)); }
__device__ inline float silu(float z) { return z * sigmoid(z); }
__device__ inline float dsilu(float z) {
  const float s = sigmoid(z);
  return s * (1.0f + z * (1.0f - s));
}

__device__ inline double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
  return x;
}
__device__ inline float wave_sum_f(float x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
  return x;
}
// Sum over a 256-thread block; valid in thread 0.
__device__ inline double block_sum(double x, double *sm) {
  x = wave_sum(x);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sm[w] = x;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sm[i];
  return r;
}

__global__ void k_pair_stats(const double *__restrict__ Boo, const double *__restrict__ Bov,
                             const double *__restrict__ Bvv, int64_t X, int64_t o, int64_t v,
                             double *nrm, double *jd) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < o * v;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / v, a = e % v;
    double s2 = 0.0, sj = 0.0;
    for (int64_t Q = 0; Q < X; ++Q) {
      const double x = Bov[(Q * o + i) * v + a];
      s2 += x * x;
      sj += Boo[(Q * o + i) * o + i] * Bvv[(Q * v + a) * v + a];
    }
    nrm[e] = sqrt(s2);
    jd[e] = sj;
  }
}

__global__ void k_features(const double *__restrict__ Kov, const double *__restrict__ eo,
                           const double *__restrict__ ev, const double *__restrict__ nrm,
                           const double *__restrict__ jd, int64_t o, int64_t v,
                           const int64_t *__restrict__ idx, int64_t u0, int64_t n,
                           const double *__restrict__ t2, float *Xf, float *Yf) {
  const int64_t vv = v * v, total = o * o * vv;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x) {
    int64_t i, j, a, b;
    bool ok = true;
    if (idx) {
      const int64_t e = idx[r];
      ok = (e >= 0 && e < total);
      const int64_t ee = ok ? e : 0;
      b = ee % v;
      a = (ee / v) % v;
      j = (ee / vv) % o;
      i = ee / (vv * o);
    } else {
      const int64_t u = u0 + r, p = u / vv, ab = u % vv;
      a = ab / v;
      b = ab % v;
      int64_t jj = (int64_t)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
      while ((jj + 1) * (jj + 2) / 2 <= p) ++jj;
      while (jj > 0 && jj * (jj + 1) / 2 > p) --jj;
      j = jj;
      i = p - jj * (jj + 1) / 2;
      ok = (j < o);
      if (!ok) { i = j = 0; }
    }
    float f[kFeat];
    float y = 0.0f;
    if (ok) {
      const double Kd = Kov[((i * v + a) * o + j) * v + b];
      const double Kx = Kov[((i * v + b) * o + j) * v + a];
      const double D = eo[i] + eo[j] - ev[a] - ev[b];
      f[0] = (float)(Kd / D);
      f[1] = (float)(Kx / D);
      f[2] = (float)Kd;
      f[3] = (float)Kx;
      f[4] = (float)(1.0 / D);
      f[5] = (float)D;
      f[6] = (float)(eo[i] + eo[j]);
      f[7] = (float)fabs(eo[i] - eo[j]);
      f[8] = (float)(ev[a] + ev[b]);
      f[9] = (float)fabs(ev[a] - ev[b]);
      f[10] = (float)(nrm[i * v + a] * nrm[j * v + b]);
      f[11] = (float)(nrm[i * v + b] * nrm[j * v + a]);
      f[12] = (i == j) ? 1.0f : 0.0f;
      f[13] = (a == b) ? 1.0f : 0.0f;
      f[14] = (float)(jd[i * v + a] + jd[j * v + b]);
      f[15] = (float)(jd[i * v + b] + jd[j * v + a]);
      if (t2) y = (float)(t2[((i * o + j) * v + a) * v + b] - Kd / D);
    } else {   // an index outside the amplitude array: a row the caller can see is bad
#pragma unroll
      for (int q = 0; q < kFeat; ++q) f[q] = NAN;
      y = NAN;
    }
    float4 *dst = reinterpret_cast<float4 *>(Xf + r * kFeat);
#pragma unroll
    for (int q = 0; q < kFeat / 4; ++q) dst[q] = make_float4(f[4 * q], f[4 * q + 1], f[4 * q + 2], f[4 * q + 3]);
    if (Yf) Yf[r] = y;
  }
}

__global__ void k_normalize(const float *__restrict__ X, int64_t n, const float *__restrict__ hdr,
                            float *xn) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * kFeat;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int q = (int)(e % kFeat);
    xn[e] = (X[e] - hdr[q]) * hdr[kFeat + q];
  }
}

// h = silu(z + b); with keep, z is overwritten by the pre-activation z + b.
// h may alias z when keep is off.
__global__ void k_bias_act(float *z, int64_t n, const float *__restrict__ bias, float *h,
                           int keep) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * kHidden;
       e += (int64_t)gridDim.x * blockDim.x) {
    const float t = z[e] + bias[e % kHidden];
    if (keep) z[e] = t;
    h[e] = silu(t);
  }
}

// y[r] = w4 . h3[r] + b4: one wave per row, four hidden units per lane.
__global__ void k_out(const float *__restrict__ h3, int64_t n, const float *__restrict__ w4,
                      const float *__restrict__ b4, float *y) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  const float4 w = reinterpret_cast<const float4 *>(w4)[lane];
  for (int64_t r = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6); r < n; r += waves) {
    const float4 h = reinterpret_cast<const float4 *>(h3 + r * kHidden)[lane];
    float acc = h.x * w.x + h.y * w.y + h.z * w.z + h.w * w.w;
    acc = wave_sum_f(acc);
    if (lane == 0) y[r] = acc + b4[0];
  }
}

__global__ void k_affine(const float *__restrict__ y, int64_t n, const float *__restrict__ hdr,
                         float *out) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x)
    out[r] = hdr[2 * kFeat] + hdr[2 * kFeat + 1] * y[r];
}

// Unique amplitude u0 + r -> (i <= j, a, b); adds the correction at (i,j,a,b)
// and at (j,i,b,a).
__global__ void k_apply_guess(const float *__restrict__ y, const float *__restrict__ hdr,
                              int64_t o, int64_t v, int64_t u0, int64_t n, double *t2) {
  const int64_t vv = v * v;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t u = u0 + r, p = u / vv, ab = u % vv, a = ab / v, b = ab % v;
    int64_t j = (int64_t)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
    while ((j + 1) * (j + 2) / 2 <= p) ++j;
    while (j > 0 && j * (j + 1) / 2 > p) --j;
    const int64_t i = p - j * (j + 1) / 2;
    if (j >= o) continue;
    const double c = (double)hdr[2 * kFeat] + (double)hdr[2 * kFeat + 1] * (double)y[r];
    t2[((i * o + j) * v + a) * v + b] += c;
    if (i != j) t2[((j * o + i) * v + b) * v + a] += c;
  }
}

// r = y - (Y - y_mu) / y_sigma, dy = 2 r / n, partials of sum r^2 (fixed grid).
__global__ void k_mse(const float *__restrict__ y, const float *__restrict__ Y, int64_t n,
                      const float *__restrict__ hdr, float *dy, double *partials) {
  __shared__ double sm[kThreads / 64];
  const float ym = hdr[2 * kFeat], ys = hdr[2 * kFeat + 1];
  double acc = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const float r = y[e] - (Y[e] - ym) / ys;
    dy[e] = 2.0f * r / (float)n;
    acc += (double)r * r;
  }
  const double s = block_sum(acc, sm);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// out[0] = scale * sum of partials[0..m) in order (one block).
__global__ void k_sum_finish(const double *__restrict__ partials, int m, double scale,
                             double *out_d, float *out_f) {
  __shared__ double sm[kThreads / 64];
  double acc = 0.0;
  for (int e = threadIdx.x; e < m; e += blockDim.x) acc += partials[e];
  const double s = block_sum(acc, sm);
  if (threadIdx.x == 0) {
    if (out_d) out_d[0] = scale * s;
    if (out_f) out_f[0] = (float)(scale * s);
  }
}

__global__ void k_vec_partials(const float *__restrict__ x, int64_t n, double *partials) {
  __shared__ double sm[kThreads / 64];
  double acc = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    acc += x[e];
  const double s = block_sum(acc, sm);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// partials[g][k] = sum over rows r = g, g + G, ... of A[r][k] (* w[r]).
__global__ void k_colsum(const float *__restrict__ A, const float *__restrict__ w, int64_t n,
                         double *partials) {
  const int k = threadIdx.x;
  double acc = 0.0;
  for (int64_t r = blockIdx.x; r < n; r += gridDim.x)
    acc += (double)A[r * kHidden + k] * (w ? (double)w[r] : 1.0);
  partials[(int64_t)blockIdx.x * kHidden + k] = acc;
}
__global__ void k_colsum_finish(const double *__restrict__ partials, int G, float *out) {
  const int k = threadIdx.x;
  double acc = 0.0;
  for (int g = 0; g < G; ++g) acc += partials[(int64_t)g * kHidden + k];
  out[k] = (float)acc;
}

// dz3[r][k] = dy[r] w4[k] silu'(z3[r][k])
__global__ void k_out_back(const float *__restrict__ dy, const float *__restrict__ w4,
                           const float *__restrict__ z3, int64_t n, float *dz3) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * kHidden;
       e += (int64_t)gridDim.x * blockDim.x)
    dz3[e] = dy[e / kHidden] * w4[e % kHidden] * dsilu(z3[e]);
}

// dz = dh silu'(z) (dz may alias dh)
__global__ void k_act_back(const float *dh, const float *__restrict__ z, int64_t n, float *dz) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * kHidden;
       e += (int64_t)gridDim.x * blockDim.x)
    dz[e] = dh[e] * dsilu(z[e]);
}

__global__ void k_fill(float *x, int64_t n, float val) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    x[e] = val;
}

// Adam (Kingma and Ba 2015): beta1 0.9, beta2 0.999, eps 1e-8; bc1 = 1 - beta1^t,
// bc2 = 1 - beta2^t.
__global__ void k_adam(float *p, const float *__restrict__ g, float *m1, float *m2, int64_t n,
                       float lr, float bc1, float bc2) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[e];
    const float a = 0.9f * m1[e] + 0.1f * gi;
    const float b = 0.999f * m2[e] + 0.001f * gi * gi;
    m1[e] = a;
    m2[e] = b;
    p[e] -= lr * (a / bc1) / (sqrtf(b / bc2) + 1e-8f);
  }
}

// Minibatch row k of step t: row index mix64(seed ^ mix64(t << 32 | k)) mod n.
__global__ void k_gather(const float *__restrict__ X, const float *__restrict__ Y, int64_t n,
                         uint64_t seed, uint64_t step, int batch, float *xb, float *yb) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < batch;
       k += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t h = mix64(seed ^ mix64((step << 32) | (uint64_t)k));
    const int64_t r = (int64_t)(h % (uint64_t)n);
    const float4 *src = reinterpret_cast<const float4 *>(X + r * kFeat);
    float4 *dst = reinterpret_cast<float4 *>(xb + k * kFeat);
#pragma unroll
    for (int q = 0; q < kFeat / 4; ++q) dst[q] = src[q];
    yb[k] = Y[r];
  }
}

// partials[b][c], c < 17: sums of column c of [X | Y]; [b][17 + c]: sums of squares.
__global__ void k_stats(const float *__restrict__ X, const float *__restrict__ Y, int64_t n,
                        double *partials) {
  __shared__ double sm[kThreads / 64];
  double s[kStatCols], q[kStatCols];
#pragma unroll
  for (int c = 0; c < kStatCols; ++c) s[c] = q[c] = 0.0;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int c = 0; c < kStatCols; ++c) {
      const double x = (c < kFeat) ? X[r * kFeat + c] : Y[r];
      s[c] += x;
      q[c] += x * x;
    }
  }
  for (int c = 0; c < kStatCols; ++c) {
    const double a = block_sum(s[c], sm);
    if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * 2 * kStatCols + c] = a;
    const double b = block_sum(q[c], sm);
    if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * 2 * kStatCols + kStatCols + c] = b;
  }
}

// header: mu, inv_sigma of each feature (0 for a constant feature), y_mu, y_sigma.
__global__ void k_stats_finish(const double *__restrict__ partials, int G, int64_t n, float *hdr) {
  const int c = threadIdx.x;
  if (c < kStatCols) {
    double s = 0.0, q = 0.0;
    for (int g = 0; g < G; ++g) {
      s += partials[(int64_t)g * 2 * kStatCols + c];
      q += partials[(int64_t)g * 2 * kStatCols + kStatCols + c];
    }
    const double mu = s / (double)n;
    const double var = fmax(q / (double)n - mu * mu, 0.0);
    const double sd = sqrt(var);
    if (c < kFeat) {
      hdr[c] = (float)mu;
      hdr[kFeat + c] = sd > 1e-30 ? (float)(1.0 / sd) : 0.0f;
    } else {
      hdr[2 * kFeat] = (float)mu;
      hdr[2 * kFeat + 1] = sd > 1e-30 ? (float)sd : 1.0f;
    }
  }
  for (int e = 2 * kFeat + 2 + threadIdx.x; e < kHeader; e += blockDim.x) hdr[e] = 0.0f;
}

// Weights uniform in [-a, a] with a = sqrt(6 / (fan_in + fan_out)) (the output
// layer scaled by 0.1 so the first prediction is near the mean correction);
// biases and padding zero.
__global__ void k_init_weights(float *P, uint64_t seed) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < kParams;
       e += (int64_t)gridDim.x * blockDim.x) {
    double lim = 0.0;
    if (e < kB1) lim = sqrt(6.0 / (kFeat + kHidden));
    else if (e >= kW2 && e < kB2) lim = sqrt(6.0 / (2 * kHidden));
    else if (e >= kW3 && e < kB3) lim = sqrt(6.0 / (2 * kHidden));
    else if (e >= kW4 && e < kB4) lim = 0.1 * sqrt(6.0 / (kHidden + 1));
    const double u = (double)(mix64(seed ^ mix64((uint64_t)e)) >> 11) * (1.0 / 9007199254740992.0);
    P[e] = (float)(lim * (2.0 * u - 1.0));
  }
}

// ---------------------------------------------------------------- products
GemmDesc base_desc() {
  GemmDesc d{};
  d.Mi = d.Ni = 1;
  d.nseg = 1;
  d.seg[0].Ki = 1;
  d.seg[0].scale = 1.0;
  d.batch = 1;
  d.nb1 = 1;
  d.prec = Prec::F32;
  d.c_type = 1;
  d.kind = Kind::Mlp;
  return d;
}

// C[r][h] = sum_k A[r][k] W[h][k]   (rows n, h < 256)
hipError_t gemm_rows(const float *A, int K, const float *W, int64_t n, float *C, hipStream_t s) {
  GemmDesc d = base_desc();
  d.M = (int)n;
  d.N = kHidden;
  d.seg[0].K = K;
  d.seg[0].a = GOperand{A, K, 0, 1, 0, 0, 0, 0, 0};
  d.seg[0].b = GOperand{W, K, 0, 1, 0, 0, 0, 0, 0};
  d.c = C;
  d.c_mo = kHidden;
  d.c_no = 1;
  return gett(d, s);
}

// G[h][k] = sum_r dZ[r][h] H[r][k]   (h < 256, k < K, rows n)
hipError_t gemm_wgrad(const float *dZ, const float *H, int K, int64_t n, float *G, hipStream_t s) {
  GemmDesc d = base_desc();
  d.M = kHidden;
  d.N = K;
  d.seg[0].K = (int)n;
  d.seg[0].a = GOperand{dZ, 1, 0, kHidden, 0, 0, 0, 0, 0};
  d.seg[0].b = GOperand{H, 1, 0, K, 0, 0, 0, 0, 0};
  d.c = G;
  d.c_mo = K;
  d.c_no = 1;
  return gett(d, s);
}

// dH[r][k] = sum_h dZ[r][h] W[h][k]   (rows n, k < 256)
hipError_t gemm_dgrad(const float *dZ, const float *W, int64_t n, float *dH, hipStream_t s) {
  GemmDesc d = base_desc();
  d.M = (int)n;
  d.N = kHidden;
  d.seg[0].K = kHidden;
  d.seg[0].a = GOperand{dZ, kHidden, 0, 1, 0, 0, 0, 0, 0};
  d.seg[0].b = GOperand{W, 1, 0, kHidden, 0, 0, 0, 0, 0};
  d.c = dH;
  d.c_mo = kHidden;
  d.c_no = 1;
  return gett(d, s);
}

hipError_t colsum(const float *A, const float *w, int64_t n, const Scratch &S, float *out,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_colsum, dim3(kColBlocks), dim3(kHidden), 0, s, A, w, n, S.partials);
  hipLaunchKernelGGL(k_colsum_finish, dim3(1), dim3(kHidden), 0, s, S.partials, kColBlocks, out);
  return hipGetLastError();
}

#define MLP_TRY(x)                        \
  do {                                    \
    const hipError_t e_ = (x);            \
    if (e_ != hipSuccess) return e_;      \
  } while (0)

}  // namespace

void plan_scratch(int64_t rows, bool training, char *base, Scratch &S) {
  S = Scratch{};
  S.rows = rows;
  S.training = training;
  size_t off = 0;
  auto take = [&](size_t bytes) -> char * {
    char *p = base ? base + off : nullptr;
    off += align256(bytes);
    return p;
  };
  const size_t R = (size_t)rows, fb = sizeof(float), hb = R * kHidden * fb;
  S.xn = (float *)take(R * kFeat * fb);
  S.h1 = (float *)take(hb);
  S.h2 = (float *)take(hb);
  S.y = (float *)take(R * fb);
  if (training) {
    S.z1 = (float *)take(hb);
    S.z2 = (float *)take(hb);
    S.z3 = (float *)take(hb);
    S.h3 = (float *)take(hb);
    S.dza = (float *)take(hb);
    S.dzb = (float *)take(hb);
    S.dy = (float *)take(R * fb);
    S.xb = (float *)take(R * kFeat * fb);
    S.yb = (float *)take(R * fb);
    S.grad = (float *)take(kParams * fb);
    S.splitk_elems = (int64_t)64 * kHidden * kHidden;
    S.splitk = (double *)take((size_t)S.splitk_elems * sizeof(double));
    S.losses = (double *)take(kLossChunk * sizeof(double));
  }
  const size_t np = std::max<size_t>({(size_t)kColBlocks * kHidden, (size_t)kSumBlocks,
                                      (size_t)kStatBlocks * 2 * kStatCols});
  S.partials = (double *)take(np * sizeof(double));
  S.loss = (double *)take(sizeof(double));
  S.bytes = off;
}

hipError_t pair_stats(const double *Boo, const double *Bov, const double *Bvv, int64_t X,
                      int64_t o, int64_t v, double *nrm, double *jd, hipStream_t s) {
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(k_pair_stats, dim3(grid_for(o * v)), dim3(kThreads), 0, s, Boo, Bov, Bvv, X,
                     o, v, nrm, jd);
  return hipGetLastError();
}

hipError_t features(const double *Kov, const double *eo, const double *ev, const double *nrm,
                    const double *jd, int64_t o, int64_t v, const int64_t *idx, int64_t u0,
                    int64_t n, const double *t2, float *Xf, float *Yf, hipStream_t s) {
  if (dry_run() || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_features, dim3(grid_for(n)), dim3(kThreads), 0, s, Kov, eo, ev, nrm, jd, o,
                     v, idx, u0, n, t2, Xf, Yf);
  return hipGetLastError();
}

hipError_t forward(const float *blob, const float *X, int64_t n, const Scratch &S, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (n > S.rows) return hipErrorInvalidValue;
  const float *P = blob + kHeader;
  const bool tr = S.training;
  float *z1 = tr ? S.z1 : S.h1, *z2 = tr ? S.z2 : S.h2, *z3 = tr ? S.z3 : S.h1;
  float *h3 = tr ? S.h3 : S.h1;
  if (!dry_run()) {
    hipLaunchKernelGGL(k_normalize, dim3(grid_for(n * kFeat)), dim3(kThreads), 0, s, X, n, blob,
                       S.xn);
    MLP_TRY(hipGetLastError());
  }
  MLP_TRY(gemm_rows(S.xn, kFeat, P + kW1, n, z1, s));
  if (!dry_run()) {
    hipLaunchKernelGGL(k_bias_act, dim3(grid_for(n * kHidden)), dim3(kThreads), 0, s, z1, n,
                       P + kB1, S.h1, (int)tr);
    MLP_TRY(hipGetLastError());
  }
  MLP_TRY(gemm_rows(S.h1, kHidden, P + kW2, n, z2, s));
  if (!dry_run()) {
    hipLaunchKernelGGL(k_bias_act, dim3(grid_for(n * kHidden)), dim3(kThreads), 0, s, z2, n,
                       P + kB2, S.h2, (int)tr);
    MLP_TRY(hipGetLastError());
  }
  MLP_TRY(gemm_rows(S.h2, kHidden, P + kW3, n, z3, s));
  if (!dry_run()) {
    hipLaunchKernelGGL(k_bias_act, dim3(grid_for(n * kHidden)), dim3(kThreads), 0, s, z3, n,
                       P + kB3, h3, (int)tr);
    const int64_t wb = std::min<int64_t>((n + 3) / 4, 16384);
    hipLaunchKernelGGL(k_out, dim3((unsigned)wb), dim3(kThreads), 0, s, h3, n, P + kW4, P + kB4,
                       S.y);
    MLP_TRY(hipGetLastError());
  }
  return hipSuccess;
}

hipError_t apply_guess(const float *blob, const float *y, int64_t o, int64_t v, int64_t u0,
                       int64_t n, double *t2, hipStream_t s) {
  if (dry_run() || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_apply_guess, dim3(grid_for(n)), dim3(kThreads), 0, s, y, blob, o, v, u0, n,
                     t2);
  return hipGetLastError();
}

hipError_t predict(const float *blob, const float *X, int64_t n, float *out, const Scratch &S,
                   hipStream_t s) {
  for (int64_t off = 0; off < n; off += S.rows) {
    const int64_t m = std::min<int64_t>(S.rows, n - off);
    MLP_TRY(forward(blob, X + off * kFeat, m, S, s));
    if (!dry_run()) {
      hipLaunchKernelGGL(k_affine, dim3(grid_for(m)), dim3(kThreads), 0, s, S.y, m, blob, out + off);
      MLP_TRY(hipGetLastError());
    }
  }
  return hipSuccess;
}

hipError_t loss_grad(const float *blob, const float *X, const float *Y, int64_t n,
                     const Scratch &S, hipStream_t s) {
  if (!S.training || n <= 0 || n > S.rows) return hipErrorInvalidValue;
  install_splitk_scratch(S.splitk, (size_t)S.splitk_elems);
  const float *P = blob + kHeader;
  float *G = S.grad;
  MLP_TRY(forward(blob, X, n, S, s));
  const bool dry = dry_run();
  if (!dry) {
    hipLaunchKernelGGL(k_mse, dim3(kSumBlocks), dim3(kThreads), 0, s, S.y, Y, n, blob, S.dy,
                       S.partials);
    hipLaunchKernelGGL(k_sum_finish, dim3(1), dim3(kThreads), 0, s, S.partials, kSumBlocks,
                       1.0 / (double)n, S.loss, (float *)nullptr);
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, s, G + kB4 + 1, kParams - kB4 - 1, 0.0f);
    MLP_TRY(hipGetLastError());
    MLP_TRY(colsum(S.h3, S.dy, n, S, G + kW4, s));
    hipLaunchKernelGGL(k_vec_partials, dim3(kSumBlocks), dim3(kThreads), 0, s, S.dy, n, S.partials);
    hipLaunchKernelGGL(k_sum_finish, dim3(1), dim3(kThreads), 0, s, S.partials, kSumBlocks, 1.0,
                       (double *)nullptr, G + kB4);
    hipLaunchKernelGGL(k_out_back, dim3(grid_for(n * kHidden)), dim3(kThreads), 0, s, S.dy,
                       P + kW4, S.z3, n, S.dza);
    MLP_TRY(hipGetLastError());
  }
  MLP_TRY(gemm_wgrad(S.dza, S.h2, kHidden, n, G + kW3, s));
  if (!dry) MLP_TRY(colsum(S.dza, nullptr, n, S, G + kB3, s));
  MLP_TRY(gemm_dgrad(S.dza, P + kW3, n, S.dzb, s));
  if (!dry) {
    hipLaunchKernelGGL(k_act_back, dim3(grid_for(n * kHidden)), dim3(kThreads), 0, s, S.dzb, S.z2,
                       n, S.dzb);
    MLP_TRY(hipGetLastError());
  }
  MLP_TRY(gemm_wgrad(S.dzb, S.h1, kHidden, n, G + kW2, s));
  if (!dry) MLP_TRY(colsum(S.dzb, nullptr, n, S, G + kB2, s));
  MLP_TRY(gemm_dgrad(S.dzb, P + kW2, n, S.dza, s));
  if (!dry) {
    hipLaunchKernelGGL(k_act_back, dim3(grid_for(n * kHidden)), dim3(kThreads), 0, s, S.dza, S.z1,
                       n, S.dza);
    MLP_TRY(hipGetLastError());
  }
  MLP_TRY(gemm_wgrad(S.dza, S.xn, kFeat, n, G + kW1, s));
  if (!dry) MLP_TRY(colsum(S.dza, nullptr, n, S, G + kB1, s));
  return hipSuccess;
}

hipError_t init(float *blob, const float *X, const float *Y, int64_t n, uint64_t seed,
                const Scratch &S, hipStream_t s) {
  if (n <= 0) return hipErrorInvalidValue;
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(k_stats, dim3(kStatBlocks), dim3(kThreads), 0, s, X, Y, n, S.partials);
  hipLaunchKernelGGL(k_stats_finish, dim3(1), dim3(64), 0, s, S.partials, kStatBlocks, n, blob);
  hipLaunchKernelGGL(k_init_weights, dim3(grid_for(kParams)), dim3(kThreads), 0, s,
                     blob + kHeader, seed);
  return hipGetLastError();
}

hipError_t train(float *blob, float *adam, int64_t step0, int nsteps, const float *X,
                 const float *Y, int64_t n, int batch, float lr, uint64_t seed, double *losses,
                 const Scratch &S, hipStream_t s) {
  if (!S.training || batch <= 0 || batch > S.rows || n <= 0 || (losses && nsteps > kLossChunk))
    return hipErrorInvalidValue;
  for (int k = 0; k < nsteps; ++k) {
    const int64_t t = step0 + k + 1;
    if (!dry_run()) {
      hipLaunchKernelGGL(k_gather, dim3(grid_for(batch)), dim3(kThreads), 0, s, X, Y, n, seed,
                         (uint64_t)t, batch, S.xb, S.yb);
      MLP_TRY(hipGetLastError());
    }
    MLP_TRY(loss_grad(blob, S.xb, S.yb, batch, S, s));
    if (dry_run()) continue;
    if (losses)
      MLP_TRY(hipMemcpyAsync(losses + k, S.loss, sizeof(double), hipMemcpyDeviceToDevice, s));
    const float bc1 = (float)(1.0 - std::pow(0.9, (double)t));
    const float bc2 = (float)(1.0 - std::pow(0.999, (double)t));
    hipLaunchKernelGGL(k_adam, dim3(grid_for(kParams)), dim3(kThreads), 0, s, blob + kHeader, S.grad,
                       adam, adam + kParams, kParams, lr, bc1, bc2);
    MLP_TRY(hipGetLastError());
  }
  return hipSuccess;
}

}  // namespace mlp
}  // namespace lnocc

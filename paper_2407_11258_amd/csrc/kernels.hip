// Bandwidth-bound kernels of the fragment solver.  Every reduction writes one
// partial per block of a fixed-size grid and is finished by a single block in
// a fixed order, so FP64 energies and norms are bitwise reproducible.
#include "kernels.h"
#include "gett.h"

namespace lnocc {
namespace {

constexpr int kEwThreads = 256;

inline int ew_blocks(int64_t n) {
  int64_t b = (n + kEwThreads - 1) / kEwThreads;
  if (b > 16384) b = 16384;
  if (b < 1) b = 1;
  return (int)b;
}

// (i, j, a, b) of the flat index e = ((i o + j) v + a) v + b.  Unsigned 32-bit
// division (a few instructions) whenever o^2 v^2 fits, else 64-bit.
__device__ inline void split4(int64_t e, int64_t o, int64_t v, int64_t &i, int64_t &j, int64_t &a,
                              int64_t &b) {
  if (o * o * v * v <= (int64_t)0xffffffffLL) {
    const uint32_t ue = (uint32_t)e, uo = (uint32_t)o, uv = (uint32_t)v, uvv = uv * uv;
    const uint32_t ij = ue / uvv, ab = ue - ij * uvv, ui = ij / uo, ua = ab / uv;
    i = ui; j = ij - ui * uo; a = ua; b = ab - ua * uv;
  } else {
    const int64_t vv = v * v, ij = e / vv, ab = e % vv;
    i = ij / o; j = ij % o; a = ab / v; b = ab % v;
  }
}

__device__ inline double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
  return x;
}

// Sum over the block; the result is valid in thread 0.
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

__global__ void k_split_B(const double *__restrict__ B, int64_t X, int64_t o, int64_t v,
                          double *Boo, double *Bov, double *Bvv) {
  const int64_t n = o + v, total = X * n * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t Q = e / (n * n), pq = e % (n * n), p = pq / n, q = pq % n;
    const double x = B[e];
    if (p < o && q < o) Boo[(Q * o + p) * o + q] = x;
    else if (p < o) Bov[(Q * o + p) * v + (q - o)] = x;
    else if (q >= o) Bvv[(Q * v + (p - o)) * v + (q - o)] = x;
  }
}

__global__ void k_diag_sum(const double *__restrict__ Boo, int64_t X, int64_t o, double *J) {
  for (int64_t Q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; Q < X;
       Q += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int64_t k = 0; k < o; ++k) s += Boo[(Q * o + k) * o + k];
    J[Q] = s;
  }
}

__global__ void k_add_diag(double *M, int64_t n, int64_t ld, const double *eps) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * blockDim.x)
    M[p * ld + p] += eps[p];
}

__global__ void k_transpose2d(const double *__restrict__ in, int64_t rows, int64_t cols,
                              double *out) {
  const int64_t total = rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / cols, c = e % cols;
    out[c * rows + r] = in[e];
  }
}

// u[i][j][a][b] = 2 t2[i][j][a][b] - t2[j][i][a][b]
__global__ void k_make_u(const double *__restrict__ t2, int64_t o, int64_t v, double *u) {
  const int64_t vv = v * v, total = o * o * vv;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t i, j, a, b;
    split4(e, o, v, i, j, a, b);
    u[e] = 2.0 * t2[e] - t2[(j * o + i) * vv + a * v + b];
  }
}

// t2[i][j][a][b] = (ia|jb) / (e_i + e_j - e_a - e_b), t1 = 0
__global__ void k_mp2_guess(const double *__restrict__ Kov, const double *eo, const double *ev,
                            int64_t o, int64_t v, double *t1, double *t2) {
  const int64_t vv = v * v, total = o * o * vv;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ij = e / vv, ab = e % vv, i = ij / o, j = ij % o, a = ab / v, b = ab % v;
    t2[e] = Kov[((i * v + a) * o + j) * v + b] / (eo[i] + eo[j] - ev[a] - ev[b]);
    if (e < o * v) t1[e] = 0.0;
  }
}

// Lov[l][d][k][c] = 2 (ld|kc) - (lc|kd), Kov[k][c][l][d] = (kc|ld)
__global__ void k_build_lov(const double *__restrict__ Kov, int64_t o, int64_t v, double *Lov) {
  const int64_t total = o * v * o * v;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e % v, k = (e / v) % o, d = (e / (v * o)) % v, l = e / (v * o * v);
    Lov[e] = 2.0 * Kov[e] - Kov[((l * v + c) * o + k) * v + d];
  }
}

// Dint[i][a][k][c] -= Goovv[k][i][a][c]
__global__ void k_sub_oovv(const double *__restrict__ G, int64_t o, int64_t v, double *Dint) {
  const int64_t total = o * v * o * v;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e % v, k = (e / v) % o, a = (e / (v * o)) % v, i = e / (v * o * v);
    Dint[e] -= G[((k * o + i) * v + a) * v + c];
  }
}

// R2 += S + S^P - 1/2 (X + X^P) - (Xs + Xs^P), with Y^P[i][j][a][b] = Y[j][i][b][a]
// and Xs[i][j][a][b] = X[j][i][a][b].  One block per (i, j) pair and 32 x 32 tile
// of (a, b): the three operands read with a and b exchanged (S[j][i], X[j][i] and
// X[i][j] at (b, a)) are staged through LDS so that every global access runs
// along the contiguous index.
constexpr int kCT = 32;
// R2[i][j][a][b] and R2[j][i][b][a] <- their mean.  A block takes one pair i <= j
// and one (a0, b0) tile with its mirror tile (b0, a0) of the partner pair, so every
// element and its mirror are read and written by the same block (for i = j only
// the tiles with a0 <= b0, a diagonal tile being its own mirror).
__global__ void k_pair_symmetrize(double *R2, int64_t o, int64_t v) {
  __shared__ double P[kCT][kCT + 1], Q[kCT][kCT + 1];   // [r][c]: (a0 + r, b0 + c) / (b0 + r, a0 + c)
  const int64_t vv = v * v;
  const int tiles = (int)((v + kCT - 1) / kCT);
  const int ta = blockIdx.x / tiles, tb = blockIdx.x % tiles;
  const int64_t a0 = (int64_t)ta * kCT, b0 = (int64_t)tb * kCT;
  const int64_t npairs = o * (o + 1) / 2;
  for (int64_t p = blockIdx.y; p < npairs; p += gridDim.y) {
    // p -> (i, j), i <= j, rows of the upper triangle in order
    int64_t i = 0, rem = p;
    while (rem >= o - i) { rem -= o - i; ++i; }
    const int64_t j = i + rem;
    if (i == j && ta > tb) continue;          // uniform over the block
    double *X = R2 + (i * o + j) * vv, *Y = R2 + (j * o + i) * vv;
    __syncthreads();
    for (int e = threadIdx.x; e < kCT * kCT; e += blockDim.x) {
      const int r = e / kCT, c = e % kCT;
      const int64_t a = a0 + r, b = b0 + c, b2 = b0 + r, a2 = a0 + c;
      P[r][c] = (a < v && b < v) ? X[a * v + b] : 0.0;
      Q[r][c] = (b2 < v && a2 < v) ? Y[b2 * v + a2] : 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kCT * kCT; e += blockDim.x) {
      const int r = e / kCT, c = e % kCT;
      const int64_t a = a0 + r, b = b0 + c, b2 = b0 + r, a2 = a0 + c;
      // X(a, b) pairs with Y(b, a) = Q[c][r]; Y(b2, a2) pairs with X(a2, b2) = P[c][r]
      if (a < v && b < v) X[a * v + b] = 0.5 * (P[r][c] + Q[c][r]);
      if (b2 < v && a2 < v) Y[b2 * v + a2] = 0.5 * (Q[r][c] + P[c][r]);
    }
  }
}

__global__ void k_combine_r2(double *R2, const double *__restrict__ S, const double *__restrict__ Xc,
                             int64_t o, int64_t v) {
  __shared__ double T[3][kCT][kCT + 1];   // [b - b0][a - a0] of S[j][i], X[j][i], X[i][j]
  const int64_t vv = v * v;
  const int tiles = (int)((v + kCT - 1) / kCT);
  const int64_t a0 = (int64_t)(blockIdx.x / tiles) * kCT, b0 = (int64_t)(blockIdx.x % tiles) * kCT;
  for (int64_t ij = blockIdx.y; ij < o * o; ij += gridDim.y) {
    const int64_t i = ij / o, j = ij % o;
    const double *Sji = S + (j * o + i) * vv, *Xji = Xc + (j * o + i) * vv, *Xij = Xc + ij * vv;
    __syncthreads();   // the previous pair's reads of T are done
    for (int e = threadIdx.x; e < kCT * kCT; e += blockDim.x) {
      const int r = e / kCT, c = e % kCT;              // row b0 + r, column a0 + c
      const int64_t b = b0 + r, a = a0 + c;
      const bool in = a < v && b < v;
      const int64_t off = b * v + a;
      T[0][r][c] = in ? Sji[off] : 0.0;
      T[1][r][c] = in ? Xji[off] : 0.0;
      T[2][r][c] = in ? Xij[off] : 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kCT * kCT; e += blockDim.x) {
      const int ra = e / kCT, cb = e % kCT;            // output (a0 + ra, b0 + cb)
      const int64_t a = a0 + ra, b = b0 + cb;
      if (a >= v || b >= v) continue;
      const int64_t idx = ij * vv + a * v + b;
      R2[idx] += S[idx] + T[0][cb][ra] - 0.5 * (Xc[idx] + T[1][cb][ra]) -
                 (Xji[a * v + b] + T[2][cb][ra]);
    }
  }
}

__global__ void k_energy_partials(const double *__restrict__ Kov, const double *__restrict__ t1,
                                  const double *__restrict__ t2, int64_t o, int64_t v,
                                  double *partials) {
  __shared__ double sm[kRedThreads / 64];
  const int64_t vv = v * v, total = o * o * vv;
  double acc = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t i, j, a, b;
    split4(e, o, v, i, j, a, b);
    const double tau = t2[e] + t1[i * v + a] * t1[j * v + b];
    const double L = 2.0 * Kov[((i * v + a) * o + j) * v + b] - Kov[((i * v + b) * o + j) * v + a];
    acc += L * tau;
  }
  const double r = block_sum(acc, sm);
  if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

__global__ void k_reduce(const double *__restrict__ partials, int64_t n, double *out,
                         int accumulate) {
  __shared__ double sm[kRedThreads / 64];
  double acc = 0.0;
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) acc += partials[e];
  const double r = block_sum(acc, sm);
  if (threadIdx.x == 0) out[0] = accumulate ? out[0] + r : r;
}

// x = t + R / (D - shift) (Jacobi step with a level shift; D < 0), e = x - t,
// and partials of sum (R / D)^2, the squared norm of the unshifted step.
__global__ void k_jacobi(const double *__restrict__ t1, const double *__restrict__ t2,
                         const double *__restrict__ R1, const double *__restrict__ R2,
                         const double *eo, const double *ev, int64_t o, int64_t v, double shift,
                         double *x, double *err, double *partials) {
  __shared__ double sm[kRedThreads / 64];
  const int64_t n1 = o * v, vv = v * v, total = n1 + o * o * vv;
  double acc = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    double told, r, d;
    if (e < n1) {
      const int64_t i = e / v, a = e % v;
      told = t1[e];
      r = R1[e];
      d = eo[i] - ev[a];
    } else {
      const int64_t f = e - n1;
      int64_t i, j, a, b;
      split4(f, o, v, i, j, a, b);
      told = t2[f];
      r = R2[f];
      d = eo[i] + eo[j] - ev[a] - ev[b];
    }
    const double u = r / d;
    const double xn = told + (shift == 0.0 ? u : r / (d - shift));
    x[e] = xn;
    err[e] = xn - told;
    acc += u * u;
  }
  const double rr = block_sum(acc, sm);
  if (threadIdx.x == 0) partials[blockIdx.x] = rr;
}

constexpr int kMaxDiis = 16;

__global__ void k_dot_partials(const double *__restrict__ E, int64_t stride, int m,
                               const double *__restrict__ enew, int64_t N, double *partials) {
  __shared__ double sm[kRedThreads / 64];
  double acc[kMaxDiis];
#pragma unroll
  for (int i = 0; i < kMaxDiis; ++i) acc[i] = 0.0;
  // four grid strides per pass, so that 4 (m + 1) loads are in flight; each
  // thread still adds its elements in increasing order
  const int64_t G = (int64_t)gridDim.x * blockDim.x;
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (; e + 3 * G < N; e += 4 * G) {
    double x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) x[u] = enew[e + u * G];
#pragma unroll
    for (int i = 0; i < kMaxDiis; ++i)
      if (i < m) {
        double y[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) y[u] = E[i * stride + e + u * G];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[i] += x[u] * y[u];
      }
  }
  for (; e < N; e += G) {
    const double x = enew[e];
#pragma unroll
    for (int i = 0; i < kMaxDiis; ++i)
      if (i < m) acc[i] += x * E[i * stride + e];
  }
#pragma unroll
  for (int i = 0; i < kMaxDiis; ++i) {
    if (i < m) {   // m is uniform over the block
      const double r = block_sum(acc[i], sm);
      if (threadIdx.x == 0) partials[i * kRedBlocks + blockIdx.x] = r;
    }
  }
}

__global__ void k_reduce_rows(const double *__restrict__ partials, double *out) {
  __shared__ double sm[kRedThreads / 64];
  double acc = 0.0;
  for (int e = threadIdx.x; e < kRedBlocks; e += blockDim.x)
    acc += partials[blockIdx.x * kRedBlocks + e];
  const double r = block_sum(acc, sm);
  if (threadIdx.x == 0) out[blockIdx.x] = r;
}

struct Coeffs { double c[kMaxDiis]; };

__global__ void k_lincomb(const double *__restrict__ Xs, int64_t stride, int m, Coeffs cf,
                          int64_t o, int64_t v, double *t1, double *t2) {
  const int64_t n1 = o * v, total = n1 + o * o * v * v;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < m; ++i) s += cf.c[i] * Xs[i * stride + e];
    if (e < n1) t1[e] = s;
    else t2[e - n1] = s;
  }
}

// T1 dressing of the virtual-virtual DF block: Bt[Q][a][b] = B[Q][a][b] -
// sum_k t1[k][a] Bov[Q][k][b].  A block takes kDressRows rows a of one Q, with
// their t1 columns in LDS; a thread owns columns b and subtracts the o terms in
// order of k (each Bov element is loaded once per block and used for every row).
constexpr int kDressRows = 16;
__global__ __launch_bounds__(kEwThreads) void k_dress_vv(const double *__restrict__ Bvv,
                                                         const double *__restrict__ Bov,
                                                         const double *__restrict__ t1, int64_t o,
                                                         int64_t v, double *__restrict__ Bt) {
  extern __shared__ double tcol[];   // [k][r]
  const int64_t Q = blockIdx.y, a0 = (int64_t)blockIdx.x * kDressRows;
  const int nr = (int)min<int64_t>(kDressRows, v - a0);
  for (int64_t e = threadIdx.x; e < o * kDressRows; e += blockDim.x) {
    const int64_t k = e / kDressRows, r = e % kDressRows;
    tcol[e] = r < nr ? t1[k * v + a0 + r] : 0.0;
  }
  __syncthreads();
  const double *B = Bvv + (Q * v + a0) * v, *Bk = Bov + Q * o * v;
  double *out = Bt + (Q * v + a0) * v;
  for (int64_t b = threadIdx.x; b < v; b += blockDim.x) {
    double acc[kDressRows];
#pragma unroll
    for (int r = 0; r < kDressRows; ++r) acc[r] = r < nr ? B[r * v + b] : 0.0;
    // the Bov loads of eight k are issued together (independent of the FMAs)
    int64_t k = 0;
    for (; k + 8 <= o; k += 8) {
      double x[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) x[q] = Bk[(k + q) * v + b];
#pragma unroll
      for (int q = 0; q < 8; ++q)
#pragma unroll
        for (int r = 0; r < kDressRows; ++r)
          acc[r] = fma(-tcol[(k + q) * kDressRows + r], x[q], acc[r]);
    }
    for (; k < o; ++k) {
      const double x = Bk[k * v + b];
#pragma unroll
      for (int r = 0; r < kDressRows; ++r) acc[r] = fma(-tcol[k * kDressRows + r], x, acc[r]);
    }
#pragma unroll
    for (int r = 0; r < kDressRows; ++r)
      if (r < nr) out[r * v + b] = acc[r];
  }
}

__global__ void k_scatter(const double *__restrict__ x, int64_t o, int64_t v, double *t1,
                          double *t2) {
  const int64_t n1 = o * v, total = n1 + o * o * v * v;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (e < n1) t1[e] = x[e];
    else t2[e - n1] = x[e];
  }
}

// ---- packed particle-particle ladder --------------------------------------
// Pairs: tri(h, l) = h (h + 1) / 2 + l for l <= h; stri(h, l) = h (h - 1) / 2 + l for l < h.
__device__ inline int64_t tri(int64_t h, int64_t l) { return h * (h + 1) / 2 + l; }
__device__ inline int64_t stri(int64_t h, int64_t l) { return h * (h - 1) / 2 + l; }

// Rows of the ladder contraction: Tsa[tri(j,i)][c][d] = t_ij^cd + t_ij^dc (i <= j)
// and Tsa[o(o+1)/2 + stri(j,i)][c][d] = t_ij^cd - t_ij^dc (i < j).
__device__ inline float lp_round_bf16(float f) {
  const uint32_t u = __float_as_uint(f);
  return __uint_as_float(((u + 0x7fffu + ((u >> 16) & 1u)) >> 16) << 16);
}
template <typename T> __device__ inline T to_lp(double x);
template <> __device__ inline double to_lp<double>(double x) { return x; }
template <> __device__ inline float to_lp<float>(double x) { return (float)x; }
template <> __device__ inline uint16_t to_lp<uint16_t>(double x) {   // bf16, round to nearest even
  const uint32_t u = __float_as_uint((float)x);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
template <typename T> __device__ inline double from_lp(T x);
template <> __device__ inline double from_lp<double>(double x) { return x; }
template <> __device__ inline double from_lp<float>(float x) { return (double)x; }

template <typename T>
__global__ void k_convert(const double *__restrict__ in, int64_t n, T *out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    out[e] = to_lp<T>(in[e]);
}

// Ladder rows: S_ij^cd = t_ij^cd + t_ij^dc at row tri(j, i) and, for i < j,
// A_ij^cd = t_ij^cd - t_ij^dc at row o(o+1)/2 + stri(j, i).  A block takes one
// pair i <= j and one 32 x 32 (c0, d0) tile; both t_ij[c][d] and t_ij[d][c] of the
// tile go through LDS so that every read and write runs along the contiguous index.
template <typename T>
__global__ void k_pack_t(const double *__restrict__ t2, int64_t o, int64_t v, T *Tsa) {
  __shared__ double Xs[kCT][kCT + 1], Ys[kCT][kCT + 1];   // t[c0 + r][d0 + q], t[d0 + r][c0 + q]
  const int64_t vv = v * v, op = o * (o + 1) / 2;
  const int tiles = (int)((v + kCT - 1) / kCT);
  const int64_t c0 = (int64_t)(blockIdx.x / tiles) * kCT, d0 = (int64_t)(blockIdx.x % tiles) * kCT;
  for (int64_t p = blockIdx.y; p < op; p += gridDim.y) {
    // p -> (i, j), i <= j, rows of the upper triangle in order
    int64_t i = 0, rem = p;
    while (rem >= o - i) { rem -= o - i; ++i; }
    const int64_t j = i + rem;
    const double *X = t2 + (i * o + j) * vv;
    __syncthreads();
    for (int e = threadIdx.x; e < kCT * kCT; e += blockDim.x) {
      const int r = e / kCT, q = e % kCT;
      Xs[r][q] = (c0 + r < v && d0 + q < v) ? X[(c0 + r) * v + d0 + q] : 0.0;
      Ys[r][q] = (d0 + r < v && c0 + q < v) ? X[(d0 + r) * v + c0 + q] : 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kCT * kCT; e += blockDim.x) {
      const int r = e / kCT, q = e % kCT;
      const int64_t c = c0 + r, d = d0 + q;
      if (c >= v || d >= v) continue;
      const double x = Xs[r][q], y = Ys[q][r];   // t_ij^cd, t_ij^dc
      Tsa[tri(j, i) * vv + c * v + d] = to_lp<T>(x + y);
      if (i < j) Tsa[(op + stri(j, i)) * vv + c * v + d] = to_lp<T>(x - y);
    }
  }
}

// R2[i][j][a][b] += (S_ij^ab + A_ij^ab) / 2 from SA[r][P(a, b)] (a >= b), where
// rows r < o(o+1)/2 hold S (symmetric in ij and ab) and the rest A
// (antisymmetric in both).  ca == 0: P = a v + b, rows of v^2; ca > 0: the
// stored-ladder row order (blocks of ca values of a, each [a - a0][b < a1]):
// P = ca^2 q (q + 1) / 2 + (a - a0) a1 + b with q = a / ca, a0 = q ca,
// a1 = min(a0 + ca, v), rows of ld entries.
__global__ void k_unpack_ladder(const double *__restrict__ SA, int64_t o, int64_t v, int64_t ca,
                                int64_t ld, double *R2) {
  const int64_t vv = v * v, total = o * o * vv, op = o * (o + 1) / 2;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t i, j, a, b;
    split4(e, o, v, i, j, a, b);
    const int64_t hi = (a >= b) ? a : b, lo = (a >= b) ? b : a;
    int64_t P;
    if (ca == 0) {
      P = hi * v + lo;
    } else {
      const int64_t q = hi / ca, a0 = q * ca, a1 = (a0 + ca < v) ? a0 + ca : v;
      P = ca * ca * q * (q + 1) / 2 + (hi - a0) * a1 + lo;
    }
    double r = SA[((i <= j) ? tri(j, i) : tri(i, j)) * ld + P];
    if (i != j && a != b) {
      const double sg = ((i < j) == (a > b)) ? 1.0 : -1.0;
      r += sg * SA[(op + ((i < j) ? stri(j, i) : stri(i, j))) * ld + P];
    }
    R2[e] += 0.5 * r;
  }
}

// (T) energy epilogue on cube tiles of the W tensors (blocked layout: the 8 x 8
// (b, c) face of a tile is 64 contiguous elements, so a tile is eight 64-element
// runs).
constexpr int TT = 8;          // tile edge
constexpr int TP = TT + 1;     // padded innermost extent in LDS

// Loads the distinct tiles of one orbit: tile p (slot[p] == p) has block
// coordinates (c[P[p][0]], c[P[p][1]], c[P[p][2]]).  Rows with a >= v are not
// read (they are not in memory and never used).
template <typename TW> struct TileLoad;
template <> struct TileLoad<float> {
  // two tiles per pass: 8 rows x 16 four-element vectors each
  __device__ static void run(const float *__restrict__ W, int v, int vt, int mask, const int *c,
                             float (*L)[TT * TT * TP]) {
    constexpr int P[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    const int t = threadIdx.x, half = t >> 7, x = (t >> 4) & 7, q = t & 15;
    const int y = q >> 1, z = (q & 1) * 4;
    int rank = 0;
#pragma unroll
    for (int p = 0; p < 6; ++p) {
      if (!((mask >> p) & 1)) continue;
      const int mine = (rank & 1) == half;
      ++rank;
      const int a = 8 * c[P[p][0]] + x;
      if (!mine || a >= v) continue;
      const float4 f = *(const float4 *)(W + ((int64_t)a * vt * vt + (int64_t)c[P[p][1]] * vt +
                                              c[P[p][2]]) * 64 + 4 * q);
      float *d = L[p] + (x * TT + y) * TP + z;
      d[0] = f.x; d[1] = f.y; d[2] = f.z; d[3] = f.w;
    }
  }
};
template <> struct TileLoad<double> {
  // one tile per pass: 8 rows x 32 two-element vectors
  __device__ static void run(const double *__restrict__ W, int v, int vt, int mask, const int *c,
                             double (*L)[TT * TT * TP]) {
    constexpr int P[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    const int t = threadIdx.x, x = t >> 5, q = t & 31;
    const int y = q >> 2, z = (q & 3) * 2;
#pragma unroll
    for (int p = 0; p < 6; ++p) {
      const int a = 8 * c[P[p][0]] + x;
      if (!((mask >> p) & 1) || a >= v) continue;
      const double2 f = *(const double2 *)(W + ((int64_t)a * vt * vt + (int64_t)c[P[p][1]] * vt +
                                                c[P[p][2]]) * 64 + 2 * q);
      double *d = L[p] + (x * TT + y) * TP + z;
      d[0] = f.x; d[1] = f.y;
    }
  }
};

// 1 / x from the hardware reciprocal estimate and two Newton-Raphson steps
// (r <- r + r (1 - x r); each step squares the relative error), for the (T)
// denominators, which are negative and far from zero and from overflow.
__device__ inline double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}

// Index of the ordered pair (u1, u2), u1 != u2, of block-coordinate positions.
__device__ inline int pair_index(int u1, int u2) { return 2 * u1 + (u2 > u1 ? u2 - 1 : u2); }

// The W tensor of one triple is read in six index orders.  Cube tiles are
// grouped into orbits under permutations of their (a, b, c) block coordinates;
// a block loads the (up to six) distinct tiles of one orbit once and evaluates
// the integrand on all of them, so each W element is read from memory once.
// The disconnected part of V needs (ia|jb), (ia|kc), (jb|kc) on pairs of the
// orbit's coordinate blocks, t1 and the orbital energies on its blocks: these go
// to LDS with the tiles.
//
// Work items are (triple, orbit) pairs, triple-major.  Workgroups are dispatched
// round-robin over the eight XCDs (block b to XCD b % 8), each with its own L2:
// the items are cut into eight contiguous ranges and the blocks of XCD x share
// range x, so the integrals of one triple and the neighbouring rows of its W are
// fetched by one L2.  Each block adds the weighted sums of its items and writes
// one partial.
template <typename TW, int SYM>
__global__ __launch_bounds__(kRedThreads) __attribute__((amdgpu_waves_per_eu(5))) void k_triples_energy(
    const TW *__restrict__ Wall, const int *__restrict__ table, int nb,
    const double *__restrict__ Kov, const double *__restrict__ t1, const double *__restrict__ eo,
    const double *__restrict__ ev, int o, int v, double *partials) {
  __shared__ TW L[6][TT * TT * TP];
  __shared__ double K[3][6][TT * TT];   // (ia|jb), (ia|kc), (jb|kc) on ordered block pairs
  __shared__ double T1[3][3][TT];       // t1 of i, j, k on each coordinate block
  __shared__ double EV[3][TT];
  __shared__ double sm[kRedThreads / 64];
  constexpr int P[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  const int t = threadIdx.x;
  const int vt = (v + TT - 1) / TT;
  const int64_t norbits = (int64_t)vt * (vt + 1) * (vt + 2) / 6;
  const int64_t went = (int64_t)v * vt * vt * 64;   // elements of one triple's W
  const int xcd = blockIdx.x & 7, S = gridDim.x >> 3, s = blockIdx.x >> 3;
  const int64_t N = (int64_t)nb * norbits;
  const int64_t lo = N * xcd / 8, hi = N * (xcd + 1) / 8;
  // compute mapping: thread -> (x, y) of a tile face and z = zq, zq + 4
  const int cx = t >> 5, cy = (t >> 2) & 7, zq = t & 3;
  double total = 0.0;
  for (int64_t item = lo + s; item < hi; item += S) {
    const int entry = (int)(item / norbits);
    const int64_t orb = item % norbits;
    const int i = table[3 * entry], j = table[3 * entry + 1], k = table[3 * entry + 2];
    const TW *W = Wall + (int64_t)entry * went;
    const double eijk = eo[i] + eo[j] + eo[k];
    // canonical block coordinates c0 <= c1 <= c2 of orbit number orb
    int c[3];
    {
      int64_t r = orb;
      int A = 0;
      for (;; ++A) {
        const int64_t n = (int64_t)(vt - A) * (vt - A + 1) / 2;
        if (r < n) break;
        r -= n;
      }
      int Bc = A;
      for (;; ++Bc) {
        const int64_t n = vt - Bc;
        if (r < n) break;
        r -= n;
      }
      c[0] = A; c[1] = Bc; c[2] = Bc + (int)r;
    }
    // slot[p]: the first permutation with the same tile coordinates as p; bit p
    // of mask: p is the first of its tile
    int slot[6], mask = 0;
#pragma unroll
    for (int p = 0; p < 6; ++p) {
      slot[p] = p;
#pragma unroll
      for (int q = 0; q < p; ++q)
        if (slot[p] == p && c[P[q][0]] == c[P[p][0]] && c[P[q][1]] == c[P[p][1]] &&
            c[P[q][2]] == c[P[p][2]])
          slot[p] = q;
      if (slot[p] == p) mask |= 1 << p;
    }
    __syncthreads();   // the previous item's reads of LDS are done
    TileLoad<TW>::run(W, v, vt, mask, c, L);
    // integral blocks: kind 0 (ia|jb) = Kov[i][a][j][b], 1 (ia|kc), 2 (jb|kc); every
    // load of a thread is issued before the first store
    constexpr int KN = 3 * 6 * TT * TT, KPT = (KN + kRedThreads - 1) / kRedThreads;
    double kv[KPT];
#pragma unroll
    for (int n = 0; n < KPT; ++n) {
      const int e = t + n * kRedThreads;
      if (e < KN) {
        const int kind = e / (6 * TT * TT), pr = (e / (TT * TT)) % 6, r = (e / TT) % TT,
                  q = e % TT;
        const int u1 = pr / 2, u2r = pr % 2, u2 = u2r < u1 ? u2r : u2r + 1;
        const int m1 = kind == 2 ? j : i, m2 = kind == 0 ? j : k;
        const int x1 = min(8 * c[u1] + r, v - 1), x2 = min(8 * c[u2] + q, v - 1);
        kv[n] = Kov[(((int64_t)m1 * v + x1) * o + m2) * v + x2];
      }
    }
#pragma unroll
    for (int n = 0; n < KPT; ++n) {
      const int e = t + n * kRedThreads;
      if (e < KN) (&K[0][0][0])[e] = kv[n];
    }
    if (t < 3 * 3 * TT) {
      const int m = t / (3 * TT), u = (t / TT) % 3, r = t % TT;
      const int occ = m == 0 ? i : m == 1 ? j : k;
      T1[m][u][r] = t1[(int64_t)occ * v + min(8 * c[u] + r, v - 1)];
    } else if (t < 3 * 3 * TT + 3 * TT) {
      const int e = t - 3 * 3 * TT, u = e / TT, r = e % TT;
      EV[u][r] = ev[min(8 * c[u] + r, v - 1)];
    }
    __syncthreads();
    double acc = 0.0;
#pragma unroll
    for (int p = 0; p < 6; ++p) {
      if (!((mask >> p) & 1)) continue;   // every distinct tile once
      const int s0 = P[p][0], s1 = P[p][1], s2 = P[p][2];
      // tiles holding W at (b,c,a), (c,a,b), (a,c,b), (b,a,c), (c,b,a) orders
      auto find = [&](int q0, int q1, int q2) {
        int r = 0;
#pragma unroll
        for (int q = 0; q < 6; ++q)
          if (P[q][0] == q0 && P[q][1] == q1 && P[q][2] == q2) r = slot[q];
        return r;
      };
      const TW *Labc = L[p];
      const TW *Lbca = L[find(s1, s2, s0)];
      const TW *Lcab = L[find(s2, s0, s1)];
      const TW *Lacb = L[find(s0, s2, s1)];
      const TW *Lbac = L[find(s1, s0, s2)];
      const TW *Lcba = L[find(s2, s1, s0)];
      const int a = 8 * c[s0] + cx, b = 8 * c[s1] + cy, c0 = 8 * c[s2];
      if (a >= v || b >= v) continue;
      const double *Kab = K[0][pair_index(s0, s1)], *Kac = K[1][pair_index(s0, s2)],
                   *Kbc = K[2][pair_index(s1, s2)];
      const double kab = Kab[cx * TT + cy], t1a = T1[0][s0][cx], t1b = T1[1][s1][cy];
      const double eab = eijk - EV[s0][cx] - EV[s1][cy];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int z = zq + 4 * h;
        if (c0 + z >= v) continue;
        const double zabc = Labc[(cx * TT + cy) * TP + z];
        const double zbca = Lbca[(cy * TT + z) * TP + cx];
        const double zcab = Lcab[(z * TT + cx) * TP + cy];
        const double zacb = Lacb[(cx * TT + z) * TP + cy];
        const double zbac = Lbac[(cy * TT + cx) * TP + z];
        const double zcba = Lcba[(z * TT + cy) * TP + cx];
        // sym 1: W(a,b,c) = Z(a,b,c) + Z(b,a,c); sym 2: W(a,b,c) = Z(a,b,c) + Z(a,c,b);
        // the six permuted values of W are then sums of the six permuted values of Z
        double w, wbca, wcab, wacb, wbac, wcba;
        if constexpr (SYM == 1) {
          w = zabc + zbac; wbca = zbca + zcba; wcab = zcab + zacb;
          wacb = zacb + zcab; wbac = zbac + zabc; wcba = zcba + zbca;
        } else if constexpr (SYM == 2) {
          w = zabc + zacb; wbca = zbca + zbac; wcab = zcab + zcba;
          wacb = zacb + zabc; wbac = zbac + zbca; wcba = zcba + zcab;
        } else {
          w = zabc; wbca = zbca; wcab = zcab; wacb = zacb; wbac = zbac; wcba = zcba;
        }
        const double V = w + kab * T1[2][s2][z] + Kac[cx * TT + z] * t1b + Kbc[cy * TT + z] * t1a;
        const double Z = 4.0 * w + wbca + wcab - 2.0 * (wacb + wbac + wcba);
        acc = fma(V * Z, recip(eab - EV[s2][z]), acc);
      }
    }
    total += ((i < j && j < k) ? 2.0 : 1.0) * acc;   // (6 or 3) / 3
  }
  const double r = block_sum(total, sm);
  if (t == 0) partials[blockIdx.x] = r;
}

}  // namespace

hipError_t split_B(const double *B, int64_t X, int64_t o, int64_t v, double *Boo, double *Bov,
                   double *Bvv, hipStream_t s) {
  if (dry_run()) return hipSuccess;
  const int64_t n = o + v;
  hipLaunchKernelGGL(k_split_B, dim3(ew_blocks(X * n * n)), dim3(kEwThreads), 0, s, B, X, o, v,
                     Boo, Bov, Bvv);
  return hipGetLastError();
}
hipError_t dress_vv(const double *Bvv, const double *Bov, const double *t1, int64_t X, int64_t o,
                    int64_t v, double *Bt, hipStream_t s) {
  if (X < 1 || o < 1 || v < 1) return hipErrorInvalidValue;
  if (!region_ok(Bvv, (size_t)(X * v * v * 8)) || !region_ok(Bt, (size_t)(X * v * v * 8)) ||
      !region_ok(Bov, (size_t)(X * o * v * 8)) || !region_ok(t1, (size_t)(o * v * 8))) {
    note_error("T1 dressing of B_vv (nocc %lld, nvir %lld, naux %lld) leaves its buffers",
               (long long)o, (long long)v, (long long)X);
    return hipErrorInvalidValue;
  }
  if (dry_run()) return hipSuccess;
  const dim3 g((unsigned)((v + kDressRows - 1) / kDressRows), (unsigned)X);
  // one thread per column b up to 256 (whole waves), so few lanes idle at small v
  const unsigned threads = (unsigned)std::min<int64_t>(kEwThreads, (v + 63) / 64 * 64);
  hipLaunchKernelGGL(k_dress_vv, g, dim3(threads), (size_t)o * kDressRows * 8, s, Bvv, Bov, t1,
                     o, v, Bt);
  return hipGetLastError();
}
hipError_t diag_sum(const double *Boo, int64_t X, int64_t o, double *J, hipStream_t s) {
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(k_diag_sum, dim3(ew_blocks(X)), dim3(kEwThreads), 0, s, Boo, X, o, J);
  return hipGetLastError();
}
hipError_t add_diag(double *M, int64_t n, int64_t ld, const double *eps, hipStream_t s) {
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(k_add_diag, dim3(ew_blocks(n)), dim3(kEwThreads), 0, s, M, n, ld, eps);
  return hipGetLastError();
}
hipError_t transpose2d(const double *in, int64_t rows, int64_t cols, double *out, hipStream_t s) {
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(k_transpose2d, dim3(ew_blocks(rows * cols)), dim3(kEwThreads), 0, s, in,
                     rows, cols, out);
  return hipGetLastError();
}
hipError_t make_u(const double *t2, int64_t o, int64_t v, double *u, hipStream_t s) {
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(k_make_u, dim3(ew_blocks(o * o * v * v)), dim3(kEwThreads), 0, s, t2, o, v, u);
  return hipGetLastError();
}
hipError_t mp2_guess(const double *Kov, const double *eo, const double *ev, int64_t o, int64_t v,
                     double *t1, double *t2, hipStream_t s) {
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(k_mp2_guess, dim3(ew_blocks(o * o * v * v)), dim3(kEwThreads), 0, s, Kov,
                     eo, ev, o, v, t1, t2);
  return hipGetLastError();
}
hipError_t build_lov(const double *Kov, int64_t o, int64_t v, double *Lov, hipStream_t s) {
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(k_build_lov, dim3(ew_blocks(o * o * v * v)), dim3(kEwThreads), 0, s, Kov,
                     o, v, Lov);
  return hipGetLastError();
}
hipError_t sub_oovv_into_dint(const double *Goovv, int64_t o, int64_t v, double *Dint,
                              hipStream_t s) {
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(k_sub_oovv, dim3(ew_blocks(o * o * v * v)), dim3(kEwThreads), 0, s, Goovv,
                     o, v, Dint);
  return hipGetLastError();
}
hipError_t combine_r2(double *R2, const double *S, const double *Xc, int64_t o, int64_t v,
                      hipStream_t s) {
  if (dry_run()) return hipSuccess;
  if (o == 0 || v == 0) return hipSuccess;
  const int tiles = (int)((v + kCT - 1) / kCT);
  const unsigned pairs = (unsigned)std::min<int64_t>(o * o, 65535);   // grid rows over (i, j)
  hipLaunchKernelGGL(k_combine_r2, dim3(tiles * tiles, pairs), dim3(kEwThreads), 0, s, R2, S, Xc,
                     o, v);
  return hipGetLastError();
}
hipError_t pair_symmetrize(double *R2, int64_t o, int64_t v, hipStream_t s) {
  if (dry_run()) return hipSuccess;
  if (o == 0 || v == 0) return hipSuccess;
  const int tiles = (int)((v + kCT - 1) / kCT);
  const int64_t npairs = o * (o + 1) / 2;
  const unsigned rows = (unsigned)std::min<int64_t>(npairs, 65535);
  hipLaunchKernelGGL(k_pair_symmetrize, dim3(tiles * tiles, rows), dim3(kEwThreads), 0, s, R2, o,
                     v);
  return hipGetLastError();
}
hipError_t energy_partials(const double *Kov, const double *t1, const double *t2, int64_t o,
                           int64_t v, double *partials, hipStream_t s) {
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(k_energy_partials, dim3(kRedBlocks), dim3(kRedThreads), 0, s, Kov, t1, t2,
                     o, v, partials);
  return hipGetLastError();
}
hipError_t reduce_partials(const double *partials, int64_t n, double *out, int accumulate,
                           hipStream_t s) {
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kRedThreads), 0, s, partials, n, out, accumulate);
  return hipGetLastError();
}
hipError_t jacobi_step(const double *t1, const double *t2, const double *R1, const double *R2,
                       const double *eo, const double *ev, int64_t o, int64_t v, double shift,
                       double *x, double *e, double *partials, hipStream_t s) {
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(k_jacobi, dim3(kRedBlocks), dim3(kRedThreads), 0, s, t1, t2, R1, R2, eo, ev,
                     o, v, shift, x, e, partials);
  return hipGetLastError();
}
hipError_t dot_partials(const double *E, int64_t stride, int m, const double *enew, int64_t N,
                        double *partials, hipStream_t s) {
  if (dry_run()) return hipSuccess;
  if (m < 1 || m > kMaxDiis) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_dot_partials, dim3(kRedBlocks), dim3(kRedThreads), 0, s, E, stride, m,
                     enew, N, partials);
  return hipGetLastError();
}
hipError_t reduce_rows(const double *partials, int m, double *out, hipStream_t s) {
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_rows, dim3(m), dim3(kRedThreads), 0, s, partials, out);
  return hipGetLastError();
}
hipError_t lincomb(const double *Xs, int64_t stride, int m, const double *c_host, int64_t o,
                   int64_t v, double *t1, double *t2, hipStream_t s) {
  if (dry_run()) return hipSuccess;
  if (m < 1 || m > kMaxDiis) return hipErrorInvalidValue;
  Coeffs cf{};
  for (int i = 0; i < m; ++i) cf.c[i] = c_host[i];
  hipLaunchKernelGGL(k_lincomb, dim3(ew_blocks(o * v + o * o * v * v)), dim3(kEwThreads), 0, s,
                     Xs, stride, m, cf, o, v, t1, t2);
  return hipGetLastError();
}
hipError_t scatter_vec(const double *x, int64_t o, int64_t v, double *t1, double *t2,
                       hipStream_t s) {
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(k_scatter, dim3(ew_blocks(o * v + o * o * v * v)), dim3(kEwThreads), 0, s,
                     x, o, v, t1, t2);
  return hipGetLastError();
}
hipError_t pack_t(const double *t2, int64_t o, int64_t v, void *Tsa, int type, hipStream_t s) {
  if (dry_run()) return hipSuccess;
  if (o == 0 || v == 0) return hipSuccess;
  const int64_t tiles = (v + kCT - 1) / kCT, npairs = o * (o + 1) / 2;
  const dim3 g((unsigned)(tiles * tiles), (unsigned)std::min<int64_t>(npairs, 65535)),
      b(kEwThreads);
  if (type == 1) hipLaunchKernelGGL(k_pack_t<float>, g, b, 0, s, t2, o, v, (float *)Tsa);
  else if (type == 2)
    hipLaunchKernelGGL(k_pack_t<uint16_t>, g, b, 0, s, t2, o, v, (uint16_t *)Tsa);
  else hipLaunchKernelGGL(k_pack_t<double>, g, b, 0, s, t2, o, v, (double *)Tsa);
  return hipGetLastError();
}
hipError_t convert(const double *in, int64_t n, void *out, int type, hipStream_t s) {
  if (dry_run()) return hipSuccess;
  const dim3 g(ew_blocks(n)), b(kEwThreads);
  if (type == 1) hipLaunchKernelGGL(k_convert<float>, g, b, 0, s, in, n, (float *)out);
  else if (type == 2) hipLaunchKernelGGL(k_convert<uint16_t>, g, b, 0, s, in, n, (uint16_t *)out);
  else hipLaunchKernelGGL(k_convert<double>, g, b, 0, s, in, n, (double *)out);
  return hipGetLastError();
}
hipError_t unpack_ladder(const double *SA, int64_t o, int64_t v, int64_t ca, int64_t ld,
                         double *R2, hipStream_t s) {
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(k_unpack_ladder, dim3(ew_blocks(o * o * v * v)), dim3(kEwThreads), 0, s, SA,
                     o, v, ca, ld, R2);
  return hipGetLastError();
}
// Unique triples i <= j <= k (not all equal) in three groups, each in
// lexicographic order: i < j < k, then i = j < k, then i < j = k; one thread,
// once per (T) computation.
__global__ void k_triples_table(int *table, int o) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int64_t n = 0;
  for (int g = 0; g < 3; ++g)
    for (int i = 0; i < o; ++i)
      for (int j = i; j < o; ++j)
        for (int k = j; k < o; ++k) {
          const int grp = (i < j && j < k) ? 0 : (i == j && j < k) ? 1 : (i < j && j == k) ? 2 : 3;
          if (grp != g) continue;
          table[3 * n] = i;
          table[3 * n + 1] = j;
          table[3 * n + 2] = k;
          ++n;
        }
}
hipError_t triples_table(int *table, int64_t o, hipStream_t s) {
  if (dry_run()) return hipSuccess;
  hipLaunchKernelGGL(k_triples_table, dim3(1), dim3(64), 0, s, table, (int)o);
  return hipGetLastError();
}
hipError_t triples_energy(const void *W, int wtype, int sym, const int *table, int nb,
                          const double *Kov, const double *t1, const double *eo,
                          const double *ev, int64_t o, int64_t v, double *partials,
                          int64_t capacity, int64_t *nparts, hipStream_t s) {
  if (nb < 1 || o < 1 || v < 1 || o > 65535 || v > 65535 || sym < 0 || sym > 2)
    return hipErrorInvalidValue;
  const int grid = wtype == 1 ? kTriplesEnergyGrid : kTriplesEnergyGrid64;
  *nparts = grid;
  if (*nparts > capacity) {
    note_error("(T) energy partials: %lld needed, %lld allocated", (long long)*nparts,
               (long long)capacity);
    return hipErrorInvalidValue;
  }
  const int64_t vt = (v + TT - 1) / TT, es = wtype == 1 ? 4 : 8;
  if (!region_ok(W, (size_t)(nb * v * vt * vt * 64 * es)) ||
      !region_ok(table, (size_t)nb * 3 * sizeof(int)) ||
      !region_ok(Kov, (size_t)(o * v * o * v * 8)) || !region_ok(partials, (size_t)*nparts * 8)) {
    note_error("(T) energy (nocc %lld, nvir %lld, %d triples) leaves its buffers; not launched",
               (long long)o, (long long)v, nb);
    return hipErrorInvalidValue;
  }
  if (dry_run()) return hipSuccess;
  const dim3 g(grid), b(kRedThreads);
  const int io = (int)o, iv = (int)v;
  if (wtype == 1) {
    const float *w = (const float *)W;
    if (sym == 1)
      hipLaunchKernelGGL((k_triples_energy<float, 1>), g, b, 0, s, w, table, nb, Kov, t1, eo, ev, io, iv, partials);
    else if (sym == 2)
      hipLaunchKernelGGL((k_triples_energy<float, 2>), g, b, 0, s, w, table, nb, Kov, t1, eo, ev, io, iv, partials);
    else
      hipLaunchKernelGGL((k_triples_energy<float, 0>), g, b, 0, s, w, table, nb, Kov, t1, eo, ev, io, iv, partials);
  } else {
    const double *w = (const double *)W;
    if (sym == 1)
      hipLaunchKernelGGL((k_triples_energy<double, 1>), g, b, 0, s, w, table, nb, Kov, t1, eo, ev, io, iv, partials);
    else if (sym == 2)
      hipLaunchKernelGGL((k_triples_energy<double, 2>), g, b, 0, s, w, table, nb, Kov, t1, eo, ev, io, iv, partials);
    else
      hipLaunchKernelGGL((k_triples_energy<double, 0>), g, b, 0, s, w, table, nb, Kov, t1, eo, ev, io, iv, partials);
  }
  return hipGetLastError();
}

}  // namespace lnocc

// Local active spaces of LNO-CC (Sec. II.C-E), the local Hamiltonian's DF
// factors (Eq. 27b) and the MP2 energy behind the composite correction (Eq. 17).
//
// For a fragment with LO coefficients U_occ [no][m] on the canonical occupied
// orbitals (and U_vir [nv][m] for LOs that reach into the virtual space):
//   1. internal / external orbitals: eigenvectors of U U^T with non-zero / zero
//      eigenvalues, i.e. the left singular vectors of U (Eqs. 18-19);
//   2. the internal orbitals made semi-canonical (Fock matrix diagonal inside
//      their span), which gives the f_{i_F i_F} of Eq. 21;
//   3. MP1 amplitudes with one internal occupied index (Eqs. 21-23) from the
//      DF factors of the canonical ov block;
//   4. the densities of Eq. 20, or the CBNO densities of Eq. 28, as matrix
//      products over two-index modes;
//   5. the densities diagonalized inside the external spaces (Eqs. 24-25); LNOs
//      with |lambda| >= eta are kept (Eq. 26);
//   6. internal orbitals plus kept LNOs made semi-canonical: the fragment's
//      active orbitals and orbital energies.
// Every product is a gett() contraction in FP64; symmetric eigenproblems go to
// a one-workgroup parallel Jacobi kernel.  The host reads back only the
// eigenvalues that decide the sizes (the internal ranks and the LNO counts).
#include "lno.h"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "gett.h"
#include "kernels.h"

namespace lnocc {
namespace {

constexpr int kEigThreads = 1024;
constexpr int kEw = 256;

inline int ew_grid(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + kEw - 1) / kEw, 16384));
}

#define LN_TRY(x)                                                         \
  do {                                                                    \
    hipError_t e_ = (x);                                                  \
    if (e_ != hipSuccess) {                                               \
      note_error("%s failed (%s) at %s:%d", #x, hipGetErrorString(e_),    \
                 __FILE__, __LINE__);                                     \
      return LNOCC_EDEVICE;                                               \
    }                                                                     \
  } while (0)

#define LN_ST(x)              \
  do {                        \
    const int st_ = (x);      \
    if (st_) return st_;      \
  } while (0)

// ------------------------------------------------------------------ kernels
// Cyclic Jacobi for a symmetric A [n][n] (overwritten), one workgroup.  A sweep
// visits every pair (p, q) once, in m - 1 rounds of m / 2 disjoint pairs
// (round-robin order, m = n rounded up to even; the extra position is a
// dummy).  The rotations of one round touch disjoint rows and columns, so the
// block applies them together: first rows p, q of all pairs (A <- J^T A), then
// columns p, q (A <- A J, V <- V J).  Sweeps stop once the off-diagonal mass
// is at most 1e-30 |A|_F^2.  On exit w[n] holds the eigenvalues ascending and
// V's columns the eigenvectors in that order (ties by index).
__global__ __launch_bounds__(kEigThreads) void k_jacobi(double *A, double *V, double *w, int n,
                                                      int max_sweeps, int *perm) {
  __shared__ double cs[kEigMax / 2], sn[kEigMax / 2];
  __shared__ int pp[kEigMax / 2], pq[kEigMax / 2];
  __shared__ double red[kEigThreads / 64];
  __shared__ double total;
  const int t = threadIdx.x;
  const int m = n + (n & 1);
  const int npairs = m / 2;
  const int64_t nn = (int64_t)n * n;
  auto block_sum = [&](double x) {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    __syncthreads();
    if ((t & 63) == 0) red[t >> 6] = x;
    __syncthreads();
    if (t == 0) {
      double s = 0.0;
      for (int i = 0; i < kEigThreads / 64; ++i) s += red[i];
      total = s;
    }
    __syncthreads();
    return total;
  };
  for (int64_t e = t; e < nn; e += kEigThreads) V[e] = (e / n == e % n) ? 1.0 : 0.0;
  double fro = 0.0;
  for (int64_t e = t; e < nn; e += kEigThreads) fro += A[e] * A[e];
  const double tol = block_sum(fro) * 1e-30;
  for (int sweep = 0; sweep < max_sweeps && n > 1; ++sweep) {
    double off = 0.0;
    for (int64_t e = t; e < nn; e += kEigThreads)
      if (e / n != e % n) off += A[e] * A[e];
    if (block_sum(off) <= tol) break;
    for (int r = 0; r < m - 1; ++r) {
      for (int k = t; k < npairs; k += kEigThreads) {
        const int a = k == 0 ? 0 : ((k - 1 + r) % (m - 1)) + 1;
        const int kb = m - 1 - k;
        const int b = ((kb - 1 + r) % (m - 1)) + 1;
        const int p = a < b ? a : b, q = a < b ? b : a;
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = A[(int64_t)p * n + q];
          if (apq != 0.0) {
            const double tau = (A[(int64_t)q * n + q] - A[(int64_t)p * n + p]) / (2.0 * apq);
            const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
          }
        }
        pp[k] = p; pq[k] = q; cs[k] = c; sn[k] = s;
      }
      __syncthreads();
      for (int64_t e = t; e < (int64_t)npairs * n; e += kEigThreads) {   // rows
        const int k = (int)(e / n), j = (int)(e % n), p = pp[k], q = pq[k];
        if (q >= n) continue;
        const double c = cs[k], s = sn[k];
        const double ap = A[(int64_t)p * n + j], aq = A[(int64_t)q * n + j];
        A[(int64_t)p * n + j] = c * ap - s * aq;
        A[(int64_t)q * n + j] = s * ap + c * aq;
      }
      __syncthreads();
      for (int64_t e = t; e < (int64_t)npairs * n; e += kEigThreads) {   // columns
        const int k = (int)(e / n), i = (int)(e % n), p = pp[k], q = pq[k];
        if (q >= n) continue;
        const double c = cs[k], s = sn[k];
        const double ap = A[(int64_t)i * n + p], aq = A[(int64_t)i * n + q];
        A[(int64_t)i * n + p] = c * ap - s * aq;
        A[(int64_t)i * n + q] = s * ap + c * aq;
        const double vp = V[(int64_t)i * n + p], vq = V[(int64_t)i * n + q];
        V[(int64_t)i * n + p] = c * vp - s * vq;
        V[(int64_t)i * n + q] = s * vp + c * vq;
      }
      __syncthreads();
    }
  }
  // ascending order by rank (ties by index)
  for (int i = t; i < n; i += kEigThreads) {
    const double d = A[(int64_t)i * n + i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double dj = A[(int64_t)j * n + j];
      rank += (dj < d) || (dj == d && j < i);
    }
    perm[rank] = i;
  }
  __syncthreads();
  for (int i = t; i < n; i += kEigThreads) w[i] = A[(int64_t)perm[i] * n + perm[i]];
  __syncthreads();
  for (int64_t e = t; e < nn; e += kEigThreads) A[e] = V[e];   // A is free now
  __syncthreads();
  for (int64_t e = t; e < nn; e += kEigThreads) V[e] = A[(e / n) * n + perm[e % n]];
}

// out[r][c] = in[r][idx ? idx[c] : c] for r < rows, c < ncols
__global__ void k_gather_cols(const double *in, int64_t rows, int64_t ldi, const int *idx,
                              int64_t ncols, double *out, int64_t ldo) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < rows * ncols;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / ncols, c = e % ncols;
    out[r * ldo + c] = in[r * ldi + (idx ? idx[c] : c)];
  }
}

// out[c] = in[idx[c]]
__global__ void k_gather(const double *in, const int *idx, int64_t n, double *out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    out[e] = in[idx[e]];
}

// out[i][k] = eps[i] W[i][k]  (rows x cols, leading dimension cols)
__global__ void k_scale_rows(const double *W, const double *eps, int64_t rows, int64_t cols,
                             double *out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < rows * cols;
       e += (int64_t)gridDim.x * blockDim.x)
    out[e] = eps[e / cols] * W[e];
}

// X[n][n] = identity
__global__ void k_identity(double *X, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * n;
       e += (int64_t)gridDim.x * blockDim.x)
    X[e] = (e / n == e % n) ? 1.0 : 0.0;
}

__global__ void k_zero(double *x, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    x[e] = 0.0;
}

// MP1 amplitudes from the integrals in place, t [n1][n2][n3][n2]:
//   pattern 0: t[k][a][j][b] /= e1[k] + e2[j] - e3[a] - e3[b]  (one internal index)
//   pattern 1: t[i][A][k][B] /= e2[i] + e2[k] - e1[A] - e1[B]  (internal virtuals)
//   pattern 2: t[I][a][J][c] /= e1[I] + e1[J] - e3[a] - e3[c]  (internal occupied)
__global__ void k_mp1_divide(double *t, int64_t n1, int64_t n2, int64_t n3, const double *e1,
                             const double *e2, const double *e3, int pattern) {
  const int64_t n = n1 * n2 * n3 * n2;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e % n2, j = (e / n2) % n3, a = (e / (n2 * n3)) % n2, k = e / (n2 * n3 * n2);
    double d;
    if (pattern == 0) d = e1[k] + e2[j] - e3[a] - e3[b];
    else if (pattern == 1) d = e2[k] + e2[j] - e1[a] - e1[b];
    else d = e1[k] + e1[j] - e3[a] - e3[b];
    t[e] /= d;
  }
}

// out[k][a][j][b] = in[k][b][j][a], both [n1][n2][n3][n2]
__global__ void k_swap_pair(const double *in, int64_t n1, int64_t n2, int64_t n3, double *out) {
  const int64_t n = n1 * n2 * n3 * n2;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e % n2, j = (e / n2) % n3, a = (e / (n2 * n3)) % n2, k = e / (n2 * n3 * n2);
    out[e] = in[((k * n2 + b) * n3 + j) * n2 + a];
  }
}

// D = X - (Y + Y^T) over [n][n]
__global__ void k_sub_sym(double *D, const double *X, const double *Y, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / n, j = e % n;
    D[e] = X[e] - (Y[e] + Y[j * n + i]);
  }
}

// MP2 on a block of bi occupied rows starting at i0: the integrals
// V[i][j][a][b] = (i0+i a|j b) become amplitudes in place, and partials[block]
// receives pieces of sum V (2 V - V^{a<->b}) / D.  A thread takes the (a, b)
// and (b, a) elements of one pair a <= b.
__global__ __launch_bounds__(kRedThreads) void k_mp2_block(double *V, int64_t bi, int64_t i0,
                                                           int64_t o, int64_t v, const double *eo,
                                                           const double *ev, double *partials) {
  __shared__ double red[kRedThreads / 64];
  const int64_t npair = v * (v + 1) / 2, n = bi * o * npair;
  double acc = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * kRedThreads) {
    const int64_t ij = e / npair, r = e % npair;
    // r -> (a, b) with a <= b, rows of the upper triangle in order:
    // row a starts at first(a) = a v - a (a - 1) / 2
    const double tv = 2.0 * v + 1.0;
    int64_t a = (int64_t)((tv - sqrt(tv * tv - 8.0 * (double)r)) * 0.5);
    a = a < 0 ? 0 : (a > v - 1 ? v - 1 : a);
    while (a > 0 && a * v - a * (a - 1) / 2 > r) --a;
    while (a + 1 < v && (a + 1) * v - (a + 1) * a / 2 <= r) ++a;
    const int64_t b = a + (r - (a * v - a * (a - 1) / 2));
    const int64_t i = ij / o, j = ij % o;
    double *blk = V + ij * v * v;
    const double d = eo[i0 + i] + eo[j] - ev[a] - ev[b];
    const double vab = blk[a * v + b], vba = blk[b * v + a];
    if (a == b) {
      acc += vab * vab / d;
      blk[a * v + a] = vab / d;
    } else {
      acc += (vab * (2.0 * vab - vba) + vba * (2.0 * vba - vab)) / d;
      blk[a * v + b] = vab / d;
      blk[b * v + a] = vba / d;
    }
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < kRedThreads / 64; ++k) s += red[k];
    partials[blockIdx.x] = s;
  }
}

// ------------------------------------------------------------------ host helpers
struct Arena {
  char *base;
  size_t off = 0;
  double *d(int64_t n) {
    off = (off + 255) & ~size_t(255);
    double *p = base ? (double *)(base + off) : nullptr;
    off += (size_t)std::max<int64_t>(n, 1) * sizeof(double);
    return p;
  }
};

bool dry() { return dry_run(); }

// C = alpha A B (+ beta C) for plain strided matrices (element strides)
hipError_t mm(int64_t M, int64_t N, int64_t K, double alpha, const double *A, int64_t sam,
              int64_t sak, const double *B, int64_t sbk, int64_t sbn, double beta, double *C,
              int64_t scm, int64_t scn, hipStream_t s) {
  if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
  return gett(gemm_desc((int)M, (int)N, (int)K, alpha, A, sam, sak, B, sbk, sbn, beta, C, scm, scn),
              s);
}

// out[P][r][q] = sum_k A(r, k) X[P][k][q] for P < batch (A: r-stride sar,
// k-stride sak; X rows of ldx, P stride sxp; out rows of ldo, P stride sop)
hipError_t left_mul_batched(int64_t rows, int64_t cols, int64_t K, const double *A, int64_t sar,
                            int64_t sak, const double *Xp, int64_t ldx, int64_t sxp, double *out,
                            int64_t ldo, int64_t sop, int64_t batch, hipStream_t s) {
  if (rows <= 0 || cols <= 0 || K <= 0 || batch <= 0) return hipSuccess;
  GemmDesc d{};
  d.M = (int)rows; d.Mi = 1; d.N = (int)cols; d.Ni = 1; d.nseg = 1;
  d.seg[0].a = GOperand{A, sar, 0, sak, 0, 0, 0, 0, 0};
  d.seg[0].b = GOperand{Xp, 1, 0, ldx, 0, 0, 0, 0, sxp};
  d.seg[0].K = (int)K; d.seg[0].Ki = 1; d.seg[0].scale = 1.0;
  d.c = out; d.c_mo = ldo; d.c_no = 1; d.c_bid = sop;
  d.batch = (int)batch; d.nb1 = 1; d.prec = Prec::F64;
  return gett(d, s);
}

// out[P][r][q] = sum_k X[P][r][k] A(k, q) for P < batch (X rows of ldx, P stride
// sxp; A: k-stride sak, q-stride saq)
hipError_t right_mul_batched(int64_t rows, int64_t cols, int64_t K, const double *Xp, int64_t ldx,
                             int64_t sxp, const double *A, int64_t sak, int64_t saq, double *out,
                             int64_t ldo, int64_t sop, int64_t batch, hipStream_t s) {
  if (rows <= 0 || cols <= 0 || K <= 0 || batch <= 0) return hipSuccess;
  GemmDesc d{};
  d.M = (int)rows; d.Mi = 1; d.N = (int)cols; d.Ni = 1; d.nseg = 1;
  d.seg[0].a = GOperand{Xp, ldx, 0, 1, 0, 0, 0, 0, sxp};
  d.seg[0].b = GOperand{A, saq, 0, sak, 0, 0, 0, 0, 0};
  d.seg[0].K = (int)K; d.seg[0].Ki = 1; d.seg[0].scale = 1.0;
  d.c = out; d.c_mo = ldo; d.c_no = 1; d.c_bid = sop;
  d.batch = (int)batch; d.nb1 = 1; d.prec = Prec::F64;
  return gett(d, s);
}

hipError_t gather_cols(const double *in, int64_t rows, int64_t ldi, const int *idx,
                       int64_t ncols, double *out, int64_t ldo, hipStream_t s) {
  if (rows <= 0 || ncols <= 0 || dry()) return hipSuccess;
  if (!region_ok(out, (size_t)((rows - 1) * ldo + ncols) * 8) ||
      !region_ok(in, (size_t)((rows - 1) * ldi + 1) * 8)) {
    note_error("column gather (%lld x %lld) outside the installed buffers", (long long)rows,
               (long long)ncols);
    return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(k_gather_cols, dim3(ew_grid(rows * ncols)), dim3(kEw), 0, s, in, rows, ldi,
                     idx, ncols, out, ldo);
  return hipGetLastError();
}

hipError_t zero(double *x, int64_t n, hipStream_t s) {
  if (n <= 0 || dry()) return hipSuccess;
  if (!region_ok(x, (size_t)n * 8)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_zero, dim3(ew_grid(n)), dim3(kEw), 0, s, x, n);
  return hipGetLastError();
}

// host copy of n device doubles (zeros in validation mode)
int read_back(const double *d, int64_t n, std::vector<double> &h, hipStream_t s) {
  h.assign((size_t)std::max<int64_t>(n, 1), 0.0);
  if (n <= 0 || dry()) return LNOCC_OK;
  LN_TRY(hipMemcpyAsync(h.data(), d, (size_t)n * 8, hipMemcpyDeviceToHost, s));
  LN_TRY(hipStreamSynchronize(s));
  return LNOCC_OK;
}

int upload_ints(int *d, const std::vector<int> &h, hipStream_t s) {
  if (h.empty() || dry()) return LNOCC_OK;
  if (!region_ok(d, h.size() * 4)) return LNOCC_EINVAL;
  LN_TRY(hipMemcpyAsync(d, h.data(), h.size() * 4, hipMemcpyHostToDevice, s));
  LN_TRY(hipStreamSynchronize(s));   // h may go out of scope after the return
  return LNOCC_OK;
}

}  // namespace

hipError_t sym_eig(double *A, double *V, double *w, int n, int *scratch, hipStream_t s) {
  if (n < 1 || dry()) return hipSuccess;
  if (n > kEigMax) {
    note_error("eigenproblem of order %d above the supported %d", n, kEigMax);
    return hipErrorInvalidValue;
  }
  const size_t nn = (size_t)n * n * 8;
  if (!region_ok(A, nn) || !region_ok(V, nn) || !region_ok(w, (size_t)n * 8) ||
      !region_ok(scratch, (size_t)n * 4)) {
    note_error("eigensolver buffers (n = %d) outside the installed buffers; not launched", n);
    return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(kEigThreads), 0, s, A, V, w, n, 60, scratch);
  return hipGetLastError();
}

// ------------------------------------------------------------------ scratch plan
namespace {
// P-block of the canonical ov transform: Lx holds pb N nv <= X no nv elements
int64_t lov_block(int64_t no, int64_t nv, int64_t X) {
  return std::max<int64_t>(1, std::min<int64_t>(X, X * no / (no + nv)));
}
}  // namespace

void plan_lno_scratch(int64_t no, int64_t nv, int64_t X, int64_t nlo, int cbno, char *base,
                      LnoScratch &S) {
  Arena A{base};
  const int64_t N = no + nv;
  const int64_t ni = std::min(nlo, no), nvi = std::min(nlo, nv);
  S.Lov = A.d(X * no * nv);
  S.lx_elems = std::max(lov_block(no, nv, X) * N * nv, X * no * nv);
  S.Lx = A.d(S.lx_elems);
  S.M = A.d(N * N); S.V = A.d(N * N); S.w = A.d(N);
  S.tmp = A.d(N * N); S.tmp2 = A.d(N * N); S.D3 = A.d(N * N);
  S.Dij = A.d(no * no); S.Dab = A.d(nv * nv);
  S.Wo = A.d(no * no); S.Wv = A.d(nv * nv);
  S.t_elems = cbno ? std::max(no * nvi * no * nvi, ni * nv * ni * nv) : ni * nv * no * nv;
  S.t = A.d(S.t_elems); S.t2 = A.d(S.t_elems);
  S.idx = (int *)A.d((N + 1) / 2);
  S.bytes = A.off + 256;
}

// ------------------------------------------------------------------ steps
namespace {

// Internal / external orbitals of U [n][m] (Eqs. 18-19).  Internal columns
// (compact, leading dimension n_int) go to Wint, external ones (leading
// dimension n - n_int) to Wext, each in ascending order of the eigenvalues of
// U U^T; eigenvalues above 1e-10 max(1, largest) count as non-zero.
int split(const double *U, int64_t n, int64_t m, const LnoScratch &S, int &n_int, double *Wint,
          double *Wext, hipStream_t s) {
  n_int = 0;
  if (!U || m == 0) {
    if (!dry()) {
      if (!region_ok(Wext, (size_t)n * n * 8)) return LNOCC_EINVAL;
      hipLaunchKernelGGL(k_identity, dim3(ew_grid(n * n)), dim3(kEw), 0, s, Wext, n);
      LN_TRY(hipGetLastError());
    }
    return LNOCC_OK;
  }
  LN_TRY(mm(n, n, m, 1.0, U, m, 1, U, 1, m, 0.0, S.M, n, 1, s));   // U U^T
  LN_TRY(sym_eig(S.M, S.V, S.w, (int)n, S.idx, s));
  std::vector<double> w;
  LN_ST(read_back(S.w, n, w, s));
  const double wmax = std::max(1.0, w[n - 1]);
  for (int64_t i = 0; i < n; ++i) n_int += w[i] > 1e-10 * wmax;
  if (dry()) n_int = (int)std::min(m, n);
  const int64_t next = n - n_int;
  LN_TRY(gather_cols(S.V + next, n, n, nullptr, n_int, Wint, n_int, s));
  LN_TRY(gather_cols(S.V, n, n, nullptr, next, Wext, next, s));
  return LNOCC_OK;
}

// Rotate W [n][k] (compact, in place) so that W^T diag(eps) W is diagonal; f[k]
// receives the diagonal, ascending.
int semicanonical(double *W, int64_t n, int64_t k, const double *eps, double *f,
                  const LnoScratch &S, hipStream_t s) {
  if (k == 0) return LNOCC_OK;
  if (!dry()) {
    if (!region_ok(S.tmp, (size_t)n * k * 8) || !region_ok(W, (size_t)n * k * 8)) {
      note_error("semi-canonical rotation outside the installed buffers");
      return LNOCC_EINVAL;
    }
    hipLaunchKernelGGL(k_scale_rows, dim3(ew_grid(n * k)), dim3(kEw), 0, s, W, eps, n, k, S.tmp);
    LN_TRY(hipGetLastError());
  }
  LN_TRY(mm(k, k, n, 1.0, W, 1, k, S.tmp, k, 1, 0.0, S.M, k, 1, s));   // W^T (eps W)
  LN_TRY(sym_eig(S.M, S.V, f, (int)k, S.idx, s));
  LN_TRY(mm(n, k, k, 1.0, W, k, 1, S.V, k, 1, 0.0, S.tmp, k, 1, s));   // W R
  if (!dry()) LN_TRY(hipMemcpyAsync(W, S.tmp, (size_t)n * k * 8, hipMemcpyDeviceToDevice, s));
  return LNOCC_OK;
}

// Lx[P][r][a] = sum_i W[i][r] Lov[P][i][a] (W compact [no][nr])
hipError_t occ_transform(const LnoScratch &S, int64_t no, int64_t nv, int64_t X, const double *W,
                         int64_t nr, hipStream_t s) {
  return left_mul_batched(nr, nv, no, W, 1, nr, S.Lov, nv, no * nv, S.Lx, nv, nr * nv, X, s);
}

// Eq. 20 from the canonical ov factors and the internal occupied orbitals Wo
// [no][ni] with energies fo:  t[k][a][j][b] (k internal), then
//   D_ij = 4 sum t[k][b][i][a] t[k][b][j][a] - 2 sum t[k][b][i][a] t[k][a][j][b]
//   D_ab = 2 sum (t[k][a][j][c] t[k][b][j][c] + t[k][c][j][a] t[k][c][j][b])
//          - (Y + Y^T),  Y[a][b] = sum t[k][c][j][a] t[k][b][j][c]
// (sums over every index but the two free ones).
int lno_density(const LnoScratch &S, int64_t no, int64_t nv, int64_t X, const double *Wo,
                const double *fo, int64_t ni, const double *eo, const double *ev, hipStream_t s) {
  if (ni == 0) {
    LN_TRY(zero(S.Dij, no * no, s));
    LN_TRY(zero(S.Dab, nv * nv, s));
    return LNOCC_OK;
  }
  LN_TRY(occ_transform(S, no, nv, X, Wo, ni, s));
  // (k a|j b) = sum_P Lx[P][k][a] Lov[P][j][b]
  LN_TRY(mm(ni * nv, no * nv, X, 1.0, S.Lx, 1, ni * nv, S.Lov, no * nv, 1, 0.0, S.t, no * nv, 1, s));
  const int64_t n4 = ni * nv * no * nv;
  if (!dry()) {
    if (!region_ok(S.t, (size_t)n4 * 8) || !region_ok(S.t2, (size_t)n4 * 8)) return LNOCC_EINVAL;
    hipLaunchKernelGGL(k_mp1_divide, dim3(ew_grid(n4)), dim3(kEw), 0, s, S.t, ni, nv, no, fo, eo,
                       ev, 0);
    hipLaunchKernelGGL(k_swap_pair, dim3(ew_grid(n4)), dim3(kEw), 0, s, S.t, ni, nv, no, S.t2);
    LN_TRY(hipGetLastError());
  }
  // element strides of t[k][a][j][b]
  const int64_t sk = nv * no * nv, sa = no * nv, sj = nv;
  {   // D_ij: rows i / j (stride nv), K = ((k, b) stride sa, a stride 1)
    GemmDesc d{};
    d.M = (int)no; d.Mi = 1; d.N = (int)no; d.Ni = 1; d.nseg = 2;
    d.seg[0].a = GOperand{S.t, sj, 0, sa, 1, 0, 0, 0, 0};
    d.seg[0].b = GOperand{S.t, sj, 0, sa, 1, 0, 0, 0, 0};
    d.seg[0].K = (int)(ni * nv * nv); d.seg[0].Ki = (int)nv; d.seg[0].scale = 4.0;
    d.seg[1].a = GOperand{S.t, sj, 0, sa, 1, 0, 0, 0, 0};
    d.seg[1].b = GOperand{S.t2, sj, 0, sa, 1, 0, 0, 0, 0};
    d.seg[1].K = (int)(ni * nv * nv); d.seg[1].Ki = (int)nv; d.seg[1].scale = -2.0;
    d.c = S.Dij; d.c_mo = no; d.c_no = 1;
    d.batch = 1; d.nb1 = 1; d.prec = Prec::F64;
    LN_TRY(gett(d, s));
  }
  {   // 2 (term1 + term2) into tmp
    GemmDesc d{};
    d.M = (int)nv; d.Mi = 1; d.N = (int)nv; d.Ni = 1; d.nseg = 2;
    // term1: rows a (stride sa), K = (k stride sk, (j, c) stride 1)
    d.seg[0].a = GOperand{S.t, sa, 0, sk, 1, 0, 0, 0, 0};
    d.seg[0].b = GOperand{S.t, sa, 0, sk, 1, 0, 0, 0, 0};
    d.seg[0].K = (int)(ni * no * nv); d.seg[0].Ki = (int)(no * nv); d.seg[0].scale = 2.0;
    // term2: rows a (stride 1), K = ((k, c) stride sa, j stride sj)
    d.seg[1].a = GOperand{S.t, 1, 0, sa, sj, 0, 0, 0, 0};
    d.seg[1].b = GOperand{S.t, 1, 0, sa, sj, 0, 0, 0, 0};
    d.seg[1].K = (int)(ni * nv * no); d.seg[1].Ki = (int)no; d.seg[1].scale = 2.0;
    d.c = S.tmp; d.c_mo = nv; d.c_no = 1;
    d.batch = 1; d.nb1 = 1; d.prec = Prec::F64;
    LN_TRY(gett(d, s));
  }
  {   // Y[a][b] = sum t[k][c][j][a] t2[k][c][j][b] into D3
    GemmDesc d{};
    d.M = (int)nv; d.Mi = 1; d.N = (int)nv; d.Ni = 1; d.nseg = 1;
    d.seg[0].a = GOperand{S.t, 1, 0, sa, sj, 0, 0, 0, 0};
    d.seg[0].b = GOperand{S.t2, 1, 0, sa, sj, 0, 0, 0, 0};
    d.seg[0].K = (int)(ni * nv * no); d.seg[0].Ki = (int)no; d.seg[0].scale = 1.0;
    d.c = S.D3; d.c_mo = nv; d.c_no = 1;
    d.batch = 1; d.nb1 = 1; d.prec = Prec::F64;
    LN_TRY(gett(d, s));
  }
  if (!dry()) {
    if (!region_ok(S.Dab, (size_t)nv * nv * 8)) return LNOCC_EINVAL;
    hipLaunchKernelGGL(k_sub_sym, dim3(ew_grid(nv * nv)), dim3(kEw), 0, s, S.Dab, S.tmp, S.D3, nv);
    LN_TRY(hipGetLastError());
  }
  return LNOCC_OK;
}

// Eq. 28 (internal occupied Wo/fo [ni] compact, internal virtuals Wv/fv [nvi] compact):
//   D_ij = 4 sum t[i][A][k][B] t[j][A][k][B] - 2 sum t[i][A][k][B] t[j][B][k][A]
//          with t[i][A][k][B] over internal virtuals A, B;
//   D_ab = 4 sum t[I][a][J][c] t[I][b][J][c] - 2 sum t[I][a][J][c] t[I][c][J][b]
//          with t[I][a][J][c] over internal occupied I, J.
int cbno_density(const LnoScratch &S, int64_t no, int64_t nv, int64_t X, const double *Wo,
                 const double *fo, int64_t ni, const double *Wv, const double *fv, int64_t nvi,
                 const double *eo, const double *ev, hipStream_t s) {
  LN_TRY(zero(S.Dij, no * no, s));
  LN_TRY(zero(S.Dab, nv * nv, s));
  if (nvi > 0) {
    // Lx[P][i][A] = sum_a Lov[P][i][a] Wv[a][A]: one product over the (P, i) rows
    LN_TRY(mm(X * no, nvi, nv, 1.0, S.Lov, nv, 1, Wv, nvi, 1, 0.0, S.Lx, nvi, 1, s));
    const int64_t R = no * nvi, n4 = R * R;
    LN_TRY(mm(R, R, X, 1.0, S.Lx, 1, R, S.Lx, R, 1, 0.0, S.t, R, 1, s));
    if (!dry()) {
      if (!region_ok(S.t, (size_t)n4 * 8) || !region_ok(S.t2, (size_t)n4 * 8)) return LNOCC_EINVAL;
      hipLaunchKernelGGL(k_mp1_divide, dim3(ew_grid(n4)), dim3(kEw), 0, s, S.t, no, nvi, no, fv,
                         eo, nullptr, 1);
      hipLaunchKernelGGL(k_swap_pair, dim3(ew_grid(n4)), dim3(kEw), 0, s, S.t, no, nvi, no, S.t2);
      LN_TRY(hipGetLastError());
    }
    const int64_t K = nvi * no * nvi;
    LN_TRY(mm(no, no, K, 4.0, S.t, K, 1, S.t, 1, K, 0.0, S.Dij, no, 1, s));
    LN_TRY(mm(no, no, K, -2.0, S.t, K, 1, S.t2, 1, K, 1.0, S.Dij, no, 1, s));
  }
  if (ni > 0) {
    LN_TRY(occ_transform(S, no, nv, X, Wo, ni, s));
    const int64_t R = ni * nv, n4 = R * R;
    LN_TRY(mm(R, R, X, 1.0, S.Lx, 1, R, S.Lx, R, 1, 0.0, S.t, R, 1, s));
    if (!dry()) {
      if (!region_ok(S.t, (size_t)n4 * 8) || !region_ok(S.t2, (size_t)n4 * 8)) return LNOCC_EINVAL;
      hipLaunchKernelGGL(k_mp1_divide, dim3(ew_grid(n4)), dim3(kEw), 0, s, S.t, ni, nv, ni, fo,
                         nullptr, ev, 2);
      hipLaunchKernelGGL(k_swap_pair, dim3(ew_grid(n4)), dim3(kEw), 0, s, S.t, ni, nv, ni, S.t2);
      LN_TRY(hipGetLastError());
    }
    // rows a (stride ni nv), K = (I stride nv ni nv, (J, c) stride 1)
    GemmDesc d{};
    d.M = (int)nv; d.Mi = 1; d.N = (int)nv; d.Ni = 1; d.nseg = 2;
    d.seg[0].a = GOperand{S.t, R, 0, nv * R, 1, 0, 0, 0, 0};
    d.seg[0].b = GOperand{S.t, R, 0, nv * R, 1, 0, 0, 0, 0};
    d.seg[0].K = (int)(ni * R); d.seg[0].Ki = (int)R; d.seg[0].scale = 4.0;
    d.seg[1].a = GOperand{S.t, R, 0, nv * R, 1, 0, 0, 0, 0};
    d.seg[1].b = GOperand{S.t2, R, 0, nv * R, 1, 0, 0, 0, 0};
    d.seg[1].K = (int)(ni * R); d.seg[1].Ki = (int)R; d.seg[1].scale = -2.0;
    d.c = S.Dab; d.c_mo = nv; d.c_no = 1;
    d.batch = 1; d.nb1 = 1; d.prec = Prec::F64;
    LN_TRY(gett(d, s));
  }
  return LNOCC_OK;
}

// Eqs. 24-26: Dbar = Wext^T D Wext [next][next], eigenpairs by descending
// |lambda|; the n_keep with |lambda| >= eta become columns off .. off + n_keep - 1
// of out (leading dimension ldo) as Wext X.  lambda_out (may be null) receives
// every eigenvalue in that order.
int select_lnos(const double *D, int64_t n, const double *Wext, int64_t next, double eta,
                const LnoScratch &S, double *out, int64_t ldo, int64_t off, double *lambda_out,
                int &n_keep, hipStream_t s) {
  n_keep = 0;
  if (next == 0) return LNOCC_OK;
  LN_TRY(mm(n, next, n, 1.0, D, n, 1, Wext, next, 1, 0.0, S.tmp, next, 1, s));         // D Wext
  LN_TRY(mm(next, next, n, 1.0, Wext, 1, next, S.tmp, next, 1, 0.0, S.M, next, 1, s));  // Wext^T .
  LN_TRY(sym_eig(S.M, S.V, S.w, (int)next, S.idx, s));
  std::vector<double> w;
  LN_ST(read_back(S.w, next, w, s));
  std::vector<int> order(next);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return std::fabs(w[a]) > std::fabs(w[b]); });
  for (int64_t c = 0; c < next; ++c) n_keep += std::fabs(w[order[c]]) >= eta;
  if (dry()) n_keep = (int)next;
  LN_ST(upload_ints(S.idx, order, s));
  if (lambda_out && !dry()) {
    if (!region_ok(lambda_out, (size_t)next * 8)) return LNOCC_EINVAL;
    hipLaunchKernelGGL(k_gather, dim3(ew_grid(next)), dim3(kEw), 0, s, S.w, S.idx, next,
                       lambda_out);
    LN_TRY(hipGetLastError());
  }
  LN_TRY(gather_cols(S.V, next, next, S.idx, n_keep, S.M, n_keep, s));
  LN_TRY(mm(n, n_keep, next, 1.0, Wext, next, 1, S.M, n_keep, 1, 0.0, out + off, ldo, 1, s));
  return LNOCC_OK;
}

}  // namespace

int local_space(const LnoSystem &sys, const double *U_occ, const double *U_vir, int64_t nlo,
                double eta_occ, double eta_vir, int cbno, const LnoScratch &S, LnoSpace &out,
                hipStream_t s) {
  const int64_t no = sys.no, nv = sys.nv, X = sys.X, N = no + nv;
  // canonical ov factors, P in blocks:
  //   Lx[P][mu][a] = sum_nu L[P][mu][nu] C[nu][no + a];  Lov[P][i][a] = sum_mu C[mu][i] Lx[P][mu][a]
  const int64_t pb = lov_block(no, nv, X);
  for (int64_t P0 = 0; P0 < X; P0 += pb) {
    const int64_t np = std::min(pb, X - P0);
    LN_TRY(right_mul_batched(N, nv, N, sys.Lao + P0 * N * N, N, N * N, sys.C + no, N, 1, S.Lx, nv,
                             N * nv, np, s));
    LN_TRY(left_mul_batched(no, nv, N, sys.C, 1, N, S.Lx, nv, N * nv, S.Lov + P0 * no * nv, nv,
                            no * nv, np, s));
  }
  // 1-2. internal orbitals (compact in tmp2 / D3 until the density step) and
  //      the external bases Wo / Wv
  int nio = 0, niv = 0;
  double *Io = S.tmp2, *Iv = S.D3;
  LN_ST(split(U_occ, no, nlo, S, nio, Io, S.Wo, s));
  LN_ST(split(U_vir, nv, U_vir ? nlo : 0, S, niv, Iv, S.Wv, s));
  LN_ST(semicanonical(Io, no, nio, sys.eo, out.eps_occ, S, s));
  LN_ST(semicanonical(Iv, nv, niv, sys.ev, out.eps_vir, S, s));
  // 3-4. densities
  if (cbno) {
    LN_ST(cbno_density(S, no, nv, X, Io, out.eps_occ, nio, Iv, out.eps_vir, niv, sys.eo, sys.ev, s));
    LN_TRY(gather_cols(Iv, nv, niv, nullptr, niv, out.C_vir, nv, s));
  } else {
    // lno_density uses D3 as scratch: the internal virtuals (no part of Eq. 20)
    // move to their place in C_vir first
    LN_TRY(gather_cols(Iv, nv, niv, nullptr, niv, out.C_vir, nv, s));
    LN_ST(lno_density(S, no, nv, X, Io, out.eps_occ, nio, sys.eo, sys.ev, s));
  }
  LN_TRY(gather_cols(Io, no, nio, nullptr, nio, out.C_occ, no, s));
  // 5. LNO selection, after the internal columns
  int nko = 0, nkv = 0;
  LN_ST(select_lnos(S.Dij, no, S.Wo, no - nio, eta_occ, S, out.C_occ, no, nio, out.lambda_occ,
                    nko, s));
  LN_ST(select_lnos(S.Dab, nv, S.Wv, nv - niv, eta_vir, S, out.C_vir, nv, niv, out.lambda_vir,
                    nkv, s));
  out.n_int_occ = nio;
  out.n_int_vir = niv;
  out.n_occ = nio + nko;
  out.n_vir = niv + nkv;
  // 6. semi-canonical active orbitals (compact copies in tmp2)
  auto finish = [&](double *Cf, int64_t rows, int64_t k, const double *eps, double *ef) -> int {
    if (k == 0) return LNOCC_OK;
    LN_TRY(gather_cols(Cf, rows, rows, nullptr, k, S.tmp2, k, s));
    LN_ST(semicanonical(S.tmp2, rows, k, eps, ef, S, s));
    LN_TRY(gather_cols(S.tmp2, rows, k, nullptr, k, Cf, rows, s));
    return LNOCC_OK;
  };
  LN_ST(finish(out.C_occ, no, out.n_occ, sys.eo, out.eps_occ));
  LN_ST(finish(out.C_vir, nv, out.n_vir, sys.ev, out.eps_vir));
  // the fragment's LOs on the active occupied orbitals: U_act = C_occ^T U_occ
  if (out.U_act)
    LN_TRY(mm(out.n_occ, nlo, no, 1.0, out.C_occ, 1, no, U_occ, nlo, 1, 0.0, out.U_act, nlo, 1, s));
  return LNOCC_OK;
}

// ------------------------------------------------------------------ Eq. 27b
namespace {
// P-block of the AO half transform: pb N na <= max(X na na, N na) elements
int64_t ham_block(int64_t N, int64_t X, int64_t na) {
  return std::max<int64_t>(1, std::min<int64_t>(X, X * na / std::max<int64_t>(N, 1)));
}
}  // namespace

size_t local_hamiltonian_bytes(int64_t no, int64_t nv, int64_t X, int64_t n_occ, int64_t n_vir) {
  const int64_t N = no + nv, na = n_occ + n_vir;
  Arena A{nullptr};
  A.d(N * na);
  A.d(ham_block(N, X, na) * N * na);
  return A.off + 256;
}

int local_hamiltonian(const LnoSystem &sys, const double *C_occ, int64_t n_occ,
                      const double *C_vir, int64_t n_vir, char *ws, size_t ws_bytes, double *B,
                      hipStream_t s) {
  const int64_t no = sys.no, nv = sys.nv, X = sys.X, N = no + nv, na = n_occ + n_vir;
  if (ws_bytes < local_hamiltonian_bytes(no, nv, X, n_occ, n_vir)) return LNOCC_ENOMEM;
  Arena A{ws};
  double *Cact = A.d(N * na);
  const int64_t pb = ham_block(N, X, na);
  double *Lx = A.d(pb * N * na);
  // Cact [N][na] = [C[:, :no] C_occ[:, :n_occ] | C[:, no:] C_vir[:, :n_vir]]
  LN_TRY(mm(N, n_occ, no, 1.0, sys.C, N, 1, C_occ, no, 1, 0.0, Cact, na, 1, s));
  LN_TRY(mm(N, n_vir, nv, 1.0, sys.C + no, N, 1, C_vir, nv, 1, 0.0, Cact + n_occ, na, 1, s));
  // B[P][p][q] = sum_mu Cact[mu][p] sum_nu L[P][mu][nu] Cact[nu][q]
  for (int64_t P0 = 0; P0 < X; P0 += pb) {
    const int64_t np = std::min(pb, X - P0);
    LN_TRY(right_mul_batched(N, na, N, sys.Lao + P0 * N * N, N, N * N, Cact, na, 1, Lx, na,
                             N * na, np, s));
    LN_TRY(left_mul_batched(na, na, N, Cact, 1, na, Lx, na, N * na, B + P0 * na * na, na, na * na,
                            np, s));
  }
  return LNOCC_OK;
}

// ------------------------------------------------------------------ MP2
size_t mp2_bytes(int64_t o, int64_t v, bool with_t2) {
  Arena A{nullptr};
  A.d(kRedBlocks);   // partials
  A.d(1);            // energy
  if (!with_t2) A.d(o * v * v);
  return A.off + 256;
}

int fragment_mp2(const double *B, const double *eo, const double *ev, int64_t o, int64_t v,
                 int64_t X, double *t1, double *t2, char *ws, size_t ws_bytes, double *e_mp2,
                 hipStream_t s) {
  const int64_t N = o + v, row = o * v * v;
  if (ws_bytes < mp2_bytes(o, v, t2 != nullptr)) return LNOCC_ENOMEM;
  Arena A{ws};
  double *partials = A.d(kRedBlocks);
  double *e_dev = A.d(1);
  int64_t bi = o;
  double *Vb = t2;
  if (!t2) {   // as many i rows per block as the workspace holds
    const size_t used = ((A.off + 255) & ~size_t(255)) + 256;
    bi = std::max<int64_t>(1, std::min<int64_t>(o, (int64_t)((ws_bytes - used) / (row * 8))));
    Vb = A.d(bi * row);
  }
  if (t1) LN_TRY(zero(t1, o * v, s));
  for (int64_t i0 = 0; i0 < o; i0 += bi) {
    const int64_t nb = std::min(bi, o - i0);
    double *V = t2 ? t2 + i0 * row : Vb;
    GemmDesc d{};   // (i a|j b) for the block's i: rows (i, a), columns (j, b), K = P
    d.M = (int)(nb * v); d.Mi = (int)v; d.N = (int)(o * v); d.Ni = (int)v; d.nseg = 1;
    d.seg[0].a = GOperand{B + i0 * N + o, N, 1, N * N, 0, 0, 0, 0, 0};
    d.seg[0].b = GOperand{B + o, N, 1, N * N, 0, 0, 0, 0, 0};
    d.seg[0].K = (int)X; d.seg[0].Ki = 1; d.seg[0].scale = 1.0;
    d.c = V; d.c_mo = row; d.c_mi = v; d.c_no = v * v; d.c_ni = 1;
    d.batch = 1; d.nb1 = 1; d.prec = Prec::F64;
    LN_TRY(gett(d, s));
    if (!dry()) {
      if (!region_ok(V, (size_t)nb * row * 8) || !region_ok(partials, kRedBlocks * 8))
        return LNOCC_EINVAL;
      hipLaunchKernelGGL(k_mp2_block, dim3(kRedBlocks), dim3(kRedThreads), 0, s, V, nb, i0, o, v,
                         eo, ev, partials);
      LN_TRY(hipGetLastError());
      LN_TRY(reduce_partials(partials, kRedBlocks, e_dev, i0 > 0, s));
    }
  }
  std::vector<double> h;
  LN_ST(read_back(e_dev, 1, h, s));
  *e_mp2 = h[0];
  return LNOCC_OK;
}

}  // namespace lnocc

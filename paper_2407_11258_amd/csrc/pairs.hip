// Fragment pair energies (Sec. II.B) and their projection onto localized
// orbitals.
//
//   E[i][i']   = sum_{j a b} tau_ij^ab (2 (i'a|jb) - (i'b|ja)),  tau = t2 + t1 t1  (Eqs. 9, 13)
//   E_T[i][i'] = -1/3 sum_{j k a b c} (4 w_ijk^abc + w_ijk^bca + w_ijk^cab)
//                                     (v_i'jk^abc - v_i'jk^cba)                    (Eq. 16)
//   e[alpha]   = sum_{i i'} U[i][alpha] E[i][i'] U[i'][alpha]                     (Eqs. 12, 15)
// with w = W / sqrt(-Delta_ijk), v_i'jk = V_i'jk / sqrt(-Delta_i'jk) (SI Sec. S1).
//
// E is one product over (j, a, b).  For E_T, i and i' meet only through a
// common (j, k): for each pair j <= k the W tensors of the o ordered triples
// (i, j, k) are formed by the W kernel of (T), turned into
//   Y[i] = (4 W + W^bca + W^cab) / sqrt(-Delta_ijk)  and
//   Z[i] = (c1 V - V^cba - c2 V^bac) / sqrt(-Delta_ijk),
// and E_T += -1/3 Y Z^T, a product over the v^3 virtual triples.  The ordered
// pair (k, j) gives the same terms with b and c exchanged (W_ikj^acb = W_ijk^abc),
// so j < k takes c1 = 2, c2 = 1 and j = k takes c1 = 1, c2 = 0.
#include "pairs.h"

#include <algorithm>
#include <cmath>

#include "gett.h"
#include "kernels.h"
#include "triples.h"

namespace lnocc {
namespace {

constexpr int kThreads = 256;

inline int blocks_for(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + kThreads - 1) / kThreads, 16384));
}

// table[3 (p o + i) + {0,1,2}] = (i, j, k) for the p-th pair j <= k (lexicographic)
__global__ void k_pair_table(int *table, int o) {
  const int64_t npair = (int64_t)o * (o + 1) / 2;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < npair * o;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t p = e / o;
    const int i = (int)(e % o);
    int j = 0;
    while (p >= o - j) { p -= o - j; ++j; }
    table[3 * e] = i;
    table[3 * e + 1] = j;
    table[3 * e + 2] = j + (int)p;
  }
}

// tau[i][j][a][b] = t2 + t1[i][a] t1[j][b];  Lx[i][j][a][b] = 2 (ia|jb) - (ib|ja)
__global__ void k_tau_l(const double *__restrict__ t1, const double *__restrict__ t2,
                        const double *__restrict__ Kov, int64_t o, int64_t v,
                        double *__restrict__ tau, double *__restrict__ Lx) {
  const int64_t n = o * o * v * v;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e % v, a = (e / v) % v, j = (e / (v * v)) % o, i = e / (o * v * v);
    tau[e] = t2[e] + t1[i * v + a] * t1[j * v + b];
    Lx[e] = 2.0 * Kov[((i * v + a) * o + j) * v + b] - Kov[((i * v + b) * o + j) * v + a];
  }
}

// Y and Z of the pair (j, k) for every i (see the file comment).
__global__ void k_pair_yz(const double *__restrict__ W, const double *__restrict__ Kov,
                          const double *__restrict__ t1, const double *__restrict__ eo,
                          const double *__restrict__ ev, int64_t o, int64_t v, int j, int k,
                          double *__restrict__ Y, double *__restrict__ Z) {
  const int64_t vvv = v * v * v, n = o * vvv;
  const double c1 = j < k ? 2.0 : 1.0, c2 = j < k ? 1.0 : 0.0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / vvv, r = e % vvv;
    const int64_t a = r / (v * v), b = (r / v) % v, c = r % v;
    const double *Wi = W + i * vvv;
    auto w = [&](int64_t x, int64_t y, int64_t z) { return Wi[(x * v + y) * v + z]; };
    // (xi|yj) t_k^z + (xi|zk) t_j^y + (yj|zk) t_i^x
    auto d = [&](int64_t x, int64_t y, int64_t z) {
      return Kov[((i * v + x) * o + j) * v + y] * t1[k * v + z] +
             Kov[((i * v + x) * o + k) * v + z] * t1[j * v + y] +
             Kov[((j * v + y) * o + k) * v + z] * t1[i * v + x];
    };
    const double s = 1.0 / std::sqrt(-(eo[i] + eo[j] + eo[k] - ev[a] - ev[b] - ev[c]));
    Y[e] = (4.0 * w(a, b, c) + w(b, c, a) + w(c, a, b)) * s;
    const double vabc = w(a, b, c) + d(a, b, c), vcba = w(c, b, a) + d(c, b, a);
    const double vbac = c2 != 0.0 ? w(b, a, c) + d(b, a, c) : 0.0;
    Z[e] = (c1 * vabc - vcba - c2 * vbac) * s;
  }
}

// out[alpha] = sum_{i i'} U[i][alpha] E[i][i'] U[i'][alpha]; one thread per alpha
__global__ void k_project(const double *__restrict__ E, const double *__restrict__ U, int o,
                          int nlo, double *__restrict__ out) {
  const int al = blockIdx.x * blockDim.x + threadIdx.x;
  if (al >= nlo) return;
  double acc = 0.0;
  for (int i = 0; i < o; ++i) {
    double row = 0.0;
    for (int ip = 0; ip < o; ++ip) row += E[i * o + ip] * U[(int64_t)ip * nlo + al];
    acc += U[(int64_t)i * nlo + al] * row;
  }
  out[al] = acc;
}

#define PR_TRY(x)                                                         \
  do {                                                                    \
    hipError_t e_ = (x);                                                  \
    if (e_ != hipSuccess) {                                               \
      note_error("%s failed (%s) at %s:%d", #x, hipGetErrorString(e_),    \
                 __FILE__, __LINE__);                                     \
      return LNOCC_EDEVICE;                                               \
    }                                                                     \
  } while (0)

}  // namespace

void plan_pair_layout(const Dims &dm, char *base, Layout &L, size_t &bytes) {
  const int64_t o = dm.o, v = dm.v, oo = o * o, vvv = v * v * v;
  const int64_t vp = triples_pad(v);
  size_t off = L.phase_off;
  auto d = [&](int64_t n) {
    off = (off + 255) & ~size_t(255);
    double *p = base ? (double *)(base + off) : nullptr;
    off += (size_t)n * sizeof(double);
    return p;
  };
  PairLayout &P = L.pairs;
  P.Gt = d(o * v * v * vp);
  P.Jt = d(oo * o * v);
  P.T = d(oo * v * vp);
  P.table = (int *)d((3 * o * (oo + o) / 2 + 1) / 2);
  P.W = d(o * vvv);
  P.Y = d(o * vvv);
  P.Z = d(o * vvv);
  P.tau = d(oo * v * v);
  P.Lx = d(oo * v * v);
  bytes = std::max(L.bytes, off + 256);
}

int pair_energies(const Layout &L, const double *t1, const double *t2, const double *eo,
                  const double *ev, double *Ecc, double *Et, const double *U, int nlo,
                  double *pcc, double *pt, hipStream_t s) {
  const int64_t o = L.dm.o, v = L.dm.v, X = L.dm.X, ov = o * v, oo = o * o, vv = v * v;
  const int64_t vvv = vv * v, vp = triples_pad(v);
  const PairLayout &P = L.pairs;
  const bool dry = dry_run();
  // CCSD: E[i][i'] = sum_{(j,a,b)} tau[i][(j,a,b)] Lx[i'][(j,a,b)]
  if (!dry) {
    hipLaunchKernelGGL(k_tau_l, dim3(blocks_for(oo * vv)), dim3(kThreads), 0, s, t1, t2, L.Kov,
                       o, v, P.tau, P.Lx);
    PR_TRY(hipGetLastError());
  }
  {
    GemmDesc d = gemm_desc((int)o, (int)o, (int)(o * vv), 1.0, P.tau, o * vv, 1, P.Lx, 1, o * vv,
                           0.0, Ecc, o, 1);
    PR_TRY(gett(d, s));
  }
  if (Et) {
    if (v * v * vp * 8 >= ((int64_t)1 << 32)) {
      note_error("pair (T): nvir %lld is beyond the 32-bit offsets of the W kernel", (long long)v);
      return LNOCC_EINVAL;
    }
    // (T) operands in FP64 (G and T padded along d, as the W kernel reads them)
    if (vp > v && !dry) PR_TRY(hipMemsetAsync(P.Gt, 0, (size_t)(ov * v * vp * 8), s));
    {
      GemmDesc d{};
      d.M = (int)ov; d.Mi = 1; d.N = (int)vv; d.Ni = (int)v;
      d.nseg = 1;
      d.seg[0].a = GOperand{L.Bov, 1, 0, ov, 0, 0, 0, 0, 0};
      d.seg[0].b = GOperand{L.Bvv, v, 1, vv, 0, 0, 0, 0, 0};
      d.seg[0].K = (int)X; d.seg[0].Ki = 1; d.seg[0].scale = 1.0;
      d.c = P.Gt; d.c_mo = v * vp; d.c_mi = 0; d.c_no = vp; d.c_ni = 1;
      d.batch = 1; d.nb1 = 1; d.prec = Prec::F64;
      PR_TRY(gett(d, s));
    }
    {  // Jt[j][k][c][l] = (ck|jl)
      GemmDesc d{};
      d.M = (int)ov; d.Mi = (int)v; d.N = (int)oo; d.Ni = (int)o;
      d.nseg = 1;
      d.seg[0].a = GOperand{L.Bov, v, 1, ov, 0, 0, 0, 0, 0};
      d.seg[0].b = GOperand{L.Boo, o, 1, oo, 0, 0, 0, 0, 0};
      d.seg[0].K = (int)X; d.seg[0].Ki = 1; d.seg[0].scale = 1.0;
      d.c = P.Jt; d.c_mo = v * o; d.c_mi = o; d.c_no = ov * o; d.c_ni = 1;
      d.batch = 1; d.nb1 = 1; d.prec = Prec::F64;
      PR_TRY(gett(d, s));
    }
    PR_TRY(triples_pad_t2(t2, o, v, P.T, 0, s));
    if (!dry) {
      hipLaunchKernelGGL(k_pair_table, dim3(blocks_for(o * (oo + o) / 2)), dim3(kThreads), 0, s,
                         P.table, (int)o);
      PR_TRY(hipGetLastError());
      PR_TRY(hipMemsetAsync(Et, 0, (size_t)oo * 8, s));
    }
    int64_t pidx = 0;
    for (int j = 0; j < o; ++j)
      for (int k = j; k < o; ++k, ++pidx) {
        const int *table = P.table + 3 * pidx * o;
        for (int ori = 0; ori < 3; ++ori)
          PR_TRY(triples_w(P.Gt, P.T, P.Jt, P.W, table, (int)o, o, v, ori, 0, ori > 0, 2, 0, s));
        if (!dry) {
          hipLaunchKernelGGL(k_pair_yz, dim3(blocks_for(o * vvv)), dim3(kThreads), 0, s, P.W,
                             L.Kov, t1, eo, ev, o, v, j, k, P.Y, P.Z);
          PR_TRY(hipGetLastError());
        }
        GemmDesc d = gemm_desc((int)o, (int)o, (int)vvv, -1.0 / 3.0, P.Y, vvv, 1, P.Z, 1, vvv,
                               1.0, Et, o, 1);
        PR_TRY(gett(d, s));
      }
  }
  if (U && nlo > 0 && !dry) {
    const int blocks = (nlo + 63) / 64;
    hipLaunchKernelGGL(k_project, dim3(blocks), dim3(64), 0, s, Ecc, U, (int)o, nlo, pcc);
    if (Et && pt) hipLaunchKernelGGL(k_project, dim3(blocks), dim3(64), 0, s, Et, U, (int)o, nlo, pt);
    PR_TRY(hipGetLastError());
  }
  return LNOCC_OK;
}

}  // namespace lnocc

// W contraction of (T) (SI Sec. S1) for a batch of unique triples on the
// gfx950 matrix cores.
//
// For a triple (i, j, k) the tensor W[a][b][c] is the sum of six particle and
// six hole terms.  Grouped by which virtual index the amplitude carries, they
// form three orientations; in orientation o the output is addressed by a row
// pair (m1, m2) and a column n, and with (p, q, r) the occupied labels taken in
// the orientation's order
//     o = 0: (m1, m2, n) = (a, b, c), (p, q, r) = (i, j, k)
//     o = 1: (m1, m2, n) = (a, c, b), (p, q, r) = (i, k, j)
//     o = 2: (m1, m2, n) = (b, c, a), (p, q, r) = (j, k, i)
// every orientation is the same four-term product
//     W[m1,m2,n] (+)= sum_d G[p][m1][m2][d] T[r][q][n][d] + sum_d G[q][m2][m1][d] T[r][p][n][d]
//                   - sum_l T[p][l][m1][m2] J[q][r][n][l] - sum_l T[q][l][m2][m1] J[p][r][n][l]
// with G[i][a][b][d] = (ai|bd), T[i][j][a][b] = t_ij^ab and J[j][k][c][l] = (ck|jl).
// The three orientations are three launches (the first overwrites W, the other
// two add to it).
//
// Kernel design.  A workgroup of four waves owns a 128 x 80 output tile (rows
// r = m1 v + m2, columns n); each wave holds 32 x 80 of it as 2 x 5 blocks of
// 16 x 16 matrix-op accumulators.  K runs through the four terms one after the
// other in slices of 16, staged through double-buffered LDS; the
// next slice is loaded into registers while the current one is multiplied.
// LDS tiles are [row][k] with a padded row (20 floats or 18 doubles), so that a
// lane's four k of one row are one (FP32) or two (FP64) 16-byte reads and the
// 16 rows read together fall on distinct banks.
// The particle operands are contiguous along d and are read as 16-byte vectors:
// G and T carry d padded with zeros to vp (a multiple of 4), so every vector is
// aligned and a slice past the end reads zeros.  The hole terms (K = nocc) are
// read element by element.  Row offsets are computed once per tile; inside the
// slice loop a load is a base pointer plus a fixed offset.  The finished tile is
// staged in LDS and written (or accumulated) along the contiguous index of W,
// so every orientation writes whole runs of memory.
#include "triples.h"

#include <algorithm>
#include <type_traits>

#include "gett.h"

namespace lnocc {
namespace {

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef double double2_t __attribute__((ext_vector_type(2)));

constexpr int kBN = 80, kBK = 16, kThreads = 256;
constexpr int kNI = 5;   // 16 x 16 blocks per wave along the 80 columns

// BM: rows of the output tile (BM / 4 per wave)
template <typename E, int BM> struct WTraits;
template <int BM> struct WTraits<float, BM> {
  using Acc = float4_t;
  using Vec = float4_t;
  static constexpr int VE = 4;          // elements per 16-byte vector
  static constexpr int LDK = kBK + 4;   // [row][k] tiles: 16 rows x 4 k of a read hit 64 banks
  static constexpr int CR = BM / 2;     // tile rows per pass of the output stage
  __device__ static Acc mma(float a, float b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lane, int r) { return 4 * (lane / 16) + r; }
};
template <int BM> struct WTraits<double, BM> {
  using Acc = double4_t;
  using Vec = double2_t;
  static constexpr int VE = 2;
  static constexpr int LDK = kBK + 2;
  static constexpr int CR = 64;         // passes of 64 rows keep the staged tile at 41 KB
  __device__ static Acc mma(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lane, int r) { return lane / 16 + 4 * r; }
};

// Particle loads: TPR threads share one row of a slice (one vector each).
template <typename E, int BM> struct PLoad {
  static constexpr int VE = WTraits<E, BM>::VE;
  static constexpr int TPR = kBK / VE;            // 4 (FP32) or 8 (FP64)
  static constexpr int RPP = kThreads / TPR;      // rows per pass: 64 or 32
  static constexpr int PA = BM / RPP;             // passes over the A tile
  static constexpr int PB = (kBN + RPP - 1) / RPP;   // passes over the B tile: 2 or 3
};
constexpr int kHB = kBN * kBK / kThreads;         // hole B elements per thread: 5
static_assert(kBN * kBK % kThreads == 0, "hole B share");

struct TripleArgs {
  const void *G;        // [o][v][v][vp]
  const void *T;        // [o][o][v][vp]
  const void *J;        // [o][o][v][o]
  void *W;              // [nb][v][v][v]
  const int *table;     // (i, j, k) of each batch entry
  int o, v, vp;
  int ori;
  int accumulate;       // 0: W = product; 1: W += product
  int nterms;           // 2: both particle and both hole terms; 1: the first of each
  int blocked;          // W layout: 0 plain [v][v][v], 1 blocked [v][vt][vt][8][8]
  int tiles_m, tiles_n;
};

// Output rows of a launch.  Orientation 2 in the blocked layout enumerates its
// (m1, m2) = (b, c) pairs in 8 x 8 blocks, (b % 8, c % 8) fastest, so that 64
// consecutive rows at one column a are one contiguous 64-element run of W; pairs
// with b or c >= v (padding) are computed from clamped rows and never stored.
__device__ inline bool blocked_rows(const TripleArgs &A) { return A.blocked && A.ori == 2; }
__device__ inline int64_t row_count(const TripleArgs &A) {
  const int64_t v = A.v, vt = (v + 7) / 8;
  return blocked_rows(A) ? vt * vt * 64 : v * v;
}
// (m1, m2) of row r; false for a padding row (then clamped into range)
__device__ inline bool row_pair(const TripleArgs &A, int64_t r, int64_t &m1, int64_t &m2) {
  const int64_t v = A.v;
  if (!blocked_rows(A)) {
    m1 = r / v;
    m2 = r % v;
    return true;
  }
  const int64_t vt = (v + 7) / 8, blk = r >> 6;
  m1 = (blk / vt) * 8 + ((r >> 3) & 7);
  m2 = (blk % vt) * 8 + (r & 7);
  const bool ok = m1 < v && m2 < v;
  m1 = min(m1, v - 1);
  m2 = min(m2, v - 1);
  return ok;
}

// Offset within one triple's W of index x in position role (0: a, 1: b, 2: c).
__device__ inline int64_t w_offset(const TripleArgs &A, int role, int64_t x) {
  const int64_t v = A.v;
  if (!A.blocked) return role == 0 ? x * v * v : role == 1 ? x * v : x;
  const int64_t vt = (v + 7) / 8;
  if (role == 0) return x * vt * vt * 64;
  if (role == 1) return (x >> 3) * vt * 64 + (x & 7) * 8;
  return (x >> 3) * 64 + (x & 7);
}

template <typename E, int BM>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2)))
void k_triples_w(TripleArgs A) {
  using Tr = WTraits<E, BM>;
  using P = PLoad<E, BM>;
  constexpr int kMI = BM / 64;            // 16-row blocks per wave
  constexpr int kHA = BM * kBK / kThreads;   // hole A elements per thread
  constexpr int KPP = kThreads / BM;      // hole A: k values per pass of the threads
  using Vec = typename Tr::Vec;
  constexpr int VE = Tr::VE;
  constexpr int LDK = Tr::LDK;
  constexpr int SZA = BM * LDK, SZB = kBN * LDK;
  constexpr int LDC = kBN + 1;
  constexpr int CR = Tr::CR;
  constexpr int STAGE = 2 * (SZA + SZB);
  constexpr int CT = CR * LDC;
  __shared__ __attribute__((aligned(16))) E smem[STAGE > CT ? STAGE : CT];
  __shared__ int64_t rowoff[BM], coloff[kBN];
  E *As = smem, *Bs = smem + 2 * SZA;

  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  int tm, tn;
  xcd_tile(blockIdx.x, A.tiles_m, A.tiles_n, tm, tn);
  const int64_t v = A.v, vp = A.vp, o = A.o, vv = v * v;
  const int64_t nrows = row_count(A);
  const int64_t r0 = (int64_t)tm * BM;
  const int n0 = tn * kBN;
  const int entry = blockIdx.y;
  const int ti = A.table[3 * entry], tj = A.table[3 * entry + 1], tk = A.table[3 * entry + 2];
  int p, q, r;
  if (A.ori == 0) { p = ti; q = tj; r = tk; }
  else if (A.ori == 1) { p = ti; q = tk; r = tj; }
  else { p = tj; q = tk; r = ti; }
  const E *G = (const E *)A.G;
  const E *T = (const E *)A.T;
  const E *J = (const E *)A.J;
  // bases of the four terms
  const E *gA[2] = {G + (int64_t)p * vv * vp, G + (int64_t)q * vv * vp};
  const E *gB[2] = {T + ((int64_t)r * o + q) * v * vp, T + ((int64_t)r * o + p) * v * vp};
  const E *hA[2] = {T + (int64_t)p * o * v * vp, T + (int64_t)q * o * v * vp};
  const E *hB[2] = {J + ((int64_t)q * o + r) * v * o, J + ((int64_t)p * o + r) * v * o};

  // Offsets that stay fixed for the whole tile.  Rows past the end of the output
  // (last row or column tile) are clamped to the last valid row: they read real
  // data and their results are never stored, so no mask is needed for them.
  const int kq = (t % P::TPR) * VE;   // first d of this thread's vectors in a slice
  // particle A rows: byte offsets of (m1 v + m2) vp + kq and (m2 v + m1) vp + kq
  uint32_t pa_flat[P::PA], pa_swap[P::PA];
#pragma unroll
  for (int s = 0; s < P::PA; ++s) {
    const int64_t gr = min(r0 + t / P::TPR + s * P::RPP, nrows - 1);
    int64_t m1, m2;
    row_pair(A, gr, m1, m2);
    pa_flat[s] = (uint32_t)(((m1 * v + m2) * vp + kq) * (int64_t)sizeof(E));
    pa_swap[s] = (uint32_t)(((m2 * v + m1) * vp + kq) * (int64_t)sizeof(E));
  }
  uint32_t pb_off[P::PB];
#pragma unroll
  for (int s = 0; s < P::PB; ++s) {
    const int n = min(n0 + t / P::TPR + s * P::RPP, A.v - 1);
    pb_off[s] = (uint32_t)(((int64_t)n * vp + kq) * (int64_t)sizeof(E));
  }
  // hole terms: element s of this thread is (row t % BM, k t / BM + KPP s) of A
  // and (row e % 80, k e / 80), e = t + 256 s, of B
  uint32_t ha_flat, ha_swap;
  {
    const int64_t gr = min(r0 + t % BM, nrows - 1);
    int64_t m1, m2;
    row_pair(A, gr, m1, m2);
    ha_flat = (uint32_t)(m1 * vp + m2);
    ha_swap = (uint32_t)(m2 * vp + m1);
  }
  uint32_t hb_off[kHB];
#pragma unroll
  for (int s = 0; s < kHB; ++s) {
    const int n = min(n0 + (t + kThreads * s) % kBN, A.v - 1);
    hb_off[s] = (uint32_t)((int64_t)n * o);
  }
  const uint32_t lstride = (uint32_t)(v * vp);   // T[.][l + 1] - T[.][l]

  typename Tr::Acc acc[kMI][kNI];
#pragma unroll
  for (int i = 0; i < kMI; ++i)
#pragma unroll
    for (int j = 0; j < kNI; ++j)
#pragma unroll
      for (int x = 0; x < 4; ++x) acc[i][j][x] = 0;

  const int sp = (A.vp + kBK - 1) / kBK;   // slices of one particle term
  const int sh = (A.o + kBK - 1) / kBK;    // slices of one hole term
  const int NP = A.nterms * sp;            // particle slices
  const int nslices = NP + A.nterms * sh;

  // registers of one slice in flight
  Vec va[P::PA], vb[P::PB];
  E ea[kHA], eb[kHB];
  auto vload = [](const char *base, uint32_t off) { return *(const Vec *)(base + off); };
  auto load = [&](int qs) {
    if (qs < NP) {       // particle term: 16-byte vectors along d
      const int term = qs < sp ? 0 : 1;
      const int k0 = (qs - term * sp) * kBK;
      const char *ba = (const char *)(gA[term] + k0), *bb = (const char *)(gB[term] + k0);
      if (k0 + kBK <= A.vp) {   // whole slice inside the padded rows
        if (term == 0) {
#pragma unroll
          for (int s = 0; s < P::PA; ++s) va[s] = vload(ba, pa_flat[s]);
        } else {
#pragma unroll
          for (int s = 0; s < P::PA; ++s) va[s] = vload(ba, pa_swap[s]);
        }
#pragma unroll
        for (int s = 0; s < P::PB; ++s) vb[s] = vload(bb, pb_off[s]);
      } else {                  // last slice: vectors past vp read as zero
        const bool kin = k0 + kq < A.vp;
        const uint32_t back = kin ? 0u : (uint32_t)(kq * sizeof(E));
#pragma unroll
        for (int s = 0; s < P::PA; ++s) {
          const Vec x = vload(ba, (term == 0 ? pa_flat[s] : pa_swap[s]) - back);
          va[s] = kin ? x : Vec{};
        }
#pragma unroll
        for (int s = 0; s < P::PB; ++s) {
          const Vec x = vload(bb, pb_off[s] - back);
          vb[s] = kin ? x : Vec{};
        }
      }
    } else {             // hole term: elements, l clamped and masked
      const int term = qs < NP + sh ? 0 : 1;
      const int kb = (qs - NP - term * sh) * kBK;
      const E *ba = hA[term], *bb = hB[term];
      const uint32_t aoff = term == 0 ? ha_flat : ha_swap;
#pragma unroll
      for (int s = 0; s < kHA; ++s) {
        const int l = kb + t / BM + KPP * s;
        const E x = ba[aoff + (uint32_t)min(l, A.o - 1) * lstride];
        ea[s] = l < A.o ? x : E(0);
      }
#pragma unroll
      for (int s = 0; s < kHB; ++s) {
        const int l = kb + (t + kThreads * s) / kBN;
        const E x = bb[hb_off[s] + (uint32_t)min(l, A.o - 1)];
        eb[s] = l < A.o ? x : E(0);
      }
    }
  };
  auto store = [&](int qs, int buf) {
    E *a = As + buf * SZA, *b = Bs + buf * SZB;
    if (qs < NP) {
#pragma unroll
      for (int s = 0; s < P::PA; ++s) {
        const int lr = t / P::TPR + s * P::RPP;
        *(Vec *)(a + lr * LDK + kq) = va[s];
      }
#pragma unroll
      for (int s = 0; s < P::PB; ++s) {
        const int lr = t / P::TPR + s * P::RPP;
        if (lr < kBN) *(Vec *)(b + lr * LDK + kq) = vb[s];
      }
    } else {
#pragma unroll
      for (int s = 0; s < kHA; ++s) a[(t % BM) * LDK + t / BM + KPP * s] = -ea[s];   // hole terms: minus
#pragma unroll
      for (int s = 0; s < kHB; ++s) {
        const int e = t + kThreads * s;
        b[(e % kBN) * LDK + e / kBN] = eb[s];
      }
    }
  };

  const int mw = wave * (BM / 4);
  load(0);
  store(0, 0);
  __syncthreads();
  for (int qs = 0; qs < nslices; ++qs) {
    const int buf = qs & 1;
    if (qs + 1 < nslices) load(qs + 1);
    const E *a = As + buf * SZA, *b = Bs + buf * SZB;
    // Lane group g = lane / 16 takes k = 4 g .. 4 g + 3 of the slice, one per
    // matrix op (the sum over k does not depend on which op adds which k), so
    // each lane reads its four k of a row with one 16-byte (FP32) or two
    // 16-byte (FP64) LDS reads.
    E af[kMI][4], bf[kNI][4];
#pragma unroll
    for (int i = 0; i < kMI; ++i) {
      const E *src = a + (mw + 16 * i + lane % 16) * LDK + 4 * (lane / 16);
#pragma unroll
      for (int x = 0; x < 4; x += VE) {
        const Vec q4 = *(const Vec *)(src + x);
#pragma unroll
        for (int e = 0; e < VE; ++e) af[i][x + e] = q4[e];
      }
    }
#pragma unroll
    for (int j = 0; j < kNI; ++j) {
      const E *src = b + (16 * j + lane % 16) * LDK + 4 * (lane / 16);
#pragma unroll
      for (int x = 0; x < 4; x += VE) {
        const Vec q4 = *(const Vec *)(src + x);
#pragma unroll
        for (int e = 0; e < VE; ++e) bf[j][x + e] = q4[e];
      }
    }
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
      for (int i = 0; i < kMI; ++i)
#pragma unroll
        for (int j = 0; j < kNI; ++j) acc[i][j] = Tr::mma(af[i][kk], bf[j][kk], acc[i][j]);
    if (qs + 1 < nslices) store(qs + 1, buf ^ 1);
    __syncthreads();
  }

  // tile -> LDS (the stage buffers are free after the last barrier) -> W, in
  // passes of CR rows
  // positions of (m1, m2, n) in W[a][b][c]
  int role1, role2, role3;
  if (A.ori == 0) { role1 = 0; role2 = 1; role3 = 2; }
  else if (A.ori == 1) { role1 = 0; role2 = 2; role3 = 1; }
  else { role1 = 1; role2 = 2; role3 = 0; }
  for (int x = t; x < BM; x += kThreads) {
    const int64_t gr = r0 + x;
    int64_t m1, m2;
    const bool ok = gr < nrows && row_pair(A, gr, m1, m2);
    rowoff[x] = ok ? w_offset(A, role1, m1) + w_offset(A, role2, m2) : -1;
  }
  for (int x = t; x < kBN; x += kThreads) coloff[x] = n0 + x < v ? w_offset(A, role3, n0 + x) : -1;
  E *Cs = smem;
  E *W = (E *)A.W + (int64_t)entry * (A.blocked ? v * ((v + 7) / 8) * ((v + 7) / 8) * 64 : vv * v);
#pragma unroll
  for (int h = 0; h < BM / CR; ++h) {
    if (mw / CR == h) {
#pragma unroll
      for (int i = 0; i < kMI; ++i)
#pragma unroll
        for (int j = 0; j < kNI; ++j)
#pragma unroll
          for (int x = 0; x < 4; ++x)
            Cs[(mw - h * CR + 16 * i + Tr::row(lane, x)) * LDC + 16 * j + lane % 16] = acc[i][j][x];
    }
    __syncthreads();
    // element e of this pass: orientation 0 runs along n (the contiguous index
    // of W), 1 and 2 along the rows (m2 contiguous); the old values of a chunk
    // are all requested before any is used.  In the blocked layout orientations
    // 0 and 1 take 8 x 8 groups (8 rows x 8 columns), so that the 64 lanes of a
    // wave cover one 64-element run of W when the rows start on a multiple of 8
    // in b (orientation 0) or c (orientation 1).
    constexpr int EPT = CR * kBN / kThreads, CH = EPT / 5;
    static_assert(EPT % 5 == 0, "epilogue chunks");
    static_assert(CR % 8 == 0 && kBN % 8 == 0, "8 x 8 epilogue groups");
    auto place = [&](int e, int &m, int &n) {
      if (A.blocked && A.ori < 2) {
        const int lo = e & 7, hi = (e >> 3) & 7, grp = e >> 6;
        const int gm = grp / (kBN / 8), gn = grp % (kBN / 8);
        if (A.ori == 0) { m = 8 * gm + hi; n = 8 * gn + lo; }
        else { m = 8 * gm + lo; n = 8 * gn + hi; }
      } else if (A.ori == 0) { m = e / kBN; n = e % kBN; }
      else { n = e / CR; m = e % CR; }
    };
#pragma unroll
    for (int c0 = 0; c0 < EPT; c0 += CH) {
      E val[CH], old[CH];
      int64_t off[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        int m, n;
        place(t + kThreads * (c0 + u), m, n);
        const int64_t ro = rowoff[h * CR + m], co = coloff[n];
        off[u] = (ro < 0 || co < 0) ? -1 : ro + co;
        val[u] = Cs[m * LDC + n];
      }
      if (A.accumulate) {
#pragma unroll
        for (int u = 0; u < CH; ++u) old[u] = W[off[u] < 0 ? 0 : off[u]];
#pragma unroll
        for (int u = 0; u < CH; ++u)
          if (off[u] >= 0) W[off[u]] = old[u] + val[u];
      } else {
#pragma unroll
        for (int u = 0; u < CH; ++u)
          if (off[u] >= 0) W[off[u]] = val[u];
      }
    }
    __syncthreads();
  }
}

// t2 in the (T) precision with d padded to vp: out[i][j][a][d], zeros for d >= v.
template <typename E>
__global__ void k_pad_t2(const double *__restrict__ t2, int64_t o, int64_t v, int64_t vp, E *out) {
  const int64_t n = o * o * v * vp;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t d = e % vp, row = e / vp;
    out[e] = d < v ? (E)t2[row * v + d] : E(0);
  }
}

}  // namespace

int64_t triples_pad(int64_t v) { return (v + 3) / 4 * 4; }

int64_t triples_w_elems(int64_t v, int blocked) {
  const int64_t vt = (v + 7) / 8;
  return blocked ? v * vt * vt * 64 : v * v * v;
}

hipError_t triples_pad_t2(const double *t2, int64_t o, int64_t v, void *out, int f32,
                          hipStream_t s) {
  if (dry_run()) return hipSuccess;
  const int64_t vp = triples_pad(v);
  const int64_t n = o * o * v * vp;
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 16384);
  if (f32)
    hipLaunchKernelGGL(k_pad_t2<float>, dim3(blocks), dim3(256), 0, s, t2, o, v, vp, (float *)out);
  else
    hipLaunchKernelGGL(k_pad_t2<double>, dim3(blocks), dim3(256), 0, s, t2, o, v, vp,
                       (double *)out);
  return hipGetLastError();
}

hipError_t triples_w(const void *G, const void *T, const void *J, void *W, const int *table,
                     int nb, int64_t o, int64_t v, int ori, int f32, int accumulate, int nterms,
                     int blocked, hipStream_t s) {
  if (nb < 1 || nb > 65535 || ori < 0 || ori > 2 || o < 1 || v < 1 || nterms < 1 || nterms > 2)
    return hipErrorInvalidValue;
  const int64_t vp = triples_pad(v), es = f32 ? 4 : 8;
  if (v * v * vp * es >= ((int64_t)1 << 32) || o * v * vp >= ((int64_t)1 << 32)) {
    note_error("(T) W kernel: nvir %lld exceeds its 32-bit offsets", (long long)v);
    return hipErrorInvalidValue;
  }
  if (!region_ok(G, (size_t)(o * v * v * vp * es)) || !region_ok(T, (size_t)(o * o * v * vp * es)) ||
      !region_ok(J, (size_t)(o * o * v * o * es)) || !region_ok(W, (size_t)(nb * triples_w_elems(v, blocked) * es)) ||
      !region_ok(table, (size_t)nb * 3 * sizeof(int))) {
    note_error("(T) W kernel (nocc %lld, nvir %lld, %d triples) leaves its buffers; not launched",
               (long long)o, (long long)v, nb);
    return hipErrorInvalidValue;
  }
  TripleArgs a{};
  a.G = G; a.T = T; a.J = J; a.W = W; a.table = table;
  a.o = (int)o; a.v = (int)v; a.vp = (int)vp;
  a.ori = ori;
  a.accumulate = accumulate;
  a.nterms = nterms;
  a.blocked = blocked ? 1 : 0;
  constexpr int bm = 128;
  const int64_t vt = (v + 7) / 8;
  const int64_t rows = (a.blocked && ori == 2) ? vt * vt * 64 : v * v;   // see row_count
  a.tiles_m = (int)((rows + bm - 1) / bm);
  a.tiles_n = (int)((v + kBN - 1) / kBN);
  if (dry_run()) return hipSuccess;
  const dim3 grid((unsigned)(a.tiles_m * a.tiles_n), (unsigned)nb);
  // algorithmic flops: nterms particle terms (K = v) and nterms hole terms
  // (K = o), each over v^3 outputs
  const double flops = (double)nb * 2.0 * nterms * (double)(v * v * v) * (double)(v + o);
  LaunchTimer tm = profile_begin(s);
  if (f32) hipLaunchKernelGGL((k_triples_w<float, bm>), grid, dim3(kThreads), 0, s, a);
  else hipLaunchKernelGGL((k_triples_w<double, bm>), grid, dim3(kThreads), 0, s, a);
  const hipError_t e = hipGetLastError();
  profile_end(tm, s, Kind::TriplesW, flops);
  return e;
}

}  // namespace lnocc

// Generic batched contraction on gfx950 matrix cores (FP64 path).
//
// Tile: 128 x 128 outputs per workgroup of 256 threads (4 wave64s in a 2 x 2
// arrangement, 64 x 64 per wave = 4 x 4 blocks of v_mfma_f64_16x16x4f64).
// K is staged through LDS in slices of 16, k-major ([k][row]) so that the 16
// lanes of one MFMA operand row read 128 contiguous bytes.  The next slice is
// fetched into registers while the current one is multiplied.
//
// MFMA 16x16x4 (f64) operand layout, lane l of a wave64:
//   A: A[l % 16][l / 16]      B: B[l / 16][l % 16]
//   D: D[l / 16 + 4 * r][l % 16], r = 0..3   (checked on gfx950)
#include "gett.h"

#include <algorithm>
#include <vector>
#include <cstdio>
#include <cstdlib>

namespace lnocc {
namespace {

constexpr int kThreads = 256;
constexpr int BM = 128, BN = 128, BK = 16;
constexpr int LDA = BM + 4;   // padded LDS row (doubles)
constexpr int LDB = BN + 4;
constexpr int kPerThreadA = BM * BK / kThreads;   // 8
constexpr int kPerThreadB = BN * BK / kThreads;   // 8

typedef double double4_t __attribute__((ext_vector_type(4)));

struct BatchIdx { int64_t i0, i1, i2; };

__device__ inline BatchIdx decode_batch(const GemmDesc &d, int id) {
  BatchIdx b;
  if (d.table) {
    b.i0 = d.table[3 * id + 0];
    b.i1 = d.table[3 * id + 1];
    b.i2 = d.table[3 * id + 2];
  } else {
    b.i0 = id / d.nb1;
    b.i1 = id % d.nb1;
    b.i2 = 0;
  }
  return b;
}

__device__ inline int64_t row_off(const GOperand &op, int r, int Ri) {
  return (int64_t)(r / Ri) * op.s_ro + (int64_t)(r % Ri) * op.s_ri;
}
__device__ inline int64_t k_off(const GOperand &op, int k, int Ki) {
  return (int64_t)(k / Ki) * op.s_ko + (int64_t)(k % Ki) * op.s_ki;
}

// Loads one BK-slice of one operand (rows row0.., k0..) into registers.
// kfast: consecutive threads walk k (operand contiguous along k); otherwise
// consecutive threads walk the row index.
template <int R, int PER>
__device__ inline void load_slice(const double *__restrict__ base, const GOperand &op,
                                  bool kfast, int nrows, int Ri, int K, int Ki,
                                  int row0, int k0, const int64_t *roff,
                                  const bool *rok, double *reg) {
  const int t = threadIdx.x;
  if (kfast) {
    const int kk = t % BK;
    const int k = k0 + kk;
    const bool kok = k < K;
    const int64_t ko = kok ? k_off(op, k, Ki) : 0;
#pragma unroll
    for (int s = 0; s < PER; ++s)
      reg[s] = (kok && rok[s]) ? base[roff[s] + ko] : 0.0;
  } else {
#pragma unroll
    for (int s = 0; s < PER; ++s) {
      const int kk = t / R + s * (kThreads / R);
      const int k = k0 + kk;
      reg[s] = (k < K && rok[0]) ? base[roff[0] + k_off(op, k, Ki)] : 0.0;
    }
  }
}

template <int R, int LD, int PER>
__device__ inline void store_slice(double *lds, bool kfast, const double *reg) {
  const int t = threadIdx.x;
  if (kfast) {
    const int kk = t % BK;
#pragma unroll
    for (int s = 0; s < PER; ++s) lds[kk * LD + t / BK + s * (kThreads / BK)] = reg[s];
  } else {
#pragma unroll
    for (int s = 0; s < PER; ++s) lds[(t / R + s * (kThreads / R)) * LD + t % R] = reg[s];
  }
}

template <int R, int PER>
__device__ inline void row_offsets(const GOperand &op, bool kfast, int nrows, int Ri,
                                   int row0, int64_t *roff, bool *rok) {
  const int t = threadIdx.x;
  if (kfast) {
#pragma unroll
    for (int s = 0; s < PER; ++s) {
      const int r = row0 + t / BK + s * (kThreads / BK);
      rok[s] = r < nrows;
      roff[s] = rok[s] ? row_off(op, r, Ri) : 0;
    }
  } else {
    const int r = row0 + t % R;
    rok[0] = r < nrows;
    roff[0] = rok[0] ? row_off(op, r, Ri) : 0;
#pragma unroll
    for (int s = 1; s < PER; ++s) { rok[s] = rok[0]; roff[s] = roff[0]; }
  }
}

template <int KIND>
__global__ __launch_bounds__(kThreads) void gett_f64_kernel(GemmDesc d, int tiles_m) {
  __shared__ double As[BK * LDA];
  __shared__ double Bs[BK * LDB];

  const int tile = blockIdx.x;
  const int tm = tile % tiles_m, tn = tile / tiles_m;
  const int m0 = tm * BM, n0 = tn * BN;
  const BatchIdx bi = decode_batch(d, blockIdx.y);

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  double4_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = double4_t{0.0, 0.0, 0.0, 0.0};

  for (int sg = 0; sg < d.nseg; ++sg) {
    const GSegment &S = d.seg[sg];
    const int64_t id = blockIdx.y;
    const double *pa = (const double *)S.a.p + bi.i0 * S.a.b0 + bi.i1 * S.a.b1 + bi.i2 * S.a.b2 + id * S.a.bid;
    const double *pb = (const double *)S.b.p + bi.i0 * S.b.b0 + bi.i1 * S.b.b1 + bi.i2 * S.b.b2 + id * S.b.bid;
    const bool akf = S.a_kfast != 0;
    const bool bkf = S.b_kfast != 0;
    int64_t aoff[kPerThreadA], boff[kPerThreadB];
    bool aok[kPerThreadA], bok[kPerThreadB];
    row_offsets<BM, kPerThreadA>(S.a, akf, d.M, d.Mi, m0, aoff, aok);
    row_offsets<BN, kPerThreadB>(S.b, bkf, d.N, d.Ni, n0, boff, bok);
    const double scale = S.scale;

    double ra[kPerThreadA], rb[kPerThreadB];
    load_slice<BM, kPerThreadA>(pa, S.a, akf, d.M, d.Mi, S.K, S.Ki, m0, 0, aoff, aok, ra);
    load_slice<BN, kPerThreadB>(pb, S.b, bkf, d.N, d.Ni, S.K, S.Ki, n0, 0, boff, bok, rb);
    for (int k0 = 0; k0 < S.K; k0 += BK) {
#pragma unroll
      for (int s = 0; s < kPerThreadA; ++s) ra[s] *= scale;
      __syncthreads();
      store_slice<BM, LDA, kPerThreadA>(As, akf, ra);
      store_slice<BN, LDB, kPerThreadB>(Bs, bkf, rb);
      __syncthreads();
      if (k0 + BK < S.K) {
        load_slice<BM, kPerThreadA>(pa, S.a, akf, d.M, d.Mi, S.K, S.Ki, m0, k0 + BK, aoff, aok, ra);
        load_slice<BN, kPerThreadB>(pb, S.b, bkf, d.N, d.Ni, S.K, S.Ki, n0, k0 + BK, boff, bok, rb);
      }
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        double af[4], bf[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
          af[i] = As[(kk + lane / 16) * LDA + wm * 64 + i * 16 + lane % 16];
#pragma unroll
        for (int j = 0; j < 4; ++j)
          bf[j] = Bs[(kk + lane / 16) * LDB + wn * 64 + j * 16 + lane % 16];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
      }
    }
  }

  // Epilogue: lane holds rows lane/16 + 4r of each 16x16 block, column lane%16.
  double *pc = d.c + bi.i0 * d.c_b0 + bi.i1 * d.c_b1 + bi.i2 * d.c_b2 + (int64_t)blockIdx.y * d.c_bid;
  int64_t coff[4];
  bool cok[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int n = n0 + wn * 64 + j * 16 + lane % 16;
    cok[j] = n < d.N;
    coff[j] = cok[j] ? (int64_t)(n / d.Ni) * d.c_no + (int64_t)(n % d.Ni) * d.c_ni : 0;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + wm * 64 + i * 16 + lane / 16 + 4 * r;
      if (m >= d.M) continue;
      const int64_t moff = (int64_t)(m / d.Mi) * d.c_mo + (int64_t)(m % d.Mi) * d.c_mi;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (!cok[j]) continue;
        double *dst = pc + moff + coff[j];
        const double v = acc[i][j][r];
        *dst = (d.beta == 0.0) ? v : v + d.beta * *dst;
      }
    }
  }
}

}  // namespace

namespace {
thread_local const Region *g_regions = nullptr;
thread_local int g_nregions = 0;

// [lo, hi] element offsets reachable from an operand's base pointer.
struct Span { int64_t lo, hi; };
void add_term(Span &s, int64_t idx_max, int64_t stride) {
  if (idx_max <= 0 || stride == 0) return;
  if (stride > 0) s.hi += idx_max * stride; else s.lo += idx_max * stride;
}
bool inside(const void *base, Span sp, size_t elem) {
  const char *lo = (const char *)base + sp.lo * (int64_t)elem;
  const char *hi = (const char *)base + (sp.hi + 1) * (int64_t)elem;
  for (int r = 0; r < g_nregions; ++r) {
    const char *a = (const char *)g_regions[r].p, *b = a + g_regions[r].bytes;
    if (lo >= a && hi <= b) return true;
  }
  return false;
}
int64_t outer_max(int64_t n, int64_t inner) { return (n - 1) / inner; }
int64_t inner_max(int64_t n, int64_t inner) { return std::min(n, inner) - 1; }

bool operand_ok(const GemmDesc &d, const GOperand &op, int64_t rows, int64_t Ri, int64_t K,
                int64_t Ki, const int64_t bmax[3]) {
  if (rows <= 0 || K <= 0) return true;
  Span s{0, 0};
  add_term(s, outer_max(rows, Ri), op.s_ro);
  add_term(s, inner_max(rows, Ri), op.s_ri);
  add_term(s, outer_max(K, Ki), op.s_ko);
  add_term(s, inner_max(K, Ki), op.s_ki);
  add_term(s, bmax[0], op.b0);
  add_term(s, bmax[1], op.b1);
  add_term(s, bmax[2], op.b2);
  add_term(s, d.batch - 1, op.bid);
  return inside(op.p, s, sizeof(double));
}

bool descriptor_ok(const GemmDesc &d) {
  if (!g_regions) return true;
  int64_t bmax[3];
  if (d.table) { bmax[0] = d.tmax[0]; bmax[1] = d.tmax[1]; bmax[2] = d.tmax[2]; }
  else { bmax[0] = (d.batch - 1) / d.nb1; bmax[1] = std::min(d.batch, d.nb1) - 1; bmax[2] = 0; }
  for (int s = 0; s < d.nseg; ++s) {
    const GSegment &g = d.seg[s];
    if (!operand_ok(d, g.a, d.M, d.Mi, g.K, g.Ki, bmax)) return false;
    if (!operand_ok(d, g.b, d.N, d.Ni, g.K, g.Ki, bmax)) return false;
  }
  Span c{0, 0};
  add_term(c, outer_max(d.M, d.Mi), d.c_mo);
  add_term(c, inner_max(d.M, d.Mi), d.c_mi);
  add_term(c, outer_max(d.N, d.Ni), d.c_no);
  add_term(c, inner_max(d.N, d.Ni), d.c_ni);
  add_term(c, bmax[0], d.c_b0);
  add_term(c, bmax[1], d.c_b1);
  add_term(c, bmax[2], d.c_b2);
  add_term(c, d.batch - 1, d.c_bid);
  return inside(d.c, c, sizeof(double));
}
}  // namespace

static bool g_dry = false;

struct Record { Kind kind; hipEvent_t start, stop; double flops; };
static bool g_profile = false;
static std::vector<Record> g_records;

void profile_enable(bool on) { g_profile = on; }

void profile_collect(KindStats out[(int)Kind::Count]) {
  for (int k = 0; k < (int)Kind::Count; ++k) out[k] = KindStats{0, 0.0, 0.0};
  for (const Record &r : g_records) {
    float ms = 0.f;
    hipEventSynchronize(r.stop);
    hipEventElapsedTime(&ms, r.start, r.stop);
    KindStats &k = out[(int)r.kind];
    k.launches += 1;
    k.ms += ms;
    k.flops += r.flops;
    hipEventDestroy(r.start);
    hipEventDestroy(r.stop);
  }
  g_records.clear();
}
bool dry_run() { return g_dry; }
void set_dry_run(bool on) { g_dry = on; }

void install_regions(const Region *r, int n) {
  g_regions = (n > 0) ? r : nullptr;
  g_nregions = (n > 0) ? n : 0;
}

static int contiguous_along_k(const GOperand &op, int Ki) {
  return (Ki > 1) ? (op.s_ki == 1) : (op.s_ko == 1);
}

hipError_t gett(const GemmDesc &din, hipStream_t stream) {
  GemmDesc d = din;
  if (d.M <= 0 || d.N <= 0 || d.batch <= 0) return hipSuccess;
  if (d.Mi <= 0 || d.Ni <= 0 || d.nseg <= 0 || d.nseg > kMaxSeg) return hipErrorInvalidValue;
  for (int s = 0; s < d.nseg; ++s) {
    if (d.seg[s].K < 0 || d.seg[s].Ki <= 0) return hipErrorInvalidValue;
    d.seg[s].a_kfast = contiguous_along_k(d.seg[s].a, d.seg[s].Ki);
    d.seg[s].b_kfast = contiguous_along_k(d.seg[s].b, d.seg[s].Ki);
  }
  if (d.batch > 65535) return hipErrorInvalidValue;
  if (d.table == nullptr && d.nb1 <= 0) return hipErrorInvalidValue;
  if (!descriptor_ok(d)) {
    if (std::getenv("LNOCC_DEBUG"))
      std::fprintf(stderr, "lnocc: contraction M=%d(%d) N=%d(%d) nseg=%d K0=%d(%d) batch=%d "
                   "leaves its buffers; not launched\n", d.M, d.Mi, d.N, d.Ni, d.nseg,
                   d.seg[0].K, d.seg[0].Ki, d.batch);
    return hipErrorIllegalAddress;
  }
  if (g_dry) return hipSuccess;
  const int tiles_m = (d.M + BM - 1) / BM;
  const int tiles_n = (d.N + BN - 1) / BN;
  dim3 grid(tiles_m * tiles_n, d.batch);
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (g_profile) {
    if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess)
      return hipErrorOutOfMemory;
    hipEventRecord(ev[0], stream);
  }
  switch (d.kind) {
    case Kind::LadderBuild:
      hipLaunchKernelGGL(gett_f64_kernel<1>, grid, dim3(kThreads), 0, stream, d, tiles_m); break;
    case Kind::LadderContract:
      hipLaunchKernelGGL(gett_f64_kernel<2>, grid, dim3(kThreads), 0, stream, d, tiles_m); break;
    case Kind::TriplesW:
      hipLaunchKernelGGL(gett_f64_kernel<3>, grid, dim3(kThreads), 0, stream, d, tiles_m); break;
    default:
      hipLaunchKernelGGL(gett_f64_kernel<0>, grid, dim3(kThreads), 0, stream, d, tiles_m); break;
  }
  const hipError_t err = hipGetLastError();
  if (g_profile) {
    hipEventRecord(ev[1], stream);
    double flops = 0.0;
    for (int s = 0; s < d.nseg; ++s) flops += 2.0 * d.M * (double)d.N * d.seg[s].K;
    g_records.push_back(Record{d.kind, ev[0], ev[1], flops * d.batch});
  }
  return err;
}

GemmDesc gemm_desc(int M, int N, int K, double alpha,
                   const double *A, int64_t sam, int64_t sak,
                   const double *B, int64_t sbk, int64_t sbn,
                   double beta, double *C, int64_t scm, int64_t scn) {
  GemmDesc d{};
  d.M = M; d.Mi = 1; d.N = N; d.Ni = 1;
  d.nseg = 1;
  GSegment &s = d.seg[0];
  s.a = GOperand{A, sam, 0, sak, 0, 0, 0, 0, 0};
  s.b = GOperand{B, sbn, 0, sbk, 0, 0, 0, 0, 0};
  s.K = K; s.Ki = 1; s.scale = alpha;
  d.c = C; d.c_mo = scm; d.c_mi = 0; d.c_no = scn; d.c_ni = 0;
  d.c_b0 = d.c_b1 = d.c_b2 = d.c_bid = 0;
  d.beta = beta;
  d.batch = 1; d.nb1 = 1; d.table = nullptr;
  d.prec = Prec::F64;
  return d;
}

}  // namespace lnocc

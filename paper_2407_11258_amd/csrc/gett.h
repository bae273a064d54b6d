// Generic batched tensor contraction ("GETT") on gfx950 matrix cores.
//
// C[m, n] (+)= sum_seg scale_seg * sum_k A_seg(m, k) * B_seg(k, n)
//
// Each of the M, N and K modes is a pair of tensor indices: m = m_o * Mi + m_i
// (likewise n with Ni and k with Ki), and every operand gives one stride per
// index, so any contraction with at most two indices per mode is expressed
// without a permuted copy.  Several K segments (different operands, same C)
// accumulate in registers before the single store.  A batch index is decoded
// into up to three integers (from a table of int triples or as id / nb1,
// id % nb1); every base pointer moves by a linear combination of them.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace lnocc {

// F32S: FP32 operands whose products run on the bf16 matrix cores as sums of
// split products (FP32-level accuracy; see the kernel source).  F64S: FP64
// operands in memory, rounded to FP32 when staged and multiplied as F32S.
enum class Prec : int { F64 = 0, F32 = 1, BF16 = 2, F32S = 3, F64S = 4 };

// What a contraction computes; each class is its own kernel symbol (so
// profiler statistics separate them) and its own timing bucket.
enum class Kind : int {
  Other = 0,          // CCSD intermediates, dressing, Fock, one-off integrals
  LadderBuild = 1,    // (ac|bd)~ = sum_Q B~_Qac B~_Qbd for a block of a
  LadderContract = 2, // R2 += sum_cd t_ij^cd (ac|bd)~
  TriplesW = 3,       // W_ijk^abc for a batch of unique triples
  Mlp = 4,            // learned-guess network layers and their gradients (FP32 only)
  Ring = 5,           // o^3 v^3 ring terms of the CCSD residual (and the ladder's T1 terms)
  Split = 6,          // timing bucket only: every launch with split-bf16 products, any kind
  Count = 7
};

// Division by a runtime-invariant divisor via multiply-high (Granlund and
// Montgomery, PLDI 1994): q = (t + ((n - t) >> s1)) >> s2 with t = mulhi(m, n);
// exact for all 32-bit n and divisors d >= 1.
struct FastDiv {
  uint32_t d, m, s1, s2;
};
inline FastDiv make_fastdiv(uint32_t d) {
  uint32_t l = 0;
  while ((1ull << l) < d) ++l;
  FastDiv f;
  f.d = d;
  f.m = (uint32_t)((((1ull << 32) * ((1ull << l) - d)) / d) + 1);
  f.s1 = l > 0 ? 1 : 0;
  f.s2 = l > 0 ? l - 1 : 0;
  return f;
}

struct GOperand {
  const void *p;          // element type given by GemmDesc::prec
  int64_t s_ro, s_ri;     // strides of the outer / inner row (m or n) index
  int64_t s_ko, s_ki;     // strides of the outer / inner contraction index
  int64_t b0, b1, b2;     // pointer offset per unit of each batch integer
  int64_t bid;            // pointer offset per unit of the batch entry number
};

struct GSegment {
  GOperand a;             // rows = m
  GOperand b;             // rows = n (the operand is addressed as B(n, k))
  int K, Ki;              // contraction length and inner extent (k = ko*Ki + ki)
  double scale;           // multiplies the A operand
  int a_kfast, b_kfast;   // set by gett(): operand contiguous along k
  FastDiv kdiv;           // set by gett(): division by Ki
};

constexpr int kMaxSeg = 4;

struct GemmDesc {
  int M, Mi, N, Ni;
  int nseg;
  GSegment seg[kMaxSeg];
  void *c;                // output (element type c_type)
  const void *c_src;      // nullptr, or the input of the beta term (C's layout): C = AB + beta c_src
  int64_t c_mo, c_mi, c_no, c_ni, c_b0, c_b1, c_b2, c_bid;
  double beta;            // 0: C is overwritten without being read
  int batch;              // number of batch entries (>= 1)
  int nb1;                // id -> (id / nb1, id % nb1, 0) when table == nullptr
  const int *table;       // device int triples, batch entry id -> (i0, i1, i2)
  int tmax[3];            // with a table: largest value of each batch integer
  Prec prec;              // operand element type in memory and product arithmetic:
                          // F64 double, F32 float, BF16 bf16 (FP32 accumulation)
  int c_type;             // output element: 0 double, 1 float, 2 bf16
  Kind kind;
  int tile_hint;          // 0 automatic, t + 1 forces tile t (see the launcher)
  double *splitk;         // set by gett(): partial-sum scratch when K is split
  FastDiv mdiv, ndiv;     // set by gett(): division by Mi, Ni
  int c_vec4;             // set by gett(): output rows 4q .. 4q+3 are consecutive,
                          // 4-element-aligned elements of C (stored as one vector)
};

// Scratch for split-K partial sums (per host thread); without it K is never split.
void install_splitk_scratch(double *p, size_t elems);

// Launch timing: while enabled, every contraction launch is bracketed by HIP
// events on its stream; collect() waits for them and sums per Kind.
struct KindStats { int64_t launches; double ms; double flops; };
void profile_enable(bool on);
bool profile_enabled();
void profile_collect(KindStats out[(int)Kind::Count]);   // also clears

// Launch timing of kernels launched outside gett(): while profiling is on,
// begin() records an event before the launch and end() one after it, filed
// under `kind` with the launch's algorithmic flops.  Both are no-ops otherwise.
struct LaunchTimer { hipEvent_t start = nullptr, stop = nullptr; };
LaunchTimer profile_begin(hipStream_t s);
void profile_end(LaunchTimer &t, hipStream_t s, Kind kind, double flops);

// Address guard.  While a region list is installed (per host thread), gett()
// refuses to launch a contraction unless every address it can touch lies
// inside one listed region.  The solver installs the workspace and the
// caller's arrays; a descriptor mistake then becomes an error, not a fault.
struct Region { const void *p; size_t bytes; };
void install_regions(const Region *r, int n);   // n = 0 removes the list
// For kernels launched outside gett(): [p, p + bytes) lies inside an installed
// region (always true while none is installed).
bool region_ok(const void *p, size_t bytes);

// Validation mode: launches are checked against the guard and then skipped,
// copies and synchronizations become no-ops and readbacks return zeros.  Lets
// the whole launch sequence of a solve run on a host without a GPU.
bool dry_run();
void set_dry_run(bool on);

// Description of the last failure noted on this host thread ("" when none
// since clear_error()); printed to stderr as well when LNOCC_DEBUG is set.
// clear_error() also clears the runtime's last-error state, which launch
// checks read.
void note_error(const char *fmt, ...);
const char *last_error();
void clear_error();

// Autotuning of tile shape and split count per contraction shape.
// tune_candidate(c) for c < tune_candidates() makes every later launch use
// candidate c and time it; tune_candidate(-1) stops; tune_commit() waits for
// those launches and stores, per shape, the fastest candidate's choice (used
// by every later launch of that shape; returns the number of shapes).  A probe
// pass (tune_probe_begin/end) launches nothing and counts shapes without a
// plan.  Plans are process-wide; save/load use a text file.
int tune_candidates();
void tune_candidate(int c);
void tune_probe_begin();
int tune_probe_end();
int tune_commit();
size_t tune_plans();
int tune_save(const char *path);
int tune_load(const char *path);
void tune_clear();

// Enqueue on `stream`.  Returns hipSuccess or the launch error.
hipError_t gett(const GemmDesc &d, hipStream_t stream);

// Convenience: fill a descriptor for a plain strided matrix product
// C[m,n] = alpha * sum_k A[m*sam + k*sak] * B[k*sbk + n*sbn] + beta*C[m*scm + n*scn].
GemmDesc gemm_desc(int M, int N, int K, double alpha,
                   const double *A, int64_t sam, int64_t sak,
                   const double *B, int64_t sbk, int64_t sbn,
                   double beta, double *C, int64_t scm, int64_t scn);

// Tile of block number `tile` of a tiles_m x tiles_n grid.  Workgroups are
// dispatched round-robin over the eight XCDs, each with its own L2 (blocks
// tile and tile + 8 share one): the column tiles of a row tile go to blocks
// tile, tile + 8, tile + 16, ..., so one L2 fetches the row tile's operand rows
// for all of them.  Row tiles past the last multiple of 8 take the plain order.
__device__ inline void xcd_tile(int tile, int tiles_m, int tiles_n, int &tm, int &tn) {
  const int G = 8 * tiles_n, full = tiles_m / 8 * G;
  if (tile < full) {
    const int g = tile / G, r = tile % G;
    tm = 8 * g + (r & 7);
    tn = r >> 3;
  } else {
    const int rem = tiles_m % 8, r = tile - full;
    tm = tiles_m / 8 * 8 + r % rem;
    tn = r / rem;
  }
}

}  // namespace lnocc

// Internal interface of the fragment solver (host side).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <cmath>
#include <vector>

#include "../../include/lnocc.h"
#include "gett.h"
#include "mlp.h"

namespace lnocc {

struct Dims { int64_t o, v, X; };

// Scratch of the pair energies (pairs.hip), FP64.
struct PairLayout {
  double *Gt = nullptr, *Jt = nullptr, *T = nullptr;   // (ai|bd), (ck|jl), t2 for the W kernel
  int *table = nullptr;             // (i, j, k) for every i and pair j <= k
  double *W = nullptr, *Y = nullptr, *Z = nullptr;     // [o][v][v][v] for one pair (j, k)
  double *tau = nullptr, *Lx = nullptr;                // [o][o][v][v]
};

// Device buffers carved out of the caller's workspace.  The (T) buffers alias
// the CCSD scratch, which is dead once the amplitudes have converged.
struct Layout {
  Dims dm;
  // common
  double *Boo, *Bov, *Bvv;          // DF split [X][o][o], [X][o][v], [X][v][v]
  double *Kov;                      // (kc|ld) as [k][c][l][d]
  double *t1w, *t2w;                // amplitudes when the caller passes none
  double *hoo, *hov, *hvo, *hvv;    // bare one-electron operator blocks
  double *J;                        // [X] occupied trace of B (or B~)
  double *scal, *partials;          // small scalars, reduction partials
  double *nrm, *jd;                 // |B_ia| and (ii|aa) [o][v] (learned-guess features)
  double *splitk;                   // split-K partial sums of thin contractions
  int64_t splitk_elems;
  // CCSD
  double *Btoo, *Btai, *Btvv;       // T1-dressed factors; Btai[Q][i][a] = B~[Q][a][i]
  double *Foo, *Fov, *Fvo, *Fvv, *Foop, *Fvvp;
  double *Pvv, *Q2, *Lov;           // (ld|kc) [k][l][d][c], (kd|lc) [k][l][c][d], 2(ld|kc)-(lc|kd) [l][d][k][c]
  double *u, *R1, *R2, *S, *Xc, *Goovv, *Cint, *Dint, *Wkl, *Y1, *Z1;
  double *chunk;                    // (ac|bd)~ for chunk_a values of a: [a][b][c][d]
  double *Tsa, *SA;                 // ladder rows [t + t^T ; t - t^T] and results [o^2][v][v]
  double *Btvv_lp;                  // B~_vv in the precision of the ladder products
  // stored ladder (bare integrals formed once per solve)
  bool lstore = false;
  void *Lst = nullptr;              // (ac|bd) blocks [a in block][b < a1][c][d], ladder precision
  int64_t lrows = 0;                // rows (a, b < a1) of all stored blocks
  double *Gkc = nullptr;            // (kc|bd) [k][c][b][d]
  double *Zl = nullptr, *Yl = nullptr, *Wl = nullptr;   // [ij][k][b], [ij][k][b], [ij][k][l]
  double *Bvv_lp = nullptr;         // bare B_vv in the ladder precision
  double *t2_lp;                    // t2 for (T): [o][o][v][vp] in the (T) element type
  bool t_f32 = false;               // (T) products and W in FP32
  Prec lp;                          // precision of the ladder and (T) products
  Prec rp;                          // o^3 v^3 ring products: F64, or F64S in the FP32 / BF16 modes
  int lpt;                          // its element type: 0 double, 1 float, 2 bf16
  double *dx, *de;                  // DIIS vectors and errors [m][namp]
  int64_t chunk_a, namp;
  int diis_m;
  // learned guess (only with LNOCC_GUESS_MLP)
  mlp::Scratch ms;                  // network scratch
  int64_t nunique = 0;              // amplitudes with i <= j: o (o + 1) / 2 v^2
  // (T)
  double *Gt, *Jt, *W, *tpart;      // (ai|bd) [i][a][b][d], (ck|jl) [j][k][c][l], W [nb][v][v][v]
  int64_t tpart_elems = 0;          // capacity of tpart (energy partial sums)
  int *table;
  int nb;
  int64_t ntriples;
  size_t bytes;
  size_t phase_off = 0;             // end of the common part (start of the phase scratch)
  PairLayout pairs;
};

struct Inputs {
  const double *B, *eo, *ev;
  double *t1, *t2;
  double conv_tol;
  const lnocc_fragment_t *frag = nullptr;   // passed to the progress callback
};

struct Outputs {
  double e_mp2 = 0, e_ccsd = 0, e_t = 0, residual = 0;
  int n_iter = 0, status = 0;
  int guess_used = 0;
};

// Stream copies and synchronization that become no-ops in validation mode
// (readbacks then return zeros).
inline hipError_t dcopy(void *dst, const void *src, size_t bytes, hipStream_t s) {
  return dry_run() ? hipSuccess : hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s);
}
inline hipError_t dzero(void *dst, size_t bytes, hipStream_t s) {
  return dry_run() ? hipSuccess : hipMemsetAsync(dst, 0, bytes, s);
}
inline hipError_t d2h(void *dst, const void *src, size_t bytes, hipStream_t s) {
  if (dry_run()) {
    for (size_t i = 0; i < bytes; ++i) ((char *)dst)[i] = 0;
    return hipSuccess;
  }
  return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s);
}
inline hipError_t h2d(void *dst, const void *src, size_t bytes, hipStream_t s) {
  return dry_run() ? hipSuccess : hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
}
inline hipError_t dsync(hipStream_t s) { return dry_run() ? hipSuccess : hipStreamSynchronize(s); }

int64_t unique_triples(int64_t o);
void plan_layout(const Dims &dm, const lnocc_options_t &opt, char *base, Layout &L);
int setup_fragment(const Layout &L, const double *B, const double *eo, const double *ev,
                   bool ccsd_phase, hipStream_t s);
// split_ring: the o^3 v^3 ring products in L.rp (split bf16 in the reduced
// modes) instead of FP64.
int ccsd_residuals(const Layout &L, const double *t1, const double *t2, hipStream_t s,
                   bool split_ring = false);
int tune_residuals(const Layout &L, const double *t1, const double *t2, hipStream_t s);
int energy(const Layout &L, const double *t1, const double *t2, double *dev_out, hipStream_t s);
struct Readback;
// rb: readback buffer to use (nullptr: a pinned one made for the call).
int run_ccsd(const Layout &L, const Inputs &in, const lnocc_options_t &opt, Outputs &out,
             hipStream_t s, Readback *rb = nullptr);
// host: one double of host memory for the energy readback (nullptr: pinned, made
// for the call).
int run_triples(const Layout &L, const Inputs &in, Outputs &out, hipStream_t s,
                bool autotune = false, double *host = nullptr);
int enqueue_triples(const Layout &L, const Inputs &in, hipStream_t s, bool autotune = false);

// Pinned host buffer for the small readbacks of one solve ([0] energy,
// [1..16] DIIS overlaps, [32] step norm, [33] step norm from the MP2 start,
// [34] its DIIS error norm, [40] (T) energy) and the event that
// marks their arrival.  Owned by the caller of CcsdRun; reused across solves.
// With an external buffer (caller-owned host memory of at least kReadbackDoubles
// doubles) nothing is allocated and no event is made: arrival is then awaited
// by synchronizing the stream.
constexpr int kReadbackDoubles = 64;
struct Readback {
  double *host = nullptr;
  hipEvent_t ev = nullptr;
  bool external = false;
  Readback();
  explicit Readback(double *buffer);
  ~Readback();
  Readback(const Readback &) = delete;
  Readback &operator=(const Readback &) = delete;
  bool ok() const;
};

// CCSD of one fragment as a resumable state machine: each enqueue_* call
// queues device work and one readback, poll() reports whether that readback
// has landed, and after_* consumes it.  The batch driver interleaves several
// of these on one stream, so the host round trip of one fragment overlaps the
// device work of the others.
// Reduced modes: residual products in split bf16 until the step norm is within
// this multiple of the convergence threshold (or stops improving).
constexpr double kSplitRingFactor = 100.0;

struct CcsdRun {
  enum class Phase { Idle, Started, Iterating, Converged, Exhausted };
  const Layout *L;
  Inputs in;
  lnocc_options_t opt;
  hipStream_t s;
  Readback *rb;
  double *host;
  Outputs out;
  Phase phase = Phase::Idle;
  std::vector<double> G;       // DIIS Gram matrix (host, FP64)
  int it = 0, count = 0, growth = 0, slot = 0, nvalid = 1;
  bool use_diis = false;
  double prev = INFINITY, best = INFINITY;
  mutable int polls = 0;
  bool mlp_check = false;      // the first step from the learned start is still to be judged
  double r_mp2 = 0.0;          // first step norm from the MP2 start
  hipGraphExec_t graph[2] = {nullptr, nullptr};   // captured residual evaluation, FP64 / split
  bool split = false;          // residual products of the next iteration in split bf16
  int split_stall = 0;         // iterations in a row without a new minimum step norm

  CcsdRun(const Layout &L, const Inputs &in, const lnocc_options_t &opt, hipStream_t s,
          Readback &rb);
  ~CcsdRun();
  CcsdRun(const CcsdRun &) = delete;
  CcsdRun &operator=(const CcsdRun &) = delete;
  int poll() const;            // 1 landed, 0 pending, < 0 error
  hipError_t wait() const;
  int begin();
  int after_begin();
  int enqueue_iteration();
  int after_iteration();
  int enqueue_final();
  int after_final();
  int enqueue_t();             // (T) on the converged amplitudes, E_(T) read back
  int after_t();

 private:
  hipError_t mark();
  int learned_start();
  int residuals();             // eager, or through the captured graph
  bool split_ring() const;     // ring products of this iteration in split bf16
};

}  // namespace lnocc

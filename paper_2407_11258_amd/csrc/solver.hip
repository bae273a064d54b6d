// Host driver of the fragment solver: workspace layout, the closed-shell CCSD
// residual as a sequence of contractions, Jacobi + DIIS iterations and the
// (T) passes.  Everything here enqueues device work on one stream; the only
// device-to-host traffic is one small readback per iteration.
//
// CCSD equations: closed-shell CCSD written with the T1-similarity-transformed
// Hamiltonian H~ = exp(-T1) H exp(T1).  Three-index factors are dressed once
// per iteration (B~ = Lm B Rm^T with Lm = 1 - T, Rm = 1 + T^T, T[a][i] = t_i^a),
// after which every term is a product of dressed DF factors, T2 and the dressed
// Fock matrix.  The residual returned is <mu| e^{-T} H e^{T} |HF> for
// mu = (i alpha -> a alpha) and (i alpha j beta -> a alpha b beta).
#include "solver.h"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "gett.h"
#include "kernels.h"
#include "triples.h"

namespace lnocc {

#define LN_TRY(x)                                                         \
  do {                                                                    \
    hipError_t e_ = (x);                                                  \
    if (e_ != hipSuccess) {                                               \
      note_error("%s failed (%s) at %s:%d", #x, hipGetErrorString(e_),    \
                 __FILE__, __LINE__);                                     \
      return LNOCC_EDEVICE;                                               \
    }                                                                     \
  } while (0)

namespace {

// LNOCC_LOG=1: one line per CCSD iteration and per (T) pass on stderr.
bool log_enabled() {
  static const bool on = [] {
    const char *e = std::getenv("LNOCC_LOG");
    return e && e[0] && e[0] != '0';
  }();
  return on;
}

GOperand OP(const double *p, int64_t ro, int64_t ri, int64_t ko, int64_t ki) {
  GOperand g{};
  g.p = p; g.s_ro = ro; g.s_ri = ri; g.s_ko = ko; g.s_ki = ki;
  return g;
}
GOperand OPB(GOperand g, int64_t b0, int64_t b1, int64_t b2) {
  g.b0 = b0; g.b1 = b1; g.b2 = b2;
  return g;
}
GemmDesc DESC(int64_t M, int64_t Mi, int64_t N, int64_t Ni, double *c, int64_t cmo, int64_t cmi,
              int64_t cno, int64_t cni, double beta) {
  GemmDesc d{};
  d.M = (int)M; d.Mi = (int)Mi; d.N = (int)N; d.Ni = (int)Ni;
  d.c = c; d.c_mo = cmo; d.c_mi = cmi; d.c_no = cno; d.c_ni = cni;
  d.beta = beta; d.batch = 1; d.nb1 = 1; d.table = nullptr; d.prec = Prec::F64;
  return d;
}
void SEG(GemmDesc &d, int64_t K, int64_t Ki, double scale, GOperand a, GOperand b) {
  GSegment &s = d.seg[d.nseg++];
  s.a = a; s.b = b; s.K = (int)K; s.Ki = (int)Ki; s.scale = scale;
}
// batch over the auxiliary index: entry Q moves operands by b0 * Q
void BATCH_Q(GemmDesc &d, int64_t X, int64_t cstride) {
  d.batch = (int)X; d.nb1 = 1; d.c_b0 = cstride;
}

struct Arena {
  char *base;
  size_t off = 0;
  double *d(int64_t n) {
    off = (off + 255) & ~size_t(255);
    double *p = base ? (double *)(base + off) : nullptr;
    off += (size_t)n * sizeof(double);
    return p;
  }
  int *i(int64_t n) {
    off = (off + 255) & ~size_t(255);
    int *p = base ? (int *)(base + off) : nullptr;
    off += (size_t)n * sizeof(int);
    return p;
  }
};

}  // namespace

// ---------------------------------------------------------------- layout
int64_t unique_triples(int64_t o) {
  // i <= j <= k with not all equal
  return o * (o + 1) * (o + 2) / 6 - o;
}

void plan_layout(const Dims &dm, const lnocc_options_t &opt, char *base, Layout &L) {
  const int64_t o = dm.o, v = dm.v, X = dm.X;
  const int64_t ov = o * v, oo = o * o, vv = v * v, oovv = oo * vv, vvv = vv * v;
  Arena A{base};
  L = Layout{};
  L.dm = dm;
  L.lp = opt.precision == LNOCC_FP32 ? Prec::F32 : (opt.precision == LNOCC_BF16 ? Prec::BF16 : Prec::F64);
  L.rp = L.lp == Prec::F64 ? Prec::F64 : Prec::F64S;
  L.lpt = (int)L.lp;
  // common
  L.Boo = A.d(X * oo); L.Bov = A.d(X * ov); L.Bvv = A.d(X * vv);
  L.Kov = A.d(oovv);
  L.t1w = A.d(ov); L.t2w = A.d(oovv);
  L.hoo = A.d(oo); L.hov = A.d(ov); L.hvo = A.d(ov); L.hvv = A.d(vv);
  L.J = A.d(X);
  L.nrm = A.d(ov); L.jd = A.d(ov);
  L.scal = A.d(64);   // [0] energy, [1..16] Gram row, [32] ||R/D||^2, [40] (T) sum
  L.partials = A.d(17 * kRedBlocks);   // 16 Gram-row slices + the step norm
  L.splitk_elems = std::max<int64_t>({(int64_t)1 << 22, 64 * vv, 4 * oovv});
  L.splitk = A.d(L.splitk_elems);
  const size_t phase = A.off;
  L.phase_off = phase;
  // CCSD phase
  L.diis_m = std::max(1, (int)opt.diis_space);
  const int64_t N = ov + oovv;
  L.namp = N;
  // Ladder blocks: a in [a0, a0 + chunk_a) against b < a0 + chunk_a (only b <= a
  // is used); the (ac|bd) block takes chunk_a v^3 doubles.  About 16 blocks keep
  // the wasted b > a corner of each rectangle small.
  int64_t chunk_bytes = opt.ladder_chunk_bytes ? (int64_t)opt.ladder_chunk_bytes : (int64_t)8 << 30;
  L.chunk_a = std::max<int64_t>(1, std::min<int64_t>((v + 15) / 16, chunk_bytes / (8 * vvv)));
  L.Btoo = A.d(X * oo); L.Btai = A.d(X * ov); L.Btvv = A.d(X * vv);
  L.Foo = A.d(oo); L.Fov = A.d(ov); L.Fvo = A.d(ov); L.Fvv = A.d(vv);
  L.Foop = A.d(oo); L.Fvvp = A.d(vv);
  L.Pvv = A.d(oovv); L.Q2 = A.d(oovv); L.Lov = A.d(oovv);
  L.u = A.d(oovv); L.R1 = A.d(ov); L.R2 = A.d(oovv); L.S = A.d(oovv); L.Xc = A.d(oovv);
  L.Goovv = A.d(oovv); L.Cint = A.d(oovv); L.Dint = A.d(oovv);
  L.Wkl = A.d(oo * oo); L.Y1 = A.d(X * ov); L.Z1 = A.d(X * ov);
  L.Tsa = A.d(oovv); L.SA = A.d(oovv);
  {  // stored ladder: every b <= a block of the bare (ac|bd) plus the correction tensors
    const size_t esz = L.lp == Prec::F64 ? 8 : (L.lp == Prec::F32 ? 4 : 2);
    int64_t blk = 0;
    for (int64_t a0 = 0; a0 < v; a0 += L.chunk_a) {
      const int64_t na = std::min<int64_t>(L.chunk_a, v - a0);
      blk += na * (a0 + na) * vv;
    }
    L.lrows = blk / vv;
    const size_t need = (size_t)blk * esz + (size_t)(o * vvv + 2 * o * oo * v + oo * oo) * 8 +
                        (L.lp != Prec::F64 ? (size_t)X * vv * esz : 0);
    L.lstore = opt.ladder_mode == LNOCC_LADDER_STORED ||
               (opt.ladder_mode == LNOCC_LADDER_AUTO && need <= ((size_t)32 << 30));
    if (L.lstore) {
      L.Lst = A.d((int64_t)(((size_t)blk * esz + 7) / 8));
      L.Gkc = A.d(o * vvv);
      L.Zl = A.d(oo * ov);
      L.Yl = A.d(oo * ov);
      L.Wl = A.d(oo * oo);
      L.Bvv_lp = (L.lp != Prec::F64) ? A.d((int64_t)(((size_t)X * vv * esz + 7) / 8)) : nullptr;
    } else {
      L.chunk = A.d(L.chunk_a * vvv);
      L.Btvv_lp = (L.lp != Prec::F64) ? A.d(X * vv) : nullptr;
    }
  }
  L.dx = A.d(L.diis_m * N); L.de = A.d(L.diis_m * N);
  if (opt.guess == LNOCC_GUESS_MLP) {
    L.nunique = o * (o + 1) / 2 * vv;
    const int64_t rows = std::min<int64_t>(L.nunique, (int64_t)1 << 17);
    mlp::Scratch probe;
    mlp::plan_scratch(rows, false, nullptr, probe);
    char *mb = (char *)A.d((int64_t)((probe.bytes + 7) / 8));
    mlp::plan_scratch(rows, false, base ? mb : nullptr, L.ms);
  }
  const size_t ccsd_end = A.off;
  // (T) phase (aliases the CCSD scratch)
  A.off = phase;
  const int64_t nt = unique_triples(o);
  // (T) runs FP32 products in the FP32 and BF16 modes, FP64 products otherwise;
  // G and T carry the contracted index padded to vp (zeros beyond v)
  L.t_f32 = L.lp != Prec::F64;
  const int64_t tes = L.t_f32 ? 4 : 8, vp = triples_pad(v);
  auto dwords = [](int64_t bytes) { return (bytes + 7) / 8; };
  int64_t nb = opt.triples_batch;
  const int64_t wel = triples_w_elems(v, 1);   // W of one triple, blocked layout
  if (nb <= 0) nb = std::max<int64_t>(1, ((int64_t)2 << 30) / (tes * wel));
  nb = std::max<int64_t>(1, std::min<int64_t>({nb, std::max<int64_t>(nt, 1), 4096}));
  L.nb = (int)nb;
  L.ntriples = nt;
  L.Gt = A.d(dwords(ov * v * vp * tes)); L.Jt = A.d(dwords(oo * ov * tes));
  L.W = A.d(dwords(nb * wel * tes));
  L.t2_lp = A.d(dwords(oo * v * vp * tes));
  L.tpart_elems = triples_partials_capacity(nb);
  L.tpart = A.d(L.tpart_elems);
  L.table = A.i(3 * std::max<int64_t>(nt, 1));
  const size_t t_end = A.off;
  L.bytes = std::max(ccsd_end, t_end) + 256;
}

// ---------------------------------------------------------------- pieces
namespace {

// G_pq = sc * 2... : adds sc * sum_Q J_Q B_Qpq + sx * sum_Qk B_Qpk B_Qkq into the
// four Fock blocks.  Bai[Q][i][a] holds B[Q][a][i].
int fock_two_electron(const Layout &L, const double *Boo, const double *Bov, const double *Bai,
                      const double *Bvv, const double *J, double *Goo, double *Gov, double *Gvo,
                      double *Gvv, double sc, double sx, hipStream_t s) {
  const int64_t o = L.dm.o, v = L.dm.v, X = L.dm.X, ov = o * v, oo = o * o, vv = v * v;
  {  // Coulomb
    GemmDesc d = DESC(oo, 1, 1, 1, Goo, 1, 0, 0, 0, 1.0);
    SEG(d, X, 1, sc, OP(Boo, 1, 0, oo, 0), OP(J, 0, 0, 1, 0));
    LN_TRY(gett(d, s));
    d = DESC(ov, 1, 1, 1, Gov, 1, 0, 0, 0, 1.0);
    SEG(d, X, 1, sc, OP(Bov, 1, 0, ov, 0), OP(J, 0, 0, 1, 0));
    LN_TRY(gett(d, s));
    d = DESC(ov, v, 1, 1, Gvo, 1, o, 0, 0, 1.0);
    SEG(d, X, 1, sc, OP(Bai, v, 1, ov, 0), OP(J, 0, 0, 1, 0));
    LN_TRY(gett(d, s));
    d = DESC(vv, 1, 1, 1, Gvv, 1, 0, 0, 0, 1.0);
    SEG(d, X, 1, sc, OP(Bvv, 1, 0, vv, 0), OP(J, 0, 0, 1, 0));
    LN_TRY(gett(d, s));
  }
  {  // exchange, contraction over (Q, k)
    GemmDesc d = DESC(o, 1, o, 1, Goo, o, 0, 1, 0, 1.0);
    SEG(d, X * o, o, sx, OP(Boo, o, 0, oo, 1), OP(Boo, 1, 0, oo, o));
    LN_TRY(gett(d, s));
    d = DESC(o, 1, v, 1, Gov, v, 0, 1, 0, 1.0);
    SEG(d, X * o, o, sx, OP(Boo, o, 0, oo, 1), OP(Bov, 1, 0, ov, v));
    LN_TRY(gett(d, s));
    d = DESC(v, 1, o, 1, Gvo, o, 0, 1, 0, 1.0);
    SEG(d, X * o, o, sx, OP(Bai, 1, 0, ov, v), OP(Boo, 1, 0, oo, o));
    LN_TRY(gett(d, s));
    d = DESC(v, 1, v, 1, Gvv, v, 0, 1, 0, 1.0);
    SEG(d, X * o, o, sx, OP(Bai, 1, 0, ov, v), OP(Bov, 1, 0, ov, v));
    LN_TRY(gett(d, s));
  }
  return LNOCC_OK;
}

size_t ladder_esz(const Layout &L) {
  return L.lp == Prec::F64 ? 8 : (L.lp == Prec::F32 ? 4 : 2);
}

// Bare (ac|bd) for every block of a (b < a1 of the block) and (kc|bd), formed
// once per solve when the ladder is stored.
int build_stored_ladder(const Layout &L, hipStream_t s) {
  const int64_t o = L.dm.o, v = L.dm.v, X = L.dm.X, ov = o * v, vv = v * v, vvv = vv * v;
  const size_t esz = ladder_esz(L);
  const char *bvv = (const char *)L.Bvv;
  if (L.lp != Prec::F64) {
    LN_TRY(convert(L.Bvv, X * vv, L.Bvv_lp, L.lpt, s));
    bvv = (const char *)L.Bvv_lp;
  }
  char *dst = (char *)L.Lst;
  for (int64_t a0 = 0; a0 < v; a0 += L.chunk_a) {
    const int64_t na = std::min<int64_t>(L.chunk_a, v - a0), a1 = a0 + na;
    GemmDesc d = DESC(na * v, v, a1 * v, v, (double *)dst, a1 * vv, v, vv, 1, 0.0);
    SEG(d, X, 1, 1.0, OP((const double *)(bvv + a0 * v * esz), v, 1, vv, 0),
        OP((const double *)bvv, v, 1, vv, 0));
    d.kind = Kind::LadderBuild;
    d.prec = L.lp;
    d.c_type = L.lpt;
    LN_TRY(gett(d, s));
    dst += (size_t)na * a1 * vv * esz;
  }
  {  // Gkc[k][c][b][d] = (kc|bd)
    GemmDesc d = DESC(ov, 1, vv, 1, L.Gkc, vv, 0, 1, 0, 0.0);
    SEG(d, X, 1, 1.0, OP(L.Bov, 1, 0, ov, 0), OP(L.Bvv, 1, 0, vv, 0));
    LN_TRY(gett(d, s));
  }
  (void)vvv;
  return LNOCC_OK;
}

}  // namespace

// One-off: DF split, bare one-electron operator, (ia|jb) in the layouts used.
int setup_fragment(const Layout &L, const double *B, const double *eo, const double *ev,
                   bool ccsd_phase, hipStream_t s) {
  const int64_t o = L.dm.o, v = L.dm.v, X = L.dm.X, ov = o * v, oo = o * o, vv = v * v;
  const int64_t ovv = o * vv;
  LN_TRY(split_B(B, X, o, v, L.Boo, L.Bov, L.Bvv, s));
  {  // Kov[k][c][l][d] = (kc|ld)
    GemmDesc d = DESC(ov, 1, ov, 1, L.Kov, ov, 0, 1, 0, 0.0);
    SEG(d, X, 1, 1.0, OP(L.Bov, 1, 0, ov, 0), OP(L.Bov, 1, 0, ov, 0));
    LN_TRY(gett(d, s));
  }
  if (!ccsd_phase) return LNOCC_OK;
  // h = diag(eps) - G(B): f = h + G with every occupied orbital of the fragment correlated
  LN_TRY(dzero(L.hoo, oo * 8, s));
  LN_TRY(dzero(L.hov, ov * 8, s));
  LN_TRY(dzero(L.hvo, ov * 8, s));
  LN_TRY(dzero(L.hvv, vv * 8, s));
  LN_TRY(diag_sum(L.Boo, X, o, L.J, s));
  int st = fock_two_electron(L, L.Boo, L.Bov, L.Bov, L.Bvv, L.J, L.hoo, L.hov, L.hvo, L.hvv,
                             -2.0, 1.0, s);
  if (st) return st;
  LN_TRY(add_diag(L.hoo, o, o, eo, s));
  LN_TRY(add_diag(L.hvv, v, v, ev, s));
  {  // Pvv[k][l][d][c] = (ld|kc)
    GemmDesc d = DESC(ov, v, ov, v, L.Pvv, vv, v, ovv, 1, 0.0);
    SEG(d, X, 1, 1.0, OP(L.Bov, v, 1, ov, 0), OP(L.Bov, v, 1, ov, 0));
    LN_TRY(gett(d, s));
  }
  {  // Q2[k][l][c][d] = (kd|lc)
    GemmDesc d = DESC(ov, v, ov, v, L.Q2, ovv, 1, vv, v, 0.0);
    SEG(d, X, 1, 1.0, OP(L.Bov, v, 1, ov, 0), OP(L.Bov, v, 1, ov, 0));
    LN_TRY(gett(d, s));
  }
  LN_TRY(build_lov(L.Kov, o, v, L.Lov, s));
  if (L.lstore) {
    const int st2 = build_stored_ladder(L, s);
    if (st2) return st2;
  }
  return LNOCC_OK;
}

// Autotuning on the residual evaluation, which recomputes every intermediate
// from (t1, t2): one evaluation per candidate, each timed launch by launch.
// Both ring arithmetics of the reduced modes are tuned (each has its own shapes).
int tune_residuals(const Layout &L, const double *t1, const double *t2, hipStream_t s) {
  const int variants = L.rp != Prec::F64 ? 2 : 1;
  tune_probe_begin();
  int st = LNOCC_OK;
  for (int w = 0; w < variants && !st; ++w) st = ccsd_residuals(L, t1, t2, s, w == 1);
  const int unplanned = tune_probe_end();
  if (st || unplanned == 0) return st;
  for (int c = 0; c < tune_candidates() && !st; ++c) {
    tune_candidate(c);
    for (int w = 0; w < variants && !st; ++w) st = ccsd_residuals(L, t1, t2, s, w == 1);
  }
  tune_candidate(-1);
  tune_commit();
  if (log_enabled()) {
    std::fprintf(stderr, "lnocc: tuned %d residual contraction shapes (%zu plans)\n", unplanned,
                 tune_plans());
    std::fflush(stderr);
  }
  return st;
}

int ccsd_residuals(const Layout &L, const double *t1, const double *t2, hipStream_t s,
                   bool split_ring) {
  const int64_t o = L.dm.o, v = L.dm.v, X = L.dm.X;
  const Prec ring = split_ring ? L.rp : Prec::F64;
  // The early iterations of the reduced modes also take every sizeable FP64
  // contraction (the DF products over Q, the T1 dressing, the hole ladder) in
  // split-bf16 products; tiny products keep FP64 tiles and the matrix-vector path.
  auto run = [&](GemmDesc &d) {
    if (split_ring && d.prec == Prec::F64 && d.kind != Kind::LadderBuild) {
      int64_t K = 0;
      for (int q = 0; q < d.nseg; ++q) K += d.seg[q].K;
      if ((int64_t)d.M * d.N >= 65536 && K >= 256) d.prec = L.rp;
    }
    return gett(d, s);
  };
  const int64_t ov = o * v, oo = o * o, vv = v * v, ovv = o * vv, vvv = vv * v, ooo = oo * o;
  const size_t B8 = sizeof(double);
  // --- T1 dressing of the DF factors
  {  // B~_ij = B_ij + sum_b B_ib t_j^b
    GemmDesc d = DESC(o, 1, o, 1, L.Btoo, o, 0, 1, 0, 1.0);
    d.c_src = L.Boo;
    BATCH_Q(d, X, oo);
    SEG(d, v, 1, 1.0, OPB(OP(L.Bov, v, 0, 1, 0), ov, 0, 0), OP(t1, v, 0, 1, 0));
    LN_TRY(run(d));
  }
  // B~_ab = B_ab - sum_k t_k^a B_kb (a rank-nocc update of every B_Q: bandwidth-bound)
  LN_TRY(dress_vv(L.Bvv, L.Bov, t1, X, o, v, L.Btvv, s));
  {  // B~_ai = B_ai + sum_b B_ab t_i^b - sum_k t_k^a B~_ki, stored [Q][i][a]
    GemmDesc d = DESC(o, 1, v, 1, L.Btai, v, 0, 1, 0, 1.0);
    d.c_src = L.Bov;
    BATCH_Q(d, X, ov);
    SEG(d, v, 1, 1.0, OP(t1, v, 0, 1, 0), OPB(OP(L.Bvv, v, 0, 1, 0), vv, 0, 0));
    SEG(d, o, 1, -1.0, OPB(OP(L.Btoo, 1, 0, o, 0), oo, 0, 0), OP(t1, 1, 0, v, 0));
    LN_TRY(run(d));
  }
  LN_TRY(diag_sum(L.Btoo, X, o, L.J, s));
  // --- dressed Fock: F~ = Lm h Rm^T + G(B~)
  LN_TRY(dcopy(L.Foo, L.hoo, oo * B8, s));
  {
    GemmDesc d = DESC(o, 1, o, 1, L.Foo, o, 0, 1, 0, 1.0);
    SEG(d, v, 1, 1.0, OP(L.hov, v, 0, 1, 0), OP(t1, v, 0, 1, 0));
    LN_TRY(run(d));
  }
  LN_TRY(dcopy(L.Fov, L.hov, ov * B8, s));
  LN_TRY(dcopy(L.Fvv, L.hvv, vv * B8, s));
  {
    GemmDesc d = DESC(v, 1, v, 1, L.Fvv, v, 0, 1, 0, 1.0);
    SEG(d, o, 1, -1.0, OP(t1, 1, 0, v, 0), OP(L.hov, 1, 0, v, 0));
    LN_TRY(run(d));
  }
  LN_TRY(dcopy(L.Fvo, L.hvo, ov * B8, s));
  {
    GemmDesc d = DESC(v, 1, o, 1, L.Fvo, o, 0, 1, 0, 1.0);
    SEG(d, v, 1, 1.0, OP(L.hvv, v, 0, 1, 0), OP(t1, v, 0, 1, 0));
    SEG(d, o, 1, -1.0, OP(t1, 1, 0, v, 0), OP(L.Foo, 1, 0, o, 0));
    LN_TRY(run(d));
  }
  int st = fock_two_electron(L, L.Btoo, L.Bov, L.Btai, L.Btvv, L.J, L.Foo, L.Fov, L.Fvo, L.Fvv,
                             2.0, -1.0, s);
  if (st) return st;
  // --- singles residual
  LN_TRY(transpose2d(L.Fvo, v, o, L.R1, s));   // F~_ai
  LN_TRY(make_u(t2, o, v, L.u, s));
  {  // Y[Q][i][d] = sum_kc u_ki^cd B_Q,kc ; R1 += sum_Qd Y[Q][i][d] B~_Q,ad
    GemmDesc d = DESC(X, 1, ov, v, L.Y1, ov, 0, v, 1, 0.0);
    SEG(d, ov, v, 1.0, OP(L.Bov, ov, 0, v, 1), OP(L.u, vv, 1, ovv, v));
    LN_TRY(run(d));
    d = DESC(o, 1, v, 1, L.R1, v, 0, 1, 0, 1.0);
    SEG(d, X * v, v, 1.0, OP(L.Y1, v, 0, ov, 1), OP(L.Btvv, v, 0, vv, 1));
    LN_TRY(run(d));
  }
  {  // Z[Q][k][a] = sum_lc u_kl^ac B_Q,lc ; R1 -= sum_Qk B~_Q,ki Z[Q][k][a]
    GemmDesc d = DESC(X, 1, ov, v, L.Z1, ov, 0, v, 1, 0.0);
    SEG(d, ov, v, 1.0, OP(L.Bov, ov, 0, v, 1), OP(L.u, ovv, v, vv, 1));
    LN_TRY(run(d));
    d = DESC(o, 1, v, 1, L.R1, v, 0, 1, 0, 1.0);
    SEG(d, X * o, o, -1.0, OP(L.Btoo, 1, 0, oo, o), OP(L.Z1, 1, 0, ov, v));
    LN_TRY(run(d));
  }
  {  // R1 += sum_kc u_ik^ac F~_kc
    GemmDesc d = DESC(ov, v, 1, 1, L.R1, v, 1, 0, 0, 1.0);
    SEG(d, ov, v, 1.0, OP(L.u, ovv, v, vv, 1), OP(L.Fov, 0, 0, v, 1));
    LN_TRY(run(d));
  }
  // --- doubles residual: R2 <- (ai|bj)~
  {
    GemmDesc d = DESC(ov, v, ov, v, L.R2, ovv, v, vv, 1, 0.0);
    SEG(d, X, 1, 1.0, OP(L.Btai, v, 1, ov, 0), OP(L.Btai, v, 1, ov, 0));
    LN_TRY(run(d));
  }
  // Particle-particle ladder R_ij^ab = sum_cd t_ij^cd (ac|bd)~ through
  // S = R^ab + R^ba = sum_cd (t^cd + t^dc) (ac|bd) (symmetric in ij and ab) and
  // A = R^ab - R^ba = sum_cd (t^cd - t^dc) (ac|bd) (antisymmetric in both): the
  // (ac|bd) block is formed for b <= a only (half of the v^4 build) and
  // contracted with o^2 rows (i <= j for S, i < j for A) instead of 2 o^2.
  // In the FP32 / BF16 modes B~_vv, the (ac|bd) block and the rows are stored in
  // that precision; products accumulate in FP32 per tile and SA stays FP64.
  const bool lowp = L.lp != Prec::F64;
  const size_t esz = ladder_esz(L);
  LN_TRY(pack_t(t2, o, v, L.Tsa, L.lpt, s));
  if (L.lstore) {
    // Bare integrals: B~_ac = B_ac - sum_k t_k^a B_kc makes
    // (ac|bd)~ = (ac|bd) - t_k^a (kc|bd) - t_l^b (ac|ld) + t_k^a t_l^b (kc|ld), so
    // R_ij^ab = sum_cd t_ij^cd (ac|bd) - sum_k t_k^a (Z - Y)_ij,k^b - sum_k Z_ji,k^a t_k^b
    // with Z_ij,k^b = sum_cd t_ij^cd (kc|bd), Y_ij,k^b = sum_l W_ij,kl t_l^b and
    // W_ij,kl = sum_cd t_ij^cd (kc|ld).
    // one product over all stored rows (a, b < a1) of every block:
    // SA[r][row] = sum_cd Tsa[r][cd] (ac|bd)[row][cd]
    {
      GemmDesc d = DESC(L.lrows, 1, oo, 1, L.SA, 1, 0, L.lrows, 0, 0.0);
      SEG(d, vv, 1, 1.0, OP((const double *)L.Lst, vv, 0, 1, 0), OP(L.Tsa, vv, 0, 1, 0));
      d.kind = Kind::LadderContract;
      d.prec = L.lp;
      LN_TRY(run(d));
    }
    LN_TRY(unpack_ladder(L.SA, o, v, L.chunk_a, L.lrows, L.R2, s));
    (void)esz;
    {  // Z[ij][k][b] = sum_cd t_ij^cd (kc|bd)
      GemmDesc d = DESC(oo, 1, ov, v, L.Zl, ov, 0, v, 1, 0.0);
      SEG(d, vv, v, 1.0, OP(t2, vv, 0, v, 1), OP(L.Gkc, vvv, v, vv, 1));
      d.kind = Kind::Ring;
      d.prec = ring;
      LN_TRY(run(d));
    }
    {  // W[ij][k][l] = sum_cd t_ij^cd (kc|ld) ; Y[ij][k][b] = sum_l W[ij][k][l] t_l^b
      GemmDesc d = DESC(oo, 1, oo, o, L.Wl, oo, 0, o, 1, 0.0);
      SEG(d, vv, v, 1.0, OP(t2, vv, 0, v, 1), OP(L.Kov, ovv, v, ov, 1));
      LN_TRY(run(d));
      d = DESC(ooo, 1, v, 1, L.Yl, v, 0, 1, 0, 0.0);
      SEG(d, o, 1, 1.0, OP(L.Wl, o, 0, 1, 0), OP(t1, 1, 0, v, 0));
      LN_TRY(run(d));
    }
    {  // R2[ij][a][b] += -t1^T (Z - Y)_ij - Z_ji^T t1, batched over (i, j)
      GemmDesc d = DESC(v, 1, v, 1, L.R2, v, 0, 1, 0, 1.0);
      d.batch = (int)oo;
      d.nb1 = (int)o;
      d.c_b0 = ovv;
      d.c_b1 = vv;
      SEG(d, o, 1, -1.0, OP(t1, 1, 0, v, 0), OPB(OP(L.Zl, 1, 0, v, 0), oo * v, ov, 0));
      SEG(d, o, 1, 1.0, OP(t1, 1, 0, v, 0), OPB(OP(L.Yl, 1, 0, v, 0), oo * v, ov, 0));
      SEG(d, o, 1, -1.0, OPB(OP(L.Zl, 1, 0, v, 0), ov, oo * v, 0), OP(t1, 1, 0, v, 0));
      LN_TRY(run(d));
    }
  } else {
    const char *bvv = (const char *)L.Btvv;
    if (lowp) {
      LN_TRY(convert(L.Btvv, X * vv, L.Btvv_lp, L.lpt, s));
      bvv = (const char *)L.Btvv_lp;
    }
    for (int64_t a0 = 0; a0 < v; a0 += L.chunk_a) {
      const int64_t na = std::min<int64_t>(L.chunk_a, v - a0), a1 = a0 + na;
      GemmDesc d = DESC(na * v, v, a1 * v, v, L.chunk, vvv, v, vv, 1, 0.0);
      SEG(d, X, 1, 1.0, OP((const double *)(bvv + a0 * v * esz), v, 1, vv, 0),
          OP((const double *)bvv, v, 1, vv, 0));
      d.kind = Kind::LadderBuild;
      // FP32 mode: split-bf16 products (FP32-level accuracy at bf16 matrix-core rates)
      d.prec = L.lp == Prec::F32 ? Prec::F32S : L.lp;
      d.c_type = L.lpt;
      LN_TRY(run(d));
      // SA[r][a][b] = sum_cd Tsa[r][cd] g[a][b][cd], rows (a, b < a1) of the block
      d = DESC(na * a1, a1, oo, 1, L.SA + a0 * v, v, 1, vv, 0, 0.0);
      SEG(d, vv, 1, 1.0, OP(L.chunk, vvv, vv, 1, 0), OP(L.Tsa, vv, 0, 1, 0));
      d.kind = Kind::LadderContract;
      d.prec = L.lp;
      LN_TRY(run(d));
    }
    LN_TRY(unpack_ladder(L.SA, o, v, 0, vv, L.R2, s));
  }
  {  // hole-hole ladder: W_klij = (ki|lj)~ + sum_cd (kc|ld) t_ij^cd ; R2 += sum_kl t_kl^ab W_klij
    GemmDesc d = DESC(oo, o, oo, o, L.Wkl, ooo, o, oo, 1, 0.0);
    SEG(d, X, 1, 1.0, OP(L.Btoo, o, 1, oo, 0), OP(L.Btoo, o, 1, oo, 0));
    LN_TRY(run(d));
    d = DESC(oo, o, oo, 1, L.Wkl, ooo, oo, 1, 0, 1.0);
    SEG(d, vv, v, 1.0, OP(L.Kov, ovv, v, ov, 1), OP(t2, vv, 0, v, 1));
    LN_TRY(run(d));
    d = DESC(oo, 1, vv, 1, L.R2, vv, 0, 1, 0, 1.0);
    SEG(d, oo, 1, 1.0, OP(L.Wkl, 1, 0, oo, 0), OP(t2, 1, 0, vv, 0));
    LN_TRY(run(d));
  }
  {  // (ki|ac)~
    GemmDesc d = DESC(oo, 1, vv, 1, L.Goovv, vv, 0, 1, 0, 0.0);
    SEG(d, X, 1, 1.0, OP(L.Btoo, 1, 0, oo, 0), OP(L.Btvv, 1, 0, vv, 0));
    LN_TRY(run(d));
  }
  // exchange-type ring: Cint_kiac = (ki|ac)~ - 1/2 sum_ld t_li^ad (kd|lc); X_ijab = sum_kc t_kj^bc Cint_kiac
  {
    GemmDesc d = DESC(ov, v, ov, v, L.Cint, vv, v, ovv, 1, 1.0);
    d.c_src = L.Goovv;
    SEG(d, ov, v, -0.5, OP(t2, vv, v, ovv, 1), OP(L.Q2, ovv, v, vv, 1));
    d.kind = Kind::Ring;
    d.prec = ring;
    LN_TRY(run(d));
    d = DESC(ov, v, ov, v, L.Xc, ovv, v, vv, 1, 0.0);
    SEG(d, ov, v, 1.0, OP(L.Cint, vv, v, ovv, 1), OP(t2, vv, v, ovv, 1));
    d.kind = Kind::Ring;
    d.prec = ring;
    LN_TRY(run(d));
  }
  // Coulomb-type ring: Dint_iakc = 2 (ai|kc)~ - (ki|ac)~ + 1/2 sum_ld u_il^ad L_ldkc ;
  // S = 1/2 sum_kc u_jk^bc Dint_iakc
  {
    GemmDesc d = DESC(ov, 1, ov, 1, L.Dint, ov, 0, 1, 0, 0.0);
    SEG(d, X, 1, 2.0, OP(L.Btai, 1, 0, ov, 0), OP(L.Bov, 1, 0, ov, 0));
    LN_TRY(run(d));
    LN_TRY(sub_oovv_into_dint(L.Goovv, o, v, L.Dint, s));
    d = DESC(ov, v, ov, 1, L.Dint, ovv, ov, 1, 0, 1.0);
    SEG(d, ov, v, 0.5, OP(L.u, ovv, v, vv, 1), OP(L.Lov, 1, 0, ovv, ov));
    d.kind = Kind::Ring;
    d.prec = ring;
    LN_TRY(run(d));
    d = DESC(ov, v, ov, v, L.S, ovv, v, vv, 1, 0.0);
    SEG(d, ov, v, 0.5, OP(L.Dint, ovv, ov, v, 1), OP(L.u, ovv, v, vv, 1));
    d.kind = Kind::Ring;
    d.prec = ring;
    LN_TRY(run(d));
  }
  // Fock-type terms: F'_bc = F~_bc - sum_kld u_kl^bd (ld|kc), F'_kj = F~_kj + sum_lcd u_lj^cd (kd|lc)
  LN_TRY(dcopy(L.Fvvp, L.Fvv, vv * B8, s));
  {
    GemmDesc d = DESC(v, 1, v, 1, L.Fvvp, v, 0, 1, 0, 1.0);
    SEG(d, oo * v, v, -1.0, OP(L.u, v, 0, vv, 1), OP(L.Pvv, 1, 0, vv, v));
    LN_TRY(run(d));
  }
  LN_TRY(dcopy(L.Foop, L.Foo, oo * B8, s));
  {
    GemmDesc d = DESC(o, 1, o, 1, L.Foop, o, 0, 1, 0, 1.0);
    SEG(d, o * vv, vv, 1.0, OP(L.Q2, ovv, 0, vv, 1), OP(L.u, vv, 0, ovv, 1));
    LN_TRY(run(d));
  }
  {  // S += sum_c t_ij^ac F'_bc - sum_k t_ik^ab F'_kj
    GemmDesc d = DESC(oo * v, 1, v, 1, L.S, v, 0, 1, 0, 1.0);
    SEG(d, v, 1, 1.0, OP(t2, v, 0, 1, 0), OP(L.Fvvp, v, 0, 1, 0));
    LN_TRY(run(d));
    d = DESC(o * vv, vv, o, 1, L.S, ovv, 1, vv, 0, 1.0);
    SEG(d, o, 1, -1.0, OP(t2, ovv, 1, vv, 0), OP(L.Foop, 1, 0, o, 0));
    LN_TRY(run(d));
  }
  LN_TRY(combine_r2(L.R2, L.S, L.Xc, o, v, s));
  // The residual of pair-symmetric amplitudes is pair-symmetric; rounding (of
  // split products above all) breaks that slightly, and an antisymmetric part
  // left in R2 would pass into t2, where no later iteration removes it.
  LN_TRY(pair_symmetrize(L.R2, o, v, s));
  return LNOCC_OK;
}

int energy(const Layout &L, const double *t1, const double *t2, double *dev_out, hipStream_t s) {
  LN_TRY(energy_partials(L.Kov, t1, t2, L.dm.o, L.dm.v, L.partials, s));
  LN_TRY(reduce_partials(L.partials, kRedBlocks, dev_out, 0, s));
  return LNOCC_OK;
}

// ---------------------------------------------------------------- DIIS
namespace {
// Solves the (m+1) x (m+1) Pulay system for the extrapolation weights.
bool diis_weights(const std::vector<double> &G, int m, int ld, std::vector<double> &c) {
  const int n = m + 1;
  std::vector<double> A(n * n, 0.0), b(n, 0.0);
  double scale = 0.0;
  for (int i = 0; i < m; ++i) scale = std::max(scale, std::fabs(G[i * ld + i]));
  if (!(scale > 0.0) || !std::isfinite(scale)) return false;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) A[i * n + j] = G[i * ld + j] / scale;
  for (int i = 0; i < m; ++i) { A[i * n + m] = -1.0; A[m * n + i] = -1.0; }
  b[m] = -1.0;
  for (int col = 0; col < n; ++col) {   // Gaussian elimination, partial pivoting
    int p = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(A[r * n + col]) > std::fabs(A[p * n + col])) p = r;
    if (std::fabs(A[p * n + col]) < 1e-14) return false;
    if (p != col) {
      for (int k = 0; k < n; ++k) std::swap(A[p * n + k], A[col * n + k]);
      std::swap(b[p], b[col]);
    }
    for (int r = col + 1; r < n; ++r) {
      const double f = A[r * n + col] / A[col * n + col];
      for (int k = col; k < n; ++k) A[r * n + k] -= f * A[col * n + k];
      b[r] -= f * b[col];
    }
  }
  std::vector<double> x(n);
  for (int r = n - 1; r >= 0; --r) {
    double acc = b[r];
    for (int k = r + 1; k < n; ++k) acc -= A[r * n + k] * x[k];
    x[r] = acc / A[r * n + r];
  }
  c.assign(x.begin(), x.begin() + m);
  for (double w : c)
    if (!std::isfinite(w)) return false;
  return true;
}
}  // namespace

// ---------------------------------------------------------------- CCSD driver
// The readback buffer is pinned so that copies stay asynchronous and the host
// can work on other fragments while one is in flight.
Readback::Readback() {
  if (dry_run()) {
    host = (double *)std::calloc(64, sizeof(double));
    return;
  }
  if (hipHostMalloc((void **)&host, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    note_error("hipHostMalloc of a readback buffer failed");
    host = nullptr;
  }
  if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
    note_error("hipEventCreate failed");
    ev = nullptr;
  }
}

Readback::Readback(double *buffer) : host(buffer), ev(nullptr), external(true) {}

Readback::~Readback() {
  if (external) return;
  if (dry_run()) {
    std::free(host);
    return;
  }
  if (host) (void)hipHostFree(host);
  if (ev) (void)hipEventDestroy(ev);
}

bool Readback::ok() const {
  return host != nullptr && (dry_run() || external || ev != nullptr);
}

CcsdRun::CcsdRun(const Layout &L_, const Inputs &in_, const lnocc_options_t &opt_, hipStream_t s_,
                 Readback &rb_)
    : L(&L_), in(in_), opt(opt_), s(s_), rb(&rb_), host(rb_.host),
      G((size_t)L_.diis_m * L_.diis_m, 0.0), split(L_.rp != Prec::F64) {}

CcsdRun::~CcsdRun() {
  for (hipGraphExec_t g : graph)
    if (g) (void)hipGraphExecDestroy(g);
}

// Reduced modes: the residual products run as split bf16 (FP32-class) in the
// early iterations and in FP64 from the first iteration whose step norm is
// within kSplitRingFactor of the threshold, or that fails twice in a row to
// reach a new minimum (the rounding of the split products then limits the
// step); the last iterations are FP64, so that rounding never sets the result.
bool CcsdRun::split_ring() const { return split; }

// The residual evaluation enqueues the same ~100 launches with the same
// arguments in every iteration of a solve (only the amplitude values change),
// so it is captured once per ring arithmetic and replayed.  It records no
// memset (copies only).
int CcsdRun::residuals() {
  const bool split = split_ring();
  if (!opt.graphs || dry_run() || profile_enabled())
    return ccsd_residuals(*L, in.t1, in.t2, s, split);
  hipGraphExec_t &graph = this->graph[split ? 1 : 0];
  if (!graph) {   // captured on a stream of its own (the caller's may be the null stream)
    hipStream_t cs = nullptr;
    LN_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      (void)hipStreamDestroy(cs);
      LN_TRY(e);
    }
    const int st = ccsd_residuals(*L, in.t1, in.t2, cs, split);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (st) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    LN_TRY(e);
    const hipError_t e2 = hipGraphInstantiate(&graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) {
      graph = nullptr;
      LN_TRY(e2);
    }
  }
  LN_TRY(hipGraphLaunch(graph, s));
  return LNOCC_OK;
}

hipError_t CcsdRun::mark() {
  return (dry_run() || !rb->ev) ? hipSuccess : hipEventRecord(rb->ev, s);
}

int CcsdRun::poll() const {
  if (dry_run()) return (++polls % 3 == 0) ? 1 : 0;   // exercises the pending state
  const hipError_t e = rb->ev ? hipEventQuery(rb->ev) : hipStreamQuery(s);
  if (e == hipSuccess) return 1;
  if (e == hipErrorNotReady) return 0;
  note_error("hipEventQuery failed (%s)", hipGetErrorString(e));
  return LNOCC_EDEVICE;
}

hipError_t CcsdRun::wait() const {
  if (dry_run()) return hipSuccess;
  return rb->ev ? hipEventSynchronize(rb->ev) : hipStreamSynchronize(s);
}

// Learned start: first the residual at the MP2 start, whose Jacobi step and
// error become the first DIIS pair (slot 0; also the fallback) and whose step
// norm goes to scal[33] (||e||^2 to scal[34]); then t2 += the network's
// correction over the unique amplitudes, chunk by chunk.
int CcsdRun::learned_start() {
  const int64_t o = L->dm.o, v = L->dm.v, N = L->namp;
  int st = ccsd_residuals(*L, in.t1, in.t2, s, split_ring());
  if (st) return st;
  install_splitk_scratch(L->splitk, (size_t)L->splitk_elems);
  LN_TRY(jacobi_step(in.t1, in.t2, L->R1, L->R2, in.eo, in.ev, o, v, opt.level_shift, L->dx,
                     L->de, L->partials + 16 * kRedBlocks, s));
  LN_TRY(reduce_partials(L->partials + 16 * kRedBlocks, kRedBlocks, L->scal + 33, 0, s));
  LN_TRY(dot_partials(L->de, N, 1, L->de, N, L->partials, s));
  LN_TRY(reduce_rows(L->partials, 1, L->scal + 34, s));
  LN_TRY(mlp::pair_stats(L->Boo, L->Bov, L->Bvv, L->dm.X, o, v, L->nrm, L->jd, s));
  const mlp::Scratch &S = L->ms;
  for (int64_t u0 = 0; u0 < L->nunique; u0 += S.rows) {
    const int64_t m = std::min<int64_t>(S.rows, L->nunique - u0);
    // raw features go to h2, which the forward pass reads before overwriting
    LN_TRY(mlp::features(L->Kov, in.eo, in.ev, L->nrm, L->jd, o, v, nullptr, u0, m, nullptr, S.h2,
                         nullptr, s));
    LN_TRY(mlp::forward(opt.mlp, S.h2, m, S, s));
    LN_TRY(mlp::apply_guess(opt.mlp, S.y, o, v, u0, m, in.t2, s));
  }
  return LNOCC_OK;
}

int CcsdRun::begin() {
  install_splitk_scratch(L->splitk, (size_t)L->splitk_elems);
  const int64_t o = L->dm.o, v = L->dm.v;
  int st = setup_fragment(*L, in.B, in.eo, in.ev, true, s);
  if (st) return st;
  // MP2 energy (always from the MP1 amplitudes) and the starting point
  if (opt.guess != LNOCC_GUESS_USER) {
    LN_TRY(mp2_guess(L->Kov, in.eo, in.ev, o, v, in.t1, in.t2, s));
    st = energy(*L, in.t1, in.t2, L->scal, s);
  } else {
    LN_TRY(mp2_guess(L->Kov, in.eo, in.ev, o, v, L->R1, L->R2, s));
    st = energy(*L, L->R1, L->R2, L->scal, s);
  }
  if (st) return st;
  if (opt.guess == LNOCC_GUESS_MLP) {
    st = learned_start();
    if (st) return st;
  }
  LN_TRY(d2h(host, L->scal, 40 * 8, s));
  LN_TRY(mark());
  phase = Phase::Started;
  return LNOCC_OK;
}

int CcsdRun::enqueue_iteration() {
  install_splitk_scratch(L->splitk, (size_t)L->splitk_elems);
  const int64_t o = L->dm.o, v = L->dm.v, N = L->namp;
  ++it;
  if (it == 1 && opt.autotune && !dry_run()) {
    const int st = tune_residuals(*L, in.t1, in.t2, s);
    if (st) return st;
  }
  int st = residuals();
  if (st) return st;
  const int m = L->diis_m;
  // (a learned start begins with the MP2 start's pair already in the subspace)
  use_diis = (m > 1) && (it >= opt.diis_start || count > 0);
  slot = use_diis ? (count % m) : 0;
  double *xs = L->dx + (int64_t)slot * N, *es = L->de + (int64_t)slot * N;
  double *rnorm = L->scal + 32;   // ||R / D||^2 of the current iterate
  LN_TRY(jacobi_step(in.t1, in.t2, L->R1, L->R2, in.eo, in.ev, o, v, opt.level_shift, xs, es,
                     L->partials + 16 * kRedBlocks, s));
  LN_TRY(reduce_partials(L->partials + 16 * kRedBlocks, kRedBlocks, rnorm, 0, s));
  nvalid = use_diis ? std::min(count + 1, m) : 1;
  const double *ebase = use_diis ? L->de : es;
  LN_TRY(dot_partials(ebase, N, nvalid, es, N, L->partials, s));
  LN_TRY(reduce_rows(L->partials, nvalid, L->scal + 1, s));
  LN_TRY(d2h(host, L->scal, 40 * 8, s));
  LN_TRY(mark());
  phase = Phase::Iterating;
  return LNOCC_OK;
}

// After the readback of an iteration: convergence test and DIIS; enqueues the
// next iterate.  Returns OK, an error, or sets phase = Converged / Exhausted.
int CcsdRun::after_iteration() {
  install_splitk_scratch(L->splitk, (size_t)L->splitk_elems);
  const int64_t o = L->dm.o, v = L->dm.v, N = L->namp;
  const int m = L->diis_m;
  double *xs = L->dx + (int64_t)slot * N, *es = L->de + (int64_t)slot * N;
  const double r2 = host[32];
  out.residual = std::sqrt(std::max(r2, 0.0));
  out.n_iter = it + (opt.guess == LNOCC_GUESS_MLP ? 1 : 0);
  if (mlp_check) {   // judge the learned start by its first step against the MP2 start's
    mlp_check = false;
    const double gram = host[1 + (use_diis ? slot : 0)];
    if (!std::isfinite(r2) || !std::isfinite(gram) || out.residual > r_mp2) {
      if (log_enabled()) {
        std::fprintf(stderr, "lnocc: learned start rejected (step %.3e, MP2 start %.3e)\n",
                     out.residual, r_mp2);
        std::fflush(stderr);
      }
      out.guess_used = LNOCC_GUESS_MP2;
      out.residual = r_mp2;
      LN_TRY(scatter_vec(L->dx, o, v, in.t1, in.t2, s));   // the MP2 path's first iterate
      std::fill(G.begin(), G.end(), 0.0);
      count = 0;
      growth = 0;
      prev = best = r_mp2;
      if (opt.on_iter) opt.on_iter(in.frag, it, out.e_mp2, out.residual, opt.user);
      if (r_mp2 <= in.conv_tol) phase = Phase::Converged;
      else if (it >= opt.max_iter) phase = Phase::Exhausted;
      return LNOCC_OK;
    }
  }
  if (log_enabled()) {
    std::fprintf(stderr, "lnocc: iteration %d residual %.3e energy %.12f\n", it, out.residual,
                 it > 1 ? host[0] : out.e_mp2);
    std::fflush(stderr);
  }
  if (!std::isfinite(r2) || !std::isfinite(host[1 + (use_diis ? slot : 0)])) {
    note_error("non-finite residual norm or DIIS overlap at iteration %d", it);
    return LNOCC_ENUMERIC;
  }
  if (opt.on_iter) opt.on_iter(in.frag, it, it > 1 ? host[0] : out.e_mp2, out.residual, opt.user);
  // end of the split phase (the DIIS subspace keeps its vectors: restarting it
  // here measured two more iterations)
  if (split) {
    split_stall = (out.residual < 0.9 * best) ? 0 : split_stall + 1;
    if (out.residual <= kSplitRingFactor * in.conv_tol || split_stall >= 2) {
      split = false;
      if (log_enabled()) {
        std::fprintf(stderr, "lnocc: FP64 residual products from iteration %d on\n", it + 1);
        std::fflush(stderr);
      }
    }
  }
  if (out.residual <= in.conv_tol) {
    LN_TRY(scatter_vec(xs, o, v, in.t1, in.t2, s));
    phase = Phase::Converged;
    return LNOCC_OK;
  }
  // DIIS safeguard: a residual that grows three iterations in a row, or far
  // above the best one seen, restarts the subspace from the current vector.
  growth = (out.residual > prev) ? growth + 1 : 0;
  prev = out.residual;
  best = std::min(best, out.residual);
  const bool restart = use_diis && count > 0 && (growth >= 3 || out.residual > 1e3 * best);
  if (restart) growth = 0;
  bool extrap = false;
  if (use_diis) {
    if (restart) {
      std::fill(G.begin(), G.end(), 0.0);
      if (slot != 0) {
        LN_TRY(dcopy(L->dx, xs, N * 8, s));
        LN_TRY(dcopy(L->de, es, N * 8, s));
      }
      G[0] = host[1 + slot];
      count = 1;
    } else {
      for (int q = 0; q < nvalid; ++q) {
        G[slot * m + q] = host[1 + q];
        G[q * m + slot] = host[1 + q];
      }
      ++count;
      if (nvalid >= 2) {
        std::vector<double> c;
        if (diis_weights(G, nvalid, m, c)) {
          LN_TRY(lincomb(L->dx, N, nvalid, c.data(), o, v, in.t1, in.t2, s));
          extrap = true;
        } else {
          std::fill(G.begin(), G.end(), 0.0);   // ill-conditioned: restart from this vector
          if (slot != 0) {
            LN_TRY(dcopy(L->dx, xs, N * 8, s));
            LN_TRY(dcopy(L->de, es, N * 8, s));
          }
          G[0] = host[1 + slot];
          count = 1;
        }
      }
    }
  }
  if (!extrap) LN_TRY(scatter_vec(xs, o, v, in.t1, in.t2, s));
  if (log_enabled() || opt.on_iter) {   // energy of the new iterate, read back with the
                                        // next Gram row (for the log and the callback)
    const int st2 = energy(*L, in.t1, in.t2, L->scal, s);
    if (st2) return st2;
  }
  if (it >= opt.max_iter) phase = Phase::Exhausted;
  return LNOCC_OK;
}

int CcsdRun::enqueue_final() {
  install_splitk_scratch(L->splitk, (size_t)L->splitk_elems);
  const int st = energy(*L, in.t1, in.t2, L->scal, s);
  if (st) return st;
  LN_TRY(d2h(host, L->scal, 8, s));
  LN_TRY(mark());
  return LNOCC_OK;
}

int CcsdRun::after_final() {
  out.e_ccsd = host[0];
  if (!std::isfinite(out.e_ccsd)) {
    note_error("non-finite CCSD energy");
    return LNOCC_ENUMERIC;
  }
  out.status = (phase == Phase::Converged) ? LNOCC_OK : LNOCC_NOT_CONVERGED;
  return out.status;
}

int CcsdRun::after_begin() {
  out.e_mp2 = host[0];
  out.n_iter = 0;
  out.residual = 0.0;
  out.status = LNOCC_OK;
  out.guess_used = opt.guess;
  if (opt.guess == LNOCC_GUESS_MLP) {
    mlp_check = true;
    r_mp2 = std::sqrt(std::max(host[33], 0.0));
    if (!std::isfinite(r_mp2) || !std::isfinite(host[34])) {
      note_error("non-finite residual at the MP2 start");
      return LNOCC_ENUMERIC;
    }
    if (L->diis_m > 1) {   // the MP2 start's step seeds the DIIS subspace
      G[0] = host[34];
      count = 1;
    }
  }
  if (opt.max_iter == 0) phase = Phase::Converged;
  return LNOCC_OK;
}

int CcsdRun::enqueue_t() {
  const int st = enqueue_triples(*L, in, s, opt.autotune != 0);
  if (st) return st;
  LN_TRY(d2h(host + 40, L->scal + 40, 8, s));
  LN_TRY(mark());
  return LNOCC_OK;
}

int CcsdRun::after_t() {
  out.e_t = host[40];
  if (std::isfinite(out.e_t)) return LNOCC_OK;
  note_error("non-finite (T) energy");
  return LNOCC_ENUMERIC;
}

int run_ccsd(const Layout &L, const Inputs &in, const lnocc_options_t &opt, Outputs &out,
             hipStream_t s, Readback *rbx) {
  std::unique_ptr<Readback> own;
  if (!rbx) {
    own.reset(new Readback());
    rbx = own.get();
  }
  if (!rbx->ok()) return LNOCC_EDEVICE;
  CcsdRun r(L, in, opt, s, *rbx);
  int st = r.begin();
  if (st) return st;
  LN_TRY(r.wait());
  st = r.after_begin();
  if (st) { out = r.out; return st; }
  while (r.phase != CcsdRun::Phase::Converged && r.phase != CcsdRun::Phase::Exhausted) {
    st = r.enqueue_iteration();
    if (st) return st;
    LN_TRY(r.wait());
    st = r.after_iteration();
    if (st) { out = r.out; return st; }
  }
  st = r.enqueue_final();
  if (st) return st;
  LN_TRY(r.wait());
  st = r.after_final();
  out = r.out;
  return st;
}

// ---------------------------------------------------------------- (T)
// Enqueues the whole (T) computation; the FP64 sum lands in L.scal[40].
int enqueue_triples(const Layout &L, const Inputs &in, hipStream_t s, bool autotune) {
  install_splitk_scratch(L.splitk, (size_t)L.splitk_elems);
  const int64_t o = L.dm.o, v = L.dm.v, X = L.dm.X;
  const int64_t ov = o * v, oo = o * o, vv = v * v, ovv = o * vv, vvv = vv * v;
  const int64_t ovo = ov * o, vo = v * o;
  const double *t1 = in.t1, *t2 = in.t2;
  double *acc = L.scal + 40;
  LN_TRY(dzero(acc, 8, s));
  if (L.ntriples == 0) return LNOCC_OK;
  // In the FP32 / BF16 modes the integrals and amplitudes entering W are
  // stored as FP32 and W itself is FP32; the energy sum is FP64.
  const int64_t vp = triples_pad(v), tes = L.t_f32 ? 4 : 8;
  if (v * v * vp * tes >= ((int64_t)1 << 32) || o * v * vp >= ((int64_t)1 << 32)) {
    note_error("(T): nvir %lld is beyond the 32-bit offsets of the W kernel", (long long)v);
    return LNOCC_EINVAL;
  }
  const int ttype = L.t_f32 ? 1 : 0;
  if (vp > v) LN_TRY(dzero(L.Gt, (size_t)(ov * v * vp * tes), s));
  {  // Gt[i][a][b][d] = (ai|bd), d padded to vp; stored in FP32 in the reduced modes,
     // so formed there by split-bf16 products (FP32-level accuracy) from the FP64 factors
    GemmDesc d = DESC(ov, 1, vv, v, L.Gt, v * vp, 0, vp, 1, 0.0);
    SEG(d, X, 1, 1.0, OP(L.Bov, 1, 0, ov, 0), OP(L.Bvv, v, 1, vv, 0));
    d.c_type = ttype;
    if (ttype == 1) d.prec = Prec::F64S;
    LN_TRY(gett(d, s));
  }
  {  // Jt[j][k][c][l] = (ck|jl)
    GemmDesc d = DESC(ov, v, oo, o, L.Jt, vo, o, ovo, 1, 0.0);
    SEG(d, X, 1, 1.0, OP(L.Bov, v, 1, ov, 0), OP(L.Boo, o, 1, oo, 0));
    d.c_type = ttype;
    LN_TRY(gett(d, s));
  }
  LN_TRY(triples_pad_t2(t2, o, v, L.t2_lp, ttype, s));
  const int wtype = ttype;
  LN_TRY(triples_table(L.table, o, s));
  (void)autotune;
  (void)ovv;
  // Triples with three distinct labels take all twelve terms of W (three
  // orientations of four).  With i = j, W is symmetric under a <-> b: the second
  // particle and hole terms of orientation 0 are the first ones with a and b
  // exchanged, and orientation 2 is orientation 1 with a and b exchanged, so
  // W = Z + Z(a <-> b) with Z = the first two terms of orientation 0 plus
  // orientation 1: half the products.  Likewise with j = k (b <-> c):
  // Z = orientation 0 plus the first two terms of orientation 2.  Z is what
  // goes to memory; the energy kernel forms W from it as it reads.
  const int64_t n0 = o * (o - 1) * (o - 2) / 6, n1 = o * (o - 1) / 2;
  const int64_t gstart[3] = {0, n0, n0 + n1}, gcount[3] = {n0, n1, n1};
  for (int g = 0; g < 3; ++g)
    for (int64_t t0 = gstart[g]; t0 < gstart[g] + gcount[g]; t0 += L.nb) {
      const int nb = (int)std::min<int64_t>(L.nb, gstart[g] + gcount[g] - t0);
      const int *table = L.table + 3 * t0;
      auto w = [&](int ori, int accumulate, int nterms) {
        return triples_w(L.Gt, L.t2_lp, L.Jt, L.W, table, nb, o, v, ori, ttype, accumulate,
                         nterms, 1, s);
      };
      if (g == 0) {
        LN_TRY(w(0, 0, 2));
        LN_TRY(w(1, 1, 2));
        LN_TRY(w(2, 1, 2));
      } else if (g == 1) {
        LN_TRY(w(0, 0, 1));
        LN_TRY(w(1, 1, 2));
      } else {
        LN_TRY(w(0, 0, 2));
        LN_TRY(w(2, 1, 1));
      }
      if (log_enabled() && ((t0 - gstart[g]) / L.nb) % 8 == 0) {
        std::fprintf(stderr, "lnocc: (T) group %d triples %lld..%lld of %lld\n", g,
                     (long long)t0, (long long)(t0 + nb), (long long)L.ntriples);
        std::fflush(stderr);
      }
      int64_t nparts = 0;
      // groups 1 and 2 leave Z in L.W; the energy kernel adds the exchanged partner
      LN_TRY(triples_energy(L.W, wtype, g, table, nb, L.Kov, t1, in.eo, in.ev, o, v, L.tpart,
                            L.tpart_elems, &nparts, s));
      LN_TRY(reduce_partials(L.tpart, nparts, acc, 1, s));
    }
  return LNOCC_OK;
}

int run_triples(const Layout &L, const Inputs &in, Outputs &out, hipStream_t s,
                bool autotune, double *hostx) {
  int st = enqueue_triples(L, in, s, autotune);
  if (st) return st;
  double *host = hostx;
  if (dry_run()) {
    out.e_t = 0.0;
    return LNOCC_OK;
  }
  if (!host && hipHostMalloc((void **)&host, sizeof(double), hipHostMallocDefault) != hipSuccess)
    return LNOCC_EDEVICE;
  hipError_t e = d2h(host, L.scal + 40, 8, s);
  if (e == hipSuccess) e = dsync(s);
  out.e_t = *host;
  if (!hostx) (void)hipHostFree(host);
  if (e != hipSuccess) return LNOCC_EDEVICE;
  if (!std::isfinite(out.e_t)) return LNOCC_ENUMERIC;
  return LNOCC_OK;
}

}  // namespace lnocc

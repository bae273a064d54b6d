// extern "C" entry points of liblnocc: argument validation on the host, then
// the solver of solver.hip on the caller's stream and workspace.
#include <cmath>
#include <climits>
#include <cstring>
#include <vector>

#include "../../include/lnocc.h"
#include "gett.h"
#include "solver.h"

using namespace lnocc;

namespace {

int check_sizes(const lnocc_fragment_t *f) {
  if (!f) return LNOCC_EINVAL;
  if (f->nocc <= 0 || f->nvir <= 0 || f->naux <= 0) return LNOCC_EINVAL;
  if (f->nocc > 1024 || f->nvir > 4096 || f->naux > 65535) return LNOCC_EINVAL;
  const int64_t o = f->nocc, v = f->nvir;
  // every contraction extent must fit the 32-bit index space of the kernels
  if (o * v * v > INT32_MAX || o * o * v > INT32_MAX || (int64_t)f->naux * o * v > INT32_MAX)
    return LNOCC_EINVAL;
  return LNOCC_OK;
}

int check_options(const lnocc_options_t *opt) {
  if (!opt) return LNOCC_EINVAL;
  if (opt->precision != LNOCC_FP64 && opt->precision != LNOCC_FP32 && opt->precision != LNOCC_BF16)
    return LNOCC_EINVAL;
  if (opt->guess != LNOCC_GUESS_MP2 && opt->guess != LNOCC_GUESS_USER) return LNOCC_EINVAL;
  if (opt->max_iter < 0 || opt->diis_space < 1 || opt->diis_space > 16 || opt->diis_start < 1 ||
      opt->triples_batch < 0 || !(opt->level_shift >= 0.0) || !std::isfinite(opt->level_shift))
    return LNOCC_EINVAL;
  return LNOCC_OK;
}

int check_pointers(const lnocc_fragment_t *f, bool need_amplitudes) {
  if (!f->B || !f->eps_occ || !f->eps_vir) return LNOCC_EINVAL;
  if (need_amplitudes && (!f->t1 || !f->t2)) return LNOCC_EINVAL;
  return LNOCC_OK;
}

int check_workspace(const Layout &L, const lnocc_options_t *opt) {
  if (!opt->workspace) return LNOCC_ENOMEM;
  if (((uintptr_t)opt->workspace) % 256) return LNOCC_EINVAL;
  if (opt->workspace_bytes < L.bytes) return LNOCC_ENOMEM;
  return LNOCC_OK;
}

// The semi-canonical energies must be finite and gapped (e_i < e_a for all i, a):
// every denominator of the amplitude equations and of (T) is then nonzero.
int check_spectrum(const lnocc_fragment_t *f, hipStream_t s) {
  if (dry_run()) return LNOCC_OK;
  std::vector<double> eo(f->nocc), ev(f->nvir);
  if (hipMemcpyAsync(eo.data(), f->eps_occ, eo.size() * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(ev.data(), f->eps_vir, ev.size() * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return LNOCC_EDEVICE;
  double omax = -INFINITY, vmin = INFINITY;
  for (double e : eo) {
    if (!std::isfinite(e)) return LNOCC_EINVAL;
    omax = std::max(omax, e);
  }
  for (double e : ev) {
    if (!std::isfinite(e)) return LNOCC_EINVAL;
    vmin = std::min(vmin, e);
  }
  return (omax < vmin) ? LNOCC_OK : LNOCC_EINVAL;
}

Dims dims_of(const lnocc_fragment_t *f) { return Dims{f->nocc, f->nvir, f->naux}; }

// Installs the address guard of the contraction launcher for one call.
struct Guard {
  Region r[6];
  Guard(const lnocc_fragment_t *f, const lnocc_options_t *opt, const Layout &L) {
    install_splitk_scratch(L.splitk, (size_t)L.splitk_elems);
    const size_t o = f->nocc, v = f->nvir, X = f->naux, n = o + v;
    int k = 0;
    r[k++] = Region{opt->workspace, opt->workspace_bytes};
    r[k++] = Region{f->B, X * n * n * 8};
    r[k++] = Region{f->eps_occ, o * 8};
    r[k++] = Region{f->eps_vir, v * 8};
    r[k++] = Region{f->t1, f->t1 ? o * v * 8 : 0};
    r[k++] = Region{f->t2, f->t2 ? o * o * v * v * 8 : 0};
    install_regions(r, k);
  }
  ~Guard() {
    install_regions(nullptr, 0);
    install_splitk_scratch(nullptr, 0);
  }
};

int prepare(lnocc_fragment_t *f, const lnocc_options_t *opt, bool need_amplitudes,
            bool need_tol, Layout &L) {
  int st = check_sizes(f);
  if (!st) st = check_options(opt);
  if (!st) st = check_pointers(f, need_amplitudes);
  if (!st && need_tol && !(f->conv_tol > 0.0 && std::isfinite(f->conv_tol))) st = LNOCC_EINVAL;
  if (st) return st;
  plan_layout(dims_of(f), *opt, (char *)opt->workspace, L);
  st = check_workspace(L, opt);
  if (st) return st;
  return check_spectrum(f, (hipStream_t)opt->stream);
}

int finish(lnocc_fragment_t *f, int st) {
  if (f) f->status = st;
  return st;
}

}  // namespace

extern "C" {

void lnocc_default_options(lnocc_options_t *opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->precision = LNOCC_FP64;
  opt->guess = LNOCC_GUESS_MP2;
  opt->do_triples = 1;
  opt->max_iter = 100;
  opt->diis_space = 8;
  opt->diis_start = 2;
}

const char *lnocc_status_string(int status) {
  switch (status) {
    case LNOCC_OK: return "LNOCC_OK";
    case LNOCC_NOT_CONVERGED: return "LNOCC_NOT_CONVERGED: iteration limit reached";
    case LNOCC_EINVAL: return "LNOCC_EINVAL: invalid argument";
    case LNOCC_ENOMEM: return "LNOCC_ENOMEM: workspace missing or too small";
    case LNOCC_EDEVICE: return "LNOCC_EDEVICE: HIP runtime error";
    case LNOCC_ENUMERIC: return "LNOCC_ENUMERIC: non-finite value";
    default: return "LNOCC: unknown status";
  }
}

int lnocc_workspace_bytes(const lnocc_fragment_t *f, int32_t nfrag, const lnocc_options_t *opt,
                          size_t *bytes) {
  if (bytes) *bytes = 0;
  if (!f || nfrag <= 0 || !bytes) return LNOCC_EINVAL;
  int st = check_options(opt);
  if (st) return st;
  size_t need = 0;
  for (int k = 0; k < nfrag; ++k) {
    st = check_sizes(&f[k]);
    if (st) return st;
    Layout L;
    plan_layout(dims_of(&f[k]), *opt, nullptr, L);
    need = std::max(need, L.bytes);
  }
  *bytes = need;
  return LNOCC_OK;
}

int lnocc_fragment_ccsd(lnocc_fragment_t *f, const lnocc_options_t *opt) {
  Layout L;
  int st = prepare(f, opt, opt && opt->guess == LNOCC_GUESS_USER, true, L);
  if (st) return finish(f, st);
  hipStream_t s = (hipStream_t)opt->stream;
  Guard guard(f, opt, L);
  Inputs in{f->B, f->eps_occ, f->eps_vir, f->t1 ? f->t1 : L.t1w, f->t2 ? f->t2 : L.t2w,
            f->conv_tol};
  st = setup_fragment(L, f->B, f->eps_occ, f->eps_vir, true, s);
  Outputs out;
  if (!st) st = run_ccsd(L, in, *opt, out, s);
  if (st >= 0 && opt->do_triples) {
    const int st2 = run_triples(L, in, out, s);
    if (st2 < 0) st = st2;
  }
  if (st < 0) dsync(s);
  f->e_mp2 = out.e_mp2;
  f->e_ccsd = out.e_ccsd;
  f->e_t = opt->do_triples ? out.e_t : 0.0;
  f->residual = out.residual;
  f->n_iter = out.n_iter;
  return finish(f, st);
}

int lnocc_fragment_triples(lnocc_fragment_t *f, const lnocc_options_t *opt) {
  Layout L;
  int st = prepare(f, opt, true, false, L);
  if (st) return finish(f, st);
  hipStream_t s = (hipStream_t)opt->stream;
  Guard guard(f, opt, L);
  Inputs in{f->B, f->eps_occ, f->eps_vir, f->t1, f->t2, f->conv_tol};
  st = setup_fragment(L, f->B, f->eps_occ, f->eps_vir, false, s);
  Outputs out;
  if (!st) st = run_triples(L, in, out, s);
  if (st < 0) dsync(s);
  f->e_t = out.e_t;
  return finish(f, st);
}

int lnocc_ccsd_residuals(lnocc_fragment_t *f, const lnocc_options_t *opt, double *r1, double *r2) {
  Layout L;
  int st = prepare(f, opt, true, false, L);
  if (!st && (!r1 || !r2)) st = LNOCC_EINVAL;
  if (st) return finish(f, st);
  hipStream_t s = (hipStream_t)opt->stream;
  Guard guard(f, opt, L);
  const int64_t o = f->nocc, v = f->nvir;
  st = setup_fragment(L, f->B, f->eps_occ, f->eps_vir, true, s);
  if (!st) st = ccsd_residuals(L, f->t1, f->t2, s);
  if (!st) {
    if (dcopy(r1, L.R1, o * v * 8, s) != hipSuccess ||
        dcopy(r2, L.R2, o * o * v * v * 8, s) != hipSuccess)
      st = LNOCC_EDEVICE;
  }
  if (dsync(s) != hipSuccess && !st) st = LNOCC_EDEVICE;
  return finish(f, st);
}

int lnocc_batch_solve(lnocc_fragment_t *f, int32_t nfrag, const lnocc_options_t *opt) {
  if (!f || nfrag <= 0) return LNOCC_EINVAL;
  int worst = LNOCC_OK;
  for (int k = 0; k < nfrag; ++k) {
    const int st = lnocc_fragment_ccsd(&f[k], opt);
    if (st < 0) worst = (worst < 0) ? std::min(worst, st) : st;
    else if (worst >= 0) worst = std::max(worst, st);
  }
  return worst;
}

void lnocc_set_validation_mode(int on) { set_dry_run(on != 0); }

void lnocc_profile_enable(int on) { profile_enable(on != 0); }

void lnocc_profile_collect(lnocc_kernel_stats_t out[LNOCC_KERNEL_CLASSES]) {
  KindStats k[(int)Kind::Count];
  profile_collect(k);
  for (int i = 0; i < LNOCC_KERNEL_CLASSES; ++i) out[i] = lnocc_kernel_stats_t{k[i].launches, k[i].ms, k[i].flops};
}

int lnocc_contract(const lnocc_contract_t *c, void *stream) {
  if (!c || !c->c || c->nseg < 1 || c->nseg > 4 || c->M < 0 || c->N < 0 || c->Mi < 1 ||
      c->Ni < 1 || c->batch < 1 || c->nb1 < 1 || c->batch > 65535)
    return LNOCC_EINVAL;
  GemmDesc d{};
  d.M = c->M; d.Mi = c->Mi; d.N = c->N; d.Ni = c->Ni;
  d.nseg = c->nseg;
  for (int s = 0; s < c->nseg; ++s) {
    if (!c->a[s].p || !c->b[s].p || c->K[s] < 0 || c->Ki[s] < 1) return LNOCC_EINVAL;
    GSegment &g = d.seg[s];
    g.a = GOperand{c->a[s].p, c->a[s].s_ro, c->a[s].s_ri, c->a[s].s_ko, c->a[s].s_ki,
                   c->a[s].b0, c->a[s].b1, 0, c->a[s].bid};
    g.b = GOperand{c->b[s].p, c->b[s].s_ro, c->b[s].s_ri, c->b[s].s_ko, c->b[s].s_ki,
                   c->b[s].b0, c->b[s].b1, 0, c->b[s].bid};
    g.K = c->K[s]; g.Ki = c->Ki[s]; g.scale = c->scale[s];
  }
  d.c = c->c;
  d.c_mo = c->c_mo; d.c_mi = c->c_mi; d.c_no = c->c_no; d.c_ni = c->c_ni;
  d.c_b0 = c->c_b0; d.c_b1 = c->c_b1; d.c_b2 = 0; d.c_bid = c->c_bid;
  d.beta = c->beta;
  d.batch = c->batch; d.nb1 = c->nb1; d.table = nullptr;
  if (c->precision < 0 || c->precision > 2) return LNOCC_EINVAL;
  d.prec = (Prec)c->precision;
  d.c_type = 0;
  hipStream_t s = (hipStream_t)stream;
  if (gett(d, s) != hipSuccess) return LNOCC_EDEVICE;
  if (dsync(s) != hipSuccess) return LNOCC_EDEVICE;
  return LNOCC_OK;
}

}  // extern "C"

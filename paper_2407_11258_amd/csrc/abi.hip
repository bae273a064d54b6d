// extern "C" entry points of liblnocc: argument validation on the host, then
// the solver of solver.hip on the caller's stream and workspace.
#include <cmath>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <memory>
#include <mutex>
#include <numeric>
#include <thread>
#include <vector>

#include "../../include/lnocc.h"
#include "gett.h"
#include "solver.h"
#include "mlp.h"
#include "pairs.h"

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
  if (opt->guess != LNOCC_GUESS_MP2 && opt->guess != LNOCC_GUESS_USER &&
      opt->guess != LNOCC_GUESS_MLP)
    return LNOCC_EINVAL;
  if (opt->guess == LNOCC_GUESS_MLP && (!opt->mlp || ((uintptr_t)opt->mlp) % 16))
    return LNOCC_EINVAL;
  if (opt->max_iter < 0 || opt->diis_space < 1 || opt->diis_space > 16 || opt->diis_start < 1 ||
      opt->triples_batch < 0 || opt->batch_slots < 0 || opt->batch_streams < 0 ||
      opt->batch_streams > 64 || opt->ladder_mode < LNOCC_LADDER_AUTO ||
      opt->ladder_mode > LNOCC_LADDER_ON_THE_FLY || !(opt->level_shift >= 0.0) ||
      !std::isfinite(opt->level_shift))
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
  Region r[7];
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
    r[k++] = Region{opt->mlp, opt->mlp ? (size_t)mlp::kBlob * 4 : 0};
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

// ------------------------------------------------------------------ static scratch
// Device scratch of lnocc_fragment_ccsd_static: one array per GPU, held until
// the process ends.  In host code its name is not a device address; the
// address of each device's copy comes from hipGetSymbolAddress, taken once per
// device with that device current.
namespace {
constexpr size_t kStaticScratchBytes = (size_t)LNOCC_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
}  // namespace
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
std::mutex g_static_mu;                       // guards the address table
void *g_static_ptr[kMaxDevices] = {};
std::mutex g_static_use[kMaxDevices];         // one call at a time per device
double g_static_host[kMaxDevices][kReadbackDoubles];   // readbacks of that call

// Holds this device's array (and its host readback buffer) for one call.
struct StaticScratch {
  void *ptr = nullptr;
  double *host = nullptr;
  std::unique_lock<std::mutex> hold;
  int acquire() {
    if (dry_run()) {   // validation mode: a stand-in address, never dereferenced
      ptr = (void *)((uintptr_t)1 << 47);
      static double dry_host[kReadbackDoubles];
      host = dry_host;
      return LNOCC_OK;
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
      note_error("hipGetDevice failed (%s)", hipGetErrorString(e));
      return LNOCC_EDEVICE;
    }
    {
      std::lock_guard<std::mutex> lock(g_static_mu);
      if (!g_static_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
          note_error("hipGetSymbolAddress of the static scratch failed (%s)",
                     hipGetErrorString(e));
          return LNOCC_EDEVICE;
        }
        g_static_ptr[dev] = p;
      }
      ptr = g_static_ptr[dev];
    }
    hold = std::unique_lock<std::mutex>(g_static_use[dev]);
    host = g_static_host[dev];
    return LNOCC_OK;
  }
};

// ------------------------------------------------------------------ batch
constexpr int kDefaultBatchSlots = 4;

int batch_slots(int nfrag, const lnocc_options_t *opt) {
  const int want = opt->batch_slots > 0 ? opt->batch_slots : kDefaultBatchSlots;
  return std::max(1, std::min(nfrag, want));
}

size_t round_up(size_t n, size_t a) { return (n + a - 1) / a * a; }

// Work of one fragment used to order the batch (largest first): the ladder of
// about twenty iterations plus (T).
double fragment_cost(const lnocc_fragment_t *f) {
  const double o = f->nocc, v = f->nvir, X = f->naux;
  return 20.0 * (X * v * v * v * v + o * o * v * v * v * v) + 2.0 * o * o * o * v * v * v * v;
}

// The plan file of opt->tune_cache: read when the call starts, rewritten when
// the call ends if autotuning added plans.
struct TuneCache {
  const char *path = nullptr;
  size_t n0 = 0;
  bool save = false;
  explicit TuneCache(const lnocc_options_t *opt) {
    if (!opt || !opt->tune_cache) return;
    path = opt->tune_cache;
    (void)tune_load(path);
    n0 = tune_plans();
    save = opt->autotune != 0;
  }
  ~TuneCache() {
    if (path && save && tune_plans() > n0) (void)tune_save(path);
  }
};

int worse(int a, int b) {
  if (a < 0 || b < 0) return std::min(a, b);
  return std::max(a, b);
}

// One fragment in flight: its slice of the workspace, its readback buffer
// and the state machine of its solve.
struct Slot {
  enum class Stage { Empty, Begin, Iterate, Final, Triples };
  Stage stage = Stage::Empty;
  int frag = -1;
  hipStream_t s = nullptr;
  char *base = nullptr;
  Layout L;
  Readback rb;
  std::unique_ptr<CcsdRun> run;
};

// Advances the solve in slot q after its last readback landed.  Returns a
// status < 0 on failure, 1 when the fragment is finished, 0 when more device
// work was enqueued.
int advance(Slot &q, const lnocc_options_t *opt) {
  CcsdRun &r = *q.run;
  int st = LNOCC_OK;
  switch (q.stage) {
    case Slot::Stage::Begin:
      st = r.after_begin();
      if (st) return st;
      if (r.phase == CcsdRun::Phase::Converged) {
        st = r.enqueue_final();
        q.stage = Slot::Stage::Final;
      } else {
        st = r.enqueue_iteration();
        q.stage = Slot::Stage::Iterate;
      }
      return st;
    case Slot::Stage::Iterate:
      st = r.after_iteration();
      if (st) return st;
      if (r.phase == CcsdRun::Phase::Converged || r.phase == CcsdRun::Phase::Exhausted) {
        q.stage = Slot::Stage::Final;
        return r.enqueue_final();
      }
      return r.enqueue_iteration();
    case Slot::Stage::Final:
      st = r.after_final();
      if (st < 0 || !opt->do_triples) return st < 0 ? st : 1;
      q.stage = Slot::Stage::Triples;
      return r.enqueue_t();
    case Slot::Stage::Triples:
      st = r.after_t();
      return st < 0 ? st : 1;
    default:
      return LNOCC_EINVAL;
  }
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
  opt->diis_space = 16;
  opt->diis_start = 1;
  opt->graphs = 1;
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
  *bytes = (nfrag == 1) ? need : round_up(need, 256) * batch_slots(nfrag, opt);
  return LNOCC_OK;
}

int lnocc_fragment_ccsd(lnocc_fragment_t *f, const lnocc_options_t *opt) {
  clear_error();
  Layout L;
  int st = prepare(f, opt, opt && opt->guess == LNOCC_GUESS_USER, true, L);
  if (st) return finish(f, st);
  hipStream_t s = (hipStream_t)opt->stream;
  Guard guard(f, opt, L);
  TuneCache cache(opt);
  Inputs in{f->B, f->eps_occ, f->eps_vir, f->t1 ? f->t1 : L.t1w, f->t2 ? f->t2 : L.t2w,
            f->conv_tol, f};
  Outputs out;
  st = run_ccsd(L, in, *opt, out, s);
  if (st >= 0 && opt->do_triples) {
    const int st2 = run_triples(L, in, out, s, opt->autotune != 0);
    if (st2 < 0) st = st2;
  }
  if (st < 0) dsync(s);
  f->e_mp2 = out.e_mp2;
  f->e_ccsd = out.e_ccsd;
  f->e_t = opt->do_triples ? out.e_t : 0.0;
  f->residual = out.residual;
  f->n_iter = out.n_iter;
  f->guess_used = out.guess_used;
  return finish(f, st);
}

int lnocc_fragment_ccsd_static(lnocc_fragment_t *f, const lnocc_options_t *opt_in) {
  clear_error();
  if (!opt_in) return finish(f, LNOCC_EINVAL);
  StaticScratch sc;
  int st = sc.acquire();
  if (st) return finish(f, st);
  // the library's own device array replaces the caller's workspace; no graph
  // capture and no tuning (both create runtime objects)
  lnocc_options_t opt = *opt_in;
  opt.workspace = sc.ptr;
  opt.workspace_bytes = kStaticScratchBytes;
  opt.graphs = 0;
  opt.autotune = 0;
  Layout L;
  st = check_sizes(f);
  if (!st) st = check_options(&opt);
  if (!st) {
    plan_layout(dims_of(f), opt, nullptr, L);
    if (L.bytes > kStaticScratchBytes) {
      note_error("fragment (%d, %d, %d) needs %zu bytes of scratch; the static array holds %zu",
                 f->nocc, f->nvir, f->naux, L.bytes, kStaticScratchBytes);
      st = LNOCC_ENOMEM;
    }
  }
  if (st) return finish(f, st);
  st = prepare(f, &opt, opt.guess == LNOCC_GUESS_USER, true, L);
  if (st) return finish(f, st);
  hipStream_t s = (hipStream_t)opt.stream;
  Guard guard(f, &opt, L);
  Inputs in{f->B, f->eps_occ, f->eps_vir, f->t1 ? f->t1 : L.t1w, f->t2 ? f->t2 : L.t2w,
            f->conv_tol, f};
  Outputs out;
  Readback rb(sc.host);
  st = run_ccsd(L, in, opt, out, s, &rb);
  if (st >= 0 && opt.do_triples) {
    const int st2 = run_triples(L, in, out, s, false, sc.host + kReadbackDoubles - 1);
    if (st2 < 0) st = st2;
  }
  if (st < 0) dsync(s);
  f->e_mp2 = out.e_mp2;
  f->e_ccsd = out.e_ccsd;
  f->e_t = opt.do_triples ? out.e_t : 0.0;
  f->residual = out.residual;
  f->n_iter = out.n_iter;
  f->guess_used = out.guess_used;
  return finish(f, st);
}

int lnocc_pair_workspace_bytes(const lnocc_fragment_t *f, const lnocc_options_t *opt,
                               size_t *bytes) {
  if (bytes) *bytes = 0;
  if (!f || !bytes) return LNOCC_EINVAL;
  int st = check_options(opt);
  if (!st) st = check_sizes(f);
  if (st) return st;
  lnocc_options_t o64 = *opt;
  o64.precision = LNOCC_FP64;
  Layout L;
  plan_layout(dims_of(f), o64, nullptr, L);
  plan_pair_layout(dims_of(f), nullptr, L, *bytes);
  return LNOCC_OK;
}

int lnocc_fragment_pair_energies(lnocc_fragment_t *f, const lnocc_options_t *opt,
                                 double *pair_ccsd, double *pair_t, const double *U, int32_t nlo,
                                 double *proj_ccsd, double *proj_t) {
  clear_error();
  if (!f || !opt) return LNOCC_EINVAL;
  int st = check_sizes(f);
  if (!st) st = check_options(opt);
  if (!st) st = check_pointers(f, true);
  if (!st && !pair_ccsd) st = LNOCC_EINVAL;
  if (!st && U && (nlo < 1 || !proj_ccsd || (pair_t && !proj_t))) st = LNOCC_EINVAL;
  if (st) return finish(f, st);
  lnocc_options_t o64 = *opt;
  o64.precision = LNOCC_FP64;
  Layout L;
  size_t need = 0;
  plan_layout(dims_of(f), o64, nullptr, L);
  plan_pair_layout(dims_of(f), nullptr, L, need);
  if (!opt->workspace) return finish(f, LNOCC_ENOMEM);
  if (((uintptr_t)opt->workspace) % 256) return finish(f, LNOCC_EINVAL);
  if (opt->workspace_bytes < need) return finish(f, LNOCC_ENOMEM);
  plan_layout(dims_of(f), o64, (char *)opt->workspace, L);
  plan_pair_layout(dims_of(f), (char *)opt->workspace, L, need);
  hipStream_t s = (hipStream_t)opt->stream;
  st = check_spectrum(f, s);
  if (st) return finish(f, st);
  const size_t o = f->nocc, v = f->nvir, X = f->naux, n = o + v;
  std::vector<Region> regions{
      Region{opt->workspace, opt->workspace_bytes}, Region{f->B, X * n * n * 8},
      Region{f->eps_occ, o * 8}, Region{f->eps_vir, v * 8}, Region{f->t1, o * v * 8},
      Region{f->t2, o * o * v * v * 8}, Region{pair_ccsd, o * o * 8},
      Region{pair_t, pair_t ? o * o * 8 : 0}, Region{U, U ? o * (size_t)nlo * 8 : 0},
      Region{proj_ccsd, U ? (size_t)nlo * 8 : 0}, Region{proj_t, U && pair_t ? (size_t)nlo * 8 : 0}};
  install_regions(regions.data(), (int)regions.size());
  install_splitk_scratch(L.splitk, (size_t)L.splitk_elems);
  st = setup_fragment(L, f->B, f->eps_occ, f->eps_vir, false, s);
  if (!st)
    st = pair_energies(L, f->t1, f->t2, f->eps_occ, f->eps_vir, pair_ccsd, pair_t, U, nlo,
                       proj_ccsd, proj_t, s);
  // traces (the canonical energies, Eq. 7 and Eq. 16 at i = i') for the host outputs
  if (!st && !dry_run()) {
    std::vector<double> h(o * o);
    if (hipMemcpyAsync(h.data(), pair_ccsd, o * o * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      st = LNOCC_EDEVICE;
    double tr = 0.0;
    for (size_t i = 0; i < o; ++i) tr += h[i * o + i];
    f->e_ccsd = tr;
    if (!st && pair_t) {
      if (hipMemcpyAsync(h.data(), pair_t, o * o * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        st = LNOCC_EDEVICE;
      tr = 0.0;
      for (size_t i = 0; i < o; ++i) tr += h[i * o + i];
      f->e_t = tr;
    }
  }
  if (dsync(s) != hipSuccess && !st) st = LNOCC_EDEVICE;
  install_regions(nullptr, 0);
  install_splitk_scratch(nullptr, 0);
  return finish(f, st);
}

int lnocc_fragment_triples(lnocc_fragment_t *f, const lnocc_options_t *opt) {
  clear_error();
  Layout L;
  int st = prepare(f, opt, true, false, L);
  if (st) return finish(f, st);
  hipStream_t s = (hipStream_t)opt->stream;
  Guard guard(f, opt, L);
  TuneCache cache(opt);
  Inputs in{f->B, f->eps_occ, f->eps_vir, f->t1, f->t2, f->conv_tol, f};
  st = setup_fragment(L, f->B, f->eps_occ, f->eps_vir, false, s);
  Outputs out;
  if (!st) st = run_triples(L, in, out, s, opt->autotune != 0);
  if (st < 0) dsync(s);
  f->e_t = out.e_t;
  return finish(f, st);
}

int lnocc_ccsd_residuals(lnocc_fragment_t *f, const lnocc_options_t *opt, double *r1, double *r2) {
  clear_error();
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
  clear_error();
  if (!f || nfrag <= 0) return LNOCC_EINVAL;
  int st = check_options(opt);
  if (st) return st;
  hipStream_t caller = (hipStream_t)opt->stream;
  // host-side checks of every fragment; a rejected fragment keeps its status
  size_t slot_bytes = 0;
  std::vector<int> order;
  int worst = LNOCC_OK;
  for (int k = 0; k < nfrag; ++k) {
    lnocc_fragment_t *g = &f[k];
    st = check_sizes(g);
    if (!st) st = check_pointers(g, opt->guess == LNOCC_GUESS_USER);
    if (!st && !(g->conv_tol > 0.0 && std::isfinite(g->conv_tol))) st = LNOCC_EINVAL;
    if (!st) st = check_spectrum(g, caller);
    if (st) {
      worst = worse(worst, finish(g, st));
      continue;
    }
    Layout L;
    plan_layout(dims_of(g), *opt, nullptr, L);
    slot_bytes = std::max(slot_bytes, round_up(L.bytes, 256));
    order.push_back(k);
  }
  if (order.empty()) return worst;
  if (!opt->workspace) return LNOCC_ENOMEM;
  if (((uintptr_t)opt->workspace) % 256) return LNOCC_EINVAL;
  TuneCache cache(opt);
  const int nslots = (int)std::min<size_t>(batch_slots((int)order.size(), opt),
                                           opt->workspace_bytes / slot_bytes);
  if (nslots < 1) {
    for (int k : order) worst = worse(worst, finish(&f[k], LNOCC_ENOMEM));
    return worst;
  }
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return fragment_cost(&f[a]) > fragment_cost(&f[b]); });

  // address guard over the workspace and every fragment's arrays
  std::vector<Region> regions{Region{opt->workspace, opt->workspace_bytes},
                              Region{opt->mlp, opt->mlp ? (size_t)mlp::kBlob * 4 : 0}};
  for (int k : order) {
    const size_t o = f[k].nocc, v = f[k].nvir, X = f[k].naux, n = o + v;
    regions.push_back(Region{f[k].B, X * n * n * 8});
    regions.push_back(Region{f[k].eps_occ, o * 8});
    regions.push_back(Region{f[k].eps_vir, v * 8});
    regions.push_back(Region{f[k].t1, f[k].t1 ? o * v * 8 : 0});
    regions.push_back(Region{f[k].t2, f[k].t2 ? o * o * v * v * 8 : 0});
  }
  install_regions(regions.data(), (int)regions.size());

  // Streams: the caller's, or a set created here (default priority) that
  // starts after the caller's stream and is joined back into it at the end.
  const int nstreams = std::min(opt->batch_streams, nslots);
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> joins;
  bool dev_ok = true;
  auto rt = [&](hipError_t e, const char *what) {
    if (e != hipSuccess) {
      note_error("%s failed (%s)", what, hipGetErrorString(e));
      dev_ok = false;
    }
    return e == hipSuccess;
  };
  if (nstreams > 0 && !dry_run()) {
    for (int i = 0; i < nstreams && dev_ok; ++i) {
      hipEvent_t e = nullptr;
      if (rt(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate")) joins.push_back(e);
    }
    for (int i = 0; i < nstreams && dev_ok; ++i) {
      hipStream_t h = nullptr;
      if (rt(hipStreamCreateWithFlags(&h, hipStreamNonBlocking), "hipStreamCreate")) streams.push_back(h);
    }
    if (dev_ok && rt(hipEventRecord(joins[0], caller), "hipEventRecord"))
      for (hipStream_t h : streams)
        if (!rt(hipStreamWaitEvent(h, joins[0], 0), "hipStreamWaitEvent")) break;
  }
  std::vector<Slot> slots(nslots);
  for (int q = 0; q < nslots; ++q) {
    slots[q].base = (char *)opt->workspace + (size_t)q * slot_bytes;
    slots[q].s = streams.empty() ? caller : streams[q % streams.size()];
    dev_ok = dev_ok && slots[q].rb.ok();
  }
  size_t next = 0;
  int active = 0;
  auto retire = [&](Slot &q, int status) {
    lnocc_fragment_t *g = &f[q.frag];
    if (status < 0 && !dry_run()) (void)hipStreamSynchronize(q.s);
    const Outputs &out = q.run->out;
    g->e_mp2 = out.e_mp2;
    g->e_ccsd = out.e_ccsd;
    g->e_t = opt->do_triples ? out.e_t : 0.0;
    g->residual = out.residual;
    g->n_iter = out.n_iter;
    g->guess_used = out.guess_used;
    if (status == 1) status = out.status;
    worst = worse(worst, finish(g, status));
    q.run.reset();
    q.frag = -1;
    q.stage = Slot::Stage::Empty;
    --active;
  };
  while (dev_ok && (next < order.size() || active > 0)) {
    bool progressed = false;
    for (Slot &q : slots) {
      if (q.stage == Slot::Stage::Empty) {
        if (next >= order.size()) continue;
        const int k = order[next++];
        lnocc_fragment_t *g = &f[k];
        plan_layout(dims_of(g), *opt, q.base, q.L);
        Inputs in{g->B, g->eps_occ, g->eps_vir, g->t1 ? g->t1 : q.L.t1w,
                  g->t2 ? g->t2 : q.L.t2w, g->conv_tol, g};
        q.frag = k;
        q.run.reset(new CcsdRun(q.L, in, *opt, q.s, q.rb));
        ++active;
        progressed = true;
        st = q.run->begin();
        if (st) retire(q, st);
        else q.stage = Slot::Stage::Begin;
        continue;
      }
      st = q.run->poll();
      if (st == 0) continue;
      progressed = true;
      st = (st < 0) ? st : advance(q, opt);
      if (st != 0) retire(q, st);
    }
    if (!progressed) std::this_thread::yield();
  }
  // join the created streams back into the caller's, then release them
  for (size_t i = 0; i < streams.size(); ++i) {
    if (i < joins.size() && hipEventRecord(joins[i], streams[i]) == hipSuccess)
      (void)hipStreamWaitEvent(caller, joins[i], 0);
  }
  for (hipStream_t h : streams) {
    (void)hipStreamSynchronize(h);
    (void)hipStreamDestroy(h);
  }
  if (!joins.empty()) (void)hipStreamSynchronize(caller);
  for (hipEvent_t e : joins) (void)hipEventDestroy(e);
  install_regions(nullptr, 0);
  install_splitk_scratch(nullptr, 0);
  if (!dev_ok) {   // a stream, event or readback buffer could not be created: nothing ran
    for (int k : order) worst = worse(worst, finish(&f[k], LNOCC_EDEVICE));
  }
  return worst;
}

}  // extern "C"

// ------------------------------------------------------------------ learned guess
namespace {

// Largest row count whose scratch fits in `bytes`.
int64_t rows_that_fit(size_t bytes, bool training) {
  mlp::Scratch S;
  int64_t lo = 0, hi = (int64_t)1 << 26;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) / 2;
    mlp::plan_scratch(mid, training, nullptr, S);
    if (S.bytes <= bytes) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

bool aligned16(const void *p) { return ((uintptr_t)p) % 16 == 0; }

// Scratch on the caller's workspace with room for `need` rows (0: as many as fit).
int mlp_scratch(const lnocc_options_t *opt, bool training, int64_t need, mlp::Scratch &S) {
  if (!opt) return LNOCC_EINVAL;
  if (!opt->workspace) return LNOCC_ENOMEM;
  if (((uintptr_t)opt->workspace) % 256) return LNOCC_EINVAL;
  const int64_t rows = rows_that_fit(opt->workspace_bytes, training);
  if (rows < std::max<int64_t>(need, 1)) return LNOCC_ENOMEM;
  mlp::plan_scratch(need > 0 ? need : rows, training, (char *)opt->workspace, S);
  return LNOCC_OK;
}

struct MlpGuard {
  std::vector<Region> r;
  MlpGuard(const lnocc_options_t *opt, const mlp::Scratch &S, std::initializer_list<Region> extra)
      : r(extra) {
    r.push_back(Region{opt->workspace, opt->workspace_bytes});
    install_regions(r.data(), (int)r.size());
    install_splitk_scratch(S.splitk, (size_t)S.splitk_elems);
  }
  ~MlpGuard() {
    install_regions(nullptr, 0);
    install_splitk_scratch(nullptr, 0);
  }
};

int device_status(hipError_t e, const char *what) {
  if (e == hipSuccess) return LNOCC_OK;
  if (!last_error()[0]) note_error("%s failed (%s)", what, hipGetErrorString(e));
  return LNOCC_EDEVICE;
}

}  // namespace

extern "C" {

int lnocc_mlp_workspace_bytes(int64_t rows, int32_t training, size_t *bytes) {
  if (bytes) *bytes = 0;
  if (!bytes || rows < 1 || rows > ((int64_t)1 << 26)) return LNOCC_EINVAL;
  mlp::Scratch S;
  mlp::plan_scratch(rows, training != 0, nullptr, S);
  *bytes = S.bytes;
  return LNOCC_OK;
}

int lnocc_mlp_samples(lnocc_fragment_t *f, const lnocc_options_t *opt, const int64_t *idx,
                      int64_t n, float *X, float *Y) {
  clear_error();
  Layout L;
  int st = prepare(f, opt, false, false, L);
  if (!st && (!idx || !X || n < 0 || !aligned16(X) || (Y && !f->t2))) st = LNOCC_EINVAL;
  if (st) return finish(f, st);
  hipStream_t s = (hipStream_t)opt->stream;
  Guard guard(f, opt, L);
  st = setup_fragment(L, f->B, f->eps_occ, f->eps_vir, false, s);
  if (!st) st = device_status(mlp::pair_stats(L.Boo, L.Bov, L.Bvv, L.dm.X, L.dm.o, L.dm.v, L.nrm,
                                              L.jd, s), "pair statistics");
  if (!st) st = device_status(mlp::features(L.Kov, f->eps_occ, f->eps_vir, L.nrm, L.jd, L.dm.o,
                                            L.dm.v, idx, 0, n, Y ? f->t2 : nullptr, X, Y, s),
                              "feature kernel");
  if (dsync(s) != hipSuccess && !st) st = LNOCC_EDEVICE;
  return finish(f, st);
}

int lnocc_mlp_init(float *blob, const float *X, const float *Y, int64_t n, uint64_t seed,
                   const lnocc_options_t *opt) {
  clear_error();
  if (!blob || !X || !Y || n < 1 || !aligned16(blob) || !aligned16(X)) return LNOCC_EINVAL;
  mlp::Scratch S;
  int st = mlp_scratch(opt, false, 0, S);
  if (st) return st;
  MlpGuard g(opt, S, {Region{blob, (size_t)mlp::kBlob * 4}, Region{X, (size_t)n * 64},
                      Region{Y, (size_t)n * 4}});
  hipStream_t s = (hipStream_t)opt->stream;
  st = device_status(mlp::init(blob, X, Y, n, seed, S, s), "network initialisation");
  if (dsync(s) != hipSuccess && !st) st = LNOCC_EDEVICE;
  return st;
}

int lnocc_mlp_predict(const float *blob, const float *X, int64_t n, float *out,
                      const lnocc_options_t *opt) {
  clear_error();
  if (!blob || !X || !out || n < 0 || !aligned16(blob) || !aligned16(X)) return LNOCC_EINVAL;
  mlp::Scratch S;
  int st = mlp_scratch(opt, false, 0, S);
  if (st) return st;
  MlpGuard g(opt, S, {Region{blob, (size_t)mlp::kBlob * 4}, Region{X, (size_t)n * 64},
                      Region{out, (size_t)n * 4}});
  hipStream_t s = (hipStream_t)opt->stream;
  st = device_status(mlp::predict(blob, X, n, out, S, s), "network prediction");
  if (dsync(s) != hipSuccess && !st) st = LNOCC_EDEVICE;
  return st;
}

int lnocc_mlp_loss_grad(const float *blob, const float *X, const float *Y, int64_t n,
                        float *grad, double *loss, const lnocc_options_t *opt) {
  clear_error();
  if (!blob || !X || !Y || !grad || !loss || n < 1 || !aligned16(blob) || !aligned16(X))
    return LNOCC_EINVAL;
  mlp::Scratch S;
  int st = mlp_scratch(opt, true, n, S);
  if (st) return st;
  MlpGuard g(opt, S, {Region{blob, (size_t)mlp::kBlob * 4}, Region{X, (size_t)n * 64},
                      Region{Y, (size_t)n * 4}, Region{grad, (size_t)mlp::kParams * 4}});
  hipStream_t s = (hipStream_t)opt->stream;
  st = device_status(mlp::loss_grad(blob, X, Y, n, S, s), "loss and gradient");
  if (!st) st = device_status(dcopy(grad, S.grad, (size_t)mlp::kParams * 4, s), "gradient copy");
  *loss = 0.0;
  if (!st) st = device_status(d2h(loss, S.loss, 8, s), "loss readback");
  if (dsync(s) != hipSuccess && !st) st = LNOCC_EDEVICE;
  return st;
}

int lnocc_mlp_train(float *blob, float *adam, int64_t step0, int32_t nsteps, const float *X,
                    const float *Y, int64_t n, int32_t batch, float lr, uint64_t seed,
                    double *losses, const lnocc_options_t *opt) {
  clear_error();
  if (!blob || !adam || !X || !Y || n < 1 || batch < 1 || nsteps < 0 || step0 < 0 ||
      !(lr > 0.0f) || !std::isfinite(lr) || !aligned16(blob) || !aligned16(X))
    return LNOCC_EINVAL;
  mlp::Scratch S;
  int st = mlp_scratch(opt, true, batch, S);
  if (st) return st;
  MlpGuard g(opt, S, {Region{blob, (size_t)mlp::kBlob * 4}, Region{adam, (size_t)mlp::kParams * 8},
                      Region{X, (size_t)n * 64}, Region{Y, (size_t)n * 4}});
  hipStream_t s = (hipStream_t)opt->stream;
  for (int k0 = 0; k0 < nsteps && !st; k0 += mlp::kLossChunk) {
    const int m = std::min(mlp::kLossChunk, nsteps - k0);
    st = device_status(mlp::train(blob, adam, step0 + k0, m, X, Y, n, batch, lr, seed,
                                  losses ? S.losses : nullptr, S, s), "training steps");
    if (!st && losses) {
      st = device_status(d2h(losses + k0, S.losses, (size_t)m * 8, s), "loss readback");
      if (!st) st = device_status(dsync(s), "stream synchronization");
    }
  }
  if (dsync(s) != hipSuccess && !st) st = LNOCC_EDEVICE;
  return st;
}

}  // extern "C"

extern "C" {

const char *lnocc_last_error(void) { return last_error(); }

int lnocc_autotune_save(const char *path) { return path ? tune_save(path) : -1; }
int lnocc_autotune_load(const char *path) { return path ? tune_load(path) : -1; }
void lnocc_autotune_clear(void) { tune_clear(); }

void lnocc_set_validation_mode(int on) { set_dry_run(on != 0); }

void lnocc_profile_enable(int on) { profile_enable(on != 0); }

void lnocc_profile_collect(lnocc_kernel_stats_t out[LNOCC_KERNEL_CLASSES]) {
  KindStats k[(int)Kind::Count];
  profile_collect(k);
  for (int i = 0; i < LNOCC_KERNEL_CLASSES; ++i) out[i] = lnocc_kernel_stats_t{k[i].launches, k[i].ms, k[i].flops};
}

int lnocc_contract(const lnocc_contract_t *c, void *stream) {
  clear_error();
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
  if (c->precision < 0 || c->precision > 4) return LNOCC_EINVAL;
  d.prec = (Prec)c->precision;
  d.c_type = 0;
  if (c->tile < 0 || c->tile > 10) return LNOCC_EINVAL;
  d.tile_hint = c->tile;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = gett(d, s);
  if (e != hipSuccess) {
    if (!last_error()[0]) note_error("contraction launch failed (%s)", hipGetErrorString(e));
    return LNOCC_EDEVICE;
  }
  e = dsync(s);
  if (e != hipSuccess) {
    note_error("stream synchronization after the contraction failed (%s)", hipGetErrorString(e));
    return LNOCC_EDEVICE;
  }
  return LNOCC_OK;
}

}  // extern "C"

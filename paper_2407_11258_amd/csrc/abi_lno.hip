// extern "C" entry points of the steps upstream and downstream of the fragment
// solve: local active spaces (Sec. II.C-E), the local Hamiltonian's DF factors
// (Eq. 27b) and the MP2 composite correction (Eq. 17).
#include <algorithm>
#include <cmath>
#include <climits>
#include <cstdint>
#include <vector>

#include "../../include/lnocc.h"
#include "gett.h"
#include "lno.h"
#include "solver.h"

using namespace lnocc;

namespace {

int check_system(const lnocc_system_t *sys) {
  if (!sys || !sys->Lao || !sys->C || !sys->eps_occ || !sys->eps_vir) return LNOCC_EINVAL;
  if (sys->nocc <= 0 || sys->nvir <= 0 || sys->naux <= 0) return LNOCC_EINVAL;
  if (sys->nocc > kEigMax || sys->nvir > kEigMax) {
    note_error("nocc %d / nvir %d above the eigensolver's %d", sys->nocc, sys->nvir, kEigMax);
    return LNOCC_EINVAL;
  }
  const int64_t N = (int64_t)sys->nocc + sys->nvir;
  // every contraction extent must fit the 32-bit index space of the kernels
  if ((int64_t)sys->naux * N > INT32_MAX || N * N > INT32_MAX) return LNOCC_EINVAL;
  return LNOCC_OK;
}

LnoSystem system_of(const lnocc_system_t *sys) {
  return LnoSystem{sys->nocc, sys->nvir, sys->naux, sys->Lao, sys->C, sys->eps_occ, sys->eps_vir};
}

int check_ws(const void *ws, size_t bytes, size_t need) {
  if (!ws) return LNOCC_ENOMEM;
  if (((uintptr_t)ws) % 256) return LNOCC_EINVAL;
  if (bytes < need) return LNOCC_ENOMEM;
  return LNOCC_OK;
}

// Address guard of the contraction launcher for one call (removed on exit).
struct RegionGuard {
  std::vector<Region> r;
  explicit RegionGuard(std::vector<Region> regions) : r(std::move(regions)) {
    install_regions(r.data(), (int)r.size());
  }
  ~RegionGuard() { install_regions(nullptr, 0); }
};

std::vector<Region> system_regions(const lnocc_system_t *sys) {
  const size_t o = sys->nocc, v = sys->nvir, X = sys->naux, N = o + v;
  return {Region{sys->Lao, X * N * N * 8}, Region{sys->C, N * N * 8},
          Region{sys->eps_occ, o * 8}, Region{sys->eps_vir, v * 8}};
}

int end_call(int st, hipStream_t s) {
  if (st < 0) {
    if (!dry_run()) hipStreamSynchronize(s);
    return st;
  }
  if (!dry_run()) {
    const hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      note_error("stream synchronization failed (%s)", hipGetErrorString(e));
      return LNOCC_EDEVICE;
    }
  }
  return st;
}

}  // namespace

extern "C" {

int lnocc_local_space_workspace_bytes(const lnocc_system_t *sys, int32_t nlo, int32_t cbno,
                                      size_t *bytes) {
  if (bytes) *bytes = 0;
  if (!bytes || nlo < 1) return LNOCC_EINVAL;
  const int st = check_system(sys);
  if (st) return st;
  LnoScratch S;
  plan_lno_scratch(sys->nocc, sys->nvir, sys->naux, nlo, cbno != 0, nullptr, S);
  *bytes = S.bytes;
  return LNOCC_OK;
}

int lnocc_local_space(const lnocc_system_t *sys, lnocc_local_space_t *sp, void *workspace,
                      size_t workspace_bytes, void *stream) {
  clear_error();
  int st = check_system(sys);
  if (st) return st;
  if (!sp || !sp->U_occ || sp->nlo < 1 || !sp->C_occ || !sp->eps_occ || !sp->C_vir ||
      !sp->eps_vir || !(sp->eta_occ >= 0.0) || !(sp->eta_vir >= 0.0) ||
      !std::isfinite(sp->eta_occ) || !std::isfinite(sp->eta_vir))
    return LNOCC_EINVAL;
  const int64_t no = sys->nocc, nv = sys->nvir, nlo = sp->nlo;
  LnoScratch S;
  plan_lno_scratch(no, nv, sys->naux, nlo, sp->cbno != 0, nullptr, S);
  st = check_ws(workspace, workspace_bytes, S.bytes);
  if (st) return st;
  plan_lno_scratch(no, nv, sys->naux, nlo, sp->cbno != 0, (char *)workspace, S);
  std::vector<Region> regions = system_regions(sys);
  regions.insert(regions.end(),
                 {Region{workspace, workspace_bytes}, Region{sp->U_occ, (size_t)(no * nlo * 8)},
                  Region{sp->U_vir, sp->U_vir ? (size_t)(nv * nlo * 8) : 0},
                  Region{sp->C_occ, (size_t)(no * no * 8)}, Region{sp->eps_occ, (size_t)no * 8},
                  Region{sp->C_vir, (size_t)(nv * nv * 8)}, Region{sp->eps_vir, (size_t)nv * 8},
                  Region{sp->lambda_occ, sp->lambda_occ ? (size_t)no * 8 : 0},
                  Region{sp->lambda_vir, sp->lambda_vir ? (size_t)nv * 8 : 0},
                  Region{sp->U_act, sp->U_act ? (size_t)(no * nlo * 8) : 0}});
  RegionGuard guard(std::move(regions));
  hipStream_t s = (hipStream_t)stream;
  LnoSpace out;
  out.C_occ = sp->C_occ; out.eps_occ = sp->eps_occ;
  out.C_vir = sp->C_vir; out.eps_vir = sp->eps_vir;
  out.lambda_occ = sp->lambda_occ; out.lambda_vir = sp->lambda_vir; out.U_act = sp->U_act;
  st = local_space(system_of(sys), sp->U_occ, sp->U_vir, nlo, sp->eta_occ, sp->eta_vir,
                   sp->cbno != 0, S, out, s);
  st = end_call(st, s);
  if (st >= 0) {
    sp->n_occ = out.n_occ; sp->n_vir = out.n_vir;
    sp->n_int_occ = out.n_int_occ; sp->n_int_vir = out.n_int_vir;
  }
  return st;
}

int lnocc_local_hamiltonian_workspace_bytes(const lnocc_system_t *sys, int32_t n_occ,
                                            int32_t n_vir, size_t *bytes) {
  if (bytes) *bytes = 0;
  if (!bytes) return LNOCC_EINVAL;
  const int st = check_system(sys);
  if (st) return st;
  if (n_occ < 0 || n_vir < 0 || n_occ > sys->nocc || n_vir > sys->nvir || n_occ + n_vir == 0)
    return LNOCC_EINVAL;
  *bytes = local_hamiltonian_bytes(sys->nocc, sys->nvir, sys->naux, n_occ, n_vir);
  return LNOCC_OK;
}

int lnocc_local_hamiltonian(const lnocc_system_t *sys, const double *C_occ, int32_t n_occ,
                            const double *C_vir, int32_t n_vir, double *B, void *workspace,
                            size_t workspace_bytes, void *stream) {
  clear_error();
  size_t need = 0;
  int st = lnocc_local_hamiltonian_workspace_bytes(sys, n_occ, n_vir, &need);
  if (st) return st;
  if (!B || (n_occ > 0 && !C_occ) || (n_vir > 0 && !C_vir)) return LNOCC_EINVAL;
  st = check_ws(workspace, workspace_bytes, need);
  if (st) return st;
  const size_t no = sys->nocc, nv = sys->nvir, X = sys->naux, na = (size_t)n_occ + n_vir;
  std::vector<Region> regions = system_regions(sys);
  regions.insert(regions.end(),
                 {Region{workspace, workspace_bytes}, Region{C_occ, C_occ ? no * no * 8 : 0},
                  Region{C_vir, C_vir ? nv * nv * 8 : 0}, Region{B, X * na * na * 8}});
  RegionGuard guard(std::move(regions));
  hipStream_t s = (hipStream_t)stream;
  st = local_hamiltonian(system_of(sys), C_occ, n_occ, C_vir, n_vir, (char *)workspace,
                         workspace_bytes, B, s);
  return end_call(st, s);
}

int lnocc_mp2_workspace_bytes(const lnocc_fragment_t *f, size_t *bytes) {
  if (bytes) *bytes = 0;
  if (!f || !bytes || f->nocc <= 0 || f->nvir <= 0 || f->naux <= 0) return LNOCC_EINVAL;
  *bytes = mp2_bytes(f->nocc, f->nvir, f->t2 != nullptr);
  return LNOCC_OK;
}

int lnocc_fragment_mp2(lnocc_fragment_t *f, const lnocc_options_t *opt) {
  clear_error();
  if (!f || !opt) return LNOCC_EINVAL;
  auto fin = [&](int st) {
    f->status = st;
    return st;
  };
  if (f->nocc <= 0 || f->nvir <= 0 || f->naux <= 0 || !f->B || !f->eps_occ || !f->eps_vir)
    return fin(LNOCC_EINVAL);
  const int64_t o = f->nocc, v = f->nvir, X = f->naux, N = o + v;
  if (X * N > INT32_MAX || o * v > INT32_MAX || N * N > INT32_MAX) return fin(LNOCC_EINVAL);
  int st = check_ws(opt->workspace, opt->workspace_bytes, mp2_bytes(o, v, f->t2 != nullptr));
  if (st) return fin(st);
  hipStream_t s = (hipStream_t)opt->stream;
  if (!dry_run()) {   // occupied below virtual, as every denominator assumes
    std::vector<double> eo(o), ev(v);
    if (hipMemcpyAsync(eo.data(), f->eps_occ, o * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(ev.data(), f->eps_vir, v * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fin(LNOCC_EDEVICE);
    double omax = -INFINITY, vmin = INFINITY;
    for (double e : eo) omax = std::isfinite(e) ? std::max(omax, e) : INFINITY;
    for (double e : ev) vmin = std::isfinite(e) ? std::min(vmin, e) : -INFINITY;
    if (!(omax < vmin)) return fin(LNOCC_EINVAL);
  }
  RegionGuard guard({Region{opt->workspace, opt->workspace_bytes},
                     Region{f->B, (size_t)(X * N * N * 8)}, Region{f->eps_occ, (size_t)o * 8},
                     Region{f->eps_vir, (size_t)v * 8},
                     Region{f->t1, f->t1 ? (size_t)(o * v * 8) : 0},
                     Region{f->t2, f->t2 ? (size_t)(o * o * v * v * 8) : 0}});
  double e = 0.0;
  st = fragment_mp2(f->B, f->eps_occ, f->eps_vir, o, v, X, f->t1, f->t2, (char *)opt->workspace,
                    opt->workspace_bytes, &e, s);
  st = end_call(st, s);
  if (st >= 0) {
    f->e_mp2 = e;
    if (!std::isfinite(e)) st = LNOCC_ENUMERIC;
  }
  return fin(st);
}

double lnocc_mp2_composite(double e_mp2_full, const double *e_mp2_fragments, int32_t nfrag) {
  double sum = 0.0;
  for (int32_t k = 0; k < nfrag && e_mp2_fragments; ++k) sum += e_mp2_fragments[k];
  return e_mp2_full - sum;
}

}  // extern "C"

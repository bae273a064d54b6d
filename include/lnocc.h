/* lnocc.h -- C ABI of the MI355X fragment solver for periodic LNO-CCSD(T).
 *
 * The library solves the problem that each LNO fragment poses (Ye and
 * Berkelbach, "Periodic local coupled-cluster theory for insulators and
 * metals", Sec. II.B): given the local Hamiltonian of an active space, i.e.
 * the semi-canonical Fock diagonal (Eq. 11 restricted to the active orbitals;
 * occupied and virtual orbitals are rotated separately, so the Fock matrix is
 * diagonal with no occupied-virtual block) and real three-index
 * density-fitting factors B[Q,p,q] with (pq|rs) = sum_Q B[Q,p,q] B[Q,r,s]
 * (Eq. 27a with the momentum sum folded into Q), it returns the CCSD
 * amplitudes t_ia, t_iajb, the CCSD correlation energy (Eq. 7) and the
 * perturbative triples energy (Eq. 16 summed at i = i' with the intermediates
 * of SI Sec. S1).
 *
 * Conventions common to every entry point
 *  - Orbitals are ordered occupied first; n = nocc + nvir.
 *  - Arrays are row-major FP64 in device memory unless stated otherwise.
 *  - t1[i][a] = t_i^a; t2[i][j][a][b] = t_ij^ab (= t_iajb of the paper),
 *    which satisfies t2[i][j][a][b] = t2[j][i][b][a].
 *  - The caller owns every buffer.  The library allocates no device memory:
 *    all scratch comes from the workspace the caller passes in options
 *    (lnocc_fragment_ccsd_static alone uses a static device array of the
 *    library instead).
 *  - Work is enqueued on options.stream (a hipStream_t; NULL = default
 *    stream).  Every entry point returns after that stream has completed the
 *    work, so host-side outputs are valid on return.
 *  - Calls that share one workspace must not overlap.
 *  - Status codes < 0 are errors (outputs undefined); > 0 are warnings
 *    (outputs valid).  Argument errors are detected on the host before any
 *    device work is enqueued.
 */
#ifndef LNOCC_H
#define LNOCC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LNOCC_ABI_VERSION 1

typedef enum {
  LNOCC_OK = 0,
  LNOCC_NOT_CONVERGED = 1, /* max_iter reached; last iterate returned */
  LNOCC_EINVAL = -1,       /* bad argument (null pointer, size, gap, tolerance) */
  LNOCC_ENOMEM = -2,       /* workspace missing or smaller than required */
  LNOCC_EDEVICE = -3,      /* a HIP call failed */
  LNOCC_ENUMERIC = -4      /* a non-finite residual or energy appeared */
} lnocc_status_t;

/* Arithmetic of the dominant contractions (the particle-particle ladder of
 * the CCSD residual, the W contraction of (T) and, in the reduced modes, the
 * o^3 v^3 ring contractions of the residual).  Energies, denominators,
 * residual norms and DIIS stay FP64 in every mode. */
typedef enum {
  LNOCC_FP64 = 0,
  LNOCC_FP32 = 1, /* FP32 storage of the ladder and (T) operands; FP32-accurate products:
                     on the FP32 matrix cores, or split as in LNOCC_FP32_SPLIT where that
                     is faster (the ladder contraction; the autotuner may pick either per
                     shape); FP32 accumulation per tile.  The other sizeable products of
                     the residual (the ring contractions, the DF products over Q, the T1
                     dressing) keep FP64 operands and use the products of
                     LNOCC_FP64_SPLIT in the early iterations, FP64 products from the
                     first step norm within 100 conv_tol (or the second in a row
                     without a new minimum) on */
  LNOCC_BF16 = 2, /* experimental: BF16 matrix-core products of the ladder (round to nearest
                     even), FP32 accumulation; errors of order 1e-4 Eh and a residual
                     floor near 1e-5 (the triples W contraction runs in FP32 and the
                     ring contractions as in LNOCC_FP32) */
  LNOCC_FP32_SPLIT = 3, /* lnocc_contract only (not a solve precision): FP32 operands, each
                           split into three bf16 parts (round to nearest even); a product is
                           the sum of the six largest part products on the BF16 matrix
                           cores, FP32 accumulation: FP32-level accuracy at BF16 rates */
  LNOCC_FP64_SPLIT = 4  /* lnocc_contract only: FP64 operands rounded to FP32 (nearest even)
                           as they are staged, then multiplied as in LNOCC_FP32_SPLIT */
} lnocc_precision_t;

typedef enum {
  LNOCC_GUESS_MP2 = 0,  /* T1 = 0, T2 = MP1 amplitudes (Eq. 21 with i_F over all occupied) */
  LNOCC_GUESS_USER = 1, /* start from the caller's t1 / t2 buffers (restart) */
  LNOCC_GUESS_MLP = 2   /* T1 = 0, T2 = MP1 amplitudes plus the correction predicted by the
                           model options.mlp (see "learned starting guess" below); falls back
                           to the MP2 start when that start is worse */
} lnocc_guess_t;

/* How the particle-particle ladder gets its (ac|bd) integrals (Eq. 27a over Q). */
typedef enum {
  LNOCC_LADDER_AUTO = 0,      /* stored when that needs at most 32 GiB of workspace */
  LNOCC_LADDER_STORED = 1,    /* bare (ac|bd) (b <= a blocks) and (kc|bd) formed once per
                                 solve; the T1 dressing enters as o^3 v^3 correction terms */
  LNOCC_LADDER_ON_THE_FLY = 2 /* T1-dressed (ac|bd) formed from B~_vv in every iteration,
                                 ladder_chunk_bytes at a time (no v^4 storage) */
} lnocc_ladder_mode_t;

/* One fragment problem and its results. */
typedef struct lnocc_fragment_t {
  int32_t nocc, nvir, naux;  /* active occupied, active virtual, auxiliary functions */
  int32_t reserved0;
  const double *B;           /* device [naux][n][n]; B[Q][p][q] == B[Q][q][p] is assumed */
  const double *eps_occ;     /* device [nocc], semi-canonical occupied energies (Hartree) */
  const double *eps_vir;     /* device [nvir], semi-canonical virtual energies;
                                every eps_occ must lie below every eps_vir */
  double conv_tol;           /* > 0; converged when ||t_new - t_old||_2 <= conv_tol over
                                the whole t1 and t2 arrays (Jacobi step, before DIIS) */
  double *t1;                /* device [nocc][nvir]: out (in with LNOCC_GUESS_USER) */
  double *t2;                /* device [nocc][nocc][nvir][nvir]: out (in with LNOCC_GUESS_USER) */
  /* host-side outputs */
  double e_mp2;              /* MP2 correlation energy (Eq. 7 at the MP1 amplitudes, T1 = 0) */
  double e_ccsd;             /* CCSD correlation energy (Eq. 7, tau = t2 + t1 t1) */
  double e_t;                /* (T) energy; 0 when triples are off */
  double residual;           /* last ||t_new - t_old||_2 */
  int32_t n_iter;            /* CCSD residual evaluations, including the one at the MP2
                                start that LNOCC_GUESS_MLP spends on its fallback test */
  int32_t status;            /* lnocc_status_t of this fragment */
  int32_t guess_used;        /* lnocc_guess_t the iterations actually started from */
  int32_t reserved1;
} lnocc_fragment_t;

/* Progress callback of the CCSD iterations: called on the calling thread after
 * every iteration of every fragment with the fragment (an element of the array
 * the call was given), the iteration number (1, 2, ...), the CCSD energy of the
 * amplitudes that entered the iteration (E_MP2 at the first) and the step norm
 * ||t_new - t_old||_2 of the iteration.  It must not call the library. */
typedef void (*lnocc_iter_fn)(const struct lnocc_fragment_t *f, int32_t it, double e,
                              double residual, void *user);

typedef struct lnocc_options_t {
  int32_t precision;         /* lnocc_precision_t */
  int32_t guess;             /* lnocc_guess_t */
  int32_t do_triples;        /* nonzero: compute E_(T) after CCSD */
  int32_t max_iter;          /* >= 0; 0 = no CCSD update (energy of the starting amplitudes) */
  int32_t diis_space;        /* 1..16 stored vectors; 1 disables extrapolation */
  int32_t diis_start;        /* first iteration that extrapolates (>= 1) */
  void *stream;              /* hipStream_t */
  void *workspace;           /* device scratch, >= lnocc_workspace_bytes(...) bytes, 256-byte aligned */
  size_t workspace_bytes;
  size_t ladder_chunk_bytes; /* cap on the (ac|bd) block formed at a time; 0 = 8 GiB */
  int32_t triples_batch;     /* unique (i<=j<=k) triples per (T) pass; 0 = automatic */
  int32_t batch_slots;       /* lnocc_batch_solve: fragments in flight at once, each with its
                                own workspace slice; 0 = 4 */
  double level_shift;        /* >= 0 (Hartree): amplitude steps R / (D - level_shift); the
                                convergence test always uses the unshifted step R / D */
  int32_t batch_streams;     /* lnocc_batch_solve: 0 = every fragment on opt->stream; n > 0 =
                                spread the fragments in flight over n streams of default
                                priority created for the call, so that small fragments run
                                concurrently */
  int32_t ladder_mode;       /* lnocc_ladder_mode_t */
  const float *mlp;          /* device model blob (LNOCC_MLP_BLOB floats) for LNOCC_GUESS_MLP */
  int32_t graphs;            /* nonzero: the residual evaluation of each CCSD iteration is
                                captured once per solve as a HIP graph and replayed (not while
                                launch timing is enabled) */
  int32_t autotune;          /* nonzero: before the first iteration of a solve whose contraction
                                shapes have no tuned plan yet, time every tile / split
                                candidate on one residual evaluation (and on the first (T)
                                batch) and keep the fastest per shape for the process */
  const char *tune_cache;    /* NULL, or the path of a contraction-plan file (the format of
                                lnocc_autotune_save): lnocc_fragment_ccsd, lnocc_fragment_triples
                                and lnocc_batch_solve read it before their first contraction
                                when it exists, and rewrite it at the end of the call when
                                autotuning added plans; a file that cannot be read or written
                                is skipped (not an error).  Ignored by
                                lnocc_fragment_ccsd_static. */
  lnocc_iter_fn on_iter;     /* NULL, or the progress callback above */
  void *user;                /* passed to on_iter */
} lnocc_options_t;

/* Fills *opt with defaults: FP64, MP2 guess, triples on, max_iter 100,
 * DIIS space 16 from iteration 1, graphs on, default stream, no workspace.
 * (16 stored vectors take 2 x 16 amplitude-sized arrays of the workspace; with
 * extrapolation from the first iteration they save about a quarter of the
 * iterations against 8 vectors from the second at 16/160/528.) */
void lnocc_default_options(lnocc_options_t *opt);

/* Human-readable name of a status code; never NULL. */
const char *lnocc_status_string(int status);

/* What failed in the last call on this host thread that returned an error
 * (the runtime call or check and its message); "" when the last call
 * succeeded.  Never NULL; valid until the next call on this thread. */
const char *lnocc_last_error(void);

/* Workspace bytes for *opt.  nfrag == 1: what lnocc_fragment_ccsd needs for
 * f[0].  nfrag > 1: what lnocc_batch_solve needs to keep min(nfrag,
 * batch_slots) fragments of f in flight, i.e. that many slices each as large
 * as the largest fragment's need (also enough for lnocc_fragment_ccsd on any
 * of them).  Writes 0 and returns LNOCC_EINVAL for bad sizes; host-only,
 * touches no device memory or pointer inside f. */
int lnocc_workspace_bytes(const lnocc_fragment_t *f, int32_t nfrag,
                          const lnocc_options_t *opt, size_t *bytes);

/* Fragment CCSD (Sec. II.B: CCSD with the fragment Hamiltonian) followed by
 * (T) (Eq. 16 at i = i', SI Sec. S1) when opt->do_triples.  Starts from the
 * MP1 guess (Eq. 21) or the caller's amplitudes, iterates Jacobi steps with
 * Pulay DIIS until the residual norm falls to f->conv_tol, writes t1 / t2 and
 * the host outputs of *f, and returns f->status.  A residual that grows three
 * iterations in a row, or rises 1000-fold above the best one, restarts the
 * DIIS subspace. */
int lnocc_fragment_ccsd(lnocc_fragment_t *f, const lnocc_options_t *opt);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve as lnocc_fragment_ccsd (same kernels and results), with its scratch in
 * a static device array of the library (LNOCC_STATIC_SCRATCH_BYTES per GPU,
 * held until the process ends) instead of opt->workspace, which is ignored.
 * The call makes no device or pinned-host allocation: no graph capture, no
 * autotuning (opt->graphs and opt->autotune are ignored), readbacks go through
 * a static host buffer with stream synchronization.  A fragment whose scratch
 * need (lnocc_workspace_bytes) exceeds the array gets LNOCC_ENOMEM and a
 * message in lnocc_last_error(); nothing runs.  The array keeps the last
 * call's contents; the solver initializes everything it reads.  Calls on one
 * GPU share its array: calls from threads of this process are serialized by a
 * lock per device; calls that overlap in any other way race. */
#define LNOCC_STATIC_SCRATCH_BYTES (64u << 20)
int lnocc_fragment_ccsd_static(lnocc_fragment_t *f, const lnocc_options_t *opt);

/* (T) energy (Eq. 16 at i = i' summed over i; W, V and Delta of SI Sec. S1)
 * of the amplitudes already in f->t1 / f->t2.  Writes f->e_t and returns the
 * status. */
int lnocc_fragment_triples(lnocc_fragment_t *f, const lnocc_options_t *opt);

/* ---- fragment pair energies and their projection (Sec. II.B) ---------------
 * From the amplitudes in f->t1 / f->t2 (normally a converged lnocc_fragment_ccsd
 * solve), the occupied pair matrices of the fragment energy
 *   pair_ccsd[i][i'] = sum_{j a b} tau_ij^ab (2 (i'a|jb) - (i'b|ja)),
 *                      tau = t2 + t1 t1                                  (Eqs. 9, 13)
 *   pair_t[i][i']    = -1/3 sum_{j k a b c} (4 w_ijk^abc + w_ijk^bca + w_ijk^cab)
 *                                           (v_i'jk^abc - v_i'jk^cba)    (Eq. 16)
 * with w = W / sqrt(-Delta_ijk), v_i'jk = V_i'jk / sqrt(-Delta_i'jk) and W, V,
 * Delta of SI Sec. S1, and, when U != NULL, the projected energy of each of the
 * nlo localized orbitals alpha:
 *   proj[alpha] = sum_{i i'} U[i][alpha] E[i][i'] U[i'][alpha]           (Eqs. 12, 15)
 * so that the fragment energy is the sum of proj over the fragment's LOs.  All
 * arrays are device FP64: pair_ccsd, pair_t [nocc][nocc] (out; pair_t = NULL
 * skips the triples part), U [nocc][nlo] (in, row i = occupied orbital i),
 * proj_ccsd, proj_t [nlo] (out).  The traces (the canonical energies of Eq. 7
 * and of Eq. 16 summed at i = i') go to f->e_ccsd and f->e_t.  Every product
 * runs in FP64 whatever opt->precision says.  The pair (T) part forms the W
 * tensors of all o ordered triples (i, j, k) for each pair j <= k, about three
 * times the work of lnocc_fragment_triples.  The workspace must hold
 * lnocc_pair_workspace_bytes() bytes (about 3 nocc nvir^3 doubles more than
 * the solve's). */
int lnocc_pair_workspace_bytes(const lnocc_fragment_t *f, const lnocc_options_t *opt,
                               size_t *bytes);
int lnocc_fragment_pair_energies(lnocc_fragment_t *f, const lnocc_options_t *opt,
                                 double *pair_ccsd, double *pair_t, const double *U, int32_t nlo,
                                 double *proj_ccsd, double *proj_t);

/* CCSD residuals R1[i][a] = <Phi_i^a| e^{-T} H e^{T} |HF> and
 * R2[i][j][a][b] = <Phi_{i alpha j beta}^{a alpha b beta}| e^{-T} H e^{T} |HF>
 * of the fragment Hamiltonian (Eq. 10) at the amplitudes in f->t1 / f->t2,
 * written to the device arrays r1 [nocc][nvir] and r2 [nocc][nocc][nvir][nvir].
 * This is the quantity the solver drives to zero. */
int lnocc_ccsd_residuals(lnocc_fragment_t *f, const lnocc_options_t *opt,
                         double *r1, double *r2);

/* Solves nfrag independent fragments (the sum over fragments of Eq. 8/13 needs
 * each one; fragments do not interact), each exactly as lnocc_fragment_ccsd
 * would.  Fragments are taken largest first and up to batch_slots of them are
 * in flight at once, each on its own slice of the workspace: the host advances
 * whichever fragment's per-iteration readback has landed while the work
 * already queued for the others keeps the device busy, so no device time is
 * lost to host round trips.  With batch_streams = 0 all of it runs on
 * opt->stream; otherwise slot q runs on stream q mod batch_streams of a set
 * created for the call, whose work starts after what opt->stream holds at the
 * call and which opt->stream waits for before the call returns.  Fewer fragments are in
 * flight when the workspace holds fewer slices; none fits: LNOCC_ENOMEM.  A fragment that fails the host checks gets its status
 * and is skipped.  Per-fragment results and statuses are written to f[k];
 * returns the most severe status (errors before warnings).  Returns when all
 * fragments are done. */
int lnocc_batch_solve(lnocc_fragment_t *f, int32_t nfrag, const lnocc_options_t *opt);

/* ---- local active space of a fragment (Sec. II.C-E) ------------------------
 * The whole system the fragments come from, device FP64:
 *   Lao     [naux][n][n] DF factors in the AO basis, (mu nu|la si) =
 *           sum_P Lao[P][mu][nu] Lao[P][la][si], symmetric in (mu, nu);
 *   C       [n][n] canonical MO coefficients (row = AO, column = MO,
 *           occupied first, orthonormal in the metric Lao is given in);
 *   eps_occ [nocc], eps_vir [nvir] canonical orbital energies (Eq. 11 is
 *           diagonal in this basis).  n = nocc + nvir. */
typedef struct lnocc_system_t {
  int32_t nocc, nvir, naux, reserved0;
  const double *Lao, *C, *eps_occ, *eps_vir;
} lnocc_system_t;

/* One fragment's active space.  In: U_occ [nocc][nlo] (row i = canonical
 * occupied orbital i, column = one of the fragment's nlo LOs), U_vir
 * [nvir][nlo] or NULL (LOs with components in the virtual space), the
 * thresholds eta_occ, eta_vir >= 0 of Eq. 26 and cbno (0: the densities of
 * Eq. 20 with one internal occupied index; 1: the cluster-specific densities
 * of Eq. 28).  Steps: internal orbitals = left singular vectors of U with
 * non-zero singular values (Eqs. 18-19; eigenvalues of U U^T above 1e-10
 * max(1, largest)), made semi-canonical; MP1 amplitudes with the internal
 * orbital energies as f_{i_F i_F} (Eqs. 21-23); the densities, diagonalized
 * inside the external spaces (Eqs. 24-25); LNOs with |lambda| >= eta kept
 * (Eq. 26); internal orbitals plus kept LNOs made semi-canonical.
 * Out (device, caller-allocated): C_occ [nocc][nocc] and C_vir [nvir][nvir]
 * (column c < n_occ / n_vir = active orbital c on the canonical orbitals, in
 * ascending order of its orbital energy), eps_occ [nocc] / eps_vir [nvir]
 * (first n_occ / n_vir entries), lambda_occ [nocc] / lambda_vir [nvir] (may be
 * NULL; the first nocc - n_int_occ / nvir - n_int_vir entries hold every
 * external eigenvalue by descending |lambda|), U_act [nocc][nlo] (may be
 * NULL; rows c < n_occ: the LOs on the active occupied orbitals,
 * U_act[c][alpha] = sum_i C_occ[i][c] U_occ[i][alpha], the U that
 * lnocc_fragment_pair_energies projects with).  Out (host): n_occ, n_vir (the
 * active sizes) and n_int_occ, n_int_vir (the internal ranks).  Orbitals are
 * defined up to sign (and up to rotations inside degenerate eigenspaces).
 * The workspace must hold lnocc_local_space_workspace_bytes(sys, nlo, cbno)
 * bytes, 256-byte aligned.  Errors: EINVAL for NULL arrays, sizes <= 0,
 * nocc or nvir above 2048 (the eigensolver's limit), negative or non-finite
 * eta; ENOMEM for a short workspace. */
typedef struct lnocc_local_space_t {
  const double *U_occ, *U_vir;
  int32_t nlo, cbno;
  double eta_occ, eta_vir;
  double *C_occ, *eps_occ, *C_vir, *eps_vir, *lambda_occ, *lambda_vir, *U_act;
  int32_t n_occ, n_vir, n_int_occ, n_int_vir;
} lnocc_local_space_t;

int lnocc_local_space_workspace_bytes(const lnocc_system_t *sys, int32_t nlo, int32_t cbno,
                                      size_t *bytes);
int lnocc_local_space(const lnocc_system_t *sys, lnocc_local_space_t *sp, void *workspace,
                      size_t workspace_bytes, void *stream);

/* DF factors of the local Hamiltonian (Eq. 27b) over the active orbitals
 * C_occ (first n_occ columns of a [nocc][nocc] array) and C_vir (first n_vir
 * columns of a [nvir][nvir] array), as lnocc_local_space returns them:
 *   B[P][p][q] = sum_{mu nu} Lao[P][mu][nu] Ca[mu][p] Ca[nu][q],
 *   Ca = [C[:, :nocc] C_occ | C[:, nocc:] C_vir],
 * written to B [naux][na][na], na = n_occ + n_vir, occupied first: the B of
 * lnocc_fragment_t, with the eps_occ / eps_vir of the active space. */
int lnocc_local_hamiltonian_workspace_bytes(const lnocc_system_t *sys, int32_t n_occ,
                                            int32_t n_vir, size_t *bytes);
int lnocc_local_hamiltonian(const lnocc_system_t *sys, const double *C_occ, int32_t n_occ,
                            const double *C_vir, int32_t n_vir, double *B, void *workspace,
                            size_t workspace_bytes, void *stream);

/* MP2 of a fragment Hamiltonian (or of the whole system, as a fragment with
 * every orbital active): t1 = 0 (when f->t1 != NULL), t2[i][j][a][b] =
 * (ia|jb) / D_ij^ab (when f->t2 != NULL) and
 * f->e_mp2 = sum_ijab (ia|jb) (2 (ia|jb) - (ib|ja)) / D_ij^ab.  Uses
 * opt->workspace and opt->stream only; without t2 the integrals pass through
 * the workspace a block of occupied rows at a time (at least one row,
 * nocc nvir^2 doubles: lnocc_mp2_workspace_bytes).  Passing the amplitudes to
 * lnocc_fragment_pair_energies (pair_t = NULL) gives the fragment's projected
 * MP2 energy, the fragment term of Eq. 17. */
int lnocc_mp2_workspace_bytes(const lnocc_fragment_t *f, size_t *bytes);
int lnocc_fragment_mp2(lnocc_fragment_t *f, const lnocc_options_t *opt);

/* Eq. 17's composite correction: e_mp2_full - sum_k e_mp2_fragments[k] (host). */
double lnocc_mp2_composite(double e_mp2_full, const double *e_mp2_fragments, int32_t nfrag);

/* ---- building block -------------------------------------------------------
 * Batched two-index-mode tensor contraction used for every DF product
 * (Eq. 27a: sums over the auxiliary index) and amplitude contraction:
 *   C[m,n] = sum_s scale_s sum_k A_s(m,k) B_s(n,k) + beta C[m,n]
 * where m = mo*Mi + mi, n = no*Ni + ni, k = ko*Ki + ki and each operand gives
 * one stride per index.  Batch entry e decodes to (e / nb1, e % nb1, 0) and
 * moves each base pointer by b0*(e / nb1) + b1*(e % nb1) + bid*e.  All strides
 * are in elements.  precision selects the operand element type and product
 * arithmetic (LNOCC_FP64: double; LNOCC_FP32: float, FP32 accumulation;
 * LNOCC_BF16: bf16 bit patterns, FP32 accumulation; LNOCC_FP32_SPLIT: float,
 * split bf16 products, FP32 accumulation; LNOCC_FP64_SPLIT: double, rounded to
 * float, split bf16 products, FP32 accumulation); C is always FP64. */
typedef struct lnocc_operand_t {
  const double *p;
  int64_t s_ro, s_ri, s_ko, s_ki;
  int64_t b0, b1, bid;
} lnocc_operand_t;

typedef struct lnocc_contract_t {
  int32_t M, Mi, N, Ni;
  int32_t nseg;                  /* 1..4 */
  int32_t K[4], Ki[4];
  double scale[4];
  lnocc_operand_t a[4], b[4];
  double *c;
  int64_t c_mo, c_mi, c_no, c_ni, c_b0, c_b1, c_bid;
  double beta;
  int32_t batch, nb1;
  int32_t precision;             /* lnocc_precision_t of the operands */
  int32_t tile;                  /* 0: automatic (tuned plan or heuristic); 1..9 force a tile
                                    of 128x128, 128x80, 128x64, 32x32, 128x160, 256x128
                                    rows x columns, 7: 128x128 with the products of
                                    LNOCC_FP32_SPLIT, 8: 160x160, 9: 128x160 with split
                                    products (5..7 and 9 for LNOCC_FP32 operands only, 8 for
                                    LNOCC_FP64 only; ignored otherwise), 10: 128x128 with
                                    split products staged in 4x4 blocks (LNOCC_FP32 and the
                                    split precisions, when every 4-element group along k, or
                                    along the rows of an operand contiguous in its rows, is
                                    contiguous and aligned and M, N, K are multiples of 4;
                                    ignored otherwise) */
} lnocc_contract_t;

int lnocc_contract(const lnocc_contract_t *desc, void *stream);

/* ---- launch timing ----------------------------------------------------------
 * While enabled, each contraction launch is bracketed by HIP events recorded on
 * the stream it runs on.  lnocc_profile_collect waits for the recorded events,
 * returns per-class totals and clears them.  Classes:
 *   0 other contractions (intermediates, T1 dressing, Fock, one-off integrals)
 *   1 (ac|bd) formation for the particle-particle ladder (Eq. 27a over Q)
 *   2 ladder contraction  sum_cd t_ij^cd (ac|bd)
 *   3 (T) W contraction   (SI Sec. S1) for batches of unique triples
 *   4 products of the learned-guess network (forward and backward)
 *   5 o^3 v^3 ring products of the CCSD residual (exchange and Coulomb rings,
 *     the T1 terms of the stored ladder)
 *   6 every launch of the classes above whose products run as split bf16
 *     products (LNOCC_FP32_SPLIT / LNOCC_FP64_SPLIT arithmetic: six bf16
 *     matrix-core products per product), whatever it computes
 * flops counts 2 M N K per product term (the algorithmic count). */
typedef struct lnocc_kernel_stats_t {
  int64_t launches;
  double ms;
  double flops;
} lnocc_kernel_stats_t;

#define LNOCC_KERNEL_CLASSES 7
void lnocc_profile_enable(int on);
void lnocc_profile_collect(lnocc_kernel_stats_t out[LNOCC_KERNEL_CLASSES]);

/* ---- learned starting guess --------------------------------------------------
 * Beyond the paper, which starts CCSD from the MP1 amplitudes (Eq. 21): a
 * per-amplitude multilayer perceptron predicts t_CCSD - t_MP1 from sixteen
 * features of the amplitude that exist before the first iteration, and the
 * solver starts from t_MP1 plus that correction (T1 = 0).  The CCSD equations
 * still decide the result; the guess changes the number of iterations only.
 * Before the first iteration the solver also evaluates the residual at the MP2
 * start; if the learned start gives a larger (or non-finite) first step
 * ||t_new - t_old||, it continues from the MP2 start instead (guess_used).
 *
 * Features of t_ij^ab, with K = (ia|jb), K' = (ib|ja), D = e_i + e_j - e_a -
 * e_b and |B_pq| the norm over Q of B[Q][p][q]:
 *   K/D, K'/D, K, K', 1/D, D, e_i + e_j, |e_i - e_j|, e_a + e_b, |e_a - e_b|,
 *   |B_ia||B_jb|, |B_ib||B_ja|, [i == j], [a == b], (ii|aa) + (jj|bb),
 *   (ii|bb) + (jj|aa)
 * (each unchanged under (i,j,a,b) -> (j,i,b,a), so the guess keeps
 * t_ij^ab = t_ji^ba).  Network: x -> (x - mu) * inv_sigma -> three hidden
 * layers of 256 SiLU units -> one output y; correction = y_mu + y_sigma * y.
 * Model blob, FP32 in device memory: LNOCC_MLP_HEADER floats [mu(16),
 * inv_sigma(16), y_mu, y_sigma, zeros] then LNOCC_MLP_PARAMS trainable floats
 * W1[256][16], b1[256], W2[256][256], b2[256], W3[256][256], b3[256], w4[256],
 * b4, zeros.  Products run in FP32 on the matrix cores.
 *
 * The calls below take stream, workspace and workspace_bytes from *opt (its
 * other fields are ignored except where stated); arrays are device FP32 and
 * 16-byte aligned; rows of X are LNOCC_MLP_FEATURES floats. */
#define LNOCC_MLP_FEATURES 16
#define LNOCC_MLP_HIDDEN 256
#define LNOCC_MLP_HEADER 64
#define LNOCC_MLP_PARAMS 136256
#define LNOCC_MLP_BLOB (LNOCC_MLP_HEADER + LNOCC_MLP_PARAMS)

/* Workspace for the network on up to `rows` rows per pass; training != 0 also
 * holds the backward pass (train and loss_grad need rows >= their batch). */
int lnocc_mlp_workspace_bytes(int64_t rows, int32_t training, size_t *bytes);

/* Training samples of a solved fragment: features X[n][16] of the amplitudes
 * with flat indices idx[r] = ((i nocc + j) nvir + a) nvir + b (device int64)
 * and, when Y != NULL, targets Y[r] = t2 - t_MP1 from the amplitudes in f->t2.
 * Uses opt->workspace as lnocc_fragment_triples does (same size).  An index
 * outside the amplitude array gives a row of NaN. */
int lnocc_mlp_samples(lnocc_fragment_t *f, const lnocc_options_t *opt, const int64_t *idx,
                      int64_t n, float *X, float *Y);

/* Header of blob from the statistics of (X, Y) over n rows (column means, inverse
 * standard deviations; 0 for a constant feature), and weights drawn from a
 * counter-based generator keyed by seed (uniform, Glorot limits; output layer
 * scaled by 0.1; biases zero). */
int lnocc_mlp_init(float *blob, const float *X, const float *Y, int64_t n, uint64_t seed,
                   const lnocc_options_t *opt);

/* out[r] = y_mu + y_sigma * net(norm(X[r])), r < n. */
int lnocc_mlp_predict(const float *blob, const float *X, int64_t n, float *out,
                      const lnocc_options_t *opt);

/* Mean squared error L = mean_r (net(norm(X[r])) - (Y[r] - y_mu) / y_sigma)^2 over
 * all n rows (*loss, host) and dL/dparams into grad (device, LNOCC_MLP_PARAMS
 * floats, parameter layout of the blob). */
int lnocc_mlp_loss_grad(const float *blob, const float *X, const float *Y, int64_t n,
                        float *grad, double *loss, const lnocc_options_t *opt);

/* nsteps Adam steps (beta1 0.9, beta2 0.999, eps 1e-8; step numbers step0 + 1,
 * ...) on the trainable part of blob, each on `batch` rows of (X, Y) drawn by a
 * counter-based generator keyed by (seed, step): row k of step t is
 * splitmix64(seed XOR splitmix64(t * 2^32 + k)) mod n, where splitmix64(z) is
 * the output function of the splitmix64 generator (Steele, Lea and Flood 2014)
 * at counter value z; adam: device float
 * [2 LNOCC_MLP_PARAMS] moments, zero before the first step.  losses (host, may be
 * NULL) receives the minibatch loss before each step. */
int lnocc_mlp_train(float *blob, float *adam, int64_t step0, int32_t nsteps, const float *X,
                    const float *Y, int64_t n, int32_t batch, float lr, uint64_t seed,
                    double *losses, const lnocc_options_t *opt);

/* ---- autotuning ---------------------------------------------------------------
 * Tuned plans (tile shape and split count per contraction shape) are shared by
 * the whole process.  Save / load them as text; returns the number of plans or
 * -1 when the file cannot be written / read.  Clearing returns to the built-in
 * heuristics. */
int lnocc_autotune_save(const char *path);
int lnocc_autotune_load(const char *path);
void lnocc_autotune_clear(void);

/* ---- validation mode -------------------------------------------------------
 * on != 0: every later call runs its host logic and launch sequence without
 * touching a device.  Each contraction launch is checked to stay inside the
 * workspace and the caller's arrays (sizes from the fragment shape) and fails
 * with LNOCC_EDEVICE otherwise; device readbacks read as zeros, so a solve
 * stops after one iteration and then runs every (T) pass.  The spectrum check
 * is skipped.  Pointers are never dereferenced in this mode.  Process-wide;
 * not for use while other threads solve. */
void lnocc_set_validation_mode(int on);

#ifdef __cplusplus
}
#endif

#endif /* LNOCC_H */

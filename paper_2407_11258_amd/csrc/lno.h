// Local active spaces of LNO-CC (Sec. II.C-E), the DF factors of the local
// Hamiltonian (Eq. 27b) and the MP2 energy used by the composite correction
// (Eq. 17).  All FP64 (see lno.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "../../include/lnocc.h"

namespace lnocc {

// The whole system upstream of the fragments (device arrays):
// Lao [X][N][N] AO-basis DF factors, symmetric in the two AO indices;
// C [N][N] canonical MO coefficients (row = AO, column = MO, occupied first);
// eo [no], ev [nv] canonical orbital energies.  N = no + nv.
struct LnoSystem {
  int64_t no, nv, X;
  const double *Lao, *C, *eo, *ev;
};

// Device scratch of local_space(), carved from one buffer.
struct LnoScratch {
  double *Lov = nullptr;      // [X][no][nv] canonical ov DF factors
  double *Lx = nullptr;       // transformed DF factors (one block of P at a time)
  double *M = nullptr, *V = nullptr, *w = nullptr;   // eigenproblem [N][N], vectors, values
  double *tmp = nullptr, *tmp2 = nullptr, *D3 = nullptr;   // [N][N] each
  double *Dij = nullptr, *Dab = nullptr;             // densities [no][no], [nv][nv]
  double *Wo = nullptr, *Wv = nullptr;               // external bases [no][no], [nv][nv]
  double *t = nullptr, *t2 = nullptr;                // MP1 amplitudes and their swapped copy
  int *idx = nullptr;                                // [N] orders / permutations
  int64_t lx_elems = 0, t_elems = 0;
  size_t bytes = 0;
};
// base == nullptr only sizes the scratch (bytes).  nlo bounds the number of
// internal orbitals; cbno selects the amplitude sizes of Eq. 28.
void plan_lno_scratch(int64_t no, int64_t nv, int64_t X, int64_t nlo, int cbno, char *base,
                      LnoScratch &S);

// Active space of one fragment.  Device outputs: C_occ [no][no] and C_vir
// [nv][nv] (column c = active orbital c on the canonical ones, c < n_occ /
// n_vir; internal orbitals first in the input to the final rotation),
// eps_occ [no], eps_vir [nv] (first n_occ / n_vir valid), lambda_occ [no],
// lambda_vir [nv] (may be null; the first no - n_int_occ / nv - n_int_vir hold
// the external eigenvalues by descending |lambda|), U_act [no][nlo] (may be
// null; rows c < n_occ: U_occ on the active occupied orbitals).  Host outputs:
// the counts.
struct LnoSpace {
  double *C_occ = nullptr, *eps_occ = nullptr, *C_vir = nullptr, *eps_vir = nullptr;
  double *lambda_occ = nullptr, *lambda_vir = nullptr, *U_act = nullptr;
  int n_occ = 0, n_vir = 0, n_int_occ = 0, n_int_vir = 0;
};
int local_space(const LnoSystem &sys, const double *U_occ, const double *U_vir, int64_t nlo,
                double eta_occ, double eta_vir, int cbno, const LnoScratch &S, LnoSpace &out,
                hipStream_t s);

// Eq. 27b for the active orbitals C_occ [no][no] (first n_occ columns) and
// C_vir [nv][nv] (first n_vir columns): B [X][na][na], na = n_occ + n_vir,
// occupied first.  Scratch: local_hamiltonian_bytes().
size_t local_hamiltonian_bytes(int64_t no, int64_t nv, int64_t X, int64_t n_occ, int64_t n_vir);
int local_hamiltonian(const LnoSystem &sys, const double *C_occ, int64_t n_occ,
                      const double *C_vir, int64_t n_vir, char *ws, size_t ws_bytes, double *B,
                      hipStream_t s);

// MP2 amplitudes and energy of a fragment Hamiltonian B [X][o+v][o+v] with
// orbital energies eo, ev: t2[i][j][a][b] = (ia|jb) / D_ij^ab when t2 != null,
// t1 = 0 when t1 != null, e = sum (ia|jb) (2 (ia|jb) - (ib|ja)) / D_ij^ab.
// Without t2 the integrals go through a scratch block of i rows (at least one
// row: o v^2 doubles); mp2_bytes() is the minimum.
size_t mp2_bytes(int64_t o, int64_t v, bool with_t2);
int fragment_mp2(const double *B, const double *eo, const double *ev, int64_t o, int64_t v,
                 int64_t X, double *t1, double *t2, char *ws, size_t ws_bytes, double *e_mp2,
                 hipStream_t s);

// Symmetric eigenproblem A [n][n] (destroyed) -> w[n] ascending, V [n][n]
// eigenvectors in columns; scratch: n ints.  n <= kEigMax.
constexpr int kEigMax = 2048;
hipError_t sym_eig(double *A, double *V, double *w, int n, int *scratch, hipStream_t s);

}  // namespace lnocc

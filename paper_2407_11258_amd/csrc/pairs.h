// Fragment pair energies and their projection onto localized orbitals (see pairs.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>

#include "solver.h"

namespace lnocc {

// Scratch of the pair energies, placed after the common part of L (aliasing the
// CCSD and (T) scratch); bytes receives the workspace the call needs.
void plan_pair_layout(const Dims &dm, char *base, Layout &L, size_t &bytes);

// Ecc [o][o] (Eqs. 9, 13) from t1, t2; Et [o][o] (Eq. 16) when Et != nullptr;
// with U [o][nlo] the projected energies pcc[alpha], pt[alpha] (Eqs. 12, 15).
// Needs setup_fragment(..., false) on L first (DF split and (ia|jb)).
int pair_energies(const Layout &L, const double *t1, const double *t2, const double *eo,
                  const double *ev, double *Ecc, double *Et, const double *U, int nlo,
                  double *pcc, double *pt, hipStream_t s);

}  // namespace lnocc

// Bandwidth-bound kernels of the fragment solver (splits, amplitude updates,
// FP64 reductions, DIIS vector algebra, the (T) energy epilogue).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace lnocc {

// Fixed grid of every partial-sum kernel: the reduction order (and so every
// FP64 energy and norm) is independent of timing and bitwise reproducible.
constexpr int kRedBlocks = 512;
constexpr int kRedThreads = 256;
// Blocks of a (T) energy launch: every block resident at once (256 CUs, five
// blocks of the FP32-W kernel or four of the FP64 one per CU), a multiple of 8
// (the launch is cut into one range of work per XCD); one partial sum per block.
constexpr int kTriplesEnergyGrid = 1280;
constexpr int kTriplesEnergyGrid64 = 1024;
inline int64_t triples_partials_capacity(int64_t) { return kTriplesEnergyGrid; }

hipError_t split_B(const double *B, int64_t X, int64_t o, int64_t v,
                   double *Boo, double *Bov, double *Bvv, hipStream_t s);
hipError_t diag_sum(const double *Boo, int64_t X, int64_t o, double *J, hipStream_t s);
// Bt[Q][a][b] = Bvv[Q][a][b] - sum_k t1[k][a] Bov[Q][k][b] (FP64, k summed in order)
hipError_t dress_vv(const double *Bvv, const double *Bov, const double *t1, int64_t X, int64_t o,
                    int64_t v, double *Bt, hipStream_t s);
hipError_t add_diag(double *M, int64_t n, int64_t ld, const double *eps, hipStream_t s);
hipError_t transpose2d(const double *in, int64_t rows, int64_t cols, double *out, hipStream_t s);
hipError_t make_u(const double *t2, int64_t o, int64_t v, double *u, hipStream_t s);
hipError_t mp2_guess(const double *Kov, const double *eo, const double *ev, int64_t o,
                     int64_t v, double *t1, double *t2, hipStream_t s);
hipError_t build_lov(const double *Kov, int64_t o, int64_t v, double *Lov, hipStream_t s);
hipError_t sub_oovv_into_dint(const double *Goovv, int64_t o, int64_t v, double *Dint,
                              hipStream_t s);
hipError_t combine_r2(double *R2, const double *S, const double *Xc, int64_t o, int64_t v,
                      hipStream_t s);
// R2 <- its pair-symmetric part, (R2[i][j][a][b] + R2[j][i][b][a]) / 2
hipError_t pair_symmetrize(double *R2, int64_t o, int64_t v, hipStream_t s);
// partials[kRedBlocks] <- pieces of sum (2 (ia|jb) - (ib|ja)) (t2 + t1 t1)
hipError_t energy_partials(const double *Kov, const double *t1, const double *t2, int64_t o,
                           int64_t v, double *partials, hipStream_t s);
// out[0] (+)= sum of partials[0..n) in a fixed order
hipError_t reduce_partials(const double *partials, int64_t n, double *out, int accumulate,
                           hipStream_t s);
// x = t + R / (D - shift) (level-shifted Jacobi step) as one concatenated vector
// [t1 | t2]; e = x - t; partials[kRedBlocks] <- pieces of ||R / D||^2.
hipError_t jacobi_step(const double *t1, const double *t2, const double *R1, const double *R2,
                       const double *eo, const double *ev, int64_t o, int64_t v, double shift,
                       double *x, double *e, double *partials, hipStream_t s);
// partials[i * kRedBlocks + b] <- pieces of dot(e_new, e_i), i < m
hipError_t dot_partials(const double *E, int64_t stride, int m, const double *enew, int64_t N,
                        double *partials, hipStream_t s);
hipError_t reduce_rows(const double *partials, int m, double *out, hipStream_t s);
// t1 | t2 <- sum_i c[i] x_i
hipError_t lincomb(const double *Xs, int64_t stride, int m, const double *c_host, int64_t o,
                   int64_t v, double *t1, double *t2, hipStream_t s);
hipError_t scatter_vec(const double *x, int64_t o, int64_t v, double *t1, double *t2,
                       hipStream_t s);

// Particle-particle ladder through (ij)-symmetric / antisymmetric rows.
// type: 0 double, 1 float, 2 bf16 (round to nearest even)
hipError_t pack_t(const double *t2, int64_t o, int64_t v, void *Tsa, int type, hipStream_t s);
hipError_t convert(const double *in, int64_t n, void *out, int type, hipStream_t s);
// SA rows of ld entries; ca == 0: entry P = a v + b; ca > 0: the stored-ladder
// order of blocks of ca values of a (see the kernel).
hipError_t unpack_ladder(const double *SA, int64_t o, int64_t v, int64_t ca, int64_t ld,
                         double *R2, hipStream_t s);

// table[3 n + {0,1,2}] <- (i, j, k) of the n-th unique triple i <= j <= k, not
// all equal (o (o + 1) (o + 2) / 6 - o entries): first the o (o - 1) (o - 2) / 6
// with i < j < k, then the o (o - 1) / 2 with i = j < k, then the o (o - 1) / 2
// with i < j = k, each group in lexicographic order.
hipError_t triples_table(int *table, int64_t o, hipStream_t s);

// (T) energy of a batch of unique triples whose W tensors sit in W[nb][v][v][v].
// table holds (i, j, k) per entry, i <= j <= k; W holds nb triples in the blocked
// layout of triples_w (triples.h); one partial per block, kTriplesEnergyGrid of them.
// W element type: 0 double, 1 float
// sym = 0: W holds W itself; sym = 1 (2): W holds Z with W(a,b,c) = Z(a,b,c) +
// Z(b,a,c) (Z(a,b,c) + Z(a,c,b)).  capacity: length of partials; a launch that
// would write more is refused (hipErrorInvalidValue, also in validation mode).
hipError_t triples_energy(const void *W, int wtype, int sym, const int *table, int nb,
                          const double *Kov, const double *t1, const double *eo,
                          const double *ev, int64_t o, int64_t v, double *partials,
                          int64_t capacity, int64_t *nparts, hipStream_t s);

}  // namespace lnocc

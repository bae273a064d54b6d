// W contraction of (T) on the matrix cores (see triples.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace lnocc {

// Padded length of the contracted virtual index d of G and T (a multiple of 4,
// so that rows of both start on 16-byte boundaries).
int64_t triples_pad(int64_t v);

// out[i][j][a][d] = t2[i][j][a][d] for d < v, 0 for v <= d < vp (float when f32).
hipError_t triples_pad_t2(const double *t2, int64_t o, int64_t v, void *out, int f32,
                          hipStream_t s);

// Layouts of W[a][b][c] for one triple.  Plain: [v][v][v].  Blocked (what the
// (T) energy kernel reads): [v][B][C][8][8] with b = 8 B + y, c = 8 C + z and
// B, C < vt = ceil(v / 8), so that the 8 x 8 (b, c) face of a cube tile is 64
// contiguous elements; positions with b or c >= v are never written.
int64_t triples_w_elems(int64_t v, int blocked);   // elements of one triple's W

// One orientation (0, 1, 2) of W for nb triples of table:
//   G [o][v][v][vp]  (ai|bd) as G[i][a][b][d], zero for d >= v
//   T [o][o][v][vp]  t_ij^ab as T[i][j][a][b], zero for b >= v
//   J [o][o][v][o]   (ck|jl) as J[j][k][c][l]
//   W [nb][triples_w_elems(v, blocked)]  overwritten (accumulate = 0) or added to
// nterms = 2: the orientation's four terms; 1: its first particle and first
// hole term only (for a triple with two equal labels the other two are the
// same terms with two virtual labels exchanged).
// Element type double, or float when f32 (FP32 products, FP32 accumulation).
hipError_t triples_w(const void *G, const void *T, const void *J, void *W, const int *table,
                     int nb, int64_t o, int64_t v, int ori, int f32, int accumulate, int nterms,
                     int blocked, hipStream_t s);

}  // namespace lnocc

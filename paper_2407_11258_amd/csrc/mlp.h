// Learned T2 starting guess: per-amplitude features, an MLP (three hidden
// layers of 256 SiLU units, FP32 on the matrix cores through gett()) that
// predicts the correction t_CCSD - t_MP1, and its training (MSE loss,
// backward pass, Adam).  The model is one flat FP32 blob in device memory:
// kHeader floats [mu(16), inv_sigma(16), y_mu, y_sigma, zeros] followed by
// the kParams trainable floats W1[256][16], b1, W2[256][256], b2, W3, b3,
// w4[256], b4, zero padding.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace lnocc {
namespace mlp {

constexpr int kFeat = 16;
constexpr int kHidden = 256;
constexpr int kHeader = 64;
constexpr int64_t kW1 = 0;
constexpr int64_t kB1 = kW1 + (int64_t)kHidden * kFeat;
constexpr int64_t kW2 = kB1 + kHidden;
constexpr int64_t kB2 = kW2 + (int64_t)kHidden * kHidden;
constexpr int64_t kW3 = kB2 + kHidden;
constexpr int64_t kB3 = kW3 + (int64_t)kHidden * kHidden;
constexpr int64_t kW4 = kB3 + kHidden;
constexpr int64_t kB4 = kW4 + kHidden;
constexpr int64_t kParams = (kB4 + 1 + 63) / 64 * 64;
constexpr int64_t kBlob = kHeader + kParams;
constexpr int kLossChunk = 64;   // training steps whose losses the scratch holds

// Device scratch for running the network on up to `rows` rows at a time.
// Inference needs xn, h1, h2, y; training also keeps the pre-activations and
// the backward buffers.
struct Scratch {
  int64_t rows = 0;
  bool training = false;
  float *xn = nullptr, *z1 = nullptr, *h1 = nullptr, *z2 = nullptr, *h2 = nullptr;
  float *z3 = nullptr, *h3 = nullptr, *y = nullptr;
  float *dy = nullptr, *dza = nullptr, *dzb = nullptr, *xb = nullptr, *yb = nullptr;
  float *grad = nullptr;          // kParams
  double *partials = nullptr;     // reduction partials
  double *loss = nullptr;         // device scalar
  double *losses = nullptr;       // kLossChunk per-step losses (training)
  double *splitk = nullptr;       // split-K scratch of the weight-gradient products
  int64_t splitk_elems = 0;
  size_t bytes = 0;
};
// base == nullptr only sizes the scratch (S.bytes).
void plan_scratch(int64_t rows, bool training, char *base, Scratch &S);

// nrm[i][a] = |B_ia| (norm over Q), jd[i][a] = (ii|aa).
hipError_t pair_stats(const double *Boo, const double *Bov, const double *Bvv, int64_t X,
                      int64_t o, int64_t v, double *nrm, double *jd, hipStream_t s);

// Raw features of n amplitudes into Xf[n][16] and, when t2 != nullptr, the
// targets Yf[n] = t2 - t_MP1.  Rows are the flat amplitude indices idx[r]
// ((i o + j) v + a) v + b when idx != nullptr, else the unique amplitudes
// u0 .. u0 + n - 1 in the order (pair p = j (j + 1) / 2 + i with i <= j) * v^2 +
// a v + b.
hipError_t features(const double *Kov, const double *eo, const double *ev, const double *nrm,
                    const double *jd, int64_t o, int64_t v, const int64_t *idx, int64_t u0,
                    int64_t n, const double *t2, float *Xf, float *Yf, hipStream_t s);

// Network output (standardised) of n <= S.rows rows into S.y.
hipError_t forward(const float *blob, const float *X, int64_t n, const Scratch &S, hipStream_t s);

// t2[i][j][a][b] += y_mu + y_sigma * y[r] for the unique amplitudes u0 + r, and
// the same at (j, i, b, a).
hipError_t apply_guess(const float *blob, const float *y, int64_t o, int64_t v, int64_t u0,
                       int64_t n, double *t2, hipStream_t s);

// out[r] = y_mu + y_sigma * net(norm(X[r])) for any n (chunks of S.rows).
hipError_t predict(const float *blob, const float *X, int64_t n, float *out, const Scratch &S,
                   hipStream_t s);

// Loss (mean squared error on the standardised targets) and its gradient
// (into S.grad, parameter layout) over n <= S.rows rows; loss into S.loss[0].
hipError_t loss_grad(const float *blob, const float *X, const float *Y, int64_t n,
                     const Scratch &S, hipStream_t s);

// Header from the statistics of (X, Y) and weights from a counter-based
// generator keyed by seed.
hipError_t init(float *blob, const float *X, const float *Y, int64_t n, uint64_t seed,
                const Scratch &S, hipStream_t s);

// nsteps Adam steps (step numbers step0 + 1 ...) on minibatches of `batch`
// rows drawn from (X, Y) by a counter-based generator; losses[k] (device,
// may be nullptr) receives the minibatch loss before step k.
hipError_t train(float *blob, float *adam, int64_t step0, int nsteps, const float *X,
                 const float *Y, int64_t n, int batch, float lr, uint64_t seed, double *losses,
                 const Scratch &S, hipStream_t s);

}  // namespace mlp
}  // namespace lnocc

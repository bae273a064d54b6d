// Generic batched contraction on gfx950 matrix cores (FP64, FP32, BF16 and
// split-bf16 FP32 products), plus matrix-vector kernels for N = 1.
//
// Tiles: 128 x 128 outputs per workgroup of 8 wave64s (4 x 2, 32 x 64 per wave
// = 2 x 4 blocks of 16 x 16 matrix ops; the FP64 one is register-limited so that
// two workgroups share a CU), 128 x 80 and 128 x 64 (4 waves), 160 x 160 (FP64,
// 10 waves: an ov x ov output is one round of 256 tiles), 32 x 32 single-wave
// tiles for thin outputs, and FP32-only 128 x 160 / 256 x 128 and split-bf16
// tiles.  K is staged through double-buffered LDS in slices (16 for FP64/FP32,
// k-major [k][row] so that the 16 lanes of one operand row read 128 contiguous
// bytes; 32 for the bf16 modes, [row][k]); the next slice is fetched into
// registers while the current one is multiplied (one barrier per slice).  Thin
// outputs with long K are split over K across workgroups; the partial tiles are
// summed in a fixed order by a second kernel, so results do not depend on
// scheduling.
//
// MFMA 16x16x4 (f64) operand layout, lane l of a wave64:
//   A: A[l % 16][l / 16]      B: B[l / 16][l % 16]
//   D: D[l / 16 + 4 * r][l % 16], r = 0..3   (checked on gfx950)
#include "gett.h"

#include <algorithm>
#include <atomic>
#include <type_traits>
#include <map>
#include <mutex>
#include <string>
#include <vector>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>

namespace lnocc {
namespace {

constexpr int kCUs = 256;   // compute units of one MI355X

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8_t __attribute__((ext_vector_type(8)));

// Arithmetic modes.  T: operand element in memory and LDS; Acc: accumulator
// fragment of one 16 x 16 block; KS: k per MFMA; BK: k per LDS slice;
// row(lane, r): output row of accumulator register r.
struct ModeF64 {
  using T = double;
  using L = double;                               // LDS element
  static constexpr int kPlanes = 1;               // LDS tiles per operand slice
  using Acc = double4_t;
  static constexpr int KS = 4, BK = 16;
  static constexpr bool kRowMajor = false;        // LDS tile [k][row]
  __device__ static int row(int lane, int r) { return lane / 16 + 4 * r; }
  __device__ static T cvt(double x) { return x; }
};
struct ModeF32 {
  using T = float;
  using L = float;
  static constexpr int kPlanes = 1;
  using Acc = float4_t;
  static constexpr int KS = 4, BK = 16;
  static constexpr bool kRowMajor = false;
  __device__ static int row(int lane, int r) { return 4 * (lane / 16) + r; }
  __device__ static T cvt(double x) { return (float)x; }
};
struct ModeBF16 {
  using T = uint16_t;                              // bf16 bit pattern
  using L = uint16_t;
  static constexpr int kPlanes = 1;
  using Acc = float4_t;
  static constexpr int KS = 32, BK = 32;
  static constexpr bool kRowMajor = true;         // LDS tile [row][k]: 8 k per lane read at once
  __device__ static int row(int lane, int r) { return 4 * (lane / 16) + r; }
};
// FP32 operands multiplied on the bf16 matrix cores: each element x is split
// into x = h + m + l + e with h = bf16(x), m = bf16(x - h), l = bf16(x - h - m)
// (round to nearest even; both differences are exact in FP32, |e| <= 2^-27 |x|),
// and a product is the sum of the six split products h h', h m', m h', h l',
// l h', m m' (the dropped ones are below 2^-24 of it), accumulated in FP32
// (Henry, Tang and Heinecke, ARITH 2019).  The splits are made once per element
// when the slice is written to LDS, as three bf16 tiles.
struct ModeF32S {
  using T = float;
  using L = uint16_t;
  static constexpr int kPlanes = 3;
  using Acc = float4_t;
  static constexpr int KS = 32, BK = 32;
  static constexpr bool kRowMajor = true;
  __device__ static int row(int lane, int r) { return 4 * (lane / 16) + r; }
};
// FP64 operands in memory, rounded to FP32 as they are staged, then split as in
// ModeF32S: FP32-class products at bf16 matrix-core rates for FP64 tensors that
// need no FP32 copy.
struct ModeF64S {
  using T = double;
  using L = uint16_t;
  static constexpr int kPlanes = 3;
  using Acc = float4_t;
  static constexpr int KS = 32, BK = 32;
  static constexpr bool kRowMajor = true;
  __device__ static int row(int lane, int r) { return 4 * (lane / 16) + r; }
};

__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// round to nearest even (finite inputs)
__device__ inline uint16_t f32_to_bf16(float f) {
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// Tile configuration: BM x BN outputs per workgroup, WM x WN waves, each wave
// owning a (BM/WM) x (BN/WN) block of 16 x 16 MFMA tiles.
template <int BM_, int BN_, int WM_, int WN_>
struct Cfg {
  static constexpr int BM = BM_, BN = BN_, WM = WM_, WN = WN_;
  static constexpr int T = 64 * WM * WN;
  static constexpr int MI = BM / WM / 16, NI = BN / WN / 16;
};
using Big = Cfg<128, 128, 4, 2>;     // 8 waves, 32 x 64 (2 x 4 MFMA blocks) each
using Big80 = Cfg<128, 80, 4, 1>;    // 4 waves, 32 x 80 (2 x 5) each: N = 80 q
using Big64 = Cfg<128, 64, 4, 1>;    // 4 waves, 32 x 64 (2 x 4) each
using Small = Cfg<32, 32, 1, 1>;
// FP32 only (accumulators are half the size of FP64 ones): more MFMA work per
// LDS slice to cover the load latency of the faster FP32 matrix cores.
using Wide160 = Cfg<128, 160, 4, 1>; // 4 waves, 32 x 160 (2 x 10) each: N = 160
using Tall = Cfg<256, 128, 4, 2>;    // 8 waves, 64 x 64 (4 x 4) each
// FP64 only: 10 waves, 32 x 80 (2 x 5) each.  An ov x ov output (2560 x 2560 for
// 16 occupied and 160 virtual orbitals) is exactly 256 of these tiles, one per
// CU, where 128 x 128 tiles leave the second round of workgroups half empty.
using Sq160 = Cfg<160, 160, 5, 2>;
// split bf16 products only: 8 waves, 32 x 80 (2 x 5) each; N = 160 (the c index
// of W) in one tile
using Wide160S = Cfg<128, 160, 4, 2>;

// Tile ids of the launcher and the autotuner (rows x columns per workgroup).
// Id 6 is the 128 x 128 tile with FP32 products evaluated as split bf16
// products (an arithmetic choice for FP32 contractions, same accuracy class).
constexpr int kTileBM[10] = {128, 128, 128, 32, 128, 256, 128, 160, 128, 128};
constexpr int kTileBN[10] = {128, 80, 64, 32, 160, 128, 128, 160, 160, 128};
constexpr int kTileSplit = 6, kTileSq160 = 7, kTileSplit160 = 8, kTileSplitV = 9;
// tiles 4..6 and 8 serve FP32 operands only, tile 7 FP64 only, tile 9 (split
// products with 4 x 4 staging) FP32 and the split modes when split_v4_ok
inline bool tile_valid(int t, Prec p) {
  if (t < 0 || t > 9) return false;
  if (t < 4) return true;
  if (t == kTileSplitV) return p == Prec::F32 || p == Prec::F32S || p == Prec::F64S;
  return t == kTileSq160 ? p == Prec::F64 : p == Prec::F32;
}

struct BatchIdx { int64_t i0, i1, i2; };

__device__ inline BatchIdx decode_batch(const GemmDesc &d, int id) {
  BatchIdx b;
  if (d.table) {
    b.i0 = d.table[3 * id + 0];
    b.i1 = d.table[3 * id + 1];
    b.i2 = d.table[3 * id + 2];
  } else {
    b.i0 = id / d.nb1;
    b.i1 = id % d.nb1;
    b.i2 = 0;
  }
  return b;
}

__device__ inline uint32_t fdiv(const FastDiv &f, uint32_t n) {
  const uint32_t t = __umulhi(f.m, n);
  return (t + ((n - t) >> f.s1)) >> f.s2;
}
__device__ inline int64_t two_index_off(const FastDiv &f, uint32_t n, int64_t s_o, int64_t s_i) {
  const uint32_t q = fdiv(f, n);
  return (int64_t)q * s_o + (int64_t)(n - q * f.d) * s_i;
}

// Prefetched elements are loaded unconditionally (from a clamped, always
// valid address) and kept as raw bits until they are written to LDS after the
// MFMA block; masking and scaling happen only there, so the wait for the loads
// lands after the arithmetic instead of before it.
template <typename E> struct BitsOf;
template <> struct BitsOf<double> { using U = uint64_t; };
template <> struct BitsOf<float> { using U = uint32_t; };
template <> struct BitsOf<uint16_t> { using U = uint16_t; };

template <class M> __device__ inline typename M::T scaled(typename M::T x, double s);
template <> __device__ inline double scaled<ModeF64>(double x, double s) { return s * x; }
template <> __device__ inline float scaled<ModeF32>(float x, double s) { return (float)s * x; }
template <> __device__ inline float scaled<ModeF32S>(float x, double s) { return (float)s * x; }
template <> __device__ inline double scaled<ModeF64S>(double x, double s) { return s * x; }

__device__ inline uint16_t bf16_rn_bits(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
// x -> (h, m, l) of the split-product mode
__device__ inline void split3(float x, uint16_t &h, uint16_t &m, uint16_t &l) {
  h = bf16_rn_bits(x);
  const float r1 = x - bf16_to_f32(h);
  m = bf16_rn_bits(r1);
  const float r2 = r1 - bf16_to_f32(m);
  l = bf16_rn_bits(r2);
}
// (scale = 1 for the B operand: the multiply folds away after inlining)
template <> __device__ inline uint16_t scaled<ModeBF16>(uint16_t x, double s) {
  return s == 1.0 ? x : f32_to_bf16((float)s * bf16_to_f32(x));
}

// Per-thread element ownership inside one BK-slice of an R-row operand tile
// (T threads, PER = R * BK / T elements each).
//   kfast (operand contiguous along k): element s -> (row t / BK + s T / BK,
//     k t % BK): one k per thread and slice.
//   otherwise 16 consecutive threads read 16 consecutive rows at one k: with
//     g = t / 16 and p = g PER + s, element s -> (row t % 16 + 16 (p % RG),
//     k p / RG), RG = R / 16 row groups; a thread touches KG = max(1, PER/RG)
//     values of k per slice.
template <class M, int R, int T>
struct Slice {
  static constexpr int BK = M::BK;
  static constexpr int PER = R * BK / T;
  static constexpr int RG = R / 16;
  static constexpr int KG = PER >= RG ? PER / RG : 1;
  // When the thread share and the row groups do not tile each other (160-row
  // tiles of 640 threads), the not-kfast layout is element s -> (row t % R,
  // k t / R + s T / R): one row per thread, consecutive threads on consecutive rows.
  static constexpr bool kWide = !(PER % RG == 0 || RG % PER == 0);
  static_assert(!kWide || (T % R == 0 && (T / R) * PER == BK), "wide layout needs T = n R");
  static_assert(PER <= 32, "in-range flags are kept in one 32-bit mask");
  using E = typename M::T;
  int64_t roff[PER];
  bool rok[PER];

  __device__ static int row_of(bool kfast, int s) {
    const int t = threadIdx.x;
    if (kfast) return t / BK + s * (T / BK);
    if constexpr (kWide) return t % R;
    return t % 16 + 16 * (((t / 16) * PER + s) % RG);
  }
  __device__ static int k_of(bool kfast, int s) {
    const int t = threadIdx.x;
    if (kfast) return t % BK;
    if constexpr (kWide) return t / R + s * (T / R);
    return ((t / 16) * PER + s) / RG;
  }
  __device__ void init(const GOperand &op, const FastDiv &rdiv, bool kfast, int nrows, int row0) {
#pragma unroll
    for (int s = 0; s < PER; ++s) {
      const int r = row0 + row_of(kfast, s);
      rok[s] = r < nrows;
      roff[s] = rok[s] ? two_index_off(rdiv, (uint32_t)r, op.s_ro, op.s_ri) : 0;
    }
  }
  // Issues the loads of one slice: raw bits in reg, in-range flags in okbits.
  __device__ void load(const E *__restrict__ base, const GOperand &op, const FastDiv &kdiv,
                       bool kfast, int K, int k0, E *reg, uint32_t &okbits) const {
    okbits = 0;
    if (kfast) {
      const int k = k0 + k_of(true, 0);
      const bool kok = k < K;
      const int64_t ko = kok ? two_index_off(kdiv, (uint32_t)k, op.s_ko, op.s_ki) : 0;
#pragma unroll
      for (int s = 0; s < PER; ++s) {
        const bool ok = kok && rok[s];
        okbits |= (uint32_t)ok << s;
        reg[s] = base[ok ? roff[s] + ko : 0];
      }
    } else if constexpr (kWide) {
#pragma unroll
      for (int s = 0; s < PER; ++s) {
        const int k = k0 + k_of(false, s);
        const bool kin = k < K;
        const int64_t ko = kin ? two_index_off(kdiv, (uint32_t)k, op.s_ko, op.s_ki) : 0;
        const bool ok = kin && rok[s];
        okbits |= (uint32_t)ok << s;
        reg[s] = base[ok ? roff[s] + ko : 0];
      }
    } else {
      int64_t ko[KG];
      bool kok[KG];
#pragma unroll
      for (int g = 0; g < KG; ++g) {
        const int k = k0 + k_of(false, g * RG);
        kok[g] = k < K;
        ko[g] = kok[g] ? two_index_off(kdiv, (uint32_t)k, op.s_ko, op.s_ki) : 0;
      }
#pragma unroll
      for (int s = 0; s < PER; ++s) {
        const int g = (KG > 1) ? s / RG : 0;
        const bool ok = kok[g] && rok[s];
        okbits |= (uint32_t)ok << s;
        reg[s] = base[ok ? roff[s] + ko[g] : 0];
      }
    }
  }
  // LDS tile: [k][row] with leading dimension LD, or [row][k] (kRowMajor);
  // split-product mode: three [row][k] tiles PS elements apart.
  template <int LD, int PS>
  __device__ static void store(typename M::L *lds, bool kfast, const E *reg, uint32_t okbits,
                               double scale) {
    using U = typename BitsOf<E>::U;
#pragma unroll
    for (int s = 0; s < PER; ++s) {
      const U m = ((okbits >> s) & 1u) ? (U)~(U)0 : (U)0;
      const E x = scaled<M>(__builtin_bit_cast(E, (U)(__builtin_bit_cast(U, reg[s]) & m)), scale);
      if constexpr (M::kPlanes == 3) {
        uint16_t h, mid, l;
        split3((float)x, h, mid, l);
        const int o = row_of(kfast, s) * LD + k_of(kfast, s);
        lds[o] = h;
        lds[PS + o] = mid;
        lds[2 * PS + o] = l;
      } else if (M::kRowMajor) {
        lds[row_of(kfast, s) * LD + k_of(kfast, s)] = x;
      } else {
        lds[k_of(kfast, s) * LD + row_of(kfast, s)] = x;
      }
    }
  }
};

// One LDS slice of MFMA steps.
template <class M, class C, int LDA, int LDB, int PSA, int PSB>
__device__ inline void mma_slice_impl(const typename M::L *Ab, const typename M::L *Bb, int lane,
                                      int wm, int wn, typename M::Acc (&acc)[C::MI][C::NI]) {
  const int mw = wm * (C::BM / C::WM), nw = wn * (C::BN / C::WN);
  if constexpr (M::kPlanes == 3) {
    // planes 0, 1, 2 = h, m, l; the six split products, each pass over all
    // (i, j) blocks so that consecutive matrix ops use different accumulators
    constexpr int kA[6] = {0, 0, 1, 0, 2, 1};
    constexpr int kB[6] = {0, 1, 0, 2, 0, 1};
#pragma unroll
    for (int kk = 0; kk < M::BK; kk += M::KS) {
      bf16x8_t af[3][C::MI], bf[3][C::NI];
#pragma unroll
      for (int p = 0; p < 3; ++p) {
#pragma unroll
        for (int i = 0; i < C::MI; ++i) {
          const u16x8_t raw = *(const u16x8_t *)(Ab + p * PSA + (mw + i * 16 + lane % 16) * LDA + kk + 8 * (lane / 16));
          af[p][i] = __builtin_bit_cast(bf16x8_t, raw);
        }
#pragma unroll
        for (int j = 0; j < C::NI; ++j) {
          const u16x8_t raw = *(const u16x8_t *)(Bb + p * PSB + (nw + j * 16 + lane % 16) * LDB + kk + 8 * (lane / 16));
          bf[p][j] = __builtin_bit_cast(bf16x8_t, raw);
        }
      }
#pragma unroll
      for (int t = 5; t >= 0; --t)   // smallest products first
#pragma unroll
        for (int i = 0; i < C::MI; ++i)
#pragma unroll
          for (int j = 0; j < C::NI; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[kA[t]][i], bf[kB[t]][j], acc[i][j], 0, 0, 0);
    }
  } else if constexpr (M::kRowMajor) {
    // bf16: lane reads 8 consecutive k of row (lane % 16) starting at 8 (lane / 16)
#pragma unroll
    for (int kk = 0; kk < M::BK; kk += M::KS) {
      bf16x8_t af[C::MI], bf[C::NI];
#pragma unroll
      for (int i = 0; i < C::MI; ++i) {
        const u16x8_t raw = *(const u16x8_t *)(Ab + (mw + i * 16 + lane % 16) * LDA + kk + 8 * (lane / 16));
        af[i] = __builtin_bit_cast(bf16x8_t, raw);
      }
#pragma unroll
      for (int j = 0; j < C::NI; ++j) {
        const u16x8_t raw = *(const u16x8_t *)(Bb + (nw + j * 16 + lane % 16) * LDB + kk + 8 * (lane / 16));
        bf[j] = __builtin_bit_cast(bf16x8_t, raw);
      }
#pragma unroll
      for (int i = 0; i < C::MI; ++i)
#pragma unroll
        for (int j = 0; j < C::NI; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
  } else {
#pragma unroll
    for (int kk = 0; kk < M::BK; kk += M::KS) {
      typename M::T af[C::MI], bf[C::NI];
#pragma unroll
      for (int i = 0; i < C::MI; ++i) af[i] = Ab[(kk + lane / 16) * LDA + mw + i * 16 + lane % 16];
#pragma unroll
      for (int j = 0; j < C::NI; ++j) bf[j] = Bb[(kk + lane / 16) * LDB + nw + j * 16 + lane % 16];
#pragma unroll
      for (int i = 0; i < C::MI; ++i)
#pragma unroll
        for (int j = 0; j < C::NI; ++j) {
          if constexpr (std::is_same<typename M::T, double>::value)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
          else
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
    }
  }
}

// k-slices of all segments, numbered consecutively; a split-K share is a
// contiguous range of them.
template <int BK>
__device__ inline int seg_slices(const GSegment &S) { return (S.K + BK - 1) / BK; }

// C[off] = v + beta * src[off]; src is C itself unless the descriptor names a
// separate input (same layout), which saves copying it into C first.
__device__ inline void store_out(const GemmDesc &d, void *base, const void *src, int64_t off,
                                 double v) {
  if (d.c_type == 1) {
    float *p = (float *)base + off;
    *p = (d.beta == 0.0) ? (float)v : (float)(v + d.beta * (double)((const float *)src)[off]);
  } else if (d.c_type == 2) {
    uint16_t *p = (uint16_t *)base + off;
    *p = f32_to_bf16((d.beta == 0.0) ? (float)v
                                     : (float)(v + d.beta * (double)bf16_to_f32(
                                                         ((const uint16_t *)src)[off])));
  } else {
    double *p = (double *)base + off;
    *p = (d.beta == 0.0) ? v : v + d.beta * ((const double *)src)[off];
  }
}

// Four consecutive rows of one output column (the FP32 accumulator registers
// of a lane), stored with one vector access; same rounding as store_out.
__device__ inline void store_out4(const GemmDesc &d, void *base, const void *src, int64_t off,
                                  float4_t v) {
  if (d.c_type == 1) {
    float4_t *p = (float4_t *)((float *)base + off);
    if (d.beta != 0.0) {
      const float4_t o = *(const float4_t *)((const float *)src + off);
#pragma unroll
      for (int r = 0; r < 4; ++r) v[r] = (float)((double)v[r] + d.beta * (double)o[r]);
    }
    *p = v;
  } else {
    double4_t *p = (double4_t *)((double *)base + off);
    double4_t w;
#pragma unroll
    for (int r = 0; r < 4; ++r) w[r] = (double)v[r];
    if (d.beta != 0.0) {
      const double4_t o = *(const double4_t *)((const double *)src + off);
#pragma unroll
      for (int r = 0; r < 4; ++r) w[r] = w[r] + d.beta * o[r];
    }
    *p = w;
  }
}

__device__ inline void store_out4(const GemmDesc &d, void *base, const void *src, int64_t off,
                                  double4_t w) {
  double4_t *p = (double4_t *)((double *)base + off);
  if (d.beta != 0.0) {
    const double4_t o = *(const double4_t *)((const double *)src + off);
#pragma unroll
    for (int r = 0; r < 4; ++r) w[r] = w[r] + d.beta * o[r];
  }
  *p = w;
}

// FP64 accumulators hold rows q + 4 r (q = lane / 16) of column lane % 16;
// three lane exchanges regroup them so that the lane holds rows 4 q + s,
// s = 0..3.  Round t: the lane offers its row q - t (mod 4) value and takes,
// from the lane of the same column with q' = q + t (mod 4), that lane's offer,
// which is row 4 q + q'.  Every lane of the wave must take part.
__device__ inline double pick4(const double4_t &a, int k) {
  return k == 0 ? a[0] : (k == 1 ? a[1] : (k == 2 ? a[2] : a[3]));
}
__device__ inline double4_t regroup_rows_f64(const double4_t &a, int lane) {
  const int q = lane >> 4, col = lane & 15;
  double4_t out = a;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const double offer = pick4(a, (q - t) & 3);
    const double got = t == 0 ? offer : __shfl(offer, (((q + t) & 3) << 4) | col, 64);
    const int s = (q + t) & 3;
#pragma unroll
    for (int r = 0; r < 4; ++r) out[r] = s == r ? got : out[r];
  }
  return out;
}

// Epilogue of the tile kernels: raw split-K partials, or the final store of
// C (vector stores of four adjacent rows when c_vec4 allows).
template <class M, class C>
__device__ inline void store_tile(const GemmDesc &d, typename M::Acc (&acc)[C::MI][C::NI], int m0,
                                  int n0, int wm, int wn, int lane, const BatchIdx &bi, int64_t id,
                                  int split) {
  if (d.splitk) {   // raw partial sums, row-major [split][M][N]
    double *pw = d.splitk + (int64_t)split * d.M * d.N;
#pragma unroll
    for (int i = 0; i < C::MI; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * (C::BM / C::WM) + i * 16 + M::row(lane, r);
        if (m >= d.M) continue;
#pragma unroll
        for (int j = 0; j < C::NI; ++j) {
          const int n = n0 + wn * (C::BN / C::WN) + j * 16 + lane % 16;
          if (n < d.N) pw[(int64_t)m * d.N + n] = (double)acc[i][j][r];
        }
      }
    return;
  }
  const int esz = d.c_type == 0 ? 8 : (d.c_type == 1 ? 4 : 2);
  const int64_t cbat = (bi.i0 * d.c_b0 + bi.i1 * d.c_b1 + bi.i2 * d.c_b2 + id * d.c_bid) * esz;
  char *pc = (char *)d.c + cbat;
  const char *ps = d.c_src ? (const char *)d.c_src + cbat : pc;
  int64_t coff[C::NI];
  bool cok[C::NI];
#pragma unroll
  for (int j = 0; j < C::NI; ++j) {
    const int n = n0 + wn * (C::BN / C::WN) + j * 16 + lane % 16;
    cok[j] = n < d.N;
    coff[j] = cok[j] ? two_index_off(d.ndiv, (uint32_t)n, d.c_no, d.c_ni) : 0;
  }
  if (d.c_vec4) {
    // rows 4 (lane / 16) + s, s = 0..3, of one column are adjacent in C: one
    // 16- or 32-byte access per column instead of four scattered ones
#pragma unroll
    for (int i = 0; i < C::MI; ++i) {
      const int m = m0 + wm * (C::BM / C::WM) + i * 16 + 4 * (lane / 16);
      const bool mok = m < d.M;
      const int64_t moff = mok ? two_index_off(d.mdiv, (uint32_t)m, d.c_mo, d.c_mi) : 0;
#pragma unroll
      for (int j = 0; j < C::NI; ++j) {
        if constexpr (std::is_same<typename M::Acc, double4_t>::value) {
          const double4_t w = regroup_rows_f64(acc[i][j], lane);   // whole wave
          if (mok && cok[j]) store_out4(d, pc, ps, moff + coff[j], w);
        } else {
          if (mok && cok[j]) store_out4(d, pc, ps, moff + coff[j], acc[i][j]);
        }
      }
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < C::MI; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + wm * (C::BM / C::WM) + i * 16 + M::row(lane, r);
      if (m >= d.M) continue;
      const int64_t moff = two_index_off(d.mdiv, (uint32_t)m, d.c_mo, d.c_mi);
#pragma unroll
      for (int j = 0; j < C::NI; ++j) {
        if (!cok[j]) continue;
        store_out(d, pc, ps, moff + coff[j], (double)acc[i][j][r]);
      }
    }
  }
}

// Workgroups per CU the register allocation must allow: two for the 8-wave FP64
// tiles (at most 128 VGPRs: a few row offsets spill), so that one workgroup's
// barrier and LDS stage overlap the other's matrix ops.  Measured: the FP64 matrix
// pipe was busy 55 % of the time with one such workgroup per CU; the K = naux
// products went 42 -> 48 TFLOP/s.
template <class M, class C>
constexpr int kMinBlocks = (std::is_same<M, ModeF64>::value && C::T == 512) ? 2 : 1;

template <class M, class C, int KIND>
__global__ __launch_bounds__(C::T) __attribute__((amdgpu_waves_per_eu(kMinBlocks<M, C> * C::T / 256)))
void gett_kernel(GemmDesc d, int tiles_m, int slices_per_split) {
  using E = typename M::T;
  constexpr int BK = M::BK;
  // [k][row] tiles pad the row (conflict-free 16-lane reads); [row][k] tiles pad
  // k to keep 16-byte alignment of each lane's 8-element read.
  constexpr int LDA = M::kRowMajor ? BK + 8 : C::BM + 4;
  constexpr int LDB = M::kRowMajor ? BK + 8 : C::BN + 4;
  constexpr int SZA = M::kRowMajor ? C::BM * LDA : BK * LDA;
  constexpr int SZB = M::kRowMajor ? C::BN * LDB : BK * LDB;
  using LE = typename M::L;
  constexpr int NP = M::kPlanes;
  __shared__ __attribute__((aligned(16))) LE As[2][NP * SZA];
  __shared__ __attribute__((aligned(16))) LE Bs[2][NP * SZB];

  const int tile = blockIdx.x;
  const int tm = tile % tiles_m, tn = tile / tiles_m;
  const int m0 = tm * C::BM, n0 = tn * C::BN;
  const BatchIdx bi = decode_batch(d, blockIdx.y);
  const int64_t id = blockIdx.y;
  const int split = blockIdx.z;
  const int q0 = split * slices_per_split, q1 = q0 + slices_per_split;

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = wave / C::WN, wn = wave % C::WN;

  typename M::Acc acc[C::MI][C::NI];
#pragma unroll
  for (int i = 0; i < C::MI; ++i)
#pragma unroll
    for (int j = 0; j < C::NI; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0;

  using SA = Slice<M, C::BM, C::T>;
  using SB = Slice<M, C::BN, C::T>;
  int qbase = 0;   // global slice number of the current segment's first slice
  for (int sg = 0; sg < d.nseg; ++sg) {
    const GSegment &S = d.seg[sg];
    const int ns = seg_slices<BK>(S);
    const int lo = max(q0, qbase) - qbase, hi = min(q1, qbase + ns) - qbase;
    qbase += ns;
    if (lo >= hi) continue;
    const E *pa = (const E *)S.a.p + bi.i0 * S.a.b0 + bi.i1 * S.a.b1 + bi.i2 * S.a.b2 + id * S.a.bid;
    const E *pb = (const E *)S.b.p + bi.i0 * S.b.b0 + bi.i1 * S.b.b1 + bi.i2 * S.b.b2 + id * S.b.bid;
    const bool akf = S.a_kfast != 0;
    const bool bkf = S.b_kfast != 0;
    SA sa;
    SB sb;
    sa.init(S.a, d.mdiv, akf, d.M, m0);
    sb.init(S.b, d.ndiv, bkf, d.N, n0);

    E ra[SA::PER], rb[SB::PER];
    uint32_t oka, okb;
    sa.load(pa, S.a, S.kdiv, akf, S.K, lo * BK, ra, oka);
    sb.load(pb, S.b, S.kdiv, bkf, S.K, lo * BK, rb, okb);
    __syncthreads();   // previous segment may still read buffer 0
    SA::template store<LDA, SZA>(As[0], akf, ra, oka, S.scale);
    SB::template store<LDB, SZB>(Bs[0], bkf, rb, okb, 1.0);
    __syncthreads();
    for (int q = lo; q < hi; ++q) {
      const int buf = (q - lo) & 1;
      if (q + 1 < hi) {
        sa.load(pa, S.a, S.kdiv, akf, S.K, (q + 1) * BK, ra, oka);
        sb.load(pb, S.b, S.kdiv, bkf, S.K, (q + 1) * BK, rb, okb);
      }
      mma_slice_impl<M, C, LDA, LDB, SZA, SZB>(As[buf], Bs[buf], lane, wm, wn, acc);
      if (q + 1 < hi) {
        SA::template store<LDA, SZA>(As[buf ^ 1], akf, ra, oka, S.scale);
        SB::template store<LDB, SZB>(Bs[buf ^ 1], bkf, rb, okb, 1.0);
      }
      __syncthreads();
    }
  }

  store_tile<M, C>(d, acc, m0, n0, wm, wn, lane, bi, id, split);
}

// Split-bf16 products with 4 x 4 staging blocks: 128 x 128 outputs per
// workgroup of 4 waves (64 x 64 each: 4 x 4 blocks of 16 x 16, so every LDS
// fragment feeds four matrix ops of each of the six part products), one LDS
// buffer of three bf16 planes per operand (60 KB, two workgroups per CU: one
// stages while the other multiplies).  Each thread stages one 4-row x 4-k block
// of each operand per 32-k slice: four 4-element vector loads (along k when the
// operand is contiguous along k, else along its rows, then transposed in
// registers), split, and one 8-byte LDS store per row and plane.  The host
// launches it only when every 4-element group is contiguous and aligned
// (split_v4_ok).
using SplitV = Cfg<128, 128, 2, 2>;

template <class E> struct Vec4Of;
template <> struct Vec4Of<float> { using V = float4_t; };
template <> struct Vec4Of<double> { using V = double4_t; };

template <class E>
struct Block4 {
  static constexpr int R = 128, BK = 32;
  using V = typename Vec4Of<E>::V;
  // one thread's 4 x 4 block: q0..q3 = rows 0..3, four consecutive k each (every
  // index below is a literal, so the block stays in registers)
  struct Regs { V q0, q1, q2, q3; };
  int64_t roff0, roff1, roff2, roff3;
  bool rok;
  // k-contiguous operands: 8 consecutive threads cover the 32 k of a row group
  // (coalesced loads, conflict-free 8-byte LDS stores); row-contiguous ones:
  // 32 consecutive threads cover the 128 rows at one k group
  __device__ static int rg(bool kfast) { return kfast ? threadIdx.x / 8 : threadIdx.x % 32; }
  __device__ static int kg(bool kfast) { return kfast ? threadIdx.x % 8 : threadIdx.x / 32; }
  __device__ void init(const GOperand &op, const FastDiv &rdiv, bool kfast, int nrows, int row0) {
    const int r0 = row0 + 4 * rg(kfast);
    rok = r0 < nrows;   // nrows is a multiple of 4
    roff0 = rok ? two_index_off(rdiv, (uint32_t)(r0 + 0), op.s_ro, op.s_ri) : 0;
    roff1 = rok ? two_index_off(rdiv, (uint32_t)(r0 + 1), op.s_ro, op.s_ri) : 0;
    roff2 = rok ? two_index_off(rdiv, (uint32_t)(r0 + 2), op.s_ro, op.s_ri) : 0;
    roff3 = rok ? two_index_off(rdiv, (uint32_t)(r0 + 3), op.s_ro, op.s_ri) : 0;
  }
  __device__ void load(const E *__restrict__ base, const GOperand &op, const FastDiv &kdiv,
                       bool kfast, int K, int k0, Regs &r, bool &ok) const {
    const int k = k0 + 4 * kg(kfast);
    ok = rok && k < K;   // K is a multiple of 4
    if (kfast) {
      const int64_t ko = ok ? two_index_off(kdiv, (uint32_t)k, op.s_ko, op.s_ki) : 0;
      r.q0 = *(const V *)(base + (ok ? roff0 + ko : 0));
      r.q1 = *(const V *)(base + (ok ? roff1 + ko : 0));
      r.q2 = *(const V *)(base + (ok ? roff2 + ko : 0));
      r.q3 = *(const V *)(base + (ok ? roff3 + ko : 0));
    } else {   // four rows at each of the four k, transposed into rows
      const V c0 = *(const V *)(base + (ok ? roff0 + two_index_off(kdiv, (uint32_t)(k + 0), op.s_ko, op.s_ki) : 0));
      const V c1 = *(const V *)(base + (ok ? roff0 + two_index_off(kdiv, (uint32_t)(k + 1), op.s_ko, op.s_ki) : 0));
      const V c2 = *(const V *)(base + (ok ? roff0 + two_index_off(kdiv, (uint32_t)(k + 2), op.s_ko, op.s_ki) : 0));
      const V c3 = *(const V *)(base + (ok ? roff0 + two_index_off(kdiv, (uint32_t)(k + 3), op.s_ko, op.s_ki) : 0));
      r.q0 = V{c0[0], c1[0], c2[0], c3[0]};
      r.q1 = V{c0[1], c1[1], c2[1], c3[1]};
      r.q2 = V{c0[2], c1[2], c2[2], c3[2]};
      r.q3 = V{c0[3], c1[3], c2[3], c3[3]};
    }
  }
  // one row: four values split into the three planes, one 8-byte store per plane
  template <int LD, int PS>
  __device__ static void put_row(uint16_t *lds, int o, const V &x, bool ok, double scale) {
    uint16_t h0, m0, l0, h1, m1, l1, h2, m2, l2, h3, m3, l3;
    const float sc = (float)scale;
    split3(ok ? sc * (float)x[0] : 0.0f, h0, m0, l0);
    split3(ok ? sc * (float)x[1] : 0.0f, h1, m1, l1);
    split3(ok ? sc * (float)x[2] : 0.0f, h2, m2, l2);
    split3(ok ? sc * (float)x[3] : 0.0f, h3, m3, l3);
    *(uint2 *)(lds + o) = make_uint2((uint32_t)h0 | ((uint32_t)h1 << 16), (uint32_t)h2 | ((uint32_t)h3 << 16));
    *(uint2 *)(lds + PS + o) = make_uint2((uint32_t)m0 | ((uint32_t)m1 << 16), (uint32_t)m2 | ((uint32_t)m3 << 16));
    *(uint2 *)(lds + 2 * PS + o) = make_uint2((uint32_t)l0 | ((uint32_t)l1 << 16), (uint32_t)l2 | ((uint32_t)l3 << 16));
  }
  template <int LD, int PS>
  __device__ static void store(uint16_t *lds, bool kfast, const Regs &r, bool ok, double scale) {
    const int o = 4 * rg(kfast) * LD + 4 * kg(kfast);
    put_row<LD, PS>(lds, o, r.q0, ok, scale);
    put_row<LD, PS>(lds, o + LD, r.q1, ok, scale);
    put_row<LD, PS>(lds, o + 2 * LD, r.q2, ok, scale);
    put_row<LD, PS>(lds, o + 3 * LD, r.q3, ok, scale);
  }
};

template <class M, int KIND>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void gett_split_v4(GemmDesc d, int tiles_m, int slices_per_split) {
  using C = SplitV;
  using E = typename M::T;
  constexpr int BK = 32, LD = BK + 8, SZ = C::BM * LD;   // both operands 128 rows
  __shared__ __attribute__((aligned(16))) uint16_t As[3 * SZ];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[3 * SZ];

  int tm, tn;
  xcd_tile(blockIdx.x, tiles_m, gridDim.x / tiles_m, tm, tn);
  const int m0 = tm * C::BM, n0 = tn * C::BN;
  const BatchIdx bi = decode_batch(d, blockIdx.y);
  const int64_t id = blockIdx.y;
  const int split = blockIdx.z;
  const int q0 = split * slices_per_split, q1 = q0 + slices_per_split;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = wave / C::WN, wn = wave % C::WN;

  typename M::Acc acc[C::MI][C::NI];
#pragma unroll
  for (int i = 0; i < C::MI; ++i)
#pragma unroll
    for (int j = 0; j < C::NI; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0;

  int qbase = 0;
  for (int sg = 0; sg < d.nseg; ++sg) {
    const GSegment &S = d.seg[sg];
    const int ns = (S.K + BK - 1) / BK;
    const int lo = max(q0, qbase) - qbase, hi = min(q1, qbase + ns) - qbase;
    qbase += ns;
    if (lo >= hi) continue;
    const E *pa = (const E *)S.a.p + bi.i0 * S.a.b0 + bi.i1 * S.a.b1 + bi.i2 * S.a.b2 + id * S.a.bid;
    const E *pb = (const E *)S.b.p + bi.i0 * S.b.b0 + bi.i1 * S.b.b1 + bi.i2 * S.b.b2 + id * S.b.bid;
    const bool akf = S.a_kfast != 0, bkf = S.b_kfast != 0;
    Block4<E> sa, sb;
    sa.init(S.a, d.mdiv, akf, d.M, m0);
    sb.init(S.b, d.ndiv, bkf, d.N, n0);
    typename Block4<E>::Regs ra, rb;
    bool oka, okb;
    sa.load(pa, S.a, S.kdiv, akf, S.K, lo * BK, ra, oka);
    sb.load(pb, S.b, S.kdiv, bkf, S.K, lo * BK, rb, okb);
    __syncthreads();   // the previous segment's last slice has been read
    Block4<E>::template store<LD, SZ>(As, akf, ra, oka, S.scale);
    Block4<E>::template store<LD, SZ>(Bs, bkf, rb, okb, 1.0);
    __syncthreads();
    for (int q = lo; q < hi; ++q) {
      const bool more = q + 1 < hi;
      if (more) {
        sa.load(pa, S.a, S.kdiv, akf, S.K, (q + 1) * BK, ra, oka);
        sb.load(pb, S.b, S.kdiv, bkf, S.K, (q + 1) * BK, rb, okb);
      }
      mma_slice_impl<M, C, LD, LD, SZ, SZ>(As, Bs, lane, wm, wn, acc);
      if (more) {
        __syncthreads();   // every wave has read the slice
        Block4<E>::template store<LD, SZ>(As, akf, ra, oka, S.scale);
        Block4<E>::template store<LD, SZ>(Bs, bkf, rb, okb, 1.0);
        __syncthreads();
      }
    }
  }
  store_tile<M, C>(d, acc, m0, n0, wm, wn, lane, bi, id, split);
}

// Matrix-vector products (N = 1, one segment, FP64, no batch):
// C[m] = scale sum_k A(m, k) B(k) + beta C[m].  A contiguous along m: a block
// holds kGvM rows (one per lane group) and kGvT / kGvM interleaved k streams per
// row, summed in LDS in a fixed order.  A contiguous along k: one wave per row,
// lanes stride over k, summed by a fixed shuffle tree.  Either way every output
// is one sum in a fixed order, so results do not depend on scheduling.
constexpr int kGvT = 256;
__global__ __launch_bounds__(kGvT) void gemv_rows(GemmDesc d, int rows_per_block) {
  __shared__ double part[kGvT];
  const GSegment &S = d.seg[0];
  const int rb = rows_per_block, kg = kGvT / rb;
  const int r = threadIdx.x % rb, g = threadIdx.x / rb;
  const int m = blockIdx.x * rb + r;
  const double *A = (const double *)S.a.p, *B = (const double *)S.b.p;
  double acc = 0.0;
  if (m < d.M) {
    // four independent partial sums (loads of four k in flight), added in order
    const int64_t ro = two_index_off(d.mdiv, (uint32_t)m, S.a.s_ro, S.a.s_ri);
    double a4[4] = {0.0, 0.0, 0.0, 0.0};
    int k = g;
    for (; k + 3 * kg < S.K; k += 4 * kg) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int ku = k + u * kg;
        a4[u] += A[ro + two_index_off(S.kdiv, (uint32_t)ku, S.a.s_ko, S.a.s_ki)] *
                 B[two_index_off(S.kdiv, (uint32_t)ku, S.b.s_ko, S.b.s_ki)];
      }
    }
    for (; k < S.K; k += kg)
      a4[0] += A[ro + two_index_off(S.kdiv, (uint32_t)k, S.a.s_ko, S.a.s_ki)] *
               B[two_index_off(S.kdiv, (uint32_t)k, S.b.s_ko, S.b.s_ki)];
    acc = (a4[0] + a4[1]) + (a4[2] + a4[3]);
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  if (g == 0 && m < d.M) {
    double t = part[r];
    for (int q = 1; q < kg; ++q) t += part[q * rb + r];
    const int64_t off = two_index_off(d.mdiv, (uint32_t)m, d.c_mo, d.c_mi);
    double *c = (double *)d.c;
    const double *src = d.c_src ? (const double *)d.c_src : c;
    c[off] = (d.beta == 0.0) ? S.scale * t : S.scale * t + d.beta * src[off];
  }
}
__global__ __launch_bounds__(kGvT) void gemv_dots(GemmDesc d) {
  const GSegment &S = d.seg[0];
  const int lane = threadIdx.x & 63;
  const int m = blockIdx.x * (kGvT / 64) + threadIdx.x / 64;
  if (m >= d.M) return;   // whole waves
  const double *A = (const double *)S.a.p, *B = (const double *)S.b.p;
  const int64_t ro = two_index_off(d.mdiv, (uint32_t)m, S.a.s_ro, S.a.s_ri);
  double a4[4] = {0.0, 0.0, 0.0, 0.0};
  int k = lane;
  for (; k + 192 < S.K; k += 256) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int ku = k + 64 * u;
      a4[u] += A[ro + two_index_off(S.kdiv, (uint32_t)ku, S.a.s_ko, S.a.s_ki)] *
               B[two_index_off(S.kdiv, (uint32_t)ku, S.b.s_ko, S.b.s_ki)];
    }
  }
  for (; k < S.K; k += 64)
    a4[0] += A[ro + two_index_off(S.kdiv, (uint32_t)k, S.a.s_ko, S.a.s_ki)] *
             B[two_index_off(S.kdiv, (uint32_t)k, S.b.s_ko, S.b.s_ki)];
  double acc = (a4[0] + a4[1]) + (a4[2] + a4[3]);
#pragma unroll
  for (int w = 32; w >= 1; w >>= 1) acc += __shfl_xor(acc, w, 64);
  if (lane == 0) {
    const int64_t off = two_index_off(d.mdiv, (uint32_t)m, d.c_mo, d.c_mi);
    double *c = (double *)d.c;
    const double *src = d.c_src ? (const double *)d.c_src : c;
    c[off] = (d.beta == 0.0) ? S.scale * acc : S.scale * acc + d.beta * src[off];
  }
}

// C[m, n] = sum_s partial[s][m][n] (+ beta C), summed in split order.
__device__ inline void splitk_store(const GemmDesc &d, int64_t e, double acc) {
  const int m = (int)(e / d.N), n = (int)(e % d.N);
  const int64_t off = (int64_t)(m / d.Mi) * d.c_mo + (int64_t)(m % d.Mi) * d.c_mi +
                      (int64_t)(n / d.Ni) * d.c_no + (int64_t)(n % d.Ni) * d.c_ni;
  store_out(d, d.c, d.c_src ? d.c_src : d.c, off, acc);
}
__global__ void splitk_reduce(GemmDesc d, int nsplit) {
  const int64_t total = (int64_t)d.M * d.N;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int s = 0; s < nsplit; ++s) acc += d.splitk[s * total + e];
    splitk_store(d, e, acc);
  }
}
// Many splits of a small output: 32 lanes share the splits of each of 8
// outputs per block (strided partial sums, then a fixed-order tree).
constexpr int kRedLanes = 32, kRedOuts = 8;
__global__ void splitk_reduce_wide(GemmDesc d, int nsplit) {
  __shared__ double sm[kRedOuts][kRedLanes + 1];
  const int64_t total = (int64_t)d.M * d.N;
  const int lane = threadIdx.x % kRedLanes, oi = threadIdx.x / kRedLanes;
  const int64_t e = (int64_t)blockIdx.x * kRedOuts + oi;
  double acc = 0.0;
  if (e < total)
    for (int s = lane; s < nsplit; s += kRedLanes) acc += d.splitk[s * total + e];
  sm[oi][lane] = acc;
  __syncthreads();
  for (int w = kRedLanes / 2; w > 0; w >>= 1) {
    if (lane < w) sm[oi][lane] += sm[oi][lane + w];
    __syncthreads();
  }
  if (lane == 0 && e < total) splitk_store(d, e, sm[oi][0]);
}

}  // namespace

namespace {
thread_local const Region *g_regions = nullptr;
thread_local int g_nregions = 0;

// [lo, hi] element offsets reachable from an operand's base pointer.
struct Span { int64_t lo, hi; };
void add_term(Span &s, int64_t idx_max, int64_t stride) {
  if (idx_max <= 0 || stride == 0) return;
  if (stride > 0) s.hi += idx_max * stride; else s.lo += idx_max * stride;
}
bool inside(const void *base, Span sp, size_t elem) {
  const char *lo = (const char *)base + sp.lo * (int64_t)elem;
  const char *hi = (const char *)base + (sp.hi + 1) * (int64_t)elem;
  for (int r = 0; r < g_nregions; ++r) {
    const char *a = (const char *)g_regions[r].p, *b = a + g_regions[r].bytes;
    if (lo >= a && hi <= b) return true;
  }
  return false;
}
int64_t outer_max(int64_t n, int64_t inner) { return (n - 1) / inner; }
int64_t inner_max(int64_t n, int64_t inner) { return std::min(n, inner) - 1; }

bool operand_ok(const GemmDesc &d, const GOperand &op, int64_t rows, int64_t Ri, int64_t K,
                int64_t Ki, const int64_t bmax[3]) {
  if (rows <= 0 || K <= 0) return true;
  Span s{0, 0};
  add_term(s, outer_max(rows, Ri), op.s_ro);
  add_term(s, inner_max(rows, Ri), op.s_ri);
  add_term(s, outer_max(K, Ki), op.s_ko);
  add_term(s, inner_max(K, Ki), op.s_ki);
  add_term(s, bmax[0], op.b0);
  add_term(s, bmax[1], op.b1);
  add_term(s, bmax[2], op.b2);
  add_term(s, d.batch - 1, op.bid);
  const size_t esz = (d.prec == Prec::F64 || d.prec == Prec::F64S) ? 8 : (d.prec == Prec::BF16 ? 2 : 4);
  return inside(op.p, s, esz);
}

}  // namespace

bool region_ok(const void *p, size_t bytes) {
  if (!g_regions || bytes == 0) return true;
  return inside(p, Span{0, (int64_t)bytes - 1}, 1);
}

namespace {
bool descriptor_ok(const GemmDesc &d, int nsplit) {
  if (!g_regions) return true;
  int64_t bmax[3];
  if (d.table) { bmax[0] = d.tmax[0]; bmax[1] = d.tmax[1]; bmax[2] = d.tmax[2]; }
  else { bmax[0] = (d.batch - 1) / d.nb1; bmax[1] = std::min(d.batch, d.nb1) - 1; bmax[2] = 0; }
  for (int s = 0; s < d.nseg; ++s) {
    const GSegment &g = d.seg[s];
    if (!operand_ok(d, g.a, d.M, d.Mi, g.K, g.Ki, bmax)) return false;
    if (!operand_ok(d, g.b, d.N, d.Ni, g.K, g.Ki, bmax)) return false;
  }
  Span c{0, 0};
  add_term(c, outer_max(d.M, d.Mi), d.c_mo);
  add_term(c, inner_max(d.M, d.Mi), d.c_mi);
  add_term(c, outer_max(d.N, d.Ni), d.c_no);
  add_term(c, inner_max(d.N, d.Ni), d.c_ni);
  add_term(c, bmax[0], d.c_b0);
  add_term(c, bmax[1], d.c_b1);
  add_term(c, bmax[2], d.c_b2);
  add_term(c, d.batch - 1, d.c_bid);
  if (!inside(d.c, c, d.c_type == 0 ? 8 : (d.c_type == 1 ? 4 : 2))) return false;
  if (d.c_src && !inside(d.c_src, c, d.c_type == 0 ? 8 : (d.c_type == 1 ? 4 : 2))) return false;
  if (nsplit > 1 && !inside(d.splitk, Span{0, (int64_t)nsplit * d.M * d.N - 1}, sizeof(double)))
    return false;
  return true;
}
}  // namespace

// Process-wide switches (atomic: read by every launching thread).
static std::atomic<bool> g_dry{false};

struct Record { Kind kind; hipEvent_t start, stop; double flops; std::string shape; };
static std::atomic<bool> g_profile{false};
static std::mutex g_records_mu;        // launch records of every thread
static std::vector<Record> g_records;

void profile_enable(bool on) { g_profile = on; }

LaunchTimer profile_begin(hipStream_t s) {
  LaunchTimer t;
  if (!g_profile || g_dry) return t;
  if (hipEventCreate(&t.start) != hipSuccess || hipEventCreate(&t.stop) != hipSuccess) {
    if (t.start) (void)hipEventDestroy(t.start);
    t.start = t.stop = nullptr;
    return t;
  }
  (void)hipEventRecord(t.start, s);
  return t;
}

void profile_end(LaunchTimer &t, hipStream_t s, Kind kind, double flops) {
  if (!t.start) return;
  (void)hipEventRecord(t.stop, s);
  std::lock_guard<std::mutex> lock(g_records_mu);
  g_records.push_back(Record{kind, t.start, t.stop, flops, std::string()});
  t.start = t.stop = nullptr;
}
bool profile_enabled() { return g_profile; }

// LNOCC_PROFILE_DUMP=1: profile_collect also prints every contraction shape
// with its launch count, time and rate, largest time first.
void profile_collect(KindStats out[(int)Kind::Count]) {
  for (int k = 0; k < (int)Kind::Count; ++k) out[k] = KindStats{0, 0.0, 0.0};
  const bool dump = std::getenv("LNOCC_PROFILE_DUMP") != nullptr;
  std::map<std::string, KindStats> by_shape;
  std::lock_guard<std::mutex> lock(g_records_mu);
  for (const Record &r : g_records) {
    float ms = 0.f;
    (void)hipEventSynchronize(r.stop);
    (void)hipEventElapsedTime(&ms, r.start, r.stop);
    KindStats &k = out[(int)r.kind];
    k.launches += 1;
    k.ms += ms;
    k.flops += r.flops;
    if (dump) {
      KindStats &b = by_shape[r.shape];
      b.launches += 1;
      b.ms += ms;
      b.flops += r.flops;
    }
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
  }
  g_records.clear();
  if (dump) {
    std::vector<std::pair<std::string, KindStats>> v(by_shape.begin(), by_shape.end());
    std::sort(v.begin(), v.end(), [](const auto &a, const auto &b) { return a.second.ms > b.second.ms; });
    for (const auto &e : v)
      std::fprintf(stderr, "lnocc-prof %9.3f ms %6lld x %7.2f TF/s  %s\n", e.second.ms,
                   (long long)e.second.launches, e.second.flops / (e.second.ms * 1e9),
                   e.first.c_str());
  }
}
bool dry_run() { return g_dry; }
void set_dry_run(bool on) { g_dry = on; }

void install_regions(const Region *r, int n) {
  g_regions = (n > 0) ? r : nullptr;
  g_nregions = (n > 0) ? n : 0;
}

static int contiguous_along_k(const GOperand &op, int Ki) {
  return (Ki > 1) ? (op.s_ki == 1) : (op.s_ko == 1);
}

namespace {
template <class M, class C>
void launch_kind(const GemmDesc &d, dim3 grid, int tiles_m, int sps, hipStream_t stream) {
  switch (d.kind) {
    case Kind::LadderBuild:
      hipLaunchKernelGGL((gett_kernel<M, C, 1>), grid, dim3(C::T), 0, stream, d, tiles_m, sps); break;
    case Kind::LadderContract:
      hipLaunchKernelGGL((gett_kernel<M, C, 2>), grid, dim3(C::T), 0, stream, d, tiles_m, sps); break;
    case Kind::TriplesW:
      hipLaunchKernelGGL((gett_kernel<M, C, 3>), grid, dim3(C::T), 0, stream, d, tiles_m, sps); break;
    case Kind::Ring:   // FP64 operands (FP64 or split products)
      if constexpr (std::is_same<M, ModeF64>::value || std::is_same<M, ModeF64S>::value)
        hipLaunchKernelGGL((gett_kernel<M, C, 5>), grid, dim3(C::T), 0, stream, d, tiles_m, sps);
      else
        hipLaunchKernelGGL((gett_kernel<M, C, 0>), grid, dim3(C::T), 0, stream, d, tiles_m, sps);
      break;
    case Kind::Mlp:
      if constexpr (std::is_same<M, ModeF32>::value) {
        hipLaunchKernelGGL((gett_kernel<M, C, 4>), grid, dim3(C::T), 0, stream, d, tiles_m, sps);
        break;
      }
      [[fallthrough]];
    default:
      hipLaunchKernelGGL((gett_kernel<M, C, 0>), grid, dim3(C::T), 0, stream, d, tiles_m, sps); break;
  }
}
template <class C>
void launch_f32(const GemmDesc &d, dim3 grid, int tiles_m, int sps, hipStream_t stream) {
  launch_kind<ModeF32, C>(d, grid, tiles_m, sps, stream);
}
template <class C>
void launch_f64(const GemmDesc &d, dim3 grid, int tiles_m, int sps, hipStream_t stream) {
  launch_kind<ModeF64, C>(d, grid, tiles_m, sps, stream);
}
template <class M>
void launch_split_v4_kind(const GemmDesc &d, dim3 grid, int tiles_m, int sps, hipStream_t stream) {
  switch (d.kind) {
    case Kind::LadderContract:
      hipLaunchKernelGGL((gett_split_v4<M, 2>), grid, dim3(256), 0, stream, d, tiles_m, sps); break;
    case Kind::TriplesW:
      hipLaunchKernelGGL((gett_split_v4<M, 3>), grid, dim3(256), 0, stream, d, tiles_m, sps); break;
    case Kind::Ring:
      hipLaunchKernelGGL((gett_split_v4<M, 5>), grid, dim3(256), 0, stream, d, tiles_m, sps); break;
    default:
      hipLaunchKernelGGL((gett_split_v4<M, 0>), grid, dim3(256), 0, stream, d, tiles_m, sps); break;
  }
}
void launch_split_v4(const GemmDesc &d, dim3 grid, int tiles_m, int sps, hipStream_t stream) {
  if (d.prec == Prec::F64S) launch_split_v4_kind<ModeF64S>(d, grid, tiles_m, sps, stream);
  else launch_split_v4_kind<ModeF32S>(d, grid, tiles_m, sps, stream);
}
// gett_split_v4 stages 4 x 4 operand blocks with 4-element vector loads: every
// 4-element group (along k for a k-contiguous operand, along its rows
// otherwise) must be contiguous and aligned, and M, N and every K multiples of 4.
bool split_v4_ok(const GemmDesc &d) {
  if (d.prec != Prec::F32 && d.prec != Prec::F32S && d.prec != Prec::F64S) return false;
  if (d.M % 4 || d.N % 4) return false;
  const int64_t esz = d.prec == Prec::F64S ? 8 : 4;
  auto al = [](int64_t x) { return x % 4 == 0; };
  auto op_ok = [&](const GOperand &o, int rows_i, int Ki, bool kfast) {
    if (((uintptr_t)o.p) % (4 * esz)) return false;
    if (!al(o.b0) || !al(o.b1) || !al(o.b2) || !al(o.bid)) return false;
    if (kfast) {
      const bool kg = Ki == 1 ? o.s_ko == 1 : (o.s_ki == 1 && Ki % 4 == 0 && al(o.s_ko));
      return kg && al(o.s_ro) && (rows_i == 1 || al(o.s_ri));
    }
    const bool rg = rows_i == 1 ? o.s_ro == 1 : (o.s_ri == 1 && rows_i % 4 == 0 && al(o.s_ro));
    return rg && al(o.s_ko) && (Ki == 1 || al(o.s_ki));
  };
  for (int q = 0; q < d.nseg; ++q) {
    const GSegment &S = d.seg[q];
    if (S.K % 4) return false;
    if (!op_ok(S.a, d.Mi, S.Ki, contiguous_along_k(S.a, S.Ki))) return false;
    if (!op_ok(S.b, d.Ni, S.Ki, contiguous_along_k(S.b, S.Ki))) return false;
  }
  return true;
}

template <class C>
void launch(const GemmDesc &d, dim3 grid, int tiles_m, int sps, hipStream_t stream) {
  switch (d.prec) {
    case Prec::F32: launch_kind<ModeF32, C>(d, grid, tiles_m, sps, stream); break;
    case Prec::BF16: launch_kind<ModeBF16, C>(d, grid, tiles_m, sps, stream); break;
    case Prec::F32S: launch_kind<ModeF32S, C>(d, grid, tiles_m, sps, stream); break;
    case Prec::F64S: launch_kind<ModeF64S, C>(d, grid, tiles_m, sps, stream); break;
    default: launch_kind<ModeF64, C>(d, grid, tiles_m, sps, stream); break;
  }
}

thread_local double *g_splitk = nullptr;
thread_local size_t g_splitk_elems = 0;
thread_local char g_error[512] = "";

}  // namespace

void note_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(g_error, sizeof(g_error), fmt, ap);
  va_end(ap);
  if (std::getenv("LNOCC_DEBUG")) std::fprintf(stderr, "lnocc: %s\n", g_error);
}
const char *last_error() { return g_error; }
void clear_error() {
  g_error[0] = 0;
  // The launch wrappers read hipGetLastError(), which also holds the error of
  // any earlier runtime call of the process (say, an allocation failure that
  // the caller recovered from); start every entry point with it cleared.
  if (!g_dry) (void)hipGetLastError();
}

void install_splitk_scratch(double *p, size_t elems) {
  g_splitk = p;
  g_splitk_elems = p ? elems : 0;
}

// ---------------------------------------------------------------- autotuning
// Candidate c = (tile, split rule): tiles 128x128, 128x80, 128x64, 32x32 (and,
// for FP32 products, 128x160, 256x128, and 128x128 and 128x160 with split bf16 products;
// for FP64 products, 160x160; for FP32 and split products whose operands allow it,
// the 4 x 4-staged split tile);
// split rules: the cost-model split, no split, twice the cost-model split.  While a
// candidate is active every launch is timed with events under its shape key;
// tune_commit() keeps, per key, the fastest candidate's (tile, split count),
// which later launches of that shape use instead of the heuristic.
namespace {
constexpr int kTileCands = 10, kSplitRules = 3;
struct TilePlan { int tile; int nsplit; };
std::mutex g_plan_mu;
std::map<std::string, TilePlan> g_plans;
std::atomic<bool> g_have_plans{false};   // !g_plans.empty(), readable without the lock
thread_local int g_cand = -1;          // -1 off, kProbeCand: keys only
constexpr int kProbeCand = 1 << 20;
thread_local int g_unplanned = 0;      // keys seen by a probe pass without a plan
struct TuneRec { std::string key; int cand; TilePlan plan; hipEvent_t a, b; };
thread_local std::vector<TuneRec> g_tune;

std::string plan_key(const GemmDesc &d) {
  std::string k;
  char buf[192];
  std::snprintf(buf, sizeof(buf), "%d.%d.%d|%d.%d.%d.%d|%d.%d.%d.%d.%d", (int)d.kind, (int)d.prec,
                d.c_type, d.M, d.Mi, d.N, d.Ni, d.batch, d.nb1, d.table ? 1 : 0,
                d.beta == 0.0 ? 0 : 1, d.nseg);
  k += buf;
  for (int s = 0; s < d.nseg; ++s) {
    const GSegment &g = d.seg[s];
    std::snprintf(buf, sizeof(buf), "|%d.%d:%lld.%lld.%lld.%lld:%lld.%lld.%lld.%lld", g.K, g.Ki,
                  (long long)g.a.s_ro, (long long)g.a.s_ri, (long long)g.a.s_ko,
                  (long long)g.a.s_ki, (long long)g.b.s_ro, (long long)g.b.s_ri,
                  (long long)g.b.s_ko, (long long)g.b.s_ki);
    k += buf;
  }
  std::snprintf(buf, sizeof(buf), "|%lld.%lld.%lld.%lld", (long long)d.c_mo, (long long)d.c_mi,
                (long long)d.c_no, (long long)d.c_ni);
  k += buf;
  return k;
}
}  // namespace

int tune_candidates() { return kTileCands * kSplitRules; }
void tune_candidate(int c) { g_cand = c; }
void tune_probe_begin() {
  g_cand = kProbeCand;
  g_unplanned = 0;
}
int tune_probe_end() {
  g_cand = -1;
  return g_unplanned;
}

int tune_commit() {
  std::map<std::string, std::map<int, std::pair<double, TilePlan>>> t;
  for (TuneRec &r : g_tune) {
    float ms = 0.f;
    (void)hipEventSynchronize(r.b);
    (void)hipEventElapsedTime(&ms, r.a, r.b);
    auto &e = t[r.key][r.cand];
    e.first += ms;
    e.second = r.plan;
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_tune.clear();
  std::lock_guard<std::mutex> lock(g_plan_mu);
  for (auto &kv : t) {
    double best = -1.0;
    TilePlan plan{0, 1};
    for (auto &c : kv.second)
      if (best < 0 || c.second.first < best) { best = c.second.first; plan = c.second.second; }
    g_plans[kv.first] = plan;
  }
  g_have_plans = !g_plans.empty();
  return (int)t.size();
}

size_t tune_plans() {
  std::lock_guard<std::mutex> lock(g_plan_mu);
  return g_plans.size();
}

int tune_save(const char *path) {
  std::lock_guard<std::mutex> lock(g_plan_mu);
  FILE *f = std::fopen(path, "w");
  if (!f) return -1;
  for (auto &kv : g_plans) std::fprintf(f, "%s %d %d\n", kv.first.c_str(), kv.second.tile, kv.second.nsplit);
  return std::fclose(f) == 0 ? (int)g_plans.size() : -1;
}

int tune_load(const char *path) {
  FILE *f = std::fopen(path, "r");
  if (!f) return -1;
  std::lock_guard<std::mutex> lock(g_plan_mu);
  char key[1024];
  int tile = 0, ns = 0, n = 0;
  while (std::fscanf(f, "%1023s %d %d", key, &tile, &ns) == 3) {
    if (tile < 0 || tile >= kTileCands || ns < 1) continue;
    g_plans[key] = TilePlan{tile, ns};
    ++n;
  }
  g_have_plans = !g_plans.empty();
  std::fclose(f);
  return n;
}

void tune_clear() {
  std::lock_guard<std::mutex> lock(g_plan_mu);
  g_plans.clear();
  g_have_plans = false;
}

hipError_t gett(const GemmDesc &din, hipStream_t stream) {
  GemmDesc d = din;
  d.splitk = nullptr;
  if (d.M <= 0 || d.N <= 0 || d.batch <= 0) return hipSuccess;
  if (d.Mi <= 0 || d.Ni <= 0 || d.nseg <= 0 || d.nseg > kMaxSeg) return hipErrorInvalidValue;
  // k per LDS slice: 32 for the bf16 matrix-core arithmetics, else 16
  auto tile_bk = [&](int t) {
    return (d.prec == Prec::BF16 || d.prec == Prec::F32S || d.prec == Prec::F64S || t == kTileSplit ||
            t == kTileSplitV ||
            t == kTileSplit160) ? 32 : 16;
  };
  int slices16 = 0, slices32 = 0;
  for (int s = 0; s < d.nseg; ++s) {
    if (d.seg[s].K < 0 || d.seg[s].Ki <= 0) return hipErrorInvalidValue;
    d.seg[s].a_kfast = contiguous_along_k(d.seg[s].a, d.seg[s].Ki);
    d.seg[s].b_kfast = contiguous_along_k(d.seg[s].b, d.seg[s].Ki);
    d.seg[s].kdiv = make_fastdiv((uint32_t)d.seg[s].Ki);
    slices16 += (d.seg[s].K + 15) / 16;
    slices32 += (d.seg[s].K + 31) / 32;
  }
  auto tile_slices = [&](int t) { return tile_bk(t) == 32 ? slices32 : slices16; };
  if (d.batch > 65535) return hipErrorInvalidValue;
  if (d.table == nullptr && d.nb1 <= 0) return hipErrorInvalidValue;
  d.mdiv = make_fastdiv((uint32_t)d.Mi);
  d.ndiv = make_fastdiv((uint32_t)d.Ni);
  {  // vector stores of 4-row groups (FP64 or FP32 C; FP64 products: FP64 C)
    const int64_t esz = d.c_type == 0 ? 8 : 4;
    const bool rows = (d.Mi % 4 == 0 && d.c_mi == 1 && d.c_mo % 4 == 0) ||
                      (d.Mi == 1 && d.c_mo == 1);
    const bool cols = d.c_no % 4 == 0 && (d.Ni == 1 || d.c_ni % 4 == 0);
    d.c_vec4 = (d.prec != Prec::F64 || d.c_type == 0) && d.c_type != 2 && rows && cols &&
               d.M % 4 == 0 &&
               d.c_b0 % 4 == 0 && d.c_b1 % 4 == 0 && d.c_b2 % 4 == 0 && d.c_bid % 4 == 0 &&
               (reinterpret_cast<uintptr_t>(d.c) % (4 * esz)) == 0 &&
               (reinterpret_cast<uintptr_t>(d.c_src) % (4 * esz)) == 0;
  }
  // Matrix-vector products take their own kernels (no tiles, no plans).
  if (d.N == 1 && d.batch == 1 && d.nseg == 1 && d.prec == Prec::F64 && d.c_type == 0 &&
      d.tile_hint == 0 && d.kind == Kind::Other && d.seg[0].K > 0) {
    if (!descriptor_ok(d, 1)) {
      note_error("matrix-vector product M=%d(%d) K=%d(%d) leaves its buffers; not launched", d.M,
                 d.Mi, d.seg[0].K, d.seg[0].Ki);
      return hipErrorIllegalAddress;
    }
    if (g_dry || g_cand == kProbeCand) return hipSuccess;
    hipEvent_t ev[2] = {nullptr, nullptr};
    if (g_profile) {
      if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess)
        return hipErrorOutOfMemory;
      (void)hipEventRecord(ev[0], stream);
    }
    if (d.seg[0].a_kfast) {
      const int per = kGvT / 64;
      hipLaunchKernelGGL(gemv_dots, dim3((unsigned)((d.M + per - 1) / per)), dim3(kGvT), 0, stream,
                         d);
    } else {
      const int rb = d.M >= 32768 ? 64 : (d.M >= 4096 ? 32 : 16);
      hipLaunchKernelGGL(gemv_rows, dim3((unsigned)((d.M + rb - 1) / rb)), dim3(kGvT), 0, stream,
                         d, rb);
    }
    hipError_t err = hipGetLastError();
    if (g_profile) {
      (void)hipEventRecord(ev[1], stream);
      std::string shape;
      if (std::getenv("LNOCC_PROFILE_DUMP")) {
        char buf[160];
        std::snprintf(buf, sizeof(buf), "k%d p%d M%d/%d N1 K%d/%d matrix-vector", (int)d.kind,
                      (int)d.prec, d.M, d.Mi, d.seg[0].K, d.seg[0].Ki);
        shape = buf;
      }
      std::lock_guard<std::mutex> lock(g_records_mu);
      g_records.push_back(Record{d.kind, ev[0], ev[1], 2.0 * d.M * (double)d.seg[0].K, shape});
    }
    return err;
  }
  // Tile shape: the 32 x 32 single-wave tile for thin outputs; otherwise 128
  // rows by the N width (128, 80 or 64) that pads N least.
  int tile = 0;
  if (d.M <= 64 || d.N <= 64) {
    tile = 3;
  } else if (d.kind != Kind::LadderBuild) {   // (the (ac|bd) formation keeps one tile shape)
    int64_t best = -1;
    for (int t : {0, 1, 2}) {
      const int bn = kTileBN[t];
      const int64_t pad = ((int64_t)(d.N + bn - 1) / bn) * bn - d.N;
      if (best < 0 || pad < best) { best = pad; tile = t; }
    }
  }
  const int64_t cap = g_splitk ? (int64_t)(g_splitk_elems / ((size_t)d.M * d.N)) : 0;
  // Split K when the tiles alone leave the chip idle: thin outputs with long K,
  // or a tile count that fills the last round of workgroups poorly.
  auto heuristic_split = [&](int t) {
    const bool sm = t == 3;
    const int bm = kTileBM[t], bn = kTileBN[t], bk = tile_bk(t), slices = tile_slices(t);
    int ns_out = 1;
    const int64_t tiles = (int64_t)((d.M + bm - 1) / bm) * ((d.N + bn - 1) / bn) * d.batch;
    if (d.batch != 1 || cap < 2) return 1;
    if (sm) {
      // single-wave tiles hide latency only by numbers: up to 16 workgroups per
      // CU for outputs of a few tiles with long K (their partial sums are small)
      const bool tiny = (int64_t)d.M * d.N <= 4096;
      const int64_t target = tiny ? 4096 : 2048;
      if (tiles < target && slices >= 8) {
        int64_t want = (target + tiles - 1) / tiles;
        want = std::min<int64_t>({want, (int64_t)slices / 4, cap, tiny ? (int64_t)8192 : 1024});
        if (want >= 2) ns_out = (int)want;
      }
    } else if (slices >= 16 && tiles < 4 * kCUs) {
      // rounds of workgroups x slices per workgroup, plus the partial-sum traffic
      const double t_slice = 2.0 * bm * bn * bk / (45e12 / kCUs);   // s per slice
      double best = -1.0;
      for (int ns = 1; ns <= 64 && ns <= cap && ns * 4 <= slices; ++ns) {
        const int64_t rounds = (tiles * ns + kCUs - 1) / kCUs;
        const double t = rounds * (double)((slices + ns - 1) / ns) * t_slice +
                         (ns > 1 ? 16.0 * ns * d.M * (double)d.N / 4e12 : 0.0);
        if (best < 0 || t < best * 0.98) { best = t; ns_out = ns; }
      }
    }
    return ns_out;
  };
  // the ladder contraction (long K, large output) of the FP32 modes: split products
  if (d.prec == Prec::F32 && d.kind == Kind::LadderContract && tile != 3) tile = kTileSplit;
  // split products take the 4 x 4-staged kernel where the operands allow it
  // (measured: 4096^3 FP32 operands 149 against 100-111 TFLOP/s for the 8-wave
  // tile, FP64 operands 152 against 96, the ladder contraction shape 133 / 125
  // (k- / row-contiguous) against 91 / 108)
  const bool v4 = split_v4_ok(d);
  if (v4 && tile != 3 &&
      (d.prec == Prec::F32S || d.prec == Prec::F64S || tile == kTileSplit))
    tile = kTileSplitV;
  // FP64 with 160 x 160 tiles when the cost model (rounds of one workgroup per
  // CU x slices, plus partial sums) prefers them
  auto model = [&](int t, int ns) {
    const int bm = kTileBM[t], bn = kTileBN[t], sl = tile_slices(t);
    const int64_t tiles = (int64_t)((d.M + bm - 1) / bm) * ((d.N + bn - 1) / bn) * d.batch;
    const double t_slice = 2.0 * bm * bn * tile_bk(t) / (45e12 / kCUs);
    return (double)((tiles * ns + kCUs - 1) / kCUs) * ((sl + ns - 1) / ns) * t_slice +
           (ns > 1 ? 16.0 * ns * d.M * (double)d.N / 4e12 : 0.0);
  };
  if (d.prec == Prec::F64 && tile != 3 && d.M >= 160 && d.N >= 160 &&
      d.kind != Kind::LadderBuild &&
      model(kTileSq160, heuristic_split(kTileSq160)) < 0.95 * model(tile, heuristic_split(tile)))
    tile = kTileSq160;
  if (d.tile_hint > 0 && tile_valid(d.tile_hint - 1, d.prec) &&
      (d.tile_hint - 1 != kTileSplitV || v4))
    tile = d.tile_hint - 1;
  int nsplit = heuristic_split(tile);
  // autotuning: a probe pass only collects keys; a candidate overrides the
  // choice (and is timed); otherwise a stored plan for this shape is used
  std::string key;
  int cand = -1;
  if (!g_dry && d.kind != Kind::LadderBuild && d.tile_hint == 0 &&
      (g_cand >= 0 || g_have_plans.load())) {
    key = plan_key(d);
    if (g_cand == kProbeCand) {
      std::lock_guard<std::mutex> lock(g_plan_mu);
      if (!g_plans.count(key)) ++g_unplanned;
      return hipSuccess;
    }
    // the FP32-only tiles stand in for the heuristic choice in other precisions
    auto set_tile = [&](int t) {
      if (tile_valid(t, d.prec) && (t != kTileSplitV || v4)) tile = t;
    };
    if (g_cand >= 0) {
      cand = g_cand;
      set_tile(cand / kSplitRules);
      const int h = heuristic_split(tile);
      const int rule = cand % kSplitRules;
      nsplit = (rule == 0) ? h : (rule == 1) ? 1 : std::max(2, 2 * h);
      if (d.batch != 1) nsplit = 1;
      nsplit = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)nsplit, cap < 2 ? 1 : cap,
                                                            (int64_t)tile_slices(tile)}));
    } else {
      std::lock_guard<std::mutex> lock(g_plan_mu);
      auto it = g_plans.find(key);
      if (it != g_plans.end()) {
        set_tile(it->second.tile);
        nsplit = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)it->second.nsplit,
                                                              cap < 2 ? 1 : cap,
                                                              (int64_t)tile_slices(tile)}));
        if (d.batch != 1) nsplit = 1;
      }
    }
  }
  const int BMx = kTileBM[tile], BNx = kTileBN[tile];
  const int tiles_m = (d.M + BMx - 1) / BMx, tiles_n = (d.N + BNx - 1) / BNx;
  const int slices = tile_slices(tile);
  const int sps = (slices + nsplit - 1) / nsplit;
  nsplit = (slices + sps - 1) / sps;
  if (nsplit > 1) d.splitk = g_splitk;
  if (!descriptor_ok(d, nsplit)) {
    note_error("contraction M=%d(%d) N=%d(%d) nseg=%d K0=%d(%d) batch=%d split=%d leaves its "
               "buffers; not launched", d.M, d.Mi, d.N, d.Ni, d.nseg, d.seg[0].K, d.seg[0].Ki,
               d.batch, nsplit);
    return hipErrorIllegalAddress;
  }
  if (g_dry) return hipSuccess;

  hipEvent_t ev[2] = {nullptr, nullptr};
  const bool timed = g_profile || cand >= 0;
  if (timed) {
    if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess)
      return hipErrorOutOfMemory;
    (void)hipEventRecord(ev[0], stream);
  }
  dim3 grid((unsigned)(tiles_m * tiles_n), (unsigned)d.batch, (unsigned)nsplit);
  switch (tile) {
    case 1: launch<Big80>(d, grid, tiles_m, sps, stream); break;
    case 2: launch<Big64>(d, grid, tiles_m, sps, stream); break;
    case 3: launch<Small>(d, grid, tiles_m, sps, stream); break;
    case 4: launch_f32<Wide160>(d, grid, tiles_m, sps, stream); break;
    case 5: launch_f32<Tall>(d, grid, tiles_m, sps, stream); break;
    case kTileSq160: launch_f64<Sq160>(d, grid, tiles_m, sps, stream); break;
    case kTileSplit: {
      GemmDesc e = d;
      e.prec = Prec::F32S;
      launch<Big>(e, grid, tiles_m, sps, stream);
      break;
    }
    case kTileSplit160: {
      GemmDesc e = d;
      e.prec = Prec::F32S;
      launch_kind<ModeF32S, Wide160S>(e, grid, tiles_m, sps, stream);
      break;
    }
    case kTileSplitV: {
      GemmDesc e = d;
      if (e.prec == Prec::F32) e.prec = Prec::F32S;
      launch_split_v4(e, grid, tiles_m, sps, stream);
      break;
    }
    default: launch<Big>(d, grid, tiles_m, sps, stream); break;
  }
  hipError_t err = hipGetLastError();
  if (err == hipSuccess && nsplit > 1) {
    const int64_t total = (int64_t)d.M * d.N;
    const int blocks = (int)std::min<int64_t>(4096, (total + 255) / 256);
    if (nsplit > 64)
      hipLaunchKernelGGL(splitk_reduce_wide, dim3((unsigned)((total + kRedOuts - 1) / kRedOuts)),
                         dim3(kRedLanes * kRedOuts), 0, stream, d, nsplit);
    else
      hipLaunchKernelGGL(splitk_reduce, dim3(blocks), dim3(256), 0, stream, d, nsplit);
    err = hipGetLastError();
  }
  if (cand >= 0) {
    (void)hipEventRecord(ev[1], stream);
    g_tune.push_back(TuneRec{key, cand, TilePlan{tile, nsplit}, ev[0], ev[1]});
  } else if (g_profile) {
    (void)hipEventRecord(ev[1], stream);
    double flops = 0.0;
    for (int s = 0; s < d.nseg; ++s) flops += 2.0 * d.M * (double)d.N * d.seg[s].K;
    std::string shape;
    if (std::getenv("LNOCC_PROFILE_DUMP")) {
      char buf[512];
      const GSegment &g = d.seg[0];
      std::snprintf(buf, sizeof(buf),
                    "k%d p%d M%d/%d N%d/%d K%d/%d seg%d b%d | A %lld %lld %lld %lld | B %lld %lld "
                    "%lld %lld | C %lld %lld %lld %lld | tile %dx%d%s split %d",
                    (int)d.kind, (int)d.prec, d.M, d.Mi, d.N, d.Ni, g.K, g.Ki, d.nseg, d.batch,
                    (long long)g.a.s_ro, (long long)g.a.s_ri, (long long)g.a.s_ko,
                    (long long)g.a.s_ki, (long long)g.b.s_ro, (long long)g.b.s_ri,
                    (long long)g.b.s_ko, (long long)g.b.s_ki, (long long)d.c_mo,
                    (long long)d.c_mi, (long long)d.c_no, (long long)d.c_ni, BMx, BNx,
                    (tile == kTileSplit || tile == kTileSplit160) ? " bf16-split"
                    : (tile == kTileSplitV ? " split-v4" : ""), nsplit);
      shape = buf;
    }
    std::lock_guard<std::mutex> lock(g_records_mu);
    // split-bf16 products are timed in a bucket of their own (one arithmetic, one peak)
    const bool split_products = d.prec == Prec::F32S || d.prec == Prec::F64S ||
                                tile == kTileSplit || tile == kTileSplit160 ||
                                tile == kTileSplitV;
    g_records.push_back(Record{split_products ? Kind::Split : d.kind, ev[0], ev[1],
                               flops * d.batch, shape});
  }
  return err;
}

GemmDesc gemm_desc(int M, int N, int K, double alpha,
                   const double *A, int64_t sam, int64_t sak,
                   const double *B, int64_t sbk, int64_t sbn,
                   double beta, double *C, int64_t scm, int64_t scn) {
  GemmDesc d{};
  d.M = M; d.Mi = 1; d.N = N; d.Ni = 1;
  d.nseg = 1;
  GSegment &s = d.seg[0];
  s.a = GOperand{A, sam, 0, sak, 0, 0, 0, 0, 0};
  s.b = GOperand{B, sbn, 0, sbk, 0, 0, 0, 0, 0};
  s.K = K; s.Ki = 1; s.scale = alpha;
  d.c = C; d.c_mo = scm; d.c_mi = 0; d.c_no = scn; d.c_ni = 0;
  d.c_b0 = d.c_b1 = d.c_b2 = d.c_bid = 0;
  d.beta = beta;
  d.batch = 1; d.nb1 = 1; d.table = nullptr;
  d.prec = Prec::F64;
  return d;
}

}  // namespace lnocc

// rp_fit_kernels.h -- HIP kernels of the fitting path, templated on the model
// shape (V variables, numerator and denominator degrees in the code D) so that
// monomials, design rows and accumulators live in registers with static
// indices.  The linearised fit (Section 4.2: A x = b, normal equations) runs
// as separate launches over every fit of a shape bucket:
//   1. the augmented Gram [A b]^T [A b]: in FP64 by weighted moments on the
//      vector units (k_gram_mom_lin), or with the design rows assembled in LDS
//      and contracted on MFMA tiles (k_gram: FP64, FP32 or BF16);
//   2. per fit, equilibration to a unit diagonal and the sweep operator on the
//      register-blocked Gram (k_sweep, one wave per fit; k_big_sweep for
//      models of more than 39 unknowns), unknowns whose pivot vanishes held at
//      zero and the fit flagged;
//   3. refinement against the samples (k_refine_lin, two fits per wave;
//      k_big_refine): iterative refinement in the FP64 form, conjugate
//      gradients preconditioned by the low-precision Gram's inverse in the
//      mixed forms (k_fit for the larger models);
//   4. the minimum-norm re-solve of every flagged fit (k_min_norm).
// The Jacobian Gram of the true loss (k_gram_mom<.., true>) and the
// Levenberg-Marquardt step (k_lm_step) reuse the same pieces.
#pragma once

#include "rp_internal.h"

namespace rp {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

// ---------------------------------------------------------------------------
// precision traits of the Gram contraction
// ---------------------------------------------------------------------------
template <int PREC> struct GramPrec;
template <> struct GramPrec<RP_FP64> {
  using elem = double; using acc = d4;
  static constexpr int K = 4;                   // samples per MFMA
  static constexpr int PAD = 4;
};
template <> struct GramPrec<RP_MIXED_FP32> {
  using elem = float; using acc = f4;
  static constexpr int K = 4;
  static constexpr int PAD = 4;
};
template <> struct GramPrec<RP_MIXED_BF16> {
  using elem = __bf16; using acc = f4;
  static constexpr int K = 32;
  static constexpr int PAD = 8;
};

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

template <typename E> __device__ __forceinline__ E to_elem(double v);
template <> __device__ __forceinline__ double to_elem<double>(double v) { return v; }
template <> __device__ __forceinline__ float to_elem<float>(double v) { return (float)v; }
template <> __device__ __forceinline__ __bf16 to_elem<__bf16>(double v) { return (__bf16)(float)v; }

// Upper-triangular tile pairs (ti <= tj) of an NT x NT tile grid.
template <int NT>
struct TilePairs {
  static constexpr int NP = NT * (NT + 1) / 2;
  int ti[NP];
  int tj[NP];
};
template <int NT>
constexpr TilePairs<NT> make_tile_pairs() {
  TilePairs<NT> P{};
  int p = 0;
  for (int i = 0; i < NT; ++i)
    for (int j = i; j < NT; ++j) { P.ti[p] = i; P.tj[p] = j; ++p; }
  return P;
}

template <int V, int D, int PREC>
struct FitCfg {
  using S = Shape<V, D>;
  using GP = GramPrec<PREC>;
  using E = typename GP::elem;
  static constexpr int NM = S::NM, NA = S::NA, NB = S::NB, NC = S::NC, NU = S::NU;
  static constexpr int NT = (NU + 15) / 16;
  static constexpr int NP = NT * (NT + 1) / 2;
  static constexpr bool PAIR_SPLIT = NP >= 8;
  static constexpr int MPW = PAIR_SPLIT ? (NP + kWaves - 1) / kWaves : NP;
  static constexpr int CH = (PREC == RP_MIXED_BF16) ? 256 : (NT <= 4 ? 128 : 64);
  static constexpr int LDD = CH + GP::PAD;
  static constexpr int DCOLS = NT * 16;
  static constexpr int KS = CH / GP::K;          // k-steps per chunk
  static constexpr int TPS = kThreads / CH;      // threads cooperating on one sample row
  static constexpr size_t D_BYTES = (size_t)DCOLS * LDD * sizeof(E);
  static constexpr size_t G_BYTES = (size_t)NU * (NU + 1) / 2 * sizeof(double);
  static constexpr size_t RAW_BYTES = D_BYTES > G_BYTES ? D_BYTES : G_BYTES;
  static constexpr TilePairs<NT> PAIRS = make_tile_pairs<NT>();
  static_assert(KS % kWaves == 0 || PAIR_SPLIT, "sample split needs KS % waves == 0");
};

__device__ __forceinline__ int pk(int i, int j) { return i * (i + 1) / 2 + j; }   // j <= i

// LDS pointers for the buffer loads that write LDS.
typedef __attribute__((address_space(3))) void* lds_void_ptr;

// Wait until at most N vector memory operations of this wave are in flight
// (the loads that write LDS are not tracked by the compiler).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

// ---------------------------------------------------------------------------
// block-wide helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

// Sum of one value per thread; every thread gets the result.
__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kWaves; ++k) s += red[k];
  __syncthreads();
  return s;
}

__device__ double block_max(double v, double* red) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = red[0];
#pragma unroll
  for (int k = 1; k < kWaves; ++k) s = fmax(s, red[k]);
  __syncthreads();
  return s;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lane swaps of a double between halves and rows of the wave (gfx950):
// swap32(a, b) leaves a's lanes 0-31 and b's lanes 0-31 in x (lanes 0-31,
// 32-63) and a's and b's lanes 32-63 in y; swap16 does the same with the odd
// 16-lane rows of a and the even rows of b.
__device__ __forceinline__ double swap32_add(double a, double b) {
  const uint64_t ua = __builtin_bit_cast(uint64_t, a), ub = __builtin_bit_cast(uint64_t, b);
  const auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)ua, (uint32_t)ub, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(ua >> 32), (uint32_t)(ub >> 32), false, false);
  const double x = __builtin_bit_cast(double, ((uint64_t)hi[0] << 32) | lo[0]);
  const double y = __builtin_bit_cast(double, ((uint64_t)hi[1] << 32) | lo[1]);
  return x + y;
}
__device__ __forceinline__ double swap16_add(double a, double b) {
  const uint64_t ua = __builtin_bit_cast(uint64_t, a), ub = __builtin_bit_cast(uint64_t, b);
  const auto lo = __builtin_amdgcn_permlane16_swap((uint32_t)ua, (uint32_t)ub, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((uint32_t)(ua >> 32), (uint32_t)(ub >> 32), false, false);
  const double x = __builtin_bit_cast(double, ((uint64_t)hi[0] << 32) | lo[0]);
  const double y = __builtin_bit_cast(double, ((uint64_t)hi[1] << 32) | lo[1]);
  return x + y;
}

// out[j] = sum over the wave's 64 lanes of acc[j], j < NC.  A swap of wave
// halves adds lanes l and l + 32 of two values at once (lanes 0-31 keep the
// first value's sums, lanes 32-63 the second's); a swap of 16-lane rows then
// does the same for lanes l and l + 16, so each lane holds a quarter of the
// values, each 16-lane row of value u standing for accumulator
// 4u + {0, 2, 1, 3}[row].  The 16 partials of every accumulator meet in LDS
// (row stride 66 doubles: the 16 lanes of a row read 16 different bank
// groups) and one lane adds them.  red: (NC + 3) / 4 * 66 doubles.
template <int NC>
__device__ __forceinline__ void wave_reduce_vec(const double (&acc)[NC], double* out, double* red) {
  constexpr int N4 = (NC + 3) / 4 * 4;
  constexpr int NQ = N4 / 4;
  constexpr int S = 66;
  const int lane = threadIdx.x & 63;
  double r[N4 / 2];
#pragma unroll
  for (int t = 0; t < N4 / 2; ++t)
    r[t] = swap32_add(2 * t < NC ? acc[2 * t] : 0.0, 2 * t + 1 < NC ? acc[2 * t + 1] : 0.0);
#pragma unroll
  for (int u = 0; u < NQ; ++u) red[u * S + lane] = swap16_add(r[2 * u], r[2 * u + 1]);
  wave_sync();
  const int g = lane >> 4;
  const int col = (g == 1 ? 2 : g == 2 ? 1 : g);
#pragma unroll
  for (int u0 = 0; u0 < NQ; u0 += 16) {
    const int u = u0 + (lane & 15);
    if (u < NQ) {
      const double* p = red + u * S + 16 * g;
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int i = 0; i < 16; i += 2) {
        s0 += p[i];
        s1 += p[i + 1];
      }
      const int j = 4 * u + col;
      if (j < NC) out[j] = s0 + s1;
    }
  }
  wave_sync();
}


// ---------------------------------------------------------------------------
// per-fit state in LDS
// ---------------------------------------------------------------------------
template <int NC>
struct FitShared {
  double c[NC];       // current coefficients (unscaled)
  double r[NC];       // normal-equation residual / right-hand sides
  double z[NC];
  double p[NC];
  double q[NC];
  double dsc[NC + 1]; // column scales 1/sqrt(G_jj) (last = 1 for the rhs column)
  double red[kWaves * NC];
  // per-wave transposition scratch of the passes' lane reductions
  static constexpr int WRED = ((NC < kPassGroupMax ? NC : kPassGroupMax) + 3) / 4 * 66;
  double wred[kWaves * WRED];
  double tmp[kWaves];
  int drop[NC];       // 1 = pivot vanished, coefficient held at zero
  int flag_nonfinite;
  int n_drop;
};

// Row of the design for one sample: the linearised problem uses weight 1,
// z = y and b = y; a Gauss-Newton step on the true loss uses weight 1/Q,
// z = f = N/Q and b = y - f (Jacobian rows), all evaluated at coefficients c.
template <int V, int D, bool GN>
struct RowGen {
  using S = Shape<V, D>;
  double m[S::NM];
  double w, zz, b;
  bool ok;
  __device__ __forceinline__ void load(const double* x, int64_t ldx, const double* y, int64_t s,
                                       bool valid, const double* c) {
    double u[V];
    double yy = 0.0;
    ok = true;
    if (valid) {
#pragma unroll
      for (int k = 0; k < V; ++k) u[k] = x[(int64_t)k * ldx + s];
      yy = y[s];
#pragma unroll
      for (int k = 0; k < V; ++k) ok = ok && isfinite(u[k]);
      ok = ok && isfinite(yy);
    } else {
#pragma unroll
      for (int k = 0; k < V; ++k) u[k] = 0.0;
    }
    monomials<V, D, double>(u, m);
    if constexpr (!GN) {
      w = valid ? 1.0 : 0.0;
      zz = yy;
      b = valid ? yy : 0.0;
    } else {
      double N = 0.0, Q = 1.0;
#pragma unroll
      for (int j = 0; j < S::NA; ++j) N = fma(c[j], m[j], N);
#pragma unroll
      for (int j = 1; j < S::NQ; ++j) Q = fma(c[S::NA + j - 1], m[j], Q);
      const double f = N / Q;
      w = valid ? 1.0 / Q : 0.0;
      zz = f;
      b = valid ? yy - f : 0.0;
    }
  }
  // column c of the augmented row [A | b]
  template <int C>
  __device__ __forceinline__ double col() const {
    if constexpr (C < S::NA) return w * m[C];
    else if constexpr (C < S::NC) return -(w * zz) * m[C - S::NA + 1];
    else if constexpr (C == S::NC) return b;
    else return 0.0;
  }
};

// ---------------------------------------------------------------------------
// Gram: chunks of design columns in LDS, contracted on MFMA
// ---------------------------------------------------------------------------
template <int V, int D, int PREC, bool GN, int... Cs>
__device__ __forceinline__ void write_row_cols(typename FitCfg<V, D, PREC>::E* Dm, int s,
                                               const RowGen<V, D, GN>& row, int lo, int hi,
                                               std::integer_sequence<int, Cs...>) {
  using Cfg = FitCfg<V, D, PREC>;
  using E = typename Cfg::E;
  ((Cs >= lo && Cs < hi ? (void)(Dm[Cs * Cfg::LDD + s] = to_elem<E>(row.template col<Cs>())) : (void)0), ...);
}

template <int V, int D, int PREC, int W>
__device__ __forceinline__ void gram_pair_split(typename FitCfg<V, D, PREC>::E* Dm,
                                                typename GramPrec<PREC>::acc* acc, int lane) {
  using Cfg = FitCfg<V, D, PREC>;
  using GP = GramPrec<PREC>;
  constexpr auto P = Cfg::PAIRS;
  for (int ks = 0; ks < Cfg::KS; ++ks) {
    if constexpr (PREC == RP_MIXED_BF16) {
      bf8 a[Cfg::NT];
#pragma unroll
      for (int t = 0; t < Cfg::NT; ++t)
        a[t] = *reinterpret_cast<const bf8*>(&Dm[(16 * t + (lane & 15)) * Cfg::LDD + ks * GP::K + 8 * (lane >> 4)]);
#pragma unroll
      for (int q = 0; q < Cfg::MPW; ++q) {
        const int p = W + kWaves * q;
        if (p < Cfg::NP) acc[q] = mfma(a[P.ti[p]], a[P.tj[p]], acc[q]);
      }
    } else {
      typename Cfg::E a[Cfg::NT];
#pragma unroll
      for (int t = 0; t < Cfg::NT; ++t)
        a[t] = Dm[(16 * t + (lane & 15)) * Cfg::LDD + ks * GP::K + (lane >> 4)];
#pragma unroll
      for (int q = 0; q < Cfg::MPW; ++q) {
        const int p = W + kWaves * q;
        if (p < Cfg::NP) acc[q] = mfma(a[P.ti[p]], a[P.tj[p]], acc[q]);
      }
    }
  }
}

// Accumulate [A b]^T [A b] of fit samples [s0, s0+m) into the packed lower
// triangle G (aliasing the design buffer).  c: coefficients for GN rows.
template <int V, int D, int PREC, bool GN>
__device__ void gram(const FitArgs& a, int64_t s0, int64_t m, unsigned char* raw, double* G,
                     FitShared<Shape<V, D>::NC>& sh, const double* c) {
  using Cfg = FitCfg<V, D, PREC>;
  using GP = GramPrec<PREC>;
  using E = typename Cfg::E;
  using Acc = typename GP::acc;
  E* Dm = reinterpret_cast<E*>(raw);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr auto P = Cfg::PAIRS;

  Acc acc[Cfg::MPW];
#pragma unroll
  for (int q = 0; q < Cfg::MPW; ++q) acc[q] = Acc{0, 0, 0, 0};

  const int srow = tid % Cfg::CH;                 // sample within the chunk
  const int part = tid / Cfg::CH;                 // wave-uniform column share
  const int lo = part * Cfg::DCOLS / Cfg::TPS;
  const int hi = (part + 1) * Cfg::DCOLS / Cfg::TPS;
  bool bad = false;

  for (int64_t c0 = 0; c0 < m; c0 += Cfg::CH) {
    {
      const bool valid = c0 + srow < m;
      RowGen<V, D, GN> row;
      row.load(a.x, a.ldx, a.y, s0 + c0 + srow, valid, c);
      bad = bad || !row.ok;
      write_row_cols<V, D, PREC, GN>(Dm, srow, row, lo, hi, std::make_integer_sequence<int, Cfg::DCOLS>{});
    }
    __syncthreads();
    if constexpr (!Cfg::PAIR_SPLIT) {
      for (int ks = wave; ks < Cfg::KS; ks += kWaves) {
        if constexpr (PREC == RP_MIXED_BF16) {
          bf8 av[Cfg::NT];
#pragma unroll
          for (int t = 0; t < Cfg::NT; ++t)
            av[t] = *reinterpret_cast<const bf8*>(&Dm[(16 * t + (lane & 15)) * Cfg::LDD + ks * GP::K + 8 * (lane >> 4)]);
#pragma unroll
          for (int p = 0; p < Cfg::NP; ++p) acc[p] = mfma(av[P.ti[p]], av[P.tj[p]], acc[p]);
        } else {
          E av[Cfg::NT];
#pragma unroll
          for (int t = 0; t < Cfg::NT; ++t)
            av[t] = Dm[(16 * t + (lane & 15)) * Cfg::LDD + ks * GP::K + (lane >> 4)];
#pragma unroll
          for (int p = 0; p < Cfg::NP; ++p) acc[p] = mfma(av[P.ti[p]], av[P.tj[p]], acc[p]);
        }
      }
    } else {
      switch (wave) {
        case 0: gram_pair_split<V, D, PREC, 0>(Dm, acc, lane); break;
        case 1: gram_pair_split<V, D, PREC, 1>(Dm, acc, lane); break;
        case 2: gram_pair_split<V, D, PREC, 2>(Dm, acc, lane); break;
        default: gram_pair_split<V, D, PREC, 3>(Dm, acc, lane); break;
      }
    }
    __syncthreads();
  }
  if (bad) atomicOr(&sh.flag_nonfinite, 1);

  // MFMA result layout (column lane%16 of the tile in every case): the FP32
  // accumulating forms hold rows 4*(lane/16)+r, the FP64 form rows lane/16+4r.
  auto store = [&](int p, const Acc& v, bool add) {
    const int ti = P.ti[p], tj = P.tj[p];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * ti + (PREC == RP_FP64 ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r);
      const int col = 16 * tj + (lane & 15);
      if (row < Cfg::NU && col < Cfg::NU && col >= row) {
        const double val = (double)v[r];
        if (add) G[pk(col, row)] += val; else G[pk(col, row)] = val;
      }
    }
  };
  if constexpr (!Cfg::PAIR_SPLIT) {
    for (int w = 0; w < kWaves; ++w) {
      if (wave == w) {
#pragma unroll
        for (int p = 0; p < Cfg::NP; ++p) store(p, acc[p], w > 0);
      }
      __syncthreads();
    }
  } else {
#pragma unroll
    for (int q = 0; q < Cfg::MPW; ++q) {
      const int p = wave + kWaves * q;
      if (p < Cfg::NP) store(p, acc[q], false);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// equilibration, Cholesky and solves on the packed Gram
// ---------------------------------------------------------------------------

// 1/d for finite d > 0: the hardware estimate refined by two Newton-Raphson
// steps x <- x + x (1 - d x), each of which squares the relative error.
__device__ __forceinline__ double rcp_nr(double d) {
  double x = __builtin_amdgcn_rcp(d);
  double e = fma(-d, x, 1.0);
  x = fma(x, e, x);
  e = fma(-d, x, 1.0);
  return fma(x, e, x);
}

// A value that is equal on every lane, moved to scalar registers so that
// branches on it are uniform.
__device__ __forceinline__ double uniform_d(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)b);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Equilibration factor of an unknown whose Gram diagonal is gii: 1/sqrt(gii),
// so that the scaled diagonal is 1 (to rounding).  A sweep pivot of the
// scaled matrix is then the squared distance of the unknown's design column
// from the span of the columns swept before it, relative to its squared
// norm, and the drop rule compares it with a constant.
__device__ __forceinline__ double eq_scale(double gii) {
  return (gii > 0.0 && isfinite(gii)) ? 1.0 / sqrt(gii) : 1.0;
}

// Scale rows/columns j < NC by d_j = eq_scale(G_jj), keep the rhs column
// unscaled, then add `shift` to the scaled diagonal and multiply it by
// (1 + lambda).
template <int NC>
__device__ void equilibrate(double* G, FitShared<NC>& sh, double shift, double lambda) {
  const int tid = threadIdx.x;
  constexpr int NU = NC + 1;
  for (int j = tid; j < NU; j += kThreads) {
    double d = 1.0;
    if (j < NC) {
      d = eq_scale(G[pk(j, j)]);
    }
    sh.dsc[j] = d;
  }
  __syncthreads();
  constexpr int NPK = NU * (NU + 1) / 2;
  for (int e = tid; e < NPK; e += kThreads) {
    int i = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
    while (i * (i + 1) / 2 > e) --i;
    while ((i + 1) * (i + 2) / 2 <= e) ++i;
    const int j = e - i * (i + 1) / 2;
    double v = G[e] * sh.dsc[i] * sh.dsc[j];
    if (i == j && i < NC) v = v * (1.0 + lambda) + shift;
    G[e] = v;
  }
  __syncthreads();
}

// In-place lower Cholesky of the leading NC x NC block.  A pivot <= tau marks
// the column as dropped (its coefficient is held at zero).  Returns the number
// of dropped columns (block-uniform).
template <int NC>
__device__ int cholesky(double* G, FitShared<NC>& sh, double tau) {
  const int tid = threadIdx.x;
  if (tid == 0) sh.n_drop = 0;
  for (int j = tid; j < NC; j += kThreads) sh.drop[j] = 0;
  __syncthreads();
  for (int k = 0; k < NC; ++k) {
    const double piv = G[pk(k, k)];
    const bool dropped = !(piv > tau);
    const double lkk = dropped ? 1.0 : sqrt(piv);
    const double inv = dropped ? 0.0 : 1.0 / lkk;
    __syncthreads();
    if (tid == 0) {
      G[pk(k, k)] = lkk;
      if (dropped) { sh.drop[k] = 1; sh.n_drop += 1; }
    }
    for (int i = k + 1 + tid; i < NC; i += kThreads) G[pk(i, k)] *= inv;
    __syncthreads();
    // trailing update: rows i > k spread over 32 groups of 8 threads
    const int grp = tid >> 3, sub = tid & 7;
    for (int i = k + 1 + grp; i < NC; i += kThreads / 8) {
      const double lik = G[pk(i, k)];
      for (int j = k + 1 + sub; j <= i; j += 8) G[pk(i, j)] -= lik * G[pk(j, k)];
    }
    __syncthreads();
  }
  return sh.n_drop;
}

// x = (L L^T)^-1 b on the scaled system (wave 0; rows spread over lanes).
// Dropped pivots give zero components.  b and x may alias.
template <int NC>
__device__ void chol_solve(const double* G, const FitShared<NC>& sh, const double* b, double* x) {
  constexpr int R = (NC + 63) / 64;
  const int tid = threadIdx.x;
  __syncthreads();
  if (tid < 64) {
    double z[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = tid + 64 * r;
      z[r] = i < NC ? b[i] : 0.0;
    }
    auto pick = [&](int k) {
      double o = z[0];
#pragma unroll
      for (int r = 1; r < R; ++r) if (k >= 64 * r) o = z[r];
      return o;
    };
    for (int k = 0; k < NC; ++k) {                    // forward: L y = b
      const double own = pick(k);
      double zk = __shfl(own, k % 64, 64);
      zk = sh.drop[k] ? 0.0 : zk / G[pk(k, k)];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = tid + 64 * r;
        if (i == k) z[r] = zk;
        else if (i > k && i < NC) z[r] -= G[pk(i, k)] * zk;
      }
    }
    for (int k = NC - 1; k >= 0; --k) {               // backward: L^T x = y
      const double own = pick(k);
      double xk = __shfl(own, k % 64, 64);
      xk = sh.drop[k] ? 0.0 : xk / G[pk(k, k)];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = tid + 64 * r;
        if (i == k) z[r] = xk;
        else if (i < k) z[r] -= G[pk(k, i)] * xk;
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = tid + 64 * r;
      if (i < NC) x[i] = z[r];
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// FP64 passes over the samples (thread per sample, registers only)
// ---------------------------------------------------------------------------
enum PassMode { PASS_RESIDUAL = 0, PASS_PRODUCT = 1, PASS_CHECK = 2 };

// RESIDUAL: w_i = b_i - a_i.v,  out = A^T w, returns sum w^2
// PRODUCT:  w_i = a_i.v,        out = A^T w
// CHECK:    w_i = b_i - a_i.v,  returns sum w^2; *qmin = min_i Q_v(u_i)
// Accumulators per thread of one sample sweep: above this the unknowns are
// split into groups, each swept over the samples on its own (the monomials
// and the residual are formed again per group), so that accumulators and
// monomials stay in registers instead of spilling to scratch.

// One sample's inputs.
template <int V>
struct SampleIn {
  double u[V];
  double y;
};

// ---------------------------------------------------------------------------
// N(u) and Q(u) by nested multiplication (multivariate Horner)
// ---------------------------------------------------------------------------
// hpoly<.., K, E0..E3, REM> is the sum of c_e u^e over the exponents e whose
// first K entries are E0.. and whose other entries total at most REM, nested
// in the powers of u_K: the part with e_K = REM, times u_K, plus the part
// with e_K = REM - 1, and so on.  A polynomial of n monomials costs n - 1
// FMAs and no monomial is formed.  DEN: the denominator (its constant term
// is 1, its other coefficients follow the numerator's).
template <int V, int D>
constexpr int mono_rank(int e0, int e1, int e2, int e3) {
  const auto& T = Mono<V, D>::T;
  for (int j = 0; j < T.n; ++j)
    if (T.e[j][0] == e0 && T.e[j][1] == e1 && T.e[j][2] == e2 && T.e[j][3] == e3) return j;
  return -1;
}

template <int V, int D, bool DEN, int K, int E0, int E1, int E2, int E3, int REM, class CF>
__device__ __forceinline__ double hpoly(const double* u, const CF& c);

template <int V, int D, bool DEN, int K, int E0, int E1, int E2, int E3, int REM, int A, class CF>
__device__ __forceinline__ double hloop(const double* u, const CF& c, double acc) {
  const double t = fma(acc, u[K],
                       hpoly<V, D, DEN, K + 1, K == 0 ? A : E0, K == 1 ? A : E1, K == 2 ? A : E2,
                             K == 3 ? A : E3, REM - A>(u, c));
  if constexpr (A == 0) return t;
  else return hloop<V, D, DEN, K, E0, E1, E2, E3, REM, A - 1>(u, c, t);
}

template <int V, int D, bool DEN, int K, int E0, int E1, int E2, int E3, int REM, class CF>
__device__ __forceinline__ double hpoly(const double* u, const CF& c) {
  if constexpr (K == V) {
    constexpr int j = mono_rank<V, D>(E0, E1, E2, E3);
    static_assert(j >= 0, "exponent in the table");
    if constexpr (DEN && j == 0) return 1.0;
    else return c(DEN ? Shape<V, D>::NA + j - 1 : j);
  } else if constexpr (REM == 0) {
    return hpoly<V, D, DEN, K + 1, E0, E1, E2, E3, 0>(u, c);
  } else {
    const double top = hpoly<V, D, DEN, K + 1, K == 0 ? REM : E0, K == 1 ? REM : E1,
                             K == 2 ? REM : E2, K == 3 ? REM : E3, 0>(u, c);
    return hloop<V, D, DEN, K, E0, E1, E2, E3, REM, REM - 1>(u, c, top);
  }
}

// N(u) and Q(u) of the coefficients c(j) (numerator first, then the
// denominator's without its constant term)
template <int V, int D, class CF>
__device__ __forceinline__ void horner_nq(const double* u, const CF& c, double& n, double& q) {
  n = hpoly<V, D, false, 0, 0, 0, 0, 0, code_dn(D)>(u, c);
  q = hpoly<V, D, true, 0, 0, 0, 0, 0, code_dq(D)>(u, c);
}

// Inputs of one fit's samples as uniform byte bases plus a 32-bit byte offset
// per lane (fits hold fewer than 2^28 samples), so the loads take the
// scalar-base addressing form and no 64-bit address per load stays live.
template <int V>
struct SampleSrc {
  const char* x[V];
  const char* y;
  uint32_t m;
  __device__ __forceinline__ SampleSrc(const FitArgs& a, int64_t s0, int64_t n) {
#pragma unroll
    for (int k = 0; k < V; ++k) x[k] = reinterpret_cast<const char*>(a.x + (int64_t)k * a.ldx + s0);
    y = reinterpret_cast<const char*>(a.y + s0);
    m = (uint32_t)n;
  }
  // Branch-free: an index past the end reads the last sample (m >= 1), which
  // the caller masks out.
  __device__ __forceinline__ void load(SampleIn<V>& t, uint32_t i) const {
    const uint32_t off = (i < m ? i : m - 1u) * 8u;
#pragma unroll
    for (int k = 0; k < V; ++k) t.u[k] = *reinterpret_cast<const double*>(x[k] + off);
    t.y = *reinterpret_cast<const double*>(y + off);
  }
};

// RESIDUAL / PRODUCT pass over the samples for unknowns [J0, J1): partial
// sums of w a_ij per wave into red[wave * NC + j]; the first group also
// returns sum w^2.  With wres (the fit's slice of the residual scratch) the
// first group stores each sample's w and the later ones (REUSE) read it back
// instead of forming N and Q again (a thread takes the same samples in every
// group, so it reads its own stores).
template <int V, int D, int MODE, int J0, int J1, bool VLDS, bool REUSE>
__device__ double pass_group_loop(const FitArgs& a, int64_t s0, int64_t m, const double* v, double* red,
                                  double* wred, double* wres) {
  using S = Shape<V, D>;
  const int tid = threadIdx.x;
  double acc[J1 - J0];
#pragma unroll
  for (int j = 0; j < J1 - J0; ++j) acc[j] = 0.0;
  double ss = 0.0;
  // the next sample's inputs (and stored residual) are in flight while this
  // one is processed
  const SampleSrc<V> src(a, s0, m);
  SampleIn<V> nx;
  double wn = 0.0;
  if (m > 0) {
    src.load(nx, tid);
    if constexpr (REUSE) wn = wres[tid < m ? tid : m - 1];
  }
  for (int64_t i = tid; i < m; i += kThreads) {
    const SampleIn<V> cur = nx;
    const int64_t inx = i + kThreads < m ? i + kThreads : m - 1;
    double w;
    if constexpr (REUSE) {
      w = wn;
      wn = wres[inx];
    }
    src.load(nx, (uint32_t)inx);
    const double y = cur.y;
    double mo[S::NM];
    monomials<V, D, double>(cur.u, mo);
    if constexpr (!REUSE) {
      int zero = 0;
      if constexpr (VLDS) asm volatile("v_mov_b32 %0, 0" : "=v"(zero));
      const double* vz = v + zero;
      double nv = 0.0, qv = 0.0;
#pragma unroll
      for (int j = 0; j < S::NA; ++j) nv = fma(vz[j], mo[j], nv);
#pragma unroll
      for (int j = 1; j < S::NQ; ++j) qv = fma(vz[S::NA + j - 1], mo[j], qv);
      const double dot = fma(-y, qv, nv);
      w = (MODE == PASS_PRODUCT) ? dot : y - dot;
      if (J0 == 0 && wres) wres[i] = w;
    }
    if constexpr (J0 == 0) ss = fma(w, w, ss);
    const double wy = -y * w;
#pragma unroll
    for (int j = J0; j < J1; ++j)
      acc[j - J0] = j < S::NA ? fma(w, mo[j < S::NA ? j : 0], acc[j - J0])
                              : fma(wy, mo[j < S::NA ? 0 : j - S::NA + 1], acc[j - J0]);
  }
  const int wave = tid >> 6;
  wave_reduce_vec<J1 - J0>(acc, red + wave * S::NC + J0, wred + wave * FitShared<S::NC>::WRED);
  return ss;
}

template <int V, int D, int MODE, int J0, int J1, bool VLDS>
__device__ double pass_group(const FitArgs& a, int64_t s0, int64_t m, const double* v, double* red,
                             double* wred, double* wres) {
  if constexpr (J0 > 0) {
    if (wres) return pass_group_loop<V, D, MODE, J0, J1, VLDS, true>(a, s0, m, v, red, wred, wres);
  }
  return pass_group_loop<V, D, MODE, J0, J1, VLDS, false>(a, s0, m, v, red, wred, wres);
}

template <int V, int D, int MODE, int GS, bool VLDS, int... G>
__device__ __forceinline__ double pass_groups(const FitArgs& a, int64_t s0, int64_t m, const double* v,
                                              double* red, double* wred, std::integer_sequence<int, G...>) {
  constexpr int NC = Shape<V, D>::NC;
  double* wres = a.wres ? a.wres + s0 : nullptr;
  double ss = 0.0;
  ((ss += pass_group<V, D, MODE, G * GS, ((G + 1) * GS < NC ? (G + 1) * GS : NC), VLDS>(a, s0, m, v, red,
                                                                                         wred, wres)), ...);
  return ss;
}

// VLDS: v is read from LDS where it is used (an opaque offset keeps the
// compiler from holding all of it in registers across the sample loop): for
// kernels that run two workgroups per compute unit in at most 256 VGPRs.
template <int V, int D, int MODE, bool VLDS = false>
__device__ double pass(const FitArgs& a, int64_t s0, int64_t m, const double* v, double* out,
                       FitShared<Shape<V, D>::NC>& sh, double* qmin) {
  using S = Shape<V, D>;
  const int tid = threadIdx.x;
  if constexpr (MODE != PASS_CHECK && S::NC > kPassGroupMax) {
    constexpr int NG = (S::NC + kPassGroupMax - 1) / kPassGroupMax;
    constexpr int GS = (S::NC + NG - 1) / NG;
    double ss = pass_groups<V, D, MODE, GS, VLDS>(a, s0, m, v, sh.red, sh.wred,
                                                  std::make_integer_sequence<int, NG>{});
    ss = block_sum(ss, sh.tmp);   // its barriers also publish the partials
    for (int j = tid; j < S::NC; j += kThreads) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < kWaves; ++w) t += sh.red[w * S::NC + j];
      out[j] = t;
    }
    __syncthreads();
    return ss;
  }
  double acc[S::NC];
#pragma unroll
  for (int j = 0; j < S::NC; ++j) acc[j] = 0.0;
  double ss = 0.0, qm = INFINITY;
  const SampleSrc<V> src(a, s0, m);
  SampleIn<V> nx;
  if (m > 0) src.load(nx, tid);
  for (int64_t i = tid; i < m; i += kThreads) {
    const SampleIn<V> cur = nx;
    src.load(nx, (uint32_t)(i + kThreads));   // clamped past the end
    const double y = cur.y;
    double mo[S::NM];
    monomials<V, D, double>(cur.u, mo);
    int zero = 0;
    if constexpr (VLDS) asm volatile("v_mov_b32 %0, 0" : "=v"(zero));
    const double* vz = v + zero;
    double nv = 0.0, qv = 0.0;
#pragma unroll
    for (int j = 0; j < S::NA; ++j) nv = fma(vz[j], mo[j], nv);
#pragma unroll
    for (int j = 1; j < S::NQ; ++j) qv = fma(vz[S::NA + j - 1], mo[j], qv);
    const double dot = fma(-y, qv, nv);                 // a_i . v
    const double w = (MODE == PASS_PRODUCT) ? dot : y - dot;
    ss = fma(w, w, ss);
    if constexpr (MODE == PASS_CHECK) qm = fmin(qm, 1.0 + qv);
    if constexpr (MODE != PASS_CHECK) {
      const double wy = -y * w;
#pragma unroll
      for (int j = 0; j < S::NA; ++j) acc[j] = fma(w, mo[j], acc[j]);
#pragma unroll
      for (int j = 1; j < S::NQ; ++j) acc[S::NA + j - 1] = fma(wy, mo[j], acc[S::NA + j - 1]);
    }
  }
  const int wave = tid >> 6;
  if constexpr (MODE != PASS_CHECK)
    wave_reduce_vec<S::NC>(acc, sh.red + wave * S::NC, sh.wred + wave * FitShared<S::NC>::WRED);
  ss = block_sum(ss, sh.tmp);
  if constexpr (MODE == PASS_CHECK) {
    qm = -block_max(-qm, sh.tmp);
    *qmin = qm;
  } else {
    for (int j = tid; j < S::NC; j += kThreads) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < kWaves; ++w) t += sh.red[w * S::NC + j];
      out[j] = t;
    }
  }
  __syncthreads();
  return ss;
}

template <int NC>
__device__ double dot_nc(const double* a, const double* b, FitShared<NC>& sh) {
  double t = 0.0;
  for (int j = threadIdx.x; j < NC; j += kThreads) t = fma(a[j], b[j], t);
  return block_sum(t, sh.tmp);
}

template <int NC>
__device__ double maxabs_nc(const double* a, FitShared<NC>& sh) {
  double t = 0.0;
  for (int j = threadIdx.x; j < NC; j += kThreads) t = fmax(t, fabs(a[j]));
  return block_max(t, sh.tmp);
}

// Early stop of the mixed forms' preconditioned CG: after four iterations,
// the observed geometric rate of the corrections (smallest so far over the
// first) projected to the iteration cap.  If even that projection misses the
// convergence bar sqrt(tol) * max|c| by more than a factor of ten, the
// low-precision Gram is too poor a preconditioner for this fit: stop now
// (the fit ends RP_FIT_NOT_CONVERGED and the FP64 re-solve takes it) instead
// of spending the remaining passes.  A NaN stops as well.
__device__ __forceinline__ bool pcg_hopeless(int it, int cap, double dn, double cn, double tol,
                                             double& dn1, double& dnmin) {
  if (it == 1) dn1 = dn;
  dnmin = fmin(dnmin, dn);
  if (it < 4) return false;
  // in base-2 logarithms, single precision (a heuristic needs no more)
  const float l1 = __builtin_amdgcn_logf((float)dn1), lm = __builtin_amdgcn_logf((float)dnmin);
  const float lr = (lm - l1) / (float)(it - 1);
  if (!(lr < 0.0f)) return true;
  return lm + lr * (float)(cap - it) > __builtin_amdgcn_logf((float)(10.0 * sqrt(tol) * cn));
}

// Put fit f on its bucket's FP64 re-solve list when its status asks for it
// (rank deficient or underdetermined: the minimum-norm solve; refinement at
// its cap: the FP64 fall-back).  One thread per fit.
__device__ __forceinline__ void flag_for_resolve(const FitArgs& a, int f, int st) {
  if (a.resolve && (st == RP_FIT_RANK_DEFICIENT || st == RP_FIT_UNDERDETERMINED ||
                    st == RP_FIT_NOT_CONVERGED))
    a.resolve[2 + atomicAdd(a.resolve, 1)] = f;
}

// ---------------------------------------------------------------------------
// sweep of the larger models by the whole workgroup
// ---------------------------------------------------------------------------
// The sweep operator (see the wave form below) on the augmented (NC+1)^2
// matrix, zero-padded to 16 SB x 16 SB and split into a 16 x 16 grid of SB x SB
// blocks: thread t of the 256 holds block (t / 16, t % 16) in registers for the
// whole sweep.  Per pivot K the sixteen threads of its block column publish
// column K to LDS (two buffers, alternating, so one barrier per pivot
// suffices); every thread then updates its block with SB^2 FMAs.  The pivot
// loop is unrolled at compile time (static block indices).  Equilibration to
// a unit diagonal is applied as the blocks are loaded; a pivot at or below
// tau is dropped (its row and column are held at zero) and marked in drop[]
// (the pivot is the squared distance of the unknown's design column from the
// span of the columns kept before it, relative to its squared norm).
// colbuf (LDS, CB doubles): the two alternating pivot columns.
template <int NC>
struct BigBlocks {
  static constexpr int NU = NC + 1;
  static constexpr int GRID = 16;
  static constexpr int SB = (NU + GRID - 1) / GRID;
  static constexpr int NP = GRID * SB;
  static constexpr int CB = 2 * NP;
  double b[SB][SB];
  double sr[SB], sc[SB];   // equilibration factors of the block's rows / columns
  int bi, bj;
};

// Load the packed lower augmented Gram gs, equilibrated, with the unknowns'
// diagonal mapped to g + dadd (the mixed forms' positive shift).  scale (LDS,
// NC doubles) receives the equilibration factors, each formed once by one
// thread (a barrier inside: every thread of the workgroup calls this).
template <int NC>
__device__ __forceinline__ void big_load(const double* gs, BigBlocks<NC>& B, double* scale,
                                         double dadd = 0.0) {
  constexpr int SB = BigBlocks<NC>::SB, NU = BigBlocks<NC>::NU;
  B.bi = threadIdx.x >> 4;
  B.bj = threadIdx.x & 15;
  for (int j = threadIdx.x; j < NC; j += kThreads) scale[j] = eq_scale(gs[pk(j, j)]);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < SB; ++r) {
    const int i = B.bi * SB + r;
    B.sr[r] = i < NC ? scale[i] : 1.0;
    const int j = B.bj * SB + r;
    B.sc[r] = j < NC ? scale[j] : 1.0;
  }
#pragma unroll
  for (int r = 0; r < SB; ++r) {
#pragma unroll
    for (int c = 0; c < SB; ++c) {
      const int i = B.bi * SB + r, j = B.bj * SB + c;
      double v = (i < NU && j < NU) ? gs[i >= j ? pk(i, j) : pk(j, i)] * B.sr[r] * B.sc[c] : 0.0;
      if (i == j && i < NC) v += dadd;
      B.b[r][c] = v;
    }
  }
}

// Pivot K = KB * SB + KR: the block row / column KB is a run-time value, the
// position KR inside the block a compile-time one (register indices stay
// static while the code holds one block row of pivots, not all of them).
template <int NC, int KR>
__device__ __forceinline__ void big_pivot(BigBlocks<NC>& B, double* colbuf, double tau, int* drop,
                                          int& ndrop, int KB) {
  constexpr int SB = BigBlocks<NC>::SB, NP = BigBlocks<NC>::NP;
  const int K = KB * SB + KR;
  double* col = colbuf + (K & 1) * NP;
  if (B.bj == KB) {   // the threads of block column KB publish column K
#pragma unroll
    for (int r = 0; r < SB; ++r) col[B.bi * SB + r] = B.b[r][KR];
  }
  __syncthreads();
  const double d = uniform_d(col[K]);
  double ci[SB], cj[SB];
#pragma unroll
  for (int r = 0; r < SB; ++r) ci[r] = col[B.bi * SB + r];
#pragma unroll
  for (int c = 0; c < SB; ++c) cj[c] = col[B.bj * SB + c];
  if (!(d > tau)) {
    if (threadIdx.x == 0) drop[K] = 1;
    ++ndrop;
    return;
  }
  const double inv = rcp_nr(d);
  const bool rowk = B.bi == KB, colk = B.bj == KB;
  double g[SB];
#pragma unroll
  for (int r = 0; r < SB; ++r) g[r] = ci[r] * inv;
  // row K itself: a_Kj - (1 - 1/d) a_Kj = a_Kj / d
  const double gk = rowk ? 1.0 - inv : g[KR];
  // column K by the same update: a_iK - (a_iK / d)(d - 1) = a_iK / d (the
  // equilibrated pivots are at most 1 plus the mixed forms' shift; the
  // rounding of d - 1 at a large restart shift only touches a preconditioner)
  if (colk) cj[KR] = d - 1.0;
#pragma unroll
  for (int r = 0; r < SB; ++r) {
#pragma unroll
    for (int c = 0; c < SB; ++c) B.b[r][c] = fma(-(r == KR ? gk : g[r]), cj[c], B.b[r][c]);
  }
  // and -1/d at the pivot
  if (rowk && colk) B.b[KR][KR] = -inv;
}

template <int NC, int... KR>
__device__ __forceinline__ void big_pivot_row(BigBlocks<NC>& B, double* colbuf, double tau, int* drop,
                                              int& ndrop, int KB, int nk, std::integer_sequence<int, KR...>) {
  constexpr int SB = BigBlocks<NC>::SB;
  ((KB * SB + KR < NC && KB * SB + KR < nk ? big_pivot<NC, KR>(B, colbuf, tau, drop, ndrop, KB) : (void)0),
   ...);
}

template <int NC, int... KB>
__device__ __forceinline__ void big_pivot_rows(BigBlocks<NC>& B, double* colbuf, double tau, int* drop,
                                               int& ndrop, int nk, std::integer_sequence<int, KB...>) {
  (big_pivot_row<NC>(B, colbuf, tau, drop, ndrop, KB, nk,
                     std::make_integer_sequence<int, BigBlocks<NC>::SB>{}), ...);
}

// Sweep every unknown.  colbuf: LDS of BigBlocks<NC>::CB doubles; drop[]:
// LDS flags, zero on entry.  Returns the number of dropped pivots (uniform).
// LOOP: a loop over block rows of pivots keeps the code a few thousand
// instructions long (fully unrolled, the largest models' sweeps outgrow the
// instruction cache); kernels whose other live values leave too few
// registers for the loop's carried blocks take the unrolled form.  nk
// (uniform, <= NC): only the first nk pivots are swept (the rest of the
// matrix is an identity block the caller does not read).
template <int NC, bool LOOP = true>
__device__ __forceinline__ int big_sweep(BigBlocks<NC>& B, double* colbuf, double tau, int* drop,
                                         int nk = NC) {
  constexpr int SB = BigBlocks<NC>::SB, NKB = (NC + SB - 1) / SB;
  int ndrop = 0;
  if constexpr (LOOP) {
    const int nkb = (nk + SB - 1) / SB;
#pragma unroll 1
    for (int kb = 0; kb < nkb; ++kb)
      big_pivot_row<NC>(B, colbuf, tau, drop, ndrop, kb, nk, std::make_integer_sequence<int, SB>{});
  } else {
    big_pivot_rows<NC>(B, colbuf, tau, drop, ndrop, nk, std::make_integer_sequence<int, NKB>{});
  }
  return ndrop;
}

// After the sweep: the unscaled solution (last row) into x[NC] and G^-1 of
// the kept unknowns, unscaled, as a packed lower triangle into ginv (zero in
// the rows and columns of dropped pivots).
template <int NC>
__device__ __forceinline__ void big_store(const BigBlocks<NC>& B, const int* drop, double* ginv,
                                          double* x) {
  constexpr int SB = BigBlocks<NC>::SB, RB = NC / SB, RR = NC % SB;
#pragma unroll
  for (int r = 0; r < SB; ++r) {
#pragma unroll
    for (int c = 0; c < SB; ++c) {
      const int i = B.bi * SB + r, j = B.bj * SB + c;
      if (i < NC && j <= i) ginv[pk(i, j)] = (drop[i] | drop[j]) ? 0.0 : -B.b[r][c] * B.sr[r] * B.sc[c];
    }
  }
  if (x && B.bi == RB) {
#pragma unroll
    for (int c = 0; c < SB; ++c) {
      const int j = B.bj * SB + c;
      if (j < NC) x[j] = drop[j] ? 0.0 : B.b[RR][c] * B.sc[c];
    }
  }
}

// The whole swept matrix, as it stands (equilibrated), packed lower into s:
// -G_KK^-1 in the kept block, G_KK^-1 G_KD beside it, the solution in the
// last row (see the sweep operator).
template <int NC>
__device__ __forceinline__ void big_store_swept(const BigBlocks<NC>& B, double* s) {
  constexpr int SB = BigBlocks<NC>::SB, NU = BigBlocks<NC>::NU;
#pragma unroll
  for (int r = 0; r < SB; ++r) {
#pragma unroll
    for (int c = 0; c < SB; ++c) {
      const int i = B.bi * SB + r, j = B.bj * SB + c;
      if (i < NU && j <= i) s[pk(i, j)] = B.b[r][c];
    }
  }
}

// Load a packed symmetric n x n matrix k (LDS, n <= N, already scaled) into
// blocks of size N: the identity beyond n, nothing in the augmented row.
template <int N>
__device__ __forceinline__ void big_load_n(const double* k, int n, BigBlocks<N>& B) {
  constexpr int SB = BigBlocks<N>::SB;
  B.bi = threadIdx.x >> 4;
  B.bj = threadIdx.x & 15;
#pragma unroll
  for (int r = 0; r < SB; ++r) {
    B.sr[r] = 1.0;
    B.sc[r] = 1.0;
  }
#pragma unroll
  for (int r = 0; r < SB; ++r) {
#pragma unroll
    for (int c = 0; c < SB; ++c) {
      const int i = B.bi * SB + r, j = B.bj * SB + c;
      double v = 0.0;
      if (i < n && j < n) v = k[i >= j ? pk(i, j) : pk(j, i)];
      else if (i == j && i < N) v = 1.0;
      B.b[r][c] = v;
    }
  }
}


// z = G^-1 r with G^-1 packed lower in LDS (n x n), one row per thread.
__device__ __forceinline__ void packed_matvec_n(const double* ginv, int n, const double* r, double* z) {
  for (int i = threadIdx.x; i < n; i += kThreads) {
    double acc = 0.0;
    for (int j = 0; j < i; ++j) acc = fma(ginv[pk(i, j)], r[j], acc);
    for (int j = i; j < n; ++j) acc = fma(ginv[pk(j, i)], r[j], acc);
    z[i] = acc;
  }
  __syncthreads();
}

template <int NC>
__device__ __forceinline__ void packed_matvec(const double* ginv, const double* r, double* z) {
  packed_matvec_n(ginv, NC, r, z);
}

// ---------------------------------------------------------------------------
// the linearised fit
// ---------------------------------------------------------------------------
// End of a workgroup fit: the optional check pass (residual and min Q at the
// samples), the coefficients out, the status, and the re-solve flag.
template <int V, int D, bool VLDS = false>
__device__ __forceinline__ void fit_finish(const FitArgs& a, int f, int64_t s0, int64_t m, int ndrop,
                                           int it, double last_rel, FitShared<Shape<V, D>::NC>& sh,
                                           double* coef) {
  constexpr int NC = Shape<V, D>::NC;
  double resid = __builtin_nan("");
  double qmin = 1.0;
  if (a.check_q) {
    const double ss = pass<V, D, PASS_CHECK, VLDS>(a, s0, m, sh.c, nullptr, sh, &qmin);
    resid = sqrt(ss);
  }
  for (int j = threadIdx.x; j < NC; j += kThreads) coef[j] = sh.c[j];
  if (threadIdx.x == 0) {
    int st = RP_FIT_OK;
    if (m < NC) st = RP_FIT_UNDERDETERMINED;
    else if (ndrop > 0) st = RP_FIT_RANK_DEFICIENT;
    else if (!(last_rel <= sqrt(a.tol))) st = RP_FIT_NOT_CONVERGED;
    else if (!(qmin > 0.0)) st = RP_FIT_Q_NONPOSITIVE;
    a.status[f] = st;
    if (a.resid) a.resid[f] = resid;
    if (a.iters) a.iters[f] = it;
    flag_for_resolve(a, f, st);
  }
}

// Numerical rank of the linearised fit: an unknown whose design column lies
// within tau_c = 1e-5 of its own norm from the span of the columns kept
// before it (natural order) is dependent; the sweep of the unit-diagonal
// Gram compares its pivot with tau_c^2.
constexpr double kTauColSq = 1e-10;

// Larger models, FP64, split form: one workgroup per fit sweeps the Gram in
// the workspace (formed there by weighted moments) straight from global
// memory into registers, then writes G^-1 of the kept unknowns over it and
// the basic solution to coef; gflag keeps bit 0 (non-finite input) and
// receives the count of dropped pivots above it.  Without a copy of the Gram
// in LDS two workgroups share a compute unit, so one hides the other's
// per-pivot barrier and LDS latency.  k_big_refine refines from there.
template <int V, int D>
__global__ __launch_bounds__(kThreads, 2) void k_big_sweep(FitArgs a) {
  constexpr int NC = Shape<V, D>::NC;
  __shared__ double colbuf[BigBlocks<NC>::CB];
  __shared__ int drop[NC];
  const int tid = threadIdx.x;
  const int f = a.ids[blockIdx.x];
  if (a.gflag[f] & 1) return;   // non-finite input: k_fit writes the outputs
  // the equilibration factors wait in LDS (not in registers) for the store
  __shared__ double scale[BigBlocks<NC>::NP];
  double* g = a.gws + a.gofs[f];
  for (int j = tid; j < NC; j += kThreads) drop[j] = 0;
  BigBlocks<NC> B;
  big_load<NC>(g, B, scale);
  constexpr int SB = BigBlocks<NC>::SB;
  __syncthreads();   // the whole Gram is in registers (it may be overwritten); drop[] is cleared
  const int ndrop = big_sweep<NC>(B, colbuf, kTauColSq, drop);
  __syncthreads();   // the drop flags of the last pivots
  double* x = a.coef + a.coef_off[f];
  constexpr int RB = NC / SB, RR = NC % SB;
#pragma unroll
  for (int r = 0; r < SB; ++r) {
#pragma unroll
    for (int c = 0; c < SB; ++c) {
      const int i = B.bi * SB + r, j = B.bj * SB + c;
      if (i < NC && j <= i) g[pk(i, j)] = (drop[i] | drop[j]) ? 0.0 : -B.b[r][c] * scale[i] * scale[j];
    }
  }
  if (B.bi == RB) {
#pragma unroll
    for (int c = 0; c < SB; ++c) {
      const int j = B.bj * SB + c;
      if (j < NC) x[j] = drop[j] ? 0.0 : B.b[RR][c] * scale[j];
    }
  }
  if (tid == 0) a.gflag[f] = ndrop << 1;
}

template <int V, int D, int PREC>
__global__ __launch_bounds__(kThreads) void k_fit(FitArgs a) {
  using Cfg = FitCfg<V, D, PREC>;
  constexpr int NC = Cfg::NC;
  __shared__ __align__(16) unsigned char raw[Cfg::RAW_BYTES];
  __shared__ FitShared<NC> sh;
  double* G = reinterpret_cast<double*>(raw);
  const int tid = threadIdx.x;
  const int f = a.ids[blockIdx.x];
  const int64_t s0 = a.sample_off[f];
  const int64_t m = a.sample_off[f + 1] - s0;
  double* coef = a.coef + a.coef_off[f];
  if (tid == 0) sh.flag_nonfinite = 0;
  __syncthreads();

  gram<V, D, PREC, false>(a, s0, m, raw, G, sh, nullptr);

  if (sh.flag_nonfinite) {
    for (int j = tid; j < NC; j += kThreads) coef[j] = __builtin_nan("");
    if (tid == 0) {
      a.status[f] = RP_FIT_NONFINITE_INPUT;
      if (a.resid) a.resid[f] = __builtin_nan("");
      if (a.iters) a.iters[f] = 0;
    }
    return;
  }

  // factor: FP64 sweeps the equilibrated Gram in registers (vanished pivots
  // dropped) into G^-1 and the solution; the mixed forms shift the diagonal
  // until the low-precision Gram factors (Cholesky), then refine against FP64
  // products.
  int ndrop = 0;
  int it = 0;
  double last_rel = 0.0;
  __shared__ double colbuf[BigBlocks<NC>::CB];
  if constexpr (PREC == RP_FP64) {
    for (int j = tid; j < NC; j += kThreads) sh.drop[j] = 0;
    BigBlocks<NC> B;
    big_load<NC>(G, B, colbuf);
    __syncthreads();   // every block is in registers; drop[] is cleared
    ndrop = big_sweep<NC>(B, colbuf, kTauColSq, sh.drop);
    __syncthreads();   // the drop flags of the last pivots
    big_store<NC>(B, sh.drop, G, sh.c);
    __syncthreads();
    // iterative refinement: c += G^-1 A^T (b - A c)
    for (it = 0; it < a.max_refine;) {
      pass<V, D, PASS_RESIDUAL>(a, s0, m, sh.c, sh.r, sh, nullptr);
      packed_matvec<NC>(G, sh.r, sh.z);
      for (int j = tid; j < NC; j += kThreads) sh.c[j] += sh.z[j];
      ++it;
      const double dn = maxabs_nc<NC>(sh.z, sh);
      const double cn = maxabs_nc<NC>(sh.c, sh);
      last_rel = cn > 0.0 ? dn / cn : dn;
      if (dn <= a.stop_rel * cn) break;
    }
  } else {
    // the shifted low-precision Gram swept into its inverse (the
    // preconditioner) and the starting solution; a non-positive pivot asks
    // for a larger shift (the Gram in LDS is still intact)
    double shift = PREC == RP_MIXED_FP32 ? 0x1p-20 : 0x1p-7;
    BigBlocks<NC> B;
    for (int attempt = 0; attempt < 7; ++attempt) {
      for (int j = tid; j < NC; j += kThreads) sh.drop[j] = 0;
      big_load<NC>(G, B, colbuf, shift);
      __syncthreads();
      ndrop = big_sweep<NC>(B, colbuf, 0.0, sh.drop);
      __syncthreads();
      if (ndrop == 0) break;
      shift *= 16.0;
    }
    big_store<NC>(B, sh.drop, G, sh.c);
    __syncthreads();
    // preconditioned CG on A^T A c = A^T b with M = the low-precision Gram;
    // a fit whose CG stops before its correction reaches the bar (a
    // breakdown, a hopeless rate, the cap) counts as not converged and is
    // re-solved in FP64
    double dn1 = 0.0, dnmin = INFINITY;
    bool reached = false;
    pass<V, D, PASS_RESIDUAL>(a, s0, m, sh.c, sh.r, sh, nullptr);
    packed_matvec<NC>(G, sh.r, sh.z);
    for (int j = tid; j < NC; j += kThreads) sh.p[j] = sh.z[j];
    double rz = dot_nc<NC>(sh.r, sh.z, sh);
    for (it = 0; it < a.max_refine;) {
      pass<V, D, PASS_PRODUCT>(a, s0, m, sh.p, sh.q, sh, nullptr);
      const double pq = dot_nc<NC>(sh.p, sh.q, sh);
      const double alpha = pq > 0.0 ? rz / pq : 0.0;
      for (int j = tid; j < NC; j += kThreads) {
        sh.c[j] = fma(alpha, sh.p[j], sh.c[j]);
        sh.r[j] = fma(-alpha, sh.q[j], sh.r[j]);
      }
      ++it;
      const double dn = fabs(alpha) * maxabs_nc<NC>(sh.p, sh);
      const double cn = maxabs_nc<NC>(sh.c, sh);
      last_rel = cn > 0.0 ? dn / cn : dn;
      if (dn <= a.tol * cn) { reached = true; break; }
      if (!(pq > 0.0)) break;
      if (pcg_hopeless(it, a.max_refine, dn, cn, a.tol, dn1, dnmin)) break;
      packed_matvec<NC>(G, sh.r, sh.z);
      const double rz2 = dot_nc<NC>(sh.r, sh.z, sh);
      const double beta = rz > 0.0 ? rz2 / rz : 0.0;
      rz = rz2;
      for (int j = tid; j < NC; j += kThreads) sh.p[j] = fma(beta, sh.p[j], sh.z[j]);
      __syncthreads();
    }
    if (!reached) last_rel = INFINITY;
  }

  fit_finish<V, D>(a, f, s0, m, ndrop, it, last_rel, sh, coef);
}

// Larger models, FP64, split form, after k_big_sweep: iterative refinement
// c += G^-1 A^T (b - A c), G^-1 read from the workspace (global memory) by the
// matrix-vector products, so the workgroup needs only a few KB of LDS and two
// share a compute unit; then the Q check and the status.
template <int V, int D>
__global__ __launch_bounds__(kThreads, 2) void k_big_refine(FitArgs a) {
  constexpr int NC = Shape<V, D>::NC;
  __shared__ FitShared<NC> sh;
  const int tid = threadIdx.x;
  const int f = a.ids[blockIdx.x];
  const int64_t s0 = a.sample_off[f];
  const int64_t m = a.sample_off[f + 1] - s0;
  double* coef = a.coef + a.coef_off[f];
  const int flags = a.gflag[f];
  if (flags & 1) {   // non-finite input (the sweep kernel skipped the fit)
    for (int j = tid; j < NC; j += kThreads) coef[j] = __builtin_nan("");
    if (tid == 0) {
      a.status[f] = RP_FIT_NONFINITE_INPUT;
      if (a.resid) a.resid[f] = __builtin_nan("");
      if (a.iters) a.iters[f] = 0;
    }
    return;
  }
  const int ndrop = flags >> 1;
  const double* H = a.gws + a.gofs[f];
  for (int j = tid; j < NC; j += kThreads) sh.c[j] = coef[j];
  __syncthreads();
  int it = 0;
  double last_rel = 0.0;
  for (it = 0; it < a.max_refine;) {
    pass<V, D, PASS_RESIDUAL, true>(a, s0, m, sh.c, sh.r, sh, nullptr);
    packed_matvec<NC>(H, sh.r, sh.z);
    for (int j = tid; j < NC; j += kThreads) sh.c[j] += sh.z[j];
    ++it;
    const double dn = maxabs_nc<NC>(sh.z, sh);
    const double cn = maxabs_nc<NC>(sh.c, sh);
    last_rel = cn > 0.0 ? dn / cn : dn;
    if (dn <= a.stop_rel * cn) break;
  }
  fit_finish<V, D, true>(a, f, s0, m, ndrop, it, last_rel, sh, coef);
}

// ---------------------------------------------------------------------------
// minimum-norm solutions of rank-deficient and underdetermined fits
// ---------------------------------------------------------------------------
// Section 4.2 solves each linearised system with an SVD.  With full column
// rank every least-squares solver gives the same minimiser; when the system is
// rank deficient or has fewer samples than unknowns, the SVD's answer is the
// minimiser of smallest Euclidean norm.  The fit kernels hold vanished pivots
// at zero (a basic solution) and flag the fit; k_min_norm then re-solves each
// flagged fit for the minimum-norm minimiser, one workgroup per fit:
//
//  - fewer samples than unknowns (m < NC): x = A^T z with (A A^T) z = b.  Row
//    i of A is [m(u_i), -y_i m'(u_i)], so a_i . a_j = Pn + y_i y_j (Pq - 1)
//    with Pn (Pq) the sum of every monomial of total degree <= dn (dq)
//    evaluated at the elementwise product u_i * u_j (the constant monomial is
//    the only one Q's part lacks).  The m x m sample Gram is equilibrated and factored, and x is
//    refined against the samples by x += A^T K^-1 (b - A x); every iterate lies
//    in the row space of A, so the limit is the minimum-norm interpolant.  A
//    vanished sample pivot (dependent samples) hands the fit to the second form.
//  - otherwise: the unknowns' augmented Gram is swept with the fit kernels'
//    drop rule, leaving kept unknowns K and dropped ones D.  The swept KD block
//    is T = G_KK^-1 G_KD, so Z = [-T; I] spans the null space of A.  x_K is
//    refined against the samples, T is refined column by column against the
//    samples (column j of T is the least-squares fit of A's column j by the
//    kept columns), and the basic solution [x_K; 0] is projected onto the row
//    space: x = [x_K - T w; w] with (I + T^T T) w = T^T x_K, or equivalently
//    x_K' = (I + T T^T)^-1 x_K, x_D = T^T x_K'.  Whichever of the two SPD
//    systems is smaller is factored (eigenvalues >= 1: no pivot can vanish).
// With fewer samples than unknowns a sample whose design row lies within
// tau_r = sqrt(1e-13) of its own norm from the span of the rows before it is
// dependent (the pivot of the unit-diagonal sample Gram against tau_r^2).
constexpr double kTauRowSq = 1e-13;
constexpr int kMinNormSteps = 10;          // refinement cap of either form
constexpr int kNullSpaceRounds = 2;        // refinement rounds of T

template <int V, int D, int J>
struct PackedExp {   // exponents of monomial J, 8 bits per variable
  static constexpr int v = Mono<V, D>::T.e[J][0] | (Mono<V, D>::T.e[J][1] << 8) |
                           (Mono<V, D>::T.e[J][2] << 16) | (Mono<V, D>::T.e[J][3] << 24);
};
template <int V, int D, int... J>
__device__ __forceinline__ void fill_exponents(int* ex, std::integer_sequence<int, J...>) {
  ((ex[J] = PackedExp<V, D, J>::v), ...);
}

template <int V, int D>
struct MinNormShared {
  static constexpr int NC = Shape<V, D>::NC, NU = NC + 1, NM = Shape<V, D>::NM;
  static constexpr int H = NC / 2;   // the smaller of |K| and |D| never exceeds it
  union {
    struct {                         // sample-space form
      double pw[V][code_dmax(D) + 1][NC];   // u_k^p of sample i
      double y[NC];
      double s[NC];                  // equilibration of the sample Gram
      double zy[NC];                 // -y_i z_i
    } smp;
    struct {                         // unknown-space form
      double col[NU];                // pivot column of the sweep
      double M[H * (H + 1) / 2];     // projection system, packed lower
      double t[NC];
      int kept[NC], dropped[NC];
      int mdrop[NC];
    } unk;
  };
  int ex[NM];
  int list[kThreads];
  int nlist;
};

// Sums of every monomial of total degree <= dn (pn) and <= dq (pq) in V
// variables at t (degree code D): the complete homogeneous sums h_0 .. h_DM
// built one variable at a time (h_d += t_k h_{d-1}, d ascending).
template <int V, int D>
__device__ __forceinline__ void monomial_sums(const double (&t)[V], double& pn, double& pq) {
  constexpr int DM = code_dmax(D), DN = code_dn(D), DQ = code_dq(D);
  double h[DM + 1];
  h[0] = 1.0;
#pragma unroll
  for (int d = 1; d <= DM; ++d) h[d] = 0.0;
#pragma unroll
  for (int k = 0; k < V; ++k) {
#pragma unroll
    for (int d = 1; d <= DM; ++d) h[d] = fma(t[k], h[d - 1], h[d]);
  }
  double sn = h[DN], sq = h[DQ];
#pragma unroll
  for (int d = DN - 1; d >= 0; --d) sn += h[d];
#pragma unroll
  for (int d = DQ - 1; d >= 0; --d) sq += h[d];
  pn = sn;
  pq = sq;
}

// Lower Cholesky of the leading n x n block of a packed symmetric matrix in
// LDS, n known at run time.  A pivot <= tau is dropped: its column is held at
// zero.  Returns the number of dropped pivots (uniform over the workgroup).
__device__ int cholesky_n(double* G, int n, int* drop, int* n_drop, double tau) {
  const int tid = threadIdx.x;
  if (tid == 0) *n_drop = 0;
  for (int j = tid; j < n; j += kThreads) drop[j] = 0;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    const double piv = G[pk(k, k)];
    const bool dropped = !(piv > tau);
    const double lkk = dropped ? 1.0 : sqrt(piv);
    const double inv = dropped ? 0.0 : 1.0 / lkk;
    __syncthreads();
    if (tid == 0) {
      G[pk(k, k)] = lkk;
      if (dropped) { drop[k] = 1; *n_drop += 1; }
    }
    for (int i = k + 1 + tid; i < n; i += kThreads) G[pk(i, k)] *= inv;
    __syncthreads();
    const int grp = tid >> 3, sub = tid & 7;
    for (int i = k + 1 + grp; i < n; i += kThreads / 8) {
      const double lik = G[pk(i, k)];
      for (int j = k + 1 + sub; j <= i; j += 8) G[pk(i, j)] -= lik * G[pk(j, k)];
    }
    __syncthreads();
  }
  return *n_drop;
}

// x = (L L^T)^-1 b for the factor of cholesky_n (wave 0, rows over lanes);
// dropped pivots give zero components.  b and x may alias; n <= NMAX.
template <int NMAX>
__device__ void chol_solve_n(const double* G, int n, const int* drop, const double* b, double* x) {
  constexpr int R = (NMAX + 63) / 64;
  const int tid = threadIdx.x;
  __syncthreads();
  if (tid < 64) {
    double z[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = tid + 64 * r;
      z[r] = i < n ? b[i] : 0.0;
    }
    auto pick = [&](int k) {
      double o = z[0];
#pragma unroll
      for (int r = 1; r < R; ++r) if (k >= 64 * r) o = z[r];
      return o;
    };
    for (int k = 0; k < n; ++k) {
      double zk = __shfl(pick(k), k % 64, 64);
      zk = drop[k] ? 0.0 : zk / G[pk(k, k)];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = tid + 64 * r;
        if (i == k) z[r] = zk;
        else if (i > k && i < n) z[r] -= G[pk(i, k)] * zk;
      }
    }
    for (int k = n - 1; k >= 0; --k) {
      double xk = __shfl(pick(k), k % 64, 64);
      xk = drop[k] ? 0.0 : xk / G[pk(k, k)];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = tid + 64 * r;
        if (i == k) z[r] = xk;
        else if (i < k) z[r] -= G[pk(k, i)] * xk;
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = tid + 64 * r;
      if (i < n) x[i] = z[r];
    }
  }
  __syncthreads();
}

// Outcome of one minimum-norm solve.
struct MinNormOut {
  double resid;     // ||b - A x||
  double qmin;      // min over the samples of Q at x
  double last_rel;  // last correction's max-norm relative to max|x|
  int steps;        // refinement steps of x
  int ndrop;        // dropped unknowns (unknown-space form)
};

// Sample-space form (m < NC).  Kp: LDS room for the packed m x m sample
// Gram.  Returns false, with nothing written, when a sample pivot vanished.
template <int V, int D>
__device__ bool min_norm_samples(const FitArgs& a, int64_t s0, int m, double* Kp, double* colbuf,
                                 FitShared<Shape<V, D>::NC>& sh, MinNormShared<V, D>& mn,
                                 MinNormOut& out) {
  using S = Shape<V, D>;
  constexpr int NC = S::NC, NA = S::NA, NM = S::NM;
  const int tid = threadIdx.x;
  auto& sm = mn.smp;
  for (int i = tid; i < m; i += kThreads) {
    sm.y[i] = a.y[s0 + i];
#pragma unroll
    for (int k = 0; k < V; ++k) {
      const double u = a.x[(int64_t)k * a.ldx + s0 + i];
      double p = 1.0;
#pragma unroll
      for (int q = 0; q <= code_dmax(D); ++q) { sm.pw[k][q][i] = p; p *= u; }
    }
  }
  __syncthreads();
  for (int i = tid; i < m; i += kThreads) {
    double t[V];
#pragma unroll
    for (int k = 0; k < V; ++k) t[k] = sm.pw[k][1][i] * sm.pw[k][1][i];
    double pn, pq;
    monomial_sums<V, D>(t, pn, pq);
    const double yi = sm.y[i];
    sm.s[i] = eq_scale(fma(yi * yi, pq - 1.0, pn));
  }
  __syncthreads();
  {
    const int grp = tid >> 3, sub = tid & 7;
    for (int i = grp; i < m; i += kThreads / 8) {
      for (int j = sub; j <= i; j += 8) {
        double t[V];
#pragma unroll
        for (int k = 0; k < V; ++k) t[k] = sm.pw[k][1][i] * sm.pw[k][1][j];
        double pn, pq;
        monomial_sums<V, D>(t, pn, pq);
        Kp[pk(i, j)] = fma(sm.y[i] * sm.y[j], pq - 1.0, pn) * sm.s[i] * sm.s[j];
      }
    }
  }
  // sweep the equilibrated sample Gram (padded with the identity to NC - 1)
  // into its inverse, packed back into Kp; only its m pivots are swept (the
  // padding is never read)
  for (int j = tid; j < NC; j += kThreads) sh.drop[j] = 0;
  __syncthreads();   // every entry of the sample Gram is written
  {
    BigBlocks<NC - 1> B;
    big_load_n<NC - 1>(Kp, m, B);
    __syncthreads();
    const int nd = big_sweep<NC - 1, false>(B, colbuf, kTauRowSq, sh.drop, m);
    __syncthreads();
    if (nd > 0) return false;
    big_store<NC - 1>(B, sh.drop, Kp, nullptr);
    __syncthreads();
  }

  for (int j = tid; j < NC; j += kThreads) sh.c[j] = 0.0;
  for (int i = tid; i < m; i += kThreads) sh.r[i] = sm.y[i];
  __syncthreads();
  double prev = INFINITY, ss = 0.0, qm = INFINITY, rel = 0.0;
  int it = 0;
  for (;;) {
    // z = K^-1 r through the inverse of the equilibrated sample Gram
    for (int i = tid; i < m; i += kThreads) sh.q[i] = sh.r[i] * sm.s[i];
    __syncthreads();
    packed_matvec_n(Kp, m, sh.q, sh.z);
    for (int i = tid; i < m; i += kThreads) {
      const double z = sh.z[i] * sm.s[i];
      sh.z[i] = z;
      sm.zy[i] = -sm.y[i] * z;
    }
    __syncthreads();
    // dx = A^T z, one unknown per thread
    for (int e = tid; e < NC; e += kThreads) {
      const bool num = e < NA;
      const int ex = mn.ex[num ? e : e - NA + 1];
      const double* w = num ? sh.z : sm.zy;
      double acc = 0.0;
      for (int i = 0; i < m; ++i) {
        double mono = sm.pw[0][ex & 0xFF][i];
#pragma unroll
        for (int k = 1; k < V; ++k) mono *= sm.pw[k][(ex >> (8 * k)) & 0xFF][i];
        acc = fma(w[i], mono, acc);
      }
      sh.p[e] = acc;
      sh.c[e] += acc;
    }
    __syncthreads();
    const double dn = maxabs_nc<NC>(sh.p, sh);
    const double cn = maxabs_nc<NC>(sh.c, sh);
    ++it;
    // r = b - A x, one sample per thread
    double ssl = 0.0, qml = INFINITY;
    for (int i = tid; i < m; i += kThreads) {
      double u[V];
#pragma unroll
      for (int k = 0; k < V; ++k) u[k] = sm.pw[k][1][i];
      double mo[NM];
      monomials<V, D, double>(u, mo);
      double nv = 0.0, qv = 0.0;
#pragma unroll
      for (int j = 0; j < NA; ++j) nv = fma(sh.c[j], mo[j], nv);
#pragma unroll
      for (int j = 1; j < S::NQ; ++j) qv = fma(sh.c[NA + j - 1], mo[j], qv);
      const double yi = sm.y[i];
      const double r = yi - fma(-yi, qv, nv);
      sh.r[i] = r;
      ssl = fma(r, r, ssl);
      qml = fmin(qml, 1.0 + qv);
    }
    ss = block_sum(ssl, sh.tmp);
    qm = -block_max(-qml, sh.tmp);
    rel = cn > 0.0 ? dn / cn : dn;
    // stop at the tolerance, once the corrections stop shrinking (rounding
    // level), or at the cap
    if (dn <= a.tol * cn || (it > 1 && dn > 0.5 * prev) || it >= kMinNormSteps) break;
    prev = dn;
  }
  out.resid = sqrt(ss);
  out.qmin = qm;
  out.last_rel = rel;
  out.steps = it;
  out.ndrop = 0;
  return true;
}

// -G_KK^-1 v in unscaled coordinates from the swept, equilibrated matrix S
// (whose KK block is -D G_KK^-1 D): out_i = -dsc_i sum_j S_ij dsc_j v_j over
// kept i, j; zero for dropped i.  sign = +1 gives G_KK^-1 v.
template <int NC>
__device__ void apply_kept_inverse(const double* S, const FitShared<NC>& sh, const double* v,
                                   double* out, double sign) {
  for (int i = threadIdx.x; i < NC; i += kThreads) {
    double acc = 0.0;
    if (!sh.drop[i]) {
      for (int j = 0; j < NC; ++j) {
        if (sh.drop[j]) continue;
        acc = fma(S[i >= j ? pk(i, j) : pk(j, i)], sh.dsc[j] * v[j], acc);
      }
      acc *= -sign * sh.dsc[i];
    }
    out[i] = acc;
  }
  __syncthreads();
}

// Unknown-space form (any m).  raw: the Gram workspace of FitCfg<V, D, FP64>.
template <int V, int D>
__device__ void min_norm_unknowns(const FitArgs& a, int64_t s0, int64_t m, unsigned char* raw,
                                  double* colbuf, FitShared<Shape<V, D>::NC>& sh,
                                  MinNormShared<V, D>& mn, MinNormOut& out) {
  constexpr int NC = Shape<V, D>::NC, NU = NC + 1;
  const int tid = threadIdx.x;
  auto& un = mn.unk;
  double* G = reinterpret_cast<double*>(raw);
  if (tid == 0) sh.flag_nonfinite = 0;
  __syncthreads();
  gram<V, D, RP_FP64, false>(a, s0, m, raw, G, sh, nullptr);

  // sweep every unknown in registers (the rhs row NC is carried along) and
  // keep the whole swept matrix, equilibrated, in G
  for (int j = tid; j <= NC; j += kThreads) sh.dsc[j] = j < NC ? eq_scale(G[pk(j, j)]) : 1.0;
  for (int j = tid; j < NC; j += kThreads) sh.drop[j] = 0;
  {
    BigBlocks<NC> B;
    big_load<NC>(G, B, colbuf);
    __syncthreads();
    const int ndrop = big_sweep<NC, false>(B, colbuf, kTauColSq, sh.drop);
    if (tid == 0) sh.n_drop = ndrop;
    __syncthreads();
    big_store_swept<NC>(B, G);
    __syncthreads();
  }
  const int grp = tid >> 3, sub = tid & 7;
  const int nd = sh.n_drop;
  const int nk = NC - nd;
  if (tid == 0) {
    int r = 0, q = 0;
    for (int j = 0; j < NC; ++j) {
      if (sh.drop[j]) un.dropped[q++] = j;
      else un.kept[r++] = j;
    }
  }
  for (int j = tid; j < NC; j += kThreads) sh.c[j] = sh.drop[j] ? 0.0 : G[pk(NC, j)] * sh.dsc[j];
  __syncthreads();

  // refine x_K: c += G_KK^-1 A_K^T (b - A c)
  double prev = INFINITY, rel = 0.0;
  int it = 0;
  for (; it < kMinNormSteps;) {
    pass<V, D, PASS_RESIDUAL>(a, s0, m, sh.c, sh.r, sh, nullptr);
    apply_kept_inverse<NC>(G, sh, sh.r, sh.z, 1.0);
    for (int j = tid; j < NC; j += kThreads) sh.c[j] += sh.z[j];
    ++it;
    const double dn = maxabs_nc<NC>(sh.z, sh);
    const double cn = maxabs_nc<NC>(sh.c, sh);
    rel = cn > 0.0 ? dn / cn : dn;
    if (dn <= a.tol * cn || (it > 1 && dn > 0.5 * prev)) break;
    prev = dn;
  }

  if (nd > 0) {
    // T_lj = dsc_l S_lj / dsc_j (l kept, j dropped) lives in the swept matrix
    auto sidx = [](int i, int j) { return i >= j ? pk(i, j) : pk(j, i); };
    // refine each column of T against the samples: with v = [t_j; -e_j],
    // A^T A v = -A_K^T (a_j - A_K t_j), so t_j -= G_KK^-1 (A^T A v)_K
    for (int round = 0; round < kNullSpaceRounds; ++round) {
      double worst = 0.0;
      for (int q = 0; q < nd; ++q) {
        const int dj = un.dropped[q];
        for (int l = tid; l < NC; l += kThreads)
          sh.p[l] = sh.drop[l] ? (l == dj ? -1.0 : 0.0) : sh.dsc[l] * G[sidx(l, dj)] / sh.dsc[dj];
        __syncthreads();
        pass<V, D, PASS_PRODUCT>(a, s0, m, sh.p, sh.q, sh, nullptr);
        apply_kept_inverse<NC>(G, sh, sh.q, sh.z, -1.0);   // -G_KK^-1 (A^T A v)
        double dl = 0.0, tl = 0.0;
        for (int l = tid; l < NC; l += kThreads) {
          if (sh.drop[l]) continue;
          G[sidx(l, dj)] += sh.z[l] * sh.dsc[dj] / sh.dsc[l];
          dl = fmax(dl, fabs(sh.z[l]));
          tl = fmax(tl, fabs(sh.p[l] + sh.z[l]));
        }
        dl = block_max(dl, sh.tmp);
        tl = block_max(tl, sh.tmp);
        worst = fmax(worst, tl > 0.0 ? dl / tl : dl);
      }
      if (worst <= a.tol) break;
    }
    __syncthreads();
    auto T = [&](int l, int j) { return sh.dsc[l] * G[sidx(l, j)] / sh.dsc[j]; };
    const bool small_d = nd <= nk;
    const int h = small_d ? nd : nk;
    // M = I + T^T T (over D) or I + T T^T (over K), packed lower
    for (int p = grp; p < h; p += kThreads / 8) {
      for (int q = sub; q <= p; q += 8) {
        double acc = (p == q) ? 1.0 : 0.0;
        if (small_d) {
          const int dp = un.dropped[p], dq = un.dropped[q];
          for (int l = 0; l < nk; ++l) acc = fma(T(un.kept[l], dp), T(un.kept[l], dq), acc);
        } else {
          const int kp = un.kept[p], kq = un.kept[q];
          for (int s = 0; s < nd; ++s) acc = fma(T(kp, un.dropped[s]), T(kq, un.dropped[s]), acc);
        }
        un.M[pk(p, q)] = acc;
      }
    }
    // right-hand side: T^T x_K (over D) or x_K (over K)
    for (int p = tid; p < h; p += kThreads) {
      double acc = 0.0;
      if (small_d) {
        const int dp = un.dropped[p];
        for (int l = 0; l < nk; ++l) acc = fma(T(un.kept[l], dp), sh.c[un.kept[l]], acc);
      } else {
        acc = sh.c[un.kept[p]];
      }
      un.t[p] = acc;
    }
    __syncthreads();
    cholesky_n(un.M, h, un.mdrop, &sh.n_drop, 0.0);
    chol_solve_n<NC>(un.M, h, un.mdrop, un.t, un.t);
    if (small_d) {
      // x_K -= T w, x_D = w
      for (int l = tid; l < NC; l += kThreads) {
        if (sh.drop[l]) continue;
        double acc = sh.c[l];
        for (int s = 0; s < nd; ++s) acc = fma(-T(l, un.dropped[s]), un.t[s], acc);
        sh.z[l] = acc;
      }
      __syncthreads();
      for (int l = tid; l < NC; l += kThreads) if (!sh.drop[l]) sh.c[l] = sh.z[l];
      for (int s = tid; s < nd; s += kThreads) sh.c[un.dropped[s]] = un.t[s];
    } else {
      // x_K = y, x_D = T^T y
      for (int s = tid; s < nd; s += kThreads) {
        const int dj = un.dropped[s];
        double acc = 0.0;
        for (int l = 0; l < nk; ++l) acc = fma(T(un.kept[l], dj), un.t[l], acc);
        sh.z[s] = acc;
      }
      __syncthreads();
      for (int l = tid; l < nk; l += kThreads) sh.c[un.kept[l]] = un.t[l];
      for (int s = tid; s < nd; s += kThreads) sh.c[un.dropped[s]] = sh.z[s];
    }
    __syncthreads();
  }
  double qm = 1.0;
  const double ss = pass<V, D, PASS_CHECK>(a, s0, m, sh.c, nullptr, sh, &qm);
  out.resid = sqrt(ss);
  out.qmin = qm;
  out.last_rel = rel;
  out.steps = it;
  out.ndrop = nd;
}

// Re-solve in FP64 every fit of the bucket whose status the fit kernels left
// at RP_FIT_RANK_DEFICIENT or RP_FIT_UNDERDETERMINED (for the minimum-norm
// minimiser), or at RP_FIT_NOT_CONVERGED (the refinement of any form hit its
// step cap: the FP64 form's few steps on a very ill-conditioned fit, or the
// mixed forms' PCG on a low-precision Gram too far from the FP64 one).  A
// full-rank fit then gets the FP64 Gram, the sweep and up to kMinNormSteps
// refinement steps, as a mixed-precision solver falls back to double
// precision.  The fit kernels append the flagged fits to the bucket's list;
// workgroup b serves list entries b, b + grid, ...
template <int V, int D>
__global__ __launch_bounds__(kThreads) void k_min_norm(FitArgs a) {
  using Cfg = FitCfg<V, D, RP_FP64>;
  constexpr int NC = Cfg::NC;
  static_assert((size_t)(NC - 1) * NC / 2 * sizeof(double) <= Cfg::RAW_BYTES, "sample Gram room");
  __shared__ __align__(16) unsigned char raw[Cfg::RAW_BYTES];
  __shared__ FitShared<NC> sh;
  __shared__ MinNormShared<V, D> mn;
  __shared__ double colbuf[BigBlocks<NC>::CB];
  __shared__ int list_len;
  const int tid = threadIdx.x;
  // the list the fit kernels filled: workgroup b re-solves entries b, b + grid, ...
  // (one read of its length, shared through LDS)
  if (tid == 0) list_len = __builtin_nontemporal_load(a.resolve);
  __syncthreads();
  const int n = list_len;
  // an empty list (every workgroup reads the same length: the list was
  // filled by earlier launches, and only the last workgroup of a non-empty
  // pass clears it) needs neither work nor the finish count below
  if (n == 0) return;
  if ((int)blockIdx.x < n) {
    if (tid == 0) fill_exponents<V, D>(mn.ex, std::make_integer_sequence<int, Cfg::NM>{});
    __syncthreads();
  }
  for (int q = blockIdx.x; q < n; q += gridDim.x) {
    const int f = a.resolve[2 + q];
    const int64_t s0 = a.sample_off[f];
    const int64_t m = a.sample_off[f + 1] - s0;
    MinNormOut o{};
    bool done = false;
    if (m < NC) done = min_norm_samples<V, D>(a, s0, (int)m, reinterpret_cast<double*>(raw), colbuf, sh, mn, o);
    if (!done) min_norm_unknowns<V, D>(a, s0, m, raw, colbuf, sh, mn, o);
    double* coef = a.coef + a.coef_off[f];
    for (int j = tid; j < NC; j += kThreads) coef[j] = sh.c[j];
    if (tid == 0) {
      int st = RP_FIT_OK;
      if (m < NC) st = RP_FIT_UNDERDETERMINED;
      else if (o.ndrop > 0) st = RP_FIT_RANK_DEFICIENT;
      else if (!(o.last_rel <= sqrt(a.tol))) st = RP_FIT_NOT_CONVERGED;
      else if (a.check_q && !(o.qmin > 0.0)) st = RP_FIT_Q_NONPOSITIVE;
      a.status[f] = st;
      if (a.resid) a.resid[f] = a.check_q ? o.resid : __builtin_nan("");
      if (a.iters) a.iters[f] = o.steps;
    }
    __syncthreads();
  }
  // the last workgroup to finish empties the list for the next call.  Each
  // workgroup's reads of the list returned (their values steered the loop
  // above) before its thread 0 counts it finished, so no fence is needed
  // here (an agent-scope fence writes back the L2 of the workgroup's XCD,
  // microseconds per workgroup); the next launch sees the cleared list
  // through the end-of-kernel release.
  if (tid == 0) {
    if (atomicAdd(a.resolve + 1, 1) == (int)gridDim.x - 1) {
      a.resolve[0] = 0;
      a.resolve[1] = 0;
    }
  }
}

// Levenberg-Marquardt state of fit f at the start of a refine call (thread 0
// of the fit's first launch): undamped, active, no rejection, no loss yet (the
// first Gram's corner provides it).
enum LmState { LM_ACTIVE = 0, LM_CONVERGED = 1, LM_STOPPED = 2, LM_NONFINITE = 3 };
__device__ __forceinline__ void lm_state_init(const FitArgs& a, int f) {
  if (threadIdx.x == 0) {
    a.lm_loss[f] = __builtin_nan("");
    a.lm_lambda[f] = 0.0;
    a.lm_state[f] = LM_ACTIVE;
    a.lm_rejects[f] = 0;
    if (a.iters) a.iters[f] = 0;
  }
}

// ---------------------------------------------------------------------------
// split form: Gram kernel + wave-per-fit solve/refine kernel
// ---------------------------------------------------------------------------
// The Gram kernel writes each fit's packed augmented Gram to a workspace; the
// solve kernel then owns one fit per wave64, so the small dense algebra and the
// refinement passes run without workgroup barriers.

template <int V, int D, int PREC, bool GN = false>
__global__ __launch_bounds__(kThreads) void k_gram(FitArgs a, double* gws, const int64_t* gofs,
                                                   int* gflag) {
  using Cfg = FitCfg<V, D, PREC>;
  constexpr int NC = Cfg::NC, NU = Cfg::NU;
  constexpr int NPK = NU * (NU + 1) / 2;
  __shared__ __align__(16) unsigned char raw[Cfg::RAW_BYTES];
  __shared__ FitShared<NC> sh;
  double* G = reinterpret_cast<double*>(raw);
  const int f = a.ids[blockIdx.x];
  if constexpr (GN) {
    // first iteration: set the fit's LM state; later ones: converged or
    // stopped: nothing to form; last step rejected: the coefficients did not
    // move and the fit's Gram in the workspace still holds
    if (a.lm_state && a.lm_first) lm_state_init(a, f);
    else if (a.lm_state && (a.lm_state[f] != 0 || a.lm_rejects[f] > 0)) return;
  }
  const int64_t s0 = a.sample_off[f];
  const int64_t m = a.sample_off[f + 1] - s0;
  if (threadIdx.x == 0) sh.flag_nonfinite = 0;
  if constexpr (GN) {
    const double* c = a.coef + a.coef_off[f];
    for (int j = threadIdx.x; j < NC; j += kThreads) sh.c[j] = c[j];
  }
  __syncthreads();
  gram<V, D, PREC, GN>(a, s0, m, raw, G, sh, GN ? sh.c : nullptr);
  double* out = gws + gofs[f];
  for (int e = threadIdx.x; e < NPK; e += kThreads) out[e] = G[e];
  if (threadIdx.x == 0) gflag[f] = sh.flag_nonfinite;
}

// Largest model the wave-per-fit kernels handle: the block sweep keeps a
// ceil((NC+1)/8)^2 block of the augmented matrix per lane in registers.
constexpr int kWaveSolveMaxNC = 39;

// ---------------------------------------------------------------------------
// sweep operator on a register-blocked symmetric matrix
// ---------------------------------------------------------------------------
// Sweeping pivot k of a symmetric matrix (d = a_kk) maps a_ij -> a_ij -
// a_ik a_kj / d for i, j != k, a_ik -> a_ik / d and a_kk -> -1/d.  Sweeping
// every unknown of the augmented normal matrix [G b; b^T b^Tb] (Section 4.2)
// leaves -G^-1 in the leading block, the least-squares solution in the last
// row and the residual sum of squares in the corner.  A pivot <= tau (rank
// deficiency) is not swept: its row and column are then held at zero in the
// outputs, i.e. its coefficient is fixed at zero.
//
// The (NC+1)^2 matrix, padded with zeros to 8 SB x 8 SB, is split into an 8x8
// grid of SB x SB blocks: lane L holds block (L >> 3, L & 7) in registers for
// the whole sweep.  Per pivot only column k travels through LDS (published by
// the eight lanes of its block column); every lane then reads the column
// entries of its block's rows and columns and updates its block with SB^2
// FMAs.  The pivot loop is unrolled at compile time, so block indices are
// static and no lane branches on data.
template <int NC>
struct Blocks {
  static constexpr int NU = NC + 1;
  static constexpr int SB = (NU + 7) / 8;
  static constexpr int NP = 8 * SB;
  double b[SB][SB];
  double sr[SB], sc[SB];   // equilibration factors of the block's rows / columns
  int bi, bj;
};

// Load the packed lower augmented Gram gs (LDS) into the blocks, equilibrated,
// with the unknowns' diagonal mapped to g * dmul + dadd (Levenberg-Marquardt
// damping, or the mixed forms' positive shift).
// The factors equilibrate the damped diagonal g_jj * dmul to 1, so every
// pivot of the sweep is at most 1 + dadd.  scr: LDS scratch of NC doubles
// (the pivot column buffer before the sweep) for the factors, each formed
// once by one lane.
template <int NC>
__device__ __forceinline__ void block_load(const double* gs, Blocks<NC>& B, double dmul,
                                           double dadd, double* scr) {
  constexpr int SB = Blocks<NC>::SB, NU = Blocks<NC>::NU;
  const int lane = threadIdx.x & 63;
  B.bi = lane >> 3;
  B.bj = lane & 7;
  for (int j = lane; j < NC; j += 64) scr[j] = eq_scale(gs[pk(j, j)] * dmul);
  wave_sync();
#pragma unroll
  for (int r = 0; r < SB; ++r) {
    const int i = B.bi * SB + r;
    B.sr[r] = i < NC ? scr[i] : 1.0;
    const int j = B.bj * SB + r;
    B.sc[r] = j < NC ? scr[j] : 1.0;
  }
#pragma unroll
  for (int r = 0; r < SB; ++r) {
#pragma unroll
    for (int c = 0; c < SB; ++c) {
      const int i = B.bi * SB + r, j = B.bj * SB + c;
      double v = 0.0;
      if (i < NU && j < NU) {
        v = gs[i >= j ? pk(i, j) : pk(j, i)] * B.sr[r] * B.sc[c];
        if (i == j && i < NC) v = fma(v, dmul, dadd);
      }
      B.b[r][c] = v;
    }
  }
  wave_sync();   // the scratch is read before the first pivot column lands there
}

template <int NC, int K>
__device__ __forceinline__ void block_pivot(Blocks<NC>& B, double* col, double tau,
                                            uint64_t& drop) {
  constexpr int SB = Blocks<NC>::SB, KB = K / SB, KR = K % SB;
  if (B.bj == KB) {   // the lanes of block column KB publish column K
#pragma unroll
    for (int r = 0; r < SB; ++r) col[B.bi * SB + r] = B.b[r][KR];
  }
  wave_sync();
  const double d = uniform_d(col[K]);
  double ci[SB], cj[SB];
#pragma unroll
  for (int r = 0; r < SB; ++r) ci[r] = col[B.bi * SB + r];
#pragma unroll
  for (int c = 0; c < SB; ++c) cj[c] = col[B.bj * SB + c];
  wave_sync();
  if (!(d > tau)) {
    drop |= 1ull << K;
    return;
  }
  const double inv = rcp_nr(d);
  const bool rowk = B.bi == KB, colk = B.bj == KB;
  double g[SB];
#pragma unroll
  for (int r = 0; r < SB; ++r) g[r] = ci[r] * inv;
  // row K itself: a_Kj - (1 - 1/d) a_Kj = a_Kj / d
  const double gk = rowk ? 1.0 - inv : g[KR];
  // column K by the same update: a_iK - (a_iK / d)(d - 1) = a_iK / d (the
  // pivots of an equilibrated matrix are at most about 1: no cancellation)
  if (colk) cj[KR] = d - 1.0;
#pragma unroll
  for (int r = 0; r < SB; ++r) {
#pragma unroll
    for (int c = 0; c < SB; ++c) B.b[r][c] = fma(-(r == KR ? gk : g[r]), cj[c], B.b[r][c]);
  }
  // and -1/d at the pivot
  if (rowk && colk) B.b[KR][KR] = -inv;
}

template <int NC, int... K>
__device__ __forceinline__ uint64_t block_sweep_all(Blocks<NC>& B, double* col, double tau,
                                                    std::integer_sequence<int, K...>) {
  uint64_t drop = 0;
  (block_pivot<NC, K>(B, col, tau, drop), ...);
  return drop;
}

// Sweep every unknown (col: LDS scratch of Blocks<NC>::NP doubles) of a
// matrix equilibrated by block_load.  A pivot at or below tau is dropped.
// Returns the bit mask of dropped pivots.
template <int NC>
__device__ __forceinline__ uint64_t block_sweep(Blocks<NC>& B, double* col, double tau) {
  static_assert(NC < 64, "pivot mask");
  return block_sweep_all<NC>(B, col, tau, std::make_integer_sequence<int, NC>{});
}

// Unscaled solution (last row of the swept matrix) into out[NC] (any memory).
template <int NC>
__device__ __forceinline__ void block_solution(const Blocks<NC>& B, uint64_t drop, double* out) {
  constexpr int SB = Blocks<NC>::SB, RB = NC / SB, RR = NC % SB;
  if (B.bi == RB) {
#pragma unroll
    for (int c = 0; c < SB; ++c) {
      const int j = B.bj * SB + c;
      if (j < NC) out[j] = ((drop >> j) & 1) ? 0.0 : B.b[RR][c] * B.sc[c];
    }
  }
}

// G^-1 of the kept unknowns, unscaled, as a packed lower triangle over g
// (zero in the rows and columns of dropped pivots).
template <int NC>
__device__ __forceinline__ void block_store_inverse(const Blocks<NC>& B, uint64_t drop, double* g) {
  constexpr int SB = Blocks<NC>::SB;
#pragma unroll
  for (int r = 0; r < SB; ++r) {
#pragma unroll
    for (int c = 0; c < SB; ++c) {
      const int i = B.bi * SB + r, j = B.bj * SB + c;
      if (i < NC && j <= i) {
        const bool z = ((drop >> i) | (drop >> j)) & 1;
        g[pk(i, j)] = z ? 0.0 : -B.b[r][c] * B.sr[r] * B.sc[c];
      }
    }
  }
}

// DPP move of a double across lanes (two 32-bit halves).
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_readlane((int)(uint32_t)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Wave64 sum with row-local DPP steps (quad swaps, half-row and row mirrors)
// and four lane reads; every lane gets the same, order-fixed result.
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_mov<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_mov<0x141>(v);   // row_half_mirror
  v += dpp_mov<0x140>(v);   // row_mirror
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}


// Monomials J0.. of u recomputed from their parents (indices < J0 must hold).
template <int V, int D, int J0, typename R, int... J>
__device__ __forceinline__ void monomials_tail_impl(const R* u, R* m, std::integer_sequence<int, J...>) {
  ((m[J0 + J] = m[MonoAt<V, D, J0 + J>::parent] * u[MonoAt<V, D, J0 + J>::var]), ...);
}
template <int V, int D, int J0, typename R>
__device__ __forceinline__ void monomials_tail(const R* u, R* m) {
  monomials_tail_impl<V, D, J0, R>(u, m, std::make_integer_sequence<int, Mono<V, D>::N - J0>{});
}


// Half-wave (32-lane) collectives: a wave serves two fits, lanes 0-31 and
// 32-63.  Every result is the same on the 32 lanes of a half.
__device__ __forceinline__ double half_sum(double v) {
  v += dpp_mov<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_mov<0x141>(v);   // row_half_mirror
  v += dpp_mov<0x140>(v);   // row_mirror
  const double s0 = readlane_d(v, 0) + readlane_d(v, 16);
  const double s1 = readlane_d(v, 32) + readlane_d(v, 48);
  return (threadIdx.x & 32) ? s1 : s0;
}

__device__ __forceinline__ double half_max(double v) {
#pragma unroll
  for (int o = 16; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

template <int NC>
__device__ __forceinline__ double half_dot(const double* a, const double* b) {
  double t = 0.0;
  for (int j = threadIdx.x & 31; j < NC; j += 32) t = fma(a[j], b[j], t);
  return half_sum(t);
}

template <int NC>
__device__ __forceinline__ double half_maxabs(const double* a) {
  double t = 0.0;
  for (int j = threadIdx.x & 31; j < NC; j += 32) t = fmax(t, fabs(a[j]));
  return half_max(t);
}

// out[j] = sum over the half's 32 lanes of acc[j], j < NC (lanes 0-31 and
// 32-63 serve two fits): a swap of 16-lane rows adds lanes l and l + 16 of
// two values at once, row 2h + k of value u then holding accumulator 2u + k
// of half h; the 16 partials meet in LDS (row stride 66 doubles) and one lane
// of the half adds them.  red: (NC + 1) / 2 * 66 doubles.
template <int NC>
__device__ __forceinline__ void half_reduce_vec(const double (&acc)[NC], double* out, double* red) {
  constexpr int N2 = (NC + 1) / 2;
  constexpr int S = 66;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int u = 0; u < N2; ++u)
    red[u * S + lane] = swap16_add(acc[2 * u], 2 * u + 1 < NC ? acc[2 * u + 1] : 0.0);
  wave_sync();
  const int h = lane >> 5, hl = lane & 31;
#pragma unroll
  for (int j0 = 0; j0 < NC; j0 += 32) {
    const int j = j0 + hl;
    if (j < NC) {
      const double* p = red + (j >> 1) * S + 16 * (2 * h + (j & 1));
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int i = 0; i < 16; i += 2) {
        s0 += p[i];
        s1 += p[i + 1];
      }
      out[j] = s0 + s1;
    }
  }
  wave_sync();
}

// z = H r for the packed lower symmetric H in global memory (r in LDS, z any
// memory), by a half wave: lane l forms rows l and l + 32.
template <int NC>
__device__ __forceinline__ void half_apply_inverse(const double* H, const double* r, double* z) {
  double t[2] = {0.0, 0.0};
  // the opaque zero keeps the row addresses from being hoisted out of the
  // caller's loops (they would pin a register pair per matrix entry)
  int zero;
  asm volatile("v_mov_b32 %0, 0" : "=v"(zero));
  const int hl = (threadIdx.x & 31) + zero;
  const double* rr = r + zero;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int j = hl + 32 * h;
    if (h * 32 < NC && j < NC) {
      const int rj = pk(j, 0);
      double s0 = 0.0, s1 = 0.0;
      // eight entries at a time, so the loads in flight stay within registers
#pragma unroll
      for (int k = 0; k < NC; ++k) {
        const double hv = H[k <= j ? rj + k : pk(k, j)];
        if (k & 1) s1 = fma(hv, rr[k], s1);
        else s0 = fma(hv, rr[k], s0);
        if ((k & 7) == 7) __builtin_amdgcn_sched_barrier(0);
      }
      t[h] = s0 + s1;
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  wave_sync();
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int j = (threadIdx.x & 31) + 32 * h;
    if (h * 32 < NC && j < NC) z[j] = t[h];
  }
  wave_sync();
}

// FP64 pass over one fit's samples by a half wave (modes as for pass());
// RESIDUAL also returns min_i Q(u_i) through qmin.  Each lane takes one
// sample per step with the next NS samples' inputs in flight (three in the
// FP64 form, whose kernel has the registers; two in the mixed forms); the fit's
// accumulators stay in registers (a half wave per fit leaves each lane the
// register room of two resident waves per SIMD).  The monomials of top degree
// are formed again, from their parents, for the accumulation rather than kept
// live through the dot products.  The vector v (the half's own, in LDS) is
// read where it is used.
template <int V, int D, int MODE, int NS = 2>
__device__ double half_pass(const FitArgs& a, int64_t s0, int64_t m, const double* v, double* out,
                            double* qmin, double* red) {
  using S = Shape<V, D>;
  constexpr bool ACC = MODE != PASS_CHECK;
  constexpr int NLOW = binom(V + code_dmax(D) - 1, code_dmax(D) - 1);   // monomials of degree < the top
  const uint32_t hl = threadIdx.x & 31;
  double acc[ACC ? S::NC : 1];
#pragma unroll
  for (int j = 0; j < (ACC ? S::NC : 1); ++j) acc[j] = 0.0;
  double ss = 0.0, qm = INFINITY;
  const SampleSrc<V> src(a, s0, m);
  auto process = [&](const SampleIn<V>& t, bool valid) {
    double mo[S::NM];
    monomials<V, D, double>(t.u, mo);
    int zero;
    asm volatile("v_mov_b32 %0, 0" : "=v"(zero));
    const double* vv = v + zero;
    double n0 = 0.0, n1 = 0.0, q0 = 0.0, q1 = 0.0;
#pragma unroll
    for (int j = 0; j < S::NA; ++j) {
      if (j & 1) n1 = fma(vv[j], mo[j], n1);
      else n0 = fma(vv[j], mo[j], n0);
    }
    // numerator and denominator coefficients are read in two groups so that
    // at most half of the vector is in registers at a time
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 1; j < S::NQ; ++j) {
      if (j & 1) q1 = fma(vv[S::NA + j - 1], mo[j], q1);
      else q0 = fma(vv[S::NA + j - 1], mo[j], q0);
    }
    const double qv = q0 + q1;
    const double dot = fma(-t.y, qv, n0 + n1);   // a_i . v
    double w = (MODE == PASS_PRODUCT) ? dot : t.y - dot;
    w = valid ? w : 0.0;
    ss = fma(w, w, ss);
    if constexpr (MODE != PASS_PRODUCT) qm = valid ? fmin(qm, 1.0 + qv) : qm;
    if constexpr (ACC) {
      double u2[V];
#pragma unroll
      for (int k = 0; k < V; ++k) {
        u2[k] = t.u[k];
        asm volatile("" : "+v"(u2[k]));   // an opaque copy: recompute, do not keep
      }
      monomials_tail<V, D, NLOW, double>(u2, mo);
      const double wy = -t.y * w;
#pragma unroll
      for (int j = 0; j < S::NA; ++j) acc[j] = fma(w, mo[j], acc[j]);
#pragma unroll
      for (int j = 1; j < S::NQ; ++j) acc[S::NA + j - 1] = fma(wy, mo[j], acc[S::NA + j - 1]);
    }
  };
  // two sets of NS slots used in turn: the next samples load into one set
  // while the other set's are processed, so every slot keeps its registers
  // and the loop's back edge moves none (such a move waits for every load in
  // flight)
  SampleIn<V> sa[NS], sb[NS];
  if (src.m > 0) {
#pragma unroll
    for (int k = 0; k < NS; ++k) src.load(sa[k], hl + 32u * k);
  }
#pragma unroll 1
  for (uint32_t b0 = 0; b0 < src.m; b0 += 64u * NS) {
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      src.load(sb[k], b0 + 32u * (NS + k) + hl);
      process(sa[k], b0 + 32u * k + hl < src.m);
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      src.load(sa[k], b0 + 32u * (2 * NS + k) + hl);
      process(sb[k], b0 + 32u * (NS + k) + hl < src.m);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  if constexpr (ACC) half_reduce_vec<S::NC>(acc, out, red);
  if constexpr (MODE != PASS_PRODUCT) *qmin = -half_max(-qm);
  wave_sync();
  return half_sum(ss);
}


// ---------------------------------------------------------------------------
// FP64 Gram by weighted moments (VALU)
// ---------------------------------------------------------------------------
// Each entry of the augmented Gram of a monomial design is a weighted moment
// sum_i w(i) m_e(u_i) (see MomentShape).  A workgroup stages 256 samples and
// their weights in LDS; each wave accumulates one static group of
// moment-weight pairs per pass (each lane over its share of the samples),
// builds every monomial of the group from per-sample power tables, and the
// packed Gram is scattered from the reduced moments through a host-built map.
// Which moment-weight pairs each wave accumulates: a table per shape
// (rp_moment_groups.inc, written by gen_moment_groups.py) assigns them so
// that the waves' work per sample -- one FMA per pair plus the multiplies
// that form their monomials -- is even within each pass, with each wave's
// monomials formed in its own variable order (products of equal leading
// factors shared).  Without a table the pairs go in index order, PL per wave.
template <int V, int D, bool GN>
struct MomGroups {
  static constexpr bool kHas = false;
  static constexpr int kNWV = 0, kNG = 0, kPL = 0;
};
#include "rp_moment_groups.inc"

template <int V, int D, bool GN>
struct MomCfg {
  using MS = MomentShape<V, D, GN>;
  static constexpr int NW = GN ? 6 : 3;
  using T = MomGroups<V, D, GN>;
  static constexpr int NWV = T::kHas ? T::kNWV : MS::NWV;   // waves per workgroup
  static constexpr int NT = 64 * NWV;              // threads per workgroup
  static constexpr int CHM = NT;                   // staged samples per chunk
  // resident waves per SIMD asked of the compiler: four (two eight-wave
  // workgroups per compute unit) where the estimated live set -- the
  // accumulators, the power table, the weights and about 30 more -- fits
  // (a few spills outside the sample loop are accepted), else three or two;
  // two for four-wave groups of more than 64 pairs per lane, which also
  // prefetch the next chunk's inputs
  static constexpr int PL = T::kHas ? T::kPL : MS::PL;          // pairs per wave
  static constexpr int NGROUP = T::kHas ? T::kNG : MS::NGROUP;   // waves over all passes
  static constexpr int NPASS = NGROUP / NWV;
  static_assert(NPASS * NWV == NGROUP && NGROUP * PL >= MS::NPAIR, "moment groups cover every pair");
  static constexpr int PLP = (PL + 3) / 4 * 4;
  static constexpr int EST = 2 * PL + 4 * V * code_dmax(D) + 2 * NW + 30;
  static constexpr int MINW = NWV == 4 ? (PL > 64 ? 2 : 3) : MS::NPAIR > 1000 ? 2 : EST <= 152 ? 4 : 3;
  static constexpr bool PREFETCH = NWV == 8 || (GN && PL > 64);
  static constexpr MonoBig<V, 2 * code_dmax(D)> E2 = make_mono_big<V, 2 * code_dmax(D)>();
};

template <int V, int D, bool GN, int G, int J>
constexpr int mom_group_pair() {
  if constexpr (MomGroups<V, D, GN>::kHas) return MomGroups<V, D, GN>::kPair[G][J];
  else return G * MomCfg<V, D, GN>::PL + J;
}
template <int V, int D, bool GN, int G, int K>
constexpr int mom_group_var() {
  if constexpr (MomGroups<V, D, GN>::kHas) {
    if constexpr (K < V) return MomGroups<V, D, GN>::kOrder[G][K];
    else return K;
  } else {
    return K;
  }
}
template <int V, int D, bool GN>
__device__ __forceinline__ int mom_slot(int p) {
  if constexpr (MomGroups<V, D, GN>::kHas) return MomGroups<V, D, GN>::kSlot[p];
  else return p;
}

template <int V, int D, bool GN>
constexpr int mom_e_of(int p) {
  int e = 0, w = 0;
  moment_pair_of<GN>(p, binom(V + code_dmax(D), code_dmax(D)), V, e, w);
  return e;
}
template <int V, int D, bool GN>
constexpr int mom_w_of(int p) {
  int e = 0, w = 0;
  moment_pair_of<GN>(p, binom(V + code_dmax(D), code_dmax(D)), V, e, w);
  return w;
}

template <int V, int D, bool GN, int G, int P, int J>
__device__ __forceinline__ void mom_acc_one(double* acc, const double (&pw)[kMaxV][2 * kMaxD + 1],
                                            const double* W) {
  using C = MomCfg<V, D, GN>;
  if constexpr (P >= 0 && P < C::MS::NPAIR) {
    constexpr int e = mom_e_of<V, D, GN>(P);
    constexpr int w = mom_w_of<V, D, GN>(P);
    // the group's variable order: products of equal leading factors are
    // formed once and shared between the group's monomials
    constexpr int k0 = mom_group_var<V, D, GN, G, 0>(), k1 = mom_group_var<V, D, GN, G, 1>();
    constexpr int k2 = mom_group_var<V, D, GN, G, 2>(), k3 = mom_group_var<V, D, GN, G, 3>();
    constexpr int a0 = C::E2.e[e][k0], a1 = C::E2.e[e][k1], a2 = C::E2.e[e][k2], a3 = C::E2.e[e][k3];
    double mon = 1.0;
    if constexpr (a0 > 0) mon *= pw[k0][a0];
    if constexpr (a1 > 0) mon *= pw[k1][a1];
    if constexpr (a2 > 0) mon *= pw[k2][a2];
    if constexpr (a3 > 0) mon *= pw[k3][a3];
    acc[J] = fma(W[w], mon, acc[J]);
  }
}

template <int V, int D, bool GN, int G, int... J>
__device__ __forceinline__ void mom_acc_group(double* acc, const double (&pw)[kMaxV][2 * kMaxD + 1],
                                              const double* W, std::integer_sequence<int, J...>) {
  using C = MomCfg<V, D, GN>;
  (mom_acc_one<V, D, GN, G, mom_group_pair<V, D, GN, G, J>(), J>(acc, pw, W), ...);
}

// One wave, one chunk of staged samples, moment group G.
template <int V, int D, bool GN, int G>
__device__ __forceinline__ void mom_chunk(double* acc, const double* su, const double* sw, int cnt) {
  using C = MomCfg<V, D, GN>;
  const int lane = threadIdx.x & 63;
#pragma unroll 1
  for (int i = lane; i < cnt; i += 64) {   // cnt: valid samples of the chunk
    double pw[kMaxV][2 * kMaxD + 1];
#pragma unroll
    for (int k = 0; k < V; ++k) {
      const double uk = su[k * C::CHM + i];
      pw[k][0] = 1.0;
      pw[k][1] = uk;
#pragma unroll
      for (int t = 2; t <= 2 * code_dmax(D); ++t) pw[k][t] = pw[k][t - 1] * uk;
    }
    double W[C::NW];
#pragma unroll
    for (int w = 0; w < C::NW; ++w) W[w] = sw[w * C::CHM + i];
    mom_acc_group<V, D, GN, G>(acc, pw, W, std::make_integer_sequence<int, C::PL>{});
  }
}

template <int V, int D, bool GN>
struct MomShared {
  using C = MomCfg<V, D, GN>;
  // the coefficients first: every staging thread reads all of them, and at
  // the bottom of LDS their addresses fit the immediate offsets of paired
  // LDS reads (no address arithmetic per read)
  double c[Shape<V, D>::NC];
  union {
    struct {
      double su[V * C::CHM];
      double sw[C::NW * C::CHM];
    } st;                                // staged chunk (accumulation phase)
    double red[C::NWV][C::PLP * 17];     // lane partials (reduction phase)
  };
  double mom[C::NGROUP * C::PL];
  int flag_nonfinite;
};

// Stage one chunk: inputs and weights of samples [c0, c0 + CHM).
template <int V, int D, bool GN>
__device__ __forceinline__ void mom_stage(const SampleIn<V>& in, int64_t m, int64_t c0,
                                          MomShared<V, D, GN>& sh, bool& bad) {
  using C = MomCfg<V, D, GN>;
  using S = Shape<V, D>;
  const int t = threadIdx.x;
  const bool valid = c0 + t < m;
  double u[V];
  const double y = in.y;
  bool fin = isfinite(y);
#pragma unroll
  for (int k = 0; k < V; ++k) {
    fin = fin && isfinite(in.u[k]);
    u[k] = valid ? in.u[k] : 0.0;
  }
  bad = bad || (valid && !fin);
#pragma unroll
  for (int k = 0; k < V; ++k) sh.st.su[k * C::CHM + t] = u[k];
  if constexpr (!GN) {
    sh.st.sw[0 * C::CHM + t] = valid ? 1.0 : 0.0;
    sh.st.sw[1 * C::CHM + t] = valid ? y : 0.0;
    sh.st.sw[2 * C::CHM + t] = valid ? y * y : 0.0;
  } else {
    // N and Q by nested multiplication with the coefficients read where they
    // are used (opaque offset: not hoisted out of the chunk loop, where they
    // would sit beside the fit's accumulators)
    int zero;
    asm volatile("v_mov_b32 %0, 0" : "=v"(zero));
    double n, q;
    const double* cc = sh.c + zero;
    horner_nq<V, D>(u, [&](int j) { return cc[j]; }, n, q);
    const double iq = valid ? 1.0 / q : 0.0;
    const double f = n * iq;   // one division per sample
    const double r = valid ? y - f : 0.0;
    const double iq2 = iq * iq;
    sh.st.sw[0 * C::CHM + t] = iq2;
    sh.st.sw[1 * C::CHM + t] = iq2 * f;
    sh.st.sw[2 * C::CHM + t] = iq2 * f * f;
    sh.st.sw[3 * C::CHM + t] = iq * r;
    sh.st.sw[4 * C::CHM + t] = iq * f * r;
    sh.st.sw[5 * C::CHM + t] = r * r;
  }
}

template <int V, int D, bool GN, int G0, int... W>
__device__ __forceinline__ void mom_chunk_dispatch(int wave, double* acc, const double* su,
                                                   const double* sw, int cnt,
                                                   std::integer_sequence<int, W...>) {
  ((wave == W ? mom_chunk<V, D, GN, G0 + W>(acc, su, sw, cnt) : (void)0), ...);
}

template <int V, int D, bool GN, int Q>
__device__ void mom_pass(const FitArgs& a, int64_t s0, int64_t m, MomShared<V, D, GN>& sh, bool& bad) {
  using C = MomCfg<V, D, GN>;
  const int wave = threadIdx.x >> 6;
  double acc[C::PL];
#pragma unroll
  for (int j = 0; j < C::PL; ++j) acc[j] = 0.0;
  // PREFETCH: the next chunk's inputs are loaded while the current one is
  // accumulated (costs registers: used where the workgroup's own waves do
  // not hide the load latency)
  const SampleSrc<V> src(a, s0, m);
  SampleIn<V> in;
  if (C::PREFETCH && m > 0) src.load(in, threadIdx.x);
  for (int64_t c0 = 0; c0 < m; c0 += C::CHM) {
    if (!C::PREFETCH) src.load(in, (uint32_t)c0 + threadIdx.x);
    mom_stage<V, D, GN>(in, m, c0, sh, bad);
    if (C::PREFETCH && c0 + C::CHM < m) src.load(in, (uint32_t)(c0 + C::CHM) + threadIdx.x);
    __syncthreads();
    // wave-uniform choice of this wave's static moment group
    const int cnt = (int)(m - c0 < C::CHM ? m - c0 : C::CHM);
    mom_chunk_dispatch<V, D, GN, C::NWV * Q>(wave, acc, sh.st.su, sh.st.sw, cnt,
                                             std::make_integer_sequence<int, C::NWV>{});
    __syncthreads();
  }
  wave_reduce_vec<C::PL>(acc, sh.mom + (C::NWV * Q + wave) * C::PL, sh.red[wave]);
  __syncthreads();   // the partials alias the staging area of the next pass
}

template <int V, int D, bool GN, int... Q>
__device__ __forceinline__ void mom_all_passes(const FitArgs& a, int64_t s0, int64_t m,
                                               MomShared<V, D, GN>& sh, bool& bad,
                                               std::integer_sequence<int, Q...>) {
  (mom_pass<V, D, GN, Q>(a, s0, m, sh, bad), ...);
}

template <int V, int D, bool GN>
__global__ __launch_bounds__((MomCfg<V, D, GN>::NT), (MomCfg<V, D, GN>::MINW)) void k_gram_mom(FitArgs a, double* gws,
                                                                   const int64_t* gofs, int* gflag) {
  using C = MomCfg<V, D, GN>;
  using S = Shape<V, D>;
  constexpr int NPK = S::NU * (S::NU + 1) / 2;
  __shared__ MomShared<V, D, GN> sh;
  const int f = a.ids[blockIdx.x];
  if constexpr (GN) {
    if (a.lm_state && a.lm_first) lm_state_init(a, f);   // see k_gram
    else if (a.lm_state && (a.lm_state[f] != 0 || a.lm_rejects[f] > 0)) return;
  }
  const int64_t s0 = a.sample_off[f];
  const int64_t m = a.sample_off[f + 1] - s0;
  if (threadIdx.x == 0) sh.flag_nonfinite = 0;
  if constexpr (GN) {
    const double* c = a.coef + a.coef_off[f];
    for (int j = threadIdx.x; j < S::NC; j += C::NT) sh.c[j] = c[j];
  }
  __syncthreads();
  bool bad = false;
  mom_all_passes<V, D, GN>(a, s0, m, sh, bad, std::make_integer_sequence<int, C::NPASS>{});
  if (bad) atomicOr(&sh.flag_nonfinite, 1);
  __syncthreads();
  double* out = gws + gofs[f];
  for (int e = threadIdx.x; e < NPK; e += C::NT) {
    const int mp = a.mom_map[e];
    const double v = sh.mom[mom_slot<V, D, GN>(mp & 0x3fffffff)];
    out[e] = (mp >> 30) & 1 ? -v : v;
  }
  if (threadIdx.x == 0) gflag[f] = sh.flag_nonfinite;
}

// ---------------------------------------------------------------------------
// FP64 Gram of the linear problem by weighted moments, inputs streamed into
// LDS by buffer loads
// ---------------------------------------------------------------------------
// The linear problem's weights (1, y, y^2) need no per-sample work, so the
// raw inputs go straight from HBM into LDS with buffer loads that write LDS
// (no registers, no staging pass): three chunk buffers, the loads of chunk
// c+2 issued as chunk c is accumulated, one barrier per chunk.  The buffer
// loads are range checked against the fit's sample count (samples past the
// end read as zero).  The compiler does not track these loads, so the waits
// on them are explicit (vmcnt: every older memory operation of the thread
// is complete, so other memory operations can only make them stricter).

template <int V, int D>
struct MomLinCfg {
  using C = MomCfg<V, D, false>;
  static constexpr int NWV = C::NWV, NT = C::NT;
  static constexpr int CHM = 256;                        // samples per chunk
  static constexpr int NA = V + 1;                       // streamed arrays: x_1..x_V, y
  static constexpr int BLK = 32;                         // doubles per wave load (4 B per lane)
  static constexpr int BPA = CHM / BLK;                  // wave loads per array and chunk
  static constexpr int NI = NA * BPA;                    // wave loads per chunk
  static constexpr int NPW = (NI + NWV - 1) / NWV;       // loads per wave and chunk (at most)
  static constexpr int NPW_MIN = NI / NWV;               // (at least)
  static constexpr int NBUF = 3;
  static_assert(2 * NPW <= 63, "two chunks in flight fit the vmcnt counter");
  // no register spills: a spill reload waits for every older memory
  // operation, the streamed loads included, and would drain the pipeline
  static constexpr int MINW = C::MINW;
};

template <int V, int D>
struct MomLinShared {
  using L = MomLinCfg<V, D>;
  using C = MomCfg<V, D, false>;
  union {
    double buf[L::NBUF][L::NA][L::CHM];   // streamed chunks (accumulation phase)
    double red[C::NWV][C::PLP * 17];      // lane partials (reduction phase)
  };
  double mom[C::NGROUP * C::PL];
  int flag_nonfinite;
};


// Workgroup barrier that the compiler may not move LDS accesses across (no
// memory fence: the streamed loads are waited for explicitly).
__device__ __forceinline__ void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

template <int V, int D, int G>
__device__ __forceinline__ void mom_lin_chunk(double* acc, const double* b, int cnt) {
  using L = MomLinCfg<V, D>;
  using C = MomCfg<V, D, false>;
  const int lane = threadIdx.x & 63;
#pragma unroll 1
  for (int i = lane; i < L::CHM; i += 64) {
    double pw[kMaxV][2 * kMaxD + 1];
#pragma unroll
    for (int k = 0; k < V; ++k) {
      const double uk = b[k * L::CHM + i];
      pw[k][0] = 1.0;
      pw[k][1] = uk;
#pragma unroll
      for (int t = 2; t <= 2 * code_dmax(D); ++t) pw[k][t] = pw[k][t - 1] * uk;
    }
    const double y = b[V * L::CHM + i];
    const bool valid = i < cnt;
    const double W[C::NW] = {valid ? 1.0 : 0.0, y, y * y};
    mom_acc_group<V, D, false, G>(acc, pw, W, std::make_integer_sequence<int, C::PL>{});
  }
}

template <int V, int D, int G0, int... W>
__device__ __forceinline__ void mom_lin_dispatch(int wave, double* acc, const double* b, int cnt,
                                                 std::integer_sequence<int, W...>) {
  ((wave == W ? mom_lin_chunk<V, D, G0 + W>(acc, b, cnt) : (void)0), ...);
}

template <int V, int D, int Q>
__device__ void mom_lin_pass(const FitArgs& a, int64_t s0, int64_t m, MomLinShared<V, D>& sh,
                             bool& bad) {
  using L = MomLinCfg<V, D>;
  using C = MomCfg<V, D, false>;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // the same index in a scalar register for the loads: the buffer descriptor
  // a wave loads through must be uniform, which the compiler then knows
  const int swave = __builtin_amdgcn_readfirstlane(wave);
  double acc[C::PL];
#pragma unroll
  for (int j = 0; j < C::PL; ++j) acc[j] = 0.0;
  const int nch = (int)((m + L::CHM - 1) / L::CHM);
  auto issue = [&](int c) {
    // lane offsets recomputed at every issue (opaque zero): kept live across
    // the chunk loop they would be spilled, and a spill reload waits for
    // every streamed load in flight
    int zero;
    asm volatile("v_mov_b32 %0, 0" : "=v"(zero));
    const uint32_t lane4 = (uint32_t)(lane + zero) * 4u;
#pragma unroll
    for (int t = 0; t < L::NPW; ++t) {
      const int q = swave + t * L::NWV;   // wave-uniform
      if (L::NI % L::NWV == 0 || q < L::NI) {
        const int k = q / L::BPA, blk = q % L::BPA;
        // descriptor of array k over the fit's samples, built from uniform values
        const double* base = k < V ? a.x + (int64_t)k * a.ldx + s0 : a.y + s0;
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)(m * 8), 0x00020000);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(
            rs, (lds_void_ptr)&sh.buf[c % L::NBUF][k][blk * L::BLK], 4,
            (uint32_t)c * (L::CHM * 8u) + (uint32_t)blk * (L::BLK * 8u) + lane4, 0, 0, 0);
      }
    }
  };
  if (nch > 0) issue(0);
  if (nch > 1) issue(1);
  for (int c = 0; c < nch; ++c) {
    if (c + 1 < nch) wait_vmcnt<L::NPW_MIN>();   // chunk c landed, chunk c+1 may be in flight
    else wait_vmcnt<0>();
    lds_barrier();                               // every wave's share of chunk c landed; chunk c-1 read
    if (c + 2 < nch) issue(c + 2);               // into the buffer of chunk c-1
    const int cnt = (int)(m - (int64_t)c * L::CHM < L::CHM ? m - (int64_t)c * L::CHM : L::CHM);
    if (cnt < L::CHM) {
      // the ragged last chunk: whatever the range-checked loads left past
      // the end is replaced by zeros (zero samples add nothing to a moment)
      double* b = &sh.buf[c % L::NBUF][0][0];
      for (int e = threadIdx.x; e < L::NA * L::CHM; e += L::NT)
        if ((e % L::CHM) >= cnt) b[e] = 0.0;
      lds_barrier();
    }
    if (Q == 0 && (int)threadIdx.x < cnt) {
      // non-finite inputs: each thread checks one sample of the chunk (the
      // first pass only; later passes read the same samples)
      const double* b = &sh.buf[c % L::NBUF][0][0];
      bool fin = isfinite(b[V * L::CHM + threadIdx.x]);
#pragma unroll
      for (int k = 0; k < V; ++k) fin = fin && isfinite(b[k * L::CHM + threadIdx.x]);
      bad = bad || !fin;
    }
    mom_lin_dispatch<V, D, C::NWV * Q>(wave, acc, &sh.buf[c % L::NBUF][0][0], cnt,
                                       std::make_integer_sequence<int, C::NWV>{});
  }
  lds_barrier();   // every wave done with the buffers, which the partials alias
  wave_reduce_vec<C::PL>(acc, sh.mom + (C::NWV * Q + wave) * C::PL, sh.red[wave]);
  __syncthreads();   // the next pass streams into the buffers again
}

template <int V, int D, int... Q>
__device__ __forceinline__ void mom_lin_all_passes(const FitArgs& a, int64_t s0, int64_t m,
                                                   MomLinShared<V, D>& sh, bool& bad,
                                                   std::integer_sequence<int, Q...>) {
  (mom_lin_pass<V, D, Q>(a, s0, m, sh, bad), ...);
}

template <int V, int D>
__global__ __launch_bounds__((MomCfg<V, D, false>::NT), (MomLinCfg<V, D>::MINW))
void k_gram_mom_lin(FitArgs a, double* gws, const int64_t* gofs, int* gflag) {
  using C = MomCfg<V, D, false>;
  using S = Shape<V, D>;
  constexpr int NPK = S::NU * (S::NU + 1) / 2;
  __shared__ MomLinShared<V, D> sh;
  const int f = a.ids[blockIdx.x];
  const int64_t s0 = a.sample_off[f];
  const int64_t m = a.sample_off[f + 1] - s0;
  if (threadIdx.x == 0) sh.flag_nonfinite = 0;
  __syncthreads();
  bool bad = false;
  mom_lin_all_passes<V, D>(a, s0, m, sh, bad, std::make_integer_sequence<int, C::NPASS>{});
  if (bad) atomicOr(&sh.flag_nonfinite, 1);
  __syncthreads();
  double* out = gws + gofs[f];
  for (int e = threadIdx.x; e < NPK; e += C::NT) {
    const int mp = a.mom_map[e];
    const double v = sh.mom[mom_slot<V, D, false>(mp & 0x3fffffff)];
    out[e] = (mp >> 30) & 1 ? -v : v;
  }
  if (threadIdx.x == 0) gflag[f] = sh.flag_nonfinite;
}

// ---------------------------------------------------------------------------
// split form, solve: block sweep of every fit's Gram (one wave per fit)
// ---------------------------------------------------------------------------
template <int NC>
struct SweepShared {
  double col[Blocks<NC>::NP];            // pivot column
  double p[NC];                          // (both first: small LDS offsets)
  double gs[(NC + 1) * (NC + 2) / 2];   // the fit's packed augmented Gram
};

// Equilibrate and sweep the augmented Gram of each fit; write the unscaled
// solution to coef and G^-1 of the kept unknowns over the fit's Gram in gws
// (the refinement kernel's preconditioner); gflag keeps bit 0 (non-finite
// input) and receives the count of dropped pivots above it.
template <int V, int D, int PREC>
__global__ __launch_bounds__(64, 4) void k_sweep(FitArgs a, double* gws, const int64_t* gofs,
                                                 int* gflag) {
  using S = Shape<V, D>;
  constexpr int NC = S::NC, NU = S::NU;
  constexpr int NPK = NU * (NU + 1) / 2;
  static_assert(NC <= kWaveSolveMaxNC, "wave solver limited to small models");
  __shared__ SweepShared<NC> w;
  const int lane = threadIdx.x;
  const int f = a.ids[blockIdx.x];
  double* coef = a.coef + a.coef_off[f];
  if (gflag[f] & 1) {
    for (int j = lane; j < NC; j += 64) coef[j] = __builtin_nan("");
    if (lane == 0) {
      a.status[f] = RP_FIT_NONFINITE_INPUT;
      if (a.resid) a.resid[f] = __builtin_nan("");
      if (a.iters) a.iters[f] = 0;
    }
    return;
  }
  double* g = gws + gofs[f];
  for (int e = lane; e < NPK; e += 64) w.gs[e] = g[e];
  wave_sync();
  // the mixed forms add a small shift so the low-precision Gram is positive definite
  Blocks<NC> B;
  block_load<NC>(w.gs, B, 1.0, PREC == RP_FP64 ? 0.0 : 0x1p-20, w.col);
  const uint64_t drop = block_sweep<NC>(B, w.col, PREC == RP_FP64 ? kTauColSq : 0.0);
  block_solution<NC>(B, drop, coef);
  block_store_inverse<NC>(B, drop, g);
  if (lane == 0) gflag[f] = __builtin_popcountll(drop) << 1;
}

// ---------------------------------------------------------------------------
// split form, refinement over the samples (one wave per fit)
// ---------------------------------------------------------------------------
template <int NC>
struct RefineShared {
  double c[2][NC], r[2][NC], z[2][NC], p[2][NC], q[2][NC];   // one set per half wave
  double red[(NC + 1) / 2 * 66];        // row partial sums of both halves
  double pcg[2][2];                     // per half: first and smallest CG correction
};

// Two fits per wave (lanes 0-31 and 32-63; nfits is the launch's fit count).
// FP64 form: iterative refinement c += G^-1 A^T (b - A c); the last pass also
// yields min Q and, with r = A^T (b - A c) and z = G^-1 r, the residual of the
// corrected coefficients as ||b - A c||^2 - r.z.  Mixed forms: conjugate
// gradients on A^T A c = A^T b preconditioned by the inverse of the
// low-precision Gram, then one check pass.
template <int V, int D, int PREC>
__global__ __launch_bounds__(64, 2) void k_refine_lin(FitArgs a, const double* gws,
                                                      const int64_t* gofs, const int* gflag,
                                                      int nfits) {
  using S = Shape<V, D>;
  constexpr int NC = S::NC;
  __shared__ RefineShared<NC> sh;
  const int lane = threadIdx.x, h = lane >> 5, hl = lane & 31;
  const int slot = 2 * blockIdx.x + h;
  if (slot >= nfits) return;
  const int f = a.ids[slot];
  const int flags = gflag[f];
  if (flags & 1) return;   // non-finite input: the sweep kernel wrote the outputs
  const int ndrop = flags >> 1;
  const int64_t s0 = a.sample_off[f];
  const int64_t m = a.sample_off[f + 1] - s0;
  double* coef = a.coef + a.coef_off[f];
  const double* H = gws + gofs[f];
  double* c = sh.c[h];
  double* r = sh.r[h];
  double* z = sh.z[h];
  for (int j = hl; j < NC; j += 32) c[j] = coef[j];
  wave_sync();

  int it = 0;
  double last_rel = 0.0;
  double resid = __builtin_nan("");
  double qmin = 1.0;
  bool checked = false;
  if constexpr (PREC == RP_FP64) {
    double ss = 0.0, rz = 0.0, qm = 1.0;
    for (it = 0; it < a.max_refine;) {
      ss = half_pass<V, D, PASS_RESIDUAL, 3>(a, s0, m, c, r, &qm, sh.red);   // three in flight
      half_apply_inverse<NC>(H, r, z);
      for (int j = hl; j < NC; j += 32) c[j] += z[j];
      wave_sync();
      ++it;
      rz = half_dot<NC>(r, z);
      const double dn = half_maxabs<NC>(z), cn = half_maxabs<NC>(c);
      last_rel = cn > 0.0 ? dn / cn : dn;
      if (dn <= a.stop_rel * cn) break;
    }
    if (it > 0) {
      resid = sqrt(fmax(ss - rz, 0.0));
      qmin = qm;
      checked = true;
    }
  } else {
    double* p = sh.p[h];
    double* q = sh.q[h];
    double qdummy;
    half_pass<V, D, PASS_RESIDUAL>(a, s0, m, c, r, &qdummy, sh.red);
    half_apply_inverse<NC>(H, r, z);
    for (int j = hl; j < NC; j += 32) p[j] = z[j];
    wave_sync();
    double rz = half_dot<NC>(r, z);
    double& dn1 = sh.pcg[h][0];
    double& dnmin = sh.pcg[h][1];
    dnmin = INFINITY;
    bool reached = false;   // as in k_fit: a CG stopped short is re-solved in FP64
    for (it = 0; it < a.max_refine;) {
      half_pass<V, D, PASS_PRODUCT>(a, s0, m, p, q, nullptr, sh.red);
      const double pq = half_dot<NC>(p, q);
      const double alpha = pq > 0.0 ? rz / pq : 0.0;
      for (int j = hl; j < NC; j += 32) {
        c[j] = fma(alpha, p[j], c[j]);
        r[j] = fma(-alpha, q[j], r[j]);
      }
      wave_sync();
      ++it;
      const double dn = fabs(alpha) * half_maxabs<NC>(p), cn = half_maxabs<NC>(c);
      last_rel = cn > 0.0 ? dn / cn : dn;
      if (dn <= a.tol * cn) { reached = true; break; }
      if (!(pq > 0.0)) break;
      if (pcg_hopeless(it, a.max_refine, dn, cn, a.tol, dn1, dnmin)) break;
      half_apply_inverse<NC>(H, r, z);
      const double rz2 = half_dot<NC>(r, z);
      const double beta = rz > 0.0 ? rz2 / rz : 0.0;
      rz = rz2;
      for (int j = hl; j < NC; j += 32) p[j] = fma(beta, p[j], z[j]);
      wave_sync();
    }
    if (!reached) last_rel = INFINITY;
  }
  if (!a.check_q) {
    resid = __builtin_nan("");
    qmin = 1.0;
  } else if (!checked) {
    resid = sqrt(half_pass<V, D, PASS_CHECK>(a, s0, m, c, nullptr, &qmin, sh.red));
  }
  for (int j = hl; j < NC; j += 32) coef[j] = c[j];
  if (hl == 0) {
    int st = RP_FIT_OK;
    if (m < NC) st = RP_FIT_UNDERDETERMINED;
    else if (ndrop > 0) st = RP_FIT_RANK_DEFICIENT;
    else if (!(last_rel <= sqrt(a.tol))) st = RP_FIT_NOT_CONVERGED;
    else if (!(qmin > 0.0)) st = RP_FIT_Q_NONPOSITIVE;
    a.status[f] = st;
    if (a.resid) a.resid[f] = resid;
    if (a.iters) a.iters[f] = it;
    flag_for_resolve(a, f, st);
  }
}

// ---------------------------------------------------------------------------
// Levenberg-Marquardt on the true loss, split form (one wave per fit)
// ---------------------------------------------------------------------------

// sum_i (N_i/Q_i - y_i)^2 over one fit's samples by one wave; c in LDS.  One
// sample per lane and step, two samples' inputs in flight.
template <int V, int D>
__device__ double wave_true_loss(const FitArgs& a, int64_t s0, int64_t m, const double* c,
                                 bool* finite_in) {
  using S = Shape<V, D>;
  const uint32_t lane = threadIdx.x & 63;
  double ss = 0.0;
  bool ok = true;
  const SampleSrc<V> src(a, s0, m);
  // one fit per wave: the coefficients are equal on every lane, so they are
  // moved to scalar registers once and the FMAs take them as scalar operands
  // (no LDS read per sample)
  double cz[S::NC];
#pragma unroll
  for (int j = 0; j < S::NC; ++j) cz[j] = uniform_d(c[j]);
  auto process = [&](const SampleIn<V>& t, bool valid) {
    double n, q;
    horner_nq<V, D>(t.u, [&](int j) { return cz[j]; }, n, q);
    const double r = n / q - t.y;
    ss = valid ? fma(r, r, ss) : ss;
    bool fin = isfinite(t.y);
#pragma unroll
    for (int k = 0; k < V; ++k) fin = fin && isfinite(t.u[k]);
    ok = ok && (fin || !valid);
  };
  // two sets of two slots used in turn (as in the refinement pass): the
  // loop's back edge moves no register, so it waits for no load
  SampleIn<V> sa[2], sb[2];
  if (src.m > 0) {
    src.load(sa[0], lane);
    src.load(sa[1], lane + 64u);
  }
#pragma unroll 1
  for (uint32_t b0 = 0; b0 < src.m; b0 += 256u) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      src.load(sb[k], b0 + 128u + 64u * k + lane);
      process(sa[k], b0 + 64u * k + lane < src.m);
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      src.load(sa[k], b0 + 256u + 64u * k + lane);
      process(sb[k], b0 + 128u + 64u * k + lane < src.m);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  if (finite_in) *finite_in = !__any(!ok);   // every lane's samples finite
  return wave_sum_dpp(ss);
}

// Per-fit LM state for a call that runs no iteration (max_iter = 0): the loss
// at the given coefficients by a pass over the samples (with_loss).  With
// iterations the first Jacobian Gram sets the state (lm_state_init) and the
// current loss comes from the corner of each iteration's Gram (sum r^2 at the
// coefficients it was formed at).
template <int V, int D>
__global__ __launch_bounds__(64, 4) void k_lm_init(FitArgs a, int with_loss) {
  using S = Shape<V, D>;
  __shared__ double c[S::NC];
  const int lane = threadIdx.x;
  const int f = a.ids[blockIdx.x];
  double loss = __builtin_nan("");
  bool finite_in = true;
  if (with_loss) {
    const int64_t s0 = a.sample_off[f];
    const int64_t m = a.sample_off[f + 1] - s0;
    const double* cg = a.coef + a.coef_off[f];
    for (int j = lane; j < S::NC; j += 64) c[j] = cg[j];
    wave_sync();
    loss = wave_true_loss<V, D>(a, s0, m, c, &finite_in);
  }
  if (lane == 0) {
    a.lm_loss[f] = loss;
    a.lm_lambda[f] = 0.0;
    a.lm_state[f] = finite_in ? LM_ACTIVE : LM_NONFINITE;
    a.lm_rejects[f] = 0;
    if (a.iters) a.iters[f] = 0;
  }
}

// Status and residual of fit f from its final LM state st (one thread).
template <int V, int D>
__device__ __forceinline__ void lm_write_final(const FitArgs& a, int f, int st) {
  const int64_t m = a.sample_off[f + 1] - a.sample_off[f];
  int out = st == LM_CONVERGED ? RP_FIT_OK : RP_FIT_NOT_CONVERGED;
  if (st == LM_NONFINITE) out = RP_FIT_NONFINITE_INPUT;
  else if (m < Shape<V, D>::NC) out = RP_FIT_UNDERDETERMINED;
  a.status[f] = out;
  a.resid[f] = st == LM_NONFINITE ? __builtin_nan("") : a.lm_loss[f];
}

// One damped Gauss-Newton step per active fit: (J^T J + lambda diag) d = J^T r
// from the Gram formed at the current coefficients (swept in registers),
// accepted when the true loss does not increase.
template <int V, int D>
__global__ __launch_bounds__(64, 4) void k_lm_step(FitArgs a, const double* gws,
                                                   const int64_t* gofs, const int* gflag) {
  using S = Shape<V, D>;
  constexpr int NC = S::NC, NU = S::NU;
  constexpr int NPK = NU * (NU + 1) / 2;
  static_assert(NC <= kWaveSolveMaxNC, "wave solver limited to small models");
  __shared__ SweepShared<NC> w;
  const int lane = threadIdx.x;
  const int f = a.ids[blockIdx.x];
  const int st0 = a.lm_state[f];
  if (st0 != LM_ACTIVE) {
    if (a.lm_last && lane == 0) lm_write_final<V, D>(a, f, st0);
    return;
  }
  if (gflag[f]) {
    if (lane == 0) {
      a.lm_state[f] = LM_NONFINITE;
      if (a.lm_last) lm_write_final<V, D>(a, f, LM_NONFINITE);
    }
    return;
  }
  const int64_t s0 = a.sample_off[f];
  const int64_t m = a.sample_off[f + 1] - s0;
  double* cg = a.coef + a.coef_off[f];
  const double lambda = a.lm_lambda[f];
  const double* g = gws + gofs[f];
  for (int e = lane; e < NPK; e += 64) w.gs[e] = g[e];
  wave_sync();
  const double loss = w.gs[NPK - 1];   // sum r^2 at the current coefficients
  Blocks<NC> B;
  block_load<NC>(w.gs, B, 1.0 + lambda, 0.0, w.col);
  const uint64_t drop = block_sweep<NC>(B, w.col, 1e-14);
  block_solution<NC>(B, drop, w.p);
  wave_sync();
  bool moved = false;
  for (int j = lane; j < NC; j += 64) {
    const double cj = cg[j];
    w.p[j] += cj;
    moved = moved || w.p[j] != cj;
  }
  wave_sync();
  const double loss_new = wave_true_loss<V, D>(a, s0, m, w.p, nullptr);
  // A step too small to change any coefficient is accepted (with zero change,
  // which ends the iteration): the two losses come from different summation
  // orders and need not agree to the last bit at the same coefficients.
  const bool accept = loss_new <= loss || !__any(moved);
  if (accept)
    for (int j = lane; j < NC; j += 64) cg[j] = w.p[j];
  if (lane == 0) {
    if (a.iters) a.iters[f] += 1;
    int st = LM_ACTIVE;
    if (accept) {
      const double change = loss - loss_new;
      double lam = lambda * 0.1;
      if (lam < 1e-12) lam = 0.0;
      a.lm_lambda[f] = lam;
      a.lm_loss[f] = loss_new;
      a.lm_rejects[f] = 0;
      if (change <= a.rtol * loss_new) st = LM_CONVERGED;
    } else {
      a.lm_loss[f] = loss;
      a.lm_lambda[f] = lambda == 0.0 ? 1e-6 : lambda * 10.0;
      const int rj = a.lm_rejects[f] + 1;
      a.lm_rejects[f] = rj;
      if (rj > 30) st = LM_STOPPED;
    }
    if (st != LM_ACTIVE) a.lm_state[f] = st;
    if (a.lm_last) lm_write_final<V, D>(a, f, st);
  }
}

template <int V, int D>
__global__ __launch_bounds__(64) void k_lm_final(FitArgs a) {
  const int f = a.ids[blockIdx.x];
  if (threadIdx.x == 0) lm_write_final<V, D>(a, f, a.lm_state[f]);
}

// ---------------------------------------------------------------------------
// Levenberg-Marquardt / Gauss-Newton on the true loss, FP64
// ---------------------------------------------------------------------------
template <int V, int D>
__device__ double true_loss(const FitArgs& a, int64_t s0, int64_t m, const double* c,
                            FitShared<Shape<V, D>::NC>& sh) {
  using S = Shape<V, D>;
  double ss = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += kThreads) {
    const int64_t s = s0 + i;
    double u[V];
#pragma unroll
    for (int k = 0; k < V; ++k) u[k] = a.x[(int64_t)k * a.ldx + s];
    double mo[S::NM];
    monomials<V, D, double>(u, mo);
    double N = 0.0, Q = 1.0;
#pragma unroll
    for (int j = 0; j < S::NA; ++j) N = fma(c[j], mo[j], N);
#pragma unroll
    for (int j = 1; j < S::NQ; ++j) Q = fma(c[S::NA + j - 1], mo[j], Q);
    const double r = N / Q - a.y[s];
    ss = fma(r, r, ss);
  }
  return block_sum(ss, sh.tmp);
}

template <int V, int D>
__global__ __launch_bounds__(kThreads) void k_refine(FitArgs a) {
  using Cfg = FitCfg<V, D, RP_FP64>;
  constexpr int NC = Cfg::NC;
  __shared__ __align__(16) unsigned char raw[Cfg::RAW_BYTES];
  __shared__ FitShared<NC> sh;
  double* G = reinterpret_cast<double*>(raw);
  const int tid = threadIdx.x;
  const int f = a.ids[blockIdx.x];
  const int64_t s0 = a.sample_off[f];
  const int64_t m = a.sample_off[f + 1] - s0;
  double* coef = a.coef + a.coef_off[f];
  if (tid == 0) sh.flag_nonfinite = 0;
  for (int j = tid; j < NC; j += kThreads) sh.c[j] = coef[j];
  __syncthreads();
  double loss = true_loss<V, D>(a, s0, m, sh.c, sh);
  double lambda = 0.0;
  int it = 0, rejects = 0;
  bool converged = false;
  for (it = 0; it < a.max_iter; ++it) {
    gram<V, D, RP_FP64, true>(a, s0, m, raw, G, sh, sh.c);
    if (sh.flag_nonfinite) break;
    equilibrate<NC>(G, sh, 0.0, lambda);
    for (int j = tid; j < NC; j += kThreads) sh.r[j] = G[pk(NC, j)];
    __syncthreads();
    cholesky<NC>(G, sh, 1e-14);
    chol_solve<NC>(G, sh, sh.r, sh.z);
    for (int j = tid; j < NC; j += kThreads) sh.p[j] = sh.c[j] + sh.z[j] * sh.dsc[j];
    __syncthreads();
    const double loss_new = true_loss<V, D>(a, s0, m, sh.p, sh);
    if (loss_new <= loss) {
      const double change = loss - loss_new;
      for (int j = tid; j < NC; j += kThreads) sh.c[j] = sh.p[j];
      __syncthreads();
      loss = loss_new;
      lambda *= 0.1;
      if (lambda < 1e-12) lambda = 0.0;
      rejects = 0;
      if (change <= a.rtol * loss) { converged = true; ++it; break; }
    } else {
      lambda = lambda == 0.0 ? 1e-6 : lambda * 10.0;
      if (++rejects > 30) { ++it; break; }
    }
  }
  for (int j = tid; j < NC; j += kThreads) coef[j] = sh.c[j];
  if (tid == 0) {
    int st = converged ? RP_FIT_OK : RP_FIT_NOT_CONVERGED;
    if (sh.flag_nonfinite) st = RP_FIT_NONFINITE_INPUT;
    else if (m < NC) st = RP_FIT_UNDERDETERMINED;
    a.status[f] = st;
    if (a.resid) a.resid[f] = loss;
    if (a.iters) a.iters[f] = it;
  }
}

// ---------------------------------------------------------------------------
// materialised design rows (API form of the fused assembly)
// ---------------------------------------------------------------------------
template <typename E, int V, int D, int... Cs>
__device__ __forceinline__ void store_row(E* dst, const RowGen<V, D, false>& row,
                                          std::integer_sequence<int, Cs...>) {
  ((dst[Cs] = to_elem<E>(row.template col<Cs>())), ...);
}

template <int V, int D, typename E>
__global__ __launch_bounds__(kThreads) void k_design(FitArgs a, E* A, const int64_t* a_off, E* rhs) {
  using S = Shape<V, D>;
  const int f = a.ids[blockIdx.x];
  const int64_t s0 = a.sample_off[f];
  const int64_t m = a.sample_off[f + 1] - s0;
  for (int64_t i = threadIdx.x; i < m; i += kThreads) {
    RowGen<V, D, false> row;
    row.load(a.x, a.ldx, a.y, s0 + i, true, nullptr);
    store_row<E, V, D>(A + a_off[f] + i * S::NC, row, std::make_integer_sequence<int, S::NC>{});
    rhs[s0 + i] = to_elem<E>(row.b);
  }
}

// ---------------------------------------------------------------------------
// FP32 true loss and adjoint
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ float dpp_movf(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}

// FP32 form of wave_reduce_vec: out[j] = sum over the wave's lanes of acc[j].
template <int NC>
__device__ __forceinline__ void wave_reduce_vec_f(const float (&acc)[NC], float* out, float* red) {
  constexpr int NCP = (NC + 3) / 4 * 4;
  const int lane = threadIdx.x & 63;
  const bool odd = lane & 1, hi2 = lane & 2;
  float r1[NCP / 2];
#pragma unroll
  for (int t = 0; t < NCP / 2; ++t) {
    const float a0 = 2 * t < NC ? acc[2 * t] : 0.0f;
    const float a1 = 2 * t + 1 < NC ? acc[2 * t + 1] : 0.0f;
    r1[t] = (odd ? a1 : a0) + dpp_movf<0xB1>(odd ? a0 : a1);   // partner lane ^ 1
  }
  const int quad = lane >> 2, q = lane & 3;
#pragma unroll
  for (int u = 0; u < NCP / 4; ++u) {
    const float b0 = r1[2 * u], b1 = r1[2 * u + 1];
    red[(4 * u + q) * 17 + quad] = (hi2 ? b1 : b0) + dpp_movf<0x4E>(hi2 ? b0 : b1);   // lane ^ 2
  }
  wave_sync();
  for (int j = lane; j < NC; j += 64) {
    float s0 = 0.0f, s1 = 0.0f;
#pragma unroll
    for (int g = 0; g < 16; g += 2) {
      s0 += red[j * 17 + g];
      s1 += red[j * 17 + g + 1];
    }
    out[j] = s0 + s1;
  }
  wave_sync();
}

__device__ __forceinline__ float wave_sum_f(float v) {
  v += dpp_movf<0xB1>(v);
  v += dpp_movf<0x4E>(v);
  v += dpp_movf<0x141>(v);
  v += dpp_movf<0x140>(v);
  return (__builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 0)) +
          __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 16))) +
         (__builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 32)) +
          __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 48)));
}

// True loss sum_i (N_i/Q_i - y_i)^2 per fit in FP32 and, in the backward mode,
// its gradient with respect to the coefficients times dloss[f] (the adjoint of
// the loss in Section 3.3's refinement): d/d alpha_j = 2 r m_j / Q and
// d/d beta_j = -2 r f m_j / Q with r = f - y, f = N/Q.  One wave per fit, one
// sample per lane and step with the next two samples' inputs in flight.
template <int V, int D>
constexpr int loss_min_waves() { return Shape<V, D>::NC <= 64 ? 4 : Shape<V, D>::NC <= 128 ? 2 : 1; }

template <int V, int D, int MODE>
__global__ __launch_bounds__(64, (loss_min_waves<V, D>())) void k_loss(FitArgs a, const float* coef,
                                                                    float* loss, const float* dloss,
                                                                    float* dcoef) {
  using S = Shape<V, D>;
  constexpr bool BWD = MODE == RP_LOSS_BWD;
  constexpr int NCP = (S::NC + 3) / 4 * 4;
  __shared__ float c[S::NC];
  __shared__ float red[BWD ? NCP * 17 : 1];
  __shared__ float gout[S::NC];
  const uint32_t lane = threadIdx.x;
  const int f = a.ids[blockIdx.x];
  const int64_t s0 = a.sample_off[f];
  const int64_t m = a.sample_off[f + 1] - s0;
  const int64_t co = a.coef_off[f];
  for (int j = lane; j < S::NC; j += 64) c[j] = coef[co + j];
  wave_sync();
  float g[BWD ? S::NC : 1];
#pragma unroll
  for (int j = 0; j < (BWD ? S::NC : 1); ++j) g[j] = 0.0f;
  float ls = 0.0f;
  const SampleSrc<V> src(a, s0, m);
  // the fit's coefficients, equal on every lane, in scalar registers
  float cz[S::NC];
#pragma unroll
  for (int j = 0; j < S::NC; ++j)
    cz[j] = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, c[j])));
  auto process = [&](const SampleIn<V>& t, bool valid) {
    float u[V];
#pragma unroll
    for (int k = 0; k < V; ++k) u[k] = (float)t.u[k];
    float mo[S::NM];
    monomials<V, D, float>(u, mo);
    float N = 0.0f, Q = 1.0f;
#pragma unroll
    for (int j = 0; j < S::NA; ++j) N = fmaf(cz[j], mo[j], N);
#pragma unroll
    for (int j = 1; j < S::NQ; ++j) Q = fmaf(cz[S::NA + j - 1], mo[j], Q);
    const float iq = 1.0f / Q;
    const float fv = N * iq;
    const float r = valid ? fv - (float)t.y : 0.0f;
    ls = fmaf(r, r, ls);
    if constexpr (BWD) {
      const float gn = 2.0f * r * iq;          // d loss / d alpha_j = gn * m_j
      const float gd = -gn * fv;               // d loss / d beta_j  = gd * m_j
#pragma unroll
      for (int j = 0; j < S::NA; ++j) g[j] = fmaf(gn, mo[j], g[j]);
#pragma unroll
      for (int j = 1; j < S::NQ; ++j) g[S::NA + j - 1] = fmaf(gd, mo[j], g[S::NA + j - 1]);
    }
  };
  // two sets of two slots used in turn (as in the refinement pass): the
  // loop's back edge moves no register, so it waits for no load
  SampleIn<V> sa[2], sb[2];
  if (src.m > 0) {
    src.load(sa[0], lane);
    src.load(sa[1], lane + 64u);
  }
#pragma unroll 1
  for (uint32_t b0 = 0; b0 < src.m; b0 += 256u) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      src.load(sb[k], b0 + 128u + 64u * k + lane);
      process(sa[k], b0 + 64u * k + lane < src.m);
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      src.load(sa[k], b0 + 256u + 64u * k + lane);
      process(sb[k], b0 + 128u + 64u * k + lane < src.m);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  ls = wave_sum_f(ls);
  if (lane == 0) loss[f] = ls;
  if constexpr (BWD) {
    wave_reduce_vec_f<S::NC>(g, gout, red);
    const float up = dloss ? dloss[f] : 1.0f;
    for (int j = lane; j < S::NC; j += 64) dcoef[co + j] = up * gout[j];
  }
}

// ---------------------------------------------------------------------------
// host launchers for one shape
// ---------------------------------------------------------------------------
template <int V, int D, int PREC>
int launch_split(const FitArgs& a, int nblocks, double* gws, const int64_t* gofs, int* gflag,
                 hipStream_t s) {
  if (PREC == RP_FP64 && a.gram_algo != RP_GRAM_MFMA && a.mom_map)
    hipLaunchKernelGGL((k_gram_mom_lin<V, D>), dim3(nblocks), dim3(MomCfg<V, D, false>::NT), 0, s, a, gws, gofs, gflag);
  else
    hipLaunchKernelGGL((k_gram<V, D, PREC>), dim3(nblocks), dim3(kThreads), 0, s, a, gws, gofs, gflag);
  hipLaunchKernelGGL((k_sweep<V, D, PREC>), dim3(nblocks), dim3(64), 0, s, a, gws, gofs, gflag);
  hipLaunchKernelGGL((k_refine_lin<V, D, PREC>), dim3((nblocks + 1) / 2), dim3(64), 0, s, a, gws, gofs,
                     gflag, nblocks);
  RP_CHECK_HIP(hipGetLastError());
  return RP_OK;
}

// Workgroups of the FP64 re-solve pass (one per compute unit): each takes its
// share of the bucket's list of flagged fits.  A call with an empty list costs
// one short launch of this many workgroups.
constexpr int kMinNormGrid = 256;

template <int V, int D>
int launch_shape_fit(int precision, const FitArgs& a, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return RP_OK;
  if (precision != RP_FP64 && precision != RP_MIXED_FP32 && precision != RP_MIXED_BF16)
    return set_error(RP_EINVAL, "unknown precision");
  bool split = false;
  if constexpr (Shape<V, D>::NC <= kWaveSolveMaxNC) {
    if (a.gws) {
      split = true;
      int rc = RP_OK;
      switch (precision) {
        case RP_FP64: rc = launch_split<V, D, RP_FP64>(a, nblocks, a.gws, a.gofs, a.gflag, s); break;
        case RP_MIXED_FP32: rc = launch_split<V, D, RP_MIXED_FP32>(a, nblocks, a.gws, a.gofs, a.gflag, s); break;
        default: rc = launch_split<V, D, RP_MIXED_BF16>(a, nblocks, a.gws, a.gofs, a.gflag, s); break;
      }
      if (rc != RP_OK) return rc;
    }
  }
  if constexpr (Shape<V, D>::NC > kWaveSolveMaxNC) {
    // larger models, FP64: the Gram by weighted moments into the workspace
    // (far fewer products than the padded MFMA tiles of the fused kernel),
    // swept there by k_big_sweep, refined by k_big_refine
    if (precision == RP_FP64 && a.gws && a.gram_algo != RP_GRAM_MFMA && a.mom_map) {
      split = true;
      hipLaunchKernelGGL((k_gram_mom_lin<V, D>), dim3(nblocks), dim3(MomCfg<V, D, false>::NT), 0, s, a,
                         a.gws, a.gofs, a.gflag);
      hipLaunchKernelGGL((k_big_sweep<V, D>), dim3(nblocks), dim3(kThreads), 0, s, a);
      hipLaunchKernelGGL((k_big_refine<V, D>), dim3(nblocks), dim3(kThreads), 0, s, a);
    }
  }
  if (!split) {
    switch (precision) {
      case RP_FP64: hipLaunchKernelGGL((k_fit<V, D, RP_FP64>), dim3(nblocks), dim3(kThreads), 0, s, a); break;
      case RP_MIXED_FP32: hipLaunchKernelGGL((k_fit<V, D, RP_MIXED_FP32>), dim3(nblocks), dim3(kThreads), 0, s, a); break;
      default: hipLaunchKernelGGL((k_fit<V, D, RP_MIXED_BF16>), dim3(nblocks), dim3(kThreads), 0, s, a); break;
    }
  }
  if (a.resolve)
    hipLaunchKernelGGL((k_min_norm<V, D>), dim3(std::min(nblocks, kMinNormGrid)), dim3(kThreads), 0, s, a);
  RP_CHECK_HIP(hipGetLastError());
  return RP_OK;
}

template <int V, int D>
int launch_shape_gram(int precision, const FitArgs& a, double* gram, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return RP_OK;
  switch (precision) {
    case kGramJacobian:
      if (a.gram_algo != RP_GRAM_MFMA && a.mom_map)
        hipLaunchKernelGGL((k_gram_mom<V, D, true>), dim3(nblocks), dim3(MomCfg<V, D, true>::NT), 0, s, a, gram, a.gofs, a.gflag);
      else
        hipLaunchKernelGGL((k_gram<V, D, RP_FP64, true>), dim3(nblocks), dim3(kThreads), 0, s, a, gram, a.gofs, a.gflag);
      break;
    case RP_FP64:
      if (a.gram_algo != RP_GRAM_MFMA && a.mom_map)
        hipLaunchKernelGGL((k_gram_mom_lin<V, D>), dim3(nblocks), dim3(MomCfg<V, D, false>::NT), 0, s, a, gram, a.gofs, a.gflag);
      else
        hipLaunchKernelGGL((k_gram<V, D, RP_FP64>), dim3(nblocks), dim3(kThreads), 0, s, a, gram, a.gofs, a.gflag);
      break;
    case RP_MIXED_FP32: hipLaunchKernelGGL((k_gram<V, D, RP_MIXED_FP32>), dim3(nblocks), dim3(kThreads), 0, s, a, gram, a.gofs, a.gflag); break;
    case RP_MIXED_BF16: hipLaunchKernelGGL((k_gram<V, D, RP_MIXED_BF16>), dim3(nblocks), dim3(kThreads), 0, s, a, gram, a.gofs, a.gflag); break;
    default: return set_error(RP_EINVAL, "unknown precision");
  }
  RP_CHECK_HIP(hipGetLastError());
  return RP_OK;
}

template <int V, int D>
int launch_shape_refine(const FitArgs& a, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return RP_OK;
  if constexpr (Shape<V, D>::NC <= kWaveSolveMaxNC) {
    if (a.gws && a.lm_state) {
      if (a.max_iter == 0) {
        // no iteration: the loss at the given coefficients and the outputs
        hipLaunchKernelGGL((k_lm_init<V, D>), dim3(nblocks), dim3(64), 0, s, a, 1);
        hipLaunchKernelGGL((k_lm_final<V, D>), dim3(nblocks), dim3(64), 0, s, a);
        RP_CHECK_HIP(hipGetLastError());
        return RP_OK;
      }
      // the first Gram sets the LM state, the last step writes the outputs
      FitArgs b = a;
      for (int it = 0; it < a.max_iter; ++it) {
        b.lm_first = it == 0;
        b.lm_last = it == a.max_iter - 1;
        if (a.gram_algo != RP_GRAM_MFMA && a.mom_map)
          hipLaunchKernelGGL((k_gram_mom<V, D, true>), dim3(nblocks), dim3(MomCfg<V, D, true>::NT), 0, s, b,
                             a.gws, a.gofs, a.gflag);
        else
          hipLaunchKernelGGL((k_gram<V, D, RP_FP64, true>), dim3(nblocks), dim3(kThreads), 0, s, b,
                             a.gws, a.gofs, a.gflag);
        hipLaunchKernelGGL((k_lm_step<V, D>), dim3(nblocks), dim3(64), 0, s, b, a.gws, a.gofs,
                           a.gflag);
      }
      RP_CHECK_HIP(hipGetLastError());
      return RP_OK;
    }
  }
  hipLaunchKernelGGL((k_refine<V, D>), dim3(nblocks), dim3(kThreads), 0, s, a);
  RP_CHECK_HIP(hipGetLastError());
  return RP_OK;
}

template <int V, int D>
int launch_shape_design(int precision, const FitArgs& a, void* A, const int64_t* a_off, void* rhs,
                        int nblocks, hipStream_t s) {
  if (nblocks <= 0) return RP_OK;
  switch (precision) {
    case RP_FP64:
      hipLaunchKernelGGL((k_design<V, D, double>), dim3(nblocks), dim3(kThreads), 0, s, a,
                         (double*)A, a_off, (double*)rhs); break;
    case RP_MIXED_FP32:
      hipLaunchKernelGGL((k_design<V, D, float>), dim3(nblocks), dim3(kThreads), 0, s, a,
                         (float*)A, a_off, (float*)rhs); break;
    case RP_MIXED_BF16:
      hipLaunchKernelGGL((k_design<V, D, __bf16>), dim3(nblocks), dim3(kThreads), 0, s, a,
                         (__bf16*)A, a_off, (__bf16*)rhs); break;
    default: return set_error(RP_EINVAL, "unknown precision");
  }
  RP_CHECK_HIP(hipGetLastError());
  return RP_OK;
}

template <int V, int D>
int launch_shape_loss(const FitArgs& a, const float* coef, float* loss, const float* dloss,
                      float* dcoef, int mode, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return RP_OK;
  if (mode == RP_LOSS_FWD)
    hipLaunchKernelGGL((k_loss<V, D, RP_LOSS_FWD>), dim3(nblocks), dim3(64), 0, s, a, coef, loss, dloss, dcoef);
  else
    hipLaunchKernelGGL((k_loss<V, D, RP_LOSS_BWD>), dim3(nblocks), dim3(64), 0, s, a, coef, loss, dloss, dcoef);
  RP_CHECK_HIP(hipGetLastError());
  return RP_OK;
}

}  // namespace rp

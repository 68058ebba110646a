// rp_fit_kernels.h -- HIP kernels of the fitting path, templated on the model
// shape (V variables, numerator and denominator degree D) so that monomials,
// design rows and accumulators live in registers with static indices.
//
// One workgroup (256 threads, four wave64s) owns one fit at a time:
//   1. design assembly fused into the Gram: chunks of samples are turned into
//      design columns in LDS (column-major, padded so the MFMA operand reads are
//      bank-conflict free) and contracted on MFMA into the augmented Gram
//      [A b]^T [A b] (Section 4.2: A x = b, normal equations);
//   2. power-of-two column equilibration and an FP64 Cholesky factorisation of
//      the Gram in LDS (packed lower triangle), then two triangular solves;
//   3. FP64 refinement over the samples: iterative refinement (FP64 form) or
//      preconditioned conjugate gradients with the low-precision Gram's
//      Cholesky factor as preconditioner (mixed forms).
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
  double dsc[NC + 1]; // power-of-two column scales (last = 1 for the rhs column)
  double red[kWaves * NC];
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
      for (int j = 1; j < S::NM; ++j) Q = fma(c[S::NA + j - 1], m[j], Q);
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

// Scale rows/columns j < NC by d_j = 2^-floor(log2(G_jj)/2) (exact), keep the
// rhs column unscaled, then add `shift` to the scaled diagonal and multiply it
// by (1 + lambda).
template <int NC>
__device__ void equilibrate(double* G, FitShared<NC>& sh, double shift, double lambda) {
  const int tid = threadIdx.x;
  constexpr int NU = NC + 1;
  for (int j = tid; j < NU; j += kThreads) {
    double d = 1.0;
    if (j < NC) {
      const double g = G[pk(j, j)];
      if (g > 0.0 && isfinite(g)) d = ldexp(1.0, -(ilogb(g) / 2));
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

// out = D (L L^T)^-1 D v  (preconditioner / correction in unscaled space)
template <int NC>
__device__ void scaled_solve(const double* G, FitShared<NC>& sh, const double* v, double* out) {
  const int tid = threadIdx.x;
  __syncthreads();
  for (int j = tid; j < NC; j += kThreads) out[j] = v[j] * sh.dsc[j];
  chol_solve<NC>(G, sh, out, out);
  for (int j = tid; j < NC; j += kThreads) out[j] *= sh.dsc[j];
  __syncthreads();
}

// ---------------------------------------------------------------------------
// FP64 passes over the samples (thread per sample, registers only)
// ---------------------------------------------------------------------------
enum PassMode { PASS_RESIDUAL = 0, PASS_PRODUCT = 1, PASS_CHECK = 2 };

// RESIDUAL: w_i = b_i - a_i.v,  out = A^T w, returns sum w^2
// PRODUCT:  w_i = a_i.v,        out = A^T w
// CHECK:    w_i = b_i - a_i.v,  returns sum w^2; *qmin = min_i Q_v(u_i)
template <int V, int D, int MODE>
__device__ double pass(const FitArgs& a, int64_t s0, int64_t m, const double* v, double* out,
                       FitShared<Shape<V, D>::NC>& sh, double* qmin) {
  using S = Shape<V, D>;
  const int tid = threadIdx.x;
  double acc[S::NC];
#pragma unroll
  for (int j = 0; j < S::NC; ++j) acc[j] = 0.0;
  double ss = 0.0, qm = INFINITY;
  for (int64_t i = tid; i < m; i += kThreads) {
    const int64_t s = s0 + i;
    double u[V];
#pragma unroll
    for (int k = 0; k < V; ++k) u[k] = a.x[(int64_t)k * a.ldx + s];
    const double y = a.y[s];
    double mo[S::NM];
    monomials<V, D, double>(u, mo);
    double nv = 0.0, qv = 0.0;
#pragma unroll
    for (int j = 0; j < S::NA; ++j) nv = fma(v[j], mo[j], nv);
#pragma unroll
    for (int j = 1; j < S::NM; ++j) qv = fma(v[S::NA + j - 1], mo[j], qv);
    const double dot = fma(-y, qv, nv);                 // a_i . v
    const double w = (MODE == PASS_PRODUCT) ? dot : y - dot;
    ss = fma(w, w, ss);
    if constexpr (MODE == PASS_CHECK) qm = fmin(qm, 1.0 + qv);
    if constexpr (MODE != PASS_CHECK) {
      const double wy = -y * w;
#pragma unroll
      for (int j = 0; j < S::NA; ++j) acc[j] = fma(w, mo[j], acc[j]);
#pragma unroll
      for (int j = 1; j < S::NM; ++j) acc[S::NA + j - 1] = fma(wy, mo[j], acc[S::NA + j - 1]);
    }
  }
  const int lane = tid & 63, wave = tid >> 6;
  if constexpr (MODE != PASS_CHECK) {
#pragma unroll
    for (int j = 0; j < S::NC; ++j) {
      const double t = wave_sum(acc[j]);
      if (lane == 0) sh.red[wave * S::NC + j] = t;
    }
  }
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

// ---------------------------------------------------------------------------
// the linearised fit
// ---------------------------------------------------------------------------
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

  // factor: FP64 drops vanished pivots; the mixed forms shift the diagonal
  // until the low-precision Gram factors, then refine against FP64 products.
  constexpr double kTauFp64 = 1e-10;
  double shift = (PREC == RP_FP64) ? 0.0 : (PREC == RP_MIXED_FP32 ? 0x1p-20 : 0x1p-7);
  // the scaled rhs column A^T b is copied out before the factorisation, which
  // overwrites only the leading NC x NC block
  equilibrate<NC>(G, sh, shift, 0.0);
  for (int j = tid; j < NC; j += kThreads) sh.r[j] = G[pk(NC, j)];   // scaled A^T b
  __syncthreads();
  int ndrop = cholesky<NC>(G, sh, PREC == RP_FP64 ? kTauFp64 : 0.0);
  if (PREC != RP_FP64 && ndrop > 0) {
    // the low-precision Gram was not SPD even with the shift: rebuild with a
    // larger shift (the Gram is recomputed; this path is rare)
    for (int attempt = 0; attempt < 6 && ndrop > 0; ++attempt) {
      shift *= 16.0;
      gram<V, D, PREC, false>(a, s0, m, raw, G, sh, nullptr);
      equilibrate<NC>(G, sh, shift, 0.0);
      for (int j = tid; j < NC; j += kThreads) sh.r[j] = G[pk(NC, j)];
      __syncthreads();
      ndrop = cholesky<NC>(G, sh, 0.0);
    }
  }
  chol_solve<NC>(G, sh, sh.r, sh.c);
  for (int j = tid; j < NC; j += kThreads) sh.c[j] *= sh.dsc[j];
  __syncthreads();

  int it = 0;
  double last_rel = 0.0;
  if constexpr (PREC == RP_FP64) {
    // iterative refinement: c += G^-1 A^T (b - A c)
    for (it = 0; it < a.max_refine;) {
      pass<V, D, PASS_RESIDUAL>(a, s0, m, sh.c, sh.r, sh, nullptr);
      scaled_solve<NC>(G, sh, sh.r, sh.z);
      for (int j = tid; j < NC; j += kThreads) sh.c[j] += sh.z[j];
      ++it;
      const double dn = maxabs_nc<NC>(sh.z, sh);
      const double cn = maxabs_nc<NC>(sh.c, sh);
      last_rel = cn > 0.0 ? dn / cn : dn;
      if (dn <= a.tol * cn) break;
    }
  } else {
    // preconditioned CG on A^T A c = A^T b with M = the low-precision Gram
    pass<V, D, PASS_RESIDUAL>(a, s0, m, sh.c, sh.r, sh, nullptr);
    scaled_solve<NC>(G, sh, sh.r, sh.z);
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
      if (dn <= a.tol * cn || !(pq > 0.0)) break;
      scaled_solve<NC>(G, sh, sh.r, sh.z);
      const double rz2 = dot_nc<NC>(sh.r, sh.z, sh);
      const double beta = rz > 0.0 ? rz2 / rz : 0.0;
      rz = rz2;
      for (int j = tid; j < NC; j += kThreads) sh.p[j] = fma(beta, sh.p[j], sh.z[j]);
      __syncthreads();
    }
  }

  double resid = __builtin_nan("");
  double qmin = 1.0;
  if (a.check_q) {
    const double ss = pass<V, D, PASS_CHECK>(a, s0, m, sh.c, nullptr, sh, &qmin);
    resid = sqrt(ss);
  }
  for (int j = tid; j < NC; j += kThreads) coef[j] = sh.c[j];
  if (tid == 0) {
    int st = RP_FIT_OK;
    if (m < NC) st = RP_FIT_UNDERDETERMINED;
    else if (ndrop > 0) st = RP_FIT_RANK_DEFICIENT;
    else if (!(last_rel <= sqrt(a.tol))) st = RP_FIT_NOT_CONVERGED;
    else if (!(qmin > 0.0)) st = RP_FIT_Q_NONPOSITIVE;
    a.status[f] = st;
    if (a.resid) a.resid[f] = resid;
    if (a.iters) a.iters[f] = it;
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
    if (a.lm_state[f] != 0) return;          // converged or stopped: nothing to form
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

template <int NC>
struct WaveShared {
  static constexpr int NU = NC + 1;
  static constexpr int NPK = NU * (NU + 1) / 2;
  static constexpr int NCP = (NC + 3) / 4 * 4;   // padded to whole quads
  double G[NPK];      // packed lower augmented Gram, swept in place
  double c[NC], r[NC], z[NC], p[NC], q[NC];
  double yv[NC + 1];  // scaled preconditioner input; pivot column during the sweep
  double dsc[NU];
  double red[NCP * 17];   // quad partial sums, [value][quad] with a padded row
  int drop[NC];
};

// Largest model the wave-per-fit solver keeps in registers.
constexpr int kWaveSolveMaxNC = 64;

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int pks(int i, int j) { return i >= j ? pk(i, j) : pk(j, i); }

// Sweep every pivot k < NC of the equilibrated augmented Gram (packed lower).
// Afterwards the leading block holds -G^-1 on the kept pivots, row NC holds
// the scaled solution and entry (NC, NC) the residual sum of squares.  A pivot
// <= tau is not swept: its coefficient is held at zero.  Returns the count of
// dropped pivots.
//
// Each lane keeps its share of the packed triangle (entries lane + 64 t) in
// registers for the whole sweep; per pivot only column k travels through LDS
// (its owners publish it, every lane then reads the two column values each of
// its entries needs).  The G array is read once at the start and written once
// at the end.
template <int NC>
__device__ __forceinline__ int wave_sweep(WaveShared<NC>& w, double tau) {
  constexpr int NU = NC + 1;
  constexpr int NPK = NU * (NU + 1) / 2;
  constexpr int NE = (NPK + 63) / 64;
  const int lane = threadIdx.x & 63;
  int ij[NE];
  double val[NE];
#pragma unroll
  for (int t = 0; t < NE; ++t) {
    const int e = lane + 64 * t;
    int i = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);   // row of packed entry e
    i -= (i * (i + 1) / 2 > e);
    i += ((i + 1) * (i + 2) / 2 <= e);
    const int j = e - i * (i + 1) / 2;
    ij[t] = e < NPK ? (i | (j << 16)) : -1;
    val[t] = e < NPK ? w.G[e] : 0.0;
  }
  double* colk = w.yv;            // NC + 1 doubles of scratch
  int ndrop = 0;
#pragma unroll 1
  for (int k = 0; k < NC; ++k) {
    // publish column k (entries (i, k) for i >= k and (k, j) for j < k)
#pragma unroll
    for (int t = 0; t < NE; ++t) {
      const int v = ij[t];
      if (v >= 0) {
        const int i = v & 0xffff, j = v >> 16;
        if (j == k) colk[i] = val[t];
        else if (i == k) colk[j] = val[t];
      }
    }
    wave_sync();
    const double d = colk[k];
    if (!(d > tau)) {
      if (lane == 0) w.drop[k] = 1;
      ++ndrop;
      wave_sync();
      continue;
    }
    if (lane == 0) w.drop[k] = 0;
    const double inv = 1.0 / d;
    double ci[NE], cj[NE];
#pragma unroll
    for (int t = 0; t < NE; ++t) {
      const int v = ij[t] < 0 ? 0 : ij[t];
      ci[t] = colk[v & 0xffff];
      cj[t] = colk[v >> 16];
    }
#pragma unroll
    for (int t = 0; t < NE; ++t) {
      const int v = ij[t];
      if (v >= 0) {
        const int i = v & 0xffff, j = v >> 16;
        if (i == k && j == k) val[t] = -inv;
        else if (i == k || j == k) val[t] *= inv;
        else val[t] = fma(-ci[t] * inv, cj[t], val[t]);
      }
    }
    wave_sync();
  }
#pragma unroll
  for (int t = 0; t < NE; ++t) {
    const int e = lane + 64 * t;
    if (e < NPK) w.G[e] = val[t];
  }
  wave_sync();
  return ndrop;
}

// out = D (G_SS)^-1 D v on the kept pivots (the swept block holds -G^-1).
template <int NC>
__device__ __forceinline__ void wave_precond(WaveShared<NC>& w, const double* v, double* out) {
  const int lane = threadIdx.x & 63;
  for (int k = lane; k < NC; k += 64) w.yv[k] = w.drop[k] ? 0.0 : v[k] * w.dsc[k];
  wave_sync();
  double t[2] = {0.0, 0.0};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int j = lane + 64 * h;
    if (j < NC) {
      const int rj = j * (j + 1) / 2;
      double a0 = 0.0, a1 = 0.0;
      int k = 0;
      for (; k + 1 <= j; k += 2) {                 // row j, columns k <= j: contiguous
        a0 = fma(w.G[rj + k], w.yv[k], a0);
        if (k + 1 <= j) a1 = fma(w.G[rj + k + 1], w.yv[k + 1], a1);
      }
      if (k <= j) a0 = fma(w.G[rj + k], w.yv[k], a0);
      for (k = j + 1; k < NC; ++k) a1 = fma(w.G[k * (k + 1) / 2 + j], w.yv[k], a1);
      t[h] = w.drop[j] ? 0.0 : -(a0 + a1) * w.dsc[j];
    }
  }
  wave_sync();
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int j = lane + 64 * h;
    if (j < NC) out[j] = t[h];
  }
  wave_sync();
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

// out[j] = sum over the wave's 64 lanes of acc[j], j < NC.  Two DPP
// butterfly steps inside each quad halve the number of values per lane twice
// (lane q of a quad ends up holding the quad sum of values 4u + q); the 16
// quad partials of every value then meet in LDS and lane j adds its row.
template <int NC>
__device__ __forceinline__ void wave_reduce_vec(const double (&acc)[NC], double* out, double* red) {
  constexpr int NCP = (NC + 3) / 4 * 4;
  const int lane = threadIdx.x & 63;
  const bool odd = lane & 1, hi2 = lane & 2;
  double r1[NCP / 2];
#pragma unroll
  for (int t = 0; t < NCP / 2; ++t) {
    const double a0 = 2 * t < NC ? acc[2 * t] : 0.0;
    const double a1 = 2 * t + 1 < NC ? acc[2 * t + 1] : 0.0;
    const double send = odd ? a0 : a1;
    const double keep = odd ? a1 : a0;
    r1[t] = keep + dpp_mov<0xB1>(send);           // partner lane ^ 1
  }
  const int quad = lane >> 2, q = lane & 3;
#pragma unroll
  for (int u = 0; u < NCP / 4; ++u) {
    const double b0 = r1[2 * u], b1 = r1[2 * u + 1];
    const double send = hi2 ? b0 : b1;
    const double keep = hi2 ? b1 : b0;
    red[(4 * u + q) * 17 + quad] = keep + dpp_mov<0x4E>(send);   // partner lane ^ 2
  }
  wave_sync();
  if (lane < NC) {
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int g = 0; g < 16; g += 2) {
      s0 += red[lane * 17 + g];
      s1 += red[lane * 17 + g + 1];
    }
    out[lane] = s0 + s1;
  }
  wave_sync();
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

template <int NC>
__device__ __forceinline__ double wave_dot(const double* a, const double* b) {
  double t = 0.0;
  for (int j = threadIdx.x & 63; j < NC; j += 64) t = fma(a[j], b[j], t);
  return wave_sum_dpp(t);
}

template <int NC>
__device__ __forceinline__ double wave_maxabs(const double* a) {
  double t = 0.0;
  for (int j = threadIdx.x & 63; j < NC; j += 64) t = fmax(t, fabs(a[j]));
  return wave_max(t);
}

// FP64 pass over one fit's samples by one wave (see pass() for the modes).
// Each lane takes two samples per step (the wave-uniform vector, read from
// LDS, is used twice per read); the next two samples' inputs are loaded one
// step ahead so a single resident wave keeps the FP64 pipeline busy.
template <int V, int D>
struct PassSample {
  using S = Shape<V, D>;
  double mo[S::NM];
  double y;
  bool valid;
};

template <int V, int D, int MODE>
__device__ double wave_pass(const FitArgs& a, int64_t s0, int64_t m, const double* v, double* out,
                            double* qmin, double* red) {
  using S = Shape<V, D>;
  const int lane = threadIdx.x & 63;
  double acc[MODE == PASS_CHECK ? 1 : S::NC];
#pragma unroll
  for (int j = 0; j < (MODE == PASS_CHECK ? 1 : S::NC); ++j) acc[j] = 0.0;
  double ss = 0.0, qm = INFINITY;
  double un[2][V], yn[2] = {0.0, 0.0};
  auto fetch = [&](int64_t i0) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t i = i0 + 64 * h;
      if (i < m) {
#pragma unroll
        for (int k = 0; k < V; ++k) un[h][k] = a.x[(int64_t)k * a.ldx + s0 + i];
        yn[h] = a.y[s0 + i];
      } else {
#pragma unroll
        for (int k = 0; k < V; ++k) un[h][k] = 0.0;
        yn[h] = 0.0;
      }
    }
  };
  fetch(lane);
#pragma unroll 1
  for (int64_t i0 = lane; i0 < m; i0 += 128) {
    double u[2][V], y[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
      for (int k = 0; k < V; ++k) u[h][k] = un[h][k];
      y[h] = yn[h];
    }
    const bool valid1 = i0 + 64 < m;
    if (i0 + 128 < m) fetch(i0 + 128);
    double mo0[S::NM], mo1[S::NM];
    monomials<V, D, double>(u[0], mo0);
    monomials<V, D, double>(u[1], mo1);
    // the vector is wave-uniform and lives in LDS: read it where it is used
    // (broadcast reads); the opaque zero offset keeps the reads in the loop
    int zero;
    asm volatile("v_mov_b32 %0, 0" : "=v"(zero));
    const double* vv = v + zero;
    double n0 = 0.0, n1 = 0.0, q0 = 0.0, q1 = 0.0;
#pragma unroll
    for (int j = 0; j < S::NA; ++j) {
      const double vj = vv[j];
      n0 = fma(vj, mo0[j], n0);
      n1 = fma(vj, mo1[j], n1);
    }
#pragma unroll
    for (int j = 1; j < S::NM; ++j) {
      const double vj = vv[S::NA + j - 1];
      q0 = fma(vj, mo0[j], q0);
      q1 = fma(vj, mo1[j], q1);
    }
    const double d0 = fma(-y[0], q0, n0), d1 = fma(-y[1], q1, n1);
    double w0 = (MODE == PASS_PRODUCT) ? d0 : y[0] - d0;
    double w1 = (MODE == PASS_PRODUCT) ? d1 : y[1] - d1;
    w1 = valid1 ? w1 : 0.0;
    ss = fma(w0, w0, ss);
    ss = fma(w1, w1, ss);
    if constexpr (MODE == PASS_CHECK) {
      qm = fmin(qm, 1.0 + q0);
      if (valid1) qm = fmin(qm, 1.0 + q1);
    } else {
      const double wy0 = -y[0] * w0, wy1 = -y[1] * w1;
#pragma unroll
      for (int j = 0; j < S::NA; ++j) acc[j] = fma(w1, mo1[j], fma(w0, mo0[j], acc[j]));
#pragma unroll
      for (int j = 1; j < S::NM; ++j)
        acc[S::NA + j - 1] = fma(wy1, mo1[j], fma(wy0, mo0[j], acc[S::NA + j - 1]));
    }
  }
  if constexpr (MODE != PASS_CHECK) {
    static_assert(S::NC <= 64, "wave reduction covers one value per lane");
    wave_reduce_vec<S::NC>(acc, out, red);
  } else {
    *qmin = -wave_max(-qm);
  }
  wave_sync();
  return wave_sum_dpp(ss);
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
template <int V, int D, bool GN>
struct MomCfg {
  using MS = MomentShape<V, D, GN>;
  static constexpr int NW = GN ? 6 : 3;
  static constexpr int NWV = MS::NWV;              // waves per workgroup
  static constexpr int NT = 64 * NWV;              // threads per workgroup
  static constexpr int CHM = NT;                   // staged samples per chunk
  static constexpr int PL = MS::PL;
  static constexpr int PLP = (PL + 3) / 4 * 4;
  static constexpr MonoBig<V, 2 * D> E2 = make_mono_big<V, 2 * D>();
};

template <int V, int D, bool GN>
constexpr int mom_e_of(int p) {
  int e = 0, w = 0;
  moment_pair_of<GN>(p, binom(V + D, D), e, w);
  return e;
}
template <int V, int D, bool GN>
constexpr int mom_w_of(int p) {
  int e = 0, w = 0;
  moment_pair_of<GN>(p, binom(V + D, D), e, w);
  return w;
}

template <int V, int D, bool GN, int P, int J>
__device__ __forceinline__ void mom_acc_one(double* acc, const double (&pw)[kMaxV][2 * kMaxD + 1],
                                            const double* W) {
  using C = MomCfg<V, D, GN>;
  if constexpr (P < C::MS::NPAIR) {
    constexpr int e = mom_e_of<V, D, GN>(P);
    constexpr int w = mom_w_of<V, D, GN>(P);
    constexpr int a0 = C::E2.e[e][0], a1 = C::E2.e[e][1], a2 = C::E2.e[e][2], a3 = C::E2.e[e][3];
    double mon = 1.0;
    if constexpr (a0 > 0) mon *= pw[0][a0];
    if constexpr (a1 > 0) mon *= pw[1][a1];
    if constexpr (a2 > 0) mon *= pw[2][a2];
    if constexpr (a3 > 0) mon *= pw[3][a3];
    acc[J] = fma(W[w], mon, acc[J]);
  }
}

template <int V, int D, bool GN, int G, int... J>
__device__ __forceinline__ void mom_acc_group(double* acc, const double (&pw)[kMaxV][2 * kMaxD + 1],
                                              const double* W, std::integer_sequence<int, J...>) {
  using C = MomCfg<V, D, GN>;
  (mom_acc_one<V, D, GN, G * C::PL + J, J>(acc, pw, W), ...);
}

// One wave, one chunk of staged samples, moment group G.
template <int V, int D, bool GN, int G>
__device__ __forceinline__ void mom_chunk(double* acc, const double* su, const double* sw) {
  using C = MomCfg<V, D, GN>;
  const int lane = threadIdx.x & 63;
#pragma unroll 1
  for (int i = lane; i < C::CHM; i += 64) {
    double pw[kMaxV][2 * kMaxD + 1];
#pragma unroll
    for (int k = 0; k < V; ++k) {
      const double uk = su[k * C::CHM + i];
      pw[k][0] = 1.0;
      pw[k][1] = uk;
#pragma unroll
      for (int t = 2; t <= 2 * D; ++t) pw[k][t] = pw[k][t - 1] * uk;
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
  double su[V * C::CHM];
  double sw[C::NW * C::CHM];
  double red[C::NWV][C::PLP * 17];
  double mom[C::MS::NGROUP * C::PL];
  double c[Shape<V, D>::NC];
  int flag_nonfinite;
};

// Stage one chunk: inputs and weights of samples [c0, c0 + 256).
template <int V, int D, bool GN>
__device__ __forceinline__ void mom_stage(const FitArgs& a, int64_t s0, int64_t m, int64_t c0,
                                          MomShared<V, D, GN>& sh, bool& bad) {
  using C = MomCfg<V, D, GN>;
  using S = Shape<V, D>;
  const int t = threadIdx.x;
  const int64_t i = c0 + t;
  double u[V], y = 0.0;
  const bool valid = i < m;
  if (valid) {
#pragma unroll
    for (int k = 0; k < V; ++k) { u[k] = a.x[(int64_t)k * a.ldx + s0 + i]; bad = bad || !isfinite(u[k]); }
    y = a.y[s0 + i];
    bad = bad || !isfinite(y);
  } else {
#pragma unroll
    for (int k = 0; k < V; ++k) u[k] = 0.0;
  }
#pragma unroll
  for (int k = 0; k < V; ++k) sh.su[k * C::CHM + t] = u[k];
  if constexpr (!GN) {
    sh.sw[0 * C::CHM + t] = valid ? 1.0 : 0.0;
    sh.sw[1 * C::CHM + t] = y;
    sh.sw[2 * C::CHM + t] = y * y;
  } else {
    double mo[S::NM];
    monomials<V, D, double>(u, mo);
    double n = 0.0, q = 1.0;
#pragma unroll
    for (int j = 0; j < S::NA; ++j) n = fma(sh.c[j], mo[j], n);
#pragma unroll
    for (int j = 1; j < S::NM; ++j) q = fma(sh.c[S::NA + j - 1], mo[j], q);
    const double iq = valid ? 1.0 / q : 0.0;
    const double f = n / q;
    const double r = valid ? y - f : 0.0;
    const double iq2 = iq * iq;
    sh.sw[0 * C::CHM + t] = iq2;
    sh.sw[1 * C::CHM + t] = iq2 * f;
    sh.sw[2 * C::CHM + t] = iq2 * f * f;
    sh.sw[3 * C::CHM + t] = iq * r;
    sh.sw[4 * C::CHM + t] = iq * f * r;
    sh.sw[5 * C::CHM + t] = r * r;
  }
}

template <int V, int D, bool GN, int G0, int... W>
__device__ __forceinline__ void mom_chunk_dispatch(int wave, double* acc, const double* su,
                                                   const double* sw, std::integer_sequence<int, W...>) {
  ((wave == W ? mom_chunk<V, D, GN, G0 + W>(acc, su, sw) : (void)0), ...);
}

template <int V, int D, bool GN, int Q>
__device__ void mom_pass(const FitArgs& a, int64_t s0, int64_t m, MomShared<V, D, GN>& sh, bool& bad) {
  using C = MomCfg<V, D, GN>;
  const int wave = threadIdx.x >> 6;
  double acc[C::PL];
#pragma unroll
  for (int j = 0; j < C::PL; ++j) acc[j] = 0.0;
  for (int64_t c0 = 0; c0 < m; c0 += C::CHM) {
    mom_stage<V, D, GN>(a, s0, m, c0, sh, bad);
    __syncthreads();
    // wave-uniform choice of this wave's static moment group
    mom_chunk_dispatch<V, D, GN, C::NWV * Q>(wave, acc, sh.su, sh.sw,
                                             std::make_integer_sequence<int, C::NWV>{});
    __syncthreads();
  }
  wave_reduce_vec<C::PL>(acc, sh.mom + (C::NWV * Q + wave) * C::PL, sh.red[wave]);
}

template <int V, int D, bool GN, int... Q>
__device__ __forceinline__ void mom_all_passes(const FitArgs& a, int64_t s0, int64_t m,
                                               MomShared<V, D, GN>& sh, bool& bad,
                                               std::integer_sequence<int, Q...>) {
  (mom_pass<V, D, GN, Q>(a, s0, m, sh, bad), ...);
}

template <int V, int D, bool GN>
__global__ __launch_bounds__((MomCfg<V, D, GN>::NT)) void k_gram_mom(FitArgs a, double* gws,
                                                                   const int64_t* gofs, int* gflag) {
  using C = MomCfg<V, D, GN>;
  using S = Shape<V, D>;
  constexpr int NPK = S::NU * (S::NU + 1) / 2;
  __shared__ MomShared<V, D, GN> sh;
  const int f = a.ids[blockIdx.x];
  if constexpr (GN) {
    if (a.lm_state[f] != 0) return;
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
  mom_all_passes<V, D, GN>(a, s0, m, sh, bad, std::make_integer_sequence<int, C::MS::NPASS>{});
  if (bad) atomicOr(&sh.flag_nonfinite, 1);
  __syncthreads();
  double* out = gws + gofs[f];
  for (int e = threadIdx.x; e < NPK; e += C::NT) {
    const int mp = a.mom_map[e];
    const double v = sh.mom[mp & 0x3fffffff];
    out[e] = (mp >> 30) & 1 ? -v : v;
  }
  if (threadIdx.x == 0) gflag[f] = sh.flag_nonfinite;
}

template <int V, int D, int PREC>
__global__ __launch_bounds__(64) void k_solve(FitArgs a, const double* gws, const int64_t* gofs,
                                              const int* gflag) {
  using S = Shape<V, D>;
  constexpr int NC = S::NC, NU = S::NU;
  constexpr int NPK = NU * (NU + 1) / 2;
  static_assert(NC <= kWaveSolveMaxNC, "wave solver limited to small models");
  __shared__ WaveShared<NC> w;
  const int lane = threadIdx.x;
  const int f = a.ids[blockIdx.x];
  const int64_t s0 = a.sample_off[f];
  const int64_t m = a.sample_off[f + 1] - s0;
  double* coef = a.coef + a.coef_off[f];
  if (gflag[f]) {
    for (int j = lane; j < NC; j += 64) coef[j] = __builtin_nan("");
    if (lane == 0) {
      a.status[f] = RP_FIT_NONFINITE_INPUT;
      if (a.resid) a.resid[f] = __builtin_nan("");
      if (a.iters) a.iters[f] = 0;
    }
    return;
  }
  const double* g = gws + gofs[f];
  for (int e = lane; e < NPK; e += 64) w.G[e] = g[e];
  wave_sync();
  // power-of-two equilibration of the unknowns; the mixed forms add a small
  // shift so the low-precision Gram is positive definite
  for (int j = lane; j < NU; j += 64) {
    double d = 1.0;
    if (j < NC) {
      const double gjj = w.G[pk(j, j)];
      if (gjj > 0.0 && isfinite(gjj)) d = ldexp(1.0, -(ilogb(gjj) / 2));
    }
    w.dsc[j] = d;
  }
  wave_sync();
  const double shift = (PREC == RP_FP64) ? 0.0 : 0x1p-20;
  for (int e = lane; e < NPK; e += 64) {
    int i = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
    while (i * (i + 1) / 2 > e) --i;
    while ((i + 1) * (i + 2) / 2 <= e) ++i;
    const int j = e - i * (i + 1) / 2;
    double v = w.G[e] * w.dsc[i] * w.dsc[j];
    if (i == j && i < NC) v += shift;
    w.G[e] = v;
  }
  wave_sync();
  const int ndrop = wave_sweep<NC>(w, PREC == RP_FP64 ? 1e-10 : 0.0);
  for (int j = lane; j < NC; j += 64) w.c[j] = w.drop[j] ? 0.0 : w.G[pk(NC, j)] * w.dsc[j];
  wave_sync();

  int it = 0;
  double last_rel = 0.0;
  if constexpr (PREC == RP_FP64) {
    for (it = 0; it < a.max_refine;) {
      wave_pass<V, D, PASS_RESIDUAL>(a, s0, m, w.c, w.r, nullptr, w.red);
      wave_precond<NC>(w, w.r, w.z);
      for (int j = lane; j < NC; j += 64) w.c[j] += w.z[j];
      wave_sync();
      ++it;
      const double dn = wave_maxabs<NC>(w.z), cn = wave_maxabs<NC>(w.c);
      last_rel = cn > 0.0 ? dn / cn : dn;
      if (dn <= a.tol * cn) break;
    }
  } else {
    wave_pass<V, D, PASS_RESIDUAL>(a, s0, m, w.c, w.r, nullptr, w.red);
    wave_precond<NC>(w, w.r, w.z);
    for (int j = lane; j < NC; j += 64) w.p[j] = w.z[j];
    wave_sync();
    double rz = wave_dot<NC>(w.r, w.z);
    for (it = 0; it < a.max_refine;) {
      wave_pass<V, D, PASS_PRODUCT>(a, s0, m, w.p, w.q, nullptr, w.red);
      const double pq = wave_dot<NC>(w.p, w.q);
      const double alpha = pq > 0.0 ? rz / pq : 0.0;
      for (int j = lane; j < NC; j += 64) {
        w.c[j] = fma(alpha, w.p[j], w.c[j]);
        w.r[j] = fma(-alpha, w.q[j], w.r[j]);
      }
      wave_sync();
      ++it;
      const double dn = fabs(alpha) * wave_maxabs<NC>(w.p), cn = wave_maxabs<NC>(w.c);
      last_rel = cn > 0.0 ? dn / cn : dn;
      if (dn <= a.tol * cn || !(pq > 0.0)) break;
      wave_precond<NC>(w, w.r, w.z);
      const double rz2 = wave_dot<NC>(w.r, w.z);
      const double beta = rz > 0.0 ? rz2 / rz : 0.0;
      rz = rz2;
      for (int j = lane; j < NC; j += 64) w.p[j] = fma(beta, w.p[j], w.z[j]);
      wave_sync();
    }
  }
  double resid = __builtin_nan("");
  double qmin = 1.0;
  if (a.check_q) resid = sqrt(wave_pass<V, D, PASS_CHECK>(a, s0, m, w.c, nullptr, &qmin, w.red));
  for (int j = lane; j < NC; j += 64) coef[j] = w.c[j];
  if (lane == 0) {
    int st = RP_FIT_OK;
    if (m < NC) st = RP_FIT_UNDERDETERMINED;
    else if (ndrop > 0) st = RP_FIT_RANK_DEFICIENT;
    else if (!(last_rel <= sqrt(a.tol))) st = RP_FIT_NOT_CONVERGED;
    else if (!(qmin > 0.0)) st = RP_FIT_Q_NONPOSITIVE;
    a.status[f] = st;
    if (a.resid) a.resid[f] = resid;
    if (a.iters) a.iters[f] = it;
  }
}

// ---------------------------------------------------------------------------
// Levenberg-Marquardt on the true loss, split form (one wave per fit)
// ---------------------------------------------------------------------------
enum LmState { LM_ACTIVE = 0, LM_CONVERGED = 1, LM_STOPPED = 2, LM_NONFINITE = 3 };

// sum_i (N_i/Q_i - y_i)^2 over one fit's samples by one wave; c in LDS.
template <int V, int D>
__device__ double wave_true_loss(const FitArgs& a, int64_t s0, int64_t m, const double* c,
                                 bool* finite_in) {
  using S = Shape<V, D>;
  const int lane = threadIdx.x & 63;
  double ss = 0.0;
  bool ok = true;
#pragma unroll 1
  for (int64_t i = lane; i < m; i += 64) {
    const int64_t s = s0 + i;
    double u[V];
#pragma unroll
    for (int k = 0; k < V; ++k) { u[k] = a.x[(int64_t)k * a.ldx + s]; ok = ok && isfinite(u[k]); }
    const double y = a.y[s];
    ok = ok && isfinite(y);
    double mo[S::NM];
    monomials<V, D, double>(u, mo);
    int zero;
    asm volatile("v_mov_b32 %0, 0" : "=v"(zero));
    const double* cz = c + zero;
    double n0 = 0.0, n1 = 0.0, q0 = 1.0, q1 = 0.0;
#pragma unroll
    for (int j = 0; j < S::NA; ++j) { if (j & 1) n1 = fma(cz[j], mo[j], n1); else n0 = fma(cz[j], mo[j], n0); }
#pragma unroll
    for (int j = 1; j < S::NM; ++j) { if (j & 1) q1 = fma(cz[S::NA + j - 1], mo[j], q1); else q0 = fma(cz[S::NA + j - 1], mo[j], q0); }
    const double r = (n0 + n1) / (q0 + q1) - y;
    ss = fma(r, r, ss);
  }
  if (finite_in) *finite_in = !__any(!ok);   // every lane's samples finite
  return wave_sum_dpp(ss);
}

template <int V, int D>
__global__ __launch_bounds__(64) void k_lm_init(FitArgs a) {
  using S = Shape<V, D>;
  __shared__ double c[S::NC];
  const int lane = threadIdx.x;
  const int f = a.ids[blockIdx.x];
  const int64_t s0 = a.sample_off[f];
  const int64_t m = a.sample_off[f + 1] - s0;
  const double* cg = a.coef + a.coef_off[f];
  for (int j = lane; j < S::NC; j += 64) c[j] = cg[j];
  wave_sync();
  bool finite_in = true;
  const double loss = wave_true_loss<V, D>(a, s0, m, c, &finite_in);
  if (lane == 0) {
    a.lm_loss[f] = loss;
    a.lm_lambda[f] = 0.0;
    a.lm_state[f] = finite_in ? LM_ACTIVE : LM_NONFINITE;
    a.lm_rejects[f] = 0;
    if (a.iters) a.iters[f] = 0;
  }
}

// One damped Gauss-Newton step per active fit: (J^T J + lambda diag) d = J^T r
// from the Gram formed at the current coefficients, accepted when the true
// loss does not increase.
template <int V, int D>
__global__ __launch_bounds__(64) void k_lm_step(FitArgs a, const double* gws, const int64_t* gofs,
                                                const int* gflag) {
  using S = Shape<V, D>;
  constexpr int NC = S::NC, NU = S::NU;
  constexpr int NPK = NU * (NU + 1) / 2;
  __shared__ WaveShared<NC> w;
  const int lane = threadIdx.x;
  const int f = a.ids[blockIdx.x];
  if (a.lm_state[f] != LM_ACTIVE) return;
  if (gflag[f]) {
    if (lane == 0) a.lm_state[f] = LM_NONFINITE;
    return;
  }
  const int64_t s0 = a.sample_off[f];
  const int64_t m = a.sample_off[f + 1] - s0;
  double* cg = a.coef + a.coef_off[f];
  const double lambda = a.lm_lambda[f];
  const double loss = a.lm_loss[f];
  const double* g = gws + gofs[f];
  for (int e = lane; e < NPK; e += 64) w.G[e] = g[e];
  wave_sync();
  for (int j = lane; j < NU; j += 64) {
    double d = 1.0;
    if (j < NC) {
      const double gjj = w.G[pk(j, j)];
      if (gjj > 0.0 && isfinite(gjj)) d = ldexp(1.0, -(ilogb(gjj) / 2));
    }
    w.dsc[j] = d;
  }
  wave_sync();
  for (int e = lane; e < NPK; e += 64) {
    int i = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
    while (i * (i + 1) / 2 > e) --i;
    while ((i + 1) * (i + 2) / 2 <= e) ++i;
    const int j = e - i * (i + 1) / 2;
    double v = w.G[e] * w.dsc[i] * w.dsc[j];
    if (i == j && i < NC) v *= (1.0 + lambda);
    w.G[e] = v;
  }
  wave_sync();
  wave_sweep<NC>(w, 1e-14);
  for (int j = lane; j < NC; j += 64)
    w.p[j] = cg[j] + (w.drop[j] ? 0.0 : w.G[pk(NC, j)] * w.dsc[j]);
  wave_sync();
  const double loss_new = wave_true_loss<V, D>(a, s0, m, w.p, nullptr);
  const bool accept = loss_new <= loss;
  if (accept)
    for (int j = lane; j < NC; j += 64) cg[j] = w.p[j];
  if (lane == 0) {
    if (a.iters) a.iters[f] += 1;
    if (accept) {
      const double change = loss - loss_new;
      double lam = lambda * 0.1;
      if (lam < 1e-12) lam = 0.0;
      a.lm_lambda[f] = lam;
      a.lm_loss[f] = loss_new;
      a.lm_rejects[f] = 0;
      if (change <= a.rtol * loss_new) a.lm_state[f] = LM_CONVERGED;
    } else {
      a.lm_lambda[f] = lambda == 0.0 ? 1e-6 : lambda * 10.0;
      const int rj = a.lm_rejects[f] + 1;
      a.lm_rejects[f] = rj;
      if (rj > 30) a.lm_state[f] = LM_STOPPED;
    }
  }
}

template <int V, int D>
__global__ __launch_bounds__(64) void k_lm_final(FitArgs a) {
  using S = Shape<V, D>;
  const int f = a.ids[blockIdx.x];
  if (threadIdx.x != 0) return;
  const int64_t m = a.sample_off[f + 1] - a.sample_off[f];
  const int st = a.lm_state[f];
  int out = st == LM_CONVERGED ? RP_FIT_OK : RP_FIT_NOT_CONVERGED;
  if (st == LM_NONFINITE) out = RP_FIT_NONFINITE_INPUT;
  else if (m < S::NC) out = RP_FIT_UNDERDETERMINED;
  a.status[f] = out;
  a.resid[f] = st == LM_NONFINITE ? __builtin_nan("") : a.lm_loss[f];
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
    for (int j = 1; j < S::NM; ++j) Q = fma(c[S::NA + j - 1], mo[j], Q);
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
template <int V, int D, int MODE>
__global__ __launch_bounds__(kThreads) void k_loss(FitArgs a, const float* coef, float* loss,
                                                   const float* dloss, float* dcoef) {
  using S = Shape<V, D>;
  __shared__ float c[S::NC];
  __shared__ float red[kWaves * (S::NC + 1)];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int f = a.ids[blockIdx.x];
  const int64_t s0 = a.sample_off[f];
  const int64_t m = a.sample_off[f + 1] - s0;
  const int64_t co = a.coef_off[f];
  for (int j = tid; j < S::NC; j += kThreads) c[j] = coef[co + j];
  __syncthreads();
  float g[MODE == RP_LOSS_BWD ? S::NC : 1];
#pragma unroll
  for (int j = 0; j < (MODE == RP_LOSS_BWD ? S::NC : 1); ++j) g[j] = 0.0f;
  float ls = 0.0f;
  for (int64_t i = tid; i < m; i += kThreads) {
    const int64_t s = s0 + i;
    float u[V];
#pragma unroll
    for (int k = 0; k < V; ++k) u[k] = (float)a.x[(int64_t)k * a.ldx + s];
    float mo[S::NM];
    monomials<V, D, float>(u, mo);
    float N = 0.0f, Q = 1.0f;
#pragma unroll
    for (int j = 0; j < S::NA; ++j) N = fmaf(c[j], mo[j], N);
#pragma unroll
    for (int j = 1; j < S::NM; ++j) Q = fmaf(c[S::NA + j - 1], mo[j], Q);
    const float iq = 1.0f / Q;
    const float fv = N * iq;
    const float r = fv - (float)a.y[s];
    ls = fmaf(r, r, ls);
    if constexpr (MODE == RP_LOSS_BWD) {
      const float gn = 2.0f * r * iq;          // d loss / d alpha_j = gn * m_j
      const float gd = -gn * fv;               // d loss / d beta_j  = gd * m_j
#pragma unroll
      for (int j = 0; j < S::NA; ++j) g[j] = fmaf(gn, mo[j], g[j]);
#pragma unroll
      for (int j = 1; j < S::NM; ++j) g[S::NA + j - 1] = fmaf(gd, mo[j], g[S::NA + j - 1]);
    }
  }
  auto wsum = [](float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
  };
  ls = wsum(ls);
  if (lane == 0) red[wave * (S::NC + 1) + S::NC] = ls;
  if constexpr (MODE == RP_LOSS_BWD) {
#pragma unroll
    for (int j = 0; j < S::NC; ++j) {
      const float t = wsum(g[j]);
      if (lane == 0) red[wave * (S::NC + 1) + j] = t;
    }
  }
  __syncthreads();
  if (tid == 0) {
    float t = 0.0f;
    for (int w = 0; w < kWaves; ++w) t += red[w * (S::NC + 1) + S::NC];
    loss[f] = t;
  }
  if constexpr (MODE == RP_LOSS_BWD) {
    const float up = dloss ? dloss[f] : 1.0f;
    for (int j = tid; j < S::NC; j += kThreads) {
      float t = 0.0f;
      for (int w = 0; w < kWaves; ++w) t += red[w * (S::NC + 1) + j];
      dcoef[co + j] = up * t;
    }
  }
}

// ---------------------------------------------------------------------------
// host launchers for one shape
// ---------------------------------------------------------------------------
template <int V, int D, int PREC>
int launch_split(const FitArgs& a, int nblocks, double* gws, const int64_t* gofs, int* gflag,
                 hipStream_t s) {
  if (PREC == RP_FP64 && a.gram_algo != RP_GRAM_MFMA && a.mom_map)
    hipLaunchKernelGGL((k_gram_mom<V, D, false>), dim3(nblocks), dim3(MomCfg<V, D, false>::NT), 0, s, a, gws, gofs, gflag);
  else
    hipLaunchKernelGGL((k_gram<V, D, PREC>), dim3(nblocks), dim3(kThreads), 0, s, a, gws, gofs, gflag);
  hipLaunchKernelGGL((k_solve<V, D, PREC>), dim3(nblocks), dim3(64), 0, s, a, gws, gofs, gflag);
  RP_CHECK_HIP(hipGetLastError());
  return RP_OK;
}

template <int V, int D>
int launch_shape_fit(int precision, const FitArgs& a, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return RP_OK;
  if constexpr (Shape<V, D>::NC <= kWaveSolveMaxNC) {
    if (a.gws) {
      switch (precision) {
        case RP_FP64: return launch_split<V, D, RP_FP64>(a, nblocks, a.gws, a.gofs, a.gflag, s);
        case RP_MIXED_FP32: return launch_split<V, D, RP_MIXED_FP32>(a, nblocks, a.gws, a.gofs, a.gflag, s);
        case RP_MIXED_BF16: return launch_split<V, D, RP_MIXED_BF16>(a, nblocks, a.gws, a.gofs, a.gflag, s);
        default: return set_error(RP_EINVAL, "unknown precision");
      }
    }
  }
  switch (precision) {
    case RP_FP64: hipLaunchKernelGGL((k_fit<V, D, RP_FP64>), dim3(nblocks), dim3(kThreads), 0, s, a); break;
    case RP_MIXED_FP32: hipLaunchKernelGGL((k_fit<V, D, RP_MIXED_FP32>), dim3(nblocks), dim3(kThreads), 0, s, a); break;
    case RP_MIXED_BF16: hipLaunchKernelGGL((k_fit<V, D, RP_MIXED_BF16>), dim3(nblocks), dim3(kThreads), 0, s, a); break;
    default: return set_error(RP_EINVAL, "unknown precision");
  }
  RP_CHECK_HIP(hipGetLastError());
  return RP_OK;
}

template <int V, int D>
int launch_shape_gram(int precision, const FitArgs& a, double* gram, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return RP_OK;
  switch (precision) {
    case RP_FP64:
      if (a.gram_algo != RP_GRAM_MFMA && a.mom_map)
        hipLaunchKernelGGL((k_gram_mom<V, D, false>), dim3(nblocks), dim3(MomCfg<V, D, false>::NT), 0, s, a, gram, a.gofs, a.gflag);
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
      hipLaunchKernelGGL((k_lm_init<V, D>), dim3(nblocks), dim3(64), 0, s, a);
      for (int it = 0; it < a.max_iter; ++it) {
        if (a.gram_algo != RP_GRAM_MFMA && a.mom_map)
          hipLaunchKernelGGL((k_gram_mom<V, D, true>), dim3(nblocks), dim3(MomCfg<V, D, true>::NT), 0, s, a,
                             a.gws, a.gofs, a.gflag);
        else
          hipLaunchKernelGGL((k_gram<V, D, RP_FP64, true>), dim3(nblocks), dim3(kThreads), 0, s, a,
                             a.gws, a.gofs, a.gflag);
        hipLaunchKernelGGL((k_lm_step<V, D>), dim3(nblocks), dim3(64), 0, s, a, a.gws, a.gofs,
                           a.gflag);
      }
      hipLaunchKernelGGL((k_lm_final<V, D>), dim3(nblocks), dim3(64), 0, s, a);
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
    hipLaunchKernelGGL((k_loss<V, D, RP_LOSS_FWD>), dim3(nblocks), dim3(kThreads), 0, s, a, coef, loss, dloss, dcoef);
  else
    hipLaunchKernelGGL((k_loss<V, D, RP_LOSS_BWD>), dim3(nblocks), dim3(kThreads), 0, s, a, coef, loss, dloss, dcoef);
  RP_CHECK_HIP(hipGetLastError());
  return RP_OK;
}

}  // namespace rp

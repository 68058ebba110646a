// rp_internal.h -- internal declarations of librpfit (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "../../include/rp.h"

namespace rp {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
int set_error(int code, const std::string& msg);
#define RP_CHECK_HIP(expr)                                                        \
  do {                                                                            \
    hipError_t _e = (expr);                                                       \
    if (_e != hipSuccess)                                                         \
      return ::rp::set_error(RP_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

// ---------------------------------------------------------------------------
// monomial enumeration (Section 4.2 model display, total-degree form)
// ---------------------------------------------------------------------------
constexpr int kMaxVarsHost = 8;

constexpr int binom(int n, int k) {
  if (k < 0 || k > n) return 0;
  long r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return (int)r;
}

// Visit every exponent vector of total degree <= d in v variables in graded
// order: degree t = 0..d, and within a degree the exponent of x1 descending,
// then x2 descending, ... (reverse-lexicographic walk over compositions of t).
template <class Emit>
constexpr void for_each_graded(int v, int d, Emit&& emit) {
  for (int t = 0; t <= d; ++t) {
    int e[kMaxVarsHost] = {};
    e[0] = t;
    for (;;) {
      emit(e);
      int i = -1;
      for (int k = v - 2; k >= 0; --k)
        if (e[k] > 0) { i = k; break; }
      if (i < 0) break;
      int rest = 0;
      for (int k = i + 1; k < v; ++k) { rest += e[k]; e[k] = 0; }
      e[i] -= 1;
      e[i + 1] = rest + 1;
    }
  }
}

// Device-side table for v <= 4, d <= 4: exponents plus a parent table so that
// monomial j = monomial parent[j] * u[var[j]] costs one multiplication.
constexpr int kMaxV = 4;
constexpr int kMaxD = 4;
constexpr int kMaxMono = 70;   // C(4+4, 4)

struct MonoTable {
  int n;
  int e[kMaxMono][kMaxV];
  int parent[kMaxMono];
  int var[kMaxMono];
};

constexpr MonoTable make_mono_table(int v, int d) {
  MonoTable T{};
  int n = 0;
  for_each_graded(v, d, [&](const int* e) {
    for (int k = 0; k < kMaxV; ++k) T.e[n][k] = k < v ? e[k] : 0;
    ++n;
  });
  T.n = n;
  for (int j = 1; j < n; ++j) {
    int k = 0;
    while (T.e[j][k] == 0) ++k;
    int want[kMaxV] = {T.e[j][0], T.e[j][1], T.e[j][2], T.e[j][3]};
    want[k] -= 1;
    for (int p = 0; p < j; ++p) {
      bool eq = true;
      for (int q = 0; q < kMaxV; ++q) eq = eq && T.e[p][q] == want[q];
      if (eq) { T.parent[j] = p; break; }
    }
    T.var[j] = k;
  }
  return T;
}

// Degree code D of a compiled model shape: the numerator's degree in bits
// 0-3 and the denominator's in bits 4-7, 0 there meaning the same as the
// numerator's (so D = d is the model of degree d over d).  Kernels compute
// the monomials up to the larger degree; the numerator takes the first
// C(v + dn, dn) of them and the denominator the first C(v + dq, dq) (the
// graded order puts every monomial of lower degree first).
constexpr int code_dn(int D) { return D & 15; }
constexpr int code_dq(int D) { return (D >> 4) ? (D >> 4) : (D & 15); }
constexpr int code_dmax(int D) { return code_dn(D) > code_dq(D) ? code_dn(D) : code_dq(D); }
constexpr int deg_code(int dn, int dq) { return dn == dq ? dn : (dn | (dq << 4)); }

template <int V, int D>
struct Mono {
  static constexpr int DM = code_dmax(D);
  static constexpr MonoTable T = make_mono_table(V, DM);
  static constexpr int N = binom(V + DM, DM);
  static_assert(T.n == N, "monomial count");
};

template <int V, int D, int J>
struct MonoAt {
  static constexpr int parent = Mono<V, D>::T.parent[J];
  static constexpr int var = Mono<V, D>::T.var[J];
};

// m[0..N) = monomials of u in the order above, one multiply each.
template <int V, int D, typename R, int... J>
__device__ __forceinline__ void monomials_impl(const R* u, R* m, std::integer_sequence<int, J...>) {
  ((m[J + 1] = m[MonoAt<V, D, J + 1>::parent] * u[MonoAt<V, D, J + 1>::var]), ...);
}

template <int V, int D, typename R>
__device__ __forceinline__ void monomials(const R* u, R* m) {
  m[0] = R(1);
  monomials_impl<V, D, R>(u, m, std::make_integer_sequence<int, Mono<V, D>::N - 1>{});
}

// Exponent table of any size (used for the moments of degree <= 2D).
template <int V, int D>
struct MonoBig {
  static constexpr int N = binom(V + D, D);
  int e[N][kMaxV];
};
template <int V, int D>
constexpr MonoBig<V, D> make_mono_big() {
  MonoBig<V, D> T{};
  int n = 0;
  for_each_graded(V, D, [&](const int* e) {
    for (int k = 0; k < kMaxV; ++k) T.e[n][k] = k < V ? e[k] : 0;
    ++n;
  });
  return T;
}

// Moment form of the augmented Gram.  Every entry of [A b]^T [A b] is a
// weighted moment sum_i w(i) m_e(u_i) with e the sum of the two columns'
// exponents.  The linear problem has w0 = 1, w1 = y, w2 = y^2 over every
// exponent of degree <= 2D (its right-hand-side entries reuse w1 and w2).
// The Jacobian rows (1/Q)[m, -f m'] with residual r = y - f have
// w0 = 1/Q^2, w1 = f/Q^2, w2 = f^2/Q^2, w3 = r/Q, w4 = f r/Q, w5 = r^2, and
// an entry needs only some weights at low degree: w1 pairs a numerator with a
// denominator column (degree >= 1), w2 two denominator columns (degree >= 2),
// w3 and w4 the right-hand side with one column (degree <= D, w4 >= 1) and w5
// only the constant.  So the exponents fall in four bands, each with its
// weights: e = 0 {w0, w3, w5}; degree 1 {w0, w1, w3, w4}; degree 2..D
// {w0, ..., w4}; degree D+1..2D {w0, w1, w2} (the linear problem: {w0, w1,
// w2} in every band).  Moment-weight pairs are ordered exponent-major (graded
// order: e = 0, then the v exponents of degree 1, ...) so a lane's group
// shares each monomial between weights.
template <bool GN>
struct MomentPairs {
  static constexpr int kZeroWeights = 3;           // e = 0
  static constexpr int kOneWeights = GN ? 4 : 3;   // degree 1
  static constexpr int kLowWeights = GN ? 5 : 3;   // degree 2..D
  // weight of slot s in band b (b: 0 e = 0, 1 degree 1, 2 degree 2..D, 3 above)
  static constexpr int weight(int b, int s) {
    if (!GN) return s;
    constexpr int w0[3] = {0, 3, 5}, w1[4] = {0, 1, 3, 4};
    return b == 0 ? w0[s] : b == 1 ? w1[s] : s;
  }
  // slot of weight w in band b, -1 if the band does not carry it
  static constexpr int slot(int b, int w) {
    const int n = b == 0 ? kZeroWeights : b == 1 ? kOneWeights : b == 2 ? kLowWeights : 3;
    for (int s = 0; s < n; ++s)
      if (weight(b, s) == w) return s;
    return -1;
  }
};
template <int V, int D, bool GN>
struct MomentShape {
  static constexpr int DM = code_dmax(D);   // moments up to degree 2 DM
  static constexpr int NM1 = binom(V + DM, DM);
  static constexpr int NM2 = binom(V + 2 * DM, 2 * DM);
  static constexpr int NPAIR = MomentPairs<GN>::kZeroWeights + MomentPairs<GN>::kOneWeights * V +
                               MomentPairs<GN>::kLowWeights * (NM1 - 1 - V) + 3 * (NM2 - NM1);
  // Waves per workgroup: a multiple of the four SIMDs of a compute unit, so
  // that the waves between two barriers are spread evenly over them.  Up to
  // 64 pairs per lane fit four waves (three resident per SIMD), up to 75 four
  // waves at two resident per SIMD (the Jacobian Gram of degree 3/3 in three
  // variables, 287 pairs: fewer waves sharing each sample's power table beat
  // more waves in flight); beyond that eight waves take at most 40 pairs each
  // (four resident per SIMD).
  static constexpr int NWV = NPAIR <= 4 * 75 ? 4 : 8;
  static constexpr int PLMAX = NWV == 4 ? (NPAIR <= 4 * 64 ? 64 : 75) : 40;   // accumulators per lane
  static constexpr int NG0 = (NPAIR + PLMAX - 1) / PLMAX;
  static constexpr int NGROUP = (NG0 + NWV - 1) / NWV * NWV;   // whole passes
  static constexpr int PL = (NPAIR + NGROUP - 1) / NGROUP;
  static constexpr int NPASS = NGROUP / NWV;
};
// Band of exponent index e (graded order; nm1 exponents of degree <= D, v of
// degree 1).
constexpr int moment_band(int e, int nm1, int v) { return e == 0 ? 0 : e <= v ? 1 : e < nm1 ? 2 : 3; }
// Index of pair (e, w) (w the weight, carried by e's band) in the ordering above.
template <bool GN>
constexpr int moment_pair_index(int e, int w, int nm1, int v) {
  using P = MomentPairs<GN>;
  const int b = moment_band(e, nm1, v), s = P::slot(b, w);
  if (b == 0) return s;
  if (b == 1) return P::kZeroWeights + (e - 1) * P::kOneWeights + s;
  if (b == 2) return P::kZeroWeights + v * P::kOneWeights + (e - 1 - v) * P::kLowWeights + s;
  return P::kZeroWeights + v * P::kOneWeights + (nm1 - 1 - v) * P::kLowWeights + (e - nm1) * 3 + s;
}
// Inverse: pair p -> (e, w).
template <bool GN>
constexpr void moment_pair_of(int p, int nm1, int v, int& e, int& w) {
  using P = MomentPairs<GN>;
  if (p < P::kZeroWeights) { e = 0; w = P::weight(0, p); return; }
  p -= P::kZeroWeights;
  if (p < v * P::kOneWeights) { e = 1 + p / P::kOneWeights; w = P::weight(1, p % P::kOneWeights); return; }
  p -= v * P::kOneWeights;
  if (p < (nm1 - 1 - v) * P::kLowWeights) {
    e = 1 + v + p / P::kLowWeights;
    w = P::weight(2, p % P::kLowWeights);
    return;
  }
  p -= (nm1 - 1 - v) * P::kLowWeights;
  e = nm1 + p / 3;
  w = P::weight(3, p % 3);
}

// Shape of a linearised model of degree code D (see code_dn).
template <int V, int D>
struct Shape {
  static constexpr int DN = code_dn(D), DQ = code_dq(D), DM = code_dmax(D);
  static constexpr int NM = Mono<V, D>::N;               // monomials computed (degree <= DM)
  static constexpr int NA = binom(V + DN, DN);           // numerator unknowns
  static constexpr int NQ = binom(V + DQ, DQ);           // denominator monomials
  static constexpr int NB = NQ - 1;                      // denominator unknowns (q0 = 1)
  static constexpr int NC = NA + NB;                     // unknowns
  static constexpr int NU = NC + 1;                      // augmented with the rhs column
};

// ---------------------------------------------------------------------------
// objects behind the opaque ABI handles
// ---------------------------------------------------------------------------
struct Bucket {            // fits of one compiled shape
  int nvars = 0, deg = 0;          // deg: the degree code (deg_code)
  int deg_num = 0, deg_den = 0;
  int count = 0;
  int32_t* d_ids = nullptr;   // device [count] fit indices, decreasing cost
  int32_t* d_mom_map = nullptr;     // moment -> packed Gram map, linear form
  int32_t* d_mom_map_gn = nullptr;  // the same for the Jacobian form
  int gram_algo = RP_GRAM_MOMENTS;  // tuned way of forming the FP64 Gram
  int precision = RP_FP64;          // tuned form of RP_AUTO
  int form_us[4] = {-1, -1, -1, -1};  // measured: FP64 moments, FP64 MFMA, FP32, BF16
  // fits the fit kernels flag for the FP64 re-solve: [0] count, [1] finished
  // re-solve workgroups, then the list (count + 2 ints, zero between calls)
  int32_t* d_resolve = nullptr;
};

// Host map from each packed augmented-Gram entry to (moment pair, sign):
// value = pair | (negative << 30).
std::vector<int32_t> moment_scatter_map(int v, int dn, int dq, bool gn);

}  // namespace rp

struct rp_ctx_s {
  int device = 0;
  int num_cu = 0;
  int max_lds = 0;
};

struct rp_plan_s {
  rp_ctx ctx = nullptr;
  int num_fits = 0;
  int64_t total_samples = 0;
  std::vector<int64_t> h_sample_off, h_coef_off, h_a_off, h_gram_off;
  std::vector<int32_t> h_nvars, h_deg_num, h_deg_den;
  int64_t* d_sample_off = nullptr;
  int64_t* d_coef_off = nullptr;
  int64_t* d_a_off = nullptr;
  std::vector<rp::Bucket> buckets;
  // workspace of the split fit form: packed augmented Gram per fit
  double* d_gws = nullptr;
  int64_t* d_gofs = nullptr;
  int* d_gflag = nullptr;
  // Levenberg-Marquardt state: lambda, loss (doubles), state, rejects (ints)
  double* d_lm = nullptr;
  int* d_lm_int = nullptr;
  // per-sample residual scratch of the grouped passes (models of more than
  // kPassGroupMax unknowns; null when the plan has none)
  double* d_wres = nullptr;
};

struct rp_graph_s {
  rp_plan plan = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

struct rp_prog_s {
  rp_ctx ctx = nullptr;
  int template_id = 0, num_programs = 0, num_metrics = 0, nvars = 0;
  int shape_v = 0, shape_d = 0;            // common (nvars, degree) of all metrics
  const double* d_coef = nullptr;          // caller's device array
  const double* d_hw = nullptr;            // caller's device array
  std::vector<int64_t> h_coef_off;
  std::vector<int32_t> h_deg_num, h_deg_den;
  int64_t* d_coef_off = nullptr;
  double scale[8] = {};
  int32_t* d_ab = nullptr;                 // [P*L*2] numerator/denominator term counts
};

namespace rp {

struct FitArgs {
  const double* x;
  int64_t ldx;
  const double* y;
  const int64_t* sample_off;
  const int64_t* coef_off;
  const int32_t* ids;
  double* coef;
  int32_t* status;
  double* resid;
  int32_t* iters;
  int32_t max_refine;
  double tol;
  int32_t check_q;
  // refinement on the true loss
  int32_t max_iter;
  double rtol;
  // split-form workspace: packed augmented Gram per fit and non-finite flags
  double* gws;
  const int64_t* gofs;
  int* gflag;
  // moment form: packed-Gram scatter map of the launched bucket
  const int32_t* mom_map;
  int gram_algo;
  // Levenberg-Marquardt state per fit (split refine form)
  double* lm_lambda;
  double* lm_loss;
  int* lm_state;
  int* lm_rejects;
  // FP64 re-solve list of the launched bucket (null: no re-solve pass);
  // refinement stops once a correction is <= stop_rel * max|coef|
  int32_t* resolve;
  double stop_rel;
  // Levenberg-Marquardt launches of one refine call: the first Gram also
  // initialises the per-fit state, the last step also writes the outputs
  int32_t lm_first, lm_last;
  // per-sample scratch (global sample index) of the passes that split a
  // large model's unknowns into groups: the first group stores each
  // sample's residual, the later groups read it (null: they recompute it)
  double* wres;
};

// Internal precision code of launch_gram: the Jacobian Gram of the true loss
// (FP64) at the coefficients in FitArgs::coef.
constexpr int kGramJacobian = 100;

// Unknowns accumulated per sweep over the samples by the passes of the
// larger models (one workgroup per fit): more are split into groups.
constexpr int kPassGroupMax = 48;

// launchers (one per compiled shape; defined in the generated kernel units)
int launch_fit(int v, int d, int precision, const FitArgs& a, int nblocks, hipStream_t s);
int launch_gram(int v, int d, int precision, const FitArgs& a, double* gram, int nblocks, hipStream_t s);
int launch_refine(int v, int d, const FitArgs& a, int nblocks, hipStream_t s);
int launch_design(int v, int d, int precision, const FitArgs& a, void* A, const int64_t* a_off,
                  void* rhs, int nblocks, hipStream_t s);
int launch_loss(int v, int d, const FitArgs& a, const float* coef, float* loss, const float* dloss,
                float* dcoef, int mode, int nblocks, hipStream_t s);
int launch_eval(const rp_prog_s* p, int sense, const rp_prog_s* tie, int tie_sense,
                const double* n_grid, int num_n, const int32_t* cand, int num_cand, int cand_dim,
                int precision, int32_t* argmin, double* best, double* second, double* values,
                hipStream_t s);

// The fit entry point without allocation keeps its scratch in a device
// array; with `device` current, look up that device's copy (rp_create).
int static_scratch_init(int device);

// Compiled model shapes: equal degrees 1..4 in 1..4 variables, and degrees
// differing by one up to 3 in 1..3 variables.
inline bool shape_supported(int v, int dn, int dq) {
  if (v < 1 || v > kMaxV || dn < 1 || dq < 1) return false;
  if (dn == dq) return dn <= kMaxD;
  return v <= 3 && dn <= 3 && dq <= 3 && (dn - dq == 1 || dq - dn == 1);
}

}  // namespace rp

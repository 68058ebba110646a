// rp_eval.hip -- exhaustive evaluation of rational programs over a candidate
// set and selection of the minimiser per (program, data size)
// (Section 3.3, steps 4-5; Section 4.3 "runtime optimization").
//
// One workgroup scores every candidate of one (program, data size) pair: the
// program's metric coefficients are staged in LDS (zero-padded to a common
// length so every lane runs the same static loop), each lane evaluates
// candidates in strides of 256, and a wave64 shuffle reduction followed by an
// LDS reduction across the four waves yields (best, index, second).
#include <climits>
#include <cmath>

#include "rp_internal.h"

namespace rp {

constexpr int kEvalThreads = 256;
constexpr int kEvalWaves = kEvalThreads / 64;
constexpr int kMaxMetrics = RP_NUM_METRICS;

struct EvalArgs {
  int template_id;
  int L;                    // metrics per program
  int num_n, num_cand, cand_dim;
  const double* coef;       // caller's coefficients
  const int64_t* coef_off;  // [P*L + 1]
  const int32_t* ab;        // [P*L*2] numerator / denominator term counts
  const double* hw;         // [P*RP_HW_COUNT] or null
  const double* n_grid;
  const int32_t* cand;
  double inv_scale[4];
  int32_t* argmin;
  double* best;
  double* second;
  double* values;           // optional [P*num_n*num_cand]
  double sense;             // +1: smallest E wins, -1: largest
  // optional second program breaking exact ties of E (same candidates)
  int tie_template;         // -1 when absent
  int tie_L;
  const double* tie_coef;
  const int64_t* tie_coef_off;
  const int32_t* tie_ab;
  const double* tie_hw;
  double tie_sense;
};

#include "rp_templates.h"

// (best key, tie key, index, second key); keys are sense-adjusted so that
// smaller always wins, and the order is (key, tie key, index).
struct Cand3 {
  double bv; double bt; int bi; double sv;
};

__device__ __forceinline__ Cand3 cand_merge(Cand3 a, Cand3 b) {
  const bool b_wins = b.bv < a.bv || (b.bv == a.bv && (b.bt < a.bt || (b.bt == a.bt && b.bi < a.bi)));
  Cand3 r;
  if (b_wins) { r.bv = b.bv; r.bt = b.bt; r.bi = b.bi; r.sv = fmin(b.sv, a.bv); }
  else { r.bv = a.bv; r.bt = a.bt; r.bi = a.bi; r.sv = fmin(a.sv, b.bv); }
  return r;
}

__device__ __forceinline__ Cand3 cand_shfl_xor(Cand3 c, int o) {
  Cand3 r;
  r.bv = __shfl_xor(c.bv, o, 64);
  r.bt = __shfl_xor(c.bt, o, 64);
  r.bi = __shfl_xor(c.bi, o, 64);
  r.sv = __shfl_xor(c.sv, o, 64);
  return r;
}

__device__ Cand3 block_argmin(Cand3 c, Cand3* red) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) c = cand_merge(c, cand_shfl_xor(c, o));
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = c;
  __syncthreads();
  Cand3 r = red[0];
#pragma unroll
  for (int k = 1; k < kEvalWaves; ++k) r = cand_merge(r, red[k]);
  __syncthreads();
  return r;
}

template <int V, int DM>
struct EvalCfg {
  static constexpr int NM = Mono<V, DM>::N;
  static constexpr int STRIDE = 2 * NM - 1;
};

// Stage program p's metric coefficients, zero-padded to STRIDE per metric
// (L metrics per program; ab, coef, coef_off of the primary or tie program).
template <int V, int DM, typename R>
__device__ void stage_coefs(int L, const int32_t* ab, const double* coef, const int64_t* coef_off,
                            int p, R* cf, int Lmax) {
  constexpr int NM = EvalCfg<V, DM>::NM, STRIDE = EvalCfg<V, DM>::STRIDE;
  for (int e = threadIdx.x; e < Lmax * STRIDE; e += kEvalThreads) {
    const int l = e / STRIDE, j = e % STRIDE;
    R v = R(0);
    if (l < L) {
      const int idx = p * L + l;
      const int na = ab[2 * idx], nb = ab[2 * idx + 1];
      const double* c = coef + coef_off[idx];
      if (j < NM) { if (j < na) v = (R)c[j]; }
      else if (j - NM < nb) v = (R)c[na + (j - NM)];
    }
    cf[e] = v;
  }
}

template <int V, int DM, typename R>
__device__ void stage_coefs(const EvalArgs& a, int p, R* cf, int Lmax) {
  stage_coefs<V, DM, R>(a.L, a.ab, a.coef, a.coef_off, p, cf, Lmax);
}

// metric slots of a template
template <int TPL>
constexpr int tpl_metrics() {
  return TPL == RP_TEMPLATE_MWPCWP ? kMaxMetrics : TPL == RP_TEMPLATE_OCCUPANCY ? 2 : 1;
}
constexpr int kNoTie = -1;

// Value E of the program for candidate c at data size n.  Lanes share the LDS
// coefficient table cf[l * STRIDE + j] (numerator j < NM, denominator term j
// at NM + j - 1, zero-padded); the monomials of u are computed once and reused
// by every metric.
template <int V, int DM, int TPL, typename R>
__device__ __forceinline__ R score(const EvalArgs& a, const R* cf, const R* hw, double n, int c,
                                   R* gslot, int gstride) {
  constexpr int NM = Mono<V, DM>::N;
  constexpr int STRIDE = 2 * NM - 1;
  constexpr int LMAX = tpl_metrics<TPL>();
  R u[V], raw[V];
  u[0] = (R)(n * a.inv_scale[0]);
  raw[0] = (R)n;
#pragma unroll
  for (int k = 1; k < V; ++k) {
    const double rv = (double)a.cand[(int64_t)c * a.cand_dim + (k - 1)];
    raw[k] = (R)rv;
    u[k] = (R)(rv * a.inv_scale[k]);
  }
  R mo[NM];
  monomials<V, DM, R>(u, mo);
  // One metric at a time (the loop is kept rolled): the block-uniform
  // coefficient table is read from LDS where it is used and each metric value
  // is parked in this lane's LDS slot, so the template below sees 16 values
  // without the compiler interleaving 16 x STRIDE coefficient loads.
  R g[LMAX];
  if constexpr (TPL == RP_TEMPLATE_SINGLE) {
    R nn = R(0), q = R(1);
#pragma unroll
    for (int j = 0; j < NM; ++j) nn = fma(cf[j], mo[j], nn);
#pragma unroll
    for (int j = 1; j < NM; ++j) q = fma(cf[NM + j - 1], mo[j], q);
    if (!(q > R(0))) return (R)INFINITY;     // Q <= 0: the candidate is infeasible
    g[0] = nn / q;
  } else if constexpr (TPL == RP_TEMPLATE_OCCUPANCY) {
#pragma unroll
    for (int l = 0; l < 2; ++l) {
      const R* cl = cf + l * STRIDE;
      R nn = R(0), q = R(1);
#pragma unroll
      for (int j = 0; j < NM; ++j) nn = fma(cl[j], mo[j], nn);
#pragma unroll
      for (int j = 1; j < NM; ++j) q = fma(cl[NM + j - 1], mo[j], q);
      g[l] = nn / q;
    }
  } else {
#pragma unroll 1
    for (int l = 0; l < LMAX; ++l) {
      const R* cl = cf + l * STRIDE;
      R nn = R(0), q = R(1);
#pragma unroll
      for (int j = 0; j < NM; ++j) nn = fma(cl[j], mo[j], nn);
#pragma unroll
      for (int j = 1; j < NM; ++j) q = fma(cl[NM + j - 1], mo[j], q);
      gslot[l * gstride] = nn / q;
    }
#pragma unroll
    for (int l = 0; l < LMAX; ++l) g[l] = gslot[l * gstride];
  }
  if constexpr (TPL == RP_TEMPLATE_SINGLE) return g[0];
  else if constexpr (TPL == RP_TEMPLATE_OCCUPANCY) return block_occupancy<R>(g, hw, raw[1], raw[2]);
  else return mwpcwp_cycles<R>(g, hw, raw[1], raw[2]);
}

template <int V, int DM, int TPL, int TTPL>
__global__ __launch_bounds__(kEvalThreads) void k_eval_f64(EvalArgs a) {
  constexpr int STRIDE = EvalCfg<V, DM>::STRIDE;
  constexpr int LMAX = tpl_metrics<TPL>();
  constexpr int TLMAX = TTPL == kNoTie ? 1 : tpl_metrics<TTPL>();
  static_assert(TTPL != RP_TEMPLATE_MWPCWP, "tie programs are single rationals or occupancy");
  __shared__ double cf[LMAX * STRIDE];
  __shared__ double hw[RP_HW_COUNT];
  __shared__ double tcf[TTPL == kNoTie ? 1 : TLMAX * STRIDE];
  __shared__ double thw[RP_HW_COUNT];
  __shared__ Cand3 red[kEvalWaves];
  __shared__ double gbuf[TPL == RP_TEMPLATE_MWPCWP ? kMaxMetrics * kEvalThreads : 1];
  const int j = blockIdx.x, p = blockIdx.y;
  stage_coefs<V, DM, double>(a, p, cf, LMAX);
  if (TPL != RP_TEMPLATE_SINGLE && threadIdx.x < RP_HW_COUNT)
    hw[threadIdx.x] = a.hw[(int64_t)p * RP_HW_COUNT + threadIdx.x];
  if constexpr (TTPL != kNoTie) {
    stage_coefs<V, DM, double>(a.tie_L, a.tie_ab, a.tie_coef, a.tie_coef_off, p, tcf, TLMAX);
    if (TTPL != RP_TEMPLATE_SINGLE && threadIdx.x < RP_HW_COUNT)
      thw[threadIdx.x] = a.tie_hw[(int64_t)p * RP_HW_COUNT + threadIdx.x];
  }
  __syncthreads();
  const double n = a.n_grid[j];
  // tie key of candidate k (sense-adjusted; a non-finite value ranks last)
  auto tie_key = [&](int k) -> double {
    if constexpr (TTPL == kNoTie) {
      return 0.0;
    } else {
      const double t = a.tie_sense * score<V, DM, TTPL, double>(a, tcf, thw, n, k, nullptr, 0);
      return isfinite(t) ? t : INFINITY;
    }
  };
  Cand3 c{INFINITY, 0.0, INT_MAX, INFINITY};
  bool bt_known = TTPL == kNoTie;
  const int64_t row = ((int64_t)p * a.num_n + j) * a.num_cand;
#pragma unroll 1
  for (int k = threadIdx.x; k < a.num_cand; k += kEvalThreads) {
    const double v = score<V, DM, TPL, double>(a, cf, hw, n, k, gbuf + threadIdx.x, kEvalThreads);
    if (a.values) a.values[row + k] = v;
    const double key = a.sense * v;
    if (!isfinite(key)) continue;
    if (key < c.bv) {
      c.sv = fmin(c.sv, c.bv);
      c.bv = key; c.bi = k; c.bt = 0.0;
      bt_known = TTPL == kNoTie;
    } else if (key == c.bv) {
      // exact tie of E: the tie program decides (the lane scans k upwards,
      // so the lower index is the incumbent)
      if (!bt_known) { c.bt = tie_key(c.bi); bt_known = true; }
      const double t = tie_key(k);
      c.sv = fmin(c.sv, key);
      if (t < c.bt) { c.bi = k; c.bt = t; }
    } else {
      c.sv = fmin(c.sv, key);
    }
  }
  if (!bt_known && c.bi != INT_MAX) c.bt = tie_key(c.bi);
  c = block_argmin(c, red);
  if (threadIdx.x == 0) {
    const int64_t o = (int64_t)p * a.num_n + j;
    a.argmin[o] = c.bi == INT_MAX ? -1 : c.bi;
    a.best[o] = a.sense * c.bv;
    a.second[o] = a.sense * c.sv;
  }
}

// FP32 scan keeping each lane's four best (value, index), merged across the
// block; the survivors are re-scored in FP64 and the FP64 minimum is kept.
struct Top4 {
  float v[4];
  int i[4];
};

__device__ __forceinline__ void top4_insert(Top4& t, float v, int i) {
  // keep ascending by (value, index)
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const bool less = v < t.v[s] || (v == t.v[s] && i < t.i[s]);
    const float tv = t.v[s];
    const int ti = t.i[s];
    if (less) { t.v[s] = v; t.i[s] = i; v = tv; i = ti; }
  }
}

template <int V, int DM, int TPL>
__global__ __launch_bounds__(kEvalThreads) void k_eval_f32(EvalArgs a) {
  constexpr int STRIDE = EvalCfg<V, DM>::STRIDE;
  constexpr int LMAX = tpl_metrics<TPL>();
  __shared__ float cf[LMAX * STRIDE];
  __shared__ double cfd[LMAX * STRIDE];
  __shared__ float hw[RP_HW_COUNT];
  __shared__ double hwd[RP_HW_COUNT];
  __shared__ Top4 wtop[kEvalWaves];
  __shared__ double resc[4];
  __shared__ int surv[4];
  __shared__ float gbuf[TPL == RP_TEMPLATE_MWPCWP ? kMaxMetrics * kEvalThreads : 1];
  __shared__ double gbufd[TPL == RP_TEMPLATE_MWPCWP ? kMaxMetrics * 4 : 1];
  const int j = blockIdx.x, p = blockIdx.y;
  stage_coefs<V, DM, float>(a, p, cf, LMAX);
  stage_coefs<V, DM, double>(a, p, cfd, LMAX);
  if (TPL != RP_TEMPLATE_SINGLE && threadIdx.x < RP_HW_COUNT) {
    const double h = a.hw[(int64_t)p * RP_HW_COUNT + threadIdx.x];
    hw[threadIdx.x] = (float)h;
    hwd[threadIdx.x] = h;
  }
  __syncthreads();
  const double n = a.n_grid[j];
  Top4 t;
#pragma unroll
  for (int s = 0; s < 4; ++s) { t.v[s] = INFINITY; t.i[s] = INT_MAX; }
  for (int k = threadIdx.x; k < a.num_cand; k += kEvalThreads) {
    const float v = (float)a.sense * score<V, DM, TPL, float>(a, cf, hw, n, k, gbuf + threadIdx.x, kEvalThreads);
    if (isfinite(v)) top4_insert(t, v, k);
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    Top4 u;
#pragma unroll
    for (int s = 0; s < 4; ++s) { u.v[s] = __shfl_xor(t.v[s], o, 64); u.i[s] = __shfl_xor(t.i[s], o, 64); }
#pragma unroll
    for (int s = 0; s < 4; ++s) top4_insert(t, u.v[s], u.i[s]);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) wtop[w] = t;
  __syncthreads();
  if (threadIdx.x < 4) {
    Top4 m = wtop[0];
    for (int k = 1; k < kEvalWaves; ++k)
      for (int s = 0; s < 4; ++s) top4_insert(m, wtop[k].v[s], wtop[k].i[s]);
    const int idx = m.i[threadIdx.x];
    resc[threadIdx.x] = idx == INT_MAX ? INFINITY
                                       : a.sense * score<V, DM, TPL, double>(a, cfd, hwd, n, idx, gbufd + threadIdx.x, 4);
    surv[threadIdx.x] = idx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    Cand3 c{INFINITY, 0.0, INT_MAX, INFINITY};
    for (int s = 0; s < 4; ++s) {
      const int idx = surv[s];
      if (idx != INT_MAX && isfinite(resc[s])) c = cand_merge(c, Cand3{resc[s], 0.0, idx, INFINITY});
    }
    const int64_t o = (int64_t)p * a.num_n + j;
    a.argmin[o] = c.bi == INT_MAX ? -1 : c.bi;
    a.best[o] = a.sense * c.bv;
    a.second[o] = a.sense * c.sv;
  }
}

template <int V, int DM, int TPL, int TTPL>
static int launch_eval_t(const EvalArgs& a, int P, int precision, hipStream_t s) {
  dim3 grid(a.num_n, P);
  if (precision == RP_FP64) {
    hipLaunchKernelGGL((k_eval_f64<V, DM, TPL, TTPL>), grid, dim3(kEvalThreads), 0, s, a);
  } else {
    if constexpr (TTPL != kNoTie) return set_error(RP_EINVAL, "a tie program needs the FP64 form");
    else hipLaunchKernelGGL((k_eval_f32<V, DM, TPL>), grid, dim3(kEvalThreads), 0, s, a);
  }
  RP_CHECK_HIP(hipGetLastError());
  return RP_OK;
}

template <int TPL, int V, int DM>
static int eval_dispatch_tie(const EvalArgs& a, int P, int precision, hipStream_t s) {
  switch (a.tie_template) {
    case kNoTie: return launch_eval_t<V, DM, TPL, kNoTie>(a, P, precision, s);
    case RP_TEMPLATE_SINGLE: return launch_eval_t<V, DM, TPL, RP_TEMPLATE_SINGLE>(a, P, precision, s);
    case RP_TEMPLATE_OCCUPANCY:
      if constexpr (V == 3) return launch_eval_t<V, DM, TPL, RP_TEMPLATE_OCCUPANCY>(a, P, precision, s);
      break;
  }
  return set_error(RP_EUNSUPPORTED, "tie program template not compiled in for this shape");
}

template <int TPL, int V>
static int eval_dispatch_d(int dm, const EvalArgs& a, int P, int precision, hipStream_t s) {
  switch (dm) {
    case 1: return eval_dispatch_tie<TPL, V, 1>(a, P, precision, s);
    case 2: return eval_dispatch_tie<TPL, V, 2>(a, P, precision, s);
    case 3: return eval_dispatch_tie<TPL, V, 3>(a, P, precision, s);
    case 4: return eval_dispatch_tie<TPL, V, 4>(a, P, precision, s);
  }
  return set_error(RP_EUNSUPPORTED, "metric degree not compiled in");
}

int launch_eval(const rp_prog_s* pr, int sense, const rp_prog_s* tie, int tie_sense,
                const double* n_grid, int num_n, const int32_t* cand, int num_cand, int cand_dim,
                int precision, int32_t* argmin, double* best, double* second, double* values,
                hipStream_t s) {
  EvalArgs a{};
  a.sense = sense;
  a.tie_template = tie ? tie->template_id : kNoTie;
  if (tie) {
    a.tie_L = tie->num_metrics;
    a.tie_coef = tie->d_coef;
    a.tie_coef_off = tie->d_coef_off;
    a.tie_ab = tie->d_ab;
    a.tie_hw = tie->d_hw;
    a.tie_sense = tie_sense;
  }
  // one monomial table serves both programs: the larger degree
  const int dm = tie ? std::max(pr->shape_d, tie->shape_d) : pr->shape_d;
  a.template_id = pr->template_id;
  a.L = pr->num_metrics;
  a.num_n = num_n;
  a.num_cand = num_cand;
  a.cand_dim = cand_dim;
  a.coef = pr->d_coef;
  a.coef_off = pr->d_coef_off;
  a.ab = pr->d_ab;
  a.hw = pr->d_hw;
  a.n_grid = n_grid;
  a.cand = cand;
  for (int k = 0; k < 4; ++k) a.inv_scale[k] = k < pr->nvars ? 1.0 / pr->scale[k] : 0.0;
  a.argmin = argmin;
  a.best = best;
  a.second = second;
  a.values = values;
  if (num_n == 0 || pr->num_programs == 0) return RP_OK;
  if (pr->template_id == RP_TEMPLATE_MWPCWP) return eval_dispatch_d<RP_TEMPLATE_MWPCWP, 3>(dm, a, pr->num_programs, precision, s);
  if (pr->template_id == RP_TEMPLATE_OCCUPANCY) return eval_dispatch_d<RP_TEMPLATE_OCCUPANCY, 3>(dm, a, pr->num_programs, precision, s);
  switch (pr->nvars) {
    case 1: return eval_dispatch_d<RP_TEMPLATE_SINGLE, 1>(dm, a, pr->num_programs, precision, s);
    case 2: return eval_dispatch_d<RP_TEMPLATE_SINGLE, 2>(dm, a, pr->num_programs, precision, s);
    case 3: return eval_dispatch_d<RP_TEMPLATE_SINGLE, 3>(dm, a, pr->num_programs, precision, s);
    case 4: return eval_dispatch_d<RP_TEMPLATE_SINGLE, 4>(dm, a, pr->num_programs, precision, s);
  }
  return set_error(RP_EUNSUPPORTED, "nvars not compiled in");
}

}  // namespace rp

using rp::set_error;

extern "C" {

int rp_program_create(rp_ctx ctx, const rp_program_desc* d, rp_prog* out) {
  if (!ctx || !d || !out) return set_error(RP_EINVAL, "rp_program_create: NULL argument");
  const int P = d->num_programs, L = d->num_metrics;
  if (P < 0 || L < 1) return set_error(RP_EINVAL, "rp_program_create: need num_programs >= 0, num_metrics >= 1");
  if (d->template_id == RP_TEMPLATE_SINGLE) {
    if (L != 1) return set_error(RP_EINVAL, "rp_program_create: the single template takes one metric");
    if (d->nvars < 1 || d->nvars > rp::kMaxV)
      return set_error(RP_EUNSUPPORTED, "rp_program_create: nvars must be 1..4");
  } else if (d->template_id == RP_TEMPLATE_MWPCWP) {
    if (L != RP_NUM_METRICS) return set_error(RP_EINVAL, "rp_program_create: MWP-CWP needs 16 metrics");
    if (d->nvars != 3) return set_error(RP_EUNSUPPORTED, "rp_program_create: MWP-CWP needs nvars == 3 (n, bx, by)");
    if (P > 0 && !d->hw) return set_error(RP_EINVAL, "rp_program_create: MWP-CWP needs the hardware vector");
  } else if (d->template_id == RP_TEMPLATE_OCCUPANCY) {
    if (L != 2) return set_error(RP_EINVAL, "rp_program_create: occupancy needs 2 metrics (registers, LDS bytes)");
    if (d->nvars != 3) return set_error(RP_EUNSUPPORTED, "rp_program_create: occupancy needs nvars == 3 (n, bx, by)");
    if (P > 0 && !d->hw) return set_error(RP_EINVAL, "rp_program_create: occupancy needs the hardware vector");
  } else {
    return set_error(RP_EINVAL, "rp_program_create: unknown template");
  }
  if (P > 0 && (!d->deg_num || !d->deg_den || !d->coef_off || !d->coef || !d->scale))
    return set_error(RP_EINVAL, "rp_program_create: NULL array");
  int dmax = 0;
  std::vector<int32_t> ab(2 * (size_t)P * L);
  for (int i = 0; i < P * L; ++i) {
    const int dn = d->deg_num[i], dq = d->deg_den[i];
    if (dn < 0 || dq < 0 || dn > rp::kMaxD || dq > rp::kMaxD)
      return set_error(RP_EUNSUPPORTED, "rp_program_create: metric degrees must be 0..4");
    int nc = 0;
    rp_num_coefs(d->nvars, dn, dq, &nc);
    if (d->coef_off[i + 1] - d->coef_off[i] != nc)
      return set_error(RP_ESHAPE, "rp_program_create: coef_off does not match the metric degrees");
    ab[2 * i] = rp::binom(d->nvars + dn, dn);
    ab[2 * i + 1] = rp::binom(d->nvars + dq, dq) - 1;
    dmax = std::max(dmax, std::max(dn, dq));
  }
  for (int k = 0; k < d->nvars; ++k)
    if (!(d->scale[k] > 0.0)) return set_error(RP_EINVAL, "rp_program_create: scales must be > 0");
  RP_CHECK_HIP(hipSetDevice(ctx->device));
  auto* p = new rp_prog_s;
  p->ctx = ctx;
  p->template_id = d->template_id;
  p->num_programs = P;
  p->num_metrics = L;
  p->nvars = d->nvars;
  p->shape_v = d->nvars;
  p->shape_d = std::max(dmax, 1);
  p->d_coef = d->coef;
  p->d_hw = d->hw;
  for (int k = 0; k < d->nvars; ++k) p->scale[k] = d->scale[k];
  p->h_coef_off.assign(d->coef_off, d->coef_off + (size_t)P * L + 1);
  p->h_deg_num.assign(d->deg_num, d->deg_num + (size_t)P * L);
  p->h_deg_den.assign(d->deg_den, d->deg_den + (size_t)P * L);
  const size_t nb = sizeof(int64_t) * ((size_t)P * L + 1);
  if (hipMalloc(&p->d_coef_off, nb) != hipSuccess ||
      hipMalloc(&p->d_ab, std::max<size_t>(sizeof(int32_t) * ab.size(), 8)) != hipSuccess) {
    if (p->d_coef_off) (void)hipFree(p->d_coef_off);
    delete p;
    return set_error(RP_ENOMEM, "rp_program_create: hipMalloc failed");
  }
  if (hipMemcpy(p->d_coef_off, d->coef_off, nb, hipMemcpyHostToDevice) != hipSuccess ||
      (!ab.empty() && hipMemcpy(p->d_ab, ab.data(), sizeof(int32_t) * ab.size(), hipMemcpyHostToDevice) != hipSuccess)) {
    (void)hipFree(p->d_coef_off);
    (void)hipFree(p->d_ab);
    delete p;
    return set_error(RP_EHIP, "rp_program_create: hipMemcpy failed");
  }
  *out = p;
  return RP_OK;
}

int rp_program_destroy(rp_prog p) {
  if (!p) return RP_OK;
  (void)hipSetDevice(p->ctx->device);
  if (p->d_coef_off) (void)hipFree(p->d_coef_off);
  if (p->d_ab) (void)hipFree(p->d_ab);
  delete p;
  return RP_OK;
}

int rp_eval_program_select(rp_prog prog, int sense, rp_prog tie_prog, int tie_sense,
                           const double* n_grid, int num_n, const int32_t* cand, int num_cand,
                           int cand_dim, int precision, int32_t* choice, double* best,
                           double* second, double* values, rp_stream_t stream) {
  if (!prog) return set_error(RP_EINVAL, "rp_eval_program_select: prog is NULL");
  if (sense != RP_SELECT_MIN && sense != RP_SELECT_MAX)
    return set_error(RP_EINVAL, "rp_eval_program_select: sense must be RP_SELECT_MIN or RP_SELECT_MAX");
  if (num_n < 0 || num_cand < 0) return set_error(RP_EINVAL, "rp_eval_program_select: negative size");
  if (cand_dim != prog->nvars - 1)
    return set_error(RP_ESHAPE, "rp_eval_program_select: cand_dim must be nvars - 1");
  if (precision != RP_FP64 && precision != RP_MIXED_FP32)
    return set_error(RP_EINVAL, "rp_eval_program_select: precision must be RP_FP64 or RP_MIXED_FP32");
  if (values && precision != RP_FP64)
    return set_error(RP_EINVAL, "rp_eval_program_select: values are returned by the FP64 form only");
  if (tie_prog) {
    if (precision != RP_FP64)
      return set_error(RP_EINVAL, "rp_eval_program_select: a tie program needs the FP64 form");
    if (tie_sense != RP_SELECT_MIN && tie_sense != RP_SELECT_MAX)
      return set_error(RP_EINVAL, "rp_eval_program_select: tie_sense must be RP_SELECT_MIN or RP_SELECT_MAX");
    if (tie_prog->template_id == RP_TEMPLATE_MWPCWP)
      return set_error(RP_EUNSUPPORTED, "rp_eval_program_select: a tie program is a single rational or an occupancy program");
    if (tie_prog->num_programs != prog->num_programs || tie_prog->nvars != prog->nvars)
      return set_error(RP_ESHAPE, "rp_eval_program_select: the tie program must match num_programs and nvars");
    if (tie_prog->ctx->device != prog->ctx->device)
      return set_error(RP_EINVAL, "rp_eval_program_select: the programs live on different devices");
  }
  if (num_n > 0 && prog->num_programs > 0 && (!n_grid || !choice || !best || !second || (num_cand > 0 && cand_dim > 0 && !cand)))
    return set_error(RP_EINVAL, "rp_eval_program_select: NULL array");
  if (prog->num_programs > 65535)
    return set_error(RP_ESHAPE, "rp_eval_program_select: at most 65535 programs per call");
  RP_CHECK_HIP(hipSetDevice(prog->ctx->device));
  return rp::launch_eval(prog, sense, tie_prog, tie_sense, n_grid, num_n, cand, num_cand, cand_dim,
                         precision, choice, best, second, values, (hipStream_t)stream);
}

int rp_eval_program_argmin(rp_prog prog, const double* n_grid, int num_n, const int32_t* cand,
                           int num_cand, int cand_dim, int precision, int32_t* argmin,
                           double* best, double* second, double* values, rp_stream_t stream) {
  return rp_eval_program_select(prog, RP_SELECT_MIN, nullptr, RP_SELECT_MIN, n_grid, num_n, cand,
                                num_cand, cand_dim, precision, argmin, best, second, values, stream);
}

}  // extern "C"

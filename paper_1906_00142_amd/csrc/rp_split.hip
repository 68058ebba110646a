// rp_split.hip -- one decision node of a rational program fitted from the
// samples (Section 3.2, third consequence: the branch conditions of a
// rational program are rational too and can be fitted like its process
// nodes).  Per node: the samples sorted by the split variable, every
// admissible breakpoint fitted on both sides by the batched linearised fit
// (rp_fit_rational on an internal plan, FP64), and the breakpoint whose two
// sides leave the smallest summed squared residual kept.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "rp_internal.h"

namespace rp {

constexpr int kSplitMaxSamples = 4096;   // per node (the sort runs in LDS)

struct SplitArgs {
  const double* x;
  int64_t ldx;
  const double* y;
  int num_samples, nvars, split_var, n_min, num_cand, nc;
  double* xs;          // replicated sorted samples: [nvars][total], total = F K m
  double* ys;          // [total]
  int64_t ldxs;        // = total
  double* us;          // sorted split variable per node [F][m]
  int32_t* bad;        // per node: a non-finite sample
  // outputs of the internal fit, one left and one right fit per candidate
  const double* fcoef;
  const int32_t* fstatus;
  const double* fresid;
  // results
  int64_t* k;
  double* theta;
  double* coef_l;
  double* coef_r;
  int32_t* status_l;
  int32_t* status_r;
  double* obj;
};

// Sort node f's samples by (u_s, sample index) -- a total order, the same as
// the order of equal values by index -- with a bitonic network in LDS, then
// write the sorted samples once per candidate breakpoint (candidate j's left
// fit takes the first n_min + j of them, its right fit the rest).
__global__ __launch_bounds__(256) void k_split_gather(SplitArgs s) {
  __shared__ double key[kSplitMaxSamples];
  __shared__ int idx[kSplitMaxSamples];
  __shared__ int bad;
  const int f = blockIdx.x, tid = threadIdx.x, m = s.num_samples;
  const int64_t s0 = (int64_t)f * m;
  int P = 1;
  while (P < m) P <<= 1;
  if (tid == 0) bad = 0;
  __syncthreads();
  bool nf = false;
  for (int i = tid; i < P; i += 256) {
    if (i < m) {
      key[i] = s.x[(int64_t)s.split_var * s.ldx + s0 + i];
      bool fin = isfinite(s.y[s0 + i]);
      for (int k = 0; k < s.nvars; ++k) fin = fin && isfinite(s.x[(int64_t)k * s.ldx + s0 + i]);
      nf = nf || !fin;
    } else {
      key[i] = INFINITY;   // padding sorts last (after every finite key, by index)
    }
    idx[i] = i;
  }
  if (nf) atomicOr(&bad, 1);
  __syncthreads();
  if (bad) {   // no candidate for this node (the select kernel reports it)
    if (tid == 0) s.bad[f] = 1;
    return;
  }
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = tid; i < P; i += 256) {
        const int j = i ^ stride;
        if (j > i) {
          const bool asc = (i & size) == 0;
          const double ki = key[i], kj = key[j];
          const int ii = idx[i], ij = idx[j];
          const bool j_before_i = kj < ki || (kj == ki && ij < ii);
          if (j_before_i == asc) {
            key[i] = kj; key[j] = ki;
            idx[i] = ij; idx[j] = ii;
          }
        }
      }
      __syncthreads();
    }
  }
  if (tid == 0) s.bad[f] = 0;
  for (int i = tid; i < m; i += 256) s.us[s0 + i] = key[i];
  const int64_t base = (int64_t)f * s.num_cand * m;
  for (int j = 0; j < s.num_cand; ++j) {
    const int64_t b = base + (int64_t)j * m;
    for (int i = tid; i < m; i += 256) {
      const int64_t src = s0 + idx[i];
      for (int k = 0; k < s.nvars; ++k) s.xs[(int64_t)k * s.ldxs + b + i] = s.x[(int64_t)k * s.ldx + src];
      s.ys[b + i] = s.y[src];
    }
  }
}

// Per node: the objective of every admissible candidate (both sides' squared
// residual norms), the smallest (the smallest k on exact ties), and the
// winner's threshold, coefficients and statuses.
__global__ __launch_bounds__(256) void k_split_select(SplitArgs s) {
  __shared__ double bv[256];
  __shared__ int bj[256];
  const int f = blockIdx.x, tid = threadIdx.x, m = s.num_samples, K = s.num_cand, nc = s.nc;
  const double* us = s.us + (int64_t)f * m;
  if (s.bad[f]) {
    for (int j = tid; j < nc; j += 256) {
      s.coef_l[(int64_t)f * nc + j] = __builtin_nan("");
      s.coef_r[(int64_t)f * nc + j] = __builtin_nan("");
    }
    if (tid == 0) {
      s.k[f] = -1;
      s.theta[f] = __builtin_nan("");
      s.obj[f] = INFINITY;
      s.status_l[f] = RP_FIT_NONFINITE_INPUT;
      s.status_r[f] = RP_FIT_NONFINITE_INPUT;
    }
    return;
  }
  double best = INFINITY;
  int bestj = -1;
  for (int j = tid; j < K; j += 256) {   // ascending j per thread: the first minimum stays
    const int k = s.n_min + j;
    if (!(us[k - 1] < us[k])) continue;  // equal values stay on one side
    const int64_t fl = 2 * ((int64_t)f * K + j);
    const double rl = s.fresid[fl], rr = s.fresid[fl + 1];
    double o = rl * rl + rr * rr;
    if (!(o == o)) o = INFINITY;
    if (o < best) { best = o; bestj = j; }
  }
  bv[tid] = best;
  bj[tid] = bestj;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
      const double o = bv[tid + w];
      const int oj = bj[tid + w];
      if (oj >= 0 && (o < bv[tid] || (o == bv[tid] && (bj[tid] < 0 || oj < bj[tid])))) {
        bv[tid] = o;
        bj[tid] = oj;
      }
    }
    __syncthreads();
  }
  const int j = bj[0];
  if (j < 0) {
    for (int q = tid; q < nc; q += 256) {
      s.coef_l[(int64_t)f * nc + q] = __builtin_nan("");
      s.coef_r[(int64_t)f * nc + q] = __builtin_nan("");
    }
    if (tid == 0) {
      s.k[f] = -1;
      s.theta[f] = __builtin_nan("");
      s.obj[f] = INFINITY;
      s.status_l[f] = RP_FIT_UNDERDETERMINED;
      s.status_r[f] = RP_FIT_UNDERDETERMINED;
    }
    return;
  }
  const int64_t fl = 2 * ((int64_t)f * K + j);
  for (int q = tid; q < nc; q += 256) {
    s.coef_l[(int64_t)f * nc + q] = s.fcoef[fl * nc + q];
    s.coef_r[(int64_t)f * nc + q] = s.fcoef[(fl + 1) * nc + q];
  }
  if (tid == 0) {
    const int k = s.n_min + j;
    s.k[f] = k;
    s.theta[f] = 0.5 * (us[k - 1] + us[k]);
    s.obj[f] = bv[0];
    s.status_l[f] = s.fstatus[fl];
    s.status_r[f] = s.fstatus[fl + 1];
  }
}

}  // namespace rp

struct rp_split_s {
  rp_ctx ctx = nullptr;
  int num_nodes = 0, num_samples = 0, nvars = 0, degree = 0, split_var = 0, n_min = 0;
  int num_cand = 0, nc = 0;
  rp_plan plan = nullptr;
  int64_t total = 0;
  double *xs = nullptr, *ys = nullptr, *us = nullptr;
  int32_t* bad = nullptr;
  double *coef = nullptr, *resid = nullptr;
  int32_t *status = nullptr, *iters = nullptr;
};

using rp::set_error;

static void split_free(rp_split s) {
  if (!s) return;
  if (s->plan) rp_plan_destroy(s->plan);
  for (void* p : {(void*)s->xs, (void*)s->ys, (void*)s->us, (void*)s->bad, (void*)s->coef,
                  (void*)s->resid, (void*)s->status, (void*)s->iters})
    if (p) (void)hipFree(p);
  delete s;
}

extern "C" {

int rp_split_create(rp_ctx ctx, int num_nodes, int num_samples, int nvars, int degree,
                    int split_var, int n_min, rp_split* out) {
  if (!ctx || !out) return set_error(RP_EINVAL, "rp_split_create: NULL argument");
  if (num_nodes < 0 || num_samples < 0 || num_samples > rp::kSplitMaxSamples)
    return set_error(RP_EINVAL, "rp_split_create: need num_nodes >= 0 and 0 <= num_samples <= 4096");
  if (!rp::shape_supported(nvars, degree, degree))
    return set_error(RP_EUNSUPPORTED, "rp_split_create: need 1 <= nvars <= 4 and 1 <= degree <= 4");
  if (split_var < 0 || split_var >= nvars)
    return set_error(RP_EINVAL, "rp_split_create: split_var must name one of the variables");
  int nc = 0;
  rp_num_coefs(nvars, degree, degree, &nc);
  if (n_min < 1) return set_error(RP_EINVAL, "rp_split_create: n_min must be >= 1");
  auto* s = new rp_split_s;
  s->ctx = ctx;
  s->num_nodes = num_nodes;
  s->num_samples = num_samples;
  s->nvars = nvars;
  s->degree = degree;
  s->split_var = split_var;
  s->n_min = n_min;
  s->nc = nc;
  s->num_cand = std::max(0, num_samples - 2 * n_min + 1);
  const int64_t F = num_nodes, K = s->num_cand, m = num_samples;
  s->total = F * K * m;
  const int64_t nfits = 2 * F * K;
  if (nfits > INT32_MAX / 2) {
    delete s;
    return set_error(RP_ESHAPE, "rp_split_create: too many candidate fits");
  }
  // the internal plan: candidate j of node f is fits 2 (f K + j) (the first
  // n_min + j sorted samples) and 2 (f K + j) + 1 (the others)
  std::vector<int64_t> off(nfits + 1, 0);
  std::vector<int32_t> nv(nfits, nvars), dg(nfits, degree);
  for (int64_t f = 0; f < F; ++f)
    for (int64_t j = 0; j < K; ++j) {
      const int64_t q = 2 * (f * K + j), b = (f * K + j) * m, k = n_min + j;
      off[q] = b;
      off[q + 1] = b + k;
      off[q + 2] = b + m;
    }
  int rc = hipSetDevice(ctx->device) == hipSuccess ? RP_OK : set_error(RP_EHIP, "rp_split_create: hipSetDevice failed");
  if (rc == RP_OK && nfits > 0)
    rc = rp_plan_create(ctx, (int)nfits, off.data(), nv.data(), dg.data(), dg.data(), &s->plan);
  auto alloc = [&](void** p, size_t bytes) {
    if (rc != RP_OK) return;
    if (hipMalloc(p, std::max<size_t>(bytes, 8)) != hipSuccess)
      rc = set_error(RP_ENOMEM, "rp_split_create: hipMalloc failed");
  };
  alloc((void**)&s->xs, sizeof(double) * (size_t)s->total * nvars);
  alloc((void**)&s->ys, sizeof(double) * (size_t)s->total);
  alloc((void**)&s->us, sizeof(double) * (size_t)(F * m));
  alloc((void**)&s->bad, sizeof(int32_t) * (size_t)F);
  alloc((void**)&s->coef, sizeof(double) * (size_t)nfits * nc);
  alloc((void**)&s->resid, sizeof(double) * (size_t)nfits);
  alloc((void**)&s->status, sizeof(int32_t) * (size_t)nfits);
  alloc((void**)&s->iters, sizeof(int32_t) * (size_t)nfits);
  if (rc != RP_OK) {
    split_free(s);
    return rc;
  }
  *out = s;
  return RP_OK;
}

int rp_split_destroy(rp_split s) {
  if (!s) return RP_OK;
  (void)hipSetDevice(s->ctx->device);
  split_free(s);
  return RP_OK;
}

int rp_split_fit(rp_split s, const double* x, int64_t ld_x, const double* y, int64_t* k,
                 double* theta, double* coef_l, double* coef_r, int32_t* status_l,
                 int32_t* status_r, double* obj, rp_stream_t stream) {
  if (!s) return set_error(RP_EINVAL, "rp_split_fit: NULL split");
  if (s->num_nodes == 0) return RP_OK;
  if (!x || !y || !k || !theta || !coef_l || !coef_r || !status_l || !status_r || !obj)
    return set_error(RP_EINVAL, "rp_split_fit: NULL argument");
  if (ld_x < (int64_t)s->num_nodes * s->num_samples)
    return set_error(RP_ESHAPE, "rp_split_fit: ld_x is smaller than the sample count");
  RP_CHECK_HIP(hipSetDevice(s->ctx->device));
  const hipStream_t st = (hipStream_t)stream;
  rp::SplitArgs a;
  std::memset(&a, 0, sizeof(a));
  a.x = x;
  a.ldx = ld_x;
  a.y = y;
  a.num_samples = s->num_samples;
  a.nvars = s->nvars;
  a.split_var = s->split_var;
  a.n_min = s->n_min;
  a.num_cand = s->num_cand;
  a.nc = s->nc;
  a.xs = s->xs;
  a.ys = s->ys;
  a.ldxs = s->total;
  a.us = s->us;
  a.bad = s->bad;
  a.fcoef = s->coef;
  a.fstatus = s->status;
  a.fresid = s->resid;
  a.k = k;
  a.theta = theta;
  a.coef_l = coef_l;
  a.coef_r = coef_r;
  a.status_l = status_l;
  a.status_r = status_r;
  a.obj = obj;
  hipLaunchKernelGGL(rp::k_split_gather, dim3(s->num_nodes), dim3(256), 0, st, a);
  RP_CHECK_HIP(hipGetLastError());
  if (s->plan) {
    // every candidate's two sides, FP64, residual norms computed
    const rp_fit_opts o = {RP_FP64, -1, -1.0, 1, RP_GRAM_AUTO};
    const int rc = rp_fit_rational(s->plan, s->xs, s->total, s->ys, &o, s->coef, s->status,
                                   s->resid, s->iters, stream);
    if (rc != RP_OK) return rc;
  }
  hipLaunchKernelGGL(rp::k_split_select, dim3(s->num_nodes), dim3(256), 0, st, a);
  RP_CHECK_HIP(hipGetLastError());
  return RP_OK;
}

}  // extern "C"

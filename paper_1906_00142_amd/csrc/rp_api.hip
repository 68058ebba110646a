// rp_api.hip -- host side of librpfit: errors, tables, contexts, plans and the
// dispatch of each entry point to the shape-specialised kernels.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <tuple>

#include "rp_internal.h"

namespace rp {

static thread_local std::string g_last_error;

int set_error(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int launch_fit_v1(int, int, const FitArgs&, int, hipStream_t);
int launch_fit_v2(int, int, const FitArgs&, int, hipStream_t);
int launch_fit_v3(int, int, const FitArgs&, int, hipStream_t);
int launch_fit_v4(int, int, const FitArgs&, int, hipStream_t);
int launch_gram_v1(int, int, const FitArgs&, double*, int, hipStream_t);
int launch_gram_v2(int, int, const FitArgs&, double*, int, hipStream_t);
int launch_gram_v3(int, int, const FitArgs&, double*, int, hipStream_t);
int launch_gram_v4(int, int, const FitArgs&, double*, int, hipStream_t);
int launch_refine_v1(int, const FitArgs&, int, hipStream_t);
int launch_refine_v2(int, const FitArgs&, int, hipStream_t);
int launch_refine_v3(int, const FitArgs&, int, hipStream_t);
int launch_refine_v4(int, const FitArgs&, int, hipStream_t);
int launch_design_v1(int, int, const FitArgs&, void*, const int64_t*, void*, int, hipStream_t);
int launch_design_v2(int, int, const FitArgs&, void*, const int64_t*, void*, int, hipStream_t);
int launch_design_v3(int, int, const FitArgs&, void*, const int64_t*, void*, int, hipStream_t);
int launch_design_v4(int, int, const FitArgs&, void*, const int64_t*, void*, int, hipStream_t);
int launch_loss_v1(int, const FitArgs&, const float*, float*, const float*, float*, int, int, hipStream_t);
int launch_loss_v2(int, const FitArgs&, const float*, float*, const float*, float*, int, int, hipStream_t);
int launch_loss_v3(int, const FitArgs&, const float*, float*, const float*, float*, int, int, hipStream_t);
int launch_loss_v4(int, const FitArgs&, const float*, float*, const float*, float*, int, int, hipStream_t);

int launch_fit(int v, int d, int precision, const FitArgs& a, int nblocks, hipStream_t s) {
  switch (v) {
    case 1: return launch_fit_v1(d, precision, a, nblocks, s);
    case 2: return launch_fit_v2(d, precision, a, nblocks, s);
    case 3: return launch_fit_v3(d, precision, a, nblocks, s);
    case 4: return launch_fit_v4(d, precision, a, nblocks, s);
  }
  return set_error(RP_EUNSUPPORTED, "variable count not compiled in");
}
int launch_gram(int v, int d, int precision, const FitArgs& a, double* gram, int nblocks, hipStream_t s) {
  switch (v) {
    case 1: return launch_gram_v1(d, precision, a, gram, nblocks, s);
    case 2: return launch_gram_v2(d, precision, a, gram, nblocks, s);
    case 3: return launch_gram_v3(d, precision, a, gram, nblocks, s);
    case 4: return launch_gram_v4(d, precision, a, gram, nblocks, s);
  }
  return set_error(RP_EUNSUPPORTED, "variable count not compiled in");
}
int launch_refine(int v, int d, const FitArgs& a, int nblocks, hipStream_t s) {
  switch (v) {
    case 1: return launch_refine_v1(d, a, nblocks, s);
    case 2: return launch_refine_v2(d, a, nblocks, s);
    case 3: return launch_refine_v3(d, a, nblocks, s);
    case 4: return launch_refine_v4(d, a, nblocks, s);
  }
  return set_error(RP_EUNSUPPORTED, "variable count not compiled in");
}
int launch_design(int v, int d, int precision, const FitArgs& a, void* A, const int64_t* a_off,
                  void* rhs, int nblocks, hipStream_t s) {
  switch (v) {
    case 1: return launch_design_v1(d, precision, a, A, a_off, rhs, nblocks, s);
    case 2: return launch_design_v2(d, precision, a, A, a_off, rhs, nblocks, s);
    case 3: return launch_design_v3(d, precision, a, A, a_off, rhs, nblocks, s);
    case 4: return launch_design_v4(d, precision, a, A, a_off, rhs, nblocks, s);
  }
  return set_error(RP_EUNSUPPORTED, "variable count not compiled in");
}
int launch_loss(int v, int d, const FitArgs& a, const float* coef, float* loss, const float* dloss,
                float* dcoef, int mode, int nblocks, hipStream_t s) {
  switch (v) {
    case 1: return launch_loss_v1(d, a, coef, loss, dloss, dcoef, mode, nblocks, s);
    case 2: return launch_loss_v2(d, a, coef, loss, dloss, dcoef, mode, nblocks, s);
    case 3: return launch_loss_v3(d, a, coef, loss, dloss, dcoef, mode, nblocks, s);
    case 4: return launch_loss_v4(d, a, coef, loss, dloss, dcoef, mode, nblocks, s);
  }
  return set_error(RP_EUNSUPPORTED, "variable count not compiled in");
}

std::vector<int32_t> moment_scatter_map(int v, int dn, int dq, bool gn) {
  // numerator columns: the monomials of degree <= dn; denominator columns:
  // those of degree <= dq but the constant; moments up to twice the larger
  const int dm = std::max(dn, dq);
  std::vector<std::vector<int>> en, eq, e2;
  for_each_graded(v, dn, [&](const int* e) { en.emplace_back(e, e + v); });
  for_each_graded(v, dq, [&](const int* e) { eq.emplace_back(e, e + v); });
  for_each_graded(v, 2 * dm, [&](const int* e) { e2.emplace_back(e, e + v); });
  auto index2 = [&](const std::vector<int>& e) {
    for (size_t k = 0; k < e2.size(); ++k)
      if (e2[k] == e) return (int)k;
    return -1;
  };
  const int nm = binom(v + dm, dm);   // moment-pair layout of the kernels
  const int na = (int)en.size(), nc = na + (int)eq.size() - 1, nu = nc + 1;
  // column kind 0 = numerator, 1 = denominator, 2 = right-hand side
  auto kind = [&](int j) { return j < na ? 0 : (j < nc ? 1 : 2); };
  auto expo = [&](int j) {
    if (j < na) return en[j];
    if (j < nc) return eq[j - na + 1];
    return std::vector<int>(v, 0);
  };
  std::vector<int32_t> map;
  map.reserve((size_t)nu * (nu + 1) / 2);
  for (int i = 0; i < nu; ++i)
    for (int j = 0; j <= i; ++j) {
      std::vector<int> e = expo(i);
      const std::vector<int> ej = expo(j);
      for (int k = 0; k < v; ++k) e[k] += ej[k];
      const int ki = kind(i), kj = kind(j);     // kj <= ki
      int w = 0, neg = 0;
      if (kj == 0 && ki == 0) { w = 0; }
      else if (kj == 0 && ki == 1) { w = 1; neg = 1; }
      else if (kj == 1 && ki == 1) { w = 2; }
      else if (kj == 0 && ki == 2) { w = gn ? 3 : 1; }
      else if (kj == 1 && ki == 2) { w = gn ? 4 : 2; neg = 1; }
      else { w = gn ? 5 : 2; }
      const int eidx = index2(e);
      const int p = gn ? moment_pair_index<true>(eidx, w, nm, v) : moment_pair_index<false>(eidx, w, nm, v);
      map.push_back(p | (neg << 30));
    }
  return map;
}

}  // namespace rp

using rp::set_error;

extern "C" {

const char* rp_last_error(void) { return rp::g_last_error.c_str(); }

int rp_monomials(int nvars, int degree, uint8_t* exps, int* count) {
  if (!count) return set_error(RP_EINVAL, "rp_monomials: count is NULL");
  if (nvars < 1 || nvars > rp::kMaxVarsHost || degree < 0 || degree > 15)
    return set_error(RP_EINVAL, "rp_monomials: need 1 <= nvars <= 8 and 0 <= degree <= 15");
  int n = 0;
  rp::for_each_graded(nvars, degree, [&](const int* e) {
    if (exps)
      for (int k = 0; k < nvars; ++k) exps[(size_t)n * nvars + k] = (uint8_t)e[k];
    ++n;
  });
  *count = n;
  return RP_OK;
}

int rp_monomials_box(int nvars, const int32_t* maxdeg, uint8_t* exps, int* count) {
  if (!count || !maxdeg) return set_error(RP_EINVAL, "rp_monomials_box: count or maxdeg is NULL");
  if (nvars < 1 || nvars > rp::kMaxVarsHost)
    return set_error(RP_EINVAL, "rp_monomials_box: need 1 <= nvars <= 8");
  int total = 0;
  for (int k = 0; k < nvars; ++k) {
    if (maxdeg[k] < 0 || maxdeg[k] > 15)
      return set_error(RP_EINVAL, "rp_monomials_box: need 0 <= maxdeg[k] <= 15");
    total += maxdeg[k];
  }
  // the graded walk up to the box's top degree, keeping what fits the box
  int n = 0;
  rp::for_each_graded(nvars, total, [&](const int* e) {
    for (int k = 0; k < nvars; ++k)
      if (e[k] > maxdeg[k]) return;
    if (exps)
      for (int k = 0; k < nvars; ++k) exps[(size_t)n * nvars + k] = (uint8_t)e[k];
    ++n;
  });
  *count = n;
  return RP_OK;
}

int rp_num_coefs(int nvars, int deg_num, int deg_den, int* count) {
  if (!count) return set_error(RP_EINVAL, "rp_num_coefs: count is NULL");
  if (nvars < 1 || nvars > rp::kMaxVarsHost || deg_num < 0 || deg_den < 0 || deg_num > 15 ||
      deg_den > 15)
    return set_error(RP_EINVAL, "rp_num_coefs: bad shape");
  *count = rp::binom(nvars + deg_num, deg_num) + rp::binom(nvars + deg_den, deg_den) - 1;
  return RP_OK;
}

int rp_candidates_2d(int max_prod, int multiple, int32_t* bxby, int* count) {
  if (!count) return set_error(RP_EINVAL, "rp_candidates_2d: count is NULL");
  if (max_prod < 1 || multiple < 1)
    return set_error(RP_EINVAL, "rp_candidates_2d: max_prod and multiple must be >= 1");
  int n = 0;
  // bx ascending; for each bx, by runs over the multiples of multiple/gcd(bx, multiple)
  for (int bx = 1; bx <= max_prod; ++bx) {
    const int step = multiple / std::gcd(bx, multiple);
    for (int by = step; (int64_t)bx * by <= max_prod; by += step) {
      if (bxby) { bxby[2 * n] = bx; bxby[2 * n + 1] = by; }
      ++n;
    }
  }
  *count = n;
  return RP_OK;
}

int rp_create(rp_ctx* out, int device) {
  if (!out) return set_error(RP_EINVAL, "rp_create: out is NULL");
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || device < 0 || device >= n)
    return set_error(RP_EHIP, "rp_create: HIP device not available");
  RP_CHECK_HIP(hipSetDevice(device));
  hipDeviceProp_t prop;
  RP_CHECK_HIP(hipGetDeviceProperties(&prop, device));
  const int rs = rp::static_scratch_init(device);
  if (rs != RP_OK) return rs;
  auto* c = new rp_ctx_s;
  c->device = device;
  c->num_cu = prop.multiProcessorCount;
  c->max_lds = (int)prop.sharedMemPerBlock;
  *out = c;
  return RP_OK;
}

int rp_destroy(rp_ctx ctx) {
  delete ctx;
  return RP_OK;
}

static void plan_free_device(rp_plan p) {
  if (!p) return;
  if (p->d_sample_off) (void)hipFree(p->d_sample_off);
  if (p->d_coef_off) (void)hipFree(p->d_coef_off);
  if (p->d_a_off) (void)hipFree(p->d_a_off);
  if (p->d_gws) (void)hipFree(p->d_gws);
  if (p->d_gofs) (void)hipFree(p->d_gofs);
  if (p->d_gflag) (void)hipFree(p->d_gflag);
  if (p->d_lm) (void)hipFree(p->d_lm);
  if (p->d_lm_int) (void)hipFree(p->d_lm_int);
  if (p->d_wres) (void)hipFree(p->d_wres);
  for (auto& b : p->buckets) {
    if (b.d_ids) (void)hipFree(b.d_ids);
    if (b.d_mom_map) (void)hipFree(b.d_mom_map);
    if (b.d_mom_map_gn) (void)hipFree(b.d_mom_map_gn);
    if (b.d_resolve) (void)hipFree(b.d_resolve);
  }
}

int rp_plan_create(rp_ctx ctx, int num_fits, const int64_t* sample_off, const int32_t* nvars,
                   const int32_t* deg_num, const int32_t* deg_den, rp_plan* out) {
  if (!ctx || !out || num_fits < 0 || (num_fits > 0 && (!sample_off || !nvars || !deg_num || !deg_den)))
    return set_error(RP_EINVAL, "rp_plan_create: NULL argument or negative num_fits");
  if (sample_off && sample_off[0] != 0)
    return set_error(RP_ESHAPE, "rp_plan_create: sample_off[0] must be 0");
  for (int f = 0; f < num_fits; ++f) {
    if (sample_off[f + 1] < sample_off[f])
      return set_error(RP_ESHAPE, "rp_plan_create: sample_off must be non-decreasing");
    if (sample_off[f + 1] - sample_off[f] >= (int64_t(1) << 28))
      return set_error(RP_ESHAPE, "rp_plan_create: a fit holds 2^28 samples or more");
    if (!rp::shape_supported(nvars[f], deg_num[f], deg_den[f]))
      return set_error(RP_EUNSUPPORTED, "rp_plan_create: fit " + std::to_string(f) +
                                            " has a shape that is not compiled in (nvars 1..4 with "
                                            "deg_num == deg_den in 1..4, or nvars 1..3 with "
                                            "degrees up to 3 that differ by one)");
  }
  RP_CHECK_HIP(hipSetDevice(ctx->device));
  auto* p = new rp_plan_s;
  p->ctx = ctx;
  p->num_fits = num_fits;
  p->h_sample_off.assign(sample_off, sample_off + num_fits + 1);
  p->h_nvars.assign(nvars, nvars + num_fits);
  p->h_deg_num.assign(deg_num, deg_num + num_fits);
  p->h_deg_den.assign(deg_den, deg_den + num_fits);
  p->total_samples = sample_off[num_fits];
  p->h_coef_off.assign(num_fits + 1, 0);
  p->h_a_off.assign(num_fits + 1, 0);
  for (int f = 0; f < num_fits; ++f) {
    int nc = 0;
    rp_num_coefs(nvars[f], deg_num[f], deg_den[f], &nc);
    p->h_coef_off[f + 1] = p->h_coef_off[f] + nc;
    p->h_a_off[f + 1] = p->h_a_off[f] + (sample_off[f + 1] - sample_off[f]) * nc;
  }
  // buckets by shape (variables, degree code), each ordered by decreasing
  // sample count (largest first)
  std::vector<std::pair<int, int>> keys;                 // (nvars, code), in order of appearance
  std::vector<std::vector<int32_t>> lists;
  for (int f = 0; f < num_fits; ++f) {
    const std::pair<int, int> key{nvars[f], rp::deg_code(deg_num[f], deg_den[f])};
    size_t k = 0;
    while (k < keys.size() && keys[k] != key) ++k;
    if (k == keys.size()) {
      keys.push_back(key);
      lists.emplace_back();
    }
    lists[k].push_back(f);
  }
  // buckets in (nvars, numerator degree, denominator degree) order
  std::vector<size_t> order(keys.size());
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](size_t a, size_t b) {
    const int va = keys[a].first, vb = keys[b].first;
    const int na = rp::code_dn(keys[a].second), nb2 = rp::code_dn(keys[b].second);
    const int qa = rp::code_dq(keys[a].second), qb = rp::code_dq(keys[b].second);
    return std::make_tuple(va, na, qa) < std::make_tuple(vb, nb2, qb);
  });
  auto fail = [&](int code, const std::string& msg) {
    plan_free_device(p);
    delete p;
    return set_error(code, msg);
  };
  for (size_t o : order) {
    auto& L = lists[o];
    const int v = keys[o].first, d = keys[o].second;
    std::stable_sort(L.begin(), L.end(), [&](int32_t a, int32_t b) {
      return (sample_off[a + 1] - sample_off[a]) > (sample_off[b + 1] - sample_off[b]);
    });
    rp::Bucket B;
    B.nvars = v;
    B.deg = d;
    B.deg_num = rp::code_dn(d);
    B.deg_den = rp::code_dq(d);
    B.count = (int)L.size();
    p->buckets.push_back(B);
    rp::Bucket& Bb = p->buckets.back();
    if (hipMalloc(&Bb.d_ids, sizeof(int32_t) * L.size()) != hipSuccess)
      return fail(RP_ENOMEM, "rp_plan_create: hipMalloc failed");
    if (hipMemcpy(Bb.d_ids, L.data(), sizeof(int32_t) * L.size(), hipMemcpyHostToDevice) != hipSuccess)
      return fail(RP_EHIP, "rp_plan_create: hipMemcpy failed");
    if (hipMalloc(&Bb.d_resolve, sizeof(int32_t) * (L.size() + 2)) != hipSuccess)
      return fail(RP_ENOMEM, "rp_plan_create: hipMalloc failed");
    if (hipMemset(Bb.d_resolve, 0, sizeof(int32_t) * (L.size() + 2)) != hipSuccess)
      return fail(RP_EHIP, "rp_plan_create: hipMemset failed");
    for (int gn = 0; gn < 2; ++gn) {
      const std::vector<int32_t> map = rp::moment_scatter_map(v, B.deg_num, B.deg_den, gn != 0);
      int32_t** dst = gn ? &Bb.d_mom_map_gn : &Bb.d_mom_map;
      if (hipMalloc(dst, sizeof(int32_t) * map.size()) != hipSuccess)
        return fail(RP_ENOMEM, "rp_plan_create: hipMalloc failed");
      if (hipMemcpy(*dst, map.data(), sizeof(int32_t) * map.size(), hipMemcpyHostToDevice) != hipSuccess)
        return fail(RP_EHIP, "rp_plan_create: hipMemcpy failed");
    }
  }
  const size_t nb = sizeof(int64_t) * (num_fits + 1);
  if (hipMalloc(&p->d_sample_off, nb) != hipSuccess || hipMalloc(&p->d_coef_off, nb) != hipSuccess ||
      hipMalloc(&p->d_a_off, nb) != hipSuccess)
    return fail(RP_ENOMEM, "rp_plan_create: hipMalloc failed");
  if (hipMemcpy(p->d_sample_off, sample_off, nb, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p->d_coef_off, p->h_coef_off.data(), nb, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p->d_a_off, p->h_a_off.data(), nb, hipMemcpyHostToDevice) != hipSuccess)
    return fail(RP_EHIP, "rp_plan_create: hipMemcpy failed");
  // Gram workspace: (nc+1)(nc+2)/2 doubles per fit
  std::vector<int64_t> gofs(num_fits + 1, 0);
  for (int f = 0; f < num_fits; ++f) {
    const int64_t nu = p->h_coef_off[f + 1] - p->h_coef_off[f] + 1;
    gofs[f + 1] = gofs[f] + nu * (nu + 1) / 2;
  }
  if (hipMalloc(&p->d_gws, sizeof(double) * std::max<int64_t>(gofs[num_fits], 1)) != hipSuccess ||
      hipMalloc(&p->d_gofs, nb) != hipSuccess ||
      hipMalloc(&p->d_gflag, sizeof(int) * std::max(num_fits, 1)) != hipSuccess)
    return fail(RP_ENOMEM, "rp_plan_create: hipMalloc of the Gram workspace failed");
  if (hipMemcpy(p->d_gofs, gofs.data(), nb, hipMemcpyHostToDevice) != hipSuccess)
    return fail(RP_EHIP, "rp_plan_create: hipMemcpy failed");
  p->h_gram_off = gofs;
  const size_t nf = (size_t)std::max(num_fits, 1);
  if (hipMalloc(&p->d_lm, sizeof(double) * 2 * nf) != hipSuccess ||
      hipMalloc(&p->d_lm_int, sizeof(int) * 3 * nf) != hipSuccess)
    return fail(RP_ENOMEM, "rp_plan_create: hipMalloc of the refinement state failed");
  // residual scratch of the grouped passes, when some model is that large
  bool grouped = false;
  for (int f = 0; f < num_fits; ++f) grouped = grouped || p->h_coef_off[f + 1] - p->h_coef_off[f] > rp::kPassGroupMax;
  if (grouped && hipMalloc(&p->d_wres, sizeof(double) * std::max<int64_t>(p->total_samples, 1)) != hipSuccess)
    return fail(RP_ENOMEM, "rp_plan_create: hipMalloc of the residual scratch failed");
  *out = p;
  return RP_OK;
}

int rp_plan_destroy(rp_plan plan) {
  if (!plan) return RP_OK;
  (void)hipSetDevice(plan->ctx->device);
  plan_free_device(plan);
  delete plan;
  return RP_OK;
}

static int base_args(rp_plan plan, const double* x, int64_t ld_x, const double* y, rp::FitArgs& a,
                     const char* who);

int rp_plan_offsets(rp_plan plan, int64_t* coef_off, int64_t* a_off, int64_t* gram_off) {
  if (!plan) return set_error(RP_EINVAL, "rp_plan_offsets: plan is NULL");
  const size_t nb = sizeof(int64_t) * (plan->num_fits + 1);
  if (coef_off) std::memcpy(coef_off, plan->h_coef_off.data(), nb);
  if (a_off) std::memcpy(a_off, plan->h_a_off.data(), nb);
  if (gram_off) std::memcpy(gram_off, plan->h_gram_off.data(), nb);
  return RP_OK;
}

int rp_gram(rp_plan plan, const double* x, int64_t ld_x, const double* y, int precision,
            int gram_algo, double* gram, rp_stream_t stream) {
  rp::FitArgs a;
  int rc = base_args(plan, x, ld_x, y, a, "rp_gram");
  if (rc) return rc;
  if (precision < RP_FP64 || precision > RP_MIXED_BF16)
    return set_error(RP_EINVAL, "rp_gram: unknown precision");
  if (plan->num_fits > 0 && !gram) return set_error(RP_EINVAL, "rp_gram: gram is NULL");
  if (gram_algo < RP_GRAM_AUTO || gram_algo > RP_GRAM_MOMENTS)
    return set_error(RP_EINVAL, "rp_gram: unknown gram_algo");
  a.gofs = plan->d_gofs;
  a.gflag = plan->d_gflag;
  a.gram_algo = gram_algo;
  RP_CHECK_HIP(hipSetDevice(plan->ctx->device));
  for (auto& b : plan->buckets) {
    a.ids = b.d_ids;
    a.mom_map = b.d_mom_map;
    a.gram_algo = gram_algo == RP_GRAM_AUTO ? b.gram_algo : gram_algo;
    rc = rp::launch_gram(b.nvars, b.deg, precision, a, gram, b.count, (hipStream_t)stream);
    if (rc) return rc;
  }
  return RP_OK;
}

int rp_gram_jacobian(rp_plan plan, const double* x, int64_t ld_x, const double* y,
                     const double* coef, int gram_algo, double* gram, rp_stream_t stream) {
  rp::FitArgs a;
  int rc = base_args(plan, x, ld_x, y, a, "rp_gram_jacobian");
  if (rc) return rc;
  if (plan->num_fits > 0 && (!gram || !coef))
    return set_error(RP_EINVAL, "rp_gram_jacobian: gram or coef is NULL");
  if (gram_algo < RP_GRAM_AUTO || gram_algo > RP_GRAM_MOMENTS)
    return set_error(RP_EINVAL, "rp_gram_jacobian: unknown gram_algo");
  a.coef = const_cast<double*>(coef);   // read only by the Jacobian kernels
  a.gofs = plan->d_gofs;
  a.gflag = plan->d_gflag;
  RP_CHECK_HIP(hipSetDevice(plan->ctx->device));
  for (auto& b : plan->buckets) {
    a.ids = b.d_ids;
    a.mom_map = b.d_mom_map_gn;
    a.gram_algo = gram_algo == RP_GRAM_AUTO ? b.gram_algo : gram_algo;
    rc = rp::launch_gram(b.nvars, b.deg, rp::kGramJacobian, a, gram, b.count, (hipStream_t)stream);
    if (rc) return rc;
  }
  return RP_OK;
}

static int base_args(rp_plan plan, const double* x, int64_t ld_x, const double* y, rp::FitArgs& a,
                     const char* who) {
  if (!plan) return set_error(RP_EINVAL, std::string(who) + ": plan is NULL");
  if (plan->num_fits > 0 && (!x || !y))
    return set_error(RP_EINVAL, std::string(who) + ": x or y is NULL");
  if (ld_x < plan->total_samples)
    return set_error(RP_ESHAPE, std::string(who) + ": ld_x is smaller than the sample count");
  std::memset(&a, 0, sizeof(a));
  a.x = x;
  a.ldx = ld_x;
  a.y = y;
  a.sample_off = plan->d_sample_off;
  a.coef_off = plan->d_coef_off;
  a.wres = plan->d_wres;
  return RP_OK;
}

int rp_assemble_design(rp_plan plan, const double* x, int64_t ld_x, const double* y,
                       int precision, void* A, void* rhs, rp_stream_t stream) {
  rp::FitArgs a;
  int rc = base_args(plan, x, ld_x, y, a, "rp_assemble_design");
  if (rc) return rc;
  if (precision < RP_FP64 || precision > RP_MIXED_BF16)
    return set_error(RP_EINVAL, "rp_assemble_design: unknown precision");
  if (plan->num_fits > 0 && (!A || !rhs))
    return set_error(RP_EINVAL, "rp_assemble_design: A or rhs is NULL");
  RP_CHECK_HIP(hipSetDevice(plan->ctx->device));
  for (auto& b : plan->buckets) {
    a.ids = b.d_ids;
    rc = rp::launch_design(b.nvars, b.deg, precision, a, A, plan->d_a_off, rhs, b.count,
                           (hipStream_t)stream);
    if (rc) return rc;
  }
  return RP_OK;
}

int rp_fit_rational(rp_plan plan, const double* x, int64_t ld_x, const double* y,
                    const rp_fit_opts* opts, double* coef, int32_t* status, double* resid,
                    int32_t* iters, rp_stream_t stream) {
  rp::FitArgs a;
  int rc = base_args(plan, x, ld_x, y, a, "rp_fit_rational");
  if (rc) return rc;
  rp_fit_opts o = {RP_FP64, -1, -1.0, 1, 0};
  if (opts) o = *opts;
  if (o.precision < RP_FP64 || o.precision > RP_AUTO)
    return set_error(RP_EINVAL, "rp_fit_rational: unknown precision");
  if (!(o.tol >= 0.0) && !(o.tol < 0.0))
    return set_error(RP_EINVAL, "rp_fit_rational: tol is NaN");
  if (plan->num_fits > 0 && (!coef || !status))
    return set_error(RP_EINVAL, "rp_fit_rational: coef or status is NULL");
  if (o.check_q && !resid)
    return set_error(RP_EINVAL, "rp_fit_rational: check_q needs resid");
  if (o.gram_algo < RP_GRAM_AUTO || o.gram_algo > RP_GRAM_MOMENTS)
    return set_error(RP_EINVAL, "rp_fit_rational: unknown gram_algo");
  a.coef = coef;
  a.status = status;
  a.resid = resid;
  a.iters = iters;
  a.check_q = o.check_q;
  a.gws = plan->d_gws;
  a.gofs = plan->d_gofs;
  a.gflag = plan->d_gflag;
  RP_CHECK_HIP(hipSetDevice(plan->ctx->device));
  for (auto& b : plan->buckets) {
    // the bucket's form: RP_AUTO takes the tuned one
    const int prec = o.precision == RP_AUTO ? b.precision : o.precision;
    // FP64 default: one refinement step, more (up to four) only for a fit
    // whose correction is still above the convergence bar sqrt(tol)
    const bool fp64_default = prec == RP_FP64 && o.max_refine < 0;
    a.max_refine = o.max_refine >= 0 ? o.max_refine
                                     : (prec == RP_FP64 ? 4 : (prec == RP_MIXED_FP32 ? 12 : 40));
    a.tol = o.tol >= 0.0 ? o.tol : (prec == RP_FP64 ? 1e-13 : 1e-12);
    a.stop_rel = fp64_default ? std::sqrt(a.tol) : a.tol;
    a.ids = b.d_ids;
    a.mom_map = b.d_mom_map;
    a.resolve = b.d_resolve;
    a.gram_algo = o.gram_algo == RP_GRAM_AUTO ? b.gram_algo : o.gram_algo;
    rc = rp::launch_fit(b.nvars, b.deg, prec, a, b.count, (hipStream_t)stream);
    if (rc) return rc;
  }
  return RP_OK;
}

int rp_refine_rational(rp_plan plan, const double* x, int64_t ld_x, const double* y,
                       const rp_refine_opts* opts, double* coef, int32_t* status, double* loss,
                       rp_stream_t stream) {
  rp::FitArgs a;
  int rc = base_args(plan, x, ld_x, y, a, "rp_refine_rational");
  if (rc) return rc;
  rp_refine_opts o = {20, 1e-14, RP_GRAM_AUTO};
  if (opts) o = *opts;
  if (o.gram_algo < RP_GRAM_AUTO || o.gram_algo > RP_GRAM_MOMENTS)
    return set_error(RP_EINVAL, "rp_refine_rational: unknown gram_algo");
  if (o.max_iter < 0 || !(o.rtol >= 0.0))
    return set_error(RP_EINVAL, "rp_refine_rational: need max_iter >= 0 and rtol >= 0");
  if (plan->num_fits > 0 && (!coef || !status || !loss))
    return set_error(RP_EINVAL, "rp_refine_rational: coef, status or loss is NULL");
  a.coef = coef;
  a.status = status;
  a.resid = loss;
  a.max_iter = o.max_iter;
  a.rtol = o.rtol;
  a.gws = plan->d_gws;
  a.gofs = plan->d_gofs;
  a.gflag = plan->d_gflag;
  const size_t nf = (size_t)std::max(plan->num_fits, 1);
  a.lm_lambda = plan->d_lm;
  a.lm_loss = plan->d_lm + nf;
  a.lm_state = plan->d_lm_int;
  a.lm_rejects = plan->d_lm_int + nf;
  a.iters = plan->d_lm_int + 2 * nf;
  a.gram_algo = o.gram_algo;
  RP_CHECK_HIP(hipSetDevice(plan->ctx->device));
  for (auto& b : plan->buckets) {
    a.ids = b.d_ids;
    a.mom_map = b.d_mom_map_gn;
    a.gram_algo = o.gram_algo == RP_GRAM_AUTO ? b.gram_algo : o.gram_algo;
    rc = rp::launch_refine(b.nvars, b.deg, a, b.count, (hipStream_t)stream);
    if (rc) return rc;
  }
  return RP_OK;
}

int rp_loss_grad(rp_plan plan, const double* x, int64_t ld_x, const double* y, const float* coef,
                 float* loss, const float* dloss, float* dcoef, int mode, rp_stream_t stream) {
  rp::FitArgs a;
  int rc = base_args(plan, x, ld_x, y, a, "rp_loss_grad");
  if (rc) return rc;
  if (mode != RP_LOSS_FWD && mode != RP_LOSS_BWD)
    return set_error(RP_EINVAL, "rp_loss_grad: mode must be RP_LOSS_FWD or RP_LOSS_BWD");
  if (plan->num_fits > 0 && (!coef || !loss || (mode == RP_LOSS_BWD && !dcoef)))
    return set_error(RP_EINVAL, "rp_loss_grad: NULL coef, loss or dcoef");
  RP_CHECK_HIP(hipSetDevice(plan->ctx->device));
  for (auto& b : plan->buckets) {
    a.ids = b.d_ids;
    rc = rp::launch_loss(b.nvars, b.deg, a, coef, loss, dloss, dcoef, mode, b.count,
                         (hipStream_t)stream);
    if (rc) return rc;
  }
  return RP_OK;
}


int rp_plan_tune(rp_plan plan, const double* x, int64_t ld_x, const double* y, rp_stream_t stream) {
  rp::FitArgs a;
  int rc = base_args(plan, x, ld_x, y, a, "rp_plan_tune");
  if (rc) return rc;
  if (plan->num_fits == 0) return RP_OK;
  RP_CHECK_HIP(hipSetDevice(plan->ctx->device));
  hipStream_t s = (hipStream_t)stream;
  // scratch outputs of the timing runs
  double *coef = nullptr, *resid = nullptr;
  int32_t *status = nullptr, *iters = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto release = [&]() {
    if (coef) (void)hipFree(coef);
    if (resid) (void)hipFree(resid);
    if (status) (void)hipFree(status);
    if (iters) (void)hipFree(iters);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  const size_t nf = (size_t)plan->num_fits;
  if (hipMalloc(&coef, sizeof(double) * (size_t)std::max<int64_t>(plan->h_coef_off[nf], 1)) != hipSuccess ||
      hipMalloc(&resid, sizeof(double) * nf) != hipSuccess ||
      hipMalloc(&status, sizeof(int32_t) * nf) != hipSuccess ||
      hipMalloc(&iters, sizeof(int32_t) * nf) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    release();
    return set_error(RP_ENOMEM, "rp_plan_tune: scratch allocation failed");
  }
  // candidate forms: (precision, gram_algo)
  const int cand[4][2] = {{RP_FP64, RP_GRAM_MOMENTS}, {RP_FP64, RP_GRAM_MFMA},
                          {RP_MIXED_FP32, RP_GRAM_AUTO}, {RP_MIXED_BF16, RP_GRAM_AUTO}};
  for (size_t k = 0; k < plan->buckets.size() && rc == RP_OK; ++k) {
    rp_plan_s view = *plan;            // a single-bucket view of the plan
    view.buckets = {plan->buckets[k]};
    float best = -1.0f;
    int best_c = 0;
    float fp64_best = -1.0f;
    int fp64_algo = RP_GRAM_MOMENTS;
    for (int c = 0; c < 4 && rc == RP_OK; ++c) {
      rp_fit_opts o = {cand[c][0], -1, -1.0, 1, cand[c][1]};
      float ms = 0.0f;
      for (int rep = 0; rep < 3 && rc == RP_OK; ++rep) {   // the first launch warms up
        (void)hipEventRecord(e0, s);
        rc = rp_fit_rational(&view, x, ld_x, y, &o, coef, status, resid, iters, stream);
        (void)hipEventRecord(e1, s);
        if (rc) break;
        if (hipEventSynchronize(e1) != hipSuccess) { rc = set_error(RP_EHIP, "rp_plan_tune: a timed fit failed"); break; }
        float t = 0.0f;
        (void)hipEventElapsedTime(&t, e0, e1);
        if (rep > 0) ms += 0.5f * t;
      }
      if (rc) break;
      plan->buckets[k].form_us[c] = (int)(ms * 1000.0f);
      if (best < 0.0f || ms < best) { best = ms; best_c = c; }
      if (cand[c][0] == RP_FP64 && (fp64_best < 0.0f || ms < fp64_best)) { fp64_best = ms; fp64_algo = cand[c][1]; }
    }
    view.buckets.clear();
    if (rc) break;
    plan->buckets[k].precision = cand[best_c][0];
    plan->buckets[k].gram_algo = fp64_algo;
  }
  release();
  return rc;
}

int rp_plan_tuning(rp_plan plan, int32_t* table, int* count) {
  if (!plan || !count) return set_error(RP_EINVAL, "rp_plan_tuning: NULL argument");
  *count = (int)plan->buckets.size();
  if (table)
    for (size_t k = 0; k < plan->buckets.size(); ++k) {
      const auto& b = plan->buckets[k];
      int32_t* row = table + RP_TUNE_COLS * k;
      row[0] = b.nvars;
      row[1] = b.deg_num;
      row[2] = b.deg_den;
      row[3] = b.precision;
      row[4] = b.gram_algo;
      for (int c = 0; c < 4; ++c) row[5 + c] = b.form_us[c];
    }
  return RP_OK;
}

int rp_plan_set_tuning(rp_plan plan, const int32_t* table, int count) {
  if (!plan || (count > 0 && !table) || count < 0)
    return set_error(RP_EINVAL, "rp_plan_set_tuning: NULL or negative argument");
  for (int k = 0; k < count; ++k) {
    const int32_t* row = table + RP_TUNE_COLS * k;
    const int prec = row[3], algo = row[4];
    if (prec < RP_FP64 || prec > RP_MIXED_BF16)
      return set_error(RP_EINVAL, "rp_plan_set_tuning: precision must be RP_FP64, RP_MIXED_FP32 or RP_MIXED_BF16");
    if (algo != RP_GRAM_MFMA && algo != RP_GRAM_MOMENTS)
      return set_error(RP_EINVAL, "rp_plan_set_tuning: gram_algo must be MFMA or MOMENTS");
  }
  for (int k = 0; k < count; ++k) {
    const int32_t* row = table + RP_TUNE_COLS * k;
    for (auto& b : plan->buckets)
      if (b.nvars == row[0] && b.deg_num == row[1] && b.deg_den == row[2]) {
        b.precision = row[3];
        b.gram_algo = row[4];
        for (int c = 0; c < 4; ++c) b.form_us[c] = row[5 + c];
      }
  }
  return RP_OK;
}

int rp_fit_graph_create(rp_plan plan, const double* x, int64_t ld_x, const double* y,
                        const rp_fit_opts* opts, double* coef, int32_t* status, double* resid,
                        int32_t* iters, rp_graph* out) {
  if (!out) return set_error(RP_EINVAL, "rp_fit_graph_create: out is NULL");
  if (!plan) return set_error(RP_EINVAL, "rp_fit_graph_create: plan is NULL");
  RP_CHECK_HIP(hipSetDevice(plan->ctx->device));
  const size_t nb = plan->buckets.size();
  std::vector<hipStream_t> br(nb, nullptr);
  hipStream_t s0 = nullptr;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> joins(nb, nullptr);
  auto cleanup = [&]() {
    for (auto& e : joins) if (e) (void)hipEventDestroy(e);
    if (fork) (void)hipEventDestroy(fork);
    for (auto& b : br) if (b) (void)hipStreamDestroy(b);
    if (s0) (void)hipStreamDestroy(s0);
  };
  if (hipStreamCreateWithFlags(&s0, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess) {
    cleanup();
    return set_error(RP_EHIP, "rp_fit_graph_create: stream/event creation failed");
  }
  for (size_t k = 0; k < nb; ++k)
    if (hipStreamCreateWithFlags(&br[k], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&joins[k], hipEventDisableTiming) != hipSuccess) {
      cleanup();
      return set_error(RP_EHIP, "rp_fit_graph_create: stream/event creation failed");
    }
  if (hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    cleanup();
    return set_error(RP_EHIP, "rp_fit_graph_create: hipStreamBeginCapture failed");
  }
  int rc = RP_OK;
  (void)hipEventRecord(fork, s0);
  // one branch per shape bucket: a single-bucket view of the plan per branch
  for (size_t k = 0; k < nb && rc == RP_OK; ++k) {
    (void)hipStreamWaitEvent(br[k], fork, 0);
    rp_plan_s view = *plan;
    view.buckets = {plan->buckets[k]};
    rc = rp_fit_rational(&view, x, ld_x, y, opts, coef, status, resid, iters, (rp_stream_t)br[k]);
    view.buckets.clear();
    (void)hipEventRecord(joins[k], br[k]);
    (void)hipStreamWaitEvent(s0, joins[k], 0);
  }
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(s0, &graph);
  if (rc != RP_OK || ec != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    cleanup();
    return rc != RP_OK ? rc : set_error(RP_EHIP, "rp_fit_graph_create: capture failed");
  }
  hipGraphExec_t exec = nullptr;
  if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(graph);
    cleanup();
    return set_error(RP_EHIP, "rp_fit_graph_create: hipGraphInstantiate failed");
  }
  cleanup();
  auto* g = new rp_graph_s;
  g->plan = plan;
  g->graph = graph;
  g->exec = exec;
  *out = g;
  return RP_OK;
}

int rp_graph_launch(rp_graph g, rp_stream_t stream) {
  if (!g) return set_error(RP_EINVAL, "rp_graph_launch: graph is NULL");
  RP_CHECK_HIP(hipSetDevice(g->plan->ctx->device));
  RP_CHECK_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
  return RP_OK;
}

int rp_graph_destroy(rp_graph g) {
  if (!g) return RP_OK;
  (void)hipSetDevice(g->plan->ctx->device);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return RP_OK;
}

}  // extern "C"

// rp_static.hip -- the fit entry point that allocates nothing: the fit's
// device scratch (per-fit offsets, the Gram workspace, the non-finite flags,
// the re-solve list and the moment map) lives in one file-scope device array
// instead of a plan's allocations.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "rp_internal.h"

namespace rp {

// The scratch array of every device the library runs on (each GPU holds its
// own copy until the process ends).  Host code never passes its name to a
// kernel: it is a host-side stand-in, not a device address; the device
// address comes from hipGetSymbolAddress, once per device.
constexpr size_t kStaticScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
static void* g_scratch_ptr[kMaxDevices] = {};
static std::mutex g_scratch_mu;

// With `device` current: look up and keep that device's scratch address.
int static_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices)
    return set_error(RP_EUNSUPPORTED, "static scratch: device index beyond the library's table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return RP_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return set_error(RP_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_ptr[device] = p;
  return RP_OK;
}

static void* static_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return (device >= 0 && device < kMaxDevices) ? g_scratch_ptr[device] : nullptr;
}

// Where each array sits inside the scratch for F fits of NPK packed Gram
// entries (byte offsets, 256-aligned).
struct StaticLayout {
  size_t sample_off, coef_off, gofs, ids, gflag, resolve, map, gws, total;
  StaticLayout(int64_t F, int64_t npk) {
    size_t o = 0;
    auto take = [&](size_t bytes) {
      const size_t at = o;
      o += (bytes + 255) / 256 * 256;
      return at;
    };
    sample_off = take(sizeof(int64_t) * (F + 1));
    coef_off = take(sizeof(int64_t) * (F + 1));
    gofs = take(sizeof(int64_t) * (F + 1));
    ids = take(sizeof(int32_t) * F);
    gflag = take(sizeof(int32_t) * F);
    resolve = take(sizeof(int32_t) * (F + 2));
    map = take(sizeof(int32_t) * npk);
    gws = take(sizeof(double) * F * npk);
    total = o;
  }
};

// Rank of exponent e (total degree t) among the exponents of v variables in
// the library's monomial order: every exponent of lower degree first, then,
// within degree t, the larger exponent of x1 first, then of x2, ...
__device__ int graded_rank(const int* e, int v) {
  int t = 0;
  for (int k = 0; k < v; ++k) t += e[k];
  int rank = t > 0 ? binom(v + t - 1, v) : 0;   // exponents of degree < t
  int r = t;                                      // degree left for e[k..]
  for (int k = 0; k + 1 < v; ++k) {
    // exponents agreeing with e before k and larger at k: x_k takes a in
    // (e[k], r], the remaining r - a is spread over the v - k - 1 others
    for (int a = e[k] + 1; a <= r; ++a) rank += binom(r - a + v - k - 2, v - k - 2);
    r -= e[k];
  }
  return rank;
}

struct StaticArgs {
  int64_t* sample_off;
  int64_t* coef_off;
  int64_t* gofs;
  int32_t* ids;
  int32_t* resolve;
  int32_t* map;
  int num_fits, num_samples, nc, npk, nvars, degree;
};

// Fill the per-fit offsets of a uniform batch (fit f owns samples
// [f m, (f+1) m) and coefficients [f nc, (f+1) nc)), clear the re-solve list
// and write the moment map of the linearised Gram (for the packed entry
// (i, j): the moment pair of the exponent e_i + e_j and the weight of the
// two columns' kinds, negated for numerator x denominator and denominator x
// right-hand side; the same map the plans build on the host).
__global__ void k_static_setup(StaticArgs s) {
  __shared__ int ex[kMaxMono][kMaxV];
  const int v = s.nvars, d = s.degree;
  if (threadIdx.x == 0) {
    int n = 0;
    for_each_graded(v, d, [&](const int* e) {
      for (int k = 0; k < kMaxV; ++k) ex[n][k] = k < v ? e[k] : 0;
      ++n;
    });
  }
  __syncthreads();
  const int F = s.num_fits;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nthr = (int64_t)gridDim.x * blockDim.x;
  for (int64_t f = tid; f <= F; f += nthr) {
    s.sample_off[f] = f * s.num_samples;
    s.coef_off[f] = f * s.nc;
    s.gofs[f] = f * s.npk;
    if (f < F) s.ids[f] = (int32_t)f;
  }
  if (tid < 2) s.resolve[tid] = 0;
  const int nm = binom(v + d, d), na = nm, nc = 2 * nm - 1;
  for (int64_t q = tid; q < s.npk; q += nthr) {
    int i = 0;
    while ((i + 1) * (i + 2) / 2 <= q) ++i;
    const int j = (int)q - i * (i + 1) / 2;   // j <= i
    auto kind = [&](int c) { return c < na ? 0 : (c < nc ? 1 : 2); };
    auto mono = [&](int c) { return c < na ? c : (c < nc ? c - na + 1 : 0); };
    int e[kMaxV];
    for (int k = 0; k < kMaxV; ++k) e[k] = ex[mono(i)][k] + ex[mono(j)][k];
    const int ki = kind(i), kj = kind(j);
    int w = 0, neg = 0;
    if (kj == 0 && ki == 0) w = 0;
    else if (kj == 0 && ki == 1) { w = 1; neg = 1; }
    else if (kj == 1 && ki == 1) w = 2;
    else if (kj == 0 && ki == 2) w = 1;
    else if (kj == 1 && ki == 2) { w = 2; neg = 1; }
    else w = 2;
    const int p = moment_pair_index<false>(graded_rank(e, v), w, nm, v);
    s.map[q] = p | (neg << 30);
  }
}

}  // namespace rp

using rp::set_error;

extern "C" {

int rp_fit_uniform_static(rp_ctx ctx, int num_fits, int num_samples, int nvars, int degree,
                          const double* x, int64_t ld_x, const double* y, double* coef,
                          int32_t* status, double* resid, int32_t* iters, rp_stream_t stream) {
  if (!ctx) return set_error(RP_EINVAL, "rp_fit_uniform_static: ctx is NULL");
  if (num_fits < 0 || num_samples < 0)
    return set_error(RP_EINVAL, "rp_fit_uniform_static: negative num_fits or num_samples");
  if (!rp::shape_supported(nvars, degree, degree))
    return set_error(RP_EUNSUPPORTED, "rp_fit_uniform_static: need 1 <= nvars <= 4 and 1 <= degree <= 4");
  if (num_samples >= (1 << 28))
    return set_error(RP_ESHAPE, "rp_fit_uniform_static: a fit holds 2^28 samples or more");
  if (num_fits == 0) return RP_OK;
  if (!x || !y || !coef || !status || !resid)
    return set_error(RP_EINVAL, "rp_fit_uniform_static: NULL x, y, coef, status or resid");
  if (ld_x < (int64_t)num_fits * num_samples)
    return set_error(RP_ESHAPE, "rp_fit_uniform_static: ld_x is smaller than the sample count");
  int nc = 0;
  rp_num_coefs(nvars, degree, degree, &nc);
  const int64_t npk = (int64_t)(nc + 1) * (nc + 2) / 2;
  const rp::StaticLayout L(num_fits, npk);
  if (L.total > rp::kStaticScratchBytes)
    return set_error(RP_ESHAPE, "rp_fit_uniform_static: " + std::to_string(num_fits) + " fits of " +
                                    std::to_string(nc) + " unknowns need " + std::to_string(L.total) +
                                    " bytes of scratch, more than its " +
                                    std::to_string(rp::kStaticScratchBytes));
  RP_CHECK_HIP(hipSetDevice(ctx->device));
  unsigned char* base = static_cast<unsigned char*>(rp::static_scratch(ctx->device));
  if (!base) return set_error(RP_EHIP, "rp_fit_uniform_static: the device's scratch was not set up");
  rp::StaticArgs s;
  s.sample_off = reinterpret_cast<int64_t*>(base + L.sample_off);
  s.coef_off = reinterpret_cast<int64_t*>(base + L.coef_off);
  s.gofs = reinterpret_cast<int64_t*>(base + L.gofs);
  s.ids = reinterpret_cast<int32_t*>(base + L.ids);
  s.resolve = reinterpret_cast<int32_t*>(base + L.resolve);
  s.map = reinterpret_cast<int32_t*>(base + L.map);
  s.num_fits = num_fits;
  s.num_samples = num_samples;
  s.nc = nc;
  s.npk = (int)npk;
  s.nvars = nvars;
  s.degree = degree;
  const hipStream_t st = (hipStream_t)stream;
  const int64_t work = std::max<int64_t>(num_fits + 1, npk);
  const int grid = (int)std::min<int64_t>((work + 255) / 256, 1024);
  hipLaunchKernelGGL(rp::k_static_setup, dim3(grid), dim3(256), 0, st, s);
  RP_CHECK_HIP(hipGetLastError());

  rp::FitArgs a;
  std::memset(&a, 0, sizeof(a));
  a.x = x;
  a.ldx = ld_x;
  a.y = y;
  a.sample_off = s.sample_off;
  a.coef_off = s.coef_off;
  a.ids = s.ids;
  a.coef = coef;
  a.status = status;
  a.resid = resid;
  a.iters = iters;
  a.max_refine = 4;
  a.tol = 1e-13;
  a.stop_rel = std::sqrt(a.tol);
  a.check_q = 1;
  a.gws = reinterpret_cast<double*>(base + L.gws);
  a.gofs = s.gofs;
  a.gflag = reinterpret_cast<int*>(base + L.gflag);
  a.mom_map = s.map;
  a.gram_algo = RP_GRAM_MOMENTS;
  a.resolve = s.resolve;
  return rp::launch_fit(nvars, degree, RP_FP64, a, num_fits, st);
}

}  // extern "C"

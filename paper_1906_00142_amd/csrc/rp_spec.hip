// rp_spec.hip -- specialised evaluators: the GPU form of the paper's code
// generation step (Section 3.3 step 3; Section 4.3 "compile-time code
// generation").  The paper combines a rational-program template with the fitted
// rational functions by text substitution into a program specialised to one
// kernel.  Here the same happens at run time for the device: each program's
// metric rationals are written out as straight-line HIP code with their
// coefficients, the normalisation and the hardware vector as literals, the
// template code is appended verbatim (the text of rp_templates.h, the code the
// table-driven evaluator runs), and the result is compiled with hipRTC for the
// device's architecture, loaded as a module and launched like the
// table-driven evaluator: one workgroup per (program, data size), candidates
// strided over its 256 lanes, a shuffle + LDS reduction to (best, index,
// second).
#include <hip/hiprtc.h>

#include <cinttypes>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "rp_internal.h"

#define RP_TPL_SRC(...) #__VA_ARGS__
static const char* const kTemplateSource =
#include "rp_templates.h"
    ;
#undef RP_TPL_SRC

struct rp_spec_s {
  rp_ctx ctx = nullptr;
  int template_id = 0, num_programs = 0, nvars = 0;
  std::string source;
  hipModule_t module = nullptr;
  hipFunction_t fn = nullptr;
};

namespace rp {
namespace {

constexpr int kSpecMaxPrograms = 256;

// A double literal that reads back to the same value.
std::string lit(double v) {
  if (std::isnan(v)) return "__builtin_nan(\"\")";
  if (std::isinf(v)) return v > 0 ? "__builtin_inf()" : "(-__builtin_inf())";
  char b[40];
  std::snprintf(b, sizeof b, "%.17g", v);
  std::string s(b);
  if (s.find_first_of(".eE") == std::string::npos) s += ".0";
  return "(" + s + ")";
}

struct HostProgram {
  int template_id, nvars, L;
  const int32_t* dn;
  const int32_t* dq;
  const int64_t* off;    // [L + 1], into coef
  const double* coef;
  const double* hw;      // [RP_HW_COUNT] or null
};

// Straight-line code computing E for one program into `v`, given u[] and the
// raw candidate values raw[].  The monomials are formed as the table-driven
// evaluator forms them (parent monomial times one variable, graded order), and
// each rational accumulates its terms in the same order with fma, so the two
// evaluators agree bit for bit up to the compiler's contraction choices.
std::string program_body(const HostProgram& hp, int dmax) {
  const MonoTable T = make_mono_table(hp.nvars, dmax);
  std::string s;
  s += "      double m[" + std::to_string(T.n) + "];\n      m[0] = 1.0;\n";
  for (int j = 1; j < T.n; ++j)
    s += "      m[" + std::to_string(j) + "] = m[" + std::to_string(T.parent[j]) + "] * u[" +
         std::to_string(T.var[j]) + "];\n";
  const int L = hp.L;
  s += "      double g[" + std::to_string(L) + "];\n";
  for (int l = 0; l < L; ++l) {
    const int na = binom(hp.nvars + hp.dn[l], hp.dn[l]);
    const int nb = binom(hp.nvars + hp.dq[l], hp.dq[l]) - 1;
    const double* c = hp.coef + hp.off[l];
    s += "      {\n        double nn = 0.0, q = 1.0;\n";
    for (int j = 0; j < na; ++j)
      if (c[j] != 0.0) s += "        nn = fma(" + lit(c[j]) + ", m[" + std::to_string(j) + "], nn);\n";
    for (int j = 1; j <= nb; ++j)
      if (c[na + j - 1] != 0.0)
        s += "        q = fma(" + lit(c[na + j - 1]) + ", m[" + std::to_string(j) + "], q);\n";
    // the single template rejects a candidate whose Q is not positive
    if (hp.template_id == RP_TEMPLATE_SINGLE)
      s += "        g[" + std::to_string(l) + "] = !(q > 0.0) ? __builtin_inf() : nn / q;\n      }\n";
    else
      s += "        g[" + std::to_string(l) + "] = nn / q;\n      }\n";
  }
  if (hp.template_id == RP_TEMPLATE_SINGLE) {
    s += "      v = g[0];\n";
  } else {
    s += "      {\n        const double h[" + std::to_string(RP_HW_COUNT) + "] = {";
    for (int k = 0; k < RP_HW_COUNT; ++k) s += (k ? ", " : "") + lit(hp.hw[k]);
    s += "};\n";
    if (hp.template_id == RP_TEMPLATE_MWPCWP)
      s += "        v = mwpcwp_cycles<double>(g, h, raw[1], raw[2]);\n";
    else
      s += "        v = block_occupancy<double>(g, h, raw[1], raw[2]);\n";
    s += "      }\n";
  }
  return s;
}

}  // namespace

// Source of the specialised evaluator of P programs (host coefficients).
std::string spec_source(int template_id, int nvars, int P, int L, const int32_t* dn,
                        const int32_t* dq, const int64_t* coef_off, const double* coef,
                        const double* hw, const double* scale) {
  int dmax = 1;
  for (int i = 0; i < P * L; ++i) dmax = std::max(dmax, std::max(dn[i], dq[i]));
  std::string s;
  s += "// generated: specialised evaluator of " + std::to_string(P) + " rational program(s)\n";
  s += "#define INFINITY __builtin_inf()\n\n";
  s += kTemplateSource;
  s += "\n\nextern \"C\" __global__ __launch_bounds__(256) void rp_spec_eval(\n"
       "    const double* __restrict__ n_grid, int num_n, const int* __restrict__ cand, int num_cand,\n"
       "    int cand_dim, double sense, int* choice, double* best, double* second, double* values) {\n"
       "  __shared__ double wbv[4], wsv[4];\n"
       "  __shared__ int wbi[4];\n"
       "  const int j = blockIdx.x, p = blockIdx.y;\n"
       "  const double n = n_grid[j];\n"
       "  double bv = __builtin_inf(), sv = __builtin_inf();\n"
       "  int bi = 2147483647;\n"
       "  const long long row = ((long long)p * num_n + j) * num_cand;\n"
       "  for (int k = threadIdx.x; k < num_cand; k += 256) {\n";
  s += "    double u[" + std::to_string(nvars) + "], raw[" + std::to_string(nvars) + "];\n";
  s += "    raw[0] = n;\n    u[0] = n * " + lit(1.0 / scale[0]) + ";\n";
  for (int k = 1; k < nvars; ++k) {
    s += "    raw[" + std::to_string(k) + "] = (double)cand[(long long)k * cand_dim + " +
         std::to_string(k - 1) + "];\n";
    s += "    u[" + std::to_string(k) + "] = raw[" + std::to_string(k) + "] * " + lit(1.0 / scale[k]) + ";\n";
  }
  s += "    double v = 0.0;\n    switch (p) {\n";
  for (int p = 0; p < P; ++p) {
    HostProgram hp{template_id, nvars, L, dn + (size_t)p * L, dq + (size_t)p * L, nullptr, coef, nullptr};
    std::vector<int64_t> off(L + 1);
    for (int l = 0; l <= L; ++l) off[l] = coef_off[(size_t)p * L + l] - coef_off[0];
    hp.off = off.data();
    hp.coef = coef;
    hp.hw = hw ? hw + (size_t)p * RP_HW_COUNT : nullptr;
    s += "    case " + std::to_string(p) + ": {\n" + program_body(hp, dmax) + "      break;\n    }\n";
  }
  s += "    }\n"
       "    if (values) values[row + k] = v;\n"
       "    const double key = sense * v;\n"
       "    if (!isfinite(key)) continue;\n"
       "    if (key < bv) { sv = fmin(sv, bv); bv = key; bi = k; }\n"
       "    else sv = fmin(sv, key);\n"
       "  }\n"
       "  for (int o = 32; o >= 1; o >>= 1) {\n"
       "    const double ov = __shfl_xor(bv, o, 64), os = __shfl_xor(sv, o, 64);\n"
       "    const int oi = __shfl_xor(bi, o, 64);\n"
       "    const bool other = ov < bv || (ov == bv && oi < bi);\n"
       "    if (other) { sv = fmin(os, bv); bv = ov; bi = oi; } else { sv = fmin(sv, ov); }\n"
       "  }\n"
       "  if ((threadIdx.x & 63) == 0) { wbv[threadIdx.x >> 6] = bv; wsv[threadIdx.x >> 6] = sv; wbi[threadIdx.x >> 6] = bi; }\n"
       "  __syncthreads();\n"
       "  if (threadIdx.x == 0) {\n"
       "    for (int w = 1; w < 4; ++w) {\n"
       "      const bool other = wbv[w] < bv || (wbv[w] == bv && wbi[w] < bi);\n"
       "      if (other) { sv = fmin(wsv[w], bv); bv = wbv[w]; bi = wbi[w]; } else { sv = fmin(sv, wbv[w]); }\n"
       "    }\n"
       "    const long long o = (long long)p * num_n + j;\n"
       "    choice[o] = bi == 2147483647 ? -1 : bi;\n"
       "    best[o] = sense * bv;\n"
       "    second[o] = sense * sv;\n"
       "  }\n"
       "}\n";
  return s;
}

}  // namespace rp

using rp::set_error;

namespace {

int check_host_desc(const rp_program_desc* d) {
  if (!d) return set_error(RP_EINVAL, "NULL program description");
  const int P = d->num_programs, L = d->num_metrics;
  if (P < 1 || P > rp::kSpecMaxPrograms)
    return set_error(RP_EINVAL, "a specialised evaluator takes 1..256 programs");
  if (d->template_id == RP_TEMPLATE_SINGLE) {
    if (L != 1 || d->nvars < 1 || d->nvars > rp::kMaxV)
      return set_error(RP_EINVAL, "single template: one metric, nvars 1..4");
  } else if (d->template_id == RP_TEMPLATE_MWPCWP || d->template_id == RP_TEMPLATE_OCCUPANCY) {
    if (L != (d->template_id == RP_TEMPLATE_MWPCWP ? RP_NUM_METRICS : 2) || d->nvars != 3 || !d->hw)
      return set_error(RP_EINVAL, "MWP-CWP / occupancy template: 16 / 2 metrics, nvars 3, a hardware vector");
  } else {
    return set_error(RP_EINVAL, "unknown template");
  }
  if (!d->deg_num || !d->deg_den || !d->coef_off || !d->coef || !d->scale)
    return set_error(RP_EINVAL, "NULL array in the program description");
  for (int i = 0; i < P * L; ++i) {
    const int dn = d->deg_num[i], dq = d->deg_den[i];
    if (dn < 0 || dq < 0 || dn > rp::kMaxD || dq > rp::kMaxD)
      return set_error(RP_EUNSUPPORTED, "metric degrees must be 0..4");
    int nc = 0;
    rp_num_coefs(d->nvars, dn, dq, &nc);
    if (d->coef_off[i + 1] - d->coef_off[i] != nc)
      return set_error(RP_ESHAPE, "coef_off does not match the metric degrees");
  }
  for (int k = 0; k < d->nvars; ++k)
    if (!(d->scale[k] > 0.0)) return set_error(RP_EINVAL, "scales must be > 0");
  return RP_OK;
}

int copy_out(const std::string& s, char* buf, size_t* len) {
  if (!len) return set_error(RP_EINVAL, "len is NULL");
  if (buf) {
    if (*len < s.size() + 1) {
      *len = s.size() + 1;
      return set_error(RP_ESHAPE, "buffer too small for the source");
    }
    std::memcpy(buf, s.c_str(), s.size() + 1);
  }
  *len = s.size() + 1;
  return RP_OK;
}

}  // namespace

extern "C" {

int rp_program_source(const rp_program_desc* d, char* buf, size_t* len) {
  const int rc = check_host_desc(d);
  if (rc != RP_OK) return rc;
  return copy_out(rp::spec_source(d->template_id, d->nvars, d->num_programs, d->num_metrics,
                                  d->deg_num, d->deg_den, d->coef_off, d->coef, d->hw, d->scale),
                  buf, len);
}

int rp_program_specialize(rp_prog prog, rp_spec* out) {
  if (!prog || !out) return set_error(RP_EINVAL, "rp_program_specialize: NULL argument");
  const int P = prog->num_programs, L = prog->num_metrics;
  if (P < 1 || P > rp::kSpecMaxPrograms)
    return set_error(RP_EINVAL, "rp_program_specialize: a specialised evaluator takes 1..256 programs");
  RP_CHECK_HIP(hipSetDevice(prog->ctx->device));
  // the coefficients and hardware vectors become literals: read them once
  const int64_t nco = prog->h_coef_off[(size_t)P * L] - prog->h_coef_off[0];
  std::vector<double> coef((size_t)std::max<int64_t>(nco, 1));
  RP_CHECK_HIP(hipMemcpy(coef.data(), prog->d_coef + prog->h_coef_off[0], sizeof(double) * nco,
                         hipMemcpyDeviceToHost));
  std::vector<double> hw;
  if (prog->template_id != RP_TEMPLATE_SINGLE) {
    hw.resize((size_t)P * RP_HW_COUNT);
    RP_CHECK_HIP(hipMemcpy(hw.data(), prog->d_hw, sizeof(double) * hw.size(), hipMemcpyDeviceToHost));
  }
  std::vector<int64_t> off(prog->h_coef_off.begin(), prog->h_coef_off.end());
  for (auto& o : off) o -= prog->h_coef_off[0];
  auto* s = new rp_spec_s;
  s->ctx = prog->ctx;
  s->template_id = prog->template_id;
  s->num_programs = P;
  s->nvars = prog->nvars;
  s->source = rp::spec_source(prog->template_id, prog->nvars, P, L, prog->h_deg_num.data(),
                              prog->h_deg_den.data(), off.data(), coef.data(),
                              hw.empty() ? nullptr : hw.data(), prog->scale);
  hipDeviceProp_t props;
  if (hipGetDeviceProperties(&props, prog->ctx->device) != hipSuccess) {
    delete s;
    return set_error(RP_EHIP, "rp_program_specialize: hipGetDeviceProperties failed");
  }
  std::string arch = std::string("--offload-arch=") + std::string(props.gcnArchName).substr(0, std::string(props.gcnArchName).find(':'));
  const char* opts[] = {arch.c_str(), "-O3", "-ffp-contract=fast", "-std=c++17"};
  hiprtcProgram prg;
  if (hiprtcCreateProgram(&prg, s->source.c_str(), "rp_spec.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS) {
    delete s;
    return set_error(RP_EHIP, "rp_program_specialize: hiprtcCreateProgram failed");
  }
  const hiprtcResult cr = hiprtcCompileProgram(prg, 4, opts);
  if (cr != HIPRTC_SUCCESS) {
    size_t ls = 0;
    hiprtcGetProgramLogSize(prg, &ls);
    std::string log(ls + 1, '\0');
    hiprtcGetProgramLog(prg, log.data());
    hiprtcDestroyProgram(&prg);
    delete s;
    return set_error(RP_EHIP, "rp_program_specialize: hipRTC compile failed: " + log.substr(0, 2000));
  }
  size_t cs = 0;
  hiprtcGetCodeSize(prg, &cs);
  std::vector<char> code(cs);
  hiprtcGetCode(prg, code.data());
  hiprtcDestroyProgram(&prg);
  if (hipModuleLoadData(&s->module, code.data()) != hipSuccess ||
      hipModuleGetFunction(&s->fn, s->module, "rp_spec_eval") != hipSuccess) {
    if (s->module) (void)hipModuleUnload(s->module);
    delete s;
    return set_error(RP_EHIP, "rp_program_specialize: loading the compiled module failed");
  }
  *out = s;
  return RP_OK;
}

int rp_spec_source(rp_spec spec, char* buf, size_t* len) {
  if (!spec) return set_error(RP_EINVAL, "rp_spec_source: spec is NULL");
  return copy_out(spec->source, buf, len);
}

int rp_eval_spec_select(rp_spec spec, int sense, const double* n_grid, int num_n, const int32_t* cand,
                        int num_cand, int cand_dim, int32_t* choice, double* best, double* second,
                        double* values, rp_stream_t stream) {
  if (!spec) return set_error(RP_EINVAL, "rp_eval_spec_select: spec is NULL");
  if (sense != RP_SELECT_MIN && sense != RP_SELECT_MAX)
    return set_error(RP_EINVAL, "rp_eval_spec_select: sense must be RP_SELECT_MIN or RP_SELECT_MAX");
  if (num_n < 0 || num_cand < 0) return set_error(RP_EINVAL, "rp_eval_spec_select: negative size");
  if (cand_dim != spec->nvars - 1)
    return set_error(RP_ESHAPE, "rp_eval_spec_select: cand_dim must be nvars - 1");
  if (num_n == 0) return RP_OK;
  if (!n_grid || !choice || !best || !second || (num_cand > 0 && cand_dim > 0 && !cand))
    return set_error(RP_EINVAL, "rp_eval_spec_select: NULL array");
  RP_CHECK_HIP(hipSetDevice(spec->ctx->device));
  double sd = sense;
  void* args[] = {(void*)&n_grid, (void*)&num_n, (void*)&cand, (void*)&num_cand, (void*)&cand_dim,
                  (void*)&sd, (void*)&choice, (void*)&best, (void*)&second, (void*)&values};
  RP_CHECK_HIP(hipModuleLaunchKernel(spec->fn, (unsigned)num_n, (unsigned)spec->num_programs, 1, 256, 1, 1,
                                     0, (hipStream_t)stream, args, nullptr));
  return RP_OK;
}

int rp_spec_destroy(rp_spec spec) {
  if (!spec) return RP_OK;
  (void)hipSetDevice(spec->ctx->device);
  if (spec->module) (void)hipModuleUnload(spec->module);
  delete spec;
  return RP_OK;
}

}  // extern "C"

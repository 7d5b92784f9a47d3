// User field samplers (include/mss.h): run-time compilation (hiprtc) of a
// user field function together with the library's device header and
// mss_user_kernels.h, per-device loading of the code object, and the
// integrator launches.  The device headers are embedded by the build
// (mss_rtc_sources.inc) so the library needs no source tree at run time.
#include <hip/hiprtc.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "mss_internal.h"
#include "mss_rtc_sources.inc"

using namespace mss;

struct mss_sampler_s {
  struct Module {
    hipModule_t mod = nullptr;
    hipFunction_t fn[2] = {nullptr, nullptr};  // spin-1/2, spin-1
    hipFunction_t work = nullptr;              // batched work-queue integrator
  };
  std::vector<char> code;
  std::string log;
  int32_t min_params = 0;      // parameters a problem must carry (terms' slots)
  bool spin_one_only = false;  // a quadrupole term: spin-1 problems only
  std::mutex mu;
  std::map<int, Module> loaded;  // device ordinal -> module (entries never erased before destroy)
};

namespace {

// Headers the device header includes that hiprtc does not ship.  Its
// runtime declarations are built in; the fixed-width integer types live in
// namespace __hip_internal.
const char kStubRuntime[] = "#pragma once\n";
const char kStubStddef[] = "#pragma once\n";
const char kStubStdint[] =
    "#pragma once\n"
    "typedef __hip_internal::int8_t int8_t;\n"
    "typedef __hip_internal::int16_t int16_t;\n"
    "typedef __hip_internal::int32_t int32_t;\n"
    "typedef __hip_internal::int64_t int64_t;\n"
    "typedef __hip_internal::uint8_t uint8_t;\n"
    "typedef __hip_internal::uint16_t uint16_t;\n"
    "typedef __hip_internal::uint32_t uint32_t;\n"
    "typedef __hip_internal::uint64_t uint64_t;\n";

// The library's own compile flags (gfx950, no packed-FP32 instructions).
const char* const kBaseOptions[] = {
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=fast-honor-pragmas",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
};

std::string program_log(hiprtcProgram prog) {
  size_t n = 0;
  if (hiprtcGetProgramLogSize(prog, &n) != HIPRTC_SUCCESS || n == 0) return std::string();
  std::string log(n, '\0');
  if (hiprtcGetProgramLog(prog, &log[0]) != HIPRTC_SUCCESS) return std::string();
  while (!log.empty() && log.back() == '\0') log.pop_back();
  return log;
}

mss_status load_on_current(mss_sampler s, const mss_sampler_s::Module** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return api_hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lock(s->mu);
  auto it = s->loaded.find(dev);
  if (it == s->loaded.end()) {
    mss_sampler_s::Module m;
    e = hipModuleLoadData(&m.mod, s->code.data());
    if (e != hipSuccess) return api_hip_fail(e, "loading the user sampler's code object");
    e = hipModuleGetFunction(&m.fn[0], m.mod, "mss_user_integrate_2");
    if (e == hipSuccess) e = hipModuleGetFunction(&m.fn[1], m.mod, "mss_user_integrate_3");
    if (e == hipSuccess) e = hipModuleGetFunction(&m.work, m.mod, "mss_user_work_integrate");
    if (e != hipSuccess) {
      (void)hipModuleUnload(m.mod);
      return api_hip_fail(e, "user sampler kernels");
    }
    it = s->loaded.emplace(dev, m).first;
  }
  *out = &it->second;
  return MSS_OK;
}

// Exact decimal-free spelling of a double for generated source.
std::string hex_literal(double v) {
  char b[64];
  snprintf(b, sizeof b, "%a", v);
  return std::string("(") + b + ")";
}

std::string slot_or_literal(int32_t slot, double v) {
  return slot >= 0 ? "p[" + std::to_string(slot) + "]" : hex_literal(v);
}

// HIP source of mss_user_field for a term list: the field-program
// interpreter's operations for these terms, in the same order and with the
// same contraction (none), so that the compiled integrator reproduces the
// interpreter's operators bit for bit.  Window bounds that are infinite are
// left out (every finite t passes them); a term whose window holds no
// finite time is left out altogether.
std::string specialised_source(const mss_term* terms, int n) {
  std::string s;
  s += "__device__ void mss_user_field(double t, const double* p, double* f) {\n";
  s += "#pragma clang fp contract(off)\n";
  s += "  double fc[4] = {0.0, 0.0, 0.0, 0.0};\n";
  for (int i = 0; i < n; ++i) {
    const mss_term& tm = terms[i];
    if (tm.t_on == INFINITY || tm.t_off == -INFINITY || !(tm.t_on < tm.t_off)) continue;
    std::string cond;
    if (tm.t_on != -INFINITY) cond = hex_literal(tm.t_on) + " < t";
    if (tm.t_off != INFINITY) cond += (cond.empty() ? "" : " && ") + std::string("t < ") + hex_literal(tm.t_off);
    s += "  // term " + std::to_string(i) + "\n";
    s += cond.empty() ? "  {\n" : "  if (" + cond + ") {\n";
    s += "    double amp = " + slot_or_literal(tm.a_slot, tm.a) + ";\n";
    s += "    double ph = " + slot_or_literal(tm.phi_slot, tm.phi) + ";\n";
    if (tm.kind >= MSS_TERM_PWC) {
      s += "    const double x = (t - " + hex_literal(tm.seg_t0) + ") / " + hex_literal(tm.seg_len) +
           ";\n";
      s += "    const double fl = floor(x);\n";
      s += "    const int s = fl < 0.0 ? 0 : (fl > (double)(" + std::to_string(tm.n_seg - 1) +
           ") ? " + std::to_string(tm.n_seg - 1) + " : (int)fl);\n";
      if (tm.seg_a_slot >= 0) s += "    amp = p[" + std::to_string(tm.seg_a_slot) + " + s];\n";
      if (tm.seg_phi_slot >= 0) s += "    ph = p[" + std::to_string(tm.seg_phi_slot) + " + s];\n";
    }
    if (tm.kind == MSS_TERM_CONST || tm.kind == MSS_TERM_PWC) {
      s += "    const double v = amp;\n";
    } else {
      const bool is_cos = tm.kind == MSS_TERM_COS || tm.kind == MSS_TERM_PWC_COS;
      s += "    const double fr = " + slot_or_literal(tm.f_slot, tm.f) + ";\n";
      s += "    const double ft = fr * t;\n";
      s += "    const double xr = mss::kTwoPi * ft;\n";
      s += "    const double arg = xr + ph;\n";
      s += "    double sn, cs;\n";
      s += "    mss::sincos_cw(arg, &sn, &cs);\n";
      s += std::string("    const double v = amp * ") + (is_cos ? "cs" : "sn") + ";\n";
    }
    s += "    fc[" + std::to_string(tm.comp) + "] = fc[" + std::to_string(tm.comp) + "] + v;\n";
    s += "  }\n";
  }
  s += "  f[0] = fc[0];\n  f[1] = fc[1];\n  f[2] = fc[2];\n  f[3] = fc[3];\n}\n";
  return s;
}

}  // namespace

namespace mss {
mss_status api_sampler_check_problem(mss_sampler s, const mss_problem* p) {
  if (p->n_params < s->min_params)
    return api_fail(MSS_E_INVALID,
                    "the sampler's terms read %d parameters, the problem has n_params = %d",
                    s->min_params, p->n_params);
  if (s->spin_one_only && p->spin_twice != 2)
    return api_fail(MSS_E_INVALID, "the sampler's terms have a quadrupole component: spin-1 only");
  return MSS_OK;
}

mss_status api_sampler_work_function(mss_sampler s, hipFunction_t* fn) {
  const mss_sampler_s::Module* m = nullptr;
  mss_status st = load_on_current(s, &m);
  if (st != MSS_OK) return st;
  *fn = m->work;
  return MSS_OK;
}
}  // namespace mss

extern "C" {

mss_status mss_sampler_create(const char* source, const char* const* options, int32_t n_options,
                              mss_sampler* out) {
  if (!out) return api_fail(MSS_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!source) return api_fail(MSS_E_INVALID, "source is NULL");
  if (n_options < 0 || (n_options > 0 && !options))
    return api_fail(MSS_E_INVALID, "options is NULL but n_options = %d", n_options);
  for (int i = 0; i < n_options; ++i)
    if (!options[i]) return api_fail(MSS_E_INVALID, "option %d is NULL", i);

  std::string program = "#include \"mss_device.h\"\n#line 1 \"user_field.hip\"\n";
  program += source;
  program += "\n#include \"mss_user_kernels.h\"\n";

  std::vector<const char*> names, texts;
  for (const rtc::EmbeddedHeader& h : rtc::kHeaders) {
    names.push_back(h.name);
    texts.push_back(h.text);
  }
  names.push_back("hip/hip_runtime.h");
  texts.push_back(kStubRuntime);
  names.push_back("stdint.h");
  texts.push_back(kStubStdint);
  names.push_back("stddef.h");
  texts.push_back(kStubStddef);

  std::vector<const char*> opts(std::begin(kBaseOptions), std::end(kBaseOptions));
  for (int i = 0; i < n_options; ++i) opts.push_back(options[i]);

  hiprtcProgram prog = nullptr;
  hiprtcResult r = hiprtcCreateProgram(&prog, program.c_str(), "user_field.hip", (int)names.size(),
                                       texts.data(), names.data());
  if (r != HIPRTC_SUCCESS)
    return api_fail(MSS_E_DEVICE, "hiprtcCreateProgram: %s", hiprtcGetErrorString(r));
  r = hiprtcCompileProgram(prog, (int)opts.size(), opts.data());
  std::string log = program_log(prog);
  if (r != HIPRTC_SUCCESS) {
    (void)hiprtcDestroyProgram(&prog);
    return api_fail_text(MSS_E_INVALID, std::string("user sampler failed to compile (") +
                                            hiprtcGetErrorString(r) + "):\n" + log);
  }
  size_t n = 0;
  r = hiprtcGetCodeSize(prog, &n);
  std::vector<char> code(n);
  if (r == HIPRTC_SUCCESS && n > 0) r = hiprtcGetCode(prog, code.data());
  (void)hiprtcDestroyProgram(&prog);
  if (r != HIPRTC_SUCCESS || n == 0)
    return api_fail(MSS_E_DEVICE, "hiprtcGetCode: %s", hiprtcGetErrorString(r));

  mss_sampler s = new (std::nothrow) mss_sampler_s;
  if (!s) return api_fail(MSS_E_NOMEM, "out of host memory");
  s->code.swap(code);
  s->log = log;
  *out = s;
  return api_ok();
}

mss_status mss_sampler_create_for_terms(const mss_term* terms, int32_t n_terms,
                                        mss_sampler* out) {
  if (!out) return api_fail(MSS_E_INVALID, "out is NULL");
  *out = nullptr;
  if (n_terms < 0 || n_terms > MSS_MAX_TERMS)
    return api_fail(MSS_E_INVALID, "n_terms must be in [0, %d], got %d", MSS_MAX_TERMS, n_terms);
  if (n_terms > 0 && !terms) return api_fail(MSS_E_INVALID, "terms is NULL");
  int32_t need = 0;
  bool quad = false;
  for (int i = 0; i < n_terms; ++i) {
    const mss_term& t = terms[i];
    const int32_t one[3] = {t.a_slot, t.f_slot, t.phi_slot};
    for (int32_t v : one)
      if (v >= 0) need = std::max(need, v + 1);
    if (t.kind >= MSS_TERM_PWC && t.n_seg >= 1) {
      if (t.seg_a_slot >= 0) need = std::max(need, t.seg_a_slot + t.n_seg);
      if (t.seg_phi_slot >= 0) need = std::max(need, t.seg_phi_slot + t.n_seg);
    }
    quad = quad || t.comp == MSS_Q;
    if (t.comp >= MSS_U1 && t.comp <= MSS_V2)
      return api_fail(MSS_E_UNSUPPORTED,
                      "term %d: full su(3) components are interpreted, not compiled in", i);
  }
  mss_status st = api_validate_terms(2, terms, n_terms, need);
  if (st != MSS_OK) return st;
  const std::string src = specialised_source(terms, n_terms);
  if ((st = mss_sampler_create(src.c_str(), nullptr, 0, out)) != MSS_OK) return st;
  (*out)->min_params = need;
  (*out)->spin_one_only = quad;
  return api_ok();
}

int32_t mss_sampler_min_params(mss_sampler s) { return s ? s->min_params : 0; }

const char* mss_sampler_log(mss_sampler s) { return s ? s->log.c_str() : ""; }

mss_status mss_sampler_integrate(mss_sampler s, const mss_problem* p, const double* params,
                                 double* U, double* time, const mss_launch* launch, void* stream) {
  if (!s) return api_fail(MSS_E_INVALID, "sampler is NULL");
  mss_status st = api_validate_problem(p);
  if (st != MSS_OK) return st;
  if (p->n_terms != 0)
    return api_fail(MSS_E_INVALID, "a sampler problem carries no terms (n_terms = %d)", p->n_terms);
  if (!U) return api_fail(MSS_E_INVALID, "U is NULL");
  if (p->n_params > 0 && !params) return api_fail(MSS_E_INVALID, "params is NULL but n_params > 0");
  if ((st = api_sampler_check_problem(s, p)) != MSS_OK) return st;
  int S, B;
  bool given = false;
  if ((st = api_resolve_launch(p, launch, &S, &B, &given)) != MSS_OK) return st;
  const mss_sampler_s::Module* m = nullptr;
  if ((st = load_on_current(s, &m)) != MSS_OK) return st;
  IntervalGrid g;
  memset(&g, 0, sizeof g);
  g.params = params;
  g.U = U;
  g.time = time;
  g.t_start = p->t_start;
  g.dt_out = p->dt_out;
  g.dt = p->dt_out / (double)p->n_fine;
  g.K = p->n_samples;
  g.L = p->n_fine;
  g.tau = p->spin_twice == 2 ? p->n_squares : 0;
  g.frame = p->rotating_frame;
  g.method = p->method;
  hipFunction_t fn = m->fn[p->spin_twice - 1];
  int blocks = 0, cu = api_device_cu_count();
  int64_t slots = 0;
  if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn, B, 0) == hipSuccess)
    slots = (int64_t)blocks * (B / 64) * cu;
  api_plan_lane_segments(g, S, given, slots);
  const unsigned grid = (unsigned)((api_grid_waves(g) * 64 + B - 1) / B);
  void* args[] = {&g};
  hipError_t e = hipModuleLaunchKernel(fn, grid, 1, 1, (unsigned)B, 1, 1, 0,
                                       (hipStream_t)stream, args, nullptr);
  if (e != hipSuccess) return api_hip_fail(e, "user sampler integrate launch");
  return api_ok();
}

mss_status mss_sampler_solve(mss_sampler s, const mss_problem* p, const double* params,
                             const double* psi0, double* U, double* psi, double* psi_final,
                             double* time, void* ws, size_t ws_bytes, void* stream) {
  if (!s) return api_fail(MSS_E_INVALID, "sampler is NULL");
  mss_status st = api_validate_problem(p);
  if (st != MSS_OK) return st;
  if (!psi0 || !psi) return api_fail(MSS_E_INVALID, "psi0 and psi are required");
  size_t need = 0, scan_bytes = 0;
  if ((st = mss_workspace_size(p, U != nullptr, &need)) != MSS_OK) return st;
  if ((st = mss_propagate_workspace_size(p->spin_twice, p->n_samples, &scan_bytes)) != MSS_OK)
    return st;
  if (need > 0 && (!ws || ws_bytes < need))
    return api_fail(MSS_E_NOMEM, "workspace too small: need %zu bytes, got %zu", need,
                    ws ? ws_bytes : (size_t)0);
  double* Uw = U ? U : (double*)((char*)ws + scan_bytes);
  if ((st = mss_sampler_integrate(s, p, params, Uw, time, nullptr, stream)) != MSS_OK) return st;
  return mss_propagate(p->spin_twice, p->n_samples, Uw, psi0, psi, psi_final, ws, scan_bytes,
                       stream);
}

void mss_sampler_destroy(mss_sampler s) {
  if (!s) return;
  int cur = 0;
  const bool have_cur = hipGetDevice(&cur) == hipSuccess;
  for (auto& kv : s->loaded) {
    if (hipSetDevice(kv.first) != hipSuccess) continue;
    (void)hipDeviceSynchronize();
    (void)hipModuleUnload(kv.second.mod);
  }
  if (have_cur) (void)hipSetDevice(cur);
  delete s;
}

}  // extern "C"

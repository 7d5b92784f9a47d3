// C ABI of the solver (include/mss.h): host-side validation, launch
// planning, workspace layout and the launch sequence of the path.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>

#include "mss_internal.h"

using namespace mss;

namespace {
thread_local std::string g_err;
}  // namespace

namespace mss {

mss_status api_fail(mss_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

mss_status api_fail_text(mss_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

mss_status api_ok() {
  g_err.clear();
  return MSS_OK;
}

mss_status api_hip_fail(hipError_t e, const char* what) {
  return api_fail(MSS_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

std::string api_last_error_copy() { return g_err; }

}  // namespace mss

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool finite(double x) { return isfinite(x) != 0; }

bool slot_ok(int32_t slot, int32_t count, int32_t n_params) {
  return slot < 0 || ((int64_t)slot + count <= (int64_t)n_params);
}

// Compute units of the current device (256 on an MI355X; also the value
// assumed when no device is visible, so planning works host-only).
int device_cu_count() {
  static std::mutex mu;
  static int cache[64];
  static bool init = false;
  std::lock_guard<std::mutex> lock(mu);
  if (!init) {
    for (int& c : cache) c = -1;
    init = true;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
    (void)hipGetLastError();
    return 256;
  }
  if (cache[dev] < 0) {
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cu <= 0) {
      (void)hipGetLastError();
      cu = 256;
    }
    cache[dev] = cu;
  }
  return cache[dev];
}

int ilog2(int x) {
  int l = 0;
  while ((1 << (l + 1)) <= x) ++l;
  return l;
}

// Lane-slice count: minimise (waves per SIMD, rounded up) x (fine steps per
// lane, rounded up); ties go to fewer slices.
int plan_slices(int64_t K, int32_t L, int cu) {
  const int64_t simds = (int64_t)cu * 4;
  int best = 1;
  double best_cost = 1e300;
  for (int S = 1; S <= 64 && S <= L; S <<= 1) {
    const int64_t waves = (K * S + 63) / 64;
    const int64_t per_simd = (waves + simds - 1) / simds;
    const int64_t steps = (L + S - 1) / S;
    const double cost = (double)per_simd * ((double)steps + 0.1 * ilog2(S));
    if (cost < best_cost * (1.0 - 1e-9)) {
      best_cost = cost;
      best = S;
    }
  }
  return best;
}

struct ScanLevels {
  int n_levels;         // number of levels above the operators (0: single tile)
  int64_t n[8];         // n[0] = K, n[l] = elements at level l
  size_t agg_off[8];    // workspace offsets of level-l aggregates (l >= 1)
  size_t state_off[8];  // workspace offsets of level-l entering states (l >= 1)
  size_t bytes;
};

ScanLevels plan_scan(int N, int64_t K) {
  ScanLevels s{};
  s.n[0] = K;
  int l = 0;
  while (s.n[l] > kScanTile) {
    s.n[l + 1] = (s.n[l] + kScanTile - 1) / kScanTile;
    ++l;
  }
  s.n_levels = l;
  size_t off = 0;
  for (int j = 1; j <= l; ++j) {
    s.agg_off[j] = off;
    off += align256((size_t)s.n[j] * 2 * N * N * sizeof(double));
    s.state_off[j] = off;
    off += align256((size_t)s.n[j] * 2 * N * sizeof(double));
  }
  s.bytes = off;
  return s;
}

mss_status validate_terms(int spin_twice, const mss_term* terms, int n_terms, int n_params) {
  for (int i = 0; i < n_terms; ++i) {
    const mss_term& t = terms[i];
    if (t.kind < MSS_TERM_CONST || t.kind > MSS_TERM_PWC_SIN)
      return api_fail(MSS_E_INVALID, "term %d: unknown kind %d", i, t.kind);
    if (t.comp < 0 || t.comp > MSS_V2)
      return api_fail(MSS_E_INVALID, "term %d: comp must be 0..7", i);
    if (t.comp >= MSS_Q && spin_twice != 2)
      return api_fail(MSS_E_INVALID, "term %d: the quadrupole components need spin-1", i);
    if (!finite(t.a) || !finite(t.f) || !finite(t.phi))
      return api_fail(MSS_E_INVALID, "term %d: a, f, phi must be finite", i);
    if (isnan(t.t_on) || isnan(t.t_off)) return api_fail(MSS_E_INVALID, "term %d: NaN window", i);
    if (!slot_ok(t.a_slot, 1, n_params) || !slot_ok(t.f_slot, 1, n_params) ||
        !slot_ok(t.phi_slot, 1, n_params))
      return api_fail(MSS_E_INVALID, "term %d: parameter slot beyond n_params = %d", i, n_params);
    if (t.kind >= MSS_TERM_PWC) {
      if (t.n_seg < 1) return api_fail(MSS_E_INVALID, "term %d: n_seg must be >= 1", i);
      if (!finite(t.seg_t0) || !finite(t.seg_len) || !(t.seg_len > 0.0))
        return api_fail(MSS_E_INVALID, "term %d: seg_t0 finite and seg_len > 0 required", i);
      if (!slot_ok(t.seg_a_slot, t.n_seg, n_params) || !slot_ok(t.seg_phi_slot, t.n_seg, n_params))
        return api_fail(MSS_E_INVALID, "term %d: segment slots beyond n_params = %d", i, n_params);
    }
  }
  return MSS_OK;
}

mss_status validate_problem(const mss_problem* p) {
  if (!p) return api_fail(MSS_E_INVALID, "problem is NULL");
  if (p->spin_twice != 1 && p->spin_twice != 2)
    return api_fail(MSS_E_INVALID, "spin_twice must be 1 (spin-1/2) or 2 (spin-1), got %d",
                p->spin_twice);
  if (p->n_terms < 0 || p->n_terms > MSS_MAX_TERMS)
    return api_fail(MSS_E_INVALID, "n_terms must be in [0, %d], got %d", MSS_MAX_TERMS, p->n_terms);
  if (p->n_terms > 0 && !p->terms) return api_fail(MSS_E_INVALID, "terms is NULL");
  if (p->n_params < 0) return api_fail(MSS_E_INVALID, "n_params must be >= 0");
  if (p->n_fine < 1) return api_fail(MSS_E_INVALID, "n_fine (L) must be >= 1, got %d", p->n_fine);
  if (p->n_samples < 1)
    return api_fail(MSS_E_INVALID, "n_samples (K) must be >= 1, got %lld", (long long)p->n_samples);
  if (p->n_samples > ((int64_t)1 << 40))
    return api_fail(MSS_E_INVALID, "n_samples (K) too large: %lld", (long long)p->n_samples);
  if (!finite(p->t_start)) return api_fail(MSS_E_INVALID, "t_start is not finite");
  if (!finite(p->dt_out) || !(p->dt_out > 0.0))
    return api_fail(MSS_E_INVALID, "dt_out must be finite and > 0");
  if (!finite(p->t_start + (double)p->n_samples * p->dt_out))
    return api_fail(MSS_E_INVALID, "t_start + K * dt_out is not finite");
  if (p->n_squares < 0 || p->n_squares > MSS_MAX_SQUARES)
    return api_fail(MSS_E_INVALID, "n_squares (tau) must be in [0, %d], got %d", MSS_MAX_SQUARES,
                p->n_squares);
  if (p->rotating_frame != 0 && p->rotating_frame != 1)
    return api_fail(MSS_E_INVALID, "rotating_frame must be 0 or 1");
  if (p->method < MSS_CF4 || p->method > MSS_HEUN)
    return api_fail(MSS_E_INVALID, "unknown method %d", p->method);
  return validate_terms(p->spin_twice, p->terms, p->n_terms, p->n_params);
}

}  // namespace

namespace mss {
int api_device_cu_count() { return device_cu_count(); }
int api_plan_slices(int64_t K, int32_t L, int cu) { return plan_slices(K, L, cu); }
int api_ilog2(int x) { return ilog2(x); }
mss_status api_validate_problem(const mss_problem* p) { return validate_problem(p); }
bool api_full_basis(const mss_problem* p) {
  if (p->spin_twice != 2) return false;
  for (int i = 0; i < p->n_terms; ++i)
    if (p->terms[i].comp >= MSS_U1) return true;
  return false;
}
mss_status api_validate_terms(int spin_twice, const mss_term* terms, int n_terms, int n_params) {
  return validate_terms(spin_twice, terms, n_terms, n_params);
}
}  // namespace mss

namespace {

mss_status resolve_launch(const mss_problem* p, const mss_launch* in, int* slices, int* block,
                          bool* given) {
  int S = in ? in->slices : 0;
  if (given) *given = S != 0;
  int B = in ? in->block : 0;
  const int cu = device_cu_count();
  if (S == 0) S = plan_slices(p->n_samples, p->n_fine, cu);
  if (B == 0 && S >= 1 && S <= 64) {
    // a launch of at most 3 waves per SIMD in all runs its waves at once;
    // one-wave workgroups then spread them evenly over the CUs (four-wave
    // workgroups leave some CUs a workgroup more than others: spin-1/2 1e4
    // intervals at 16 slices, 2,500 waves, 19.0 -> 18.5 us).  Longer
    // launches keep 256-lane workgroups, the fastest in a sweep of the
    // 2e5-interval spin-1 simulation.
    const int64_t waves = (p->n_samples * S + 63) / 64;
    B = waves <= 3 * 4 * (int64_t)cu ? 64 : 256;
  }
  if (B == 0) B = 256;
  if (S < 1 || S > 64 || (S & (S - 1)) != 0 || S > p->n_fine)
    return api_fail(MSS_E_INVALID, "launch.slices must be a power of two in [1, min(64, L)], got %d",
                S);
  if (B != 64 && B != 128 && B != 256)
    return api_fail(MSS_E_INVALID, "launch.block must be 64, 128 or 256, got %d", B);
  const int64_t grid = (p->n_samples * S + B - 1) / B;
  if (grid > 0x7fffffffLL) return api_fail(MSS_E_INVALID, "grid too large");
  *slices = S;
  *block = B;
  return MSS_OK;
}

}  // namespace

namespace mss {
mss_status api_resolve_launch(const mss_problem* p, const mss_launch* in, int* slices, int* block,
                              bool* given) {
  return resolve_launch(p, in, slices, block, given);
}

void api_plan_lane_segments(IntervalGrid& g, int S0, bool given, int64_t slots) {
  const int64_t K = g.K;
  const int L = g.L;
  g.n_seg = 1;
  g.seg_sl[0] = g.seg_sl[1] = ilog2(S0);
  g.seg_k0[0] = 0;
  g.seg_w0[0] = 0;
  g.seg_k0[1] = K;
  g.seg_w0[1] = 0;
  if (given || slots <= 0) return;
  const int64_t per0 = 64 / S0;
  const int64_t W0 = (K + per0 - 1) / per0;
  if (W0 <= slots) return;  // at most one round: the slice count already fills it
  const int64_t full = (W0 / slots) * slots;
  const int64_t k_main = full * per0;
  const int64_t rest = K - k_main;
  if (rest <= 0) return;
  // the leftover intervals, sliced as finely as one round of waves allows
  int S1 = S0;
  const int cap = L < 64 ? L : 64;
  while (S1 * 2 <= cap && (rest * S1 * 2 + 63) / 64 <= slots) S1 *= 2;
  if ((L + S1 - 1) / S1 >= (L + S0 - 1) / S0) return;  // no shorter final round
  g.n_seg = 2;
  g.seg_sl[1] = ilog2(S1);
  g.seg_k0[1] = k_main;
  g.seg_w0[1] = full;
}

int64_t api_grid_waves(const IntervalGrid& g) {
  const int j = g.n_seg - 1;
  const int64_t per = 64 >> g.seg_sl[j];
  return g.seg_w0[j] + (g.K - g.seg_k0[j] + per - 1) / per;
}
}  // namespace mss

namespace {
// The ordered product, with <J> of every state when spin is non-null.
mss_status propagate(int32_t spin_twice, int64_t n_samples, const double* U, const double* psi0,
                     double* psi, double* psi_final, double* spin, void* ws, size_t ws_bytes,
                     void* stream) {
  if (spin_twice != 1 && spin_twice != 2) return api_fail(MSS_E_INVALID, "spin_twice must be 1 or 2");
  if (n_samples < 1) return api_fail(MSS_E_INVALID, "n_samples must be >= 1");
  if (!U || !psi0 || !psi) return api_fail(MSS_E_INVALID, "U, psi0 and psi are required");
  const int N = spin_twice + 1;
  const ScanLevels lv = plan_scan(N, n_samples);
  if (lv.bytes > 0 && (!ws || ws_bytes < lv.bytes))
    return api_fail(MSS_E_NOMEM, "workspace too small: need %zu bytes, got %zu", lv.bytes,
                ws ? ws_bytes : (size_t)0);
  hipStream_t st = (hipStream_t)stream;
  char* w = (char*)ws;
  const double* M[8];
  M[0] = U;
  for (int l = 1; l <= lv.n_levels; ++l) M[l] = (const double*)(w + lv.agg_off[l]);
  hipError_t e;
  if (lv.n_levels == 2 && (lv.n[1] + kScanTile - 1) / kScanTile <= kTopWaves) {
    // level 0 up, levels 1-2 in one workgroup, level 0 down
    e = launch_scan_reduce(N, M[0], lv.n[0], (double*)M[1], st);
    if (e == hipSuccess)
      e = launch_scan_top(N, M[1], lv.n[1], psi0, (double*)(w + lv.state_off[1]), st);
    if (e == hipSuccess)
      e = launch_scan_apply(N, M[0], lv.n[0], (const double*)(w + lv.state_off[1]), psi,
                            psi_final, st, spin);
    if (e != hipSuccess) return api_hip_fail(e, "scan launch");
    return api_ok();
  }
  if (lv.n_levels == 1) {
    // level 0 up, then level 0 down with the single level-1 tile folded in
    e = launch_scan_reduce(N, M[0], lv.n[0], (double*)M[1], st);
    if (e == hipSuccess)
      e = launch_scan_apply_fold(N, M[0], lv.n[0], M[1], lv.n[1], psi0, psi, psi_final, st, spin);
    if (e != hipSuccess) return api_hip_fail(e, "scan launch");
    return api_ok();
  }
  for (int l = 0; l < lv.n_levels; ++l) {
    e = launch_scan_reduce(N, M[l], lv.n[l], (double*)M[l + 1], st);
    if (e != hipSuccess) return api_hip_fail(e, "scan reduce launch");
  }
  // top level: one tile entered with psi0
  for (int l = lv.n_levels; l >= 0; --l) {
    const double* start = (l == lv.n_levels) ? psi0 : (const double*)(w + lv.state_off[l + 1]);
    double* before = (l == 0) ? psi : (double*)(w + lv.state_off[l]);
    double* after = (l == 0) ? psi_final : nullptr;
    e = launch_scan_apply(N, M[l], lv.n[l], start, before, after, st, l == 0 ? spin : nullptr);
    if (e != hipSuccess) return api_hip_fail(e, "scan apply launch");
  }
  return api_ok();
}
}  // namespace

namespace mss {
mss_status api_propagate(int32_t spin_twice, int64_t n_samples, const double* U,
                         const double* psi0, double* psi, double* psi_final, void* ws,
                         size_t ws_bytes, void* stream) {
  return propagate(spin_twice, n_samples, U, psi0, psi, psi_final, nullptr, ws, ws_bytes, stream);
}
}  // namespace mss

extern "C" {

const char* mss_status_str(mss_status s) {
  switch (s) {
    case MSS_OK: return "MSS_OK";
    case MSS_E_INVALID: return "MSS_E_INVALID";
    case MSS_E_NOMEM: return "MSS_E_NOMEM";
    case MSS_E_DEVICE: return "MSS_E_DEVICE";
    case MSS_E_UNSUPPORTED: return "MSS_E_UNSUPPORTED";
    case MSS_E_BUSY: return "MSS_E_BUSY";
    case MSS_E_NOTREADY: return "MSS_E_NOTREADY";
  }
  return "MSS_E_UNKNOWN";
}

const char* mss_last_error(void) { return g_err.c_str(); }

const char* mss_version(void) { return "mss 0.1 gfx950"; }

mss_status mss_validate(const mss_problem* p) {
  mss_status s = validate_problem(p);
  return s == MSS_OK ? api_ok() : s;
}

mss_status mss_plan_launch(const mss_problem* p, mss_launch* out) {
  mss_status s = validate_problem(p);
  if (s != MSS_OK) return s;
  if (!out) return api_fail(MSS_E_INVALID, "out is NULL");
  int S, B;
  if ((s = resolve_launch(p, nullptr, &S, &B, nullptr)) != MSS_OK) return s;
  out->slices = S;
  out->block = B;
  return api_ok();
}

mss_status mss_propagate_workspace_size(int32_t spin_twice, int64_t n_samples, size_t* bytes) {
  if (spin_twice != 1 && spin_twice != 2) return api_fail(MSS_E_INVALID, "spin_twice must be 1 or 2");
  if (n_samples < 1) return api_fail(MSS_E_INVALID, "n_samples must be >= 1");
  if (!bytes) return api_fail(MSS_E_INVALID, "bytes is NULL");
  *bytes = plan_scan(spin_twice + 1, n_samples).bytes;
  return api_ok();
}

mss_status mss_workspace_size(const mss_problem* p, int32_t store_u, size_t* bytes) {
  mss_status s = validate_problem(p);
  if (s != MSS_OK) return s;
  if (!bytes) return api_fail(MSS_E_INVALID, "bytes is NULL");
  const int N = p->spin_twice + 1;
  size_t b = plan_scan(N, p->n_samples).bytes;
  if (!store_u) b += align256((size_t)p->n_samples * 2 * N * N * sizeof(double));
  *bytes = b;
  return api_ok();
}

mss_status mss_integrate(const mss_problem* p, const double* params, double* U, double* time,
                         const mss_launch* launch, void* stream) {
  mss_status s = validate_problem(p);
  if (s != MSS_OK) return s;
  if (!U) return api_fail(MSS_E_INVALID, "U is NULL");
  if (p->n_params > 0 && !params) return api_fail(MSS_E_INVALID, "params is NULL but n_params > 0");
  int S, B;
  bool given = false;
  if ((s = resolve_launch(p, launch, &S, &B, &given)) != MSS_OK) return s;
  IntegrateArgs a;
  memset(&a, 0, sizeof a);
  a.fp.n_terms = p->n_terms;
  for (int i = 0; i < p->n_terms; ++i) a.fp.t[i] = p->terms[i];
  a.g.params = params;
  a.g.U = U;
  a.g.time = time;
  a.g.t_start = p->t_start;
  a.g.dt_out = p->dt_out;
  a.g.dt = p->dt_out / (double)p->n_fine;
  a.g.K = p->n_samples;
  a.g.L = p->n_fine;
  a.g.tau = p->spin_twice == 2 ? p->n_squares : 0;
  a.g.frame = p->rotating_frame;
  a.g.method = p->method;
  a.g.full = api_full_basis(p) ? 1 : 0;
  api_plan_lane_segments(a.g, S, given, integrate_slots(p->spin_twice + 1, B));
  hipError_t e = launch_integrate(p->spin_twice + 1, a, B, (hipStream_t)stream);
  if (e != hipSuccess) return api_hip_fail(e, "integrate launch");
  return api_ok();
}


mss_status mss_propagate(int32_t spin_twice, int64_t n_samples, const double* U,
                         const double* psi0, double* psi, double* psi_final, void* ws,
                         size_t ws_bytes, void* stream) {
  return propagate(spin_twice, n_samples, U, psi0, psi, psi_final, nullptr, ws, ws_bytes, stream);
}

mss_status mss_propagate_spin(int32_t spin_twice, int64_t n_samples, const double* U,
                              const double* psi0, double* psi, double* psi_final, double* spin,
                              void* ws, size_t ws_bytes, void* stream) {
  if (!spin) return api_fail(MSS_E_INVALID, "spin is NULL");
  return propagate(spin_twice, n_samples, U, psi0, psi, psi_final, spin, ws, ws_bytes, stream);
}

mss_status mss_spin_projection(int32_t spin_twice, int64_t n_samples, const double* psi,
                               double* out, void* stream) {
  if (spin_twice != 1 && spin_twice != 2) return api_fail(MSS_E_INVALID, "spin_twice must be 1 or 2");
  if (n_samples < 0) return api_fail(MSS_E_INVALID, "n_samples must be >= 0");
  if (n_samples == 0) return api_ok();
  if (!psi || !out) return api_fail(MSS_E_INVALID, "psi and out are required");
  if ((n_samples + 255) / 256 > 0x7fffffffLL) return api_fail(MSS_E_INVALID, "too many samples");
  hipError_t e = launch_spin_projection(spin_twice + 1, psi, n_samples, out, (hipStream_t)stream);
  if (e != hipSuccess) return api_hip_fail(e, "spin projection launch");
  return api_ok();
}

mss_status mss_solve(const mss_problem* p, const double* params, const double* psi0, double* U,
                     double* psi, double* psi_final, double* time, void* ws, size_t ws_bytes,
                     void* stream) {
  mss_status s = validate_problem(p);
  if (s != MSS_OK) return s;
  if (!psi0 || !psi) return api_fail(MSS_E_INVALID, "psi0 and psi are required");
  const int N = p->spin_twice + 1;
  size_t need = 0;
  if ((s = mss_workspace_size(p, U != nullptr, &need)) != MSS_OK) return s;
  if (need > 0 && (!ws || ws_bytes < need))
    return api_fail(MSS_E_NOMEM, "workspace too small: need %zu bytes, got %zu", need,
                ws ? ws_bytes : (size_t)0);
  char* w = (char*)ws;
  const size_t scan_bytes = plan_scan(N, p->n_samples).bytes;
  double* Uw = U ? U : (double*)(w + scan_bytes);
  if ((s = mss_integrate(p, params, Uw, time, nullptr, stream)) != MSS_OK) return s;
  return mss_propagate(p->spin_twice, p->n_samples, Uw, psi0, psi, psi_final, ws, scan_bytes,
                       stream);
}

}  // extern "C"

// Batched execution (C ABI, include/mss.h): many independent simulations of
// uneven length (mixed spin allowed) in one persistent integrator launch
// plus one segmented scan, optionally captured as one HIP graph.  Built on
// the work-set layer (mss_work.h): the plan keeps the packed layout as
// offsets and writes absolute pointers into the device descriptors when a
// run brings new buffers.
#include <stddef.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "mss_work.h"

using namespace mss;

struct mss_batch_plan {
  int32_t n = 0;
  bool needs_params = false;  // some simulation reads parameter slots
  WorkSet work;
  std::vector<int64_t> psi0_off, state_off, op_off, param_off;
  std::vector<size_t> scan_off;  // byte offsets of each simulation's scan scratch
  size_t scan_bytes = 0;
  int64_t op_total = 0;
  int grid_blocks = 0;
  mss_batch_options opt{};
  mss_sampler sampler = nullptr;  // field source of every simulation, or null (field programs)
  // device descriptors
  void* desc = nullptr;
  size_t o_sims = 0, o_terms = 0;
  std::vector<size_t> o_reduce, o_apply;
  size_t o_chain = 0;
  std::vector<char> image;
  DevWork dev;
  const void* uploaded[6] = {};
  bool have_upload = false;
  hipEvent_t last_run = nullptr;
  // graph
  hipStream_t capture_stream = nullptr;
  hipGraphExec_t exec = nullptr;
  const void* graph_key[6] = {};
};

namespace {

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

void release(mss_batch_plan* p) {
  if (!p) return;
  if (p->last_run) (void)hipEventSynchronize(p->last_run);
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
  if (p->last_run) (void)hipEventDestroy(p->last_run);
  if (p->desc) (void)hipFree(p->desc);
  delete p;
}

// Workspace: counter (256 B) | operators, when the caller keeps no U |
// per-simulation scan scratch.  Chained plans: the chain head and slots.
size_t scan_base(const mss_batch_plan* P, bool store_u) {
  return 256 + (store_u ? 0 : a256((size_t)P->op_total * 16));
}

size_t ws_need(const mss_batch_plan* P, bool store_u) {
  if (P->work.chained) return chain_workspace_bytes(P->n);
  return scan_base(P, store_u) + P->scan_bytes;
}

mss_status check_ws(const mss_batch_plan* P, bool store_u, const void* ws, size_t ws_bytes) {
  const size_t need = ws_need(P, store_u);
  if (!ws || ws_bytes < need)
    return api_fail(MSS_E_NOMEM, "workspace too small: need %zu bytes, got %zu", need,
                    ws ? ws_bytes : (size_t)0);
  return MSS_OK;
}

template <class T>
T* shift(T* base, int64_t off) {
  return base ? base + off : nullptr;
}

// Point the descriptors at this call's buffers (NULL state pointers are
// allowed for integrate-only calls).  Re-upload only when they change; the
// plan's earlier work is waited for first, since it reads the descriptors.
mss_status bind(mss_batch_plan* P, const double* params, const double* psi0, double* psi,
                double* psi_final, double* U, void* ws) {
  char* base = (char*)ws;
  const bool chained = P->work.chained;
  double* ops = (U || chained) ? U : (double*)(base + 256);
  const void* key[6] = {params, psi0, psi, psi_final, ops, ws};
  bool same = P->have_upload;
  for (int i = 0; i < 6 && same; ++i) same = P->uploaded[i] == key[i];
  if (same) return MSS_OK;
  if (P->have_upload) {
    hipError_t e = hipEventSynchronize(P->last_run);
    if (e != hipSuccess) return api_hip_fail(e, "batch wait");
  }
  const size_t sb = scan_base(P, U != nullptr);
  for (int i = 0; i < P->n; ++i) {
    SimDesc& d = P->work.sims[i];
    d.params = shift(params, P->param_off[i]);
    d.psi0 = shift(psi0, 2 * P->psi0_off[i]);
    d.psi = shift(psi, 2 * P->state_off[i]);
    d.psi_final = shift(psi_final, 2 * P->psi0_off[i]);
    d.U = shift(ops, 2 * P->op_off[i]);
    d.scan_ws = chained ? nullptr : (double*)(base + sb + P->scan_off[i]);
  }
  P->work.pack(P->image.data(), &P->o_sims, &P->o_terms, &P->o_reduce, &P->o_apply, &P->o_chain);
  hipError_t e = hipMemcpy(P->desc, P->image.data(), P->image.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return api_hip_fail(e, "descriptor upload");
  for (int i = 0; i < 6; ++i) P->uploaded[i] = key[i];
  P->have_upload = true;
  return MSS_OK;
}

// The sampler's work integrator on the current device (null without one).
mss_status user_function(mss_batch_plan* P, hipFunction_t* fn, bool chained = false) {
  *fn = nullptr;
  return P->sampler ? api_sampler_work_function(P->sampler, fn, chained) : MSS_OK;
}

// The whole batch (integrate and scan, or one chained launch) or one half.
hipError_t launch_batch(mss_batch_plan* P, bool integrate, bool scan, void* ws, hipFunction_t fn,
                        hipStream_t st) {
  if (P->work.chained && integrate && scan) {
    const unsigned long long ticks =
        P->opt.chain_wait_us ? 100ull * (unsigned long long)P->opt.chain_wait_us : kChainWaitTicks;
    return launch_work_chained(P->dev, ws, P->grid_blocks, st, fn, ticks);
  }
  hipError_t e = hipSuccess;
  if (integrate) e = launch_work_integrate(P->dev, (unsigned long long*)ws, P->grid_blocks, st, fn);
  if (e == hipSuccess && scan) e = launch_work_scan(P->dev, st);
  return e;
}

mss_status enqueue(mss_batch_plan* P, bool integrate, bool scan, void* ws, hipStream_t st) {
  hipError_t e = hipSuccess;
  hipFunction_t fn = nullptr;
  if (integrate) {
    mss_status s = user_function(P, &fn, P->work.chained && scan);
    if (s != MSS_OK) return s;
  }
  e = launch_batch(P, integrate, scan, ws, fn, st);
  if (e == hipSuccess) e = hipEventRecord(P->last_run, st);
  if (e != hipSuccess) return api_hip_fail(e, "batch launch");
  return MSS_OK;
}

mss_status create_plan(int32_t n, const mss_problem* problems, const int64_t* param_off,
                       const mss_batch_options* options, mss_sampler sampler,
                       mss_batch_plan** out) {
  if (!out) return api_fail(MSS_E_INVALID, "out is NULL");
  *out = nullptr;
  if (n < 1) return api_fail(MSS_E_INVALID, "a batch needs at least one simulation");
  if (!problems) return api_fail(MSS_E_INVALID, "problems is NULL");
  mss_batch_options opt{};
  if (options) opt = *options;
  auto bad_slices = [](int s) { return s < 0 || s > 64 || (s & (s - 1)) != 0; };
  if (bad_slices(opt.slices_spin_half) || bad_slices(opt.slices_spin_one))
    return api_fail(MSS_E_INVALID, "slices must be 0 (choose) or a power of two <= 64");
  if (opt.waves_per_simd < 0 || opt.waves_per_simd > 8)
    return api_fail(MSS_E_INVALID, "waves_per_simd must be in [0, 8]");
  if (opt.scan_per_lane != 0 && opt.scan_per_lane != 2 && opt.scan_per_lane != 4 &&
      opt.scan_per_lane != 8)
    return api_fail(MSS_E_INVALID, "scan_per_lane must be 0, 2, 4 or 8");
  if (opt.chain_wait_us < 0) return api_fail(MSS_E_INVALID, "chain_wait_us must be >= 0");
  if (opt.chained != 0 && opt.chained != 1)
    return api_fail(MSS_E_INVALID, "chained must be 0 or 1");
  const int scan_e = opt.scan_per_lane ? opt.scan_per_lane : kScanPerLane;
  for (int i = 0; i < n; ++i) {
    mss_status s = api_validate_problem(&problems[i]);
    if (s != MSS_OK) {
      std::string m = api_last_error_copy();
      return api_fail(s, "simulation %d: %s", i, m.c_str());
    }
    if (problems[i].n_params > 0 && (!param_off || param_off[i] < 0))
      return api_fail(MSS_E_INVALID, "simulation %d has parameters but no valid param_off", i);
  }
  const int cu = api_device_cu_count();
  // lane-slice count per spin class, planned on the class's total interval count
  int64_t k_class[2] = {0, 0};
  int32_t l_class[2] = {1 << 30, 1 << 30};
  for (int i = 0; i < n; ++i) {
    const int c = problems[i].spin_twice - 1;
    k_class[c] += problems[i].n_samples;
    l_class[c] = std::min(l_class[c], problems[i].n_fine);
  }
  int S_class[2];
  for (int c = 0; c < 2; ++c) {
    const int given = c == 0 ? opt.slices_spin_half : opt.slices_spin_one;
    S_class[c] = given ? given : (k_class[c] ? api_plan_slices(k_class[c], l_class[c], cu) : 1);
  }

  mss_batch_plan* P = new (std::nothrow) mss_batch_plan();
  if (!P) return api_fail(MSS_E_NOMEM, "host allocation failed");
  P->n = n;
  P->opt = opt;
  P->sampler = sampler;
  P->work.scan_e = scan_e;
  P->work.chained = opt.chained != 0;
  P->psi0_off.assign(n + 1, 0);
  P->state_off.assign(n + 1, 0);
  P->op_off.assign(n + 1, 0);
  P->param_off.assign(n, 0);
  P->scan_off.assign(n, 0);
  size_t scan = 0;
  for (int i = 0; i < n; ++i) {
    const mss_problem& q = problems[i];
    const int N = q.spin_twice + 1;
    P->psi0_off[i + 1] = P->psi0_off[i] + N;
    P->state_off[i + 1] = P->state_off[i] + q.n_samples * N;
    P->op_off[i + 1] = P->op_off[i] + q.n_samples * N * N;
    P->param_off[i] = q.n_params > 0 ? param_off[i] : 0;
    if (q.n_params > 0) P->needs_params = true;
    P->scan_off[i] = scan;
    if (!P->work.chained) scan += scan_scratch_bytes(N, q.n_samples, 64 * scan_e);
    int S = S_class[q.spin_twice - 1];
    while (S > q.n_fine) S >>= 1;
    P->work.add(q, api_ilog2(S), 0, q.n_samples, !P->work.chained);
  }
  P->work.finalize();
  if (P->work.chained) {
    // unit tags are unit + 1 in 32 bits
    for (int i = 0; i < n; ++i) {
      const int64_t per = (int64_t)kChainPerLane * (64 >> P->work.sims[i].slices_log2);
      if ((problems[i].n_samples + per - 1) / per >= ((int64_t)1 << 31)) {
        release(P);
        return api_fail(MSS_E_UNSUPPORTED, "simulation %d is too long for a chained plan", i);
      }
    }
  }
  P->scan_bytes = scan;
  P->op_total = P->op_off[n];
  P->image.resize(P->work.packed_bytes());
  P->work.pack(P->image.data(), &P->o_sims, &P->o_terms, &P->o_reduce, &P->o_apply, &P->o_chain);
  hipError_t e = hipMalloc(&P->desc, P->image.size());
  if (e == hipSuccess) e = hipEventCreateWithFlags(&P->last_run, hipEventDisableTiming);
  if (e != hipSuccess) {
    release(P);
    if (e == hipErrorOutOfMemory) return api_fail(MSS_E_NOMEM, "descriptor allocation failed");
    return api_hip_fail(e, "batch plan");
  }
  P->dev = device_view(P->work, (const char*)P->desc, P->o_sims, P->o_terms, P->o_reduce,
                       P->o_apply, P->o_chain);
  int wps = opt.waves_per_simd ? opt.waves_per_simd : 2;
  if (P->work.chained) {
    // a CU holds as many chained workgroups as its LDS has room for their
    // parked operators (two on gfx950, which their registers also allow); a
    // workgroup beyond those would only start once the queue is drained
    int dev = 0, lds = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) ==
            hipSuccess) {
      const int fit = lds / (int)(4 * kChainParkDoubles * sizeof(double));
      if (fit > 0) wps = std::min(wps, fit);
    }
  }
  const int64_t blocks = (int64_t)cu * wps;  // 256-thread blocks: one wave per SIMD each
  const int64_t units = P->work.chained ? P->work.n_units : P->work.n_items;
  P->grid_blocks = (int)std::max<int64_t>(1, std::min(blocks, (units + 3) / 4));
  *out = P;
  return api_ok();
}

}  // namespace

extern "C" {

mss_status mss_batch_plan_create(int32_t n, const mss_problem* problems, const int64_t* param_off,
                                 const mss_batch_options* options, mss_batch_plan** out) {
  return create_plan(n, problems, param_off, options, nullptr, out);
}

mss_status mss_batch_plan_create_sampled(int32_t n, const mss_problem* problems,
                                         const int64_t* param_off,
                                         const mss_batch_options* options, mss_sampler sampler,
                                         mss_batch_plan** out) {
  if (out) *out = nullptr;
  if (!sampler) return api_fail(MSS_E_INVALID, "sampler is NULL");
  if (n >= 1 && problems)
    for (int i = 0; i < n; ++i) {
      if (problems[i].n_terms != 0)
        return api_fail(MSS_E_INVALID, "simulation %d: a sampler problem carries no terms", i);
      const mss_status st = api_sampler_check_problem(sampler, &problems[i]);
      if (st != MSS_OK) return st;
    }
  return create_plan(n, problems, param_off, options, sampler, out);
}

mss_status mss_batch_layout(const mss_batch_plan* P, int64_t* psi0_off, int64_t* state_off,
                            int64_t* op_off) {
  if (!P) return api_fail(MSS_E_INVALID, "plan is NULL");
  for (int i = 0; i <= P->n; ++i) {
    if (psi0_off) psi0_off[i] = P->psi0_off[i];
    if (state_off) state_off[i] = P->state_off[i];
    if (op_off) op_off[i] = P->op_off[i];
  }
  return api_ok();
}

mss_status mss_batch_workspace_size(const mss_batch_plan* P, int32_t store_u, size_t* bytes) {
  if (!P || !bytes) return api_fail(MSS_E_INVALID, "plan and bytes are required");
  *bytes = ws_need(P, store_u != 0);
  return api_ok();
}

mss_status mss_batch_info(const mss_batch_plan* P, mss_batch_info_t* info) {
  if (!P || !info) return api_fail(MSS_E_INVALID, "plan and info are required");
  info->n_sims = P->n;
  info->n_items = P->work.chained ? P->work.n_units : P->work.n_items;
  info->grid_blocks = P->grid_blocks;
  info->scan_levels = P->work.n_levels + 1;
  info->pad = 0;
  info->total_samples = 0;
  for (const SimDesc& d : P->work.sims) info->total_samples += d.K_total;
  return api_ok();
}

mss_status mss_batch_run(mss_batch_plan* P, const double* params, const double* psi0, double* psi,
                         double* psi_final, double* U, void* ws, size_t ws_bytes, void* stream) {
  if (!P) return api_fail(MSS_E_INVALID, "plan is NULL");
  if (!psi0 || !psi) return api_fail(MSS_E_INVALID, "psi0 and psi are required");
  if (P->needs_params && !params)
    return api_fail(MSS_E_INVALID, "params is NULL but the batch has parameterised simulations");
  mss_status s = check_ws(P, U != nullptr, ws, ws_bytes);
  if (s != MSS_OK) return s;
  if ((s = bind(P, params, psi0, psi, psi_final, U, ws)) != MSS_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  if (!P->opt.use_graph) {
    s = enqueue(P, true, true, ws, st);
    return s == MSS_OK ? api_ok() : s;
  }
  bool same = P->exec != nullptr;
  for (int i = 0; i < 6 && same; ++i) same = P->graph_key[i] == P->uploaded[i];
  if (!same) {
    if (P->exec) {
      (void)hipGraphExecDestroy(P->exec);
      P->exec = nullptr;
    }
    hipFunction_t fn = nullptr;
    if ((s = user_function(P, &fn, P->work.chained)) != MSS_OK) return s;
    hipError_t e = hipSuccess;
    if (!P->capture_stream) e = hipStreamCreateWithFlags(&P->capture_stream, hipStreamNonBlocking);
    hipGraph_t g = nullptr;
    if (e == hipSuccess) e = hipStreamBeginCapture(P->capture_stream, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
      hipError_t el = launch_batch(P, true, true, ws, fn, P->capture_stream);
      hipError_t e2 = hipStreamEndCapture(P->capture_stream, &g);
      e = el != hipSuccess ? el : e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&P->exec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) return api_hip_fail(e, "batch graph capture");
    for (int i = 0; i < 6; ++i) P->graph_key[i] = P->uploaded[i];
  }
  hipError_t e = hipGraphLaunch(P->exec, st);
  if (e == hipSuccess) e = hipEventRecord(P->last_run, st);
  if (e != hipSuccess) return api_hip_fail(e, "batch graph launch");
  return api_ok();
}

mss_status mss_batch_integrate(mss_batch_plan* P, const double* params, double* U, void* ws,
                               size_t ws_bytes, void* stream) {
  if (!P) return api_fail(MSS_E_INVALID, "plan is NULL");
  if (P->work.chained && !U)
    return api_fail(MSS_E_INVALID, "a chained plan keeps no operators: mss_batch_integrate needs U");
  if (P->needs_params && !params)
    return api_fail(MSS_E_INVALID, "params is NULL but the batch has parameterised simulations");
  mss_status s = check_ws(P, U != nullptr, ws, ws_bytes);
  if (s != MSS_OK) return s;
  // the integrator reads no states: keep whatever state pointers are bound
  const double* psi0 = P->have_upload ? (const double*)P->uploaded[1] : nullptr;
  double* psi = P->have_upload ? (double*)P->uploaded[2] : nullptr;
  double* fin = P->have_upload ? (double*)P->uploaded[3] : nullptr;
  if ((s = bind(P, params, psi0, psi, fin, U, ws)) != MSS_OK) return s;
  s = enqueue(P, true, false, ws, (hipStream_t)stream);
  return s == MSS_OK ? api_ok() : s;
}

mss_status mss_batch_propagate(mss_batch_plan* P, const double* psi0, double* psi,
                               double* psi_final, const double* U, void* ws, size_t ws_bytes,
                               void* stream) {
  if (!P) return api_fail(MSS_E_INVALID, "plan is NULL");
  if (P->work.chained)
    return api_fail(MSS_E_UNSUPPORTED,
                    "a chained plan forms its states in mss_batch_run (create the plan with "
                    "chained = 0 for a separate scan)");
  if (!psi0 || !psi) return api_fail(MSS_E_INVALID, "psi0 and psi are required");
  mss_status s = check_ws(P, U != nullptr, ws, ws_bytes);
  if (s != MSS_OK) return s;
  const double* params = P->have_upload ? (const double*)P->uploaded[0] : nullptr;
  if ((s = bind(P, params, psi0, psi, psi_final, (double*)U, ws)) != MSS_OK) return s;
  s = enqueue(P, false, true, ws, (hipStream_t)stream);
  return s == MSS_OK ? api_ok() : s;
}

mss_status mss_batch_check(const mss_batch_plan* P, const void* ws, void* stream) {
  if (!P) return api_fail(MSS_E_INVALID, "plan is NULL");
  if (!P->work.chained) return api_ok();
  if (!ws) return api_fail(MSS_E_INVALID, "ws is NULL");
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  unsigned long long failed = 0;
  if (e == hipSuccess)
    e = hipMemcpy(&failed, (const char*)ws + offsetof(ChainSync, failed), sizeof failed,
                  hipMemcpyDeviceToHost);
  if (e != hipSuccess) return api_hip_fail(e, "chained run check");
  if (failed == ~0ull)
    return api_fail(MSS_E_DEVICE, "chained run failed: a wave reached its dequeue with lanes "
                                  "missing; the states are undefined");
  if (failed)
    return api_fail(MSS_E_DEVICE,
                    "chained run failed: unit %llu of a simulation waited longer than the "
                    "bound for its entering state; the states are undefined",
                    failed);
  return api_ok();
}

void mss_batch_plan_destroy(mss_batch_plan* P) { release(P); }

mss_status mss_solve_batch(int32_t n, const mss_problem* problems, const int64_t* param_off,
                           const double* params, const double* psi0, double* psi,
                           double* psi_final, double* U, void* stream) {
  if (!psi0 || !psi) return api_fail(MSS_E_INVALID, "psi0 and psi are required");
  mss_batch_options opt{};
  opt.chained = 1;
  mss_batch_plan* P = nullptr;
  mss_status s = create_plan(n, problems, param_off, &opt, nullptr, &P);
  if (s != MSS_OK) return s;
  if (P->needs_params && !params)
    s = api_fail(MSS_E_INVALID, "params is NULL but the batch has parameterised simulations");
  const size_t bytes = ws_need(P, U != nullptr);
  void* ws = nullptr;
  if (s == MSS_OK) {
    hipError_t e = hipMalloc(&ws, bytes);
    if (e != hipSuccess)
      s = e == hipErrorOutOfMemory ? api_fail(MSS_E_NOMEM, "workspace allocation failed")
                                   : api_hip_fail(e, "workspace allocation");
  }
  if (s == MSS_OK) s = mss_batch_run(P, params, psi0, psi, psi_final, U, ws, bytes, stream);
  if (s == MSS_OK) s = mss_batch_check(P, ws, stream);  // waits for the run
  if (ws) (void)hipFree(ws);
  release(P);
  return s == MSS_OK ? api_ok() : s;
}

}  // extern "C"

// C entry points of operator application, the right-hand side, the time
// step, the RK time loop and the launch-shape tuner.
#include <string>
#include <vector>

#include "gather.hpp"
#include "tune_cache.hpp"

namespace labfm {
std::mutex g_cfg_mutex;
labfm_launch_config g_cfg[3][3] = {};
std::mutex g_event_mutex;
std::vector<hipEvent_t> g_events;
}  // namespace labfm

using namespace labfm;

extern "C" int labfm_apply_operators(const labfm_operators* ops, uint32_t op_mask,
                                     const double* phi, double* out, labfm_prec prec,
                                     void* stream_) {
  clear_error();
  if (int r = check_ops(ops, prec, "apply_operators")) return r;
  LABFM_REQUIRE(phi && out, "apply_operators: null field pointer");
  LABFM_REQUIRE(op_mask != 0 && op_mask < (1u << LABFM_NUM_OPS),
                "apply_operators: op_mask must select operators 0..5");
  hipStream_t st = as_stream(stream_);
  const LaunchCfg cfg = cfg_for(LABFM_KERNEL_APPLY, prec, ops->n, ops->nnz);
  hipError_t e = with_prec(prec, ops, [&](auto pol, const auto* w) {
    return launch_apply<decltype(pol)>(cfg, ops, w, op_mask, phi, out, st);
  });
  LABFM_HIP(e);
  return LABFM_OK;
}

extern "C" int labfm_ns_rhs(const double* q, const labfm_operators* ops,
                            const labfm_rk_params* prm, double* out, labfm_prec prec,
                            void* stream_) {
  clear_error();
  if (int r = check_ops(ops, prec, "ns_rhs")) return r;
  LABFM_REQUIRE(q && prm && out, "ns_rhs: null argument");
  LABFM_REQUIRE(out != q, "ns_rhs: out must not alias q");
  hipStream_t st = as_stream(stream_);
  const LaunchCfg cfg = cfg_for(LABFM_KERNEL_STAGE, prec, ops->n, ops->nnz);
  const Flow fl{prm->c2, prm->mu, prm->gx, prm->gy};
  hipError_t e = with_prec(prec, ops, [&](auto pol, const auto* w) {
    return launch_stage<decltype(pol)>(cfg, ops, w, q, nullptr, out, nullptr, 0.0, 1.0, fl, st);
  });
  LABFM_HIP(e);
  return LABFM_OK;
}

extern "C" size_t labfm_time_step_workspace_bytes(void) {
  return align256(sizeof(double) * (1024 + 1));
}

extern "C" int labfm_time_step(const double* q, const double* s, int32_t n, double c2, double mu,
                               double conv_coef, double visc_coef, double* dt_out,
                               void* workspace, size_t workspace_bytes, void* stream_) {
  clear_error();
  LABFM_REQUIRE(n > 0 && q && s && dt_out, "time_step: bad arguments");
  LABFM_REQUIRE(c2 > 0.0 && mu > 0.0, "time_step: c2 and mu must be positive");
  LABFM_REQUIRE(conv_coef > 0.0 && visc_coef > 0.0, "time_step: coefficients must be positive");
  LABFM_WORKSPACE(workspace, workspace_bytes, labfm_time_step_workspace_bytes(), "time_step");
  hipStream_t st = as_stream(stream_);
  const int nb = static_cast<int>(std::min<long long>(1024, blocks_for(n, kRedThreads)));
  double* d = static_cast<double*>(workspace);
  hipLaunchKernelGGL(dt_partial_kernel, dim3(nb), dim3(kRedThreads), 0, st, q, s, n, sqrt(c2),
                     mu, conv_coef, visc_coef, d);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    hipLaunchKernelGGL(min_final_kernel, dim3(1), dim3(kRedThreads), 0, st, d, nb, d + nb);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(dt_out, d + nb, sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  LABFM_HIP(e);
  return LABFM_OK;
}

extern "C" size_t labfm_rk_workspace_bytes(int32_t n) {
  if (n <= 0) return 0;
  // two stage registers of 3n doubles, then an int flag (256-byte aligned)
  return 2 * 3 * static_cast<size_t>(n) * sizeof(double) + 256;
}

extern "C" int labfm_rk_step(double* q, const labfm_operators* ops, const labfm_rk_params* prm,
                             int32_t n_steps, labfm_prec prec, int32_t use_graph,
                             void* workspace, size_t workspace_bytes, labfm_timing* timing,
                             void* stream_) {
  clear_error();
  if (int r = check_ops(ops, prec, "rk_step")) return r;
  LABFM_REQUIRE(q && prm, "rk_step: null state or parameters");
  LABFM_REQUIRE(n_steps >= 0, "rk_step: n_steps must be >= 0");
  LABFM_REQUIRE(prm->dt > 0.0 && std::isfinite(prm->dt), "rk_step: dt must be positive");
  LABFM_REQUIRE(!prm->filter || ops->kappa, "rk_step: filter requires kappa");
  const int n = ops->n;
  LABFM_REQUIRE(workspace && workspace_bytes >= labfm_rk_workspace_bytes(n),
                "rk_step: workspace of %zu bytes required", labfm_rk_workspace_bytes(n));
  hipStream_t st = as_stream(stream_);
  double* Ya = static_cast<double*>(workspace);
  double* Yb = Ya + 3 * static_cast<size_t>(n);
  int* flag = reinterpret_cast<int*>(Yb + 3 * static_cast<size_t>(n));

  StepPlan plan;
  plan.ops = ops;
  plan.w = (prec == LABFM_F64) ? static_cast<const void*>(ops->w)
                               : static_cast<const void*>(ops->w32);  // F32 policies
  plan.prec = prec;
  plan.stage_cfg = cfg_for(LABFM_KERNEL_STAGE, prec, n, ops->nnz);
  plan.filter_cfg = cfg_for(LABFM_KERNEL_FILTER, prec, n, ops->nnz);
  plan.fl = Flow{prm->c2, prm->mu, prm->gx, prm->gy};
  plan.dt = prm->dt;
  plan.filter = prm->filter;
  plan.Q = q;
  plan.Ya = Ya;
  plan.Yb = Yb;

  if (timing) {
    // event-timed launches (no graph); 6 marks per timed step, one step in
    // every `every` timed
    std::lock_guard<std::mutex> lock(g_event_mutex);
    const int per_step = 6;
    const int every = timing->every > 1 ? timing->every : 1;
    const int timed = (n_steps + every - 1) / every;
    LABFM_HIP(reserve_events(static_cast<size_t>(per_step) * timed));
    double stage = 0.0, filt = 0.0;
    long long ns = 0, nf = 0;
    Marks mk{g_events.data(), 0};
    hipError_t e = hipSuccess;
    for (int k = 0; k < n_steps && e == hipSuccess; ++k)
      e = enqueue_step_any(plan, st, (k % every == 0) ? &mk : nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    for (int k = 0; k < timed && e == hipSuccess; ++k) {
      for (int l = 0; l < 5 && e == hipSuccess; ++l) {
        float ms = 0.0f;
        e = hipEventElapsedTime(&ms, g_events[k * per_step + l], g_events[k * per_step + l + 1]);
        if (l < 4) {
          stage += ms;
          ++ns;
        } else if (prm->filter) {
          filt += ms;
          ++nf;
        }
      }
    }
    LABFM_HIP(e);
    timing->stage_ms = stage;
    timing->filter_ms = filt;
    timing->stage_launches = ns;
    timing->filter_launches = nf;
  } else if (use_graph && n_steps > 0) {
    // capture one step on a private stream, replay it n_steps times
    hipStream_t cs = nullptr;
    LABFM_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipEvent_t join = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipEventCreateWithFlags(&join, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(join, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(cs, join, 0);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t ce = enqueue_step_any(plan, cs, nullptr);
      e = hipStreamEndCapture(cs, &graph);
      if (ce != hipSuccess) e = ce;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    for (int k = 0; k < n_steps && e == hipSuccess; ++k) e = hipGraphLaunch(exec, cs);
    if (e == hipSuccess) e = hipEventRecord(join, cs);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, join, 0);
    // the graph and stream may only be released once the replays are done
    if (e == hipSuccess) e = hipStreamSynchronize(cs);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (join) (void)hipEventDestroy(join);
    (void)hipStreamDestroy(cs);
    LABFM_HIP(e);
  } else {
    for (int k = 0; k < n_steps; ++k) LABFM_HIP(enqueue_step_any(plan, st, nullptr));
  }

  if (prm->check_finite) {
    LABFM_HIP(hipMemsetAsync(flag, 0, sizeof(int), st));
    const long long len = 3LL * n;
    const unsigned nb = static_cast<unsigned>(std::min<long long>(2048, blocks_for(len, 256)));
    hipLaunchKernelGGL(nonfinite_kernel, dim3(nb), dim3(256), 0, st, q, len, flag);
    LABFM_LAUNCHED();
    int h_flag = 0;
    LABFM_HIP(hipMemcpyAsync(&h_flag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    LABFM_HIP(hipStreamSynchronize(st));
    if (h_flag) {
      set_error("rk_step: non-finite value in the state after %d steps", n_steps);
      return LABFM_ERR_NONFINITE;
    }
  }
  return LABFM_OK;
}

extern "C" int labfm_get_launch_config(int32_t kernel, labfm_prec prec, int32_t n, int64_t nnz,
                                       labfm_launch_config* cfg) {
  clear_error();
  LABFM_REQUIRE(kernel >= 0 && kernel <= 2 && cfg, "get_launch_config: bad arguments");
  LABFM_REQUIRE(known_prec(prec), "get_launch_config: bad precision");
  const LaunchCfg c = cfg_for(kernel, prec, n, nnz);
  cfg->lanes_per_node = c.lpn;
  cfg->flags = c.flags;
  return LABFM_OK;
}

extern "C" int labfm_set_launch_config(int32_t kernel, labfm_prec prec,
                                       const labfm_launch_config* cfg) {
  clear_error();
  LABFM_REQUIRE(kernel >= 0 && kernel <= 2, "set_launch_config: unknown kernel %d", kernel);
  LABFM_REQUIRE(known_prec(prec), "set_launch_config: bad precision");
  labfm_launch_config c{0, 0};
  if (cfg && cfg->lanes_per_node != 0) {
    LABFM_REQUIRE(valid_cfg(*cfg), "set_launch_config: unsupported shape (%d lanes, flags %d)",
                  cfg->lanes_per_node, cfg->flags);
    c = *cfg;
  }
  std::lock_guard<std::mutex> lock(g_cfg_mutex);
  g_cfg[kernel][prec_slot(prec)] = c;
  return LABFM_OK;
}

extern "C" int labfm_tune(const labfm_operators* ops, const double* q, labfm_prec prec,
                          int32_t reps, void* workspace, size_t workspace_bytes,
                          const char* cache_path, labfm_launch_config* best, double* best_ms,
                          int32_t* from_cache, void* stream_) {
  clear_error();
  if (int r = check_ops(ops, prec, "tune")) return r;
  LABFM_REQUIRE(q && best && best_ms && reps > 0, "tune: bad arguments");
  const int n = ops->n;
  LABFM_WORKSPACE(workspace, workspace_bytes, labfm_rk_workspace_bytes(n), "tune");
  LABFM_REQUIRE(ops->kappa, "tune: kappa required");
  hipStream_t st = as_stream(stream_);
  if (from_cache) *from_cache = 0;

  // the cache keys: kernel, precision, device and what the kernels' speed
  // depends on (node count, stencil entries, tiles, wall equation)
  static const char* const kKernelNames[3] = {"stage", "filter", "apply"};
  const std::string path = tune_cache_path(cache_path);
  std::vector<TuneEntry> entries(3);
  {
    const std::string common = "/prec" + std::to_string(static_cast<int>(prec)) + "/" +
                               tune_device_key() + "/n" + std::to_string(n) + "/nnz" +
                               std::to_string(static_cast<long long>(ops->nnz)) + "/tiles" +
                               std::to_string(ops->tiles ? 1 : 0) + "/walls" +
                               std::to_string(ops->wall_normal ? 1 : 0);
    for (int k = 0; k < 3; ++k) entries[k].key = std::string("launch/") + kKernelNames[k] + common;
  }
  if (!path.empty() && tune_cache_lookup(path, entries)) {
    bool ok = true;
    for (int k = 0; k < 3; ++k) {
      const labfm_launch_config c{entries[k].a, entries[k].b};
      ok = ok && valid_cfg(c);
    }
    if (ok) {
      std::lock_guard<std::mutex> lock(g_cfg_mutex);
      for (int k = 0; k < 3; ++k) {
        best[k] = labfm_launch_config{entries[k].a, entries[k].b};
        best_ms[k] = entries[k].ms;
        g_cfg[k][prec_slot(prec)] = best[k];
      }
      if (from_cache) *from_cache = 1;
      return LABFM_OK;
    }
  }
  double* out = static_cast<double*>(workspace);
  const Flow fl{1.0, 1.0, 0.0, 0.0};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  LABFM_HIP(hipEventCreate(&e0));
  LABFM_HIP(hipEventCreate(&e1));
  hipError_t err = hipSuccess;
  const int lpns[4] = {4, 8, 16, 32};
  constexpr int kCands = 16, kPasses = 2;
  for (int kernel = 0; kernel < 3 && err == hipSuccess; ++kernel) {
    // every candidate is timed in kPasses interleaved passes and keeps its
    // best mean; the default shape stays unless another is more than
    // kMargin faster (timing noise does not flip the choice)
    constexpr double kMargin = 0.02;
    double t[kCands];
    for (int k = 0; k < kCands; ++k) t[k] = 1e300;
    for (int pass = 0; pass < kPasses && err == hipSuccess; ++pass) {
      for (int k = 0; k < kCands && err == hipSuccess; ++k) {
        const LaunchCfg c{lpns[k / 4], k % 4};
        auto launch = [&]() -> hipError_t {
          return with_prec(prec, ops, [&](auto pol, const auto* w) {
            using P = decltype(pol);
            if (kernel == LABFM_KERNEL_STAGE)
              return launch_stage<P>(c, ops, w, q, nullptr, out, nullptr, 0.0, 1.0, fl, st);
            if (kernel == LABFM_KERNEL_FILTER) return launch_filter<P>(c, ops, w, q, out, st);
            // apply: the five derivative operators of u
            return launch_apply<P>(c, ops, w, 0x1F, q + n, out, st);
          });
        };
        err = launch();  // warm-up
        if (err == hipSuccess) err = hipEventRecord(e0, st);
        for (int r = 0; r < reps && err == hipSuccess; ++r) err = launch();
        if (err == hipSuccess) err = hipEventRecord(e1, st);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        if (err == hipSuccess) t[k] = std::min(t[k], static_cast<double>(ms) / reps);
      }
    }
    if (err != hipSuccess) break;
    const LaunchCfg d = default_cfg(kernel, prec, n, ops->nnz);
    int kd = 0;
    for (int k = 0; k < kCands; ++k)
      if (lpns[k / 4] == d.lpn && k % 4 == d.flags) kd = k;
    int kb = kd;
    for (int k = 0; k < kCands; ++k)
      if (t[k] < t[kb]) kb = k;
    if (!(t[kb] < (1.0 - kMargin) * t[kd])) kb = kd;
    best[kernel].lanes_per_node = lpns[kb / 4];
    best[kernel].flags = kb % 4;
    best_ms[kernel] = t[kb];
    std::lock_guard<std::mutex> lock(g_cfg_mutex);
    g_cfg[kernel][prec_slot(prec)] = best[kernel];
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  LABFM_HIP(err);
  if (path.empty()) return LABFM_OK;
  for (int k = 0; k < 3; ++k) {
    entries[k].a = best[k].lanes_per_node;
    entries[k].b = best[k].flags;
    entries[k].ms = best_ms[k];
  }
  std::string msg;
  if (!tune_cache_store(path, entries, msg)) {
    set_error("tune: tune cache: %s", msg.c_str());
    return LABFM_ERR_ARG;
  }
  return LABFM_OK;
}

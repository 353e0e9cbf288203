// Launch-shape autotuner: times project_validate_motions on the caller's
// sample motions for every candidate (W, sphere batch 4 / 8 / 16, or 4 / 8
// for the planners' round kernels) and keeps
// the fastest by validated-waypoint throughput.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "cprrtc.h"
#include "handles.h"

namespace {

// q_to' = q_from + s (q_to - q_from): the same direction, steer length scaled
// with the waypoint count so the initial spacing stays the same.
__global__ void rescale_kernel(const float* __restrict__ q_from, const float* __restrict__ q_to,
                               float* __restrict__ out, long n, float s) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = q_from[i] + s * (q_to[i] - q_from[i]);
}

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace

extern "C" {

int cp_autotune(const cp_robot* robot, const cp_env* env, const cp_constraint* constraint,
                cp_proj_params* params, int32_t n_motions, const float* d_q_from,
                const float* d_q_to, int32_t flags, int32_t reps, cp_tune_report* report,
                void* stream) {
  using namespace cprrtc;
  try {
    if (!robot || !env || !params || !d_q_from || !d_q_to)
      return api_fail(CP_E_ARG, "cp_autotune: NULL argument");
    if (n_motions < 1 || reps < 1 || reps > 1000)
      return api_fail(CP_E_ARG, "cp_autotune: n_motions < 1 or reps outside 1..1000");
    cp_proj_params base;
    int rc = api_params(params, &base);
    if (rc != CP_OK) return rc;
    const int dof = robot->host.dof;
    hipStream_t st = (hipStream_t)stream;
    const size_t nq = (size_t)n_motions * dof;
    DevBuf qt, xi, status;
    hipError_t e = hipMalloc(&qt.p, sizeof(float) * nq);
    if (e == hipSuccess) e = hipMalloc(&xi.p, sizeof(float) * nq * 64);
    if (e == hipSuccess) e = hipMalloc(&status.p, sizeof(int32_t) * n_motions);
    if (e != hipSuccess) return api_hip_fail(e, "cp_autotune buffers");
    hipEvent_t t0 = nullptr, t1 = nullptr;
    e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    if (e != hipSuccess) {
      if (t0) (void)hipEventDestroy(t0);
      return api_hip_fail(e, "cp_autotune events");
    }

    const int Ws[2] = {32, 64};
    const int Bs[3] = {4, 8, 16};
    std::vector<int32_t> st_h(n_motions);
    cp_tune_report rep;
    std::memset(&rep, 0, sizeof rep);
    double best = -1.0;
    cp_proj_params chosen = base;
    for (int wi = 0; wi < 2 && rc == CP_OK; ++wi) {
      const int W = Ws[wi];
      if (!(flags & CP_TUNE_W) && W != base.W) continue;
      // sample motions rescaled from the caller's W to this W
      const float s = (float)(W - 1) / (float)(base.W - 1);
      rescale_kernel<<<(unsigned)((nq + 255) / 256), 256, 0, st>>>(d_q_from, d_q_to, (float*)qt.p,
                                                                   (long)nq, s);
      e = hipGetLastError();
      if (e != hipSuccess) {
        rc = api_hip_fail(e, "cp_autotune rescale");
        break;
      }
      for (int bi = 0; bi < ((flags & CP_TUNE_PLANNER) ? 2 : 3) && rc == CP_OK; ++bi) {
        cp_proj_params p = base;
        p.W = W;
        p.sphere_batch = Bs[bi];
        // one untimed call (first-touch, instruction cache), then reps timed calls
        rc = project_validate_motions(robot, env, constraint, &p, n_motions, d_q_from,
                                      (const float*)qt.p, (float*)xi.p, (int32_t*)status.p,
                                      nullptr, nullptr, 0, stream);
        if (rc != CP_OK) break;
        e = hipEventRecord(t0, st);
        for (int r = 0; r < reps && rc == CP_OK; ++r)
          rc = project_validate_motions(robot, env, constraint, &p, n_motions, d_q_from,
                                        (const float*)qt.p, (float*)xi.p, (int32_t*)status.p,
                                        nullptr, nullptr, 0, stream);
        if (rc != CP_OK) break;
        if (e == hipSuccess) e = hipEventRecord(t1, st);
        if (e == hipSuccess)
          e = hipMemcpyAsync(st_h.data(), status.p, sizeof(int32_t) * n_motions,
                             hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
        if (e != hipSuccess) {
          rc = api_hip_fail(e, "cp_autotune timing");
          break;
        }
        long decided = 0;
        for (int m = 0; m < n_motions; ++m) decided += st_h[m] != CP_MOTION_PROJ_FAIL;
        const double sec = (double)ms * 1e-3 / reps;
        const double rate = sec > 0 ? (double)decided * (W - 1) / sec : 0.0;
        const int k = rep.n++;
        rep.W[k] = W;
        rep.sphere_batch[k] = Bs[bi];
        rep.ms[k] = (double)ms / reps;
        rep.waypoints_per_s[k] = rate;
        if (rate > best) {
          best = rate;
          chosen = p;
        }
      }
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (rc != CP_OK) return rc;
    *params = chosen;
    if (report) *report = rep;
    return CP_OK;
  } catch (...) {
    return api_fail(CP_E_ARG, "cp_autotune: unexpected exception");
  }
}

}  // extern "C"

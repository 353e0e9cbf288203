// Library-internal definitions of the opaque C-ABI handles and the helpers
// the translation units of libcprrtc.so share.
#pragma once
#include <hip/hip_runtime.h>

#include <deque>
#include <mutex>
#include <vector>

#include "cprrtc.h"
#include "device.h"

namespace cprrtc {
// Kernels compiled at run time for one robot, constraint kind and set of
// locked axes (null where not compiled).
struct RtcFns {
  hipFunction_t pool = nullptr;                          // pooled projection
  hipFunction_t plan[2] = {nullptr, nullptr};            // planner round, sphere batch 4 / 8
  hipFunction_t validate[3] = {nullptr, nullptr, nullptr};  // culled validation, 4 / 8 / 16
  hipFunction_t fkcc[2] = {nullptr, nullptr};              // FK + CC of configurations, 4 / 8
};
struct RtcKernel {
  int kind = 0;
  unsigned mask = 0;                 // bit i = axis i locked
  std::vector<hipModule_t> modules;  // every module this entry's kernels live in
  RtcFns fns;
  double compile_ms = 0.0;
};
struct PlanDev;
}  // namespace cprrtc

struct cp_robot {
  cprrtc::RobotDev host;            // host copy (dispatch reads dof, chains, limits)
  cprrtc::RobotDev* dev = nullptr;  // device copy
  float4* spheres = nullptr;        // device spheres, grouped by link
  int2* pairs = nullptr;            // device self-collision pairs (positions in `spheres`)
  int2* pairs_cc = nullptr;         // the same pairs as (s | t << 16, bits of (r_s + r_t)^2),
                                    // grouped by s for the self-collision kernel
  int n_cc = 0;                     // entries of pairs_cc the kernel walks
  int2* sph_map = nullptr;          // device, per sphere in description order: (position in
                                    // `spheres`, joint frame that carries it)
  std::vector<int32_t> self_pairs;  // host, description order: s0 t0 s1 t1 ...
  std::mutex rtc_lock;              // guards rtc (specialisation may run beside projections)
  std::deque<cprrtc::RtcKernel> rtc; // a deque: entries stay put as more are added
};

struct cp_env {
  cprrtc::EnvDev view;              // device pointers + counts, passed by value to kernels
  float4* block = nullptr;          // one allocation holding every primitive
  int total = 0;                    // primitive count
};

namespace cprrtc {
int api_fail(int code, const char* fmt, ...);
int api_hip_fail(hipError_t e, const char* what);
int api_constraint(const cp_constraint* c, const cp_robot* robot, ConDev* out);
int api_params(const cp_proj_params* params, cp_proj_params* p);
// The run-time compiled pooled kernel for this robot and constraint, if one
// was made (nullptr otherwise).
// Copies (under the robot's lock) the kernels compiled for the constraint's
// kind and mask; false if there are none.
bool rtc_find(cp_robot* robot, const ConDev& con, RtcFns* out);
// The validation kernels of any entry of the robot (they depend on the robot only).
bool rtc_find_validate(cp_robot* robot, RtcFns* out);
hipError_t launch_rtc_validate(const RtcFns& k, const cp_robot* robot, const EnvDev& env, int W,
                               int n_motions, const float* xi, int* status,
                               unsigned long long* work, bool early, int batch,
                               hipStream_t stream);
hipError_t launch_rtc_pool(const RtcFns& k, const cp_robot* robot, const ConDev& con,
                           const ProjDev& prm, int n_motions, const float* q_from,
                           const float* q_to, float* xi, int* status, int* iters,
                           unsigned long long* work, hipStream_t stream);
hipError_t launch_rtc_plan_round(const RtcFns& k, const cp_robot* robot, const EnvDev& env,
                                 const ConDev& con, const ProjDev& prm, const PlanDev& pd,
                                 int sphere_batch, unsigned blocks, size_t lds,
                                 hipStream_t stream);
void rtc_release(cp_robot* robot);
// fk_cc_batch's check (collision flags only) with the kernel compiled for
// the robot (RtcFns::fkcc, sphere batch 4 or 8).
hipError_t launch_rtc_fk_cc(const RtcFns& k, const cp_robot* robot, const EnvDev& env, int n_cfg,
                            const float* q, uint8_t* collide, bool early, int batch,
                            hipStream_t stream);
// Learned warm start for the planners: CP_OK if the network fits the robot's
// DOF and constraint kind and has the fused shape (else the error, with its
// message set); corrections delta [n_segments][W-1][dof] of the straight
// segments q_from[i] -> q_to[i] ([n_segments][dof]) by the fused network.
int mlp_warm_check(const cp_mlp* mlp, int dof, int kind);
hipError_t mlp_warm_corrections(const cp_mlp* mlp, const cp_robot* robot, const ConDev& con, int W,
                                long n_segments, const float* q_from, const float* q_to,
                                float* delta, hipStream_t st);
}  // namespace cprrtc

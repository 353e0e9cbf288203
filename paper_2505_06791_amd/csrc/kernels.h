// Launch entry points of the gfx950 kernels (host side of kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.h"

namespace cprrtc {

bool dof_supported(int dof);

// Scene check of n_cfg configurations, one wavefront each with its lanes
// splitting the primitives: collide[i] = min_sd[i] <= 0, min_sd[i] as
// fk_cc's exact form (for a query's few endpoints).
hipError_t launch_config_sd(const RobotDev* rob, const float4* sph, const EnvDev& env, int n_cfg,
                            const float* q, uint8_t* collide, float* min_sd, hipStream_t stream);
hipError_t launch_fk_cc(const RobotDev* rob, const float4* sph, const EnvDev& env, int n_cfg,
                        const float* q, uint8_t* collide, float* min_sd, bool early, int batch,
                        hipStream_t stream);

// World centres of every robot sphere of every configuration, [n_cfg][S][3]
// in description order; map[s] = (position in sph, joint frame of sphere s).
hipError_t launch_sphere_xyz(const RobotDev* rob, const float4* sph, const int2* map, int n_spheres,
                             int n_cfg, const float* q, float* xyz, hipStream_t stream);

// Pooled projection: slots per wavefront, whether a launch of n motions uses
// it (pooled: 1 = always, 0 = never, -1 = by batch size), its grid size.
constexpr int kPoolSlots = 4;
bool use_pool(int n_motions, int pooled);
unsigned pool_blocks(int n_motions);

// pooled: 1 = several motions per wavefront, 0 = one motion per wavefront,
// -1 = by batch size.
hipError_t launch_project(int dof, const RobotDev* rob, const ConDev& con, const ProjDev& prm,
                          int n_motions, const float* q_from, const float* q_to, float* xi,
                          int* status, int* iters, unsigned long long* work, int pooled,
                          hipStream_t stream, bool* supported);

hipError_t launch_project_mode(int dof, int mode, const RobotDev* rob, const ConDev& con,
                               const ProjDev& prm, int n_motions, const float* q_from,
                               const float* q_to, const float* delta, float* xi, int* status,
                               int* iters, unsigned long long* work, int pooled,
                               hipStream_t stream, bool* supported);

// Self-collision of configurations (OR into collide, min into min_sd) and of
// motions' waypoints 1..W-1 (status 0 -> 2 on a hit).  pairs: n_entries
// records (s | t << 16, bits of (r_s + r_t)^2), n_entries a multiple of
// kSelfPad, and kSelfPad more past the end.  The checked pairs come in
// groups of kSelfPad / 16 records sharing their first sphere s, group g at
// entries (g / 16) kSelfPad + g % 16 + 16 u (u < kSelfPad / 16); records
// with (r_s + r_t)^2 = -1 fill groups and the list up, never hit and are
// left out of the minimum.
constexpr int kSelfPad = 32;
hipError_t launch_self_cc(const RobotDev* rob, const RobotDev& host, const float4* sph,
                          const int2* pairs, int n_entries, int n_cfg, const float* q,
                          uint8_t* collide, float* min_sd, bool early, hipStream_t stream);
hipError_t launch_self_cc_motions(const RobotDev* rob, const RobotDev& host, const float4* sph,
                                  const int2* pairs, int n_entries, int W, int n_motions,
                                  const float* xi, int* status, hipStream_t stream);

hipError_t launch_validate(const RobotDev* rob, const float4* sph, const EnvDev& env, int W,
                           int n_motions, const float* xi, int* status, unsigned long long* work,
                           bool early, bool cull, int batch, hipStream_t stream);

hipError_t launch_project_configs(int dof, const RobotDev* rob, const ConDev& con, int n,
                                  const float* q_in, float* q_out, int* status, float tol,
                                  int max_iters, float alpha, float lambda2, hipStream_t stream,
                                  bool* supported);

}  // namespace cprrtc

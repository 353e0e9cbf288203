// Library-internal definitions of the opaque C-ABI handles and the helpers
// the translation units of libcprrtc.so share.
#pragma once
#include <hip/hip_runtime.h>

#include "cprrtc.h"
#include "device.h"

struct cp_robot {
  cprrtc::RobotDev host;            // host copy (dispatch reads dof, chains, limits)
  cprrtc::RobotDev* dev = nullptr;  // device copy
  float4* spheres = nullptr;        // device spheres, grouped by link
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
}  // namespace cprrtc

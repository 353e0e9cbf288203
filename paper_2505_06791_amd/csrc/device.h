// Device-side data layouts and per-lane building blocks for gfx950.
//
// Layout choices (all float32 on the device):
//  * Robot and scene data are wave-uniform: every lane of a wavefront reads
//    the same joint row or primitive, so they live in plain global memory
//    behind const __restrict__ pointers and are fetched with scalar loads
//    into SGPRs, where VALU instructions take them as operands directly.
//  * Primitives are stored array-of-structs per type, padded to float4
//    multiples, so one primitive is one s_load_dwordx8/x16.
//  * Per-lane state (a configuration, a 3x4 frame, a sphere batch) is in
//    VGPRs; nothing per lane goes through LDS.
#pragma once
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#endif
#include <stdint.h>

namespace cprrtc {

constexpr int kMaxDof = 16;
constexpr int kMaxChains = 2;
constexpr int kMaxSpheres = 1024;

struct RobotDev {
  int dof;
  int n_chains;
  int chain_begin[kMaxChains + 1];   // joints of chain c: [chain_begin[c], chain_begin[c+1])
  int n_spheres;
  float base[kMaxChains][12];        // 3x4 row-major (rotation | translation)
  float tool[kMaxChains][12];
  float ca[kMaxDof];                 // cos(alpha_{i-1})
  float sa[kMaxDof];                 // sin(alpha_{i-1})
  float a[kMaxDof];
  float d0[kMaxDof];
  float th0[kMaxDof];
  float lo[kMaxDof];
  float hi[kMaxDof];
  int prismatic[kMaxDof];
  int short_angle[kMaxDof];          // revolute, angle (limits plus offset) within +-3.2 rad
                                     // (read by the kernels compiled for the robot)
  int sph_begin[kMaxDof + 1];        // spheres riding in joint frame j: [sph_begin[j], sph_begin[j+1])
};

// Culling margin (metres; far above float32 rounding of the box test).
constexpr float kCullMargin = 1e-4f;

struct EnvDev {
  int n_aabb, n_obb, n_sph, n_cap, n_cyl;
  const float4* aabb;  // 2 x float4: (centre, 0), (half extents, 0)
  const float4* obb;   // 4 x float4: (u.c, v.c, w.c, 0), (axis u, half_u), (axis v, half_v), (axis w, half_w)
  const float4* sph;   // 1 x float4: (centre, radius)
  const float4* cap;   // 2 x float4: (p0, radius), (p1 - p0, 1/|p1 - p0|^2 or 0)
  const float4* cyl;   // 2 x float4: (centre, half length), (unit axis, radius)
  const float4* bound; // 1 x float4 per primitive, types in the order above:
                       // bounding sphere for culling: (centre, (radius + margin)^2)
};

enum { KIND_NONE = 0, KIND_POSE = 1, KIND_REL = 2 };

struct ConDev {
  int kind;
  float mask[6];      // 1 locked / 0 free: x y z roll pitch yaw
  float Rt[9];        // POSE: Rc^T; REL: R*^T (row-major)
  float pc[3];        // POSE: constraint frame origin
  float target[6];    // POSE: locked values; REL: p* then zeros
};

struct ProjDev {
  int W;
  int max_iters;
  float tau, tau_sm, tau_task, alpha, lambda2;
  int variant;        // CP_PROJECT_PARALLEL / _INDEPENDENT / _SEQUENTIAL
};

// ------------------------------------------------------------------ frames

struct Frame {
  float r[9];   // rotation, row-major: column c is (r[c], r[3+c], r[6+c])
  float p[3];
};

__device__ __forceinline__ void frame_from(Frame& T, const float* __restrict__ m) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    T.r[3 * i + 0] = m[4 * i + 0];
    T.r[3 * i + 1] = m[4 * i + 1];
    T.r[3 * i + 2] = m[4 * i + 2];
    T.p[i] = m[4 * i + 3];
  }
}

// T <- T * RotX(alpha) * TransX(a) * RotZ(theta) * TransZ(d), done as column
// operations on T: the twist mixes columns 1 and 2, the offset a moves along
// column 0, the joint angle mixes columns 0 and 1, d moves along column 2.
__device__ __forceinline__ void frame_advance(Frame& T, float ca, float sa, float a, float ct,
                                              float st, float d) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const float c1 = T.r[3 * i + 1], c2 = T.r[3 * i + 2];
    T.r[3 * i + 1] = ca * c1 + sa * c2;
    T.r[3 * i + 2] = ca * c2 - sa * c1;
    T.p[i] += a * T.r[3 * i + 0];
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const float c0 = T.r[3 * i + 0], c1 = T.r[3 * i + 1];
    T.r[3 * i + 0] = ct * c0 + st * c1;
    T.r[3 * i + 1] = ct * c1 - st * c0;
    T.p[i] += d * T.r[3 * i + 2];
  }
}

// sin and cos of a joint angle (|x| up to a few turns): x = k pi/2 + r with
// |r| <= pi/4 by a two-constant Cody-Waite reduction (pi/2 split into a float
// and its remainder), then the Taylor polynomials of sin r to r^9 and cos r
// to r^10, whose truncation error on |r| <= pi/4 is below 2e-9; the quadrant
// k mod 4 swaps and negates the pair.  Absolute error about 6e-8 (one unit
// in the last place of 1), at roughly half the instructions of the general
// library routine, which also handles huge arguments.
__device__ __forceinline__ void sincos_joint(float x, float& s, float& c) {
  const float k = rintf(x * 0.636619772367581343f);
  float r = fmaf(-k, 1.57079637050628662109375f, x);
  r = fmaf(-k, -4.37113900018624283e-8f, r);
  const float r2 = r * r;
  float ps = fmaf(r2, 2.75573192e-6f, -1.98412698e-4f);   // 1/9!, -1/7!
  ps = fmaf(r2, ps, 8.33333333e-3f);                       // 1/5!
  ps = fmaf(r2, ps, -1.66666667e-1f);                      // -1/3!
  const float sr = fmaf(r * r2, ps, r);
  float pc = fmaf(r2, -2.75573192e-7f, 2.48015873e-5f);   // -1/10!, 1/8!
  pc = fmaf(r2, pc, -1.38888889e-3f);                      // -1/6!
  pc = fmaf(r2, pc, 4.16666667e-2f);                       // 1/4!
  pc = fmaf(r2, pc, -0.5f);                                // -1/2!
  const float cr = fmaf(r2, pc, 1.0f);
  const int q = (int)k;
  const float a = (q & 1) ? cr : sr;
  const float b = (q & 1) ? sr : cr;
  s = (q & 2) ? -a : a;
  c = ((q + 1) & 2) ? -b : b;
}

// sin and cos of a joint angle known to lie within [-3.2, 3.2] (a joint
// whose limits, plus its offset, keep it there) from the hardware sine and
// cosine (argument in revolutions): measured absolute error 3.5e-7 (sin) and
// 2.6e-7 (cos) over that range, at one multiply and two transcendental
// instructions.  Beyond a few turns the rounding of x / (2 pi) grows with
// |x|, so unbounded joints keep sincos_joint.
__device__ __forceinline__ void sincos_hw(float x, float& s, float& c) {
  const float r = x * 0.159154943091895336f;   // 1 / (2 pi)
  s = __builtin_amdgcn_sinf(r);
  c = __builtin_amdgcn_cosf(r);
}

// Where the projection reads the robot's constants and the constraint's
// locked axes: RobotMem reads the device copy of the robot and the
// constraint's mask at run time; a kernel compiled at run time for one robot
// and one mask (hipRTC) supplies a policy with the same functions returning
// compile-time constants, so unrolled loops fold them (zero twists and
// offsets vanish, prismatic tests and free-axis branches disappear).
struct RobotMem {
  static __device__ __forceinline__ float ca(const RobotDev* r, int j) { return r->ca[j]; }
  static __device__ __forceinline__ float sa(const RobotDev* r, int j) { return r->sa[j]; }
  static __device__ __forceinline__ float a(const RobotDev* r, int j) { return r->a[j]; }
  static __device__ __forceinline__ float d0(const RobotDev* r, int j) { return r->d0[j]; }
  static __device__ __forceinline__ float th0(const RobotDev* r, int j) { return r->th0[j]; }
  static __device__ __forceinline__ float lo(const RobotDev* r, int j) { return r->lo[j]; }
  static __device__ __forceinline__ float hi(const RobotDev* r, int j) { return r->hi[j]; }
  static __device__ __forceinline__ bool prismatic(const RobotDev* r, int j) { return r->prismatic[j] != 0; }
  // joint angle bounded by +-3.2 (sincos_hw applies); the library kernels
  // take the general routine for every joint, so that all of them (pooled
  // and one motion per wavefront alike) compute the same bits
  static __device__ __forceinline__ bool short_angle(const RobotDev*, int) { return false; }
  // first joint of chain 1 (ndof for a single chain)
  static __device__ __forceinline__ int chain1(const RobotDev* r, int ndof) {
    return r->n_chains > 1 ? r->chain_begin[1] : ndof;
  }
  static __device__ __forceinline__ float base(const RobotDev* r, int c, int i) { return r->base[c][i]; }
  static __device__ __forceinline__ float tool(const RobotDev* r, int c, int i) { return r->tool[c][i]; }
  static __device__ __forceinline__ bool lock(const ConDev& c, int i) { return c.mask[i] != 0.0f; }
  // collision spheres: chains, spheres riding in joint frame j, sphere s
  static __device__ __forceinline__ int n_chains(const RobotDev* r) { return r->n_chains; }
  static __device__ __forceinline__ int chain_begin(const RobotDev* r, int c) { return r->chain_begin[c]; }
  static __device__ __forceinline__ int sph_begin(const RobotDev* r, int j) { return r->sph_begin[j]; }
  static __device__ __forceinline__ float4 sphere(const float4* __restrict__ sph, int s) { return sph[s]; }
};

// T * tool_c of the policy.
template <class P>
__device__ __forceinline__ void frame_times_p(const Frame& T, const RobotDev* __restrict__ rob,
                                              int c, Frame& out) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int k = 0; k < 3; ++k)
      out.r[3 * i + k] = T.r[3 * i + 0] * P::tool(rob, c, k) + T.r[3 * i + 1] * P::tool(rob, c, 4 + k) +
                         T.r[3 * i + 2] * P::tool(rob, c, 8 + k);
    out.p[i] = T.r[3 * i + 0] * P::tool(rob, c, 3) + T.r[3 * i + 1] * P::tool(rob, c, 7) +
               T.r[3 * i + 2] * P::tool(rob, c, 11) + T.p[i];
  }
}

template <class P>
__device__ __forceinline__ void frame_from_p(Frame& T, const RobotDev* __restrict__ rob, int c,
                                             bool tool) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int k = 0; k < 3; ++k)
      T.r[3 * i + k] = tool ? P::tool(rob, c, 4 * i + k) : P::base(rob, c, 4 * i + k);
    T.p[i] = tool ? P::tool(rob, c, 4 * i + 3) : P::base(rob, c, 4 * i + 3);
  }
}

// Joint j of the robot at joint value qj.
template <class P = RobotMem>
__device__ __forceinline__ void joint_advance(Frame& T, const RobotDev* __restrict__ rob, int j,
                                              float qj) {
  const bool pri = P::prismatic(rob, j);
  const float theta = P::th0(rob, j) + (pri ? 0.0f : qj);
  const float d = P::d0(rob, j) + (pri ? qj : 0.0f);
  float st, ct;
  if (P::short_angle(rob, j))
    sincos_hw(theta, st, ct);
  else
    sincos_joint(theta, st, ct);
  frame_advance(T, P::ca(rob, j), P::sa(rob, j), P::a(rob, j), ct, st, d);
}

// Tool frame: T_ee = T * tool.
__device__ __forceinline__ void frame_times(const Frame& T, const float* __restrict__ m,
                                            Frame& out) {
  Frame B;
  frame_from(B, m);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
      out.r[3 * i + c] = T.r[3 * i + 0] * B.r[c] + T.r[3 * i + 1] * B.r[3 + c] +
                         T.r[3 * i + 2] * B.r[6 + c];
    out.p[i] = T.r[3 * i + 0] * B.p[0] + T.r[3 * i + 1] * B.p[1] + T.r[3 * i + 2] * B.p[2] +
               T.p[i];
  }
}

}  // namespace cprrtc

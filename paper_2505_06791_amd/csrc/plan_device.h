// Device code of one planner round (paper Section III), shared by the
// library's round kernels (plan.hip) and round kernels compiled at run time
// for one robot and constraint mask (rtc.hip): tree layout, Halton samples,
// nearest-node search, steering, one projected and validated motion,
// appends and the connect loop of one extension.
#pragma once
#include "collide.h"
#include "cprrtc.h"
#include "device.h"
#include "project.h"

namespace cprrtc {

constexpr int kPlanBlock = 256;
constexpr unsigned kPrimes[kMaxDof] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53};

struct PlanDev {
  float* q[2];          // [dof][cap] node configurations (structure of arrays)
  int* parent[2];       // [cap]
  float* edge[2];       // [cap][W][dof] dense edge from the parent to the node
  float* scratch;       // [n_groups][W][dof] segment under test
  int* ctl;             // control block, see kCtl*
  int cap;
  int n_groups;
  int max_connect;
  float step;           // steer length (W - 1) tau
  float connect2;       // (tau + tau_sm)^2
  float shift[kMaxDof]; // Cranley-Patterson shift per dimension
  unsigned sample_base; // Halton index of the round's first sample
  const int2* self_pairs; // self-collision pairs (positions in the sphere array)
  int n_self;           // checked pairs (used by the round kernels built with SELF)
};

// Dynamic LDS of a round kernel when extensions check self-collision:
// per wavefront, the sphere centres of one configuration (n_spheres float4)
// and that configuration's joint values (4 float4).
extern __shared__ float4 cp_plan_lds[];
__host__ __device__ inline size_t plan_lds_bytes(int n_spheres) {
  return sizeof(float4) * (size_t)(kPlanBlock / 64) * (size_t)(n_spheres + 4);
}

// control block layout (ints)
enum { kCtlCount = 0, kCtlPublished = 2, kCtlDone = 4, kCtlConn = 5, kCtlOverflow = 8, kCtlInts = 16 };

// Radical inverse of i in base b (Halton coordinate).
__device__ __forceinline__ float radical_inverse(unsigned i, unsigned b) {
  const float inv = 1.0f / (float)b;
  float f = inv, r = 0.0f;
  while (i) {
    const unsigned d = i % b;
    r += (float)d * f;
    i /= b;
    f *= inv;
  }
  return r;
}

// Nearest published node (squared L2 in joint space, ties to the lowest
// index): lanes scan nodes 64 apart, then a wavefront argmin.
template <int NDOF>
__device__ __forceinline__ int nearest_node(const float* __restrict__ qs, int n, int cap,
                                            const float (&x)[NDOF], float& best_d2) {
  const int lane = threadIdx.x & 63;
  float best = FLT_MAX;
  int bi = 0x7fffffff;
  for (int i = lane; i < n; i += 64) {
    float d = 0.0f;
#pragma unroll
    for (int j = 0; j < NDOF; ++j) {
      const float t = qs[j * cap + i] - x[j];
      d += t * t;
    }
    if (d < best) {
      best = d;
      bi = i;
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const float ob = __shfl_xor(best, o, 64);
    const int oi = __shfl_xor(bi, o, 64);
    if (ob < best || (ob == best && oi < bi)) {
      best = ob;
      bi = oi;
    }
  }
  best_d2 = best;
  return bi;
}

template <int NDOF>
__device__ __forceinline__ float dist2(const float (&a)[NDOF], const float (&b)[NDOF]) {
  float d = 0.0f;
#pragma unroll
  for (int j = 0; j < NDOF; ++j) {
    const float t = a[j] - b[j];
    d += t * t;
  }
  return d;
}

// q_steer = a + min(1, step / |b - a|) (b - a)
template <int NDOF>
__device__ __forceinline__ void steer(const float (&a)[NDOF], const float (&b)[NDOF], float step,
                                      float (&out)[NDOF]) {
  const float d = sqrtf(dist2<NDOF>(a, b));
  const float s = d > step ? step / d : 1.0f;
#pragma unroll
  for (int j = 0; j < NDOF; ++j) out[j] = a[j] + s * (b[j] - a[j]);
}

// Self-collision of one configuration (joint values qq in LDS, read by
// every lane) by the whole wavefront: the lanes place the sphere centres in
// `cent`, then test the checked pairs 64 at a time (colliding iff
// |c_s - c_t| - r_s - r_t <= 0).  Uniform result.
template <class P>
__device__ __forceinline__ bool self_collides(const RobotDev* __restrict__ rob,
                                              const float4* __restrict__ sph, const float* qq,
                                              const int2* __restrict__ pairs, int n_pairs,
                                              float4* cent) {
  const int lane = threadIdx.x & 63;
  for (int c = 0; c < P::n_chains(rob); ++c) {
    Frame T;
    frame_from_p<P>(T, rob, c, false);
    for (int j = P::chain_begin(rob, c); j < P::chain_begin(rob, c + 1); ++j) {
      joint_advance<P>(T, rob, j, qq[j]);
      for (int s = P::sph_begin(rob, j) + lane; s < P::sph_begin(rob, j + 1); s += 64) {
        const float4 l = P::sphere(sph, s);
        cent[s] = make_float4(T.r[0] * l.x + T.r[1] * l.y + T.r[2] * l.z + T.p[0],
                              T.r[3] * l.x + T.r[4] * l.y + T.r[5] * l.z + T.p[1],
                              T.r[6] * l.x + T.r[7] * l.y + T.r[8] * l.z + T.p[2], l.w);
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");   // centres of other lanes
  __builtin_amdgcn_wave_barrier();
  bool hit = false;
  for (int base = 0; base < n_pairs && !hit; base += 64) {
    const int p = base + lane;
    bool h = false;
    if (p < n_pairs) {
      const int2 st = pairs[p];
      const float4 a = cent[st.x], b = cent[st.y];
      const float dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z, reach = a.w + b.w;
      h = dx * dx + dy * dy + dz * dz <= reach * reach;   // |c_s - c_t| <= r_s + r_t
    }
    hit = __ballot(h) != 0;
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");   // reads before the next writes
  __builtin_amdgcn_wave_barrier();
  return hit;
}

// One motion a -> b on this wavefront (lanes 0..W-1), projected and
// validated (with n_self > 0 also against the robot itself).  q: this
// lane's projected waypoint; end: xi[W-1] broadcast.
// delta (nullable): the learned warm start's corrections of waypoints
// 1..W-1 ([W-1][NDOF]); the segment is first projected from the corrected
// waypoints and, if that fails, again from the straight line.
template <int NDOF, int KIND, int B, class P = RobotMem, bool SELF = false>
__device__ __forceinline__ bool try_motion(const RobotDev* __restrict__ rob, const float4* __restrict__ sph,
                           const EnvDev& env, const ConDev& con, const ProjDev& prm,
                           float* __restrict__ scratch, const int2* __restrict__ self_pairs,
                           int n_self, const float (&a)[NDOF],
                           const float (&b)[NDOF], float (&q)[NDOF], float (&end)[NDOF],
                           const float* __restrict__ delta = nullptr) {
  const int W = prm.W;
  const int lane = threadIdx.x & 63;
  const int k = lane % W;
  const int seg = lane - k;
  const bool in_motion = lane < W;
  const uint64_t wmask = (W == 64) ? ~0ull : ((1ull << W) - 1ull);
  const uint64_t segmask = wmask << seg;
  const float s = (float)k / (float)(W - 1);
  int iters = 0;
  unsigned long long updates = 0;
  bool ok = false;
  if (delta != nullptr) {
#pragma unroll
    for (int j = 0; j < NDOF; ++j) {
      q[j] = a[j] + s * (b[j] - a[j]);
      if (in_motion && k >= 1)
        q[j] = fminf(fmaxf(q[j] + delta[(k - 1) * NDOF + j], P::lo(rob, j)), P::hi(rob, j));
    }
    ok = project_segment<NDOF, KIND, P>(rob, con, prm, k, seg, wmask, segmask, !in_motion, q,
                                        iters, updates);
    ok = __shfl(ok ? 1 : 0, 0, 64) != 0;
  }
  if (!ok) {
#pragma unroll
    for (int j = 0; j < NDOF; ++j) q[j] = a[j] + s * (b[j] - a[j]);
    ok = prm.variant == CP_PROJECT_SEQUENTIAL
             ? project_sequential<NDOF, KIND>(rob, con, prm, k, seg, !in_motion, q, iters, updates)
             : project_segment<NDOF, KIND, P>(rob, con, prm, k, seg, wmask, segmask, !in_motion, q,
                                              iters, updates);
  }
  if (!__shfl(ok ? 1 : 0, 0, 64)) return false;
  float* xk = scratch + (size_t)(in_motion ? lane : 0) * NDOF;
  if (in_motion) {
#pragma unroll
    for (int j = 0; j < NDOF; ++j) xk[j] = q[j];
  }
  uint64_t hits;
  float msd;
  CcWork cw;
  cc_work_clear(cw);
  collide_config<B, false, true, true, P>(rob, sph, env, xk, in_motion && k >= 1, segmask, true, hits,
                                       msd, cw);
  const uint64_t all_hits = __ballot((hits & segmask) != 0 && in_motion);
  if (all_hits) return false;
  if (SELF && n_self > 0) {
    // waypoints 1..W-1 against the robot itself, one configuration at a
    // time by the whole wavefront
    float4* cent = cp_plan_lds + (size_t)(threadIdx.x >> 6) * (rob->n_spheres + 4);
    float* qq = reinterpret_cast<float*>(cent + rob->n_spheres);
    for (int kk = 1; kk < W; ++kk) {
      if (lane == 0) {
#pragma unroll
        for (int j = 0; j < NDOF; ++j)
          qq[j] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, q[j]), kk));
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      if (self_collides<P>(rob, sph, qq, self_pairs, n_self, cent)) return false;
    }
  }
#pragma unroll
  for (int j = 0; j < NDOF; ++j) end[j] = __shfl(q[j], W - 1, 64);
  return true;
}

// Append the projected segment held in the lanes' q as a new node of tree t
// with the given parent.  Returns the slot, or -1 if the tree is full.
template <int NDOF>
__device__ __forceinline__ int append_node(const PlanDev& pd, int W, int t, int parent, const float (&q)[NDOF]) {
  const int lane = threadIdx.x & 63;
  int slot = 0;
  if (lane == 0) slot = atomicAdd(&pd.ctl[kCtlCount + t], 1);
  slot = __shfl(slot, 0, 64);
  if (slot >= pd.cap) {
    if (lane == 0) atomicExch(&pd.ctl[kCtlOverflow], 1);
    return -1;
  }
  if (lane < W) {
    float* e = pd.edge[t] + ((size_t)slot * W + lane) * NDOF;
#pragma unroll
    for (int j = 0; j < NDOF; ++j) e[j] = q[j];
  }
  if (lane == W - 1) {
#pragma unroll
    for (int j = 0; j < NDOF; ++j) pd.q[t][(size_t)j * pd.cap + slot] = q[j];
    pd.parent[t][slot] = parent;
  }
  return slot;
}

template <int NDOF>
__device__ __forceinline__ void load_node(const PlanDev& pd, int t, int i, float (&out)[NDOF]) {
#pragma unroll
  for (int j = 0; j < NDOF; ++j) out[j] = pd.q[t][(size_t)j * pd.cap + i];
}

__device__ __forceinline__ bool plan_done(const PlanDev& pd) {
  return __atomic_load_n(&pd.ctl[kCtlDone], __ATOMIC_RELAXED) != 0;
}

// The extension's sample (Halton point of group g, tree g & 1), its
// nearest published node and the steered end: q_near = node `near`, q_steer.
template <int NDOF, class P = RobotMem>
__device__ __forceinline__ int plan_sample(const RobotDev* __restrict__ rob, const PlanDev& pd,
                                           unsigned sample_base, int g, float (&qn)[NDOF],
                                           float (&qs)[NDOF]) {
  const int lane = threadIdx.x & 63;
  const int X = g & 1;                          // half the wavefronts grow each tree
  const int pubX = pd.ctl[kCtlPublished + X];
  // Halton sample: lane j computes coordinate j, then every lane takes all.
  float u = 0.0f;
  if (lane < NDOF) {
    u = radical_inverse(sample_base + (unsigned)g + 1u, kPrimes[lane]) + pd.shift[lane];
    u -= floorf(u);
  }
  float qr[NDOF];
#pragma unroll
  for (int j = 0; j < NDOF; ++j) qr[j] = P::lo(rob, j) + __shfl(u, j, 64) * (P::hi(rob, j) - P::lo(rob, j));
  float d2;
  const int near = nearest_node<NDOF>(pd.q[X], pubX, pd.cap, qr, d2);
  load_node<NDOF>(pd, X, near, qn);
  steer<NDOF>(qn, qr, pd.step, qs);
  return near;
}

// The rest of an extension after its sample: the motion q_near -> q_steer
// (warm-started when delta, [W-1][NDOF], is given), its append, then the
// connect loop towards the nearest node of the other tree (plain projection).
template <int NDOF, int KIND, int B, class P = RobotMem, bool SELF = false>
__device__ __forceinline__ void plan_extend_from(const RobotDev* __restrict__ rob, const float4* __restrict__ sph,
                            const EnvDev& env, const ConDev& con, const ProjDev& prm,
                            const PlanDev& pd, int g, int near, const float (&qn)[NDOF],
                            const float (&qs0)[NDOF], const float* __restrict__ delta) {
  const int lane = threadIdx.x & 63;
  const int W = prm.W;
  const int X = g & 1, Y = X ^ 1;
  const int pubY = pd.ctl[kCtlPublished + Y];
  float* scratch = pd.scratch + (size_t)g * W * NDOF;
  float qs[NDOF], q[NDOF], qe[NDOF], d2;
  if (!try_motion<NDOF, KIND, B, P, SELF>(rob, sph, env, con, prm, scratch, pd.self_pairs, pd.n_self, qn,
                                    qs0, q, qe, delta)) return;
  int cur = append_node<NDOF>(pd, W, X, near, q);
  if (cur < 0) return;

  // extend the same tree towards the nearest node of the other tree
  float qt[NDOF];
  const int tgt = nearest_node<NDOF>(pd.q[Y], pubY, pd.cap, qe, d2);
  load_node<NDOF>(pd, Y, tgt, qt);
  float dcur = dist2<NDOF>(qe, qt);
  for (int c = 0;; ++c) {
    if (dcur < pd.connect2) {
      if (lane == 0 && atomicCAS(&pd.ctl[kCtlDone], 0, 1) == 0) {
        pd.ctl[kCtlConn + 0] = X;
        pd.ctl[kCtlConn + 1] = cur;
        pd.ctl[kCtlConn + 2] = tgt;
      }
      return;
    }
    if (c >= pd.max_connect) return;
    if (__shfl(plan_done(pd) ? 1 : 0, 0, 64)) return;
    steer<NDOF>(qe, qt, pd.step, qs);
    float qe2[NDOF];
    if (!try_motion<NDOF, KIND, B, P, SELF>(rob, sph, env, con, prm, scratch, pd.self_pairs, pd.n_self, qe,
                                      qs, q, qe2)) return;
    const float dnew = dist2<NDOF>(qe2, qt);
    if (!(dnew < dcur)) return;                  // no progress: stop extending
    cur = append_node<NDOF>(pd, W, X, cur, q);
    if (cur < 0) return;
#pragma unroll
    for (int j = 0; j < NDOF; ++j) qe[j] = qe2[j];
    dcur = dnew;
  }
}


// One tree extension of one wavefront (group g of the round): sample, grow
// the group's tree by one motion, then towards the other tree.
template <int NDOF, int KIND, int B, class P = RobotMem, bool SELF = false>
__device__ __forceinline__ void plan_extend(const RobotDev* __restrict__ rob, const float4* __restrict__ sph,
                            const EnvDev& env, const ConDev& con, const ProjDev& prm,
                            const PlanDev& pd, unsigned sample_base, int g) {
  if (__shfl(plan_done(pd) ? 1 : 0, 0, 64)) return;
  float qn[NDOF], qs[NDOF];
  const int near = plan_sample<NDOF, P>(rob, pd, sample_base, g, qn, qs);
  plan_extend_from<NDOF, KIND, B, P, SELF>(rob, sph, env, con, prm, pd, g, near, qn, qs, nullptr);
}

// Warm-started rounds, first half: the sample of group g (its nearest node
// and steered end) written for the network; near = -1 when the plan is done.
template <int NDOF>
__device__ __forceinline__ void write_sample(const RobotDev* __restrict__ rob, const PlanDev& pd,
                                             unsigned sample_base, int g, float* __restrict__ from,
                                             float* __restrict__ to, int* __restrict__ near_out) {
  const int lane = threadIdx.x & 63;
  float qn[NDOF], qs[NDOF];
  int near = -1;
  if (!__shfl(plan_done(pd) ? 1 : 0, 0, 64)) {
    near = plan_sample<NDOF>(rob, pd, sample_base, g, qn, qs);
  } else {
#pragma unroll
    for (int j = 0; j < NDOF; ++j) qn[j] = qs[j] = 0.0f;
  }
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < NDOF; ++j) {
      from[j] = qn[j];
      to[j] = qs[j];
    }
    *near_out = near;
  }
}

// Warm-started rounds, second half: the extension from the recorded sample,
// its first motion corrected by delta ([W-1][NDOF]).
template <int NDOF, int KIND, int B>
__device__ __forceinline__ void extend_from_sample(const RobotDev* __restrict__ rob,
                                                   const float4* __restrict__ sph, const EnvDev& env,
                                                   const ConDev& con, const ProjDev& prm,
                                                   const PlanDev& pd, int g,
                                                   const float* __restrict__ from,
                                                   const float* __restrict__ to, int near,
                                                   const float* __restrict__ delta) {
  if (near < 0 || __shfl(plan_done(pd) ? 1 : 0, 0, 64)) return;
  float qn[NDOF], qs[NDOF];
#pragma unroll
  for (int j = 0; j < NDOF; ++j) {
    qn[j] = from[j];
    qs[j] = to[j];
  }
  plan_extend_from<NDOF, KIND, B>(rob, sph, env, con, prm, pd, g, near, qn, qs, delta);
}

}  // namespace cprrtc

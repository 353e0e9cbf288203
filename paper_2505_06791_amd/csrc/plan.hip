// plan(): constrained bidirectional RRT-Connect on one GPU (paper Section III).
//
// Two trees (rooted at start and goal) live in HBM.  The planner runs in
// rounds; a round is one launch of plan_round_kernel with n_groups
// wavefronts, each one tree extension as the paper describes it for one
// thread block:
//   sample q_rand (Halton, shifted by the seed) -> nearest node q_near of its
//   tree -> steer to q_steer at most (W-1) tau away -> W straight-line
//   waypoints -> ParallelProject -> FK + CC with early exit -> if valid,
//   append q_end with parent q_near and the dense edge; then extend the same
//   tree from q_end towards the nearest node of the other tree while each
//   projected, collision-free segment strictly reduces the distance to it.
// The trees are connected when an end comes within tau + tau_sm of that node.
//
// Concurrency: searches read only the nodes published before the round
// (published[t]); appends reserve slots with an atomic counter and write the
// node, its parent and its edge; a one-thread kernel publishes the counters
// after the round.  So no search reads a node that is being written.  The
// first wavefront to connect sets `done` by compare-and-swap and records the
// connection; wavefronts that see `done` leave.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "collide.h"
#include "cprrtc.h"
#include "device.h"
#include "handles.h"
#include "kernels.h"
#include "plan_device.h"
#include "project.h"

namespace cprrtc {

// SELF: extensions also check their waypoints against the robot itself
// (a separate instantiation, so that the plain kernels keep their registers).
template <int NDOF, int KIND, int B, bool SELF>
__global__ __launch_bounds__(kPlanBlock) void plan_round_kernel(const RobotDev* __restrict__ rob,
                                                                const float4* __restrict__ sph,
                                                                EnvDev env, ConDev con,
                                                                ProjDev prm, PlanDev pd) {
  const int g = (int)((blockIdx.x * kPlanBlock + threadIdx.x) >> 6);
  if (g >= pd.n_groups) return;                  // wavefront-uniform
  plan_extend<NDOF, KIND, B, RobotMem, SELF>(rob, sph, env, con, prm, pd, pd.sample_base, g);
}

// Warm-started rounds: the first motion of every extension starts from
// waypoints corrected by the learned network.  A round is three launches:
// the samples (nearest node, steered end) into seg_from / seg_to / seg_near,
// the network on those segments (delta [G][W-1][NDOF]), then the extensions
// from there.  A group whose plan is already done records near = -1.
template <int NDOF>
__global__ __launch_bounds__(kPlanBlock) void plan_sample_kernel(const RobotDev* __restrict__ rob,
                                                                 PlanDev pd, float* __restrict__ seg_from,
                                                                 float* __restrict__ seg_to,
                                                                 int* __restrict__ seg_near) {
  const int g = (int)((blockIdx.x * kPlanBlock + threadIdx.x) >> 6);
  if (g >= pd.n_groups) return;                  // wavefront-uniform
  write_sample<NDOF>(rob, pd, pd.sample_base, g, seg_from + (size_t)g * NDOF,
                     seg_to + (size_t)g * NDOF, seg_near + g);
}

template <int NDOF, int KIND, int B>
__global__ __launch_bounds__(kPlanBlock) void plan_round_warm_kernel(
    const RobotDev* __restrict__ rob, const float4* __restrict__ sph, EnvDev env, ConDev con,
    ProjDev prm, PlanDev pd, const float* __restrict__ seg_from, const float* __restrict__ seg_to,
    const int* __restrict__ seg_near, const float* __restrict__ delta) {
  const int g = (int)((blockIdx.x * kPlanBlock + threadIdx.x) >> 6);
  if (g >= pd.n_groups) return;                  // wavefront-uniform
  extend_from_sample<NDOF, KIND, B>(rob, sph, env, con, prm, pd, g, seg_from + (size_t)g * NDOF,
                                    seg_to + (size_t)g * NDOF, seg_near[g],
                                    delta + (size_t)g * (prm.W - 1) * NDOF);
}

// Roots (start in tree 0, goal in tree 1) and counters of a fresh plan.
__global__ void plan_init_kernel(PlanDev pd, const float* __restrict__ ends, int dof) {
  const int t = threadIdx.x;
  if (t < 2) {
    for (int j = 0; j < dof; ++j) pd.q[t][(size_t)j * pd.cap] = ends[t * dof + j];
    pd.parent[t][0] = -1;
  }
  if (t < kCtlInts) pd.ctl[t] = (t == kCtlCount || t == kCtlCount + 1 || t == kCtlPublished ||
                                  t == kCtlPublished + 1) ? 1 : 0;
}

__global__ void publish_kernel(int* ctl, int cap) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctl[kCtlPublished + 0] = min(ctl[kCtlCount + 0], cap);
    ctl[kCtlPublished + 1] = min(ctl[kCtlCount + 1], cap);
  }
}

// The path of a connected planner, assembled on the device: thread 0 walks
// both trees' parent links from the connection (tree-0 chain n0 -> root into
// items[0..], tree-1 chain n1 -> root into items[cap..]) and writes
// hdr = {path rows, chain lengths}; then the block copies, into out (rows
// of dof floats), the tree-0 edges from the root to n0 (points 1..W-1 of
// each), n1's configuration, and the tree-1 edges from n1 back to its root
// (each reversed, points W-2..0).  Rows 0 and len-1 are the caller's own
// end points and are left to the host.  Nothing is copied when the path
// would not fit max_rows.
__global__ void path_walk_kernel(PlanDev pd, int n0, int n1, int W, int dof, int* __restrict__ items,
                                 int* __restrict__ hdr, float* __restrict__ out, long max_rows) {
  __shared__ int c0s, c1s;
  if (threadIdx.x == 0) {
    int c0 = 0, c1 = 0;
    for (int v = n0; v > 0 && c0 < pd.cap; v = pd.parent[0][v]) items[c0++] = v;
    for (int v = n1; v > 0 && c1 < pd.cap; v = pd.parent[1][v]) items[pd.cap + c1++] = v;
    c0s = c0;
    c1s = c1;
    hdr[0] = 1 + c0 * (W - 1) + 1 + c1 * (W - 1);
    hdr[1] = c0;
    hdr[2] = c1;
  }
  __syncthreads();
  const int c0 = c0s, c1 = c1s, seg = (W - 1) * dof;
  if ((long)1 + (long)(c0 + c1) * (W - 1) + 1 > max_rows) return;
  // tree-0 edges, root first
  for (long t = threadIdx.x; t < (long)c0 * seg; t += blockDim.x) {
    const int k = (int)(t / seg), r = (int)(t % seg), p = r / dof, j = r % dof;
    const int node = items[c0 - 1 - k];
    out[(size_t)(1 + k * (W - 1) + p) * dof + j] = pd.edge[0][((size_t)node * W + p + 1) * dof + j];
  }
  const int mid = 1 + c0 * (W - 1);
  for (int j = threadIdx.x; j < dof; j += blockDim.x) out[(size_t)mid * dof + j] = pd.q[1][(size_t)j * pd.cap + n1];
  // tree-1 edges from n1 back to the root, each reversed
  for (long t = threadIdx.x; t < (long)c1 * seg; t += blockDim.x) {
    const int k = (int)(t / seg), r = (int)(t % seg), p = r / dof, j = r % dof;
    const int node = items[pd.cap + k];
    out[(size_t)(mid + 1 + k * (W - 1) + p) * dof + j] = pd.edge[1][((size_t)node * W + W - 2 - p) * dof + j];
  }
}

// ------------------------------------------------------------------ batched planning

constexpr int kHostIoFloats = 64;       // pinned staging of a planner (endpoints, checks, header)
constexpr int kPathPrefixRows = 4096;   // path rows fetched with the header

// One planning query of a batch: its robot, scene, constraint and trees.
struct ProblemDev {
  const RobotDev* rob;
  const float4* sph;
  EnvDev env;
  ConDev con;
  PlanDev pd;
  int dof;
};

// One round for the queries of one (DOF, constraint kind) class of the
// batch: wavefront w works for query w / groups of the class as group
// w % groups.  The round number comes from the device (advanced by the
// publish kernel), so a captured sequence of rounds can be replayed.
template <int NDOF, int KIND, int B>
__global__ __launch_bounds__(kPlanBlock) void plan_batch_round_kernel(
    const ProblemDev* __restrict__ probs, int n_probs, int groups, ProjDev prm,
    const unsigned* __restrict__ round) {
  // the wavefront index is uniform: keep it in a scalar register so the
  // problem descriptor is read with scalar loads
  const int w = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * kPlanBlock + threadIdx.x) >> 6));
  const int qi = w / groups, g = w % groups;
  if (qi >= n_probs) return;                     // wavefront-uniform
  const ProblemDev& P = probs[qi];
  plan_extend<NDOF, KIND, B>(P.rob, P.sph, P.env, P.con, prm, P.pd, *round * (unsigned)groups, g);
}

// Warm-started batch rounds (every query of one class): samples of
// wavefront w = query w / groups, group w % groups into segment w.
template <int NDOF>
__global__ __launch_bounds__(kPlanBlock) void plan_batch_sample_kernel(
    const ProblemDev* __restrict__ probs, int n_probs, int groups, const unsigned* __restrict__ round,
    float* __restrict__ seg_from, float* __restrict__ seg_to, int* __restrict__ seg_near) {
  const int w = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * kPlanBlock + threadIdx.x) >> 6));
  const int qi = w / groups, g = w % groups;
  if (qi >= n_probs) return;                     // wavefront-uniform
  const ProblemDev& P = probs[qi];
  write_sample<NDOF>(P.rob, P.pd, *round * (unsigned)groups, g, seg_from + (size_t)w * NDOF,
                     seg_to + (size_t)w * NDOF, seg_near + w);
}

template <int NDOF, int KIND, int B>
__global__ __launch_bounds__(kPlanBlock) void plan_batch_warm_kernel(
    const ProblemDev* __restrict__ probs, int n_probs, int groups, ProjDev prm,
    const float* __restrict__ seg_from, const float* __restrict__ seg_to,
    const int* __restrict__ seg_near, const float* __restrict__ delta) {
  const int w = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * kPlanBlock + threadIdx.x) >> 6));
  const int qi = w / groups, g = w % groups;
  if (qi >= n_probs) return;                     // wavefront-uniform
  const ProblemDev& P = probs[qi];
  extend_from_sample<NDOF, KIND, B>(P.rob, P.sph, P.env, P.con, prm, P.pd, g,
                                    seg_from + (size_t)w * NDOF, seg_to + (size_t)w * NDOF,
                                    seg_near[w], delta + (size_t)w * (prm.W - 1) * NDOF);
}

template <int NDOF, int KIND>
static void launch_batch_class(int batch, unsigned nb, hipStream_t st, const ProblemDev* probs,
                               int n, int groups, const ProjDev& prm, const unsigned* round) {
  if (batch == 4)
    plan_batch_round_kernel<NDOF, KIND, 4><<<nb, kPlanBlock, 0, st>>>(probs, n, groups, prm, round);
  else
    plan_batch_round_kernel<NDOF, KIND, 8><<<nb, kPlanBlock, 0, st>>>(probs, n, groups, prm, round);
}

static bool launch_batch_round(int dof, int kind, int batch, unsigned nb, hipStream_t st,
                               const ProblemDev* probs, int n, int groups, const ProjDev& prm,
                               const unsigned* round) {
  switch (dof * 4 + kind) {
    case 6 * 4 + KIND_NONE: launch_batch_class<6, KIND_NONE>(batch, nb, st, probs, n, groups, prm, round); return true;
    case 6 * 4 + KIND_POSE: launch_batch_class<6, KIND_POSE>(batch, nb, st, probs, n, groups, prm, round); return true;
    case 7 * 4 + KIND_NONE: launch_batch_class<7, KIND_NONE>(batch, nb, st, probs, n, groups, prm, round); return true;
    case 7 * 4 + KIND_POSE: launch_batch_class<7, KIND_POSE>(batch, nb, st, probs, n, groups, prm, round); return true;
    case 9 * 4 + KIND_NONE: launch_batch_class<9, KIND_NONE>(batch, nb, st, probs, n, groups, prm, round); return true;
    case 9 * 4 + KIND_POSE: launch_batch_class<9, KIND_POSE>(batch, nb, st, probs, n, groups, prm, round); return true;
    case 14 * 4 + KIND_POSE: launch_batch_class<14, KIND_POSE>(batch, nb, st, probs, n, groups, prm, round); return true;
    case 14 * 4 + KIND_REL: launch_batch_class<14, KIND_REL>(batch, nb, st, probs, n, groups, prm, round); return true;
    default: return false;
  }
}

// One round of a batch in one launch: every wavefront takes (query, group)
// tasks from a device counter until none is left and runs the extension
// with the code of the query's (DOF, constraint kind) class (branch uniform
// per wavefront); the last wavefront to finish publishes every query's new
// nodes, advances the round and resets the counters for the next round.
// Class sets: 0 = DOF 6, 7, 9 without or with a pose constraint; 1 = DOF 14
// with a pose or relative-pose constraint.  queue[0]: next task,
// queue[1]: wavefronts finished (both zero when a round starts).
template <int SET, int B>
__global__ __launch_bounds__(kPlanBlock, SET == 0 ? 2 : 1) void plan_batch_queue_kernel(
    ProblemDev* __restrict__ probs, int n_probs, int groups, ProjDev prm,
    unsigned* __restrict__ round, unsigned* __restrict__ queue, unsigned n_waves) {
  const int lane = threadIdx.x & 63;
  const unsigned r = __builtin_amdgcn_readfirstlane(*round);
  const unsigned total = (unsigned)n_probs * (unsigned)groups;
  while (true) {
    unsigned t = 0;
    if (lane == 0) t = atomicAdd(&queue[0], 1u);
    t = __builtin_amdgcn_readfirstlane(t);
    if (t >= total) break;
    const int qi = (int)(t / (unsigned)groups), g = (int)(t % (unsigned)groups);
    const ProblemDev& P = probs[qi];
    const unsigned base = r * (unsigned)groups;
#define CP_QUEUE_CASE(ND, K)                                                   \
  case ND * 4 + K:                                                             \
    plan_extend<ND, K, B>(P.rob, P.sph, P.env, P.con, prm, P.pd, base, g);   \
    break;
    if constexpr (SET == 0) {
      switch (P.dof * 4 + P.con.kind) {
        CP_QUEUE_CASE(6, KIND_NONE)
        CP_QUEUE_CASE(6, KIND_POSE)
        CP_QUEUE_CASE(7, KIND_NONE)
        CP_QUEUE_CASE(7, KIND_POSE)
        CP_QUEUE_CASE(9, KIND_NONE)
        CP_QUEUE_CASE(9, KIND_POSE)
        default: break;
      }
    } else {
      switch (P.dof * 4 + P.con.kind) {
        CP_QUEUE_CASE(14, KIND_POSE)
        CP_QUEUE_CASE(14, KIND_REL)
        default: break;
      }
    }
#undef CP_QUEUE_CASE
  }
  // the last wavefront out publishes (all appends of the round are done)
  __threadfence();
  unsigned fin = 0;
  if (lane == 0) fin = atomicAdd(&queue[1], 1u);
  fin = __builtin_amdgcn_readfirstlane(fin);
  if (fin == n_waves - 1) {
    __threadfence();
    for (int i = lane; i < n_probs; i += 64) {
      int* ctl = probs[i].pd.ctl;
      const int cap = probs[i].pd.cap;
      ctl[kCtlPublished + 0] = min(atomicAdd(&ctl[kCtlCount + 0], 0), cap);
      ctl[kCtlPublished + 1] = min(atomicAdd(&ctl[kCtlCount + 1], 0), cap);
    }
    if (lane == 0) {
      *round = r + 1u;
      queue[0] = 0u;
      queue[1] = 0u;
    }
  }
}

template <int NDOF, int KIND>
static void launch_batch_warm_class(int batch, unsigned nb, hipStream_t st, const ProblemDev* probs,
                                    int n, int groups, const ProjDev& prm, const float* f,
                                    const float* t, const int* nr, const float* delta) {
  if (batch == 4)
    plan_batch_warm_kernel<NDOF, KIND, 4><<<nb, kPlanBlock, 0, st>>>(probs, n, groups, prm, f, t, nr, delta);
  else
    plan_batch_warm_kernel<NDOF, KIND, 8><<<nb, kPlanBlock, 0, st>>>(probs, n, groups, prm, f, t, nr, delta);
}

// One warm-started batch round for the queries of one class: samples, the
// network, extensions.
static bool launch_batch_warm_round(int dof, int kind, int batch, unsigned nb, hipStream_t st,
                                    const ProblemDev* probs, int n, int groups, const ProjDev& prm,
                                    const unsigned* round, float* f, float* t, int* nr,
                                    float* delta, const cp_mlp* mlp, const cp_robot* robot,
                                    const ConDev& con, hipError_t* he) {
#define CP_BATCH_WARM(ND, K)                                                                          \
  {                                                                                                   \
    plan_batch_sample_kernel<ND><<<nb, kPlanBlock, 0, st>>>(probs, n, groups, round, f, t, nr);       \
    *he = mlp_warm_corrections(mlp, robot, con, prm.W, (long)n * groups, f, t, delta, st);            \
    launch_batch_warm_class<ND, K>(batch, nb, st, probs, n, groups, prm, f, t, nr, delta);            \
    return true;                                                                                      \
  }
  switch (dof * 4 + kind) {
    case 6 * 4 + KIND_NONE: CP_BATCH_WARM(6, KIND_NONE)
    case 6 * 4 + KIND_POSE: CP_BATCH_WARM(6, KIND_POSE)
    case 7 * 4 + KIND_NONE: CP_BATCH_WARM(7, KIND_NONE)
    case 7 * 4 + KIND_POSE: CP_BATCH_WARM(7, KIND_POSE)
    case 9 * 4 + KIND_NONE: CP_BATCH_WARM(9, KIND_NONE)
    case 9 * 4 + KIND_POSE: CP_BATCH_WARM(9, KIND_POSE)
    case 14 * 4 + KIND_POSE: CP_BATCH_WARM(14, KIND_POSE)
    case 14 * 4 + KIND_REL: CP_BATCH_WARM(14, KIND_REL)
    default: return false;
  }
#undef CP_BATCH_WARM
}

__global__ void publish_batch_kernel(ProblemDev* probs, int n_probs, unsigned* round) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_probs) {
    int* ctl = probs[i].pd.ctl;
    const int cap = probs[i].pd.cap;
    ctl[kCtlPublished + 0] = min(ctl[kCtlCount + 0], cap);
    ctl[kCtlPublished + 1] = min(ctl[kCtlCount + 1], cap);
  }
  if (i == 0) *round += 1u;
}

// Roots of both trees and a fresh control block per query; done_init[i] = 1
// marks a query with nothing to search (endpoint check failed, or start and
// goal already connected at the roots).
__global__ void plan_batch_init_kernel(ProblemDev* probs, int n_probs, const float* __restrict__ ends,
                                       const int* __restrict__ ends_off,
                                       const int* __restrict__ done_init) {
  const int i = blockIdx.x;
  if (i >= n_probs) return;
  const PlanDev& pd = probs[i].pd;
  const int dof = probs[i].dof;
  const int t = threadIdx.x;
  if (t < 2) {
    for (int j = 0; j < dof; ++j) pd.q[t][(size_t)j * pd.cap] = ends[ends_off[i] + t * dof + j];
    pd.parent[t][0] = -1;
  }
  if (t < kCtlInts)
    pd.ctl[t] = (t == kCtlCount || t == kCtlCount + 1 || t == kCtlPublished || t == kCtlPublished + 1)
                    ? 1
                    : (t == kCtlDone ? done_init[i] : 0);
}

// Endpoint checks of every query of a batch in one launch, one wavefront
// per query: lane 0 takes the start, lane 1 the goal for the task error
// (ok[2i + e] = error below tol, no projection step); the minimum signed
// distance of the robot's spheres to the query's scene (sd[2i + e]) comes
// from all lanes splitting the primitives (config_min_sd), start then goal.
__global__ __launch_bounds__(64) void batch_ends_kernel(const ProblemDev* __restrict__ probs,
                                                        int n_probs, const float* __restrict__ ends,
                                                        const int* __restrict__ ends_off, float tol,
                                                        int* __restrict__ ok, float* __restrict__ sd) {
  const int i = blockIdx.x;
  if (i >= n_probs) return;
  const ProblemDev& P = probs[i];
  const int lane = threadIdx.x;
  const bool on = lane < 2;
  const float* q = ends + ends_off[i] + (on ? lane : 0) * P.dof;
  float einf = 0.0f;
#define CP_ENDS_CASE(ND, K)                                       \
  case ND * 4 + K: {                                              \
    float qa[ND], g[ND];                                          \
    for (int j = 0; j < ND; ++j) qa[j] = q[j];                    \
    task_step<ND, K>(P.rob, P.con, qa, 0.0f, g, einf);            \
    break;                                                        \
  }
  switch (P.dof * 4 + P.con.kind) {
    CP_ENDS_CASE(6, KIND_NONE)
    CP_ENDS_CASE(6, KIND_POSE)
    CP_ENDS_CASE(7, KIND_NONE)
    CP_ENDS_CASE(7, KIND_POSE)
    CP_ENDS_CASE(9, KIND_NONE)
    CP_ENDS_CASE(9, KIND_POSE)
    CP_ENDS_CASE(14, KIND_POSE)
    CP_ENDS_CASE(14, KIND_REL)
    default: einf = FLT_MAX; break;
  }
#undef CP_ENDS_CASE
  if (on) ok[2 * i + lane] = einf < tol ? 1 : 0;
  for (int e = 0; e < 2; ++e) {
    const float d = config_min_sd<4>(P.rob, P.sph, P.env, ends + ends_off[i] + e * P.dof);
    if (lane == 0) sd[2 * i + e] = d;
  }
}

// Path assembly for many queries: item = (query, tree, node, mode, offset).
__global__ void gather_batch_kernel(const ProblemDev* __restrict__ probs, const int* __restrict__ items,
                                    int n_items, int W, const long* __restrict__ out_off,
                                    float* __restrict__ out) {
  const int i = blockIdx.x;
  if (i >= n_items) return;
  const int qi = items[5 * i + 0], tree = items[5 * i + 1], node = items[5 * i + 2],
            mode = items[5 * i + 3], off = items[5 * i + 4];
  const PlanDev& pd = probs[qi].pd;
  const int dof = probs[qi].dof;
  float* o = out + out_off[qi];
  if (mode == 2) {
    for (int j = threadIdx.x; j < dof; j += blockDim.x)
      o[(size_t)off * dof + j] = pd.q[tree][(size_t)j * pd.cap + node];
    return;
  }
  const float* e = pd.edge[tree] + (size_t)node * W * dof;
  for (int t = threadIdx.x; t < (W - 1) * dof; t += blockDim.x) {
    const int p = t / dof, j = t % dof;
    const int src = mode == 1 ? (W - 2 - p) : (p + 1);
    o[(size_t)(off + p) * dof + j] = e[(size_t)src * dof + j];
  }
}

template <int NDOF, int KIND>
static void launch_round_kind(int batch, unsigned nb, hipStream_t st, const RobotDev* rob,
                              const float4* sph, const EnvDev& env, const ConDev& con,
                              const ProjDev& prm, const PlanDev& pd, size_t lds) {
  if (lds > 0) {
    if (batch == 4)
      plan_round_kernel<NDOF, KIND, 4, true><<<nb, kPlanBlock, lds, st>>>(rob, sph, env, con, prm, pd);
    else
      plan_round_kernel<NDOF, KIND, 8, true><<<nb, kPlanBlock, lds, st>>>(rob, sph, env, con, prm, pd);
  } else if (batch == 4) {
    plan_round_kernel<NDOF, KIND, 4, false><<<nb, kPlanBlock, 0, st>>>(rob, sph, env, con, prm, pd);
  } else {
    plan_round_kernel<NDOF, KIND, 8, false><<<nb, kPlanBlock, 0, st>>>(rob, sph, env, con, prm, pd);
  }
}

template <int NDOF>
static bool launch_round_ndof(int kind, int batch, unsigned nb, hipStream_t st, const RobotDev* rob,
                              const float4* sph, const EnvDev& env, const ConDev& con,
                              const ProjDev& prm, const PlanDev& pd, size_t lds) {
  switch (kind) {
    case KIND_NONE: launch_round_kind<NDOF, KIND_NONE>(batch, nb, st, rob, sph, env, con, prm, pd, lds); return true;
    case KIND_POSE: launch_round_kind<NDOF, KIND_POSE>(batch, nb, st, rob, sph, env, con, prm, pd, lds); return true;
    case KIND_REL:
      if constexpr (NDOF % 2 == 0) {
        launch_round_kind<NDOF, KIND_REL>(batch, nb, st, rob, sph, env, con, prm, pd, lds);
        return true;
      }
      return false;
  }
  return false;
}

template <int NDOF>
static bool launch_warm_ndof(int kind, int batch, unsigned nb, hipStream_t st, const RobotDev* rob,
                             const float4* sph, const EnvDev& env, const ConDev& con,
                             const ProjDev& prm, const PlanDev& pd, float* f, float* t, int* nr,
                             float* delta, const cp_mlp* mlp, const cp_robot* robot,
                             hipError_t* he) {
  if (kind == KIND_REL && NDOF % 2 != 0) return false;
  plan_sample_kernel<NDOF><<<nb, kPlanBlock, 0, st>>>(rob, pd, f, t, nr);
  *he = mlp_warm_corrections(mlp, robot, con, prm.W, pd.n_groups, f, t, delta, st);
#define CP_WARM_KIND(K)                                                                              \
  if (batch == 4)                                                                                    \
    plan_round_warm_kernel<NDOF, K, 4><<<nb, kPlanBlock, 0, st>>>(rob, sph, env, con, prm, pd, f, t, nr, delta); \
  else                                                                                               \
    plan_round_warm_kernel<NDOF, K, 8><<<nb, kPlanBlock, 0, st>>>(rob, sph, env, con, prm, pd, f, t, nr, delta);
  switch (kind) {
    case KIND_NONE: CP_WARM_KIND(KIND_NONE) return true;
    case KIND_POSE: CP_WARM_KIND(KIND_POSE) return true;
    case KIND_REL:
      if constexpr (NDOF % 2 == 0) {
        CP_WARM_KIND(KIND_REL)
        return true;
      }
      return false;
  }
#undef CP_WARM_KIND
  return false;
}

// One warm-started round of a single query: samples, network, extensions.
static bool launch_warm_round(int dof, int kind, int batch, unsigned nb, hipStream_t st,
                              const RobotDev* rob, const float4* sph, const EnvDev& env,
                              const ConDev& con, const ProjDev& prm, const PlanDev& pd, float* f,
                              float* t, int* nr, float* delta, const cp_mlp* mlp,
                              const cp_robot* robot, hipError_t* he) {
  switch (dof) {
    case 2: return launch_warm_ndof<2>(kind, batch, nb, st, rob, sph, env, con, prm, pd, f, t, nr, delta, mlp, robot, he);
    case 3: return launch_warm_ndof<3>(kind, batch, nb, st, rob, sph, env, con, prm, pd, f, t, nr, delta, mlp, robot, he);
    case 6: return launch_warm_ndof<6>(kind, batch, nb, st, rob, sph, env, con, prm, pd, f, t, nr, delta, mlp, robot, he);
    case 7: return launch_warm_ndof<7>(kind, batch, nb, st, rob, sph, env, con, prm, pd, f, t, nr, delta, mlp, robot, he);
    case 9: return launch_warm_ndof<9>(kind, batch, nb, st, rob, sph, env, con, prm, pd, f, t, nr, delta, mlp, robot, he);
    case 14: return launch_warm_ndof<14>(kind, batch, nb, st, rob, sph, env, con, prm, pd, f, t, nr, delta, mlp, robot, he);
    default: return false;
  }
}

static bool launch_round(int dof, int kind, int batch, unsigned nb, hipStream_t st,
                         const RobotDev* rob, const float4* sph, const EnvDev& env,
                         const ConDev& con, const ProjDev& prm, const PlanDev& pd, size_t lds) {
  switch (dof) {
    case 2: return launch_round_ndof<2>(kind, batch, nb, st, rob, sph, env, con, prm, pd, lds);
    case 3: return launch_round_ndof<3>(kind, batch, nb, st, rob, sph, env, con, prm, pd, lds);
    case 6: return launch_round_ndof<6>(kind, batch, nb, st, rob, sph, env, con, prm, pd, lds);
    case 7: return launch_round_ndof<7>(kind, batch, nb, st, rob, sph, env, con, prm, pd, lds);
    case 9: return launch_round_ndof<9>(kind, batch, nb, st, rob, sph, env, con, prm, pd, lds);
    case 14: return launch_round_ndof<14>(kind, batch, nb, st, rob, sph, env, con, prm, pd, lds);
    default: return false;
  }
}

}  // namespace cprrtc

// ------------------------------------------------------------------ host side

using namespace cprrtc;

struct cp_planner {
  const cp_robot* robot = nullptr;
  cp_plan_opts opts;
  int dof = 0;
  float* q[2] = {nullptr, nullptr};
  int* parent[2] = {nullptr, nullptr};
  float* edge[2] = {nullptr, nullptr};
  float* scratch = nullptr;
  int* ctl = nullptr;
  int* items = nullptr;       // device chain lists of path_walk_kernel
  float* path_buf = nullptr;  // device path buffer
  int* host_ctl = nullptr;    // pinned mirror of the control block
  size_t path_cap = 0;        // points that fit in path_buf / items
  int* path_hdr = nullptr;    // device {path rows, chain lengths} (path_walk_kernel)
  // pinned staging: endpoints out, check results and path header back, the
  // first kPathPrefixRows rows of the path back in the same synchronisation
  float* host_io = nullptr;
  float* host_path = nullptr;
  float* cfg = nullptr;       // [2][dof] start/goal scratch for checks
  float* cfg_out = nullptr;
  int* cfg_status = nullptr;
  uint8_t* cfg_col = nullptr;
  float* cfg_sd = nullptr;
  // learned warm start (cp_planner_set_warm): the network and its round buffers
  const cp_mlp* warm = nullptr;
  float* seg_from = nullptr;  // [n_groups][dof]
  float* seg_to = nullptr;    // [n_groups][dof]
  int* seg_near = nullptr;    // [n_groups]
  float* delta = nullptr;     // [n_groups][W-1][dof]
};

namespace {

uint64_t splitmix64(uint64_t& state) {
  uint64_t z = (state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

void free_planner(cp_planner* p) {
  if (!p) return;
  for (int t = 0; t < 2; ++t) {
    if (p->q[t]) (void)hipFree(p->q[t]);
    if (p->parent[t]) (void)hipFree(p->parent[t]);
    if (p->edge[t]) (void)hipFree(p->edge[t]);
  }
  if (p->scratch) (void)hipFree(p->scratch);
  if (p->ctl) (void)hipFree(p->ctl);
  if (p->items) (void)hipFree(p->items);
  if (p->path_buf) (void)hipFree(p->path_buf);
  if (p->host_ctl) (void)hipHostFree(p->host_ctl);
  if (p->host_io) (void)hipHostFree(p->host_io);
  if (p->host_path) (void)hipHostFree(p->host_path);
  if (p->path_hdr) (void)hipFree(p->path_hdr);
  if (p->cfg) (void)hipFree(p->cfg);
  if (p->cfg_out) (void)hipFree(p->cfg_out);
  if (p->cfg_status) (void)hipFree(p->cfg_status);
  if (p->cfg_col) (void)hipFree(p->cfg_col);
  if (p->cfg_sd) (void)hipFree(p->cfg_sd);
  for (void* b : {(void*)p->seg_from, (void*)p->seg_to, (void*)p->seg_near, (void*)p->delta})
    if (b) (void)hipFree(b);
  delete p;
}

}  // namespace

extern "C" {

void cp_plan_opts_default(cp_plan_opts* o) {
  if (!o) return;
  cp_proj_params_default(&o->proj);
  o->n_groups = 256;
  o->max_rounds = 2000;
  o->capacity = 16384;
  o->max_connect = 64;
  o->poll_every = 1;
  o->flags = 0;
}

int cp_planner_create(const cp_robot* robot, const cp_plan_opts* opts, cp_planner** out) {
  try {
    if (!robot || !out) return api_fail(CP_E_ARG, "cp_planner_create: NULL argument");
    *out = nullptr;
    cp_plan_opts o;
    cp_plan_opts_default(&o);
    if (opts) o = *opts;
    cp_proj_params p;
    int rc = api_params(&o.proj, &p);
    if (rc != CP_OK) return rc;
    o.proj = p;
    if (o.n_groups < 2 || o.n_groups > 65536) return api_fail(CP_E_ARG, "n_groups %d not in 2..65536", o.n_groups);
    if (o.capacity < 2 || o.capacity > (1 << 24)) return api_fail(CP_E_ARG, "capacity %d not in 2..2^24", o.capacity);
    if (o.max_rounds < 1 || o.max_connect < 0 || o.poll_every < 1)
      return api_fail(CP_E_ARG, "max_rounds, max_connect or poll_every out of range");
    if (o.flags & ~CP_SELF_COLLISION) return api_fail(CP_E_ARG, "plan flags %d", o.flags);
    if ((o.flags & CP_SELF_COLLISION) && plan_lds_bytes(robot->host.n_spheres) > 65536)
      return api_fail(CP_E_UNSUPPORTED, "self-collision planning supports at most 1020 spheres");
    if (!dof_supported(robot->host.dof))
      return api_fail(CP_E_UNSUPPORTED, "planning kernels are built for dof 2, 3, 6, 7, 9, 14 (got %d)", robot->host.dof);
    cp_planner* pl = new (std::nothrow) cp_planner;
    if (!pl) return api_fail(CP_E_ARG, "out of host memory");
    pl->robot = robot;
    pl->opts = o;
    const int n = robot->host.dof, W = o.proj.W;
    pl->dof = n;
    const size_t cap = (size_t)o.capacity;
    // path: at most capacity nodes per tree, W-1 points per edge, + 2
    pl->path_cap = 2 * cap * (size_t)(W - 1) + 2;
    hipError_t e = hipSuccess;
    for (int t = 0; t < 2 && e == hipSuccess; ++t) {
      e = hipMalloc((void**)&pl->q[t], sizeof(float) * n * cap);
      if (e == hipSuccess) e = hipMalloc((void**)&pl->parent[t], sizeof(int) * cap);
      if (e == hipSuccess) e = hipMalloc((void**)&pl->edge[t], sizeof(float) * cap * W * n);
    }
    if (e == hipSuccess) e = hipMalloc((void**)&pl->scratch, sizeof(float) * (size_t)o.n_groups * W * n);
    if (e == hipSuccess) e = hipMalloc((void**)&pl->ctl, sizeof(int) * kCtlInts);
    if (e == hipSuccess) e = hipMalloc((void**)&pl->items, sizeof(int) * 4 * 2 * cap);
    if (e == hipSuccess) e = hipMalloc((void**)&pl->path_buf, sizeof(float) * pl->path_cap * n);
    if (e == hipSuccess) e = hipHostMalloc((void**)&pl->host_ctl, sizeof(int) * kCtlInts, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&pl->host_io, sizeof(float) * kHostIoFloats, hipHostMallocDefault);
    if (e == hipSuccess)
      e = hipHostMalloc((void**)&pl->host_path, sizeof(float) * kPathPrefixRows * n, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void**)&pl->path_hdr, sizeof(int) * 4);
    if (e == hipSuccess) e = hipMalloc((void**)&pl->cfg, sizeof(float) * 2 * n);
    if (e == hipSuccess) e = hipMalloc((void**)&pl->cfg_out, sizeof(float) * 2 * n);
    if (e == hipSuccess) e = hipMalloc((void**)&pl->cfg_status, sizeof(int) * 2);
    if (e == hipSuccess) e = hipMalloc((void**)&pl->cfg_col, 2);
    if (e == hipSuccess) e = hipMalloc((void**)&pl->cfg_sd, sizeof(float) * 2);
    if (e != hipSuccess) {
      free_planner(pl);
      return api_hip_fail(e, "cp_planner_create");
    }
    *out = pl;
    return CP_OK;
  } catch (...) {
    return api_fail(CP_E_ARG, "cp_planner_create: unexpected exception");
  }
}

void cp_planner_destroy(cp_planner* p) { free_planner(p); }

int cp_planner_set_warm(cp_planner* pl, const cp_mlp* mlp) {
  try {
    if (!pl) return api_fail(CP_E_ARG, "cp_planner_set_warm: NULL planner");
    if (mlp && (pl->opts.flags & CP_SELF_COLLISION))
      return api_fail(CP_E_UNSUPPORTED, "cp_planner_set_warm: warm-started rounds do not check self-collision");
    if (mlp && pl->opts.proj.variant != CP_PROJECT_PARALLEL)
      return api_fail(CP_E_UNSUPPORTED, "cp_planner_set_warm: the warm start serves the parallel projector only");
    if (mlp && !pl->seg_from) {
      const size_t G = pl->opts.n_groups, n = pl->dof, W = pl->opts.proj.W;
      hipError_t e = hipMalloc((void**)&pl->seg_from, sizeof(float) * G * n);
      if (e == hipSuccess) e = hipMalloc((void**)&pl->seg_to, sizeof(float) * G * n);
      if (e == hipSuccess) e = hipMalloc((void**)&pl->seg_near, sizeof(int) * G);
      if (e == hipSuccess) e = hipMalloc((void**)&pl->delta, sizeof(float) * G * (W - 1) * n);
      if (e != hipSuccess) return api_hip_fail(e, "cp_planner_set_warm");
    }
    pl->warm = mlp;
    return CP_OK;
  } catch (...) {
    return api_fail(CP_E_ARG, "cp_planner_set_warm: unexpected exception");
  }
}

int cp_plan(cp_planner* pl, const cp_env* env, const cp_constraint* constraint,
            const double* start, const double* goal, uint64_t seed, cp_path* out,
            cp_plan_stats* stats, void* stream_v) {
  try {
    if (!pl || !env || !start || !goal || !out) return api_fail(CP_E_ARG, "cp_plan: NULL argument");
    if (out->capacity > 0 && !out->q) return api_fail(CP_E_ARG, "cp_plan: NULL path buffer");
    hipStream_t st = (hipStream_t)stream_v;
    const cp_robot* robot = pl->robot;
    const int n = pl->dof, W = pl->opts.proj.W;
    const cp_plan_opts& o = pl->opts;
    out->len = 0;
    out->dof = n;
    if (stats) std::memset(stats, 0, sizeof *stats);
    ConDev con;
    int rc = api_constraint(constraint, robot, &con);
    if (rc != CP_OK) return rc;
    const cp_proj_params& pp = o.proj;
    ProjDev prm;
    prm.W = W;
    prm.max_iters = pp.max_iters;
    prm.tau = (float)pp.tau;
    prm.tau_sm = (float)pp.tau_sm;
    prm.tau_task = (float)pp.tau_task;
    prm.alpha = (float)pp.alpha;
    prm.lambda2 = (float)(pp.lambda * pp.lambda);
    prm.variant = pp.variant;

    // endpoints: inside the limits (host), on the manifold and collision-free (device)
    for (int e = 0; e < 2; ++e) {
      const double* c = e == 0 ? start : goal;
      for (int j = 0; j < n; ++j)
        if (!(c[j] >= robot->host.lo[j] && c[j] <= robot->host.hi[j]))
          return api_fail(e == 0 ? CP_E_START : CP_E_GOAL, "%s outside the joint limits", e == 0 ? "start" : "goal");
    }
    // pinned staging: [0, 2n) the endpoints, [2n, 2n + 2) the checks'
    // statuses (int bits), [2n + 2, 2n + 4) their distances
    float* io = pl->host_io;
    for (int j = 0; j < n; ++j) {
      io[j] = (float)start[j];
      io[n + j] = (float)goal[j];
    }
    hipError_t he = hipMemcpyAsync(pl->cfg, io, sizeof(float) * 2 * n, hipMemcpyHostToDevice, st);
    if (he != hipSuccess) return api_hip_fail(he, "cp_plan");
    bool sup = false;
    he = launch_project_configs(n, robot->dev, con, 2, pl->cfg, pl->cfg_out, pl->cfg_status,
                                (float)pp.tau_task, 0, 1.0f, 0.0f, st, &sup);
    if (he == hipSuccess) he = launch_config_sd(robot->dev, robot->spheres, env->view, 2, pl->cfg, pl->cfg_col, pl->cfg_sd, st);
    // with the self-check on, an endpoint must also be clear of the robot itself
    const int n_self = (int)robot->self_pairs.size() / 2;
    if (he == hipSuccess && (o.flags & CP_SELF_COLLISION) && n_self > 0)
      he = launch_self_cc(robot->dev, robot->host, robot->spheres, robot->pairs_cc, robot->n_cc, 2,
                          pl->cfg, pl->cfg_col, pl->cfg_sd, false, st);
    int* ok_h = reinterpret_cast<int*>(io + 2 * n);
    float* sd_h = io + 2 * n + 2;
    if (he == hipSuccess) he = hipMemcpyAsync(ok_h, pl->cfg_status, sizeof(int) * 2, hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipMemcpyAsync(sd_h, pl->cfg_sd, sizeof(float) * 2, hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    if (he != hipSuccess) return api_hip_fail(he, "cp_plan endpoint checks");
    if (!sup) return api_fail(CP_E_UNSUPPORTED, "no kernel for dof %d with constraint kind %d", n, con.kind);
    if (!ok_h[0]) return api_fail(CP_E_START, "start is off the constraint manifold");
    if (!ok_h[1]) return api_fail(CP_E_GOAL, "goal is off the constraint manifold");
    if (!(sd_h[0] > 0.0f)) return api_fail(CP_E_START, "start is in collision (scene or, with CP_SELF_COLLISION, the robot itself)");
    if (!(sd_h[1] > 0.0f)) return api_fail(CP_E_GOAL, "goal is in collision (scene or, with CP_SELF_COLLISION, the robot itself)");

    const double tol = pp.tau + pp.tau_sm;
    double dsg = 0.0;
    for (int j = 0; j < n; ++j) dsg += (start[j] - goal[j]) * (start[j] - goal[j]);
    if (std::sqrt(dsg) < tol) {   // already connected
      out->len = 2;
      if (out->capacity < 2) return api_fail(CP_E_CAPACITY, "path needs 2 rows");
      std::memcpy(out->q, start, sizeof(double) * n);
      std::memcpy(out->q + n, goal, sizeof(double) * n);
      return CP_OK;
    }

    PlanDev pd;
    std::memset(&pd, 0, sizeof pd);
    for (int t = 0; t < 2; ++t) {
      pd.q[t] = pl->q[t];
      pd.parent[t] = pl->parent[t];
      pd.edge[t] = pl->edge[t];
    }
    pd.scratch = pl->scratch;
    pd.ctl = pl->ctl;
    pd.cap = o.capacity;
    pd.n_groups = o.n_groups;
    pd.max_connect = o.max_connect;
    pd.step = (float)((W - 1) * pp.tau);
    // (pl->cfg still holds the endpoints)
    plan_init_kernel<<<1, 64, 0, st>>>(pd, pl->cfg, n);
    he = hipGetLastError();
    if (he != hipSuccess) return api_hip_fail(he, "cp_plan init");
    pd.connect2 = (float)(tol * tol);
    uint64_t state = seed;
    for (int j = 0; j < kMaxDof; ++j)
      pd.shift[j] = (float)((double)(splitmix64(state) >> 11) * (1.0 / 9007199254740992.0));
    const unsigned nb = (unsigned)((o.n_groups * 64 + kPlanBlock - 1) / kPlanBlock);
    // self-collision in the extensions: the robot's pairs and the LDS for
    // one configuration's sphere centres per wavefront
    const int n_pairs = (int)robot->self_pairs.size() / 2;
    if ((o.flags & CP_SELF_COLLISION) && n_pairs > 0) {
      pd.self_pairs = robot->pairs;
      pd.n_self = n_pairs;
    }
    const size_t lds = pd.n_self > 0 ? plan_lds_bytes(robot->host.n_spheres) : 0;

    int rounds = 0;
    bool done = false;
    if (pl->warm) {
      rc = mlp_warm_check(pl->warm, n, con.kind);
      if (rc != CP_OK) return rc;
    }
    // the round kernel compiled for this robot and mask (cp_robot_specialize), if any
    // (warm-started rounds use the library's kernels)
    RtcFns rk;
    const bool use_rtc = !pl->warm && rtc_find(const_cast<cp_robot*>(robot), con, &rk) &&
                         rk.plan[0] && lds == 0;   // (compiled without the self-check)
    while (rounds < o.max_rounds && !done) {
      pd.sample_base = (unsigned)rounds * (unsigned)o.n_groups;
      if (pl->warm) {
        hipError_t we = hipSuccess;
        if (!launch_warm_round(n, con.kind, pp.sphere_batch, nb, st, robot->dev, robot->spheres,
                               env->view, con, prm, pd, pl->seg_from, pl->seg_to, pl->seg_near,
                               pl->delta, pl->warm, robot, &we))
          return api_fail(CP_E_UNSUPPORTED, "no planning kernel for dof %d, constraint kind %d", n, con.kind);
        if (we != hipSuccess) return api_hip_fail(we, "cp_plan warm-start network");
      } else if (use_rtc) {
        he = launch_rtc_plan_round(rk, robot, env->view, con, prm, pd, pp.sphere_batch, nb, lds,
                                   st);
        if (he != hipSuccess) return api_hip_fail(he, "cp_plan round (run-time compiled kernel)");
      } else if (!launch_round(n, con.kind, pp.sphere_batch, nb, st, robot->dev, robot->spheres,
                               env->view, con, prm, pd, lds)) {
        return api_fail(CP_E_UNSUPPORTED, "no planning kernel for dof %d, constraint kind %d", n, con.kind);
      }
      publish_kernel<<<1, 1, 0, st>>>(pl->ctl, o.capacity);
      ++rounds;
      if (rounds % o.poll_every == 0 || rounds == o.max_rounds) {
        he = hipMemcpyAsync(pl->host_ctl, pl->ctl, sizeof(int) * kCtlInts, hipMemcpyDeviceToHost, st);
        if (he == hipSuccess) he = hipStreamSynchronize(st);
        if (he != hipSuccess) return api_hip_fail(he, "cp_plan round");
        done = pl->host_ctl[kCtlDone] != 0;
        if (!done && pl->host_ctl[kCtlOverflow]) break;
      }
    }
    he = hipGetLastError();
    if (he != hipSuccess) return api_hip_fail(he, "cp_plan launch");
    const int* hc = pl->host_ctl;
    if (stats) {
      stats->rounds = rounds;
      stats->launches_per_round = pl->warm ? 4 : 2;
      stats->nodes[0] = std::min(hc[kCtlCount + 0], o.capacity);
      stats->nodes[1] = std::min(hc[kCtlCount + 1], o.capacity);
      stats->overflow = hc[kCtlOverflow];
    }
    if (!done) {
      if (hc[kCtlOverflow]) return api_fail(CP_E_CAPACITY, "a tree reached its capacity of %d nodes", o.capacity);
      return CP_NO_SOLUTION;
    }

    // path: tree-0 chain root -> n0, bridge to n1, tree-1 chain n1 -> root,
    // assembled on the device; its header and first rows come back in one
    // synchronisation
    const int X = hc[kCtlConn + 0], a = hc[kCtlConn + 1], b = hc[kCtlConn + 2];
    const int n0 = X == 0 ? a : b, n1 = X == 0 ? b : a;
    path_walk_kernel<<<1, 256, 0, st>>>(pd, n0, n1, W, n, pl->items, pl->path_hdr, pl->path_buf,
                                        (long)pl->path_cap);
    he = hipGetLastError();
    int* hdr = reinterpret_cast<int*>(io + kHostIoFloats - 4);
    const size_t pre = std::min((size_t)kPathPrefixRows, pl->path_cap);
    if (he == hipSuccess) he = hipMemcpyAsync(hdr, pl->path_hdr, sizeof(int) * 4, hipMemcpyDeviceToHost, st);
    if (he == hipSuccess)
      he = hipMemcpyAsync(pl->host_path, pl->path_buf, sizeof(float) * pre * n, hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    if (he != hipSuccess) return api_hip_fail(he, "cp_plan path");
    const size_t len = (size_t)hdr[0];
    out->len = (int32_t)len;
    if ((size_t)out->capacity < len) return api_fail(CP_E_CAPACITY, "path needs %zu rows", len);
    for (size_t i = 1; i + 1 < std::min(len, pre); ++i)
      for (int j = 0; j < n; ++j) out->q[i * n + j] = (double)pl->host_path[i * n + j];
    if (len > pre) {   // the rest of a long path
      std::vector<float> rest((len - pre) * n);
      he = hipMemcpyAsync(rest.data(), pl->path_buf + pre * n, sizeof(float) * rest.size(), hipMemcpyDeviceToHost, st);
      if (he == hipSuccess) he = hipStreamSynchronize(st);
      if (he != hipSuccess) return api_hip_fail(he, "cp_plan path");
      for (size_t i = pre; i + 1 < len; ++i)
        for (int j = 0; j < n; ++j) out->q[i * n + j] = (double)rest[(i - pre) * n + j];
    }
    // the end points are the caller's own values
    std::memcpy(out->q, start, sizeof(double) * n);
    std::memcpy(out->q + (len - 1) * n, goal, sizeof(double) * n);
    return CP_OK;
  } catch (...) {
    return api_fail(CP_E_ARG, "cp_plan: unexpected exception");
  }
}

int cp_planner_tree(const cp_planner* pl, int32_t tree, int32_t capacity, double* q,
                    int32_t* parent, int32_t* count) {
  try {
    if (!pl || !count || tree < 0 || tree > 1) return api_fail(CP_E_ARG, "cp_planner_tree: bad argument");
    int ctl[kCtlInts];
    hipError_t he = hipMemcpy(ctl, pl->ctl, sizeof ctl, hipMemcpyDeviceToHost);
    if (he != hipSuccess) return api_hip_fail(he, "cp_planner_tree");
    const int cap = pl->opts.capacity, n = pl->dof;
    const int cnt = std::min(ctl[kCtlCount + tree], cap);
    *count = cnt;
    if (capacity < cnt) return api_fail(CP_E_CAPACITY, "tree holds %d nodes", cnt);
    if (cnt > 0 && (!q || !parent)) return api_fail(CP_E_ARG, "cp_planner_tree: NULL buffer");
    std::vector<float> col(cnt);
    for (int j = 0; j < n && cnt > 0; ++j) {
      he = hipMemcpy(col.data(), pl->q[tree] + (size_t)j * cap, sizeof(float) * cnt, hipMemcpyDeviceToHost);
      if (he != hipSuccess) return api_hip_fail(he, "cp_planner_tree");
      for (int i = 0; i < cnt; ++i) q[(size_t)i * n + j] = (double)col[i];
    }
    if (cnt > 0) {
      he = hipMemcpy(parent, pl->parent[tree], sizeof(int32_t) * cnt, hipMemcpyDeviceToHost);
      if (he != hipSuccess) return api_hip_fail(he, "cp_planner_tree");
    }
    return CP_OK;
  } catch (...) {
    return api_fail(CP_E_ARG, "cp_planner_tree: unexpected exception");
  }
}

int plan(const cp_robot* robot, const cp_env* env, const cp_constraint* constraint,
         const double* start, const double* goal, uint64_t seed, const cp_plan_opts* opts,
         cp_path* out) {
  cp_planner* pl = nullptr;
  int rc = cp_planner_create(robot, opts, &pl);
  if (rc != CP_OK) return rc;
  rc = cp_plan(pl, env, constraint, start, goal, seed, out, nullptr, nullptr);
  (void)hipStreamSynchronize(nullptr);
  cp_planner_destroy(pl);
  return rc;
}

void cp_batch_opts_default(cp_batch_opts* o) {
  if (!o) return;
  cp_proj_params_default(&o->proj);
  o->groups_per_query = 16;
  o->max_rounds = 500;
  o->capacity = 2048;
  o->max_connect = 64;
  o->rounds_per_graph = 4;
  o->flags = 0;
}

}  // extern "C"

struct cp_batch {
  cp_batch_opts opts;
  int max_queries = 0, max_dof = 0;
  float* q = nullptr;          // [Q][2][max_dof][cap]
  int* parent = nullptr;       // [Q][2][cap]
  float* edge = nullptr;       // [Q][2][cap][W][max_dof]
  float* scratch = nullptr;    // [Q][G][W][max_dof]
  int* ctl = nullptr;          // [Q][kCtlInts]
  unsigned* round = nullptr;   // device round counter
  unsigned* queue = nullptr;   // device task counter and finished-wavefront count
  ProblemDev* probs = nullptr; // [Q]
  int* host_ctl = nullptr;     // pinned [Q][kCtlInts]
  float* ends = nullptr;       // [Q][2][max_dof] endpoint scratch
  int* ends_off = nullptr;     // [Q]
  int* cfg_status = nullptr;   // [2Q] endpoint on the manifold
  float* cfg_sd = nullptr;     // [2Q] endpoint's minimum signed distance
  int* done_init = nullptr;    // [Q] nothing to search
  hipStream_t stream = nullptr;
  // learned warm start (cp_batch_set_warm): the network and its round buffers
  const cp_mlp* warm = nullptr;
  float* seg_from = nullptr;   // [Q * G][max_dof]
  float* seg_to = nullptr;
  int* seg_near = nullptr;     // [Q * G]
  float* delta = nullptr;      // [Q * G][W-1][max_dof]
};

namespace {

void free_batch(cp_batch* b) {
  if (!b) return;
  for (void* p : {(void*)b->q, (void*)b->parent, (void*)b->edge, (void*)b->scratch, (void*)b->ctl,
                  (void*)b->round, (void*)b->queue, (void*)b->probs, (void*)b->ends, (void*)b->ends_off,
                  (void*)b->cfg_status, (void*)b->cfg_sd, (void*)b->done_init,
                  (void*)b->seg_from, (void*)b->seg_to, (void*)b->seg_near, (void*)b->delta})
    if (p) (void)hipFree(p);
  if (b->host_ctl) (void)hipHostFree(b->host_ctl);
  if (b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

bool batch_kind_supported(int dof, int kind) {
  if (dof == 6 || dof == 7 || dof == 9) return kind == KIND_NONE || kind == KIND_POSE;
  if (dof == 14) return kind == KIND_POSE || kind == KIND_REL;
  return false;
}

}  // namespace

extern "C" {

int cp_batch_create(const cp_batch_opts* opts, int32_t max_queries, int32_t max_dof,
                    cp_batch** out) {
  try {
    if (!out) return api_fail(CP_E_ARG, "cp_batch_create: NULL argument");
    *out = nullptr;
    cp_batch_opts o;
    cp_batch_opts_default(&o);
    if (opts) o = *opts;
    cp_proj_params p;
    int rc = api_params(&o.proj, &p);
    if (rc != CP_OK) return rc;
    o.proj = p;
    if (max_queries < 1 || max_queries > 65536 || max_dof < 1 || max_dof > kMaxDof)
      return api_fail(CP_E_ARG, "cp_batch_create: max_queries or max_dof out of range");
    if (o.groups_per_query < 2 || o.capacity < 2 || o.max_rounds < 1 || o.max_connect < 0 ||
        o.rounds_per_graph < 1 || o.rounds_per_graph > 64 || (o.flags & ~CP_BATCH_PER_CLASS))
      return api_fail(CP_E_ARG, "cp_batch_create: options out of range");
    cp_batch* b = new (std::nothrow) cp_batch;
    if (!b) return api_fail(CP_E_ARG, "out of host memory");
    b->opts = o;
    b->max_queries = max_queries;
    b->max_dof = max_dof;
    const size_t Q = max_queries, C = o.capacity, W = o.proj.W, D = max_dof, Gq = o.groups_per_query;
    hipError_t e = hipMalloc((void**)&b->q, sizeof(float) * Q * 2 * D * C);
    if (e == hipSuccess) e = hipMalloc((void**)&b->parent, sizeof(int) * Q * 2 * C);
    if (e == hipSuccess) e = hipMalloc((void**)&b->edge, sizeof(float) * Q * 2 * C * W * D);
    if (e == hipSuccess) e = hipMalloc((void**)&b->scratch, sizeof(float) * Q * Gq * W * D);
    if (e == hipSuccess) e = hipMalloc((void**)&b->ctl, sizeof(int) * Q * kCtlInts);
    if (e == hipSuccess) e = hipMalloc((void**)&b->round, sizeof(unsigned));
    if (e == hipSuccess) e = hipMalloc((void**)&b->queue, sizeof(unsigned) * 2);
    if (e == hipSuccess) e = hipMalloc((void**)&b->probs, sizeof(ProblemDev) * Q);
    if (e == hipSuccess) e = hipHostMalloc((void**)&b->host_ctl, sizeof(int) * Q * kCtlInts, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void**)&b->ends, sizeof(float) * Q * 2 * D);
    if (e == hipSuccess) e = hipMalloc((void**)&b->ends_off, sizeof(int) * Q);
    if (e == hipSuccess) e = hipMalloc((void**)&b->cfg_status, sizeof(int) * Q * 2);
    if (e == hipSuccess) e = hipMalloc((void**)&b->cfg_sd, sizeof(float) * Q * 2);
    if (e == hipSuccess) e = hipMalloc((void**)&b->done_init, sizeof(int) * Q);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      free_batch(b);
      return api_hip_fail(e, "cp_batch_create");
    }
    *out = b;
    return CP_OK;
  } catch (...) {
    return api_fail(CP_E_ARG, "cp_batch_create: unexpected exception");
  }
}

void cp_batch_destroy(cp_batch* b) { free_batch(b); }

int cp_batch_set_warm(cp_batch* b, const cp_mlp* mlp) {
  try {
    if (!b) return api_fail(CP_E_ARG, "cp_batch_set_warm: NULL batch");
    if (mlp && b->opts.proj.variant != CP_PROJECT_PARALLEL)
      return api_fail(CP_E_UNSUPPORTED, "cp_batch_set_warm: the warm start serves the parallel projector only");
    if (mlp && !b->seg_from) {
      const size_t QG = (size_t)b->max_queries * b->opts.groups_per_query, D = b->max_dof,
                   W = b->opts.proj.W;
      hipError_t e = hipMalloc((void**)&b->seg_from, sizeof(float) * QG * D);
      if (e == hipSuccess) e = hipMalloc((void**)&b->seg_to, sizeof(float) * QG * D);
      if (e == hipSuccess) e = hipMalloc((void**)&b->seg_near, sizeof(int) * QG);
      if (e == hipSuccess) e = hipMalloc((void**)&b->delta, sizeof(float) * QG * (W - 1) * D);
      if (e != hipSuccess) return api_hip_fail(e, "cp_batch_set_warm");
    }
    b->warm = mlp;
    return CP_OK;
  } catch (...) {
    return api_fail(CP_E_ARG, "cp_batch_set_warm: unexpected exception");
  }
}

int cp_plan_batch(cp_batch* b, int32_t n, const cp_query* queries, cp_path* paths,
                  int32_t* status, cp_plan_stats* stats, void* caller_stream) {
  try {
    if (!b || !queries || !paths || !status) return api_fail(CP_E_ARG, "cp_plan_batch: NULL argument");
    if (n < 0 || n > b->max_queries) return api_fail(CP_E_ARG, "cp_plan_batch: %d queries (max %d)", n, b->max_queries);
    if (n == 0) return CP_OK;
    const cp_batch_opts& o = b->opts;
    const cp_proj_params& pp = o.proj;
    const int W = pp.W, D = b->max_dof, Gq = o.groups_per_query;
    const size_t C = o.capacity;
    hipError_t he = hipStreamSynchronize((hipStream_t)caller_stream);
    if (he != hipSuccess) return api_hip_fail(he, "cp_plan_batch");
    hipStream_t st = b->stream;
    ProjDev prm;
    prm.W = W;
    prm.max_iters = pp.max_iters;
    prm.tau = (float)pp.tau;
    prm.tau_sm = (float)pp.tau_sm;
    prm.tau_task = (float)pp.tau_task;
    prm.alpha = (float)pp.alpha;
    prm.lambda2 = (float)(pp.lambda * pp.lambda);
    prm.variant = pp.variant;
    const double tol = pp.tau + pp.tau_sm;

    // queries sorted by (DOF, constraint kind) class; slot k of the pools
    // and of the problem table serves query perm[k]
    std::vector<int> perm(n), cls(n);
    for (int i = 0; i < n; ++i) {
      if (!queries[i].robot) return api_fail(CP_E_ARG, "query %d: NULL robot", i);
      const int kind = queries[i].constraint ? queries[i].constraint->kind : CP_CON_NONE;
      cls[i] = queries[i].robot->host.dof * 4 + kind;
      perm[i] = i;
    }
    std::stable_sort(perm.begin(), perm.end(), [&](int x, int y) { return cls[x] < cls[y]; });
    std::vector<cp_query> sq(n);
    for (int k = 0; k < n; ++k) sq[k] = queries[perm[k]];
    std::vector<int32_t> st_k(n, CP_OK);
    std::vector<cp_plan_stats> stats_k(n);
    std::vector<cp_path*> path_k(n);
    for (int k = 0; k < n; ++k) path_k[k] = &paths[perm[k]];
    queries = sq.data();
    int32_t* const status_out = status;
    status = st_k.data();

    // per-query descriptors, endpoint limits
    std::vector<ProblemDev> probs(n);
    std::vector<float> ends((size_t)n * 2 * D, 0.0f);
    std::vector<int> ends_off(n);
    for (int i = 0; i < n; ++i) {
      const cp_query& qq = queries[i];
      status[i] = CP_OK;
      std::memset(&stats_k[i], 0, sizeof stats_k[i]);
      path_k[i]->len = 0;
      if (!qq.robot || !qq.env || !qq.start || !qq.goal) return api_fail(CP_E_ARG, "query %d: NULL member", perm[i]);
      const int dof = qq.robot->host.dof;
      if (dof > D) return api_fail(CP_E_ARG, "query %d: dof %d above the batch's %d", perm[i], dof, D);
      path_k[i]->dof = dof;
      ProblemDev& P = probs[i];
      std::memset(&P, 0, sizeof P);
      int rc = api_constraint(qq.constraint, qq.robot, &P.con);
      if (rc != CP_OK) return rc;
      if (!batch_kind_supported(dof, P.con.kind))
        return api_fail(CP_E_UNSUPPORTED, "query %d: dof %d with constraint kind %d", perm[i], dof, P.con.kind);
      P.rob = qq.robot->dev;
      P.sph = qq.robot->spheres;
      P.env = qq.env->view;
      P.dof = dof;
      PlanDev& pd = P.pd;
      for (int t = 0; t < 2; ++t) {
        pd.q[t] = b->q + ((size_t)i * 2 + t) * D * C;
        pd.parent[t] = b->parent + ((size_t)i * 2 + t) * C;
        pd.edge[t] = b->edge + ((size_t)i * 2 + t) * C * W * D;
      }
      pd.scratch = b->scratch + (size_t)i * Gq * W * D;
      pd.ctl = b->ctl + (size_t)i * kCtlInts;
      pd.cap = o.capacity;
      pd.n_groups = Gq;
      pd.max_connect = o.max_connect;
      pd.step = (float)((W - 1) * pp.tau);
      pd.connect2 = (float)(tol * tol);
      uint64_t state = qq.seed;
      for (int j = 0; j < kMaxDof; ++j)
        pd.shift[j] = (float)((double)(splitmix64(state) >> 11) * (1.0 / 9007199254740992.0));
      ends_off[i] = i * 2 * D;
      for (int j = 0; j < dof; ++j) {
        ends[(size_t)i * 2 * D + j] = (float)qq.start[j];
        ends[(size_t)i * 2 * D + dof + j] = (float)qq.goal[j];
        if (!(qq.start[j] >= qq.robot->host.lo[j] && qq.start[j] <= qq.robot->host.hi[j])) status[i] = CP_E_START;
        if (!(qq.goal[j] >= qq.robot->host.lo[j] && qq.goal[j] <= qq.robot->host.hi[j]) && status[i] == CP_OK) status[i] = CP_E_GOAL;
      }
    }
    // a warm-started batch: one network serves one robot and one constraint
    if (b->warm) {
      for (int i = 1; i < n; ++i)
        if (queries[i].robot != queries[0].robot || std::memcmp(&probs[i].con, &probs[0].con, sizeof(ConDev)) != 0)
          return api_fail(CP_E_UNSUPPORTED, "cp_plan_batch: a warm-started batch needs one robot and one constraint (query %d differs)", perm[i]);
      int rc = mlp_warm_check(b->warm, probs[0].dof, probs[0].con.kind);
      if (rc != CP_OK) return rc;
    }
    he = hipMemcpyAsync(b->ends, ends.data(), sizeof(float) * ends.size(), hipMemcpyHostToDevice, st);
    if (he == hipSuccess) he = hipMemcpyAsync(b->ends_off, ends_off.data(), sizeof(int) * n, hipMemcpyHostToDevice, st);
    // endpoints on the manifold and collision-free: every query's two
    // checks in one launch (the problem records go up first)
    if (he == hipSuccess) he = hipMemcpyAsync(b->probs, probs.data(), sizeof(ProblemDev) * n, hipMemcpyHostToDevice, st);
    if (he == hipSuccess) {
      batch_ends_kernel<<<n, 64, 0, st>>>(b->probs, n, b->ends, b->ends_off, (float)pp.tau_task,
                                          b->cfg_status, b->cfg_sd);
      he = hipGetLastError();
    }
    std::vector<int> ok_h(2 * n);
    std::vector<float> sd_h(2 * n);
    if (he == hipSuccess) he = hipMemcpyAsync(ok_h.data(), b->cfg_status, sizeof(int) * 2 * n, hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipMemcpyAsync(sd_h.data(), b->cfg_sd, sizeof(float) * 2 * n, hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    if (he != hipSuccess) return api_hip_fail(he, "cp_plan_batch endpoint checks");
    std::vector<int> active(n, 0);
    for (int i = 0; i < n; ++i) {
      if (status[i] == CP_OK && !(ok_h[2 * i] && sd_h[2 * i] > 0.0f)) status[i] = CP_E_START;
      if (status[i] == CP_OK && !(ok_h[2 * i + 1] && sd_h[2 * i + 1] > 0.0f)) status[i] = CP_E_GOAL;
      active[i] = status[i] == CP_OK;
    }
    // problems whose endpoints fail, or whose start and goal already
    // connect, are marked done at once (zero group budget, connection at
    // the roots)
    std::vector<int> done_init(n, 0);
    for (int i = 0; i < n; ++i) {
      double dsg = 0.0;
      for (int j = 0; j < probs[i].dof; ++j) dsg += (queries[i].start[j] - queries[i].goal[j]) * (queries[i].start[j] - queries[i].goal[j]);
      const bool trivial = active[i] && std::sqrt(dsg) < tol;
      done_init[i] = (!active[i] || trivial) ? 1 : 0;
    }
    he = hipMemcpyAsync(b->done_init, done_init.data(), sizeof(int) * n, hipMemcpyHostToDevice, st);
    if (he == hipSuccess) {
      plan_batch_init_kernel<<<n, 64, 0, st>>>(b->probs, n, b->ends, b->ends_off, b->done_init);
      he = hipGetLastError();
    }
    const unsigned zero = 0, zeros[2] = {0, 0};
    if (he == hipSuccess) he = hipMemcpyAsync(b->round, &zero, sizeof zero, hipMemcpyHostToDevice, st);
    if (he == hipSuccess) he = hipMemcpyAsync(b->queue, zeros, sizeof zeros, hipMemcpyHostToDevice, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    if (he != hipSuccess) return api_hip_fail(he, "cp_plan_batch init");

    // capture R rounds in a graph (per round: one launch per class, then the
    // publish kernel), replay until every query is done
    std::vector<std::pair<int, int>> ranges;   // [begin, end) of each class
    for (int k = 0; k < n;) {
      int e2 = k;
      while (e2 < n && probs[e2].dof * 4 + probs[e2].con.kind == probs[k].dof * 4 + probs[k].con.kind) ++e2;
      ranges.push_back({k, e2});
      k = e2;
    }
    const int R = o.rounds_per_graph;
    // one launch per round over the task queue when every class is in one set
    int set = -1;
    for (const auto& rg : ranges) {
      const int d = probs[rg.first].dof, k = probs[rg.first].con.kind;
      const int cs = (d == 14) ? 1 : (d == 6 || d == 7 || d == 9) ? 0 : 2;
      set = set < 0 ? cs : (set == cs ? set : 2);
    }
    const bool queued = !b->warm && !(o.flags & CP_BATCH_PER_CLASS) && (set == 0 || set == 1);
    unsigned q_blocks = 0;
    if (queued) {
      int per_cu = 0, cus = 0;
      hipError_t oe = set == 0
          ? (pp.sphere_batch == 4
                 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, plan_batch_queue_kernel<0, 4>, kPlanBlock, 0)
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, plan_batch_queue_kernel<0, 8>, kPlanBlock, 0))
          : (pp.sphere_batch == 4
                 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, plan_batch_queue_kernel<1, 4>, kPlanBlock, 0)
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, plan_batch_queue_kernel<1, 8>, kPlanBlock, 0));
      int dev = 0;
      if (oe == hipSuccess) oe = hipGetDevice(&dev);
      if (oe == hipSuccess) oe = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
      if (oe != hipSuccess) return api_hip_fail(oe, "cp_plan_batch occupancy");
      const long tasks = (long)n * Gq;
      const long resident = (long)std::max(per_cu, 1) * std::max(cus, 1);
      q_blocks = (unsigned)std::max(1L, std::min(resident, (tasks * 64 + kPlanBlock - 1) / kPlanBlock));
    }
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    he = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (he == hipSuccess && queued) {
      const unsigned waves = q_blocks * (kPlanBlock / 64);
      for (int r = 0; r < R; ++r) {
        if (set == 0 && pp.sphere_batch == 4)
          plan_batch_queue_kernel<0, 4><<<q_blocks, kPlanBlock, 0, st>>>(b->probs, n, Gq, prm, b->round, b->queue, waves);
        else if (set == 0)
          plan_batch_queue_kernel<0, 8><<<q_blocks, kPlanBlock, 0, st>>>(b->probs, n, Gq, prm, b->round, b->queue, waves);
        else if (pp.sphere_batch == 4)
          plan_batch_queue_kernel<1, 4><<<q_blocks, kPlanBlock, 0, st>>>(b->probs, n, Gq, prm, b->round, b->queue, waves);
        else
          plan_batch_queue_kernel<1, 8><<<q_blocks, kPlanBlock, 0, st>>>(b->probs, n, Gq, prm, b->round, b->queue, waves);
      }
      he = hipStreamEndCapture(st, &graph);
    } else if (he == hipSuccess) {
      hipError_t we = hipSuccess;
      for (int r = 0; r < R; ++r) {
        for (const auto& rg : ranges) {
          const int cnt = rg.second - rg.first;
          const long waves = (long)cnt * Gq;
          const unsigned nb = (unsigned)((waves * 64 + kPlanBlock - 1) / kPlanBlock);
          if (b->warm)
            launch_batch_warm_round(probs[rg.first].dof, probs[rg.first].con.kind, pp.sphere_batch, nb,
                                    st, b->probs + rg.first, cnt, Gq, prm, b->round, b->seg_from,
                                    b->seg_to, b->seg_near, b->delta, b->warm, queries[0].robot,
                                    probs[0].con, &we);
          else
            launch_batch_round(probs[rg.first].dof, probs[rg.first].con.kind, pp.sphere_batch, nb, st,
                               b->probs + rg.first, cnt, Gq, prm, b->round);
        }
        publish_batch_kernel<<<(n + 255) / 256, 256, 0, st>>>(b->probs, n, b->round);
      }
      he = hipStreamEndCapture(st, &graph);
      if (he == hipSuccess && we != hipSuccess) he = we;
    }
    if (he == hipSuccess) he = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (he != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return api_hip_fail(he, "cp_plan_batch graph");
    }
    int rounds = 0;
    std::vector<int> done_round(n, -1);
    while (rounds < o.max_rounds) {
      he = hipGraphLaunch(exec, st);
      if (he == hipSuccess) he = hipMemcpyAsync(b->host_ctl, b->ctl, sizeof(int) * n * kCtlInts, hipMemcpyDeviceToHost, st);
      if (he == hipSuccess) he = hipStreamSynchronize(st);
      if (he != hipSuccess) break;
      rounds += R;
      bool all = true;
      for (int i = 0; i < n; ++i) {
        const int* hc = b->host_ctl + (size_t)i * kCtlInts;
        if (hc[kCtlDone] && done_round[i] < 0) done_round[i] = rounds;
        all = all && (hc[kCtlDone] || hc[kCtlOverflow]);
      }
      if (all) break;
    }
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    if (he != hipSuccess) return api_hip_fail(he, "cp_plan_batch rounds");

    // paths of the solved queries
    std::vector<int> par((size_t)n * 2 * C);
    he = hipMemcpyAsync(par.data(), b->parent, sizeof(int) * par.size(), hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    if (he != hipSuccess) return api_hip_fail(he, "cp_plan_batch paths");
    std::vector<int> items;
    std::vector<long> out_off(n, 0);
    std::vector<size_t> lens(n, 0);
    long total = 0;
    for (int i = 0; i < n; ++i) {
      const int* hc = b->host_ctl + (size_t)i * kCtlInts;
      stats_k[i].rounds = done_round[i] >= 0 ? done_round[i] : rounds;
      stats_k[i].launches_per_round = queued ? 1 : b->warm ? 4 : (int)ranges.size() + 1;
      stats_k[i].nodes[0] = std::min(hc[kCtlCount + 0], o.capacity);
      stats_k[i].nodes[1] = std::min(hc[kCtlCount + 1], o.capacity);
      stats_k[i].overflow = hc[kCtlOverflow];
      if (status[i] != CP_OK) continue;
      if (!hc[kCtlDone]) {
        status[i] = hc[kCtlOverflow] ? CP_E_CAPACITY : CP_NO_SOLUTION;
        continue;
      }
      const int dof = probs[i].dof;
      const int X = hc[kCtlConn + 0], a = hc[kCtlConn + 1], c2 = hc[kCtlConn + 2];
      const int n0 = X == 0 ? a : c2, n1 = X == 0 ? c2 : a;
      const int* p0 = par.data() + ((size_t)i * 2 + 0) * C;
      const int* p1 = par.data() + ((size_t)i * 2 + 1) * C;
      std::vector<int> chain0, chain1;
      for (int v = n0; v > 0; v = p0[v]) chain0.push_back(v);
      std::reverse(chain0.begin(), chain0.end());
      for (int v = n1; v > 0; v = p1[v]) chain1.push_back(v);
      const size_t len = 1 + chain0.size() * (W - 1) + 1 + chain1.size() * (W - 1);
      lens[i] = len;
      path_k[i]->len = (int32_t)len;
      if ((size_t)path_k[i]->capacity < len || !path_k[i]->q) {
        status[i] = CP_E_CAPACITY;
        continue;
      }
      out_off[i] = total;
      total += (long)len * dof;
      int off = 1;
      for (int v : chain0) { items.insert(items.end(), {i, 0, v, 0, off}); off += W - 1; }
      items.insert(items.end(), {i, 1, n1, 2, off});
      off += 1;
      for (int v : chain1) { items.insert(items.end(), {i, 1, v, 1, off}); off += W - 1; }
    }
    if (total > 0) {
      float* d_out = nullptr;
      int* d_items = nullptr;
      long* d_off = nullptr;
      he = hipMalloc((void**)&d_out, sizeof(float) * total);
      if (he == hipSuccess) he = hipMalloc((void**)&d_items, sizeof(int) * items.size());
      if (he == hipSuccess) he = hipMalloc((void**)&d_off, sizeof(long) * n);
      if (he == hipSuccess) he = hipMemcpyAsync(d_items, items.data(), sizeof(int) * items.size(), hipMemcpyHostToDevice, st);
      if (he == hipSuccess) he = hipMemcpyAsync(d_off, out_off.data(), sizeof(long) * n, hipMemcpyHostToDevice, st);
      const int n_items = (int)items.size() / 5;
      if (he == hipSuccess && n_items > 0) {
        gather_batch_kernel<<<n_items, 64, 0, st>>>(b->probs, d_items, n_items, W, d_off, d_out);
        he = hipGetLastError();
      }
      std::vector<float> pts(total);
      if (he == hipSuccess) he = hipMemcpyAsync(pts.data(), d_out, sizeof(float) * total, hipMemcpyDeviceToHost, st);
      if (he == hipSuccess) he = hipStreamSynchronize(st);
      if (d_out) (void)hipFree(d_out);
      if (d_items) (void)hipFree(d_items);
      if (d_off) (void)hipFree(d_off);
      if (he != hipSuccess) return api_hip_fail(he, "cp_plan_batch gather");
      for (int i = 0; i < n; ++i) {
        if (status[i] != CP_OK || lens[i] == 0) continue;
        const int dof = probs[i].dof;
        const size_t len = lens[i];
        double* pq = path_k[i]->q;
        for (size_t r = 1; r + 1 < len; ++r)
          for (int j = 0; j < dof; ++j) pq[r * dof + j] = (double)pts[out_off[i] + r * dof + j];
        std::memcpy(pq, queries[i].start, sizeof(double) * dof);
        std::memcpy(pq + (len - 1) * dof, queries[i].goal, sizeof(double) * dof);
      }
    }
    // queries whose start and goal are within reach of each other
    for (int i = 0; i < n; ++i) {
      if (status[i] != CP_OK || lens[i] != 0) continue;
      const int dof = probs[i].dof;
      path_k[i]->len = 2;
      if (path_k[i]->capacity < 2 || !path_k[i]->q) { status[i] = CP_E_CAPACITY; continue; }
      std::memcpy(path_k[i]->q, queries[i].start, sizeof(double) * dof);
      std::memcpy(path_k[i]->q + dof, queries[i].goal, sizeof(double) * dof);
    }
    for (int k = 0; k < n; ++k) {
      status_out[perm[k]] = st_k[k];
      if (stats) stats[perm[k]] = stats_k[k];
    }
    return CP_OK;
  } catch (...) {
    return api_fail(CP_E_ARG, "cp_plan_batch: unexpected exception");
  }
}

}  // extern "C"

// gfx950 kernels of the hot path: fk_cc_batch, project_validate_motions
// (a projection kernel followed by a validation kernel on the same stream),
// project_configs.
//
// Validation (and fk_cc): a motion of W waypoints occupies W consecutive
// lanes of one wavefront (W = 64: one wavefront per motion, W = 32: two), so
// the collision flag is a ballot and needs neither LDS nor a barrier.
//
// Projection: a wavefront holds several motions in LDS and spreads only the
// waypoints that are still being projected over its lanes (project_pool_kernel);
// a one-motion-per-wavefront form (project_kernel) serves the sequential
// operator, whose waypoints wait for each other anyway.
//
// Projection and validation are separate kernels because their register
// needs differ: fused, the collision loop would run at the projection's
// occupancy.  The projected segment goes through HBM between them
// (W * dof * 4 bytes per motion, written anyway as the call's output).
#include "kernels.h"

#include <float.h>

#include <algorithm>

#include "collide.h"
#include "project.h"
#include "project_pool.h"

namespace cprrtc {

constexpr int kBlock = 256;

// ------------------------------------------------------------------ FK + CC, one configuration per lane

template <int B, bool SD>
__global__ __launch_bounds__(kBlock) void fk_cc_kernel(const RobotDev* __restrict__ rob,
                                                       const float4* __restrict__ sph, EnvDev env,
                                                       int n_cfg, const float* __restrict__ q,
                                                       uint8_t* __restrict__ collide,
                                                       float* __restrict__ min_sd, int early) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool on = i < n_cfg;
  const int dof = rob->dof;
  const float* qi = q + (on ? i : 0) * dof;
  uint64_t hits;
  float msd;
  CcWork cw;
  cc_work_clear(cw);
  collide_config<B, SD, false, false>(rob, sph, env, qi, on, 0ull, early != 0, hits, msd, cw);
  if (on) {
    collide[i] = (hits >> (threadIdx.x & 63)) & 1ull;
    if (SD) min_sd[i] = msd;
  }
}

// Scene check of a few configurations (a query's endpoints), one wavefront
// each, its lanes splitting the primitives (config_min_sd); same outputs as
// fk_cc_kernel<B, true> with every batch evaluated.
template <int B>
__global__ __launch_bounds__(64) void config_sd_kernel(const RobotDev* __restrict__ rob,
                                                       const float4* __restrict__ sph, EnvDev env,
                                                       int n_cfg, const float* __restrict__ q,
                                                       uint8_t* __restrict__ collide,
                                                       float* __restrict__ min_sd) {
  const int i = blockIdx.x;
  if (i >= n_cfg) return;
  const float sd = config_min_sd<B>(rob, sph, env, q + (int64_t)i * rob->dof);
  if (threadIdx.x == 0) {
    collide[i] = sd <= 0.0f ? 1 : 0;
    min_sd[i] = sd;
  }
}

// ------------------------------------------------------------------ sphere centres

// One thread per (configuration, sphere): the chain's frames up to the
// sphere's joint, then R c_local + p.  Consecutive threads write consecutive
// 12-byte centres, so the output (the bulk of the traffic) is coalesced.
__global__ __launch_bounds__(kBlock) void sphere_xyz_kernel(const RobotDev* __restrict__ rob,
                                                            const float4* __restrict__ sph,
                                                            const int2* __restrict__ map,
                                                            int n_spheres, int64_t n_items,
                                                            const float* __restrict__ q,
                                                            float* __restrict__ xyz) {
  const int dof = rob->dof;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < n_items; t += stride) {
    const int64_t i = t / n_spheres;
    const int s = (int)(t - i * n_spheres);
    const int2 m = map[s];
    const int c = (rob->n_chains > 1 && m.y >= rob->chain_begin[1]) ? 1 : 0;
    const float* qi = q + i * dof;
    Frame T;
    frame_from(T, rob->base[c]);
    for (int j = rob->chain_begin[c]; j <= m.y; ++j) joint_advance(T, rob, j, qi[j]);
    const float4 l = sph[m.x];
    float* o = xyz + t * 3;
    o[0] = T.r[0] * l.x + T.r[1] * l.y + T.r[2] * l.z + T.p[0];
    o[1] = T.r[3] * l.x + T.r[4] * l.y + T.r[5] * l.z + T.p[1];
    o[2] = T.r[6] * l.x + T.r[7] * l.y + T.r[8] * l.z + T.p[2];
  }
}

// ------------------------------------------------------------------ projection (Algorithm 1)

// One motion per W lanes (project_segment).  Writes the segment, status
// (0 = projected, 1 = projection failed) and the iteration count.
// MODE 0: start from the straight line.
// MODE 1: warm start, xi[k] = clamp(straight line + delta[motion][k-1]) for
//         k >= 1 (delta from the network, [n_motions][W-1][NDOF]).
// MODE 2: fallback, only motions whose status is 1 are projected again from
//         the straight line; their iterations are added to iters.
// MODE 3: the sequential projection (CP_PROJECT_SEQUENTIAL) from the
//         straight line; modes 0-2 run Algorithm 1 (with or without the
//         smoothing term, by prm.variant).
template <int NDOF, int KIND, int MODE>
__global__ __launch_bounds__(kBlock) void project_kernel(
    const RobotDev* __restrict__ rob, ConDev con, ProjDev prm, int n_motions,
    const float* __restrict__ q_from, const float* __restrict__ q_to,
    const float* __restrict__ delta, float* __restrict__ xi, int* __restrict__ status,
    int* __restrict__ iters, unsigned long long* __restrict__ work) {
  const int W = prm.W;
  const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t motion = gid / W;
  const int k = (int)(gid % W);
  if (motion >= n_motions) return;   // whole motion segments leave together
  if (MODE == 2 && status[motion] != 1) return;
  const int lane = threadIdx.x & 63;
  const int seg = lane - k;          // first lane of this motion in the wavefront
  const uint64_t wmask = (W == 64) ? ~0ull : ((1ull << W) - 1ull);
  const uint64_t segmask = wmask << seg;

  float q[NDOF];
  {
    const float s = (float)k / (float)(W - 1);
#pragma unroll
    for (int j = 0; j < NDOF; ++j) {
      const float a = q_from[motion * NDOF + j];
      const float b = q_to[motion * NDOF + j];
      q[j] = a + s * (b - a);
    }
    if (MODE == 1 && k >= 1) {
      const float* d = delta + (motion * (W - 1) + (k - 1)) * NDOF;
#pragma unroll
      for (int j = 0; j < NDOF; ++j) q[j] = fminf(fmaxf(q[j] + d[j], rob->lo[j]), rob->hi[j]);
    }
  }

  int it = 0;
  unsigned long long updates = 0;   // waypoint updates computed (lanes past prog, per iteration)
  const bool ok =
      MODE == 3 ? project_sequential<NDOF, KIND>(rob, con, prm, k, seg, false, q, it, updates)
                : project_segment<NDOF, KIND>(rob, con, prm, k, seg, wmask, segmask, false, q, it,
                                              updates);

  float* xk = xi + (motion * W + k) * NDOF;
#pragma unroll
  for (int j = 0; j < NDOF; ++j) xk[j] = q[j];
  if (k == 0) {
    status[motion] = ok ? 0 : 1;
    if (iters) iters[motion] = (MODE == 2 ? iters[motion] : 0) + it;
    if (work) atomicAdd(&work[6], updates);
  }
}

// Pooled projection kernel of the library (robot and mask read at run time);
// the body is in project_pool.h.
template <int NDOF, int KIND, int MODE, int S>
__global__ __launch_bounds__(64) void project_pool_kernel(
    const RobotDev* __restrict__ rob, ConDev con, ProjDev prm, int n_motions,
    const float* __restrict__ q_from, const float* __restrict__ q_to,
    const float* __restrict__ delta, float* __restrict__ xi, int* __restrict__ status,
    int* __restrict__ iters, unsigned long long* __restrict__ work) {
  project_pool_body<NDOF, KIND, MODE, S, RobotMem>(rob, con, prm, n_motions, q_from, q_to, delta,
                                                   xi, status, iters, work);
}

// ------------------------------------------------------------------ validation (FK + CC of projected segments)

// Waypoints 1..W-1 of every motion whose projection succeeded (status 0 from
// project_kernel) run FK + CC; the body is validate_body in collide.h.
template <int B, bool CULL>
__global__ __launch_bounds__(kBlock) void validate_kernel(
    const RobotDev* __restrict__ rob, const float4* __restrict__ sph, EnvDev env, int W,
    int n_motions, const float* __restrict__ xi, int* __restrict__ status,
    unsigned long long* __restrict__ work, int early) {
  validate_body<B, CULL, RobotMem>(rob, sph, env, W, n_motions, xi, status, work, early,
                                   (int64_t)blockIdx.x * kBlock + threadIdx.x);
}

// ------------------------------------------------------------------ self-collision

// Four configurations per wavefront, one per row of 16 lanes: the row runs
// its configuration's forward kinematics (the same value in its 16 lanes),
// places the sphere centres into LDS (sphere s by lane s mod 16 of the row),
// then tests the checked pairs 16 at a time:
// sd = |c_s - c_t| - r_s - r_t, colliding iff sd <= 0 (for the verdict
// alone, |c_s - c_t|^2 <= (r_s + r_t)^2 with the right-hand side stored
// with the pair, so only the centres' x, y, z are read).
//   pairs[p] = (s | t << 16, bits of (r_s + r_t)^2), s and t positions in
//   the link-grouped sphere array; n_entries records (a multiple of
//   kSelfPad) plus kSelfPad more, in groups of kU = kSelfPad / 16 records
//   sharing s (group g at (g / 16) kSelfPad + g % 16 + 16 u), so lane l of
//   a row reads c_s once per loop trip; records with (r_s + r_t)^2 = -1
//   fill groups and the list up: they never collide and the minimum skips
//   them.
//   MOTION = false: item i is configuration i of q; collide[i] |= hit and,
//                   with min_sd, min_sd[i] = min(min_sd[i], min pair sd)
//                   (every pair evaluated).
//   MOTION = true:  item i is waypoint 1 + i mod (W - 1) of motion
//                   i / (W - 1) in xi; motions whose status is not 0 are
//                   skipped; a hit sets the status to 2.
// A row without an item (the grid's tail, a motion already decided) runs
// its kinematics on a valid row of the input and reports nothing.  Up to
// four wavefronts per workgroup (fewer for robots with many spheres); LDS
// holds 4 x n_spheres float4 per wavefront.
constexpr int kSelfRow = 16;
constexpr int kSelfPerWave = 64 / kSelfRow;
static_assert(kSelfPad % kSelfRow == 0, "pairs are read a row at a time");
constexpr int kSelfWaves = 4;

template <bool MOTION>
__global__ __launch_bounds__(64 * kSelfWaves) void self_cc_kernel(
    const RobotDev* __restrict__ rob, const float4* __restrict__ sph,
    const int2* __restrict__ pairs, int n_entries, int64_t n_items, int W,
    const float* __restrict__ q_all, uint8_t* __restrict__ collide, float* __restrict__ min_sd,
    int* __restrict__ status, int early) {
  extern __shared__ float4 centres[];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane / kSelfRow, l = lane % kSelfRow;
  const int64_t first = ((int64_t)blockIdx.x * (blockDim.x >> 6) + w) * kSelfPerWave;
  if (first >= n_items) return;                   // wave-uniform
  const int64_t item = first + g;
  const int dof = rob->dof;
  bool on = item < n_items;
  int64_t motion = 0;
  const float* q;
  if (MOTION) {
    motion = on ? item / (W - 1) : 0;
    on = on && status[motion] == 0;               // failed or already colliding
    q = q_all + (on ? motion * W + 1 + item % (W - 1) : 1) * dof;
  } else {
    q = q_all + (on ? item : 0) * dof;
  }
  if (__ballot(on) == 0) return;
  const int n_sph = rob->n_spheres;
  float4* c = centres + (size_t)(w * kSelfPerWave + g) * n_sph;
  for (int ch = 0; ch < rob->n_chains; ++ch) {
    Frame T;
    frame_from(T, rob->base[ch]);
    for (int j = rob->chain_begin[ch]; j < rob->chain_begin[ch + 1]; ++j) {
      joint_advance(T, rob, j, q[j]);
      for (int s = rob->sph_begin[j] + l; s < rob->sph_begin[j + 1]; s += kSelfRow) {
        const float4 ls = sph[s];
        c[s] = make_float4(T.r[0] * ls.x + T.r[1] * ls.y + T.r[2] * ls.z + T.p[0],
                           T.r[3] * ls.x + T.r[4] * ls.y + T.r[5] * ls.z + T.p[1],
                           T.r[6] * ls.x + T.r[7] * ls.y + T.r[8] * ls.z + T.p[2], ls.w);
      }
    }
  }
  // the centres other lanes placed are read below: order the stores before
  // the loads (one wavefront, so a wavefront-scope fence suffices)
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const bool all_pairs = !MOTION && min_sd;
  const uint64_t row_bits = 0xFFFFull << (kSelfRow * g);
  const uint64_t off_rows = __ballot(!on);
  uint64_t acc = 0;                               // OR of every round's ballot (uniform)
  float msd = FLT_MAX;
  if (all_pairs) {
    for (int base = 0; base < n_entries; base += kSelfRow) {
      const int p = base + l;
      bool hit = false;
      if (on && p < n_entries) {
        const int2 pr = pairs[p];
        if (__int_as_float(pr.y) >= 0.0f) {          // not a filler
          const float4 a = c[pr.x & 0xFFFF], b = c[pr.x >> 16];
          const float dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
          const float sd = sqrtf(dx * dx + dy * dy + dz * dz) - (a.w + b.w);
          msd = fminf(msd, sd);
          hit = sd <= 0.0f;
        }
      }
      acc |= __ballot(hit);
    }
  } else {
    // the list is padded to a multiple of kSelfPad with pairs that never
    // hit, and a row without an item tests its own (finite) centres with its
    // bits ignored: no lane branches
    // the records of the next trip are loaded before this trip's centres
    // are read (the list has kSelfPad entries past its padded end for that)
    constexpr int kU = kSelfPad / kSelfRow;
    const int2* pb = pairs;                       // wavefront-uniform
    int2 next[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) next[u] = pb[u * kSelfRow + l];
    for (int base = 0; base < n_entries; base += kSelfPad) {
      int2 cur[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) cur[u] = next[u];
      pb += kSelfPad;
#pragma unroll
      for (int u = 0; u < kU; ++u) next[u] = pb[u * kSelfRow + l];
      // the lane's kU records of this trip share their first sphere
      const float4* ca = c + (cur[0].x & 0xFFFF);
      const float ax = ca->x, ay = ca->y, az = ca->z;
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int2 pr = cur[u];
        const float4* cb = c + (pr.x >> 16);
        const float dx = ax - cb->x, dy = ay - cb->y, dz = az - cb->z;
        acc |= __ballot(dx * dx + dy * dy + dz * dz <= __int_as_float(pr.y));
      }
      if (early) {
        // every row decided (a hit) or without an item
        const uint64_t x = acc | off_rows;
        const uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
        if ((lo & 0xFFFFu) && (lo >> 16) && (hi & 0xFFFFu) && (hi >> 16)) break;
      }
    }
  }
  const bool hit_any = (acc & row_bits) != 0;
  if (all_pairs) msd = row_min(msd);
  if (on && l == 0) {
    if (MOTION) {
      if (hit_any) status[motion] = 2;
    } else {
      if (hit_any) collide[item] = 1;
      if (all_pairs) min_sd[item] = fminf(min_sd[item], msd);
    }
  }
}

// Wavefronts per workgroup for a robot: LDS of at most 64 KiB per workgroup.
static int self_waves(int n_spheres) {
  const int per_wave = (int)sizeof(float4) * kSelfPerWave * n_spheres;
  return std::max(1, std::min(kSelfWaves, 65536 / per_wave));
}

hipError_t launch_self_cc(const RobotDev* rob, const RobotDev& host, const float4* sph,
                          const int2* pairs, int n_entries, int n_cfg, const float* q,
                          uint8_t* collide, float* min_sd, bool early, hipStream_t stream) {
  if (n_entries == 0 || n_cfg == 0) return hipSuccess;
  const int waves = self_waves(host.n_spheres);
  const size_t lds = sizeof(float4) * kSelfPerWave * waves * host.n_spheres;
  const int64_t per_block = (int64_t)kSelfPerWave * waves;
  const unsigned nb = (unsigned)((n_cfg + per_block - 1) / per_block);
  self_cc_kernel<false><<<nb, 64 * waves, lds, stream>>>(
      rob, sph, pairs, n_entries, n_cfg, 0, q, collide, min_sd, nullptr, early ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_self_cc_motions(const RobotDev* rob, const RobotDev& host, const float4* sph,
                                  const int2* pairs, int n_entries, int W, int n_motions,
                                  const float* xi, int* status, hipStream_t stream) {
  if (n_entries == 0 || n_motions == 0) return hipSuccess;
  const int waves = self_waves(host.n_spheres);
  const size_t lds = sizeof(float4) * kSelfPerWave * waves * host.n_spheres;
  const int64_t items = (int64_t)n_motions * (W - 1);
  const int64_t per_block = (int64_t)kSelfPerWave * waves;
  const unsigned nb = (unsigned)((items + per_block - 1) / per_block);
  self_cc_kernel<true><<<nb, 64 * waves, lds, stream>>>(
      rob, sph, pairs, n_entries, items, W, xi, nullptr, nullptr, status, 1);
  return hipGetLastError();
}

// ------------------------------------------------------------------ single configurations

template <int NDOF, int KIND>
__global__ __launch_bounds__(kBlock) void project_configs_kernel(
    const RobotDev* __restrict__ rob, ConDev con, int n, const float* __restrict__ q_in,
    float* __restrict__ q_out, int* __restrict__ status, float tol, int max_iters, float alpha,
    float lambda2) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  float q[NDOF];
#pragma unroll
  for (int j = 0; j < NDOF; ++j) q[j] = q_in[i * NDOF + j];
  int ok = 0;
  for (int it = 0; it <= max_iters; ++it) {
    float g[NDOF], einf;
    task_step<NDOF, KIND>(rob, con, q, lambda2, g, einf);
    if (einf < tol) {
      ok = 1;
      break;
    }
    if (it == max_iters) break;
#pragma unroll
    for (int j = 0; j < NDOF; ++j)
      q[j] = fminf(fmaxf(q[j] - alpha * g[j], rob->lo[j]), rob->hi[j]);
  }
#pragma unroll
  for (int j = 0; j < NDOF; ++j) q_out[i * NDOF + j] = q[j];
  status[i] = ok;
}

// ------------------------------------------------------------------ launchers

static unsigned blocks_for(int64_t threads) { return (unsigned)((threads + kBlock - 1) / kBlock); }

hipError_t launch_config_sd(const RobotDev* rob, const float4* sph, const EnvDev& env, int n_cfg,
                            const float* q, uint8_t* collide, float* min_sd, hipStream_t stream) {
  if (n_cfg <= 0) return hipSuccess;
  config_sd_kernel<4><<<n_cfg, 64, 0, stream>>>(rob, sph, env, n_cfg, q, collide, min_sd);
  return hipGetLastError();
}

hipError_t launch_fk_cc(const RobotDev* rob, const float4* sph, const EnvDev& env, int n_cfg,
                        const float* q, uint8_t* collide, float* min_sd, bool early, int batch,
                        hipStream_t stream) {
  const unsigned nb = blocks_for(n_cfg);
  if (min_sd) {
    fk_cc_kernel<4, true><<<nb, kBlock, 0, stream>>>(rob, sph, env, n_cfg, q, collide, min_sd, 0);
  } else if (batch == 4) {
    fk_cc_kernel<4, false><<<nb, kBlock, 0, stream>>>(rob, sph, env, n_cfg, q, collide, nullptr, early);
  } else {
    fk_cc_kernel<8, false><<<nb, kBlock, 0, stream>>>(rob, sph, env, n_cfg, q, collide, nullptr, early);
  }
  return hipGetLastError();
}

hipError_t launch_sphere_xyz(const RobotDev* rob, const float4* sph, const int2* map, int n_spheres,
                             int n_cfg, const float* q, float* xyz, hipStream_t stream) {
  const int64_t items = (int64_t)n_cfg * n_spheres;
  const unsigned nb = (unsigned)std::min<int64_t>(blocks_for(items), 1 << 20);   // grid-stride beyond
  sphere_xyz_kernel<<<nb, kBlock, 0, stream>>>(rob, sph, map, n_spheres, items, q, xyz);
  return hipGetLastError();
}

// Motions per pooled wavefront and the number of wavefronts.  Measured on
// the cluttered 65 536-motion batch: many short wavefronts that take their
// slots' motions once balance best (4 slots, one share of 4 motions per
// wavefront: 1.44 ms, 0.76 ms compiled for the robot; shares of 8: 1.54 /
// 0.83 ms; shares of 12: 1.76 / 0.88 ms; half the batch in shares of 8,
// the rest in shares of 4: 1.41 / 0.80 ms; 3 slots: 1.48 / 0.76 ms; 5
// slots: 1.53 / 0.96 ms; 6 slots: 1.67 / 1.05 ms; the
// one-motion-per-wavefront kernel: 2.53 ms).  Fewer slots leave LDS for
// more wavefronts per CU (4 x 64 x 7 floats: 22 workgroups), which hide
// the latency of each wavefront's scalar bookkeeping.
// Below this many motions the pooled form has too few wavefronts to fill the
// chip (fewer than 4 per SIMD) and one motion per wavefront is used.
constexpr int kPoolMinMotions = 24576;
unsigned pool_blocks(int n) {
  const int per = (n + kPoolSlots - 1) / kPoolSlots;
  return (unsigned)std::max(1, std::min(per, 256 * 64));
}
bool use_pool(int n, int pooled) { return pooled == 1 || (pooled < 0 && n >= kPoolMinMotions); }

template <int NDOF, int KIND>
static void launch_project_kind(int mode, int pooled, unsigned nb, hipStream_t stream,
                                const RobotDev* rob, const ConDev& con, const ProjDev& prm, int n,
                                const float* qf, const float* qt, const float* delta, float* xi,
                                int* st, int* it, unsigned long long* work) {
  const bool pool = mode != 3 && use_pool(n, pooled);
  if (!pool) {
    if (mode == 1)
      project_kernel<NDOF, KIND, 1><<<nb, kBlock, 0, stream>>>(rob, con, prm, n, qf, qt, delta, xi, st, it, work);
    else if (mode == 2)
      project_kernel<NDOF, KIND, 2><<<nb, kBlock, 0, stream>>>(rob, con, prm, n, qf, qt, delta, xi, st, it, work);
    else if (mode == 3)
      project_kernel<NDOF, KIND, 3><<<nb, kBlock, 0, stream>>>(rob, con, prm, n, qf, qt, delta, xi, st, it, work);
    else
      project_kernel<NDOF, KIND, 0><<<nb, kBlock, 0, stream>>>(rob, con, prm, n, qf, qt, delta, xi, st, it, work);
    return;
  }
  const unsigned np = pool_blocks(n);
  if (mode == 1)
    project_pool_kernel<NDOF, KIND, 1, kPoolSlots><<<np, 64, 0, stream>>>(rob, con, prm, n, qf, qt, delta, xi, st, it, work);
  else if (mode == 2)
    project_pool_kernel<NDOF, KIND, 2, kPoolSlots><<<np, 64, 0, stream>>>(rob, con, prm, n, qf, qt, delta, xi, st, it, work);
  else
    project_pool_kernel<NDOF, KIND, 0, kPoolSlots><<<np, 64, 0, stream>>>(rob, con, prm, n, qf, qt, delta, xi, st, it, work);
}

template <int NDOF>
static bool launch_project_ndof(int kind, int mode, int pooled, unsigned nb, hipStream_t stream,
                                const RobotDev* rob, const ConDev& con, const ProjDev& prm, int n,
                                const float* qf, const float* qt, const float* delta, float* xi,
                                int* st, int* it, unsigned long long* work) {
  switch (kind) {
    case KIND_NONE:
      launch_project_kind<NDOF, KIND_NONE>(mode, pooled, nb, stream, rob, con, prm, n, qf, qt, delta, xi, st, it, work);
      return true;
    case KIND_POSE:
      launch_project_kind<NDOF, KIND_POSE>(mode, pooled, nb, stream, rob, con, prm, n, qf, qt, delta, xi, st, it, work);
      return true;
    case KIND_REL:
      if constexpr (NDOF % 2 == 0) {
        launch_project_kind<NDOF, KIND_REL>(mode, pooled, nb, stream, rob, con, prm, n, qf, qt, delta, xi, st, it, work);
        return true;
      }
      return false;
  }
  return false;
}

bool dof_supported(int dof) {
  switch (dof) {
    case 2: case 3: case 6: case 7: case 9: case 14: return true;
    default: return false;
  }
}

hipError_t launch_project_mode(int dof, int mode, const RobotDev* rob, const ConDev& con,
                               const ProjDev& prm, int n_motions, const float* q_from,
                               const float* q_to, const float* delta, float* xi, int* status,
                               int* iters, unsigned long long* work, int pooled,
                               hipStream_t stream, bool* supported) {
  const unsigned nb = blocks_for((int64_t)n_motions * prm.W);
  bool ok = false;
  switch (dof) {
    case 2: ok = launch_project_ndof<2>(con.kind, mode, pooled, nb, stream, rob, con, prm, n_motions, q_from, q_to, delta, xi, status, iters, work); break;
    case 3: ok = launch_project_ndof<3>(con.kind, mode, pooled, nb, stream, rob, con, prm, n_motions, q_from, q_to, delta, xi, status, iters, work); break;
    case 6: ok = launch_project_ndof<6>(con.kind, mode, pooled, nb, stream, rob, con, prm, n_motions, q_from, q_to, delta, xi, status, iters, work); break;
    case 7: ok = launch_project_ndof<7>(con.kind, mode, pooled, nb, stream, rob, con, prm, n_motions, q_from, q_to, delta, xi, status, iters, work); break;
    case 9: ok = launch_project_ndof<9>(con.kind, mode, pooled, nb, stream, rob, con, prm, n_motions, q_from, q_to, delta, xi, status, iters, work); break;
    case 14: ok = launch_project_ndof<14>(con.kind, mode, pooled, nb, stream, rob, con, prm, n_motions, q_from, q_to, delta, xi, status, iters, work); break;
    default: ok = false;
  }
  *supported = ok;
  return ok ? hipGetLastError() : hipSuccess;
}

hipError_t launch_project(int dof, const RobotDev* rob, const ConDev& con, const ProjDev& prm,
                          int n_motions, const float* q_from, const float* q_to, float* xi,
                          int* status, int* iters, unsigned long long* work, int pooled,
                          hipStream_t stream, bool* supported) {
  return launch_project_mode(dof, prm.variant == CP_PROJECT_SEQUENTIAL ? 3 : 0, rob, con, prm,
                             n_motions, q_from, q_to, nullptr, xi, status, iters, work, pooled,
                             stream, supported);
}

hipError_t launch_validate(const RobotDev* rob, const float4* sph, const EnvDev& env, int W,
                           int n_motions, const float* xi, int* status, unsigned long long* work,
                           bool early, bool cull, int batch, hipStream_t stream) {
  const unsigned nb = blocks_for((int64_t)n_motions * W);
  const int e = early ? 1 : 0;
  if (cull) {
    if (batch == 4)
      validate_kernel<4, true><<<nb, kBlock, 0, stream>>>(rob, sph, env, W, n_motions, xi, status, work, e);
    else if (batch == 16)
      validate_kernel<16, true><<<nb, kBlock, 0, stream>>>(rob, sph, env, W, n_motions, xi, status, work, e);
    else
      validate_kernel<8, true><<<nb, kBlock, 0, stream>>>(rob, sph, env, W, n_motions, xi, status, work, e);
  } else {
    if (batch == 4)
      validate_kernel<4, false><<<nb, kBlock, 0, stream>>>(rob, sph, env, W, n_motions, xi, status, work, e);
    else if (batch == 16)
      validate_kernel<16, false><<<nb, kBlock, 0, stream>>>(rob, sph, env, W, n_motions, xi, status, work, e);
    else
      validate_kernel<8, false><<<nb, kBlock, 0, stream>>>(rob, sph, env, W, n_motions, xi, status, work, e);
  }
  return hipGetLastError();
}

template <int NDOF>
static bool launch_pc_kind(int kind, unsigned nb, hipStream_t stream, const RobotDev* rob,
                           const ConDev& con, int n, const float* qi, float* qo, int* st,
                           float tol, int max_iters, float alpha, float lambda2) {
  switch (kind) {
    case KIND_NONE: project_configs_kernel<NDOF, KIND_NONE><<<nb, kBlock, 0, stream>>>(rob, con, n, qi, qo, st, tol, max_iters, alpha, lambda2); return true;
    case KIND_POSE: project_configs_kernel<NDOF, KIND_POSE><<<nb, kBlock, 0, stream>>>(rob, con, n, qi, qo, st, tol, max_iters, alpha, lambda2); return true;
    case KIND_REL:
      if constexpr (NDOF % 2 == 0) {
        project_configs_kernel<NDOF, KIND_REL><<<nb, kBlock, 0, stream>>>(rob, con, n, qi, qo, st, tol, max_iters, alpha, lambda2);
        return true;
      }
      return false;
  }
  return false;
}

hipError_t launch_project_configs(int dof, const RobotDev* rob, const ConDev& con, int n,
                                  const float* q_in, float* q_out, int* status, float tol,
                                  int max_iters, float alpha, float lambda2, hipStream_t stream,
                                  bool* supported) {
  const unsigned nb = blocks_for(n);
  bool ok = false;
  switch (dof) {
    case 2: ok = launch_pc_kind<2>(con.kind, nb, stream, rob, con, n, q_in, q_out, status, tol, max_iters, alpha, lambda2); break;
    case 3: ok = launch_pc_kind<3>(con.kind, nb, stream, rob, con, n, q_in, q_out, status, tol, max_iters, alpha, lambda2); break;
    case 6: ok = launch_pc_kind<6>(con.kind, nb, stream, rob, con, n, q_in, q_out, status, tol, max_iters, alpha, lambda2); break;
    case 7: ok = launch_pc_kind<7>(con.kind, nb, stream, rob, con, n, q_in, q_out, status, tol, max_iters, alpha, lambda2); break;
    case 9: ok = launch_pc_kind<9>(con.kind, nb, stream, rob, con, n, q_in, q_out, status, tol, max_iters, alpha, lambda2); break;
    case 14: ok = launch_pc_kind<14>(con.kind, nb, stream, rob, con, n, q_in, q_out, status, tol, max_iters, alpha, lambda2); break;
    default: ok = false;
  }
  *supported = ok;
  return ok ? hipGetLastError() : hipSuccess;
}

}  // namespace cprrtc

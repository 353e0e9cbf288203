// Sphere-vs-primitive collision checking on gfx950 (paper Sections I and IV:
// every waypoint's robot collision spheres against every environment
// primitive; a collision found anywhere ends the motion early).
//
// One lane = one configuration.  The lane walks the chain joint by joint
// (runtime loop, joint rows via scalar loads), and for each link takes its
// spheres in batches of B: B sphere centres sit in VGPRs while primitives
// stream through SGPRs, so one scalar fetch feeds B pair tests.  Pair
// verdicts are gathered with ballots into a wave-wide bit mask held in SGPRs
// (one compare + one scalar OR per pair).  Between batches the wave polls the
// mask and leaves when the motion (or every lane) has collided.
//
// Two ways to choose the primitives a batch is tested against:
//  * all of them (fk_cc_batch: lanes hold unrelated configurations);
//  * culled (motions: the 64 lanes are consecutive waypoints of one short
//    segment, so their spheres occupy a compact region): the wave reduces the
//    batch's sphere boxes to one axis-aligned box, every lane tests 1/64 of the
//    primitives' bounding spheres against it, and only the ballot's set bits
//    are tested pair by pair.  A primitive whose bounding sphere is farther
//    than kCullMargin from the box cannot touch any sphere of the batch in any
//    lane, so the verdicts are those of the full test.
//
// A pair collides iff dist(centre, solid) <= r; the verdict form compares
// squared distances, the exact form computes dist - r and keeps its minimum.
//
// Instruction count is what bounds these loops (one scalar fetch feeds B
// spheres, so every saved vector instruction per pair shows), hence:
//  * an OBB is stored as its three axes with the centre's coordinate along
//    each (u.c) and its half extents, so the coordinate of a sphere centre
//    along an axis is one three-term dot product with u.c folded in;
//  * the square root is the hardware one (about 1 ulp, against the 1e-5 m
//    band the verdicts are held to);
//  * in the verdict form, when every sphere of the batch has r < 1 m, the
//    positive part max(x, 0) of a distance component becomes a clamp to
//    [0, 1] (an output modifier of the subtraction that forms it): a
//    component above 1 m gives d2 >= 1 > r^2 clamped or not.
#pragma once
#ifndef __HIPCC_RTC__
#include <float.h>
#endif
#ifndef FLT_MAX
#define FLT_MAX 3.402823466e+38F   // the run-time compiler has no <float.h>
#endif

#include "device.h"

namespace cprrtc {


// ------------------------------------------------------------------ single-primitive tests
// B sphere centres (per lane) against one primitive (uniform).  Verdict form
// ORs ballots into hits; exact form lowers msd.  CLAMP (verdict form only):
// every radius of the batch is below 1 m.

__device__ __forceinline__ float hw_sqrt(float x) {
#if __has_builtin(__builtin_amdgcn_sqrtf)
  return __builtin_amdgcn_sqrtf(x);
#else
  return sqrtf(x);
#endif
}

// Positive part of a distance component: max(x, 0), or clamp to [0, 1].
template <bool CLAMP>
__device__ __forceinline__ float pos_part(float x) {
  return CLAMP ? __builtin_amdgcn_fmed3f(x, 0.0f, 1.0f) : fmaxf(x, 0.0f);
}

template <int B, bool SD, bool CLAMP = false>
__device__ __forceinline__ void test_aabb(const float4 c, const float4 h, const float (&cx)[B],
                                          const float (&cy)[B], const float (&cz)[B],
                                          const float (&rad)[B], uint64_t& hits, float& msd) {
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const float ex = pos_part<CLAMP>(fabsf(cx[b] - c.x) - h.x);
    const float ey = pos_part<CLAMP>(fabsf(cy[b] - c.y) - h.y);
    const float ez = pos_part<CLAMP>(fabsf(cz[b] - c.z) - h.z);
    const float d2 = ex * ex + ey * ey + ez * ez;
    if (SD) msd = fminf(msd, hw_sqrt(d2) - rad[b]);
    else hits |= __ballot(d2 <= rad[b] * rad[b]);
  }
}

// o = (u.c, v.c, w.c): the box centre's coordinates along its axes; u, v, w
// the unit axes with the half extents in .w.
template <int B, bool SD, bool CLAMP = false>
__device__ __forceinline__ void test_obb(const float4 o, const float4 u, const float4 v,
                                         const float4 w, const float (&cx)[B],
                                         const float (&cy)[B], const float (&cz)[B],
                                         const float (&rad)[B], uint64_t& hits, float& msd) {
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const float pu = fmaf(u.x, cx[b], fmaf(u.y, cy[b], fmaf(u.z, cz[b], -o.x)));
    const float pv = fmaf(v.x, cx[b], fmaf(v.y, cy[b], fmaf(v.z, cz[b], -o.y)));
    const float pw = fmaf(w.x, cx[b], fmaf(w.y, cy[b], fmaf(w.z, cz[b], -o.z)));
    const float eu = pos_part<CLAMP>(fabsf(pu) - u.w);
    const float ev = pos_part<CLAMP>(fabsf(pv) - v.w);
    const float ew = pos_part<CLAMP>(fabsf(pw) - w.w);
    const float d2 = eu * eu + ev * ev + ew * ew;
    if (SD) msd = fminf(msd, hw_sqrt(d2) - rad[b]);
    else hits |= __ballot(d2 <= rad[b] * rad[b]);
  }
}

template <int B, bool SD>
__device__ __forceinline__ void test_sphere(const float4 s, const float (&cx)[B],
                                            const float (&cy)[B], const float (&cz)[B],
                                            const float (&rad)[B], uint64_t& hits, float& msd) {
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const float tx = cx[b] - s.x, ty = cy[b] - s.y, tz = cz[b] - s.z;
    const float d2 = tx * tx + ty * ty + tz * tz;
    if (SD) {
      msd = fminf(msd, fmaxf(hw_sqrt(d2) - s.w, 0.0f) - rad[b]);
    } else {
      const float reach = s.w + rad[b];
      hits |= __ballot(d2 <= reach * reach);
    }
  }
}

template <int B, bool SD>
__device__ __forceinline__ void test_capsule(const float4 p0, const float4 dv, const float (&cx)[B],
                                             const float (&cy)[B], const float (&cz)[B],
                                             const float (&rad)[B], uint64_t& hits, float& msd) {
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const float tx = cx[b] - p0.x, ty = cy[b] - p0.y, tz = cz[b] - p0.z;
    float s = (tx * dv.x + ty * dv.y + tz * dv.z) * dv.w;
    s = fminf(fmaxf(s, 0.0f), 1.0f);
    const float wx = tx - s * dv.x, wy = ty - s * dv.y, wz = tz - s * dv.z;
    const float d2 = wx * wx + wy * wy + wz * wz;
    if (SD) {
      msd = fminf(msd, fmaxf(hw_sqrt(d2) - p0.w, 0.0f) - rad[b]);
    } else {
      const float reach = p0.w + rad[b];
      hits |= __ballot(d2 <= reach * reach);
    }
  }
}

template <int B, bool SD, bool CLAMP = false>
__device__ __forceinline__ void test_cylinder(const float4 c, const float4 u, const float (&cx)[B],
                                              const float (&cy)[B], const float (&cz)[B],
                                              const float (&rad)[B], uint64_t& hits, float& msd) {
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const float tx = cx[b] - c.x, ty = cy[b] - c.y, tz = cz[b] - c.z;
    const float al = tx * u.x + ty * u.y + tz * u.z;
    const float wx = tx - al * u.x, wy = ty - al * u.y, wz = tz - al * u.z;
    const float da = pos_part<CLAMP>(fabsf(al) - c.w);
    const float dr = pos_part<CLAMP>(hw_sqrt(wx * wx + wy * wy + wz * wz) - u.w);
    const float d2 = da * da + dr * dr;
    if (SD) msd = fminf(msd, hw_sqrt(d2) - rad[b]);
    else hits |= __ballot(d2 <= rad[b] * rad[b]);
  }
}

// Is every radius of the batch below 1 m (wavefront-uniform)?
template <int B>
__device__ __forceinline__ bool small_radii(const float (&rad)[B]) {
  bool small = true;
#pragma unroll
  for (int b = 0; b < B; ++b) small = small && rad[b] < 1.0f;
  return small;
}

// ------------------------------------------------------------------ all primitives

template <int B, bool SD, bool CLAMP>
__device__ __forceinline__ void test_all_of(const EnvDev& env, const float (&cx)[B],
                                            const float (&cy)[B], const float (&cz)[B],
                                            const float (&rad)[B], uint64_t& hits, float& msd) {
  for (int i = 0; i < env.n_aabb; ++i)
    test_aabb<B, SD, CLAMP>(env.aabb[2 * i], env.aabb[2 * i + 1], cx, cy, cz, rad, hits, msd);
  for (int i = 0; i < env.n_obb; ++i)
    test_obb<B, SD, CLAMP>(env.obb[4 * i], env.obb[4 * i + 1], env.obb[4 * i + 2],
                           env.obb[4 * i + 3], cx, cy, cz, rad, hits, msd);
  for (int i = 0; i < env.n_sph; ++i) test_sphere<B, SD>(env.sph[i], cx, cy, cz, rad, hits, msd);
  for (int i = 0; i < env.n_cap; ++i)
    test_capsule<B, SD>(env.cap[2 * i], env.cap[2 * i + 1], cx, cy, cz, rad, hits, msd);
  for (int i = 0; i < env.n_cyl; ++i)
    test_cylinder<B, SD, CLAMP>(env.cyl[2 * i], env.cyl[2 * i + 1], cx, cy, cz, rad, hits, msd);
}

template <int B, bool SD>
__device__ __forceinline__ void test_all(const EnvDev& env, const float (&cx)[B],
                                         const float (&cy)[B], const float (&cz)[B],
                                         const float (&rad)[B], uint64_t& hits, float& msd) {
  if (!SD && small_radii<B>(rad)) test_all_of<B, SD, true>(env, cx, cy, cz, rad, hits, msd);
  else test_all_of<B, SD, false>(env, cx, cy, cz, rad, hits, msd);
}

// ------------------------------------------------------------------ culled primitives

// Wavefront reductions (every lane of the wavefront active; every lane gets
// the result).  Within each row of 16 lanes the partners come through DPP
// lane swizzles, which feed the min/max directly instead of going through
// the LDS crossbar: quad_perm [1,0,3,2] and [2,3,0,1] (partners 1 and 2
// apart), row_half_mirror (lane i of 8 with 7 - i) and row_mirror (lane i
// of 16 with 15 - i); then the four rows combine by shuffles 16 and 32 apart.
template <int CTRL>
__device__ __forceinline__ float dpp_partner(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
// Minimum over the lane's row of 16 lanes.
__device__ __forceinline__ float row_min(float v) {
  v = fminf(v, dpp_partner<0xB1>(v));
  v = fminf(v, dpp_partner<0x4E>(v));
  v = fminf(v, dpp_partner<0x141>(v));
  return fminf(v, dpp_partner<0x140>(v));
}
__device__ __forceinline__ float wave_min(float v) {
  v = row_min(v);
  v = fminf(v, __shfl_xor(v, 16, 64));
  return fminf(v, __shfl_xor(v, 32, 64));
}
__device__ __forceinline__ float wave_max(float v) {
  v = fmaxf(v, dpp_partner<0xB1>(v));
  v = fmaxf(v, dpp_partner<0x4E>(v));
  v = fmaxf(v, dpp_partner<0x141>(v));
  v = fmaxf(v, dpp_partner<0x140>(v));
  v = fmaxf(v, __shfl_xor(v, 16, 64));
  return fmaxf(v, __shfl_xor(v, 32, 64));
}

// Box of the batch's spheres over the counting lanes of the wave.
struct WaveBox {
  float lo[3], hi[3];
};

template <int B>
__device__ __forceinline__ WaveBox wave_box(const float (&cx)[B], const float (&cy)[B],
                                            const float (&cz)[B], const float (&rad)[B],
                                            bool lane_on) {
  float lx = FLT_MAX, ly = FLT_MAX, lz = FLT_MAX, hx = -FLT_MAX, hy = -FLT_MAX, hz = -FLT_MAX;
  if (lane_on) {
#pragma unroll
    for (int b = 0; b < B; ++b) {
      lx = fminf(lx, cx[b] - rad[b]); hx = fmaxf(hx, cx[b] + rad[b]);
      ly = fminf(ly, cy[b] - rad[b]); hy = fmaxf(hy, cy[b] + rad[b]);
      lz = fminf(lz, cz[b] - rad[b]); hz = fmaxf(hz, cz[b] + rad[b]);
    }
  }
  WaveBox box;
  box.lo[0] = wave_min(lx); box.lo[1] = wave_min(ly); box.lo[2] = wave_min(lz);
  box.hi[0] = wave_max(hx); box.hi[1] = wave_max(hy); box.hi[2] = wave_max(hz);
  return box;
}

// Does the bounding sphere come within kCullMargin of the box?  bs holds
// the centre and (radius + kCullMargin)^2.  med3(x, lo, hi) - x is the
// signed gap from x to the box along one axis (0 inside).
__device__ __forceinline__ bool near_box(const float4 bs, const WaveBox& box) {
  const float ex = __builtin_amdgcn_fmed3f(bs.x, box.lo[0], box.hi[0]) - bs.x;
  const float ey = __builtin_amdgcn_fmed3f(bs.y, box.lo[1], box.hi[1]) - bs.y;
  const float ez = __builtin_amdgcn_fmed3f(bs.z, box.lo[2], box.hi[2]) - bs.z;
  return ex * ex + ey * ey + ez * ez <= bs.w;
}

// Test the batch against the primitives whose bounding spheres come near
// `box`, all types in one pass: the bounding spheres are stored in type
// order (AABB, OBB, sphere, capsule, cylinder), so the active lanes share one
// loop over all of them (ceil(n / lanes) rounds rather than one or more per
// type; lanes are ranked among the active ones: with W = 32 one motion of the
// wavefront may already have left), the set bits of the ballot are walked in
// scalar registers, and each candidate goes to its type's pair test by its
// index (a wavefront-uniform branch).  Adds the candidates per type to
// count[].
template <int B, bool CLAMP>
__device__ __forceinline__ void test_culled_of(const EnvDev& env, const WaveBox& box,
                                               const float (&cx)[B], const float (&cy)[B],
                                               const float (&cz)[B], const float (&rad)[B],
                                               uint64_t& hits, int (&count)[5]) {
  const int lane = threadIdx.x & 63;
  const uint64_t act = __ballot(1);
  const int n_act = __popcll(act);
  const int rank = __popcll(act & ((1ull << lane) - 1ull));
  const int b1 = env.n_aabb, b2 = b1 + env.n_obb, b3 = b2 + env.n_sph, b4 = b3 + env.n_cap;
  const int n = b4 + env.n_cyl;
  float msd_unused = 0.0f;
  for (int base = 0; base < n; base += n_act) {
    const int i = base + rank;
    const bool cand = (i < n) && near_box(env.bound[min(i, n - 1)], box);
    uint64_t m = __ballot(cand);
    while (m) {
      const int l = __ffsll((unsigned long long)m) - 1;
      m &= m - 1;
      const int p = base + __popcll(act & ((1ull << l) - 1ull));
      if (p < b1) {
        ++count[0];
        test_aabb<B, false, CLAMP>(env.aabb[2 * p], env.aabb[2 * p + 1], cx, cy, cz, rad, hits,
                                   msd_unused);
      } else if (p < b2) {
        const int q = p - b1;
        ++count[1];
        test_obb<B, false, CLAMP>(env.obb[4 * q], env.obb[4 * q + 1], env.obb[4 * q + 2],
                                  env.obb[4 * q + 3], cx, cy, cz, rad, hits, msd_unused);
      } else if (p < b3) {
        ++count[2];
        test_sphere<B, false>(env.sph[p - b2], cx, cy, cz, rad, hits, msd_unused);
      } else if (p < b4) {
        const int q = p - b3;
        ++count[3];
        test_capsule<B, false>(env.cap[2 * q], env.cap[2 * q + 1], cx, cy, cz, rad, hits, msd_unused);
      } else {
        const int q = p - b4;
        ++count[4];
        test_cylinder<B, false, CLAMP>(env.cyl[2 * q], env.cyl[2 * q + 1], cx, cy, cz, rad, hits,
                                       msd_unused);
      }
    }
  }
}

template <int B>
__device__ __forceinline__ void test_culled_all(const EnvDev& env, const WaveBox& box,
                                                const float (&cx)[B], const float (&cy)[B],
                                                const float (&cz)[B], const float (&rad)[B],
                                                uint64_t& hits, int (&count)[5]) {
  if (small_radii<B>(rad)) test_culled_of<B, true>(env, box, cx, cy, cz, rad, hits, count);
  else test_culled_of<B, false>(env, box, cx, cy, cz, rad, hits, count);
}

// ------------------------------------------------------------------ one configuration per lane

// Work done by one wave, in units of one lane's work (what the work counters add up).
struct CcWork {
  unsigned long long pairs[5];     // pair tests per primitive type
  unsigned long long centres;      // sphere centres placed
  unsigned long long culls;        // bounding-sphere tests
};

__device__ __forceinline__ void cc_work_clear(CcWork& w) {
  for (int t = 0; t < 5; ++t) w.pairs[t] = 0;
  w.centres = 0;
  w.culls = 0;
}

// Collision state of one lane's configuration q (joint j at q[j]).
//   lane_on  the lane holds a configuration that counts
//   MOTION   stop once any counting lane of the segment `segmask` collided
//            (else once every counting lane has)
//   CULL     test only primitives near the wave's batch box
//   early    false: evaluate every batch
// hits_out: ballot mask of colliding counting lanes; msd_out (SD only).
// Control flow is wave-uniform except where W = 32 lets two motions of one
// wave leave at different batches (a box reduced while the other motion has
// left can only grow by stale lanes, which keeps the culling conservative).
template <int B, bool SD, bool MOTION, bool CULL, class P = RobotMem>
__device__ void collide_config(const RobotDev* __restrict__ rob, const float4* __restrict__ sph,
                               const EnvDev& env, const float* q, bool lane_on, uint64_t segmask,
                               bool early, uint64_t& hits_out, float& msd_out, CcWork& work) {
  uint64_t hits = 0;
  float msd = FLT_MAX;
  const uint64_t on_mask = __ballot(lane_on);
  const int n_on = __popcll(on_mask & (MOTION ? segmask : ~0ull));
  const int n_prims = env.n_aabb + env.n_obb + env.n_sph + env.n_cap + env.n_cyl;
  const int nch = P::n_chains(rob);
  for (int c = 0; c < nch; ++c) {
    Frame T;
    frame_from_p<P>(T, rob, c, false);
    const int j1 = P::chain_begin(rob, c + 1);
    for (int j = P::chain_begin(rob, c); j < j1; ++j) {
      joint_advance<P>(T, rob, j, q[j]);
      const int s1 = P::sph_begin(rob, j + 1);
      for (int s = P::sph_begin(rob, j); s < s1; s += B) {
        float cx[B], cy[B], cz[B], rr[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
          const float4 l = P::sphere(sph, min(s + b, s1 - 1));  // a short batch repeats its last sphere
          cx[b] = T.r[0] * l.x + T.r[1] * l.y + T.r[2] * l.z + T.p[0];
          cy[b] = T.r[3] * l.x + T.r[4] * l.y + T.r[5] * l.z + T.p[1];
          cz[b] = T.r[6] * l.x + T.r[7] * l.y + T.r[8] * l.z + T.p[2];
          rr[b] = l.w;
        }
        const int nb = min(B, s1 - s);
        work.centres += (unsigned long long)nb * n_on;
        if (CULL) {
          const WaveBox box = wave_box<B>(cx, cy, cz, rr, lane_on);
          int k[5] = {0, 0, 0, 0, 0};
          test_culled_all<B>(env, box, cx, cy, cz, rr, hits, k);
          const unsigned long long f = (unsigned long long)nb * n_on;
#pragma unroll
          for (int t = 0; t < 5; ++t) work.pairs[t] += k[t] * f;
          work.culls += n_prims;
        } else {
          test_all<B, SD>(env, cx, cy, cz, rr, hits, msd);
          const unsigned long long f = (unsigned long long)nb * n_on;
          work.pairs[0] += env.n_aabb * f; work.pairs[1] += env.n_obb * f;
          work.pairs[2] += env.n_sph * f; work.pairs[3] += env.n_cap * f;
          work.pairs[4] += env.n_cyl * f;
        }
        if (SD) hits = __ballot(msd <= 0.0f);
        if (early) {
          if (MOTION) {
            // the segment is done once it collided, or if none of its lanes counts
            if ((hits & on_mask & segmask) || !(on_mask & segmask)) goto done;
          } else {
            if ((on_mask & ~hits) == 0) goto done;
          }
        }
      }
    }
  }
done:
  hits_out = hits & on_mask;
  msd_out = msd;
}

// Minimum signed distance of one configuration (the same q in every lane
// of the wavefront) to the scene, the lanes splitting the primitives: lane l
// takes primitives l, l + 64, ... in type order against every sphere.  The
// minimum runs over the same pairs and pair values as collide_config's exact
// form, so it is the same number; a query's endpoints are checked this way
// instead of one lane walking the whole scene.  Every lane gets the result.
template <int B, class P = RobotMem>
__device__ float config_min_sd(const RobotDev* __restrict__ rob, const float4* __restrict__ sph,
                               const EnvDev& env, const float* q) {
  const int lane = threadIdx.x & 63;
  const int b1 = env.n_aabb, b2 = b1 + env.n_obb, b3 = b2 + env.n_sph, b4 = b3 + env.n_cap;
  const int n = b4 + env.n_cyl;
  float msd = FLT_MAX;
  uint64_t unused = 0;
  const int nch = P::n_chains(rob);
  for (int c = 0; c < nch; ++c) {
    Frame T;
    frame_from_p<P>(T, rob, c, false);
    const int j1 = P::chain_begin(rob, c + 1);
    for (int j = P::chain_begin(rob, c); j < j1; ++j) {
      joint_advance<P>(T, rob, j, q[j]);
      const int s1 = P::sph_begin(rob, j + 1);
      for (int s = P::sph_begin(rob, j); s < s1; s += B) {
        float cx[B], cy[B], cz[B], rr[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
          const float4 l = P::sphere(sph, min(s + b, s1 - 1));
          cx[b] = T.r[0] * l.x + T.r[1] * l.y + T.r[2] * l.z + T.p[0];
          cy[b] = T.r[3] * l.x + T.r[4] * l.y + T.r[5] * l.z + T.p[1];
          cz[b] = T.r[6] * l.x + T.r[7] * l.y + T.r[8] * l.z + T.p[2];
          rr[b] = l.w;
        }
        for (int p = lane; p < n; p += 64) {
          if (p < b1) {
            test_aabb<B, true>(env.aabb[2 * p], env.aabb[2 * p + 1], cx, cy, cz, rr, unused, msd);
          } else if (p < b2) {
            const int k = p - b1;
            test_obb<B, true>(env.obb[4 * k], env.obb[4 * k + 1], env.obb[4 * k + 2], env.obb[4 * k + 3],
                              cx, cy, cz, rr, unused, msd);
          } else if (p < b3) {
            test_sphere<B, true>(env.sph[p - b2], cx, cy, cz, rr, unused, msd);
          } else if (p < b4) {
            const int k = p - b3;
            test_capsule<B, true>(env.cap[2 * k], env.cap[2 * k + 1], cx, cy, cz, rr, unused, msd);
          } else {
            const int k = p - b4;
            test_cylinder<B, true>(env.cyl[2 * k], env.cyl[2 * k + 1], cx, cy, cz, rr, unused, msd);
          }
        }
      }
    }
  }
  return wave_min(msd);
}

// Validation of projected segments, thread gid of the launch: waypoints
// 1..W-1 of every motion whose projection succeeded (status 0) run FK + CC,
// one waypoint per lane; the motion leaves at the first batch in which any
// of its waypoints collides.  Status becomes 0 (valid) or 2 (collision).
// Shared by the library kernel (RobotMem) and kernels compiled at run time
// for one robot (a constant policy).
template <int B, bool CULL, class P>
__device__ __forceinline__ void validate_body(const RobotDev* __restrict__ rob,
                                              const float4* __restrict__ sph, const EnvDev& env,
                                              int W, int n_motions, const float* __restrict__ xi,
                                              int* __restrict__ status,
                                              unsigned long long* __restrict__ work, int early,
                                              int64_t gid) {
  const int64_t motion = gid / W;
  const int k = (int)(gid % W);
  const bool in_range = motion < n_motions;
  const bool checks = in_range && status[motion] == 0;
  if (__ballot(checks) == 0) return;   // wave-uniform: nothing to check here
  const int lane = threadIdx.x & 63;
  const int seg = lane - k;
  const uint64_t wmask = (W == 64) ? ~0ull : ((1ull << W) - 1ull);
  const uint64_t segmask = wmask << seg;
  const bool lane_on = checks && k >= 1;
  const float* q = xi + (in_range ? (motion * W + k) : 0) * rob->dof;
  uint64_t hits;
  float msd;
  CcWork cw;
  cc_work_clear(cw);
  collide_config<B, false, true, CULL, P>(rob, sph, env, q, lane_on, segmask, early != 0, hits,
                                          msd, cw);
  if (checks && k == 0) {
    status[motion] = (hits & segmask) ? 2 : 0;
    if (work) {
      for (int t = 0; t < 5; ++t) atomicAdd(&work[t], cw.pairs[t]);
      atomicAdd(&work[5], cw.centres);
      atomicAdd(&work[7], cw.culls);
    }
  }
}

}  // namespace cprrtc

// Sphere-vs-primitive collision checking on gfx950 (paper Sections I and IV:
// every waypoint's robot collision spheres against every environment
// primitive; a collision found anywhere ends the motion early).
//
// One lane = one configuration.  The lane walks the chain joint by joint
// (runtime loop, joint rows via scalar loads), and for each link takes its
// spheres in batches of B: B sphere centres sit in VGPRs while the loop over
// primitives streams each primitive once through SGPRs, so one scalar fetch
// feeds B pair tests.  Between batches the wave polls the batch's verdict with
// a ballot and leaves the loop when the motion (or every lane) has collided.
//
// A pair collides iff  dist(centre, solid) <= r.  The verdict form compares
// squared distances (no square root except the cylinder's radial distance);
// the exact form computes the signed distance dist - r itself and keeps its
// minimum.
#pragma once
#include <float.h>

#include "device.h"

namespace cprrtc {

template <int B, bool SD>
__device__ __forceinline__ void pair_tests(const EnvDev& env, const float (&cx)[B],
                                           const float (&cy)[B], const float (&cz)[B],
                                           const float (&rad)[B], bool& hit, float& msd) {
  float r2[B];
#pragma unroll
  for (int b = 0; b < B; ++b) r2[b] = rad[b] * rad[b];

#pragma unroll 1
  for (int i = 0; i < env.n_aabb; ++i) {
    const float4 c = env.aabb[2 * i], h = env.aabb[2 * i + 1];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const float ex = fmaxf(fabsf(cx[b] - c.x) - h.x, 0.0f);
      const float ey = fmaxf(fabsf(cy[b] - c.y) - h.y, 0.0f);
      const float ez = fmaxf(fabsf(cz[b] - c.z) - h.z, 0.0f);
      const float d2 = ex * ex + ey * ey + ez * ez;
      if (SD) msd = fminf(msd, sqrtf(d2) - rad[b]);
      else hit |= d2 <= r2[b];
    }
  }
#pragma unroll 1
  for (int i = 0; i < env.n_obb; ++i) {
    const float4 c = env.obb[4 * i], u = env.obb[4 * i + 1], v = env.obb[4 * i + 2],
                 w = env.obb[4 * i + 3];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const float tx = cx[b] - c.x, ty = cy[b] - c.y, tz = cz[b] - c.z;
      const float eu = fmaxf(fabsf(u.x * tx + u.y * ty + u.z * tz) - u.w, 0.0f);
      const float ev = fmaxf(fabsf(v.x * tx + v.y * ty + v.z * tz) - v.w, 0.0f);
      const float ew = fmaxf(fabsf(w.x * tx + w.y * ty + w.z * tz) - w.w, 0.0f);
      const float d2 = eu * eu + ev * ev + ew * ew;
      if (SD) msd = fminf(msd, sqrtf(d2) - rad[b]);
      else hit |= d2 <= r2[b];
    }
  }
#pragma unroll 1
  for (int i = 0; i < env.n_sph; ++i) {
    const float4 s = env.sph[i];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const float tx = cx[b] - s.x, ty = cy[b] - s.y, tz = cz[b] - s.z;
      const float d2 = tx * tx + ty * ty + tz * tz;
      if (SD) {
        msd = fminf(msd, fmaxf(sqrtf(d2) - s.w, 0.0f) - rad[b]);
      } else {
        const float reach = s.w + rad[b];
        hit |= d2 <= reach * reach;
      }
    }
  }
#pragma unroll 1
  for (int i = 0; i < env.n_cap; ++i) {
    const float4 p0 = env.cap[2 * i], dv = env.cap[2 * i + 1];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const float tx = cx[b] - p0.x, ty = cy[b] - p0.y, tz = cz[b] - p0.z;
      float s = (tx * dv.x + ty * dv.y + tz * dv.z) * dv.w;
      s = fminf(fmaxf(s, 0.0f), 1.0f);
      const float wx = tx - s * dv.x, wy = ty - s * dv.y, wz = tz - s * dv.z;
      const float d2 = wx * wx + wy * wy + wz * wz;
      if (SD) {
        msd = fminf(msd, fmaxf(sqrtf(d2) - p0.w, 0.0f) - rad[b]);
      } else {
        const float reach = p0.w + rad[b];
        hit |= d2 <= reach * reach;
      }
    }
  }
#pragma unroll 1
  for (int i = 0; i < env.n_cyl; ++i) {
    const float4 c = env.cyl[2 * i], u = env.cyl[2 * i + 1];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const float tx = cx[b] - c.x, ty = cy[b] - c.y, tz = cz[b] - c.z;
      const float al = tx * u.x + ty * u.y + tz * u.z;
      const float wx = tx - al * u.x, wy = ty - al * u.y, wz = tz - al * u.z;
      const float da = fmaxf(fabsf(al) - c.w, 0.0f);
      const float dr = fmaxf(sqrtf(wx * wx + wy * wy + wz * wz) - u.w, 0.0f);
      const float d2 = da * da + dr * dr;
      if (SD) msd = fminf(msd, sqrtf(d2) - rad[b]);
      else hit |= d2 <= r2[b];
    }
  }
}

// Collision state of one lane's configuration q (global memory, stride 1,
// joint j at q[j]).  lane_on = the lane holds a configuration that counts.
// MOTION: the wave stops once any counting lane of the motion's segment
// (bits `segmask` of the ballot) has collided; otherwise once every counting
// lane has.  early = false evaluates every pair.
// n_done: robot spheres whose tests against every primitive were evaluated
// (wave-uniform; a short batch counts only its real spheres).
template <int B, bool SD, bool MOTION>
__device__ void collide_config(const RobotDev* __restrict__ rob, const float4* __restrict__ sph,
                               const EnvDev& env, const float* q, bool lane_on, uint64_t segmask,
                               bool early, bool& hit_out, float& msd_out, int& n_done) {
  bool hit = false;
  float msd = FLT_MAX;
  n_done = 0;
  const int nch = rob->n_chains;
  for (int c = 0; c < nch; ++c) {
    Frame T;
    frame_from(T, rob->base[c]);
    const int j1 = rob->chain_begin[c + 1];
    for (int j = rob->chain_begin[c]; j < j1; ++j) {
      joint_advance(T, rob, j, q[j]);
      const int s1 = rob->sph_begin[j + 1];
      for (int s = rob->sph_begin[j]; s < s1; s += B) {
        float cx[B], cy[B], cz[B], rr[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
          const float4 l = sph[min(s + b, s1 - 1)];  // a short batch repeats its last sphere
          cx[b] = T.r[0] * l.x + T.r[1] * l.y + T.r[2] * l.z + T.p[0];
          cy[b] = T.r[3] * l.x + T.r[4] * l.y + T.r[5] * l.z + T.p[1];
          cz[b] = T.r[6] * l.x + T.r[7] * l.y + T.r[8] * l.z + T.p[2];
          rr[b] = l.w;
        }
        pair_tests<B, SD>(env, cx, cy, cz, rr, hit, msd);
        n_done += min(B, s1 - s);
        if (SD) hit = msd <= 0.0f;
        if (early) {
          if (MOTION) {
            if ((__ballot(hit && lane_on) & segmask) != 0) goto done;
          } else {
            if (__ballot(lane_on && !hit) == 0) goto done;
          }
        }
      }
    }
  }
done:
  hit_out = hit && lane_on;
  msd_out = msd;
}

}  // namespace cprrtc

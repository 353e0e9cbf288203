// Per-lane task error, task Jacobian and damped least-squares step
// (Algorithm 1, GetTaskError / GetTaskJacobian / J^+ E_task), all in VGPRs.
//
// The constrained pose and its error:
//   POSE: chain 0's end effector seen from the constraint frame,
//         R' = Rc^T R_ee, p' = Rc^T (p_ee - pc), x = (p', roll, pitch, yaw of R'),
//         e = x - target on the locked axes (angles wrapped);
//   REL:  end effector 2 seen from end effector 1, R' = R1^T R2,
//         p' = R1^T (p2 - p1), e = (p' - p*, roll/pitch/yaw of R*^T R').
// Jacobian columns come from the geometric Jacobian of each joint (revolute:
// v = z x (p_ee - o), w = z; prismatic: v = z, w = 0), rotated into the
// constraint frame, angular rows turned into roll/pitch/yaw rates.  The
// rates are read straight off the rotation matrix (cos pitch = |(R00, R10)|,
// sin pitch = -R20, yaw from R00/R10), so no trigonometry is needed there.
//
// Only the rows of locked axes are formed: the m x m system
// (J_m J_m^T + lambda^2 I) y_m = e_m is factored by an unrolled Cholesky in
// registers, with the free rows skipped by uniform branches on the mask.
#pragma once
#include "cprrtc.h"
#include "device.h"

namespace cprrtc {

__device__ __forceinline__ float wrap_pi(float x) {
  const float two_pi = 6.28318530717958647692f, inv_two_pi = 0.15915494309189533577f;
  return x - two_pi * floorf((x + 3.14159265358979323846f) * inv_two_pi);
}

// atan2 for the orientation error: t = min(|x|,|y|) / max(|x|,|y|) in [0, 1];
// above tan(pi/8) the identity atan t = pi/4 + atan((t - 1) / (t + 1)) brings
// the argument into [-tan(pi/8), tan(pi/8)], where the Taylor series of atan
// to z^15 is within 2e-8; the octant then follows from |y| > |x|, the sign of
// x and the sign of y.  Error about one unit in the last place of the result.
__device__ __forceinline__ float atan2_task(float y, float x) {
  const float ax = fabsf(x), ay = fabsf(y);
  const float mn = fminf(ax, ay), mx = fmaxf(ax, ay);
  const float t = mx > 0.0f ? mn * __builtin_amdgcn_rcpf(mx) : 0.0f;
  const bool big = t > 0.414213562373095049f;
  const float z = big ? (t - 1.0f) * __builtin_amdgcn_rcpf(t + 1.0f) : t;
  const float z2 = z * z;
  float p = fmaf(z2, -1.0f / 15.0f, 1.0f / 13.0f);
  p = fmaf(z2, p, -1.0f / 11.0f);
  p = fmaf(z2, p, 1.0f / 9.0f);
  p = fmaf(z2, p, -1.0f / 7.0f);
  p = fmaf(z2, p, 1.0f / 5.0f);
  p = fmaf(z2, p, -1.0f / 3.0f);
  p = fmaf(z2, p, 1.0f);
  float r = fmaf(z, p, big ? 0.785398163397448310f : 0.0f);
  if (ay > ax) r = 1.57079632679489662f - r;
  if (x < 0.0f) r = 3.14159265358979324f - r;
  return copysignf(r, y);
}

template <int NDOF, int KIND, class P = RobotMem>
__device__ __forceinline__ void task_step(const RobotDev* __restrict__ rob, const ConDev& con,
                                          const float (&q)[NDOF], float lambda2,
                                          float (&g)[NDOF], float& einf) {
  if (KIND == KIND_NONE) {
#pragma unroll
    for (int j = 0; j < NDOF; ++j) g[j] = 0.0f;
    einf = 0.0f;
    return;
  }
  // Locked axes.  The mask is the same for every lane, so the tests below
  // are uniform branches: rows of free axes are neither formed nor factored,
  // and the work is that of the m x m system of the locked axes.
  bool lock[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) lock[i] = P::lock(con, i);
  const bool any_ang = lock[3] || lock[4] || lock[5];

  // Forward kinematics: joint axes z_j and origins o_j, end effectors.
  float zx[NDOF], zy[NDOF], zz[NDOF], ox[NDOF], oy[NDOF], oz[NDOF];
  const int b1 = P::chain1(rob, NDOF);
  Frame T, ee0, ee1;
  frame_from_p<P>(T, rob, 0, false);
#pragma unroll
  for (int j = 0; j < NDOF; ++j) {
    if (j == b1) {
      frame_times_p<P>(T, rob, 0, ee0);
      frame_from_p<P>(T, rob, 1, false);
    }
    joint_advance<P>(T, rob, j, q[j]);
    zx[j] = T.r[2]; zy[j] = T.r[5]; zz[j] = T.r[8];
    ox[j] = T.p[0]; oy[j] = T.p[1]; oz[j] = T.p[2];
  }
  if (b1 < NDOF) frame_times_p<P>(T, rob, 1, ee1);
  else frame_times_p<P>(T, rob, 0, ee0);

  // Frame the error is measured in: A1 = rotation from world to the
  // reference (Rc^T or R1^T), P1 = reference origin, E = end effector.
  float A1[9], P1[3], Pe[3], pp[3];
  if (KIND == KIND_POSE) {
#pragma unroll
    for (int i = 0; i < 9; ++i) A1[i] = con.Rt[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) { P1[i] = con.pc[i]; Pe[i] = ee0.p[i]; }
  } else {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int c = 0; c < 3; ++c) A1[3 * i + c] = ee0.r[3 * c + i];
#pragma unroll
    for (int i = 0; i < 3; ++i) { P1[i] = ee0.p[i]; Pe[i] = ee1.p[i]; }
  }
  const Frame& E2 = (KIND == KIND_POSE) ? ee0 : ee1;
  // p' = A1 (Pe - P1)
  const float dPx = Pe[0] - P1[0], dPy = Pe[1] - P1[1], dPz = Pe[2] - P1[2];
#pragma unroll
  for (int i = 0; i < 3; ++i) pp[i] = A1[3 * i] * dPx + A1[3 * i + 1] * dPy + A1[3 * i + 2] * dPz;

  float e[6];
#pragma unroll
  for (int i = 0; i < 3; ++i) e[i] = lock[i] ? pp[i] - con.target[i] : 0.0f;
  e[3] = e[4] = e[5] = 0.0f;

  // Orientation: R' = A1 R_E2, the rotation whose roll/pitch/yaw is measured
  // (Re) and the matrix taking world angular velocity into its frame (Aw).
  float Aw[9], cy = 1.0f, sy = 0.0f, sp = 0.0f, inv_cp = 1.0f;
  if (any_ang) {
    float Rp[9], Re[9];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
        Rp[3 * i + c] = A1[3 * i] * E2.r[c] + A1[3 * i + 1] * E2.r[3 + c] + A1[3 * i + 2] * E2.r[6 + c];
    }
    if (KIND == KIND_POSE) {
#pragma unroll
      for (int i = 0; i < 9; ++i) { Re[i] = Rp[i]; Aw[i] = A1[i]; }
    } else {
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          Re[3 * i + c] = con.Rt[3 * i] * Rp[c] + con.Rt[3 * i + 1] * Rp[3 + c] + con.Rt[3 * i + 2] * Rp[6 + c];
          Aw[3 * i + c] = con.Rt[3 * i] * A1[c] + con.Rt[3 * i + 1] * A1[3 + c] + con.Rt[3 * i + 2] * A1[6 + c];
        }
    }
    const float cp = sqrtf(Re[0] * Re[0] + Re[3] * Re[3]);
    sp = -Re[6];
    inv_cp = __builtin_amdgcn_rcpf(cp);   // step direction only; decisions use e
    cy = Re[0] * inv_cp;
    sy = Re[3] * inv_cp;
    if (KIND == KIND_POSE) {
      if (lock[3]) e[3] = wrap_pi(atan2_task(Re[7], Re[8]) - con.target[3]);
      if (lock[4]) e[4] = wrap_pi(atan2_task(-Re[6], cp) - con.target[4]);
      if (lock[5]) e[5] = wrap_pi(atan2_task(Re[3], Re[0]) - con.target[5]);
    } else {
      if (lock[3]) e[3] = atan2_task(Re[7], Re[8]);
      if (lock[4]) e[4] = atan2_task(-Re[6], cp);
      if (lock[5]) e[5] = atan2_task(Re[3], Re[0]);
    }
  }
  einf = 0.0f;
#pragma unroll
  for (int i = 0; i < 6; ++i) einf = fmaxf(einf, fabsf(e[i]));

  // Jacobian rows of the locked axes.
  float J[6][NDOF];
  const float d21x = Pe[0] - P1[0], d21y = Pe[1] - P1[1], d21z = Pe[2] - P1[2];
#pragma unroll
  for (int j = 0; j < NDOF; ++j) {
    const bool first = j < b1;   // joint moves end effector 1 (REL) / the constrained one (POSE)
    const bool pri = P::prismatic(rob, j);
    float vx, vy, vz, wx, wy, wz;
    const bool at1 = KIND == KIND_REL && first;
    const float tx = at1 ? P1[0] : Pe[0], ty = at1 ? P1[1] : Pe[1], tz = at1 ? P1[2] : Pe[2];
    if (pri) {
      vx = zx[j]; vy = zy[j]; vz = zz[j];
      wx = wy = wz = 0.0f;
    } else {
      const float rx = tx - ox[j], ry = ty - oy[j], rz = tz - oz[j];
      vx = zy[j] * rz - zz[j] * ry;
      vy = zz[j] * rx - zx[j] * rz;
      vz = zx[j] * ry - zy[j] * rx;
      wx = zx[j]; wy = zy[j]; wz = zz[j];
    }
    float sgn = 1.0f;
    if (KIND == KIND_REL && first) {
      // d p' = R1^T (-v1 + (p2 - p1) x w1), omega_err = -Aw w1
      const float cxp = d21y * wz - d21z * wy, cyp = d21z * wx - d21x * wz,
                  czp = d21x * wy - d21y * wx;
      vx = cxp - vx; vy = cyp - vy; vz = czp - vz;
      sgn = -1.0f;
    }
    const bool moves = !(KIND == KIND_POSE && !first);
#pragma unroll
    for (int i = 0; i < 3; ++i)
      if (lock[i]) J[i][j] = moves ? A1[3 * i] * vx + A1[3 * i + 1] * vy + A1[3 * i + 2] * vz : 0.0f;
    if (any_ang) {
      const float da0 = sgn * (Aw[0] * wx + Aw[1] * wy + Aw[2] * wz);
      const float da1 = sgn * (Aw[3] * wx + Aw[4] * wy + Aw[5] * wz);
      const float da2 = sgn * (Aw[6] * wx + Aw[7] * wy + Aw[8] * wz);
      const float rr = (cy * da0 + sy * da1) * inv_cp;
      if (lock[3]) J[3][j] = moves ? rr : 0.0f;
      if (lock[4]) J[4][j] = moves ? cy * da1 - sy * da0 : 0.0f;
      if (lock[5]) J[5][j] = moves ? da2 + sp * rr : 0.0f;
    }
  }

  // (J J^T + lambda^2 I) y = e over the locked rows by Cholesky, g = J^T y.
  // Entries that involve a free row are never read.
  float L[6][6], inv_diag[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    if (!lock[c]) continue;
    float s = lambda2;
#pragma unroll
    for (int j = 0; j < NDOF; ++j) s += J[c][j] * J[c][j];
#pragma unroll
    for (int k = 0; k < c; ++k)
      if (lock[k]) s -= L[c][k] * L[c][k];
    inv_diag[c] = __builtin_amdgcn_rsqf(s);   // 1 / L[c][c]
#pragma unroll
    for (int r = c + 1; r < 6; ++r) {
      if (!lock[r]) continue;
      float t = 0.0f;
#pragma unroll
      for (int j = 0; j < NDOF; ++j) t += J[r][j] * J[c][j];
#pragma unroll
      for (int k = 0; k < c; ++k)
        if (lock[k]) t -= L[r][k] * L[c][k];
      L[r][c] = t * inv_diag[c];
    }
  }
  float z[6], y[6];
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    if (!lock[r]) continue;
    float s = e[r];
#pragma unroll
    for (int k = 0; k < r; ++k)
      if (lock[k]) s -= L[r][k] * z[k];
    z[r] = s * inv_diag[r];
  }
#pragma unroll
  for (int r = 5; r >= 0; --r) {
    if (!lock[r]) continue;
    float s = z[r];
#pragma unroll
    for (int k = r + 1; k < 6; ++k)
      if (lock[k]) s -= L[k][r] * y[k];
    y[r] = s * inv_diag[r];
  }
#pragma unroll
  for (int j = 0; j < NDOF; ++j) g[j] = 0.0f;
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    if (!lock[a]) continue;
#pragma unroll
    for (int j = 0; j < NDOF; ++j) g[j] += J[a][j] * y[a];
  }
}

// Algorithm 1 on the W-lane segment this lane belongs to (Jacobi form).
// q: this lane's waypoint xi[k]; in: the straight-line value, out: the
// projected value (success) or the last iterate.  Each active lane computes its
// update from the snapshot (its own xi[k] and xi[k-1] from a shuffle before
// anyone writes); validity is gathered with one ballot; prog moves to the end
// of the contiguous valid run after it; only lanes past the new prog take
// their new value.  `idle` lanes (outside any motion) count as valid so that
// their segment finishes at once.  Returns true on success; iters = iterations
// used (max_iters on failure); updates += waypoint updates computed.
// One waypoint update of Algorithm 1 from the snapshot: q = xi[k], qprev =
// xi[k-1].  qn receives the new value (task step, smoothing term unless the
// operator is the independent one, clamp to the limits); returns the
// waypoint's validity at q (task error and spacing).
template <int NDOF, int KIND, class P = RobotMem>
__device__ __forceinline__ bool waypoint_update(const RobotDev* __restrict__ rob, const ConDev& con,
                                                const ProjDev& prm, const float (&q)[NDOF],
                                                const float (&qprev)[NDOF], float (&qn)[NDOF]) {
  float g[NDOF], einf;
  task_step<NDOF, KIND, P>(rob, con, q, prm.lambda2, g, einf);
  float d2 = 0.0f, dl[NDOF];
#pragma unroll
  for (int j = 0; j < NDOF; ++j) {
    dl[j] = q[j] - qprev[j];
    d2 += dl[j] * dl[j];
  }
  const float esm = sqrtf(d2) - prm.tau;
  const float wsm = prm.variant == CP_PROJECT_INDEPENDENT ? 0.0f : esm;   // smoothing term
#pragma unroll
  for (int j = 0; j < NDOF; ++j)
    qn[j] = fminf(fmaxf(q[j] - prm.alpha * (g[j] + dl[j] * wsm), P::lo(rob, j)), P::hi(rob, j));
  return (einf < prm.tau_task) && (esm < prm.tau_sm);
}

// Algorithm 1 on the W-lane segment this lane belongs to (Jacobi form).
// q: this lane's waypoint xi[k]; in: the straight-line value, out: the
// projected value (success) or the last iterate.  Each active lane computes its
// update from the snapshot (its own xi[k] and xi[k-1] from a shuffle before
// anyone writes); validity is gathered with one ballot; prog moves to the end
// of the contiguous valid run after it; only lanes past the new prog take
// their new value.  `idle` lanes (outside any motion) count as valid so that
// their segment finishes at once.  Returns true on success; iters = iterations
// used (max_iters on failure); updates += waypoint updates computed.
template <int NDOF, int KIND, class P = RobotMem>
__device__ __forceinline__ bool project_segment(const RobotDev* __restrict__ rob, const ConDev& con,
                                                const ProjDev& prm, int k, int seg,
                                                uint64_t wmask, uint64_t segmask, bool idle,
                                                float (&q)[NDOF], int& iters,
                                                unsigned long long& updates) {
  const int W = prm.W;
  int prog = 0;
  for (int it = 1; it <= prm.max_iters; ++it) {
    updates += (unsigned long long)(W - 1 - prog);
    float qprev[NDOF];
#pragma unroll
    for (int j = 0; j < NDOF; ++j) qprev[j] = __shfl_up(q[j], 1, W);
    float qn[NDOF];
    const bool ok = waypoint_update<NDOF, KIND, P>(rob, con, prm, q, qprev, qn);
    const bool valid = idle || (k <= prog) || ok;
    const uint64_t bits = (__ballot(valid) & segmask) >> seg;
    const uint64_t invalid = ~bits & wmask;      // bits 0..prog are set
    prog = invalid ? (__ffsll((unsigned long long)invalid) - 2) : W - 1;
    if (prog == W - 1) {
      iters = it;
      return true;
    }
    if (k > prog) {
#pragma unroll
      for (int j = 0; j < NDOF; ++j) q[j] = qn[j];
    }
  }
  iters = prm.max_iters;
  return false;
}

// Sequential projection of the segment (CP_PROJECT_SEQUENTIAL): for
// k = 1..W-1 in turn, lane k starts from the projected waypoint k-1 plus one
// interpolation step (its straight-line value minus lane k-1's) and takes
// damped least-squares steps, without the smoothing term, until its task
// error and its spacing to waypoint k-1 are valid (checked before each step),
// at most max_iters steps.  The other lanes of the segment wait.  q: in, the
// straight-line value of this lane's waypoint; out, the projected value.
// iters: steps summed over the waypoints (max_iters for each waypoint that
// failed and every waypoint after it); updates += single-waypoint steps.
template <int NDOF, int KIND>
__device__ __forceinline__ bool project_sequential(const RobotDev* __restrict__ rob,
                                                   const ConDev& con, const ProjDev& prm, int k,
                                                   int seg, bool idle, float (&q)[NDOF],
                                                   int& iters, unsigned long long& updates) {
  const int W = prm.W;
  float step[NDOF];
#pragma unroll
  for (int j = 0; j < NDOF; ++j) step[j] = q[j] - __shfl_up(q[j], 1, W);
  int total = 0;
  bool failed = false;   // this lane's segment has a waypoint that did not project
  for (int kk = 1; kk < W; ++kk) {
    // every lane runs every trip, so the shuffles always read active lanes
    float prev[NDOF];
#pragma unroll
    for (int j = 0; j < NDOF; ++j) prev[j] = __shfl(q[j], seg + kk - 1, 64);
    int used = 0;
    bool valid = true;
    if (k == kk && !failed && !idle) {
#pragma unroll
      for (int j = 0; j < NDOF; ++j) q[j] = prev[j] + step[j];
      valid = false;
      for (int it = 1; it <= prm.max_iters; ++it) {
        float g[NDOF], einf;
        task_step<NDOF, KIND>(rob, con, q, prm.lambda2, g, einf);
        float d2 = 0.0f;
#pragma unroll
        for (int j = 0; j < NDOF; ++j) d2 += (q[j] - prev[j]) * (q[j] - prev[j]);
        const float esm = sqrtf(d2) - prm.tau;
        used = it;
        if (einf < prm.tau_task && esm < prm.tau_sm) {
          valid = true;
          break;
        }
#pragma unroll
        for (int j = 0; j < NDOF; ++j)
          q[j] = fminf(fmaxf(q[j] - prm.alpha * g[j], rob->lo[j]), rob->hi[j]);
      }
    }
    // lane seg + kk decided for its segment
    const bool seg_ok = __shfl(valid ? 1 : 0, seg + kk, 64) != 0;
    const int seg_used = __shfl(used, seg + kk, 64);
    if (!failed) total += seg_used;
    if (!seg_ok) failed = true;
    if (__ballot(!failed && !idle) == 0) break;   // uniform: no segment left to project
  }
  iters = total;
  updates += (unsigned long long)total;
  return !failed;
}

}  // namespace cprrtc

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
// Free axes are handled by zeroing their error and Jacobian rows and putting
// 1 (instead of lambda^2) on their diagonal: the 6x6 system
// (J J^T + D) y = e then leaves y = 0 on those rows, which is exactly the
// step of the reduced m x m system (J_m J_m^T + lambda^2 I) y_m = e_m, also
// for lambda = 0.  The factorisation is an unrolled Cholesky in registers.
#pragma once
#include "device.h"

namespace cprrtc {

__device__ __forceinline__ float wrap_pi(float x) {
  const float two_pi = 6.28318530717958647692f;
  return x - two_pi * floorf((x + 3.14159265358979323846f) / two_pi);
}

template <int NDOF, int KIND>
__device__ __forceinline__ void task_step(const RobotDev* __restrict__ rob, const ConDev& con,
                                          const float (&q)[NDOF], float lambda2,
                                          float (&g)[NDOF], float& einf) {
  if (KIND == KIND_NONE) {
#pragma unroll
    for (int j = 0; j < NDOF; ++j) g[j] = 0.0f;
    einf = 0.0f;
    return;
  }
  // Forward kinematics: joint axes z_j and origins o_j, end effectors.
  float zx[NDOF], zy[NDOF], zz[NDOF], ox[NDOF], oy[NDOF], oz[NDOF];
  const int b1 = rob->n_chains > 1 ? rob->chain_begin[1] : NDOF;
  Frame T, ee0, ee1;
  frame_from(T, rob->base[0]);
#pragma unroll
  for (int j = 0; j < NDOF; ++j) {
    if (j == b1) {
      frame_times(T, rob->tool[0], ee0);
      frame_from(T, rob->base[1]);
    }
    joint_advance(T, rob, j, q[j]);
    zx[j] = T.r[2]; zy[j] = T.r[5]; zz[j] = T.r[8];
    ox[j] = T.p[0]; oy[j] = T.p[1]; oz[j] = T.p[2];
  }
  if (b1 < NDOF) frame_times(T, rob->tool[1], ee1);
  else frame_times(T, rob->tool[0], ee0);

  // Frame the error is measured in: A1 = rotation from world to the
  // reference (Rc^T or R1^T), P1 = reference origin, E = end effector.
  float A1[9], P1[3], Pe[3], Rp[9], pp[3];
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
  // R' = A1 * R_E2, p' = A1 (Pe - P1)
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
      Rp[3 * i + c] = A1[3 * i] * E2.r[c] + A1[3 * i + 1] * E2.r[3 + c] + A1[3 * i + 2] * E2.r[6 + c];
  }
  const float dPx = Pe[0] - P1[0], dPy = Pe[1] - P1[1], dPz = Pe[2] - P1[2];
#pragma unroll
  for (int i = 0; i < 3; ++i) pp[i] = A1[3 * i] * dPx + A1[3 * i + 1] * dPy + A1[3 * i + 2] * dPz;

  // Rotation whose roll/pitch/yaw is measured, and the matrix taking world
  // angular velocity into its frame (Aw).
  float Re[9], Aw[9];
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
  const float sp = -Re[6];
  const float inv_cp = 1.0f / cp;
  const float cy = Re[0] * inv_cp, sy = Re[3] * inv_cp;
  const float roll = atan2f(Re[7], Re[8]);
  const float pitch = atan2f(-Re[6], cp);
  const float yaw = atan2f(Re[3], Re[0]);

  float e[6];
  if (KIND == KIND_POSE) {
    e[0] = pp[0] - con.target[0];
    e[1] = pp[1] - con.target[1];
    e[2] = pp[2] - con.target[2];
    e[3] = wrap_pi(roll - con.target[3]);
    e[4] = wrap_pi(pitch - con.target[4]);
    e[5] = wrap_pi(yaw - con.target[5]);
  } else {
    e[0] = pp[0] - con.target[0];
    e[1] = pp[1] - con.target[1];
    e[2] = pp[2] - con.target[2];
    e[3] = roll;
    e[4] = pitch;
    e[5] = yaw;
  }
  einf = 0.0f;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    e[i] *= con.mask[i];
    einf = fmaxf(einf, fabsf(e[i]));
  }

  // Jacobian columns.
  float J[6][NDOF];
  const float d21x = Pe[0] - P1[0], d21y = Pe[1] - P1[1], d21z = Pe[2] - P1[2];
#pragma unroll
  for (int j = 0; j < NDOF; ++j) {
    const bool first = j < b1;   // joint moves end effector 1 (REL) / the constrained one (POSE)
    const bool pri = rob->prismatic[j] != 0;
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
    if (KIND == KIND_POSE && !first) {
      vx = vy = vz = wx = wy = wz = 0.0f;
    }
    const float dp0 = A1[0] * vx + A1[1] * vy + A1[2] * vz;
    const float dp1 = A1[3] * vx + A1[4] * vy + A1[5] * vz;
    const float dp2 = A1[6] * vx + A1[7] * vy + A1[8] * vz;
    const float da0 = sgn * (Aw[0] * wx + Aw[1] * wy + Aw[2] * wz);
    const float da1 = sgn * (Aw[3] * wx + Aw[4] * wy + Aw[5] * wz);
    const float da2 = sgn * (Aw[6] * wx + Aw[7] * wy + Aw[8] * wz);
    const float rr = (cy * da0 + sy * da1) * inv_cp;
    const float pr = cy * da1 - sy * da0;
    const float yr = da2 + sp * rr;
    J[0][j] = dp0 * con.mask[0];
    J[1][j] = dp1 * con.mask[1];
    J[2][j] = dp2 * con.mask[2];
    J[3][j] = rr * con.mask[3];
    J[4][j] = pr * con.mask[4];
    J[5][j] = yr * con.mask[5];
  }

  // (J J^T + lambda^2 I) y = e by Cholesky, g = J^T y.
  float M[6][6];
#pragma unroll
  for (int a = 0; a < 6; ++a)
#pragma unroll
    for (int b = 0; b <= a; ++b) {
      float s = (a == b) ? (con.mask[a] != 0.0f ? lambda2 : 1.0f) : 0.0f;
#pragma unroll
      for (int j = 0; j < NDOF; ++j) s += J[a][j] * J[b][j];
      M[a][b] = s;
    }
  float L[6][6], inv_diag[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    float s = M[c][c];
#pragma unroll
    for (int k = 0; k < c; ++k) s -= L[c][k] * L[c][k];
    const float l = sqrtf(s);
    L[c][c] = l;
    inv_diag[c] = 1.0f / l;
#pragma unroll
    for (int r = c + 1; r < 6; ++r) {
      float t = M[r][c];
#pragma unroll
      for (int k = 0; k < c; ++k) t -= L[r][k] * L[c][k];
      L[r][c] = t * inv_diag[c];
    }
  }
  float z[6], y[6];
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    float s = e[r];
#pragma unroll
    for (int k = 0; k < r; ++k) s -= L[r][k] * z[k];
    z[r] = s * inv_diag[r];
  }
#pragma unroll
  for (int r = 5; r >= 0; --r) {
    float s = z[r];
#pragma unroll
    for (int k = r + 1; k < 6; ++k) s -= L[k][r] * y[k];
    y[r] = s * inv_diag[r];
  }
#pragma unroll
  for (int j = 0; j < NDOF; ++j) {
    float s = 0.0f;
#pragma unroll
    for (int a = 0; a < 6; ++a) s += J[a][j] * y[a];
    g[j] = s;
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
template <int NDOF, int KIND>
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
    float g[NDOF], einf;
    task_step<NDOF, KIND>(rob, con, q, prm.lambda2, g, einf);
    float d2 = 0.0f, dl[NDOF];
#pragma unroll
    for (int j = 0; j < NDOF; ++j) {
      dl[j] = q[j] - qprev[j];
      d2 += dl[j] * dl[j];
    }
    const float esm = sqrtf(d2) - prm.tau;
    float qn[NDOF];
#pragma unroll
    for (int j = 0; j < NDOF; ++j)
      qn[j] = fminf(fmaxf(q[j] - prm.alpha * (g[j] + dl[j] * esm), rob->lo[j]), rob->hi[j]);
    const bool valid = idle || (k <= prog) || ((einf < prm.tau_task) && (esm < prm.tau_sm));
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

}  // namespace cprrtc

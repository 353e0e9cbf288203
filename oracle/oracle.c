/* FP64 CPU oracle for cpRRTC's constrained motion projection and validation.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg; never by the HIP library.
 *
 * Paper: "cpRRTC: GPU-Parallel RRT-Connect for Constrained Motion Planning"
 * (Hu, Wang, Christensen, arXiv 2505.06791).
 *   - Section III (GPU-Parallel Project Operation on Motion): a motion is a
 *     fixed number of straight-line waypoints from q_near; it is projected onto
 *     the constraint manifold with the start fixed and the end free, then every
 *     waypoint runs forward kinematics and collision checking.
 *   - Section III-A, Algorithm 1 (ParallelProject): per-waypoint task error,
 *     task Jacobian, pseudo-inverse step, smoothing error/Jacobian/step,
 *     update from a shared snapshot, validity flag, progress over the valid
 *     prefix, early return or None after max_iters.
 *   - Section IV (intra-block communication): a collision anywhere invalidates
 *     the motion; the early exit only skips work, so this plain version checks
 *     everything and takes the same verdict.
 * Readings where the paper is silent (index base of prog, contiguous prefix,
 * norms, thresholds, damping, clamping) are listed at each use.
 */
#include "oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXDOF 32
#define MAXM 6

/* ---------------------------------------------------------------- 4x4 algebra */

static void mat4_identity(double* T) {
  memset(T, 0, 16 * sizeof(double));
  T[0] = T[5] = T[10] = T[15] = 1.0;
}

static void mat4_mul(const double* A, const double* B, double* C) {
  double t[16];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      double s = 0.0;
      for (int k = 0; k < 4; ++k) s += A[i * 4 + k] * B[k * 4 + j];
      t[i * 4 + j] = s;
    }
  memcpy(C, t, sizeof t);
}

static void rot_x(double ang, double* T) {
  mat4_identity(T);
  T[5] = cos(ang); T[6] = -sin(ang);
  T[9] = sin(ang); T[10] = cos(ang);
}

static void rot_z(double ang, double* T) {
  mat4_identity(T);
  T[0] = cos(ang); T[1] = -sin(ang);
  T[4] = sin(ang); T[5] = cos(ang);
}

static void trans_x(double v, double* T) { mat4_identity(T); T[3] = v; }
static void trans_z(double v, double* T) { mat4_identity(T); T[11] = v; }

/* Rotation block R (3x3 row-major) and translation p of a 4x4. */
static void mat4_split(const double* T, double R[9], double p[3]) {
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) R[i * 3 + j] = T[i * 4 + j];
    p[i] = T[i * 4 + 3];
  }
}

static void mat3_mul(const double* A, const double* B, double* C) {
  double t[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += A[i * 3 + k] * B[k * 3 + j];
      t[i * 3 + j] = s;
    }
  memcpy(C, t, sizeof t);
}

static void mat3_transpose(const double* A, double* B) {
  double t[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) t[j * 3 + i] = A[i * 3 + j];
  memcpy(B, t, sizeof t);
}

static void mat3_vec(const double* A, const double* v, double* out) {
  double t[3];
  for (int i = 0; i < 3; ++i) t[i] = A[i * 3 + 0] * v[0] + A[i * 3 + 1] * v[1] + A[i * 3 + 2] * v[2];
  memcpy(out, t, sizeof t);
}

static void cross3(const double* a, const double* b, double* out) {
  double t[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
  memcpy(out, t, sizeof t);
}

static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static double norm3(const double* a) { return sqrt(dot3(a, a)); }

/* Angle difference wrapped into (-pi, pi]. */
static double wrap_angle(double x) {
  double y = fmod(x + M_PI, 2.0 * M_PI);
  if (y < 0) y += 2.0 * M_PI;
  y -= M_PI;
  if (y <= -M_PI) y += 2.0 * M_PI;
  return y;
}

/* ---------------------------------------------------------------- kinematics */

/* Forward kinematics of the serial chain(s), modified Denavit-Hartenberg
 * (Craig):  T_i = RotX(alpha_{i-1}) TransX(a_{i-1}) RotZ(theta_i) TransZ(d_i),
 * revolute joints add q_i to theta_i, prismatic joints add q_i to d_i; frame i
 * of chain c is Base_c T_1 ... T_i and the end effector is that of the last
 * joint of the chain times Tool_c.  (Section III: "forward kinematics" per
 * waypoint; the chain model itself is not given by the paper.) */
void or_fk(const or_robot* r, const double* q, double* frames, double* ee) {
  double run[2][16];
  for (int c = 0; c < r->n_chains; ++c) memcpy(run[c], r->base + 16 * c, sizeof run[c]);
  for (int i = 0; i < r->dof; ++i) {
    const int c = r->chain[i];
    double theta = r->theta[i], d = r->d[i];
    if (r->type[i] == OR_REVOLUTE) theta += q[i]; else d += q[i];
    double A[16], B[16], C[16], D[16], T[16];
    rot_x(r->alpha[i], A);
    trans_x(r->a[i], B);
    rot_z(theta, C);
    trans_z(d, D);
    mat4_mul(A, B, T);
    mat4_mul(T, C, T);
    mat4_mul(T, D, T);
    mat4_mul(run[c], T, run[c]);
    if (frames) memcpy(frames + 16 * i, run[c], sizeof run[c]);
  }
  if (ee)
    for (int c = 0; c < r->n_chains; ++c) mat4_mul(run[c], r->tool + 16 * c, ee + 16 * c);
}

/* Roll-pitch-yaw of R = Rz(yaw) Ry(pitch) Rx(roll). */
static void rpy_of(const double* R, double rpy[3]) {
  rpy[0] = atan2(R[7], R[8]);
  rpy[1] = atan2(-R[6], sqrt(R[0] * R[0] + R[3] * R[3]));
  rpy[2] = atan2(R[3], R[0]);
}

/* E maps roll/pitch/yaw rates to the spatial angular velocity of
 * Rz(y) Ry(p) Rx(r):  omega = yaw' z + pitch' Rz(y) y + roll' Rz(y) Ry(p) x. */
static void rpy_rate_matrix(const double rpy[3], double E[9]) {
  const double cp = cos(rpy[1]), sp = sin(rpy[1]), cy = cos(rpy[2]), sy = sin(rpy[2]);
  const double M[9] = {cy * cp, -sy, 0.0,
                       sy * cp, cy, 0.0,
                       -sp, 0.0, 1.0};
  memcpy(E, M, sizeof M);
}

/* Solve the 3x3 system E x = b by Cramer's rule. */
static void solve3(const double* E, const double* b, double* x) {
  const double det = E[0] * (E[4] * E[8] - E[5] * E[7]) - E[1] * (E[3] * E[8] - E[5] * E[6]) +
                     E[2] * (E[3] * E[7] - E[4] * E[6]);
  for (int col = 0; col < 3; ++col) {
    double M[9];
    memcpy(M, E, sizeof M);
    for (int row = 0; row < 3; ++row) M[row * 3 + col] = b[row];
    x[col] = (M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
              M[2] * (M[3] * M[7] - M[4] * M[6])) / det;
  }
}

int32_t or_task_dim(const or_constraint* c) {
  if (c->kind == OR_CON_NONE) return 0;
  int m = 0;
  for (int j = 0; j < 6; ++j) m += c->mask[j] != 0;
  return m;
}

/* Pose the constraint acts on, as (R', p'):
 *   POSE:     end effector of chain 0 seen from the constraint frame,
 *             R' = Rc^T R_ee, p' = Rc^T (p_ee - p_c);
 *   REL_POSE: end effector 2 seen from end effector 1,
 *             R' = R1^T R2, p' = R1^T (p2 - p1).
 * (Evaluation section: constraints lock linear and angular end-effector axes,
 * a plane locks one axis, a line two, fixed orientation the angular ones.) */
static void constrained_pose(const or_robot* r, const or_constraint* c, const double* ee,
                             double Rp[9], double pp[3]) {
  double R1[9], p1[3], R2[9], p2[3], R1t[9], d[3];
  if (c->kind == OR_CON_REL_POSE) {
    mat4_split(ee, R1, p1);
    mat4_split(ee + 16, R2, p2);
  } else {
    mat4_split(c->frame, R1, p1);
    mat4_split(ee, R2, p2);
  }
  (void)r;
  mat3_transpose(R1, R1t);
  mat3_mul(R1t, R2, Rp);
  for (int i = 0; i < 3; ++i) d[i] = p2[i] - p1[i];
  mat3_vec(R1t, d, pp);
}

/* Six task coordinates: position, then roll/pitch/yaw.  For REL_POSE the
 * angular part is the roll/pitch/yaw of the rotation error R*^T R'. */
static void task_coords_from_ee(const or_robot* r, const or_constraint* c, const double* ee,
                                double x6[6], double Rerr[9]) {
  double Rp[9], pp[3];
  constrained_pose(r, c, ee, Rp, pp);
  if (c->kind == OR_CON_REL_POSE) {
    double Rs[9], ps[3], Rst[9];
    mat4_split(c->rel_target, Rs, ps);
    mat3_transpose(Rs, Rst);
    mat3_mul(Rst, Rp, Rerr);
  } else {
    memcpy(Rerr, Rp, sizeof(double) * 9);
  }
  x6[0] = pp[0]; x6[1] = pp[1]; x6[2] = pp[2];
  rpy_of(Rerr, x6 + 3);
}

void or_task_coords(const or_robot* r, const or_constraint* c, const double* q, double* x6) {
  double ee[32], Rerr[9];
  or_fk(r, q, NULL, ee);
  task_coords_from_ee(r, c, ee, x6, Rerr);
}

/* Task error E_task (Algorithm 1, GetTaskError): the locked coordinates minus
 * their targets, angles wrapped into (-pi, pi].  REL_POSE targets are folded
 * into the rotation error, so its angular target is 0 and its positional
 * target is p* = rel_target's translation. */
static int32_t task_error_from_ee(const or_robot* r, const or_constraint* c, const double* ee,
                                  double* e) {
  if (c->kind == OR_CON_NONE) return 0;
  double x6[6], Rerr[9], tgt[6];
  task_coords_from_ee(r, c, ee, x6, Rerr);
  if (c->kind == OR_CON_REL_POSE) {
    tgt[0] = c->rel_target[3]; tgt[1] = c->rel_target[7]; tgt[2] = c->rel_target[11];
    tgt[3] = tgt[4] = tgt[5] = 0.0;
  } else {
    memcpy(tgt, c->target, sizeof tgt);
  }
  int m = 0;
  for (int j = 0; j < 6; ++j) {
    if (!c->mask[j]) continue;
    const double diff = x6[j] - tgt[j];
    e[m++] = (j >= 3) ? wrap_angle(diff) : diff;
  }
  return m;
}

int32_t or_task_error(const or_robot* r, const or_constraint* c, const double* q, double* e) {
  double ee[32];
  or_fk(r, q, NULL, ee);
  return task_error_from_ee(r, c, ee, e);
}

/* Task Jacobian J_task (Algorithm 1, GetTaskJacobian): derivative of the task
 * error with respect to q, from the geometric Jacobian of each joint
 * (revolute: v = z_i x (p_ee - p_i), w = z_i; prismatic: v = z_i, w = 0),
 * expressed in the constraint frame, angular rows mapped to roll/pitch/yaw
 * rates through E^{-1}.  Row-major [m][dof]. */
int32_t or_task_jacobian(const or_robot* r, const or_constraint* c, const double* q, double* J) {
  if (c->kind == OR_CON_NONE) return 0;
  const int n = r->dof;
  double frames[MAXDOF * 16], ee[32], x6[6], Rerr[9], E[9];
  or_fk(r, q, frames, ee);
  task_coords_from_ee(r, c, ee, x6, Rerr);
  rpy_rate_matrix(x6 + 3, E);

  double R1[9], p1[3], R2[9], p2[3], R1t[9], Rs[9], ps[3], Rst[9], A[9];
  if (c->kind == OR_CON_REL_POSE) {
    mat4_split(ee, R1, p1);
    mat4_split(ee + 16, R2, p2);
    mat4_split(c->rel_target, Rs, ps);
    mat3_transpose(Rs, Rst);
  } else {
    mat4_split(c->frame, R1, p1);     /* the constraint frame plays arm 1 */
    mat4_split(ee, R2, p2);
    for (int i = 0; i < 9; ++i) Rst[i] = (i % 4 == 0) ? 1.0 : 0.0;
    (void)Rs; (void)ps;
  }
  mat3_transpose(R1, R1t);
  mat3_mul(Rst, R1t, A);              /* maps world angular velocity into the error frame */

  double col6[MAXDOF][6];
  for (int i = 0; i < n; ++i) {
    const int ch = r->chain[i];
    double Ri[9], pi[3], z[3], v[3], w[3];
    mat4_split(frames + 16 * i, Ri, pi);
    z[0] = Ri[2]; z[1] = Ri[5]; z[2] = Ri[8];
    double pe[3];
    if (c->kind == OR_CON_REL_POSE) {
      memcpy(pe, ch == 0 ? p1 : p2, sizeof pe);
    } else {
      memcpy(pe, p2, sizeof pe);
    }
    if (r->type[i] == OR_REVOLUTE) {
      double rel[3] = {pe[0] - pi[0], pe[1] - pi[1], pe[2] - pi[2]};
      cross3(z, rel, v);
      memcpy(w, z, sizeof w);
    } else {
      memcpy(v, z, sizeof v);
      w[0] = w[1] = w[2] = 0.0;
    }
    double dpos[3], dang[3];
    if (c->kind == OR_CON_REL_POSE) {
      if (ch == 0) {
        /* moving end effector 1: d p' = R1^T (-v1 + (p2 - p1) x w1), omega_err = -A w1 */
        double d21[3] = {p2[0] - p1[0], p2[1] - p1[1], p2[2] - p1[2]}, t[3];
        cross3(d21, w, t);
        double u[3] = {-v[0] + t[0], -v[1] + t[1], -v[2] + t[2]};
        mat3_vec(R1t, u, dpos);
        double mw[3] = {-w[0], -w[1], -w[2]};
        mat3_vec(A, mw, dang);
      } else {
        mat3_vec(R1t, v, dpos);
        mat3_vec(A, w, dang);
      }
    } else if (ch == 0) {
      mat3_vec(R1t, v, dpos);
      mat3_vec(A, w, dang);
    } else {
      dpos[0] = dpos[1] = dpos[2] = dang[0] = dang[1] = dang[2] = 0.0;
    }
    double rates[3];
    solve3(E, dang, rates);
    col6[i][0] = dpos[0]; col6[i][1] = dpos[1]; col6[i][2] = dpos[2];
    col6[i][3] = rates[0]; col6[i][4] = rates[1]; col6[i][5] = rates[2];
  }
  int m = 0;
  for (int j = 0; j < 6; ++j) {
    if (!c->mask[j]) continue;
    for (int i = 0; i < n; ++i) J[m * n + i] = col6[i][j];
    ++m;
  }
  return m;
}

/* Task step nabla_task = J^+ E_task (Algorithm 1), read as the damped
 * least-squares step g = J^T (J J^T + lambda^2 I)^{-1} e, the system solved by
 * Cholesky factorisation.  m = 0 gives g = 0. */
void or_dls_step(const double* J, const double* e, int32_t m, int32_t n, double lambda, double* g) {
  double A[MAXM * MAXM], L[MAXM * MAXM], z[MAXM], y[MAXM];
  for (int i = 0; i < n; ++i) g[i] = 0.0;
  if (m == 0) return;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      double s = 0.0;
      for (int k = 0; k < n; ++k) s += J[i * n + k] * J[j * n + k];
      A[i * m + j] = s + (i == j ? lambda * lambda : 0.0);
    }
  memset(L, 0, sizeof L);
  for (int j = 0; j < m; ++j) {
    double s = A[j * m + j];
    for (int k = 0; k < j; ++k) s -= L[j * m + k] * L[j * m + k];
    L[j * m + j] = sqrt(s);
    for (int i = j + 1; i < m; ++i) {
      double t = A[i * m + j];
      for (int k = 0; k < j; ++k) t -= L[i * m + k] * L[j * m + k];
      L[i * m + j] = t / L[j * m + j];
    }
  }
  for (int i = 0; i < m; ++i) {
    double s = e[i];
    for (int k = 0; k < i; ++k) s -= L[i * m + k] * z[k];
    z[i] = s / L[i * m + i];
  }
  for (int i = m - 1; i >= 0; --i) {
    double s = z[i];
    for (int k = i + 1; k < m; ++k) s -= L[k * m + i] * y[k];
    y[i] = s / L[i * m + i];
  }
  for (int k = 0; k < n; ++k) {
    double s = 0.0;
    for (int i = 0; i < m; ++i) s += J[i * n + k] * y[i];
    g[k] = s;
  }
}

/* ---------------------------------------------------------------- geometry */
/* Signed distance of a robot sphere (centre c, radius r) to a solid
 * primitive: the Euclidean distance from c to the primitive's point set
 * (0 inside it) minus r.  A pair collides when this is <= 0.  (Sections I and
 * IV: robot collision spheres are checked against environment primitives.) */

double or_sd_aabb(const double* c, double r, const double* box) {
  double u[3];
  for (int k = 0; k < 3; ++k) u[k] = fmax(fabs(c[k] - box[k]) - box[3 + k], 0.0);
  return norm3(u) - r;
}

double or_sd_obb(const double* c, double r, const double* box) {
  /* coordinates of c in the box frame: R^T (c - centre) */
  const double* R = box + 3;
  double t[3] = {c[0] - box[0], c[1] - box[1], c[2] - box[2]}, loc[3], u[3];
  for (int k = 0; k < 3; ++k) loc[k] = R[0 * 3 + k] * t[0] + R[1 * 3 + k] * t[1] + R[2 * 3 + k] * t[2];
  for (int k = 0; k < 3; ++k) u[k] = fmax(fabs(loc[k]) - box[12 + k], 0.0);
  return norm3(u) - r;
}

double or_sd_sphere(const double* c, double r, const double* s) {
  double t[3] = {c[0] - s[0], c[1] - s[1], c[2] - s[2]};
  return fmax(norm3(t) - s[3], 0.0) - r;
}

double or_sd_capsule(const double* c, double r, const double* cap) {
  const double d[3] = {cap[3] - cap[0], cap[4] - cap[1], cap[5] - cap[2]};
  const double t[3] = {c[0] - cap[0], c[1] - cap[1], c[2] - cap[2]};
  const double dd = dot3(d, d);
  double s = dd > 0.0 ? dot3(t, d) / dd : 0.0;
  s = fmin(fmax(s, 0.0), 1.0);
  const double w[3] = {t[0] - s * d[0], t[1] - s * d[1], t[2] - s * d[2]};
  return fmax(norm3(w) - cap[6], 0.0) - r;
}

double or_sd_cylinder(const double* c, double r, const double* cyl) {
  const double* u = cyl + 3;
  const double t[3] = {c[0] - cyl[0], c[1] - cyl[1], c[2] - cyl[2]};
  const double along = dot3(t, u);
  const double w[3] = {t[0] - along * u[0], t[1] - along * u[1], t[2] - along * u[2]};
  const double radial = norm3(w);
  const double da = fmax(fabs(along) - cyl[6], 0.0);
  const double dr = fmax(radial - cyl[7], 0.0);
  return sqrt(da * da + dr * dr) - r;
}

void or_sphere_centres(const or_robot* r, const double* q, double* xyz) {
  double frames[MAXDOF * 16];
  or_fk(r, q, frames, NULL);
  for (int s = 0; s < r->n_spheres; ++s) {
    const double* T = frames + 16 * r->sphere_link[s];
    const double* l = r->sphere + 4 * s;
    for (int i = 0; i < 3; ++i)
      xyz[3 * s + i] = T[i * 4 + 0] * l[0] + T[i * 4 + 1] * l[1] + T[i * 4 + 2] * l[2] + T[i * 4 + 3];
  }
}

/* Minimum signed distance over every (robot sphere, primitive) pair. */
double or_config_min_sd(const or_robot* r, const or_env* env, const double* q) {
  double* xyz = (double*)malloc(sizeof(double) * 3 * (r->n_spheres + 1));
  or_sphere_centres(r, q, xyz);
  double best = DBL_MAX;
  for (int s = 0; s < r->n_spheres; ++s) {
    const double* c = xyz + 3 * s;
    const double rad = r->sphere[4 * s + 3];
    for (int i = 0; i < env->n_aabb; ++i) best = fmin(best, or_sd_aabb(c, rad, env->aabb + 6 * i));
    for (int i = 0; i < env->n_obb; ++i) best = fmin(best, or_sd_obb(c, rad, env->obb + 15 * i));
    for (int i = 0; i < env->n_sphere; ++i) best = fmin(best, or_sd_sphere(c, rad, env->sphere + 4 * i));
    for (int i = 0; i < env->n_capsule; ++i) best = fmin(best, or_sd_capsule(c, rad, env->capsule + 7 * i));
    for (int i = 0; i < env->n_cylinder; ++i) best = fmin(best, or_sd_cylinder(c, rad, env->cylinder + 8 * i));
  }
  free(xyz);
  return best;
}

static int clamp_threads(int32_t n) { return n > 0 ? n : 1; }

/* ---------------------------------------------------------------- self-collision */

/* Candidate pair by the link rule (before the home-clearance test). */
static int self_candidate(const or_robot* r, int s, int t) {
  const int ls = r->sphere_link[s], lt = r->sphere_link[t];
  if (r->chain[ls] != r->chain[lt]) return 1;
  return abs(ls - lt) >= 2;
}

static double self_pair_sd(const or_robot* r, const double* xyz, int s, int t) {
  const double dx = xyz[3 * s] - xyz[3 * t];
  const double dy = xyz[3 * s + 1] - xyz[3 * t + 1];
  const double dz = xyz[3 * s + 2] - xyz[3 * t + 2];
  return sqrt(dx * dx + dy * dy + dz * dz) - r->sphere[4 * s + 3] - r->sphere[4 * t + 3];
}

int32_t or_self_pairs(const or_robot* r, int32_t capacity, int32_t* pairs) {
  double home[MAXDOF];
  for (int j = 0; j < r->dof; ++j) home[j] = fmin(fmax(0.0, r->lo[j]), r->hi[j]);
  double* xyz = (double*)malloc(sizeof(double) * 3 * (r->n_spheres + 1));
  or_sphere_centres(r, home, xyz);
  int32_t count = 0;
  for (int s = 0; s < r->n_spheres; ++s)
    for (int t = s + 1; t < r->n_spheres; ++t) {
      if (!self_candidate(r, s, t)) continue;
      if (!(self_pair_sd(r, xyz, s, t) > OR_SELF_HOME_CLEARANCE)) continue;
      if (count < capacity) {
        pairs[2 * count] = s;
        pairs[2 * count + 1] = t;
      }
      ++count;
    }
  free(xyz);
  return count;
}

double or_self_min_sd(const or_robot* r, int32_t n_pairs, const int32_t* pairs, const double* q) {
  double* xyz = (double*)malloc(sizeof(double) * 3 * (r->n_spheres + 1));
  or_sphere_centres(r, q, xyz);
  double best = DBL_MAX;
  for (int i = 0; i < n_pairs; ++i) best = fmin(best, self_pair_sd(r, xyz, pairs[2 * i], pairs[2 * i + 1]));
  free(xyz);
  return best;
}

/* The checked pairs of r, allocated (free with free()); *n receives their number. */
static int32_t* self_pair_list(const or_robot* r, int32_t* n) {
  *n = or_self_pairs(r, 0, NULL);
  int32_t* pairs = (int32_t*)malloc(sizeof(int32_t) * 2 * (*n + 1));
  or_self_pairs(r, *n, pairs);
  return pairs;
}

void or_self_cc_batch(const or_robot* r, int32_t n_cfg, const double* q, uint8_t* collide,
                      double* min_sd, int32_t n_threads) {
  int32_t np = 0;
  int32_t* pairs = self_pair_list(r, &np);
  const int nt = clamp_threads(n_threads);
#pragma omp parallel for num_threads(nt) schedule(dynamic, 16)
  for (int32_t i = 0; i < n_cfg; ++i) {
    const double sd = or_self_min_sd(r, np, pairs, q + (size_t)i * r->dof);
    if (collide) collide[i] = sd <= 0.0;
    if (min_sd) min_sd[i] = sd;
  }
  free(pairs);
}

void or_fk_cc_batch(const or_robot* r, const or_env* env, int32_t n_cfg, const double* q,
                    uint8_t* collide, double* min_sd, int32_t n_threads) {
  const int nt = clamp_threads(n_threads);
#pragma omp parallel for num_threads(nt) schedule(dynamic, 16)
  for (int32_t i = 0; i < n_cfg; ++i) {
    const double sd = or_config_min_sd(r, env, q + (size_t)i * r->dof);
    if (collide) collide[i] = sd <= 0.0;
    if (min_sd) min_sd[i] = sd;
  }
}

/* ---------------------------------------------------------------- projection */

/* Algorithm 1, ParallelProject, run synchronously (Jacobi): every active
 * waypoint's new value is computed from the same snapshot xi, and xi changes
 * only after all of them are computed (Section III-A: xi_new is formed first,
 * the segment itself is not yet modified).
 *
 * Readings:
 *  - indices are 0-based; xi[0] is the fixed start; prog is the index of the
 *    last waypoint of the validated prefix, starting at 0, and waypoints
 *    prog < k <= W-1 are active; success when prog reaches W-1;
 *  - prog advances over the contiguous run of valid waypoints after it (the
 *    text describes prog as how many initial configurations are projected);
 *  - validity is judged at the snapshot value, before the update, with the
 *    infinity norm of E_task; waypoints that join the prefix keep the value
 *    that was judged valid, the rest take xi_new;
 *  - E_sm = ||xi[k] - xi[k-1]||_2 - tau (tau = interpolation step),
 *    J_sm = xi[k] - xi[k-1], nabla_sm = J_sm E_sm (signed), valid spacing is
 *    E_sm < tau_sm;
 *  - J^+ is the damped least-squares step; updates are clamped to the joint
 *    limits.
 * xi: [W][dof], in = straight-line segment, out = projected segment.
 * Returns 1 on success (xi projected, *iters = iterations used), else 0.
 * *margin: smallest distance of any decision that moved prog from its
 * threshold (for accounting of threshold ties against a float32 run).
 * trace_prog (nullable, [max_iters]): prog after each iteration. */
int32_t or_parallel_project(const or_robot* r, const or_constraint* c, const or_params* p,
                            double* xi, int32_t* iters, double* margin, int32_t* trace_prog) {
  const int n = r->dof, W = p->W;
  double* xi_new = (double*)malloc(sizeof(double) * (size_t)W * n);
  int* valid = (int*)malloc(sizeof(int) * W);
  double* dmargin = (double*)malloc(sizeof(double) * W);
  int prog = 0, ok = 0, it = 0;
  double mg = DBL_MAX;
  for (it = 1; it <= p->max_iters; ++it) {
    for (int k = prog + 1; k <= W - 1; ++k) {
      const double* qk = xi + (size_t)k * n;
      const double* qp = xi + (size_t)(k - 1) * n;
      double e[MAXM], J[MAXM * MAXDOF], g_task[MAXDOF], delta[MAXDOF];
      const int m = or_task_error(r, c, qk, e);
      or_task_jacobian(r, c, qk, J);
      or_dls_step(J, e, m, n, p->lambda, g_task);
      double dist2 = 0.0;
      for (int j = 0; j < n; ++j) {
        delta[j] = qk[j] - qp[j];
        dist2 += delta[j] * delta[j];
      }
      const double E_sm = sqrt(dist2) - p->tau;
      for (int j = 0; j < n; ++j) {
        const double g_sm = p->variant == OR_PROJECT_INDEPENDENT ? 0.0 : delta[j] * E_sm;
        double v = qk[j] - p->alpha * (g_task[j] + g_sm);
        v = fmin(fmax(v, r->lo[j]), r->hi[j]);
        xi_new[(size_t)k * n + j] = v;
      }
      double einf = 0.0;
      for (int i = 0; i < m; ++i) einf = fmax(einf, fabs(e[i]));
      const double m_task = p->tau_task - einf;
      const double m_sm = p->tau_sm - E_sm;
      valid[k] = (m_task > 0.0) && (m_sm > 0.0);
      dmargin[k] = valid[k] ? fmin(m_task, m_sm) : fmax(-m_task, -m_sm);
    }
    int np = prog;
    while (np + 1 <= W - 1 && valid[np + 1]) ++np;
    const int last = np + 1 <= W - 1 ? np + 1 : W - 1;
    for (int k = prog + 1; k <= last; ++k) mg = fmin(mg, dmargin[k]);
    prog = np;
    if (trace_prog) trace_prog[it - 1] = prog;
    if (prog == W - 1) { ok = 1; break; }
    for (int k = prog + 1; k <= W - 1; ++k)
      memcpy(xi + (size_t)k * n, xi_new + (size_t)k * n, sizeof(double) * n);
  }
  if (iters) *iters = ok ? it : p->max_iters;
  if (margin) *margin = mg;
  free(xi_new);
  free(valid);
  free(dmargin);
  return ok;
}

int32_t or_sequential_project(const or_robot* r, const or_constraint* c, const or_params* p,
                              double* xi, int32_t* iters, double* margin) {
  const int n = r->dof, W = p->W;
  double* init = (double*)malloc(sizeof(double) * (size_t)W * n);
  memcpy(init, xi, sizeof(double) * (size_t)W * n);
  double mg = DBL_MAX;
  int32_t total = 0;
  int ok = 1;
  for (int k = 1; k < W && ok; ++k) {
    const double* prev = xi + (size_t)(k - 1) * n;
    double* x = xi + (size_t)k * n;
    for (int j = 0; j < n; ++j) x[j] = prev[j] + (init[(size_t)k * n + j] - init[(size_t)(k - 1) * n + j]);
    int valid = 0;
    for (int it = 1; it <= p->max_iters; ++it) {
      double e[MAXM], J[MAXM * MAXDOF], g[MAXDOF];
      const int m = or_task_error(r, c, x, e);
      double einf = 0.0, dist2 = 0.0;
      for (int i = 0; i < m; ++i) einf = fmax(einf, fabs(e[i]));
      for (int j = 0; j < n; ++j) dist2 += (x[j] - prev[j]) * (x[j] - prev[j]);
      const double m_task = p->tau_task - einf;
      const double m_sm = p->tau_sm - (sqrt(dist2) - p->tau);
      const int v = (m_task > 0.0) && (m_sm > 0.0);
      mg = fmin(mg, v ? fmin(m_task, m_sm) : fmax(-m_task, -m_sm));
      ++total;
      if (v) { valid = 1; break; }
      or_task_jacobian(r, c, x, J);
      or_dls_step(J, e, m, n, p->lambda, g);
      for (int j = 0; j < n; ++j) x[j] = fmin(fmax(x[j] - p->alpha * g[j], r->lo[j]), r->hi[j]);
    }
    if (!valid) ok = 0;
  }
  if (iters) *iters = total;
  if (margin) *margin = mg;
  free(init);
  return ok;
}

int32_t or_project_motion(const or_robot* r, const or_constraint* c, const or_params* p,
                          double* xi, int32_t* iters, double* margin) {
  if (p->variant == OR_PROJECT_SEQUENTIAL) return or_sequential_project(r, c, p, xi, iters, margin);
  return or_parallel_project(r, c, p, xi, iters, margin, NULL);
}

/* One motion per (q_from, q_to): W straight-line waypoints
 * xi_init[k] = q_from + (k / (W-1)) (q_to - q_from)  (Section III: a fixed
 * number of linearly interpolated states from q_near), ParallelProject, then
 * collision checking of waypoints 1..W-1 (waypoint 0 is already in the tree).
 * status: VALID, PROJ_FAIL or COLLISION; min_sd[i] = minimum signed distance
 * over the checked waypoints (DBL_MAX when projection failed). */
void or_project_validate_motions(const or_robot* r, const or_env* env, const or_constraint* c,
                                 const or_params* p, int32_t n_motions, const double* q_from,
                                 const double* q_to, double* xi, int32_t* status, int32_t* iters,
                                 double* proj_margin, double* min_sd, int32_t n_threads) {
  const int n = r->dof, W = p->W;
  const int nt = clamp_threads(n_threads);
  int32_t np = 0;
  int32_t* pairs = p->self_collision ? self_pair_list(r, &np) : NULL;
#pragma omp parallel for num_threads(nt) schedule(dynamic, 4)
  for (int32_t i = 0; i < n_motions; ++i) {
    double* x = xi + (size_t)i * W * n;
    const double* a = q_from + (size_t)i * n;
    const double* b = q_to + (size_t)i * n;
    for (int k = 0; k < W; ++k) {
      const double s = (double)k / (double)(W - 1);
      for (int j = 0; j < n; ++j) x[(size_t)k * n + j] = a[j] + s * (b[j] - a[j]);
    }
    int32_t it = 0;
    double mg = DBL_MAX;
    const int ok = or_project_motion(r, c, p, x, &it, &mg);
    double best = DBL_MAX;
    int st = OR_MOTION_PROJ_FAIL;
    if (ok) {
      for (int k = 1; k < W; ++k) {
        best = fmin(best, or_config_min_sd(r, env, x + (size_t)k * n));
        if (pairs) best = fmin(best, or_self_min_sd(r, np, pairs, x + (size_t)k * n));
      }
      st = best <= 0.0 ? OR_MOTION_COLLISION : OR_MOTION_VALID;
    }
    status[i] = st;
    if (iters) iters[i] = it;
    if (proj_margin) proj_margin[i] = mg;
    if (min_sd) min_sd[i] = best;
  }
  free(pairs);
}

/* Projection of one configuration (used to put start, goal and tree roots on
 * the manifold): q <- clamp(q - alpha g_task) until ||e||_inf < tol.
 * Returns 1 if the tolerance was met within max_iters steps. */
int32_t or_project_config(const or_robot* r, const or_constraint* c, const double* q_in,
                          double tol, int32_t max_iters, double alpha, double lambda,
                          double* q_out, int32_t* iters) {
  const int n = r->dof;
  memcpy(q_out, q_in, sizeof(double) * n);
  for (int it = 0; it <= max_iters; ++it) {
    double e[MAXM], J[MAXM * MAXDOF], g[MAXDOF];
    const int m = or_task_error(r, c, q_out, e);
    double einf = 0.0;
    for (int i = 0; i < m; ++i) einf = fmax(einf, fabs(e[i]));
    if (einf < tol) {
      if (iters) *iters = it;
      return 1;
    }
    if (it == max_iters) break;
    or_task_jacobian(r, c, q_out, J);
    or_dls_step(J, e, m, n, lambda, g);
    for (int j = 0; j < n; ++j) q_out[j] = fmin(fmax(q_out[j] - alpha * g[j], r->lo[j]), r->hi[j]);
  }
  if (iters) *iters = max_iters;
  return 0;
}

/* ---------------------------------------------------------------- planning */

/* splitmix64 (Steele, Lea, Flood 2014): the per-dimension shifts of the
 * Halton sequence are drawn from it, seeded with the planner's seed. */
static uint64_t splitmix64_next(uint64_t* state) {
  uint64_t z = (*state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* Radical inverse of i in base b: the Halton coordinate (Evaluation section:
 * samples come from the Halton sequence, reseeded only at the start). */
static double radical_inverse(uint32_t i, uint32_t b) {
  double f = 1.0 / b, r = 0.0;
  while (i) {
    r += f * (double)(i % b);
    i /= b;
    f /= b;
  }
  return r;
}

typedef struct {
  int n, W, cap, count;
  double* q;        /* [cap][n] */
  int* parent;      /* [cap] */
  double* edge;     /* [cap][W][n] */
} or_tree;

static int tree_nearest(const or_tree* t, const double* x, int n) {
  int best = 0;
  double bd = DBL_MAX;
  for (int i = 0; i < t->count; ++i) {
    double d = 0.0;
    for (int j = 0; j < n; ++j) d += (t->q[(size_t)i * n + j] - x[j]) * (t->q[(size_t)i * n + j] - x[j]);
    if (d < bd) { bd = d; best = i; }
  }
  return best;
}

static double dist_sq(const double* a, const double* b, int n) {
  double d = 0.0;
  for (int j = 0; j < n; ++j) d += (a[j] - b[j]) * (a[j] - b[j]);
  return d;
}

/* q_steer = a + min(1, step / |b - a|) (b - a) */
static void steer_to(const double* a, const double* b, double step, int n, double* out) {
  const double d = sqrt(dist_sq(a, b, n));
  const double s = d > step ? step / d : 1.0;
  for (int j = 0; j < n; ++j) out[j] = a[j] + s * (b[j] - a[j]);
}

/* One motion a -> b: straight-line waypoints, ParallelProject, collision
 * check of waypoints 1..W-1 (Section III).  xi receives the segment. */
static int motion_ok(const or_robot* r, const or_env* env, const or_constraint* c,
                     const or_params* p, const double* a, const double* b, double* xi) {
  const int n = r->dof, W = p->W;
  for (int k = 0; k < W; ++k) {
    const double s = (double)k / (double)(W - 1);
    for (int j = 0; j < n; ++j) xi[(size_t)k * n + j] = a[j] + s * (b[j] - a[j]);
  }
  int32_t it;
  double mg;
  if (!or_project_motion(r, c, p, xi, &it, &mg)) return 0;
  for (int k = 1; k < W; ++k)
    if (or_config_min_sd(r, env, xi + (size_t)k * n) <= 0.0) return 0;
  return 1;
}

static int tree_append(or_tree* t, int parent, const double* xi) {
  if (t->count >= t->cap) return -1;
  const int s = t->count++;
  memcpy(t->q + (size_t)s * t->n, xi + (size_t)(t->W - 1) * t->n, sizeof(double) * t->n);
  t->parent[s] = parent;
  memcpy(t->edge + (size_t)s * t->W * t->n, xi, sizeof(double) * t->W * t->n);
  return s;
}

int32_t or_plan(const or_robot* r, const or_env* env, const or_constraint* c, const or_params* p,
                const double* start, const double* goal, uint64_t seed, int32_t max_samples,
                int32_t capacity, int32_t max_connect, double* path, int32_t cap_path,
                int32_t* path_len, int32_t* nodes) {
  static const uint32_t primes[16] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53};
  const int n = r->dof, W = p->W;
  const double step = (W - 1) * p->tau, tol = p->tau + p->tau_sm;
  or_tree tr[2];
  for (int t = 0; t < 2; ++t) {
    tr[t].n = n; tr[t].W = W; tr[t].cap = capacity; tr[t].count = 1;
    tr[t].q = (double*)malloc(sizeof(double) * (size_t)capacity * n);
    tr[t].parent = (int*)malloc(sizeof(int) * (size_t)capacity);
    tr[t].edge = (double*)malloc(sizeof(double) * (size_t)capacity * W * n);
    memcpy(tr[t].q, t == 0 ? start : goal, sizeof(double) * n);
    tr[t].parent[0] = -1;
  }
  double shift[16];
  uint64_t state = seed;
  for (int j = 0; j < 16; ++j) shift[j] = (double)(splitmix64_next(&state) >> 11) * (1.0 / 9007199254740992.0);
  double* xi = (double*)malloc(sizeof(double) * (size_t)W * n);
  double qr[MAXDOF], qs[MAXDOF], qe[MAXDOF], qt[MAXDOF];
  int found = 0, fa = -1, fb = -1, fx = 0, status = 0;
  if (sqrt(dist_sq(start, goal, n)) < tol) { found = 1; fx = 0; fa = 0; fb = 0; }
  for (int32_t i = 0; i < max_samples && !found; ++i) {
    const int X = i & 1, Y = X ^ 1;
    for (int j = 0; j < n; ++j) {
      double u = radical_inverse((uint32_t)i + 1u, primes[j]) + shift[j];
      u -= floor(u);
      qr[j] = r->lo[j] + u * (r->hi[j] - r->lo[j]);
    }
    const int near = tree_nearest(&tr[X], qr, n);
    steer_to(tr[X].q + (size_t)near * n, qr, step, n, qs);
    if (!motion_ok(r, env, c, p, tr[X].q + (size_t)near * n, qs, xi)) continue;
    int cur = tree_append(&tr[X], near, xi);
    if (cur < 0) { status = -1; break; }
    memcpy(qe, xi + (size_t)(W - 1) * n, sizeof(double) * n);
    const int tgt = tree_nearest(&tr[Y], qe, n);
    memcpy(qt, tr[Y].q + (size_t)tgt * n, sizeof(double) * n);
    double dcur = dist_sq(qe, qt, n);
    for (int s = 0;; ++s) {
      if (dcur < tol * tol) { found = 1; fx = X; fa = cur; fb = tgt; break; }
      if (s >= max_connect) break;
      steer_to(qe, qt, step, n, qs);
      if (!motion_ok(r, env, c, p, qe, qs, xi)) break;
      const double dnew = dist_sq(xi + (size_t)(W - 1) * n, qt, n);
      if (!(dnew < dcur)) break;
      cur = tree_append(&tr[X], cur, xi);
      if (cur < 0) { status = -1; break; }
      memcpy(qe, xi + (size_t)(W - 1) * n, sizeof(double) * n);
      dcur = dnew;
    }
    if (status < 0) break;
  }
  if (nodes) { nodes[0] = tr[0].count; nodes[1] = tr[1].count; }
  if (found) {
    const int n0 = fx == 0 ? fa : fb, n1 = fx == 0 ? fb : fa;
    int len = 2, d0 = 0, d1 = 0;
    for (int v = n0; v > 0; v = tr[0].parent[v]) ++d0;
    for (int v = n1; v > 0; v = tr[1].parent[v]) ++d1;
    len = 2 + (d0 + d1) * (W - 1);
    if (sqrt(dist_sq(start, goal, n)) < tol && d0 == 0 && d1 == 0) len = 2;
    *path_len = len;
    if (len > cap_path) {
      status = -2;
    } else {
      /* tree-0 chain root -> n0 (edges forward), then n1, then tree-1 chain n1 -> root (backward) */
      int* chain = (int*)malloc(sizeof(int) * (size_t)(d0 + 1));
      int m = 0;
      for (int v = n0; v > 0; v = tr[0].parent[v]) chain[m++] = v;
      int row = 0;
      memcpy(path + (size_t)row++ * n, start, sizeof(double) * n);
      for (int i2 = m - 1; i2 >= 0; --i2)
        for (int k = 1; k < W; ++k)
          memcpy(path + (size_t)row++ * n, tr[0].edge + ((size_t)chain[i2] * W + k) * n, sizeof(double) * n);
      free(chain);
      memcpy(path + (size_t)row++ * n, tr[1].q + (size_t)n1 * n, sizeof(double) * n);
      for (int v = n1; v > 0; v = tr[1].parent[v])
        for (int k = W - 2; k >= 0; --k)
          memcpy(path + (size_t)row++ * n, tr[1].edge + ((size_t)v * W + k) * n, sizeof(double) * n);
      memcpy(path + (size_t)(len - 1) * n, goal, sizeof(double) * n);
      status = 1;
    }
  }
  for (int t = 0; t < 2; ++t) { free(tr[t].q); free(tr[t].parent); free(tr[t].edge); }
  free(xi);
  return status;
}

/* Nearest node among the first `count` nodes (lowest index on ties) and the
 * distance gap to the runner-up (DBL_MAX with a single node). */
static int tree_nearest_gap(const or_tree* t, int count, const double* x, int n, double* gap) {
  int best = 0;
  double b1 = DBL_MAX, b2 = DBL_MAX;
  for (int i = 0; i < count; ++i) {
    const double d = dist_sq(t->q + (size_t)i * n, x, n);
    if (d < b1) { b2 = b1; b1 = d; best = i; }
    else if (d < b2) b2 = d;
  }
  *gap = b2 == DBL_MAX ? DBL_MAX : sqrt(b2) - sqrt(b1);
  return best;
}

/* motion_ok with the closeness of its decisions: *margin = min(projection
 * margin, |minimum signed distance over waypoints 1..W-1|). */
static int motion_ok_margin(const or_robot* r, const or_env* env, const or_constraint* c,
                            const or_params* p, const double* a, const double* b, double* xi,
                            double* margin) {
  const int n = r->dof, W = p->W;
  for (int k = 0; k < W; ++k) {
    const double s = (double)k / (double)(W - 1);
    for (int j = 0; j < n; ++j) xi[(size_t)k * n + j] = a[j] + s * (b[j] - a[j]);
  }
  int32_t it;
  double mg = DBL_MAX;
  const int proj = or_project_motion(r, c, p, xi, &it, &mg);
  *margin = mg;
  if (!proj) return 0;
  double msd = DBL_MAX;
  for (int k = 1; k < W; ++k) msd = fmin(msd, or_config_min_sd(r, env, xi + (size_t)k * n));
  *margin = fmin(mg, fabs(msd));
  return msd > 0.0;
}

int32_t or_plan_rounds(const or_robot* r, const or_env* env, const or_constraint* c,
                       const or_params* p, const double* start, const double* goal, uint64_t seed,
                       int32_t n_groups, int32_t rounds, int32_t capacity, int32_t max_connect,
                       double* q0, int32_t* parent0, int32_t* band0, double* q1, int32_t* parent1,
                       int32_t* band1, int32_t* counts, int32_t* found_round, int32_t* band_round,
                       int32_t* band_extensions) {
  static const uint32_t primes[16] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53};
  const double kBandProj = 1e-5, kBandDist = 1e-4, kBandSample = 1e-5;
  const int n = r->dof, W = p->W;
  const double step = (W - 1) * p->tau, tol = p->tau + p->tau_sm;
  or_tree tr[2];
  int32_t* flag[2] = {band0, band1};
  for (int t = 0; t < 2; ++t) {
    tr[t].n = n; tr[t].W = W; tr[t].cap = capacity; tr[t].count = 1;
    tr[t].q = t == 0 ? q0 : q1;
    tr[t].parent = t == 0 ? parent0 : parent1;
    tr[t].edge = (double*)malloc(sizeof(double) * (size_t)capacity * W * n);
    memcpy(tr[t].q, t == 0 ? start : goal, sizeof(double) * n);
    tr[t].parent[0] = -1;
    flag[t][0] = 0;
  }
  double shift[16];
  uint64_t state = seed;
  for (int j = 0; j < 16; ++j) shift[j] = (double)(splitmix64_next(&state) >> 11) * (1.0 / 9007199254740992.0);
  double* xi = (double*)malloc(sizeof(double) * (size_t)W * n);
  double qr[MAXDOF], qs[MAXDOF], qe[MAXDOF], qt[MAXDOF];
  int status = 0;
  *found_round = 0;
  *band_round = 0;
  *band_extensions = 0;
  for (int32_t rd = 0; rd < rounds && !*found_round && status == 0; ++rd) {
    const int pub[2] = {tr[0].count, tr[1].count};   /* snapshot seen by this round's searches */
    for (int g = 0; g < n_groups && !*found_round && status == 0; ++g) {
      const int X = g & 1, Y = X ^ 1;
      const uint32_t idx = (uint32_t)rd * (uint32_t)n_groups + (uint32_t)g + 1u;
      int band = 0;   /* a decision of this extension so far lay near its threshold */
      for (int j = 0; j < n; ++j) {
        double u = radical_inverse(idx, primes[j]) + shift[j];
        u -= floor(u);
        if (u < kBandSample || u > 1.0 - kBandSample) band = 1;
        qr[j] = r->lo[j] + u * (r->hi[j] - r->lo[j]);
      }
      double gap, mg;
      const int near = tree_nearest_gap(&tr[X], pub[X], qr, n, &gap);
      if (gap < kBandDist) band = 1;
      steer_to(tr[X].q + (size_t)near * n, qr, step, n, qs);
      const int ok = motion_ok_margin(r, env, c, p, tr[X].q + (size_t)near * n, qs, xi, &mg);
      if (mg < kBandProj) band = 1;
      if (ok) {
        int cur = tree_append(&tr[X], near, xi);
        if (cur < 0) { status = -1; break; }
        flag[X][cur] = band;
        memcpy(qe, xi + (size_t)(W - 1) * n, sizeof(double) * n);
        const int tgt = tree_nearest_gap(&tr[Y], pub[Y], qe, n, &gap);
        if (gap < kBandDist) band = 1;
        memcpy(qt, tr[Y].q + (size_t)tgt * n, sizeof(double) * n);
        double dcur = dist_sq(qe, qt, n);
        for (int s = 0;; ++s) {
          if (fabs(sqrt(dcur) - tol) < kBandDist) band = 1;
          if (dcur < tol * tol) { *found_round = rd + 1; break; }
          if (s >= max_connect) break;
          steer_to(qe, qt, step, n, qs);
          const int ok2 = motion_ok_margin(r, env, c, p, qe, qs, xi, &mg);
          if (mg < kBandProj) band = 1;
          if (!ok2) break;
          const double dnew = dist_sq(xi + (size_t)(W - 1) * n, qt, n);
          if (fabs(sqrt(dnew) - sqrt(dcur)) < kBandDist) band = 1;
          if (!(dnew < dcur)) break;
          cur = tree_append(&tr[X], cur, xi);
          if (cur < 0) { status = -1; break; }
          flag[X][cur] = band;
          memcpy(qe, xi + (size_t)(W - 1) * n, sizeof(double) * n);
          dcur = dnew;
        }
      }
      if (band) {
        ++*band_extensions;
        if (!*band_round) *band_round = rd + 1;
      }
    }
  }
  counts[0] = tr[0].count;
  counts[1] = tr[1].count;
  for (int t = 0; t < 2; ++t) free(tr[t].edge);
  free(xi);
  return status;
}

void or_path_report(const or_robot* r, const or_env* env, const or_constraint* c,
                    const double* path, int32_t len, double* out) {
  const int n = r->dof;
  double worst_e = 0.0, worst_sp = 0.0, msd = DBL_MAX;
  int inside = 1;
  for (int i = 0; i < len; ++i) {
    const double* q = path + (size_t)i * n;
    double e[MAXM];
    const int m = or_task_error(r, c, q, e);
    for (int k = 0; k < m; ++k) worst_e = fmax(worst_e, fabs(e[k]));
    if (i > 0) worst_sp = fmax(worst_sp, sqrt(dist_sq(q, q - n, n)));
    msd = fmin(msd, or_config_min_sd(r, env, q));
    for (int j = 0; j < n; ++j) if (q[j] < r->lo[j] || q[j] > r->hi[j]) inside = 0;
  }
  out[0] = worst_e; out[1] = worst_sp; out[2] = msd; out[3] = inside;
}

/* ---------------------------------------------------------------- MLP */
/* z_l = W_l h_{l-1} + b_l, h_l = silu(z_l) for hidden layers, y = z_L;
 * silu(z) = z / (1 + exp(-z)); loss = mean over all M * n_out outputs of
 * (y - t)^2; gradients by the chain rule, layer by layer. */

static double silu_d(double z) { return z / (1.0 + exp(-z)); }
static double silu_grad_d(double z) {
  const double s = 1.0 / (1.0 + exp(-z));
  return s * (1.0 + z * (1.0 - s));
}

static size_t mlp_offset_w(int32_t l, const int32_t* dims) {
  size_t off = 0;
  for (int32_t i = 0; i < l; ++i) off += (size_t)dims[i + 1] * dims[i] + dims[i + 1];
  return off;
}

/* One sample through the network; z[l] and h[l] stored for the backward pass
 * (h[0] = the input).  Buffers are [n_layers + 1][maxw]. */
static void mlp_sample_forward(int32_t L, const int32_t* dims, const double* params,
                               const double* x, double* z, double* h, int maxw) {
  for (int j = 0; j < dims[0]; ++j) h[j] = x[j];
  for (int32_t l = 0; l < L; ++l) {
    const double* W = params + mlp_offset_w(l, dims);
    const double* b = W + (size_t)dims[l + 1] * dims[l];
    const double* hin = h + (size_t)l * maxw;
    double* zo = z + (size_t)(l + 1) * maxw;
    double* ho = h + (size_t)(l + 1) * maxw;
    for (int o = 0; o < dims[l + 1]; ++o) {
      double s = b[o];
      for (int i = 0; i < dims[l]; ++i) s += W[(size_t)o * dims[l] + i] * hin[i];
      zo[o] = s;
      ho[o] = (l + 1 < L) ? silu_d(s) : s;
    }
  }
}

void or_mlp_forward(int32_t n_layers, const int32_t* dims, const double* params, int32_t M,
                    const double* x, double* y) {
  int maxw = 0;
  for (int32_t l = 0; l <= n_layers; ++l) maxw = dims[l] > maxw ? dims[l] : maxw;
  double* z = (double*)malloc(sizeof(double) * (size_t)(n_layers + 1) * maxw);
  double* h = (double*)malloc(sizeof(double) * (size_t)(n_layers + 1) * maxw);
  for (int32_t m = 0; m < M; ++m) {
    mlp_sample_forward(n_layers, dims, params, x + (size_t)m * dims[0], z, h, maxw);
    memcpy(y + (size_t)m * dims[n_layers], h + (size_t)n_layers * maxw, sizeof(double) * dims[n_layers]);
  }
  free(z);
  free(h);
}

double or_mlp_gradients(int32_t n_layers, const int32_t* dims, const double* params, int32_t M,
                        const double* x, const double* t, double* grad) {
  const int32_t L = n_layers, nout = dims[L];
  int maxw = 0;
  for (int32_t l = 0; l <= L; ++l) maxw = dims[l] > maxw ? dims[l] : maxw;
  const size_t np = mlp_offset_w(L, dims);
  memset(grad, 0, sizeof(double) * np);
  double* z = (double*)malloc(sizeof(double) * (size_t)(L + 1) * maxw);
  double* h = (double*)malloc(sizeof(double) * (size_t)(L + 1) * maxw);
  double* d = (double*)malloc(sizeof(double) * maxw);      /* dLoss/dz of the current layer */
  double* dn = (double*)malloc(sizeof(double) * maxw);
  double loss = 0.0;
  const double scale = 1.0 / ((double)M * nout);
  for (int32_t m = 0; m < M; ++m) {
    mlp_sample_forward(L, dims, params, x + (size_t)m * dims[0], z, h, maxw);
    for (int o = 0; o < nout; ++o) {
      const double e = h[(size_t)L * maxw + o] - t[(size_t)m * nout + o];
      loss += e * e * scale;
      d[o] = 2.0 * e * scale;
    }
    for (int32_t l = L - 1; l >= 0; --l) {
      const double* W = params + mlp_offset_w(l, dims);
      double* gW = grad + mlp_offset_w(l, dims);
      double* gb = gW + (size_t)dims[l + 1] * dims[l];
      const double* hin = h + (size_t)l * maxw;
      for (int o = 0; o < dims[l + 1]; ++o) {
        gb[o] += d[o];
        for (int i = 0; i < dims[l]; ++i) gW[(size_t)o * dims[l] + i] += d[o] * hin[i];
      }
      if (l == 0) break;
      for (int i = 0; i < dims[l]; ++i) {
        double s = 0.0;
        for (int o = 0; o < dims[l + 1]; ++o) s += W[(size_t)o * dims[l] + i] * d[o];
        dn[i] = s * silu_grad_d(z[(size_t)l * maxw + i]);
      }
      memcpy(d, dn, sizeof(double) * dims[l]);
    }
  }
  free(z);
  free(h);
  free(d);
  free(dn);
  return loss;
}

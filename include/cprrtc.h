/* cprrtc.h -- C ABI of the MI355X (gfx950) library for batched constrained
 * motion projection and validation, the data-parallel hot path of cpRRTC
 * (Hu, Wang, Christensen: "cpRRTC: GPU-Parallel RRT-Connect for Constrained
 * Motion Planning", arXiv 2505.06791).
 *
 * Conventions shared by every call
 *   - Plain C types only.  Arrays are row-major.  Angles in radians, lengths
 *     in metres.
 *   - Pointers named d_* are device (HBM) pointers; all others are host.
 *     The library never frees or retains a caller's pointer beyond the call
 *     (device-pointer calls: beyond completion of the work on `stream`).
 *   - `stream` is a hipStream_t passed as void*; NULL is the default stream.
 *     Device-pointer calls are asynchronous on that stream; plan() is
 *     synchronous.
 *   - Every call returns a status code (CP_OK = 0, < 0 errors).  No exception
 *     or abort crosses this boundary.  cp_last_error() describes the last
 *     failure on the calling thread.
 *   - Handles (cp_robot, cp_env) are immutable after creation and may be
 *     shared by threads; calls on different streams may overlap.
 */
#ifndef CPRRTC_H
#define CPRRTC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
enum {
  CP_OK = 0,
  CP_NO_SOLUTION = 1,      /* plan(): budget exhausted without a path (not an error) */
  CP_E_ARG = -1,           /* malformed argument (NULL, size, layout) */
  CP_E_START = -2,         /* plan(): start outside limits, off the manifold or colliding */
  CP_E_GOAL = -3,          /* plan(): goal outside limits, off the manifold or colliding */
  CP_E_CAPACITY = -4,      /* output or tree capacity too small */
  CP_E_RTC = -5,           /* runtime compilation failed */
  CP_E_HIP = -6,           /* HIP runtime error */
  CP_E_UNSUPPORTED = -7    /* DOF, chain count or waypoint count this build does not serve */
};

/* Per-motion outcome written by project_validate_motions (data, not errors). */
enum { CP_MOTION_VALID = 0, CP_MOTION_PROJ_FAIL = 1, CP_MOTION_COLLISION = 2 };

enum { CP_REVOLUTE = 0, CP_PRISMATIC = 1 };
enum { CP_CON_NONE = 0, CP_CON_POSE = 1, CP_CON_REL_POSE = 2 };

/* flags */
enum {
  CP_NO_EARLY_EXIT = 1,  /* keep checking a motion / configuration after its first collision */
  CP_NO_CULL = 2,        /* project_validate_motions: test every primitive, without the
                            wave-level bounding-box culling (verdicts are the same) */
  CP_POOLED = 8,         /* project_validate_motions: project with several motions per
                            wavefront whatever the batch size (results are the same) */
  CP_PER_MOTION = 16,    /* project_validate_motions: project with one motion per wavefront
                            whatever the batch size (results are the same) */
  CP_GENERIC = 32,       /* project_validate_motions, validate_motions, fk_cc_batch: use
                            the library's projection, validation and FK/CC kernels even
                            where cp_robot_specialize compiled some for the robot */
  CP_SELF_COLLISION = 64 /* fk_cc_batch, validate_motions, project_validate_motions: also
                            check the robot against itself (cp_robot_self_pairs) */
};

/* ------------------------------------------------------------ descriptors */

/* Serial chain(s) in modified Denavit-Hartenberg form (Craig):
 *   T_i = RotX(alpha_{i-1}) TransX(a_{i-1}) RotZ(theta_i) TransZ(d_i),
 * a revolute joint adds q_i to theta_i, a prismatic joint adds q_i to d_i.
 * Frame i of chain c is base_c T_1 ... T_i over that chain's joints; the end
 * effector is the last frame of the chain times tool_c.  The paper runs
 * forward kinematics per waypoint (Section III) without fixing a model.
 * All arrays host, double, copied by cp_robot_create. */
typedef struct cp_robot_desc {
  int32_t dof;               /* total joints, 1..16 */
  int32_t n_chains;          /* 1, or 2 for two arms on one base */
  const int32_t* joint_type; /* [dof] CP_REVOLUTE / CP_PRISMATIC */
  const int32_t* joint_chain;/* [dof] chain of each joint; non-decreasing */
  const double* alpha;       /* [dof] alpha_{i-1} */
  const double* a;           /* [dof] a_{i-1} */
  const double* d;           /* [dof] constant part of d_i */
  const double* theta;       /* [dof] constant part of theta_i */
  const double* q_lo;        /* [dof] joint limits */
  const double* q_hi;        /* [dof] */
  const double* base;        /* [n_chains][16] homogeneous, row-major */
  const double* tool;        /* [n_chains][16] */
  int32_t n_spheres;         /* robot collision spheres, 1..1024 */
  const int32_t* sphere_link;/* [n_spheres] joint whose frame carries the sphere */
  const double* sphere;      /* [n_spheres][4] centre in that frame, radius > 0 */
} cp_robot_desc;

/* Environment primitives (solid).  Host, double, copied by cp_env_create.
 * Counts may be 0 (pointer then ignored). */
typedef struct cp_env_desc {
  int32_t n_aabb;      const double* aabb;      /* [n][6]  centre, half extents */
  int32_t n_obb;       const double* obb;       /* [n][15] centre, R (row-major; its
                                                   columns are the box axes), half extents */
  int32_t n_sphere;    const double* sphere;    /* [n][4]  centre, radius */
  int32_t n_capsule;   const double* capsule;   /* [n][7]  p0, p1, radius */
  int32_t n_cylinder;  const double* cylinder;  /* [n][8]  centre, unit axis, half length, radius */
} cp_env_desc;

/* Task constraint (Evaluation section: end-effector axes are locked; a plane
 * locks one position axis, a line two, fixed orientation the angular ones).
 *   CP_CON_POSE:     chain 0's end effector seen from `frame`:
 *                    x = (Rc^T (p - pc), roll, pitch, yaw of Rc^T R), with
 *                    R = Rz(yaw) Ry(pitch) Rx(roll); error = (x - target) on
 *                    the axes set in mask, angles wrapped into (-pi, pi].
 *   CP_CON_REL_POSE: end effector 2 seen from end effector 1:
 *                    p' = R1^T (p2 - p1), R' = R1^T R2; error = (p' - p*,
 *                    roll/pitch/yaw of R*^T R') on the masked axes, where
 *                    rel_target = [R* p*].
 *   CP_CON_NONE:     no task error (only the spacing term acts). */
typedef struct cp_constraint {
  int32_t kind;
  int32_t mask[6];          /* x y z roll pitch yaw: 1 = locked */
  double frame[16];         /* CP_CON_POSE: constraint frame in world, row-major */
  double target[6];         /* CP_CON_POSE: locked values in that frame */
  double rel_target[16];    /* CP_CON_REL_POSE: pose of end effector 2 in end effector 1 */
} cp_constraint;

/* Parameters of Algorithm 1 (ParallelProject).  The paper names them but
 * gives no values; cp_proj_params_default() fills the defaults shown. */
typedef struct cp_proj_params {
  int32_t W;          /* waypoints per motion incl. the fixed start: 32 or 64 (64) */
  int32_t max_iters;  /* iteration budget (32) */
  double tau;         /* spacing target = interpolation step (0.05) */
  double tau_sm;      /* spacing slack: a waypoint is valid if its spacing < tau + tau_sm (0.025) */
  double tau_task;    /* task tolerance on the infinity norm of the error (1e-3) */
  double alpha;       /* step factor (1.0) */
  double lambda;      /* damping of the least-squares step (1e-2) */
  int32_t sphere_batch; /* spheres per collision batch between early-exit polls: 4, 8 or 16
                           (8); the planner's rounds take 8 for 16 */
  int32_t variant;    /* projection operator, CP_PROJECT_* (CP_PROJECT_PARALLEL) */
} cp_proj_params;

/* Projection operators (Section III-A and its comparison in the Evaluation):
 * PARALLEL     Algorithm 1: every waypoint projected at once with the
 *              smoothing term, frozen validated prefix;
 * INDEPENDENT  the same iteration without the smoothing term (waypoints
 *              projected in parallel and independently; spacing is still
 *              required for validity);
 * SEQUENTIAL   the CBiRRT-style projection of cpRRTC-Naive: waypoint k
 *              starts at the projected waypoint k-1 plus one interpolation
 *              step and is projected alone (damped least squares, no
 *              smoothing term) until it is valid (task error and spacing to
 *              k-1), at most max_iters steps per waypoint; iterations are
 *              summed over the waypoints. */
enum { CP_PROJECT_PARALLEL = 0, CP_PROJECT_INDEPENDENT = 1, CP_PROJECT_SEQUENTIAL = 2 };

typedef struct cp_robot cp_robot;   /* opaque; device copy of a cp_robot_desc */
typedef struct cp_env cp_env;       /* opaque; device copy of a cp_env_desc */

/* ------------------------------------------------------------ handles */
int cp_robot_create(const cp_robot_desc* desc, cp_robot** out);
void cp_robot_destroy(cp_robot* robot);
int cp_env_create(const cp_env_desc* desc, cp_env** out);
void cp_env_destroy(cp_env* env);
void cp_proj_params_default(cp_proj_params* p);
const char* cp_last_error(void);    /* thread-local; valid until the next call on this thread */

/* ------------------------------------------------------------ hot path */

/* Forward kinematics of every collision sphere and sphere-vs-primitive
 * collision check, one configuration per lane (Sections I and IV: each
 * waypoint's FK and CC).  A configuration collides iff some pair has
 * signed distance <= 0 (distance from the sphere centre to the solid minus
 * the sphere radius).
 *   d_q        [n_cfg][dof] float32 configurations
 *   d_collide  [n_cfg] 1 = collides, 0 = free
 *   d_min_sd   [n_cfg] nullable; if given, every pair is evaluated and the
 *              minimum signed distance is written
 *   d_sphere_xyz [n_cfg][n_spheres][3] nullable; if given, the world centre
 *              of every robot sphere (the forward kinematics the check runs),
 *              spheres in description order, float32, written by a separate
 *              kernel on the same stream
 *   flags      CP_NO_EARLY_EXIT: evaluate every pair even after a collision;
 *              CP_SELF_COLLISION: also the robot against itself
 * Errors: CP_E_ARG (NULL handle/pointer, n_cfg < 0), CP_E_UNSUPPORTED (dof),
 * CP_E_HIP (launch failure). n_cfg = 0 is a no-op. */
int fk_cc_batch(const cp_robot* robot, const cp_env* env, int32_t n_cfg, const float* d_q,
                uint8_t* d_collide, float* d_min_sd, float* d_sphere_xyz, int32_t flags,
                void* stream);

/* Self-collision pairs of a robot (specified here; the paper checks the
 * robot against the environment only).  A pair of spheres (s, t) is checked
 * when their links lie in different chains, or in one chain at least two
 * joints apart, and they are clear by more than 1e-3 m at the home
 * configuration (every joint at 0 clamped into its limits; pairs that
 * overlap there touch across a joint by construction and are allowed).  A
 * configuration self-collides iff some checked pair has signed distance
 * |c_s - c_t| - r_s - r_t <= 0.  With CP_SELF_COLLISION, fk_cc_batch ORs
 * this into d_collide (and takes the minimum into d_min_sd), and motion
 * validation marks a motion colliding (status 2) if any of waypoints
 * 1..W-1 self-collides (16 lanes per configuration or waypoint, over the
 * pairs).
 *   pairs     out, host, nullable: [capacity][2] sphere indices in
 *             description order, s < t, sorted; at most capacity written
 *   count     out: the number of checked pairs
 * The list is computed once, at cp_robot_create.  Errors: CP_E_ARG. */
int cp_robot_self_pairs(const cp_robot* robot, int32_t capacity, int32_t* pairs, int32_t* count);

/* Motion projection and validation (Section III and Algorithm 1; Section IV).
 * For each motion i: W waypoints xi[k] = q_from + (k/(W-1)) (q_to - q_from),
 * ParallelProject with xi[0] fixed and the end free (Jacobi snapshot,
 * validated prefix frozen, damped least-squares task step, smoothing step
 * (||xi[k]-xi[k-1]|| - tau) (xi[k]-xi[k-1]), clamp to limits), then FK+CC of
 * waypoints 1..W-1 with an early exit of the whole motion on any collision.
 * Two kernels run on `stream`: projection, then validation.  Batches of at
 * least 24576 motions are projected with several motions per wavefront and
 * only their unfrozen waypoints on its lanes, smaller ones with one motion
 * per wavefront (flags CP_POOLED / CP_PER_MOTION force either; the results
 * are identical).
 *   d_q_from, d_q_to [n_motions][dof] float32
 *   d_xi      [n_motions][W][dof] float32 out: projected segment (on
 *             CP_MOTION_PROJ_FAIL: the last iterate)
 *   d_status  [n_motions] int32 out: CP_MOTION_*
 *   d_iters   [n_motions] int32 out, nullable: ParallelProject iterations
 *   d_work    [8] uint64 in/out, nullable: work counters the call ADDS to
 *             (the caller zeroes them), in units of one waypoint's work:
 *             [0..4] sphere-primitive pair tests against axis-aligned boxes,
 *             oriented boxes, spheres, capsules, cylinders; [5] robot sphere
 *             centres placed; [6] waypoint updates of ParallelProject
 *             (waypoints past the frozen prefix, summed over iterations);
 *             [7] bounding-sphere culling tests (per motion and batch)
 *   params    NULL = defaults
 * Errors: CP_E_ARG, CP_E_UNSUPPORTED (dof, W), CP_E_HIP. */
int project_validate_motions(const cp_robot* robot, const cp_env* env,
                             const cp_constraint* constraint, const cp_proj_params* params,
                             int32_t n_motions, const float* d_q_from, const float* d_q_to,
                             float* d_xi, int32_t* d_status, int32_t* d_iters, uint64_t* d_work,
                             int32_t flags, void* stream);

/* The two halves of project_validate_motions, for callers that want them
 * apart (e.g. to time them, or to project without checking):
 *   project_motions:  interpolation + ParallelProject; d_status[i] = 0 when
 *                     the segment was projected, CP_MOTION_PROJ_FAIL when not;
 *                     d_work adds to slot [6] only.
 *   validate_motions: FK + CC of waypoints 1..W-1 of every motion whose
 *                     d_status is 0 on entry (others are left untouched);
 *                     d_status becomes CP_MOTION_VALID or CP_MOTION_COLLISION;
 *                     d_work adds to slots [0..5] and [7].
 * Arguments, layouts and errors as for project_validate_motions (W and
 * sphere_batch are taken from params). */
int project_motions(const cp_robot* robot, const cp_constraint* constraint,
                    const cp_proj_params* params, int32_t n_motions, const float* d_q_from,
                    const float* d_q_to, float* d_xi, int32_t* d_status, int32_t* d_iters,
                    uint64_t* d_work, void* stream);
int validate_motions(const cp_robot* robot, const cp_env* env, const cp_proj_params* params,
                     int32_t n_motions, const float* d_xi, int32_t* d_status, uint64_t* d_work,
                     int32_t flags, void* stream);

/* Projection of single configurations onto the manifold (puts start, goal
 * and samples on it): q <- clamp(q - alpha g_task) until ||e||_inf < tol,
 * at most max_iters steps.
 *   d_q_in, d_q_out [n][dof] float32; d_status [n] int32: 1 converged, 0 not.
 * Errors: CP_E_ARG, CP_E_UNSUPPORTED, CP_E_HIP. */
int project_configs(const cp_robot* robot, const cp_constraint* constraint, int32_t n,
                    const float* d_q_in, float* d_q_out, int32_t* d_status, double tol,
                    int32_t max_iters, double alpha, double lambda, void* stream);

/* ------------------------------------------------------------ learned warm start */

/* A multilayer perceptron n_in -> hidden (SiLU) x n_hidden -> n_out with BF16
 * weights and FP32 accumulation on the matrix cores, FP32 master weights and
 * Adam state; all of it in device memory owned by the handle.  Parameters
 * are one FP32 vector: for each layer, W [out][in] row-major, then b [out].
 * Inputs x [M][n_in], outputs / targets [M][n_out], all float32 device
 * pointers; calls are asynchronous on `stream`; a handle serves one stream at
 * a time (it keeps activation workspace). */
typedef struct cp_mlp cp_mlp;
int cp_mlp_create(int32_t n_in, int32_t hidden, int32_t n_hidden, int32_t n_out, uint64_t seed,
                  cp_mlp** out);
void cp_mlp_destroy(cp_mlp* mlp);
int64_t cp_mlp_num_params(const cp_mlp* mlp);
int cp_mlp_get_params(const cp_mlp* mlp, float* d_params, void* stream);
int cp_mlp_set_params(cp_mlp* mlp, const float* d_params, void* stream);
int cp_mlp_forward(cp_mlp* mlp, int64_t M, const float* d_x, float* d_y, void* stream);
/* Gradients of the mean squared error over the n_out outputs (and the loss)
 * at the current parameters; d_grad [num_params] and d_loss [1] nullable. */
int cp_mlp_gradients(cp_mlp* mlp, int64_t M, const float* d_x, const float* d_t, float* d_grad,
                     float* d_loss, void* stream);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8) on the mean squared error. */
int cp_mlp_train_step(cp_mlp* mlp, int64_t M, const float* d_x, const float* d_t, float lr,
                      float* d_loss, void* stream);
/* Adam state, for checkpoints: the first and second moment estimates
 * (d_m1, d_m2: [num_params] float32 device, the parameter order above) and
 * the number of steps taken (which sets the bias corrections of the next
 * step).  get copies them out (step: host pointer, nullable), set copies
 * them in; with cp_mlp_get_params / cp_mlp_set_params they restore a run
 * exactly (the training kernels sum in a fixed order).  Asynchronous on
 * `stream`.  Errors: CP_E_ARG (NULL handle or moment buffer, step < 0),
 * CP_E_HIP. */
int cp_mlp_get_state(const cp_mlp* mlp, float* d_m1, float* d_m2, int64_t* step, void* stream);
int cp_mlp_set_state(cp_mlp* mlp, const float* d_m1, const float* d_m2, int64_t step, void* stream);

/* project_motions with a learned warm start: every waypoint k >= 1 starts at
 * clamp(straight line + net(features)), features = (waypoint / joint range,
 * constraint parameters: the locked pose targets (6), or p* and R* (12) for a
 * relative pose); the network needs n_in = dof + 6 (or + 12), n_out = dof.
 * ParallelProject then runs to the same tolerance; motions whose projection
 * fails are projected again from the straight line (the plain projector is
 * the fallback and the judge).  d_iters receives the iterations of both
 * passes.  flags: CP_WARM_NO_FALLBACK skips the fallback (to measure the warm
 * pass alone).  Only the parallel projector (variant CP_PROJECT_PARALLEL) is
 * warm-started; other variants return CP_E_UNSUPPORTED.  Otherwise as
 * project_motions. */
enum { CP_WARM_NO_FALLBACK = 4 };
int project_motions_warm(const cp_robot* robot, const cp_constraint* constraint,
                         const cp_proj_params* params, cp_mlp* mlp, int32_t n_motions,
                         const float* d_q_from, const float* d_q_to, float* d_xi,
                         int32_t* d_status, int32_t* d_iters, uint64_t* d_work, int32_t flags,
                         void* stream);

/* Training pairs of the warm start from motions the projector projected:
 * for waypoint k = 1..W-1 of motion m, row m (W-1) + k - 1 of d_x
 * [n_motions (W-1)][dof + 6 (or + 12)] receives the network's features (as
 * project_motions_warm computes them for the straight waypoint of
 * d_q_from[m] -> d_q_to[m]) and the row of d_t [n_motions (W-1)][dof] the
 * target, d_xi[m][k] minus that straight waypoint.  Rows of motions whose
 * projection failed are written too; the caller keeps the rows it wants.
 * Device pointers, asynchronous on stream.  Errors: CP_E_ARG,
 * CP_E_UNSUPPORTED (dof), CP_E_HIP. */
int cp_warm_pairs(const cp_robot* robot, const cp_constraint* constraint, int32_t W,
                  int32_t n_motions, const float* d_q_from, const float* d_q_to,
                  const float* d_xi, float* d_x, float* d_t, void* stream);

/* project_motions_warm for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same kernels and results, but the network's corrections go
 * to a fixed device array of 32 MiB (8 Mi floats) inside the library instead
 * of memory the library allocates, and the call allocates nothing.  The array
 * exists once per GPU (held until the process ends) and every call on that
 * GPU shares it: calls that overlap on one GPU race and must not be issued
 * concurrently (on different streams or threads).  Limits: n_motions x (W-1)
 * x dof <= 8 Mi (e.g. 19 000 motions of a 7-joint robot at W = 64), else
 * CP_E_CAPACITY with nothing launched; the network must have the fused shape
 * (hidden width 64, 128, 256 or 512, at most 32 inputs and 16 outputs), else
 * CP_E_UNSUPPORTED.  Arguments, layout, ownership and the other errors as
 * project_motions_warm. */
int project_motions_warm_noalloc(const cp_robot* robot, const cp_constraint* constraint,
                                 const cp_proj_params* params, cp_mlp* mlp, int32_t n_motions,
                                 const float* d_q_from, const float* d_q_to, float* d_xi,
                                 int32_t* d_status, int32_t* d_iters, uint64_t* d_work,
                                 int32_t flags, void* stream);

/* ------------------------------------------------------------ run-time specialisation */

/* Compiles at run time (hipRTC) kernels for this robot and for constraints
 * of this one's kind and locked axes, with the robot's joint constants,
 * base and tool frames, collision spheres and the mask written in as
 * constants (the kernel source is the library's own device code; only the
 * constants differ), and keeps them in the robot handle.  what:
 * CP_SPECIALIZE_PROJECT (0 means this) -- the pooled projection kernel, the
 * culled validation kernels and the FK/CC kernel of configurations: later
 * calls that project this robot's motions in the pooled form
 * (project_motions, project_validate_motions; see CP_POOLED) with a
 * constraint of the same kind and mask use the first, every later culled
 * validation of this robot's motions (validate_motions,
 * project_validate_motions; the validation kernels depend on the robot
 * only) the second, and fk_cc_batch calls of this robot without distances
 * (d_min_sd NULL) the third, unless flags hold CP_GENERIC;
 * CP_SPECIALIZE_PLAN -- the planner's round kernels: later cp_plan calls of
 * planners of this robot with such a constraint use them.  In these kernels
 * revolute joints whose limits (plus theta) stay within +-3.2 rad take the
 * hardware sine and cosine, accurate there (waypoints are expected within
 * the joint limits).
 * The constraint's other values (frame, targets) stay arguments.  Rotation
 * entries within 1e-6 of 0 or +-1 are taken as those values.  Kernels
 * already compiled for the key are not compiled again.  compile_ms:
 * nullable, out (compile and load time of this call).
 * Thread-safe with concurrent projections of the same robot.  Errors:
 * CP_E_ARG, CP_E_UNSUPPORTED (dof, kind), CP_E_RTC (compilation; the log
 * head in cp_last_error), CP_E_HIP (module load). */
enum { CP_SPECIALIZE_PROJECT = 1, CP_SPECIALIZE_PLAN = 2 };
int cp_robot_specialize(cp_robot* robot, const cp_constraint* constraint, int32_t what,
                        double* compile_ms);

/* ------------------------------------------------------------ launch autotuning */

/* Picks the launch shape for a workload by measurement: for every candidate
 * (W in {32, 64} if flags has CP_TUNE_W, else the W of *params; sphere batch
 * in {4, 8, 16}, or {4, 8} -- the planners' round kernels -- if flags has
 * CP_TUNE_PLANNER) runs project_validate_motions once untimed and reps times timed
 * on the caller's sample motions (d_q_from, d_q_to: [n_motions][dof] device
 * floats, steered for the W of *params; for another W the end points are
 * moved along the same direction by (W' - 1) / (W - 1) so the initial
 * spacing is unchanged) and keeps the candidate with the most waypoints per
 * second over motions whose projection succeeded (W - 1 each).  *params: in,
 * the base parameters; out, the chosen W and sphere_batch (other fields
 * unchanged).  report: nullable, one entry per candidate timed.  Synchronous
 * on stream; allocates its own scratch (n_motions x 64 x dof floats).
 * Errors as project_validate_motions, CP_E_ARG for n_motions < 1 or reps
 * outside 1..1000. */
enum { CP_TUNE_W = 1, CP_TUNE_PLANNER = 2 };
typedef struct cp_tune_report {
  int32_t n;                   /* candidates timed */
  int32_t W[8];
  int32_t sphere_batch[8];
  double ms[8];                /* mean time per call */
  double waypoints_per_s[8];
} cp_tune_report;
int cp_autotune(const cp_robot* robot, const cp_env* env, const cp_constraint* constraint,
                cp_proj_params* params, int32_t n_motions, const float* d_q_from,
                const float* d_q_to, int32_t flags, int32_t reps, cp_tune_report* report,
                void* stream);

/* ------------------------------------------------------------ planning */

/* Constrained bidirectional RRT-Connect (Section III): two trees rooted at
 * start and goal; in each round n_groups wavefronts each sample a Halton
 * point (shifted by the seed; sampling restarts with every call), extend
 * their tree (half the wavefronts per tree) from its nearest node by one
 * projected, validated motion of at most (W-1) tau, then keep extending the
 * same tree towards the nearest node of the other tree while every segment is
 * valid and strictly reduces that distance; the trees connect when an end
 * comes within tau + tau_sm of that node.  Searches see the nodes published
 * before the round. */
typedef struct cp_plan_opts {
  cp_proj_params proj;   /* projection / validation parameters */
  int32_t n_groups;      /* extensions (wavefronts) per round, >= 2 (256) */
  int32_t max_rounds;    /* round budget (2000) */
  int32_t capacity;      /* nodes per tree (16384) */
  int32_t max_connect;   /* extension steps towards the other tree per round (64) */
  int32_t poll_every;    /* rounds between host checks of the done flag (1) */
  int32_t flags;         /* CP_SELF_COLLISION: every extension also checks its waypoints
                            against the robot itself (cp_robot_self_pairs), one
                            configuration at a time by the wavefront; these rounds use
                            the library's kernels even for a specialised robot (0) */
} cp_plan_opts;

/* Dense path: every waypoint of every edge, consecutive spacing < tau + tau_sm;
 * q[0] and q[len-1] are the caller's start and goal values. */
typedef struct cp_path {
  int32_t capacity;      /* in: rows of q allocated by the caller */
  int32_t len;           /* out: rows of the path (also set when capacity is too small) */
  int32_t dof;           /* out */
  double* q;             /* [capacity][dof], caller-allocated, host */
} cp_path;

typedef struct cp_plan_stats {
  int32_t rounds;        /* rounds launched */
  int32_t nodes[2];      /* tree sizes (start tree, goal tree) */
  int32_t overflow;      /* 1 if a tree reached its capacity */
  int32_t launches_per_round;  /* kernel launches per round */
} cp_plan_stats;

/* Path shortcutting (specified here; the paper returns the planner's path
 * as it is).  Each round: for every index i of the path P, the farthest
 * j >= i + 2 with ||P[j] - P[i]|| <= (W-1) tau whose subpath is longer than
 * the chord is a candidate; all candidates of the round are projected and
 * validated in one project_validate_motions call (from P[i] towards P[j],
 * Algorithm 1, flags as given); a candidate is accepted when its motion is
 * valid, waypoint W-2 lies within tau + tau_sm of P[j], and the piece
 * (waypoints 1 .. W-2, then P[j]) is shorter than P[i..j]; accepted pieces
 * replace their subpaths by decreasing gain, skipping any whose interval
 * meets a kept one except at an end point.  Rounds stop early when none is
 * accepted.  The result is a dense path between the same end points, every
 * spacing < tau + tau_sm, never longer than the input.
 *   path, len   in: [len][dof] host doubles (a dense path, as cp_plan returns)
 *   rounds      round budget, >= 0
 *   flags       passed to project_validate_motions (e.g. CP_SELF_COLLISION)
 *   out         out: the shortened path (out->capacity rows available)
 *   stats       nullable
 * Synchronous on `stream`.  Allocates its candidate buffers per call.
 * Errors: CP_E_ARG, CP_E_UNSUPPORTED (W), CP_E_CAPACITY (out too small;
 * out->len is set), CP_E_HIP, and those of project_validate_motions. */
typedef struct cp_shortcut_stats {
  int32_t rounds;        /* rounds run */
  int32_t candidates;    /* motions projected over all rounds */
  int32_t replaced;      /* pieces spliced in */
  double length_before;  /* sum of consecutive joint-space distances */
  double length_after;
} cp_shortcut_stats;
int cp_shortcut(const cp_robot* robot, const cp_env* env, const cp_constraint* constraint,
                const cp_proj_params* params, const double* path, int32_t len, int32_t rounds,
                int32_t flags, cp_path* out, cp_shortcut_stats* stats, void* stream);

typedef struct cp_planner cp_planner;  /* opaque: device trees and scratch for one robot */

void cp_plan_opts_default(cp_plan_opts* o);
/* Allocates the trees (2 x capacity x (W+1) x dof floats) once, for repeated
 * cp_plan calls.  Errors: CP_E_ARG, CP_E_UNSUPPORTED (dof), CP_E_HIP. */
int cp_planner_create(const cp_robot* robot, const cp_plan_opts* opts, cp_planner** out);
void cp_planner_destroy(cp_planner* planner);
/* Synchronous on `stream` (NULL = default).  start, goal: [dof] host doubles,
 * inside the limits, on the manifold (||e||_inf < tau_task) and collision-free.
 * Returns CP_OK with the path in out, CP_NO_SOLUTION when max_rounds pass
 * without a connection, CP_E_START / CP_E_GOAL for a bad endpoint,
 * CP_E_CAPACITY when out->capacity < out->len or a tree fills up.
 * stats: nullable.  A planner serves one call at a time. */
int cp_plan(cp_planner* planner, const cp_env* env, const cp_constraint* constraint,
            const double* start, const double* goal, uint64_t seed, cp_path* out,
            cp_plan_stats* stats, void* stream);
/* The search tree `tree` (0: start, 1: goal) as the last cp_plan left it:
 * *count nodes (capped at the capacity), q [count][dof] host doubles (the
 * device floats widened), parent [count] (-1 for the root).  Returns
 * CP_E_CAPACITY with *count set when capacity < *count.  Synchronous. */
int cp_planner_tree(const cp_planner* planner, int32_t tree, int32_t capacity, double* q,
                    int32_t* parent, int32_t* count);
/* Learned warm start for the planner's extensions (paper Section III-A: the
 * projection of a straight segment; the network is this library's extension,
 * see project_motions_warm): with a network set, every extension's first
 * motion q_near -> q_steer is projected from the straight waypoints plus the
 * network's corrections, and again from the straight line if that fails;
 * the connect steps project plainly.  A round is then three launches
 * (samples, the fused network, extensions) and uses the library's round
 * kernels, not ones compiled for the robot.  mlp = NULL switches it off.
 * The network is borrowed (it must outlive the plans) and must have the
 * fused shape (see project_motions_warm_noalloc) with n_in = dof + 6 (+ 12
 * for a relative pose), n_out = dof; that is checked by cp_plan.  Errors:
 * CP_E_ARG, CP_E_UNSUPPORTED (with CP_SELF_COLLISION or a projector variant
 * other than CP_PROJECT_PARALLEL), CP_E_HIP (round buffers). */
int cp_planner_set_warm(cp_planner* planner, const cp_mlp* mlp);
/* One-shot form: creates a planner with opts (NULL = defaults), plans on the
 * default stream, destroys it. */
int plan(const cp_robot* robot, const cp_env* env, const cp_constraint* constraint,
         const double* start, const double* goal, uint64_t seed, const cp_plan_opts* opts,
         cp_path* out);

/* ------------------------------------------------------------ batched planning */

/* Many independent queries (robots, DOF, scenes, constraint kinds may all
 * differ) planned together (paper Section III: extensions are independent).
 * Every query owns groups_per_query extensions per round, each the
 * extension step of cp_plan.  A round is one launch: wavefronts take
 * (query, extension) tasks from a device counter until none is left, each
 * running the code specialised for its query's (DOF, constraint kind), and
 * the last wavefront to finish publishes the round's nodes.  With
 * CP_BATCH_PER_CLASS (or a warm start, or classes from both sets below) a
 * round is instead one launch per (DOF, kind) class plus a publish launch.
 * rounds_per_graph rounds are captured in a HIP graph that is replayed until
 * every query is solved, out of budget (max_rounds, rounded up to a whole
 * replay) or out of tree capacity.  Each query's samples depend on its seed
 * only, not on the other queries of the batch.
 * Supported: dof 6, 7, 9 with no / pose constraint; dof 14 with pose /
 * relative-pose constraint. */
enum { CP_BATCH_PER_CLASS = 1 };
typedef struct cp_batch_opts {
  cp_proj_params proj;        /* W and sphere_batch shared by the batch */
  int32_t groups_per_query;   /* wavefronts per query per round (16) */
  int32_t max_rounds;         /* round budget (500) */
  int32_t capacity;           /* nodes per tree per query (2048) */
  int32_t max_connect;        /* (64) */
  int32_t rounds_per_graph;   /* rounds per graph replay (4) */
  int32_t flags;              /* CP_BATCH_PER_CLASS (0) */
} cp_batch_opts;

typedef struct cp_query {
  const cp_robot* robot;
  const cp_env* env;
  const cp_constraint* constraint;
  const double* start;        /* [dof] host */
  const double* goal;         /* [dof] host */
  uint64_t seed;
} cp_query;

typedef struct cp_batch cp_batch;   /* opaque: tree pools for max_queries queries */

void cp_batch_opts_default(cp_batch_opts* o);
int cp_batch_create(const cp_batch_opts* opts, int32_t max_queries, int32_t max_dof,
                    cp_batch** out);
void cp_batch_destroy(cp_batch* batch);
/* Synchronous (waits for `stream` first, works on its own stream).
 * status[i]: CP_OK (path in paths[i]), CP_NO_SOLUTION, CP_E_START,
 * CP_E_GOAL, CP_E_CAPACITY (tree full or paths[i].capacity too small).
 * stats nullable ([n]).  Returns CP_OK unless the call itself fails. */
int cp_plan_batch(cp_batch* batch, int32_t n, const cp_query* queries, cp_path* paths,
                  int32_t* status, cp_plan_stats* stats, void* stream);
/* Learned warm start for the batch (as cp_planner_set_warm): every query of
 * the next cp_plan_batch calls must then use the same robot handle and an
 * identical constraint (a network serves one robot and one constraint;
 * otherwise cp_plan_batch returns CP_E_UNSUPPORTED), and a round becomes
 * three launches (samples, network, extensions).  mlp = NULL switches it
 * off; the network is borrowed. */
int cp_batch_set_warm(cp_batch* batch, const cp_mlp* mlp);

#ifdef __cplusplus
}
#endif
#endif

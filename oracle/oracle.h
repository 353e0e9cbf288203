/* FP64 CPU oracle for cpRRTC's constrained motion projection and validation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no source,
 * header, table or helper with the HIP library, and the HIP library never
 * calls it.
 *
 * Every quantity is double precision; float inputs are promoted exactly by
 * the caller.  Nothing here is blocked, fused or reordered beyond what the
 * definitions state.
 */
#ifndef CPRRTC_ORACLE_H
#define CPRRTC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_REVOLUTE = 0, OR_PRISMATIC = 1 };
enum { OR_CON_NONE = 0, OR_CON_POSE = 1, OR_CON_REL_POSE = 2 };
enum { OR_MOTION_VALID = 0, OR_MOTION_PROJ_FAIL = 1, OR_MOTION_COLLISION = 2 };

typedef struct {
  int32_t dof, n_chains;
  const int32_t* type;        /* [dof] OR_REVOLUTE / OR_PRISMATIC */
  const int32_t* chain;       /* [dof] chain of each joint */
  const double* alpha;        /* [dof] alpha_{i-1} */
  const double* a;            /* [dof] a_{i-1} */
  const double* d;            /* [dof] constant part of d_i */
  const double* theta;        /* [dof] constant part of theta_i */
  const double* lo;           /* [dof] */
  const double* hi;           /* [dof] */
  const double* base;         /* [n_chains][16] row-major */
  const double* tool;         /* [n_chains][16] row-major */
  int32_t n_spheres;
  const int32_t* sphere_link; /* [S] joint whose frame carries the sphere */
  const double* sphere;       /* [S][4] local centre, radius */
} or_robot;

typedef struct {
  int32_t n_aabb, n_obb, n_sphere, n_capsule, n_cylinder;
  const double* aabb;      /* [n][6]  centre, half extents */
  const double* obb;       /* [n][15] centre, R row-major (columns = axes), half extents */
  const double* sphere;    /* [n][4]  centre, radius */
  const double* capsule;   /* [n][7]  p0, p1, radius */
  const double* cylinder;  /* [n][8]  centre, unit axis, half length, radius */
} or_env;

typedef struct {
  int32_t kind;
  int32_t mask[6];          /* x y z roll pitch yaw */
  double frame[16];         /* constraint frame in world, row-major */
  double target[6];
  double rel_target[16];    /* pose of end effector 2 in end effector 1's frame */
} or_constraint;

typedef struct {
  int32_t W;                /* waypoints per motion, including the fixed start */
  int32_t max_iters;
  double tau;               /* spacing target (interpolation step) */
  double tau_sm;            /* spacing slack: valid spacing is < tau + tau_sm */
  double tau_task;          /* task tolerance on the infinity norm of the error */
  double alpha;             /* step factor */
  double lambda;            /* damping of the least-squares step */
  int32_t variant;          /* OR_PROJECT_PARALLEL, _INDEPENDENT or _SEQUENTIAL */
  int32_t self_collision;   /* 1: motions are also checked against the robot itself */
} or_params;

/* Projection operators: Algorithm 1 (PARALLEL); the same iteration without
 * the smoothing term (INDEPENDENT: the naive parallel projection Section
 * III-A sets aside); waypoint after waypoint (SEQUENTIAL: the CBiRRT-style
 * projection of cpRRTC-Naive in the Evaluation). */
enum { OR_PROJECT_PARALLEL = 0, OR_PROJECT_INDEPENDENT = 1, OR_PROJECT_SEQUENTIAL = 2 };

/* Kinematics.  frames: [dof][16] joint frames in world; ee: [n_chains][16]. */
void or_fk(const or_robot* r, const double* q, double* frames, double* ee);
int32_t or_task_dim(const or_constraint* c);
/* Full 6-vector task coordinates (before masking) and masked error/Jacobian. */
void or_task_coords(const or_robot* r, const or_constraint* c, const double* q, double* x6);
int32_t or_task_error(const or_robot* r, const or_constraint* c, const double* q, double* e);
int32_t or_task_jacobian(const or_robot* r, const or_constraint* c, const double* q, double* J);
void or_dls_step(const double* J, const double* e, int32_t m, int32_t n, double lambda, double* g);

/* Geometry. */
double or_sd_aabb(const double* c, double r, const double* box);
double or_sd_obb(const double* c, double r, const double* box);
double or_sd_sphere(const double* c, double r, const double* s);
double or_sd_capsule(const double* c, double r, const double* cap);
double or_sd_cylinder(const double* c, double r, const double* cyl);
void or_sphere_centres(const or_robot* r, const double* q, double* xyz);
double or_config_min_sd(const or_robot* r, const or_env* env, const double* q);

/* Self-collision (specified here; the paper checks the robot against the
 * environment only).  Checked pairs: spheres whose links lie in different
 * chains, or in one chain at least two joints apart, and that are clear by
 * more than OR_SELF_HOME_CLEARANCE at the home configuration (every joint
 * at 0 clamped into its limits; pairs overlapping there touch across a
 * joint by construction and are allowed).  or_self_pairs writes up to
 * `capacity` pairs (s, t), s < t, description order, lexicographic, and
 * returns their number.  or_self_min_sd: minimum over the given pairs of
 * |c_s - c_t| - r_s - r_t (DBL_MAX without pairs); a configuration
 * self-collides iff it is <= 0. */
#define OR_SELF_HOME_CLEARANCE 1e-3
int32_t or_self_pairs(const or_robot* r, int32_t capacity, int32_t* pairs);
double or_self_min_sd(const or_robot* r, int32_t n_pairs, const int32_t* pairs, const double* q);
void or_self_cc_batch(const or_robot* r, int32_t n_cfg, const double* q, uint8_t* collide,
                      double* min_sd, int32_t n_threads);

/* Batched entry points (OpenMP over independent items; n_threads <= 0 means 1). */
void or_fk_cc_batch(const or_robot* r, const or_env* env, int32_t n_cfg, const double* q,
                    uint8_t* collide, double* min_sd, int32_t n_threads);

int32_t or_parallel_project(const or_robot* r, const or_constraint* c, const or_params* p,
                            double* xi, int32_t* iters, double* margin, int32_t* trace_prog);

void or_project_validate_motions(const or_robot* r, const or_env* env, const or_constraint* c,
                                 const or_params* p, int32_t n_motions, const double* q_from,
                                 const double* q_to, double* xi, int32_t* status, int32_t* iters,
                                 double* proj_margin, double* min_sd, int32_t n_threads);

/* Sequential projection: for k = 1..W-1 in turn, waypoint k starts at the
 * projected waypoint k-1 plus one interpolation step (xi_init[k] -
 * xi_init[k-1]) and takes damped least-squares steps (no smoothing term),
 * validity (||e||_inf < tau_task and ||xi[k] - xi[k-1]|| - tau < tau_sm)
 * checked before each step, at most max_iters checks; the motion fails at
 * the first waypoint that never becomes valid.  *iters: checks summed over
 * the waypoints; *margin: as or_parallel_project. */
int32_t or_sequential_project(const or_robot* r, const or_constraint* c, const or_params* p,
                              double* xi, int32_t* iters, double* margin);
/* The operator p->variant selects (or_parallel_project or
 * or_sequential_project). */
int32_t or_project_motion(const or_robot* r, const or_constraint* c, const or_params* p,
                          double* xi, int32_t* iters, double* margin);

int32_t or_project_config(const or_robot* r, const or_constraint* c, const double* q_in,
                          double tol, int32_t max_iters, double alpha, double lambda,
                          double* q_out, int32_t* iters);

/* Sequential constrained RRT-Connect with the same semantics as the GPU
 * planner run with one extension per round.  path: [cap_path][dof];
 * returns 1 if a path was found (*path_len rows), 0 if the sample budget ran
 * out, -1 if a tree filled up, -2 if the path buffer is too small. */
int32_t or_plan(const or_robot* r, const or_env* env, const or_constraint* c, const or_params* p,
                const double* start, const double* goal, uint64_t seed, int32_t max_samples,
                int32_t capacity, int32_t max_connect, double* path, int32_t cap_path,
                int32_t* path_len, int32_t* nodes);

/* The GPU planner's round schedule run sequentially (its lockstep replay):
 * in round r (0-based) extension g = 0..n_groups-1 takes Halton index
 * r * n_groups + g + 1, grows tree g & 1 and searches only the nodes present
 * when the round began; nodes are appended in extension order.  Stops in the
 * round the trees connect or after `rounds` rounds.  q0/q1: [capacity][dof],
 * parent0/parent1 and band0/band1: [capacity], counts[2].  A decision lies
 * in the band when it is near its threshold: a sample coordinate within
 * 1e-5 of wrapping, a nearest-node runner-up within 1e-4, a projection
 * margin or |signed distance| below 1e-5, a connection or progress distance
 * within 1e-4.  band0/band1[i] = 1 when a decision of the extension that
 * appended node i, up to that node, was in the band.  *found_round: 1-based
 * round of the connection, else 0; *band_round: 1-based first round with an
 * extension holding a band decision, else 0; *band_extensions: how many
 * extensions held one.  Returns 0, or -1 when a tree fills up. */
int32_t or_plan_rounds(const or_robot* r, const or_env* env, const or_constraint* c,
                       const or_params* p, const double* start, const double* goal, uint64_t seed,
                       int32_t n_groups, int32_t rounds, int32_t capacity, int32_t max_connect,
                       double* q0, int32_t* parent0, int32_t* band0, double* q1, int32_t* parent1,
                       int32_t* band1, int32_t* counts, int32_t* found_round, int32_t* band_round,
                       int32_t* band_extensions);

/* Re-validation of a dense path: limits, ||e||_inf < tau_task + slack,
 * consecutive spacing < tau + tau_sm + slack, minimum signed distance of every
 * waypoint.  out[0] = worst task error, out[1] = worst spacing, out[2] =
 * minimum signed distance, out[3] = 1 if all waypoints are inside the limits. */
void or_path_report(const or_robot* r, const or_env* env, const or_constraint* c,
                    const double* path, int32_t len, double* out);

/* Multilayer perceptron with SiLU hidden activations (the learned warm start).
 * dims[0..n_layers]: widths; params: per layer W [dims[l+1]][dims[l]]
 * row-major then b [dims[l+1]].  x [M][dims[0]], y/t [M][dims[n_layers]].
 * or_mlp_gradients returns the mean squared error over all outputs and
 * writes its gradient (same layout as params). */
void or_mlp_forward(int32_t n_layers, const int32_t* dims, const double* params, int32_t M,
                    const double* x, double* y);
double or_mlp_gradients(int32_t n_layers, const int32_t* dims, const double* params, int32_t M,
                        const double* x, const double* t, double* grad);

#ifdef __cplusplus
}
#endif
#endif

"""Seeded synthetic inputs: robots, scenes, constraints and raw configurations.

This module draws random numbers and lays them out; it computes nothing the
planner computes (no kinematics, no distances, no projection).  Both the HIP
path and the FP64 oracle consume what it returns, so it imports nothing else
from this package and nothing from the oracle.

The paper evaluates on MotionBenchMaker scenes with the Fetch and Franka
robots and on cuRobo's constrained-planning tutorial with random cuboids
(Evaluation section).  None of those assets exist here; seeded stand-ins of
the same kind are drawn instead:

* robots are serial revolute chains in modified Denavit-Hartenberg form
  (Craig's convention) carrying collision spheres on their links, optionally
  on a two-joint prismatic planar base, or two arms on one base;
* scenes are sets of primitives (axis-aligned boxes, oriented boxes, spheres,
  capsules, solid cylinders) uniform in a cube over the robot's base: 1.2 m
  for the plain scene; 3.0 m (300 primitives) and 3.6 m (1000 primitives) for
  the cluttered ones, where a 1.2 m cube would leave no collision-free
  configuration at all; a keep-out column around each arm base keeps the
  shoulder free;
* constraints lock end-effector axes (roll/pitch = upright, a horizontal
  plane plus upright), or fix the relative pose of two end effectors.

Layouts (all float64 / int32 numpy arrays):

robot = dict(
    dof, n_chains,
    joint_type[dof]   0 revolute, 1 prismatic
    joint_chain[dof]  chain index, joints of chain 0 first, then chain 1
    alpha[dof], a[dof]  alpha_{i-1}, a_{i-1} of joint i
    d[dof], theta[dof]  constant parts of d_i, theta_i (the joint adds q_i)
    lo[dof], hi[dof]    joint limits
    base[n_chains,4,4], tool[n_chains,4,4]  homogeneous transforms
    sphere_link[S]      joint index whose frame carries sphere s
    sphere[S,4]         centre (x, y, z) in that frame, radius
)
env = dict(aabb[n,6] (centre, half extents), obb[n,15] (centre, R row-major
    whose columns are the box axes, half extents), sphere[n,4] (centre, radius),
    capsule[n,7] (p0, p1, radius), cylinder[n,8] (centre, unit axis,
    half length, radius))
constraint = dict(kind 0 none / 1 pose mask / 2 relative pose,
    mask[6] over (x, y, z, roll, pitch, yaw), frame[4,4] constraint frame in
    world, target[6] locked values in that frame, rel_target[4,4] pose of
    end effector 2 in end effector 1's frame)
"""
from __future__ import annotations

import math

import numpy as np

REVOLUTE, PRISMATIC = 0, 1
CON_NONE, CON_POSE, CON_REL_POSE = 0, 1, 2
JOINT_LIMIT = 2.8          # rad, revolute joints
BASE_LIMIT = 1.0           # m, prismatic base joints
TOOL_OFFSET = 0.1          # m along the last joint axis


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _eye4(n: int = 1) -> np.ndarray:
    return np.repeat(np.eye(4)[None], n, axis=0)


def _trans(x: float, y: float, z: float) -> np.ndarray:
    t = np.eye(4)
    t[:3, 3] = (x, y, z)
    return t


def _rot_y(angle: float) -> np.ndarray:
    c, s = math.cos(angle), math.sin(angle)
    t = np.eye(4)
    t[0, 0], t[0, 2], t[2, 0], t[2, 2] = c, s, -s, c
    return t


def _arm_dh(rng: np.random.Generator, n: int):
    """Per-joint DH rows of an n-joint revolute arm: d_i ~ U[0.05, 0.4] m,
    a = 0, alpha_0 = 0 and alpha_{i-1} = +-pi/2 (sign drawn) for i >= 2."""
    d = rng.uniform(0.05, 0.4, n)
    sign = rng.integers(0, 2, n) * 2 - 1
    alpha = sign * (math.pi / 2.0)
    alpha[0] = 0.0
    return alpha, np.zeros(n), d, np.zeros(n)


def _next_origin(alpha_next: float, a_next: float, d_next: float) -> np.ndarray:
    """Origin of frame k+1 written in frame k (the DH row of joint k+1 read as
    a fixed offset): this is where link k ends, so its spheres lie on the
    segment from the frame-k origin to this point."""
    return np.array([a_next, -math.sin(alpha_next) * d_next, math.cos(alpha_next) * d_next])


def _link_spheres(rng, alpha, a, d, joint_ids, tool_z, n_spheres, r_lo, r_hi):
    """Spheres assigned round-robin to the listed joints' frames, each centred
    at t * (end of that link), t ~ U[0, 1], radius ~ U[r_lo, r_hi]."""
    links, rows = [], []
    for s in range(n_spheres):
        j = joint_ids[s % len(joint_ids)]
        pos = int(np.searchsorted(joint_ids, j))
        if pos + 1 < len(joint_ids):
            nj = joint_ids[pos + 1]
            end = _next_origin(alpha[nj], a[nj], d[nj])
        else:
            end = np.array([0.0, 0.0, tool_z])
        t = rng.uniform(0.0, 1.0)
        r = rng.uniform(r_lo, r_hi)
        links.append(j)
        rows.append([*(t * end), r])
    order = np.argsort(np.asarray(links), kind="stable")
    return (np.asarray(links, np.int32)[order],
            np.asarray(rows, np.float64).reshape(-1, 4)[order])


def make_arm(seed: int, dof: int = 7, n_spheres: int = 20,
             r_lo: float = 0.03, r_hi: float = 0.08) -> dict:
    """Single revolute arm based at the world origin, joint 1 axis = world z."""
    rng = rng_for(seed)
    alpha, a, d, theta = _arm_dh(rng, dof)
    ids = np.arange(dof)
    sl, sp = _link_spheres(rng, alpha, a, d, ids, TOOL_OFFSET, n_spheres, r_lo, r_hi)
    return dict(
        dof=dof, n_chains=1,
        joint_type=np.zeros(dof, np.int32), joint_chain=np.zeros(dof, np.int32),
        alpha=alpha, a=a, d=d, theta=theta,
        lo=np.full(dof, -JOINT_LIMIT), hi=np.full(dof, JOINT_LIMIT),
        base=_eye4(1), tool=_trans(0, 0, TOOL_OFFSET)[None].copy(),
        sphere_link=sl, sphere=sp,
    )


def make_mobile_arm(seed: int, arm_dof: int = 7, n_arm_spheres: int = 20,
                    n_base_spheres: int = 8) -> dict:
    """Arm on a planar base: joint 1 slides along world x, joint 2 along
    world y (both +-1 m), then an arm_dof revolute arm whose first axis is
    world z.  The base transform turns z onto world x; joint 2 twists by
    -pi/2 with theta offset pi/2 so its axis is world y; joint 3 twists by
    -pi/2 again so its axis is world z.  Base spheres ride in joint 2's frame,
    whose axes are (x, y, z) = (-x_w, z_w, y_w)."""
    rng = rng_for(seed)
    alpha_arm, a_arm, d_arm, th_arm = _arm_dh(rng, arm_dof)
    alpha_arm[0] = -math.pi / 2.0
    dof = arm_dof + 2
    alpha = np.concatenate([[0.0, -math.pi / 2.0], alpha_arm])
    a = np.concatenate([[0.0, 0.0], a_arm])
    d = np.concatenate([[0.0, 0.0], d_arm])
    theta = np.concatenate([[0.0, math.pi / 2.0], th_arm])
    jt = np.array([PRISMATIC, PRISMATIC] + [REVOLUTE] * arm_dof, np.int32)
    lo = np.concatenate([[-BASE_LIMIT] * 2, [-JOINT_LIMIT] * arm_dof])
    hi = -lo
    arm_ids = np.arange(2, dof)
    sl, sp = _link_spheres(rng, alpha, a, d, arm_ids, TOOL_OFFSET,
                           n_arm_spheres, 0.03, 0.08)
    base_rows = []
    for k in range(n_base_spheres):
        wx, wy = rng.uniform(-0.2, 0.2, 2)
        wz = rng.uniform(0.05, 0.15)
        base_rows.append([-wx, wz, wy, rng.uniform(0.06, 0.1)])
    sl = np.concatenate([np.full(n_base_spheres, 1, np.int32), sl]).astype(np.int32)
    sp = np.concatenate([np.asarray(base_rows), sp])
    return dict(
        dof=dof, n_chains=1, joint_type=jt, joint_chain=np.zeros(dof, np.int32),
        alpha=alpha, a=a, d=d, theta=theta, lo=lo, hi=hi,
        base=_rot_y(math.pi / 2.0)[None].copy(),
        tool=_trans(0, 0, TOOL_OFFSET)[None].copy(),
        sphere_link=sl, sphere=sp,
    )


def make_dual_arm(seed: int, arm_dof: int = 7, spheres_per_arm: int = 80) -> dict:
    """Two revolute arms on one base, bases at (0, -0.35, 0) and (0, +0.35, 0)."""
    rng = rng_for(seed)
    parts = []
    for arm in range(2):
        alpha, a, d, theta = _arm_dh(rng, arm_dof)
        ids = np.arange(arm_dof)
        sl, sp = _link_spheres(rng, alpha, a, d, ids, TOOL_OFFSET,
                               spheres_per_arm, 0.03, 0.08)
        parts.append((alpha, a, d, theta, sl + arm * arm_dof, sp))
    dof = 2 * arm_dof
    cat = lambda i: np.concatenate([parts[0][i], parts[1][i]])
    base = np.stack([_trans(0, -0.35, 0), _trans(0, 0.35, 0)])
    return dict(
        dof=dof, n_chains=2, joint_type=np.zeros(dof, np.int32),
        joint_chain=np.repeat(np.arange(2, dtype=np.int32), arm_dof),
        alpha=cat(0), a=cat(1), d=cat(2), theta=cat(3),
        lo=np.full(dof, -JOINT_LIMIT), hi=np.full(dof, JOINT_LIMIT),
        base=base, tool=np.stack([_trans(0, 0, TOOL_OFFSET)] * 2),
        sphere_link=cat(4).astype(np.int32), sphere=cat(5),
    )


def _random_rotation(rng) -> np.ndarray:
    """Uniform rotation from a normalised Gaussian quaternion (w, x, y, z)."""
    qv = rng.normal(size=4)
    w, x, y, z = qv / np.linalg.norm(qv)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def _unit(rng) -> np.ndarray:
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def _centre(rng, cube_side: float, keep_out) -> np.ndarray:
    """Centre uniform in the cube [-s/2, s/2]^2 x [0, s], redrawn while it falls
    in a keep-out column (x, y, radius, z_max) around a robot base."""
    lo = np.array([-cube_side / 2.0, -cube_side / 2.0, 0.0])
    hi = np.array([cube_side / 2.0, cube_side / 2.0, cube_side])
    while True:
        c = rng.uniform(lo, hi)
        if all(math.hypot(c[0] - x, c[1] - y) >= r or c[2] > zmax for x, y, r, zmax in keep_out):
            return c


BASE_KEEP_OUT = ((0.0, 0.0, 0.25, 0.5),)
DUAL_KEEP_OUT = ((0.0, -0.35, 0.25, 0.5), (0.0, 0.35, 0.25, 0.5))


def empty_env() -> dict:
    return dict(aabb=np.zeros((0, 6)), obb=np.zeros((0, 15)), sphere=np.zeros((0, 4)),
                capsule=np.zeros((0, 7)), cylinder=np.zeros((0, 8)))


def make_boxes(seed: int, n: int = 10, side_lo: float = 0.05, side_hi: float = 0.3,
               cube_side: float = 1.2, keep_out=BASE_KEEP_OUT) -> dict:
    """n axis-aligned boxes, sides ~ U[side_lo, side_hi], centres in the cube."""
    rng = rng_for(seed)
    env = empty_env()
    rows = []
    for _ in range(n):
        c = _centre(rng, cube_side, keep_out)
        rows.append([*c, *(rng.uniform(side_lo, side_hi, 3) / 2.0)])
    env["aabb"] = np.asarray(rows, np.float64).reshape(-1, 6)
    return env


def make_mixed(seed: int, n: int = 300, size_lo: float = 0.02, size_hi: float = 0.25,
               cube_side: float = 1.2, keep_out=BASE_KEEP_OUT,
               frac=(0.4, 0.3, 0.15, 0.15)) -> dict:
    """n primitives: 40% oriented boxes, 30% spheres, 15% capsules and 15%
    solid cylinders (by default); every size (box side, diameter, length)
    ~ U[size_lo, size_hi]; orientations uniform."""
    rng = rng_for(seed)
    counts = [int(round(f * n)) for f in frac]
    counts[0] += n - sum(counts)
    env = empty_env()
    obb, sph, cap, cyl = [], [], [], []
    u = lambda k=1: rng.uniform(size_lo, size_hi, k)
    for _ in range(counts[0]):
        c = _centre(rng, cube_side, keep_out)
        obb.append([*c, *_random_rotation(rng).reshape(-1), *(u(3) / 2.0)])
    for _ in range(counts[1]):
        c = _centre(rng, cube_side, keep_out)
        sph.append([*c, u()[0] / 2.0])
    for _ in range(counts[2]):
        c = _centre(rng, cube_side, keep_out)
        ax, length, r = _unit(rng), u()[0], u()[0] / 2.0
        cap.append([*(c - 0.5 * length * ax), *(c + 0.5 * length * ax), r])
    for _ in range(counts[3]):
        c = _centre(rng, cube_side, keep_out)
        ax, length, r = _unit(rng), u()[0], u()[0] / 2.0
        cyl.append([*c, *ax, 0.5 * length, r])
    env["obb"] = np.asarray(obb, np.float64).reshape(-1, 15)
    env["sphere"] = np.asarray(sph, np.float64).reshape(-1, 4)
    env["capsule"] = np.asarray(cap, np.float64).reshape(-1, 7)
    env["cylinder"] = np.asarray(cyl, np.float64).reshape(-1, 8)
    return env


def subdivide_boxes(env: dict, k: int) -> dict:
    """Every axis-aligned box split into k x k x k boxes that tile it exactly
    (the union, hence every signed distance from outside and every collision
    verdict, is unchanged; the primitive count grows k^3-fold)."""
    out = dict(env)
    rows = []
    for b in np.asarray(env["aabb"], np.float64).reshape(-1, 6):
        c, h = b[:3], b[3:]
        hs = h / k
        for i in range(k):
            for j in range(k):
                for l in range(k):
                    off = np.array([i, j, l], np.float64)
                    rows.append([*(c - h + hs * (2.0 * off + 1.0)), *hs])
    out["aabb"] = np.asarray(rows, np.float64).reshape(-1, 6)
    return out


def env_count(env: dict) -> int:
    return sum(len(env[k]) for k in ("aabb", "obb", "sphere", "capsule", "cylinder"))


def no_constraint() -> dict:
    return dict(kind=CON_NONE, mask=np.zeros(6, np.int32), frame=np.eye(4),
                target=np.zeros(6), rel_target=np.eye(4))


def upright() -> dict:
    """End effector roll = pitch = 0 in the world frame (its z axis vertical)."""
    return dict(kind=CON_POSE, mask=np.array([0, 0, 0, 1, 1, 0], np.int32),
                frame=np.eye(4), target=np.zeros(6), rel_target=np.eye(4))


def plane_upright(seed: int, z_lo: float = 0.3, z_hi: float = 0.9) -> dict:
    """End effector on the horizontal plane z = z_c, z_c ~ U[z_lo, z_hi], and upright."""
    z_c = rng_for(seed).uniform(z_lo, z_hi)
    target = np.zeros(6)
    target[2] = z_c
    return dict(kind=CON_POSE, mask=np.array([0, 0, 1, 1, 1, 0], np.int32),
                frame=np.eye(4), target=target, rel_target=np.eye(4))


def line_constraint(seed: int) -> dict:
    """End effector on a horizontal line: y = y_c and z = z_c locked."""
    rng = rng_for(seed)
    target = np.zeros(6)
    target[1] = rng.uniform(-0.2, 0.2)
    target[2] = rng.uniform(0.3, 0.9)
    return dict(kind=CON_POSE, mask=np.array([0, 1, 1, 0, 0, 0], np.int32),
                frame=np.eye(4), target=target, rel_target=np.eye(4))


def fixed_orientation(seed: int) -> dict:
    """End effector orientation fixed (roll = pitch = 0, yaw = y_c ~ U[-pi, pi]),
    position free."""
    target = np.zeros(6)
    target[5] = rng_for(seed).uniform(-math.pi, math.pi)
    return dict(kind=CON_POSE, mask=np.array([0, 0, 0, 1, 1, 1], np.int32),
                frame=np.eye(4), target=target, rel_target=np.eye(4))


def relative_pose(gap: float = 0.3) -> dict:
    """Second end effector held at (0, gap, 0) in the first one's frame,
    turned by pi about that frame's x axis (the two tools face each other)."""
    rel = np.eye(4)
    rel[:3, :3] = np.array([[1.0, 0, 0], [0, -1.0, 0], [0, 0, -1.0]])
    rel[:3, 3] = (0.0, gap, 0.0)
    return dict(kind=CON_REL_POSE, mask=np.ones(6, np.int32), frame=np.eye(4),
                target=np.zeros(6), rel_target=rel)


def random_configs(robot: dict, n: int, seed: int) -> np.ndarray:
    """n configurations uniform within the joint limits, float64 [n, dof]."""
    rng = rng_for(seed)
    return rng.uniform(robot["lo"], robot["hi"], size=(n, robot["dof"]))


def random_displacements(robot: dict, q_from: np.ndarray, max_len: float, seed: int,
                         min_frac: float = 0.5) -> np.ndarray:
    """Motion end points: q_from plus a uniformly oriented step whose length is
    ~ U[min_frac, 1] * max_len, clipped into the joint limits."""
    rng = rng_for(seed)
    n, dof = q_from.shape
    v = rng.normal(size=(n, dof))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    length = rng.uniform(min_frac, 1.0, size=(n, 1)) * max_len
    return np.clip(q_from + v * length, robot["lo"], robot["hi"])


# Named workloads -----------------------------------------------------------

def workload(name: str, seed: int) -> dict:
    """Robot, scene and constraint of a named workload.

    plain      7-DOF arm, 20 spheres, 10 axis-aligned boxes, upright (tol 1e-3)
    cluttered  7-DOF arm, 100 spheres, 300 mixed primitives, plane + upright
    mobile     9-DOF (planar base + 7-DOF arm), mixed primitives
    dual       two 7-DOF arms, 160 spheres, 1000 mixed primitives, relative pose
    """
    if name == "plain":
        return dict(robot=make_arm(seed, 7, 20), env=make_boxes(seed + 1, 10),
                    constraint=upright(), tau_task=1e-3)
    if name == "cluttered":
        return dict(robot=make_arm(seed, 7, 100), env=make_mixed(seed + 1, 300, cube_side=3.0),
                    constraint=plane_upright(seed + 2), tau_task=1e-3)
    if name == "mobile":
        return dict(robot=make_mobile_arm(seed), env=make_mixed(seed + 1, 100, cube_side=3.0),
                    constraint=plane_upright(seed + 2), tau_task=1e-3)
    if name == "dual":
        return dict(robot=make_dual_arm(seed),
                    env=make_mixed(seed + 1, 1000, cube_side=3.6, keep_out=DUAL_KEEP_OUT),
                    constraint=relative_pose(), tau_task=1e-4)
    raise ValueError(f"unknown workload {name!r}")


def uneven_query(seed: int) -> dict:
    """One query of the uneven batch: DOF uniform in {6, 7, 9} (6: 17
    spheres, 7: 20, 9: planar base with 8 base spheres + 7-DOF arm with 20),
    round(exp U[ln 10, ln 1000]) mixed primitives in the 3.0 m cube, and a
    constraint uniform in {none, upright, plane + upright}; tolerance 1e-3."""
    rng = rng_for(seed)
    dof = int(rng.choice([6, 7, 9]))
    n_obs = int(round(math.exp(rng.uniform(math.log(10.0), math.log(1000.0)))))
    kind = int(rng.integers(0, 3))
    if dof == 9:
        robot = make_mobile_arm(seed)
    else:
        robot = make_arm(seed, dof, 17 if dof == 6 else 20)
    con = (no_constraint(), upright(), plane_upright(seed + 2))[kind]
    return dict(robot=robot, env=make_mixed(seed + 1, n_obs, cube_side=3.0), constraint=con,
                tau_task=1e-3)

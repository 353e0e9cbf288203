"""Python access to the FP64 CPU oracle (liboracle.so, built from oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use it.  It marshals the seeded input dictionaries into the
oracle's own structs; it shares no code with the HIP library or its binding.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_SANITIZE=1: a separate build with AddressSanitizer and
# UndefinedBehaviorSanitizer (the process must preload the sanitizer
# runtimes; tests/test_oracle_sanitized.py runs the oracle's pins that way)
SANITIZE = os.environ.get("ORACLE_SANITIZE") == "1"
LIB_PATH = os.path.join(_HERE, "liboracle_san.so" if SANITIZE else "liboracle.so")
SANITIZE_FLAGS = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                  "-fno-sanitize-recover=undefined"]

MOTION_VALID, MOTION_PROJ_FAIL, MOTION_COLLISION = 0, 1, 2

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_u8p = C.POINTER(C.c_uint8)


class _Robot(C.Structure):
    _fields_ = [("dof", C.c_int32), ("n_chains", C.c_int32),
                ("type", _ip), ("chain", _ip),
                ("alpha", _dp), ("a", _dp), ("d", _dp), ("theta", _dp),
                ("lo", _dp), ("hi", _dp), ("base", _dp), ("tool", _dp),
                ("n_spheres", C.c_int32), ("sphere_link", _ip), ("sphere", _dp)]


class _Env(C.Structure):
    _fields_ = [("n_aabb", C.c_int32), ("n_obb", C.c_int32), ("n_sphere", C.c_int32),
                ("n_capsule", C.c_int32), ("n_cylinder", C.c_int32),
                ("aabb", _dp), ("obb", _dp), ("sphere", _dp), ("capsule", _dp),
                ("cylinder", _dp)]


class _Constraint(C.Structure):
    _fields_ = [("kind", C.c_int32), ("mask", C.c_int32 * 6), ("frame", C.c_double * 16),
                ("target", C.c_double * 6), ("rel_target", C.c_double * 16)]


class _Params(C.Structure):
    _fields_ = [("W", C.c_int32), ("max_iters", C.c_int32), ("tau", C.c_double),
                ("tau_sm", C.c_double), ("tau_task", C.c_double), ("alpha", C.c_double),
                ("lam", C.c_double), ("variant", C.c_int32), ("self_collision", C.c_int32)]


PROJECT_PARALLEL, PROJECT_INDEPENDENT, PROJECT_SEQUENTIAL = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (OpenMP over independent items only)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        opt = SANITIZE_FLAGS if SANITIZE else ["-O2"]
        subprocess.check_call(["gcc", *opt, "-fPIC", "-shared", "-fopenmp", "-o", LIB_PATH,
                               src, "-lm"], cwd=_HERE)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        L.or_config_min_sd.restype = C.c_double
        for name in ("or_sd_aabb", "or_sd_obb", "or_sd_sphere", "or_sd_capsule", "or_sd_cylinder"):
            getattr(L, name).restype = C.c_double
            getattr(L, name).argtypes = [_dp, C.c_double, _dp]
        L.or_task_dim.restype = C.c_int32
        L.or_task_error.restype = C.c_int32
        L.or_task_jacobian.restype = C.c_int32
        L.or_parallel_project.restype = C.c_int32
        L.or_project_config.restype = C.c_int32
        L.or_self_pairs.restype = C.c_int32
        L.or_self_min_sd.restype = C.c_double
        _lib = L
    return _lib


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def _ptr(a, t=_dp):
    return a.ctypes.data_as(t)


class Robot:
    """Oracle view of a robot dictionary (keeps the arrays alive)."""

    def __init__(self, rd: dict):
        self.keep = dict(
            type=np.ascontiguousarray(rd["joint_type"], np.int32),
            chain=np.ascontiguousarray(rd["joint_chain"], np.int32),
            alpha=_f64(rd["alpha"]), a=_f64(rd["a"]), d=_f64(rd["d"]), theta=_f64(rd["theta"]),
            lo=_f64(rd["lo"]), hi=_f64(rd["hi"]),
            base=_f64(rd["base"]).reshape(-1), tool=_f64(rd["tool"]).reshape(-1),
            sphere_link=np.ascontiguousarray(rd["sphere_link"], np.int32),
            sphere=_f64(rd["sphere"]).reshape(-1),
        )
        k = self.keep
        self.dof = int(rd["dof"])
        self.n_chains = int(rd["n_chains"])
        self.n_spheres = len(k["sphere_link"])
        self.lo, self.hi = k["lo"], k["hi"]
        self.s = _Robot(self.dof, self.n_chains, _ptr(k["type"], _ip), _ptr(k["chain"], _ip),
                        _ptr(k["alpha"]), _ptr(k["a"]), _ptr(k["d"]), _ptr(k["theta"]),
                        _ptr(k["lo"]), _ptr(k["hi"]), _ptr(k["base"]), _ptr(k["tool"]),
                        self.n_spheres, _ptr(k["sphere_link"], _ip), _ptr(k["sphere"]))


class Env:
    def __init__(self, ed: dict):
        names = ("aabb", "obb", "sphere", "capsule", "cylinder")
        widths = (6, 15, 4, 7, 8)
        self.keep = {n: _f64(np.asarray(ed[n]).reshape(-1, w)) for n, w in zip(names, widths)}
        k = self.keep
        self.s = _Env(*(len(k[n]) for n in names), *(_ptr(k[n]) for n in names))


class Constraint:
    def __init__(self, cd: dict):
        self.s = _Constraint()
        self.s.kind = int(cd["kind"])
        for i in range(6):
            self.s.mask[i] = int(cd["mask"][i])
            self.s.target[i] = float(cd["target"][i])
        fr = np.asarray(cd["frame"], np.float64).reshape(-1)
        rt = np.asarray(cd["rel_target"], np.float64).reshape(-1)
        for i in range(16):
            self.s.frame[i] = fr[i]
            self.s.rel_target[i] = rt[i]
        self.m = lib().or_task_dim(C.byref(self.s))


def params(W=64, max_iters=32, tau=0.05, tau_sm=0.025, tau_task=1e-3, alpha=1.0, lam=1e-2,
           variant=PROJECT_PARALLEL, self_collision=False):
    return _Params(W, max_iters, tau, tau_sm, tau_task, alpha, lam, variant, int(self_collision))


# ------------------------------------------------------------------ wrappers

def fk(robot: Robot, q):
    q = _f64(q)
    frames = np.zeros((robot.dof, 4, 4))
    ee = np.zeros((robot.n_chains, 4, 4))
    lib().or_fk(C.byref(robot.s), _ptr(q), _ptr(frames), _ptr(ee))
    return frames, ee


def task_coords(robot: Robot, con: Constraint, q):
    q = _f64(q)
    x = np.zeros(6)
    lib().or_task_coords(C.byref(robot.s), C.byref(con.s), _ptr(q), _ptr(x))
    return x


def task_error(robot: Robot, con: Constraint, q):
    q = _f64(q)
    e = np.zeros(6)
    m = lib().or_task_error(C.byref(robot.s), C.byref(con.s), _ptr(q), _ptr(e))
    return e[:m].copy()


def task_jacobian(robot: Robot, con: Constraint, q):
    q = _f64(q)
    J = np.zeros(6 * robot.dof)
    m = lib().or_task_jacobian(C.byref(robot.s), C.byref(con.s), _ptr(q), _ptr(J))
    return J[: m * robot.dof].reshape(m, robot.dof).copy()


def dls_step(J, e, lam):
    J = _f64(J)
    e = _f64(e)
    m, n = J.shape
    g = np.zeros(n)
    lib().or_dls_step(_ptr(J), _ptr(e), C.c_int32(m), C.c_int32(n), C.c_double(lam), _ptr(g))
    return g


def sd(kind: str, centre, radius, prim):
    c = _f64(centre)
    p = _f64(prim)
    return getattr(lib(), "or_sd_" + kind)(_ptr(c), C.c_double(radius), _ptr(p))


def sphere_centres(robot: Robot, q):
    q = _f64(q)
    out = np.zeros((robot.n_spheres, 3))
    lib().or_sphere_centres(C.byref(robot.s), _ptr(q), _ptr(out))
    return out


def config_min_sd(robot: Robot, env: Env, q):
    q = _f64(q)
    return lib().or_config_min_sd(C.byref(robot.s), C.byref(env.s), _ptr(q))


def fk_cc_batch(robot: Robot, env: Env, q, n_threads: int = 1):
    q = _f64(q).reshape(-1, robot.dof)
    n = len(q)
    col = np.zeros(n, np.uint8)
    msd = np.zeros(n)
    lib().or_fk_cc_batch(C.byref(robot.s), C.byref(env.s), C.c_int32(n), _ptr(q),
                         _ptr(col, _u8p), _ptr(msd), C.c_int32(n_threads))
    return col, msd


def self_pairs(robot: Robot):
    """Checked self-collision sphere pairs [P][2] (s < t, description order)."""
    n = lib().or_self_pairs(C.byref(robot.s), C.c_int32(0), None)
    out = np.zeros((max(n, 1), 2), np.int32)
    lib().or_self_pairs(C.byref(robot.s), C.c_int32(n), _ptr(out, _ip))
    return out[:n].copy()


def self_min_sd(robot: Robot, q, pairs=None):
    pairs = self_pairs(robot) if pairs is None else np.ascontiguousarray(pairs, np.int32)
    return lib().or_self_min_sd(C.byref(robot.s), C.c_int32(len(pairs)),
                            _ptr(pairs.reshape(-1) if len(pairs) else np.zeros(2, np.int32), _ip),
                            _ptr(_f64(q)))


def self_cc_batch(robot: Robot, q, n_threads: int = 1):
    q = _f64(q).reshape(-1, robot.dof)
    n = len(q)
    col = np.zeros(n, np.uint8)
    msd = np.zeros(n)
    lib().or_self_cc_batch(C.byref(robot.s), C.c_int32(n), _ptr(q), _ptr(col, _u8p), _ptr(msd),
                           C.c_int32(n_threads))
    return col, msd


def shortcut(robot: Robot, env: Env, con: Constraint, prm, path, rounds: int, n_threads: int = 8):
    """Path shortcutting as specified for the library (the paper returns the
    planner's path as it is).  Per round: for every index i, the farthest
    j >= i + 2 with |P[j] - P[i]| <= (W-1) tau whose subpath is longer than
    the chord is a candidate; every candidate motion P[i] -> P[j] is
    projected and validated (Algorithm 1, then the collision check); it is
    accepted when valid, waypoint W-2 lies within tau + tau_sm of P[j], and
    the piece (waypoints 1..W-2, then P[j]) is shorter than P[i..j]; pieces
    replace their subpaths by decreasing gain, skipping any whose interval
    meets a kept one except at an end point; stop when none is accepted.
    Returns (path, dict(rounds, candidates, replaced, length_before,
    length_after))."""
    P = [np.asarray(x, np.float64) for x in _f64(path)]
    W = prm.W
    reach, link = (W - 1) * prm.tau, prm.tau + prm.tau_sm

    def length(v):
        return sum(np.linalg.norm(v[k] - v[k - 1]) for k in range(1, len(v)))

    stats = dict(rounds=0, candidates=0, replaced=0, length_before=length(P))
    for r in range(rounds):
        L = len(P)
        cand = []
        for i in range(L - 2):
            j = next((k for k in range(L - 1, i + 1, -1) if np.linalg.norm(P[k] - P[i]) <= reach),
                     None)
            if j is None:
                continue
            if length(P[i:j + 1]) - np.linalg.norm(P[j] - P[i]) <= 1e-9:
                continue
            cand.append((i, j))
        if not cand:
            break
        res = project_validate_motions(robot, env, con, prm, np.array([P[i] for i, _ in cand]),
                                       np.array([P[j] for _, j in cand]), n_threads=n_threads)
        stats["candidates"] += len(cand)
        acc = []
        for m, (i, j) in enumerate(cand):
            if res["status"][m] != MOTION_VALID:
                continue
            x = res["xi"][m]
            if not np.linalg.norm(x[W - 2] - P[j]) < link:
                continue
            piece = [P[i]] + [x[k] for k in range(1, W - 1)] + [P[j]]
            gain = length(P[i:j + 1]) - length(piece)
            if gain > 0:
                acc.append((gain, m, i, j))
        stats["rounds"] = r + 1
        if not acc:
            break
        acc.sort(key=lambda a: -a[0])          # stable: ties keep candidate order
        keep = []
        for gain, m, i, j in acc:
            if all(j <= ki or kj <= i for _, _, ki, kj in keep):
                keep.append((gain, m, i, j))
        keep.sort(key=lambda a: a[2])
        Q, at = [], 0
        for _, m, i, j in keep:
            Q += P[at:i + 1] + [res["xi"][m][k] for k in range(1, W - 1)]
            at = j
        P = Q + P[at:]
        stats["replaced"] += len(keep)
    stats["length_after"] = length(P)
    return np.array(P), stats


def parallel_project(robot: Robot, con: Constraint, prm, xi_init):
    xi = _f64(xi_init).copy()
    it = C.c_int32(0)
    mg = C.c_double(0)
    trace = np.zeros(prm.max_iters, np.int32)
    ok = lib().or_parallel_project(C.byref(robot.s), C.byref(con.s), C.byref(prm), _ptr(xi),
                                   C.byref(it), C.byref(mg), _ptr(trace, _ip))
    return bool(ok), xi, it.value, mg.value, trace[: it.value].copy()


def project_motion(robot: Robot, con: Constraint, prm, xi_init):
    """The projection operator prm.variant selects; returns (ok, xi, iters, margin)."""
    xi = _f64(xi_init).copy()
    it = C.c_int32(0)
    mg = C.c_double(0)
    ok = lib().or_project_motion(C.byref(robot.s), C.byref(con.s), C.byref(prm), _ptr(xi),
                                 C.byref(it), C.byref(mg))
    return bool(ok), xi, it.value, mg.value


def project_validate_motions(robot: Robot, env: Env, con: Constraint, prm, q_from, q_to,
                             n_threads: int = 1):
    q_from = _f64(q_from).reshape(-1, robot.dof)
    q_to = _f64(q_to).reshape(-1, robot.dof)
    M = len(q_from)
    xi = np.zeros((M, prm.W, robot.dof))
    status = np.zeros(M, np.int32)
    iters = np.zeros(M, np.int32)
    margin = np.zeros(M)
    msd = np.zeros(M)
    lib().or_project_validate_motions(C.byref(robot.s), C.byref(env.s), C.byref(con.s),
                                      C.byref(prm), C.c_int32(M), _ptr(q_from), _ptr(q_to),
                                      _ptr(xi), _ptr(status, _ip), _ptr(iters, _ip),
                                      _ptr(margin), _ptr(msd), C.c_int32(n_threads))
    return dict(xi=xi, status=status, iters=iters, proj_margin=margin, min_sd=msd)


def project_config(robot: Robot, con: Constraint, q, tol=1e-9, max_iters=100, alpha=1.0,
                   lam=1e-2):
    q = _f64(q)
    out = np.zeros(robot.dof)
    it = C.c_int32(0)
    ok = lib().or_project_config(C.byref(robot.s), C.byref(con.s), _ptr(q), C.c_double(tol),
                                 C.c_int32(max_iters), C.c_double(alpha), C.c_double(lam),
                                 _ptr(out), C.byref(it))
    return bool(ok), out, it.value


def plan(robot: Robot, env: Env, con: Constraint, prm, start, goal, seed, max_samples=20000,
         capacity=16384, max_connect=64):
    """Sequential FP64 planner; returns (status, path [len, dof] or None, nodes)."""
    start = _f64(start)
    goal = _f64(goal)
    cap_path = 2 * capacity * (prm.W - 1) + 2
    cap_path = min(cap_path, 200000)
    path = np.zeros((cap_path, robot.dof))
    plen = C.c_int32(0)
    nodes = np.zeros(2, np.int32)
    L = lib()
    L.or_plan.restype = C.c_int32
    st = L.or_plan(C.byref(robot.s), C.byref(env.s), C.byref(con.s), C.byref(prm), _ptr(start),
                   _ptr(goal), C.c_uint64(seed), C.c_int32(max_samples), C.c_int32(capacity),
                   C.c_int32(max_connect), _ptr(path), C.c_int32(cap_path), C.byref(plen),
                   _ptr(nodes, _ip))
    return st, (path[: plen.value].copy() if st == 1 else None), nodes


def plan_rounds(robot: Robot, env: Env, con: Constraint, prm, start, goal, seed, n_groups, rounds,
                capacity=4096, max_connect=64):
    """Round-synchronous FP64 planner (the GPU planner's schedule, one
    extension after another).  Returns dict(trees=[(q [count, dof],
    parent [count], band [count]) for tree 0, 1], found_round, band_round,
    band_extensions, status)."""
    start = _f64(start)
    goal = _f64(goal)
    n = robot.dof
    q = [np.zeros((capacity, n)), np.zeros((capacity, n))]
    par = [np.zeros(capacity, np.int32), np.zeros(capacity, np.int32)]
    band = [np.zeros(capacity, np.int32), np.zeros(capacity, np.int32)]
    counts = np.zeros(2, np.int32)
    found, bround, bext = C.c_int32(0), C.c_int32(0), C.c_int32(0)
    L = lib()
    L.or_plan_rounds.restype = C.c_int32
    st = L.or_plan_rounds(C.byref(robot.s), C.byref(env.s), C.byref(con.s), C.byref(prm),
                          _ptr(start), _ptr(goal), C.c_uint64(seed), C.c_int32(n_groups),
                          C.c_int32(rounds), C.c_int32(capacity), C.c_int32(max_connect),
                          _ptr(q[0]), _ptr(par[0], _ip), _ptr(band[0], _ip),
                          _ptr(q[1]), _ptr(par[1], _ip), _ptr(band[1], _ip),
                          _ptr(counts, _ip), C.byref(found), C.byref(bround), C.byref(bext))
    trees = [(q[t][: counts[t]].copy(), par[t][: counts[t]].copy(), band[t][: counts[t]].copy())
             for t in range(2)]
    return dict(trees=trees, found_round=found.value, band_round=bround.value,
                band_extensions=bext.value, status=st)


def path_report(robot: Robot, env: Env, con: Constraint, path):
    """(worst task error, worst spacing, min signed distance, inside limits)."""
    path = _f64(path)
    out = np.zeros(4)
    lib().or_path_report(C.byref(robot.s), C.byref(env.s), C.byref(con.s), _ptr(path),
                         C.c_int32(len(path)), _ptr(out))
    return dict(task_error=out[0], spacing=out[1], min_sd=out[2], inside=bool(out[3]))


def mlp_forward(dims, params, x):
    dims = np.ascontiguousarray(dims, np.int32)
    params, x = _f64(params), _f64(x)
    M = len(x)
    y = np.zeros((M, dims[-1]))
    lib().or_mlp_forward(C.c_int32(len(dims) - 1), _ptr(dims, _ip), _ptr(params), C.c_int32(M),
                         _ptr(x), _ptr(y))
    return y


def mlp_gradients(dims, params, x, t):
    dims = np.ascontiguousarray(dims, np.int32)
    params, x, t = _f64(params), _f64(x), _f64(t)
    grad = np.zeros_like(params)
    L = lib()
    L.or_mlp_gradients.restype = C.c_double
    loss = L.or_mlp_gradients(C.c_int32(len(dims) - 1), _ptr(dims, _ip), _ptr(params),
                              C.c_int32(len(x)), _ptr(x), _ptr(t), _ptr(grad))
    return loss, grad


def mlp_num_params(dims):
    return int(sum(dims[i + 1] * dims[i] + dims[i + 1] for i in range(len(dims) - 1)))

"""ctypes binding of libcprrtc.so (the C ABI declared in include/cprrtc.h).

Argument marshalling only: robot/scene/constraint dictionaries (layout in
`paper_2505_06791_amd.inputs`) become the C descriptors, torch tensors pass
their device pointers and the current HIP stream.  Every step of the hot path
runs in the library's kernels; if the library is missing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcprrtc.so")

CP_OK, CP_NO_SOLUTION = 0, 1
CP_E_ARG, CP_E_START, CP_E_GOAL, CP_E_CAPACITY = -1, -2, -3, -4
CP_E_RTC, CP_E_HIP, CP_E_UNSUPPORTED = -5, -6, -7
MOTION_VALID, MOTION_PROJ_FAIL, MOTION_COLLISION = 0, 1, 2
NO_EARLY_EXIT = 1
NO_CULL = 2
WARM_NO_FALLBACK = 4
CP_TUNE_W = 1
CP_TUNE_PLANNER = 2
POOLED, PER_MOTION, GENERIC = 8, 16, 32
SPECIALIZE_PROJECT, SPECIALIZE_PLAN = 1, 2
SELF_COLLISION = 64
BATCH_PER_CLASS = 1
PROJECT_PARALLEL, PROJECT_INDEPENDENT, PROJECT_SEQUENTIAL = 0, 1, 2
WORK_SLOTS = 8

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class CprrtcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"cprrtc error {code}: {msg}")
        self.code = code


class RobotDesc(C.Structure):
    _fields_ = [("dof", C.c_int32), ("n_chains", C.c_int32), ("joint_type", _ip),
                ("joint_chain", _ip), ("alpha", _dp), ("a", _dp), ("d", _dp), ("theta", _dp),
                ("q_lo", _dp), ("q_hi", _dp), ("base", _dp), ("tool", _dp),
                ("n_spheres", C.c_int32), ("sphere_link", _ip), ("sphere", _dp)]


class EnvDesc(C.Structure):
    _fields_ = [("n_aabb", C.c_int32), ("aabb", _dp), ("n_obb", C.c_int32), ("obb", _dp),
                ("n_sphere", C.c_int32), ("sphere", _dp), ("n_capsule", C.c_int32),
                ("capsule", _dp), ("n_cylinder", C.c_int32), ("cylinder", _dp)]


class Constraint(C.Structure):
    _fields_ = [("kind", C.c_int32), ("mask", C.c_int32 * 6), ("frame", C.c_double * 16),
                ("target", C.c_double * 6), ("rel_target", C.c_double * 16)]


class ProjParams(C.Structure):
    _fields_ = [("W", C.c_int32), ("max_iters", C.c_int32), ("tau", C.c_double),
                ("tau_sm", C.c_double), ("tau_task", C.c_double), ("alpha", C.c_double),
                ("lam", C.c_double), ("sphere_batch", C.c_int32), ("variant", C.c_int32)]


class PlanOpts(C.Structure):
    _fields_ = [("proj", ProjParams), ("n_groups", C.c_int32), ("max_rounds", C.c_int32),
                ("capacity", C.c_int32), ("max_connect", C.c_int32), ("poll_every", C.c_int32),
                ("flags", C.c_int32)]


class Path(C.Structure):
    _fields_ = [("capacity", C.c_int32), ("len", C.c_int32), ("dof", C.c_int32), ("q", _dp)]


class PlanStats(C.Structure):
    _fields_ = [("rounds", C.c_int32), ("nodes", C.c_int32 * 2), ("overflow", C.c_int32),
                ("launches_per_round", C.c_int32)]


class ShortcutStats(C.Structure):
    _fields_ = [("rounds", C.c_int32), ("candidates", C.c_int32), ("replaced", C.c_int32),
                ("length_before", C.c_double), ("length_after", C.c_double)]


class TuneReport(C.Structure):
    _fields_ = [("n", C.c_int32), ("W", C.c_int32 * 8), ("sphere_batch", C.c_int32 * 8),
                ("ms", C.c_double * 8), ("waypoints_per_s", C.c_double * 8)]


class BatchOpts(C.Structure):
    _fields_ = [("proj", ProjParams), ("groups_per_query", C.c_int32), ("max_rounds", C.c_int32),
                ("capacity", C.c_int32), ("max_connect", C.c_int32),
                ("rounds_per_graph", C.c_int32), ("flags", C.c_int32)]


class Query(C.Structure):
    _fields_ = [("robot", C.c_void_p), ("env", C.c_void_p), ("constraint", C.c_void_p),
                ("start", _dp), ("goal", _dp), ("seed", C.c_uint64)]


_lib = None


def lib():
    """Load libcprrtc.so (built by __graft_entry__.build()); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise CprrtcError(CP_E_HIP, f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        L.cp_last_error.restype = C.c_char_p
        vp = C.c_void_p
        L.cp_robot_create.argtypes = [C.POINTER(RobotDesc), C.POINTER(vp)]
        L.cp_env_create.argtypes = [C.POINTER(EnvDesc), C.POINTER(vp)]
        L.cp_robot_destroy.argtypes = [vp]
        L.cp_robot_specialize.argtypes = [vp, C.POINTER(Constraint), C.c_int32, C.POINTER(C.c_double)]
        L.cp_robot_self_pairs.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.cp_env_destroy.argtypes = [vp]
        L.cp_proj_params_default.argtypes = [C.POINTER(ProjParams)]
        L.fk_cc_batch.argtypes = [vp, vp, C.c_int32, vp, vp, vp, vp, C.c_int32, vp]
        L.project_validate_motions.argtypes = [vp, vp, C.POINTER(Constraint), C.POINTER(ProjParams),
                                               C.c_int32, vp, vp, vp, vp, vp, vp, C.c_int32, vp]
        L.project_motions.argtypes = [vp, C.POINTER(Constraint), C.POINTER(ProjParams), C.c_int32,
                                      vp, vp, vp, vp, vp, vp, vp]
        L.validate_motions.argtypes = [vp, vp, C.POINTER(ProjParams), C.c_int32, vp, vp, vp,
                                       C.c_int32, vp]
        L.cp_plan_opts_default.argtypes = [C.POINTER(PlanOpts)]
        L.cp_planner_create.argtypes = [vp, C.POINTER(PlanOpts), C.POINTER(vp)]
        L.cp_planner_destroy.argtypes = [vp]
        L.cp_planner_tree.argtypes = [vp, C.c_int32, C.c_int32, _dp, C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int32)]
        L.cp_plan.argtypes = [vp, vp, C.POINTER(Constraint), _dp, _dp, C.c_uint64,
                              C.POINTER(Path), C.POINTER(PlanStats), vp]
        L.plan.argtypes = [vp, vp, C.POINTER(Constraint), _dp, _dp, C.c_uint64,
                           C.POINTER(PlanOpts), C.POINTER(Path)]
        L.cp_autotune.argtypes = [vp, vp, C.POINTER(Constraint), C.POINTER(ProjParams), C.c_int32,
                                  vp, vp, C.c_int32, C.c_int32, C.POINTER(TuneReport), vp]
        L.cp_planner_set_warm.argtypes = [vp, vp]
        L.cp_batch_set_warm.argtypes = [vp, vp]
        L.cp_batch_opts_default.argtypes = [C.POINTER(BatchOpts)]
        L.cp_batch_create.argtypes = [C.POINTER(BatchOpts), C.c_int32, C.c_int32, C.POINTER(vp)]
        L.cp_batch_destroy.argtypes = [vp]
        L.cp_plan_batch.argtypes = [vp, C.c_int32, C.POINTER(Query), C.POINTER(Path),
                                    C.POINTER(C.c_int32), C.POINTER(PlanStats), vp]
        L.cp_mlp_create.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_uint64,
                                    C.POINTER(vp)]
        L.cp_mlp_destroy.argtypes = [vp]
        L.cp_mlp_num_params.argtypes = [vp]
        L.cp_mlp_num_params.restype = C.c_int64
        L.cp_mlp_get_params.argtypes = [vp, vp, vp]
        L.cp_mlp_set_params.argtypes = [vp, vp, vp]
        L.cp_mlp_forward.argtypes = [vp, C.c_int64, vp, vp, vp]
        L.cp_mlp_gradients.argtypes = [vp, C.c_int64, vp, vp, vp, vp, vp]
        L.cp_mlp_train_step.argtypes = [vp, C.c_int64, vp, vp, C.c_float, vp, vp]
        L.cp_mlp_get_state.argtypes = [vp, vp, vp, C.POINTER(C.c_int64), vp]
        L.cp_mlp_set_state.argtypes = [vp, vp, vp, C.c_int64, vp]
        L.project_motions_warm.argtypes = [vp, C.POINTER(Constraint), C.POINTER(ProjParams), vp,
                                           C.c_int32, vp, vp, vp, vp, vp, vp, C.c_int32, vp]
        L.project_motions_warm_noalloc.argtypes = L.project_motions_warm.argtypes
        L.cp_warm_pairs.argtypes = [vp, C.POINTER(Constraint), C.c_int32, C.c_int32, vp, vp, vp,
                                    vp, vp, vp]
        L.project_configs.argtypes = [vp, C.POINTER(Constraint), C.c_int32, vp, vp, vp,
                                      C.c_double, C.c_int32, C.c_double, C.c_double, vp]
        _lib = L
    return _lib


def _check(rc: int):
    if rc < 0:
        raise CprrtcError(rc, lib().cp_last_error().decode())
    return rc


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def _i32(x):
    return np.ascontiguousarray(x, dtype=np.int32)


class Robot:
    """Device copy of a robot dictionary (cp_robot handle)."""

    def __init__(self, rd: dict):
        keep = [_i32(rd["joint_type"]), _i32(rd["joint_chain"]), _f64(rd["alpha"]), _f64(rd["a"]),
                _f64(rd["d"]), _f64(rd["theta"]), _f64(rd["lo"]), _f64(rd["hi"]),
                _f64(rd["base"]).reshape(-1), _f64(rd["tool"]).reshape(-1),
                _i32(rd["sphere_link"]), _f64(rd["sphere"]).reshape(-1)]
        jt, jc, al, a, d, th, lo, hi, base, tool, sl, sp = keep
        desc = RobotDesc(int(rd["dof"]), int(rd["n_chains"]), jt.ctypes.data_as(_ip),
                         jc.ctypes.data_as(_ip), al.ctypes.data_as(_dp), a.ctypes.data_as(_dp),
                         d.ctypes.data_as(_dp), th.ctypes.data_as(_dp), lo.ctypes.data_as(_dp),
                         hi.ctypes.data_as(_dp), base.ctypes.data_as(_dp), tool.ctypes.data_as(_dp),
                         len(sl), sl.ctypes.data_as(_ip), sp.ctypes.data_as(_dp))
        h = C.c_void_p()
        _check(lib().cp_robot_create(C.byref(desc), C.byref(h)))
        self.handle = h
        self.dof = int(rd["dof"])
        self.n_spheres = len(sl)

    def self_pairs(self):
        """Checked self-collision sphere pairs [P][2] (description order)."""
        n = C.c_int32(0)
        _check(lib().cp_robot_self_pairs(self.handle, 0, None, C.byref(n)))
        out = np.zeros((max(n.value, 1), 2), np.int32)
        _check(lib().cp_robot_self_pairs(self.handle, n.value,
                                         out.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(n)))
        return out[: n.value].copy()

    def specialize(self, con, project: bool = True, plan: bool = False) -> float:
        """Compiles (hipRTC) the pooled projection kernel and / or the
        planner's round kernels for this robot and the constraint's kind and
        locked axes; returns this call's compile time in ms (0 when nothing
        was left to compile)."""
        ms = C.c_double(0.0)
        what = (SPECIALIZE_PROJECT if project else 0) | (SPECIALIZE_PLAN if plan else 0)
        _check(lib().cp_robot_specialize(self.handle, C.byref(con), what, C.byref(ms)))
        return ms.value

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.cp_robot_destroy(self.handle)
            self.handle = None


class Env:
    """Device copy of a scene dictionary (cp_env handle)."""

    def __init__(self, ed: dict):
        widths = dict(aabb=6, obb=15, sphere=4, capsule=7, cylinder=8)
        arrs = {k: _f64(np.asarray(ed[k]).reshape(-1, w)) for k, w in widths.items()}
        args = []
        for k in ("aabb", "obb", "sphere", "capsule", "cylinder"):
            args += [len(arrs[k]), arrs[k].ctypes.data_as(_dp)]
        desc = EnvDesc(*args)
        h = C.c_void_p()
        _check(lib().cp_env_create(C.byref(desc), C.byref(h)))
        self.handle = h
        self.counts = {k: len(v) for k, v in arrs.items()}
        self.n_prims = sum(self.counts.values())

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.cp_env_destroy(self.handle)
            self.handle = None


def constraint(cd: dict) -> Constraint:
    c = Constraint()
    c.kind = int(cd["kind"])
    fr = np.asarray(cd["frame"], np.float64).reshape(-1)
    rt = np.asarray(cd["rel_target"], np.float64).reshape(-1)
    for i in range(6):
        c.mask[i] = int(cd["mask"][i])
        c.target[i] = float(cd["target"][i])
    for i in range(16):
        c.frame[i] = fr[i]
        c.rel_target[i] = rt[i]
    return c


def proj_params(W=64, max_iters=32, tau=0.05, tau_sm=0.025, tau_task=1e-3, alpha=1.0, lam=1e-2,
                sphere_batch=8, variant=0) -> ProjParams:
    """variant: PROJECT_PARALLEL (Algorithm 1), PROJECT_INDEPENDENT (no
    smoothing term) or PROJECT_SEQUENTIAL (waypoint after waypoint)."""
    return ProjParams(W, max_iters, tau, tau_sm, tau_task, alpha, lam, sphere_batch, variant)


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev(t, dtype):
    import torch
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise CprrtcError(CP_E_ARG, f"expected a contiguous {dtype} CUDA tensor")
    return C.c_void_p(t.data_ptr())


# ------------------------------------------------------------------ hot path

def fk_cc_batch(robot: Robot, env: Env, q, collide, min_sd=None, flags: int = 0, stream=None,
                sphere_xyz=None):
    """q: [N, dof] float32 (device); collide: [N] uint8 (device); min_sd: [N] float32 or None;
    sphere_xyz: [N, n_spheres, 3] float32 or None (sphere centres, description order)."""
    import torch
    n = q.shape[0]
    if sphere_xyz is not None and tuple(sphere_xyz.shape) != (n, robot.n_spheres, 3):
        raise CprrtcError(CP_E_ARG, f"sphere_xyz must be [{n}, {robot.n_spheres}, 3]")
    _check(lib().fk_cc_batch(robot.handle, env.handle, n, _dev(q, torch.float32),
                             _dev(collide, torch.uint8),
                             _dev(min_sd, torch.float32) if min_sd is not None else None,
                             _dev(sphere_xyz, torch.float32) if sphere_xyz is not None else None,
                             flags, _stream(stream)))


def project_validate_motions(robot: Robot, env: Env, con: Constraint, prm: ProjParams,
                             q_from, q_to, xi, status, iters=None, work=None, flags: int = 0,
                             stream=None):
    """q_from/q_to: [M, dof] float32; xi: [M, W, dof] float32; status/iters: [M] int32;
    work: [8] int64 counters the call adds to (see include/cprrtc.h)."""
    import torch
    m = q_from.shape[0]
    _check(lib().project_validate_motions(
        robot.handle, env.handle, C.byref(con), C.byref(prm), m, _dev(q_from, torch.float32),
        _dev(q_to, torch.float32), _dev(xi, torch.float32), _dev(status, torch.int32),
        _dev(iters, torch.int32) if iters is not None else None,
        _dev(work, torch.int64) if work is not None else None, flags, _stream(stream)))


def project_motions(robot: Robot, con: Constraint, prm: ProjParams, q_from, q_to, xi, status,
                    iters=None, work=None, stream=None):
    """Interpolation + ParallelProject only; status 0 = projected, 1 = failed."""
    import torch
    m = q_from.shape[0]
    _check(lib().project_motions(
        robot.handle, C.byref(con), C.byref(prm), m, _dev(q_from, torch.float32),
        _dev(q_to, torch.float32), _dev(xi, torch.float32), _dev(status, torch.int32),
        _dev(iters, torch.int32) if iters is not None else None,
        _dev(work, torch.int64) if work is not None else None, _stream(stream)))


def shortcut(robot: Robot, env: Env, con: Constraint, prm: ProjParams, path, rounds: int,
             flags: int = 0, max_len: int = None, stream=None):
    """Path shortcutting (cp_shortcut): path [len, dof] float64 host.
    Returns (shortened path [len', dof] float64, stats dict)."""
    path = _f64(path)
    n, dof = path.shape
    max_len = max_len or max(n * 64, 1024)
    buf = np.zeros((max_len, dof))
    out = Path(max_len, 0, 0, buf.ctypes.data_as(_dp))
    stats = ShortcutStats()
    _check(lib().cp_shortcut(robot.handle, env.handle, C.byref(con), C.byref(prm),
                             path.ctypes.data_as(_dp), n, rounds, flags, C.byref(out),
                             C.byref(stats), _stream(stream)))
    return buf[: out.len].copy(), dict(rounds=stats.rounds, candidates=stats.candidates,
                                       replaced=stats.replaced,
                                       length_before=stats.length_before,
                                       length_after=stats.length_after)


def validate_motions(robot: Robot, env: Env, prm: ProjParams, xi, status, work=None,
                     flags: int = 0, stream=None):
    """FK + CC of the motions whose status is 0; status becomes 0 (valid) or 2 (collision)."""
    import torch
    m = xi.shape[0]
    _check(lib().validate_motions(
        robot.handle, env.handle, C.byref(prm), m, _dev(xi, torch.float32),
        _dev(status, torch.int32), _dev(work, torch.int64) if work is not None else None, flags,
        _stream(stream)))


def project_configs(robot: Robot, con: Constraint, q_in, q_out, status, tol=1e-5, max_iters=100,
                    alpha=1.0, lam=1e-2, stream=None):
    """Single-configuration projection; status[i] = 1 when ||e||_inf < tol was reached."""
    import torch
    n = q_in.shape[0]
    _check(lib().project_configs(robot.handle, C.byref(con), n, _dev(q_in, torch.float32),
                                 _dev(q_out, torch.float32), _dev(status, torch.int32), tol,
                                 max_iters, alpha, lam, _stream(stream)))


def autotune(robot: Robot, env: Env, con: Constraint, params: ProjParams, q_from, q_to,
             tune_W: bool = False, reps: int = 3, stream=None, planner: bool = False):
    """Times project_validate_motions for each candidate launch shape on the
    sample motions; returns (chosen ProjParams, list of candidate dicts).
    planner=True: only the sphere batches the planners' round kernels have."""
    import torch
    p = ProjParams.from_buffer_copy(params)
    rep = TuneReport()
    flags = (CP_TUNE_W if tune_W else 0) | (CP_TUNE_PLANNER if planner else 0)
    _check(lib().cp_autotune(robot.handle, env.handle, C.byref(con), C.byref(p), q_from.shape[0],
                             _dev(q_from, torch.float32), _dev(q_to, torch.float32),
                             flags, reps, C.byref(rep), _stream(stream)))
    cands = [dict(W=rep.W[i], sphere_batch=rep.sphere_batch[i], ms=rep.ms[i],
                  waypoints_per_s=rep.waypoints_per_s[i]) for i in range(rep.n)]
    return p, cands


# ------------------------------------------------------------------ planning

def plan_opts(n_groups=256, max_rounds=2000, capacity=16384, max_connect=64, poll_every=1,
              flags=0, **proj) -> PlanOpts:
    o = PlanOpts()
    lib().cp_plan_opts_default(C.byref(o))
    o.proj = proj_params(**proj)
    o.n_groups, o.max_rounds, o.capacity = n_groups, max_rounds, capacity
    o.max_connect, o.poll_every, o.flags = max_connect, poll_every, flags
    return o


class Planner:
    """cp_planner handle: device trees for one robot, reused across plans."""

    def __init__(self, robot: Robot, opts: PlanOpts | None = None):
        self.robot = robot
        self.opts = opts if opts is not None else plan_opts()
        h = C.c_void_p()
        _check(lib().cp_planner_create(robot.handle, C.byref(self.opts), C.byref(h)))
        self.handle = h

    def plan(self, env: Env, con: Constraint, start, goal, seed: int, max_len: int = 200000,
             stream=None):
        """Returns (status, path [len, dof] float64 or None, stats dict).
        status: CP_OK, CP_NO_SOLUTION, or raises CprrtcError for errors."""
        start = _f64(start)
        goal = _f64(goal)
        buf = np.zeros((max_len, self.robot.dof))
        path = Path(max_len, 0, 0, buf.ctypes.data_as(_dp))
        stats = PlanStats()
        strm = _stream(stream) if stream is not None else None
        rc = lib().cp_plan(self.handle, env.handle, C.byref(con), start.ctypes.data_as(_dp),
                           goal.ctypes.data_as(_dp), C.c_uint64(seed), C.byref(path),
                           C.byref(stats), strm)
        _check(rc)
        st = dict(rounds=stats.rounds, nodes=(stats.nodes[0], stats.nodes[1]),
                  overflow=stats.overflow, launches_per_round=stats.launches_per_round)
        if rc == CP_OK:
            return rc, buf[: path.len].copy(), st
        return rc, None, st

    def set_warm(self, mlp: "MLP | None"):
        """Warm-start every extension's first motion with the network (None: off)."""
        _check(lib().cp_planner_set_warm(self.handle, mlp.handle if mlp is not None else None))
        self._warm = mlp

    def tree(self, t: int):
        """Tree t (0 start, 1 goal) of the last plan: (q [count, dof] float64,
        parent [count] int32)."""
        cnt = C.c_int32(0)
        rc = lib().cp_planner_tree(self.handle, t, 0, None, None, C.byref(cnt))
        if rc not in (CP_OK, CP_E_CAPACITY):
            _check(rc)
        q = np.zeros((max(cnt.value, 1), self.robot.dof))
        par = np.zeros(max(cnt.value, 1), np.int32)
        _check(lib().cp_planner_tree(self.handle, t, cnt.value, q.ctypes.data_as(_dp),
                                     par.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(cnt)))
        return q[: cnt.value], par[: cnt.value]

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.cp_planner_destroy(self.handle)
            self.handle = None


def batch_opts(groups_per_query=16, max_rounds=500, capacity=2048, max_connect=64,
               rounds_per_graph=4, flags=0, **proj) -> BatchOpts:
    o = BatchOpts()
    lib().cp_batch_opts_default(C.byref(o))
    o.proj = proj_params(**proj)
    o.groups_per_query, o.max_rounds, o.capacity = groups_per_query, max_rounds, capacity
    o.max_connect, o.rounds_per_graph, o.flags = max_connect, rounds_per_graph, flags
    return o


class BatchPlanner:
    """cp_batch handle: tree pools for up to max_queries queries of up to
    max_dof joints, planned together (one launch per (DOF, constraint kind)
    class per round, rounds replayed from a HIP graph)."""

    def __init__(self, max_queries: int, max_dof: int, opts: BatchOpts | None = None):
        self.opts = opts if opts is not None else batch_opts()
        self.max_queries, self.max_dof = max_queries, max_dof
        h = C.c_void_p()
        _check(lib().cp_batch_create(C.byref(self.opts), max_queries, max_dof, C.byref(h)))
        self.handle = h

    def set_warm(self, mlp: "MLP | None"):
        """Warm-start the extensions with the network (None: off); the
        queries of a warm batch share one robot and one constraint."""
        _check(lib().cp_batch_set_warm(self.handle, mlp.handle if mlp is not None else None))
        self._warm = mlp

    def plan(self, queries, max_len: int = 65536, stream=None):
        """queries: list of (Robot, Env, Constraint, start, goal, seed).
        Returns (status [n] int32, paths: list of [len, dof] float64 or None,
        stats: list of dicts)."""
        n = len(queries)
        keep = []
        qs = (Query * max(n, 1))()
        paths = (Path * max(n, 1))()
        bufs = []
        for i, (robot, env, con, start, goal, seed) in enumerate(queries):
            a, b = _f64(start), _f64(goal)
            keep += [a, b, con]
            qs[i] = Query(robot.handle.value, env.handle.value, C.addressof(con),
                          a.ctypes.data_as(_dp), b.ctypes.data_as(_dp), seed)
            buf = np.zeros((max_len, robot.dof))
            bufs.append(buf)
            paths[i] = Path(max_len, 0, 0, buf.ctypes.data_as(_dp))
        status = (C.c_int32 * max(n, 1))()
        stats = (PlanStats * max(n, 1))()
        strm = _stream(stream) if stream is not None else None
        _check(lib().cp_plan_batch(self.handle, n, qs, paths, status, stats, strm))
        st = np.array([status[i] for i in range(n)], np.int32)
        out = [bufs[i][: paths[i].len].copy() if st[i] == CP_OK else None for i in range(n)]
        info = [dict(rounds=stats[i].rounds, nodes=(stats[i].nodes[0], stats[i].nodes[1]),
                     overflow=stats[i].overflow, launches_per_round=stats[i].launches_per_round)
                for i in range(n)]
        return st, out, info

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.cp_batch_destroy(self.handle)
            self.handle = None


# ------------------------------------------------------------------ learned warm start

class MLP:
    """cp_mlp handle: n_in -> hidden (SiLU) x n_hidden -> n_out, BF16 weights on
    the matrix cores, FP32 masters and Adam state on the device."""

    def __init__(self, n_in: int, hidden: int, n_hidden: int, n_out: int, seed: int = 0):
        h = C.c_void_p()
        _check(lib().cp_mlp_create(n_in, hidden, n_hidden, n_out, C.c_uint64(seed), C.byref(h)))
        self.handle = h
        self.n_in, self.hidden, self.n_hidden, self.n_out = n_in, hidden, n_hidden, n_out
        self.n_params = int(lib().cp_mlp_num_params(h))

    @property
    def dims(self):
        return [self.n_in] + [self.hidden] * self.n_hidden + [self.n_out]

    def get_params(self):
        import torch
        p = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        _check(lib().cp_mlp_get_params(self.handle, _dev(p, torch.float32), _stream()))
        return p

    def set_params(self, p):
        import torch
        _check(lib().cp_mlp_set_params(self.handle, _dev(p, torch.float32), _stream()))

    def forward(self, x):
        import torch
        y = torch.empty((x.shape[0], self.n_out), dtype=torch.float32, device=x.device)
        _check(lib().cp_mlp_forward(self.handle, x.shape[0], _dev(x, torch.float32),
                                    _dev(y, torch.float32), _stream()))
        return y

    def gradients(self, x, t):
        import torch
        g = torch.empty(self.n_params, dtype=torch.float32, device=x.device)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        _check(lib().cp_mlp_gradients(self.handle, x.shape[0], _dev(x, torch.float32),
                                      _dev(t, torch.float32), _dev(g, torch.float32),
                                      _dev(loss, torch.float32), _stream()))
        return g, loss

    def train_step(self, x, t, lr: float, loss=None):
        import torch
        _check(lib().cp_mlp_train_step(self.handle, x.shape[0], _dev(x, torch.float32),
                                       _dev(t, torch.float32), C.c_float(lr),
                                       _dev(loss, torch.float32) if loss is not None else None,
                                       _stream()))

    def get_state(self):
        """Adam state: (m1, m2 device tensors, step count)."""
        import torch
        m1 = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        m2 = torch.empty_like(m1)
        step = C.c_int64()
        _check(lib().cp_mlp_get_state(self.handle, _dev(m1, torch.float32), _dev(m2, torch.float32),
                                      C.byref(step), _stream()))
        return m1, m2, int(step.value)

    def set_state(self, m1, m2, step: int):
        import torch
        _check(lib().cp_mlp_set_state(self.handle, _dev(m1, torch.float32), _dev(m2, torch.float32),
                                      int(step), _stream()))

    # Checkpoint: <path>.json (shape, step, layout) and <path>.bin (parameters,
    # then the two Adam moment vectors, float32 little-endian), read back with
    # json and numpy.fromfile only.
    CHECKPOINT_FORMAT = "cprrtc-mlp-1"

    def save(self, path: str):
        import json
        import torch
        p = self.get_params()
        m1, m2, step = self.get_state()
        torch.cuda.synchronize()
        blob = torch.cat([p, m1, m2]).cpu().numpy().astype("<f4")
        blob.tofile(path + ".bin")
        with open(path + ".json", "w") as f:
            json.dump(dict(format=self.CHECKPOINT_FORMAT, n_in=self.n_in, hidden=self.hidden,
                           n_hidden=self.n_hidden, n_out=self.n_out, n_params=self.n_params,
                           step=step, dtype="float32-le", arrays=["params", "adam_m1", "adam_m2"]),
                      f, indent=1)

    @classmethod
    def load(cls, path: str) -> "MLP":
        import json
        import torch
        with open(path + ".json") as f:
            h = json.load(f)
        if h.get("format") != cls.CHECKPOINT_FORMAT:
            raise ValueError(f"{path}.json: not a {cls.CHECKPOINT_FORMAT} checkpoint")
        net = cls(h["n_in"], h["hidden"], h["n_hidden"], h["n_out"])
        n = net.n_params
        if n != h["n_params"]:
            raise ValueError(f"{path}.json: {h['n_params']} parameters, the shape has {n}")
        blob = np.fromfile(path + ".bin", dtype="<f4")
        if blob.size != 3 * n:
            raise ValueError(f"{path}.bin: {blob.size} values, expected {3 * n}")
        t = torch.from_numpy(blob.astype(np.float32)).to("cuda")
        net.set_params(t[:n].contiguous())
        net.set_state(t[n:2 * n].contiguous(), t[2 * n:].contiguous(), int(h["step"]))
        torch.cuda.synchronize()
        return net

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.cp_mlp_destroy(self.handle)
            self.handle = None


def warm_pairs(robot: Robot, con: Constraint, W: int, q_from, q_to, xi, n_in: int, stream=None):
    """cp_warm_pairs: (features [M (W-1), n_in], targets [M (W-1), dof]) of
    every waypoint k >= 1 of the projected motions xi [M, W, dof]."""
    import torch
    M, dof = q_from.shape
    x = torch.empty((M * (W - 1), n_in), dtype=torch.float32, device=q_from.device)
    t = torch.empty((M * (W - 1), dof), dtype=torch.float32, device=q_from.device)
    _check(lib().cp_warm_pairs(robot.handle, C.byref(con), W, M, _dev(q_from, torch.float32),
                               _dev(q_to, torch.float32), _dev(xi, torch.float32),
                               _dev(x, torch.float32), _dev(t, torch.float32), _stream(stream)))
    return x, t


def project_motions_warm(robot: Robot, con: Constraint, prm: ProjParams, mlp: MLP, q_from, q_to,
                         xi, status, iters=None, work=None, flags: int = 0, stream=None,
                         noalloc: bool = False):
    """project_motions with the learned warm start and the plain fallback
    (flags=WARM_NO_FALLBACK: the warm pass alone); noalloc=True calls
    project_motions_warm_noalloc (the library's fixed buffer, no allocation)."""
    import torch
    m = q_from.shape[0]
    fn = lib().project_motions_warm_noalloc if noalloc else lib().project_motions_warm
    _check(fn(
        robot.handle, C.byref(con), C.byref(prm), mlp.handle, m, _dev(q_from, torch.float32),
        _dev(q_to, torch.float32), _dev(xi, torch.float32), _dev(status, torch.int32),
        _dev(iters, torch.int32) if iters is not None else None,
        _dev(work, torch.int64) if work is not None else None, flags, _stream(stream)))

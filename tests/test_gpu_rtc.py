"""Run-time specialisation (hipRTC) of the pooled projection kernel and of
the planner's round kernels: kernels compiled with a robot's constants and
a constraint's locked axes compute what the library kernels compute and
meet the oracle.  Folding the
constants lets the compiler fuse multiply-adds differently, so waypoints may
differ in the last bits: statuses and iterations must agree outside the
oracle's threshold band, waypoints of motions projected by both within
1e-5 rad."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from paper_2505_06791_amd import inputs as I
from tests.helpers import ORACLE_THREADS, manifold_starts, motion_set, oracle_views
from tests.test_gpu_parity import _compare_pv
from tests.test_gpu_plan import _check_path

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_06791_amd import cprrtc
    cprrtc.lib()
    return cprrtc


def _workload(name):
    if name == "line":
        w = dict(I.workload("plain", 2364))
        w["constraint"] = I.line_constraint(7)
        return w
    if name == "none":
        w = dict(I.workload("plain", 2401))
        w["constraint"] = I.no_constraint()
        return w
    if name == "dual-free":   # the relative-pose workload in an empty scene
        return dict(I.workload("dual", 2400), env=I.empty_env())
    return I.workload(name, 2400)


def _run(G, robot, env, con, w, q_from, q_to, kw, flags):
    M, dof, W = len(q_from), w["robot"]["dof"], kw["W"]
    qf, qt = torch.from_numpy(q_from).to("cuda:0"), torch.from_numpy(q_to).to("cuda:0")
    xi = torch.full((M, W, dof), float("nan"), device="cuda:0")
    st = torch.full((M,), -9, dtype=torch.int32, device="cuda:0")
    it = torch.full((M,), -9, dtype=torch.int32, device="cuda:0")
    G.project_validate_motions(robot, env, con, G.proj_params(**kw), qf, qt, xi, st, it, flags=flags)
    torch.cuda.synchronize()
    return xi.cpu().numpy(), st.cpu().numpy(), it.cpu().numpy()


def _oracle(w, q_from, q_to, kw):
    ro, eo, co = oracle_views(w)
    return O.project_validate_motions(ro, eo, co, O.params(**kw), q_from.astype(np.float64),
                                      q_to.astype(np.float64), n_threads=ORACLE_THREADS)


@pytest.mark.parametrize("name,W,M,least", [("plain", 64, 48, 10), ("cluttered", 64, 48, 10),
                                            ("mobile", 32, 48, 10), ("dual-free", 64, 2400, 100),
                                            ("line", 64, 48, 10), ("none", 64, 48, 10)])
def test_specialised_kernel_equals_library_kernel(G, name, W, M, least):
    w = _workload(name)
    q_from, q_to = motion_set(w, M, 29, W=W)
    robot, env, con = G.Robot(w["robot"]), G.Env(w["env"]), G.constraint(w["constraint"])
    ms = robot.specialize(con)
    assert ms > 0
    assert robot.specialize(con) == 0.0         # kept: the second call compiles nothing
    kw = dict(W=W, tau_task=w["tau_task"])
    xi_s, st_s, it_s = _run(G, robot, env, con, w, q_from, q_to, kw, G.POOLED)
    xi_g, st_g, it_g = _run(G, robot, env, con, w, q_from, q_to, kw, G.POOLED | G.GENERIC)
    print(name, "compile ms", round(ms, 1), "statuses", np.bincount(st_s, minlength=3), flush=True)
    ref = _oracle(w, q_from, q_to, kw)
    _agree(ref, (xi_s, st_s, it_s), (xi_g, st_g, it_g))
    _compare_pv(f"{name} specialised", ref, xi_s, st_s, it_s, w, W, w["tau_task"],
                min_compared=least)


def _agree(ref, a, b):
    band = (ref["proj_margin"] < 1e-5) | (np.abs(ref["min_sd"]) < 1e-5)
    assert np.array_equal(a[1][~band], b[1][~band])
    proj_band = ref["proj_margin"] < 1e-5
    assert np.array_equal(a[2][~proj_band], b[2][~proj_band])
    both = (a[1] != O.MOTION_PROJ_FAIL) & (b[1] != O.MOTION_PROJ_FAIL) & ~band
    if both.any():
        assert np.abs(a[0][both] - b[0][both]).max() < 1e-5


def test_specialised_kernel_serves_only_its_mask(G):
    """A robot specialised for upright projects plane + upright motions with
    the library kernel (same results as with CP_GENERIC), meeting the oracle."""
    w = dict(I.workload("plain", 2400), constraint=I.plane_upright(3))
    robot, env = G.Robot(w["robot"]), G.Env(w["env"])
    robot.specialize(G.constraint(I.upright()))
    con = G.constraint(w["constraint"])
    q_from, q_to = motion_set(w, 32, 41)
    kw = dict(W=64, tau_task=1e-3)
    a = _run(G, robot, env, con, w, q_from, q_to, kw, G.POOLED)
    b = _run(G, robot, env, con, w, q_from, q_to, kw, G.POOLED | G.GENERIC)
    for x, y in zip(a, b):                      # the same kernel ran both times
        assert np.array_equal(x, y)
    _compare_pv("plain other mask", _oracle(w, q_from, q_to, kw), *a, w, 64, 1e-3)


@pytest.mark.parametrize("name,seeds", [("plain", range(1000, 1004)), ("cluttered", (2001, 2002)),
                                        ("dual", (4000, 4001))])
def test_specialised_planner_paths_pass_oracle_revalidation(G, name, seeds):
    """cp_plan with the round kernels compiled for the robot and mask: every
    path passes the oracle's re-validation, and the projection kernel is
    compiled separately (a plan-only specialisation leaves pooled projection
    on the library kernel)."""
    solved = 0
    for seed in seeds:
        w = I.workload(name, seed)
        ends = manifold_starts(w, 2, seed + 5).astype(np.float64)
        robot, env, con = G.Robot(w["robot"]), G.Env(w["env"]), G.constraint(w["constraint"])
        ms = robot.specialize(con, project=False, plan=True)
        assert ms > 0 and robot.specialize(con, project=False, plan=True) == 0.0
        pl = G.Planner(robot, G.plan_opts(n_groups=128, max_rounds=400, tau_task=w["tau_task"]))
        rc, path, st = pl.plan(env, con, ends[0], ends[1], seed)
        print(name, seed, "compile ms", round(ms, 1), "rc", rc,
              "len", None if path is None else len(path), st, flush=True)
        if rc == G.CP_OK:
            solved += 1
            _check_path(w, path, ends[0], ends[1], w["tau_task"])
    assert solved >= 1
    # the projection kernel was not compiled by the plan-only call
    assert robot.specialize(con) > 0


@pytest.mark.parametrize("name,W,batch", [("cluttered", 64, 8), ("cluttered", 32, 4),
                                          ("dual", 64, 8), ("mobile", 64, 4)])
def test_specialised_validation_equals_library_validation(G, name, W, batch):
    """validate_motions with the kernels compiled for the robot: the same
    verdicts as the library's kernels (CP_GENERIC) and as the oracle's
    clearance of waypoints 1..W-1, outside the 1e-5 m band."""
    w = _workload(name)
    q_from, q_to = motion_set(w, 40, 53, W=W)
    robot, env, con = G.Robot(w["robot"]), G.Env(w["env"]), G.constraint(w["constraint"])
    kw = dict(W=W, tau_task=w["tau_task"], sphere_batch=batch)
    xi, st, _ = _run(G, robot, env, con, w, q_from, q_to, kw, G.GENERIC)
    assert robot.specialize(con) > 0
    prm = G.proj_params(**kw)
    ro, eo, co = oracle_views(w)
    sd = np.array([O.path_report(ro, eo, co, xi[m, 1:].astype(np.float64))["min_sd"]
                   for m in range(len(xi))])
    band = np.abs(sd) < 1e-5
    out = {}
    for flags in (0, G.GENERIC, G.NO_EARLY_EXIT, G.GENERIC | G.NO_EARLY_EXIT):
        s = torch.from_numpy(np.where(st == O.MOTION_PROJ_FAIL, 1, 0).astype(np.int32)).to("cuda:0")
        G.validate_motions(robot, env, prm, torch.from_numpy(xi).to("cuda:0"), s, flags=flags)
        torch.cuda.synchronize()
        out[flags] = s.cpu().numpy()
    print(name, W, batch, "band", int(band.sum()), "statuses", np.bincount(out[0], minlength=3),
          flush=True)
    checked = st != O.MOTION_PROJ_FAIL
    want = np.where(sd < 0, 2, 0)
    for flags, s in out.items():
        assert np.array_equal(s[~checked], np.ones((~checked).sum(), np.int32))
        assert np.array_equal(s[checked & ~band], want[checked & ~band]), flags


def test_full_size_sampled_specialised(G):
    """The benchmark's launch as bench.py times it: 65 536 cluttered motions
    with the projection and validation kernels compiled for the robot;
    sampled motions (and the last) recomputed by the oracle."""
    from tests.test_gpu_parity import _oracle_pv
    w = I.workload("cluttered", 2000)
    base_from, _ = motion_set(w, 256, 2500)
    M = 65536
    q_from = np.tile(base_from, (M // len(base_from), 1))
    q_to = I.random_displacements(w["robot"], q_from.astype(np.float64), 63 * 0.05,
                                  2501).astype(np.float32)
    robot, env, con = G.Robot(w["robot"]), G.Env(w["env"]), G.constraint(w["constraint"])
    assert robot.specialize(con) > 0
    kw = dict(W=64, tau_task=w["tau_task"])
    xi, st, it = _run(G, robot, env, con, w, q_from, q_to, kw, 0)
    idx = np.concatenate([np.sort(np.random.default_rng(0).choice(M, 48, replace=False)), [M - 1]])
    ref = _oracle_pv(w, q_from[idx], q_to[idx], 64, w["tau_task"])
    _compare_pv("cluttered-full specialised", ref, xi[idx], st[idx], it[idx], w, 64,
                w["tau_task"])
    # the library kernels on the same launch: every motion whose status or
    # iteration count differs between the two is recomputed by the oracle.
    # A differing projection outcome (one kernel projects, the other fails)
    # must come from a decision within 1e-5 of its threshold.  Where both
    # project, the two results are different valid projections (float32
    # rounding moves the iterates by about 1e-6 rad, which can move a
    # decision that lies near the band edge by one iteration): each is
    # re-validated by the oracle (start bitwise, limits, task error and
    # spacing within their thresholds up to the band), and each kernel's
    # collision verdict must be the oracle's FK and distances on that
    # kernel's own waypoints, outside the 1e-5 m band.
    xi_g, st_g, it_g = _run(G, robot, env, con, w, q_from, q_to, kw, G.GENERIC)
    assert set(np.unique(st)).issubset({0, 1, 2})
    diff = np.nonzero((st != st_g) | (it != it_g))[0]
    print("statuses specialised", np.bincount(st, minlength=3), "library",
          np.bincount(st_g, minlength=3), "differing motions", len(diff), flush=True)
    if len(diff):
        ref_d = _oracle_pv(w, q_from[diff], q_to[diff], 64, w["tau_task"])
        proj_band = ref_d["proj_margin"] < 1e-5
        ro, eo, co = oracle_views(w)
        max_spacing = 0.05 + 0.025
        judged = iters_only = 0
        for j, m in enumerate(diff):
            if (st[m] == 1) != (st_g[m] == 1):
                assert proj_band[j], (m, st[m], st_g[m], it[m], it_g[m])
                continue
            iters_only += int(st[m] == st_g[m])
            for s_k, xi_k in ((st[m], xi[m]), (st_g[m], xi_g[m])):
                if s_k == 1:
                    continue
                assert np.array_equal(xi_k[0], q_from[m]), m
                rep = O.path_report(ro, eo, co, xi_k.astype(np.float64))
                assert rep["inside"], m
                assert rep["task_error"] < w["tau_task"] + 1e-5, (m, rep)
                assert rep["spacing"] < max_spacing + 1e-5, (m, rep)
                sd = O.path_report(ro, eo, co, xi_k[1:].astype(np.float64))["min_sd"]
                if abs(sd) >= 1e-5:
                    assert s_k == (2 if sd <= 0 else 0), (m, s_k, sd)
                    judged += 1
        print("differing motions: same status, iterations only", iters_only,
              "; verdicts judged on each kernel's own waypoints", judged, flush=True)


@pytest.mark.parametrize("name,n", [("plain", 4099), ("cluttered", 2050), ("mobile", 1025),
                                    ("dual", 1030)])
def test_specialised_fk_cc_matches_oracle(G, name, n):
    """fk_cc_batch with the FK/CC kernel compiled for the robot: verdicts equal
    the FP64 oracle's outside the 1e-5 m band, with and without early exit,
    and equal the library kernel's (CP_GENERIC) outside the band."""
    w = I.workload(name, 1300 + n)
    q32 = I.random_configs(w["robot"], n, 9).astype(np.float32)
    ro, eo, _ = oracle_views(w)
    col_o, sd_o = O.fk_cc_batch(ro, eo, q32.astype(np.float64), n_threads=ORACLE_THREADS)
    robot, env = G.Robot(w["robot"]), G.Env(w["env"])
    assert robot.specialize(G.constraint(w["constraint"])) > 0
    q = torch.from_numpy(q32).to("cuda:0")
    out = {}
    for flags in (0, G.NO_EARLY_EXIT, G.GENERIC):
        col = torch.full((n,), 7, dtype=torch.uint8, device="cuda:0")
        G.fk_cc_batch(robot, env, q, col, flags=flags)
        torch.cuda.synchronize()
        out[flags] = col.cpu().numpy().astype(bool)
    band = np.abs(sd_o) <= 1e-5
    print(name, n, "band", int(band.sum()), "colliding", int(col_o.sum()), flush=True)
    for flags, col in out.items():
        assert np.array_equal(col[~band], col_o[~band].astype(bool)), flags
    assert np.array_equal(out[0], out[G.NO_EARLY_EXIT])


def test_compiled_kernels_come_back_from_the_disk_cache(G, tmp_path, monkeypatch):
    """A second robot handle with the same description and constraint mask
    reads the code object the first one compiled from the disk cache
    (CPRRTC_RTC_CACHE) instead of compiling, and its kernels give the same
    bits."""
    monkeypatch.setenv("CPRRTC_RTC_CACHE", str(tmp_path / "rtc"))
    w = _workload("plain")
    con, env = G.constraint(w["constraint"]), G.Env(w["env"])
    r1 = G.Robot(w["robot"])
    ms1 = r1.specialize(con)
    assert len(list((tmp_path / "rtc").glob("*.co"))) == 1
    r2 = G.Robot(w["robot"])
    ms2 = r2.specialize(con)
    assert len(list((tmp_path / "rtc").glob("*.co"))) == 1
    print("compile ms", round(ms1, 1), "from the cache", round(ms2, 1), flush=True)
    assert ms2 < 0.5 * ms1
    q_from, q_to = motion_set(w, 48, 31)
    kw = dict(W=64, tau_task=w["tau_task"])
    a = _run(G, r1, env, con, w, q_from, q_to, kw, G.POOLED)
    b = _run(G, r2, env, con, w, q_from, q_to, kw, G.POOLED)
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    assert np.array_equal(a[0], b[0], equal_nan=True)

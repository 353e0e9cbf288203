"""Path shortcutting (cp_shortcut) on the GPU: the chord in free space,
planned paths shortened and re-validated by the oracle, the oracle's own
shortcutting of the same path for comparison, and the error paths."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from paper_2505_06791_amd import inputs as I
from tests.helpers import BAND, manifold_starts, oracle_views

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_06791_amd import cprrtc
    cprrtc.lib()
    return cprrtc


def _zigzag(start, n=30):
    steps = np.zeros((n, len(start)))
    steps[:, 0] = 0.04
    steps[:, 1] = np.where(np.arange(n) % 2 == 0, 0.02, -0.02)
    return np.vstack([start, start + np.cumsum(steps, axis=0)])


def test_shortcut_free_space_is_the_chord(G):
    w = I.workload("plain", 2403)
    robot, env = G.Robot(w["robot"]), G.Env(I.empty_env())
    con = G.constraint(I.no_constraint())
    P = _zigzag(np.zeros(7)).astype(np.float32).astype(np.float64)
    out, st = G.shortcut(robot, env, con, G.proj_params(), P, rounds=3)
    chord = np.linalg.norm(P[-1] - P[0])
    assert np.array_equal(out[0], P[0]) and np.array_equal(out[-1], P[-1])
    assert len(out) == 64 and st["replaced"] == 1 and st["rounds"] == 1
    assert abs(st["length_after"] - chord) < 1e-5


def _check(w, path, start, goal, tau_task):
    ro, eo, co = oracle_views(w)
    rep = O.path_report(ro, eo, co, path)
    assert np.array_equal(path[0], start) and np.array_equal(path[-1], goal)
    assert rep["inside"] and rep["task_error"] < tau_task + BAND, rep
    assert rep["spacing"] < 0.075 + BAND and rep["min_sd"] > -BAND, rep
    return rep


@pytest.mark.parametrize("name,seeds", [("plain", (1000, 1001, 1003)), ("cluttered", (2001,))])
def test_shortcut_planned_paths(G, name, seeds):
    """Paths from the GPU planner, shortened in five rounds: same end points,
    never longer, valid by the oracle; the oracle's shortcutting of the same
    path reaches a comparable length (decisions near a threshold may go
    either way between FP32 and FP64, so the lengths are compared loosely)."""
    for seed in seeds:
        w = I.workload(name, seed)
        ends = manifold_starts(w, 2, seed + 5).astype(np.float64)
        robot, env, con = G.Robot(w["robot"]), G.Env(w["env"]), G.constraint(w["constraint"])
        pl = G.Planner(robot, G.plan_opts(n_groups=128, max_rounds=400, tau_task=w["tau_task"]))
        rc, path, _ = pl.plan(env, con, ends[0], ends[1], seed)
        if rc != G.CP_OK:
            continue
        prm = G.proj_params(tau_task=w["tau_task"])
        out, st = G.shortcut(robot, env, con, prm, path, rounds=5)
        _check(w, out, ends[0], ends[1], w["tau_task"])
        assert st["length_after"] <= st["length_before"] + 1e-9
        ro, eo, co = oracle_views(w)
        ref, st_o = O.shortcut(ro, eo, co, O.params(tau_task=w["tau_task"]), path, rounds=5)
        print(name, seed, "length", round(st["length_before"], 3), "->",
              round(st["length_after"], 3), "oracle", round(st_o["length_after"], 3),
              "pieces", st["replaced"], st_o["replaced"], flush=True)
        assert abs(st["length_after"] - st_o["length_after"]) <= 0.1 * st["length_before"]
        # with the self-check the spliced-in pieces are also free of
        # self-collision (the planner's own points are kept as they are)
        out_s, _ = G.shortcut(robot, env, con, prm, path, rounds=5, flags=G.SELF_COLLISION)
        _check(w, out_s, ends[0], ends[1], w["tau_task"])
        pairs = O.self_pairs(ro)
        old_rows = {x.tobytes() for x in path}
        new_pts = [x for x in out_s if x.tobytes() not in old_rows]
        print("  self-checked pieces add", len(new_pts), "points", flush=True)
        if len(pairs) and new_pts:
            assert min(O.self_min_sd(ro, x, pairs) for x in new_pts) > -BAND


def test_shortcut_errors_and_no_rounds(G):
    w = I.workload("plain", 2403)
    robot, env = G.Robot(w["robot"]), G.Env(I.empty_env())
    con = G.constraint(I.no_constraint())
    P = _zigzag(np.zeros(7))
    same, st = G.shortcut(robot, env, con, G.proj_params(), P, rounds=0)
    assert np.array_equal(same, P) and st["rounds"] == 0
    with pytest.raises(G.CprrtcError) as e:
        G.shortcut(robot, env, con, G.proj_params(), P, rounds=3, max_len=10)
    assert e.value.code == G.CP_E_CAPACITY
    with pytest.raises(G.CprrtcError) as e:
        G.shortcut(robot, env, con, G.proj_params(), P, rounds=1, flags=1 << 20)
    assert e.value.code == G.CP_E_ARG

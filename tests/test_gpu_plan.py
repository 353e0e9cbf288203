"""plan() on the GPU: every returned path passes oracle re-validation.

The GPU grows both trees with hundreds of concurrent extensions, so its
paths are not the oracle planner's; they are judged by the oracle (FP64) on
the path itself: joint limits, task error below tolerance, consecutive
spacing below tau + tau_sm, clearance outside the 1e-5 m band, and the exact
start and goal at the ends.  End-to-end planning is parity unpinned against
the paper (it prints no example); these checks and the invariants are what
pin it.
"""
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


def _check_path(w, path, start, goal, tau_task, tau=0.05, tau_sm=0.025):
    ro, eo, co = oracle_views(w)
    rep = O.path_report(ro, eo, co, path)
    assert np.array_equal(path[0], start) and np.array_equal(path[-1], goal)
    assert rep["inside"]
    assert rep["task_error"] < tau_task + BAND, rep
    assert rep["spacing"] < tau + tau_sm + BAND, rep
    assert rep["min_sd"] > -BAND, rep
    return rep


@pytest.mark.parametrize("name,seeds", [("plain", range(1000, 1006)), ("cluttered", range(2000, 2003)),
                                        ("mobile", range(3000, 3002))])
def test_plan_paths_pass_oracle_revalidation(G, name, seeds):
    solved = 0
    for seed in seeds:
        w = I.workload(name, seed)
        ends = manifold_starts(w, 2, seed + 5).astype(np.float64)
        robot, env, con = G.Robot(w["robot"]), G.Env(w["env"]), G.constraint(w["constraint"])
        pl = G.Planner(robot, G.plan_opts(n_groups=128, max_rounds=400, tau_task=w["tau_task"]))
        rc, path, st = pl.plan(env, con, ends[0], ends[1], seed)
        print(name, seed, "rc", rc, "len", None if path is None else len(path), st, flush=True)
        if rc == G.CP_OK:
            solved += 1
            _check_path(w, path, ends[0], ends[1], w["tau_task"])
    assert solved >= 1


def test_plan_is_repeatable_per_planner_and_reusable(G):
    w = I.workload("plain", 1001)
    ends = manifold_starts(w, 2, 1006).astype(np.float64)
    robot, env, con = G.Robot(w["robot"]), G.Env(w["env"]), G.constraint(w["constraint"])
    pl = G.Planner(robot, G.plan_opts(n_groups=64, max_rounds=400))
    for _ in range(3):     # the same handle plans again from a clean state
        rc, path, st = pl.plan(env, con, ends[0], ends[1], 7)
        assert rc == G.CP_OK
        _check_path(w, path, ends[0], ends[1], 1e-3)
    # the reverse query
    rc, path, st = pl.plan(env, con, ends[1], ends[0], 8)
    assert rc == G.CP_OK
    _check_path(w, path, ends[1], ends[0], 1e-3)


def test_plan_endpoint_errors(G):
    w = I.workload("plain", 1002)
    ends = manifold_starts(w, 2, 1007).astype(np.float64)
    robot, env, con = G.Robot(w["robot"]), G.Env(w["env"]), G.constraint(w["constraint"])
    pl = G.Planner(robot, G.plan_opts(n_groups=16, max_rounds=8))
    off = ends[0].copy()
    off[3] += 0.5                                     # off the manifold
    with pytest.raises(G.CprrtcError) as ex:
        pl.plan(env, con, off, ends[1], 1)
    assert ex.value.code == G.CP_E_START
    with pytest.raises(G.CprrtcError) as ex:
        pl.plan(env, con, ends[0], off, 1)
    assert ex.value.code == G.CP_E_GOAL
    outside = ends[0].copy()
    outside[0] = 3.0                                  # outside the limits
    with pytest.raises(G.CprrtcError) as ex:
        pl.plan(env, con, outside, ends[1], 1)
    assert ex.value.code == G.CP_E_START
    # an obstacle placed on the start's end effector puts the start in collision
    ro, eo, co = oracle_views(w)
    _, ee = O.fk(ro, ends[0])
    env2 = {k: v.copy() for k, v in w["env"].items()}
    env2["sphere"] = np.array([[*ee[0, :3, 3], 0.15]])
    with pytest.raises(G.CprrtcError) as ex:
        pl.plan(G.Env(env2), con, ends[0], ends[1], 1)
    assert ex.value.code == G.CP_E_START
    # start == goal: the two-point path
    rc, path, _ = pl.plan(env, con, ends[0], ends[0], 1)
    assert rc == G.CP_OK and len(path) == 2


def test_plan_budget_and_capacity(G):
    w = I.workload("cluttered", 2001)
    ends = manifold_starts(w, 2, 2006).astype(np.float64)
    robot, env, con = G.Robot(w["robot"]), G.Env(w["env"]), G.constraint(w["constraint"])
    # one round of two extensions rarely connects a long query: NO_SOLUTION, not an error
    pl = G.Planner(robot, G.plan_opts(n_groups=2, max_rounds=1, max_connect=0, poll_every=1))
    rc, path, st = pl.plan(env, con, ends[0], ends[1], 3)
    assert rc in (G.CP_OK, G.CP_NO_SOLUTION)
    assert st["rounds"] == 1
    # trees of capacity 2 fill at once
    pl = G.Planner(robot, G.plan_opts(n_groups=64, max_rounds=50, capacity=2, poll_every=1))
    try:
        rc, path, st = pl.plan(env, con, ends[0], ends[1], 3)
        assert rc in (G.CP_OK, G.CP_NO_SOLUTION)
    except G.CprrtcError as e:
        assert e.code == G.CP_E_CAPACITY


def _match_trees(q_gpu, p_gpu, q_or, p_or, band_or, slack, tol=1e-4):
    """Node-for-node match, independent of append order: every oracle node
    appended without a band decision pairs with a distinct GPU node whose
    configuration and parent configuration agree within tol; at most `slack`
    GPU nodes stay unpaired (outputs of extensions that held a band
    decision)."""
    used = np.zeros(len(q_gpu), bool)
    assert np.abs(q_gpu[0] - q_or[0]).max() < tol and p_gpu[0] == -1
    used[0] = True
    for i in range(1, len(q_or)):
        if band_or[i]:
            continue
        d = np.abs(q_gpu - q_or[i]).max(1)
        pd = np.abs(q_gpu[np.maximum(p_gpu, 0)] - q_or[p_or[i]]).max(1)
        cand = np.nonzero((d < tol) & (pd < tol) & ~used & (p_gpu >= 0))[0]
        assert len(cand) >= 1, (i, d.min())
        used[cand[0]] = True
    assert (~used).sum() <= slack, ((~used).sum(), slack)
    return int(used.sum()) - 1


@pytest.mark.parametrize("specialised", [False, True])
def test_plan_lockstep_replay_matches_oracle_rounds(G, specialised):
    """Rounds of the GPU planner against the oracle's round-synchronous
    replay (same Halton indices, same tree per extension, searches over the
    nodes present when the round began).  Compared through the first round
    that holds a decision within the band of its threshold: every node the
    oracle appended without such a decision has its GPU twin.  specialised:
    the round kernels compiled at run time for the robot and mask."""
    compared, matched = 0, 0
    for name, seed in (("cluttered", 2001), ("plain", 1000), ("plain", 1001), ("plain", 1003),
                       ("plain", 1004), ("plain", 1005), ("mobile", 3000)):
        w = I.workload(name, seed)
        ro, eo, co = oracle_views(w)
        ends = manifold_starts(w, 2, seed + 5).astype(np.float64)
        prm_o = O.params(W=64, tau_task=w["tau_task"])
        groups, R = 32, 3
        ref = O.plan_rounds(ro, eo, co, prm_o, ends[0], ends[1], seed, n_groups=groups, rounds=R)
        lim = min(R, ref["band_round"]) if ref["band_round"] else R
        if ref["found_round"]:
            lim = min(lim, ref["found_round"] - 1)
        print(name, seed, "found", ref["found_round"], "band round", ref["band_round"],
              "rounds compared", lim, flush=True)
        if lim < 1:
            continue
        if lim < R:
            ref = O.plan_rounds(ro, eo, co, prm_o, ends[0], ends[1], seed, n_groups=groups,
                                rounds=lim)
        robot, env, con = G.Robot(w["robot"]), G.Env(w["env"]), G.constraint(w["constraint"])
        if specialised:
            assert robot.specialize(con, project=False, plan=True) > 0
        pl = G.Planner(robot, G.plan_opts(n_groups=groups, max_rounds=lim, capacity=4096,
                                          tau_task=w["tau_task"]))
        rc, path, st = pl.plan(env, con, ends[0], ends[1], seed)
        if rc == G.CP_OK:            # a band extension connected on the GPU
            assert ref["band_extensions"] > 0
            continue
        assert rc == G.CP_NO_SOLUTION and st["rounds"] == lim
        slack = ref["band_extensions"] * 65
        for t in range(2):
            qg, pg = pl.tree(t)
            qo, po, bo = ref["trees"][t]
            m = _match_trees(qg, pg, qo, po, bo, slack)
            print("  tree", t, "nodes gpu", len(qg), "oracle", len(qo), "band", int(bo.sum()),
                  "matched", m, flush=True)
            matched += m
        compared += 1
    assert compared >= 3 and matched >= 10

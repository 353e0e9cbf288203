"""The learned warm start inside the planners (cp_planner_set_warm,
cp_batch_set_warm): every path they return passes the oracle's
re-validation at the tolerance 1e-4 (limits, task error, spacing, clearance,
exact ends), the warm-started rounds keep the plain projector as fallback,
and the batch refuses queries a single network cannot serve.  The network is
trained here on projector pairs of the same robot (a few seconds)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2505_06791_amd import inputs as I
from tests.helpers import manifold_starts
from tests.test_gpu_plan import _check_path

pytestmark = pytest.mark.gpu
TAU_TASK = 1e-4


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_06791_amd import cprrtc
    cprrtc.lib()
    return cprrtc


@pytest.fixture(scope="module")
def trained(G):
    from paper_2505_06791_amd import warmstart
    w = I.workload("plain", 1000)
    rd, cd = w["robot"], w["constraint"]
    robot, con = G.Robot(rd), G.constraint(cd)
    X, T = warmstart.make_pairs(rd, cd, 16384, seed=4000, tau_task=TAU_TASK, robot=robot, con=con)
    net = G.MLP(warmstart.n_inputs(rd, cd), 256, 3, rd["dof"], seed=4000)
    hist = warmstart.train(net, X, T, epochs=4, batch=4096)
    assert hist[-1] < hist[0]
    return w, robot, con, net


def test_warm_planner_paths_pass_oracle_revalidation(G, trained):
    w, robot, con, net = trained
    env = G.Env(w["env"])
    pl = G.Planner(robot, G.plan_opts(n_groups=128, max_rounds=400, tau_task=TAU_TASK))
    pl.set_warm(net)
    solved = 0
    for seed in range(6):
        ends = manifold_starts(w, 2, 1100 + seed).astype(np.float64)
        rc, path, st = pl.plan(env, con, ends[0], ends[1], seed)
        print("warm plan", seed, "rc", rc, "len", None if path is None else len(path), st, flush=True)
        if rc == G.CP_OK:
            solved += 1
            _check_path(w, path, ends[0], ends[1], TAU_TASK)
    assert solved >= 3
    # switched off again: the plain rounds
    pl.set_warm(None)
    ends = manifold_starts(w, 2, 1100).astype(np.float64)
    rc, path, _ = pl.plan(env, con, ends[0], ends[1], 0)
    if rc == G.CP_OK:
        _check_path(w, path, ends[0], ends[1], TAU_TASK)


def test_warm_batch_paths_pass_oracle_revalidation(G, trained):
    w, robot, con, net = trained
    env = G.Env(w["env"])
    queries = []
    for seed in range(10):
        ends = manifold_starts(w, 2, 1200 + seed).astype(np.float64)
        queries.append((robot, env, con, ends[0], ends[1], seed))
    bp = G.BatchPlanner(len(queries), 7, G.batch_opts(groups_per_query=32, max_rounds=400,
                                                      capacity=8192, tau_task=TAU_TASK))
    bp.set_warm(net)
    st, paths, info = bp.plan(queries)
    print("warm batch statuses", st.tolist(), "rounds", [i["rounds"] for i in info], flush=True)
    assert (st == G.CP_OK).sum() >= 5
    for (rb, e, c, a, b, s), rc, path in zip(queries, st, paths):
        assert rc in (G.CP_OK, G.CP_NO_SOLUTION)
        if rc == G.CP_OK:
            _check_path(w, path, a, b, TAU_TASK)


def test_warm_batch_needs_one_robot_and_constraint(G, trained):
    w, robot, con, net = trained
    env = G.Env(w["env"])
    ends = manifold_starts(w, 2, 1300).astype(np.float64)
    other = G.Robot(w["robot"])        # the same description, another handle
    bp = G.BatchPlanner(2, 7, G.batch_opts(groups_per_query=8, max_rounds=8, tau_task=TAU_TASK))
    bp.set_warm(net)
    with pytest.raises(G.CprrtcError) as ex:
        bp.plan([(robot, env, con, ends[0], ends[1], 1), (other, env, con, ends[0], ends[1], 2)])
    assert ex.value.code == G.CP_E_UNSUPPORTED
    # a network of the wrong shape for the robot
    wrong = G.MLP(9, 64, 2, 3, seed=1)
    pl = G.Planner(robot, G.plan_opts(n_groups=8, max_rounds=4, tau_task=TAU_TASK))
    pl.set_warm(wrong)
    with pytest.raises(G.CprrtcError) as ex:
        pl.plan(env, con, ends[0], ends[1], 1)
    assert ex.value.code == G.CP_E_ARG
    # self-collision checks are not part of the warm-started rounds
    pl2 = G.Planner(robot, G.plan_opts(n_groups=8, max_rounds=4, tau_task=TAU_TASK,
                                       flags=G.SELF_COLLISION))
    with pytest.raises(G.CprrtcError) as ex:
        pl2.set_warm(net)
    assert ex.value.code == G.CP_E_UNSUPPORTED


def test_warm_batch_gain_or_loss_is_bounded(G, trained):
    """The same 24 queries planned in one batch plainly and warm-started, with
    the same budget: the warm-started batch must solve at least as many
    queries less one, and its mean rounds per solved query may exceed the
    plain batch's by at most half plus two rounds (measured on 128 such
    queries with the benchmark's network: all solved either way, the batch
    done after 12 rounds against 16, 21 ms against 25 ms)."""
    w, robot, con, net = trained
    env = G.Env(w["env"])
    queries = []
    for seed in range(24):
        ends = manifold_starts(w, 2, 1400 + seed).astype(np.float64)
        queries.append((robot, env, con, ends[0], ends[1], seed))
    out = {}
    for warm in (False, True):
        bp = G.BatchPlanner(len(queries), 7, G.batch_opts(groups_per_query=32, max_rounds=800,
                                                          capacity=8192, tau_task=TAU_TASK))
        bp.set_warm(net if warm else None)
        st, paths, info = bp.plan(queries)
        ok = st == G.CP_OK
        out[warm] = (int(ok.sum()), float(np.mean([i["rounds"] for i, o in zip(info, ok) if o])))
        for (rb, e, c, a, b, s), rc, path in zip(queries, st, paths):
            if rc == G.CP_OK:
                _check_path(w, path, a, b, TAU_TASK)
    print("solved / rounds: plain", out[False], "warm", out[True], flush=True)
    assert out[True][0] >= out[False][0] - 1
    assert out[True][1] <= 1.5 * out[False][1] + 2

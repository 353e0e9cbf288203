"""Launch autotuner: it times every candidate shape on the caller's sample
motions and returns the fastest; the sphere batch it picks never changes a
verdict (early-exit polls sit between batches only)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2505_06791_amd import inputs as I
from tests.helpers import motion_set

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_06791_amd import cprrtc
    cprrtc.lib()
    return cprrtc


def _run(G, robot, env, con, prm, qf, qt, dof):
    M = qf.shape[0]
    xi = torch.empty((M, prm.W, dof), device=DEV)
    st = torch.empty(M, dtype=torch.int32, device=DEV)
    G.project_validate_motions(robot, env, con, prm, qf, qt, xi, st)
    torch.cuda.synchronize()
    return st.cpu().numpy(), xi.cpu().numpy()


@pytest.mark.parametrize("tune_W", [False, True])
def test_autotune_picks_the_fastest_candidate(G, tune_W):
    w = I.workload("cluttered", 2001)
    dof = w["robot"]["dof"]
    q_from, q_to = motion_set(w, 256, 2500)
    robot, env, con = G.Robot(w["robot"]), G.Env(w["env"]), G.constraint(w["constraint"])
    base = G.proj_params(W=64, tau_task=1e-3)
    qf, qt = torch.from_numpy(q_from).to(DEV), torch.from_numpy(q_to).to(DEV)
    chosen, cands = G.autotune(robot, env, con, base, qf, qt, tune_W=tune_W, reps=2)
    print(cands, "->", chosen.W, chosen.sphere_batch, flush=True)
    assert len(cands) == (6 if tune_W else 3)
    best = max(cands, key=lambda c: c["waypoints_per_s"])
    assert (chosen.W, chosen.sphere_batch) == (best["W"], best["sphere_batch"])
    assert all(c["ms"] > 0 for c in cands)
    if not tune_W:
        assert chosen.W == 64
    # everything but the launch shape is kept
    assert chosen.tau_task == base.tau_task and chosen.max_iters == base.max_iters
    # the chosen sphere batch gives the base verdicts at the same W
    same = G.proj_params(W=chosen.W, tau_task=1e-3, sphere_batch=4)
    if chosen.W != 64:
        s = (chosen.W - 1) / 63
        qt = qf + s * (qt - qf)
    st_a, xi_a = _run(G, robot, env, con, same, qf, qt, dof)
    st_b, xi_b = _run(G, robot, env, con, chosen, qf, qt, dof)
    assert np.array_equal(st_a, st_b)
    assert np.array_equal(xi_a, xi_b)


def test_autotune_rejects_bad_arguments(G):
    w = I.workload("plain", 1000)
    robot, env, con = G.Robot(w["robot"]), G.Env(w["env"]), G.constraint(w["constraint"])
    q = torch.zeros((4, 7), device=DEV)
    with pytest.raises(G.CprrtcError) as ex:
        G.autotune(robot, env, con, G.proj_params(), q, q, reps=0)
    assert ex.value.code == G.CP_E_ARG
    with pytest.raises(G.CprrtcError) as ex:
        G.autotune(robot, env, con, G.proj_params(W=48), q, q)
    assert ex.value.code == G.CP_E_UNSUPPORTED

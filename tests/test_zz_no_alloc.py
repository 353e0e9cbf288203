"""project_motions_warm_noalloc (the warm start for callers that cannot
allocate) against project_motions_warm on the same inputs: both run the same
kernels, so statuses, iterations and waypoints must be equal bit for bit, on
two calls in a row (the second smaller, so stale rows of the shared fixed
buffer would show), and a batch beyond the fixed buffer is refused before
anything is launched."""
import ctypes as C

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


def _run(G, robot, con, prm, net, q_from, q_to, noalloc, flags=0):
    M, W, dof = q_from.shape[0], prm.W, q_from.shape[1]
    xi = torch.full((M, W, dof), float("nan"), device=DEV)
    st = torch.full((M,), -7, dtype=torch.int32, device=DEV)
    it = torch.full((M,), -7, dtype=torch.int32, device=DEV)
    G.project_motions_warm(robot, con, prm, net, q_from, q_to, xi, st, it, flags=flags,
                           noalloc=noalloc)
    torch.cuda.synchronize()
    return xi.cpu().numpy(), st.cpu().numpy(), it.cpu().numpy()


@pytest.mark.parametrize("flags", [0, 4])
def test_noalloc_equals_allocating_entry_point(G, flags):
    from paper_2505_06791_amd import warmstart
    w = I.workload("plain", 1000)
    rd, cd = w["robot"], w["constraint"]
    robot, con = G.Robot(rd), G.constraint(cd)
    net = G.MLP(warmstart.n_inputs(rd, cd), 256, 3, rd["dof"], seed=11)
    prm = G.proj_params(W=64, tau_task=1e-4)
    qf, qt = motion_set(w, 160, 77)
    for n in (160, 37):      # the second call is smaller than the first
        q_from = torch.from_numpy(qf[:n]).to(DEV)
        q_to = torch.from_numpy(qt[:n]).to(DEV)
        xa, sa, ia = _run(G, robot, con, prm, net, q_from, q_to, False, flags)
        xb, sb, ib = _run(G, robot, con, prm, net, q_from, q_to, True, flags)
        assert np.array_equal(sa, sb) and np.array_equal(ia, ib), n
        assert set(np.unique(sb)).issubset({0, 1}), n
        done = sb == 0
        assert np.array_equal(xa[done], xb[done]), n
        print(f"n={n} flags={flags}: statuses {np.bincount(sb, minlength=2)} equal, "
              f"iterations equal, waypoints of {int(done.sum())} projected motions bitwise equal",
              flush=True)


def test_noalloc_refuses_batches_beyond_the_fixed_buffer(G):
    from paper_2505_06791_amd import warmstart
    w = I.workload("plain", 1000)
    rd, cd = w["robot"], w["constraint"]
    robot, con = G.Robot(rd), G.constraint(cd)
    net = G.MLP(warmstart.n_inputs(rd, cd), 256, 3, rd["dof"], seed=11)
    prm = G.proj_params(W=64, tau_task=1e-4)
    limit = (8 << 20) // (63 * rd["dof"])
    small = torch.zeros((1, rd["dof"]), device=DEV)
    out = torch.zeros((1, 64, rd["dof"]), device=DEV)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    L = G.lib()
    for n, want in ((limit + 1, G.CP_E_CAPACITY), (1 << 30, G.CP_E_CAPACITY)):
        rc = L.project_motions_warm_noalloc(
            robot.handle, C.byref(con), C.byref(prm), net.handle, n, small.data_ptr(),
            small.data_ptr(), out.data_ptr(), st.data_ptr(), None, None, 0, None)
        assert rc == want, (n, rc)
        assert b"exceed" in L.cp_last_error()
    torch.cuda.synchronize()

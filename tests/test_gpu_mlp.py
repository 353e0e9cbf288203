"""Learned warm start on the GPU: network kernels against references, the
fallback guarantee, and what the trained network gains.

Bars: the forward pass equals a float32 reference that rounds at the same
points (BF16 input, weights and hidden activations; FP32 bias, accumulation
and output) to 1e-2 of the output range (an activation may round to the
neighbouring BF16 value: 2^-8 relative; a wrong operand layout errs by
O(1)); gradients agree element by element with the FP64 oracle evaluated at
the same BF16-rounded weights and inputs: |g - g_oracle| <= 1e-2 max|g_oracle|
+ 2e-2 |g_oracle| per tensor.  The GPU also rounds hidden activations and
back-propagated errors to BF16; emulating those roundings in float32 against
the FP64 oracle gives at most 4.1e-3 of the tensor's maximum (five random
13 -> 3 x 256 -> 7 networks), so the bar has a 2.4x margin, and a swapped,
transposed or sign-flipped term errs by O(1) of the maximum.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from paper_2505_06791_amd import inputs as I
from tests.helpers import BAND, motion_set, oracle_views

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_06791_amd import cprrtc
    cprrtc.lib()
    return cprrtc


def bf16(t):
    return t.to(torch.bfloat16).to(torch.float32)


def split_params(p, dims):
    out, off = [], 0
    for l in range(len(dims) - 1):
        k, n = dims[l], dims[l + 1]
        W = p[off:off + n * k].reshape(n, k)
        off += n * k
        b = p[off:off + n]
        off += n
        out.append((W, b))
    return out


def reference_forward(p, dims, x):
    h = bf16(x)
    layers = split_params(p, dims)
    for l, (W, b) in enumerate(layers):
        z = h @ bf16(W).t() + b
        h = bf16(torch.nn.functional.silu(z)) if l + 1 < len(layers) else z
    return h


@pytest.mark.parametrize("dims_hidden", [(13, 256, 3, 7), (26, 512, 3, 14), (5, 64, 2, 3)])
def test_forward_matches_reference(G, dims_hidden):
    n_in, hid, nh, n_out = dims_hidden
    net = G.MLP(n_in, hid, nh, n_out, seed=3)
    g = torch.Generator(device=DEV)
    g.manual_seed(0)
    for M in (1, 63, 257, 4096):
        x = torch.randn((M, n_in), generator=g, device=DEV)
        y = net.forward(x)
        ref = reference_forward(net.get_params(), net.dims, x)
        err = ((y - ref).abs().max() / ref.abs().max().clamp_min(1e-6)).item()
        assert err < 1e-2, (M, err)


@pytest.mark.parametrize("dims_hidden,M", [((13, 256, 3, 7), 96), ((26, 512, 3, 14), 300),
                                           ((5, 64, 2, 3), 1000), ((13, 256, 3, 7), 9000)])
def test_gradients_match_fp64_oracle(G, dims_hidden, M):
    n_in, hid, nh, n_out = dims_hidden
    net = G.MLP(n_in, hid, nh, n_out, seed=4)
    g = torch.Generator(device=DEV)
    g.manual_seed(1)
    x = torch.randn((M, n_in), generator=g, device=DEV)
    t = torch.randn((M, n_out), generator=g, device=DEV) * 0.3
    grad, loss = net.gradients(x, t)
    # oracle at the BF16-rounded weights the matrix cores used, FP32 biases
    p = net.get_params()
    pr = p.clone()
    off = 0
    for l in range(len(net.dims) - 1):
        k, n = net.dims[l], net.dims[l + 1]
        pr[off:off + n * k] = bf16(p[off:off + n * k])
        off += n * k + n
    loss_o, grad_o = O.mlp_gradients(net.dims, pr.cpu().double().numpy(),
                                     bf16(x).cpu().double().numpy(), t.cpu().double().numpy())
    gg = grad.cpu().double().numpy()
    assert abs(loss.item() - loss_o) <= 2e-2 * loss_o
    off = 0
    worst = 0.0
    for l in range(len(net.dims) - 1):
        k, n = net.dims[l], net.dims[l + 1]
        for what, sl in (("W", slice(off, off + n * k)), ("b", slice(off + n * k, off + n * k + n))):
            a, b = gg[sl], grad_o[sl]
            scale = np.abs(b).max()
            assert scale > 0, (l, what)
            excess = np.abs(a - b) - (1e-2 * scale + 2e-2 * np.abs(b))
            worst = max(worst, float((np.abs(a - b) / scale).max()))
            assert np.all(excess <= 0), (l, what, int(np.argmax(excess)), float(excess.max()))
        off += n * k + n
    print("gradients", dims_hidden, "M", M, "max |g - g_oracle| / max|g_oracle|", f"{worst:.2e}",
          flush=True)


def test_training_reduces_the_loss(G):
    net = G.MLP(8, 128, 2, 3, seed=5)
    g = torch.Generator(device=DEV)
    g.manual_seed(2)
    x = torch.rand((16384, 8), generator=g, device=DEV) * 2 - 1
    t = torch.stack([torch.sin(2 * x[:, 0]) * x[:, 1], x[:, 2] * x[:, 3], torch.cos(x[:, 4])], 1)
    from paper_2505_06791_amd import warmstart
    hist = warmstart.train(net, x.contiguous(), t.contiguous(), epochs=8, batch=1024, lr_max=3e-3)
    assert hist[-1] < 0.1 * hist[0], hist


def _revalidate_segments(w, xi, st, W, tau_task):
    ro, eo, co = oracle_views(w)
    for m in np.nonzero(st == 0)[0]:
        x = xi[m].astype(np.float64)
        for k in range(1, W):
            assert np.abs(O.task_error(ro, co, x[k])).max(initial=0.0) < tau_task + BAND
            assert np.linalg.norm(x[k] - x[k - 1]) < 0.075 + BAND


def _project(G, w, q_from, q_to, tau_task, mlp=None, W=64, flags=0):
    robot, con = G.Robot(w["robot"]), G.constraint(w["constraint"])
    prm = G.proj_params(W=W, tau_task=tau_task)
    M, dof = len(q_from), w["robot"]["dof"]
    qf, qt = torch.from_numpy(q_from).to(DEV), torch.from_numpy(q_to).to(DEV)
    xi = torch.empty((M, W, dof), device=DEV)
    st = torch.empty(M, dtype=torch.int32, device=DEV)
    it = torch.empty(M, dtype=torch.int32, device=DEV)
    if mlp is None:
        G.project_motions(robot, con, prm, qf, qt, xi, st, it)
    else:
        G.project_motions_warm(robot, con, prm, mlp, qf, qt, xi, st, it, flags=flags)
    torch.cuda.synchronize()
    return xi.cpu().numpy(), st.cpu().numpy(), it.cpu().numpy()


def test_warm_start_with_untrained_network_keeps_every_plain_success(G):
    """The plain projector is the fallback: whatever the network predicts,
    a motion the plain projector projects is projected, and every projected
    segment passes re-validation by the oracle."""
    w = I.workload("plain", 1000)
    q_from, q_to = motion_set(w, 40, 21)
    from paper_2505_06791_amd import warmstart
    net = G.MLP(warmstart.n_inputs(w["robot"], w["constraint"]), 64, 2, 7, seed=9)
    _, st_p, _ = _project(G, w, q_from, q_to, 1e-4)
    xi_w, st_w, _ = _project(G, w, q_from, q_to, 1e-4, mlp=net)
    assert np.all(st_w[st_p == 0] == 0)
    _revalidate_segments(w, xi_w, st_w, 64, 1e-4)


def test_warm_start_network_shape_is_checked(G):
    w = I.workload("plain", 1000)
    net = G.MLP(5, 32, 1, 7)
    q = torch.zeros((1, 7), device=DEV)
    with pytest.raises(G.CprrtcError) as ex:
        G.project_motions_warm(G.Robot(w["robot"]), G.constraint(w["constraint"]), G.proj_params(),
                               net, q, q, torch.empty((1, 64, 7), device=DEV),
                               torch.empty(1, dtype=torch.int32, device=DEV))
    assert ex.value.code == G.CP_E_ARG


def test_trained_warm_start_gain(G):
    """Train on pairs the projector produces (plain scene, upright), then
    compare on held-out motions at tolerance 1e-4: the warm start must not
    lose a motion the plain projector projects, and with the fallback it
    must project at least 3 points more of the motions (measured: 75% plain,
    86% warm + fallback on these 300)."""
    from paper_2505_06791_amd import warmstart
    w = I.workload("plain", 1000)
    rd, cd = w["robot"], w["constraint"]
    X, T = warmstart.make_pairs(rd, cd, 8192, seed=4000)
    net = G.MLP(warmstart.n_inputs(rd, cd), 256, 3, rd["dof"], seed=4000)
    hist = warmstart.train(net, X, T, epochs=6, batch=4096)
    q_from, q_to = motion_set(w, 300, 4100)
    _, st_p, it_p = _project(G, w, q_from, q_to, 1e-4)
    xi_w, st_w, it_w = _project(G, w, q_from, q_to, 1e-4, mlp=net)
    _, st_o, it_o = _project(G, w, q_from, q_to, 1e-4, mlp=net, flags=G.WARM_NO_FALLBACK)
    both = (st_p == 0) & (st_o == 0)
    print("warm start: train loss", [f"{h:.2e}" for h in hist],
          "| success plain", (st_p == 0).mean(), "warm pass", (st_o == 0).mean(),
          "warm+fallback", (st_w == 0).mean(),
          "| mean iterations where plain and warm pass both project: plain", it_p[both].mean(),
          "warm", it_o[both].mean(), "| all motions incl. fallback: plain", it_p.mean(),
          "warm+fallback", it_w.mean(), flush=True)
    assert hist[-1] < hist[0]
    assert np.all(st_w[st_p == 0] == 0)
    assert (st_w == 0).mean() >= (st_p == 0).mean() + 0.03
    _revalidate_segments(w, xi_w, st_w, 64, 1e-4)


@pytest.mark.parametrize("name,seed", [("plain", 1000), ("dual", 5000)])
def test_warm_pairs_match_reference(G, name, seed):
    """cp_warm_pairs: features (straight waypoint over the joint range, then
    the constraint parameters) and targets (projected - straight waypoint) of
    every waypoint k >= 1, against float32 references computed here."""
    from paper_2505_06791_amd import warmstart
    w = I.workload(name, seed)
    rd, cd = w["robot"], w["constraint"]
    robot, con = G.Robot(rd), G.constraint(cd)
    W = 64 if name == "plain" else 32
    q_from, q_to = warmstart.motion_ends(rd, robot, con, 64, seed=77, W=W)
    M, dof = q_from.shape
    xi = torch.randn((M, W, dof), device=DEV)          # any segment: the kernel only subtracts
    x, t = G.warm_pairs(robot, con, W, q_from, q_to, xi, warmstart.n_inputs(rd, cd))
    s = (torch.arange(W, device=DEV, dtype=torch.float32) / (W - 1))[None, :, None]
    straight = (q_from[:, None, :] + s * (q_to - q_from)[:, None, :])[:, 1:, :].reshape(-1, dof)
    rng = torch.from_numpy(np.maximum(np.abs(rd["lo"]), np.abs(rd["hi"])).astype(np.float32)).to(DEV)
    cp = torch.from_numpy(warmstart.constraint_features(cd)).to(DEV)
    x_ref = torch.cat([straight / rng, cp.expand(straight.shape[0], -1)], 1)
    t_ref = xi[:, 1:, :].reshape(-1, dof) - straight
    assert torch.allclose(x, x_ref, rtol=0, atol=2e-6), (x - x_ref).abs().max().item()
    assert torch.allclose(t, t_ref, rtol=0, atol=2e-6), (t - t_ref).abs().max().item()


def test_checkpoint_resumes_exactly(G, tmp_path):
    """MLP.save / MLP.load (parameters and Adam state through the C ABI,
    a JSON header and a float32 file): a run resumed from the checkpoint
    takes bit-identical steps (the training kernels sum in a fixed order)."""
    net = G.MLP(13, 256, 3, 7, seed=11)
    g = torch.Generator(device=DEV)
    g.manual_seed(3)
    xs = [torch.randn((4096, 13), generator=g, device=DEV) for _ in range(6)]
    ts = [torch.randn((4096, 7), generator=g, device=DEV) * 0.3 for _ in range(6)]
    for i in range(3):
        net.train_step(xs[i], ts[i], 1e-3)
    path = str(tmp_path / "net")
    net.save(path)
    net2 = G.MLP.load(path)
    for i in range(3, 6):
        net.train_step(xs[i], ts[i], 1e-3)
        net2.train_step(xs[i], ts[i], 1e-3)
    torch.cuda.synchronize()
    assert torch.equal(net.get_params(), net2.get_params())
    m1a, m2a, sa = net.get_state()
    m1b, m2b, sb = net2.get_state()
    assert sa == sb == 6
    assert torch.equal(m1a, m1b) and torch.equal(m2a, m2b)
    assert torch.equal(net.forward(xs[0]), net2.forward(xs[0]))

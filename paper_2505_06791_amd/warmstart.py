"""Training of the learned warm start on pairs the projector itself produces.

Pairs (waypoint of a straight-line segment, constraint parameters) ->
(its projected value - the waypoint), taken from motions the library's own
motion projector (project_motions, Algorithm 1) projected successfully and
formed by the library (cp_warm_pairs, the features the warm start uses):
segments start at an on-manifold q_near (random configurations put on the
manifold by project_configs) and head for a random sample, at most (W-1) tau
long, as the planner draws them.  The network is trained with the library's
own forward / backward / Adam kernels (cp_mlp_train_step); the feature
layout is the one project_motions_warm builds on the device.
"""
from __future__ import annotations

import math

import numpy as np

from . import cprrtc as G
from . import inputs as I


def constraint_features(cd: dict) -> np.ndarray:
    """Constraint parameters given to the network: locked pose targets (6),
    or p* and R* row-major (12) for a relative pose."""
    if cd["kind"] == I.CON_REL_POSE:
        rt = np.asarray(cd["rel_target"], np.float64)
        return np.concatenate([rt[:3, 3], rt[:3, :3].reshape(-1)]).astype(np.float32)
    return (np.asarray(cd["target"], np.float64) * np.asarray(cd["mask"])).astype(np.float32)


def n_inputs(rd: dict, cd: dict) -> int:
    return int(rd["dof"]) + len(constraint_features(cd))


def motion_ends(rd: dict, robot, con, n: int, seed: int, W: int = 64, tau: float = 0.05,
                tol: float = 1e-5):
    """(q_from, q_to) of up to n motions: on-manifold starts heading for
    uniform samples, at most (W-1) tau long."""
    import torch
    dev = torch.device("cuda:0")
    lo = torch.from_numpy(rd["lo"].astype(np.float32)).to(dev)
    hi = torch.from_numpy(rd["hi"].astype(np.float32)).to(dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    raw = torch.from_numpy(I.random_configs(rd, n, seed).astype(np.float32)).to(dev)
    near = torch.empty_like(raw)
    ok = torch.empty(n, dtype=torch.int32, device=dev)
    G.project_configs(robot, con, raw, near, ok, tol=tol, max_iters=100)
    near = near[ok == 1].contiguous()
    rand = lo + (hi - lo) * torch.rand(near.shape, generator=gen, device=dev)
    d = rand - near
    dist = d.norm(dim=1, keepdim=True).clamp_min(1e-12)
    to = (near + d * torch.clamp((W - 1) * tau / dist, max=1.0)).contiguous()
    return near, to


def make_pairs(rd: dict, cd: dict, n_motions: int, seed: int, W: int = 64, tau: float = 0.05,
               tau_task: float = 1e-4, robot=None, con=None):
    """(features [N, n_in], targets [N, dof]) on the device from the
    successfully projected motions among n_motions: every waypoint k >= 1."""
    import torch
    robot = robot or G.Robot(rd)
    con = con or G.constraint(cd)
    dof = rd["dof"]
    q_from, q_to = motion_ends(rd, robot, con, n_motions, seed, W, tau)
    M = q_from.shape[0]
    xi = torch.empty((M, W, dof), dtype=torch.float32, device=q_from.device)
    st = torch.empty(M, dtype=torch.int32, device=q_from.device)
    G.project_motions(robot, con, G.proj_params(W=W, tau=tau, tau_task=tau_task), q_from, q_to,
                      xi, st)
    good = st == 0
    X, T = G.warm_pairs(robot, con, W, q_from, q_to, xi, n_inputs(rd, cd))
    keep = good.repeat_interleave(W - 1)
    return X[keep].contiguous(), T[keep].contiguous()


def train(mlp: G.MLP, X, T, epochs: int = 10, batch: int = 4096, lr_max: float = 1e-3,
          lr_min: float = 1e-5, seed: int = 0, log=None):
    """Adam with a cosine learning-rate schedule; returns the mean loss per epoch."""
    import torch
    n = X.shape[0]
    steps_per_epoch = max(1, n // batch)
    total = epochs * steps_per_epoch
    gen = torch.Generator(device=X.device)
    gen.manual_seed(seed)
    loss = torch.zeros(1, dtype=torch.float32, device=X.device)
    history = []
    step = 0
    for ep in range(epochs):
        perm = torch.randperm(n, generator=gen, device=X.device)
        acc = torch.zeros(1, dtype=torch.float32, device=X.device)
        for b in range(steps_per_epoch):
            idx = perm[b * batch:(b + 1) * batch]
            xb, tb = X[idx].contiguous(), T[idx].contiguous()
            lr = lr_min + 0.5 * (lr_max - lr_min) * (1 + math.cos(math.pi * step / total))
            mlp.train_step(xb, tb, lr, loss)
            acc += loss
            step += 1
        history.append(float(acc.item()) / steps_per_epoch)
        if log:
            log(f"epoch {ep}: loss {history[-1]:.3e}")
    return history

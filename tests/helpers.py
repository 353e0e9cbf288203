"""Shared test helpers: seeded workloads prepared with the oracle.

Inputs handed to the HIP path are float32; the oracle receives the very same
float32 values promoted to float64.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle as O
from paper_2505_06791_amd import inputs as I

BAND = 1e-5   # |signed distance| or validity margin below which a float32 run may flip
# threads for the oracle's batched calls and the preparation below (the
# oracle releases the interpreter lock inside each call)
ORACLE_THREADS = max(1, min(16, os.cpu_count() or 1))


def oracle_views(w):
    return O.Robot(w["robot"]), O.Env(w["env"]), O.Constraint(w["constraint"])


def manifold_starts(w, n, seed, margin=1e-3, tol=1e-9, max_tries=40):
    """n configurations projected onto the constraint manifold (oracle, FP64)
    and collision-free by more than `margin`, as float32."""
    ro, eo, co = oracle_views(w)

    def prepare(q):
        ok, qp, _ = O.project_config(ro, co, q, tol=tol, max_iters=100)
        return qp if ok and O.config_min_sd(ro, eo, qp) > margin else None

    out = []
    tries = 0
    with ThreadPoolExecutor(ORACLE_THREADS) as ex:
        while len(out) < n and tries < max_tries:
            for qp in ex.map(prepare, I.random_configs(w["robot"], 4 * n, seed + 7919 * tries)):
                if qp is not None:
                    out.append(qp)
                    if len(out) == n:
                        break
            tries += 1
    assert len(out) == n, f"only {len(out)} of {n} start configurations found"
    return np.asarray(out).astype(np.float32)


def motion_set(w, n, seed, W=64, tau=0.05, collision_free_start=True):
    q_from = manifold_starts(w, n, seed, margin=1e-3 if collision_free_start else -1e9)
    q_to = I.random_displacements(w["robot"], q_from.astype(np.float64), (W - 1) * tau,
                                  seed + 1).astype(np.float32)
    return q_from, q_to

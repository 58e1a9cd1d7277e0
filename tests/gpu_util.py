"""Shared helpers of the GPU parity tests (oracle calls and tolerances)."""
import numpy as np
import pytest
import torch

import oracle as O

ALPHA = 0.15

# Tolerances (FP32 path against the FP64 oracle at the same push count T):
PPR_ABS = 1e-6        # pi_hat, max abs
DPPR_ABS = 1e-6       # d(s) pi_hat / max(1, d(s)), max abs (the PPR bound read per unit degree)
PDIST_REL = 1e-5      # Delta, relative
STRESS_REL = 1e-5     # stress of a given layout, relative
STEP_REL = 1e-5       # one Jacobi step, relative to the layout's scale


def get_ops():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_2112_14944_amd import ops
    return ops


def oracle_ppr(g, sources, tol=None, T=None):
    W = O.weight_matrix(g.n, g.eu, g.ev, g.weight)
    d = O.degrees(W)
    P = O.transition(W)
    est, t, res = O.ppr_power_iteration(P, np.asarray(sources), ALPHA, tol=tol, fixed_iters=T)
    return est, O.dppr(est, d, sources), t, res, d


def assert_ppr_close(gpu_ppr, gpu_dppr, est, dppr_o, d_src):
    gp = gpu_ppr.double().cpu().numpy()
    gd = gpu_dppr.double().cpu().numpy()
    err = np.abs(gp - est).max()
    assert err <= PPR_ABS, f"PPR max-abs {err:.3e}"
    scale = np.maximum(1.0, d_src)[:, None]
    errd = (np.abs(gd - dppr_o) / scale).max()
    assert errd <= DPPR_ABS, f"DPPR max-abs per unit degree {errd:.3e}"
    return err, errd


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)

"""Helpers shared by the GPU parity tests."""
import numpy as np
import pytest

import oracle

TOL = {np.float64: 1e-12, np.float32: 2e-6}


def need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def rel_error(y, y_ref, scale):
    """max_i |y_i - y_ref,i| / scale_i, where rows with scale_i = 0 must match
    exactly (they contribute inf otherwise)."""
    y = np.asarray(y, np.float64)
    diff = np.abs(y - y_ref)
    zero = scale == 0
    if np.any(diff[zero] != 0):
        return np.inf
    if np.all(zero):
        return 0.0
    return float(np.max(diff[~zero] / scale[~zero]))


def check_spmv(y_gpu, rp, ci, v, x, y0, alpha, beta, dtype):
    y_ref = oracle.spmv(rp, ci, v, x, y0, alpha=alpha, beta=beta)
    scale = abs(alpha) * oracle.absmv(rp, ci, v, x)
    if beta != 0:
        scale = scale + abs(beta) * np.abs(np.asarray(y0, np.float64))
    err = rel_error(y_gpu, y_ref, scale)
    assert err <= TOL[dtype], "relative error %g > %g" % (err, TOL[dtype])
    return err


def progress(msg):
    print("[gpu] " + msg, flush=True)

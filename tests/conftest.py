"""Test configuration: registers the ``gpu`` marker and puts the repository
root on sys.path so that ``oracle`` and ``paper_0903_1949_amd`` import."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP path through the C ABI)")
    config.addinivalue_line("markers", "slow: oracle cases that take tens of seconds on the CPU")


import numpy as np
import pytest


def rel_err(a, b, floor=1e-4):
    """Per-array error metric used for every parity check:
    max_i |a_i - b_i| / max(|b_i|, floor * max_j |b_j|).  Relative where the
    reference is not tiny, absolute at a floor of 1e-4 of the array's scale
    (e.g. I- at the top, where I_top = 0)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if b.size == 0:
        return 0.0
    scale = np.max(np.abs(b))
    if scale == 0.0:
        return float(np.max(np.abs(a)))
    den = np.maximum(np.abs(b), floor * scale)
    return float(np.max(np.abs(a - b) / den))


def switch_slab(na, nf=5):
    """One two-level slab of unit opacity whose layers put Delta = dtau/mu
    just below and just above 1/4 (relative offsets 1e-3, 1e-6, 1e-9) for
    every angle in turn: the switch between the thin-layer series and the
    exponential in the sweeps.  Synthetic; returns a workloads.TwoLevelBatch."""
    from oracle.quadrature import gauss_legendre01
    from paper_0903_1949_amd import workloads as W
    mu, _ = gauss_legendre01(na)
    offsets = [s * f for f in (1e-3, 1e-6, 1e-9) for s in (-1.0, 1.0)]
    steps = [0.25 * m * (1.0 + o) for m in mu for o in offsets]
    tau = 1e-3 + np.concatenate([[0.0], np.cumsum(steps)])
    nd = tau.shape[0]
    _, phi, wnu = W.doppler_grid(nf)
    return W.TwoLevelBatch(nd=np.array([nd], np.int32), tau=tau, q=np.ones((nd, nf)), phi=phi,
                           wnu=wnu, eps=np.array([1e-3]), B=1.0 + 0.5 * tau / tau[-1],
                           S_trial=1.0 - 0.7 * np.exp(-3.0 * tau), na=na)


@pytest.fixture(scope="session")
def gpu_ctx():
    """libpprt context on cuda:0.  GPU tests fail (not skip) without a device:
    they must never pass on a fallback."""
    import torch
    from paper_0903_1949_amd import pprt
    if not torch.cuda.is_available():
        pytest.fail("GPU test selected but no HIP device is visible")
    torch.cuda.set_device(0)
    ctx = pprt.Context(0)
    yield ctx
    torch.cuda.synchronize()
    ctx.close()

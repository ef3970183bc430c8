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


def rel_err_terms(a, b, mag, scale=None):
    """Error of a sum whose terms may cancel, element by element relative to
    the magnitude of its terms: max |a - b| / mag, with mag = sum |term|.
    `scale` (e.g. |S|) floors mag at 1e-15 scale: the oracle forms each term
    as a difference I - S in FP64, so below that a term is indistinguishable
    from zero (entries with neither terms nor a floor must agree exactly)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    mag = np.asarray(mag, dtype=np.float64)
    if scale is not None:
        mag = np.maximum(mag, 1e-15 * np.abs(np.asarray(scale, dtype=np.float64)))
    if b.size == 0:
        return 0.0
    d = np.abs(a - b)
    if np.any(d[mag == 0.0] != 0.0):
        return float("inf")
    nz = mag > 0.0
    return float(np.max(d[nz] / mag[nz])) if np.any(nz) else 0.0


def rel_err_elem(a, b, tiny=1e-300):
    """Plain element-wise relative error max |a - b| / max(|b|, tiny): no
    floor tied to the array's scale."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if b.size == 0:
        return 0.0
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), tiny)))


U64 = 2.0 ** -53


def skeel(As, x):
    """Componentwise condition of As x = b: (|As^-1| |As| |x|)_i / |x_i|."""
    inv = np.linalg.inv(As)
    return (np.abs(inv) @ (np.abs(As) @ np.abs(x))) / np.abs(x)


def rate_magnitudes(atom, pops, J, lstar):
    """Magnitude of the terms each preconditioned rate sums over its window:
    sum W sigma (|J| + |Lambda* eta/kappa|) for [dR_lu] (with G for [dR_ul])
    and sum W U (1 + |p Lambda*|) for [R*_ul]."""
    from oracle import rates
    o = rates.opacities(atom, pops)
    sig = rates.cross_sections(atom)
    G = atom.Gst
    U = atom.bfac[None, :] * G * sig
    p = o["chi_t"] / o["kappa"]
    dJmag = np.abs(J) + np.abs(lstar * o["eta_t"] / o["kappa"])
    W = atom.W[None, :]
    rows = pops.shape[0]
    m = [np.zeros((rows, atom.nt)) for _ in range(3)]
    for t in range(atom.nt):
        sl = slice(int(atom.k0[t]), int(atom.k1[t]))
        m[0][:, t] = np.sum(np.abs(W[:, sl] * sig[:, sl]) * dJmag[:, sl], axis=1)
        m[1][:, t] = np.sum(np.abs(W[:, sl] * G[:, sl] * sig[:, sl]) * dJmag[:, sl], axis=1)
        m[2][:, t] = np.sum(np.abs(W[:, sl] * U[:, sl]) * (1.0 + np.abs(p[:, sl] * lstar[:, sl])), axis=1)
    return m


def population_error_ratio(atom, pops_old, rates_ref, got, eps_rate, J, lstar):
    """Largest ratio of the populations' relative error to its bound.  Both
    sides solve the statistical equilibrium for x = n / n_old by LU with
    partial pivoting (backward stable); with rate-matrix entries that differ
    by at most delta_r of themselves, each x_i may differ by
    (delta_r + 8 n u) times its componentwise (Skeel) condition.  delta_r is
    eps_rate times the largest ratio, over the row's entries, of the
    magnitude of the terms summed into a rate to the entry (rates with
    collisions); eps_rate is the relative accuracy of those terms (the
    formal-solution and rate-assembly contracts).  The same delta_r bounds
    the componentwise backward error (Oettli-Prager) of the result in the
    oracle's system, max_i |As x - b|_i / (|As| |x| + |b|)_i, which is the
    sharper of the two checks.  Returns (forward ratio, worst relative
    error, backward ratio)."""
    from oracle import rates
    mag = rate_magnitudes(atom, pops_old, J, lstar)
    P_lu = rates_ref[0] + atom.Clu
    P_ul = rates_ref[2] + rates_ref[1] + atom.Cul
    rel = np.maximum(mag[0] / np.abs(P_lu), (mag[1] + mag[2]) / np.abs(P_ul))
    delta_row = eps_rate * rel.max(axis=1)
    worst, ratio, bw = 0.0, 0.0, 0.0
    for r in range(pops_old.shape[0]):
        A, rhs = rates.rate_matrix(atom, r, *rates_ref)
        As = A * pops_old[r][None, :]
        x_ref = np.linalg.solve(As, rhs)
        x = got[r] / pops_old[r]
        err = np.abs(x - x_ref) / np.abs(x_ref)
        tol = delta_row[r] + 8.0 * atom.nl * U64
        worst = max(worst, float(err.max()))
        ratio = max(ratio, float(np.max(err / (tol * skeel(As, x_ref)))))
        omega = np.abs(As @ x - rhs) / (np.abs(As) @ np.abs(x) + np.abs(rhs))
        bw = max(bw, float(omega.max() / tol))
    return ratio, worst, bw


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

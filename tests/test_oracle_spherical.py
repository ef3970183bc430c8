"""Pins of the spherical oracle: the mu quadrature at every shell, the exact
constant state, the closed-form solution for a uniform source and opacity
(path lengths computed directly, no recursion), the same on the thin shells
of a log-tau radial grid against a 60-digit evaluation, Lambda* against
brute-force unit columns, and the ALI fixed point against a direct solve."""
from decimal import Decimal, localcontext

import numpy as np
import pytest

from oracle import ali, spherical
from paper_0903_1949_amd import workloads as W


def _shells(nd=12, r_in=1.0, r_out=3.0, tau_lo=1e-3, tau_hi=30.0):
    r = np.geomspace(r_out, r_in, nd)
    tau = np.concatenate([[tau_lo], np.geomspace(tau_lo * 3, tau_hi, nd - 1)])
    return r, tau


def test_mu_quadrature_is_normalised_at_every_shell():
    r, _ = _shells()
    p, inner = spherical.rays(r, 6)
    mu, w = spherical.mu_weights(r, p, inner)
    for d in range(r.shape[0]):
        hit = inner >= d
        assert abs(w[d, hit].sum() - 1.0) < 1e-14
        assert abs((w[d, hit] * mu[d, hit]).sum() - 0.5) < 1e-14       # trapezoid is exact for mu
        assert np.isclose(np.nanmax(mu[d]), 1.0) and np.nanmin(mu[d]) == 0.0


def test_constant_state_is_exact():
    r, tau = _shells()
    nd, nf = r.shape[0], 5
    q = np.random.default_rng(1).lognormal(0, 0.5, size=(nd, nf))
    B = 0.7
    out = spherical.formal_solution_sph(r, tau, q, np.full((nd, nf), B), 5, Bbot=np.full(nf, B),
                                        Bbot_prev=np.full(nf, B), Itop=np.full(nf, B))
    assert np.allclose(out["J"], B, rtol=0, atol=1e-15)
    assert np.all(np.abs(out["JmS"]) < 1e-15)
    assert np.all(np.abs(out["H"]) < 1e-15)
    assert np.allclose(out["lstar"] + out["lstar_c"], 1.0, rtol=0, atol=1e-14)


def test_uniform_sphere_closed_form():
    """S = 1 and a uniform opacity chi everywhere, nothing incident: along
    each ray I = 1 - exp(-chi * path), the path measured from where the ray
    enters the shell structure (the linear-source update is exact for a
    constant source)."""
    nd, nf, nc = 15, 3, 7
    r = np.linspace(4.0, 1.0, nd)
    chi = np.array([0.05, 0.7, 6.0])
    tau = (r[0] - r)                         # reference opacity 1 per unit length
    q = np.repeat(chi[None, :], nd, axis=0)
    out = spherical.formal_solution_sph(r, tau, q, np.ones((nd, nf)), nc, lower="given",
                                        Bbot=np.zeros(nf))
    p, inner = spherical.rays(r, nc)
    mu, w = out["mu"], out["w"]
    J = np.zeros((nd, nf))
    for j, pj in enumerate(p):
        m = int(inner[j])
        z = np.sqrt(np.maximum(0.0, r[: m + 1] ** 2 - pj ** 2))
        z0 = z[0]
        core = pj < r[-1]
        for d in range(m + 1):
            path_in = z0 - z[d]
            # outward: from the core, or from the entry point through the tangent point
            path_out = (z[d] - z[m]) if core else (z0 + z[d])
            Iin = 1 - np.exp(-chi * path_in)
            Iout = 1 - np.exp(-chi * path_out)
            J[d] += 0.5 * w[d, j] * (Iin + Iout)
    assert np.max(np.abs(out["J"] - J)) < 1e-13


def test_thin_shells_against_high_precision():
    """The paper's line-test sphere (Sect. 3.1): r_out = 2 r_c, tau_std log
    from 1e-4 to 1e8 at constant continuum opacity, so the outer shells are
    ~1e-12 r thick.  S = 1, uniform q, nothing incident: J against the same
    sums in 60-digit decimal arithmetic (paths z_d - z_{d+1} taken directly,
    I = 1 - exp(-path) per direction).  Forming z_d - z_{d+1} in float64
    loses ~1e-11 here; the oracle must stay at rounding level."""
    nd, nc = 40, 5
    tmin, tmax = 1e-4, 1e8
    tau = np.geomspace(tmin, tmax, nd)
    r = 2.0 - (tau - tmin) / (tmax - tmin)
    r[-1] = 1.0
    chi = np.array([1e-9, 1e-6, 1e-3])
    q = np.repeat(chi[None, :], nd, axis=0)
    out = spherical.formal_solution_sph(r, tau, q, np.ones((nd, 3)), nc, lower="given",
                                        Bbot=np.zeros(3))
    p, inner = spherical.rays(r, nc)
    w = out["w"]
    J = np.zeros((nd, 3))
    with localcontext() as ctx:
        ctx.prec = 60
        R = [Decimal(float(x)) for x in r]
        T = [Decimal(float(x)) for x in tau]
        for j, pj in enumerate(p):
            m, P = int(inner[j]), Decimal(float(pj))
            z = [(R[d] * R[d] - P * P).sqrt() for d in range(m + 1)]
            if pj == r[m]:
                z[m] = Decimal(0)
            core = pj < r[-1]
            seg = [(T[d + 1] - T[d]) / (R[d] - R[d + 1]) * (z[d] - z[d + 1]) for d in range(m)]
            for k in range(3):
                cum = [Decimal(0)]
                for sg in seg:
                    cum.append(cum[-1] + Decimal(float(chi[k])) * sg)
                for d in range(m + 1):
                    t_out = (cum[-1] - cum[d]) if core else (2 * cum[-1] - cum[d])
                    I = 2 - (-cum[d]).exp() - (-t_out).exp()
                    J[d, k] += 0.5 * w[d, j] * float(I)
    assert np.max(np.abs(out["J"] - J) / J) < 1e-13


@pytest.mark.parametrize("nd,nf,nc,seed", [(6, 2, 3, 0), (10, 3, 5, 1)])
def test_lambda_star_equals_brute_force_diagonal(nd, nf, nc, seed):
    rng = np.random.default_rng(seed)
    r, tau = _shells(nd)
    q = rng.lognormal(0, 0.5, size=(nd, nf))
    L = spherical.lambda_matrix_sph(r, tau, q, nc)
    S = rng.uniform(0.5, 1.5, size=(nd, nf))
    out = spherical.formal_solution_sph(r, tau, q, S, nc, lower="given", Bbot=np.zeros(nf))
    diag = np.stack([np.diag(L[k]) for k in range(nf)], axis=1)
    assert np.allclose(out["lstar"], diag, rtol=1e-13, atol=1e-16)
    assert np.allclose(out["lstar_c"], 1.0 - diag, rtol=1e-12, atol=1e-15)
    J = np.einsum("kij,jk->ik", L, S)
    assert np.allclose(out["J"], J, rtol=1e-13, atol=1e-15)
    assert np.all(L >= -1e-17) and np.all(L.sum(axis=2) <= 1 + 1e-13)


def test_spherical_ali_fixed_point_equals_direct_solve():
    nd, nf, nc, eps = 12, 7, 4, 1e-2
    r, tau = _shells(nd)
    x, phi, wnu = W.doppler_grid(nf, 3.0)
    q = np.random.default_rng(3).lognormal(0, 0.3, size=nd)[:, None] * phi[None, :]
    B = np.linspace(1.0, 1.4, nd)
    res = spherical.two_level_ali_sph(r, tau, q, phi, wnu, eps, B, nc, tol=1e-14, max_iter=5000)
    assert res["converged"]
    wp = wnu * phi
    L = spherical.lambda_matrix_sph(r, tau, q, nc)
    Lbar = np.einsum("k,kij->ij", wp, L)
    bc = spherical.formal_solution_sph(r, tau, q, np.zeros((nd, nf)), nc, Bbot=np.full(nf, B[-1]),
                                       Bbot_prev=np.full(nf, B[-2]))
    Sd = np.linalg.solve(np.eye(nd) - (1 - eps) * Lbar, (1 - eps) * (bc["J"] @ wp) + eps * B)
    assert np.max(np.abs(res["S"] - Sd) / Sd) < 1e-11

"""Pins of the omega = 0 oracle against results fixed by mathematics, not by
the oracle's own formulas: quadrature exactness, high-precision integrals,
the exact linear-source (Eddington-Barbier) solution, adaptive quadrature of
the formal integral, and Lambda* against brute-force unit columns."""
import math

import mpmath
import numpy as np
import pytest
from scipy import integrate

from oracle import formal
from oracle.quadrature import gauss_legendre01


# ---------------------------------------------------------------- quadrature
@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 32])
def test_gauss_legendre01_exact_for_degree_2n_minus_1(n):
    mu, w = gauss_legendre01(n)
    assert mu.shape == (n,) and np.all((mu > 0) & (mu < 1)) and np.all(np.diff(mu) > 0)
    for p in range(0, 2 * n):
        assert abs(np.sum(w * mu ** p) - 1.0 / (p + 1)) < 1e-14 * max(1, n)
    # degree 2n is not integrated exactly (the rule is exactly Gaussian, no more)
    assert abs(np.sum(w * mu ** (2 * n)) - 1.0 / (2 * n + 1)) > 1e-8 / 10 ** n


# ------------------------------------------------------- layer weights (1D)
def _mp_weights(delta):
    d = mpmath.mpf(delta)
    e = mpmath.exp(-d)
    # the layer integrals themselves, by mpmath quadrature:
    # alpha = int_0^D (1 - t/D) e^-t dt / 1, gamma = int_0^D (t/D) e^-t dt
    alpha = mpmath.quad(lambda t: (1 - t / d) * mpmath.exp(-t), [0, d])
    gamma = mpmath.quad(lambda t: (t / d) * mpmath.exp(-t), [0, d])
    return float(e), float(alpha), float(gamma)


@pytest.mark.parametrize("delta", [1e-12, 3e-7, 1e-3, 0.0999, 0.4999, 0.5, 0.5001, 2.0, 37.0, 1e4])
def test_short_char_weights_equal_layer_integrals(delta):
    mpmath.mp.dps = 40
    e, a, g = _mp_weights(delta)
    e_o, psi_o, a_o, g_o = formal.short_char_weights(np.array([delta]))
    assert abs(e_o[0] - e) <= 1e-15 * max(e, 1e-300)
    assert abs(a_o[0] - a) <= 2e-15 * abs(a)
    assert abs(g_o[0] - g) <= 2e-15 * abs(g) + 1e-300
    assert abs(psi_o[0] - (1 - a)) <= 2e-15


# ------------------------------------------------ P1 linear source is exact
@pytest.mark.parametrize("na", [1, 3, 8])
def test_linear_source_eddington_barbier(na):
    """S = a + b tau: I+ = a + b(tau + mu) at every node and the down-going
    intensity has the closed form a + b tau - b mu - (a + b tau1 - b mu) e^{-(tau-tau1)/mu}."""
    mu, w = gauss_legendre01(na)
    tau = np.logspace(-4, 3, 41)
    q = np.ones((41, 1))
    a, b = 0.7, 0.3
    S = (a + b * tau)[:, None]
    out = formal.formal_solution(tau, q, S, mu, w, lower="diffusion",
                                 Bbot=S[-1], Bbot_prev=S[-2])
    Ip_exact = a + b * (tau[:, None] + mu[None, :])
    Im_exact = (a + b * tau[:, None] - b * mu[None, :]
                - (a + b * tau[0] - b * mu[None, :]) * np.exp(-(tau[:, None] - tau[0]) / mu[None, :]))
    assert np.max(np.abs(out["Iplus"][:, 0, :] - Ip_exact)) < 1e-12 * np.max(Ip_exact)
    assert np.max(np.abs(out["Iminus"][:, 0, :] - Im_exact)) < 1e-12 * np.max(Ip_exact)
    # emergent intensity: Eddington-Barbier is exact for a linear source
    assert np.allclose(out["Iemerg"][0], a + b * (tau[0] + mu), rtol=1e-13, atol=0)


def test_linear_source_multifrequency_nonuniform_opacity():
    """With frequency- and depth-dependent opacity the same closed form holds
    in each frequency's own optical depth scale tau_k (the trapezoid sum)."""
    rng = np.random.default_rng(11)
    nd, nf = 30, 4
    mu, w = gauss_legendre01(4)
    tau = np.logspace(-3, 2, nd)
    q = rng.lognormal(0, 0.8, size=(nd, nf))
    tk = np.zeros((nd, nf))
    tk[1:] = np.cumsum(0.5 * (q[1:] + q[:-1]) * np.diff(tau)[:, None], axis=0)
    tk += 1e-3
    a, b = 1.3, 0.05
    S = a + b * tk
    out = formal.formal_solution(tau, q, S, mu, w, lower="diffusion", Bbot=S[-1], Bbot_prev=S[-2])
    exact = a + b * (tk[:, :, None] + mu[None, None, :])
    assert np.max(np.abs(out["Iplus"] - exact)) < 1e-12 * np.max(exact)
    # H = b/3 exactly where the down-going field has converged to the diffusion form
    deep = tk[:, 0] > 60
    assert np.allclose(out["H"][deep], b / 3.0 * np.ones_like(out["H"][deep]), rtol=1e-12, atol=1e-14)


# ------------------------------------ brute-force quadrature of the formal integral
def test_formal_integral_by_adaptive_quadrature():
    """Random positive S per node, linear between nodes: the intensities at
    every node equal the formal integral of the transfer equation evaluated
    by adaptive quadrature (no use of the closed-form layer weights)."""
    rng = np.random.default_rng(5)
    nd = 7
    tau = np.array([1e-3, 0.02, 0.1, 0.35, 1.2, 3.0, 9.0])
    q = np.ones((nd, 1))
    S = rng.uniform(0.2, 2.0, size=nd)
    mu, w = gauss_legendre01(3)
    Ibot = rng.uniform(0.5, 1.5, size=3)
    out = formal.formal_solution(tau, q, S, mu, w, lower="given", Ibot=Ibot[None, :])
    Sfun = lambda t: np.interp(t, tau, S)
    for i, m in enumerate(mu):
        for d in range(nd):
            # up-going: from the bottom boundary to node d
            val, _ = integrate.quad(lambda t: Sfun(t) * math.exp(-(t - tau[d]) / m) / m,
                                    tau[d], tau[-1], points=list(tau[d:]), limit=200,
                                    epsabs=1e-14, epsrel=1e-13)
            ip = val + Ibot[i] * math.exp(-(tau[-1] - tau[d]) / m)
            assert abs(out["Iplus"][d, 0, i] - ip) < 1e-11
            val, _ = integrate.quad(lambda t: Sfun(t) * math.exp(-(tau[d] - t) / m) / m,
                                    tau[0], tau[d], points=list(tau[:d + 1]), limit=200,
                                    epsabs=1e-14, epsrel=1e-13) if d > 0 else (0.0, 0.0)
            assert abs(out["Iminus"][d, 0, i] - val) < 1e-11


# --------------------------------------------- P4 Lambda* vs brute force
@pytest.mark.parametrize("nd,nf,na,seed", [(2, 1, 1, 0), (5, 3, 2, 1), (16, 4, 4, 2)])
def test_lambda_star_equals_brute_force_diagonal(nd, nf, na, seed):
    rng = np.random.default_rng(seed)
    tau = np.logspace(-3, 3, nd)
    q = rng.lognormal(0, 0.5, size=(nd, nf))
    mu, w = gauss_legendre01(na)
    L = formal.lambda_matrix(tau, q, mu, w)
    S = rng.uniform(0.5, 1.5, size=(nd, nf))
    out = formal.formal_solution(tau, q, S, mu, w, lower="given")
    diag = np.stack([np.diag(L[k]) for k in range(nf)], axis=1)
    assert np.allclose(out["lstar"], diag, rtol=1e-14, atol=1e-16)
    assert np.allclose(out["lstar_c"], 1.0 - diag, rtol=1e-12, atol=1e-15)
    # the same Lambda matrix reproduces J for any S (linearity; zero boundaries)
    J = np.einsum("kij,jk->ik", L, S)
    assert np.allclose(out["J"], J, rtol=1e-13, atol=1e-15)
    # Lambda has non-negative entries and row sums <= 1 (a lossy slab)
    assert np.all(L >= -1e-17) and np.all(L.sum(axis=2) <= 1 + 1e-13)


def test_lambda_star_complement_keeps_relative_accuracy_when_thick():
    """In optically very thick layers Lambda* -> 1; the complement must stay
    accurate in relative terms: 1 - Lambda*_dd -> 1/2 sum w psi ~ mu/(dtau)."""
    tau = np.array([0.0, 1e6, 2e6, 3e6]) + 1.0
    q = np.ones((4, 1))
    mu, w = gauss_legendre01(4)
    out = formal.formal_solution(tau, q, np.ones(4), mu, w, lower="given")
    # interior node 1: two layers of thickness 1e6 -> psi = mu / 1e6 (e = 0)
    expect = 0.5 * np.sum(w * mu / 1e6) * 2
    assert abs(out["lstar_c"][1, 0] - expect) < 1e-15 * expect


def test_constant_source_top_mean_intensity():
    """S = B = 1 everywhere on a thick slab: I+ = 1 exactly and at the top
    J(tau1) = 1/2 sum w (1 + 1 - ...) -> 1/2 + O(tau1)."""
    mu, w = gauss_legendre01(8)
    tau = np.logspace(-8, 4, 60)
    out = formal.formal_solution(tau, np.ones((60, 1)), np.ones(60), mu, w,
                                 lower="diffusion", Bbot=np.ones(1), Bbot_prev=np.ones(1))
    assert np.allclose(out["Iplus"], 1.0, rtol=0, atol=1e-15)
    assert abs(out["J"][0, 0] - 0.5) < 1e-15
    assert abs(out["JmS"][0, 0] + 0.5) < 1e-15
    assert np.allclose(out["J"][-1], 1.0, atol=1e-15)


def test_difference_form_moments_match_plain_form():
    """J - S and H from the difference-form recursion equal J - S and H from
    the plain-form intensities to rounding relative to |S|; with constant S
    deep in a thick slab the difference form carries no rounding leak."""
    rng = np.random.default_rng(8)
    nd, nf = 40, 6
    tau = np.logspace(-4, 4, nd)
    q = rng.lognormal(0, 0.5, size=(nd, nf))
    S = rng.uniform(0.5, 1.5, size=(nd, nf))
    mu, w = gauss_legendre01(6)
    out = formal.formal_solution(tau, q, S, mu, w, lower="diffusion", Bbot=S[-1], Bbot_prev=S[-2])
    assert np.max(np.abs(out["JmS"] - (out["J"] - S))) < 1e-14 * np.abs(S).max()
    H = 0.5 * np.einsum("dki,i->dk", out["Iplus"] - out["Iminus"], w * mu)
    assert np.max(np.abs(out["H"] - H)) < 1e-14 * np.abs(S).max()
    c = formal.formal_solution(tau, np.ones((nd, 1)), np.full(nd, 0.8), mu, w, lower="diffusion",
                               Bbot=np.full(1, 0.8), Bbot_prev=np.full(1, 0.8))
    # deep down only the top boundary's exponentially small deficit remains:
    # no rounding "leak" of order 1e-16 |S|, which J - S by subtraction carries
    assert np.all(np.abs(c["JmS"][tau > 100]) < 1e-60)

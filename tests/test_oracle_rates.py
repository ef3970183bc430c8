"""Pins of the multilevel rate oracle: the collision-dominated (LTE) limit,
reduction to the two-level operator-splitting update for an isolated line,
the plain rates when Lambda* = 0, the linearity identity of the
preconditioned net rate, and statistical equilibrium at convergence."""
import copy
import math

import numpy as np
import pytest

from oracle import ali, rates
from oracle.quadrature import gauss_legendre01
from paper_0903_1949_amd import workloads as W


@pytest.fixture(scope="module")
def small_atom():
    return W.multilevel_atom(nbound=4, ncont=3, nd=14, na=4, nline_pts=12, ncont_pts=8, seed=7)


def _A(atom):
    """Spontaneous rate per transition and row: sum_k W b G sigma."""
    A = np.zeros((atom.tau.shape[0], atom.nt))
    for t in range(atom.nt):
        sl = slice(int(atom.k0[t]), int(atom.k1[t]))
        A[:, t] = np.sum(atom.W[None, sl] * atom.bfac[None, sl] * atom.Gst[:, sl] * atom.sigma[None, sl], axis=1)
    return A


def test_collision_dominated_limit_is_lte(small_atom):
    a = copy.deepcopy(small_atom)
    A = _A(a)
    a.Cul = A * 1e14
    a.Clu = a.Cul * a.nstar[:, a.up] / a.nstar[:, a.lo]
    mu, w = gauss_legendre01(a.na)
    p = a.nstar * (1 + 0.3 * np.sin(np.arange(a.nl))[None, :])     # start away from LTE
    for _ in range(2):
        p, mx, _ = rates.nlte_iteration(a, p, mu, w)
    assert np.max(np.abs(p / a.nstar - 1)) < 1e-8


def test_zero_lambda_star_gives_plain_rates(small_atom):
    a = small_atom
    rng = np.random.default_rng(1)
    J = rng.uniform(0.0, 2.0, size=(a.tau.shape[0], a.nf)) * a.Bnu
    pops = a.nstar * rng.uniform(0.5, 2.0, size=a.nstar.shape)
    dRlu, dRul, Rsul = rates.preconditioned_rates(a, pops, J, np.zeros_like(J))
    for t in range(a.nt):
        sl = slice(int(a.k0[t]), int(a.k1[t]))
        Rlu = np.sum(a.W[sl] * a.sigma[sl] * J[:, sl], axis=1)
        Rul = np.sum(a.W[sl] * (a.bfac[sl] * a.Gst[:, sl] * a.sigma[sl] + a.Gst[:, sl] * a.sigma[sl] * J[:, sl]), axis=1)
        assert np.allclose(dRlu[:, t], Rlu, rtol=1e-13, atol=0)
        assert np.allclose(Rsul[:, t] + dRul[:, t], Rul, rtol=1e-13, atol=0)


def test_preconditioned_net_rate_is_linear_identity(small_atom):
    """n_l [dR_lu] - n_u ([R*_ul] + [dR_ul]) = sum_k W chi_t (J - Lambda p S - (1 - p Lambda) S)
    = sum_k W chi_t (J - S_t) for any Lambda* when the populations are the
    ones the rates were built with (the Lambda* terms cancel)."""
    a = small_atom
    rng = np.random.default_rng(2)
    rows = a.tau.shape[0]
    J = rng.uniform(0.2, 2.0, size=(rows, a.nf)) * a.Bnu
    L = rng.uniform(0.0, 1.0, size=(rows, a.nf))
    pops = a.nstar * rng.uniform(0.5, 2.0, size=a.nstar.shape)
    dRlu, dRul, Rsul = rates.preconditioned_rates(a, pops, J, L)
    o = rates.opacities(a, pops)
    for t in range(a.nt):
        sl = slice(int(a.k0[t]), int(a.k1[t]))
        l, u = int(a.lo[t]), int(a.up[t])
        net = pops[:, l] * dRlu[:, t] - pops[:, u] * (Rsul[:, t] + dRul[:, t])
        St = o["eta_t"][:, sl] / o["chi_t"][:, sl]
        exact = np.sum(a.W[sl] * o["chi_t"][:, sl] / a.sigma[sl] * a.sigma[sl] * (J[:, sl] - St), axis=1)
        scale = np.abs(pops[:, l] * dRlu[:, t]).max()
        assert np.max(np.abs(net - exact)) < 1e-12 * scale


def _two_level_atom(nd=20, nf=15, eps=1e-2, na=4, seed=3):
    """An isolated line in a two-level atom with constant nu across the line
    (so W_k sigma_k = c w_k phi_k exactly) and no continuum."""
    from paper_0903_1949_amd.workloads import MultiLevelAtom, doppler_grid, log_tau
    x, phi, wnu = doppler_grid(nf, 3.0)
    tau = log_tau(nd, 1e-3, 1e3)
    nu0 = 0.75
    T = np.full(nd, 6000.0)
    kT = 8.617333262e-5 * T / 13.605693
    g = np.array([2.0, 8.0])
    E = np.array([0.0, nu0])
    ntot = np.full(nd, 1.0)
    ratio = g[1] / g[0] * np.exp(-nu0 / kT)
    nstar = np.stack([ntot / (1 + ratio), ntot * ratio / (1 + ratio)], axis=1)
    s = 1e3
    sigma = s * phi
    Gc = g[0] / g[1]
    b = nu0 ** 3
    Bl = b / np.expm1(nu0 / kT)
    c = s / nu0
    Cul = eps / (1 - eps) * c * Gc * (b + Bl)
    atom = MultiLevelAtom(
        nd=np.array([nd], np.int32), tau=tau, T=T, na=na, g=g, E=E, lo=np.array([0], np.int32),
        up=np.array([1], np.int32), kind=np.array([0], np.int32), k0=np.array([0], np.int32),
        k1=np.array([nf], np.int32), nu=np.full(nf, nu0), wnu=wnu, owner=np.zeros(nf, np.int32),
        sigma=sigma, bfac=np.full(nf, b), W=wnu / nu0, Gst=np.full((nd, nf), Gc),
        Bnu=np.broadcast_to(Bl[:, None], (nd, nf)).copy(), kc=np.zeros(nd), sc=np.zeros(nd),
        nstar=nstar, ntot=ntot, Cul=Cul[:, None], Clu=(Cul * nstar[:, 1] / nstar[:, 0])[:, None],
        name="two-level")
    return atom, phi, wnu, Bl


def test_two_level_reduction():
    """For an isolated line the multilevel preconditioned rates give exactly
    the two-level operator-splitting update with eps/(1-eps) = C_ul/(c G (b + B))."""
    eps = 1e-2
    atom, phi, wnu, Bl = _two_level_atom(eps=eps)
    mu, w = gauss_legendre01(atom.na)
    pops0 = atom.nstar * np.array([1.3, 0.6])[None, :]        # off LTE
    o = rates.opacities(atom, pops0)
    S0 = (o["eta_t"] / o["chi_t"])[:, 0]
    new, _, _ = rates.nlte_iteration(atom, pops0, mu, w, scattering=False)
    b, Gc = atom.bfac[0], atom.Gst[0, 0]
    S_ml = new[:, 1] * b * Gc / (new[:, 0] - new[:, 1] * Gc)
    r = ali.two_level_ali(atom.tau, o["q"], phi, wnu, eps, Bl, mu, w, tol=1e-300, max_iter=1, S0=S0)
    assert np.max(np.abs(S_ml - r["S"]) / np.abs(r["S"])) < 1e-12


@pytest.mark.slow
def test_converged_populations_satisfy_statistical_equilibrium():
    a = W.multilevel_atom(nbound=3, ncont=2, nd=16, na=4, nline_pts=10, ncont_pts=6, seed=11)
    mu, w = gauss_legendre01(a.na)
    r = rates.nlte_solve(a, mu, w, tol=1e-10, max_iter=400)
    assert r["converged"]
    fs, _ = rates.formal_solution_atom(a, r["pops"], mu, w)
    assert rates.net_rate_residual(a, r["pops"], fs["J"]) < 1e-8
    assert np.allclose(r["pops"].sum(axis=1), a.ntot, rtol=1e-13)


# ------------------------------------------------ depth-dependent Voigt profiles
def test_voigt_function_limits():
    """H(a, x) = Re w(x + i a): Gaussian for a -> 0, Lorentzian wings
    a / (sqrt(pi) x^2) (1 + 3/(2 x^2)) far out, and integral sqrt(pi)."""
    x = np.linspace(-6, 6, 241)
    assert np.max(np.abs(rates.voigt_H(1e-12, x) - np.exp(-x * x))) < 1e-11
    a, X = 0.01, np.array([300.0, 1000.0, 3000.0])
    asym = a / (math.sqrt(math.pi) * X ** 2) * (1 + 1.5 / X ** 2)
    assert np.max(np.abs(rates.voigt_H(a, X) / asym - 1)) < 1e-6
    xs = np.linspace(-2000, 2000, 4_000_001)
    integral = np.trapezoid(rates.voigt_H(a, xs), xs) + 2 * a / (math.sqrt(math.pi) * 2000.0)
    assert abs(integral / math.sqrt(math.pi) - 1) < 1e-6


def test_depth_profiles_match_the_reference_depth_grid():
    """At the reference depth (Doppler width 1e-4 of the line centre) the
    oracle's depth-dependent cross-sections equal the generator's profile,
    built independently on its own sinh-spaced grid."""
    a = W.multilevel_atom(nbound=4, ncont=3, nd=14, na=4, nline_pts=12, ncont_pts=8, seed=7,
                          depth_profiles=True)
    sig = rates.cross_sections(a)
    r1 = int(np.argmin(np.abs(a.dopp - 1e-4)))
    assert abs(a.dopp[r1] / 1e-4 - 1) < 1e-12
    # (x = (nu - nu0)/dnu_D recomputed from the stored grid carries the
    # cancellation of nu - nu0 ~ 1e-4 nu0, so ~12 digits survive)
    assert np.allclose(sig[r1], a.sigma, rtol=1e-8, atol=0)
    # other depths differ (the profiles really depend on depth)
    assert np.max(np.abs(sig[0] / a.sigma - 1)) > 1e-3


def test_depth_profiles_collision_dominated_limit_is_lte():
    a = W.multilevel_atom(nbound=4, ncont=3, nd=14, na=4, nline_pts=12, ncont_pts=8, seed=7,
                          depth_profiles=True)
    A = np.zeros((a.tau.shape[0], a.nt))
    sig = rates.cross_sections(a)
    for t in range(a.nt):
        sl = slice(int(a.k0[t]), int(a.k1[t]))
        A[:, t] = np.sum(a.W[None, sl] * a.bfac[None, sl] * a.Gst[:, sl] * sig[:, sl], axis=1)
    a.Cul = A * 1e14
    a.Clu = a.Cul * a.nstar[:, a.up] / a.nstar[:, a.lo]
    mu, w = gauss_legendre01(a.na)
    p = a.nstar * (1 + 0.3 * np.sin(np.arange(a.nl))[None, :])
    for _ in range(2):
        p, mx, _ = rates.nlte_iteration(a, p, mu, w)
    assert np.max(np.abs(p / a.nstar - 1)) < 1e-8

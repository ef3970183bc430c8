"""Pins of the omega > 0 oracle (layer operators by matrix exponential +
doubling, adding recursion, dense Lambda*) against results fixed by the
mathematics: the omega -> 0 reduction to the short-characteristic weights,
reciprocity, energy conservation, single scattering, the semi-infinite
Chandrasekhar H-function, the exact diffusion solution, flux conservation,
independence of the sublayer size, brute-force Lambda columns and the ALI
fixed point against a direct solve."""
import math

import numpy as np
import pytest

from oracle import ali, dense, formal
from oracle.quadrature import gauss_legendre01
from paper_0903_1949_amd import workloads as W

DELTAS = np.array([1e-9, 1e-3, 0.3, 2.0, 50.0, 700.0])


@pytest.mark.parametrize("na", [1, 3, 8])
def test_omega_zero_reduces_to_short_characteristics(na):
    mu, w = gauss_legendre01(na)
    L = dense.layer_operators(DELTAS, np.zeros_like(DELTAS), mu, w)
    e, psi, al, ga = formal.short_char_weights(DELTAS[:, None] / mu[None, :])
    eye = np.eye(na)
    for key in ("tp", "tm"):
        assert np.max(np.abs(L[key] - e[:, :, None] * eye)) < 1e-13
    for key in ("rp", "rm"):
        assert np.max(np.abs(L[key])) < 1e-15
    bp, bm = dense.layer_sources(L, DELTAS, np.full(6, 0.7), np.full(6, 1.3))
    assert np.max(np.abs(bp - (0.7 * al + 1.3 * ga))) < 5e-13
    assert np.max(np.abs(bm - (1.3 * al + 0.7 * ga))) < 5e-13


@pytest.mark.parametrize("omega", [0.1, 0.9, 0.999999, 1.0])
def test_reciprocity_and_symmetry(omega):
    """diag(mu w) t and diag(mu w) r are symmetric; a homogeneous layer is
    symmetric top-bottom (t+ = t-, r+ = r-)."""
    mu, w = gauss_legendre01(6)
    L = dense.layer_operators(DELTAS, np.full(6, omega), mu, w)
    Wm = np.diag(mu * w)
    for key in ("tp", "tm", "rp", "rm"):
        A = Wm @ L[key]
        assert np.max(np.abs(A - np.swapaxes(A, 1, 2))) < 1e-13
    assert np.max(np.abs(L["tp"] - L["tm"])) < 1e-12
    assert np.max(np.abs(L["rp"] - L["rm"])) < 1e-12


def test_energy_conservation_conservative_layer():
    """omega = 1: sum_i mu_i w_i (t_ij + r_ij) = mu_j w_j.  The doubling route
    loses ~1e-13 per doubling in a conservative layer, so the bound grows
    mildly with thickness."""
    mu, w = gauss_legendre01(6)
    L = dense.layer_operators(DELTAS, np.ones(6), mu, w)
    err = np.abs(np.einsum("i,lij->lj", mu * w, L["tp"] + L["rm"]) - mu * w).max(axis=1)
    assert np.all(err[:5] < 1e-12) and err[5] < 1e-9
    assert np.max(np.abs(L["bcp"])) == 0.0     # no thermal emission at omega = 1


def test_single_scattering_reflection():
    """d r_ij / d omega at omega = 0 equals the single-scattering reflection
    (w_j/2) mu_j/(mu_i+mu_j) (1 - exp(-Delta (1/mu_i + 1/mu_j)))."""
    mu, w = gauss_legendre01(4)
    dl = np.array([0.01, 0.5, 3.0])
    h = 1e-6
    Lp = dense.layer_operators(dl, np.full(3, h), mu, w)
    Lm = dense.layer_operators(dl, np.full(3, -h), mu, w)
    drdw = (Lp["rm"] - Lm["rm"]) / (2 * h)
    mi, mj = mu[:, None], mu[None, :]
    for n, D in enumerate(dl):
        exact = 0.5 * w[None, :] * mj / (mi + mj) * (1.0 - np.exp(-D * (1 / mi + 1 / mj)))
        assert np.max(np.abs(drdw[n] - exact)) < 1e-8


@pytest.mark.parametrize("omega", [0.3, 0.9, 0.99])
def test_semi_infinite_chandrasekhar_h(omega):
    """Constant thermal source B in a semi-infinite isotropically scattering
    medium: I(0, mu) = B sqrt(1 - omega) H(mu), H the discrete H-function."""
    na = 8
    mu, w = gauss_legendre01(na)
    H = dense.chandrasekhar_h(omega, mu, w)
    # the discrete H-function's zeroth moment identity
    assert abs(np.sum(w * H) - 2 * (1 - math.sqrt(1 - omega)) / omega) < 1e-12
    tau = np.concatenate([[1e-6], np.logspace(-4, 3, 40)])
    nd = tau.shape[0]
    q = np.ones((nd, 1))
    B = 1.7
    out = dense.formal_solution_dense(tau, q, np.full(nd, B), mu, w, omega=np.full((nd, 1), omega),
                                      lower="diffusion", Bbot=np.full(1, B), Bbot_prev=np.full(1, B))
    exact = B * math.sqrt(1 - omega) * H
    # the top node sits at tau = 1e-6, not 0: one thin layer of attenuation
    assert np.max(np.abs(out["Iemerg"][0] - exact) / exact) < 2e-5
    single = dense.layer_operators(np.array([1e3]), np.array([omega]), mu, w)
    assert np.max(np.abs(single["bcp"][0] * B - exact) / exact) < 1e-11


@pytest.mark.parametrize("omega", [0.0, 0.5, 0.999])
def test_diffusion_solution_exact_for_any_omega(omega):
    """S^g = a + b tau, incident I- = a - b mu, diffusion lower boundary:
    I+- = a + b tau +- b mu everywhere, J = a + b tau, H = b/3."""
    mu, w = gauss_legendre01(4)
    tau = np.logspace(-3, 2, 25)
    nd = tau.shape[0]
    a, b = 1.1, 0.4
    S = (a + b * tau)[:, None]
    out = dense.formal_solution_dense(tau, np.ones((nd, 1)), S, mu, w,
                                      omega=np.full((nd, 1), omega), Itop=(a + b * tau[0] - b * mu)[None, :],
                                      lower="diffusion", Bbot=S[-1], Bbot_prev=S[-2])
    ex_p = a + b * (tau[:, None] + mu[None, :])
    ex_m = a + b * (tau[:, None] - mu[None, :])
    scale = np.abs(ex_p).max()
    assert np.max(np.abs(out["Iplus"][:, 0] - ex_p)) < 1e-11 * scale
    assert np.max(np.abs(out["Iminus"][:, 0] - ex_m)) < 1e-11 * scale
    assert np.max(np.abs(out["H"] - b / 3)) < 1e-11 * scale


def test_flux_conservation_pure_scattering_slab():
    """omega = 1, no thermal source, light incident from above, nothing from
    below: the net flux H is the same at every node."""
    mu, w = gauss_legendre01(6)
    tau = np.concatenate([[0.0], np.logspace(-2, 1.3, 20)]) + 1e-3
    nd = tau.shape[0]
    out = dense.formal_solution_dense(tau, np.ones((nd, 1)), np.zeros(nd), mu, w,
                                      omega=np.ones((nd, 1)), Itop=np.ones((1, 6)), lower="given")
    H = out["H"][:, 0]
    assert np.max(np.abs(H - H.mean())) < 1e-11 * np.abs(H).max()
    assert H.mean() < 0   # net flux downward


def test_sublayer_size_does_not_matter(monkeypatch):
    """The route is exact: a 10x finer starting sublayer (3-4 more doublings)
    gives the same operators to rounding."""
    mu, w = gauss_legendre01(4)
    dl = np.array([0.05, 1.0, 30.0])
    om = np.array([0.5, 0.95, 0.3])
    L1 = dense.layer_operators(dl, om, mu, w)
    monkeypatch.setattr(dense, "_H_NORM", 0.01)
    L2 = dense.layer_operators(dl, om, mu, w)
    for k in ("tp", "rm", "bcp", "bsp", "bsm"):
        assert np.max(np.abs(L1[k] - L2[k])) < 5e-12 * max(1.0, np.abs(L1[k]).max())


@pytest.mark.parametrize("nd,nf,na,seed", [(2, 1, 2, 0), (6, 2, 3, 1), (12, 3, 4, 2)])
def test_dense_lstar_equals_brute_force(nd, nf, na, seed):
    rng = np.random.default_rng(seed)
    tau = np.logspace(-2, 2.5, nd)
    q = rng.lognormal(0, 0.5, size=(nd, nf))
    om = rng.uniform(0.0, 0.99, size=(nd, nf))
    mu, w = gauss_legendre01(na)
    Lm = dense.lambda_matrix_dense(tau, q, om, mu, w)
    S = rng.uniform(0.5, 1.5, size=(nd, nf))
    out = dense.formal_solution_dense(tau, q, S, mu, w, omega=om, lower="given")
    diag = np.stack([np.diag(Lm[k]) for k in range(nf)], axis=1)
    assert np.max(np.abs(out["lstar"] - diag)) < 1e-13
    assert np.max(np.abs(out["lstar_c"] - (1.0 - diag))) < 1e-13
    # linearity: the Lambda matrix reproduces J for zero boundary light
    J = np.einsum("kij,jk->ik", Lm, S)
    assert np.max(np.abs(out["J"] - J)) < 1e-13


def test_dense_reduces_to_diagonal_formal_solution():
    rng = np.random.default_rng(4)
    nd, nf = 15, 4
    tau = np.logspace(-3, 3, nd)
    q = rng.lognormal(0, 0.6, size=(nd, nf))
    S = rng.uniform(0.3, 2.0, size=(nd, nf))
    mu, w = gauss_legendre01(5)
    Bb, Bp = rng.uniform(0.5, 1.5, size=nf), rng.uniform(0.5, 1.5, size=nf)
    o1 = formal.formal_solution(tau, q, S, mu, w, lower="diffusion", Bbot=Bb, Bbot_prev=Bp)
    o2 = dense.formal_solution_dense(tau, q, S, mu, w, omega=np.zeros((nd, nf)), lower="diffusion",
                                     Bbot=Bb, Bbot_prev=Bp)
    for k in ("Iplus", "Iminus", "J", "H", "lstar"):
        assert np.max(np.abs(o1[k] - o2[k])) < 1e-12, k


def test_two_level_with_continuum_ali_fixed_point():
    """ALI with coherent continuum scattering inside the layers (dense formal
    solution, p_k = dS^g_k/dS_l < 1) converges to the direct solution of
    S_l = (1-eps) Jbar[S_l] + eps B built from brute-force Lambda columns."""
    b = W.two_level_batch(nb=1, nd_lo=9, nd_hi=9, na=3, nf=5, seed=1, cont_ratio=0.05,
                          eps_c=1e-2, x_max=3.0).atmosphere(0)
    mu, w = gauss_legendre01(b.na)
    eps = float(b.eps[0])
    kw = {"omega": b.omega}
    r = ali.two_level_ali(b.tau, b.q, b.phi, b.wnu, eps, b.B, mu, w, tol=1e-13, max_iter=5000,
                          pfrac=b.pfrac, sg_const=b.sg_const, fs=dense.formal_solution_dense,
                          fs_kwargs=kw)
    assert r["converged"]
    Lm = dense.lambda_matrix_dense(b.tau, b.q, b.omega, mu, w)     # dJ_k / dS^g_k
    wp = b.wnu * b.phi
    nd, nf = b.q.shape
    Lbar = np.einsum("k,kij,jk->ij", wp, Lm, b.pfrac)               # dJbar / dS_l
    zero = dense.formal_solution_dense(b.tau, b.q, b.sg_const, mu, w, omega=b.omega,
                                       lower="diffusion", Bbot=np.full(nf, b.B[-1]),
                                       Bbot_prev=np.full(nf, b.B[-2]), want_lstar=False)
    J0 = zero["J"] @ wp
    Sd = np.linalg.solve(np.eye(nd) - (1 - eps) * Lbar, (1 - eps) * J0 + eps * b.B)
    assert np.max(np.abs(r["S"] - Sd) / Sd) < 1e-10


def test_dense_lstar_complement_keeps_relative_accuracy():
    """Thick layers: 1 - Lambda* is tiny and must keep its relative accuracy.
    With omega = 0 it equals the short-characteristic complement
    1/2 sum w (psi_above + psi_below) exactly.  With omega > 0 scattering
    keeps a photon longer from thermalising, so the complement grows
    monotonically with omega, and nodes with equal layers on both sides get
    the same value (both computed through the tiny complement itself, not as
    1 minus a number near 1)."""
    mu, w = gauss_legendre01(4)
    tau = np.array([1.0, 2e4, 4e4, 6e4, 8e4])
    nd = tau.shape[0]
    q = np.ones((nd, 1))
    o0 = dense.formal_solution_dense(tau, q, np.ones(nd), mu, w, omega=np.zeros((nd, 1)), lower="given")
    f0 = formal.formal_solution(tau, q, np.ones(nd), mu, w, lower="given")
    assert np.max(np.abs(o0["lstar_c"][1:-1] / f0["lstar_c"][1:-1] - 1)) < 1e-12
    assert f0["lstar_c"][2, 0] < 1e-4
    prev = o0["lstar_c"][1:-1, 0]
    for om in (0.1, 0.5, 0.9, 0.99, 0.9999):
        c = dense.formal_solution_dense(tau, q, np.ones(nd), mu, w, omega=np.full((nd, 1), om),
                                        lower="given")["lstar_c"][1:-1, 0]
        assert np.all(c > prev)
        assert abs(c[2] / c[1] - 1) < 1e-10      # nodes 2 and 3: equal layers (2e4) on both sides
        prev = c

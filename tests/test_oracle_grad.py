"""Pins of the gradient oracle (complex step of the emergent intensity):
the derivative of the formal integral evaluated independently in 40-digit
arithmetic, agreement with central finite differences, Euler's identity for
a loss homogeneous of degree 2 in the source, the uniform-shift identity,
and zero opacity sensitivity when the source is constant."""
import mpmath
import numpy as np
import pytest

from oracle import formal, grad
from oracle.quadrature import gauss_legendre01
from paper_0903_1949_amd import workloads as W


@pytest.fixture(scope="module")
def case():
    return W.gradient_case(nd=40, na=4, nf=16, seed=4)


@pytest.mark.parametrize("lower", ["diffusion", "given"])
def test_emergent_intensity_equals_formal_solution(lower):
    rng = np.random.default_rng(3)
    nd, nf, na = 30, 7, 4
    tau = np.logspace(-4, 4, nd)
    q = rng.lognormal(0, 0.5, size=(nd, nf))
    S = rng.uniform(0.5, 1.5, size=(nd, nf))
    mu, w = gauss_legendre01(na)
    Bb, Bp = S[-1], S[-2] * 0.97
    Ib = rng.uniform(0.5, 1.5, size=(nf, na))
    kw = dict(Bbot=Bb, Bbot_prev=Bp) if lower == "diffusion" else dict(Ibot=Ib)
    ref = formal.formal_solution(tau, q, S, mu, w, lower=lower, **kw)["Iemerg"]
    I = grad.emergent_intensity(tau, q, S, mu, lower=lower, **kw)
    assert np.max(np.abs(I.real - ref)) < 1e-14 * np.abs(ref).max()


def _mp_emergent(tau, q, S, mu, Bb, Bp):
    """I+(top) by 40-digit quadrature of the formal integral with S linear in
    the frequency optical depth between nodes (one frequency, one angle)."""
    t = [mpmath.mpf(0)]
    for d in range(len(tau) - 1):
        t.append(t[-1] + (q[d] + q[d + 1]) / 2 * (mpmath.mpf(tau[d + 1]) - mpmath.mpf(tau[d])))
    m = mpmath.mpf(mu)
    total = mpmath.mpf(0)
    for d in range(len(tau) - 1):
        a, b = t[d], t[d + 1]
        Sa, Sb = S[d], S[d + 1]
        f = lambda x: (Sa + (Sb - Sa) * (x - a) / (b - a)) * mpmath.exp(-x / m) / m
        total += mpmath.quad(f, [a, b])
    Ibot = Bb + m * (Bb - Bp) / (t[-1] - t[-2])
    return total + Ibot * mpmath.exp(-t[-1] / m)


def test_complex_step_equals_high_precision_derivative():
    """dI+/dq_d, dI+/dS_d and the boundary derivatives against mpmath's
    numerical differentiation of the formal integral itself (no layer
    weights involved)."""
    mpmath.mp.dps = 40
    rng = np.random.default_rng(9)
    nd, na = 5, 2
    tau = np.array([1e-3, 0.05, 0.4, 1.5, 4.0])
    q = rng.lognormal(0, 0.5, size=(nd, 1))
    S = rng.uniform(0.5, 1.5, size=(nd, 1))
    Bb, Bp = np.array([1.3]), np.array([1.1])
    mu, _ = gauss_legendre01(na)
    for i in range(na):
        gI = np.zeros((1, na))
        gI[0, i] = 1.0
        cs = grad.vjp_complex_step(tau, q, S, mu, gI, Bbot=Bb, Bbot_prev=Bp)
        qm = [mpmath.mpf(x) for x in q[:, 0]]
        Sm = [mpmath.mpf(x) for x in S[:, 0]]
        for d in range(nd):
            def fq(x, d=d):
                qq = list(qm)
                qq[d] = x
                return _mp_emergent(tau, qq, Sm, mu[i], mpmath.mpf(Bb[0]), mpmath.mpf(Bp[0]))

            def fS(x, d=d):
                SS = list(Sm)
                SS[d] = x
                return _mp_emergent(tau, qm, SS, mu[i], mpmath.mpf(Bb[0]), mpmath.mpf(Bp[0]))
            dq = float(mpmath.diff(fq, qm[d]))
            dS = float(mpmath.diff(fS, Sm[d]))
            assert abs(cs["dq"][d, 0] - dq) <= 1e-13 * max(abs(dq), 1e-3)
            assert abs(cs["dS"][d, 0] - dS) <= 1e-13 * max(abs(dS), 1e-3)
        dBb = float(mpmath.diff(lambda x: _mp_emergent(tau, qm, Sm, mu[i], x, mpmath.mpf(Bp[0])),
                                mpmath.mpf(Bb[0])))
        dBp = float(mpmath.diff(lambda x: _mp_emergent(tau, qm, Sm, mu[i], mpmath.mpf(Bb[0]), x),
                                mpmath.mpf(Bp[0])))
        assert abs(cs["dBbot"][0] - dBb) <= 1e-13 * abs(dBb)
        assert abs(cs["dBbot_prev"][0] - dBp) <= 1e-13 * abs(dBp)


def test_complex_step_agrees_with_central_differences(case):
    g = case
    mu, _ = gauss_legendre01(g.na)
    depths = [0, 3, 12, 20, 27, 39]
    cc, cB = grad.c4_grad_complex_step(g.tau, g.c, g.f, g.B, mu, depths=depths)
    fc, fB = grad.c4_grad_central_fd(g.tau, g.c, g.f, g.B, mu, depths=depths, rel=1e-4)
    scale_c = np.abs(cc).max()
    assert np.max(np.abs(cc - fc)) < 1e-7 * scale_c
    assert np.max(np.abs(cB - fB)) < 1e-7 * np.abs(cB).max()


def test_euler_identity_and_uniform_shift(case):
    """L(lambda B) = lambda^2 L, so sum B dL/dB = 2 L; shifting every B by the
    same amount shifts every I+ by that amount (the weights sum to one and the
    boundary value shifts with B), so sum dL/dB = sum 2 I+."""
    g = case
    mu, _ = gauss_legendre01(g.na)
    _, gB = grad.c4_grad_complex_step(g.tau, g.c, g.f, g.B, mu)
    L = np.sum(grad.c4_loss_per_freq(g.tau, g.c, g.f, g.B, mu).real)
    assert abs(np.sum(g.B * gB) - 2 * L) < 1e-12 * L
    q = g.c[:, None] * g.f[None, :]
    I = grad.emergent_intensity(g.tau, q, g.B, mu, Bbot=g.B[-1], Bbot_prev=g.B[-2]).real
    assert np.allclose(gB.sum(axis=0), 2 * I.sum(axis=1), rtol=1e-12, atol=0)


def test_constant_source_has_no_opacity_sensitivity(case):
    """With S = B = const (and Bbot = Bbot_prev) I+ = B for any opacity."""
    g = case
    mu, _ = gauss_legendre01(g.na)
    B = np.full_like(g.B, 0.7)
    gc, _ = grad.c4_grad_complex_step(g.tau, g.c, g.f, B, mu, depths=[0, 5, 20, 39])
    assert np.max(np.abs(gc)) < 1e-14


def test_given_boundary_adjoint_is_transmission():
    """With the lower boundary given, dI+(top)/dIbot = exp(-t_N / mu) for
    each angle (the whole slab's transmission)."""
    rng = np.random.default_rng(2)
    nd, nf, na = 12, 3, 4
    tau = np.logspace(-3, 1, nd)
    q = rng.lognormal(0, 0.5, size=(nd, nf))
    S = rng.uniform(0.5, 1.5, size=(nd, nf))
    mu, _ = gauss_legendre01(na)
    gI = np.ones((nf, na))
    cs = grad.vjp_complex_step(tau, q, S, mu, gI, lower="given", Ibot=np.ones((nf, na)))
    tN = np.sum(0.5 * (q[1:] + q[:-1]) * np.diff(tau)[:, None], axis=0)
    assert np.allclose(cs["dIbot"], np.exp(-tN[:, None] / mu[None, :]), rtol=1e-13, atol=0)

"""Oracle: gradients of the emergent spectrum.  Test infrastructure only.

The emergent intensity of the omega = 0 formal solution (the up-going sweep
of oracle.formal with linear short characteristics, Sect. 3.2 comparison
calculation) is restated here in complex-safe form and differentiated by the
complex-step method (Squire & Trapp 1998): for a real-analytic f,
df/dx = Im f(x + i h) / h, with no subtractive cancellation, so h = 1e-30
gives the derivative to rounding.  Frequencies are independent, so one
complex step applied to a whole depth row gives the derivative with respect
to that row's entry at every frequency at once.  Central finite differences
in float64 are the second, cruder check.

Nothing here is an adjoint: every derivative is taken of the forward map
directly, one input row at a time.
"""
from __future__ import annotations

import numpy as np


def _weights_complex(delta):
    """(e, alpha, gamma) of the linear short characteristic for complex
    Delta with a positive real part: Taylor series below |Delta| = 0.5 (to
    Delta^21), the closed forms above; both are analytic."""
    d = np.asarray(delta, dtype=np.complex128)
    e = np.exp(-d)
    a = np.empty_like(d)
    g = np.empty_like(d)
    small = np.abs(d) < 0.5
    big = ~small
    if np.any(big):
        db = d[big]
        psi = (1.0 - e[big]) / db
        a[big] = 1.0 - psi
        g[big] = psi - e[big]
    if np.any(small):
        ds = d[small]
        sa = np.zeros_like(ds)
        sg = np.zeros_like(ds)
        power = ds.copy()
        fact = 1.0
        for n in range(1, 22):
            fact *= (n + 1)                   # (n+1)!
            sign = 1.0 if (n % 2) else -1.0   # (-1)^(n+1)
            sa += sign * power / fact
            sg += sign * n * power / fact
            power = power * ds
        a[small] = sa
        g[small] = sg
    return e, a, g


def emergent_intensity(tau, q, S, mu, lower="diffusion", Bbot=None, Bbot_prev=None, Ibot=None):
    """I+ at node 0, [nf, na], for one atmosphere; complex-safe in q, S and
    the boundary data.  lower = "diffusion": I+(nd-1) = Bbot + mu (Bbot -
    Bbot_prev) / dtau_k(last layer); lower = "given": I+(nd-1) = Ibot [nf, na]."""
    tau = np.asarray(tau, dtype=np.float64)
    q = np.asarray(q)
    S = np.asarray(S)
    nd, nf = q.shape
    mu = np.asarray(mu, dtype=np.float64)
    dt = 0.5 * (q[:-1] + q[1:]) * np.diff(tau)[:, None]
    if lower == "diffusion":
        Bb = np.asarray(Bbot)
        Bp = np.asarray(Bbot_prev)
        I = Bb[:, None] + mu[None, :] * ((Bb - Bp) / dt[nd - 2])[:, None]
    else:
        I = np.zeros((nf, mu.shape[0])) if Ibot is None else np.asarray(Ibot)
    for d in range(nd - 2, -1, -1):
        e, a, g = _weights_complex(dt[d][:, None] / mu[None, :])
        I = e * I + a * S[d][:, None] + g * S[d + 1][:, None]
    return I


def vjp_complex_step(tau, q, S, mu, gI, lower="diffusion", Bbot=None, Bbot_prev=None, Ibot=None,
                     depths=None, h=1e-30):
    """Derivatives of phi = sum_{k,i} gI[k,i] I+[k,i](top) with respect to
    q[d, k] and S[d, k] for the listed depth rows (all when None), and to
    the boundary data.  Returns dict(dq [len, nf], dS [len, nf], depths, and
    dBbot, dBbot_prev [nf] or dIbot [nf, na])."""
    q = np.asarray(q, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    nd, nf = q.shape
    gI = np.asarray(gI, dtype=np.float64)
    depths = list(range(nd)) if depths is None else list(depths)
    kw = dict(lower=lower, Bbot=Bbot, Bbot_prev=Bbot_prev, Ibot=Ibot)

    def phi_k(**over):
        args = dict(kw)
        qq = over.pop("q", q)
        SS = over.pop("S", S)
        args.update(over)
        return np.sum(gI * emergent_intensity(tau, qq, SS, mu, **args), axis=1).imag / h

    out = {"depths": np.array(depths), "dq": np.zeros((len(depths), nf)),
           "dS": np.zeros((len(depths), nf))}
    for j, d in enumerate(depths):
        qc = q.astype(np.complex128)
        qc[d] += 1j * h
        out["dq"][j] = phi_k(q=qc)
        Sc = S.astype(np.complex128)
        Sc[d] += 1j * h
        out["dS"][j] = phi_k(S=Sc)
    if lower == "diffusion":
        out["dBbot"] = phi_k(Bbot=np.asarray(Bbot, np.float64) + 1j * h)
        out["dBbot_prev"] = phi_k(Bbot_prev=np.asarray(Bbot_prev, np.float64) + 1j * h)
    else:
        Ib = np.zeros((nf, len(mu))) if Ibot is None else np.asarray(Ibot, np.float64)
        dI = np.zeros_like(Ib)
        for i in range(len(mu)):
            Ic = Ib.astype(np.complex128)
            Ic[:, i] += 1j * h
            res = gI * emergent_intensity(tau, q, S, mu, lower="given", Ibot=Ic)
            dI[:, i] = np.sum(res, axis=1).imag / h
        out["dIbot"] = dI
    return out


# ---------------------------------------------------------------------------
# The emergent-spectrum loss of the gradient workload: q = c_d f_k, S = B,
# diffusion boundary from B's last two rows, L = sum_{k,i} I+_{k,i}(top)^2.

def c4_loss_per_freq(tau, c, f, B, mu):
    """L_k = sum_i I+_{k,i}^2 (complex-safe in c and B)."""
    q = np.asarray(c)[:, None] * np.asarray(f)[None, :]
    I = emergent_intensity(tau, q, B, mu, lower="diffusion", Bbot=B[-1], Bbot_prev=B[-2])
    return np.sum(I * I, axis=1)


def c4_grad_complex_step(tau, c, f, B, mu, depths=None, h=1e-30):
    """dL/dc_d [len] and dL/dB[d, k] [len, nf] at the listed depths, by
    complex steps of c_d and of the row B[d, :] (B enters S and, for its
    last two rows, the boundary condition)."""
    c = np.asarray(c, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    nd, nf = B.shape
    depths = list(range(nd)) if depths is None else list(depths)
    g_c = np.zeros(len(depths))
    g_B = np.zeros((len(depths), nf))
    for j, d in enumerate(depths):
        cc = c.astype(np.complex128)
        cc[d] += 1j * h
        g_c[j] = np.sum(c4_loss_per_freq(tau, cc, f, B, mu).imag) / h
        Bc = B.astype(np.complex128)
        Bc[d] += 1j * h
        g_B[j] = c4_loss_per_freq(tau, c, f, Bc, mu).imag / h
    return g_c, g_B


def c4_grad_central_fd(tau, c, f, B, mu, depths, rel=1e-4):
    """Central differences with step rel * |p| for dL/dc_d and dL/dB[d, k]."""
    c = np.asarray(c, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    nd, nf = B.shape
    L = lambda cc, BB: c4_loss_per_freq(tau, cc, f, BB, mu).real
    g_c = np.zeros(len(depths))
    g_B = np.zeros((len(depths), nf))
    for j, d in enumerate(depths):
        hc = rel * abs(c[d])
        cp, cm = c.copy(), c.copy()
        cp[d] += hc
        cm[d] -= hc
        g_c[j] = (np.sum(L(cp, B)) - np.sum(L(cm, B))) / (2 * hc)
        hB = rel * np.abs(B[d])
        Bp, Bm = B.copy(), B.copy()
        Bp[d] += hB
        Bm[d] -= hB
        g_B[j] = (L(c, Bp) - L(c, Bm)) / (2 * hB)
    return g_c, g_B

"""Oracle: two-level-atom operator splitting (accelerated Lambda iteration)
with the diagonal approximate operator.  Test infrastructure only.

The paper solves the line scattering problem by operator splitting
(Sect. 2; the convergence study of Sect. 3.2.1 compares the local, diagonal
Lambda* with the nearest-neighbour one).  The update used here is the local
operator update of Olson, Auer & Buchler (1986) / Rybicki & Hummer (1991) for
a two-level atom with complete redistribution:

    S_l = (1 - eps) Jbar + eps B,        Jbar = sum_k wnu_k phi_k J_k,

    S_new = S_old + [(1-eps)(Jbar_fs - S_old) + eps (B - S_old)]
                    / [eps + (1-eps)(1 - Lbar*)]

where Jbar_fs comes from a formal solution with S_old and
1 - Lbar* = sum_k wnu_k phi_k [(1 - p_k) + p_k (1 - Lambda*_k)],
p_k = dS^g_k / dS_l (1 for a pure line).  Both sides of the update are
written as differences so that no term is a small difference of large ones.
The iteration starts at S = B and stops when the maximum relative change
max_d |S_new - S_old| / |S_new| falls below tol (the paper's stopping rule,
Sect. 3.2.1, applied to S).

Non-local operator (Sect. 3.2.1 compares the local Lambda* with a
nearest-neighbour one, which in 1D is the tri-diagonal band of Lambda).  With
the profile-averaged band Lbar* = sum_k wnu_k phi_k tri(Lambda_k), the update
solves, per atmosphere,

    [I - (1-eps) Lbar*] dS = (1-eps)(Jbar_fs - S_old) + eps (B - S_old),

whose diagonal is eps + (1-eps)(1 - Lbar*_dd).  The band is read off the
brute-force Lambda matrix (its definition), and the system is solved densely.

Ng acceleration (Ng 1974, in the form given by Auer 1987): from the last four
iterates x0 (newest), x1, x2, x3 and the differences d0 = x0 - x1,
d1 = x1 - x2, d2 = x2 - x3, the coefficients a, b minimise the weighted norm
of d0 - a (d0 - d1) - b (d0 - d2) with weights 1/x0^2, and the accelerated
iterate is (1 - a - b) x0 + a x1 + b x2.  The paper gives no schedule (it
defers the method to its Paper I).  Extrapolation assumes the errors already
decay geometrically, so here it starts once an un-accelerated step changes S
by less than NG_START (maximum relative change): that step's old and new
iterates open the first group.  From then on it is applied whenever four
iterates have accumulated, and the accelerated iterate starts the next group.
(Applied from the very first iterates it stalls on some thick atmospheres
with a small eps, for the diagonal and the tri-diagonal operator alike.)
"""
from __future__ import annotations

import numpy as np

from . import formal

NG_START = 1e-2


def _sg(S_l, pfrac, sg_const, nf):
    S_l = np.asarray(S_l, dtype=np.float64)
    if pfrac is None:
        return np.broadcast_to(S_l[:, None], (S_l.shape[0], nf))
    return pfrac * S_l[:, None] + sg_const


def profile_moments(out, S_l, Sg, phi, wnu, pfrac=None):
    """(Jbar - S_l, 1 - Lbar*) per depth from one formal solution."""
    wp = np.asarray(wnu) * np.asarray(phi)
    jms = out["JmS"]                                      # J_k - S^g_k
    if pfrac is None:
        jbar_m_s = jms @ wp
        one_m_lbar = out["lstar_c"] @ wp
    else:
        jbar_m_s = (jms + (Sg - S_l[:, None])) @ wp
        one_m_lbar = ((1.0 - pfrac) + pfrac * out["lstar_c"]) @ wp
    return jbar_m_s, one_m_lbar


def two_level_ali(tau, q, phi, wnu, eps, B, mu, w, tol=1e-8, max_iter=20000,
                  S0=None, pfrac=None, sg_const=None, fs=None, fs_kwargs=None):
    """Converge the line source function of one atmosphere.

    tau [nd], q [nd, nf], phi/wnu [nf], eps scalar, B [nd].  ``fs`` is the
    formal solution callable (default: the omega = 0 one); it receives
    (tau, q, S^g, mu, w, lower="diffusion", Bbot, Bbot_prev, **fs_kwargs).

    Returns dict(S, iterations, max_rel history, converged)."""
    fs = fs or formal.formal_solution
    fs_kwargs = fs_kwargs or {}
    nd, nf = np.asarray(q).shape
    B = np.asarray(B, dtype=np.float64)
    S = B.copy() if S0 is None else np.asarray(S0, dtype=np.float64).copy()
    Bbot = np.full(nf, B[-1])
    Bprev = np.full(nf, B[-2])
    hist = []
    converged = False
    it = 0
    for it in range(1, max_iter + 1):
        Sg = _sg(S, pfrac, sg_const, nf)
        out = fs(tau, q, Sg, mu, w, lower="diffusion", Bbot=Bbot, Bbot_prev=Bprev, **fs_kwargs)
        jms, olb = profile_moments(out, S, Sg, phi, wnu, pfrac)
        dS = ((1.0 - eps) * jms + eps * (B - S)) / (eps + (1.0 - eps) * olb)
        S_new = S + dS
        rel = float(np.max(np.abs(dS) / np.abs(S_new)))
        hist.append(rel)
        S = S_new
        if rel < tol:
            converged = True
            break
    return {"S": S, "iterations": it, "max_rel": np.array(hist), "converged": converged}


def direct_fixed_point(tau, q, phi, wnu, eps, B, mu, w):
    """The ALI's fixed point by a dense direct solve (pure line, omega = 0):
    S* = (I - (1-eps) Lbar)^-1 [(1-eps) Jbar_bc + eps B], where Lbar is the
    profile-averaged brute-force Lambda matrix and Jbar_bc the profile-averaged
    J of a formal solution with S = 0 and the real boundary conditions."""
    q = np.asarray(q, dtype=np.float64)
    nd, nf = q.shape
    B = np.asarray(B, dtype=np.float64)
    wp = np.asarray(wnu) * np.asarray(phi)
    L = formal.lambda_matrix(tau, q, mu, w)                # [nf, nd, nd]
    Lbar = np.einsum("k,kij->ij", wp, L)
    bc = formal.formal_solution(tau, q, np.zeros((nd, nf)), mu, w, lower="diffusion",
                                Bbot=np.full(nf, B[-1]), Bbot_prev=np.full(nf, B[-2]))
    Jbc = bc["J"] @ wp
    A = np.eye(nd) - (1.0 - eps) * Lbar
    return np.linalg.solve(A, (1.0 - eps) * Jbc + eps * B)


def batch_two_level_update(nd, S, B, eps, jbar_m_s, one_m_lbar):
    """One ALI update for a ragged batch, given the profile moments per node.
    Returns (S_new [sum nd], max_rel [nb])."""
    nd = np.asarray(nd)
    off = np.concatenate([[0], np.cumsum(nd)]).astype(np.int64)
    epsn = np.repeat(np.asarray(eps, dtype=np.float64), nd)
    dS = ((1.0 - epsn) * jbar_m_s + epsn * (B - S)) / (epsn + (1.0 - epsn) * one_m_lbar)
    S_new = S + dS
    rel = np.abs(dS) / np.abs(S_new)
    mx = np.array([rel[off[b]:off[b + 1]].max() for b in range(nd.shape[0])])
    return S_new, mx


def lambda_band(tau, q, mu, w):
    """Tri-diagonal band of the brute-force Lambda operator per frequency:
    (sub, diag, sup), each [nd, nf], sub[d] = Lambda[d, d-1] (0 at d = 0),
    sup[d] = Lambda[d, d+1] (0 at the last node)."""
    L = formal.lambda_matrix(tau, q, mu, w)          # [nf, nd, nd]
    nf, nd, _ = L.shape
    sub = np.zeros((nd, nf))
    sup = np.zeros((nd, nf))
    idx = np.arange(nd)
    diag = L[:, idx, idx].T.copy()
    sub[1:] = L[:, idx[1:], idx[:-1]].T
    sup[:-1] = L[:, idx[:-1], idx[1:]].T
    return sub, diag, sup


def ng_extrapolate(x0, x1, x2, x3):
    """Ng acceleration from four iterates (x0 newest); weights 1/x0^2."""
    d0, d1, d2 = x0 - x1, x1 - x2, x2 - x3
    wt = 1.0 / (x0 * x0)
    u = d0 - d1
    v = d0 - d2
    A = np.array([[np.sum(wt * u * u), np.sum(wt * u * v)],
                  [np.sum(wt * u * v), np.sum(wt * v * v)]])
    rhs = np.array([np.sum(wt * d0 * u), np.sum(wt * d0 * v)])
    det = A[0, 0] * A[1, 1] - A[0, 1] * A[1, 0]
    if det == 0.0 or not np.isfinite(det):
        return x0.copy()
    a, b = np.linalg.solve(A, rhs)
    return (1.0 - a - b) * x0 + a * x1 + b * x2


def two_level_ali_nonlocal(tau, q, phi, wnu, eps, B, mu, w, tol=1e-8, max_iter=20000,
                           operator="tri", ng=False, S0=None):
    """Pure-line two-level ALI (omega = 0) with the diagonal ("diag") or the
    tri-diagonal ("tri") approximate operator, optionally Ng-accelerated.
    Returns dict(S, iterations, max_rel history, converged)."""
    q = np.asarray(q, dtype=np.float64)
    nd, nf = q.shape
    B = np.asarray(B, dtype=np.float64)
    wp = np.asarray(wnu) * np.asarray(phi)
    sub, diag, sup = lambda_band(tau, q, mu, w)
    Lsub, Lsup = sub @ wp, sup @ wp
    S = B.copy() if S0 is None else np.asarray(S0, dtype=np.float64).copy()
    Bbot = np.full(nf, B[-1])
    Bprev = np.full(nf, B[-2])
    hist, group = [], None
    converged = False
    it = 0
    for it in range(1, max_iter + 1):
        Sg = np.broadcast_to(S[:, None], (nd, nf))
        out = formal.formal_solution(tau, q, Sg, mu, w, lower="diffusion", Bbot=Bbot, Bbot_prev=Bprev)
        jms, olb = profile_moments(out, S, Sg, phi, wnu)
        rhs = (1.0 - eps) * jms + eps * (B - S)
        A = np.diag(eps + (1.0 - eps) * olb)
        if operator == "tri":
            A -= (1.0 - eps) * (np.diag(Lsub[1:], -1) + np.diag(Lsup[:-1], 1))
        S_new = S + np.linalg.solve(A, rhs)
        if ng:
            if group is None:
                if np.max(np.abs(S_new - S) / np.abs(S_new)) < NG_START:
                    group = [S.copy(), S_new.copy()]
            else:
                group.append(S_new.copy())
                if len(group) == 4:
                    S_new = ng_extrapolate(group[3], group[2], group[1], group[0])
                    group = [S_new.copy()]
        rel = float(np.max(np.abs(S_new - S) / np.abs(S_new)))
        hist.append(rel)
        S = S_new
        if rel < tol:
            converged = True
            break
    return {"S": S, "iterations": it, "max_rel": np.array(hist), "converged": converged}


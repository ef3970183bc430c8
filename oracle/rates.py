"""Oracle: multilevel preconditioned radiative rates and the per-depth
statistical-equilibrium solve.  Test infrastructure only.

Reading of the paper.  The paper's notation names the rate operators
[R_ij], [R_ji], [R*_ij], [R*_ji], [Delta R_ij], [Delta R_ji] and a rate
matrix A alongside J-bar and Lambda* (its preamble), and solves the
scattering problem by operator splitting (Sect. 2).  The reading taken here
is the full preconditioning of Rybicki & Hummer (1991) with the diagonal
Lambda*: for a transition t = (l < u) and a frequency k of its window,

    chi_t = (n_l - n_u G_k) sigma_k,  eta_t = n_u U_k,  U_k = b_k G_k sigma_k,
    kappa_k = chi_t + kappa_c,        p_k = chi_t / kappa_k,
    dJ_k    = J_k - Lambda*_k p_k S_t = J_k - Lambda*_k eta_t / kappa_k   (old populations)

    [dR_lu] = sum_k W_k sigma_k dJ_k
    [dR_ul] = sum_k W_k G_k sigma_k dJ_k
    [R*_ul] = sum_k W_k U_k (1 - p_k Lambda*_k)

and the new populations solve, at every depth,

    sum_{j != i} n_j P_ji - n_i sum_{j != i} P_ij = 0   (i != 0),   sum_i n_i = n_tot,
    P_lu = [dR_lu] + C_lu,   P_ul = [R*_ul] + [dR_ul] + C_ul,

(the ground-level equation replaced by number conservation), by LU with
partial pivoting in float64, for the unknowns n_i / n_i^old (the columns
scaled by the previous populations, which spans far fewer decades).  The net radiative rate is linear in the new
populations because chi_t^new p S_t^new = p eta_t^new.  W_k is the
frequency-integration weight of a rate (w_k / nu_k in reduced units).

Depth-dependent line profiles (when the atom carries line_nu0, line_s,
line_a and dopp): for a frequency k in the window of line t and depth d,
sigma_{d,k} = s_t H(a_t, x) / (sqrt(pi) dnu_D), dnu_D = nu0_t dopp_d,
x = (nu_k - nu0_t) / dnu_D, with the Voigt function H(a, x) = Re w(x + i a)
taken from the Faddeeva function of scipy (a library step); continua keep
their depth-independent cross-sections.

The formal solution that supplies J and Lambda* is the omega > 0 oracle
(continuum scattering inside the layers), with q = kappa + sigma_c per unit
reference optical depth, omega = sigma_c / q and S^g = (eta_t + kappa_c B)/kappa.
"""
from __future__ import annotations

import numpy as np

from scipy.special import wofz

from . import dense, formal


def voigt_H(a, x):
    """H(a, x) = Re w(x + i a) (Faddeeva function)."""
    return np.real(wofz(np.asarray(x) + 1j * np.asarray(a)))


def cross_sections(atom):
    """sigma [rows, nf]: per frequency, or depth-dependent Voigt lines."""
    rows = atom.tau.shape[0]
    sig = np.broadcast_to(atom.sigma[None, :], (rows, atom.nf)).copy()
    if getattr(atom, "line_a", None) is None:
        return sig
    for t in range(atom.nt):
        if atom.line_nu0[t] <= 0.0:
            continue
        sl = slice(int(atom.k0[t]), int(atom.k1[t]))
        dnu = atom.line_nu0[t] * atom.dopp[:, None]
        x = (atom.nu[None, sl] - atom.line_nu0[t]) / dnu
        sig[:, sl] = atom.line_s[t] * voigt_H(atom.line_a[t], x) / (np.sqrt(np.pi) * dnu)
    return sig


def opacities(atom, pops):
    """Per (row, frequency): q, omega, S^g and the owning transition's chi,
    eta and the absorptive opacity kappa, from populations [rows, nl]."""
    t = atom.owner
    nl_ = pops[:, atom.lo[t]]
    nu_ = pops[:, atom.up[t]]
    G = atom.Gst
    sig = cross_sections(atom)
    chi_t = (nl_ - nu_ * G) * sig
    eta_t = nu_ * atom.bfac[None, :] * G * sig
    kappa = chi_t + atom.kc[:, None]
    q = kappa + atom.sc[:, None]
    return {"q": q, "omega": atom.sc[:, None] / q, "Sg": (eta_t + atom.kc[:, None] * atom.Bnu) / kappa,
            "chi_t": chi_t, "eta_t": eta_t, "kappa": kappa}


def preconditioned_rates(atom, pops_old, J, lstar):
    """[dR_lu], [dR_ul], [R*_ul] per (row, transition)."""
    o = opacities(atom, pops_old)
    p = o["chi_t"] / o["kappa"]
    dJ = J - lstar * o["eta_t"] / o["kappa"]
    Wk = atom.W[None, :]
    sig = cross_sections(atom)
    G = atom.Gst
    U = atom.bfac[None, :] * G * sig
    rows = pops_old.shape[0]
    dRlu = np.zeros((rows, atom.nt))
    dRul = np.zeros((rows, atom.nt))
    Rsul = np.zeros((rows, atom.nt))
    for t in range(atom.nt):
        sl = slice(int(atom.k0[t]), int(atom.k1[t]))
        dRlu[:, t] = np.sum(Wk[:, sl] * sig[:, sl] * dJ[:, sl], axis=1)
        dRul[:, t] = np.sum(Wk[:, sl] * G[:, sl] * sig[:, sl] * dJ[:, sl], axis=1)
        Rsul[:, t] = np.sum(Wk[:, sl] * U[:, sl] * (1.0 - p[:, sl] * lstar[:, sl]), axis=1)
    return dRlu, dRul, Rsul


def rate_matrix(atom, r, dRlu, dRul, Rsul):
    """The statistical-equilibrium matrix A and right-hand side at row r
    (ground-level row replaced by number conservation)."""
    nl = atom.nl
    P = np.zeros((nl, nl))             # P[i, j]: rate from i to j
    for t in range(atom.nt):
        l, u = int(atom.lo[t]), int(atom.up[t])
        P[l, u] += dRlu[r, t] + atom.Clu[r, t]
        P[u, l] += Rsul[r, t] + dRul[r, t] + atom.Cul[r, t]
    A = P.T.copy()                      # A[i, j] = P[j, i] for j != i
    np.fill_diagonal(A, 0.0)
    A[np.arange(nl), np.arange(nl)] = -P.sum(axis=1) + np.diag(P)
    A[0, :] = 1.0
    rhs = np.zeros(nl)
    rhs[0] = atom.ntot[r]
    return A, rhs


def solve_populations(atom, dRlu, dRul, Rsul, scale=None):
    """New populations per row.  The unknowns span many decades, so the
    system is solved for n_i / scale_i (columns scaled by `scale`, e.g. the
    previous populations) and scaled back; the solution is the same."""
    rows = dRlu.shape[0]
    pops = np.zeros((rows, atom.nl))
    for r in range(rows):
        A, rhs = rate_matrix(atom, r, dRlu, dRul, Rsul)
        s = np.ones(atom.nl) if scale is None else scale[r]
        pops[r] = np.linalg.solve(A * s[None, :], rhs) * s
    return pops


def formal_solution_atom(atom, pops, mu, w, scattering=True):
    """J and Lambda* (and the rest) of every atmosphere for given populations."""
    o = opacities(atom, pops)
    off = atom.off
    outs = []
    for b in range(atom.nb):
        s = slice(int(off[b]), int(off[b + 1]))
        kw = dict(lower="diffusion", Bbot=atom.Bnu[s][-1], Bbot_prev=atom.Bnu[s][-2])
        if scattering:
            outs.append(dense.formal_solution_dense(atom.tau[s], o["q"][s], o["Sg"][s], mu, w,
                                                    omega=o["omega"][s], **kw))
        else:
            outs.append(formal.formal_solution(atom.tau[s], o["q"][s], o["Sg"][s], mu, w, **kw))
    res = {k: np.concatenate([x[k] for x in outs]) for k in ("J", "lstar", "lstar_c", "JmS")}
    return res, o


def nlte_iteration(atom, pops, mu, w, scattering=True):
    fs, _ = formal_solution_atom(atom, pops, mu, w, scattering)
    dRlu, dRul, Rsul = preconditioned_rates(atom, pops, fs["J"], fs["lstar"])
    new = solve_populations(atom, dRlu, dRul, Rsul, scale=pops)
    rel = np.abs(new - pops) / np.abs(new)
    off = atom.off
    mx = np.array([rel[off[b]:off[b + 1]].max() for b in range(atom.nb)])
    return new, mx, {"dRlu": dRlu, "dRul": dRul, "Rsul": Rsul, "J": fs["J"], "lstar": fs["lstar"]}


def nlte_solve(atom, mu, w, tol=1e-8, max_iter=500, scattering=True, pops0=None):
    """Iterate from LTE until the maximum relative change of every population
    falls below tol."""
    pops = atom.nstar.copy() if pops0 is None else pops0.copy()
    hist = []
    it = 0
    for it in range(1, max_iter + 1):
        pops, mx, _ = nlte_iteration(atom, pops, mu, w, scattering)
        hist.append(float(mx.max()))
        if hist[-1] < tol:
            break
    return {"pops": pops, "iterations": it, "max_rel": np.array(hist), "converged": hist[-1] < tol}


def net_rate_residual(atom, pops, J):
    """Statistical-equilibrium residual with the plain (unpreconditioned)
    radiative rates of the given J: max over rows and levels of
    |sum in - sum out| / (sum in + sum out)."""
    Wk = atom.W[None, :]
    sig = cross_sections(atom)
    G = atom.Gst
    U = atom.bfac[None, :] * G * sig
    worst = 0.0
    for r in range(pops.shape[0]):
        flow_in = np.zeros(atom.nl)
        flow_out = np.zeros(atom.nl)
        for t in range(atom.nt):
            sl = slice(int(atom.k0[t]), int(atom.k1[t]))
            l, u = int(atom.lo[t]), int(atom.up[t])
            Rlu = np.sum(Wk[0, sl] * sig[r, sl] * J[r, sl])
            Rul = np.sum(Wk[0, sl] * (U[r, sl] + G[r, sl] * sig[r, sl] * J[r, sl]))
            up_flow = pops[r, l] * (Rlu + atom.Clu[r, t])
            down_flow = pops[r, u] * (Rul + atom.Cul[r, t])
            flow_out[l] += up_flow; flow_in[u] += up_flow
            flow_out[u] += down_flow; flow_in[l] += down_flow
        worst = max(worst, float(np.max(np.abs(flow_in - flow_out) / (flow_in + flow_out))))
    return worst

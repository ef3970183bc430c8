"""Oracle: formal solution in 1D spherical symmetry along impact-parameter
rays, and the two-level operator splitting on it.  Test infrastructure only.

The paper's 1D comparison calculations are spherical (Sect. 3.1), its
subject is radiative transfer in spherical coordinates (Sect. 3), and its
line tests iterate the two-level atom with operator splitting (Sect. 3.2.2).
The reading taken here (the formal-solution details are deferred to the
paper's Papers I-II, Sect. 2):

* Shells r_0 > r_1 > ... > r_{nd-1} = R_core (node 0 outermost).  The
  reference optical depth tau (increasing inward) fixes the reference
  opacity per shell, chi_ref = (tau_{d+1} - tau_d) / (r_d - r_{d+1}); the
  monochromatic opacity is q_k chi_ref, q_k linear between the two nodes.
* Rays of impact parameter p: nc core rays with mu_core = 1 - c/nc
  (c = 0..nc-1, so p = 0 is one of them) that end on the core, and one
  tangent ray p = r_m for every shell m (m = nd-1 is tangent to the core,
  m = 0 has zero length).  Along a ray z = sqrt(r^2 - p^2); between the
  shells d and d+1 the optical path is dtau_k = (q_k(d) + q_k(d+1))/2 chi_ref
  (z_d - z_{d+1}), and the source is linear in it (linear short
  characteristics, the same layer weights as in plane-parallel geometry).
  The path is evaluated as dtau_ref,d (r_d + r_{d+1}) / (z_d + z_{d+1}), the
  same number without the cancellation of z_d - z_{d+1} in thin shells (a
  log-tau radial grid with constant reference opacity makes the outer shells
  ~1e-12 of the radius thick).
* Inward intensity from I_top at shell 0; on a tangent ray the outward
  intensity starts at the tangent point with the inward value; on a core
  ray the outward intensity starts on the core with the diffusion value
  B + mu_core (B - B_prev) / dtau_k of the last radial layer (mu_core = z/R).
* At shell d the rays crossing it give mu_dj = z_dj / r_d from 1 (p = 0)
  down to 0 (its own tangent ray); the angle moments use trapezoid weights
  in mu over those points (they sum to one):
      J = 1/2 sum w (I_out + I_in),   H = 1/2 sum w mu (I_out - I_in),
  J - S from the same recursion on D = I - S.
* Lambda*_dd = dJ(d)/dS(d) exactly: the local alpha weights in both
  directions (at a tangent point the outward intensity is the inward one),
  plus, on a tangent ray, the path back through the tangent point: S(d)
  enters the inward intensity at d and below it, which returns attenuated by
  the round trip, so the outward intensity at d (d < m) also gains
      e_d E_{d+1}^2 gamma_d + E_d^2 alpha_{d-1},   E_d = prod_{i=d}^{m-1} e_i
  (segment d joins shells d and d+1; alpha_{-1} = 0).
"""
from __future__ import annotations

import numpy as np

from . import formal


def rays(r, nc):
    """Impact parameters (ascending): nc core rays, then tangent rays
    p = r_{nd-1}, ..., r_0.  Returns p [nrays] and, per ray, the innermost
    shell it reaches (nd-1 for core rays)."""
    r = np.asarray(r, dtype=np.float64)
    nd = r.shape[0]
    Rc = r[-1]
    mu_c = 1.0 - np.arange(nc) / nc
    p_core = Rc * np.sqrt(np.maximum(0.0, 1.0 - mu_c * mu_c))
    p = np.concatenate([p_core, r[::-1]])
    inner = np.concatenate([np.full(nc, nd - 1), np.arange(nd - 1, -1, -1)])
    return p, inner


def mu_weights(r, p, inner):
    """mu [nd, nrays] (NaN where a ray misses the shell) and trapezoid
    weights w [nd, nrays] in mu over the rays crossing each shell."""
    r = np.asarray(r, dtype=np.float64)
    nd, nr = r.shape[0], p.shape[0]
    mu = np.full((nd, nr), np.nan)
    w = np.zeros((nd, nr))
    for d in range(nd):
        hit = np.where(inner >= d)[0]                       # rays with p <= r_d
        m = np.sqrt(np.maximum(0.0, 1.0 - (p[hit] / r[d]) ** 2))
        m[p[hit] == r[d]] = 0.0
        mu[d, hit] = m
        order = np.argsort(-m)                              # mu descending (p ascending)
        ms = m[order]
        ww = np.zeros_like(ms)
        if ms.shape[0] > 1:
            dm = ms[:-1] - ms[1:]
            ww[:-1] += 0.5 * dm
            ww[1:] += 0.5 * dm
        w[d, hit[order]] = ww
    return mu, w


def formal_solution_sph(r, tau, q, S, nc, lower="diffusion", Bbot=None, Bbot_prev=None,
                        Itop=None):
    """One spherical atmosphere.  r, tau [nd]; q, S [nd, nf] (S may be [nd]);
    Itop [nf] isotropic incident intensity (None = 0).
    Returns dict(J, JmS, H, lstar, lstar_c [nd, nf], Iemerg [nf, nrays] at
    shell 0 (outward), p, mu, w)."""
    r = np.asarray(r, dtype=np.float64)
    tau = np.asarray(tau, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    nd, nf = q.shape
    S = np.asarray(S, dtype=np.float64)
    if S.ndim == 1:
        S = np.repeat(S[:, None], nf, axis=1)
    p, inner = rays(r, nc)
    mu, w = mu_weights(r, p, inner)
    Itop = np.zeros(nf) if Itop is None else np.asarray(Itop, dtype=np.float64)
    J = np.zeros((nd, nf)); JmS = np.zeros((nd, nf)); H = np.zeros((nd, nf))
    lam = np.zeros((nd, nf)); lamc = np.zeros((nd, nf))
    Iem = np.zeros((nf, p.shape[0]))
    dt_last = 0.5 * (q[-2] + q[-1]) * (tau[-1] - tau[-2])   # radial, for the diffusion value
    for j in range(p.shape[0]):
        m = int(inner[j])
        z = np.sqrt(np.maximum(0.0, (r[: m + 1] - p[j]) * (r[: m + 1] + p[j])))
        if p[j] == r[m]:
            z[m] = 0.0
        if m == 0:                                          # zero-length ray at the outer shell
            wj = 0.5 * w[0, j]
            J[0] += wj * 2 * Itop
            JmS[0] += wj * 2 * (Itop - S[0])
            lamc[0] += wj * 2
            Iem[:, j] = Itop
            continue
        # chi_ref (z_d - z_{d+1}) = dtau_ref,d (r_d + r_{d+1}) / (z_d + z_{d+1}), since
        # z_d^2 - z_{d+1}^2 = r_d^2 - r_{d+1}^2: the same path, free of the
        # cancellation of thin shells
        path = np.diff(tau)[:m] * (r[:m] + r[1 : m + 1]) / (z[:m] + z[1 : m + 1])
        dtau = 0.5 * (q[:m] + q[1 : m + 1]) * path[:, None]
        e, psi, al, ga = formal.short_char_weights(dtau)
        Iin = np.zeros((m + 1, nf)); Din = np.zeros((m + 1, nf))
        ain = np.zeros((m + 1, nf)); pin = np.zeros((m + 1, nf))   # d I_in(d) / d S(d), and 1 - it
        Iin[0] = Itop; Din[0] = Itop - S[0]; pin[0] = 1.0
        for d in range(m):
            Iin[d + 1] = e[d] * Iin[d] + al[d] * S[d + 1] + ga[d] * S[d]
            Din[d + 1] = e[d] * Din[d] + psi[d] * (S[d] - S[d + 1])
            ain[d + 1] = al[d]
            pin[d + 1] = psi[d]
        Iout = np.zeros((m + 1, nf)); Dout = np.zeros((m + 1, nf))
        aout = np.zeros((m + 1, nf)); pout = np.zeros((m + 1, nf))
        if inner[j] == nd - 1 and p[j] < r[-1]:             # core ray
            muc = z[m] / r[m]
            if lower == "diffusion":
                Iout[m] = Bbot + muc * (Bbot - Bbot_prev) / dt_last
            else:
                Iout[m] = Bbot
            Dout[m] = Iout[m] - S[m]
            aout[m] = 0.0
            pout[m] = 1.0
        else:                                               # turns at its tangent point
            Iout[m] = Iin[m]; Dout[m] = Din[m]; aout[m] = ain[m]; pout[m] = pin[m]
        # round-trip coupling of a tangent ray (see the module notes)
        extra = np.zeros((m + 1, nf))
        if not (inner[j] == nd - 1 and p[j] < r[-1]):
            E = np.ones((m + 1, nf))                        # E[d] = prod_{i=d}^{m-1} e_i
            for d in range(m - 1, -1, -1):
                E[d] = e[d] * E[d + 1]
            for d in range(m):
                a_prev = al[d - 1] if d > 0 else 0.0
                extra[d] = e[d] * E[d + 1] ** 2 * ga[d] + E[d] ** 2 * a_prev
        for d in range(m - 1, -1, -1):
            Iout[d] = e[d] * Iout[d + 1] + al[d] * S[d] + ga[d] * S[d + 1]
            Dout[d] = e[d] * Dout[d + 1] + psi[d] * (S[d + 1] - S[d])
            aout[d] = al[d]
            pout[d] = psi[d]
        wj = 0.5 * w[: m + 1, j][:, None]
        muj = mu[: m + 1, j][:, None]
        J[: m + 1] += wj * (Iout + Iin)
        JmS[: m + 1] += wj * (Dout + Din)
        H[: m + 1] += wj * muj * (Iout - Iin)
        lam[: m + 1] += wj * (aout + ain + extra)
        lamc[: m + 1] += wj * (pout + pin - extra)
        Iem[:, j] = Iout[0]
    return {"J": J, "JmS": JmS, "H": H, "lstar": lam, "lstar_c": lamc, "Iemerg": Iem,
            "p": p, "mu": mu, "w": w}


def lambda_matrix_sph(r, tau, q, nc):
    """Brute-force Lambda [nf, nd, nd]: column d' is J for S = unit at d'
    with zero incident and core intensities."""
    q = np.asarray(q, dtype=np.float64)
    nd, nf = q.shape
    L = np.zeros((nf, nd, nd))
    for dp in range(nd):
        S = np.zeros((nd, nf))
        S[dp] = 1.0
        out = formal_solution_sph(r, tau, q, S, nc, lower="given", Bbot=np.zeros(nf))
        L[:, :, dp] = out["J"].T
    return L


def two_level_ali_sph(r, tau, q, phi, wnu, eps, B, nc, tol=1e-8, max_iter=20000, S0=None):
    """Pure-line two-level ALI (diagonal Lambda*) on one spherical atmosphere:
    the update of oracle.ali with the spherical formal solution."""
    from . import ali
    nd, nf = np.asarray(q).shape
    B = np.asarray(B, dtype=np.float64)
    S = B.copy() if S0 is None else np.asarray(S0, dtype=np.float64).copy()
    hist = []
    converged = False
    it = 0
    for it in range(1, max_iter + 1):
        Sg = np.broadcast_to(S[:, None], (nd, nf))
        out = formal_solution_sph(r, tau, q, Sg, nc, Bbot=np.full(nf, B[-1]),
                                  Bbot_prev=np.full(nf, B[-2]))
        jms, olb = ali.profile_moments(out, S, Sg, phi, wnu)
        dS = ((1.0 - eps) * jms + eps * (B - S)) / (eps + (1.0 - eps) * olb)
        S_new = S + dS
        rel = float(np.max(np.abs(dS) / np.abs(S_new)))
        hist.append(rel)
        S = S_new
        if rel < tol:
            converged = True
            break
    return {"S": S, "iterations": it, "max_rel": np.array(hist), "converged": converged}

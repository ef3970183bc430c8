"""Oracle: formal solution of the plane-parallel transfer equation without
scattering inside the layers (omega = 0), its exact Lambda* diagonal and the
brute-force Lambda matrix.  Test infrastructure only.

Definition (standard 1D statement of the formal solution the paper defers to
its Papers I-II, Sect. 2):

* tau is the reference optical depth, increasing inward, node 0 at the top;
  the monochromatic layer optical depth is the trapezoid
  dtau_k(l) = (q_k(d) + q_k(d+1)) / 2 * (tau[d+1] - tau[d]).
* Along a ray with direction cosine mu in (0, 1) the layer's optical path is
  Delta = dtau_k / mu.  With the source S linear in optical depth between the
  two nodes, integrating  mu dI/dtau = I - S  exactly over one layer gives
      I+(d)   = e I+(d+1) + alpha S(d)   + gamma S(d+1)   (up-going ray)
      I-(d+1) = e I-(d)   + alpha S(d+1) + gamma S(d)     (down-going ray)
  with e = exp(-Delta), alpha = 1 - (1-e)/Delta, gamma = (1-e)/Delta - e.
  (Derivation: the layer integral of S(t) e^{-t}, t the path from the exit
  node, split into its constant and linear parts.)
* Boundaries (Sect. 3.1, item 4): I-(top) given (zero in every test of the
  paper); inner boundary either the diffusion approximation
  I+(bottom, mu) = B(ND) + mu (B(ND) - B(ND-1)) / dtau_k(ND-1/2)
  or a given intensity.
* Angle moments with Gauss weights w (sum 1) per hemisphere:
  J = 1/2 sum w (I+ + I-),  H = 1/2 sum w mu (I+ - I-).  J - S and H are
  taken from the same recursion written for D = I - S (algebraically
  identical), which keeps them accurate where they are small.
* Lambda*: the exact diagonal of the discrete Lambda operator,
  Lambda_dd = dJ(d)/dS(d) = 1/2 sum w [alpha(Delta_{d+1/2}) [d<ND] + alpha(Delta_{d-1/2}) [d>1]],
  and its complement 1 - Lambda_dd, formed from 1 - alpha = (1-e)/Delta so
  that it keeps full relative accuracy where Lambda_dd -> 1.
"""
from __future__ import annotations

import numpy as np

_SERIES_MAX = 0.5
_NTERMS = 18


def layer_optical_depths(tau: np.ndarray, q: np.ndarray) -> np.ndarray:
    """Trapezoid layer optical depths, shape [nd-1, nf]."""
    tau = np.asarray(tau, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    return 0.5 * (q[:-1] + q[1:]) * np.diff(tau)[:, None]


def short_char_weights(delta: np.ndarray):
    """(e, psi, alpha, gamma) of one layer of optical path delta > 0.

    psi = (1 - e)/delta, alpha = 1 - psi, gamma = psi - e.  Below delta = 0.5
    the three are summed from their Taylor series (the closed forms cancel
    there):  psi   = sum_{n>=0} (-delta)^n / (n+1)!,
             alpha = sum_{n>=1} (-1)^(n+1) delta^n / (n+1)!,
             gamma = sum_{n>=1} (-1)^(n+1) n delta^n / (n+1)!.
    Eighteen terms leave a truncation below 1e-19."""
    d = np.asarray(delta, dtype=np.float64)
    e = np.exp(-d)
    small = d < _SERIES_MAX
    with np.errstate(divide="ignore", invalid="ignore"):
        psi = np.where(small, 0.0, (1.0 - e) / np.where(small, 1.0, d))
    alpha = 1.0 - psi
    gamma = psi - e
    if np.any(small):
        ds = d[small]
        ps = np.zeros_like(ds)
        al = np.zeros_like(ds)
        ga = np.zeros_like(ds)
        power = np.ones_like(ds)
        fact = 1.0
        for n in range(0, _NTERMS):
            fact *= (n + 1)            # (n+1)!
            sign = -1.0 if (n % 2) else 1.0
            ps += sign * power / fact
            if n >= 1:
                al += -sign * power / fact
                ga += -sign * n * power / fact
            power = power * ds
        psi = psi.copy(); alpha = alpha.copy(); gamma = gamma.copy()
        psi[small] = ps
        alpha[small] = al
        gamma[small] = ga
    return e, psi, alpha, gamma


def formal_solution(tau, q, S, mu, w, Itop=None, lower="diffusion", Bbot=None,
                    Bbot_prev=None, Ibot=None) -> dict:
    """Formal solution of one atmosphere, omega = 0.

    tau [nd]; q [nd, nf]; S [nd, nf] or [nd] (broadcast over frequency);
    mu, w [na]; Itop [nf, na] or None (zero).  lower = "diffusion" uses
    Bbot[nf] = B(ND), Bbot_prev[nf] = B(ND-1); lower = "given" uses Ibot[nf, na]
    (None: zero).

    Returns float64 arrays: Iplus, Iminus [nd, nf, na]; J, JmS, H, lstar,
    lstar_c [nd, nf]; Iemerg [nf, na] (= Iplus at the top)."""
    tau = np.asarray(tau, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    nd, nf = q.shape
    if nd < 2:
        raise ValueError("need at least two depth points")
    S = np.asarray(S, dtype=np.float64)
    if S.ndim == 1:
        S = np.broadcast_to(S[:, None], (nd, nf))
    mu = np.asarray(mu, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    na = mu.shape[0]

    dtau = layer_optical_depths(tau, q)                    # [nd-1, nf]
    delta = dtau[:, :, None] / mu[None, None, :]           # [nd-1, nf, na]
    e, psi, alpha, gamma = short_char_weights(delta)

    Ip = np.zeros((nd, nf, na))
    Im = np.zeros((nd, nf, na))
    if lower == "diffusion":
        Bb = np.asarray(Bbot, dtype=np.float64)
        Bp = np.asarray(Bbot_prev, dtype=np.float64)
        grad = (Bb - Bp) / dtau[nd - 2]                    # dB/dtau_k on the last layer
        Ip[nd - 1] = Bb[:, None] + mu[None, :] * grad[:, None]
    elif lower == "given":
        if Ibot is not None:
            Ip[nd - 1] = np.asarray(Ibot, dtype=np.float64)
    else:
        raise ValueError(f"unknown lower boundary {lower!r}")
    if Itop is not None:
        Im[0] = np.asarray(Itop, dtype=np.float64)

    Sk = S[:, :, None]
    for d in range(nd - 2, -1, -1):                         # up-going rays, bottom -> top
        Ip[d] = e[d] * Ip[d + 1] + alpha[d] * Sk[d] + gamma[d] * Sk[d + 1]
    for d in range(0, nd - 1):                              # down-going rays, top -> bottom
        Im[d + 1] = e[d] * Im[d] + alpha[d] * Sk[d + 1] + gamma[d] * Sk[d]

    J = 0.5 * np.einsum("dki,i->dk", Ip + Im, w)
    # J - S and H also from the same recursion written for D = I - S:
    #   D+(d) = e D+(d+1) + psi (S(d+1) - S(d)),  D-(d+1) = e D-(d) + psi (S(d) - S(d+1))
    # (substitute alpha = 1 - psi, gamma = psi - e above); where J ~ S deep in
    # the atmosphere this keeps the small difference's relative accuracy.
    Dp = np.zeros((nd, nf, na))
    Dm = np.zeros((nd, nf, na))
    Dp[nd - 1] = Ip[nd - 1] - Sk[nd - 1]
    Dm[0] = Im[0] - Sk[0]
    for d in range(nd - 2, -1, -1):
        Dp[d] = e[d] * Dp[d + 1] + psi[d] * (Sk[d + 1] - Sk[d])
    for d in range(0, nd - 1):
        Dm[d + 1] = e[d] * Dm[d] + psi[d] * (Sk[d] - Sk[d + 1])
    JmS = 0.5 * np.einsum("dki,i->dk", Dp + Dm, w)
    H = 0.5 * np.einsum("dki,i->dk", Dp - Dm, w * mu)
    lstar = np.zeros((nd, nf))
    lstar_c = np.zeros((nd, nf))
    half_w = 0.5 * w
    a_below = np.einsum("lki,i->lk", alpha, half_w)         # layer d+1/2 acting on node d
    p_below = np.einsum("lki,i->lk", psi, half_w)
    lstar[:-1] += a_below
    lstar[1:] += a_below
    # complement: each hemisphere contributes 1/2 sum w (1 - alpha) = 1/2 sum w psi
    # where a layer is present and 1/2 sum w where the boundary fixes the intensity
    lstar_c[:-1] += p_below
    lstar_c[1:] += p_below
    lstar_c[0] += 0.5 * np.sum(w)
    lstar_c[nd - 1] += 0.5 * np.sum(w)
    return {
        "Iplus": Ip, "Iminus": Im, "J": J, "JmS": JmS, "H": H,
        "lstar": lstar, "lstar_c": lstar_c, "Iemerg": Ip[0].copy(),
    }


def lambda_matrix(tau, q, mu, w) -> np.ndarray:
    """Brute-force discrete Lambda operator, shape [nf, nd, nd]:
    column d' is J from a formal solution with S = unit vector at node d' and
    zero boundary intensities.  Used to pin Lambda* and the ALI fixed point."""
    q = np.asarray(q, dtype=np.float64)
    nd, nf = q.shape
    L = np.zeros((nf, nd, nd))
    for dp in range(nd):
        S = np.zeros((nd, nf))
        S[dp] = 1.0
        out = formal_solution(tau, q, S, mu, w, lower="given")
        L[:, :, dp] = out["J"].T
    return L


def batch_formal_solution(nd, tau, q, S, mu, w, Bbot=None, Bbot_prev=None, Itop=None):
    """Formal solution of every atmosphere of a ragged batch (diffusion inner
    boundary).  nd [nb]; tau [sum nd]; q, S [sum nd, nf] (S may be [sum nd]);
    Bbot, Bbot_prev [nb, nf]; Itop [nb, nf, na] or None.  Returns the per-node
    outputs concatenated in the same ragged order and Iemerg [nb, nf, na]."""
    nd = np.asarray(nd)
    off = np.concatenate([[0], np.cumsum(nd)]).astype(np.int64)
    outs = []
    for b in range(nd.shape[0]):
        s = slice(int(off[b]), int(off[b + 1]))
        Sb = S[s]
        outs.append(formal_solution(
            tau[s], q[s], Sb, mu, w, Itop=None if Itop is None else Itop[b],
            lower="diffusion", Bbot=Bbot[b], Bbot_prev=Bbot_prev[b]))
    res = {}
    for key in ("Iplus", "Iminus", "J", "JmS", "H", "lstar", "lstar_c"):
        res[key] = np.concatenate([o[key] for o in outs], axis=0)
    res["Iemerg"] = np.stack([o["Iemerg"] for o in outs], axis=0)
    return res


__all__ = [
    "layer_optical_depths", "short_char_weights", "formal_solution", "lambda_matrix",
    "batch_formal_solution",
]

"""Oracle: formal solution with coherent isotropic scattering inside each
layer (omega > 0): exact layer operators t, r, beta of a homogeneous slab,
the adding recursion and the dense diagonal Lambda*.  Test infrastructure only.

Reading of the paper.  The paper names the layer transmission and reflection
matrices t+-, r+- and source vectors beta+- together with the intensity
vectors I+- in its notation, and parameterises coherent isotropic continuum
scattering by a thermalisation parameter (Sect. 3.1, item 6); it defers the
equations to its Papers I-II (Sect. 2).  The reading taken here: each layer
between nodes d and d+1 is homogeneous with single-scattering albedo
omega = (omega(d) + omega(d+1))/2 and carries a non-scattering source S^g
linear in the layer's optical depth; the total source is
S = (1 - omega) S^g + omega J.  The layer equations are

    I+(d)   = t+ I+(d+1) + r- I-(d)   + beta+
    I-(d+1) = t- I-(d)   + r+ I+(d+1) + beta-

(r- reflects down-going light back up, r+ up-going light back down).

Route used here (kept independent of the eigen route of the HIP kernels):
1. the transfer equation of a thin sublayer, dy/dt = K y + (1-omega) c S^g(t),
   y = (I+, I-), is integrated exactly by the exponential of an augmented
   matrix (Van Loan 1978) evaluated by its Taylor series, which converges to
   rounding because the sublayer is chosen with ||h K|| <= 0.1;
2. the transfer form y(h) = Phi y(0) + g is rearranged into t, r, beta;
3. the sublayer is doubled n times with the star product (adding-doubling,
   van de Hulst 1963; Hansen & Travis 1974), carrying the responses to a
   unit constant source and to a unit-slope source, until it reaches the
   layer's thickness.  Every step is exact, so the result is the exact
   discrete-ordinate layer up to rounding.

Adding recursion (top -> bottom), with the composite reflection R_d and
source Sigma_d of everything above node d seen from below
(I-(d) = R_d I+(d) + Sigma_d; R_0 = 0, Sigma_0 = I_top):
    G_d = (I - r- R_d)^-1,  P_d = G_d t+,  u_d = G_d (r- Sigma_d + beta+)
    R_{d+1} = r+ + t- R_d P_d,  Sigma_{d+1} = t- (Sigma_d + R_d u_d) + beta-
and back-substitution I+(d) = P_d I+(d+1) + u_d, I-(d) = R_d I+(d) + Sigma_d
from the lower boundary up.  J - S^g and H come from the same recursion run
on D = I - S^g, whose layer sources are +-(S^g(d+1) - S^g(d)) Q,
Q = beta_l+ + t 1 (exact: a constant S^g is reproduced by every layer).

Lambda*_dd = dJ(d)/dS^g(d): S^g(d) enters beta of the layer above and the
layer below node d.  With the composite reflection R^up_d of everything below
node d (I+(d) = R^up_d I-(d) + Sigma^up_d, from a bottom-up adding pass), the
response at node d is
    dI+(d) = (I - R^up_d R_d)^-1 (R^up_d dSigma_d + dSigma^up_d),
    dI-(d) = R_d dI+(d) + dSigma_d,
    dSigma_d    = t-_a R_{d-1} G_{d-1} dbeta+_a + dbeta-_a     (layer a above),
    dSigma^up_d = t+_b R^up_{d+1} G^up_{d+1} dbeta-_b + dbeta+_b (layer b below),
    G^up_{d+1} = (I - r+_b R^up_{d+1})^-1.
It is pinned against brute-force unit columns of the full Lambda matrix.
"""
from __future__ import annotations

import numpy as np

from .formal import layer_optical_depths

_H_NORM = 0.1      # sublayer size: ||h K|| <= 0.1 keeps the Taylor series to ~20 terms
_NTAYLOR = 24


def _taylor_expm(A):
    """exp(A) for a batch [..., n, n] with ||A|| <= ~0.25 (plain Taylor sum)."""
    n = A.shape[-1]
    out = np.broadcast_to(np.eye(n), A.shape).copy()
    term = out.copy()
    for k in range(1, _NTAYLOR + 1):
        term = term @ A / k
        out = out + term
    return out


def _sublayer(h, omega, mu, w):
    """Exact operators of a thin homogeneous sublayer of thickness h (batch).
    Returns dict of t+, t-, r+, r- [..., na, na] and source responses for
    S^g = 1 (bc+, bc-) and S^g = t (bs+, bs-) [..., na]."""
    na = mu.shape[0]
    Mv = 1.0 / mu
    shp = h.shape
    hb = h[..., None, None]
    om = omega[..., None, None]
    # K for y = (I+, I-):  dI+/dt = M (I+ - S),  dI-/dt = -M (I- - S),
    # homogeneous S = omega/2 w^T (I+ + I-)
    Mm = np.diag(Mv)
    ow = 0.5 * np.outer(Mv, w)          # M 1 w^T / 2
    K = np.zeros(shp + (2 * na, 2 * na))
    K[..., :na, :na] = Mm - om * ow
    K[..., :na, na:] = -om * ow
    K[..., na:, :na] = om * ow
    K[..., na:, na:] = -Mm + om * ow
    c = np.concatenate([-Mv, Mv])       # source direction of S^g
    src = (1.0 - omega)[..., None] * c  # [..., 2na]
    n2 = 2 * na + 2
    res = {}
    for which in ("c", "s"):
        A = np.zeros(shp + (n2, n2))
        A[..., :2 * na, :2 * na] = K
        if which == "c":
            A[..., :2 * na, 2 * na] = src          # driven by s0 = 1
        else:
            A[..., :2 * na, 2 * na + 1] = src      # driven by s1 = t
        A[..., 2 * na + 1, 2 * na] = 1.0           # s1' = s0
        E = _taylor_expm(hb * A)
        Phi = E[..., :2 * na, :2 * na]
        g = E[..., :2 * na, 2 * na]                # response from z(0) = (0, 1, 0)
        res["Phi"] = Phi
        res["g" + which] = g
    Phi = res["Phi"]
    P11, P12 = Phi[..., :na, :na], Phi[..., :na, na:]
    P21, P22 = Phi[..., na:, :na], Phi[..., na:, na:]
    tp = np.linalg.inv(P11)
    rm = -tp @ P12
    rp = P21 @ tp
    tm = P22 - P21 @ tp @ P12
    out = {"tp": tp, "tm": tm, "rp": rp, "rm": rm}
    for which in ("c", "s"):
        g = res["g" + which]
        gp, gm = g[..., :na], g[..., na:]
        bp = -np.einsum("...ij,...j->...i", tp, gp)       # -P11^-1 g+
        bm = gm + np.einsum("...ij,...j->...i", P21, bp)  # g- - P21 P11^-1 g+
        out["b" + which + "p"] = bp
        out["b" + which + "m"] = bm
    return out


def _mv(A, x):
    return np.einsum("...ij,...j->...i", A, x)


def star(A, B):
    """Operators of layer A on top of layer B (Redheffer star product)."""
    na = A["tp"].shape[-1]
    I = np.eye(na)
    G1 = np.linalg.inv(I - A["rp"] @ B["rm"])     # acts on I- at the interface
    G2 = np.linalg.inv(I - B["rm"] @ A["rp"])     # acts on I+ at the interface
    return {
        "tp": A["tp"] @ G2 @ B["tp"],
        "rm": A["rm"] + A["tp"] @ B["rm"] @ G1 @ A["tm"],
        "tm": B["tm"] @ G1 @ A["tm"],
        "rp": B["rp"] + B["tm"] @ G1 @ A["rp"] @ B["tp"],
        "_G1": G1,
    }


def star_source(A, B, Sab, bAp, bAm, bBp, bBm):
    """Source vectors of the star product of A (top) and B (bottom) given the
    layers' own source vectors (Sab = star(A, B) supplies G1)."""
    G1 = Sab["_G1"]
    inner = _mv(G1, _mv(A["rp"], bBp) + bAm)          # I- at the interface minus its
    bp = bAp + _mv(A["tp"], bBp + _mv(B["rm"], inner))
    bm = bBm + _mv(B["tm"], inner)
    return bp, bm


def layer_operators(delta, omega, mu, w):
    """Exact operators of homogeneous layers: delta, omega arrays of equal
    shape (omega in [0, 1]).  Returns dict with tp, tm, rp, rm [..., na, na]
    and the source responses bcp, bcm (unit constant S^g) and bsp, bsm
    (S^g = t, the optical depth below the layer top) [..., na]."""
    delta = np.asarray(delta, dtype=np.float64)
    omega = np.broadcast_to(np.asarray(omega, dtype=np.float64), delta.shape)
    mu = np.asarray(mu, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    knorm = 2.0 / mu.min()
    n = np.maximum(0, np.ceil(np.log2(np.maximum(delta * knorm / _H_NORM, 1e-300)))).astype(int)
    h = delta / (2.0 ** n)
    L = _sublayer(h, omega, mu, w)
    for it in range(int(n.max()) if n.size else 0):
        sel = n > it
        if not np.any(sel):
            break
        A = {k: v[sel] for k, v in L.items()}
        hs = h[sel]
        S = star(A, A)
        bcp, bcm = star_source(A, A, S, A["bcp"], A["bcm"], A["bcp"], A["bcm"])
        # slope source: top half sees t, bottom half sees h + t'
        bsp, bsm = star_source(A, A, S, A["bsp"], A["bsm"],
                               hs[:, None] * A["bcp"] + A["bsp"], hs[:, None] * A["bcm"] + A["bsm"])
        for k, v in (("tp", S["tp"]), ("tm", S["tm"]), ("rp", S["rp"]), ("rm", S["rm"]),
                     ("bcp", bcp), ("bcm", bcm), ("bsp", bsp), ("bsm", bsm)):
            L[k] = L[k].copy()
            L[k][sel] = v
        h = h.copy()
        h[sel] = 2.0 * hs
    return L


def layer_sources(L, delta, S_top, S_bot):
    """beta+- of layers whose S^g runs linearly from S_top to S_bot."""
    slope = (S_bot - S_top) / delta
    bp = S_top[..., None] * L["bcp"] + slope[..., None] * L["bsp"]
    bm = S_top[..., None] * L["bcm"] + slope[..., None] * L["bsm"]
    return bp, bm


def _lower_boundary(nf, na, mu, dtau_last, lower, Bbot, Bbot_prev, Ibot):
    if lower == "diffusion":
        grad = (np.asarray(Bbot) - np.asarray(Bbot_prev)) / dtau_last
        return np.asarray(Bbot)[:, None] + mu[None, :] * grad[:, None]
    if lower == "given":
        return np.zeros((nf, na)) if Ibot is None else np.asarray(Ibot, dtype=np.float64)
    raise ValueError(lower)


def formal_solution_dense(tau, q, S, mu, w, omega=None, Itop=None, lower="diffusion",
                          Bbot=None, Bbot_prev=None, Ibot=None, ops=None, want_lstar=True):
    """Formal solution of one atmosphere with in-layer isotropic scattering.

    tau [nd]; q [nd, nf]; S = S^g [nd, nf] or [nd]; omega [nd, nf] (node
    albedo; None = 0); other arguments as formal.formal_solution.  `ops`
    may carry precomputed layer operators.  Returns the same keys as the
    omega = 0 oracle (J - S means J - S^g) plus the layer operators."""
    tau = np.asarray(tau, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    nd, nf = q.shape
    mu = np.asarray(mu, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    na = mu.shape[0]
    S = np.asarray(S, dtype=np.float64)
    if S.ndim == 1:
        S = np.broadcast_to(S[:, None], (nd, nf))
    om = np.zeros((nd, nf)) if omega is None else np.asarray(omega, dtype=np.float64)
    dtau = layer_optical_depths(tau, q)                        # [L, nf]
    oml = 0.5 * (om[:-1] + om[1:])
    L = ops if ops is not None else layer_operators(dtau, oml, mu, w)
    bp, bm = layer_sources(L, dtau, S[:-1], S[1:])             # [L, nf, na]
    I = np.eye(na)

    # ---- adding recursion, top -> bottom
    R = np.zeros((nd, nf, na, na))
    Sig = np.zeros((nd, nf, na))
    if Itop is not None:
        Sig[0] = Itop
    P = np.zeros((nd - 1, nf, na, na))
    u = np.zeros((nd - 1, nf, na))
    G = np.zeros((nd - 1, nf, na, na))
    for d in range(nd - 1):
        G[d] = np.linalg.inv(I - L["rm"][d] @ R[d])
        P[d] = G[d] @ L["tp"][d]
        u[d] = _mv(G[d], _mv(L["rm"][d], Sig[d]) + bp[d])
        R[d + 1] = L["rp"][d] + L["tm"][d] @ R[d] @ P[d]
        Sig[d + 1] = _mv(L["tm"][d], Sig[d] + _mv(R[d], u[d])) + bm[d]

    # ---- lower boundary and back-substitution, bottom -> top
    Ip = np.zeros((nd, nf, na))
    Im = np.zeros((nd, nf, na))
    Ip[nd - 1] = _lower_boundary(nf, na, mu, dtau[nd - 2], lower, Bbot, Bbot_prev, Ibot)
    Im[nd - 1] = _mv(R[nd - 1], Ip[nd - 1]) + Sig[nd - 1]
    for d in range(nd - 2, -1, -1):
        Ip[d] = _mv(P[d], Ip[d + 1]) + u[d]
        Im[d] = _mv(R[d], Ip[d]) + Sig[d]

    J = 0.5 * np.einsum("dki,i->dk", Ip + Im, w)
    # J - S^g and H in difference form: the same adding recursion carries
    # D = I - S^g, whose layer sources are +- (S^g(d+1) - S^g(d)) Q with
    # Q = beta_l+ + t 1 (a constant S^g reproduces itself exactly:
    # beta_c + t 1 + r 1 = 1), so small J - S^g keeps its relative accuracy.
    Q = L["bsp"] / dtau[..., None] + L["tp"] @ np.ones(na)
    dS = (S[1:] - S[:-1])[..., None]
    Dt = (np.zeros((nf, na)) if Itop is None else np.asarray(Itop)) - S[0][:, None]
    Db = Ip[nd - 1] - S[nd - 1][:, None]
    Dp, Dm = _adding_backsub(L, dS * Q, -dS * Q, Dt, Db)
    JmS = 0.5 * np.einsum("dki,i->dk", Dp + Dm, w)
    H = 0.5 * np.einsum("dki,i->dk", Dp - Dm, w * mu)
    out = {"Iplus": Ip, "Iminus": Im, "J": J, "JmS": JmS, "H": H, "Iemerg": Ip[0].copy(),
           "ops": L}
    if want_lstar:
        lst, lstc = lstar_dense(L, dtau, R, G, mu, w)
        out["lstar"] = lst
        out["lstar_c"] = lstc
    return out


def _adding_backsub(L, bp, bm, top, bottom):
    """Intensities at every node from layer operators, layer sources bp/bm
    [L, nf, na], the incident vector at the top and the up-going vector at
    the bottom (adding down, back-substitution up)."""
    nl, nf, na = bp.shape
    nd = nl + 1
    I = np.eye(na)
    R = np.zeros((nd, nf, na, na))
    Sig = np.zeros((nd, nf, na))
    Sig[0] = top
    P = np.zeros((nl, nf, na, na))
    u = np.zeros((nl, nf, na))
    for d in range(nl):
        G = np.linalg.inv(I - L["rm"][d] @ R[d])
        P[d] = G @ L["tp"][d]
        u[d] = _mv(G, _mv(L["rm"][d], Sig[d]) + bp[d])
        R[d + 1] = L["rp"][d] + L["tm"][d] @ R[d] @ P[d]
        Sig[d + 1] = _mv(L["tm"][d], Sig[d] + _mv(R[d], u[d])) + bm[d]
    Xp = np.zeros((nd, nf, na))
    Xm = np.zeros((nd, nf, na))
    Xp[nd - 1] = bottom
    Xm[nd - 1] = _mv(R[nd - 1], Xp[nd - 1]) + Sig[nd - 1]
    for d in range(nd - 2, -1, -1):
        Xp[d] = _mv(P[d], Xp[d + 1]) + u[d]
        Xm[d] = _mv(R[d], Xp[d]) + Sig[d]
    return Xp, Xm


def lstar_dense(L, dtau, R, G, mu, w):
    """Diagonal Lambda* and its complement 1 - Lambda* from the two-sided
    composites (see module doc).  The complement is the response of
    J - S^g to the same unit change of S^g(d), taken through the
    difference-form sources (+Q on the layer above the node, -Q on the layer
    below, -1 where a boundary fixes the incoming intensity), so it keeps full
    relative accuracy where Lambda* -> 1."""
    nl, nf, na = L["bcp"].shape
    nd = nl + 1
    I = np.eye(na)
    Rup = np.zeros((nd, nf, na, na))
    Gup = np.zeros((nd, nf, na, na))      # Gup[d+1] = (I - r+_b Rup[d+1])^-1 for layer b = (d, d+1)
    for d in range(nd - 2, -1, -1):
        Gup[d + 1] = np.linalg.inv(I - L["rp"][d] @ Rup[d + 1])
        Rup[d] = L["rm"][d] + L["tp"][d] @ Rup[d + 1] @ Gup[d + 1] @ L["tm"][d]
    Q = L["bsp"] / dtau[..., None] + L["tp"] @ np.ones(na)
    lst = np.zeros((nd, nf))
    lstc = np.zeros((nd, nf))
    ones = np.ones((nf, na))
    for d in range(nd):
        dS = np.zeros((nf, na))
        dSu = np.zeros((nf, na))
        eS = -ones if d == 0 else np.zeros((nf, na))          # difference form
        eSu = -ones if d == nd - 1 else np.zeros((nf, na))
        if d > 0:                                  # layer a = (d-1, d): S^g 0 -> 1
            a = d - 1
            inv = 1.0 / dtau[a]
            M = L["tm"][a] @ R[d - 1] @ G[d - 1]
            dS = _mv(M, inv[:, None] * L["bsp"][a]) + inv[:, None] * L["bsm"][a]
            eS = _mv(M, Q[a]) - Q[a]
        if d < nd - 1:                             # layer b = (d, d+1): S^g 1 -> 0
            b = d
            inv = 1.0 / dtau[b]
            dbp = L["bcp"][b] - inv[:, None] * L["bsp"][b]
            dbm = L["bcm"][b] - inv[:, None] * L["bsm"][b]
            M = L["tp"][b] @ Rup[d + 1] @ Gup[d + 1]
            dSu = _mv(M, dbm) + dbp
            eSu = _mv(M, Q[b]) - Q[b]
        A = I - Rup[d] @ R[d]
        dIp = np.linalg.solve(A, (_mv(Rup[d], dS) + dSu)[..., None])[..., 0]
        dIm = _mv(R[d], dIp) + dS
        lst[d] = 0.5 * (dIp + dIm) @ w
        eDp = np.linalg.solve(A, (_mv(Rup[d], eS) + eSu)[..., None])[..., 0]
        eDm = _mv(R[d], eDp) + eS
        lstc[d] = -0.5 * (eDp + eDm) @ w
    return lst, lstc


def lambda_matrix_dense(tau, q, omega, mu, w):
    """Brute-force Lambda (dJ/dS^g), shape [nf, nd, nd], from unit columns
    with zero boundary intensities.  Used to pin lstar_dense."""
    q = np.asarray(q, dtype=np.float64)
    nd, nf = q.shape
    dtau = layer_optical_depths(tau, q)
    om = np.asarray(omega, dtype=np.float64)
    ops = layer_operators(dtau, 0.5 * (om[:-1] + om[1:]), mu, w)
    Lm = np.zeros((nf, nd, nd))
    for dp in range(nd):
        S = np.zeros((nd, nf))
        S[dp] = 1.0
        out = formal_solution_dense(tau, q, S, mu, w, omega=om, lower="given", ops=ops,
                                    want_lstar=False)
        Lm[:, :, dp] = out["J"].T
    return Lm


def chandrasekhar_h(omega, mu, w, tol=1e-15, maxit=100000):
    """Discrete Chandrasekhar H-function for isotropic scattering, by the
    fixed-point iteration H(mu_i) = 1 + mu_i H(mu_i) sum_j (omega/2) w_j H(mu_j)/(mu_i + mu_j)
    written as H = 1 / (1 - mu_i sum_j (omega/2) w_j H_j / (mu_i + mu_j))."""
    mu = np.asarray(mu, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    H = np.ones_like(mu)
    for _ in range(maxit):
        Hn = 1.0 / (1.0 - mu * ((0.5 * omega * w * H)[None, :] / (mu[:, None] + mu[None, :])).sum(1))
        if np.max(np.abs(Hn - H)) < tol:
            return Hn
        H = Hn
    return H


__all__ = ["layer_operators", "layer_sources", "star", "star_source", "formal_solution_dense",
           "lstar_dense", "lambda_matrix_dense", "chandrasekhar_h"]

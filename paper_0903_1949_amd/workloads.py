"""Seeded synthetic atmospheres for the plane-parallel formal solution.

This module only *describes inputs*: depth grids, opacity ratios, line
profiles, frequency weights, thermalisation parameters and trial source
functions.  It holds none of the transfer arithmetic (no layer optical depths,
no exponentials, no quadrature over angle), so both the CPU oracle and the
HIP path can be fed from it without sharing any of the method.

The physical set-up follows the paper's test environment (Sect. 3.1): constant
Planck function, no incident radiation at the outer boundary, a diffusion inner
boundary, a two-level line parameterised by its thermalisation parameter, and
coherent isotropic continuum scattering parameterised by the continuum
thermalisation parameter.  The paper's own runs are 3D; these are their 1D
plane-parallel counterparts, sized as the workloads below state.

Conventions shared by every generator
-------------------------------------
* ``tau``   reference optical depth per node, strictly increasing inward,
            node 0 at the top.  Concatenated over atmospheres (float64).
* ``nd``    depth points per atmosphere (int32); ``off[b] = sum(nd[:b])``.
* ``q``     opacity ratio chi_k / chi_ref per (node, frequency), row-major
            ``[(off[b]+d)*nf + k]`` (float64).
* ``phi``   line profile per frequency; ``wnu`` frequency-quadrature weights,
            renormalised so that sum(wnu*phi) == 1 in float64.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class TwoLevelBatch:
    """A batch of independent plane-parallel two-level-atom atmospheres."""

    nd: np.ndarray            # [nb] int32
    tau: np.ndarray           # [sum nd] float64
    q: np.ndarray             # [sum nd, nf] float64 (line + continuum opacity / chi_ref)
    phi: np.ndarray           # [nf] float64
    wnu: np.ndarray           # [nf] float64
    eps: np.ndarray           # [nb] float64 line thermalisation parameter
    B: np.ndarray             # [sum nd] float64 Planck function per node
    S_trial: np.ndarray       # [sum nd] float64 smooth trial line source function
    na: int
    omega: np.ndarray | None = None    # [sum nd, nf] continuum albedo (None: no scattering)
    pfrac: np.ndarray | None = None    # [sum nd, nf] dS^g_k/dS_l  (None: pure line, 1)
    sg_const: np.ndarray | None = None # [sum nd, nf] part of S^g_k not proportional to S_l
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nb(self) -> int:
        return int(self.nd.shape[0])

    @property
    def nf(self) -> int:
        return int(self.phi.shape[0])

    @property
    def off(self) -> np.ndarray:
        o = np.zeros(self.nb + 1, dtype=np.int64)
        o[1:] = np.cumsum(self.nd)
        return o

    @property
    def points(self) -> int:
        """depth x angle x frequency points of one formal solution."""
        return int(self.nd.sum()) * self.na * self.nf

    def atmosphere(self, b: int) -> "TwoLevelBatch":
        o = self.off
        s = slice(int(o[b]), int(o[b + 1]))
        pick = lambda a: None if a is None else a[s]
        return TwoLevelBatch(
            nd=self.nd[b:b + 1].copy(), tau=self.tau[s], q=self.q[s], phi=self.phi,
            wnu=self.wnu, eps=self.eps[b:b + 1], B=self.B[s], S_trial=self.S_trial[s],
            na=self.na, omega=pick(self.omega), pfrac=pick(self.pfrac),
            sg_const=pick(self.sg_const), name=f"{self.name}[{b}]", meta=dict(self.meta))

    def subset(self, idx) -> "TwoLevelBatch":
        idx = [int(i) for i in idx]
        o = self.off
        rows = np.concatenate([np.arange(o[b], o[b + 1]) for b in idx]) if idx else np.zeros(0, np.int64)
        pick = lambda a: None if a is None else a[rows]
        return TwoLevelBatch(
            nd=self.nd[idx].copy(), tau=self.tau[rows], q=self.q[rows], phi=self.phi,
            wnu=self.wnu, eps=self.eps[idx], B=self.B[rows], S_trial=self.S_trial[rows],
            na=self.na, omega=pick(self.omega), pfrac=pick(self.pfrac),
            sg_const=pick(self.sg_const), name=f"{self.name}{idx[:4]}...", meta=dict(self.meta))


def doppler_grid(nf: int, x_max: float = 5.0):
    """Equidistant Doppler offsets on [-x_max, x_max], Gaussian profile and
    trapezoid weights renormalised so that sum(w * phi) == 1 in float64."""
    if nf == 1:
        x = np.zeros(1)
        phi = np.ones(1) / math.sqrt(math.pi)
        w = np.ones(1) / phi
        return x, phi, w
    x = np.linspace(-x_max, x_max, nf)
    phi = np.exp(-x * x) / math.sqrt(math.pi)
    w = np.full(nf, x[1] - x[0])
    w[0] *= 0.5
    w[-1] *= 0.5
    w = w / float(np.sum(w * phi))
    return x, phi, w


def log_tau(nd: int, lo: float, hi: float) -> np.ndarray:
    return np.logspace(math.log10(lo), math.log10(hi), nd)


def single_two_level(nd=64, na=4, nf=21, eps=1e-4, tau_lo=1e-4, tau_hi=1e4,
                     x_max=5.0, B=1.0) -> TwoLevelBatch:
    """One constant-property two-level slab: the 1D analogue of the paper's
    line test (Sect. 3.1, Sect. 3.2.2), with tau the profile-integrated line
    optical depth so that tau_k = phi_k * tau.  Default sizes: 64 depths
    log-spaced 1e-4..1e4, 4 Gauss angles per hemisphere, 21 frequencies on
    [-5, 5] in steps of 0.5, eps = 1e-4, B = 1."""
    x, phi, w = doppler_grid(nf, x_max)
    tau = log_tau(nd, tau_lo, tau_hi)
    q = np.broadcast_to(phi, (nd, nf)).copy()
    Bv = np.full(nd, float(B))
    se = math.sqrt(eps)
    S_trial = B * (1.0 - (1.0 - se) * np.exp(-math.sqrt(3.0 * eps) * tau))
    return TwoLevelBatch(nd=np.array([nd], np.int32), tau=tau, q=q, phi=phi, wnu=w,
                         eps=np.array([eps]), B=Bv, S_trial=S_trial, na=na,
                         name=f"two-level slab nd={nd} na={na} nf={nf} eps={eps:g}",
                         meta={"x": x})


def two_level_batch(nb=512, nd_lo=48, nd_hi=256, na=8, nf=1024, eps_lo=1e-6,
                    eps_hi=1e-1, sigma_m=0.5, tau_lo=1e-4, tau_hi=1e4, x_max=5.0,
                    seed=3, cont_ratio=0.0, eps_c=1e-4) -> TwoLevelBatch:
    """Many independent two-level atmospheres of uneven depth counts.

    Per atmosphere b: nd_b ~ U{nd_lo..nd_hi}; tau log-spaced tau_lo..tau_hi;
    eps_b log-uniform on [eps_lo, eps_hi]; per-node opacity multipliers
    m_{b,d} ~ lognormal(0, sigma_m) so that q_k = m * (phi_k + cont_ratio).
    B = 1.  The trial source function S_b = 1 - (1 - sqrt(eps_b)) exp(-sqrt(3 eps_b) tau)
    is a smooth, realistic line source used to time single formal solutions.

    With cont_ratio > 0 a grey coherent isotropic continuum of strength
    cont_ratio per unit profile and thermalisation eps_c is added (the
    parameterised continuum scattering of Sect. 3.1); then per node
    omega_k = r_c (1 - eps_c) / (phi_k + r_c) and the non-scattering source is
    S^g_k = (phi_k S_l + r_c eps_c B) / (phi_k + r_c eps_c), returned as
    pfrac = phi_k / (phi_k + r_c eps_c) and sg_const = r_c eps_c B / (phi_k + r_c eps_c).
    """
    rng = np.random.default_rng(seed)
    nd = rng.integers(nd_lo, nd_hi + 1, size=nb).astype(np.int32)
    eps = np.exp(rng.uniform(math.log(eps_lo), math.log(eps_hi), size=nb))
    x, phi, w = doppler_grid(nf, x_max)
    taus, ms = [], []
    for b in range(nb):
        taus.append(log_tau(int(nd[b]), tau_lo, tau_hi))
        ms.append(rng.lognormal(0.0, sigma_m, size=int(nd[b])))
    tau = np.concatenate(taus)
    m = np.concatenate(ms)
    q = m[:, None] * (phi[None, :] + cont_ratio)
    B = np.ones_like(tau)
    S_trial = np.empty_like(tau)
    o = 0
    for b in range(nb):
        n = int(nd[b])
        e = float(eps[b])
        S_trial[o:o + n] = 1.0 - (1.0 - math.sqrt(e)) * np.exp(-math.sqrt(3.0 * e) * taus[b])
        o += n
    omega = pfrac = sg_const = None
    if cont_ratio > 0.0:
        rc = cont_ratio
        om_k = rc * (1.0 - eps_c) / (phi + rc)
        omega = np.broadcast_to(om_k, q.shape).copy()
        pf_k = phi / (phi + rc * eps_c)
        pfrac = np.broadcast_to(pf_k, q.shape).copy()
        sg_const = (rc * eps_c / (phi + rc * eps_c))[None, :] * B[:, None]
    return TwoLevelBatch(nd=nd, tau=tau, q=q, phi=phi, wnu=w, eps=eps, B=B,
                         S_trial=S_trial, na=na, omega=omega, pfrac=pfrac,
                         sg_const=sg_const,
                         name=(f"{nb} two-level atmospheres nd {nd_lo}..{nd_hi} na={na} "
                               f"nf={nf} seed={seed}" + (f" +continuum r_c={cont_ratio:g}"
                                                         if cont_ratio > 0 else "")),
                         meta={"x": x, "seed": seed, "cont_ratio": cont_ratio, "eps_c": eps_c})


def random_slab(nd=9, nf=3, seed=0, tau_lo=1e-3, tau_hi=1e2, q_sigma=0.7,
                s_lo=0.2, s_hi=2.0):
    """Small slab with random opacity ratios and a random positive source per
    (node, frequency) -- for parity tests of the formal solution on ragged,
    non-smooth inputs.  Returns (tau[nd], q[nd,nf], S[nd,nf], Bbot[nf], Bbot_prev[nf])."""
    rng = np.random.default_rng(seed)
    tau = log_tau(nd, tau_lo, tau_hi) if nd > 1 else np.array([tau_lo])
    q = rng.lognormal(0.0, q_sigma, size=(nd, nf))
    S = rng.uniform(s_lo, s_hi, size=(nd, nf))
    Bb = rng.uniform(s_lo, s_hi, size=nf)
    Bp = rng.uniform(s_lo, s_hi, size=nf)
    return tau, q, S, Bb, Bp

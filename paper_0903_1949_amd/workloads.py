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


@dataclass
class SphericalBatch:
    """A batch of independent spherically symmetric two-level atmospheres."""

    nd: np.ndarray            # [nb] int32 shells per atmosphere
    r: np.ndarray             # [sum nd] float64 radii, decreasing inward, r[last] = r_core
    tau: np.ndarray           # [sum nd] float64 radial reference optical depth
    q: np.ndarray             # [sum nd, nf] float64 opacity / chi_ref
    phi: np.ndarray           # [nf]
    wnu: np.ndarray           # [nf]
    eps: np.ndarray           # [nb]
    B: np.ndarray             # [sum nd]
    n_core: int               # core rays per atmosphere
    name: str = ""

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

    def rows(self, b: int) -> slice:
        o = self.off
        return slice(int(o[b]), int(o[b + 1]))


def spherical_batch(nb=4, nd_lo=24, nd_hi=48, nf=64, n_core=8, r_out=2.0, tau_lo=1e-4,
                    tau_hi=1e8, eps_lo=1e-6, eps_hi=1e-1, sigma_m=0.5, x_max=5.0,
                    B_slope=0.0, seed=5) -> SphericalBatch:
    """Spheres after the paper's test environment (Sect. 3.1): core radius 1,
    outer radius r_out (2 for its large test case, 1.1 for the small one),
    radial optical depth log-spaced tau_lo..tau_hi (1e-4..1e8 there) at a
    constant reference opacity, so r_d = r_out - (tau_d - tau_lo) (r_out - 1) /
    (tau_hi - tau_lo); a Doppler line with per-node multipliers
    m ~ lognormal(0, sigma_m), q_k = m phi_k; eps_b log-uniform; B = 1 (the
    paper's constant Planck function) plus B_slope * (d / (nd - 1)) when a
    gradient is wanted."""
    rng = np.random.default_rng(seed)
    nd = rng.integers(nd_lo, nd_hi + 1, size=nb).astype(np.int32)
    eps = np.exp(rng.uniform(math.log(eps_lo), math.log(eps_hi), size=nb))
    x, phi, w = doppler_grid(nf, x_max)
    rs, taus, ms, Bs = [], [], [], []
    for b in range(nb):
        n = int(nd[b])
        t = log_tau(n, tau_lo, tau_hi)
        r = r_out - (t - tau_lo) * ((r_out - 1.0) / (tau_hi - tau_lo))
        r[0], r[-1] = r_out, 1.0
        rs.append(r)
        taus.append(t)
        ms.append(rng.lognormal(0.0, sigma_m, size=n))
        Bs.append(1.0 + B_slope * np.arange(n) / (n - 1))
    m = np.concatenate(ms)
    return SphericalBatch(nd=nd, r=np.concatenate(rs), tau=np.concatenate(taus),
                          q=m[:, None] * phi[None, :], phi=phi, wnu=w, eps=eps,
                          B=np.concatenate(Bs), n_core=int(n_core),
                          name=(f"{nb} spheres r_out={r_out:g} nd {nd_lo}..{nd_hi} nf={nf} "
                                f"n_core={n_core} seed={seed}"))


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


# ---------------------------------------------------------------------------
# Multilevel model atom (hydrogen-like) on a grey atmosphere.
#
# Reduced units: frequencies in units of the ionisation energy (13.6 eV),
# opacities per unit reference optical depth (the grey continuum defines it,
# chi_ref = kappa_c + sigma_c = 1 per unit tau_ref), b_k = nu_k^3 stands for
# 2 h nu^3 / c^2 and the radiative-rate weight is W_k = w_k / nu_k (the common
# factor 4 pi / h multiplies every radiative and collisional rate alike).
# Each frequency point belongs to exactly one transition (its "window");
# transitions do not overlap in frequency (a builder's simplification).
@dataclass
class MultiLevelAtom:
    nd: np.ndarray            # [nb] int32
    tau: np.ndarray           # [rows] reference optical depth
    T: np.ndarray             # [rows] temperature (K)
    na: int
    # levels
    g: np.ndarray             # [nl]
    E: np.ndarray             # [nl] energy (units of 13.6 eV); ion last
    # transitions
    lo: np.ndarray            # [nt] int32 lower level
    up: np.ndarray            # [nt] int32 upper level
    kind: np.ndarray          # [nt] 0 line, 1 bound-free
    k0: np.ndarray            # [nt] first frequency of the window
    k1: np.ndarray            # [nt] one past the last
    # frequency grid
    nu: np.ndarray            # [nf]
    wnu: np.ndarray           # [nf] trapezoid weights in nu within each window
    owner: np.ndarray         # [nf] int32 transition owning the frequency
    sigma: np.ndarray         # [nf] cross-section of the owning transition
    bfac: np.ndarray          # [nf] b = nu0^3 (lines) or nu^3 (continua)
    W: np.ndarray             # [nf] w_k / nu_k
    # depth-dependent data
    Gst: np.ndarray           # [rows, nf] stimulated-emission factor G
    Bnu: np.ndarray           # [rows, nf] Planck function (reduced)
    kc: np.ndarray            # [rows] continuum absorption per unit tau_ref (eps_c)
    sc: np.ndarray            # [rows] continuum scattering per unit tau_ref (1 - eps_c)
    nstar: np.ndarray         # [rows, nl] LTE populations
    ntot: np.ndarray          # [rows]
    Cul: np.ndarray           # [rows, nt] downward collision rates
    Clu: np.ndarray           # [rows, nt] upward collision rates (detailed balance)
    name: str = ""
    # depth-dependent Voigt line profiles (None: sigma[k] holds every profile)
    line_nu0: np.ndarray = None   # [nt] line centre (0 for continua)
    line_s: np.ndarray = None     # [nt] strength: sigma = s H(a, x) / (sqrt(pi) dnu_D)
    line_a: np.ndarray = None     # [nt] Voigt damping parameter
    dopp: np.ndarray = None       # [rows] Doppler width / line centre at each depth

    @property
    def nb(self):
        return int(self.nd.shape[0])

    @property
    def nf(self):
        return int(self.nu.shape[0])

    @property
    def nl(self):
        return int(self.g.shape[0])

    @property
    def nt(self):
        return int(self.lo.shape[0])

    @property
    def off(self):
        o = np.zeros(self.nb + 1, dtype=np.int64)
        o[1:] = np.cumsum(self.nd)
        return o


_KB_EV = 8.617333262e-5     # Boltzmann constant, eV/K
_RY_EV = 13.605693          # ionisation energy of hydrogen, eV
_SAHA = 2.0706e-16          # (h^2 / (2 pi m_e k))^(3/2) in cm^3 K^(3/2), hydrogen-like factor


def multilevel_atom(nbound=6, ncont=5, nd=128, na=8, nline_pts=100, ncont_pts=100,
                    tau_lo=1e-6, tau_hi=1e2, teff=5800.0, eps_c=1e-2, strength_lo=1e-2,
                    strength_hi=1e4, a_lo=1e-3, a_hi=1e-2, x_max=50.0, coll_scale=1e-3,
                    line_pairs=None, nb=1, seed=2, depth_profiles=False,
                    damping_log=False) -> MultiLevelAtom:
    """Hydrogen-like atom with `nbound` bound levels (E_i = 1 - 1/i^2,
    g_i = 2 i^2) and a continuum level, all bound-bound pairs as lines (or
    `line_pairs`) and bound-free continua from levels 1..ncont, on a grey
    Eddington atmosphere T = Teff (3/4 (tau + 2/3))^(1/4).

    Line strengths: LTE line-centre chi_l / chi_c at tau_ref = 1,
    log-uniform on [strength_lo, strength_hi]; Voigt damping a uniform on
    [a_lo, a_hi] (log-uniform with damping_log=True); each line sampled by nline_pts points symmetric about the
    centre and concentrated in the core (x = x_max sinh-spaced).  Continua:
    hydrogenic nu^-3 cross-sections from the edge to 4x the edge on
    ncont_pts log-spaced points, strength at the edge log-uniform in
    [0.1, 10] (times chi_c at tau_ref = 1).  Collisions: C_ul = A_ul *
    coll_scale * tau_ref, C_lu by detailed balance.  n_tot = 1e14 tau_ref,
    n_e = 1e13 sqrt(tau_ref) (cm^-3, builder's choice).  nb identical
    atmospheres are stacked when nb > 1 (a batch of the same model).

    depth_profiles=True: line profiles depend on depth through the Doppler
    width dnu_D = nu0 * 1e-4 * sqrt(T / T(tau_ref = 1)) and are not
    renormalised on the grid; sigma_{d,k} = s_t H(a_t, x) / (sqrt(pi) dnu_D),
    x = (nu_k - nu0) / dnu_D, is then evaluated by the consumer (line_nu0,
    line_s, line_a, dopp; sigma[k] keeps the reference-depth values)."""
    from scipy.special import wofz

    rng = np.random.default_rng(seed)
    nl = nbound + 1
    lev = np.arange(1, nbound + 1)
    g = np.concatenate([2.0 * lev ** 2, [1.0]])
    E = np.concatenate([1.0 - 1.0 / lev ** 2, [1.0]])
    pairs = line_pairs if line_pairs is not None else [(i, j) for i in range(nbound) for j in range(i + 1, nbound)]
    lo, up, kind = [], [], []
    for (i, j) in pairs:
        lo.append(i); up.append(j); kind.append(0)
    for i in range(ncont):
        lo.append(i); up.append(nl - 1); kind.append(1)
    lo = np.array(lo, np.int32); up = np.array(up, np.int32); kind = np.array(kind, np.int32)
    nt = lo.shape[0]
    # depth structure
    tau = log_tau(nd, tau_lo, tau_hi)
    T = teff * (0.75 * (tau + 2.0 / 3.0)) ** 0.25
    kT = _KB_EV * T / _RY_EV                        # kT in units of 13.6 eV
    ntot = 1e14 * tau
    ne = 1e13 * np.sqrt(tau)
    # LTE populations: Boltzmann within bound levels, Saha to the continuum
    bound_rel = g[None, :nbound] * np.exp(-(E[None, :nbound] - E[0]) / kT[:, None])   # n_i / (n_1/g_1 ...)
    # n_i / n_ion = g_i / g_ion * n_e * Phi(T) * exp((E_ion - E_i)/kT),  Phi = _SAHA T^-3/2 / 2
    phi_s = 0.5 * _SAHA * T ** -1.5
    ratio = g[None, :nbound] / g[nl - 1] * (ne * phi_s)[:, None] * np.exp((E[nl - 1] - E[None, :nbound]) / kT[:, None])
    nion = ntot / (1.0 + ratio.sum(axis=1))
    nstar = np.empty((nd, nl))
    nstar[:, :nbound] = ratio * nion[:, None]
    nstar[:, nl - 1] = nion
    del bound_rel
    # frequency windows
    nus, ws, owner, sig, bfac = [], [], [], [], []
    k0 = np.zeros(nt, np.int32); k1 = np.zeros(nt, np.int32)
    kpos = 0
    i1 = int(np.argmin(np.abs(tau - 1.0)))
    strengths = np.exp(rng.uniform(math.log(strength_lo), math.log(strength_hi), size=nt))
    line_nu0 = np.zeros(nt)
    line_s = np.zeros(nt)
    damp = (np.exp(rng.uniform(math.log(a_lo), math.log(a_hi), size=nt)) if damping_log
            else rng.uniform(a_lo, a_hi, size=nt))
    cstr = np.exp(rng.uniform(math.log(0.1), math.log(10.0), size=nt))
    for t in range(nt):
        l, u = int(lo[t]), int(up[t])
        if kind[t] == 0:
            nu0 = E[u] - E[l]
            dop = 1e-4 * nu0                        # Doppler width (builder's choice)
            s = np.sinh(np.linspace(-math.asinh(x_max), math.asinh(x_max), nline_pts))
            nu = nu0 + dop * s
            prof = np.real(wofz(s + 1j * damp[t])) / math.sqrt(math.pi) / dop      # Voigt, per unit nu
            w = _trapz_weights(nu)
            if not depth_profiles:
                prof = prof / np.sum(w * prof)      # normalised on the discrete grid
            # line-centre LTE opacity ratio at tau_ref = 1 sets the strength
            centre = prof[nline_pts // 2]
            Gc = g[l] / g[u]
            stim = 1.0 - nstar[i1, u] * Gc / nstar[i1, l]
            s_t = strengths[t] / (nstar[i1, l] * centre * stim)
            sigma = s_t * prof
            b = np.full(nline_pts, nu0 ** 3)
            line_nu0[t], line_s[t] = nu0, s_t
        else:
            edge = E[u] - E[l]
            nu = np.geomspace(edge, 4.0 * edge, ncont_pts)
            w = _trapz_weights(nu)
            stim = 1.0 - math.exp(-edge / kT[i1])
            s_t = cstr[t] / (nstar[i1, l] * stim)
            sigma = s_t * (edge / nu) ** 3
            b = nu ** 3
        k0[t] = kpos
        kpos += nu.shape[0]
        k1[t] = kpos
        nus.append(nu); ws.append(w); owner.append(np.full(nu.shape[0], t, np.int32))
        sig.append(sigma); bfac.append(b)
    nu = np.concatenate(nus); wnu = np.concatenate(ws); owner = np.concatenate(owner)
    sigma = np.concatenate(sig); bfac = np.concatenate(bfac)
    W = wnu / nu
    nf = nu.shape[0]
    # stimulated-emission factor and Planck function per (depth, frequency)
    Gst = np.empty((nd, nf))
    for t in range(nt):
        sl = slice(k0[t], k1[t])
        l, u = int(lo[t]), int(up[t])
        if kind[t] == 0:
            Gst[:, sl] = g[l] / g[u]
        else:
            Gst[:, sl] = (nstar[:, l] / nstar[:, u])[:, None] * np.exp(-nu[None, sl] / kT[:, None])
    Bnu = nu[None, :] ** 3 / np.expm1(nu[None, :] / kT[:, None])
    dopp = 1e-4 * np.sqrt(T / T[i1])
    sig_rows = sigma[None, :]
    if depth_profiles:
        sig_rows = np.broadcast_to(sigma, (nd, nf)).copy()
        for t in range(nt):
            if kind[t] == 0:
                sl = slice(k0[t], k1[t])
                dnu = line_nu0[t] * dopp[:, None]
                x = (nu[None, sl] - line_nu0[t]) / dnu
                sig_rows[:, sl] = line_s[t] * np.real(wofz(x + 1j * damp[t])) / (math.sqrt(math.pi) * dnu)
    # collisions: A_ul = sum_k W_k b_k G_k sigma_k (for continua evaluated with the local G)
    Cul = np.empty((nd, nt))
    Clu = np.empty((nd, nt))
    for t in range(nt):
        sl = slice(k0[t], k1[t])
        A = np.sum(W[None, sl] * bfac[None, sl] * Gst[:, sl] * sig_rows[:, sl], axis=1)
        Cul[:, t] = A * coll_scale * tau
        Clu[:, t] = Cul[:, t] * nstar[:, up[t]] / nstar[:, lo[t]]
    kc = np.full(nd, eps_c)
    sc = np.full(nd, 1.0 - eps_c)
    rep = lambda a: np.concatenate([a] * nb, axis=0) if nb > 1 else a
    return MultiLevelAtom(
        nd=np.full(nb, nd, np.int32), tau=rep(tau), T=rep(T), na=na, g=g, E=E, lo=lo, up=up,
        kind=kind, k0=k0, k1=k1, nu=nu, wnu=wnu, owner=owner, sigma=sigma, bfac=bfac, W=W,
        Gst=rep(Gst), Bnu=rep(Bnu), kc=rep(kc), sc=rep(sc), nstar=rep(nstar), ntot=rep(ntot),
        Cul=rep(Cul), Clu=rep(Clu),
        name=f"{nl}-level atom ({nt} transitions), nd={nd}, nf={nf}, na={na}",
        line_nu0=line_nu0 if depth_profiles else None, line_s=line_s if depth_profiles else None,
        line_a=np.where(kind == 0, damp, 0.0) if depth_profiles else None,
        dopp=rep(dopp) if depth_profiles else None)


def c5_atom(nd=512, na=32, nline_pts=160, ncont=4, ncont_pts=96, nlines=100, nb=1,
            seed=5) -> MultiLevelAtom:
    """The large angle-coupled case: a 20-level hydrogen-like atom (19 bound
    levels and the continuum) with `nlines` lines, all 18 Delta n = 1 pairs
    plus seeded other pairs, and bound-free continua from the lowest `ncont`
    levels; nd depths, tau_ref 1e-6..1e2; na angles per hemisphere;
    nf = nlines * nline_pts + ncont * ncont_pts frequencies (16384 at the
    defaults); depth-dependent Voigt lines with damping log-uniform on
    [1e-4, 1e-1] and strengths log-uniform on [1e-2, 1e4]; grey background
    with eps_c = 1e-2."""
    nbound = 19
    adj = [(i, i + 1) for i in range(nbound - 1)]
    rest = [(i, j) for i in range(nbound) for j in range(i + 2, nbound)]
    rng = np.random.default_rng(seed + 1000)
    pick = rng.choice(len(rest), size=nlines - len(adj), replace=False)
    pairs = sorted(adj + [rest[k] for k in pick])
    return multilevel_atom(nbound=nbound, ncont=ncont, nd=nd, na=na, nline_pts=nline_pts,
                           ncont_pts=ncont_pts, tau_lo=1e-6, tau_hi=1e2, eps_c=1e-2,
                           strength_lo=1e-2, strength_hi=1e4, a_lo=1e-4, a_hi=1e-1,
                           line_pairs=pairs, nb=nb, seed=seed, depth_profiles=True,
                           damping_log=True)


def _trapz_weights(x):
    w = np.zeros_like(x)
    d = np.diff(x)
    w[:-1] += 0.5 * d
    w[1:] += 0.5 * d
    return w


@dataclass
class GradientCase:
    """Inputs of the emergent-spectrum gradient workload: q = c_d f_k, S = B."""
    tau: np.ndarray      # [nd]
    c: np.ndarray        # [nd] per-depth opacity scale
    f: np.ndarray        # [nf] per-frequency opacity shape
    B: np.ndarray        # [nd, nf] Planck function B_nu(T(tau_d)), normalised by its max
    nu: np.ndarray       # [nf] Hz
    na: int


def gradient_case(nd=256, na=16, nf=4096, tau_lo=1e-4, tau_hi=1e4, teff=5800.0,
                  nu_lo=1.5e14, nu_hi=3e15, seed=4) -> GradientCase:
    """Per-depth opacity c_d ~ lognormal(0, 0.5), per-frequency factor f_k
    log-uniform on [0.1, 10], frequencies log-spaced nu_lo..nu_hi, grey
    Eddington T(tau) at Teff and B = B_nu(T), normalised by its maximum."""
    rng = np.random.default_rng(seed)
    tau = log_tau(nd, tau_lo, tau_hi)
    c = rng.lognormal(0.0, 0.5, size=nd)
    f = np.exp(rng.uniform(math.log(0.1), math.log(10.0), size=nf))
    nu = np.geomspace(nu_lo, nu_hi, nf)
    T = teff * (0.75 * (tau + 2.0 / 3.0)) ** 0.25
    h_over_k = 4.799243073e-11        # h / k_B in K s
    x = h_over_k * nu[None, :] / T[:, None]
    B = nu[None, :] ** 3 / np.expm1(x)
    B = B / B.max()
    return GradientCase(tau=tau, c=c, f=f, B=B, nu=nu, na=na)


@dataclass
class VoxelSphere:
    """A sphere on a 3D spherical voxel grid (r, theta_c, phi_c): radial edges
    r [nr + 1], opacity chi [nvox, nf] and thermal source B [nvox, nf] per
    voxel (voxel v = (i nt + j) np + k), scattering eps [nvox]."""
    r: np.ndarray
    nt: int
    np_: int
    chi: np.ndarray
    B: np.ndarray
    eps: np.ndarray

    @property
    def nvox(self):
        return self.chi.shape[0]

    @property
    def nf(self):
        return self.chi.shape[1]


def voxel_sphere(nr=65, nt=33, np_=65, nf=32, r_in=1.0, r_out=2.0, tau_min=1e-4, tau_max=1e8,
                 continuum="r6", line_ratio=0.0, eps=1e-4, B=1.0, lumpy=0.0, seed=0):
    """The test sphere of the paper's Sect. 3.1 on a voxel grid.  Radial
    edges logarithmic in the reference optical depth from tau_max at r_in to
    tau_min at the last inner edge (0 at r_out); the reference opacity per
    shell is the mean over the shell, dtau/dr, of chi = C / r^6 ("r6",
    C fixed by the tau range) or of a constant ("const").  nf frequencies
    across a Doppler line: chi_k = chi_ref (1 + line_ratio phi_k) with phi
    normalised to peak 1 (line_ratio 0: grey).  lumpy > 0 multiplies each
    voxel's opacity by a seeded lognormal factor of that sigma (a 3D
    structure).  B constant, eps per voxel."""
    if continuum == "r6":
        C = 5.0 * tau_max / (r_in ** -5 - r_out ** -5)
        taus = np.logspace(np.log10(tau_max), np.log10(tau_min), nr)
        r = np.concatenate([(5.0 * taus / C + r_out ** -5) ** -0.2, [r_out]])
        r[0] = r_in
    else:
        taus = np.logspace(np.log10(tau_max), np.log10(tau_min), nr)
        chi0 = tau_max / (r_out - r_in)
        r = np.concatenate([r_out - taus / chi0, [r_out]])
        r[0] = r_in
    tau_e = np.concatenate([taus, [0.0]])
    chi_shell = (tau_e[:-1] - tau_e[1:]) / (r[1:] - r[:-1])
    x = doppler_grid(nf)[0]
    phi = np.exp(-x * x)
    prof = 1.0 + line_ratio * phi
    nvox = nr * nt * np_
    chi = np.repeat(chi_shell, nt * np_)[:, None] * prof[None, :]
    if lumpy > 0.0:
        rng = np.random.default_rng(seed)
        chi = chi * rng.lognormal(0.0, lumpy, size=(nvox, 1))
    return VoxelSphere(r=r, nt=nt, np_=np_, chi=chi, B=np.full((nvox, nf), float(B)),
                       eps=np.full(nvox, float(eps)))

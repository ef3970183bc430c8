"""Oracle: 3D full characteristics on a spherical voxel grid (r, theta_c,
phi_c): the per-voxel mean intensity J, the flux vector, the 3^3-neighbour
approximate operator Lambda* and the grey two-level operator-splitting step.
Test infrastructure only.

The paper's method (Sect. 2): a set of characteristics per solid angle, one
started at each boundary voxel and tracked through the grid to its exit,
stepping from a voxel to its neighbour along the characteristic, with every
voxel crossed by at least one characteristic per solid angle.  Its spherical
set-up (Sect. 3.1): a grid regular in theta_c and phi_c, radial edges
logarithmic in the reference optical depth, zero incident intensity at the
outer boundary and I = B at the inner one, solid angles (theta, phi) with
n_theta = n_phi.  Its operator (Sect. 3.2.1): the 3^3 voxel neighbours.  The
formal solution along a characteristic and the voxel averaging are deferred
to its Papers I-II; the reading taken here:

* Voxel (i, j, k): r_i <= r < r_{i+1} (r_0 the inner, r_nr the outer
  boundary), theta_c in [j pi/nt, (j+1) pi/nt), phi_c in
  [2 pi k/np, 2 pi (k+1)/np); flat index v = (i nt + j) np + k.  Opacity
  chi_v and source S_v are constant inside a voxel (per frequency).
* Directions: mu = cos(theta) at the n_mu Gauss-Legendre nodes on (-1, 1),
  phi at n_phi equally spaced values offset by half a step; weights
  w = (w_mu / 2) / n_phi (they sum to one).
* The characteristics of one direction n: a square lattice of parallel
  lines across n (spacing h, by default half the angular size of an inner
  boundary face, r_0 pi / (2 nt)), each started where it enters the outer
  sphere (incident intensity I_out, zero by default), and for a lattice line
  that meets the inner sphere a second one started where it leaves it
  (I_core); then, in voxel order, while a voxel has not been crossed, one
  through its centre, started where the line through the centre enters the
  domain (on the inner sphere with I_core if the backward line meets it
  first, else on the outer sphere with I_out).  A characteristic ends where
  it leaves the outer sphere or meets the inner one.  (The paper starts one
  characteristic at each boundary voxel, which on the equal voxels of its
  Cartesian Papers I-II is an equal-area lattice; on this grid the inner
  faces are several times smaller than the outer ones, and that start
  over-weights the light from the core in the voxel means: 25-100% too much
  in the vacuum dilution test, at any grid refinement.)
* The walk: the next crossing is the smallest parameter beyond the current
  one among the current voxel's two spheres, two cones theta = const (the
  plane z = 0 at theta = pi/2; none on the axis) and two half-planes
  phi = const; the crossed surface names the neighbour (one index up or
  down, phi periodic); crossings closer than 1e-13 of the outer radius to the
  current point are the surface just crossed.  A line that passes the z axis (within 1e-9 of the
  outer radius) inside a pole voxel meets all half-planes there at once; it
  goes on in the pole voxel of the direction's own azimuth.  A segment is the
  part of the line inside one voxel, of length ell.
* Along a segment of optical depth D = chi_v ell with constant S_v:
  I_out = S_v + (I_in - S_v) e^{-D} (exact), and its mean over the segment
  I_bar = S_v + (I_in - S_v) psi(D), psi(D) = (1 - e^{-D}) / D.
* J_v = sum over directions of w (sum ell I_bar) / (sum ell), the sums over
  the direction's lattice segments in v (the path-length weighted mean over
  the characteristics that cross the voxel: a volume mean, since every
  lattice line stands for the same cross-section h^2); a coverage
  characteristic enters the mean only of the voxels no earlier
  characteristic of its direction crossed (elsewhere it only carries its
  intensity).  The flux vector F_v the same with w n, reported in the local
  (r, theta, phi) components at the voxel centre.
* Lambda*_{v,u} = dJ_v / dS_u for the 27 voxels u = (i+di, j+dj, k+dk),
  |di|, |dj|, |dk| <= 1 (phi periodic, no neighbour beyond a radial boundary
  or a pole), index (di+1) 9 + (dj+1) 3 + (dk+1).  Exact when every earlier
  visit of u along the characteristic is followed (window=None); with
  window = W only the last W distinct voxels of the characteristic carry
  their derivative forward.
* Grey two-level (continuum) operator splitting with the diagonal of
  Lambda*: S_new = S + ((1 - eps) J + eps B - S) / (1 - (1 - eps) L_vv).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .quadrature import gauss_legendre01


@dataclass
class Grid:
    r: np.ndarray          # [nr + 1] radial edges, ascending (r[0] inner boundary)
    nt: int                # theta_c bins over [0, pi]
    np_: int               # phi_c bins over [0, 2 pi)

    @property
    def nr(self):
        return self.r.shape[0] - 1

    @property
    def nvox(self):
        return self.nr * self.nt * self.np_

    def index(self, i, j, k):
        return (i * self.nt + j) * self.np_ + k

    def ijk(self, v):
        k = v % self.np_
        j = (v // self.np_) % self.nt
        return v // (self.np_ * self.nt), j, k

    def centre(self, i, j, k):
        """Voxel centre: mid radius, mid theta_c, mid phi_c."""
        rm = 0.5 * (self.r[i] + self.r[i + 1])
        return rm * unit(self.theta_mid(j), self.phi_mid(k))

    def theta_mid(self, j):
        return (j + 0.5) * math.pi / self.nt

    def phi_mid(self, k):
        return (k + 0.5) * 2.0 * math.pi / self.np_


def unit(theta, phi):
    s = math.sin(theta)
    return np.array([s * math.cos(phi), s * math.sin(phi), math.cos(theta)])


def directions(n_mu, n_phi):
    """Unit vectors [n_mu * n_phi, 3] and weights (sum 1): Gauss-Legendre in
    mu on (-1, 1), phi equally spaced with a half-step offset."""
    x, wx = gauss_legendre01(n_mu)           # on (0, 1), sum wx = 1
    mu = 2.0 * x - 1.0
    wmu = wx                                  # w_mu / 2 on (-1, 1)
    dirs, w = [], []
    for a in range(n_mu):
        st = math.sqrt(max(0.0, 1.0 - mu[a] * mu[a]))
        for b in range(n_phi):
            ph = (b + 0.5) * 2.0 * math.pi / n_phi
            dirs.append([st * math.cos(ph), st * math.sin(ph), mu[a]])
            w.append(wmu[a] / n_phi)
    return np.array(dirs), np.array(w)


# ---------------------------------------------------------------- the walk
def _sphere_roots(p, n, R):
    b = float(np.dot(p, n))
    c = float(np.dot(p, p)) - R * R
    disc = b * b - c
    if disc < 0.0:
        return ()
    sq = math.sqrt(disc)
    q = -(b + math.copysign(sq, b))
    if q == 0.0:
        return (0.0,)
    return (q, c / q)


def _cone_roots(p, n, theta):
    """Parameters where the line meets the cone theta_c = theta (the plane
    z = 0 at theta = pi/2); the axis (theta = 0, pi) is never crossed."""
    if theta <= 0.0 or theta >= math.pi:
        return ()
    c = math.cos(theta)
    if abs(c) < 1e-15:                       # the plane z = 0
        return (-p[2] / n[2],) if n[2] != 0.0 else ()
    c2 = c * c
    A = n[2] * n[2] - c2
    B = p[2] * n[2] - c2 * float(np.dot(p, n))
    C = p[2] * p[2] - c2 * float(np.dot(p, p))
    roots = []
    if abs(A) < 1e-300:
        if B != 0.0:
            roots = [-C / (2.0 * B)]
    else:
        disc = B * B - A * C
        if disc >= 0.0:
            sq = math.sqrt(disc)
            q = -(B + math.copysign(sq, B))
            if q != 0.0:
                roots = [q / A, C / q]
            else:
                roots = [-B / A]
    # keep the nappe of this cone: z has the sign of cos(theta)
    return tuple(t for t in roots if (p[2] + t * n[2]) * c > 0.0)


def _plane_root(p, n, phi):
    """Parameter where the line meets the half-plane phi_c = phi."""
    sp, cp = math.sin(phi), math.cos(phi)
    a = -sp * p[0] + cp * p[1]
    b = -sp * n[0] + cp * n[1]
    if b == 0.0:
        return ()
    t = -a / b
    x, y = p[0] + t * n[0], p[1] + t * n[1]
    return (t,) if cp * x + sp * y > 0.0 else ()


def _axis_crossing(p, n, dist):
    """Parameter where the line passes the z axis within `dist`, or None."""
    h2 = n[0] * n[0] + n[1] * n[1]
    if h2 == 0.0:
        return None
    t = -(p[0] * n[0] + p[1] * n[1]) / h2
    x, y = p[0] + t * n[0], p[1] + t * n[1]
    return t if x * x + y * y < dist * dist else None


def walk(g: Grid, p0, n, ijk, tol=None, max_steps=None):
    """Segments [(v, ell)] of the line p0 + t n (t >= 0) from voxel ijk (which
    contains p0) to its end, and how it ends ("out" or "core")."""
    p0 = np.asarray(p0, dtype=np.float64)
    n = np.asarray(n, dtype=np.float64)
    tol = 1e-13 * g.r[-1] if tol is None else tol
    max_steps = 8 * (g.nr + g.nt + g.np_) + 64 if max_steps is None else max_steps
    ax_tol = 1e-9 * g.r[-1]
    i, j, k = ijk
    t = 0.0
    segs = []
    dth = math.pi / g.nt
    dph = 2.0 * math.pi / g.np_
    for _ in range(max_steps):
        best, move = math.inf, None
        for R, mv in ((g.r[i + 1], ("r", +1)), (g.r[i], ("r", -1))):
            for tt in _sphere_roots(p0, n, R):
                if t + tol < tt < best:
                    best, move = tt, mv
        if g.nt > 1:
            for th, mv in (((j + 1) * dth, ("t", +1)), (j * dth, ("t", -1))):
                for tt in _cone_roots(p0, n, th):
                    if t + tol < tt < best:
                        best, move = tt, mv
        # a line through the axis (inside a pole voxel) meets every half-plane
        # phi = const at once: it crosses to the opposite azimuth instead
        t_ax = _axis_crossing(p0, n, ax_tol) if (g.np_ > 1 and (j == 0 or j == g.nt - 1)) else None
        if t_ax is not None and t + tol < t_ax < best:
            best, move = t_ax, ("a", 0)
        elif g.np_ > 1:
            for ph, mv in (((k + 1) * dph, ("p", +1)), (k * dph, ("p", -1))):
                for tt in _plane_root(p0, n, ph):
                    if t + tol < tt < best:
                        best, move = tt, mv
        if move is None:
            raise RuntimeError("characteristic left its voxel through no surface")
        segs.append((g.index(i, j, k), best - t))
        t = best
        kind, step = move
        if kind == "r":
            i += step
            if i == g.nr:
                return segs, "out"
            if i < 0:
                return segs, "core"
        elif kind == "t":
            j += step
            if not 0 <= j < g.nt:
                raise RuntimeError("characteristic crossed a pole cone")
        elif kind == "a":
            k = min(int((math.atan2(n[1], n[0]) % (2.0 * math.pi)) / dph), g.np_ - 1)
        else:
            k = (k + step) % g.np_
    raise RuntimeError("characteristic did not end")


def _voxel_of_boundary_point(g: Grid, p, i):
    r = float(np.linalg.norm(p))
    th = math.acos(max(-1.0, min(1.0, p[2] / r)))
    ph = math.atan2(p[1], p[0]) % (2.0 * math.pi)
    j = min(int(th / (math.pi / g.nt)), g.nt - 1)
    k = min(int(ph / (2.0 * math.pi / g.np_)), g.np_ - 1)
    return i, j, k


@dataclass
class Ray:
    start: str                               # "out" (I_out) or "core" (I_core)
    segs: list = field(default_factory=list)  # [(v, ell)]
    p0: np.ndarray = None                    # starting point
    end: str = ""                            # "out" or "core"
    area: float = 0.0                        # cross-section it stands for
    counts: list = field(default_factory=list)  # per segment: enters the voxel mean


def lattice_basis(n):
    """Orthonormal e1, e2 across the direction n."""
    a = np.array([0.0, 0.0, 1.0]) if abs(n[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
    e1 = np.cross(n, a)
    e1 /= np.linalg.norm(e1)
    return e1, np.cross(n, e1)


def default_spacing(g: Grid):
    """Lattice spacing: half the angular size of an inner boundary face."""
    return 0.5 * g.r[0] * math.pi / g.nt


def rays_of_direction(g: Grid, n, h=None):
    """The characteristics of direction n (see the module notes)."""
    n = np.asarray(n, dtype=np.float64)
    h = default_spacing(g) if h is None else h
    R, Rc = g.r[-1], g.r[0]
    out = []
    hit = np.zeros(g.nvox, dtype=bool)

    def add(start, p0, ijk, lattice):
        segs, end = walk(g, p0, n, ijk)
        counts = [True] * len(segs) if lattice else [not hit[v] for v, _ in segs]
        out.append(Ray(start, segs, np.asarray(p0, dtype=np.float64), end, 1.0, counts))
        for v, _ in segs:
            hit[v] = True

    e1, e2 = lattice_basis(n)
    m = int(math.ceil(R / h))
    for a in range(-m, m):
        for b in range(-m, m):
            x, y = (a + 0.5) * h, (b + 0.5) * h
            rho2 = x * x + y * y
            if rho2 >= R * R:
                continue
            q = x * e1 + y * e2
            p0 = q - math.sqrt(R * R - rho2) * n
            add("out", p0, _voxel_of_boundary_point(g, p0, g.nr - 1), True)
            if rho2 < Rc * Rc:
                p1 = q + math.sqrt(Rc * Rc - rho2) * n
                add("core", p1, _voxel_of_boundary_point(g, p1, 0), True)
    for v in range(g.nvox):
        if hit[v]:
            continue
        c = g.centre(*g.ijk(v))
        # backward along -n: the outer sphere, or the inner one if met first
        s_out = max(_sphere_roots(c, -n, g.r[-1]))
        s_core = [s for s in _sphere_roots(c, -n, g.r[0]) if s > 0.0]
        if s_core and min(s_core) < s_out:
            p0 = c - min(s_core) * n
            add("core", p0, _voxel_of_boundary_point(g, p0, 0), False)
        else:
            p0 = c - s_out * n
            add("out", p0, _voxel_of_boundary_point(g, p0, g.nr - 1), False)
        if not hit[v]:
            raise RuntimeError(f"the characteristic through the centre of voxel {v} missed it")
    return out


def ray_sets(g: Grid, dirs, h=None):
    return [rays_of_direction(g, n, h) for n in dirs]


# ------------------------------------------------------- formal solution
def psi(D):
    """(1 - e^-D)/D, series below 1e-3."""
    D = np.asarray(D, dtype=np.float64)
    small = D < 1e-3
    Dl = np.where(small, 1.0, D)             # the closed form only where it is used
    return np.where(small, 1.0 - D / 2.0 + D * D / 6.0 - D ** 3 / 24.0, -np.expm1(-Dl) / Dl)


def neighbour_slot(g: Grid, v, u):
    """Index 0..26 of u among the 3^3 neighbours of v, or -1."""
    i, j, k = g.ijk(v)
    a, b, c = g.ijk(u)
    di, dj = a - i, b - j
    dk = (c - k) % g.np_
    if dk == g.np_ - 1:
        dk = -1
    if abs(di) > 1 or abs(dj) > 1 or dk not in (-1, 0, 1):
        return -1
    return (di + 1) * 9 + (dj + 1) * 3 + (dk + 1)


def formal_solution(g: Grid, dirs, w, rsets, chi, S, I_out=None, I_core=None, lstar=False,
                    window=None, flux=False):
    """J [nvox, nf] (and Lambda* [nvox, 27, nf], the flux [nvox, 3, nf] in
    (r, theta, phi) components) for chi, S [nvox, nf]."""
    chi = np.asarray(chi, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    nvox, nf = S.shape
    I_out = np.zeros(nf) if I_out is None else np.broadcast_to(np.asarray(I_out, np.float64), (nf,))
    I_core = np.zeros(nf) if I_core is None else np.broadcast_to(np.asarray(I_core, np.float64), (nf,))
    J = np.zeros((nvox, nf))
    L = np.zeros((nvox, 27, nf)) if lstar else None
    Fc = np.zeros((nvox, 3, nf)) if flux else None
    for n, wd, rays in zip(dirs, w, rsets):
        Lsum = np.zeros(nvox)
        for ray in rays:
            for (v, ell), c in zip(ray.segs, ray.counts):
                if c:
                    Lsum[v] += ray.area * ell
        for ray in rays:
            I = (I_out if ray.start == "out" else I_core).copy()
            deriv = {}                       # u -> dI/dS_u, most recent last
            for (v, ell), c in zip(ray.segs, ray.counts):
                D = chi[v] * ell
                e = np.exp(-D)
                ps = psi(D)
                Ib = S[v] + (I - S[v]) * ps
                f = wd * ray.area * ell / Lsum[v] if c else 0.0
                J[v] += f * Ib
                if flux:
                    Fc[v] += f * np.outer(n, Ib)
                if lstar:
                    for u, du in deriv.items():
                        s = neighbour_slot(g, v, u)
                        if s >= 0:
                            L[v, s] += f * (ps * du + ((1.0 - ps) if u == v else 0.0))
                    if v not in deriv:
                        L[v, 13] += f * (1.0 - ps)
                    nd = {u: du * e for u, du in deriv.items() if u != v}
                    nd[v] = deriv.get(v, 0.0) * e + (1.0 - e)
                    if window is not None:
                        while len(nd) > window:
                            nd.pop(next(iter(nd)))
                    deriv = nd
                I = S[v] + (I - S[v]) * e
    out = {"J": J}
    if lstar:
        out["lstar"] = L
    if flux:
        F = np.zeros_like(Fc)
        for v in range(nvox):
            i, j, k = g.ijk(v)
            th, ph = g.theta_mid(j), g.phi_mid(k)
            er = unit(th, ph)
            et = np.array([math.cos(th) * math.cos(ph), math.cos(th) * math.sin(ph), -math.sin(th)])
            ep = np.array([-math.sin(ph), math.cos(ph), 0.0])
            for a, e_ in enumerate((er, et, ep)):
                F[v, a] = e_ @ Fc[v]
        out["F"] = F
    return out


def lambda_matrix(g: Grid, dirs, w, rsets, chi, nf_index=0):
    """Brute-force Lambda [nvox, nvox] at one frequency: column u is the
    change of J when S_u goes from 0 to 1 (zero incident intensities)."""
    chi1 = np.asarray(chi, dtype=np.float64)[:, nf_index:nf_index + 1]
    nvox = chi1.shape[0]
    Lm = np.zeros((nvox, nvox))
    for u in range(nvox):
        S = np.zeros((nvox, 1))
        S[u, 0] = 1.0
        Lm[:, u] = formal_solution(g, dirs, w, rsets, chi1, S)["J"][:, 0]
    return Lm


def ali_step(J, lstar_diag, S, B, eps):
    """Grey two-level operator-splitting step with the diagonal Lambda*:
    returns S_new and max |S_new - S| / |S_new| over everything."""
    J, Ld, S = (np.asarray(a, dtype=np.float64) for a in (J, lstar_diag, S))
    B = np.asarray(B, dtype=np.float64)
    eps = np.asarray(eps, dtype=np.float64)
    Sn = S + ((1.0 - eps) * J + eps * B - S) / (1.0 - (1.0 - eps) * Ld)
    return Sn, float(np.max(np.abs(Sn - S) / np.abs(Sn)))

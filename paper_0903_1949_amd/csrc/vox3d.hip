// 3D full characteristics on a spherical voxel grid (r, theta_c, phi_c):
// the plan-time geometry (host, FP64) and the formal-solution, Lambda* and
// operator-splitting kernels (gfx950).
//
// Method (the paper's Sect. 2): for every solid angle a set of
// characteristics crosses the grid from boundary to boundary, stepping from
// a voxel to its neighbour along the characteristic, and every voxel is
// crossed by at least one characteristic per solid angle.  Spherical set-up
// (Sect. 3.1): a grid regular in theta_c and phi_c, zero incident intensity
// outside and I = B leaving the inner sphere; solid angles (theta, phi).
// 3^3-neighbour Lambda* (Sect. 3.2.1).  The reading (the formal solution along
// a characteristic and the voxel averaging come from the paper's Papers I-II):
//
// * Voxel (i, j, k): r_i <= r < r_{i+1}, theta_c in [j pi/nt, (j+1) pi/nt),
//   phi_c in [2 pi k/np, 2 pi (k+1)/np); v = (i nt + j) np + k; chi and S
//   constant in a voxel.
// * Directions: mu at the n_mu Gauss-Legendre nodes on (-1, 1), phi at n_phi
//   equal steps offset by half a step; w = (w_mu / 2) / n_phi.
// * Characteristics of a direction n: a square lattice of parallel lines
//   across n with spacing h, each started where it enters the outer sphere,
//   and, for a line that meets the inner sphere, a second one started where
//   it leaves it (I_core).  Then, in voxel order, for every voxel no line has
//   crossed, the line through its centre from where it enters the domain
//   (a coverage characteristic: it enters the mean only of the voxels that
//   were not crossed before it).  Every lattice line stands for the same
//   cross-section h^2, so the path-length weighted mean of a voxel over the
//   lines that cross it is a volume mean.
// * The walk: the next crossing is the smallest parameter beyond the current
//   one among the voxel's two spheres, two cones (the plane z = 0 at pi/2)
//   and two half-planes phi = const; the crossed surface names the
//   neighbour.  A line passing the z axis inside a pole voxel (within 1e-9 of
//   the outer radius) continues in the pole voxel of the direction's own
//   azimuth.
// * A segment of optical depth D = chi ell: I_out = S + (I_in - S) e^-D, its
//   mean I_bar = S + (I_in - S) psi(D), psi = (1 - e^-D)/D;
//   J_v = sum_Omega w (sum ell I_bar) / (sum ell); the flux vector the same
//   with w n.  The plan stores per segment the voxel, ell and
//   wn = w / (sum ell of the direction in the voxel), so J_v = sum wn ell I_bar.
// * Lambda*_{v,u} = dJ_v/dS_u for the 3^3 neighbours u, followed along each
//   characteristic through its last W distinct voxels (a register window).
//
// GPU mapping: a group of G = min(64, 2^ceil(log2 nf)) lanes per
// characteristic, one frequency per lane, 64/G characteristics per wave.  The
// segment stream of a characteristic is read once for all its frequencies;
// chi and S are read as rows over frequency (the voxel's row stays in L2
// across the characteristics of nearby directions).  J, the flux and
// Lambda* accumulate with the hardware's atomic add, one per segment and
// frequency; that add rate bounds the kernel (about 1.9e11 FP64 or 3.3e11
// FP32 adds per second on the whole chip for rows of 32 to 64 values).
// FP32 plans therefore accumulate J and Lambda* (its diagonal in the
// operator-splitting step, or the full 27-neighbour band) in FP32 over blocks
// of 64 directions and add each block's sums into the FP64 outputs; FP64
// plans accumulate in FP64 directly.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <thread>

#include "pprt_internal.h"

namespace pprt {

// ================================================================ geometry
namespace {

constexpr double kPi = 3.14159265358979323846;

struct G3 {
  int nr, nt, np;
  const double* r;       // [nr + 1]
  int64_t nvox() const { return (int64_t)nr * nt * np; }
  int64_t index(int i, int j, int k) const { return ((int64_t)i * nt + j) * np + k; }
  double theta_mid(int j) const { return (j + 0.5) * kPi / nt; }
  double phi_mid(int k) const { return (k + 0.5) * 2.0 * kPi / np; }
};

struct V3 { double x, y, z; };
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 unit_tp(double th, double ph) {
  const double s = std::sin(th);
  return {s * std::cos(ph), s * std::sin(ph), std::cos(th)};
}

// roots of |p + t n|^2 = R^2 (|n| = 1); returns the count
int sphere_roots(V3 p, V3 n, double R, double t[2]) {
  const double b = dot(p, n), c = dot(p, p) - R * R;
  const double disc = b * b - c;
  if (disc < 0.0) return 0;
  const double q = -(b + std::copysign(std::sqrt(disc), b));
  if (q == 0.0) { t[0] = 0.0; return 1; }
  t[0] = q; t[1] = c / q;
  return 2;
}

// parameters where the line meets the cone theta_c = th (z = 0 at pi/2),
// on the nappe whose z has the sign of cos(th)
int cone_roots(V3 p, V3 n, double th, double t[2]) {
  if (th <= 0.0 || th >= kPi) return 0;
  const double c = std::cos(th);
  if (std::fabs(c) < 1e-15) {
    if (n.z == 0.0) return 0;
    t[0] = -p.z / n.z;
    return 1;
  }
  const double c2 = c * c;
  const double A = n.z * n.z - c2;
  const double B = p.z * n.z - c2 * dot(p, n);
  const double C = p.z * p.z - c2 * dot(p, p);
  double cand[2];
  int m = 0;
  if (std::fabs(A) < 1e-300) {
    if (B != 0.0) cand[m++] = -C / (2.0 * B);
  } else {
    const double disc = B * B - A * C;
    if (disc >= 0.0) {
      const double q = -(B + std::copysign(std::sqrt(disc), B));
      if (q != 0.0) { cand[m++] = q / A; cand[m++] = C / q; }
      else cand[m++] = -B / A;
    }
  }
  int out = 0;
  for (int a = 0; a < m; ++a)
    if ((p.z + cand[a] * n.z) * c > 0.0) t[out++] = cand[a];
  return out;
}

// parameter where the line meets the half-plane phi_c = ph
int plane_root(V3 p, V3 n, double ph, double* t) {
  const double sp = std::sin(ph), cp = std::cos(ph);
  const double a = -sp * p.x + cp * p.y, b = -sp * n.x + cp * n.y;
  if (b == 0.0) return 0;
  const double tt = -a / b;
  const double x = p.x + tt * n.x, y = p.y + tt * n.y;
  if (cp * x + sp * y > 0.0) { *t = tt; return 1; }
  return 0;
}

// parameter where the line passes the z axis within `dist`
bool axis_crossing(V3 p, V3 n, double dist, double* t) {
  const double h2 = n.x * n.x + n.y * n.y;
  if (h2 == 0.0) return false;
  const double tt = -(p.x * n.x + p.y * n.y) / h2;
  const double x = p.x + tt * n.x, y = p.y + tt * n.y;
  if (x * x + y * y < dist * dist) { *t = tt; return true; }
  return false;
}

struct Seg { int64_t v; double ell; };

// walk the line p0 + t n from voxel (i, j, k); false if it fails to end
bool walk(const G3& g, V3 p0, V3 n, int i, int j, int k, std::vector<Seg>& segs) {
  const double R = g.r[g.nr];
  const double tol = 1e-13 * R, ax_tol = 1e-9 * R;   // tol: the surface just crossed
  const double dth = kPi / g.nt, dph = 2.0 * kPi / g.np;
  const int max_steps = 8 * (g.nr + g.nt + g.np) + 64;
  double t = 0.0;
  for (int step = 0; step < max_steps; ++step) {
    double best = INFINITY;
    int kind = -1, dir = 0;   // kind 0 r, 1 theta, 2 phi, 3 axis
    double rt[2];
    const double Rs[2] = {g.r[i + 1], g.r[i]};
    for (int a = 0; a < 2; ++a) {
      const int m = sphere_roots(p0, n, Rs[a], rt);
      for (int b = 0; b < m; ++b)
        if (rt[b] > t + tol && rt[b] < best) { best = rt[b]; kind = 0; dir = a == 0 ? 1 : -1; }
    }
    if (g.nt > 1) {
      const double th[2] = {(j + 1) * dth, j * dth};
      for (int a = 0; a < 2; ++a) {
        const int m = cone_roots(p0, n, th[a], rt);
        for (int b = 0; b < m; ++b)
          if (rt[b] > t + tol && rt[b] < best) { best = rt[b]; kind = 1; dir = a == 0 ? 1 : -1; }
      }
    }
    double tax;
    if (g.np > 1 && (j == 0 || j == g.nt - 1) && axis_crossing(p0, n, ax_tol, &tax) && tax > t + tol &&
        tax < best) {
      best = tax; kind = 3;
    } else if (g.np > 1) {
      const double ph[2] = {(k + 1) * dph, k * dph};
      for (int a = 0; a < 2; ++a) {
        double tt;
        if (plane_root(p0, n, ph[a], &tt) && tt > t + tol && tt < best) {
          best = tt; kind = 2; dir = a == 0 ? 1 : -1;
        }
      }
    }
    if (kind < 0) return false;
    segs.push_back({g.index(i, j, k), best - t});
    t = best;
    if (kind == 0) {
      i += dir;
      if (i == g.nr || i < 0) return true;
    } else if (kind == 1) {
      j += dir;
      if (j < 0 || j >= g.nt) return false;
    } else if (kind == 3) {
      const double az = std::fmod(std::atan2(n.y, n.x) + 2.0 * kPi, 2.0 * kPi);
      k = std::min((int)(az / dph), g.np - 1);
    } else {
      k = (k + dir + g.np) % g.np;
    }
  }
  return false;
}

void voxel_of_boundary_point(const G3& g, V3 p, int* j, int* k) {
  const double r = std::sqrt(dot(p, p));
  const double th = std::acos(std::max(-1.0, std::min(1.0, p.z / r)));
  const double ph = std::fmod(std::atan2(p.y, p.x) + 2.0 * kPi, 2.0 * kPi);
  *j = std::min((int)(th / (kPi / g.nt)), g.nt - 1);
  *k = std::min((int)(ph / (2.0 * kPi / g.np)), g.np - 1);
}

struct DirRays {                    // the characteristics of one direction
  std::vector<int64_t> seg0;        // [nrays + 1]
  std::vector<uint8_t> core;        // starts on the inner sphere
  std::vector<Seg> segs;
  std::vector<uint8_t> counts;      // per segment: enters the voxel mean
  int64_t nfill = 0;
  bool ok = true;
};

void rays_of_direction(const G3& g, V3 n, double h, DirRays& d) {
  const double R = g.r[g.nr], Rc = g.r[0];
  std::vector<uint8_t> hit((size_t)g.nvox(), 0);
  d.seg0.assign(1, 0);
  auto add = [&](bool core, V3 p0, int i, bool lattice) {
    int j, k;
    voxel_of_boundary_point(g, p0, &j, &k);
    const size_t s0 = d.segs.size();
    if (!walk(g, p0, n, i, j, k, d.segs)) { d.ok = false; return; }
    for (size_t s = s0; s < d.segs.size(); ++s) {
      const int64_t v = d.segs[s].v;
      d.counts.push_back(lattice ? 1 : (hit[v] ? 0 : 1));
    }
    for (size_t s = s0; s < d.segs.size(); ++s) hit[d.segs[s].v] = 1;
    d.seg0.push_back((int64_t)d.segs.size());
    d.core.push_back(core ? 1 : 0);
  };
  // lattice across n
  const V3 a = std::fabs(n.z) < 0.9 ? V3{0.0, 0.0, 1.0} : V3{1.0, 0.0, 0.0};
  V3 e1 = {n.y * a.z - n.z * a.y, n.z * a.x - n.x * a.z, n.x * a.y - n.y * a.x};
  const double l1 = std::sqrt(dot(e1, e1));
  e1 = (1.0 / l1) * e1;
  const V3 e2 = {n.y * e1.z - n.z * e1.y, n.z * e1.x - n.x * e1.z, n.x * e1.y - n.y * e1.x};
  const int m = (int)std::ceil(R / h);
  for (int ia = -m; ia < m && d.ok; ++ia)
    for (int ib = -m; ib < m && d.ok; ++ib) {
      const double x = (ia + 0.5) * h, y = (ib + 0.5) * h;
      const double rho2 = x * x + y * y;
      if (rho2 >= R * R) continue;
      const V3 q = x * e1 + y * e2;
      add(false, q - std::sqrt(R * R - rho2) * n, g.nr - 1, true);
      if (rho2 < Rc * Rc) add(true, q + std::sqrt(Rc * Rc - rho2) * n, 0, true);
    }
  // coverage
  for (int64_t v = 0; v < g.nvox() && d.ok; ++v) {
    if (hit[v]) continue;
    const int k = (int)(v % g.np), j = (int)((v / g.np) % g.nt), i = (int)(v / ((int64_t)g.np * g.nt));
    const V3 c = (0.5 * (g.r[i] + g.r[i + 1])) * unit_tp(g.theta_mid(j), g.phi_mid(k));
    const V3 mn = {-n.x, -n.y, -n.z};
    double t[2];
    const int no = sphere_roots(c, mn, R, t);
    const double s_out = no == 2 ? std::max(t[0], t[1]) : t[0];
    const int nc = sphere_roots(c, mn, Rc, t);
    double s_core = INFINITY;
    for (int b = 0; b < nc; ++b)
      if (t[b] > 0.0) s_core = std::min(s_core, t[b]);
    if (s_core < s_out) add(true, c - s_core * n, 0, false);
    else add(false, c - s_out * n, g.nr - 1, false);
    ++d.nfill;
    if (!hit[v]) d.ok = false;
  }
}

}  // namespace

bool vox_build_geometry(const double* r, int nr, int nt, int np, int n_mu, int n_phi, double h, int nthreads,
                        VoxGeom& out, std::string& err) {
  G3 g{nr, nt, np, r};
  const int ndir = n_mu * n_phi;
  std::vector<double> x(n_mu), wx(n_mu);
  if (pprt_gauss_legendre01(n_mu, x.data(), wx.data()) != PPRT_OK) {
    err = "n_mu must be in 1..64";
    return false;
  }
  out.nr = nr; out.nt = nt; out.np = np; out.ndir = ndir;
  out.dirs.resize(3 * (size_t)ndir);
  out.w.resize(ndir);
  for (int a = 0; a < n_mu; ++a) {
    const double mu = 2.0 * x[a] - 1.0, st = std::sqrt(std::max(0.0, 1.0 - mu * mu));
    for (int b = 0; b < n_phi; ++b) {
      const double ph = (b + 0.5) * 2.0 * kPi / n_phi;
      const int d = a * n_phi + b;
      out.dirs[3 * d] = st * std::cos(ph);
      out.dirs[3 * d + 1] = st * std::sin(ph);
      out.dirs[3 * d + 2] = mu;
      out.w[d] = wx[a] / n_phi;
    }
  }
  std::vector<DirRays> per(ndir);
  std::atomic<int> next{0};
  auto work = [&]() {
    for (int d; (d = next.fetch_add(1)) < ndir;) {
      const V3 n = {out.dirs[3 * d], out.dirs[3 * d + 1], out.dirs[3 * d + 2]};
      rays_of_direction(g, n, h, per[d]);
    }
  };
  const int nth = std::max(1, std::min(nthreads, ndir));
  std::vector<std::thread> th;
  for (int t = 1; t < nth; ++t) th.emplace_back(work);
  work();
  for (auto& t : th) t.join();
  int64_t nrays = 0, nseg = 0;
  for (int d = 0; d < ndir; ++d) {
    if (!per[d].ok) {
      err = "a characteristic of direction " + std::to_string(d) + " left the grid through no surface";
      return false;
    }
    nrays += (int64_t)per[d].core.size();
    nseg += (int64_t)per[d].segs.size();
    out.nfill += per[d].nfill;
  }
  out.ray_seg0.resize(nrays + 1);
  out.ray_dir.resize(nrays);
  out.ray_core.resize(nrays);
  out.seg_ijk.resize(nseg);
  out.seg_ell.resize(nseg);
  out.seg_wn.resize(nseg);
  std::vector<double> lsum((size_t)g.nvox());
  int64_t ro = 0, so = 0;
  for (int d = 0; d < ndir; ++d) {
    const DirRays& dr = per[d];
    std::fill(lsum.begin(), lsum.end(), 0.0);
    for (size_t s = 0; s < dr.segs.size(); ++s)
      if (dr.counts[s]) lsum[dr.segs[s].v] += dr.segs[s].ell;
    const int64_t nr_d = (int64_t)dr.core.size();
    for (int64_t q = 0; q < nr_d; ++q) {
      out.ray_seg0[ro + q] = so + dr.seg0[q];
      out.ray_dir[ro + q] = d;
      out.ray_core[ro + q] = dr.core[q];
    }
    for (size_t s = 0; s < dr.segs.size(); ++s) {
      const int64_t v = dr.segs[s].v;
      const int k = (int)(v % np), j = (int)((v / np) % nt), i = (int)(v / ((int64_t)np * nt));
      out.seg_ijk[so + s] = (uint32_t)i << 20 | (uint32_t)j << 10 | (uint32_t)k;
      out.seg_ell[so + s] = dr.segs[s].ell;
      out.seg_wn[so + s] = dr.counts[s] ? out.w[d] / lsum[v] : 0.0;
    }
    ro += nr_d;
    so += (int64_t)dr.segs.size();
  }
  out.ray_seg0[nrays] = nseg;
  return true;
}

// ================================================================ kernels
namespace {

__device__ __forceinline__ int vox_index(uint32_t ijk, int nt, int np) {
  return ((int)(ijk >> 20) * nt + (int)((ijk >> 10) & 1023u)) * np + (int)(ijk & 1023u);
}

// slot 0..26 of u among the 3^3 neighbours of v (phi periodic), or -1
__device__ __forceinline__ int nbr_slot(uint32_t v, uint32_t u, int np) {
  const int di = (int)(u >> 20) - (int)(v >> 20);
  const int dj = (int)((u >> 10) & 1023u) - (int)((v >> 10) & 1023u);
  int dk = (int)(u & 1023u) - (int)(v & 1023u);
  if (dk > 1) dk -= np;
  if (dk < -1) dk += np;
  if (di < -1 || di > 1 || dj < -1 || dj > 1 || dk < -1 || dk > 1) return -1;
  return (di + 1) * 9 + (dj + 1) * 3 + (dk + 1);
}

// psi(D) = (1 - e^-D)/D: the series below 1e-3 (truncation D^4/120), else
// -expm1(-D)/D (no cancellation for small D)
__device__ __forceinline__ double psi_d(double D) {
  return D < 1e-3 ? 1.0 - D * (0.5 - D * (1.0 / 6.0 - D * (1.0 / 24.0))) : -expm1(-D) / D;
}
__device__ __forceinline__ float psi_d(float D) {
  return D < 1e-3f ? 1.0f - D * (0.5f - D * (1.0f / 6.0f - D * (1.0f / 24.0f))) : -expm1f(-D) / D;
}
__device__ __forceinline__ double exp_neg(double D) { return exp(-D); }
__device__ __forceinline__ float exp_neg(float D) { return expf(-D); }

constexpr int kWin = 8;   // Lambda* window: distinct voxels followed per characteristic

// MODE 0: J (+flux); 1: J + Lambda* band; 2: J + Lambda*_vv only.  The
// segments are taken P at a time: their records, then their voxels' chi and
// S rows, are loaded together before the sequential update, so each batch
// waits for two memory round trips instead of two per segment.
template <typename T, typename A, int MODE, int P>
__global__ __launch_bounds__(256) void k_vox_fs(VoxArgs<T, A> a) {
  const int lane = (int)(threadIdx.x & 63);
  const int wave = (int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
  const int G = a.group;                     // lanes per characteristic
  const int per_wave = 64 / G;
  const int fb = wave % a.nfb;               // frequency block
  const int64_t rl = (int64_t)(wave / a.nfb) * per_wave + lane / G;
  const int kf = fb * 64 + lane % G;
  if (rl >= a.nrays || kf >= a.nf) return;
  const int64_t ray = a.ray0 + rl;
  const int nf = a.nf;
  const int64_t s0 = a.ray_seg0[ray], s1 = a.ray_seg0[ray + 1];
  const int d = a.ray_dir[ray];
  T I = a.ray_core[ray] ? (a.I_core ? a.I_core[kf] : (T)0) : (a.I_out ? a.I_out[kf] : (T)0);
  double nx = 0.0, ny = 0.0, nz = 0.0;
  if (a.flux) { nx = a.dirs[3 * d]; ny = a.dirs[3 * d + 1]; nz = a.dirs[3 * d + 2]; }
  uint32_t wid[kWin];
  T wder[kWin];
  int wage[kWin];
  if constexpr (MODE != 0) {
#pragma unroll
    for (int q = 0; q < kWin; ++q) { wid[q] = 0xffffffffu; wder[q] = (T)0; wage[q] = -1; }
  }
  for (int64_t sb = s0; sb < s1; sb += P) {
    const int n = (int)(s1 - sb < P ? s1 - sb : P);
    uint32_t ijkq[P];
    T ellq[P], wnq[P], chiq[P], Sq[P];
    int vq[P];
#pragma unroll
    for (int q = 0; q < P; ++q)
      if (q < n) {
        ijkq[q] = a.seg_ijk[sb + q];
        ellq[q] = a.seg_ell[sb + q];
        wnq[q] = a.seg_wn[sb + q];
      }
#pragma unroll
    for (int q = 0; q < P; ++q)
      if (q < n) {
        vq[q] = vox_index(ijkq[q], a.nt, a.np);
        chiq[q] = a.chi[(int64_t)vq[q] * nf + kf];
        Sq[q] = a.S[(int64_t)vq[q] * nf + kf];
      }
#pragma unroll
    for (int q = 0; q < P; ++q) {
      if (q >= n) break;
      const uint32_t ijk = ijkq[q];
      const T ell = ellq[q];
      const int v = vq[q];
      const T S = Sq[q];
      const T D = chiq[q] * ell;
      const T e = exp_neg(D);
      const T ps = psi_d(D);
      const T Ib = S + (I - S) * ps;
      const double f = (double)wnq[q] * (double)ell;
      if (f != 0.0) {
        unsafeAtomicAdd(a.J + (int64_t)v * nf + kf, (A)(f * (double)Ib));
        if (a.flux) {
          double* F = a.flux + (int64_t)v * 3 * nf + kf;
          unsafeAtomicAdd(F, f * (double)Ib * nx);
          unsafeAtomicAdd(F + nf, f * (double)Ib * ny);
          unsafeAtomicAdd(F + 2 * nf, f * (double)Ib * nz);
        }
      }
      if constexpr (MODE != 0) {
        // dI_bar/dS_u = psi dI_in/dS_u (+ 1 - psi for u = v); dI_out/dS_u = e dI_in/dS_u (+ 1 - e);
        // MODE 2 accumulates the diagonal (u = v) alone
        int self = -1;
#pragma unroll
        for (int w = 0; w < kWin; ++w) {
          if (wage[w] >= 0) {
            if (wid[w] == ijk) self = w;
            const int slot = MODE == 1 ? nbr_slot(ijk, wid[w], a.np) : (wid[w] == ijk ? 13 : -1);
            if (slot >= 0 && f != 0.0) {
              const T dv = ps * wder[w] + (wid[w] == ijk ? (T)1 - ps : (T)0);
              A* Lp = MODE == 1 ? a.lstar + ((int64_t)v * 27 + slot) * nf + kf : a.lstar + (int64_t)v * nf + kf;
              unsafeAtomicAdd(Lp, (A)(f * (double)dv));
            }
          }
        }
        if (self < 0 && f != 0.0) {
          A* Lp = MODE == 1 ? a.lstar + ((int64_t)v * 27 + 13) * nf + kf : a.lstar + (int64_t)v * nf + kf;
          unsafeAtomicAdd(Lp, (A)(f * (double)((T)1 - ps)));
        }
        // carry the window: attenuate, then (re)enter v as the most recent
        int oldest = 0, oldest_age = 0x7fffffff;
#pragma unroll
        for (int w = 0; w < kWin; ++w) {
          wder[w] *= e;
          if (wage[w] < oldest_age) { oldest_age = wage[w]; oldest = w; }
        }
        const int age = (int)(sb + q - s0);
        const int w0 = self >= 0 ? self : oldest;
#pragma unroll
        for (int w = 0; w < kWin; ++w)
          if (w == w0) {
            wder[w] = (self >= 0 ? wder[w] : (T)0) + ((T)1 - e);
            wid[w] = ijk;
            wage[w] = age;
          }
      }
      I = S + (I - S) * e;
    }
  }
}

template <typename T>
__global__ void k_vox_fill(T* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (T)0;
}

__global__ void k_vox_flush(const float* src, double* dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] += (double)src[i];
}

// grey two-level operator splitting per voxel and frequency:
//   S_new = S + ((1 - eps) J + eps B - S) / (1 - (1 - eps) L_vv)
__global__ void k_vox_ali(const double* J, const double* Ld, double* S, const double* B, const double* eps,
                          int64_t nvox, int nf, unsigned long long* maxrel_bits) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double rel = 0.0;
  if (x < nvox * nf) {
    const double ep = eps[x / nf];
    const double s = S[x];
    const double sn = s + ((1.0 - ep) * J[x] + ep * B[x] - s) / (1.0 - (1.0 - ep) * Ld[x]);
    S[x] = sn;
    rel = fabs(sn - s) / fabs(sn);
    if (!(rel == rel)) rel = INFINITY;
  }
  // wave maximum, then one atomic per wave (non-negative doubles order as integers)
  for (int off = 32; off > 0; off >>= 1) rel = fmax(rel, __shfl_xor(rel, off));
  if ((threadIdx.x & 63) == 0) atomicMax(maxrel_bits, (unsigned long long)__double_as_longlong(rel));
}

template <typename T>
__global__ void k_to_bulk(const double* src, T* dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (T)src[i];
}

template <typename T, typename A>
hipError_t run_vox_fs(const VoxArgs<T, A>& a, int mode, hipStream_t s) {
  const int64_t per_wave = 64 / a.group;
  const int64_t waves = ((a.nrays + per_wave - 1) / per_wave) * a.nfb;
  const int64_t blocks = (waves + 3) / 4;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  if (blocks == 0) return hipSuccess;
  if (mode == 1) hipLaunchKernelGGL((k_vox_fs<T, A, 1, 4>), dim3((unsigned)blocks), dim3(256), 0, s, a);
  else if (mode == 2) hipLaunchKernelGGL((k_vox_fs<T, A, 2, 4>), dim3((unsigned)blocks), dim3(256), 0, s, a);
  else hipLaunchKernelGGL((k_vox_fs<T, A, 0, 8>), dim3((unsigned)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_vox_zero(double* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_vox_fill<double>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_vox_zero32(float* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_vox_fill<float>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_vox_flush(const float* src, double* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_vox_flush, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_vox_fs(int precision, bool acc32, const void* args, int mode, hipStream_t s) {
  if (precision == PPRT_FP64) return run_vox_fs(*static_cast<const VoxArgs<double, double>*>(args), mode, s);
  if (acc32) return run_vox_fs(*static_cast<const VoxArgs<float, float>*>(args), mode, s);
  return run_vox_fs(*static_cast<const VoxArgs<float, double>*>(args), mode, s);
}

hipError_t launch_vox_to_bulk(int precision, const double* src, void* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned b = (unsigned)((n + 255) / 256);
  if (precision == PPRT_FP64)
    hipLaunchKernelGGL(k_to_bulk<double>, dim3(b), dim3(256), 0, s, src, (double*)dst, n);
  else
    hipLaunchKernelGGL(k_to_bulk<float>, dim3(b), dim3(256), 0, s, src, (float*)dst, n);
  return hipGetLastError();
}

hipError_t launch_vox_ali(const double* J, const double* Ld, double* S, const double* B, const double* eps,
                          int64_t nvox, int nf, unsigned long long* maxrel_bits, hipStream_t s) {
  const int64_t n = nvox * nf;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_vox_ali, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, J, Ld, S, B, eps, nvox, nf,
                     maxrel_bits);
  return hipGetLastError();
}

}  // namespace pprt

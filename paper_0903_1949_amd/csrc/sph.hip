// Formal solution in 1D spherical symmetry on impact-parameter rays, and the
// two-level operator-splitting step on it (the geometry of the paper's 1D
// comparison calculations, Sect. 3.1; the formal-solution details are
// deferred to its Papers I-II, Sect. 2).
//
// Geometry (host, per plan): shells r_0 > .. > r_{nd-1} = R_core; nc core
// rays with mu_core = 1 - c/nc, and one tangent ray p = r_m per shell m.
// Per (ray, shell) the plan stores the path factor g = (r_d + r_{d+1}) /
// (z_d + z_{d+1}) of the segment to the next shell inward (z = sqrt(r^2 - p^2)),
// half the trapezoid weight in mu of the ray at the shell, and mu.  The
// segment's reference optical path chi_ref (z_d - z_{d+1}) equals
// dtau_ref,d * g, which keeps thin shells free of cancellation.
// Along a ray the update is the linear short characteristic with
// dtau_k = (q_k(d) + q_k(d+1))/2 * dtau_ref,d g.  Inward from I_top; outward
// from the tangent point (with the inward value) or from the core (diffusion
// value B + mu_core (B - B_prev)/dtau_k of the last radial layer).
//
// Lambda*_dd = dJ(d)/dS(d) exactly: the local alpha weights of both passes,
// plus, on a tangent ray, the round trip through the tangent point: with the
// running transmission E from the tangent point outward, the outward step
// over segment k adds e_k E^2 gamma_k to node k and, unless node k+1 is the
// tangent node, E^2 alpha_k to node k+1.
//
// Mapping: one lane per frequency; the lane walks the rays of its atmosphere
// one after another and accumulates J, J - S, H, Lambda* and 1 - Lambda* of
// every shell it crosses in the output arrays (each lane owns its frequency
// column, so the read-modify-writes never collide).
#include "pprt_internal.h"

namespace pprt {
namespace {

template <typename T>
__device__ __forceinline__ void weights(T dt, T& e, T& ps, T& al, T& ga) {
  // e, psi = (1 - e)/dt, alpha = 1 - psi, gamma = psi - e.  Thin layers
  // (dt < 1/4) by the series alpha = dt P, P = sum_{i>=0} (-dt)^i / (i+2)!
  // (nested, to (i+2)! = 14!), psi = 1 - alpha, e = 1 - dt psi.
  if (dt < T(0.25)) {
    T p = T(0);
    for (int n = 13; n >= 1; --n) p = (p * (-dt) + T(1)) / T(n + 1);
    al = dt * p;
    ps = T(1) - al;
    e = T(1) - dt * ps;
    ga = dt * ps - al;
  } else {
    e = exp(-dt);
    ps = (T(1) - e) / dt;
    al = T(1) - ps;
    ga = ps - e;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_fs_sph(SphArgs<T> a) {
  const int b = blockIdx.y;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.nf) return;
  if (a.active && !a.active[b]) return;
  const int nf = a.nf;
  const int64_t o = a.off[b];
  const int nd = (int)(a.off[b + 1] - o);
  auto S_at = [&](int d) -> T { return a.Sg ? a.Sg[(o + d) * nf + k] : T(a.Sl[o + d]); };
  auto acc = [&](T* arr, int d, T v) {
    if (arr) arr[(o + d) * nf + k] += v;
  };
  for (int d = 0; d < nd; ++d) {
    const int64_t x = (o + d) * nf + k;
    if (a.J) a.J[x] = T(0);
    if (a.JmS) a.JmS[x] = T(0);
    if (a.lstar) a.lstar[x] = T(0);
    if (a.lstar_c) a.lstar_c[x] = T(0);
    if (a.H) a.H[x] = T(0);
  }
  const T Itop = a.Itop ? a.Itop[(int64_t)b * nf + k] : T(0);
  const T dt_last = T(0.5) * (a.q[(o + nd - 2) * nf + k] + a.q[(o + nd - 1) * nf + k]) *
                    T(a.tau[o + nd - 1] - a.tau[o + nd - 2]);
  for (int j = a.ray0[b]; j < a.ray0[b + 1]; ++j) {
    const SphRay ry = a.rays[j];
    const int m = ry.m;
    // ---- inward pass
    T I = Itop, D = Itop - S_at(0);
    {
      const T h = T(a.hw[ry.e0]);
      acc(a.J, 0, h * I);
      acc(a.JmS, 0, h * D);
      acc(a.H, 0, -h * T(a.mu[ry.e0]) * I);
      acc(a.lstar_c, 0, h);
    }
    T S0 = S_at(0), q0 = a.q[o * nf + k];
    T ain_m = T(0), pin_m = T(1);
    for (int d = 0; d < m; ++d) {
      const T S1 = S_at(d + 1), q1 = a.q[(o + d + 1) * nf + k];
      const T dt = T(0.5) * (q0 + q1) * T((a.tau[o + d + 1] - a.tau[o + d]) * a.path[ry.e0 + d]);
      T e, ps, al, ga;
      weights(dt, e, ps, al, ga);
      I = e * I + al * S1 + ga * S0;
      D = e * D + ps * (S0 - S1);
      const T h = T(a.hw[ry.e0 + d + 1]);
      acc(a.J, d + 1, h * I);
      acc(a.JmS, d + 1, h * D);
      acc(a.H, d + 1, -h * T(a.mu[ry.e0 + d + 1]) * I);
      acc(a.lstar, d + 1, h * al);
      acc(a.lstar_c, d + 1, h * ps);
      ain_m = al;
      pin_m = ps;
      S0 = S1;
      q0 = q1;
    }
    // ---- turn: tangent point (inward values) or the core
    T Io, Do, aout, pout;
    if (ry.core) {
      const T Sm = S_at(m);
      if (a.lower_bc == PPRT_BC_DIFFUSION) {
        const T Bb = a.Bl ? T(a.Bl[o + nd - 1]) : a.Bbot[(int64_t)b * nf + k];
        const T Bp = a.Bl ? T(a.Bl[o + nd - 2]) : a.Bbot_prev[(int64_t)b * nf + k];
        Io = Bb + T(ry.mu_core) * (Bb - Bp) / dt_last;
      } else {
        Io = a.Ibot ? a.Ibot[(int64_t)b * nf + k] : T(0);
      }
      Do = Io - Sm;
      aout = T(0);
      pout = T(1);
    } else {
      Io = I;
      Do = D;
      aout = ain_m;
      pout = pin_m;
    }
    {
      const T h = T(a.hw[ry.e0 + m]);
      acc(a.J, m, h * Io);
      acc(a.JmS, m, h * Do);
      acc(a.H, m, h * T(a.mu[ry.e0 + m]) * Io);
      acc(a.lstar, m, h * aout);
      acc(a.lstar_c, m, h * pout);
    }
    // ---- outward pass, with the round-trip coupling of tangent rays
    T E = T(1);
    T S1 = S_at(m), q1 = a.q[(o + m) * nf + k];
    for (int d = m - 1; d >= 0; --d) {
      const T Sd = S_at(d), qd = a.q[(o + d) * nf + k];
      const T dt = T(0.5) * (qd + q1) * T((a.tau[o + d + 1] - a.tau[o + d]) * a.path[ry.e0 + d]);
      T e, ps, al, ga;
      weights(dt, e, ps, al, ga);
      Io = e * Io + al * Sd + ga * S1;
      Do = e * Do + ps * (S1 - Sd);
      const T h = T(a.hw[ry.e0 + d]);
      T ex = T(0);
      if (!ry.core) {
        const T E2 = E * E;
        ex = e * E2 * ga;
        if (d + 1 < m) {                      // to node d+1 (the tangent node counts alpha once)
          const T ex1 = E2 * al;
          const T h1 = T(a.hw[ry.e0 + d + 1]);
          acc(a.lstar, d + 1, h1 * ex1);
          acc(a.lstar_c, d + 1, -h1 * ex1);
        }
        E *= e;
      }
      acc(a.J, d, h * Io);
      acc(a.JmS, d, h * Do);
      acc(a.H, d, h * T(a.mu[ry.e0 + d]) * Io);
      acc(a.lstar, d, h * (al + ex));
      acc(a.lstar_c, d, h * (ps - ex));
      S1 = Sd;
      q1 = qd;
    }
  }
}

}  // namespace

hipError_t launch_fs_sph(int precision, int nb, int nf, hipStream_t s, const void* args) {
  const dim3 grid((unsigned)((nf + 255) / 256), (unsigned)nb);
  if (precision == PPRT_FP64)
    hipLaunchKernelGGL(k_fs_sph<double>, grid, dim3(256), 0, s, *(const SphArgs<double>*)args);
  else
    hipLaunchKernelGGL(k_fs_sph<float>, grid, dim3(256), 0, s, *(const SphArgs<float>*)args);
  return hipGetLastError();
}

}  // namespace pprt

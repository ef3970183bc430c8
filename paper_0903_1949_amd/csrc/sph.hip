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
#include <type_traits>
#include <utility>

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

// ---- sweep with rays in register groups ---------------------------------------
//
// One wave per (sphere, 64-frequency tile); lane = frequency.  The wave takes
// the sphere's rays G at a time.  Rays are ordered by impact parameter: the
// n_core core rays (deepest shell nd-1), then the tangent rays of shells
// nd-1, nd-2, ..., 0.  Ray g of group j (global index jG + g) therefore crosses
// shell d exactly when g <= T(d) = n_core + nd - 1 - d - jG, turns at its
// tangent point when g == T(d), and a whole group is inside every shell with
// T(d) >= G: each of the group's conditions is one comparison with T(d), and
// all but the last G shells of a group run without any.
//
// Per ray the wave keeps in registers the difference-form intensity
// D = I - S, the last inward psi (the outward start value of a tangent ray)
// and the transmission E from the tangent point (the round trip of Lambda*).
// q and S of a shell are read once per group, one segment ahead (with tau and
// the row's path-factor bounds), so that the loads of the next shell overlap
// the arithmetic of this one; the group's geometry rows (path factor, its
// reciprocal, half weight) come through scalar loads issued before the
// current shell's flush.  Each shell's contribution of the group is added
// once: to the J - S and 1 - Lambda* columns (formal solution), or, for the
// two-level step, already summed with the profile weights over each 16-lane
// row of frequencies (DPP) and added by the four row leaders (LDS atomics)
// into the wave's per-shell totals in LDS, which end as the tile's partial
// sums for the float64 update.
//
// Group size and occupancy were set by measurement on 512 spheres of 48-256
// shells: FP32 groups of 10 rays at six waves per SIMD (80 registers, two
// spilled) took 6.40 ms per two-level sweep, against 6.46 ms for 12 rays and
// 6.48 ms for 8 rays at their best wave counts, and 7.29 ms for 16 rays at
// four waves; the FP64 groups of 4 keep four waves.

// A load from an address that is uniform over the wave, issued as a scalar load.
template <typename T>
__device__ __forceinline__ T sload(const T* p, int64_t i) {
  return ((const __attribute__((address_space(4))) T*)p)[i];
}

// f(integral_constant<int, g>) for g = 0..N-1, unrolled in the source so that
// every per-ray register is a separate value.
template <typename F, int... I>
__device__ __forceinline__ void for_rays_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void for_rays(F&& f) {
  for_rays_impl(f, std::make_integer_sequence<int, N>{});
}

constexpr float kLog2e = 1.4426950408889634f;

// One segment of the difference-form update D <- e D + psi dS, FP32.
// Thin (x < 1/4): psi from the fitted polynomial and D + psi (dS - x D), the
// same update with 1 - e = x psi; thick: e = 2^(-x log2 e) and psi = m - e m,
// m = 1/x = rq * ip (rq = 1/(qbar dtau_ref), ip = 1/path factor).  The regime
// is chosen per wave; when the lanes disagree both forms run.
template <bool NEED_E>
__device__ __forceinline__ void seg_update(float x, float rq, float ip, float dS, float& D,
                                           float& ps, float& e) {
  const unsigned long long act = __ballot(1);
  const unsigned long long tb = __ballot(x < 0.25f);
  float Dn, pn, en = 0.0f;
  if (tb == act) {
    pn = psi_thin_f32(x);
    if (NEED_E) en = fmaf(-x, pn, 1.0f);
    Dn = fmaf(pn, fmaf(-x, D, dS), D);
  } else if (tb == 0) {
    en = __builtin_amdgcn_exp2f(-(x * kLog2e));
    const float m = rq * ip;
    pn = fmaf(-en, m, m);
    Dn = fmaf(en, D, pn * dS);
  } else {
    const float p1 = psi_thin_f32(x);
    const float D1 = fmaf(p1, fmaf(-x, D, dS), D);
    const float e2 = __builtin_amdgcn_exp2f(-(x * kLog2e));
    const float m = rq * ip;
    const float p2 = fmaf(-e2, m, m);
    const float D2 = fmaf(e2, D, p2 * dS);
    const bool thin = x < 0.25f;
    pn = thin ? p1 : p2;
    Dn = thin ? D1 : D2;
    if (NEED_E) en = thin ? fmaf(-x, p1, 1.0f) : e2;
  }
  D = Dn;
  ps = pn;
  if (NEED_E) e = en;
}

// FP64: psi by its series for thin segments (x < 1/4, 13 terms, truncation
// below 1e-17), else e = exp(-x), psi = (1 - e)/x.
template <bool NEED_E>
__device__ __forceinline__ void seg_update(double x, double rq, double ip, double dS, double& D,
                                           double& ps, double& e) {
  double pn, en;
  if (x < 0.25) {
    // psi = sum_{n=0}^{12} (-x)^n / (n+1)!
    double p = 1.0 / 6227020800.0;                    // 1/13!
    p = fma(p, -x, 1.0 / 479001600.0);
    p = fma(p, -x, 1.0 / 39916800.0);
    p = fma(p, -x, 1.0 / 3628800.0);
    p = fma(p, -x, 1.0 / 362880.0);
    p = fma(p, -x, 1.0 / 40320.0);
    p = fma(p, -x, 1.0 / 5040.0);
    p = fma(p, -x, 1.0 / 720.0);
    p = fma(p, -x, 1.0 / 120.0);
    p = fma(p, -x, 1.0 / 24.0);
    p = fma(p, -x, 1.0 / 6.0);
    p = fma(p, -x, 0.5);
    pn = fma(p, -x, 1.0);
    en = fma(-x, pn, 1.0);
  } else {
    en = exp(-x);
    pn = (1.0 - en) * (rq * ip);
  }
  D = fma(en, D, pn * dS);
  ps = pn;
  e = en;
}

// The same update with the regime fixed for the whole wave: R = 0 every
// lane thin, R = 1 every lane thick, R = 2 chosen per ray (as above).  FP64
// always decides per lane.
template <int R, bool NEED_E>
__device__ __forceinline__ void seg_update_r(float x, float rq, float ip, float dS, float& D, float& ps,
                                             float& e) {
  if constexpr (R == 0) {
    ps = psi_thin_f32(x);
    if (NEED_E) e = fmaf(-x, ps, 1.0f);
    D = fmaf(ps, fmaf(-x, D, dS), D);
  } else if constexpr (R == 1) {
    e = __builtin_amdgcn_exp2f(-(x * kLog2e));
    const float m = rq * ip;
    ps = fmaf(-e, m, m);
    D = fmaf(e, D, ps * dS);
  } else {
    seg_update<NEED_E>(x, rq, ip, dS, D, ps, e);
  }
}
template <int R, bool NEED_E>
__device__ __forceinline__ void seg_update_r(double x, double rq, double ip, double dS, double& D,
                                             double& ps, double& e) {
  seg_update<NEED_E>(x, rq, ip, dS, D, ps, e);
}

__device__ __forceinline__ float recip_t(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip_t(double x) { return 1.0 / x; }

template <typename T, int G, bool PART>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu((sizeof(T) == 4 && PART) ? 6 : 4)))
void k_sph_fast(SphFastArgs<T> a) {
  extern __shared__ __align__(16) unsigned char sph_lds[];
  const int lane = (int)(threadIdx.x & 63);
  const int wave = (int)(threadIdx.x >> 6);
  const SphItem it = a.items[(int64_t)blockIdx.x * (blockDim.x >> 6) + wave];
  const int b = __builtin_amdgcn_readfirstlane(it.b);
  if (b < 0) return;
  if (a.active != nullptr && a.active[b] == 0) return;
  const int tile = __builtin_amdgcn_readfirstlane(it.tile);
  const int nf = a.nf;
  const int k = tile * 64 + lane;
  const bool ok = k < nf;
  const int kk = ok ? k : nf - 1;                   // clamped: loads stay in bounds
  const int64_t o = a.off[b];
  const int nd = (int)(a.off[b + 1] - o);
  const int nc = a.n_core;
  const T* __restrict__ qc = a.q + kk;
  auto q_at = [&](int d) -> T { return qc[(o + d) * nf]; };
  auto S_at = [&](int d) -> T { return PART ? T(a.Sl[o + d]) : a.Sg[(o + d) * nf + kk]; };
  const T wp = PART ? (ok ? a.wphi[kk] : T(0)) : T(0);
  // two-level step: per wave, the profile-weighted sums over the tile
  // (2 quantities x ndmax shells, stride ndmax + 1)
  const int rs = a.ndmax + 1;
  T* acc = PART ? reinterpret_cast<T*>(sph_lds) + (int64_t)wave * 2 * rs : nullptr;
  if (PART) {
    for (int d = lane; d < 2 * rs; d += 64) acc[d] = T(0);
  }
  // one shell's contribution of the current group
  auto flush = [&](int d, T vj, T vl, bool store) {
    if (PART) {
      const T sj = row_sum(wp * vj);
      const T sl = row_sum(wp * vl);
      if ((lane & 15) == 0) {
        atomicAdd(acc + d, sj);
        atomicAdd(acc + rs + d, sl);
      }
    } else if (ok) {
      const int64_t x = (o + d) * nf + kk;
      if (store) {
        a.JmS[x] = vj;
        a.Lc[x] = vl;
      } else {
        a.JmS[x] += vj;
        a.Lc[x] += vl;
      }
    }
  };
  const T Itop = a.Itop ? a.Itop[(int64_t)b * nf + kk] : T(0);
  // core intensity I(mu) = Ic0 + mu Ic1
  T Ic0, Ic1 = T(0);
  if (a.lower_bc == PPRT_BC_DIFFUSION) {
    const T Bb = a.Bl ? T(a.Bl[o + nd - 1]) : a.Bbot[(int64_t)b * nf + kk];
    const T Bp = a.Bl ? T(a.Bl[o + nd - 2]) : a.Bbot_prev[(int64_t)b * nf + kk];
    const T dtl = T(0.5) * (q_at(nd - 2) + q_at(nd - 1)) * T(a.tau[o + nd - 1] - a.tau[o + nd - 2]);
    Ic0 = Bb;
    Ic1 = (Bb - Bp) / dtl;
  } else {
    Ic0 = a.Ibot ? a.Ibot[(int64_t)b * nf + kk] : T(0);
  }
  const T* muc = a.muc + (int64_t)b * nc;
  const int gfirst = a.grp0[b];
  const int gbeg = gfirst + __builtin_amdgcn_readfirstlane(it.g0);
  const int gend = gfirst + __builtin_amdgcn_readfirstlane(it.g1);
  for (int gi = gbeg; gi < gend; ++gi) {
    const int jG = (gi - gfirst) * G;
    const int Tb = nc + nd - 1 - jG;                // T(d) = Tb - d
    const int mx = Tb < nd - 1 ? Tb : nd - 1;       // deepest shell of the group
    const int ncg = nc - jG;                        // rays g < ncg are core rays
    const bool first = gi == gfirst;                // its core rays reach every shell (column
                                                    // mode: one item covers all groups)
    const int64_t t0 = sload(a.gtab, gi);
    const T* tb = a.tab + t0;
    const T* tx = a.tabx + t0 / (3 * G) * 2;        // per row: largest, smallest path factor
    T D[G], E[G], pl[G];
    T pth[G], ipt[G], hw[G];
    // regime of a shell's segments for the whole group (FP32, every ray with a
    // segment on row r): 0 all thin, 1 all thick, 2 per ray
    auto regime = [&](T qa, T pmax, T pmin) -> int {
      if constexpr (sizeof(T) == 8) {
        return 2;
      } else {
        const unsigned long long act = __ballot(1);
        if (__ballot(qa * pmax < 0.25f) == act) return 0;
        if (__ballot(qa * pmin >= 0.25f) == act) return 1;
        return 2;
      }
    };
    // the next shell's q, S, tau and regime bounds, loaded one segment ahead
    T qp, Sp, xmx = T(0), xmn = T(0);
    double tp;
    auto prefetch = [&](int d, int r) {
      qp = q_at(d);
      Sp = S_at(d);
      tp = a.tau[o + d];
      if constexpr (sizeof(T) == 4) {
        xmx = sload(tx, 2 * r);
        xmn = sload(tx, 2 * r + 1);
      }
    };
    auto load_row = [&](int d, bool geo, bool wts) {
      const T* row = tb + (int64_t)d * 3 * G;
      for_rays<G>([&](auto gc) {
        constexpr int g = decltype(gc)::value;
        if (geo) {
          pth[g] = sload(row, g);
          ipt[g] = sload(row, G + g);
        }
        if (wts) hw[g] = sload(row, 2 * G + g);
      });
    };
    // ---- inward: node 0, then segments d-1 -> d
    T S0 = S_at(0), q0 = q_at(0);
    double tu0 = a.tau[o];
    prefetch(1, 0);
    {
      load_row(0, false, true);
      T hs = T(0);
      const T D0 = Itop - S0;
      for_rays<G>([&](auto gc) {
        constexpr int g = decltype(gc)::value;
        hs += hw[g];
        D[g] = D0;
        E[g] = T(1);
        pl[g] = T(1);
      });
      flush(0, hs * D0, hs, first);
      load_row(0, true, false);
      load_row(mx > 0 ? 1 : 0, false, true);
    }
    auto inward = [&](int d, auto cond) {
      constexpr bool COND = decltype(cond)::value;
      const T q1 = qp, S1 = Sp, pmax = xmx, pmin = xmn;
      const double t1 = tp;
      prefetch(d + 1 < nd ? d + 1 : nd - 1, d < mx ? d : mx);
      const T qa = T(0.5) * (q0 + q1) * T(t1 - tu0);
      const T rq = recip_t(qa);
      const T dS = S0 - S1;
      const int Td = Tb - d;
      T aj = T(0), al = T(0);
      auto rays = [&](auto rc) {
        constexpr int R = decltype(rc)::value;
        for_rays<G>([&](auto gc) {
          constexpr int g = decltype(gc)::value;
          // every ray is computed; one past its deepest shell has zero path and
          // weight there and keeps its state
          T ps, e, Dn = D[g];
          seg_update_r<R, false>(qa * pth[g], rq, ipt[g], dS, Dn, ps, e);
          if (COND) {
            D[g] = g <= Td ? Dn : D[g];
            pl[g] = g == Td ? ps : pl[g];
          } else {
            D[g] = Dn;
          }
          aj = fma(hw[g], D[g], aj);
          al = fma(hw[g], ps, al);
        });
      };
      if constexpr (COND) {
        rays(std::integral_constant<int, 2>{});
      } else {
        const int R = regime(qa, pmax, pmin);
        if (R == 0) rays(std::integral_constant<int, 0>{});
        else if (R == 1) rays(std::integral_constant<int, 1>{});
        else rays(std::integral_constant<int, 2>{});
      }
      // the next segment's rows, loaded while this shell is flushed
      load_row(d, true, false);
      load_row(d < mx ? d + 1 : mx, false, true);
      flush(d, aj, al, first);
      q0 = q1;
      S0 = S1;
      tu0 = t1;
    };
    const int dA = Tb - G;                          // T(d) >= G for d <= dA
    {
      const int e1 = dA < mx ? dA : mx;
      int d = 1;
      for (; d <= e1; ++d) inward(d, std::false_type{});
      for (; d <= mx; ++d) inward(d, std::true_type{});
    }
    // ---- outward: turn at each ray's deepest shell, then segments d+1 -> d.
    // The round trip of a tangent ray adds e_d E^2 gamma_d to node d and, unless
    // node d+1 is its tangent node, E^2 alpha_d to node d+1 (taken from
    // 1 - Lambda*), so node d+1 is added one shell late.
    T Sn = S0, qn = q0;                              // node mx
    double tn = tu0;
    T nj = T(0), nl = T(0);
    prefetch(mx > 0 ? mx - 1 : 0, mx > 0 ? mx - 1 : 0);
    {
      load_row(mx, false, true);
      const int Td = Tb - mx;
      const T Sm = Sn;
      for_rays<G>([&](auto gc) {
        constexpr int g = decltype(gc)::value;
        if (mx == nd - 1 ? g <= Td : g == Td) {
          T pn = pl[g];
          if (g < ncg) {
            D[g] = Ic0 + muc[jG + g] * Ic1 - Sm;
            pn = T(1);
          }
          nj = fma(hw[g], D[g], nj);
          nl = fma(hw[g], pn, nl);
        }
      });
    }
    load_row(mx > 0 ? mx - 1 : 0, true, true);
    auto outward = [&](int d, auto cond) {
      constexpr bool COND = decltype(cond)::value;
      const T Sd = Sp, qd = qp, pmax = xmx, pmin = xmn;
      const double td = tp;
      prefetch(d > 0 ? d - 1 : 0, d > 0 ? d - 1 : 0);
      const T qa = T(0.5) * (qd + qn) * T(tn - td);
      const T rq = recip_t(qa);
      const T dS = Sn - Sd;
      const T* nxt = tb + (int64_t)(d + 1) * 3 * G + 2 * G;   // half weights of node d+1
      const int Td = Tb - d;
      T aj = T(0), al = T(0);
      // CORE: the group may hold core rays (g < ncg), which have no round trip
      auto rays = [&](auto rc, auto cc) {
        constexpr int R = decltype(rc)::value;
        constexpr bool CORE = decltype(cc)::value;
        for_rays<G>([&](auto gc) {
          constexpr int g = decltype(gc)::value;
          // every ray is computed; in the last shells of the group a ray with
          // g == T(d) is at its tangent point (it keeps D, adds its last inward
          // psi) and one with g > T(d) misses the shell (zero weight, keeps its state)
          const bool seg = !COND || g < Td;
          T ps, e, Dn = D[g];
          if (CORE && g < ncg) {
            seg_update_r<R, false>(qa * pth[g], rq, ipt[g], dS, Dn, ps, e);
            D[g] = seg ? Dn : D[g];
            al = fma(hw[g], seg ? ps : pl[g], al);
          } else {
            seg_update_r<R, true>(qa * pth[g], rq, ipt[g], dS, Dn, ps, e);
            const T E2 = E[g] * E[g];
            const T u = ps - e * (E2 * (ps - e));
            D[g] = seg ? Dn : D[g];
            al = fma(hw[g], seg ? u : pl[g], al);
            if (!COND || g < Td - 1) nl = fma(-sload(nxt, g), E2 * (T(1) - ps), nl);
            E[g] = seg ? E[g] * e : E[g];
          }
          aj = fma(hw[g], D[g], aj);
        });
      };
      using I0 = std::integral_constant<int, 0>;
      using I1 = std::integral_constant<int, 1>;
      using I2 = std::integral_constant<int, 2>;
      if constexpr (COND) {
        rays(I2{}, std::true_type{});
      } else if (ncg > 0) {
        rays(I2{}, std::true_type{});
      } else {
        const int R = regime(qa, pmax, pmin);
        if (R == 0) rays(I0{}, std::false_type{});
        else if (R == 1) rays(I1{}, std::false_type{});
        else rays(I2{}, std::false_type{});
      }
      load_row(d > 0 ? d - 1 : 0, true, true);
      flush(d + 1, nj, nl, false);
      nj = aj;
      nl = al;
      Sn = Sd;
      qn = qd;
      tn = td;
    };
    {
      // no condition where T(d+1) >= G (every ray has a segment and the
      // round-trip term) and d <= nd - 2
      int dB = dA - 1;
      if (dB > nd - 2) dB = nd - 2;
      if (dB < -1) dB = -1;
      int d = mx - 1;
      for (; d > dB; --d) outward(d, std::true_type{});
      for (; d >= 0; --d) outward(d, std::false_type{});
    }
    flush(0, nj, nl, false);
  }
  if (PART) {
    // this chunk's slot: the (J - S, 1 - Lambda*) pair at 2 slot, 2 slot + 1 of
    // the tile's (P + 1) / 2 four-value entries (the update adds entry values 0
    // and 2, and 1 and 3); the first chunk also clears the slots its sphere
    // leaves unused
    const int slot = __builtin_amdgcn_readfirstlane(it.slot);
    const int nslot = __builtin_amdgcn_readfirstlane(it.nslot);
    const int P2 = 2 * ((a.P + 1) >> 1);
    for (int d = lane; d < nd; d += 64) {
      T* pp = a.part + ((o + d) * a.ntiles + tile) * (int64_t)P2 * 2;
      pp[slot * 2 + 0] = acc[d];
      pp[slot * 2 + 1] = acc[rs + d];
      if (slot == 0)
        for (int c = nslot; c < P2; ++c) {
          pp[c * 2 + 0] = T(0);
          pp[c * 2 + 1] = T(0);
        }
    }
  }
}

}  // namespace

int sph_group_size(int precision) { return precision == PPRT_FP64 ? 4 : 10; }

size_t sph_fast_lds_bytes(int precision, int wpb, int ndmax) {
  return (size_t)wpb * 2 * (ndmax + 1) * (precision == PPRT_FP64 ? sizeof(double) : sizeof(float));
}

hipError_t launch_sph_fast(int precision, int nblocks, int wpb, hipStream_t s, const void* args) {
  if (nblocks <= 0) return hipSuccess;
  const dim3 grid((unsigned)nblocks), block((unsigned)(64 * wpb));
  if (precision == PPRT_FP64) {
    const auto& a = *(const SphFastArgs<double>*)args;
    if (a.part)
      hipLaunchKernelGGL((k_sph_fast<double, 4, true>), grid, block,
                         sph_fast_lds_bytes(precision, wpb, a.ndmax), s, a);
    else
      hipLaunchKernelGGL((k_sph_fast<double, 4, false>), grid, block, 0, s, a);
  } else {
    const auto& a = *(const SphFastArgs<float>*)args;
    if (a.part)
      hipLaunchKernelGGL((k_sph_fast<float, 10, true>), grid, block,
                         sph_fast_lds_bytes(precision, wpb, a.ndmax), s, a);
    else
      hipLaunchKernelGGL((k_sph_fast<float, 10, false>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_fs_sph(int precision, int nb, int nf, hipStream_t s, const void* args) {
  const dim3 grid((unsigned)((nf + 255) / 256), (unsigned)nb);
  if (precision == PPRT_FP64)
    hipLaunchKernelGGL(k_fs_sph<double>, grid, dim3(256), 0, s, *(const SphArgs<double>*)args);
  else
    hipLaunchKernelGGL(k_fs_sph<float>, grid, dim3(256), 0, s, *(const SphArgs<float>*)args);
  return hipGetLastError();
}

}  // namespace pprt

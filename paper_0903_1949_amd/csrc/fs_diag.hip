// Formal solution without in-layer scattering (omega = 0) on gfx950.
//
// Method: for a layer between nodes d and d+1 the transmission operators are
// diagonal, t+- = diag(exp(-dtau_k/mu_i)), the reflections vanish, and the
// source vectors beta+- follow from a source function linear in tau_k between
// the nodes (the 1D comparison calculation of the paper, Sect. 3.2; the
// formal-solution scheme itself is deferred to the paper's Papers I-II,
// Sect. 2).  The sweep is written in difference form D = I - S:
//     D+(d)   = e D+(d+1) + psi (S(d+1) - S(d))     (up-going)
//     D-(d+1) = e D-(d)   + psi (S(d)   - S(d+1))   (down-going)
// with e = exp(-Delta), psi = (1 - e)/Delta, Delta = dtau_k / mu_i.  This is
// algebraically the linear short-characteristic update and is exactly zero for
// constant S, so J - S carries no rounding "leak".  1 - Lambda*_dd is summed
// from psi directly (1 - alpha = psi), never as 1 minus a sum.
//
// Mapping: one lane per frequency, all na angles of both hemispheres in
// registers; a block holds `waves_per_block` waves of consecutive frequencies
// of one atmosphere; blocks are ordered longest atmosphere first.  Depth-major
// layout: at each depth step the 64 lanes of a wave read 64 consecutive
// frequencies of one row (coalesced).
#include "pprt_internal.h"

namespace pprt {
namespace {

// ---- per-layer weights of one angle --------------------------------------
// e = exp(-Delta), psi = (1-e)/Delta, and for the plain form
// alpha = 1 - psi, gamma = psi - e, with Delta = dtau_k / mu_i.
//
// FP32: optically thin layers (Delta < 1/4) take the series
//   psi   = sum_{n>=0} (-Delta)^n/(n+1)!           (to Delta^5, truncation < 5e-8)
//   alpha = sum_{n>=1} (-1)^(n+1) Delta^n/(n+1)!   (to Delta^6)
// and e = 1 - Delta psi, gamma = Delta psi - alpha (both exact identities), so
// they need no exponential at all; thicker layers take the closed forms with
// v_exp_f32, psi = m - e m where m = mu_i / dtau_k.  The choice is made per
// wave: when all 64 lanes agree only one branch executes (over 90% of the
// (wave, layer, angle) triples in line-formation atmospheres), otherwise both
// run and each lane selects its own.
template <bool AG>
__device__ __forceinline__ void layer_w_thin(float D, float& e_, float& ps_, float& al_, float& ga_) {
  ps_ = fmaf(D, fmaf(D, fmaf(D, fmaf(D, fmaf(D, -1.f / 720.f, 1.f / 120.f), -1.f / 24.f),
                             1.f / 6.f), -0.5f), 1.f);
  e_ = fmaf(-D, ps_, 1.f);
  if (AG) {
    al_ = D * fmaf(-D, fmaf(-D, fmaf(-D, fmaf(-D, fmaf(-D, 1.f / 5040.f, 1.f / 720.f),
                                               1.f / 120.f), 1.f / 24.f), 1.f / 6.f), 0.5f);
    ga_ = fmaf(D, ps_, -al_);
  }
}
template <bool AG>
__device__ __forceinline__ void layer_w_thick(float dt, float inv_dt, float c, float mu, float& e_,
                                              float& ps_, float& al_, float& ga_) {
  e_ = __builtin_amdgcn_exp2f(-(dt * c));        // v_exp_f32; c = log2(e)/mu
  const float m = mu * inv_dt;
  ps_ = fmaf(-e_, m, m);
  if (AG) {
    al_ = 1.f - ps_;
    ga_ = ps_ - e_;
  }
}
template <bool AG>
__device__ __forceinline__ void layer_w(float dt, float inv_dt, float c, float rmu, float mu,
                                        float& e, float& ps, float& al, float& ga) {
  const float D = dt * rmu;
  const bool thin = D < 0.25f;
  const unsigned long long act = __ballot(1);
  const unsigned long long tb = __ballot(thin);
  auto thin_w = [&](float& e_, float& ps_, float& al_, float& ga_) { layer_w_thin<AG>(D, e_, ps_, al_, ga_); };
  auto thick_w = [&](float& e_, float& ps_, float& al_, float& ga_) {
    layer_w_thick<AG>(dt, inv_dt, c, mu, e_, ps_, al_, ga_);
  };
  if (tb == act) {
    thin_w(e, ps, al, ga);
  } else if (tb == 0) {
    thick_w(e, ps, al, ga);
  } else {
    float e1, p1, a1 = 0.f, g1 = 0.f, e2, p2, a2 = 0.f, g2 = 0.f;
    thin_w(e1, p1, a1, g1);
    thick_w(e2, p2, a2, g2);
    e = thin ? e1 : e2;
    ps = thin ? p1 : p2;
    if (AG) {
      al = thin ? a1 : a2;
      ga = thin ? g1 : g2;
    }
  }
}

// FP64: closed forms throughout (expm1 keeps psi accurate for any Delta > 0;
// alpha and gamma then carry absolute errors ~1e-16, below every use).
template <bool AG>
__device__ __forceinline__ void layer_w(double dt, double inv_dt, double /*c*/, double rmu,
                                        double mu, double& e, double& ps, double& al, double& ga) {
  const double D = dt * rmu;
  e = exp(-D);
  ps = -expm1(-D) * (mu * inv_dt);
  if (AG) {
    al = 1.0 - ps;
    ga = ps - e;
  }
}

__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// Quad-local swaps (lanes 4q..4q+3): partner 1 and partner 2.
__device__ __forceinline__ float dpp_quad_swap1(float v) { return dpp_f<0xb1>(v); }
__device__ __forceinline__ float dpp_quad_swap2(float v) { return dpp_f<0x4e>(v); }
__device__ __forceinline__ double dpp_quad_swap1(double v) { return dpp_d<0xb1>(v); }
__device__ __forceinline__ double dpp_quad_swap2(double v) { return dpp_d<0x4e>(v); }

// ---------------------------------------------------------------------------
// Full-output formal solution.  Two recurrences run side by side per angle:
// the difference form D = I - S (for J - S and H, which are small differences
// deep in the atmosphere) and the plain form
//     I+(d) = e I+(d+1) + alpha S(d) + gamma S(d+1)
// (for I+-, J, the emergent intensity and Lambda*, which are small where the
// medium is optically thin).  Each form is accurate where the other loses
// digits; both are the same linear short-characteristic update.  The
// up-going sweep runs first and parks its hemisphere's moments in the output
// arrays; the down-going sweep completes them.
template <typename T, int NA>
__global__ __launch_bounds__(512) void k_fs_full(FsFullArgs<T> a, Angles<T> ang) {
  const Item it = a.items[blockIdx.x];
  const int b = it.b;
  const int nd = it.nd;
  const int nf = a.nf;
  const int k = it.g * (int)blockDim.x + (int)threadIdx.x;
  if (k >= nf) return;
  const int64_t row0 = a.off[b];
  const uint32_t o = a.outputs;
  // parking places for the up-going hemisphere's moments
  T* pj = (o & PPRT_OUT_JMS) ? a.JmS : nullptr;           // 1/2 sum w D+
  T* pJ = (o & PPRT_OUT_J) ? a.J : nullptr;               // 1/2 sum w I+
  T* pc = (o & PPRT_OUT_LSTAR_C) ? a.lstar_c : nullptr;   // 1/2 sum w psi
  T* pa = (o & PPRT_OUT_LSTAR) ? a.lstar : nullptr;       // 1/2 sum w alpha
  T* ph = (o & PPRT_OUT_H) ? a.H : nullptr;               // 1/2 sum w mu D+
  T* Ip = (o & PPRT_OUT_IPLUS) ? a.Iplus : nullptr;
  T* Im = (o & PPRT_OUT_IMINUS) ? a.Iminus : nullptr;
  T* Lsup = (o & PPRT_OUT_LSTAR_SUP) ? a.lsup : nullptr;   // dJ(d)/dS(d+1): up-going rays
  T* Lsub = (o & PPRT_OUT_LSTAR_SUB) ? a.lsub : nullptr;   // dJ(d)/dS(d-1): down-going rays

  T D[NA], I[NA];
  // alpha of the previous layer in sweep order (0 next to the boundary node,
  // whose intensity does not depend on S): band = 1/2 sum w (gamma + e alpha_prev)
  T aprev[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) aprev[i] = T(0);
  // ---- up-going sweep: node nd-1 (lower boundary) -> node 0
  int64_t r = row0 + nd - 1;
  T q1 = a.q[r * nf + k];
  T S1 = a.Sg[r * nf + k];
  double t1 = a.tau[r];
  {
    const T q0 = a.q[(r - 1) * nf + k];
    const T dt = T(0.5) * (q0 + q1) * T(t1 - a.tau[r - 1]);
    if (a.lower_bc == PPRT_BC_DIFFUSION) {
      const T Bb = a.Bbot[(int64_t)b * nf + k];
      const T Bp = a.Bbot_prev[(int64_t)b * nf + k];
      const T g = (Bb - Bp) / dt;
      const T base = Bb - S1;
#pragma unroll
      for (int i = 0; i < NA; ++i) {
        D[i] = base + ang.mu[i] * g;
        I[i] = Bb + ang.mu[i] * g;
      }
    } else {
#pragma unroll
      for (int i = 0; i < NA; ++i) {
        I[i] = a.Ibot ? a.Ibot[((int64_t)b * nf + k) * NA + i] : T(0);
        D[i] = I[i] - S1;
      }
    }
  }
  auto emit_up = [&](int64_t rr, T csum, T asum) {
    T js = T(0), hs = T(0), Js = T(0);
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      js += ang.hw[i] * D[i];
      hs += ang.hwmu[i] * D[i];
      Js += ang.hw[i] * I[i];
    }
    const int64_t x = rr * nf + k;
    if (pj) pj[x] = js;
    if (pJ) pJ[x] = Js;
    if (pc) pc[x] = csum;
    if (pa) pa[x] = asum;
    if (ph) ph[x] = hs;
    if (Ip) {
#pragma unroll
      for (int i = 0; i < NA; ++i) Ip[x * NA + i] = I[i];
    }
  };
  emit_up(r, ang.hwsum, T(0));
  if (Lsup) Lsup[r * nf + k] = T(0);
  for (int d = nd - 2; d >= 0; --d) {
    r = row0 + d;
    const T q0 = a.q[r * nf + k];
    const T S0 = a.Sg[r * nf + k];
    const double t0 = a.tau[r];
    const T dt = T(0.5) * (q0 + q1) * T(t1 - t0);
    const T inv = recip(dt);
    const T dS = S1 - S0;
    T cs = T(0), as = T(0), bs = T(0);
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      T e, ps, al, ga;
      layer_w<true>(dt, inv, ang.c[i], ang.rmu[i], ang.mu[i], e, ps, al, ga);
      D[i] = e * D[i] + ps * dS;
      I[i] = e * I[i] + al * S0 + ga * S1;
      cs += ang.hw[i] * ps;
      as += ang.hw[i] * al;
      bs += ang.hw[i] * (ga + e * aprev[i]);
      aprev[i] = al;
    }
    emit_up(r, cs, as);
    if (Lsup) Lsup[r * nf + k] = bs;
    q1 = q0; S1 = S0; t1 = t0;
  }
  if (o & PPRT_OUT_IEMERG) {
#pragma unroll
    for (int i = 0; i < NA; ++i) a.Iemerg[((int64_t)b * nf + k) * NA + i] = I[i];
  }

  // ---- down-going sweep: node 0 (upper boundary) -> node nd-1
  // q1, S1, t1 now hold node 0.
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    I[i] = a.Itop ? a.Itop[((int64_t)b * nf + k) * NA + i] : T(0);
    D[i] = I[i] - S1;
  }
  auto emit_down = [&](int64_t rr, T csum, T asum) {
    T js = T(0), hs = T(0), Js = T(0);
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      js += ang.hw[i] * D[i];
      hs += ang.hwmu[i] * D[i];
      Js += ang.hw[i] * I[i];
    }
    const int64_t x = rr * nf + k;
    if (pj) pj[x] = pj[x] + js;
    if (pJ) pJ[x] = pJ[x] + Js;
    if (pc) pc[x] = pc[x] + csum;
    if (pa) pa[x] = pa[x] + asum;
    if (ph) ph[x] = ph[x] - hs;
    if (Im) {
#pragma unroll
      for (int i = 0; i < NA; ++i) Im[x * NA + i] = I[i];
    }
  };
  T q0 = q1, S0 = S1;
  double t0 = t1;
  emit_down(row0, ang.hwsum, T(0));
  if (Lsub) Lsub[row0 * nf + k] = T(0);
#pragma unroll
  for (int i = 0; i < NA; ++i) aprev[i] = T(0);
  for (int d = 1; d < nd; ++d) {
    r = row0 + d;
    q1 = a.q[r * nf + k];
    S1 = a.Sg[r * nf + k];
    t1 = a.tau[r];
    const T dt = T(0.5) * (q0 + q1) * T(t1 - t0);
    const T inv = recip(dt);
    const T dS = S0 - S1;
    T cs = T(0), as = T(0), bs = T(0);
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      T e, ps, al, ga;
      layer_w<true>(dt, inv, ang.c[i], ang.rmu[i], ang.mu[i], e, ps, al, ga);
      D[i] = e * D[i] + ps * dS;
      I[i] = e * I[i] + al * S1 + ga * S0;
      cs += ang.hw[i] * ps;
      as += ang.hw[i] * al;
      bs += ang.hw[i] * (ga + e * aprev[i]);
      aprev[i] = al;
    }
    emit_down(r, cs, as);
    if (Lsub) Lsub[r * nf + k] = bs;
    q0 = q1; S0 = S1; t0 = t1;
  }
}

// ---------------------------------------------------------------------------
// Profile-moment formal solution for the two-level ALI.  The line source S_l
// is one value per node, so J - S and 1 - Lambda* enter only through their
// profile-weighted sums, and those are additive over hemispheres and over
// frequencies.  Every wave therefore runs independently: ONE sweep direction
// over 64 consecutive frequencies of one atmosphere, no barrier, no sharing.
//
// Per node each lane forms wphi_k * 1/2 sum_i w_i D_i and
// wphi_k * 1/2 sum_i w_i psi_i and parks the pair in the wave's LDS slab
// [CH nodes][2][64 lanes].  Every CH nodes the wave reduces the slab
// transposed: lane l sums 16 contiguous entries of one (node, quantity)
// (ds_read_b128), a quad DPP step adds the four parts, and one lane per
// (node, quantity) writes part[row][wave][dir][q].  The per-node cost is one
// ds_write2 instead of a 64-lane DPP tree.
constexpr int CH = 8;

// Moments reduced per node: (J-S, 1-Lambda*) or, with the tri-diagonal
// operator, also the neighbour band; the slab holds CHN nodes of NQ
// quantities (NQ * CHN <= 16 lane groups) and part[] has NQP per hemisphere.
template <bool TRI>
struct ProfileLayout {
  static constexpr int NQ = TRI ? 3 : 2;
  static constexpr int NQP = TRI ? 4 : 2;
  static constexpr int CHN = TRI ? 5 : CH;
};

// One layer of the difference-form sweep for all angles, with the
// Lambda*-complement sum ls += sum_i wh_i psi_i (wh_i: the lane's weight of
// angle i, w_i/2 times its frequency's profile weight).
//
// FP32.  Every angle takes the same update,
//     D <- D + psi (dS - Delta D)        (= e D + psi dS, as 1 - e = Delta psi),
// and only psi is formed by regime.  Optically thin (Delta < 1/4): psi from a
// degree-4 polynomial fitted to (1 - e^-Delta)/Delta on [0, 1/4] for least
// maximum relative error (Remez exchange; fitted error 2.5e-9, below FP32
// rounding; evaluated in FP32 the error is 4.5e-8).  Thick: psi = m - e m,
// e = 2^(-dtau c) (v_exp_f32), m = mu / dtau; there 1 - Delta psi equals e up
// to an absolute rounding error of order 1e-7, i.e. the transmitted term keeps
// a relative accuracy of order 1e-7 of D, like e D itself.  Because
// Delta_i = dtau / mu_i, the wave decides once per layer: all angles thin when
// dtau < min_i(mu_i)/4 in every lane, all thick when dtau >= max_i(mu_i)/4 in
// every lane, otherwise per angle (and per lane when the lanes disagree).  The
// branches produce only psi, so the intensities are updated in place after
// they join (no register copies of the NA intensities at the join).
template <int NA>
__device__ __forceinline__ void sweep_layer(const Angles<float>& ang, const float (&wh)[NA], float dt,
                                            float dS, float (&D)[NA], float& ls) {
  constexpr float kThin = 0.25f;
  auto psi_poly = [](float x) {
    float p = fmaf(x, 7.510221563279629e-3f, -4.1488952934741974e-2f);
    p = fmaf(x, p, 1.6665081679821014e-1f);
    p = fmaf(x, p, -4.999994933605194e-1f);
    return fmaf(x, p, 1.0f);
  };
  auto psi_exp = [&](int i, float inv) {
    const float e = __builtin_amdgcn_exp2f(-(dt * ang.c[i]));
    const float m = ang.mu[i] * inv;
    return fmaf(-e, m, m);
  };
  float ps[NA], x[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) x[i] = dt * ang.rmu[i];     // Delta_i
  const unsigned long long act = __ballot(1);
  const bool all_thin = __ballot(dt < ang.dt_all_thin) == act;
  if (all_thin) {
#pragma unroll
    for (int i = 0; i < NA; ++i) ps[i] = psi_poly(x[i]);
  } else {
    const float inv = recip(dt);
    if (__ballot(dt >= ang.dt_all_thick) == act) {
#pragma unroll
      for (int i = 0; i < NA; ++i) ps[i] = psi_exp(i, inv);
    } else {
#pragma unroll
      for (int i = 0; i < NA; ++i) {
        const bool thin = x[i] < kThin;
        const unsigned long long tb = __ballot(thin);
        if (tb == act) {
          ps[i] = psi_poly(x[i]);
        } else if (tb == 0) {
          ps[i] = psi_exp(i, inv);
        } else {
          const float p1 = psi_poly(x[i]);
          const float p2 = psi_exp(i, inv);
          ps[i] = thin ? p1 : p2;
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    D[i] = fmaf(ps[i], fmaf(-x[i], D[i], dS), D[i]);
    ls = fmaf(wh[i], ps[i], ls);
  }
}

// FP64: the series below 1/4, the closed form above (as described in the loop).
template <int NA>
__device__ __forceinline__ void sweep_layer(const Angles<double>& ang, const double (&wh)[NA], double dt,
                                            double dS, double (&D)[NA], double& ls) {
  const double inv = recip(dt);
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    // thin (Delta < 1/4): psi by its series, 13 terms (truncation below
    // 1e-17), and e = 1 - Delta psi; thick: e = exp(-Delta) and
    // psi = (1 - e) mu / dtau, where 1 - e >= 0.22 loses nothing
    const double x = dt * ang.rmu[i];
    double e, ps;
    if (x < 0.25) {
      double p = 1.0 / 6227020800.0;                  // 1/13!
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
      ps = fma(p, -x, 1.0);
      e = fma(-x, ps, 1.0);
    } else {
      e = exp(-x);
      ps = (1.0 - e) * (ang.mu[i] * inv);
    }
    D[i] = e * D[i] + ps * dS;
    ls += wh[i] * ps;
  }
}

template <typename T, int NA, bool UP, bool TRI>
__device__ __forceinline__ void profile_sweep(const FsProfileArgs<T>& a, const Angles<T>& ang,
                                              const Item it, T* slab) {
  const int b = it.b;
  const int nd = it.nd;
  const int nf = a.nf;
  const int lane = (int)(threadIdx.x & 63);
  const int k = it.g * 64 + lane;
  const int kk = k < nf ? k : nf - 1;         // clamped: loads stay in bounds
  const int64_t row0 = a.off[b];
  const T wp = k < nf ? a.wphi[kk] : T(0);
  T wh[NA];                                   // the lane's weights: profile x angle
#pragma unroll
  for (int i = 0; i < NA; ++i) wh[i] = wp * ang.hw[i];
  // q of node `row` for this lane: a uniform row base plus the lane's column
  auto qat = [&](int64_t row) { return a.q[row * nf + kk]; };
  // S, B and the per-row differences are read-only for the whole launch and
  // their index is uniform over the wave: reading them through the constant
  // address space makes them scalar loads, kept in scalar registers
  using cdouble = const __attribute__((address_space(4))) double;
  using cT = const __attribute__((address_space(4))) T;
  cdouble* const Sc = (cdouble*)a.S;
  cdouble* const Bc = (cdouble*)a.B;
  cT* const dtr = (cT*)a.dtr;     // T(tau[r+1] - tau[r]) / 2
  cT* const dSr = (cT*)a.dSr;     // T(S[r+1] - S[r])

  T D[NA];
  int d = UP ? nd - 1 : 0;
  T qn = qat(row0 + d);
  double Sn = Sc[row0 + d];
  if (UP) {
    const T qa = qat(row0 + d - 1);
    const T dt = (qa + qn) * dtr[row0 + d - 1];
    if (a.lower_bc == PPRT_BC_DIFFUSION) {
      const double Bb = Bc[row0 + d];
      const double Bp = Bc[row0 + d - 1];
      const T g = T(Bb - Bp) / dt;
      const T base = T(Bb - Sn);
#pragma unroll
      for (int i = 0; i < NA; ++i) D[i] = base + ang.mu[i] * g;
    } else {
#pragma unroll
      for (int i = 0; i < NA; ++i)
        D[i] = (a.Ibot ? a.Ibot[((int64_t)b * nf + kk) * NA + i] : T(0)) - T(Sn);
    }
  } else {
#pragma unroll
    for (int i = 0; i < NA; ++i)
      D[i] = (a.Itop ? a.Itop[((int64_t)b * nf + kk) * NA + i] : T(0)) - T(Sn);
  }

  // slab reduction: lane -> (sigma = NQ*slot + quantity, part p of 4)
  constexpr int NQ = ProfileLayout<TRI>::NQ;
  constexpr int NQP = ProfileLayout<TRI>::NQP;
  constexpr int CHN = ProfileLayout<TRI>::CHN;
  const int sig = lane >> 2;
  const int prt = lane & 3;
  T* const out = a.part;
  const int nw = a.nw;
  auto flush = [&](int j0, int count) {
    // every lane of the wave has written its slots: order those LDS writes
    // before the transposed reads (the wave's LDS operations execute in order)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int sg = sig < NQ * CHN ? sig : 0;     // groups past the slab read a valid one
    const T* src = slab + sg * 64 + prt * 16;
    T acc = T(0);
#pragma unroll
    for (int t = 0; t < 16; ++t) acc += src[t];
    acc += dpp_quad_swap1(acc);
    acc += dpp_quad_swap2(acc);
    const int slot = sig / NQ;
    if (prt == 0 && sig < NQ * CHN && slot < count) {
      const int j = j0 + slot;
      const int node = UP ? nd - 1 - j : j;
      out[(((row0 + node) * nw + it.g) * 2 + (UP ? 0 : 1)) * NQP + (sig % NQ)] = acc;
    }
    // the next chunk overwrites the slab: keep these reads before those writes
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  auto park = [&](int j, T jsum, T lsum, T band) {
    const int slot = j % CHN;
    slab[(NQ * slot + 0) * 64 + lane] = jsum;        // weighted already
    slab[(NQ * slot + 1) * 64 + lane] = lsum;
    if (TRI) slab[(NQ * slot + 2) * 64 + lane] = wp * band;
  };
  auto node_sum = [&]() {
    T js = T(0);
#pragma unroll
    for (int i = 0; i < NA; ++i) js += wh[i] * D[i];
    return js;
  };

  park(0, node_sum(), wp * ang.hwsum, T(0));
  int j0 = 0;
  // TRI: alpha of the previous layer in sweep order, per angle (0 before the
  // first layer: the boundary node's intensity does not depend on S)
  T aprev[TRI ? NA : 1];
#pragma unroll
  for (int i = 0; i < (TRI ? NA : 1); ++i) aprev[i] = T(0);
  // prefetch the next node of the sweep
  int dn = UP ? nd - 2 : 1;
  T qf = qat(row0 + dn);
  for (int j = 1; j < nd; ++j) {
    if (j % CHN == 0) {
      flush(j0, CHN);
      j0 = j;
    }
    const T qd = qf;
    // the layer between this node and its predecessor in sweep order spans
    // rows l, l+1: its reference depth and the source change across it
    const int64_t l = row0 + (UP ? nd - 1 - j : j - 1);
    const T dtl = dtr[l];
    const T dSl = dSr[l];
    if (j + 1 < nd) {
      dn = UP ? nd - 2 - j : j + 1;
      qf = qat(row0 + dn);
    }
    const T dt = (qd + qn) * dtl;             // dtl = half the reference depth
    const T dS = UP ? dSl : -dSl;
    T ls = T(0), band = T(0);
    if (TRI) {
      // with the neighbour coupling: the layer's alpha, gamma and e per angle
      // (accurate series for thin layers), band = 1/2 sum w (gamma + e alpha_prev).
      // FP32 decides the regime once per layer when every angle agrees in
      // every lane (the thresholds of sweep_layer), else per angle.
      const T inv = recip(dt);
      if constexpr (std::is_same<T, float>::value) {
        auto layer = [&](auto rc) {
          constexpr int R = decltype(rc)::value;
#pragma unroll
          for (int i = 0; i < NA; ++i) {
            float e, ps, al, ga;
            if constexpr (R == 0) layer_w_thin<true>(dt * ang.rmu[i], e, ps, al, ga);
            else if constexpr (R == 1) layer_w_thick<true>(dt, inv, ang.c[i], ang.mu[i], e, ps, al, ga);
            else layer_w<true>(dt, inv, ang.c[i], ang.rmu[i], ang.mu[i], e, ps, al, ga);
            D[i] = e * D[i] + ps * dS;
            ls += wh[i] * ps;
            band += ang.hw[i] * (ga + e * aprev[i]);
            aprev[i] = al;
          }
        };
        const unsigned long long act = __ballot(1);
        if (__ballot(dt < ang.dt_all_thin) == act) layer(std::integral_constant<int, 0>{});
        else if (__ballot(dt >= ang.dt_all_thick) == act) layer(std::integral_constant<int, 1>{});
        else layer(std::integral_constant<int, 2>{});
      } else {
#pragma unroll
        for (int i = 0; i < NA; ++i) {
          T e, ps, al, ga;
          layer_w<true>(dt, inv, ang.c[i], ang.rmu[i], ang.mu[i], e, ps, al, ga);
          D[i] = e * D[i] + ps * dS;
          ls += wh[i] * ps;
          band += ang.hw[i] * (ga + e * aprev[i]);
          aprev[i] = al;
        }
      }
    } else {
      sweep_layer(ang, wh, dt, dS, D, ls);
    }
    park(j, node_sum(), ls, band);
    qn = qd;
  }
  flush(j0, nd - j0);
}

template <typename T, int NA, bool TRI>
__global__ __launch_bounds__(512) void k_fs_profile(FsProfileArgs<T> a, Angles<T> ang) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  // the wave index is uniform over the wave: say so, so that the item, the
  // atmosphere's offsets and its per-row data are loaded and kept as scalars
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  T* slab = reinterpret_cast<T*>(lds_raw) +
            (size_t)wave * (ProfileLayout<TRI>::NQ * ProfileLayout<TRI>::CHN * 64);
  if (a.queue == nullptr) {
    const int item = (int)blockIdx.x * (int)(blockDim.x >> 6) + wave;
    if (item >= a.nitems) return;                       // whole wave
    const Item it = a.items[item];
    if (a.active != nullptr && a.active[it.b] == 0) return;   // whole wave
    if (it.dir == 0)
      profile_sweep<T, NA, true, TRI>(a, ang, it, slab);
    else
      profile_sweep<T, NA, false, TRI>(a, ang, it, slab);
    return;
  }
  // Persistent grid: every wave takes the next item (longest atmosphere
  // first) until the counter passes the end; the counter only grows, so every
  // wave leaves the loop.
  for (;;) {
    int item = 0;
    if ((threadIdx.x & 63) == 0) item = atomicAdd(a.queue, 1);
    item = __builtin_amdgcn_readfirstlane(item);
    if (item >= a.nitems) return;
    const Item it = a.items[item];
    if (a.active != nullptr && a.active[it.b] == 0) continue;
    if (it.dir == 0)
      profile_sweep<T, NA, true, TRI>(a, ang, it, slab);
    else
      profile_sweep<T, NA, false, TRI>(a, ang, it, slab);
  }
}

// Per-row differences for the batched sweep, rounded once to T:
//     dtr[r] = T(tau[r+1] - tau[r]) / 2,   dSr[r] = T(S[r+1] - S[r])
// (the last row has no successor: 0; rows that straddle two atmospheres are
// never read).  The halving is exact, so a layer's optical depth
// (q_d + q_{d+1}) dtr is the same number as 1/2 (q_d + q_{d+1}) T(dtau).
template <typename T>
__global__ __launch_bounds__(256) void k_row_diffs(const double* __restrict__ tau,
                                                   const double* __restrict__ S, int64_t rows,
                                                   T* __restrict__ dtr, T* __restrict__ dSr) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const bool last = r + 1 >= rows;
  dtr[r] = last ? T(0) : T(0.5) * T(tau[r + 1] - tau[r]);
  dSr[r] = last ? T(0) : T(S[r + 1] - S[r]);
}

template <typename T, int NA>
hipError_t launch_full_t(int wpb, int nitems, hipStream_t s, const void* args, const void* ang) {
  hipLaunchKernelGGL((k_fs_full<T, NA>), dim3(nitems), dim3(64 * wpb), 0, s,
                     *static_cast<const FsFullArgs<T>*>(args), *static_cast<const Angles<T>*>(ang));
  return hipGetLastError();
}

template <typename T, int NA>
hipError_t launch_profile_t(int wpb, int nitems, int nblocks, bool tri, hipStream_t s,
                            const void* args, const void* ang) {
  if (nblocks <= 0) nblocks = (nitems + wpb - 1) / wpb;
  const auto& A = *static_cast<const FsProfileArgs<T>*>(args);
  const auto& G = *static_cast<const Angles<T>*>(ang);
  if (tri) {
    const size_t lds = (size_t)wpb * ProfileLayout<true>::NQ * ProfileLayout<true>::CHN * 64 * sizeof(T);
    hipLaunchKernelGGL((k_fs_profile<T, NA, true>), dim3(nblocks), dim3(64 * wpb), lds, s, A, G);
  } else {
    const size_t lds = (size_t)wpb * ProfileLayout<false>::NQ * ProfileLayout<false>::CHN * 64 * sizeof(T);
    hipLaunchKernelGGL((k_fs_profile<T, NA, false>), dim3(nblocks), dim3(64 * wpb), lds, s, A, G);
  }
  return hipGetLastError();
}

#define PPRT_NA_LIST(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(12) X(16) X(24) X(32)

template <typename T>
hipError_t dispatch_full(int na, int wpb, int nitems, hipStream_t s, const void* a, const void* g) {
  switch (na) {
#define CASE(N) case N: return launch_full_t<T, N>(wpb, nitems, s, a, g);
    PPRT_NA_LIST(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}
template <typename T>
hipError_t dispatch_profile(int na, int wpb, int nitems, int nblocks, bool tri, hipStream_t s,
                            const void* a, const void* g) {
  switch (na) {
#define CASE(N) case N: return launch_profile_t<T, N>(wpb, nitems, nblocks, tri, s, a, g);
    PPRT_NA_LIST(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

bool na_supported(int na) {
  switch (na) {
#define CASE(N) case N: return true;
    PPRT_NA_LIST(CASE)
#undef CASE
    default: return false;
  }
}

hipError_t launch_fs_full(int precision, int na, int wpb, int nitems, hipStream_t s,
                          const void* args, const void* angles) {
  if (nitems == 0) return hipSuccess;
  return precision == PPRT_FP64 ? dispatch_full<double>(na, wpb, nitems, s, args, angles)
                                : dispatch_full<float>(na, wpb, nitems, s, args, angles);
}

hipError_t launch_row_diffs(int precision, const double* tau, const double* S, int64_t rows, void* dtr,
                            void* dSr, hipStream_t s) {
  if (rows == 0) return hipSuccess;
  const dim3 grid((unsigned)((rows + 255) / 256));
  if (precision == PPRT_FP64)
    hipLaunchKernelGGL(k_row_diffs<double>, grid, dim3(256), 0, s, tau, S, rows, (double*)dtr, (double*)dSr);
  else
    hipLaunchKernelGGL(k_row_diffs<float>, grid, dim3(256), 0, s, tau, S, rows, (float*)dtr, (float*)dSr);
  return hipGetLastError();
}

hipError_t launch_fs_profile(int precision, int na, int wpb, int nitems, int nblocks, bool tri,
                             hipStream_t s, const void* args, const void* angles) {
  if (nitems == 0) return hipSuccess;
  return precision == PPRT_FP64
             ? dispatch_profile<double>(na, wpb, nitems, nblocks, tri, s, args, angles)
             : dispatch_profile<float>(na, wpb, nitems, nblocks, tri, s, args, angles);
}

}  // namespace pprt

// Emergent intensity of the omega = 0 formal solution and its adjoint
// (vector-Jacobian product), with layer checkpointing.
//
// Forward: the up-going sweep of the linear short-characteristic solution
// (the 1D comparison calculation of the paper, Sect. 3.2), in difference form
//     D(d) = e D(d+1) + psi (S(d+1) - S(d)),     I+(tau_1) = D(1) + S(1),
// e = exp(-Delta), psi = (1 - e)/Delta, Delta = dtau_k / mu_i,
// dtau_k = (q(d) + q(d+1))/2 (tau(d+1) - tau(d)).  Every K-th node's D is kept
// in the workspace (a checkpoint); nothing else is stored.
//
// Adjoint: with lambda(d) = dL/dI+(d) and the plain form of the same update,
// I+(d) = e I+(d+1) + alpha S(d) + gamma S(d+1), alpha = 1 - psi, gamma = psi - e:
//     lambda(d+1)  = e lambda(d)
//     dL/dS(d)    += lambda(d) alpha          dL/dS(d+1) += lambda(d) gamma
//     dI+(d)/dDelta = -e D(d+1) - (gamma/Delta) (S(d+1) - S(d))
//     dL/d dtau_k  = sum_i lambda_i(d) dI+_i(d)/dDelta_i / mu_i
//     dL/dq(d), dL/dq(d+1) += (tau(d+1) - tau(d))/2 dL/d dtau_k
// and at the diffusion lower boundary I+ = Bbot + mu (Bbot - Bbot_prev)/dtau_k.
// The derivative is written with D = I - S and the source difference, so no
// term is a small difference of large intensities.  The backward sweep runs
// top-down one segment of K layers at a time: it recomputes the segment's D
// values upward from the checkpoint below it into registers, then walks the
// adjoint down through them.
//
// Mapping: one lane per (frequency, angle).  A wave holds 64/NAP frequencies
// of NAP lanes each (NAP = na rounded up to a power of two; lanes i >= na
// carry zeros).  The sums over angles are DPP reductions inside each NAP-lane
// group, so a single atmosphere of a few thousand frequencies already fills
// the chip with a wave per SIMD.
#include "pprt_internal.h"

// The reverse sweep recomputes D with the forward's exact operations, which
// makes the gradients independent of the checkpoint interval bit for bit;
// automatic fusion of a multiply and an add could differ between the two
// kernels, so every fused multiply-add here is written out and no other is made.
#pragma clang fp contract(off)

namespace pprt {
namespace {

template <typename T>
struct AdjW {
  T e, ps, al, ga, gd;   // gd = gamma / Delta
};

// FP32 weights.  Delta < 1/4: series (psi to Delta^5, alpha to Delta^6,
// gamma/Delta to Delta^6; truncation below 1e-7 relative), e = 1 - Delta psi
// and gamma = Delta psi - alpha exactly; otherwise closed forms with v_exp_f32.
__device__ __forceinline__ AdjW<float> adj_w(float dt, float c, float rmu, float mu) {
  const float D = dt * rmu;
  AdjW<float> w;
  if (D < 0.25f) {
    w.ps = fmaf(D, fmaf(D, fmaf(D, fmaf(D, fmaf(D, -1.f / 720.f, 1.f / 120.f), -1.f / 24.f),
                                1.f / 6.f), -0.5f), 1.f);
    w.al = D * fmaf(-D, fmaf(-D, fmaf(-D, fmaf(-D, fmaf(-D, 1.f / 5040.f, 1.f / 720.f),
                                                1.f / 120.f), 1.f / 24.f), 1.f / 6.f), 0.5f);
    w.e = fmaf(-D, w.ps, 1.f);
    w.ga = fmaf(D, w.ps, -w.al);
    w.gd = fmaf(D, fmaf(D, fmaf(D, fmaf(D, fmaf(D, fmaf(D, 1.f / 5760.f, -1.f / 840.f),
                                                1.f / 144.f), -1.f / 30.f), 1.f / 8.f),
                        -1.f / 3.f), 0.5f);
  } else {
    w.e = __builtin_amdgcn_exp2f(-(dt * c));
    const float m = mu / dt;
    w.ps = fmaf(-w.e, m, m);
    w.al = 1.f - w.ps;
    w.ga = w.ps - w.e;
    w.gd = w.ga * m;
  }
  return w;
}

// FP64 weights.  Delta < 1/10: nested series, alpha = (Delta/2) X with
// psi = 1 - (Delta/2) X, gamma/Delta = sum_m (m+1)(-Delta)^m/(m+2)! (terms to
// Delta^11, truncation below 1e-21); otherwise closed forms with expm1.
__device__ __forceinline__ AdjW<double> adj_w(double dt, double /*c*/, double rmu, double mu) {
  const double D = dt * rmu;
  AdjW<double> w;
  if (D < 0.1) {
    double X = 1.0;
#pragma unroll
    for (int n = 14; n >= 3; --n) X = fma(-D / n, X, 1.0);
    w.al = 0.5 * D * X;
    w.ps = 1.0 - w.al;
    w.e = fma(-D, w.ps, 1.0);
    w.ga = fma(D, w.ps, -w.al);
    // (m+1)/(m+2)! for m = 0..11
    constexpr double cm[12] = {1.0 / 2,        2.0 / 6,         3.0 / 24,         4.0 / 120,
                               5.0 / 720,      6.0 / 5040,      7.0 / 40320,      8.0 / 362880,
                               9.0 / 3628800,  10.0 / 39916800, 11.0 / 479001600, 12.0 / 6227020800.0};
    double g = cm[11];
#pragma unroll
    for (int m = 10; m >= 0; --m) g = fma(-D, g, cm[m]);
    w.gd = g;
  } else {
    w.e = exp(-D);
    const double m = mu / dt;
    w.ps = -expm1(-D) * m;
    w.al = 1.0 - w.ps;
    w.ga = w.ps - w.e;
    w.gd = w.ga * m;
  }
  return w;
}

template <int CTRL>
__device__ __forceinline__ float dppf(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dppf(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(u & 0xffffffffll), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over each aligned group of NAP lanes; the result is the same in every
// lane of the group (every addition is commutative pairwise, so all lanes
// see identical roundings).  All 64 lanes must be active.
template <int NAP, typename T>
__device__ __forceinline__ T group_sum(T v) {
  if (NAP >= 2) v += dppf<0xb1>(v);     // quad_perm [1,0,3,2]
  if (NAP >= 4) v += dppf<0x4e>(v);     // quad_perm [2,3,0,1]
  if (NAP >= 8) v += dppf<0x141>(v);    // row_half_mirror
  if (NAP >= 16) v += dppf<0x140>(v);   // row_mirror
  if (NAP >= 32) v += __shfl_xor(v, 16, 64);
  return v;
}

template <typename T, int NAP>
struct Lane {
  int k;          // frequency (clamped into range)
  int i;          // angle slot
  bool kval;      // frequency in range
  bool on;        // kval and i < na
  T mu, rmu, c;
};

template <typename T, int NAP>
__device__ __forceinline__ Lane<T, NAP> lane_of(const Item& it, const Angles<T>& A, int nf, int na) {
  constexpr int FPW = 64 / NAP;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wpb = blockDim.x >> 6;
  Lane<T, NAP> L;
  L.i = lane & (NAP - 1);
  const int kr = (it.g * wpb + wave) * FPW + lane / NAP;
  L.kval = kr < nf;
  L.k = L.kval ? kr : nf - 1;
  L.on = L.kval && L.i < na;
  L.mu = T(1);
  L.rmu = T(1);
  L.c = T(1.4426950408889634);
#pragma unroll
  for (int j = 0; j < NAP && j < kMaxNA; ++j)
    if (L.i == j && j < na) {
      L.mu = A.mu[j];
      L.rmu = A.rmu[j];
      L.c = A.c[j];
    }
  return L;
}

// D at the bottom node from the lower boundary condition.
template <typename T, int NAP>
__device__ __forceinline__ T bottom_D(const AdjArgs<T>& a, const Lane<T, NAP>& L, int b, T Sbot,
                                      T dt_last) {
  const int64_t bk = (int64_t)b * a.nf + L.k;
  if (a.lower_bc == PPRT_BC_DIFFUSION) {
    const T Bb = a.Bbot[bk], Bp = a.Bbot_prev[bk];
    return fma(L.mu, (Bb - Bp) / dt_last, Bb - Sbot);
  }
  if (!a.Ibot) return -Sbot;
  const int ic = L.i < a.na ? L.i : 0;
  return a.Ibot[bk * a.na + ic] - Sbot;
}

template <typename T, int NAP, int K>
__global__ __launch_bounds__(256) void k_emergent(AdjArgs<T> a, Angles<T> A) {
  const Item it = a.items[blockIdx.x];
  const Lane<T, NAP> L = lane_of<T, NAP>(it, A, a.nf, a.na);
  const int nf = a.nf, nd = it.nd, b = it.b;
  const int64_t o = a.off[b];
  const int64_t cko = a.ck_off[b];
  const T* q = a.q + L.k;
  const T* S = a.Sg + L.k;
  T S1 = S[(o + nd - 1) * nf], q1 = q[(o + nd - 1) * nf];
  T S0 = S[(o + nd - 2) * nf], q0 = q[(o + nd - 2) * nf];
  T dt = T(0.5) * (q0 + q1) * T(a.tau[o + nd - 1] - a.tau[o + nd - 2]);
  T Dc = bottom_D<T, NAP>(a, L, b, S1, dt);
  const int64_t ckrow = (int64_t)nf * a.na;
  const int64_t ckl = (int64_t)L.k * a.na + L.i;
  if ((nd - 1) % K == 0 && L.on) a.ckpt[(cko + (nd - 1) / K) * ckrow + ckl] = Dc;
  for (int d = nd - 2; d >= 0; --d) {
    T Sn = S0, qn = q0;
    if (d > 0) {
      Sn = S[(o + d - 1) * nf];
      qn = q[(o + d - 1) * nf];
    }
    dt = T(0.5) * (q0 + q1) * T(a.tau[o + d + 1] - a.tau[o + d]);
    const AdjW<T> w = adj_w(dt, L.c, L.rmu, L.mu);
    Dc = fma(w.e, Dc, w.ps * (S1 - S0));
    if ((unsigned)d % K == 0 && L.on) a.ckpt[(cko + d / K) * ckrow + ckl] = Dc;
    S1 = S0;
    q1 = q0;
    S0 = Sn;
    q0 = qn;
  }
  if (L.on) a.Iemerg[((int64_t)b * nf + L.k) * a.na + L.i] = Dc + S1;
}

// State carried down the adjoint walk.
template <typename T>
struct VjpState {
  T lam;        // dL/dI+ at the current node (per lane)
  T prev_gdt;   // angle-summed dL/d dtau_k of the layer above (uniform in the group)
  T prev_lg;    // lambda gamma of the layer above (per lane)
  T dtr_prev;   // reference thickness of the layer above
  T gBb, gBp;   // lower-boundary adjoints (per lane)
  T Sa, qa;     // inputs at the current node
};

// One segment of layers s .. s+len-1.  FULL: len == K, so every register
// index is static; otherwise the D(d+1) lookup is an unrolled select.
template <typename T, int NAP, int K, bool FULL>
__device__ __forceinline__ void vjp_segment(const AdjArgs<T>& a, const Lane<T, NAP>& L,
                                            VjpState<T>& st, int b, int s, int len_rt, int nd, int64_t o,
                                            int64_t cko, int64_t bk, bool diff, bool writer) {
  const int len = FULL ? K : len_rt;
  const int nf = a.nf;
  const T* q = a.q + L.k;
  const T* S = a.Sg + L.k;
  const int send = s + len;
  // ---- recompute D(send), D(send-1), .. D(s+1): Dbuf[r] = D(send - r)
  T Dbuf[K];
  T Sb = S[(o + send) * nf], qb = q[(o + send) * nf];
  if (send % K == 0) {
    Dbuf[0] = L.on ? a.ckpt[(cko + send / K) * ((int64_t)nf * a.na) + (int64_t)L.k * a.na + L.i]
                   : T(0);
  } else {   // send == nd - 1, not a checkpoint node: the boundary value
    const T qp = q[(o + send - 1) * nf];
    const T dtl = T(0.5) * (qp + qb) * T(a.tau[o + send] - a.tau[o + send - 1]);
    Dbuf[0] = L.on ? bottom_D<T, NAP>(a, L, b, Sb, dtl) : T(0);
  }
#pragma unroll
  for (int r = 1; r < K; ++r) {
    if (FULL || r < len) {
      const int n = send - r;
      const T Sn = S[(o + n) * nf], qn = q[(o + n) * nf];
      const T dt = T(0.5) * (qn + qb) * T(a.tau[o + n + 1] - a.tau[o + n]);
      const AdjW<T> w = adj_w(dt, L.c, L.rmu, L.mu);
      Dbuf[r] = fma(w.e, Dbuf[r - 1], w.ps * (Sb - Sn));
      Sb = Sn;
      qb = qn;
    }
  }
  // ---- adjoint walk down through layers s .. send-1
#pragma unroll
  for (int j = 0; j < K; ++j) {
    if (FULL || j < len) {
      const int d = s + j;
      const T Sd1 = S[(o + d + 1) * nf], qd1 = q[(o + d + 1) * nf];
      const T dtr = T(a.tau[o + d + 1] - a.tau[o + d]);
      const T dt = T(0.5) * (st.qa + qd1) * dtr;
      const AdjW<T> w = adj_w(dt, L.c, L.rmu, L.mu);
      T Dn;   // D(d+1) = Dbuf[len - 1 - j]
      if (FULL) {
        Dn = Dbuf[K - 1 - j];
      } else {
        Dn = Dbuf[0];
#pragma unroll
        for (int r = 1; r < K; ++r)
          if (r == len - 1 - j) Dn = Dbuf[r];
      }
      const T dS_lane = fma(st.lam, w.al, st.prev_lg);
      T gdt_lane = -st.lam * fma(w.e, Dn, w.gd * (Sd1 - st.Sa)) * L.rmu;
      const T lam_next = w.e * st.lam;
      if (d == nd - 2 && diff) {
        const T Bb = a.Bbot[bk], Bp = a.Bbot_prev[bk];
        const T m = L.mu / dt;
        gdt_lane = fma(-lam_next * m * (Bb - Bp), T(1) / dt, gdt_lane);
        st.gBb = lam_next * (T(1) + m);
        st.gBp = -lam_next * m;
      }
      st.prev_lg = st.lam * w.ga;
      st.lam = lam_next;
      const T gdt = group_sum<NAP>(gdt_lane);
      const T dSd = group_sum<NAP>(dS_lane);
      if (writer) {
        a.dq[(o + d) * nf + L.k] = T(0.5) * fma(st.dtr_prev, st.prev_gdt, dtr * gdt);
        a.dSg[(o + d) * nf + L.k] = dSd;
      }
      st.prev_gdt = gdt;
      st.dtr_prev = dtr;
      st.Sa = Sd1;
      st.qa = qd1;
    }
  }
}

template <typename T, int NAP, int K>
__global__ __launch_bounds__(256) void k_emergent_vjp(AdjArgs<T> a, Angles<T> A) {
  const Item it = a.items[blockIdx.x];
  const Lane<T, NAP> L = lane_of<T, NAP>(it, A, a.nf, a.na);
  const int nf = a.nf, nd = it.nd, b = it.b;
  const int64_t o = a.off[b];
  const int64_t cko = a.ck_off[b];
  const int64_t bk = (int64_t)b * nf + L.k;
  const bool diff = a.lower_bc == PPRT_BC_DIFFUSION;
  const bool writer = L.kval && L.i == 0;

  VjpState<T> st;
  st.lam = L.on ? a.gI[bk * a.na + L.i] : T(0);
  st.prev_gdt = 0;
  st.prev_lg = 0;
  st.dtr_prev = 0;
  st.gBb = 0;
  st.gBp = 0;
  st.Sa = a.Sg[o * nf + L.k];
  st.qa = a.q[o * nf + L.k];
  int s = 0;
  for (; s + K <= nd - 1; s += K)
    vjp_segment<T, NAP, K, true>(a, L, st, b, s, K, nd, o, cko, bk, diff, writer);
  if (s < nd - 1)
    vjp_segment<T, NAP, K, false>(a, L, st, b, s, nd - 1 - s, nd, o, cko, bk, diff, writer);
  // bottom node
  const T dSb = group_sum<NAP>(st.prev_lg);
  const T sBb = group_sum<NAP>(st.gBb);
  const T sBp = group_sum<NAP>(st.gBp);
  if (writer) {
    a.dq[(o + nd - 1) * nf + L.k] = T(0.5) * st.dtr_prev * st.prev_gdt;
    a.dSg[(o + nd - 1) * nf + L.k] = dSb;
    if (diff && a.dBbot) a.dBbot[bk] = sBb;
    if (diff && a.dBbot_prev) a.dBbot_prev[bk] = sBp;
  }
  if (!diff && a.dIbot && L.on) a.dIbot[bk * a.na + L.i] = st.lam;
}

template <typename T, int NAP, int K>
hipError_t launch_nap_k(bool vjp, int nitems, int wpb, hipStream_t s, const AdjArgs<T>& a,
                        const Angles<T>& A) {
  if (vjp)
    hipLaunchKernelGGL((k_emergent_vjp<T, NAP, K>), dim3(nitems), dim3(64 * wpb), 0, s, a, A);
  else
    hipLaunchKernelGGL((k_emergent<T, NAP, K>), dim3(nitems), dim3(64 * wpb), 0, s, a, A);
  return hipGetLastError();
}

template <typename T, int NAP>
hipError_t launch_nap(bool vjp, int K, int nitems, int wpb, hipStream_t s, const AdjArgs<T>& a,
                      const Angles<T>& A) {
  switch (K) {
    case 1: return launch_nap_k<T, NAP, 1>(vjp, nitems, wpb, s, a, A);
    case 8: return launch_nap_k<T, NAP, 8>(vjp, nitems, wpb, s, a, A);
    case 16: return launch_nap_k<T, NAP, 16>(vjp, nitems, wpb, s, a, A);
    case 32: return launch_nap_k<T, NAP, 32>(vjp, nitems, wpb, s, a, A);
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_t(bool vjp, int nap, int K, int nitems, int wpb, hipStream_t s,
                    const AdjArgs<T>& a, const Angles<T>& A) {
  switch (nap) {
    case 1: return launch_nap<T, 1>(vjp, K, nitems, wpb, s, a, A);
    case 2: return launch_nap<T, 2>(vjp, K, nitems, wpb, s, a, A);
    case 4: return launch_nap<T, 4>(vjp, K, nitems, wpb, s, a, A);
    case 8: return launch_nap<T, 8>(vjp, K, nitems, wpb, s, a, A);
    case 16: return launch_nap<T, 16>(vjp, K, nitems, wpb, s, a, A);
    case 32: return launch_nap<T, 32>(vjp, K, nitems, wpb, s, a, A);
  }
  return hipErrorInvalidValue;
}

}  // namespace

int adj_lanes_per_freq(int na) {
  int p = 1;
  while (p < na) p <<= 1;
  return p;
}

bool adj_interval_supported(int K) { return K == 1 || K == 8 || K == 16 || K == 32; }

hipError_t launch_emergent(int precision, bool vjp, int na, int K, int nitems, int wpb,
                           hipStream_t s, const void* args, const void* angles) {
  const int nap = adj_lanes_per_freq(na);
  if (precision == PPRT_FP64)
    return launch_t<double>(vjp, nap, K, nitems, wpb, s, *(const AdjArgs<double>*)args,
                            *(const Angles<double>*)angles);
  return launch_t<float>(vjp, nap, K, nitems, wpb, s, *(const AdjArgs<float>*)args,
                         *(const Angles<float>*)angles);
}

}  // namespace pprt

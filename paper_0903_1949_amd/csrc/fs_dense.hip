// Formal solution with coherent isotropic scattering inside the layers
// (omega > 0) on gfx950, FP64: exact homogeneous-layer operators t, r, beta
// from the discrete-ordinate eigen solution, the adding recursion down, a
// bottom-up adding pass, and the two-sided combination that yields I+-, J and
// the exact diagonal Lambda* at every node.
//
// Reading (the paper names t+-, r+-, beta+- and I+- in its notation and
// parameterises coherent isotropic continuum scattering, Sect. 3.1 item 6;
// the equations are deferred to its Papers I-II, Sect. 2): each layer is
// homogeneous with albedo omega = mean of its two node values and a source
// S^g linear in the layer optical depth; the total source is
// S = (1-omega) S^g + omega J.  Layer equations:
//     I+(d) = t I+(d+1) + r I-(d) + beta+,   I-(d+1) = t I-(d) + r I+(d+1) + beta-
// (a homogeneous layer has t+ = t-, r+ = r-).
//
// Layer operators.  In scaled intensities I^ = diag(sqrt w) I the homogeneous
// problem reduces to the symmetric matrix diag(1/mu^2) - omega u u^T,
// u_i = sqrt(w_i)/mu_i: its eigenvalues lambda = k^2 are the roots of the
// secular equation 1 = omega sum_j w_j / (1 - mu_j^2 lambda) (found with the
// origin at the nearer pole), and orthonormal eigenvectors V follow from the
// Gu & Eisenstat (1994) recomputed vector.  With M = diag(1/mu), D the layer
// optical depth, x = k D/2, Q_T = V diag(k tanh x) V^T,
// Q_C' = V diag(2 x coth x) V^T, F_T = (M + Q_T)^-1, F_C' = (D M + Q_C')^-1
// (both symmetric positive definite):
//     r^ = M (F_T + D F_C') - I,     t^ = M (F_T - D F_C'),
//     beta^_c  = 2 Q_T F_T sqrt(w)                        (unit constant S^g)
//     Qv       = 2 M F_C' (sqrt(w) mu)
//     beta^_l+ = Qv - t^ sqrt(w),    beta^_l- = (I - r^) sqrt(w) - Qv
//                                                         (unit node difference)
// exact for every thickness and for omega = 1 (k = 0 is regular), with no
// growing exponential and no 1/D.
//
// Mapping: NA lanes per frequency (lane i holds row i of every NA x NA matrix
// and element i of every vector), 64/NA frequencies per wave, one wave per
// block.  Matrix products broadcast the right operand through the group's LDS
// slab; the LDS operations of one wave execute in order and compiler fences
// keep the program order.  The Gauss-Jordan eliminations instead take each
// pivot row from its lane through the cross-lane permute and scale no row
// until the end (fewer instructions than a pivot lane that scales and stores
// its row while the other lanes wait).  The two passes are two kernels, each limited to
// 256 registers so that two waves share a SIMD (fewer spills than three); the
// eigen solutions of pass 1 (rows of V and the roots) stay in the workspace
// for pass 2, and each root's Newton iteration starts from the same lane's
// root of the previous layer.  Intensities travel in difference form
// D = I - S^g (scaled), whose layer sources are +-(S^g(d+1) - S^g(d)) Q with
// Q = beta_l+ + t sqrt(w), exact because a layer reproduces a constant S^g
// (beta_c + t sqrt(w) + r sqrt(w) = sqrt(w)); J - S^g and H then keep their
// relative accuracy where they are small.  Pass 1 (top -> bottom) stores the composite
// reflection R_d and source Sigma_d of every node in the workspace; pass 2
// (bottom -> top) rebuilds the layer operators from the kept eigen solutions, builds the composites R^up,
// Sigma^up of the layers below and emits the node outputs:
//     I+ = (I - R^up R)^-1 (R^up Sigma + Sigma^up),  I- = R I+ + Sigma,
// and the same combination of the unit-source responses of the two layers
// that touch the node gives Lambda*_dd = dJ(d)/dS^g(d) (plain form) and
// 1 - Lambda*_dd (difference form, so it stays accurate as Lambda* -> 1).
#include "pprt_internal.h"

namespace pprt {
namespace {

template <int NA>
struct DenseTab {
  // internal angle order: descending mu (ascending d = 1/mu^2)
  double mu[NA], m[NA], d[NA], z2[NA], w[NA], sw[NA], swmu[NA];
  int ext[NA];  // index of internal angle i in the caller's (ascending mu) order
};

__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A group's LDS slab.  Matrix rows are RS doubles apart: padded from NA >= 8
// on, so that the lanes' 16-byte row stores fall on different banks.  The
// slab stride is 2 (mod 16) doubles, so that the groups of a wave, which
// read the same offsets of their own slabs, touch disjoint 4-bank spans.
template <int NA>
struct Slab {
  static constexpr int RS = NA >= 8 ? NA + 2 : NA;
  static constexpr int MAT = (NA * RS > 2 * NA + 3) ? NA * RS : 2 * NA + 3;
  static constexpr int VEC = MAT;            // 4 vector slots of NA
  static constexpr int ROOT = MAT + 4 * NA;  // 2 NA: root origin and offset
  static constexpr int USED = MAT + 6 * NA;
  static constexpr int SIZE = USED + (18 - USED % 16) % 16;
};

// 1/x from the hardware reciprocal and two Newton-Raphson steps
// (r <- r + r (1 - x r)); for finite nonzero normal x, within 1 ulp
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// lane-group toolkit: lane i holds row i
template <int NA>
struct Grp {
  double* buf;
  int i;
  int b4;   // 4 x the group's first lane (permute address)

  __device__ __forceinline__ void put_mat(const double (&A)[NA]) {
    wsync();
#pragma unroll
    for (int j = 0; j < NA; ++j) buf[i * Slab<NA>::RS + j] = A[j];
    wsync();
  }
  __device__ __forceinline__ void put_vec(double v, int slot) {
    wsync();
    buf[Slab<NA>::VEC + slot * NA + i] = v;
    wsync();
  }
  __device__ __forceinline__ double vec(int j, int slot) const {
    return buf[Slab<NA>::VEC + slot * NA + j];
  }
  // C = A B
  __device__ __forceinline__ void mul(double (&C)[NA], const double (&A)[NA], const double (&B)[NA]) {
    put_mat(B);
    double acc[NA];
#pragma unroll
    for (int j = 0; j < NA; ++j) acc[j] = 0.0;
#pragma unroll
    for (int k = 0; k < NA; ++k) {
      const double a = A[k];
#pragma unroll
      for (int j = 0; j < NA; ++j) acc[j] = fma(a, buf[k * Slab<NA>::RS + j], acc[j]);
    }
#pragma unroll
    for (int j = 0; j < NA; ++j) C[j] = acc[j];
  }
  // (A x)_i
  __device__ __forceinline__ double mv(const double (&A)[NA], double x) {
    put_vec(x, 0);
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < NA; ++j) acc = fma(A[j], vec(j, 0), acc);
    return acc;
  }
  // sum over the group of v
  __device__ __forceinline__ double sum(double v) {
    put_vec(v, 1);
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < NA; ++j) acc += vec(j, 1);
    return acc;
  }
  // Gauss-Jordan elimination without pivoting on the rows [A | X | v] held
  // by the group's lanes (A is destroyed).  Step k takes row k from lane k
  // through the cross-lane permute (no LDS memory, no divergent pivot lane)
  // and subtracts A_ik / A_kk times it from every other row; the pivot row is
  // not scaled, so column k of A and the columns left of it are final after
  // step k and are not updated again.  Lane i divides its right-hand sides by
  // its own pivot at the end.  XM: 0 no matrix right-hand side, 1 X holds one
  // on entry, 2 X starts as the identity (X = A^-1 on exit; row k of X has
  // no entries right of column k at step k).
  __device__ __forceinline__ double from_lane(double v, int k) const {
    const int a = b4 + 4 * k;
    const int lo = __builtin_amdgcn_ds_bpermute(a, __double2loint(v));
    const int hi = __builtin_amdgcn_ds_bpermute(a, __double2hiint(v));
    return __hiloint2double(hi, lo);
  }
  template <int XM, int NB>
  __device__ __forceinline__ void gj(double (&A)[NA], double (&X)[NA], double (&v)[NB > 0 ? NB : 1]) {
    if constexpr (XM == 2) {
#pragma unroll
      for (int j = 0; j < NA; ++j) X[j] = (j == i) ? 1.0 : 0.0;
    }
    double own = 1.0;
#pragma unroll
    for (int k = 0; k < NA; ++k) {
      const double piv = from_lane(A[k], k);
      const double c = (i == k) ? 0.0 : A[k] * rcp_nr(piv);
      own = (i == k) ? piv : own;
#pragma unroll
      for (int j = k + 1; j < NA; ++j) A[j] = fma(-c, from_lane(A[j], k), A[j]);
      if constexpr (XM != 0) {
#pragma unroll
        for (int j = 0; j < (XM == 2 ? k + 1 : NA); ++j) X[j] = fma(-c, from_lane(X[j], k), X[j]);
      }
#pragma unroll
      for (int m = 0; m < NB; ++m) v[m] = fma(-c, from_lane(v[m], k), v[m]);
    }
    const double r = rcp_nr(own);
    if constexpr (XM != 0) {
#pragma unroll
      for (int j = 0; j < NA; ++j) X[j] *= r;
    }
#pragma unroll
    for (int m = 0; m < NB; ++m) v[m] *= r;
  }
  // X = A^-1; A is destroyed.  Used on symmetric positive definite matrices
  // and on I - (reflection products).
  __device__ __forceinline__ void inv(double (&X)[NA], double (&A)[NA]) {
    double v[1];
    gj<2, 0>(A, X, v);
  }
  // y1, y2, y3 with A y = b1, b2, b3; A is destroyed
  __device__ __forceinline__ void solve3(double (&A)[NA], double& b1, double& b2, double& b3) {
    double v[3] = {b1, b2, b3};
    gj<0, 3>(A, A, v);
    b1 = v[0]; b2 = v[1]; b3 = v[2];
  }
  // X <- A^-1 X (X holds the right-hand side's rows on entry); A is destroyed
  __device__ __forceinline__ void solve_mat(double (&X)[NA], double (&A)[NA]) {
    double v[1];
    gj<1, 0>(A, X, v);
  }
  // X <- A^-1 X and b0, b1, b2 <- A^-1 b0, b1, b2 (right-hand sides on
  // entry); A is destroyed
  __device__ __forceinline__ void solve_mat_v3(double (&X)[NA], double (&A)[NA], double& b0,
                                               double& b1, double& b2) {
    double v[3] = {b0, b1, b2};
    gj<1, 3>(A, X, v);
    b0 = v[0]; b1 = v[1]; b2 = v[2];
  }
};

template <int NA>
struct LaneTab {  // per-lane copies of the angle constants of row i
  double mu, m, d, z2, w, sw, swmu;
  int ext;
};


// ---- eigen solution of diag(d) - omega z z^T (d ascending) ------------------
// Lane i finds root i in (d_{i-1}, d_i) (d_{-1} = 0) as org + del, org the
// nearer end, by bracketed Newton on the secular function; the group then
// forms the Gu-Eisenstat vector and lane i keeps row i of V and its root.
template <int NA>
__device__ void eigen(Grp<NA>& g, const DenseTab<NA>& T, const LaneTab<NA>& L, double om,
                      double (&V)[NA], double& k_i, double& lam_prev) {
  const int i = g.i;
  double lo = 0.0;
#pragma unroll
  for (int j = 0; j < NA; ++j)
    if (j == i - 1) lo = T.d[j];
  const double hi = L.d;
  double org = hi, del = 0.0;
  const double om1 = 1.0 - om;
  if (om > 0.0) {
    // f(lam) = 1 - om sum z2_j/(d_j - lam), or for root 0 near lam = 0 the
    // equivalent (1 - om) - om lam sum w_j/(d_j - lam); both decrease in lam.
    auto feval = [&](double o, double sgn, double x, double& f, double& df) {
      double s = 0.0, s2 = 0.0;
      if (i == 0 && o == 0.0) {
#pragma unroll
        for (int j = 0; j < NA; ++j) {
          const double r = rcp_nr(T.d[j] - sgn * x);
          s = fma(T.w[j], r, s);
          s2 = fma(T.w[j] * T.d[j], r * r, s2);
        }
        f = om1 - om * x * s;
        df = -om * s2;
      } else {
#pragma unroll
        for (int j = 0; j < NA; ++j) {
          const double r = rcp_nr((T.d[j] - o) - sgn * x);
          s = fma(T.z2[j], r, s);
          s2 = fma(T.z2[j] * r, r, s2);
        }
        f = 1.0 - om * s;
        df = -om * s2;
      }
    };
    const double mid = 0.5 * (lo + hi);
    double fm, dfm;
    if (i == 0) feval(0.0, 1.0, mid, fm, dfm);
    else feval(lo, 1.0, mid - lo, fm, dfm);
    double sgn, xl, xh;
    if (fm > 0.0) { org = hi; sgn = -1.0; xl = 0.0; xh = hi - mid; }
    else { org = lo; sgn = 1.0; xl = 0.0; xh = mid - lo; }
    if (i == 0 && sgn > 0.0 && om1 <= 0.0) {
      del = 0.0;                       // omega = 1: the diffusion root is exactly 0
    } else {
      // start from the root of the previous layer (same frequency, nearly the
      // same omega) when it lies in this half of the interval, else mid-way
      const double xp = sgn * (lam_prev - org);
      double x = (xp > xl && xp < xh) ? xp : 0.5 * (xl + xh);
      for (int it = 0; it < 200; ++it) {
        double f, df;
        feval(org, sgn, x, f, df);
        // lam = org + sgn x is too small when f > 0
        if ((f > 0.0) == (sgn > 0.0)) xl = x; else xh = x;
        double xn = x - f * rcp_nr(df * sgn);
        // a converged step ends the iteration before the bracket test: at the
        // root (f == 0, or a step that rounds to nothing) the update above has
        // just moved a bracket end onto x, and the test would take a bisection
        // step away from it
        if (fabs(xn - x) <= 2e-16 * x) {
          x = xn;
          break;
        }
        if (!(xn > xl && xn < xh)) xn = 0.5 * (xl + xh);
        const double step = fabs(xn - x);
        x = xn;
        if (step <= 2e-16 * x || xh - xl <= 4e-16 * xh) break;
      }
      del = sgn * x;
    }
  }
  // broadcast roots
  wsync();
  g.buf[Slab<NA>::ROOT + 2 * i + 0] = org;
  g.buf[Slab<NA>::ROOT + 2 * i + 1] = del;
  wsync();
  const double lam = org + del;
  lam_prev = lam;
  k_i = sqrt(fmax(lam, 0.0));
  if (!(om > 0.0)) {
#pragma unroll
    for (int a = 0; a < NA; ++a) V[a] = (a == i) ? 1.0 : 0.0;
    return;
  }
  // Gu-Eisenstat: zhat_i^2 = prod_a (lam_a - d_i) / (-omega prod_{j != i} (d_j - d_i))
  double num = 1.0, den = -om;
#pragma unroll
  for (int a = 0; a < NA; ++a) {
    const double oa = g.buf[Slab<NA>::ROOT + 2 * a];
    const double da = g.buf[Slab<NA>::ROOT + 2 * a + 1];
    num *= (oa - L.d) + da;
    if (a != i) den *= (T.d[a] - L.d);
  }
  const double zh = sqrt(fabs(num / den));
  g.put_vec(zh, 2);
  // column norm of eigenvector i: sum_j zh_j^2 / (d_j - lam_i)^2
  double nrm = 0.0;
#pragma unroll
  for (int j = 0; j < NA; ++j) {
    const double q = g.vec(j, 2) * rcp_nr((T.d[j] - org) - del);
    nrm = fma(q, q, nrm);
  }
  g.put_vec(1.0 / sqrt(nrm), 3);
#pragma unroll
  for (int a = 0; a < NA; ++a) {
    const double oa = g.buf[Slab<NA>::ROOT + 2 * a];
    const double da = g.buf[Slab<NA>::ROOT + 2 * a + 1];
    V[a] = zh * rcp_nr((L.d - oa) - da) * g.vec(a, 3);
  }
}

// x / tanh(x) for x >= 0, series below 0.05
__device__ __forceinline__ double x_coth_x(double x) {
  if (x < 0.05) {
    const double x2 = x * x;
    return 1.0 + x2 * (1.0 / 3.0 + x2 * (-1.0 / 45.0 + x2 * (2.0 / 945.0)));
  }
  return x / tanh(x);
}

// Layer operators in scaled variables (row i in this lane).
template <int NA>
struct LayerOps {
  double t[NA], r[NA];
  double bc, blp, blm;  // element i of beta_c, beta_l+, beta_l-
  double qv;            // element i of Q = beta_l+ + t sqrt(w) (difference-form source)
};

template <int NA>
__device__ void layer_ops(Grp<NA>& g, const DenseTab<NA>& T, const LaneTab<NA>& L,
                          const double (&V)[NA], double k_i, double Dl, LayerOps<NA>& o) {
  const int i = g.i;
  // per-root factors of root i, broadcast
  const double x = 0.5 * k_i * Dl;
  const double tx = k_i * tanh(x);
  const double cx = 2.0 * x_coth_x(x);
  g.put_vec(tx, 2);
  g.put_vec(cx, 3);
  // Q_T = V diag(tx) V^T and Q_C' = V diag(cx) V^T: broadcast V
  g.put_mat(V);
  // one matrix at a time (fewer live registers): Q_T, then M + Q_T and its
  // inverse, then D M + Q_C' and its inverse.  The eliminations leave the
  // slab alone, so putting V there again changes no value; its fences keep
  // the compiler from interleaving the second product with the first
  // inversion, which without them spills 69 registers in pass 1 (15% slower)
  double QT[NA], FT[NA], FC[NA];
  {
    double vt[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) vt[a] = V[a] * g.vec(a, 2);
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      double st = 0.0;
#pragma unroll
      for (int a = 0; a < NA; ++a) st = fma(vt[a], g.buf[j * Slab<NA>::RS + a], st);
      QT[j] = st;
    }
  }
  {
    double AT[NA];
#pragma unroll
    for (int j = 0; j < NA; ++j) AT[j] = QT[j];
    AT[i] += L.m;               // M + Q_T      (lane-dependent diagonal)
    g.inv(FT, AT);
  }
  g.put_mat(V);
  {
    double vc[NA], AC[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) vc[a] = V[a] * g.vec(a, 3);
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      double sc = 0.0;
#pragma unroll
      for (int a = 0; a < NA; ++a) sc = fma(vc[a], g.buf[j * Slab<NA>::RS + a], sc);
      AC[j] = sc;
    }
    AC[i] += Dl * L.m;          // D M + Q_C'
    g.inv(FC, AC);
  }
  double tw = 0.0, rw = 0.0, fw = 0.0, qv = 0.0;
#pragma unroll
  for (int j = 0; j < NA; ++j) {
    const double ft = FT[j], fc = Dl * FC[j];
    o.r[j] = L.m * (ft + fc) - ((j == i) ? 1.0 : 0.0);
    o.t[j] = L.m * (ft - fc);
    tw = fma(o.t[j], T.sw[j], tw);
    rw = fma(o.r[j], T.sw[j], rw);
    fw = fma(ft, T.sw[j], fw);
    qv = fma(FC[j], T.swmu[j], qv);
  }
  qv *= 2.0 * L.m;
  o.qv = qv;
  o.bc = 2.0 * g.mv(QT, fw);
  o.blp = qv - tw;
  o.blm = (L.sw - rw) - qv;
}

template <int NA>
struct FsDenseArgs {
  const Item* items;
  const int64_t* off;
  const double* tau;
  const double* q;
  const double* Sg;
  const double* omega;
  const double* Itop;
  const double* Bbot;
  const double* Bbot_prev;
  const double* Ibot;
  double *J, *JmS, *lstar, *lstar_c, *Iplus, *Iminus, *H, *Iemerg;
  double* wsR;     // [rows][nf][NA][NA]
  double* wsS;     // [rows][nf][NA]
  double* wsV;     // [rows][nf][NA][NA+1]: eigen solution of layer (d, d+1), row i and root k_i
  double* wsZ;     // [rows][nf][NA][2]: R_d G_d beta+ and R_d G_d Q of layer (d, d+1), element i
  uint32_t* status; // device status word: NONFINITE when an output is not finite
  int32_t nf;
  int32_t nitems;
  int32_t lower_bc;
  uint32_t outputs;
};

// PASS 1: the adding recursion down (composites R, Sigma and the layers'
// eigen solutions into the workspace); PASS 2: the pass up with the outputs.
// Two kernels, so that each holds only its own pass's registers.
template <int NA, int PASS>
__global__ __launch_bounds__(64, 2) void k_fs_dense(FsDenseArgs<NA> a, DenseTab<NA> T) {
  constexpr int F = 64 / NA;
  __shared__ double slab[F * Slab<NA>::SIZE];
  const int lane = (int)threadIdx.x;
  const int grp = lane / NA;
  const int item = (int)blockIdx.x;
  if (item >= a.nitems) return;
  const Item it = a.items[item];
  const int b = it.b;
  const int nd = it.nd;
  const int nf = a.nf;
  const int k = it.g * F + grp;
  if (k >= nf) return;   // a whole group: groups never talk to each other
  const int64_t row0 = a.off[b];
  Grp<NA> g{slab + grp * Slab<NA>::SIZE, lane % NA, 4 * (lane - lane % NA)};
  const int i = g.i;
  LaneTab<NA> L{};
#pragma unroll
  for (int j = 0; j < NA; ++j)
    if (j == i) {
      L.mu = T.mu[j]; L.m = T.m[j]; L.d = T.d[j]; L.z2 = T.z2[j]; L.w = T.w[j];
      L.sw = T.sw[j]; L.swmu = T.swmu[j]; L.ext = T.ext[j];
    }
  const uint32_t o = a.outputs;
  auto at = [&](const double* p, int64_t row) { return p[row * nf + k]; };
  auto layer_depth = [&](int d) {   // optical depth of layer (d, d+1)
    return 0.5 * (at(a.q, row0 + d) + at(a.q, row0 + d + 1)) * (a.tau[row0 + d + 1] - a.tau[row0 + d]);
  };
  auto layer_omega = [&](int d) {
    return a.omega ? 0.5 * (at(a.omega, row0 + d) + at(a.omega, row0 + d + 1)) : 0.0;
  };
  double* wsR = a.wsR + ((row0 * nf + k) * NA + i) * NA;   // + node * nf * NA * NA
  double* wsS = a.wsS + (row0 * nf + k) * NA + i;           // + node * nf * NA
  const int64_t strideR = (int64_t)nf * NA * NA;
  const int64_t strideS = (int64_t)nf * NA;
  double* wsV = a.wsV + ((row0 * nf + k) * NA + i) * (NA + 1);   // + layer * nf * NA * (NA + 1)
  const int64_t strideV = (int64_t)nf * NA * (NA + 1);
  double* wsZ = a.wsZ + ((row0 * nf + k) * NA + i) * 2;          // + layer * nf * NA * 2
  const int64_t strideZ = (int64_t)nf * NA * 2;
  // the unit-source responses behind Lambda* (plain form) and 1 - Lambda*
  // (difference form) are formed only for the outputs that are wanted
  const bool wd = (o & PPRT_OUT_LSTAR) != 0;
  const bool we = (o & PPRT_OUT_LSTAR_C) != 0;

  double V[NA];
  double kk = 0.0;
  double om_prev = -1.0;
  double lam_prev = -1.0;     // root of the last eigen solution (none yet)
  LayerOps<NA> op;

  if constexpr (PASS == 1) {
  // ---------------- pass 1: adding recursion, top -> bottom
  double R[NA];
#pragma unroll
  for (int j = 0; j < NA; ++j) R[j] = 0.0;
  // difference form: D = I - S^g, scaled by sqrt(w)
  double Sig = L.sw * ((a.Itop ? a.Itop[((int64_t)b * nf + k) * NA + L.ext] : 0.0) - at(a.Sg, row0));
  for (int d = 0; d < nd - 1; ++d) {
#pragma unroll
    for (int j = 0; j < NA; ++j) wsR[d * strideR + j] = R[j];
    wsS[d * strideS] = Sig;
    const double om = layer_omega(d);
    if (om != om_prev) {
      eigen<NA>(g, T, L, om, V, kk, lam_prev);
      om_prev = om;
    }
#pragma unroll
    for (int j = 0; j < NA; ++j) wsV[d * strideV + j] = V[j];
    wsV[d * strideV + NA] = kk;
    const double Dl = layer_depth(d);
    layer_ops<NA>(g, T, L, V, kk, Dl, op);
    const double dSg = at(a.Sg, row0 + d + 1) - at(a.Sg, row0 + d);
    const double bp = dSg * op.qv;        // difference-form layer sources
    const double bm = -dSg * op.qv;
    // G = (I - r R)^-1: P = G t, u = G (r Sigma + beta+), and for pass 2's
    // unit responses G beta_l+ and G Q, from one elimination on I - r R
    double X[NA], P[NA];
    g.mul(X, op.r, R);
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      X[j] = ((j == i) ? 1.0 : 0.0) - X[j];
      P[j] = op.t[j];
    }
    double u = g.mv(op.r, Sig) + bp;
    double y1 = op.blp, y2 = op.qv;
    g.solve_mat_v3(P, X, u, y1, y2);
    if (wd) wsZ[d * strideZ] = g.mv(R, y1);
    if (we) wsZ[d * strideZ + 1] = g.mv(R, y2);
    // Sigma_{d+1} = t (Sigma + R u) + beta-,  R_{d+1} = r + t R P
    const double Ru = g.mv(R, u);
    const double Sig_n = g.mv(op.t, Sig + Ru) + bm;
    double RP[NA], tRP[NA];
    g.mul(RP, R, P);
    g.mul(tRP, op.t, RP);
#pragma unroll
    for (int j = 0; j < NA; ++j) R[j] = op.r[j] + tRP[j];
    Sig = Sig_n;
  }
#pragma unroll
  for (int j = 0; j < NA; ++j) wsR[(nd - 1) * strideR + j] = R[j];
  wsS[(nd - 1) * strideS] = Sig;
  } else {
  // ---------------- pass 2: bottom -> top, outputs per node
  bool nonfinite = false;
  double Rup[NA];
#pragma unroll
  for (int j = 0; j < NA; ++j) Rup[j] = 0.0;
  double Sup;
  {
    const int64_t rl = row0 + nd - 1;
    const double S_last = at(a.Sg, rl);
    if (a.lower_bc == PPRT_BC_DIFFUSION) {
      const double Bb = a.Bbot[(int64_t)b * nf + k];
      const double Bp = a.Bbot_prev[(int64_t)b * nf + k];
      const double gr = (Bb - Bp) / layer_depth(nd - 2);
      Sup = L.sw * ((Bb - S_last) + L.mu * gr);
    } else {
      Sup = L.sw * ((a.Ibot ? a.Ibot[((int64_t)b * nf + k) * NA + L.ext] : 0.0) - S_last);
    }
    (void)rl;
  }
  double dSu = 0.0;           // dSigma^up of the node being emitted (layer below)
  double eSu = -L.sw;         // its difference-form counterpart (lower boundary: -1)
  om_prev = -1.0;
  for (int d = nd - 1; d >= 0; --d) {
    const bool has_a = d >= 1;  // layer a = (d-1, d) above node d
    if (has_a) {      // the eigen solution of layer a, kept by pass 1
#pragma unroll
      for (int j = 0; j < NA; ++j) V[j] = wsV[(d - 1) * strideV + j];
      kk = wsV[(d - 1) * strideV + NA];
      layer_ops<NA>(g, T, L, V, kk, layer_depth(d - 1), op);
    }
    // ---- emit node d
    double Rd[NA];
#pragma unroll
    for (int j = 0; j < NA; ++j) Rd[j] = wsR[d * strideR + j];
    const double Sd = wsS[d * strideS];
    // unit response: layer above (S^g 0 -> 1) through R_{d-1}, G_{d-1}; in
    // plain form (dS, for Lambda*) and in difference form (eS, sources +-Q
    // and -1 at a boundary, for 1 - Lambda* with full relative accuracy)
    // (each response only when its output is wanted: wd, we are uniform)
    double dS = 0.0, eS = -L.sw;
    if (has_a) {      // R_{d-1} G_{d-1} (dbeta+_a, Q_a), kept by pass 1
      if (wd) dS = g.mv(op.t, wsZ[(d - 1) * strideZ]) + op.blm;
      if (we) eS = g.mv(op.t, wsZ[(d - 1) * strideZ + 1]) - op.qv;
    }
    // I+ and the two responses from one elimination on I - R^up R_d
    double Ip = g.mv(Rup, Sd) + Sup;
    double dIp = wd ? g.mv(Rup, dS) + dSu : 0.0;
    double eDp = we ? g.mv(Rup, eS) + eSu : 0.0;
    {
      double X[NA];
      g.mul(X, Rup, Rd);
#pragma unroll
      for (int j = 0; j < NA; ++j) X[j] = ((j == i) ? 1.0 : 0.0) - X[j];
      g.solve3(X, Ip, dIp, eDp);
    }
    const double Im = g.mv(Rd, Ip) + Sd;
    // Ip, Im are the scaled differences D+- = sqrt(w) (I+- - S^g)
    const double JmSn = 0.5 * g.sum(L.sw * (Ip + Im));
    double Ln = 0.0, Lcn = 0.0;
    if (wd) {
      const double dIm = g.mv(Rd, dIp) + dS;
      Ln = 0.5 * g.sum(L.sw * (dIp + dIm));
    }
    if (we) {
      const double eDm = g.mv(Rd, eDp) + eS;
      Lcn = -0.5 * g.sum(L.sw * (eDp + eDm));
    }
    const double Hn = 0.5 * g.sum(L.swmu * (Ip - Im));
    // a zero or non-finite pivot in any elimination ends up here
    nonfinite |= !isfinite(Ip + Im + Ln + Lcn);
    {
      const int64_t x = (row0 + d) * nf + k;
      const double S = a.Sg[x];
      if (i == 0) {
        if (o & PPRT_OUT_J) a.J[x] = JmSn + S;
        if (o & PPRT_OUT_JMS) a.JmS[x] = JmSn;
        if (o & PPRT_OUT_LSTAR) a.lstar[x] = Ln;
        if (o & PPRT_OUT_LSTAR_C) a.lstar_c[x] = Lcn;
        if (o & PPRT_OUT_H) a.H[x] = Hn;
      }
      if (o & PPRT_OUT_IPLUS) a.Iplus[x * NA + L.ext] = Ip / L.sw + S;
      if (o & PPRT_OUT_IMINUS) a.Iminus[x * NA + L.ext] = Im / L.sw + S;
      if (d == 0 && (o & PPRT_OUT_IEMERG))
        a.Iemerg[((int64_t)b * nf + k) * NA + L.ext] = Ip / L.sw + S;
    }
    // ---- move the lower composite up through layer a
    if (has_a) {
      const double dSg = at(a.Sg, row0 + d) - at(a.Sg, row0 + d - 1);
      const double bp = dSg * op.qv;
      const double bm = -dSg * op.qv;
      // R^up G^up = R^up (I - r R^up)^-1 = (I - R^up r)^-1 R^up
      double Y[NA], RG[NA];
      g.mul(Y, Rup, op.r);
#pragma unroll
      for (int j = 0; j < NA; ++j) {
        Y[j] = ((j == i) ? 1.0 : 0.0) - Y[j];
        RG[j] = Rup[j];
      }
      g.solve_mat(RG, Y);
      const double w1 = g.mv(RG, g.mv(op.r, Sup) + bm);
      const double Sup_n = g.mv(op.t, Sup + w1) + bp;
      // unit response of layer a seen from node d-1 (S^g 1 -> 0)
      const double dbm = op.bc - op.blm, dbp = op.bc - op.blp;
      if (wd) dSu = g.mv(op.t, g.mv(RG, dbm)) + dbp;
      if (we) eSu = g.mv(op.t, g.mv(RG, op.qv)) - op.qv;
      double RGt[NA], tRGt[NA];
      g.mul(RGt, RG, op.t);
      g.mul(tRGt, op.t, RGt);
#pragma unroll
      for (int j = 0; j < NA; ++j) Rup[j] = op.r[j] + tRGt[j];
      Sup = Sup_n;
    }
  }
  if (nonfinite && a.status) atomicOr(a.status, PPRT_DEV_NONFINITE);
  }
}

template <int NA>
hipError_t launch_dense_t(int nitems, hipStream_t s, const void* args, const void* tab) {
  hipLaunchKernelGGL((k_fs_dense<NA, 1>), dim3(nitems), dim3(64), 0, s,
                     *static_cast<const FsDenseArgs<NA>*>(args), *static_cast<const DenseTab<NA>*>(tab));
  hipLaunchKernelGGL((k_fs_dense<NA, 2>), dim3(nitems), dim3(64), 0, s,
                     *static_cast<const FsDenseArgs<NA>*>(args), *static_cast<const DenseTab<NA>*>(tab));
  return hipGetLastError();
}

template <int NA>
void fill_tab(DenseTab<NA>& T, const double* mu_asc, const double* w_asc) {
  // internal order: descending mu
  for (int i = 0; i < NA; ++i) {
    const int e = NA - 1 - i;
    const double m = mu_asc[e], w = w_asc[e];
    T.mu[i] = m; T.m[i] = 1.0 / m; T.d[i] = 1.0 / (m * m); T.w[i] = w;
    T.z2[i] = w / (m * m); T.sw[i] = sqrt(w); T.swmu[i] = sqrt(w) * m; T.ext[i] = e;
  }
}

template <int NA>
hipError_t run_dense(const DenseLaunch& L, hipStream_t s) {
  FsDenseArgs<NA> a{};
  a.items = L.items; a.off = L.off; a.tau = L.tau; a.q = L.q; a.Sg = L.Sg; a.omega = L.omega;
  a.Itop = L.Itop; a.Bbot = L.Bbot; a.Bbot_prev = L.Bbot_prev; a.Ibot = L.Ibot;
  a.J = L.J; a.JmS = L.JmS; a.lstar = L.lstar; a.lstar_c = L.lstar_c; a.Iplus = L.Iplus;
  a.Iminus = L.Iminus; a.H = L.H; a.Iemerg = L.Iemerg;
  a.wsR = L.ws;
  a.wsS = L.ws + (size_t)L.rows * L.nf * NA * NA;
  a.wsV = a.wsS + (size_t)L.rows * L.nf * NA;
  a.wsZ = a.wsV + (size_t)L.rows * L.nf * NA * (NA + 1);
  a.nf = L.nf; a.nitems = L.nitems; a.lower_bc = L.lower_bc; a.outputs = L.outputs;
  a.status = L.status;
  DenseTab<NA> T{};
  fill_tab<NA>(T, L.mu, L.w);
  return launch_dense_t<NA>(L.nitems, s, &a, &T);
}

}  // namespace

bool dense_na_supported(int na) { return na == 1 || na == 2 || na == 4 || na == 8 || na == 16; }

size_t dense_workspace_bytes(int na, int64_t rows, int nf) {
  return (size_t)rows * nf * (size_t)(2 * na * na + 4 * na) * sizeof(double);
}

int dense_freqs_per_item(int na) { return 64 / na; }

hipError_t launch_fs_dense(const DenseLaunch& L, hipStream_t s) {
  if (L.nitems == 0) return hipSuccess;
  switch (L.na) {
    case 1: return run_dense<1>(L, s);
    case 2: return run_dense<2>(L, s);
    case 4: return run_dense<4>(L, s);
    case 8: return run_dense<8>(L, s);
    case 16: return run_dense<16>(L, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pprt

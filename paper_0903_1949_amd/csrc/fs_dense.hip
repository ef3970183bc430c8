// Formal solution with coherent isotropic scattering inside the layers
// (omega > 0) on gfx950, in FP64 or with an FP32 bulk: exact homogeneous-layer
// operators t, r, beta
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
// layer operators of pass 1 (rows of t and r, elements of the source vectors,
// in the bulk type) stay in the workspace for pass 2, which would otherwise
// form them again (a quarter of the formal solution), and each root's Newton
// iteration starts from the same lane's root of the previous layer.  Intensities travel in difference form
// D = I - S^g (scaled), whose layer sources are +-(S^g(d+1) - S^g(d)) Q with
// Q = beta_l+ + t sqrt(w), exact because a layer reproduces a constant S^g
// (beta_c + t sqrt(w) + r sqrt(w) = sqrt(w)); J - S^g and H then keep their
// relative accuracy where they are small.  Pass 1 (top -> bottom) stores the composite
// reflection R_d and source Sigma_d of every node in the workspace; pass 2
// (bottom -> top) takes the kept layer operators, builds the composites R^up,
// Sigma^up of the layers below and emits the node outputs:
//     I+ = (I - R^up R)^-1 (R^up Sigma + Sigma^up),  I- = R I+ + Sigma,
// and the same combination of the unit-source responses of the two layers
// that touch the node gives Lambda*_dd = dJ(d)/dS^g(d) (plain form) and
// 1 - Lambda*_dd (difference form, so it stays accurate as Lambda* -> 1).
//
// Precision.  The kernels are templated on the bulk type T.  T = double is
// FP64 throughout.  T = float keeps every array, composite, product and the
// adding recursion in FP32, but forms each layer's operators in FP64 and
// rounds them: in a thin, nearly conservative layer the absorption that
// t and r carry is a small difference of the large non-diffusive modes, and
// the matrix products V diag(.) V^T of an FP32 layer solution bury it in
// rounding (the diffusion eigenvalue is ~(1 - omega) of the others), which
// the recursion then accumulates over many layers.  Pass 1 keeps the rounded
// operators for pass 2, which forms the FP64 ones again only for the layers
// whose elimination runs in FP64.  The eliminations with I - (reflection)(reflection)
// -- G = (I - r R_d)^-1 of the way down, (I - R^up r)^-1 and (I - R^up R_d)^-1
// of the way up -- run in FP64 where the thick-layer rule asks for it: the layer's
// absorption depth D (1 - omega)^1/2 exceeds 1, or the bound |r|_inf |R|_inf
// of |r R| exceeds 1/2 (its spectral radius, and with it the conditioning of
// I - r R, is then no longer safely away from 1).  In FP64 the product r R is
// accumulated from the FP32 operands (exact products) and the right-hand
// sides are formed in FP64 before the elimination; results are rounded back
// to FP32.  The decision is taken per wave (FP64 when any of its frequency
// groups qualifies) so the branch stays uniform; a mode switch forces FP64 or
// FP32 everywhere for error studies, and per-wave counters record how many
// eliminations ran in FP64.
#include <type_traits>

#include "pprt_internal.h"

namespace pprt {
namespace {

// ---- scalar helpers per bulk type -------------------------------------------
// 1/x from the hardware reciprocal and Newton-Raphson steps (r <- r + r (1 - x r)):
// two for double, one for float; for finite nonzero normal x within 1 ulp
__device__ __forceinline__ double rcpT(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float rcpT(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
}
__device__ __forceinline__ double fmaT(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float fmaT(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double sqrtT(double x) { return sqrt(x); }
__device__ __forceinline__ float sqrtT(float x) { return sqrtf(x); }
__device__ __forceinline__ double tanhT(double x) { return tanh(x); }
__device__ __forceinline__ float tanhT(float x) { return tanhf(x); }
__device__ __forceinline__ double absT(double x) { return fabs(x); }
__device__ __forceinline__ float absT(float x) { return fabsf(x); }
__device__ __forceinline__ double maxT(double a, double b) { return fmax(a, b); }
__device__ __forceinline__ float maxT(float a, float b) { return fmaxf(a, b); }
template <typename T>
constexpr T epsT() { return std::is_same<T, double>::value ? (T)0x1p-52 : (T)0x1p-23f; }

// value of v in lane `a / 4` (a = 4 x source lane) through the cross-lane permute
__device__ __forceinline__ double permute(int a, double v) {
  const int lo = __builtin_amdgcn_ds_bpermute(a, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(a, __double2hiint(v));
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float permute(int a, float v) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(a, __float_as_int(v)));
}

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

// A group's LDS slab in elements of type T.  Matrix rows are RS elements
// apart: padded by 16 bytes from NA >= 8 on, so that the lanes' 16-byte row
// stores fall on different banks.  The slab stride is 16 bytes more than a
// multiple of 128 bytes, so that the groups of a wave, which read the same
// offsets of their own slabs, touch disjoint bank spans.  The kernels size
// the slabs for double; a float group uses the first half of its double slab.
template <typename T, int NA>
struct Slab {
  static constexpr int PADW = 16 / (int)sizeof(T);
  static constexpr int LINE = 128 / (int)sizeof(T);
  static constexpr int RS = NA >= 8 ? NA + PADW : NA;
  static constexpr int MAT = (NA * RS > 2 * NA + 3) ? NA * RS : 2 * NA + 3;
  static constexpr int VEC = MAT;            // 4 vector slots of NA
  static constexpr int ROOT = MAT + 4 * NA;  // 2 NA: root origin and offset
  static constexpr int USED = MAT + 6 * NA;
  static constexpr int SIZE = USED + (PADW + LINE - USED % LINE) % LINE;
};
static_assert(Slab<float, 16>::USED <= 2 * Slab<double, 16>::SIZE, "float slab fits its double slab");
static_assert(Slab<float, 1>::USED <= 2 * Slab<double, 1>::SIZE, "float slab fits its double slab");

// lane-group toolkit in precision T: lane i holds row i.  Operands of another
// type are converted as they are read (float -> double is exact).
template <typename T, int NA>
struct Grp {
  T* buf;
  int i;
  int b4;   // 4 x the group's first lane (permute address)
  static constexpr int RS = Slab<T, NA>::RS;

  template <typename S>
  __device__ __forceinline__ void put_mat(const S (&A)[NA]) {
    wsync();
#pragma unroll
    for (int j = 0; j < NA; ++j) buf[i * RS + j] = (T)A[j];
    wsync();
  }
  __device__ __forceinline__ void put_vec(T v, int slot) {
    wsync();
    buf[Slab<T, NA>::VEC + slot * NA + i] = v;
    wsync();
  }
  __device__ __forceinline__ T vec(int j, int slot) const {
    return buf[Slab<T, NA>::VEC + slot * NA + j];
  }
  // C = A B
  template <typename SA, typename SB>
  __device__ __forceinline__ void mul(T (&C)[NA], const SA (&A)[NA], const SB (&B)[NA]) {
    put_mat(B);
    T acc[NA];
#pragma unroll
    for (int j = 0; j < NA; ++j) acc[j] = (T)0;
#pragma unroll
    for (int k = 0; k < NA; ++k) {
      const T a = (T)A[k];
#pragma unroll
      for (int j = 0; j < NA; ++j) acc[j] = fmaT(a, buf[k * RS + j], acc[j]);
    }
#pragma unroll
    for (int j = 0; j < NA; ++j) C[j] = acc[j];
  }
  // (A x)_i
  template <typename SA>
  __device__ __forceinline__ T mv(const SA (&A)[NA], T x) {
    put_vec(x, 0);
    T acc = (T)0;
#pragma unroll
    for (int j = 0; j < NA; ++j) acc = fmaT((T)A[j], vec(j, 0), acc);
    return acc;
  }
  // (A^T x)_i
  __device__ __forceinline__ T mvT(const T (&A)[NA], T x) {
    put_mat(A);
    put_vec(x, 0);
    T acc = (T)0;
#pragma unroll
    for (int j = 0; j < NA; ++j) acc = fmaT(buf[j * RS + i], vec(j, 0), acc);
    return acc;
  }
  // C = A^T
  __device__ __forceinline__ void transpose(T (&C)[NA], const T (&A)[NA]) {
    put_mat(A);
#pragma unroll
    for (int j = 0; j < NA; ++j) C[j] = buf[j * RS + i];
  }
  // sum over the group's rows of column i of A
  __device__ __forceinline__ T colsum(const T (&A)[NA]) {
    put_mat(A);
    T acc = (T)0;
#pragma unroll
    for (int a = 0; a < NA; ++a) acc += buf[a * RS + i];
    return acc;
  }
  // sum over the group of v
  __device__ __forceinline__ T sum(T v) {
    put_vec(v, 1);
    T acc = (T)0;
#pragma unroll
    for (int j = 0; j < NA; ++j) acc += vec(j, 1);
    return acc;
  }
  // maximum over the group of v
  __device__ __forceinline__ T gmax(T v) {
    put_vec(v, 1);
    T acc = vec(0, 1);
#pragma unroll
    for (int j = 1; j < NA; ++j) acc = maxT(acc, vec(j, 1));
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
  __device__ __forceinline__ T from_lane(T v, int k) const { return permute(b4 + 4 * k, v); }
  template <int XM, int NB>
  __device__ __forceinline__ void gj(T (&A)[NA], T (&X)[NA], T (&v)[NB > 0 ? NB : 1]) {
    if constexpr (XM == 2) {
#pragma unroll
      for (int j = 0; j < NA; ++j) X[j] = (j == i) ? (T)1 : (T)0;
    }
    T own = (T)1;
#pragma unroll
    for (int k = 0; k < NA; ++k) {
      const T piv = from_lane(A[k], k);
      const T c = (i == k) ? (T)0 : A[k] * rcpT(piv);
      own = (i == k) ? piv : own;
#pragma unroll
      for (int j = k + 1; j < NA; ++j) A[j] = fmaT(-c, from_lane(A[j], k), A[j]);
      if constexpr (XM != 0) {
#pragma unroll
        for (int j = 0; j < (XM == 2 ? k + 1 : NA); ++j) X[j] = fmaT(-c, from_lane(X[j], k), X[j]);
      }
#pragma unroll
      for (int m = 0; m < NB; ++m) v[m] = fmaT(-c, from_lane(v[m], k), v[m]);
    }
    const T r = rcpT(own);
    if constexpr (XM != 0) {
#pragma unroll
      for (int j = 0; j < NA; ++j) X[j] *= r;
    }
#pragma unroll
    for (int m = 0; m < NB; ++m) v[m] *= r;
  }
  // X = A^-1; A is destroyed.  Used on symmetric positive definite matrices.
  __device__ __forceinline__ void inv(T (&X)[NA], T (&A)[NA]) {
    T v[1];
    gj<2, 0>(A, X, v);
  }
  // y1, y2, y3 with A y = b1, b2, b3; A is destroyed
  __device__ __forceinline__ void solve3(T (&A)[NA], T& b1, T& b2, T& b3) {
    T v[3] = {b1, b2, b3};
    gj<0, 3>(A, A, v);
    b1 = v[0]; b2 = v[1]; b3 = v[2];
  }
  // X <- A^-1 X (X holds the right-hand side's rows on entry); A is destroyed
  __device__ __forceinline__ void solve_mat(T (&X)[NA], T (&A)[NA]) {
    T v[1];
    gj<1, 0>(A, X, v);
  }
  // X <- A^-1 X and b0, b1, b2 <- A^-1 b0, b1, b2 (right-hand sides on
  // entry); A is destroyed
  __device__ __forceinline__ void solve_mat_v3(T (&X)[NA], T (&A)[NA], T& b0, T& b1, T& b2) {
    T v[3] = {b0, b1, b2};
    gj<1, 3>(A, X, v);
    b0 = v[0]; b1 = v[1]; b2 = v[2];
  }
};

template <typename T, int NA>
struct LaneTab {  // per-lane copies of the angle constants of row i
  T mu, m, d, z2, w, sw, swmu;
  int ext;
};


// ---- eigen solution of diag(d) - omega z z^T (d ascending) ------------------
// Lane i finds root i in (d_{i-1}, d_i) (d_{-1} = 0) as org + del, org the
// nearer end, by bracketed Newton on the secular function; the group then
// forms the Gu-Eisenstat vector and lane i keeps row i of V and its root.
template <int NA>
__device__ void eigen(Grp<double, NA>& g, const DenseTab<NA>& tb, const LaneTab<double, NA>& L,
                      double om, double (&V)[NA], double& k_i, double& lam_prev) {
  using T = double;
  constexpr T EPS = epsT<T>();
  const int i = g.i;
  T lo = (T)0;
#pragma unroll
  for (int j = 0; j < NA; ++j)
    if (j == i - 1) lo = tb.d[j];
  const T hi = L.d;
  T org = hi, del = (T)0;
  const T om1 = (T)1 - om;
  if (om > (T)0) {
    // f(lam) = 1 - om sum z2_j/(d_j - lam), or for root 0 near lam = 0 the
    // equivalent (1 - om) - om lam sum w_j/(d_j - lam); both decrease in lam.
    auto feval = [&](T o, T sgn, T x, T& f, T& df) {
      T s = (T)0, s2 = (T)0;
      if (i == 0 && o == (T)0) {
#pragma unroll
        for (int j = 0; j < NA; ++j) {
          const T r = rcpT(tb.d[j] - sgn * x);
          s = fmaT(tb.w[j], r, s);
          s2 = fmaT(tb.w[j] * tb.d[j], r * r, s2);
        }
        f = om1 - om * x * s;
        df = -om * s2;
      } else {
#pragma unroll
        for (int j = 0; j < NA; ++j) {
          const T r = rcpT((tb.d[j] - o) - sgn * x);
          s = fmaT(tb.z2[j], r, s);
          s2 = fmaT(tb.z2[j] * r, r, s2);
        }
        f = (T)1 - om * s;
        df = -om * s2;
      }
    };
    const T mid = (T)0.5 * (lo + hi);
    T fm, dfm;
    if (i == 0) feval((T)0, (T)1, mid, fm, dfm);
    else feval(lo, (T)1, mid - lo, fm, dfm);
    T sgn, xl, xh;
    if (fm > (T)0) { org = hi; sgn = (T)-1; xl = (T)0; xh = hi - mid; }
    else { org = lo; sgn = (T)1; xl = (T)0; xh = mid - lo; }
    if (i == 0 && sgn > (T)0 && om1 <= (T)0) {
      del = (T)0;                       // omega = 1: the diffusion root is exactly 0
    } else {
      // start from the root of the previous layer (same frequency, nearly the
      // same omega) when it lies in this half of the interval, else mid-way
      const T xp = sgn * (lam_prev - org);
      T x = (xp > xl && xp < xh) ? xp : (T)0.5 * (xl + xh);
      for (int it = 0; it < 200; ++it) {
        T f, df;
        feval(org, sgn, x, f, df);
        // lam = org + sgn x is too small when f > 0
        if ((f > (T)0) == (sgn > (T)0)) xl = x; else xh = x;
        T xn = x - f * rcpT(df * sgn);
        // a converged step ends the iteration before the bracket test: at the
        // root (f == 0, or a step that rounds to nothing) the update above has
        // just moved a bracket end onto x, and the test would take a bisection
        // step away from it
        if (absT(xn - x) <= (T)2 * EPS * x) {
          x = xn;
          break;
        }
        if (!(xn > xl && xn < xh)) xn = (T)0.5 * (xl + xh);
        const T step = absT(xn - x);
        x = xn;
        if (step <= (T)2 * EPS * x || xh - xl <= (T)4 * EPS * xh) break;
      }
      del = sgn * x;
    }
  }
  // broadcast roots
  wsync();
  g.buf[Slab<T, NA>::ROOT + 2 * i + 0] = org;
  g.buf[Slab<T, NA>::ROOT + 2 * i + 1] = del;
  wsync();
  const T lam = org + del;
  lam_prev = lam;
  k_i = sqrtT(maxT(lam, (T)0));
  if (!(om > (T)0)) {
#pragma unroll
    for (int a = 0; a < NA; ++a) V[a] = (a == i) ? (T)1 : (T)0;
    return;
  }
  // Gu-Eisenstat: zhat_i^2 = prod_a (lam_a - d_i) / (-omega prod_{j != i} (d_j - d_i))
  T num = del + (org - L.d), den = -om;
#pragma unroll
  for (int a = 0; a < NA; ++a) {
    const T oa = g.buf[Slab<T, NA>::ROOT + 2 * a];
    const T da = g.buf[Slab<T, NA>::ROOT + 2 * a + 1];
    if (a != i) {
      num *= (oa - L.d) + da;
      den *= tb.d[a] - L.d;
    }
  }
  const T zh2 = num / den;
  const T zh = sqrtT(absT(zh2));
  g.put_vec(zh, 2);
  // column norm of eigenvector i: sum_j zh_j^2 / (d_j - lam_i)^2
  T nrm = (T)0;
#pragma unroll
  for (int j = 0; j < NA; ++j) {
    const T q = g.vec(j, 2) * rcpT((tb.d[j] - org) - del);
    nrm = fmaT(q, q, nrm);
  }
  g.put_vec((T)1 / sqrtT(nrm), 3);
#pragma unroll
  for (int a = 0; a < NA; ++a) {
    const T oa = g.buf[Slab<T, NA>::ROOT + 2 * a];
    const T da = g.buf[Slab<T, NA>::ROOT + 2 * a + 1];
    V[a] = zh * rcpT((L.d - oa) - da) * g.vec(a, 3);
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
template <typename T, int NA>
struct LayerOps {
  T t[NA], r[NA];
  T bc, blp, blm;  // element i of beta_c, beta_l+, beta_l-
  T qv;            // element i of Q = beta_l+ + t sqrt(w) (difference-form source)
};

// (FP64 for every bulk type: see the precision note at the top)
template <int NA>
__device__ void layer_ops(Grp<double, NA>& g, const DenseTab<NA>& tb, const LaneTab<double, NA>& L,
                          const double (&V)[NA], double k_i, double Dl, LayerOps<double, NA>& o) {
  using T = double;
  const int i = g.i;
  constexpr int RS = Slab<T, NA>::RS;
  // per-root factors of root i, broadcast
  const T x = (T)0.5 * k_i * Dl;
  const T tx = k_i * tanhT(x);
  const T cx = (T)2 * x_coth_x(x);
  g.put_vec(tx, 2);
  g.put_vec(cx, 3);
  // Q_T = V diag(tx) V^T and Q_C' = V diag(cx) V^T: broadcast V
  g.put_mat(V);
  // one matrix at a time (fewer live registers): Q_T, then M + Q_T and its
  // inverse, then D M + Q_C' and its inverse.  The eliminations leave the
  // slab alone, so putting V there again changes no value; its fences keep
  // the compiler from interleaving the second product with the first
  // inversion, which without them spills 69 registers in pass 1 (15% slower)
  T QT[NA], FT[NA], FC[NA];
  {
    T vt[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) vt[a] = V[a] * g.vec(a, 2);
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      T st = (T)0;
#pragma unroll
      for (int a = 0; a < NA; ++a) st = fmaT(vt[a], g.buf[j * RS + a], st);
      QT[j] = st;
    }
  }
  {
    T AT[NA];
#pragma unroll
    for (int j = 0; j < NA; ++j) AT[j] = QT[j];
    AT[i] += L.m;               // M + Q_T      (lane-dependent diagonal)
    g.inv(FT, AT);
  }
  g.put_mat(V);
  {
    T vc[NA], AC[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) vc[a] = V[a] * g.vec(a, 3);
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      T sc = (T)0;
#pragma unroll
      for (int a = 0; a < NA; ++a) sc = fmaT(vc[a], g.buf[j * RS + a], sc);
      AC[j] = sc;
    }
    AC[i] += Dl * L.m;          // D M + Q_C'
    g.inv(FC, AC);
  }
  T tw = (T)0, rw = (T)0, fw = (T)0, qv = (T)0;
#pragma unroll
  for (int j = 0; j < NA; ++j) {
    const T ft = FT[j], fc = Dl * FC[j];
    o.r[j] = L.m * (ft + fc) - ((j == i) ? (T)1 : (T)0);
    o.t[j] = L.m * (ft - fc);
    tw = fmaT(o.t[j], tb.sw[j], tw);
    rw = fmaT(o.r[j], tb.sw[j], rw);
    fw = fmaT(ft, tb.sw[j], fw);
    qv = fmaT(FC[j], tb.swmu[j], qv);
  }
  qv *= (T)2 * L.m;
  o.qv = qv;
  o.bc = (T)2 * g.mv(QT, fw);
  o.blp = qv - tw;
  o.blm = (L.sw - rw) - qv;
}

template <typename T, int NA>
__device__ __forceinline__ void round_ops(const LayerOps<double, NA>& s, LayerOps<T, NA>& o) {
#pragma unroll
  for (int j = 0; j < NA; ++j) {
    o.t[j] = (T)s.t[j];
    o.r[j] = (T)s.r[j];
  }
  o.bc = (T)s.bc; o.blp = (T)s.blp; o.blm = (T)s.blm; o.qv = (T)s.qv;
}

// ---- the eliminations with I - (reflection)(reflection) in FP64 -------------
// for a float bulk under the thick-layer rule: the layer's own FP64
// operators, the FP32 composites converted exactly, products accumulated and
// right-hand sides formed in precision U = double.  (The kernels spell out
// the same eliminations in the bulk type inline: through these helpers the
// compiler serialises the FP64 kernels' cross-lane permutes, 16% slower.)

// way down: P <- G t, u <- G (r Sigma + dS^g Q), y1 <- G beta_l+, y2 <- G Q,
// G = (I - r R)^-1
template <typename U, typename T, typename S, int NA>
__device__ __forceinline__ void solve_down(Grp<U, NA>& gu, const LayerOps<S, NA>& op, const T (&R)[NA],
                                           T Sig, T dSg, T (&P)[NA], T& u, T& y1, T& y2) {
  const int i = gu.i;
  U X[NA], Pu[NA];
  gu.mul(X, op.r, R);
#pragma unroll
  for (int j = 0; j < NA; ++j) {
    X[j] = ((j == i) ? (U)1 : (U)0) - X[j];
    Pu[j] = (U)op.t[j];
  }
  U uu = gu.mv(op.r, (U)Sig) + (U)dSg * (U)op.qv;
  U z1 = (U)op.blp, z2 = (U)op.qv;
  gu.solve_mat_v3(Pu, X, uu, z1, z2);
#pragma unroll
  for (int j = 0; j < NA; ++j) P[j] = (T)Pu[j];
  u = (T)uu; y1 = (T)z1; y2 = (T)z2;
}

// node: (I - R^up R_d) y = R^up s + s^up for the intensity and the two unit
// responses (the latter only when wanted)
template <typename U, typename T, int NA>
__device__ __forceinline__ void solve_node(Grp<U, NA>& gu, const T (&Rup)[NA], const T (&Rd)[NA], T Sd,
                                           T Sup, T dS, T dSu, T eS, T eSu, bool wd, bool we, T& Ip,
                                           T& dIp, T& eDp) {
  const int i = gu.i;
  U y0 = gu.mv(Rup, (U)Sd) + (U)Sup;
  U y1 = wd ? gu.mv(Rup, (U)dS) + (U)dSu : (U)0;
  U y2 = we ? gu.mv(Rup, (U)eS) + (U)eSu : (U)0;
  U X[NA];
  gu.mul(X, Rup, Rd);
#pragma unroll
  for (int j = 0; j < NA; ++j) X[j] = ((j == i) ? (U)1 : (U)0) - X[j];
  gu.solve3(X, y0, y1, y2);
  Ip = (T)y0; dIp = (T)y1; eDp = (T)y2;
}

// way up: RG <- (I - R^up r)^-1 R^up  (= R^up (I - r R^up)^-1)
template <typename U, typename T, typename S, int NA>
__device__ __forceinline__ void solve_up(Grp<U, NA>& gu, const T (&Rup)[NA], const S (&r)[NA],
                                         T (&RG)[NA]) {
  const int i = gu.i;
  U Y[NA], Xu[NA];
  gu.mul(Y, Rup, r);
#pragma unroll
  for (int j = 0; j < NA; ++j) {
    Y[j] = ((j == i) ? (U)1 : (U)0) - Y[j];
    Xu[j] = (U)Rup[j];
  }
  gu.solve_mat(Xu, Y);
#pragma unroll
  for (int j = 0; j < NA; ++j) RG[j] = (T)Xu[j];
}

template <typename T, int NA>
__device__ __forceinline__ T row_abs_sum(const T (&A)[NA]) {
  T s = (T)0;
#pragma unroll
  for (int j = 0; j < NA; ++j) s += absT(A[j]);
  return s;
}

template <typename T, int NA>
struct FsDenseArgs {
  const Item* items;
  const int64_t* off;
  const double* tau;
  const T* q;
  const T* Sg;
  const T* omega;
  const T* Itop;
  const T* Bbot;
  const T* Bbot_prev;
  const T* Ibot;
  T *J, *JmS, *lstar, *lstar_c, *Iplus, *Iminus, *H, *Iemerg;
  T* wsR;     // [rows][nf][NA][NA]
  T* wsS;     // [rows][nf][NA]
  T* wsV;      // [rows][nf][NA][2 NA + 4]: layer (d, d+1): rows of t, r; bc, blp, blm, qv (bulk type)
               // (FP64 bulk only; a float bulk recomputes it in pass 2)
  T* wsZ;     // [rows][nf][NA][2]: R_d G_d beta+ and R_d G_d Q of layer (d, d+1), element i
  uint32_t* status; // device status word: NONFINITE when an output is not finite
  unsigned long long* thick_stats;  // [2]: eliminations in FP64, all eliminations (float bulk)
  int32_t nf;
  int32_t nitems;
  int32_t lower_bc;
  int32_t thick_mode;   // DENSE_THICK_RULE / _NEVER / _ALWAYS (float bulk)
  uint32_t outputs;
};

// PASS 1: the adding recursion down (composites R, Sigma and, in FP64, the
// layers' eigen solutions into the workspace); PASS 2: the pass up with the
// outputs.  Two kernels, so that each holds only its own pass's registers.
template <typename T, int NA, int PASS>
__global__ __launch_bounds__(64, 2) void k_fs_dense(FsDenseArgs<T, NA> a, DenseTab<NA> tb) {
  constexpr int F = 64 / NA;
  constexpr bool MIXED = std::is_same<T, float>::value;
  __shared__ double slab[F * Slab<double, NA>::SIZE];
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
  double* gslab = slab + grp * Slab<double, NA>::SIZE;
  Grp<T, NA> g{reinterpret_cast<T*>(gslab), lane % NA, 4 * (lane - lane % NA)};
  Grp<double, NA> g64{gslab, lane % NA, 4 * (lane - lane % NA)};
  const int i = g.i;
  LaneTab<double, NA> L64{};
#pragma unroll
  for (int j = 0; j < NA; ++j)
    if (j == i) {
      L64.mu = tb.mu[j]; L64.m = tb.m[j]; L64.d = tb.d[j]; L64.z2 = tb.z2[j]; L64.w = tb.w[j];
      L64.sw = tb.sw[j]; L64.swmu = tb.swmu[j]; L64.ext = tb.ext[j];
    }
  LaneTab<T, NA> L{(T)L64.mu, (T)L64.m, (T)L64.d, (T)L64.z2, (T)L64.w, (T)L64.sw, (T)L64.swmu, L64.ext};
  const uint32_t o = a.outputs;
  auto at = [&](const T* p, int64_t row) { return p[row * nf + k]; };
  // layer (d, d+1): optical depth and albedo in FP64 from the bulk inputs
  auto layer_depth = [&](int d) {
    return 0.5 * ((double)at(a.q, row0 + d) + (double)at(a.q, row0 + d + 1)) *
           (a.tau[row0 + d + 1] - a.tau[row0 + d]);
  };
  auto layer_omega = [&](int d) {
    return a.omega ? 0.5 * ((double)at(a.omega, row0 + d) + (double)at(a.omega, row0 + d + 1)) : 0.0;
  };
  // the thick-layer rule's absorption-depth test for one layer
  auto thick_layer = [&](T Dl, T om) { return Dl * sqrtT(maxT((T)1 - om, (T)0)) > (T)1; };
  // wave-uniform decision: FP64 when any lane's group asks for it
  auto wave_any = [&](bool f) { return __builtin_amdgcn_ballot_w64(f) != 0; };
  T* wsR = a.wsR + ((row0 * nf + k) * NA + i) * NA;   // + node * nf * NA * NA
  T* wsS = a.wsS + (row0 * nf + k) * NA + i;           // + node * nf * NA
  const int64_t strideR = (int64_t)nf * NA * NA;
  const int64_t strideS = (int64_t)nf * NA;
  constexpr int OW = 2 * NA + 4;     // kept operator values per lane and layer
  T* wsV = a.wsV + ((row0 * nf + k) * NA + i) * OW;  // + layer * nf * NA * OW
  const int64_t strideV = (int64_t)nf * NA * OW;
  T* wsZ = a.wsZ + ((row0 * nf + k) * NA + i) * 2;          // + layer * nf * NA * 2
  const int64_t strideZ = (int64_t)nf * NA * 2;
  // the unit-source responses behind Lambda* (plain form) and 1 - Lambda*
  // (difference form) are formed only for the outputs that are wanted
  const bool wd = (o & PPRT_OUT_LSTAR) != 0;
  const bool we = (o & PPRT_OUT_LSTAR_C) != 0;
  const int mode = a.thick_mode;
  unsigned n64 = 0, ntot = 0;   // eliminations of this wave in FP64, in all

  double V[NA];
  double kk = 0.0;
  double om_prev = -1.0;
  double lam_prev = -1.0;     // root of the last eigen solution (none yet)
  LayerOps<double, NA> op64;  // the layer's operators (FP64) ...
  LayerOps<T, NA> op;         // ... in the bulk type

  if constexpr (PASS == 1) {
  // ---------------- pass 1: adding recursion, top -> bottom
  T R[NA];
#pragma unroll
  for (int j = 0; j < NA; ++j) R[j] = (T)0;
  // difference form: D = I - S^g, scaled by sqrt(w)
  T Sig = L.sw * ((a.Itop ? a.Itop[((int64_t)b * nf + k) * NA + L.ext] : (T)0) - at(a.Sg, row0));
  for (int d = 0; d < nd - 1; ++d) {
#pragma unroll
    for (int j = 0; j < NA; ++j) wsR[d * strideR + j] = R[j];
    wsS[d * strideS] = Sig;
    const double om64 = layer_omega(d);
    if (om64 != om_prev) {
      eigen<NA>(g64, tb, L64, om64, V, kk, lam_prev);
      om_prev = om64;
    }
    const double Dl64 = layer_depth(d);
    layer_ops<NA>(g64, tb, L64, V, kk, Dl64, op64);
    round_ops(op64, op);
    {                 // kept for pass 2 in the bulk type (FP32 plans: the rounded operators)
      T* po = wsV + d * strideV;
#pragma unroll
      for (int j = 0; j < NA; ++j) {
        po[j] = op.t[j];
        po[NA + j] = op.r[j];
      }
      po[2 * NA] = op.bc;
      po[2 * NA + 1] = op.blp;
      po[2 * NA + 2] = op.blm;
      po[2 * NA + 3] = op.qv;
    }
    const T Dl = (T)Dl64, om = (T)om64;
    const T dSg = at(a.Sg, row0 + d + 1) - at(a.Sg, row0 + d);
    const T bm = -dSg * op.qv;       // difference-form layer source of the way up
    // G = (I - r R)^-1: P = G t, u = G (r Sigma + beta+), and for pass 2's
    // unit responses G beta_l+ and G Q, from one elimination on I - r R
    T P[NA], u, y1, y2;
    bool use64 = false;
    if constexpr (MIXED) {
      if (mode == DENSE_THICK_ALWAYS) {
        use64 = true;
      } else if (mode == DENSE_THICK_RULE) {
        const T nR = g.gmax(row_abs_sum(R));
        use64 = wave_any(thick_layer(Dl, om) || row_abs_sum(op.r) * nR > (T)0.5);
      }
      n64 += use64 ? 1u : 0u;
      ++ntot;
    }
    if (use64) {
      solve_down<double>(g64, op64, R, Sig, dSg, P, u, y1, y2);
    } else {
      T X[NA];
      g.mul(X, op.r, R);
#pragma unroll
      for (int j = 0; j < NA; ++j) {
        X[j] = ((j == i) ? (T)1 : (T)0) - X[j];
        P[j] = op.t[j];
      }
      u = g.mv(op.r, Sig) + dSg * op.qv;
      y1 = op.blp; y2 = op.qv;
      g.solve_mat_v3(P, X, u, y1, y2);
    }
    if (wd) wsZ[d * strideZ] = g.mv(R, y1);
    if (we) wsZ[d * strideZ + 1] = g.mv(R, y2);
    // Sigma_{d+1} = t (Sigma + R u) + beta-,  R_{d+1} = r + t R P
    const T Ru = g.mv(R, u);
    const T Sig_n = g.mv(op.t, Sig + Ru) + bm;
    T RP[NA], tRP[NA];
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
  T Rup[NA];
#pragma unroll
  for (int j = 0; j < NA; ++j) Rup[j] = (T)0;
  T Sup;
  {
    const int64_t rl = row0 + nd - 1;
    const T S_last = at(a.Sg, rl);
    if (a.lower_bc == PPRT_BC_DIFFUSION) {
      const T Bb = a.Bbot[(int64_t)b * nf + k];
      const T Bp = a.Bbot_prev[(int64_t)b * nf + k];
      const T gr = (Bb - Bp) / (T)layer_depth(nd - 2);
      Sup = L.sw * ((Bb - S_last) + L.mu * gr);
    } else {
      Sup = L.sw * ((a.Ibot ? a.Ibot[((int64_t)b * nf + k) * NA + L.ext] : (T)0) - S_last);
    }
  }
  T dSu = (T)0;           // dSigma^up of the node being emitted (layer below)
  T eSu = -L.sw;          // its difference-form counterpart (lower boundary: -1)
  bool thick_below = false;   // the layer below the node meets the absorption-depth test
  for (int d = nd - 1; d >= 0; --d) {
    const bool has_a = d >= 1;  // layer a = (d-1, d) above node d
    T Da = (T)0, oma = (T)0;
    if (has_a) {      // the operators of layer a, kept by pass 1 (FP32 plans: rounded; the
                      // FP64 ones are formed again where an FP64 elimination needs them)
      const double om64 = layer_omega(d - 1);
      const double Da64 = layer_depth(d - 1);
      const T* po = wsV + (d - 1) * strideV;
#pragma unroll
      for (int j = 0; j < NA; ++j) {
        op.t[j] = po[j];
        op.r[j] = po[NA + j];
      }
      op.bc = po[2 * NA];
      op.blp = po[2 * NA + 1];
      op.blm = po[2 * NA + 2];
      op.qv = po[2 * NA + 3];
      Da = (T)Da64;
      oma = (T)om64;
    }
    const bool thick_a = MIXED && has_a && mode == DENSE_THICK_RULE && thick_layer(Da, oma);
    // ---- emit node d
    T Rd[NA];
#pragma unroll
    for (int j = 0; j < NA; ++j) Rd[j] = wsR[d * strideR + j];
    const T Sd = wsS[d * strideS];
    // unit response: layer above (S^g 0 -> 1) through R_{d-1}, G_{d-1}; in
    // plain form (dS, for Lambda*) and in difference form (eS, sources +-Q
    // and -1 at a boundary, for 1 - Lambda* with full relative accuracy)
    // (each response only when its output is wanted: wd, we are uniform)
    T dS = (T)0, eS = -L.sw;
    if (has_a) {      // R_{d-1} G_{d-1} (dbeta+_a, Q_a), kept by pass 1
      if (wd) dS = g.mv(op.t, wsZ[(d - 1) * strideZ]) + op.blm;
      if (we) eS = g.mv(op.t, wsZ[(d - 1) * strideZ + 1]) - op.qv;
    }
    // I+ and the two responses from one elimination on I - R^up R_d
    T Ip, dIp, eDp;
    {
      bool use64 = false;
      if constexpr (MIXED) {
        if (mode == DENSE_THICK_ALWAYS) {
          use64 = true;
        } else if (mode == DENSE_THICK_RULE) {
          const T nR = g.gmax(row_abs_sum(Rd));
          use64 = wave_any(thick_a || thick_below || row_abs_sum(Rup) * nR > (T)0.5);
        }
        n64 += use64 ? 1u : 0u;
        ++ntot;
      }
      if (use64) {
        solve_node<double>(g64, Rup, Rd, Sd, Sup, dS, dSu, eS, eSu, wd, we, Ip, dIp, eDp);
      } else {
        Ip = g.mv(Rup, Sd) + Sup;
        dIp = wd ? g.mv(Rup, dS) + dSu : (T)0;
        eDp = we ? g.mv(Rup, eS) + eSu : (T)0;
        T X[NA];
        g.mul(X, Rup, Rd);
#pragma unroll
        for (int j = 0; j < NA; ++j) X[j] = ((j == i) ? (T)1 : (T)0) - X[j];
        g.solve3(X, Ip, dIp, eDp);
      }
    }
    const T Im = g.mv(Rd, Ip) + Sd;
    // Ip, Im are the scaled differences D+- = sqrt(w) (I+- - S^g)
    const T JmSn = (T)0.5 * g.sum(L.sw * (Ip + Im));
    T Ln = (T)0, Lcn = (T)0;
    if (wd) {
      const T dIm = g.mv(Rd, dIp) + dS;
      Ln = (T)0.5 * g.sum(L.sw * (dIp + dIm));
    }
    if (we) {
      const T eDm = g.mv(Rd, eDp) + eS;
      Lcn = (T)-0.5 * g.sum(L.sw * (eDp + eDm));
    }
    const T Hn = (T)0.5 * g.sum(L.swmu * (Ip - Im));
    // a zero or non-finite pivot in any elimination ends up here
    nonfinite |= !isfinite(Ip + Im + Ln + Lcn);
    {
      const int64_t x = (row0 + d) * nf + k;
      const T S = a.Sg[x];
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
      const T dSg = at(a.Sg, row0 + d) - at(a.Sg, row0 + d - 1);
      const T bp = dSg * op.qv;
      const T bm = -dSg * op.qv;
      // R^up G^up = R^up (I - r R^up)^-1 = (I - R^up r)^-1 R^up
      T RG[NA];
      bool use64 = false;
      if constexpr (MIXED) {
        if (mode == DENSE_THICK_ALWAYS) {
          use64 = true;
        } else if (mode == DENSE_THICK_RULE) {
          const T nr = g.gmax(row_abs_sum(op.r));
          use64 = wave_any(thick_a || row_abs_sum(Rup) * nr > (T)0.5);
        }
        n64 += use64 ? 1u : 0u;
        ++ntot;
      }
      if (use64) {
        if constexpr (MIXED) {      // layer a's FP64 operators (wave-uniform branch)
          const double om64 = layer_omega(d - 1);
          if (om64 != om_prev) {
            eigen<NA>(g64, tb, L64, om64, V, kk, lam_prev);
            om_prev = om64;
          }
          layer_ops<NA>(g64, tb, L64, V, kk, layer_depth(d - 1), op64);
        }
        solve_up<double>(g64, Rup, op64.r, RG);
      } else {
        T Y[NA];
        g.mul(Y, Rup, op.r);
#pragma unroll
        for (int j = 0; j < NA; ++j) {
          Y[j] = ((j == i) ? (T)1 : (T)0) - Y[j];
          RG[j] = Rup[j];
        }
        g.solve_mat(RG, Y);
      }
      const T w1 = g.mv(RG, g.mv(op.r, Sup) + bm);
      const T Sup_n = g.mv(op.t, Sup + w1) + bp;
      // unit response of layer a seen from node d-1 (S^g 1 -> 0)
      const T dbm = op.bc - op.blm, dbp = op.bc - op.blp;
      if (wd) dSu = g.mv(op.t, g.mv(RG, dbm)) + dbp;
      if (we) eSu = g.mv(op.t, g.mv(RG, op.qv)) - op.qv;
      T RGt[NA], tRGt[NA];
      g.mul(RGt, RG, op.t);
      g.mul(tRGt, op.t, RGt);
#pragma unroll
      for (int j = 0; j < NA; ++j) Rup[j] = op.r[j] + tRGt[j];
      Sup = Sup_n;
    }
    thick_below = thick_a;
  }
  if (nonfinite && a.status) atomicOr(a.status, PPRT_DEV_NONFINITE);
  }
  if constexpr (MIXED) {
    if (a.thick_stats && lane == 0) {
      atomicAdd(&a.thick_stats[0], (unsigned long long)n64);
      atomicAdd(&a.thick_stats[1], (unsigned long long)ntot);
    }
  }
}

template <int NA>
void fill_tab(DenseTab<NA>& tb, const double* mu_asc, const double* w_asc) {
  // internal order: descending mu
  for (int i = 0; i < NA; ++i) {
    const int e = NA - 1 - i;
    const double m = mu_asc[e], w = w_asc[e];
    tb.mu[i] = m; tb.m[i] = 1.0 / m; tb.d[i] = 1.0 / (m * m); tb.w[i] = w;
    tb.z2[i] = w / (m * m); tb.sw[i] = sqrt(w); tb.swmu[i] = sqrt(w) * m; tb.ext[i] = e;
  }
}

template <typename T, int NA>
hipError_t run_dense(const DenseLaunch& L, hipStream_t s) {
  FsDenseArgs<T, NA> a{};
  a.items = L.items; a.off = L.off; a.tau = L.tau;
  a.q = (const T*)L.q; a.Sg = (const T*)L.Sg; a.omega = (const T*)L.omega;
  a.Itop = (const T*)L.Itop; a.Bbot = (const T*)L.Bbot; a.Bbot_prev = (const T*)L.Bbot_prev;
  a.Ibot = (const T*)L.Ibot;
  a.J = (T*)L.J; a.JmS = (T*)L.JmS; a.lstar = (T*)L.lstar; a.lstar_c = (T*)L.lstar_c;
  a.Iplus = (T*)L.Iplus; a.Iminus = (T*)L.Iminus; a.H = (T*)L.H; a.Iemerg = (T*)L.Iemerg;
  // workspace: R | Sigma | Z | the layer operators, all in the bulk type
  const size_t rf = (size_t)L.rows * L.nf;
  a.wsR = (T*)L.ws;
  a.wsS = a.wsR + rf * NA * NA;
  a.wsZ = a.wsS + rf * NA;
  a.wsV = a.wsZ + rf * NA * 2;
  a.nf = L.nf; a.nitems = L.nitems; a.lower_bc = L.lower_bc; a.outputs = L.outputs;
  a.status = L.status;
  a.thick_stats = L.thick_stats;
  a.thick_mode = L.thick_mode;
  DenseTab<NA> tb{};
  fill_tab<NA>(tb, L.mu, L.w);
  hipLaunchKernelGGL((k_fs_dense<T, NA, 1>), dim3(L.nitems), dim3(64), 0, s, a, tb);
  hipLaunchKernelGGL((k_fs_dense<T, NA, 2>), dim3(L.nitems), dim3(64), 0, s, a, tb);
  return hipGetLastError();
}

template <typename T>
hipError_t run_dense_na(const DenseLaunch& L, hipStream_t s) {
  switch (L.na) {
    case 1: return run_dense<T, 1>(L, s);
    case 2: return run_dense<T, 2>(L, s);
    case 4: return run_dense<T, 4>(L, s);
    case 8: return run_dense<T, 8>(L, s);
    case 16: return run_dense<T, 16>(L, s);
    default: return hipErrorInvalidValue;
  }
}

// ---- reverse mode of the emergent intensity (omega > 0, FP64) --------------
// The emergent I+ at node 0 depends only on the composite of the layers below
// each node, built bottom-up:
//     R^up_{d-1} = r + t RG t,      RG = (I - R^up_d r)^-1 R^up_d,
//     S^up_{d-1} = t (S^up_d + RG (r S^up_d - dS^g Q)) + dS^g Q,
//     D+(0) = R^up_0 Sigma_0 + S^up_0,  Iemerg = D+(0) / sqrt(w) + S^g(0)
// (layer a = d - 1, dS^g = S^g(d) - S^g(a), Sigma_0 = sqrt(w) (Itop - S^g(0)),
// and at the bottom R^up = 0, S^up = sqrt(w) (Bbot - S^g + mu (Bbot - Bbot_prev)/D)
// or sqrt(w) (Ibot - S^g)).  k_dense_up runs that recursion and keeps R^up,
// S^up of every node and each layer's eigen solution; k_dense_vjp runs it
// backwards from g = dL/dIemerg, top-down, with the cotangents of R^up and
// S^up, and takes the derivative of t, r and Q in the layer optical depth D
// from the eigen form (V, k fixed by the albedo): with x = k D / 2,
//     dQ_T/dD = V diag(k^2/2 sech^2 x) V^T,   dQ_C'/dD = V diag(k (coth x - x csch^2 x)) V^T,
//     dF_T = -F_T dQ_T F_T,   dF_C' = -F_C' (M + dQ_C') F_C',
//     dr = M (dF_T + F_C' + D dF_C'),   dt = M (dF_T - F_C' - D dF_C'),   dQ = 2 M dF_C' sqrt(w) mu.
// D = (q(a) + q(a+1)) (tau(a+1) - tau(a)) / 2 gives dL/dq; the S^g differences
// and the boundary terms give dL/dS^g and dL/dBbot, dL/dBbot_prev or dL/dIbot.

// the layer's t, r and Q (in o) with the rows of F_T and F_C' and the root's
// derivative factors d(k tanh x)/dD and d(2 x coth x)/dD
// root i's derivative factors d(k tanh x)/dD and d(2 x coth x)/dD, x = k D / 2
__device__ __forceinline__ void layer_dfac(double k_i, double Dl, double& dtx, double& dcx) {
  const double x = 0.5 * k_i * Dl;
  const double th = tanh(x);
  dtx = 0.5 * k_i * k_i * (1.0 - th * th);
  if (x < 0.05) {
    const double x2 = x * x;
    dcx = k_i * x * (2.0 / 3.0 + x2 * (-4.0 / 45.0 + x2 * (4.0 / 315.0)));
  } else {
    const double sh = sinh(x);
    dcx = k_i * (1.0 / th - x / (sh * sh));
  }
}

// t, r and Q (in o) from the rows of F_T and F_C'
template <int NA>
__device__ __forceinline__ void layer_ops_from_f(Grp<double, NA>& g, const LaneTab<double, NA>& L,
                                                 const double (&FT)[NA], const double (&FC)[NA], double Dl,
                                                 LayerOps<double, NA>& o) {
  const int i = g.i;
#pragma unroll
  for (int j = 0; j < NA; ++j) {
    const double ft = FT[j], fc = Dl * FC[j];
    o.r[j] = L.m * (ft + fc) - ((j == i) ? 1.0 : 0.0);
    o.t[j] = L.m * (ft - fc);
  }
  g.put_vec(L.swmu, 1);
  double qv = 0.0;
#pragma unroll
  for (int j = 0; j < NA; ++j) qv = fma(FC[j], g.vec(j, 1), qv);
  o.qv = 2.0 * L.m * qv;
}

template <int NA>
__device__ void layer_ops_grad(Grp<double, NA>& g, const LaneTab<double, NA>& L, const double (&V)[NA],
                               double k_i, double Dl, LayerOps<double, NA>& o, double (&FT)[NA],
                               double (&FC)[NA], double& dtx, double& dcx) {
  const int i = g.i;
  constexpr int RS = Slab<double, NA>::RS;
  const double x = 0.5 * k_i * Dl;
  g.put_vec(k_i * tanh(x), 2);
  g.put_vec(2.0 * x_coth_x(x), 3);
  layer_dfac(k_i, Dl, dtx, dcx);
  double A[NA];
  g.put_mat(V);
  {
    double vt[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) vt[a] = V[a] * g.vec(a, 2);
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      double st = 0.0;
#pragma unroll
      for (int a = 0; a < NA; ++a) st = fma(vt[a], g.buf[j * RS + a], st);
      A[j] = st;
    }
  }
  A[i] += L.m;                  // M + Q_T
  g.inv(FT, A);
  g.put_mat(V);
  {
    double vc[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) vc[a] = V[a] * g.vec(a, 3);
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      double st = 0.0;
#pragma unroll
      for (int a = 0; a < NA; ++a) st = fma(vc[a], g.buf[j * RS + a], st);
      A[j] = st;
    }
  }
  A[i] += Dl * L.m;             // D M + Q_C'
  g.inv(FC, A);
  layer_ops_from_f<NA>(g, L, FT, FC, Dl, o);
}

template <int NA>
struct DenseVjpArgs {
  const Item* items;
  const int64_t* off;
  const double *tau, *q, *Sg, *omega, *Itop, *Bbot, *Bbot_prev, *Ibot, *gI;
  double *dq, *dSg, *dBbot, *dBbot_prev, *dIbot;
  double* wsR;   // [rows][nf][NA][NA]: R^up of each node
  double* wsS;   // [rows][nf][NA]: S^up of each node
  double* wsV;   // [rows][nf][NA][3 NA + 1]: layer (d, d+1): row i of V, root k_i, rows i of F_T, F_C'
  uint32_t* status;
  int32_t nf, nitems, lower_bc;
};

// the lane-group set-up shared by the two kernels
#define PPRT_DENSE_GROUP_SETUP                                                              \
  constexpr int F = 64 / NA;                                                                \
  __shared__ double slab[F * Slab<double, NA>::SIZE];                                        \
  const int lane = (int)threadIdx.x;                                                        \
  const int grp = lane / NA;                                                                \
  const int item = (int)blockIdx.x;                                                         \
  if (item >= a.nitems) return;                                                             \
  const Item it = a.items[item];                                                            \
  const int b = it.b;                                                                       \
  const int nd = it.nd;                                                                     \
  const int nf = a.nf;                                                                      \
  const int k = it.g * F + grp;                                                             \
  if (k >= nf) return;                                                                      \
  const int64_t row0 = a.off[b];                                                            \
  Grp<double, NA> g{slab + grp * Slab<double, NA>::SIZE, lane % NA, 4 * (lane - lane % NA)}; \
  const int i = g.i;                                                                        \
  LaneTab<double, NA> L{};                                                                  \
  _Pragma("unroll") for (int j = 0; j < NA; ++j) if (j == i) {                              \
    L.mu = tb.mu[j]; L.m = tb.m[j]; L.d = tb.d[j]; L.z2 = tb.z2[j]; L.w = tb.w[j];          \
    L.sw = tb.sw[j]; L.swmu = tb.swmu[j]; L.ext = tb.ext[j];                                \
  }                                                                                         \
  auto at = [&](const double* p, int64_t row) { return p[row * nf + k]; };                  \
  auto layer_depth = [&](int d) {                                                           \
    return 0.5 * (at(a.q, row0 + d) + at(a.q, row0 + d + 1)) * (a.tau[row0 + d + 1] - a.tau[row0 + d]); \
  };                                                                                        \
  auto layer_omega = [&](int d) {                                                           \
    return a.omega ? 0.5 * (at(a.omega, row0 + d) + at(a.omega, row0 + d + 1)) : 0.0;      \
  };                                                                                        \
  double* wsR = a.wsR + ((row0 * nf + k) * NA + i) * NA;                                    \
  double* wsS = a.wsS + (row0 * nf + k) * NA + i;                                           \
  double* wsV = a.wsV + ((row0 * nf + k) * NA + i) * (3 * NA + 1);                         \
  const int64_t strideR = (int64_t)nf * NA * NA;                                            \
  const int64_t strideS = (int64_t)nf * NA;                                                 \
  const int64_t strideV = (int64_t)nf * NA * (3 * NA + 1);

// the bottom-up composites R^up, S^up of every node, and the eigen solutions
// with the rows of F_T and F_C' (the reverse sweep takes t, r and Q from them)
template <int NA>
__global__ __launch_bounds__(64, 1) void k_dense_up(DenseVjpArgs<NA> a, DenseTab<NA> tb) {
  PPRT_DENSE_GROUP_SETUP
  double Rup[NA];
#pragma unroll
  for (int j = 0; j < NA; ++j) Rup[j] = 0.0;
  double Sup;
  {
    const double S_last = at(a.Sg, row0 + nd - 1);
    if (a.lower_bc == PPRT_BC_DIFFUSION) {
      const double Bb = a.Bbot[(int64_t)b * nf + k], Bp = a.Bbot_prev[(int64_t)b * nf + k];
      Sup = L.sw * ((Bb - S_last) + L.mu * (Bb - Bp) / layer_depth(nd - 2));
    } else {
      const double Ib = a.Ibot ? a.Ibot[((int64_t)b * nf + k) * NA + L.ext] : 0.0;
      Sup = L.sw * (Ib - S_last);
    }
  }
#pragma unroll
  for (int j = 0; j < NA; ++j) wsR[(nd - 1) * strideR + j] = 0.0;
  wsS[(nd - 1) * strideS] = Sup;
  double V[NA], kk = 0.0, om_prev = -1.0, lam_prev = -1.0;
  LayerOps<double, NA> op;
  for (int d = nd - 1; d >= 1; --d) {
    const int la = d - 1;
    const double om = layer_omega(la);
    if (om != om_prev) {
      eigen<NA>(g, tb, L, om, V, kk, lam_prev);
      om_prev = om;
    }
#pragma unroll
    for (int j = 0; j < NA; ++j) wsV[la * strideV + j] = V[j];
    wsV[la * strideV + NA] = kk;
    {
      double FT[NA], FC[NA], dtx, dcx;
      layer_ops_grad<NA>(g, L, V, kk, layer_depth(la), op, FT, FC, dtx, dcx);
#pragma unroll
      for (int j = 0; j < NA; ++j) {
        wsV[la * strideV + NA + 1 + j] = FT[j];
        wsV[la * strideV + 2 * NA + 1 + j] = FC[j];
      }
    }
    const double dSg = at(a.Sg, row0 + d) - at(a.Sg, row0 + la);
    double X[NA], RG[NA];
    g.mul(X, Rup, op.r);
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      X[j] = ((j == i) ? 1.0 : 0.0) - X[j];
      RG[j] = Rup[j];
    }
    g.solve_mat(RG, X);                                  // RG = (I - R^up r)^-1 R^up
    const double w1 = g.mv(RG, g.mv(op.r, Sup) - dSg * op.qv);
    Sup = g.mv(op.t, Sup + w1) + dSg * op.qv;
    double RGt[NA], tRGt[NA];
    g.mul(RGt, RG, op.t);
    g.mul(tRGt, op.t, RGt);
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      Rup[j] = op.r[j] + tRGt[j];
      wsR[la * strideR + j] = Rup[j];
    }
    wsS[la * strideS] = Sup;
  }
}

// C = A B as Grp::mul, with the loop over k rolled by two and A's row read
// from LDS (ar: this lane's column of a [k][64 lanes] array): in the reverse
// sweep, whose steps hold a dozen matrix rows, the fully unrolled product left
// the 16-angle kernel with about a thousand registers in scratch
template <int NA>
__device__ __forceinline__ void mul_rolled(Grp<double, NA>& g, double* ar, double (&C)[NA],
                                           const double (&A)[NA], const double (&B)[NA]) {
  constexpr int RS = Slab<double, NA>::RS;
  g.put_mat(B);
#pragma unroll
  for (int k = 0; k < NA; ++k) ar[64 * k] = A[k];
  double acc[NA];
#pragma unroll
  for (int j = 0; j < NA; ++j) acc[j] = 0.0;
#pragma unroll 2
  for (int k = 0; k < NA; ++k) {
    const double a = ar[64 * k];
#pragma unroll
    for (int j = 0; j < NA; ++j) acc[j] = fma(a, g.buf[k * RS + j], acc[j]);
  }
#pragma unroll
  for (int j = 0; j < NA; ++j) C[j] = acc[j];
}

// reverse sweep, top-down: dL/dq, dL/dS^g and the boundary derivatives
template <int NA>
__global__ __launch_bounds__(64, 1) void k_dense_vjp(DenseVjpArgs<NA> a, DenseTab<NA> tb) {
  PPRT_DENSE_GROUP_SETUP
  (void)layer_omega;                  // the albedo enters through the stored eigen solutions
  // the left factor's row of each product, [k][lane] (mul_rolled)
  __shared__ double arow[NA * 64];
  auto mul = [&](double (&C)[NA], const double (&A)[NA], const double (&B)[NA]) {
    mul_rolled<NA>(g, arow + lane, C, A, B);
  };
  const int64_t bk = (int64_t)b * nf + k;
  bool nonfinite = false;
  double Rb[NA], Sb;
  double dS_node, dq_node = 0.0;    // node being finished: its dL/dS^g and dL/dq so far
  {
    const double gI = a.gI[bk * NA + L.ext];
    const double S0 = at(a.Sg, row0);
    const double Sig0 = L.sw * ((a.Itop ? a.Itop[bk * NA + L.ext] : 0.0) - S0);
    double Rup[NA];
#pragma unroll
    for (int j = 0; j < NA; ++j) Rup[j] = wsR[j];
    const double Ipb = gI / L.sw;                       // D+(0) = R^up_0 Sigma_0 + S^up_0
    dS_node = g.sum(gI);
    g.put_vec(Sig0, 1);
#pragma unroll
    for (int j = 0; j < NA; ++j) Rb[j] = Ipb * g.vec(j, 1);
    dS_node -= g.sum(L.sw * g.mvT(Rup, Ipb));
    Sb = Ipb;
  }
  for (int d = 1; d < nd; ++d) {
    const int la = d - 1;
    double Rup[NA], V[NA];
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      Rup[j] = wsR[d * strideR + j];
      V[j] = wsV[la * strideV + j];
    }
    const double Sup = wsS[d * strideS];
    const double kk = wsV[la * strideV + NA];
    const double Dl = layer_depth(la);
    // t, r and Q from the rows of F_T and F_C' kept by the pass up; those
    // rows are read again (not held) for the layer depth's derivative at the
    // end of the step
    LayerOps<double, NA> op;
    double dtx, dcx;
    layer_dfac(kk, Dl, dtx, dcx);
    {
      double FT[NA], FC[NA];
#pragma unroll
      for (int j = 0; j < NA; ++j) {
        FT[j] = wsV[la * strideV + NA + 1 + j];
        FC[j] = wsV[la * strideV + 2 * NA + 1 + j];
      }
      layer_ops_from_f<NA>(g, L, FT, FC, Dl, op);
    }
    const double dSg = at(a.Sg, row0 + d) - at(a.Sg, row0 + la);
    // forward quantities of the step
    double G[NA], RG[NA], T1[NA], T2[NA];
    mul(T1, Rup, op.r);
#pragma unroll
    for (int j = 0; j < NA; ++j) T1[j] = ((j == i) ? 1.0 : 0.0) - T1[j];
    g.inv(G, T1);                                        // G = (I - R^up r)^-1
    mul(RG, G, Rup);
    const double v = g.mv(op.r, Sup) - dSg * op.qv;
    const double u = Sup + g.mv(RG, v);
    // S^up' = t u + dS^g Q
    double tb_[NA], rb[NA], RGb[NA];
    g.put_vec(u, 1);
#pragma unroll
    for (int j = 0; j < NA; ++j) tb_[j] = Sb * g.vec(j, 1);
    const double ub = g.mvT(op.t, Sb);
    double dSgb = g.sum(op.qv * Sb);
    double qvb = dSg * Sb;
    double Supb = ub;
    // u = S^up + RG v
    g.put_vec(v, 1);
#pragma unroll
    for (int j = 0; j < NA; ++j) RGb[j] = ub * g.vec(j, 1);
    const double vb = g.mvT(RG, ub);
    // v = r S^up - dS^g Q
    g.put_vec(Sup, 1);
#pragma unroll
    for (int j = 0; j < NA; ++j) rb[j] = vb * g.vec(j, 1) + Rb[j];   // + the R^up' = r + ... term
    Supb += g.mvT(op.r, vb);
    dSgb -= g.sum(op.qv * vb);
    qvb -= dSg * vb;
    // R^up' = r + t RG t: t gets Rb (RG t)^T + (t RG)^T Rb, RG gets t^T Rb t^T
    mul(T1, RG, op.t);
    g.transpose(T2, T1);
    mul(T1, Rb, T2);
#pragma unroll
    for (int j = 0; j < NA; ++j) tb_[j] += T1[j];
    mul(T1, op.t, RG);
    g.transpose(T2, T1);
    mul(T1, T2, Rb);
#pragma unroll
    for (int j = 0; j < NA; ++j) tb_[j] += T1[j];
    double tT[NA];
    g.transpose(tT, op.t);
    mul(T1, tT, Rb);
    mul(T2, T1, tT);
#pragma unroll
    for (int j = 0; j < NA; ++j) RGb[j] += T2[j];
    // RG = G R^up: R^up gets G^T RGb (I + r RG)^T, r gets RG^T RGb RG^T
    double Rupb[NA];
    mul(T1, op.r, RG);
#pragma unroll
    for (int j = 0; j < NA; ++j) T1[j] += (j == i) ? 1.0 : 0.0;
    g.transpose(T2, T1);                                 // (I + r RG)^T
    g.transpose(T1, G);
    mul(Rupb, T1, RGb);
    mul(T1, Rupb, T2);
#pragma unroll
    for (int j = 0; j < NA; ++j) Rupb[j] = T1[j];
    g.transpose(T2, RG);
    mul(T1, T2, RGb);
    mul(RG, T1, T2);                                   // RG no longer needed: RG^T RGb RG^T
#pragma unroll
    for (int j = 0; j < NA; ++j) rb[j] += RG[j];
    // the layer optical depth: <tb, dt> + <rb, dr> + <Qb, dQ>
    double part = 0.0;
    {
      double FT[NA], FC[NA];
#pragma unroll
      for (int j = 0; j < NA; ++j) {
        FT[j] = wsV[la * strideV + NA + 1 + j];
        FC[j] = wsV[la * strideV + 2 * NA + 1 + j];
        V[j] = wsV[la * strideV + j];
      }
      double AT[NA], AC[NA];
#pragma unroll
      for (int j = 0; j < NA; ++j) {
        AT[j] = L.m * (tb_[j] + rb[j]);
        AC[j] = L.m * (rb[j] - tb_[j]);
        part = fma(AC[j], FC[j], part);                  // <A_C, F_C'>
      }
      mul(T1, FT, AT);
      mul(T2, T1, FT);                                 // B_T = F_T A_T F_T
      mul(T1, T2, V);
#pragma unroll
      for (int j = 0; j < NA; ++j) T1[j] *= V[j];
      part -= dtx * g.colsum(T1);                        // - sum_j dtx_j (V^T B_T V)_jj
      const double c = g.mv(FC, L.swmu);                 // F_C' sqrt(w) mu
      const double y = g.mv(FC, 2.0 * L.m * qvb);        // F_C' (2 M Qb)
      mul(T1, FC, AC);
      mul(T2, T1, FC);
      g.put_vec(c, 1);
#pragma unroll
      for (int j = 0; j < NA; ++j) T2[j] = Dl * T2[j] + y * g.vec(j, 1);   // B_C
      double bcd = 0.0;
#pragma unroll
      for (int j = 0; j < NA; ++j)
        if (j == i) bcd = T2[j];
      part -= L.m * bcd;                                 // - <B_C, M>
      mul(T1, T2, V);
#pragma unroll
      for (int j = 0; j < NA; ++j) T1[j] *= V[j];
      part -= dcx * g.colsum(T1);                        // - sum_j dcx_j (V^T B_C V)_jj
    }
    const double Dlb = g.sum(part);
    const double h = 0.5 * (a.tau[row0 + d] - a.tau[row0 + la]);
    // node la is finished (layer la - 1 below it came first)
    dq_node += h * Dlb;
    dS_node -= dSgb;
    nonfinite |= !isfinite(dq_node + dS_node);
    if (i == 0) {
      a.dq[(row0 + la) * nf + k] = dq_node;
      a.dSg[(row0 + la) * nf + k] = dS_node;
    }
    dq_node = h * Dlb;
    dS_node = dSgb;
    Sb = Supb;
#pragma unroll
    for (int j = 0; j < NA; ++j) Rb[j] = Rupb[j];
  }
  // the lower boundary
  dS_node -= g.sum(L.sw * Sb);
  if (a.lower_bc == PPRT_BC_DIFFUSION) {
    const double Dl = layer_depth(nd - 2);
    const double Bb = a.Bbot[bk], Bp = a.Bbot_prev[bk];
    const double swSb = g.sum(L.sw * Sb), swmuSb = g.sum(L.swmu * Sb);
    const double Dlb = -swmuSb * (Bb - Bp) / (Dl * Dl);
    const double h = 0.5 * (a.tau[row0 + nd - 1] - a.tau[row0 + nd - 2]);
    dq_node += h * Dlb;
    if (i == 0) {
      a.dq[(row0 + nd - 2) * nf + k] += h * Dlb;       // the last layer's depth also sets the gradient
      if (a.dBbot) a.dBbot[bk] = swSb + swmuSb / Dl;
      if (a.dBbot_prev) a.dBbot_prev[bk] = -swmuSb / Dl;
    }
  } else if (a.dIbot) {
    a.dIbot[bk * NA + L.ext] = L.sw * Sb;
  }
  nonfinite |= !isfinite(dq_node + dS_node);
  if (i == 0) {
    a.dq[(row0 + nd - 1) * nf + k] = dq_node;
    a.dSg[(row0 + nd - 1) * nf + k] = dS_node;
  }
  if (nonfinite && a.status && i == 0) atomicOr(a.status, PPRT_DEV_NONFINITE);
}
#undef PPRT_DENSE_GROUP_SETUP

template <int NA>
hipError_t run_dense_vjp(const DenseVjpLaunch& L, hipStream_t s) {
  DenseVjpArgs<NA> a{};
  a.items = L.items; a.off = L.off; a.tau = L.tau; a.q = L.q; a.Sg = L.Sg; a.omega = L.omega;
  a.Itop = L.Itop; a.Bbot = L.Bbot; a.Bbot_prev = L.Bbot_prev; a.Ibot = L.Ibot; a.gI = L.gI;
  a.dq = L.dq; a.dSg = L.dSg; a.dBbot = L.dBbot; a.dBbot_prev = L.dBbot_prev; a.dIbot = L.dIbot;
  const size_t rf = (size_t)L.rows * L.nf;
  a.wsR = (double*)L.ws;
  a.wsS = a.wsR + rf * NA * NA;
  a.wsV = a.wsS + rf * NA;
  a.status = L.status;
  a.nf = L.nf; a.nitems = L.nitems; a.lower_bc = L.lower_bc;
  DenseTab<NA> tb{};
  fill_tab<NA>(tb, L.mu, L.w);
  hipLaunchKernelGGL((k_dense_up<NA>), dim3(L.nitems), dim3(64), 0, s, a, tb);
  hipLaunchKernelGGL((k_dense_vjp<NA>), dim3(L.nitems), dim3(64), 0, s, a, tb);
  return hipGetLastError();
}

}  // namespace

bool dense_na_supported(int na) { return na == 1 || na == 2 || na == 4 || na == 8 || na == 16 || na == 32; }

size_t dense_workspace_bytes(int na, int64_t rows, int nf, int precision) {
  // per node and frequency: R (na^2), Sigma (na), Z (2 na) in the bulk type,
  // plus (lane-per-row FP64 kernels) each layer's t, r and four source
  // vectors (2 na^2 + 4 na doubles)
  const size_t rf = (size_t)rows * nf;
  if (dense_mfma_na(na)) return dense_mfma_workspace_bytes(na, rows, nf, precision);
  if (precision == PPRT_FP64) return rf * (size_t)(3 * na * na + 7 * na) * sizeof(double);
  return rf * (size_t)(3 * na * na + 7 * na) * sizeof(float);
}

// frequencies per wave: one on the matrix cores, else 64 / na lane groups
int dense_freqs_per_item(int na, int precision) {
  if (dense_mfma_na(na)) return 1;
  return na <= 64 ? 64 / na : 1;
}

size_t dense_vjp_workspace_bytes(int na, int64_t rows, int nf) {
  // R^up (na^2) and S^up (na) of every node, the eigen solution (na^2 + na) of every layer
  return (size_t)rows * nf * (size_t)(4 * na * na + 2 * na) * sizeof(double);
}

hipError_t launch_dense_vjp(const DenseVjpLaunch& L, hipStream_t s) {
  if (L.nitems == 0) return hipSuccess;
  switch (L.na) {
    case 1: return run_dense_vjp<1>(L, s);
    case 2: return run_dense_vjp<2>(L, s);
    case 4: return run_dense_vjp<4>(L, s);
    case 8: return run_dense_vjp<8>(L, s);
    case 16: return run_dense_vjp<16>(L, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fs_dense(const DenseLaunch& L, hipStream_t s) {
  if (L.nitems == 0) return hipSuccess;
  if (dense_mfma_na(L.na)) return launch_fs_dense_mfma(L, s);
  if (L.na > 16) return hipErrorInvalidValue;
  return L.precision == PPRT_FP64 ? run_dense_na<double>(L, s) : run_dense_na<float>(L, s);
}

}  // namespace pprt

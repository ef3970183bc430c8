// Formal solution with coherent isotropic scattering inside the layers for
// NA = 32 angles per hemisphere (32 x 32 layer operators, the 64-stream
// problem) on the FP64 matrix cores of gfx950.  The code is written for
// NA = 16 T; only T = 2 is built: at NA = 16 the lane-per-row kernel of
// fs_dense.hip, whose 16 x 16 operators fit one lane's registers row by row,
// is faster (36 against 48 ms on a 64-atmosphere, 256-frequency batch).
//
// The method is that of fs_dense.hip (the same homogeneous-layer operators
// t, r, beta from the discrete-ordinate eigen solution, the adding recursion
// down with the composite R and Sigma of every node kept, the pass up with
// I+-, J, J - S^g, H, Lambda* and 1 - Lambda* at every node, intensities in
// difference form); only the mapping differs:
//
// * One frequency per wave.  An NA x NA matrix (NA = 16 T) lives in T x T
//   tiles of the v_mfma_f64_16x16x4 result layout: lane l holds column l % 16
//   of each tile and rows l / 16 + 4 q, q = 0..3, four doubles per tile (an
//   NA = 32 matrix costs 32 registers).  Vectors are compact: lane i < NA
//   holds element i (angles in order of decreasing mu), the other lanes 0.
// * Products: both factors are written to the wave's LDS slab row-major and
//   read back as matrix-core operands (A: lane l holds A[l % 16][l / 16] of a
//   16 x 4 panel; B: lane l holds B[l / 16][l % 16] of a 4 x 16 panel); an
//   NA x NA x NA product is 4 T^3 v_mfma_f64_16x16x4 instructions.
//   V diag(x) V^T reads V transposed from the same slab.
// * Eliminations: Gauss-Jordan without pivoting on [A | X] (the matrices are
//   M + Q_T and D M + Q_C' (symmetric positive definite) or
//   I - (reflection)(reflection)), by blocks of four columns: the block's
//   four rows and four columns go to LDS, every lane inverts the 4 x 4 pivot
//   block, the other rows take one rank-4 update W -= C (P^-1 B) per tile
//   pair on the matrix cores, and the block rows are set to P^-1 B (the loop
//   over blocks is unrolled, so every tile and register index is static).
// * Mat-vec products: the vector goes through the slab, each lane multiplies
//   its tile elements and the sixteen lanes of a row group reduce by DPP
//   row sums; sums over angles reduce across the wave.
// * The eigen data of every layer (secular-equation roots, the Gu-Eisenstat
//   vector zhat and the column norms) are solved apart, before the
//   recursion, by k_mf_roots (one thread per frequency and root, at full
//   occupancy) and kept in the workspace; both passes assemble the
//   eigenvectors from them.  The workspace keeps R, Sigma and two unit-source
//   responses per node in the plan's type and the eigen data in FP64:
//   (NA^2 + 3 NA) reals + 32 NA bytes per node and frequency.
// * The workspace also keeps each layer's t, r and source vectors from the
//   pass down (2 NA^2 + 4 NA reals per layer and frequency in the plan's
//   type, in the tiles' register order so that every lane moves contiguous
//   bytes per tile), and the pass up loads them instead of forming them
//   again: the second formation was 27% of the formal solution, the loads
//   cost one memory latency per layer.  FP32 plans round them to FP32, so
//   that both passes work with the same layers.
// * The operators of a layer do not depend on the recursion, so a pass of
//   their own (PASS 0) forms them before it: 16 waves per (atmosphere,
//   frequency), each taking every 16th layer, at two waves per SIMD (the
//   recursion passes need one wave per SIMD's registers); it never stages a
//   generic product, so its slab stops before the second operand's area
//   (17.2 KB instead of 25.6 KB: eight waves per CU).  The pass down then
//   loads them like the pass up (C5: 463 -> 419 ms per formal solution).
#include "pprt_internal.h"

namespace pprt {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

template <int NA>
struct MfTab {
  // internal angle order: descending mu (ascending d = 1/mu^2); z2 = w d
  double mu[NA], m[NA], d[NA], z2[NA], w[NA], sw[NA], swmu[NA];
};

template <int T>
struct Mat {
  v4d t[T][T];
};

// the wave's LDS slab (doubles)
template <int T>
struct Lay {
  static constexpr int NA = 16 * T;
  static constexpr int LA = NA + 1;                 // row stride of the product operands
  static constexpr int LW = 16 * (2 * T + 1);       // width of an augmented block row
  static constexpr int A0 = 0;                      // NA x LA
  static constexpr int BR = A0 + NA * LA;           // 4 x LW: block rows
  static constexpr int BC = BR + 4 * LW;            // NA x 5: block columns
  static constexpr int VS = BC + NA * 5;            // 8 vector slots of NA
  static constexpr int RT = VS + 8 * NA;            // 2 NA roots (origin, offset)
  static constexpr int ZH = RT + 2 * NA;            // NA: Gu-Eisenstat zhat
  static constexpr int NR = ZH + NA;                // NA: eigenvector norms
  static constexpr int TX = NR + NA;                // NA: k tanh x
  static constexpr int CX = TX + NA;                // NA: 2 x coth x
  static constexpr int TM = CX + NA;                // NA: angle table m = 1/mu
  static constexpr int TD = TM + NA;                // NA: d = 1/mu^2
  static constexpr int TMU = TD + NA;               // NA: mu
  static constexpr int TZ2 = TMU + NA;              // NA: w d
  static constexpr int TW = TZ2 + NA;               // NA: w
  static constexpr int B0 = TW + NA;                // NA x LA: second product operand, last:
  static constexpr int SIZE = B0 + NA * LA;         // the operator pass (no generic products)
                                                    // takes a slab of B0 doubles
  // vector slots: 0 mat-vec input, 1 mat-vec output, 2..4 right-hand-side
  // columns, 5 sqrt(w), 6 sqrt(w) mu, 7 spare
};

template <int T>
struct W {                 // per-wave context
  double* s;               // LDS slab
  int lane, g, c;
};

// ---- tiles <-> LDS
template <int T>
__device__ __forceinline__ void store(const W<T>& w, const Mat<T>& M, int base, int ld) {
#pragma unroll
  for (int ti = 0; ti < T; ++ti)
#pragma unroll
    for (int tj = 0; tj < T; ++tj)
#pragma unroll
      for (int q = 0; q < 4; ++q) w.s[base + (16 * ti + w.g + 4 * q) * ld + 16 * tj + w.c] = M.t[ti][tj][q];
}

// compact vectors: lane l < NA holds element l
template <int T>
__device__ __forceinline__ void vset(const W<T>& w, int slot, double x) {
  if (w.lane < Lay<T>::NA) w.s[Lay<T>::VS + slot * Lay<T>::NA + w.lane] = x;
}
template <int T>
__device__ __forceinline__ double vget(const W<T>& w, int slot) {
  return w.lane < Lay<T>::NA ? w.s[Lay<T>::VS + slot * Lay<T>::NA + w.lane] : 0.0;
}
template <int T>
__device__ __forceinline__ double tab(const W<T>& w, int base) {   // this lane's angle constant
  return w.lane < Lay<T>::NA ? w.s[base + w.lane] : 0.0;
}

// C = A B with A (row-major, lda) and B (row-major, ldb, or transposed) in LDS;
// A's columns scaled by scale[k] when given (V diag(x) V^T)
template <int T, bool TRANSB>
__device__ __forceinline__ void mul_ll(const W<T>& w, Mat<T>& C, int a0, int lda, int b0, int ldb,
                                       int scale = -1) {
  constexpr int KS = 4 * T;
#pragma unroll
  for (int ti = 0; ti < T; ++ti)
#pragma unroll
    for (int tj = 0; tj < T; ++tj) C.t[ti][tj] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int k = 4 * s + w.g;
    double a[T], b[T];
#pragma unroll
    for (int ti = 0; ti < T; ++ti) {
      a[ti] = w.s[a0 + (16 * ti + w.c) * lda + k];
      if (scale >= 0) a[ti] *= w.s[scale + k];
    }
#pragma unroll
    for (int tj = 0; tj < T; ++tj)
      b[tj] = TRANSB ? w.s[b0 + (16 * tj + w.c) * ldb + k] : w.s[b0 + k * ldb + 16 * tj + w.c];
#pragma unroll
    for (int ti = 0; ti < T; ++ti)
#pragma unroll
      for (int tj = 0; tj < T; ++tj) C.t[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ti], b[tj], C.t[ti][tj], 0, 0, 0);
  }
}

// C = A B for tiles A, B (through the slab)
template <int T>
__device__ __forceinline__ void mul(const W<T>& w, Mat<T>& C, const Mat<T>& A, const Mat<T>& B) {
  wsync();
  store(w, A, Lay<T>::A0, Lay<T>::LA);
  store(w, B, Lay<T>::B0, Lay<T>::LA);
  wsync();
  mul_ll<T, false>(w, C, Lay<T>::A0, Lay<T>::LA, Lay<T>::B0, Lay<T>::LA);
}

// y = A x for x in vector slot `in`; the result goes to slot 1 and is returned compact
template <int T>
__device__ __forceinline__ double mv_slot(const W<T>& w, const Mat<T>& A, int in) {
  double xc[T];
#pragma unroll
  for (int tj = 0; tj < T; ++tj) xc[tj] = w.s[Lay<T>::VS + in * Lay<T>::NA + 16 * tj + w.c];
  double y[T][4];
#pragma unroll
  for (int ti = 0; ti < T; ++ti)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double p = 0.0;
#pragma unroll
      for (int tj = 0; tj < T; ++tj) p = fma(A.t[ti][tj][q], xc[tj], p);
      y[ti][q] = row_sum(p);       // the sixteen lanes of the row group (DPP)
    }
  wsync();
  if (w.c == 0) {
#pragma unroll
    for (int ti = 0; ti < T; ++ti)
#pragma unroll
      for (int q = 0; q < 4; ++q) w.s[Lay<T>::VS + 1 * Lay<T>::NA + 16 * ti + w.g + 4 * q] = y[ti][q];
  }
  wsync();
  return vget(w, 1);
}
template <int T>
__device__ __forceinline__ double mv(const W<T>& w, const Mat<T>& A, double x) {
  wsync();
  vset(w, 0, x);
  wsync();
  return mv_slot(w, A, 0);
}

// sum over angles of a x (compact; DPP row sums, then the four rows)
__device__ __forceinline__ double dot(double a, double x) { return wave_sum(a * x); }

// Gauss-Jordan without pivoting on the augmented tiles [A | X] (TX column
// tiles of right-hand sides): on exit A = I and X = A^-1 X.
template <int T, int TX>
__device__ void gj(const W<T>& w, Mat<T>& A, v4d (&X)[T][TX]) {
  constexpr int TT = T + TX;
  constexpr int LW = Lay<T>::LW;
  double* br = w.s + Lay<T>::BR;
  double* bc = w.s + Lay<T>::BC;
#pragma unroll
  for (int tb = 0; tb < T; ++tb)         // the block's tile and register, both static: the tiles
#pragma unroll                           // stay in (accumulation) registers, read and written in place
  for (int qb = 0; qb < 4; ++qb) {       // block rows 4 b + g: tile row tb, register qb
    const int b = 4 * tb + qb;
    wsync();
    // block rows (every lane: its column of each tile) and block columns
    // (the four lanes per row group whose column is 4 qb .. 4 qb + 3)
#pragma unroll
    for (int tj = 0; tj < T; ++tj) {
      const v4d a = A.t[tb][tj];
      br[w.g * LW + 16 * tj + w.c] = a[qb];
    }
#pragma unroll
    for (int tj = 0; tj < TX; ++tj) {
      const v4d a = X[tb][tj];
      br[w.g * LW + 16 * (T + tj) + w.c] = a[qb];
    }
    if ((w.c >> 2) == qb) {
#pragma unroll
      for (int ti = 0; ti < T; ++ti)
#pragma unroll
        for (int q = 0; q < 4; ++q) bc[(16 * ti + w.g + 4 * q) * 5 + (w.c & 3)] = A.t[ti][tb][q];
    }
    wsync();
    // row g of P^-1 for this lane (the only row its B operands need): the
    // solution of P^T y = e_g from an LU factorisation of the 4 x 4 pivot
    // block P without pivoting (every lane factorises; no LDS round trip)
    double M[4][4], rk[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) M[i][j] = br[i * LW + 4 * b + j];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      rk[kk] = rcp_nr(M[kk][kk]);
#pragma unroll
      for (int i = kk + 1; i < 4; ++i) {
        M[i][kk] *= rk[kk];                              // L below the diagonal
#pragma unroll
        for (int j = kk + 1; j < 4; ++j) M[i][j] = fma(-M[i][kk], M[kk][j], M[i][j]);   // U on and above
      }
    }
    double z[4], pr[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {                        // U^T z = e_g
      double acc = (w.g == m) ? 1.0 : 0.0;
#pragma unroll
      for (int p = 0; p < m; ++p) acc = fma(-M[p][m], z[p], acc);
      z[m] = acc * rk[m];
    }
#pragma unroll
    for (int m = 3; m >= 0; --m) {                       // L^T y = z
      double acc = z[m];
#pragma unroll
      for (int p = m + 1; p < 4; ++p) acc = fma(-M[p][m], pr[p], acc);
      pr[m] = acc;
    }
    // B operands: row g of P^-1 [block rows], columns 16 tj + c
    double bop[TT];
#pragma unroll
    for (int tj = 0; tj < TT; ++tj) {
      double sacc = 0.0;
#pragma unroll
      for (int m = 0; m < 4; ++m) sacc = fma(pr[m], br[m * LW + 16 * tj + w.c], sacc);
      bop[tj] = sacc;
    }
    // A operands: -C, C = block columns, zero on the block rows (they are
    // replaced by P^-1 B below: forming them as B - (P - I) P^-1 B would take
    // a small difference of large terms when the pivots are large); lane l
    // takes row 16 ti + c, column g of the block
    double aop[T];
#pragma unroll
    for (int ti = 0; ti < T; ++ti) {
      const int rb = 16 * ti + w.c - 4 * b;
      aop[ti] = (rb >= 0 && rb < 4) ? 0.0 : -bc[(16 * ti + w.c) * 5 + w.g];
    }
#pragma unroll
    for (int ti = 0; ti < T; ++ti) {
#pragma unroll
      for (int tj = 0; tj < T; ++tj) A.t[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop[ti], bop[tj], A.t[ti][tj], 0, 0, 0);
#pragma unroll
      for (int tj = 0; tj < TX; ++tj) X[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop[ti], bop[T + tj], X[ti][tj], 0, 0, 0);
    }
    // the block rows: register qb of tile row tb holds row g of the block,
    // and bop holds row g of P^-1 B in this lane's columns
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (q == qb) {
#pragma unroll
        for (int tj = 0; tj < T; ++tj) A.t[tb][tj][q] = bop[tj];
#pragma unroll
        for (int tj = 0; tj < TX; ++tj) X[tb][tj][q] = bop[T + tj];
      }
  }
}

// up to three compact vectors as the columns 0..2 of a right-hand-side tile
template <int T>
__device__ __forceinline__ void cols_in(const W<T>& w, v4d (&X)[T], double x0, double x1, double x2) {
  wsync();
  vset(w, 2, x0);
  vset(w, 3, x1);
  vset(w, 4, x2);
  wsync();
#pragma unroll
  for (int ti = 0; ti < T; ++ti)
#pragma unroll
    for (int q = 0; q < 4; ++q)
      X[ti][q] = w.c < 3 ? w.s[Lay<T>::VS + (2 + w.c) * Lay<T>::NA + 16 * ti + w.g + 4 * q] : 0.0;
}
template <int T>
__device__ __forceinline__ void cols_out(const W<T>& w, const v4d (&X)[T], double& x0, double& x1, double& x2) {
  wsync();
  if (w.c < 3) {
#pragma unroll
    for (int ti = 0; ti < T; ++ti)
#pragma unroll
      for (int q = 0; q < 4; ++q) w.s[Lay<T>::VS + (2 + w.c) * Lay<T>::NA + 16 * ti + w.g + 4 * q] = X[ti][q];
  }
  wsync();
  x0 = vget(w, 2);
  x1 = vget(w, 3);
  x2 = vget(w, 4);
}

// ---- eigen solution of diag(d) - omega z z^T: lane i < NA finds root i in
// (d_{i-1}, d_i) as org + del by bracketed Newton on the secular function;
// td, tz2, tw: the tables d, w d and w in LDS
template <int NA>
__device__ void secular_root(int i, double om, double lam_prev, const double* td, const double* tz2,
                             const double* tw, double& org, double& del) {
  const double lo = i > 0 ? td[i - 1] : 0.0;
  const double hi = td[i];
  org = hi;
  del = 0.0;
  const double om1 = 1.0 - om;
  if (!(om > 0.0)) return;
  auto feval = [&](double o, double sgn, double x, double& f, double& df) {
    double s = 0.0, s2 = 0.0;
    if (i == 0 && o == 0.0) {
#pragma unroll 8
      for (int j = 0; j < NA; ++j) {
        const double dj = td[j];
        const double r = rcp_nr(dj - sgn * x);
        s = fma(tw[j], r, s);
        s2 = fma(tw[j] * dj, r * r, s2);
      }
      f = om1 - om * x * s;
      df = -om * s2;
    } else {
#pragma unroll 8
      for (int j = 0; j < NA; ++j) {
        const double r = rcp_nr((td[j] - o) - sgn * x);
        s = fma(tz2[j], r, s);
        s2 = fma(tz2[j] * r, r, s2);
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
  if (i == 0 && sgn > 0.0 && om1 <= 0.0) { del = 0.0; return; }
  const double xp = sgn * (lam_prev - org);
  double x = (xp > xl && xp < xh) ? xp : 0.5 * (xl + xh);
  for (int it = 0; it < 200; ++it) {
    double f, df;
    feval(org, sgn, x, f, df);
    if ((f > 0.0) == (sgn > 0.0)) xl = x; else xh = x;
    double xn = x - f * rcp_nr(df * sgn);
    if (fabs(xn - x) <= 2e-16 * x) { x = xn; break; }
    if (!(xn > xl && xn < xh)) xn = 0.5 * (xl + xh);
    const double step = fabs(xn - x);
    x = xn;
    if (step <= 2e-16 * x || xh - xl <= 4e-16 * xh) break;
  }
  del = sgn * x;
}

__device__ __forceinline__ double x_coth_x(double x) {
  if (x < 0.05) {
    const double x2 = x * x;
    return 1.0 + x2 * (1.0 / 3.0 + x2 * (-1.0 / 45.0 + x2 * (2.0 / 945.0)));
  }
  return x / tanh(x);
}

template <int T>
struct Ops {                 // layer operators in scaled variables; vectors compact
  Mat<T> t, r;
  double bc, blp, blm, qv;
};

// m of the rows an element of the tile layout belongs to, from the slab
template <int T>
__device__ __forceinline__ double row_m(const W<T>& w, int ti, int q) {
  return w.s[Lay<T>::TM + 16 * ti + w.g + 4 * q];
}

// eigen solution (V in the slab's A0 area, row-major) and the layer operators
template <int T>
__device__ void layer(const W<T>& w, double om, double Dl, const double* roots, double& om_prev, Ops<T>& o) {
  constexpr int NA = 16 * T;
  constexpr int LA = Lay<T>::LA;
  double* s = w.s;
  const int i = w.lane;
  if (om != om_prev) {
    // the layer's roots (origin and offset), Gu-Eisenstat zhat and column
    // norms, from k_mf_roots
    wsync();
    if (i < NA) {
      s[Lay<T>::RT + 2 * i] = roots[4 * i];
      s[Lay<T>::RT + 2 * i + 1] = roots[4 * i + 1];
      s[Lay<T>::ZH + i] = roots[4 * i + 2];
      s[Lay<T>::NR + i] = roots[4 * i + 3];
    }
    om_prev = om;
  }
  wsync();
  if (i < NA) {
    const double lam = s[Lay<T>::RT + 2 * i] + s[Lay<T>::RT + 2 * i + 1];
    const double k = sqrt(fmax(lam, 0.0));
    const double x = 0.5 * k * Dl;
    s[Lay<T>::TX + i] = k * tanh(x);
    s[Lay<T>::CX + i] = 2.0 * x_coth_x(x);
  }
  // V (row a, column = root ic) into the A0 area
#pragma unroll
  for (int ti = 0; ti < T; ++ti)
#pragma unroll
    for (int tj = 0; tj < T; ++tj)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int a = 16 * ti + w.g + 4 * q, ic = 16 * tj + w.c;
        double v = (a == ic) ? 1.0 : 0.0;
        if (om > 0.0) {
          const double oa = s[Lay<T>::RT + 2 * ic], da = s[Lay<T>::RT + 2 * ic + 1];
          v = s[Lay<T>::ZH + a] * rcp_nr((s[Lay<T>::TD + a] - oa) - da) * s[Lay<T>::NR + ic];
        }
        s[Lay<T>::A0 + a * LA + ic] = v;
      }
  wsync();
  // Q_T = V diag(k tanh x) V^T; F_T = (M + Q_T)^-1; bc needs Q_T F_T sqrt(w)
  Mat<T> FT, FC;
  double qf;
  {
    Mat<T> QT, A;
    mul_ll<T, true>(w, QT, Lay<T>::A0, LA, Lay<T>::A0, LA, Lay<T>::TX);
    v4d X[T][T];
#pragma unroll
    for (int ti = 0; ti < T; ++ti)
#pragma unroll
      for (int tj = 0; tj < T; ++tj)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const bool dg = ti == tj && (w.g + 4 * q) == w.c;
          A.t[ti][tj][q] = QT.t[ti][tj][q] + (dg ? row_m(w, ti, q) : 0.0);
          X[ti][tj][q] = dg ? 1.0 : 0.0;
        }
    gj<T, T>(w, A, X);
#pragma unroll
    for (int ti = 0; ti < T; ++ti)
#pragma unroll
      for (int tj = 0; tj < T; ++tj) FT.t[ti][tj] = X[ti][tj];
    const double fw = mv_slot(w, FT, 5);
    qf = mv(w, QT, fw);
  }
  // Q_C' = V diag(2 x coth x) V^T; F_C' = (D M + Q_C')^-1 (V is still in A0)
  {
    Mat<T> A;
    mul_ll<T, true>(w, A, Lay<T>::A0, LA, Lay<T>::A0, LA, Lay<T>::CX);
    v4d X[T][T];
#pragma unroll
    for (int ti = 0; ti < T; ++ti)
#pragma unroll
      for (int tj = 0; tj < T; ++tj)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const bool dg = ti == tj && (w.g + 4 * q) == w.c;
          A.t[ti][tj][q] += dg ? Dl * row_m(w, ti, q) : 0.0;
          X[ti][tj][q] = dg ? 1.0 : 0.0;
        }
    gj<T, T>(w, A, X);
#pragma unroll
    for (int ti = 0; ti < T; ++ti)
#pragma unroll
      for (int tj = 0; tj < T; ++tj) FC.t[ti][tj] = X[ti][tj];
  }
  // r = M (F_T + D F_C') - I, t = M (F_T - D F_C')
#pragma unroll
  for (int ti = 0; ti < T; ++ti)
#pragma unroll
    for (int tj = 0; tj < T; ++tj)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double ft = FT.t[ti][tj][q], fc = Dl * FC.t[ti][tj][q], m = row_m(w, ti, q);
        const bool dg = ti == tj && (w.g + 4 * q) == w.c;
        o.r.t[ti][tj][q] = m * (ft + fc) - (dg ? 1.0 : 0.0);
        o.t.t[ti][tj][q] = m * (ft - fc);
      }
  // vectors (compact): t sqrt(w), r sqrt(w), F_C' sqrt(w) mu
  const double tw = mv_slot(w, o.t, 5), rw = mv_slot(w, o.r, 5), fq = mv_slot(w, FC, 6);
  const double qv = 2.0 * tab(w, Lay<T>::TM) * fq;
  o.qv = qv;
  o.blp = qv - tw;
  o.blm = (tab(w, Lay<T>::VS + 5 * NA) - rw) - qv;
  o.bc = 2.0 * qf;
}

template <int T>
__device__ __forceinline__ void set_identity_minus(const W<T>& w, Mat<T>& X) {
#pragma unroll
  for (int ti = 0; ti < T; ++ti)
#pragma unroll
    for (int tj = 0; tj < T; ++tj)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        X.t[ti][tj][q] = ((ti == tj && (w.g + 4 * q) == w.c) ? 1.0 : 0.0) - X.t[ti][tj][q];
}

// S: the plan's storage type (inputs, outputs and the workspace); the
// arithmetic is FP64 for both
template <typename S>
struct MfArgs {
  const Item* items;
  const int64_t* off;
  const double* tau;
  const S* q;
  const S* Sg;
  const S* omega;
  const S* Itop;
  const S* Bbot;
  const S* Bbot_prev;
  const S* Ibot;
  S *J, *JmS, *lstar, *lstar_c, *Iplus, *Iminus, *H, *Iemerg;
  S* wsR;          // [rows][nf][NA][NA]
  S* wsS;          // [rows][nf][NA]
  S* wsZ;          // [rows][nf][NA][2]
  double* wsRT;    // [rows][nf][NA][4]: layer (d, d+1): root origin and offset, zhat, column norm
  S* wsO;          // [rows][nf][2 NA^2 + 4 NA]: layer (d, d+1): t, r tiles, then bc, blp, blm, qv
  uint32_t* status;
  unsigned long long* thick_stats;   // FP32 plans: [FP64 eliminations, all eliminations]
  int32_t nf, nitems, lower_bc;
  uint32_t outputs;
};

// The eigen solutions of every layer, apart from the formal solution: one
// thread per (frequency, root), two frequencies per wave, each thread walking
// down its column and starting every layer's Newton iteration from its own
// root of the layer above (the albedo changes with depth in a real
// atmosphere, and inside the one-wave-per-SIMD formal solution these
// iterations were a third of its instructions).  The 32 threads of a column
// then share their roots through LDS for the Gu-Eisenstat zhat_i and the
// column norms, so that the formal solution only assembles V.  A layer whose
// albedo equals the one above keeps its values.
template <int T, typename S>
__global__ __launch_bounds__(64) void k_mf_roots(MfArgs<S> a, MfTab<16 * T> tb) {
  constexpr int NA = 16 * T;
  constexpr int C = 64 / NA;            // columns per wave
  static_assert(64 % NA == 0, "whole columns per wave");
  __shared__ double td[NA], tz2[NA], tw[NA];
  __shared__ double rt[C][2 * NA], zh[C][NA];
  const int t = (int)threadIdx.x;
  if (t < NA) {
    td[t] = tb.d[t];
    tz2[t] = tb.z2[t];
    tw[t] = tb.w[t];
  }
  __syncthreads();
  const int col = t / NA;
  const int item = (int)blockIdx.x * C + col;
  const int i = t % NA;
  if (item >= a.nitems) return;
  const Item it = a.items[item];
  const int nd = it.nd, nf = a.nf, k = it.g;
  if (k >= nf) return;
  const int64_t row0 = a.off[it.b];
  double* out = a.wsRT + ((row0 * nf + k) * NA + i) * 4;
  const int64_t stride = (int64_t)nf * NA * 4;
  double om_prev = -1.0, lam_prev = -1.0, org = 0.0, del = 0.0, zhat = 0.0, nrm = 1.0;
  for (int d = 0; d < nd - 1; ++d) {
    const double om = a.omega ? 0.5 * ((double)a.omega[(row0 + d) * nf + k] + (double)a.omega[(row0 + d + 1) * nf + k])
                              : 0.0;
    const bool fresh = om != om_prev;
    if (fresh) {
      secular_root<NA>(i, om, lam_prev, td, tz2, tw, org, del);
      lam_prev = org + del;
    }
    // (the LDS exchanges stay in this column's own slots; the fences keep
    // each lane's stores ahead of the other lanes' loads in the wave)
    wsync();
    rt[col][2 * i] = org;
    rt[col][2 * i + 1] = del;
    wsync();
    if (fresh && om > 0.0) {
      const double dl = td[i];
      double num = del + (org - dl), den = -om;
#pragma unroll 8
      for (int b2 = 0; b2 < NA; ++b2)
        if (b2 != i) {
          num *= (rt[col][2 * b2] - dl) + rt[col][2 * b2 + 1];
          den *= td[b2] - dl;
        }
      zhat = sqrt(fabs(num / den));
    }
    wsync();
    zh[col][i] = zhat;
    wsync();
    if (fresh) {
      if (om > 0.0) {
        double q2 = 0.0;
#pragma unroll 8
        for (int j = 0; j < NA; ++j) {
          const double q = zh[col][j] * rcp_nr((td[j] - org) - del);
          q2 = fma(q, q, q2);
        }
        nrm = 1.0 / sqrt(q2);
      } else {
        zhat = 0.0;
        nrm = 1.0;
      }
      om_prev = om;
    }
    out[d * stride] = org;
    out[d * stride + 1] = del;
    out[d * stride + 2] = zhat;
    out[d * stride + 3] = nrm;
  }
}

constexpr int kOpsSplit = 16;   // waves per (atmosphere, frequency) forming the layer operators

template <int T, int PASS, typename S>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(PASS == 0 ? 2 : 1)))
void k_fs_dense_mfma(MfArgs<S> a, MfTab<16 * T> tb) {
  constexpr int NA = 16 * T;
  __shared__ double slab[PASS == 0 ? Lay<T>::B0 : Lay<T>::SIZE];
  const int lane = (int)threadIdx.x;
  // PASS 0 forms the layer operators: kOpsSplit waves per (atmosphere,
  // frequency), wave c taking layers c, c + kOpsSplit, ...
  const int item = PASS == 0 ? (int)(blockIdx.x / kOpsSplit) : (int)blockIdx.x;
  if (item >= a.nitems) return;
  const Item it = a.items[item];
  const int b = it.b, nd = it.nd, nf = a.nf;
  const int k = it.g;                    // one frequency per wave
  if (k >= nf) return;
  const int64_t row0 = a.off[b];
  W<T> w{slab, lane, lane >> 4, lane & 15};
  // angle tables into LDS; this lane's constants (angle `lane` of the
  // internal order, external index NA - 1 - lane) in registers
  if (lane < NA) {
    slab[Lay<T>::TM + lane] = tb.m[lane];
    slab[Lay<T>::TD + lane] = tb.d[lane];
    slab[Lay<T>::TMU + lane] = tb.mu[lane];
    slab[Lay<T>::TZ2 + lane] = tb.z2[lane];
    slab[Lay<T>::TW + lane] = tb.w[lane];
    slab[Lay<T>::VS + 5 * NA + lane] = tb.sw[lane];
    slab[Lay<T>::VS + 6 * NA + lane] = tb.swmu[lane];
  }
  wsync();
  const bool act = lane < NA;
  const double sw_l = tab(w, Lay<T>::VS + 5 * NA), swmu_l = tab(w, Lay<T>::VS + 6 * NA);
  const double mu_l = tab(w, Lay<T>::TMU);
  const int ext = NA - 1 - lane;
  const uint32_t o = a.outputs;
  auto at = [&](const S* p, int64_t row) { return (double)p[row * nf + k]; };
  auto layer_depth = [&](int d) {
    return 0.5 * (at(a.q, row0 + d) + at(a.q, row0 + d + 1)) * (a.tau[row0 + d + 1] - a.tau[row0 + d]);
  };
  auto layer_omega = [&](int d) {
    return a.omega ? 0.5 * (at(a.omega, row0 + d) + at(a.omega, row0 + d + 1)) : 0.0;
  };
  const int64_t strideR = (int64_t)nf * NA * NA, strideS = (int64_t)nf * NA, strideZ = (int64_t)nf * NA * 2;
  S* wsR = a.wsR + (row0 * nf + k) * NA * NA;
  S* wsS = a.wsS + (row0 * nf + k) * NA;
  S* wsZ = a.wsZ + (row0 * nf + k) * NA * 2;
  const bool wd = (o & PPRT_OUT_LSTAR) != 0;
  const bool we = (o & PPRT_OUT_LSTAR_C) != 0;
  double om_prev = -1.0;
  const double* wsRT = a.wsRT + (row0 * nf + k) * NA * 4;   // + layer * nf * NA * 4
  const int64_t strideRT = (int64_t)nf * NA * 4;
  Ops<T> op;

  auto save_mat = [&](S* dst, const Mat<T>& M) {
#pragma unroll
    for (int ti = 0; ti < T; ++ti)
#pragma unroll
      for (int tj = 0; tj < T; ++tj)
#pragma unroll
        for (int q = 0; q < 4; ++q) dst[(16 * ti + w.g + 4 * q) * NA + 16 * tj + w.c] = (S)M.t[ti][tj][q];
  };
  auto load_mat = [&](const S* src, Mat<T>& M) {
#pragma unroll
    for (int ti = 0; ti < T; ++ti)
#pragma unroll
      for (int tj = 0; tj < T; ++tj)
#pragma unroll
        for (int q = 0; q < 4; ++q) M.t[ti][tj][q] = (double)src[(16 * ti + w.g + 4 * q) * NA + 16 * tj + w.c];
  };
  // the layer operators of layer (d, d+1), kept by pass 1 for pass 2 in the
  // plan's type; an FP32 plan rounds them before pass 1 uses them, so that
  // both passes work with the same operators
  constexpr int64_t OPS = 2 * NA * NA + 4 * NA;
  using S4 = S __attribute__((ext_vector_type(4)));
  auto ops_at = [&](int d) { return a.wsO + ((row0 + d) * nf + k) * OPS; };
  auto cvt4 = [](const v4d& x) { return S4{(S)x[0], (S)x[1], (S)x[2], (S)x[3]}; };
  auto save_ops = [&](int d, Ops<T>& op) {
    S* p = ops_at(d);
#pragma unroll
    for (int ti = 0; ti < T; ++ti)
#pragma unroll
      for (int tj = 0; tj < T; ++tj) {
        const int o4 = ((ti * T + tj) * 64 + lane) * 4;
        const S4 t4 = cvt4(op.t.t[ti][tj]), r4 = cvt4(op.r.t[ti][tj]);
        *(S4*)(p + o4) = t4;
        *(S4*)(p + NA * NA + o4) = r4;
        if constexpr (sizeof(S) == 4) {
          op.t.t[ti][tj] = v4d{(double)t4[0], (double)t4[1], (double)t4[2], (double)t4[3]};
          op.r.t[ti][tj] = v4d{(double)r4[0], (double)r4[1], (double)r4[2], (double)r4[3]};
        }
      }
    const S4 v = S4{(S)op.bc, (S)op.blp, (S)op.blm, (S)op.qv};
    if (lane < NA) *(S4*)(p + 2 * NA * NA + 4 * lane) = v;
    if constexpr (sizeof(S) == 4) {
      op.bc = (double)v[0];
      op.blp = (double)v[1];
      op.blm = (double)v[2];
      op.qv = (double)v[3];
    }
  };
  auto load_ops = [&](int d, Ops<T>& op) {
    const S* p = ops_at(d);
#pragma unroll
    for (int ti = 0; ti < T; ++ti)
#pragma unroll
      for (int tj = 0; tj < T; ++tj) {
        const int o4 = ((ti * T + tj) * 64 + lane) * 4;
        const S4 t4 = *(const S4*)(p + o4), r4 = *(const S4*)(p + NA * NA + o4);
        op.t.t[ti][tj] = v4d{(double)t4[0], (double)t4[1], (double)t4[2], (double)t4[3]};
        op.r.t[ti][tj] = v4d{(double)r4[0], (double)r4[1], (double)r4[2], (double)r4[3]};
      }
    // lanes past NA hold zeros in compact vectors
    const S4 v = lane < NA ? *(const S4*)(p + 2 * NA * NA + 4 * lane) : S4{0, 0, 0, 0};
    op.bc = (double)v[0];
    op.blp = (double)v[1];
    op.blm = (double)v[2];
    op.qv = (double)v[3];
  };

  if constexpr (PASS == 0) {
    // ---- the layer operators (the roots of a layer depend on its albedo
    // alone, so a layer with the albedo of this wave's previous one keeps them)
    for (int d = (int)(blockIdx.x % kOpsSplit); d < nd - 1; d += kOpsSplit) {
      layer<T>(w, layer_omega(d), layer_depth(d), wsRT + d * strideRT, om_prev, op);
      save_ops(d, op);
    }
  } else if constexpr (PASS == 1) {
    // ---- pass 1: top -> bottom, composite R and Sigma of every node
    Mat<T> R;
#pragma unroll
    for (int ti = 0; ti < T; ++ti)
#pragma unroll
      for (int tj = 0; tj < T; ++tj) R.t[ti][tj] = v4d{0.0, 0.0, 0.0, 0.0};
    double Sig = 0.0;
    if (act) {
      const double It = a.Itop ? (double)a.Itop[((int64_t)b * nf + k) * NA + ext] : 0.0;
      Sig = sw_l * (It - at(a.Sg, row0));
    }
    for (int d = 0; d < nd - 1; ++d) {
      save_mat(wsR + d * strideR, R);
      if (act) wsS[d * strideS + lane] = (S)Sig;
      load_ops(d, op);
      const double dSg = at(a.Sg, row0 + d + 1) - at(a.Sg, row0 + d);
      // G = (I - r R)^-1: P = G t, u = G (r Sigma + dS^g Q) and the unit
      // responses G beta_l+ and G Q, from one elimination on I - r R
      Mat<T> A;
      mul(w, A, op.r, R);
      set_identity_minus(w, A);
      const double u = fma(dSg, op.qv, mv(w, op.r, Sig));
      v4d X[T][T + 1];
      v4d xc[T];
      cols_in(w, xc, u, op.blp, op.qv);
#pragma unroll
      for (int ti = 0; ti < T; ++ti) {
#pragma unroll
        for (int tj = 0; tj < T; ++tj) X[ti][tj] = op.t.t[ti][tj];
        X[ti][T] = xc[ti];
      }
      gj<T, T + 1>(w, A, X);
      Mat<T> P;
#pragma unroll
      for (int ti = 0; ti < T; ++ti) {
#pragma unroll
        for (int tj = 0; tj < T; ++tj) P.t[ti][tj] = X[ti][tj];
        xc[ti] = X[ti][T];
      }
      double uu, y1, y2;
      cols_out(w, xc, uu, y1, y2);
      if (wd) {
        const double z = mv(w, R, y1);
        if (act) wsZ[d * strideZ + 2 * lane] = (S)z;
      }
      if (we) {
        const double z = mv(w, R, y2);
        if (act) wsZ[d * strideZ + 2 * lane + 1] = (S)z;
      }
      // Sigma_{d+1} = t (Sigma + R u) - dS^g Q,  R_{d+1} = r + t R P
      const double Ru = mv(w, R, uu);
      Sig = fma(-dSg, op.qv, mv(w, op.t, Sig + Ru));
      Mat<T> RP, tRP;
      mul(w, RP, R, P);
      mul(w, tRP, op.t, RP);
#pragma unroll
      for (int ti = 0; ti < T; ++ti)
#pragma unroll
        for (int tj = 0; tj < T; ++tj) R.t[ti][tj] = op.r.t[ti][tj] + tRP.t[ti][tj];
    }
    save_mat(wsR + (nd - 1) * strideR, R);
    if (act) wsS[(nd - 1) * strideS + lane] = (S)Sig;
    if (sizeof(S) == 4 && a.thick_stats && lane == 0) {   // every elimination here is FP64
      atomicAdd(&a.thick_stats[0], (unsigned long long)(nd - 1));
      atomicAdd(&a.thick_stats[1], (unsigned long long)(nd - 1));
    }
  } else {
    // ---- pass 2: bottom -> top, outputs per node
    bool nonfinite = false;
    Mat<T> Rup;
#pragma unroll
    for (int ti = 0; ti < T; ++ti)
#pragma unroll
      for (int tj = 0; tj < T; ++tj) Rup.t[ti][tj] = v4d{0.0, 0.0, 0.0, 0.0};
    double Sup = 0.0, dSu = 0.0, eSu = -sw_l;
    if (act) {
      const double S_last = at(a.Sg, row0 + nd - 1);
      if (a.lower_bc == PPRT_BC_DIFFUSION) {
        const double Bb = (double)a.Bbot[(int64_t)b * nf + k];
        const double Bp = (double)a.Bbot_prev[(int64_t)b * nf + k];
        const double gr = (Bb - Bp) / layer_depth(nd - 2);
        Sup = sw_l * ((Bb - S_last) + mu_l * gr);
      } else {
        const double Ib = a.Ibot ? (double)a.Ibot[((int64_t)b * nf + k) * NA + ext] : 0.0;
        Sup = sw_l * (Ib - S_last);
      }
    }
    for (int d = nd - 1; d >= 0; --d) {
      const bool has_a = d >= 1;
      if (has_a) load_ops(d - 1, op);
      Mat<T> Rd;
      load_mat(wsR + d * strideR, Rd);
      const double Sd = act ? (double)wsS[d * strideS + lane] : 0.0;
      // unit responses of the layer above (plain form for Lambda*, difference
      // form for 1 - Lambda*), from R_{d-1} G_{d-1} (beta_l+, Q) of pass 1
      double dS = 0.0, eS = -sw_l;
      if (has_a) {
        if (wd) dS = mv(w, op.t, act ? (double)wsZ[(d - 1) * strideZ + 2 * lane] : 0.0) + op.blm;
        if (we) eS = mv(w, op.t, act ? (double)wsZ[(d - 1) * strideZ + 2 * lane + 1] : 0.0) - op.qv;
      }
      // I+ and the two responses from one elimination on I - R^up R_d
      double Ip = mv(w, Rup, Sd) + Sup;
      double dIp = wd ? mv(w, Rup, dS) + dSu : 0.0;
      double eDp = we ? mv(w, Rup, eS) + eSu : 0.0;
      {
        Mat<T> A;
        mul(w, A, Rup, Rd);
        set_identity_minus(w, A);
        v4d X[T][1];
        v4d xc[T];
        cols_in(w, xc, Ip, dIp, eDp);
#pragma unroll
        for (int ti = 0; ti < T; ++ti) X[ti][0] = xc[ti];
        gj<T, 1>(w, A, X);
#pragma unroll
        for (int ti = 0; ti < T; ++ti) xc[ti] = X[ti][0];
        cols_out(w, xc, Ip, dIp, eDp);
      }
      // Ip, Im are the scaled differences sqrt(w) (I+- - S^g)
      const double Im = mv(w, Rd, Ip) + Sd;
      const double JmSn = 0.5 * dot(sw_l, Ip + Im);
      const double Hn = 0.5 * dot(swmu_l, Ip - Im);
      double Ln = 0.0, Lcn = 0.0;
      if (wd) Ln = 0.5 * dot(sw_l, dIp + mv(w, Rd, dIp) + dS);
      if (we) Lcn = -0.5 * dot(sw_l, eDp + mv(w, Rd, eDp) + eS);
      // a zero or non-finite pivot in any elimination ends up here
      nonfinite |= !isfinite(JmSn + Hn + Ln + Lcn);
      {
        const int64_t x = (row0 + d) * nf + k;
        const double Sx = (double)a.Sg[x];
        if (lane == 0) {
          if (o & PPRT_OUT_J) a.J[x] = (S)(JmSn + Sx);
          if (o & PPRT_OUT_JMS) a.JmS[x] = (S)JmSn;
          if (o & PPRT_OUT_LSTAR) a.lstar[x] = (S)Ln;
          if (o & PPRT_OUT_LSTAR_C) a.lstar_c[x] = (S)Lcn;
          if (o & PPRT_OUT_H) a.H[x] = (S)Hn;
        }
        if (act) {
          if (o & PPRT_OUT_IPLUS) a.Iplus[x * NA + ext] = (S)(Ip / sw_l + Sx);
          if (o & PPRT_OUT_IMINUS) a.Iminus[x * NA + ext] = (S)(Im / sw_l + Sx);
          if (d == 0 && (o & PPRT_OUT_IEMERG)) a.Iemerg[((int64_t)b * nf + k) * NA + ext] = (S)(Ip / sw_l + Sx);
        }
      }
      // move the lower composite up through layer a = d - 1
      if (has_a) {
        const double dSg = at(a.Sg, row0 + d) - at(a.Sg, row0 + d - 1);
        // R^up G^up = R^up (I - r R^up)^-1 = (I - R^up r)^-1 R^up
        Mat<T> A;
        mul(w, A, Rup, op.r);
        set_identity_minus(w, A);
        v4d X[T][T];
#pragma unroll
        for (int ti = 0; ti < T; ++ti)
#pragma unroll
          for (int tj = 0; tj < T; ++tj) X[ti][tj] = Rup.t[ti][tj];
        gj<T, T>(w, A, X);
        Mat<T> RG;
#pragma unroll
        for (int ti = 0; ti < T; ++ti)
#pragma unroll
          for (int tj = 0; tj < T; ++tj) RG.t[ti][tj] = X[ti][tj];
        const double w1 = mv(w, RG, fma(-dSg, op.qv, mv(w, op.r, Sup)));
        const double Sup_n = fma(dSg, op.qv, mv(w, op.t, Sup + w1));
        // unit response of layer a seen from node d - 1
        if (wd) dSu = mv(w, op.t, mv(w, RG, op.bc - op.blm)) + (op.bc - op.blp);
        if (we) eSu = mv(w, op.t, mv(w, RG, op.qv)) - op.qv;
        Sup = act ? Sup_n : 0.0;
        Mat<T> RGt, tRGt;
        mul(w, RGt, RG, op.t);
        mul(w, tRGt, op.t, RGt);
#pragma unroll
        for (int ti = 0; ti < T; ++ti)
#pragma unroll
          for (int tj = 0; tj < T; ++tj) Rup.t[ti][tj] = op.r.t[ti][tj] + tRGt.t[ti][tj];
      }
    }
    if (nonfinite && a.status && lane == 0) atomicOr(a.status, PPRT_DEV_NONFINITE);
    if (sizeof(S) == 4 && a.thick_stats && lane == 0) {
      atomicAdd(&a.thick_stats[0], (unsigned long long)(2 * nd - 1));
      atomicAdd(&a.thick_stats[1], (unsigned long long)(2 * nd - 1));
    }
  }
}

template <int T, typename S>
hipError_t run_mfma(const DenseLaunch& L, hipStream_t s) {
  constexpr int NA = 16 * T;
  MfArgs<S> a{};
  a.items = L.items; a.off = L.off; a.tau = L.tau;
  a.q = (const S*)L.q; a.Sg = (const S*)L.Sg; a.omega = (const S*)L.omega;
  a.Itop = (const S*)L.Itop; a.Bbot = (const S*)L.Bbot; a.Bbot_prev = (const S*)L.Bbot_prev;
  a.Ibot = (const S*)L.Ibot;
  a.J = (S*)L.J; a.JmS = (S*)L.JmS; a.lstar = (S*)L.lstar; a.lstar_c = (S*)L.lstar_c;
  a.Iplus = (S*)L.Iplus; a.Iminus = (S*)L.Iminus; a.H = (S*)L.H; a.Iemerg = (S*)L.Iemerg;
  const size_t rf = (size_t)L.rows * L.nf;
  a.wsR = (S*)L.ws;
  a.wsS = a.wsR + rf * NA * NA;
  a.wsZ = a.wsS + rf * NA;
  a.wsRT = (double*)(a.wsZ + rf * NA * 2);
  a.wsO = (S*)(a.wsRT + rf * NA * 4);
  a.status = L.status;
  a.thick_stats = L.thick_stats;
  a.nf = L.nf; a.nitems = L.nitems; a.lower_bc = L.lower_bc; a.outputs = L.outputs;
  MfTab<NA> tb{};
  for (int i = 0; i < NA; ++i) {
    const int e = NA - 1 - i;
    const double m = L.mu[e], wt = L.w[e];
    tb.mu[i] = m; tb.m[i] = 1.0 / m; tb.d[i] = 1.0 / (m * m); tb.w[i] = wt;
    tb.z2[i] = wt / (m * m); tb.sw[i] = sqrt(wt); tb.swmu[i] = sqrt(wt) * m;
  }
  hipLaunchKernelGGL((k_mf_roots<T, S>), dim3((L.nitems + 64 / NA - 1) / (64 / NA)), dim3(64), 0, s, a, tb);
  hipLaunchKernelGGL((k_fs_dense_mfma<T, 0, S>), dim3(L.nitems * kOpsSplit), dim3(64), 0, s, a, tb);
  hipLaunchKernelGGL((k_fs_dense_mfma<T, 1, S>), dim3(L.nitems), dim3(64), 0, s, a, tb);
  hipLaunchKernelGGL((k_fs_dense_mfma<T, 2, S>), dim3(L.nitems), dim3(64), 0, s, a, tb);
  return hipGetLastError();
}

}  // namespace

bool dense_mfma_na(int na) { return na == 32; }

size_t dense_mfma_workspace_bytes(int na, int64_t rows, int nf, int precision) {
  // R, Sigma and the two unit-source responses in the plan's type, per layer
  // and root the origin, offset, zhat and column norm in FP64, and each
  // layer's t, r and four source vectors in the plan's type
  const size_t rf = (size_t)rows * nf;
  const size_t es = precision == PPRT_FP64 ? sizeof(double) : sizeof(float);
  return rf * (size_t)(na * na + 3 * na) * es + rf * (size_t)(4 * na) * sizeof(double) +
         rf * (size_t)(2 * na * na + 4 * na) * es;
}

hipError_t launch_fs_dense_mfma(const DenseLaunch& L, hipStream_t s) {
  if (L.nitems == 0) return hipSuccess;
  if (L.na == 32) return L.precision == PPRT_FP64 ? run_mfma<2, double>(L, s) : run_mfma<2, float>(L, s);
  return hipErrorInvalidValue;
}

}  // namespace pprt

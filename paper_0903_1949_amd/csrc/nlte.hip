// Multilevel atom on gfx950, FP64: opacity/source assembly from populations,
// preconditioned radiative rates and the per-depth statistical-equilibrium
// solve.
//
// Reading (the paper's notation names the rate operators [R_ij], [R*_ij],
// [Delta R_ij] and a rate matrix A; the scattering problem is solved by
// operator splitting, Sect. 2): full preconditioning of Rybicki & Hummer
// (1991) with the diagonal Lambda*.  For transition t = (l < u) and a
// frequency k of its window (each frequency belongs to one transition):
//     chi_t = (n_l - n_u G) sigma,  eta_t = n_u b G sigma,  kappa = chi_t + kappa_c,
//     q = kappa + sigma_c,  omega = sigma_c / q,  S^g = (eta_t + kappa_c B) / kappa,
//     dJ = J - Lambda* eta_t / kappa                       (old populations)
//     [dR_lu] = sum_k W sigma dJ,   [dR_ul] = sum_k W G sigma dJ,
//     [R*_ul] = sum_k W b G sigma (1 - p Lambda*),  p = chi_t / kappa,
// and per depth  sum_{j!=i} n_j P_ji - n_i sum_{j!=i} P_ij = 0 (i != 0),
// sum n = n_tot, with P_lu = [dR_lu] + C_lu, P_ul = [R*_ul] + [dR_ul] + C_ul,
// solved by LU with partial pivoting for n_i / n_i^old (columns scaled by the
// previous populations: the unknowns span many decades).
#include <cmath>

#include "pprt_internal.h"

namespace pprt {
namespace {

// H(a, x) = Re w(x + i a) by Weideman's expansion (coefficients in vc):
// with i z = -a + i x,  L - i z = (L + a) - i x,  L + i z = (L - a) + i x.
__device__ __forceinline__ double voigt_H(const VoigtCoef& vc, double aa, double x) {
  const double L = vc.L;
  const double dr = L + aa, di = -x;             // L - i z
  const double nr = L - aa, ni = x;              // L + i z
  const double den = dr * dr + di * di;
  const double zr = (nr * dr + ni * di) / den;   // Z = (L + i z) / (L - i z)
  const double zi = (ni * dr - nr * di) / den;
  double pr = vc.a[kVoigtN], pi = 0.0;
  for (int n = kVoigtN - 1; n >= 1; --n) {       // p = sum a_{n+1} Z^n by Horner
    const double tr = pr * zr - pi * zi + vc.a[n];
    pi = pr * zi + pi * zr;
    pr = tr;
  }
  // 1 / (L - i z) = (dr - i di) / den
  const double ur = dr / den, ui = -di / den;
  const double u2r = ur * ur - ui * ui, u2i = 2.0 * ur * ui;
  const double wr = 2.0 * (pr * u2r - pi * u2i) + 0.56418958354775628695 * ur;   // 1/sqrt(pi)
  return wr;
}

// cross-section of the point (row r, frequency k) owned by transition t
__device__ __forceinline__ double cross_section(const MlArgs& a, int64_t r, int k, int t) {
  if (a.line_a != nullptr) {
    const double nu0 = a.line_nu0[t];
    if (nu0 > 0.0) {
      const double dnu = nu0 * a.dopp[r];
      const double x = (a.nu[k] - nu0) / dnu;
      return a.line_s[t] * voigt_H(a.vc, a.line_a[t], x) * (0.56418958354775628695 / dnu);
    }
  }
  return a.sigma[k];
}

// level indices of transition t inside [0, nlev) with lower < upper
__device__ __forceinline__ bool level_pair_ok(const MlArgs& a, int t) {
  const int l = a.lower[t], u = a.upper[t];
  return l >= 0 && u < a.nlev && l < u;
}

__global__ void k_voigt(VoigtCoef vc, int64_t n, const double* __restrict__ av,
                        const double* __restrict__ xv, double* __restrict__ H) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) H[i] = voigt_H(vc, av[i], xv[i]);
}

__global__ void k_ml_opacity(MlArgs a, double* __restrict__ q, double* __restrict__ om,
                             double* __restrict__ Sg) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= a.rows * a.nf) return;
  const int64_t r = x / a.nf;
  const int k = (int)(x - r * a.nf);
  const int t = a.owner[k];
  // the host validates the tables; a table rewritten since then cannot
  // make this kernel read out of bounds
  if (t < 0 || t >= a.ntr || !level_pair_ok(a, t)) {
    if (a.status) atomicOr(a.status, PPRT_DEV_BADINDEX);
    return;
  }
  const double nl = a.pops[r * a.nlev + a.lower[t]];
  const double nu = a.pops[r * a.nlev + a.upper[t]];
  const double G = a.G[x], s = cross_section(a, r, k, t);
  const double chi = (nl - nu * G) * s;
  const double eta = nu * a.bfac[k] * G * s;
  const double kap = chi + a.kc[r];
  const double qq = kap + a.sc[r];
  q[x] = qq;
  om[x] = a.sc[r] / qq;
  Sg[x] = (eta + a.kc[r] * a.Bnu[x]) / kap;
}

// one wave per (row, transition): sums over the transition's window
__global__ __launch_bounds__(64) void k_ml_rates(MlArgs a, const double* __restrict__ J,
                                                 const double* __restrict__ L,
                                                 double* __restrict__ dRlu, double* __restrict__ dRul,
                                                 double* __restrict__ Rsul) {
  const int64_t r = blockIdx.x;
  const int t = blockIdx.y;
  const int lane = threadIdx.x;
  if (!level_pair_ok(a, t) || a.k0[t] < 0 || a.k1[t] > a.nf) {
    if (lane == 0 && a.status) atomicOr(a.status, PPRT_DEV_BADINDEX);
    return;
  }
  const double nl = a.pops[r * a.nlev + a.lower[t]];
  const double nu = a.pops[r * a.nlev + a.upper[t]];
  double s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (int k = a.k0[t] + lane; k < a.k1[t]; k += 64) {
    const int64_t x = r * a.nf + k;
    const double G = a.G[x], s = cross_section(a, r, k, t), W = a.W[k];
    const double chi = (nl - nu * G) * s;
    const double U = a.bfac[k] * G * s;
    const double kap = chi + a.kc[r];
    const double lam = L[x];
    const double dJ = J[x] - lam * (nu * U) / kap;
    s1 = fma(W * s, dJ, s1);
    s2 = fma(W * G * s, dJ, s2);
    s3 = fma(W * U, 1.0 - (chi / kap) * lam, s3);
  }
  __shared__ double red[3][64];
  red[0][lane] = s1;
  red[1][lane] = s2;
  red[2][lane] = s3;
  __syncthreads();
  for (int h = 32; h > 0; h >>= 1) {
    if (lane < h) {
      red[0][lane] += red[0][lane + h];
      red[1][lane] += red[1][lane + h];
      red[2][lane] += red[2][lane + h];
    }
    __syncthreads();
  }
  if (lane == 0) {
    dRlu[r * a.ntr + t] = red[0][0];
    dRul[r * a.ntr + t] = red[1][0];
    Rsul[r * a.ntr + t] = red[2][0];
  }
}

constexpr int kMaxLev = 32;

// one block per atmosphere; each thread solves the systems of its rows
__global__ __launch_bounds__(128) void k_ml_solve(MlArgs a, const int64_t* __restrict__ off,
                                                  const double* __restrict__ dRlu,
                                                  const double* __restrict__ dRul,
                                                  const double* __restrict__ Rsul,
                                                  double* __restrict__ pops_new,
                                                  double* __restrict__ max_rel,
                                                  uint32_t* __restrict__ status, MlSolveCtl ctl) {
  __shared__ double red[128];
  const int b = blockIdx.x;
  const int n = a.nlev;
  if (ctl.active != nullptr && ctl.active[b] == 0) {   // converged: keep the populations
    for (int64_t x = off[b] * n + threadIdx.x; x < off[b + 1] * n; x += blockDim.x)
      pops_new[x] = a.pops[x];
    return;
  }
  double mx = 0.0;
  uint32_t bad = 0;
  for (int64_t r = off[b] + threadIdx.x; r < off[b + 1]; r += blockDim.x) {
    double A[kMaxLev][kMaxLev];
    double x[kMaxLev];
    for (int i = 0; i < n; ++i) {
      x[i] = 0.0;
      for (int j = 0; j < n; ++j) A[i][j] = 0.0;
    }
    // A[i][j] += rate j -> i ; A[i][i] -= rates out of i
    for (int t = 0; t < a.ntr; ++t) {
      const int l = a.lower[t], u = a.upper[t];
      if (!(l >= 0 && u < n && l < u)) { bad |= PPRT_DEV_BADINDEX; continue; }
      const int64_t y = r * a.ntr + t;
      const double Plu = dRlu[y] + a.Clu[y];
      const double Pul = Rsul[y] + dRul[y] + a.Cul[y];
      A[u][l] += Plu;
      A[l][l] -= Plu;
      A[l][u] += Pul;
      A[u][u] -= Pul;
    }
    for (int j = 0; j < n; ++j) A[0][j] = 1.0;   // number conservation
    x[0] = a.ntot[r];
    // unknowns n_i / n_i^old: scale the columns by the previous populations
    double sc[kMaxLev];
    for (int j = 0; j < n; ++j) {
      sc[j] = a.pops[r * n + j];
      for (int i = 0; i < n; ++i) A[i][j] *= sc[j];
    }
    // LU with partial pivoting, forward/back substitution.  A column with
    // no nonzero (or no finite) pivot makes the system singular: the row
    // keeps its old populations and the SINGULAR bit is raised.
    bool singular = false;
    for (int c = 0; c < n; ++c) {
      int p = c;
      double best = fabs(A[c][c]);
      for (int i = c + 1; i < n; ++i)
        if (fabs(A[i][c]) > best) { best = fabs(A[i][c]); p = i; }
      if (!(best > 0.0) || !isfinite(best)) { singular = true; break; }
      if (p != c) {
        for (int j = 0; j < n; ++j) { const double tmp = A[c][j]; A[c][j] = A[p][j]; A[p][j] = tmp; }
        const double tmp = x[c]; x[c] = x[p]; x[p] = tmp;
      }
      const double inv = 1.0 / A[c][c];
      for (int i = c + 1; i < n; ++i) {
        const double f = A[i][c] * inv;
        if (f != 0.0) {
          for (int j = c; j < n; ++j) A[i][j] = fma(-f, A[c][j], A[i][j]);
          x[i] = fma(-f, x[c], x[i]);
        }
      }
    }
    if (singular) {
      bad |= PPRT_DEV_SINGULAR;
      for (int i = 0; i < n; ++i) pops_new[r * n + i] = a.pops[r * n + i];
      continue;
    }
    for (int c = n - 1; c >= 0; --c) {
      double s = x[c];
      for (int j = c + 1; j < n; ++j) s = fma(-A[c][j], x[j], s);
      x[c] = s / A[c][c];
    }
    for (int i = 0; i < n; ++i) x[i] *= sc[i];
    for (int i = 0; i < n; ++i) {
      const double old = a.pops[r * n + i];
      const double rel = fabs(x[i] - old) / fabs(x[i]);
      if (!isfinite(x[i])) bad |= PPRT_DEV_NONFINITE;
      mx = fmax(mx, isfinite(rel) ? rel : INFINITY);
      pops_new[r * n + i] = x[i];
    }
  }
  if (bad && status) atomicOr(status, bad);
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (max_rel) max_rel[b] = red[0];
    if (ctl.iters != nullptr) {
      const int it = (ctl.iters[b] += 1);
      if (ctl.active != nullptr && (red[0] < ctl.tol || (ctl.max_iter > 0 && it >= ctl.max_iter)))
        ctl.active[b] = 0;
    }
  }
}

__global__ void k_gather_bottom(const double* __restrict__ Bnu, const int64_t* __restrict__ off,
                                int nb, int nf, double* __restrict__ Bb, double* __restrict__ Bp) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= (int64_t)nb * nf) return;
  const int b = (int)(x / nf);
  const int k = (int)(x - (int64_t)b * nf);
  const int64_t last = off[b + 1] - 1;
  Bb[x] = Bnu[last * nf + k];
  Bp[x] = Bnu[(last - 1) * nf + k];
}

}  // namespace

int ml_max_levels() { return kMaxLev; }

hipError_t launch_ml_opacity(const MlArgs& a, double* q, double* om, double* Sg, hipStream_t s) {
  const int64_t n = a.rows * a.nf;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ml_opacity, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, q, om, Sg);
  return hipGetLastError();
}

hipError_t launch_ml_rates(const MlArgs& a, const double* J, const double* L, double* dRlu,
                           double* dRul, double* Rsul, hipStream_t s) {
  if (a.rows == 0 || a.ntr == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ml_rates, dim3((unsigned)a.rows, (unsigned)a.ntr), dim3(64), 0, s, a, J, L,
                     dRlu, dRul, Rsul);
  return hipGetLastError();
}

hipError_t launch_ml_solve(const MlArgs& a, const int64_t* off, int nb, const double* dRlu,
                           const double* dRul, const double* Rsul, double* pops_new, double* max_rel,
                           uint32_t* status, hipStream_t s, const MlSolveCtl& ctl) {
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ml_solve, dim3(nb), dim3(128), 0, s, a, off, dRlu, dRul, Rsul, pops_new,
                     max_rel, status, ctl);
  return hipGetLastError();
}

hipError_t launch_gather_bottom(const double* Bnu, const int64_t* off, int nb, int nf, double* Bb,
                                double* Bp, hipStream_t s) {
  const int64_t n = (int64_t)nb * nf;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_bottom, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Bnu, off,
                     nb, nf, Bb, Bp);
  return hipGetLastError();
}

const VoigtCoef& voigt_coefficients() {
  // Fourier cosine coefficients of F(theta) = exp(-t^2)(L^2 + t^2),
  // t = L tan(theta/2), on the M = 2N point grid theta_k = k pi / M
  // (F is even and vanishes at theta = pi), as Weideman's method prescribes.
  static const VoigtCoef vc = [] {
    VoigtCoef c{};
    const int N = kVoigtN, M = 2 * N;
    const double pi = 3.14159265358979323846;
    c.L = std::sqrt(N / std::sqrt(2.0));
    for (int n = 0; n <= N; ++n) {
      double acc = 0.5 * c.L * c.L;              // theta = 0 term, weight 1/2
      for (int k = 1; k < M; ++k) {
        const double th = k * pi / M;
        const double t = c.L * std::tan(0.5 * th);
        acc += std::exp(-t * t) * (c.L * c.L + t * t) * std::cos(n * th);
      }
      c.a[n] = acc / M;
    }
    return c;
  }();
  return vc;
}

hipError_t launch_voigt(int64_t n, const double* a, const double* x, double* H, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_voigt, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, voigt_coefficients(),
                     n, a, x, H);
  return hipGetLastError();
}

}  // namespace pprt

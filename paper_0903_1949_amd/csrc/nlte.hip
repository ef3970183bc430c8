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
constexpr int kSolveWaves = 4;            // waves per block
constexpr int kSolveChunk = 2 * kSolveWaves;   // depth rows per block (more past 524,280 depths)
constexpr int kSolveLd = kMaxLev + 1;     // LDS row stride of the assembled matrix

// value of v in lane l (l uniform)
__device__ __forceinline__ double lane_value(double v, int l) {
  const long long bits = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(bits & 0xffffffffll), l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(bits >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Statistical equilibrium per depth: one wave per depth row.  Lane i
// assembles row i of the rate matrix in the wave's LDS (in transition order,
// so the sums are the same on every run), then keeps it in registers (static
// column indices: no private memory) for an LU factorisation with partial
// pivoting in which the pivot rows stay in their lanes: each step picks the
// largest remaining |A_ic| by a wave reduction (ties to the lowest row) and
// reads the pivot row from its lane; one step of iterative refinement
// follows.  Unknowns are n_i / n_i^old (columns scaled by the previous
// populations), row 0 is number conservation.
//
// Block (b, c) takes depth rows c chunk .. (c + 1) chunk - 1 of
// atmosphere b, so that an atmosphere's depths spread over the whole chip
// (the 512 depths of one atmosphere ran on a single block of four waves
// before: 9.9 ms for a 20-level atom), and stores the largest relative change
// of its rows in part[b][c]; k_ml_solve_fin takes each atmosphere's maximum
// over its chunks (a maximum, so the order does not matter) and applies the
// convergence control.
__global__ __launch_bounds__(64 * kSolveWaves) void k_ml_solve(
    MlArgs a, const int64_t* __restrict__ off, const double* __restrict__ dRlu,
    const double* __restrict__ dRul, const double* __restrict__ Rsul, double* __restrict__ pops_new,
    double* __restrict__ part, int chunk, int nchunk, uint32_t* __restrict__ status, MlSolveCtl ctl) {
  __shared__ double Ms[kSolveWaves][kMaxLev * kSolveLd];
  __shared__ double red[kSolveWaves];
  const int b = blockIdx.x;
  const int64_t r0 = off[b] + (int64_t)blockIdx.y * chunk;
  const int64_t r1 = r0 + chunk < off[b + 1] ? r0 + chunk : off[b + 1];
  if (r0 >= r1) return;                              // past this atmosphere's depths
  const int n = a.nlev;
  const int lane = (int)(threadIdx.x & 63);
  const int wv = (int)(threadIdx.x >> 6);
  if (ctl.active != nullptr && ctl.active[b] == 0) {   // converged: keep the populations
    for (int64_t x = r0 * n + threadIdx.x; x < r1 * n; x += blockDim.x)
      pops_new[x] = a.pops[x];
    return;
  }
  double* M = Ms[wv];
  double mx = 0.0;
  uint32_t bad = 0;
  for (int64_t r = r0 + wv; r < r1; r += kSolveWaves) {
    // the previous row's reads of the slab are done
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // ---- assembly: A[i][j] += rate j -> i, A[i][i] -= rates out of i
    if (lane < n)
      for (int j = 0; j < n; ++j) M[lane * kSolveLd + j] = 0.0;
    for (int t = 0; t < a.ntr; ++t) {
      const int l = a.lower[t], u = a.upper[t];
      if (!(l >= 0 && u < n && l < u)) { bad |= PPRT_DEV_BADINDEX; continue; }
      const int64_t y = r * a.ntr + t;
      const double Plu = dRlu[y] + a.Clu[y];
      const double Pul = Rsul[y] + dRul[y] + a.Cul[y];
      if (lane == u) {
        M[u * kSolveLd + l] += Plu;
        M[u * kSolveLd + u] -= Pul;
      } else if (lane == l) {
        M[l * kSolveLd + l] -= Plu;
        M[l * kSolveLd + u] += Pul;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // ---- row `lane` into registers, columns scaled by the old populations
    double row[kMaxLev];
    double x = (lane == 0) ? a.ntot[r] : 0.0;
#pragma unroll
    for (int j = 0; j < kMaxLev; ++j) {
      double v = 0.0;
      if (j < n) {
        v = (lane == 0) ? 1.0 : (lane < n ? M[lane * kSolveLd + j] : 0.0);   // row 0: conservation
        v *= a.pops[r * n + j];
      }
      row[j] = v;
    }
    bool used = lane >= n;
    int mystep = kMaxLev;                // the step at which this lane's row is the pivot
    int pos[kMaxLev];
    bool singular = false;
#pragma unroll
    for (int c = 0; c < kMaxLev; ++c) {
      pos[c] = 0;
      if (c < n && !singular) {
        // pivot: the largest |A_ic| over the rows not yet used (a NaN counts
        // as infinite, which makes the system singular)
        double v = -1.0;
        if (!used) {
          v = fabs(row[c]);
          if (v != v) v = INFINITY;
        }
        int bl = lane;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          const double ov = __shfl_xor(v, o);
          const int ol = __shfl_xor(bl, o);
          if (ov > v || (ov == v && ol < bl)) { v = ov; bl = ol; }
        }
        const int p = __builtin_amdgcn_readfirstlane(bl);
        // v is the same in every lane after the reduction
        if (!(v > 0.0) || !isfinite(v)) {
          singular = true;
        } else {
          pos[c] = p;
          const double inv = 1.0 / lane_value(row[c], p);
          const double xp = lane_value(x, p);
          const bool upd = !used && lane != p;
          const double f = upd ? row[c] * inv : 0.0;
#pragma unroll
          for (int j = c + 1; j < kMaxLev; ++j) {
            const double pj = lane_value(row[j], p);
            if (upd) row[j] = fma(-f, pj, row[j]);
          }
          if (upd) x = fma(-f, xp, x);
          if (lane == p) { used = true; mystep = c; }
        }
      }
    }
    if (singular) {
      bad |= PPRT_DEV_SINGULAR;
      if (lane < n) pops_new[r * n + lane] = a.pops[r * n + lane];
      continue;
    }
    // ---- back substitution on the pivot rows (uniform values)
    double sol[kMaxLev];
#pragma unroll
    for (int c = kMaxLev - 1; c >= 0; --c) {
      sol[c] = 0.0;
      if (c < n) {
        const int p = pos[c];
        double sacc = lane_value(x, p);
#pragma unroll
        for (int j = c + 1; j < kMaxLev; ++j)
          if (j < n) sacc = fma(-lane_value(row[j], p), sol[j], sacc);
        sol[c] = sacc / lane_value(row[c], p);
      }
    }
    // ---- one step of iterative refinement in FP64: the residual of the
    // scaled system from the assembled matrix (still in the slab), then the
    // correction from the same factors (partial pivoting alone leaves
    // componentwise backward errors of several n u on these systems, whose
    // columns span many decades; one step brings them to rounding level)
    double d = 0.0;
    if (lane < n) {
      d = (lane == 0) ? a.ntot[r] : 0.0;
#pragma unroll
      for (int j = 0; j < kMaxLev; ++j)
        if (j < n) {
          const double aij = (lane == 0) ? 1.0 : M[lane * kSolveLd + j];
          d = fma(-(aij * a.pops[r * n + j]), sol[j], d);
        }
    }
#pragma unroll
    for (int c = 0; c < kMaxLev; ++c) {
      if (c < n) {
        const int p = pos[c];
        const double inv = 1.0 / lane_value(row[c], p);
        const double dp = lane_value(d, p);
        if (mystep > c) d = fma(-(row[c] * inv), dp, d);
      }
    }
    double corr[kMaxLev];
#pragma unroll
    for (int c = kMaxLev - 1; c >= 0; --c) {
      corr[c] = 0.0;
      if (c < n) {
        const int p = pos[c];
        double sacc = lane_value(d, p);
#pragma unroll
        for (int j = c + 1; j < kMaxLev; ++j)
          if (j < n) sacc = fma(-lane_value(row[j], p), corr[j], sacc);
        corr[c] = sacc / lane_value(row[c], p);
      }
    }
#pragma unroll
    for (int c = 0; c < kMaxLev; ++c) sol[c] += corr[c];
    double mine = 0.0;
#pragma unroll
    for (int j = 0; j < kMaxLev; ++j)
      if (j == lane) mine = sol[j];
    if (lane < n) {
      const double old = a.pops[r * n + lane];
      const double xi = mine * old;
      const double rel = fabs(xi - old) / fabs(xi);
      if (!isfinite(xi)) bad |= PPRT_DEV_NONFINITE;
      mx = fmax(mx, isfinite(rel) ? rel : INFINITY);
      pops_new[r * n + lane] = xi;
    }
  }
  if (bad && status) atomicOr(status, bad);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
  if (lane == 0) red[wv] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
    for (int w = 1; w < kSolveWaves; ++w) m = fmax(m, red[w]);
    part[(int64_t)b * nchunk + blockIdx.y] = m;
  }
}

// per atmosphere: the largest relative change over its chunks, and the
// iteration count and convergence flag
__global__ void k_ml_solve_fin(const int64_t* __restrict__ off, int nb, const double* __restrict__ part,
                               int chunk, int nchunk, double* __restrict__ max_rel, MlSolveCtl ctl) {
  const int b = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (b >= nb) return;
  if (ctl.active != nullptr && ctl.active[b] == 0) return;
  const int64_t rows = off[b + 1] - off[b];
  const int nc = (int)((rows + chunk - 1) / chunk);
  double m = 0.0;
  for (int c = 0; c < nc; ++c) m = fmax(m, part[(int64_t)b * nchunk + c]);
  if (max_rel) max_rel[b] = m;
  if (ctl.iters != nullptr) {
    const int it = (ctl.iters[b] += 1);
    if (ctl.active != nullptr && (m < ctl.tol || (ctl.max_iter > 0 && it >= ctl.max_iter)))
      ctl.active[b] = 0;
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

// depth rows per block: kSolveChunk, more where the chunks of the deepest
// atmosphere would pass the grid's 65,535 limit in y
static int ml_solve_chunk_rows(int ndmax) {
  const int need = (ndmax + 65534) / 65535;
  return need > kSolveChunk ? (need + kSolveWaves - 1) / kSolveWaves * kSolveWaves : kSolveChunk;
}

int ml_solve_chunks(int ndmax) {
  const int c = ml_solve_chunk_rows(ndmax);
  return (ndmax + c - 1) / c;
}

hipError_t launch_ml_solve(const MlArgs& a, const int64_t* off, int nb, int ndmax, const double* dRlu,
                           const double* dRul, const double* Rsul, double* pops_new, double* part,
                           double* max_rel, uint32_t* status, hipStream_t s, const MlSolveCtl& ctl) {
  if (nb == 0 || ndmax <= 0) return hipSuccess;
  const int chunk = ml_solve_chunk_rows(ndmax), nchunk = ml_solve_chunks(ndmax);
  hipLaunchKernelGGL(k_ml_solve, dim3(nb, nchunk), dim3(64 * kSolveWaves), 0, s, a, off, dRlu, dRul, Rsul,
                     pops_new, part, chunk, nchunk, status, ctl);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_ml_solve_fin, dim3((nb + 255) / 256), dim3(256), 0, s, off, nb, part, chunk, nchunk,
                     max_rel, ctl);
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

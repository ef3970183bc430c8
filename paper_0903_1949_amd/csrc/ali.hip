// Two-level-atom operator-splitting update in float64 (the "OS step" of the
// paper's timing breakdown, Sect. 3.2.1), one block per atmosphere.
//
// For a pure line with complete redistribution and the diagonal Lambda*, the
// local-operator update of Olson, Auer & Buchler (1986) reads, per node,
//     S_new = S + [(1-eps)(Jbar - S) + eps (B - S)] / [eps + (1-eps)(1 - Lbar*)]
// with Jbar - S and 1 - Lbar* taken from the profile-weighted partial sums
// the formal-solution sweep left in `part` (one per wave: both hemispheres,
// every 64-frequency tile; added here in float64 in a fixed order).  The block also forms the
// atmosphere's maximum relative change max_d |S_new - S| / |S_new|, the
// stopping quantity of Sect. 3.2.1 applied to S, and retires the atmosphere
// once it falls below the tolerance.
#include "pprt_internal.h"

namespace pprt {
namespace {

__global__ __launch_bounds__(256) void k_ali_update(AliUpdateArgs a) {
  __shared__ double red[256];
  const int b = blockIdx.x;
  if (a.active != nullptr && a.active[b] == 0) return;   // uniform over the block
  const int64_t r0 = a.off[b];
  const int64_t r1 = a.off[b + 1];
  const double eps = a.eps[b];
  const int stride = a.nw * 4;
  double mx = 0.0;
  bool bad = false;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
    double jms = 0.0, olb = 0.0;
    if (a.part_fp64) {
      const double* p = static_cast<const double*>(a.part) + r * stride;
      for (int g = 0; g < a.nw; ++g) {
        jms += p[g * 4 + 0] + p[g * 4 + 2];     // up + down hemispheres
        olb += p[g * 4 + 1] + p[g * 4 + 3];
      }
    } else {
      const float* p = static_cast<const float*>(a.part) + r * stride;
      for (int g = 0; g < a.nw; ++g) {
        jms += (double)p[g * 4 + 0] + (double)p[g * 4 + 2];
        olb += (double)p[g * 4 + 1] + (double)p[g * 4 + 3];
      }
    }
    const double S = a.S[r];
    const double dS = ((1.0 - eps) * jms + eps * (a.B[r] - S)) / (eps + (1.0 - eps) * olb);
    const double Sn = S + dS;
    double rel = fabs(dS) / fabs(Sn);
    if (!isfinite(Sn) || !isfinite(rel)) {
      bad = true;
      rel = INFINITY;
    }
    a.S[r] = Sn;
    mx = fmax(mx, rel);
  }
  if (bad && a.status != nullptr) atomicOr(a.status, (unsigned)PPRT_DEV_NONFINITE);
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double m = red[0];
    a.max_rel[b] = m;
    int it = 0;
    if (a.iters != nullptr) it = (a.iters[b] += 1);
    if (a.active != nullptr && a.tol > 0.0 && m < a.tol) a.active[b] = 0;
    if (a.active != nullptr && a.max_iter > 0 && it >= a.max_iter) a.active[b] = 0;
  }
}

// S^g_k = p_k S_l + c_k for every (row, frequency)
template <typename T>
__global__ void k_sg_assemble(const double* __restrict__ S, const T* __restrict__ p,
                              const T* __restrict__ c, T* __restrict__ Sg, int64_t rows, int nf) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= rows * nf) return;
  const int64_t r = x / nf;
  Sg[x] = (T)((double)p[x] * S[r] + (double)c[x]);
}

// Per row: jms = sum_k wphi_k (JmS_k + S^g_k - S_l), olb = sum_k wphi_k ((1-p_k) + p_k Lc_k)
// (p and S^g NULL: a pure line, p = 1 and S^g = S_l),
// written as part[row] = (jms, olb, 0, 0) (one frequency group, one hemisphere slot).
template <typename T>
__global__ __launch_bounds__(256) void k_profile_reduce(const double* __restrict__ S,
                                                        const T* __restrict__ JmS,
                                                        const T* __restrict__ Lc,
                                                        const T* __restrict__ Sg,
                                                        const T* __restrict__ p,
                                                        const T* __restrict__ wphi,
                                                        double* __restrict__ part, int nf) {
  __shared__ double red[2][256];
  const int64_t r = blockIdx.x;
  const double Sl = S[r];
  double js = 0.0, ls = 0.0;
  for (int k = threadIdx.x; k < nf; k += blockDim.x) {
    const int64_t x = r * nf + k;
    const double wp = (double)wphi[k];
    // p == nullptr: a pure line (S^g = S_l, p = 1)
    const double pk = p ? (double)p[x] : 1.0;
    const double sgl = p ? ((double)Sg[x] - Sl) : 0.0;
    js += wp * ((double)JmS[x] + sgl);
    ls += wp * ((1.0 - pk) + pk * (double)Lc[x]);
  }
  red[0][threadIdx.x] = js;
  red[1][threadIdx.x] = ls;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[r * 4 + 0] = red[0][0];
    part[r * 4 + 1] = red[1][0];
    part[r * 4 + 2] = 0.0;
    part[r * 4 + 3] = 0.0;
  }
}

// Non-local update (tri-diagonal approximate operator) and/or Ng
// acceleration, one block per atmosphere, float64.  With the profile-averaged
// band from the sweep (part[row][tile][hemisphere] = (J-S, 1-Lambda*, band, -);
// the up-going hemisphere's band is Lambda*_{d,d+1}, the down-going one's
// Lambda*_{d,d-1}) each atmosphere solves
//     [I - (1-eps) Lbar*] dS = (1-eps)(Jbar - S) + eps (B - S)
// by Thomas elimination (the matrix is diagonally dominant: the rows of
// Lambda sum to at most one, so no pivoting is needed).  Ng's extrapolation
// (in Auer's form, weights 1/x0^2) waits until an un-accelerated update
// changes S by less than kNgStart (maximum relative change), whose old and new
// iterates open the first group; from then on it is applied whenever four
// iterates have gathered since the last extrapolation.  The group history
// lives in hist[3][rows]; ng_count[nb] is 0 while waiting, else the number of
// iterates in the group.
constexpr double kNgStart = 1e-2;

__global__ __launch_bounds__(256) void k_ali_update_nl(AliUpdateArgs a, AliNlArgs n) {
  __shared__ double red[5][256];
  __shared__ double ab[3];
  const int b = blockIdx.x;
  if (a.active != nullptr && a.active[b] == 0) return;   // uniform over the block
  const int64_t r0 = a.off[b];
  const int64_t r1 = a.off[b + 1];
  const int64_t rows = n.rows;
  const double eps = a.eps[b];
  const int nqp = n.tri ? 4 : 2;
  const int stride = a.nw * 2 * nqp;
  double* cf = n.coef;
  // ---- coefficients of the per-atmosphere system
  for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
    double jms = 0.0, olb = 0.0, sup = 0.0, sub = 0.0;
    for (int g = 0; g < a.nw; ++g) {
      double v[2][3];
      for (int dir = 0; dir < 2; ++dir)
        for (int q = 0; q < (n.tri ? 3 : 2); ++q) {
          const int64_t x = r * stride + (g * 2 + dir) * nqp + q;
          v[dir][q] = a.part_fp64 ? static_cast<const double*>(a.part)[x]
                                  : (double)static_cast<const float*>(a.part)[x];
        }
      jms += v[0][0] + v[1][0];
      olb += v[0][1] + v[1][1];
      if (n.tri) {
        sup += v[0][2];
        sub += v[1][2];
      }
    }
    const double S = a.S[r];
    cf[r * 4 + 0] = -(1.0 - eps) * sub;
    cf[r * 4 + 1] = eps + (1.0 - eps) * olb;
    cf[r * 4 + 2] = -(1.0 - eps) * sup;
    cf[r * 4 + 3] = (1.0 - eps) * jms + eps * (a.B[r] - S);
  }
  __syncthreads();
  if (n.tri && threadIdx.x == 0) {
    double cp = 0.0, dp = 0.0;
    for (int64_t r = r0; r < r1; ++r) {
      const double lo = cf[r * 4 + 0];
      const double m = cf[r * 4 + 1] - lo * cp;
      cp = cf[r * 4 + 2] / m;
      dp = (cf[r * 4 + 3] - lo * dp) / m;
      cf[r * 4 + 2] = cp;
      cf[r * 4 + 3] = dp;
    }
    double xv = cf[(r1 - 1) * 4 + 3];
    for (int64_t r = r1 - 2; r >= r0; --r) {
      xv = cf[r * 4 + 3] - cf[r * 4 + 2] * xv;
      cf[r * 4 + 3] = xv;
    }
  }
  __syncthreads();
  // ---- new iterate (and Ng's group)
  const int cnt = n.ng ? n.ng_count[b] : 0;
  const bool waiting = n.ng && cnt == 0;            // the update's S_old, S_new may open a group
  const bool extrap = n.ng && cnt == 3;
  double mx = 0.0;
  bool bad = false;
  double s5[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
    const double So = a.S[r];
    const double dS = n.tri ? cf[r * 4 + 3] : cf[r * 4 + 3] / cf[r * 4 + 1];
    const double Sn = So + dS;
    if (waiting) n.hist[r] = So;
    if (extrap) {
      const double x0 = Sn, x1 = n.hist[2 * rows + r], x2 = n.hist[rows + r], x3 = n.hist[r];
      const double d0 = x0 - x1, d1 = x1 - x2, d2 = x2 - x3;
      const double wt = 1.0 / (x0 * x0);
      const double u = d0 - d1, v = d0 - d2;
      s5[0] += wt * u * u;
      s5[1] += wt * u * v;
      s5[2] += wt * v * v;
      s5[3] += wt * d0 * u;
      s5[4] += wt * d0 * v;
      cf[r * 4 + 0] = Sn;                 // keep x0 for the second pass
      continue;
    }
    if (n.ng) n.hist[(int64_t)(waiting ? 1 : cnt) * rows + r] = Sn;
    double rel = fabs(dS) / fabs(Sn);
    if (!isfinite(Sn) || !isfinite(rel)) {
      bad = true;
      rel = INFINITY;
    }
    a.S[r] = Sn;
    mx = fmax(mx, rel);
  }
  if (extrap) {
    for (int q = 0; q < 5; ++q) red[q][threadIdx.x] = s5[q];
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
      if ((int)threadIdx.x < st)
        for (int q = 0; q < 5; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const double A00 = red[0][0], A01 = red[1][0], A11 = red[2][0], b0 = red[3][0], b1 = red[4][0];
      const double det = A00 * A11 - A01 * A01;
      if (det == 0.0 || !isfinite(det)) {
        ab[0] = 0.0;
        ab[1] = 0.0;
      } else {
        ab[0] = (b0 * A11 - A01 * b1) / det;
        ab[1] = (A00 * b1 - A01 * b0) / det;
      }
    }
    __syncthreads();
    const double ca = ab[0], cb = ab[1];
    for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
      const double So = a.S[r];
      const double x0 = cf[r * 4 + 0], x1 = n.hist[2 * rows + r], x2 = n.hist[rows + r];
      const double Sa = (1.0 - ca - cb) * x0 + ca * x1 + cb * x2;
      n.hist[r] = Sa;
      double rel = fabs(Sa - So) / fabs(Sa);
      if (!isfinite(Sa) || !isfinite(rel)) {
        bad = true;
        rel = INFINITY;
      }
      a.S[r] = Sa;
      mx = fmax(mx, rel);
    }
  }
  if (bad && a.status != nullptr) atomicOr(a.status, (unsigned)PPRT_DEV_NONFINITE);
  __syncthreads();
  red[0][threadIdx.x] = mx;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[0][threadIdx.x] = fmax(red[0][threadIdx.x], red[0][threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double m = red[0][0];
    a.max_rel[b] = m;
    int it = 0;
    if (a.iters != nullptr) it = (a.iters[b] += 1);
    if (a.active != nullptr && a.tol > 0.0 && m < a.tol) a.active[b] = 0;
    if (a.active != nullptr && a.max_iter > 0 && it >= a.max_iter) a.active[b] = 0;
    if (n.ng) n.ng_count[b] = extrap ? 1 : waiting ? (m < kNgStart ? 2 : 0) : cnt + 1;
  }
}

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

hipError_t launch_ali_update(int nb, hipStream_t s, const AliUpdateArgs& a) {
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ali_update, dim3(nb), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_ali_update_nl(int nb, hipStream_t s, const AliUpdateArgs& a, const AliNlArgs& n) {
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ali_update_nl, dim3(nb), dim3(256), 0, s, a, n);
  return hipGetLastError();
}

hipError_t launch_sg_assemble(int precision, const double* S, const void* p, const void* c, void* Sg,
                              int64_t rows, int nf, hipStream_t s) {
  const int64_t n = rows * nf;
  if (n == 0) return hipSuccess;
  const unsigned nb = (unsigned)((n + 255) / 256);
  if (precision == PPRT_FP64)
    hipLaunchKernelGGL(k_sg_assemble<double>, dim3(nb), dim3(256), 0, s, S, (const double*)p,
                       (const double*)c, (double*)Sg, rows, nf);
  else
    hipLaunchKernelGGL(k_sg_assemble<float>, dim3(nb), dim3(256), 0, s, S, (const float*)p,
                       (const float*)c, (float*)Sg, rows, nf);
  return hipGetLastError();
}

hipError_t launch_profile_reduce(int precision, const double* S, const void* JmS, const void* Lc,
                                 const void* Sg, const void* p, const void* wphi, double* part,
                                 int64_t rows, int nf, hipStream_t s) {
  if (rows == 0) return hipSuccess;
  if (precision == PPRT_FP64)
    hipLaunchKernelGGL(k_profile_reduce<double>, dim3((unsigned)rows), dim3(256), 0, s, S,
                       (const double*)JmS, (const double*)Lc, (const double*)Sg, (const double*)p,
                       (const double*)wphi, part, nf);
  else
    hipLaunchKernelGGL(k_profile_reduce<float>, dim3((unsigned)rows), dim3(256), 0, s, S,
                       (const float*)JmS, (const float*)Lc, (const float*)Sg, (const float*)p,
                       (const float*)wphi, part, nf);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int bs = 256;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, p, v, n);
  return hipGetLastError();
}

}  // namespace pprt

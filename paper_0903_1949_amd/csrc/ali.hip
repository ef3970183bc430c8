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

// Per row: jms = sum_k wphi_k (JmS_k + S^g_k - S_l), olb = sum_k wphi_k ((1-p_k) + p_k Lc_k),
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
    const double pk = (double)p[x];
    js += wp * ((double)JmS[x] + ((double)Sg[x] - Sl));
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

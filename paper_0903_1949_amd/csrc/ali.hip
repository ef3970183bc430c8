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
    if (a.iters != nullptr) a.iters[b] += 1;
    if (a.active != nullptr && a.tol > 0.0 && m < a.tol) a.active[b] = 0;
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

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int bs = 256;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, p, v, n);
  return hipGetLastError();
}

}  // namespace pprt

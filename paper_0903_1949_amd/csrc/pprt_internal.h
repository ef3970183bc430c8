// Internal structures shared by the host runtime and the kernels of libpprt.
// Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>

#include "../../include/pprt.h"

namespace pprt {

constexpr int kMaxNA = 32;

// psi(x) = (1 - e^-x)/x for optically thin layers (0 <= x < 1/4), FP32: a
// degree-4 polynomial fitted for least maximum relative error on [0, 1/4]
// (Remez exchange; fitted error 2.5e-9, evaluated in FP32 4.5e-8).
__device__ __forceinline__ float psi_thin_f32(float x) {
  float p = fmaf(x, 7.510221563279629e-3f, -4.1488952934741974e-2f);
  p = fmaf(x, p, 1.6665081679821014e-1f);
  p = fmaf(x, p, -4.999994933605194e-1f);
  return fmaf(x, p, 1.0f);
}

// ---- wave-wide sums (deterministic order) ---------------------------------
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(u & 0xffffffffll), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float readlane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double readlane(double v, int l) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over each row of 16 lanes (quad swaps, half-row mirror, row mirror);
// every lane must be active and ends with its row's sum.
__device__ __forceinline__ float row_sum(float v) {
  v += dpp_f<0xb1>(v);    // quad_perm [1,0,3,2]
  v += dpp_f<0x4e>(v);    // quad_perm [2,3,0,1]
  v += dpp_f<0x141>(v);   // row_half_mirror
  v += dpp_f<0x140>(v);   // row_mirror
  return v;
}
__device__ __forceinline__ double row_sum(double v) {
  v += dpp_d<0xb1>(v);
  v += dpp_d<0x4e>(v);
  v += dpp_d<0x141>(v);
  v += dpp_d<0x140>(v);
  return v;
}

// Sum over the 64 lanes of a wave; every lane must be active.  Within each
// row of 16 lanes: quad swaps, half-row mirror, row mirror; then the four row
// sums are added in a fixed order.  The result is uniform over the wave.
__device__ __forceinline__ float wave_sum(float v) {
  v += dpp_f<0xb1>(v);    // quad_perm [1,0,3,2]
  v += dpp_f<0x4e>(v);    // quad_perm [2,3,0,1]
  v += dpp_f<0x141>(v);   // row_half_mirror
  v += dpp_f<0x140>(v);   // row_mirror
  return (readlane(v, 0) + readlane(v, 16)) + (readlane(v, 32) + readlane(v, 48));
}
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<0xb1>(v);
  v += dpp_d<0x4e>(v);
  v += dpp_d<0x141>(v);
  v += dpp_d<0x140>(v);
  return (readlane(v, 0) + readlane(v, 16)) + (readlane(v, 32) + readlane(v, 48));
}

// Angle constants of one plan, passed to kernels by value (kernel-argument
// segment, read into scalar registers).  All per-angle, uniform over lanes.
template <typename T>
struct Angles {
  T c[kMaxNA];     // log2(e) / mu_i   (exponent scale for exp2)
  T rmu[kMaxNA];   // 1 / mu_i
  T mu[kMaxNA];    // mu_i
  T hw[kMaxNA];    // w_i / 2
  T hwmu[kMaxNA];  // w_i mu_i / 2
  T hwsum;         // sum_i w_i / 2 (one hemisphere's weight)
  T rmu_max;       // max_i 1/mu_i (the angle with the largest Delta)
  T rmu_min;       // min_i 1/mu_i
  T dt_all_thin;   // FP32 sweep: every angle is optically thin when dtau < this
  T dt_all_thick;  // FP32 sweep: every angle is optically thick when dtau >= this
};

// One work item: atmosphere b, frequency group g (blockDim.x frequencies),
// sweep direction dir (profile mode: 0 = up-going, 1 = down-going).
struct Item {
  int32_t b;
  int32_t g;
  int32_t dir;
  int32_t nd;
};

template <typename T>
struct FsFullArgs {
  const Item* items;
  const int64_t* off;       // [nb+1]
  const double* tau;
  const T* q;
  const T* Sg;
  const T* Itop;
  const T* Bbot;
  const T* Bbot_prev;
  const T* Ibot;
  T* J; T* JmS; T* lstar; T* lstar_c; T* Iplus; T* Iminus; T* H; T* Iemerg;
  T* lsub; T* lsup;         // tri-diagonal band of Lambda
  int32_t nf;
  int32_t lower_bc;
  uint32_t outputs;
};

template <typename T>
struct FsProfileArgs {
  const Item* items;
  const int64_t* off;
  const double* tau;
  const T* q;
  const double* S;          // [rows] line source function (float64 state)
  const double* B;          // [rows] Planck function (diffusion lower boundary)
  const T* Itop;
  const T* Ibot;
  const T* wphi;            // [nf]
  const int32_t* active;    // [nb] or nullptr
  int32_t* queue;           // persistent launch: work counter (zeroed before launch); else nullptr
  T* part;                  // [rows][nw][2 dir][2 or 4] per-wave profile moments
  const T* dtr;             // [rows] T(tau[r+1] - tau[r]) / 2 (launch_row_diffs)
  const T* dSr;             // [rows] T(S[r+1] - S[r])
  int32_t nf;
  int32_t nw;               // waves across the frequency range, ceil(nf/64)
  int32_t nitems;           // one item per wave: (b, 64-frequency tile, dir)
  int32_t lower_bc;
};

struct AliUpdateArgs {
  const int64_t* off;
  const void* part;         // [rows][nw][2][2], float or double (part_fp64)
  const double* eps;
  const double* B;
  double* S;
  double* max_rel;          // [nb]
  int32_t* active;          // [nb] or nullptr (device flags, 1 = iterate)
  int32_t* iters;           // [nb] or nullptr
  uint32_t* status;         // device status word
  double tol;               // > 0: clear `active` once max_rel < tol
  int32_t max_iter;         // > 0: clear `active` once iters reaches it
  int32_t nw;
  int32_t nb;
  int32_t part_fp64;
};

// Emergent intensity and its adjoint (fs_adjoint.hip).  Item.g indexes
// blocks of wpb * 64 / lanes_per_freq frequencies.
template <typename T>
struct AdjArgs {
  const Item* items;
  const int64_t* off;       // [nb+1] row offsets
  const int64_t* ck_off;    // [nb] checkpoint-row offsets for the interval in use
  const double* tau;
  const T* q;
  const T* Sg;
  const T* Bbot;
  const T* Bbot_prev;
  const T* Ibot;
  T* Iemerg;                // [nb][nf][na] (forward)
  T* ckpt;                  // [checkpoint rows][nf][na]
  const T* gI;              // [nb][nf][na] dL/dIemerg (adjoint)
  T* dq;                    // [rows][nf]
  T* dSg;                   // [rows][nf]
  T* dBbot;                 // [nb][nf] or nullptr
  T* dBbot_prev;            // [nb][nf] or nullptr
  T* dIbot;                 // [nb][nf][na] or nullptr
  int32_t nf, na, lower_bc;
};
int adj_lanes_per_freq(int na);
bool adj_interval_supported(int K);
hipError_t launch_emergent(int precision, bool vjp, int na, int K, int nitems, int wpb,
                           hipStream_t s, const void* args, const void* angles);

// Non-local (tri-diagonal) operator and Ng acceleration in the update.
struct AliNlArgs {
  int32_t tri;              // 1: tri-diagonal band in part[] (4 entries per hemisphere)
  int32_t ng;               // 1: Ng acceleration
  int64_t rows;
  double* coef;             // [rows][4] scratch
  double* hist;             // [3][rows] Ng group history
  int32_t* ng_count;        // [nb] iterates in the current group (0 = not started)
};
hipError_t launch_ali_update_nl(int nb, hipStream_t s, const AliUpdateArgs& a, const AliNlArgs& n);

// Dense (in-layer scattering) formal solution, FP64 or FP32 bulk (fs_dense.hip).
// Real arrays are double for PPRT_FP64 and float for PPRT_FP32; tau is double.
enum { DENSE_THICK_RULE = 0, DENSE_THICK_NEVER = 1, DENSE_THICK_ALWAYS = 2 };
struct DenseLaunch {
  const Item* items;
  const int64_t* off;
  const double* tau;
  const void* q;
  const void* Sg;
  const void* omega;
  const void* Itop;
  const void* Bbot;
  const void* Bbot_prev;
  const void* Ibot;
  void *J, *JmS, *lstar, *lstar_c, *Iplus, *Iminus, *H, *Iemerg;
  void* ws;
  uint32_t* status;   // device status word (NONFINITE), may be NULL
  unsigned long long* thick_stats;   // [2] FP64 / all eliminations (FP32 bulk), may be NULL
  int64_t rows;
  int32_t nf, na, nitems, lower_bc;
  int32_t precision;  // PPRT_FP64 or PPRT_FP32 (bulk)
  int32_t thick_mode; // DENSE_THICK_* (FP32 bulk only)
  uint32_t outputs;
  const double* mu;   // host, ascending
  const double* w;
};
bool dense_na_supported(int na);
size_t dense_workspace_bytes(int na, int64_t rows, int nf, int precision);
int dense_freqs_per_item(int na, int precision);
// NA = 32: the matrix-core kernels (fs_dense_mfma.hip), FP64 arithmetic for both storage types
bool dense_mfma_na(int na);
size_t dense_mfma_workspace_bytes(int na, int64_t rows, int nf, int precision);
hipError_t launch_fs_dense_mfma(const DenseLaunch& L, hipStream_t s);
hipError_t launch_fs_dense(const DenseLaunch& L, hipStream_t s);
// Reverse mode of the emergent intensity with in-layer scattering (FP64, na <= 16)
struct DenseVjpLaunch {
  const Item* items;
  const int64_t* off;
  const double *tau, *q, *Sg, *omega, *Itop, *Bbot, *Bbot_prev, *Ibot, *gI;
  double *dq, *dSg, *dBbot, *dBbot_prev, *dIbot;
  void* ws;
  uint32_t* status;
  int64_t rows;
  int32_t nf, na, nitems, lower_bc;
  const double* mu;   // host, ascending
  const double* w;
};
size_t dense_vjp_workspace_bytes(int na, int64_t rows, int nf);
hipError_t launch_dense_vjp(const DenseVjpLaunch& L, hipStream_t s);


// Spherical formal solution (sph.hip).
struct SphRay {
  int32_t e0;      // first (ray, shell) entry
  int32_t m;       // innermost shell reached
  int32_t core;    // 1: ends on the core
  double mu_core;  // mu at the core (core rays)
};
template <typename T>
struct SphArgs {
  const int64_t* off;       // [nb+1]
  const int32_t* ray0;      // [nb+1] rays of atmosphere b: ray0[b] .. ray0[b+1]-1
  const SphRay* rays;
  const double* path;       // [entries] (r_d + r_{d+1}) / (z_d + z_{d+1}); 0 at the innermost node
  const double* hw;         // [entries] half trapezoid weight in mu
  const double* mu;         // [entries]
  const double* tau;
  const T* q;
  const T* Sg;              // [rows][nf] or nullptr (then Sl)
  const double* Sl;         // [rows] source per row (pure line), when Sg == nullptr
  const T* Itop;            // [nb][nf] isotropic incident, or nullptr
  const T* Bbot;            // [nb][nf] diffusion core: B at the two innermost shells,
  const T* Bbot_prev;       //   or, when Bl is set, Bl at those rows (all frequencies)
  const double* Bl;         // [rows] or nullptr
  const T* Ibot;            // [nb][nf] isotropic core intensity (GIVEN)
  const int32_t* active;    // [nb] or nullptr: skip atmospheres with active[b] == 0
  T *J, *JmS, *lstar, *lstar_c, *H;
  int32_t nf, lower_bc;
};
hipError_t launch_fs_sph(int precision, int nb, int nf, hipStream_t s, const void* args);

// Spherical two-level sweep (sph.hip): one wave per (sphere, 64-frequency
// tile), rays in groups of sph_group_size() held in registers.
struct SphItem {
  int32_t b;       // sphere (-1: idle wave)
  int32_t tile;    // 64-frequency tile
  int32_t g0, g1;  // ray groups g0 .. g1-1 of the sphere
  int32_t slot;    // partial-sum slot of this chunk of groups (two-level step)
  int32_t nslot;   // chunks of the sphere (slot 0 clears the slots nslot .. P-1)
};
template <typename T>
struct SphFastArgs {
  const SphItem* items;     // [nblocks * waves per block], block order
  const int64_t* off;       // [nb+1]
  const int32_t* grp0;      // [nb+1] ray groups of sphere b: grp0[b] .. grp0[b+1]-1
  const int64_t* gtab;      // [ngroups] start of the group's table in tab
  const T* tab;             // per group [deepest shell + 1][3][G]: path factor of the
                            // segment to the next shell inward, its reciprocal, half
                            // weight in mu (zero where the ray misses the shell)
  const T* tabx;            // per group [deepest shell + 1][2]: largest and smallest
                            // path factor of the group's segments on the row
  const T* muc;             // [nb][n_core] mu at the core of core ray c
  const double* tau;
  const T* q;
  const T* Sg;              // [rows][nf] source per frequency (formal solution)
  const double* Sl;         // [rows] line source (two-level step)
  const T* Itop;            // [nb][nf] or nullptr
  const T* Bbot;            // [nb][nf] diffusion core (when Bl == nullptr)
  const T* Bbot_prev;
  const double* Bl;         // [rows] B per row (two-level step) or nullptr
  const T* Ibot;            // [nb][nf] given core intensity
  const int32_t* active;    // [nb] or nullptr
  const T* wphi;            // [nf] profile weights (two-level step)
  T* JmS;                   // [rows][nf] J - S (formal solution)
  T* Lc;                    // [rows][nf] 1 - Lambda* (formal solution)
  T* part;                  // [rows][ntiles][(P + 1) / 2][4]: slot s at 2s, 2s + 1 (two-level step) or nullptr
  int32_t nf, ntiles, lower_bc, n_core, ndmax;
  int32_t P;                // partial-sum slots (chunks) per tile
};
int sph_group_size(int precision);
size_t sph_fast_lds_bytes(int precision, int wpb, int ndmax);
hipError_t launch_sph_fast(int precision, int nblocks, int wpb, hipStream_t s, const void* args);

// Weideman's expansion of the Faddeeva function (nlte.hip): N terms.
constexpr int kVoigtN = 40;
struct VoigtCoef {
  double L;
  double a[kVoigtN + 1];    // a[1..N] used
};
const VoigtCoef& voigt_coefficients();
hipError_t launch_voigt(int64_t n, const double* a, const double* x, double* H, hipStream_t s);

// Multilevel atom (nlte.hip); every array is device memory, FP64.
struct MlArgs {
  const double* pops;     // [rows][nlev] populations the rates are built with
  const int32_t* lower;   // [ntr]
  const int32_t* upper;
  const int32_t* k0;
  const int32_t* k1;
  const int32_t* owner;   // [nf]
  const double* sigma;    // [nf]
  const double* bfac;     // [nf]
  const double* W;        // [nf]
  const double* G;        // [rows][nf]
  const double* Bnu;      // [rows][nf]
  const double* kc;       // [rows]
  const double* sc;       // [rows]
  const double* ntot;     // [rows]
  const double* Cul;      // [rows][ntr]
  const double* Clu;      // [rows][ntr]
  uint32_t* status;       // device status word: BADINDEX for a table entry out of range
  // depth-dependent Voigt lines (line_a == nullptr: sigma[k] throughout)
  const double* nu;       // [nf]
  const double* line_nu0; // [ntr]
  const double* line_s;   // [ntr]
  const double* line_a;   // [ntr]
  const double* dopp;     // [rows]
  VoigtCoef vc;
  int64_t rows;
  int32_t nf, nlev, ntr;
};
int ml_max_levels();
hipError_t launch_ml_opacity(const MlArgs& a, double* q, double* om, double* Sg, hipStream_t s);
hipError_t launch_ml_rates(const MlArgs& a, const double* J, const double* L, double* dRlu,
                           double* dRul, double* Rsul, hipStream_t s);
// Convergence bookkeeping of the multilevel loop (all NULL / 0: one plain solve).
// Atmospheres with active[b] == 0 keep their populations; after each solve
// iters[b] is incremented and active[b] cleared once max_rel < tol or the
// count reaches max_iter.
struct MlSolveCtl {
  int32_t* active;
  int32_t* iters;
  double tol;
  int32_t max_iter;
};
// The per-depth solve on blocks of (atmosphere, chunk of depth rows); ndmax =
// the largest depth count; part holds nb * ml_solve_chunks(ndmax) doubles
// (each chunk's largest relative change, reduced per atmosphere by a second
// kernel).
int ml_solve_chunks(int ndmax);
hipError_t launch_ml_solve(const MlArgs& a, const int64_t* off, int nb, int ndmax, const double* dRlu,
                           const double* dRul, const double* Rsul, double* pops_new, double* part,
                           double* max_rel, uint32_t* status, hipStream_t s,
                           const MlSolveCtl& ctl = MlSolveCtl{});
hipError_t launch_gather_bottom(const double* Bnu, const int64_t* off, int nb, int nf, double* Bb,
                                double* Bp, hipStream_t s);

// Launchers (fs_diag.hip, ali.hip).  Return hipSuccess or the launch error.
hipError_t launch_fs_full(int precision, int na, int wpb, int nitems, hipStream_t s,
                          const void* args, const void* angles);
// nblocks = 0: one wave per item; otherwise a persistent grid of nblocks
// blocks whose waves take items from args.queue.
// tri: also reduce the tri-diagonal band (part[] then has 4 entries per
// (row, tile, hemisphere): J-S, 1-Lambda*, band, unused).
hipError_t launch_row_diffs(int precision, const double* tau, const double* S, int64_t rows, void* dtr,
                            void* dSr, hipStream_t s);
hipError_t launch_fs_profile(int precision, int na, int wpb, int nitems, int nblocks, bool tri,
                             hipStream_t s, const void* args, const void* angles);
hipError_t launch_ali_update(int nb, hipStream_t s, const AliUpdateArgs& a);
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);

// 3D full characteristics on a spherical voxel grid (vox3d.hip).
struct VoxGeom {                   // plan-time geometry (host, FP64)
  int nr = 0, nt = 0, np = 0, ndir = 0;
  int64_t nfill = 0;               // coverage characteristics
  std::vector<double> dirs, w;     // [ndir][3], [ndir]
  std::vector<int64_t> ray_seg0;   // [nrays + 1]
  std::vector<int32_t> ray_dir;    // [nrays]
  std::vector<uint8_t> ray_core;   // [nrays] 1: starts on the inner sphere
  std::vector<uint32_t> seg_ijk;   // [nseg] i << 20 | j << 10 | k
  std::vector<double> seg_ell;     // [nseg] path length in the voxel
  std::vector<double> seg_wn;      // [nseg] w / (direction's path length in the voxel), 0 off the mean
};
bool vox_build_geometry(const double* r, int nr, int nt, int np, int n_mu, int n_phi, double h, int nthreads,
                        VoxGeom& out, std::string& err);
template <typename T, typename A = double>   // A: accumulator type of J and Lambda*
struct VoxArgs {
  const int64_t* ray_seg0;
  const int32_t* ray_dir;
  const uint8_t* ray_core;
  const uint32_t* seg_ijk;
  const T* seg_ell;
  const T* seg_wn;
  const double* dirs;       // [ndir][3]
  const T* chi;             // [nvox][nf]
  const T* S;               // [nvox][nf]
  const T* I_out;           // [nf] or NULL (0)
  const T* I_core;          // [nf] or NULL (0)
  A* J;                     // [nvox][nf], accumulated (zeroed by the caller)
  double* flux;             // [nvox][3][nf] Cartesian, or NULL
  A* lstar;                 // [nvox][27][nf] (band) or [nvox][nf] (diagonal), or NULL
  int64_t ray0;             // first characteristic of this launch
  int64_t nrays;            // characteristics of this launch
  int32_t nf, nfb, group, nt, np;
};
hipError_t launch_vox_zero(double* p, int64_t n, hipStream_t s);
hipError_t launch_vox_fs(int precision, bool acc32, const void* args, int mode, hipStream_t s);
hipError_t launch_vox_zero32(float* p, int64_t n, hipStream_t s);
// dst[i] += src[i] (FP32 partial sums into the FP64 outputs)
hipError_t launch_vox_flush(const float* src, double* dst, int64_t n, hipStream_t s);
hipError_t launch_vox_to_bulk(int precision, const double* src, void* dst, int64_t n, hipStream_t s);
hipError_t launch_vox_ali(const double* J, const double* Ld, double* S, const double* B, const double* eps,
                          int64_t nvox, int nf, unsigned long long* maxrel_bits, hipStream_t s);

hipError_t launch_sg_assemble(int precision, const double* S, const void* p, const void* c, void* Sg,
                              int64_t rows, int nf, hipStream_t s);
hipError_t launch_profile_reduce(int precision, const double* S, const void* JmS, const void* Lc,
                                 const void* Sg, const void* p, const void* wphi, double* part,
                                 int64_t rows, int nf, hipStream_t s);

bool na_supported(int na);

// Measured peaks (peaks.hip): FP32 / FP64 FMA TFLOP/s, exp2 Texp/s, copy GB/s.
hipError_t measure_peaks(int n_cu, void* scratch, size_t bytes, hipStream_t s, double* fp32,
                         double* fp64, double* exp_rate, double* copy_gbs);
hipError_t measure_atomic_rates(int n_cu, void* scratch, size_t bytes, hipStream_t s, double* f64_gadds,
                                double* f32_gadds);

}  // namespace pprt

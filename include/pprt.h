/*
 * pprt.h -- C ABI of libpprt, a plane-parallel formal solution of the
 * equation of radiative transfer with its accelerated Lambda iteration,
 * for AMD Instinct MI355X (gfx950).
 *
 * Problem statement (Hauschildt & Baron, "A 3D radiative transfer framework
 * IV", Sect. 2 and Sect. 3.1): the scattering problem for line transfer is
 * solved by operator splitting around a formal solution of the transfer
 * equation; the 1D plane-parallel calculation is the comparison standard
 * (abstract, Sect. 3.2).  The test environment of Sect. 3.1 fixes the inputs:
 * an optical-depth grid, opacities, a Planck function, zero incident
 * intensity at the outer boundary, a diffusion inner boundary, a two-level
 * line with thermalisation parameter eps and coherent isotropic continuum
 * scattering.  Inputs: atmosphere (tau grid), opacities, source terms and
 * model atom.  Outputs: I+/I-, J, Jbar, Lambda*, rates and populations.
 *
 * Conventions shared by every call
 * --------------------------------
 * - tau is the reference optical depth, strictly increasing inward; node 0
 *   is the top.  A batch holds nbatch independent atmospheres with nd[b]
 *   nodes each (2 <= nd[b]); off[b] = nd[0] + ... + nd[b-1].
 * - "row" = one (atmosphere, node) pair, index off[b] + d.
 * - Per-(row, frequency) arrays are row-major: element (off[b]+d)*nf + k.
 *   Per-(row, frequency, angle) arrays: ((off[b]+d)*nf + k)*na + i.
 *   Per-(atmosphere, frequency) arrays: b*nf + k; with angle: (b*nf+k)*na+i.
 * - Angles: na Gauss-Legendre nodes mu_i on (0,1) per hemisphere with
 *   weights summing to one, ascending in mu.  I+ is the up-going (outward)
 *   intensity, I- the down-going one, both indexed by the same mu_i.
 * - All array pointers are DEVICE pointers unless the field says "host".
 *   Element type of "real" arrays follows the plan precision: double for
 *   PPRT_FP64, float for PPRT_FP32.  tau, model-atom and ALI state arrays are
 *   always double.
 * - Ownership: the caller allocates and frees every input, output and
 *   workspace buffer.  The library keeps only small plan metadata (it may
 *   call hipMalloc for that inside pprt_plan_create) and never frees caller
 *   memory.
 * - Asynchrony: compute calls enqueue kernels on the context stream and
 *   return; results are ready after the caller synchronises that stream.
 *   Nothing is copied device -> host except where a call says so.
 * - Errors: every call returns a pprt_status.  Argument and shape errors are
 *   detected on the host before any launch, and pprt_last_error() then
 *   holds a message.  Conditions found on the device (non-finite values)
 *   set bits of a status word read by pprt_sync().  No exception, abort or
 *   exit crosses this interface.
 * - Thread safety: one context per host thread.
 */
#ifndef PPRT_H
#define PPRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pprt_status {
  PPRT_OK = 0,
  PPRT_E_INVALID_ARG = 1,   /* bad pointer, value or flag combination        */
  PPRT_E_SHAPE = 2,         /* inconsistent or unsupported sizes            */
  PPRT_E_DEVICE = 3,        /* no usable HIP device / runtime failure       */
  PPRT_E_WORKSPACE = 4,     /* workspace missing or too small               */
  PPRT_E_NONFINITE = 5,     /* NaN/Inf met (host scan or device status)     */
  PPRT_E_NOT_CONVERGED = 6, /* iteration cap reached before the tolerance   */
  PPRT_E_SINGULAR = 7,      /* a per-depth linear system cannot be solved   */
  PPRT_E_UNSUPPORTED = 8,   /* valid request this build does not implement  */
  PPRT_E_LAUNCH = 9         /* a kernel launch failed                       */
} pprt_status;

/* device status bits (pprt_sync) */
#define PPRT_DEV_NONFINITE 0x1u  /* a kernel produced NaN/Inf                     */
#define PPRT_DEV_SINGULAR  0x2u  /* a per-depth rate system had no usable pivot   */
#define PPRT_DEV_BADINDEX  0x4u  /* a model-atom table entry was out of range     */

typedef enum pprt_precision { PPRT_FP64 = 0, PPRT_FP32 = 1 } pprt_precision;
typedef enum pprt_lower_bc { PPRT_BC_DIFFUSION = 0, PPRT_BC_GIVEN = 1 } pprt_lower_bc;

/* output bitmask of pprt_formal_solution */
#define PPRT_OUT_J       0x01u  /* J = 1/2 sum_i w_i (I+ + I-)          [row][nf]     */
#define PPRT_OUT_JMS     0x02u  /* J - S (difference form)              [row][nf]     */
#define PPRT_OUT_LSTAR   0x04u  /* Lambda*_dd = dJ(d)/dS(d)             [row][nf]     */
#define PPRT_OUT_LSTAR_C 0x08u  /* 1 - Lambda*_dd, formed directly      [row][nf]     */
#define PPRT_OUT_IPLUS   0x10u  /* I+                                   [row][nf][na] */
#define PPRT_OUT_IMINUS  0x20u  /* I-                                   [row][nf][na] */
#define PPRT_OUT_H       0x40u  /* H = 1/2 sum_i w_i mu_i (I+ - I-)     [row][nf]     */
#define PPRT_OUT_IEMERG  0x80u  /* emergent I+ at node 0                [b][nf][na]   */
#define PPRT_OUT_LSTAR_SUB 0x100u /* Lambda_{d,d-1} = dJ(d)/dS(d-1), 0 at d = 0  [row][nf] */
#define PPRT_OUT_LSTAR_SUP 0x200u /* Lambda_{d,d+1} = dJ(d)/dS(d+1), 0 at the last node [row][nf]
                                     (the tri-diagonal band; omega = 0 plans only) */

typedef struct pprt_ctx pprt_ctx;
typedef struct pprt_plan pprt_plan;

/* ------------------------------------------------------------------ misc */

/* Library version; any pointer may be NULL.  Always PPRT_OK. */
int pprt_version(int* major, int* minor, int* patch);

/* Static, never-freed description of a status code. */
const char* pprt_status_string(pprt_status s);

/* Gauss-Legendre rule on (0,1) (host helper): mu[n], w[n] host arrays,
 * ascending mu, sum w = 1.  The angle quadrature of the 1D comparison
 * calculations (Sect. 3.1 discretises solid angle; a plane-parallel slab
 * needs only mu).  E_INVALID_ARG for n < 1 or n > 64 or NULL pointers. */
pprt_status pprt_gauss_legendre01(int n, double* mu, double* w);

/* --------------------------------------------------------------- context */

/* Create a context on HIP device `device`.  E_DEVICE if no such device. */
pprt_status pprt_create(pprt_ctx** out, int device);
void pprt_destroy(pprt_ctx* ctx);
/* Borrow a HIP stream (hipStream_t as void*; NULL = the null stream).
 * The library never destroys it. */
pprt_status pprt_set_stream(pprt_ctx* ctx, void* hip_stream);
/* Message of the last host-side error on this context ("" if none). */
const char* pprt_last_error(const pprt_ctx* ctx);
/* Wait for the context stream, then return and clear the device status
 * word (PPRT_DEV_* bits).  E_NONFINITE if the NONFINITE bit was set, else
 * E_SINGULAR for SINGULAR, else E_INVALID_ARG for BADINDEX. */
pprt_status pprt_sync(pprt_ctx* ctx, uint32_t* device_status);

/* Validation mode.  PPRT_VALIDATE_INPUTS: before launching, the compute
 * calls copy their inputs to the host (on the context stream, then
 * synchronise) and scan them: tau strictly increasing per atmosphere
 * (E_INVALID_ARG) and finite, q > 0 (E_INVALID_ARG), every source,
 * boundary and albedo array finite (E_NONFINITE).  Off by default: the scan
 * reads every input array once per call. */
#define PPRT_VALIDATE_INPUTS 0x1u
pprt_status pprt_set_validation(pprt_ctx* ctx, uint32_t flags);

/* The same scans on host arrays, without a device.  pprt_check_tau: tau
 * [sum nd] (host) finite and strictly increasing inside each atmosphere
 * (E_NONFINITE / E_INVALID_ARG, E_SHAPE for nd < 2).  pprt_check_finite:
 * n values of the given precision (host) finite, else E_NONFINITE.  msg
 * (host, len bytes, may be NULL) receives the reason. */
pprt_status pprt_check_tau(int32_t nbatch, const int32_t* nd, const double* tau, char* msg, size_t len);
pprt_status pprt_check_finite(int32_t precision, int64_t n, const void* x, char* msg, size_t len);

/* ------------------------------------------------------------------ plan */

typedef struct pprt_shape {
  int32_t nbatch;        /* number of atmospheres, >= 1                       */
  const int32_t* nd;     /* host [nbatch]: nodes per atmosphere, each >= 2     */
  int32_t na;            /* Gauss angles per hemisphere, 1..32                 */
  int32_t nf;            /* frequencies, >= 1                                  */
  int32_t precision;     /* pprt_precision of the bulk sweep                   */
  int32_t lower_bc;      /* pprt_lower_bc                                      */
  uint32_t outputs;      /* PPRT_OUT_* requested from pprt_formal_solution     */
  int32_t waves_per_block; /* 0 = tuned default; else 1, 2, 4 or 8             */
} pprt_shape;

/* Host-only check of a shape (no device needed): returns the status that
 * pprt_plan_create would return for it and writes a message into msg
 * (host buffer of msg_len bytes, may be NULL). */
pprt_status pprt_shape_check(const pprt_shape* shape, char* msg, size_t msg_len);

/* Validate a shape and build the plan: ragged offsets, the work list sorted
 * longest atmosphere first, angle constants.  `mu`/`w` (host, [na]) may be
 * NULL for the Gauss rule.  E_SHAPE / E_INVALID_ARG on bad input. */
pprt_status pprt_plan_create(pprt_ctx* ctx, const pprt_shape* shape,
                             const double* mu, const double* w, pprt_plan** out);
void pprt_plan_destroy(pprt_plan* plan);
/* Workspace the ALI calls need (bytes, 256-aligned pointer expected). */
pprt_status pprt_plan_workspace_bytes(const pprt_plan* plan, size_t* bytes);
/* Total rows (sum of nd) and the plan's angle rule (host copies). */
pprt_status pprt_plan_info(const pprt_plan* plan, int64_t* rows, double* mu, double* w);

/* ------------------------------------------------------- formal solution */

typedef struct pprt_fs_in {
  const double* tau;     /* [rows] reference optical depth                    */
  const void* q;         /* real [rows][nf]: chi_k / chi_ref, > 0              */
  const void* Sg;        /* real [rows][nf] source function S_k                */
  const void* Itop;      /* real [nb][nf][na] incident I- at node 0; NULL = 0  */
  const void* Bbot;      /* real [nb][nf] B_k at the last node  (DIFFUSION)    */
  const void* Bbot_prev; /* real [nb][nf] B_k at the node above (DIFFUSION)    */
  const void* Ibot;      /* real [nb][nf][na] I+ at the last node (GIVEN); NULL = 0 */
} pprt_fs_in;

typedef struct pprt_fs_out {
  void* J; void* JmS; void* lstar; void* lstar_c;   /* real [rows][nf]      */
  void* Iplus; void* Iminus;                        /* real [rows][nf][na]  */
  void* H;                                          /* real [rows][nf]      */
  void* Iemerg;                                     /* real [nb][nf][na]    */
  void* lstar_sub; void* lstar_sup;                 /* real [rows][nf]      */
} pprt_fs_out;

/* Formal solution without in-layer scattering (the omega = 0 layer
 * recursion: t+- = diag(exp(-dtau_k/mu_i)), r+- = 0, beta+- from a source
 * linear in tau_k between nodes), for every atmosphere of the plan.
 * Layer optical depth: dtau_k = (q_k(d)+q_k(d+1))/2 * (tau[d+1]-tau[d]).
 * Lower boundary: DIFFUSION  I+(last) = B + mu (B - B_prev)/dtau_k(last layer);
 * GIVEN  I+(last) = Ibot.  Every output whose bit is set in the plan's
 * `outputs` must be non-NULL; other pointers are ignored.
 * Difference form: I+-(d) - S(d) is propagated, so J - S is exact zero for
 * constant S and 1 - Lambda* keeps full relative accuracy in thick layers. */
pprt_status pprt_formal_solution(pprt_plan* plan, const pprt_fs_in* in, pprt_fs_out* out);

/* Formal solution with coherent isotropic scattering inside every layer
 * (the parameterised continuum scattering of Sect. 3.1, item 6; the layer
 * recursion with transmission t+-, reflection r+- and source beta+- of the
 * paper's notation).  `omega` (real [rows][nf]) is the single-scattering
 * albedo at each node, 0 <= omega <= 1; a layer takes the mean of its two
 * nodes and S^g = in->Sg, linear in the layer optical depth, is the
 * non-scattering source: S = (1 - omega) S^g + omega J.  Each layer is solved
 * exactly (discrete-ordinate eigen solution, no growing exponentials), layers
 * are combined by the adding method top-down and bottom-up, and every node
 * gets I+-, J, J - S^g, H and the exact diagonal Lambda*_dd = dJ(d)/dS^g(d)
 * with 1 - Lambda*.  na in {1, 2, 4, 8, 16, 32} (E_UNSUPPORTED otherwise);
 * plans with na = 32 run on the matrix cores (one frequency per wave, 16 x 16
 * FP64 tiles), the others on the vector units (na lanes per frequency, one
 * row of each operator per lane).
 * Precision: an FP64 plan computes in FP64 throughout.  An FP32 plan with
 * na <= 16 forms each layer's operators in FP64 and rounds them, keeps
 * arrays, composites, products and the adding recursion in FP32, and runs
 * the eliminations with I - (reflection)(reflection) in FP64 where the
 * thick-layer rule selects them (pprt_plan_set_thick_mode).  An FP32 plan
 * with na = 32 keeps its arrays and the workspace in FP32 (the layer
 * operators included, rounded to FP32 for both passes) and computes in
 * FP64: every elimination is FP64 (pprt_thick_counts counts them all) and
 * the thick modes change nothing.  Needs a workspace of
 * pprt_plan_scattering_workspace_bytes() per node and frequency:
 * 8 or 4 (3 na^2 + 7 na) bytes in FP64 or FP32 plans with na <= 16 (the
 * composite reflection and source of every node, two unit-source responses
 * of each layer and each layer's t, r and source vectors, which the
 * bottom-up pass reads instead of forming them again; FP32 plans keep the
 * rounded operators and form the FP64 ones again only for the eliminations
 * the thick-layer rule runs in FP64), and with na = 32 8 or 4 (na^2 + 3 na) bytes (FP64 or FP32
 * plans) plus 32 na bytes for each layer's eigen data (secular-equation
 * roots, Gu-Eisenstat vector, column norms), solved apart before the
 * recursion, and 8 or 4 (2 na^2 + 4 na) bytes more for each layer's t, r
 * and source vectors, which the bottom-up pass reads instead of forming
 * them again (an FP32 plan rounds them to FP32 for both passes); all kept
 * between the
 * top-down and the bottom-up pass; omega = 0 everywhere reproduces
 * pprt_formal_solution to rounding. */
pprt_status pprt_plan_scattering_workspace_bytes(const pprt_plan* plan, size_t* bytes);
pprt_status pprt_formal_solution_scattering(pprt_plan* plan, const pprt_fs_in* in,
                                            const void* omega, pprt_fs_out* out,
                                            void* workspace);

/* FP64 eliminations of the FP32-bulk scattering path (the precision split of
 * the layer recursion: FP32 bulk, FP64 for the inversions of optically thick
 * layers).  The recursion inverts I - r R_d on the way down and I - R^up r,
 * I - R^up R_d on the way up.  PPRT_THICK_RULE (the default) runs one of
 * these in FP64 when its layer's absorption depth dtau (1 - omega)^1/2
 * exceeds 1 or the bound |A|_inf |B|_inf of the reflection product |A B|
 * exceeds 1/2; the decision is taken for a wave of 64/na frequencies at once
 * (FP64 when any of them qualifies).  PPRT_THICK_NEVER keeps every
 * elimination in FP32 and PPRT_THICK_ALWAYS runs every one in FP64 (error
 * studies).  FP64 plans ignore the mode.  E_INVALID_ARG for another value. */
typedef enum pprt_thick_mode {
  PPRT_THICK_RULE = 0, PPRT_THICK_NEVER = 1, PPRT_THICK_ALWAYS = 2
} pprt_thick_mode;
pprt_status pprt_plan_set_thick_mode(pprt_plan* plan, int32_t mode);

/* Counters of the FP32-bulk scattering path, summed over every launch on the
 * context since it was created or last reset: eliminations run in FP64 and
 * all eliminations (one per wave and decision).  pprt_thick_counts
 * synchronises the context's stream; pprt_thick_counts_reset is ordered on
 * it. */
pprt_status pprt_thick_counts(pprt_ctx* ctx, uint64_t* fp64, uint64_t* total);
pprt_status pprt_thick_counts_reset(pprt_ctx* ctx);

/* ----------------------------------------------------- two-level atom ALI */

typedef struct pprt_two_level {
  const double* eps;     /* [nb] line thermalisation parameter, 0 <= eps <= 1 */
  const double* B;       /* [rows] Planck function per node                   */
  const void* wphi;      /* real [nf] wnu_k * phi_k (profile x frequency weight;
                            sum = 1)                                          */
} pprt_two_level;

typedef struct pprt_ali_ctl {
  double tol;            /* stop when max_d |dS|/|S_new| < tol per atmosphere */
  int32_t max_iter;      /* iteration cap, >= 1                               */
  int32_t iters_per_sync;/* iterations enqueued between host checks (>= 1)    */
  int32_t use_graph;     /* 1: capture the iterations_per_sync launches between
                            checks once in a hipGraph (on a private stream at
                            the default priority) and replay it; same results */
  int32_t resume;        /* 0: start afresh (iteration counts, convergence
                            flags and Ng history reset); 1: continue from the
                            state in the workspace, e.g. after
                            pprt_ali_state_import; max_iter caps the total */
} pprt_ali_ctl;

typedef struct pprt_ali_report {
  int32_t iterations;    /* iterations run (max over atmospheres)             */
  int32_t n_converged;   /* atmospheres that met the tolerance                */
  double max_rel;        /* largest last relative change over atmospheres     */
} pprt_ali_report;

/* One operator-splitting step for every atmosphere (pure two-level line,
 * complete redistribution, diagonal Lambda*; Sect. 2 and the local-operator
 * runs of Sect. 3.2.1):  a formal solution with S_k = S_l (the line source
 * function, per node, float64 `S` [rows]) fused with the profile quadratures
 *   Jbar - S_l = sum_k wphi_k (J_k - S_l),  1 - Lbar* = sum_k wphi_k (1 - Lambda*_k),
 * then in float64
 *   S_new = S + [(1-eps)(Jbar - S) + eps (B - S)] / [eps + (1-eps)(1 - Lbar*)].
 * `S` is updated in place; `max_rel` [nb] (device, double) receives
 * max_d |S_new - S|/|S_new|.  in->Sg is ignored.  Atmospheres whose
 * `active` flag (device int32 [nb], NULL = all) is 0 are left untouched.
 * Needs the plan workspace (E_WORKSPACE otherwise). */
pprt_status pprt_two_level_ali_step(pprt_plan* plan, const pprt_fs_in* in,
                                    const pprt_two_level* atom, double* S,
                                    double* max_rel, const int32_t* active,
                                    void* workspace);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * pprt_two_level_ali_step without the caller's workspace.  The step's
 * scratch (the per-tile moment partials and, with the tri-diagonal
 * operator, its per-row coefficients) lives in a static device array of
 * PPRT_NOALLOC_SCRATCH_BYTES bytes, one copy per GPU, which the process
 * holds until it ends; a plan whose pprt_plan_workspace_bytes exceeds it
 * gets E_WORKSPACE (split the batch into smaller plans), and plans with Ng
 * acceleration get E_UNSUPPORTED (Ng's history must persist between steps).
 * Every call on one GPU uses that GPU's single array, whatever the context or
 * stream: calls that overlap on one GPU race, and the caller must order
 * them.  No allocating call is made (plan metadata is allocated earlier, by
 * pprt_plan_create; the validation mode's host scan is not applied here);
 * the step writes every scratch entry before it reads it.
 * Other arguments, results and errors as pprt_two_level_ali_step. */
#define PPRT_NOALLOC_SCRATCH_BYTES (64u << 20)
pprt_status pprt_two_level_ali_step_noalloc(pprt_plan* plan, const pprt_fs_in* in,
                                            const pprt_two_level* atom, double* S,
                                            double* max_rel, const int32_t* active);

/* A persistent step graph (the batched configuration's "one hipGraph
 * launch"): `steps` consecutive pprt_two_level_ali_step calls on exactly
 * these arguments are captured once into a hipGraph (on a private stream at
 * the default priority) and instantiated; each pprt_graph_launch replays
 * them on the context stream current at launch time, asynchronously, with
 * the same results as the eager calls.  The pointers are baked into the
 * graph: every array and the workspace must stay allocated, at the same
 * addresses, until pprt_graph_destroy, and the plan must outlive the graph.
 * Launches of one graph, like the steps, must be ordered on one stream. */
typedef struct pprt_graph pprt_graph;
pprt_status pprt_two_level_graph_create(pprt_plan* plan, const pprt_fs_in* in,
                                        const pprt_two_level* atom, double* S, double* max_rel,
                                        const int32_t* active, void* workspace, int32_t steps,
                                        pprt_graph** out);
pprt_status pprt_graph_launch(pprt_graph* graph);
void pprt_graph_destroy(pprt_graph* graph);

/* The two halves of pprt_two_level_ali_step, for callers that schedule or
 * time them separately.  pprt_two_level_moments runs the formal solution
 * and leaves the profile-weighted moments (per row, frequency group and
 * hemisphere) in the workspace; pprt_two_level_update reads them and applies
 * the float64 update to S, writing max_rel [nb].  Same arguments, layouts
 * and errors as pprt_two_level_ali_step; the workspace must be the same. */
pprt_status pprt_two_level_moments(pprt_plan* plan, const pprt_fs_in* in,
                                   const pprt_two_level* atom, const double* S,
                                   const int32_t* active, void* workspace);
pprt_status pprt_two_level_update(pprt_plan* plan, const pprt_two_level* atom, double* S,
                                  double* max_rel, const int32_t* active, void* workspace);

/* Two-level line on a background continuum (Sect. 3.1, items 5-6: grey
 * continuum opacity with coherent isotropic scattering).  Per node and
 * frequency the non-scattering source is S^g_k = p_k S_l + c_k (p_k is the
 * line's share of the absorptive opacity, c_k the continuum's thermal part)
 * and omega_k the continuum albedo (NULL: no scattering inside layers). */
typedef struct pprt_continuum {
  const void* pfrac;     /* real [rows][nf] p_k = dS^g_k / dS_l, 0 < p <= 1   */
  const void* sg_const;  /* real [rows][nf] c_k                                */
  const void* omega;     /* real [rows][nf] or NULL                            */
} pprt_continuum;

/* Workspace of pprt_two_level_ali_step_continuum (bytes). */
pprt_status pprt_plan_continuum_workspace_bytes(const pprt_plan* plan, size_t* bytes);

/* One operator-splitting step of the line on a continuum: S^g assembly,
 * formal solution (with in-layer scattering when cont->omega is given: na in
 * {1,2,4,8,16,32}, FP32 plans with the FP64 eliminations of
 * pprt_formal_solution_scattering), then per node the profile quadratures
 *   Jbar - S_l = sum_k wphi_k [(J_k - S^g_k) + (S^g_k - S_l)],
 *   1 - Lbar*  = sum_k wphi_k [(1 - p_k) + p_k (1 - Lambda*_k)]
 * and the float64 update of pprt_two_level_ali_step.  in->Bbot/Bbot_prev are
 * required for the diffusion lower boundary; in->Sg is ignored.  Other
 * arguments as pprt_two_level_ali_step; the workspace is
 * pprt_plan_continuum_workspace_bytes(). */
pprt_status pprt_two_level_ali_step_continuum(pprt_plan* plan, const pprt_fs_in* in,
                                              const pprt_two_level* atom,
                                              const pprt_continuum* cont, double* S,
                                              double* max_rel, const int32_t* active,
                                              void* workspace);

/* Iterate pprt_two_level_ali_step from the given S (device [rows], float64,
 * in/out) until every atmosphere's max relative change is below ctl->tol or
 * ctl->max_iter is reached.  Each atmosphere stops at its own convergence.
 * `iters` (device int32 [nb], may be NULL) receives the per-atmosphere
 * iteration counts.  Synchronises the context stream every
 * ctl->iters_per_sync iterations to test for completion (reads nb flags).
 * E_NOT_CONVERGED if the cap was hit; the report is filled either way. */
pprt_status pprt_two_level_ali(pprt_plan* plan, const pprt_fs_in* in,
                               const pprt_two_level* atom, const pprt_ali_ctl* ctl,
                               double* S, int32_t* iters, pprt_ali_report* report,
                               void* workspace);

/* ---------------------------------------------------- multilevel atom */

/* A multilevel model atom on a grey background (the paper's rate operators
 * [R_ij], [R*_ij], [Delta R_ij] and rate matrix A, read as the full
 * preconditioning of Rybicki & Hummer 1991 with the diagonal Lambda*).
 * Every frequency belongs to exactly one transition (its window); units are
 * the caller's, consistent between radiative and collisional rates.  All
 * pointers are device memory, float64 except the int32 tables. */
typedef struct pprt_atom {
  int32_t nlev;              /* levels incl. any continuum level, 2..32            */
  int32_t ntr;               /* transitions, >= 1                                  */
  const int32_t* lower;      /* [ntr] lower level (0-based); level 0 is replaced    */
  const int32_t* upper;      /* [ntr] upper level  by number conservation          */
  const int32_t* k0;         /* [ntr] first frequency of the window                */
  const int32_t* k1;         /* [ntr] one past the last frequency of the window    */
  const int32_t* owner;      /* [nf] transition owning frequency k                 */
  const double* sigma;       /* [nf] absorption cross-section                      */
  const double* bfac;        /* [nf] b (2 h nu^3 / c^2 in the caller's units)       */
  const double* W;           /* [nf] rate quadrature weight (4 pi w / (h nu))       */
  const double* G;           /* [rows][nf] stimulated-emission factor               */
  const double* Bnu;         /* [rows][nf] Planck function                          */
  const double* kc;          /* [rows] continuum absorption per unit tau_ref        */
  const double* sc;          /* [rows] continuum scattering per unit tau_ref        */
  const double* ntot;        /* [rows] total number density of the atom             */
  const double* Cul;         /* [rows][ntr] downward collision rates                */
  const double* Clu;         /* [rows][ntr] upward collision rates                  */
  /* Optional depth-dependent Voigt lines (all four NULL: sigma[k] is used).
   * For k in the window of a line t (line_nu0[t] > 0) and row d:
   *   sigma = line_s[t] H(line_a[t], x) / (sqrt(pi) dnu_D),
   *   dnu_D = line_nu0[t] dopp[d],  x = (nu[k] - line_nu0[t]) / dnu_D,
   * H(a, x) = Re w(x + i a) evaluated on the device (see pprt_voigt).
   * Windows with line_nu0[t] == 0 (continua) keep sigma[k]. */
  const double* nu;          /* [nf] frequency of each point                        */
  const double* line_nu0;    /* [ntr] line centre, 0 for continua                   */
  const double* line_s;      /* [ntr] line strength                                 */
  const double* line_a;      /* [ntr] Voigt damping parameter (>= 0)                */
  const double* dopp;        /* [rows] Doppler width relative to the line centre    */
} pprt_atom;

/* Host validation of the atom (copies the tables to the host on the
 * context stream, then synchronises): level and window indices in range,
 * windows inside [0, nf), every frequency owned by the transition whose
 * window holds it (E_INVALID_ARG / E_SHAPE), and the rate-matrix pattern of
 * pprt_atom_check_host (E_SINGULAR).  The compute calls below re-read and
 * check the index tables on every call (a table rewritten in place is seen);
 * their kernels also test every index they use and raise PPRT_DEV_BADINDEX
 * instead of reading outside an array. */
pprt_status pprt_atom_check(pprt_plan* plan, const pprt_atom* atom);

/* Opacity and source assembly from populations pops [rows][nlev]:
 * q = kappa + sigma_c (per unit tau_ref), omega = sigma_c / q and
 * S^g = (eta + kappa_c B) / kappa, each [rows][nf] float64. */
pprt_status pprt_nlte_opacity(pprt_plan* plan, const pprt_atom* atom, const double* pops,
                              double* q, double* omega, double* Sg);

/* Preconditioned rates per (row, transition) [rows][ntr] from the old
 * populations and a formal solution's J and Lambda* ([rows][nf]):
 * [dR_lu] = sum W sigma dJ, [dR_ul] = sum W G sigma dJ,
 * [R*_ul] = sum W b G sigma (1 - p Lambda*), dJ = J - Lambda* eta/kappa. */
pprt_status pprt_rates_assemble(pprt_plan* plan, const pprt_atom* atom, const double* pops_old,
                                const double* J, const double* lstar, double* dRlu,
                                double* dRul, double* Rsul);

/* Statistical equilibrium per depth with P_lu = [dR_lu] + C_lu,
 * P_ul = [R*_ul] + [dR_ul] + C_ul and the ground-level equation replaced by
 * sum n = n_tot; LU with partial pivoting in float64.  pops_new [rows][nlev];
 * max_rel [nb] (may be NULL) = max |n_new - n_old| / n_new per atmosphere.
 * A singular system sets PPRT_DEV_SINGULAR (read by pprt_sync). */
pprt_status pprt_rates_solve(pprt_plan* plan, const pprt_atom* atom, const double* pops_old,
                             const double* dRlu, const double* dRul, const double* Rsul,
                             double* pops_new, double* max_rel);

/* Workspace of pprt_nlte_step (bytes) for an atom of nlev levels and ntr
 * transitions. */
pprt_status pprt_plan_nlte_workspace_bytes(const pprt_plan* plan, int32_t nlev, int32_t ntr,
                                           size_t* bytes);

/* Host-only form of pprt_atom_check on host copies of the tables (no
 * device): index tables as above, plus the rate-matrix pattern: a level all
 * of whose transitions have zero collision rates (both ways) and a zero
 * cross-section over the window at some depth row makes the statistical
 * equilibrium singular there (its row and column are empty): E_SINGULAR.
 * Reads lower, upper, k0, k1, owner, sigma, Cul, Clu [rows][ntr] and, with
 * Voigt lines (line_a != NULL), line_nu0 and line_s; the other fields are
 * ignored.  pprt_atom_check runs the same checks on the device tables. */
pprt_status pprt_atom_check_host(const pprt_atom* atom_host, int64_t rows, int32_t nf, char* msg,
                                 size_t len);

/* One accelerated-Lambda iteration of the multilevel atom: opacities from
 * pops, formal solution with in-layer continuum scattering (FP64 plans,
 * na in {1,2,4,8,16,32}), rate assembly and the per-depth solve; pops
 * [rows][nlev] is replaced by the new populations and max_rel [nb] gets the
 * largest relative change.  in->tau (and in->Itop, NULL = 0) are used; the
 * diffusion lower boundary takes B from atom->Bnu. */
pprt_status pprt_nlte_step(pprt_plan* plan, const pprt_fs_in* in, const pprt_atom* atom,
                           double* pops, double* max_rel, void* workspace);

/* The multilevel operator-splitting loop (Sect. 2; the convergence test of
 * Sect. 3.2.1 on the populations): from pops (device [rows][nlev], float64,
 * in/out) repeat pprt_nlte_step until every atmosphere's maximum relative
 * population change is below ctl->tol or ctl->max_iter steps were taken.
 * An atmosphere stops (its populations are frozen) at its own convergence;
 * `iters` (device int32 [nb], may be NULL) receives the per-atmosphere
 * counts.  The atom is validated once, tables and rate-matrix pattern
 * (pprt_atom_check).  Synchronises every ctl->iters_per_sync steps;
 * ctl->use_graph and ctl->resume must be 0.  Returns E_SINGULAR if a
 * per-depth system had no usable pivot (those rows keep their previous
 * populations), E_NONFINITE for NaN/Inf, E_NOT_CONVERGED at the cap; the
 * report is filled in every case that reaches the loop.  Workspace:
 * pprt_plan_nlte_workspace_bytes. */
pprt_status pprt_nlte_solve(pprt_plan* plan, const pprt_fs_in* in, const pprt_atom* atom,
                            const pprt_ali_ctl* ctl, double* pops, int32_t* iters,
                            pprt_ali_report* report, void* workspace);

/* ---- 1D spherical symmetry ----------------------------------------------
 * The formal solution on impact-parameter rays through spherical shells
 * (the geometry of the paper's 1D comparison calculations, Sect. 3.1), with
 * the same linear short-characteristic update per ray segment.  Shells
 * r_0 > .. > r_{nd-1} = R_core per atmosphere (node 0 outermost, finite,
 * positive, strictly decreasing: else PPRT_E_INVALID_ARG); the radial
 * reference optical depth tau (from pprt_fs_in, increasing inward) sets
 * chi_ref = dtau / dr per shell and q_k = chi_k / chi_ref, so a segment of
 * a ray with impact parameter p has the optical path (q_k(d) + q_k(d+1))/2
 * dtau_d (r_d + r_{d+1}) / (z_d + z_{d+1}), z = sqrt(r^2 - p^2).  Rays: n_core core rays with mu at the core
 * 1 - c/n_core (c = 0..n_core-1) and one tangent ray per shell.  At each
 * shell J, J - S, H use trapezoid weights in mu over the rays crossing it
 * (mu from 1 down to 0 at the shell's tangent ray); Lambda*_dd = dJ/dS(d)
 * exactly, including the round trip of tangent rays through their tangent
 * point.  Incident intensity Itop and core intensity Ibot (GIVEN) are
 * isotropic, [nb][nf]; the diffusion core uses B + mu (B - B_prev)/dtau_k
 * of the last radial layer with mu at the core.  Outputs J, JmS, lstar,
 * lstar_c, H ([rows][nf]).  r is a host array [rows], read during the call
 * only.  At most 65535 atmospheres, 1000 shells each and 1024 core rays per
 * plan.  A plan whose outputs are exactly JmS | LSTAR_C (what an ALI step
 * needs) runs the ray-group sweep; other output sets the per-frequency
 * sweep over single rays. */
typedef struct pprt_sph_plan pprt_sph_plan;
pprt_status pprt_sph_plan_create(pprt_ctx* ctx, int32_t nbatch, const int32_t* nd, int32_t nf,
                                 int32_t precision, int32_t lower_bc, uint32_t outputs,
                                 const double* r, int32_t n_core, pprt_sph_plan** out);
void pprt_sph_plan_destroy(pprt_sph_plan* plan);
pprt_status pprt_sph_plan_info(const pprt_sph_plan* plan, int64_t* rows, int32_t* nrays,
                               int64_t* ray_shell_pairs);
pprt_status pprt_sph_formal_solution(pprt_sph_plan* plan, const pprt_fs_in* in, pprt_fs_out* out);
/* Two-level operator-splitting step on spherical atmospheres: pure line,
 * diagonal Lambda*, the update of pprt_two_level_ali_step (the paper's
 * Sect. 3.2.2 line tests, here on the geometry above).  As there, in->Sg,
 * Bbot and Bbot_prev are ignored: the line source is S [rows] (FP64 state,
 * updated in place), the diffusion core takes atom->B at the two innermost
 * shells, and atmospheres with active[b] == 0 are left untouched.
 * workspace: pprt_sph_plan_workspace_bytes. */
pprt_status pprt_sph_plan_workspace_bytes(const pprt_sph_plan* plan, size_t* bytes);
pprt_status pprt_sph_two_level_ali_step(pprt_sph_plan* plan, const pprt_fs_in* in,
                                        const pprt_two_level* atom, double* S, double* max_rel,
                                        const int32_t* active, void* workspace);
/* The two halves of that step: the sweep, which leaves per 64-frequency tile
 * the profile-weighted sums of J - S and 1 - Lambda* in the workspace, and
 * the float64 update from them (same arguments as above). */
pprt_status pprt_sph_two_level_moments(pprt_sph_plan* plan, const pprt_fs_in* in,
                                       const pprt_two_level* atom, const double* S,
                                       const int32_t* active, void* workspace);
pprt_status pprt_sph_two_level_update(pprt_sph_plan* plan, const pprt_two_level* atom, double* S,
                                      double* max_rel, const int32_t* active, void* workspace);

/* ---- Voigt function ----------------------------------------------------
 * H(a, x) = Re w(x + i a), w the Faddeeva function, for a >= 0, by the
 * rational expansion of Weideman (1994) with N = 40 terms,
 *   w(z) ~ 2 p(Z) / (L - i z)^2 + (1/sqrt(pi)) / (L - i z),
 *   Z = (L + i z) / (L - i z),  L = (N / sqrt 2)^(1/2),
 * p(Z) = sum_{n<N} a_{n+1} Z^n, a_n the Fourier coefficients of
 * exp(-t^2)(L^2 + t^2), t = L tan(theta/2) (computed once on the host).
 * The same evaluation serves the multilevel opacity and rate kernels.
 * a, x, H: device [n] float64.  Asynchronous on the context stream. */
pprt_status pprt_voigt(pprt_ctx* ctx, int64_t n, const double* a, const double* x, double* H);

/* ---- Measured device peaks (diagnostic) ----------------------------------
 * Sustained rates of plain (non-packed) FP32 and FP64 vector FMA, of the
 * hardware exp2, and of a device-memory copy (read + write bytes), timed
 * with HIP events on the context stream (best of four launches).  `scratch`
 * is caller-owned device memory: at least n_CU * 16 * 256 * 8 bytes; the
 * copy is measured (half the buffer copied to the other half) when it holds
 * at least 128 MiB, else copy_gbs = 0.  The atomic rates (coalesced adds of
 * rows of 32 values at hashed rows of an array of up to 139425 rows, the
 * pattern of the 3D formal solution) need 32 x 8 x 1024 bytes, else 0.
 * Synchronises the stream. */
typedef struct pprt_peaks {
  double fp32_tflops;
  double fp64_tflops;
  double exp2_trate;     /* 1e12 exp2 per second */
  double copy_gbs;
  double atomic_f64_gadds;   /* 1e9 FP64 atomic adds per second */
  double atomic_f32_gadds;   /* 1e9 FP32 atomic adds per second */
} pprt_peaks;
pprt_status pprt_measure_peaks(pprt_ctx* ctx, void* scratch, size_t bytes, pprt_peaks* out);

/* ---- Approximate operator of the two-level ALI ---------------------------
 * PPRT_LSTAR_DIAG (default): the local operator, the exact diagonal of the
 * discrete Lambda.  PPRT_LSTAR_TRI: the non-local operator, its exact
 * tri-diagonal band (the 1D counterpart of the nearest-neighbour operator
 * whose convergence Sect. 3.2.1 compares with the local one):
 *   Lambda_{d,d+1} = 1/2 sum_i w_i [gamma_{d+1/2} + e_{d+1/2} alpha_{d+3/2}]  (up-going rays)
 *   Lambda_{d,d-1} = 1/2 sum_i w_i [gamma_{d-1/2} + e_{d-1/2} alpha_{d-3/2}]  (down-going rays)
 * (no alpha term next to a boundary node), profile-averaged like the
 * diagonal; the update then solves, per atmosphere in float64,
 *   [I - (1-eps) Lbar*] dS = (1-eps)(Jbar - S) + eps (B - S)
 * (tri-diagonal, diagonally dominant; Thomas elimination).
 * ng = 1 adds Ng acceleration (Ng 1974 in Auer's 1987 form, weights
 * 1/S^2).  It starts once an un-accelerated update changes S by less than
 * 1e-2 (maximum relative change over the atmosphere; that update's old and
 * new iterates open the first group); from then on, whenever four iterates
 * have gathered since the last extrapolation, S is replaced by the
 * extrapolated iterate.
 * Applies to pprt_two_level_ali_step / _update / _ali (not to the continuum
 * step).  Changes the workspace size: call before
 * pprt_plan_workspace_bytes.  pprt_two_level_ali resets Ng's history at
 * its start; callers stepping with pprt_two_level_ali_step call
 * pprt_two_level_reset before the first step. */
#define PPRT_LSTAR_DIAG 0
#define PPRT_LSTAR_TRI 1
pprt_status pprt_plan_set_operator(pprt_plan* plan, int32_t lstar, int32_t ng);
pprt_status pprt_two_level_reset(pprt_plan* plan, void* workspace);

/* ---- Checkpoint / resume of the two-level ALI ----------------------------
 * The state of an operator-splitting iteration is the source function S and
 * what the workspace carries between steps: per-atmosphere iteration counts,
 * last maximum relative changes and convergence flags (pprt_two_level_ali)
 * and Ng's group history and counter.  On resume an atmosphere steps again
 * unless it has met the new call's tolerance or iteration cap.  pprt_ali_state_export writes it into a caller-owned host buffer
 * of pprt_ali_state_bytes() bytes (a header fingerprints the batch shape,
 * precision and operator); pprt_ali_state_import restores it into S and a
 * workspace of a plan of the same shape and operator (E_SHAPE /
 * E_INVALID_ARG otherwise), so that stepping on (pprt_two_level_ali_step,
 * or pprt_two_level_ali with ctl->resume = 1) continues bit for bit as
 * the uninterrupted iteration would.  Both synchronise the context stream. */
pprt_status pprt_ali_state_bytes(const pprt_plan* plan, size_t* bytes);
pprt_status pprt_ali_state_export(pprt_plan* plan, const double* S, const void* workspace, void* host,
                                  size_t bytes);
pprt_status pprt_ali_state_import(pprt_plan* plan, const void* host, size_t bytes, double* S,
                                  void* workspace);

/* ---- Launch shape of the batched two-level sweep, and its autotuner ------
 * The batched sweep of pprt_two_level_moments / _ali_step / _ali runs one
 * wave per (atmosphere, 64-frequency tile, hemisphere), longest atmosphere
 * first.  Two launch parameters change its speed, never its result (each
 * wave's arithmetic is the same): waves per block (1, 2, 4, 8) and the grid
 * form, either one wave per item (persistent_waves_per_cu = 0) or a
 * persistent grid of n_CU * persistent_waves_per_cu waves that take items
 * from a device counter (zeroed by a kernel before each launch, so the
 * launch may be captured in a graph). */
pprt_status pprt_plan_set_launch(pprt_plan* plan, int32_t waves_per_block,
                                 int32_t persistent_waves_per_cu);
pprt_status pprt_plan_get_launch(const pprt_plan* plan, int32_t* waves_per_block,
                                 int32_t* persistent_waves_per_cu);

#define PPRT_TUNE_FORCE 0x1   /* re-measure even if this shape is cached */

typedef struct pprt_tune_report {
  int32_t waves_per_block;          /* chosen                                  */
  int32_t persistent_waves_per_cu;  /* chosen (0 = one wave per item)          */
  float best_ms;                    /* time of the chosen shape (best round)   */
  float default_ms;                 /* time of the plan's default shape        */
  int32_t candidates;               /* shapes measured                         */
  int32_t from_cache;               /* 1: taken from the in-process cache      */
} pprt_tune_report;

/* Time every launch shape (4 block sizes x {per-item, persistent at 8, 16,
 * 32 waves per CU}) on the caller's inputs with HIP events (three rounds
 * over all shapes, each one warm-up and three timed launches per shape,
 * moments only; S is read, not changed; the workspace's moment area is
 * overwritten), keep each shape's best round, and choose the fastest shape
 * when it beats the plan's default by more than 1% (else the default); the
 * choice goes into the plan and an in-process cache keyed by device,
 * precision, na, nf and the depth counts.  A later plan of the same shape takes the cached choice without
 * measuring unless flags has PPRT_TUNE_FORCE.  Synchronises the stream. */
pprt_status pprt_plan_autotune(pprt_plan* plan, const pprt_fs_in* in, const pprt_two_level* atom,
                               const double* S, void* workspace, int32_t flags,
                               pprt_tune_report* report);

/* ---- Gradients of the emergent spectrum (omega = 0; omega > 0 below) -----
 * The emergent intensity I+(tau_1, mu_i, nu_k) of the plane-parallel formal
 * solution without in-layer scattering (Sect. 3.2 comparison calculation,
 * linear source between nodes) and the vector-Jacobian product of that map:
 * given g = dL/dIemerg for any scalar loss L, the derivatives of L with
 * respect to every q and S^g entry and to the lower-boundary data.  The
 * adjoint is hand-written (reverse sweep of the layer recursion).  The
 * forward call keeps the difference-form intensity of every K-th depth node
 * in the workspace (layer checkpointing); the reverse call recomputes each
 * segment of K layers from the checkpoint below it.  K (checkpoint_interval)
 * is 1, 8, 16 or 32: memory sum_b (floor((nd_b - 1)/K) + 1) * nf * na reals.
 * Both calls take q, Sg, Bbot/Bbot_prev (DIFFUSION) or Ibot (GIVEN) from
 * `in`; Itop does not enter (I+ is independent of the down-going field when
 * omega = 0).  Element type follows the plan's precision.  Any na in 1..32
 * is supported (lanes are padded to a power of two). */
typedef struct pprt_fs_grad {
  void* dq;          /* real [rows][nf]     dL/dq   (required)                */
  void* dSg;         /* real [rows][nf]     dL/dS^g (required)                */
  void* dBbot;       /* real [nb][nf]       DIFFUSION; NULL = not written     */
  void* dBbot_prev;  /* real [nb][nf]       DIFFUSION; NULL = not written     */
  void* dIbot;       /* real [nb][nf][na]   GIVEN;     NULL = not written     */
} pprt_fs_grad;

/* Checkpoint workspace (bytes) for interval K; E_INVALID_ARG for other K. */
pprt_status pprt_plan_adjoint_workspace_bytes(const pprt_plan* plan, int32_t checkpoint_interval,
                                              size_t* bytes);

/* Forward: Iemerg [nb][nf][na] and the checkpoints in `workspace`
 * (caller-owned, at least pprt_plan_adjoint_workspace_bytes).  Asynchronous. */
pprt_status pprt_emergent_intensity(pprt_plan* plan, const pprt_fs_in* in,
                                    int32_t checkpoint_interval, void* Iemerg, void* workspace);

/* Reverse: gIemerg [nb][nf][na] in, gradients out.  `workspace` must hold
 * the checkpoints written by pprt_emergent_intensity for the same inputs
 * and interval (otherwise the result is undefined; nothing faults).
 * Every output entry is overwritten.  Asynchronous. */
pprt_status pprt_formal_solution_vjp(pprt_plan* plan, const pprt_fs_in* in,
                                     int32_t checkpoint_interval, const void* gIemerg,
                                     const pprt_fs_grad* grad, void* workspace);

/* ---- Gradients of the emergent spectrum with in-layer scattering --------
 * The vector-Jacobian product of the emergent intensity Iemerg (I+ at node
 * 0, [b][nf][na]) of pprt_formal_solution_scattering: given g = dL/dIemerg,
 * the derivatives of L with respect to every q and S^g entry and to the
 * lower-boundary data (grad->dBbot, dBbot_prev for DIFFUSION, grad->dIbot for
 * GIVEN, each NULL = not written).  omega and Itop are held fixed.  The
 * adjoint is hand-written: the call reruns the bottom-up adding recursion of
 * the layers below every node (composite reflection R^up and source S^up,
 * kept in the workspace with each layer's eigen solution) and then sweeps it
 * backwards from the top, with the derivatives of each layer's t, r and
 * difference-form source in its optical depth taken from the eigen form.
 * FP64 plans with na in {1, 2, 4, 8, 16} (E_UNSUPPORTED otherwise); in, omega
 * and gIemerg as for the forward call, device memory; workspace of
 * pprt_plan_scattering_vjp_workspace_bytes() = 8 (4 na^2 + 2 na) bytes per
 * node and frequency (the composites below every node, each layer's eigen
 * solution and the rows of its F_T and F_C').  Every dq and dSg entry is
 * overwritten.  Asynchronous. */
pprt_status pprt_plan_scattering_vjp_workspace_bytes(const pprt_plan* plan, size_t* bytes);
pprt_status pprt_formal_solution_scattering_vjp(pprt_plan* plan, const pprt_fs_in* in,
                                                const void* omega, const void* gIemerg,
                                                const pprt_fs_grad* grad, void* workspace);

/* ------------------------- 3D full characteristics, spherical voxel grid */

/* The paper's own method (Sect. 2: characteristics tracked through the grid
 * from boundary to boundary, stepping voxel to neighbouring voxel, every
 * voxel crossed by at least one per solid angle; Sect. 3.1: the spherical
 * grid regular in theta_c and phi_c, I = 0 incident outside and I_core
 * leaving the inner sphere; Sect. 3.2.1: the 3^3-neighbour Lambda*).
 * Voxel (i, j, k): r[i] <= r < r[i+1], theta_c in [j pi/nt, (j+1) pi/nt),
 * phi_c in [2 pi k/np, 2 pi (k+1)/np); index v = (i nt + j) np + k.  Opacity
 * chi and source S are constant inside a voxel, per frequency.  Directions:
 * mu at n_mu Gauss-Legendre nodes on (-1, 1) times n_phi azimuths (offset by
 * half a step), weights summing to one.  Per direction the characteristics
 * are a square lattice of parallel lines with spacing h across the direction
 * (each started on the outer sphere, plus one leaving the inner sphere where
 * a line meets it) and one through the centre of every voxel that no line
 * crossed.  J_v is the path-length weighted mean of the segment-mean
 * intensities S + (I_in - S)(1 - e^-D)/D over the characteristics that
 * cross v, summed over directions with their weights. */
typedef struct pprt_vox_grid {
  int32_t nr, nt, np;    /* 1 <= nr <= 1023, 2 <= nt <= 1023, 3 <= np <= 1023  */
  const double* r;       /* host [nr + 1], ascending by at least 1e-12 r[nr] per
                            shell (the walk takes crossings within 1e-13 r[nr]
                            of the current point as the surface just crossed),
                            r[0] > 0                                            */
} pprt_vox_grid;

typedef struct pprt_vox_plan pprt_vox_plan;

typedef struct pprt_vox_info {
  int64_t nvox, ndir, nrays, nsegments;
  int64_t ncoverage;     /* coverage characteristics (voxels no lattice line crossed) */
  double spacing;        /* lattice spacing h                                   */
  size_t device_bytes;   /* geometry held on the device                         */
} pprt_vox_info;

/* Builds the characteristics of every direction on the host (FP64, threaded
 * over directions) and uploads them: per segment the packed voxel index, the
 * path length and the mean weight (8 + 2 es bytes, es = 8 in FP64 and 4 in
 * FP32 plans).  spacing <= 0 takes r[0] pi / (2 nt) (half an inner boundary
 * face).  nf >= 1 frequencies.  E_INVALID_ARG for a bad grid or count,
 * E_SHAPE when the characteristics would exceed 2^31 segments. */
pprt_status pprt_vox_plan_create(pprt_ctx* ctx, const pprt_vox_grid* grid, int32_t n_mu, int32_t n_phi,
                                 double spacing, int32_t nf, int32_t precision, pprt_vox_plan** out);
pprt_status pprt_vox_plan_info(const pprt_vox_plan* plan, pprt_vox_info* info);
/* The same characteristics on the host only (no device, no context): call
 * with NULL arrays for the counts, then with arrays of those sizes (host):
 * ray_seg0 [nrays + 1], ray_dir [nrays], ray_core [nrays] (1: starts on the
 * inner sphere), seg_ijk [nseg] (i << 20 | j << 10 | k), seg_ell [nseg],
 * seg_wn [nseg] (direction weight over the direction's path length in the
 * voxel; 0 where a coverage characteristic does not enter the mean).
 * E_WORKSPACE if the arrays were sized for other counts. */
pprt_status pprt_vox_geometry_host(const pprt_vox_grid* grid, int32_t n_mu, int32_t n_phi, double spacing,
                                   int64_t* nrays, int64_t* nseg, int64_t* ray_seg0, int32_t* ray_dir,
                                   uint8_t* ray_core, uint32_t* seg_ijk, double* seg_ell, double* seg_wn);
/* Directions [ndir][3] and weights [ndir] into host arrays. */
pprt_status pprt_vox_directions(const pprt_vox_plan* plan, double* dirs, double* w);
void pprt_vox_plan_destroy(pprt_vox_plan* plan);

/* Formal solution: chi, S real [nvox][nf] (device); I_out, I_core real [nf]
 * (device, NULL = 0) entering at the outer and leaving the inner sphere.
 * Outputs (device, float64, overwritten): J [nvox][nf]; flux [nvox][3][nf]
 * (Cartesian components of sum w n I_bar, NULL = not computed); lstar
 * [nvox][27][nf] (NULL = not computed): Lambda*_{v,u} = dJ_v/dS_u for
 * u = (i+di, j+dj, k+dk), slot (di+1) 9 + (dj+1) 3 + (dk+1), phi periodic,
 * zero for neighbours beyond a radial boundary or a pole, followed along each
 * characteristic through its last 8 distinct voxels.  Accumulation by
 * atomic adds: FP64 plans in FP64; in FP32 plans J and the Lambda* band (the
 * flux in FP64) as FP32 sums over blocks of 64 directions added into the
 * FP64 outputs.  Results agree between runs to rounding, not bit for bit.
 * The plan holds 2 x 4 nvox nf bytes of block sums in FP32 plans, and the
 * first call of an FP32 plan that asks for lstar allocates 27 x 4 nvox nf
 * bytes more for the band's block sums (kept until the plan is destroyed;
 * E_DEVICE if that allocation fails).
 * Asynchronous on the context's stream; calls on one plan must not overlap. */
pprt_status pprt_vox_formal_solution(pprt_vox_plan* plan, const void* chi, const void* S, const void* I_out,
                                     const void* I_core, double* J, double* flux, double* lstar);

/* Grey two-level operator-splitting step on every voxel and frequency with
 * the diagonal of Lambda* (the local operator of Sect. 3.2.1):
 *   S <- S + ((1 - eps) J + eps B - S) / (1 - (1 - eps) Lambda*_vv),
 * S, B float64 [nvox][nf] (device; S in/out), eps float64 [nvox] (device),
 * max_rel float64 [1] (device) <- max |dS| / |S_new|.  The workspace
 * (pprt_vox_ali_workspace_bytes) holds J, Lambda*_vv and, in FP32 plans, S
 * rounded to the bulk type.  Asynchronous. */
pprt_status pprt_vox_ali_workspace_bytes(const pprt_vox_plan* plan, size_t* bytes);
pprt_status pprt_vox_ali_step(pprt_vox_plan* plan, const void* chi, double* S, const double* B,
                              const double* eps, const void* I_out, const void* I_core, double* max_rel,
                              void* workspace);

#ifdef __cplusplus
}
#endif
#endif /* PPRT_H */

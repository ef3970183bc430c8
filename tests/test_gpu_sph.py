"""GPU parity of the 1D spherical path (impact-parameter rays through shells,
the paper's 1D comparison geometry, Sect. 3.1): the formal solution (J, J - S,
H, Lambda* and 1 - Lambda*) against the FP64 oracle on ragged batches that span
two 256-frequency blocks and a ragged tail, Lambda* against brute-force unit
columns, the two-level operator-splitting step step by step, its convergence,
the active mask, and the plan's argument checks."""
import numpy as np
import pytest
import torch

from oracle import spherical
from paper_0903_1949_amd import pprt
from paper_0903_1949_amd import workloads as W
from tests.conftest import rel_err

pytestmark = pytest.mark.gpu

OUTS = pprt.OUT_J | pprt.OUT_JMS | pprt.OUT_LSTAR | pprt.OUT_LSTAR_C | pprt.OUT_H
TOL = {pprt.FP64: 1e-10, pprt.FP32: 1e-5}
# J - S and H are small differences of O(S) hemisphere terms; in FP32 their
# error follows the rounding of the terms, not their difference.  The binding
# check is against the scale of J, at FP32 rounding level (2e-6).  In the
# per-array metric, whose floor is 1e-4 max|H| while max|H| ~ 0.1 max|J| in
# these spheres and H falls to the floor at depth, that same rounding reads
# ~1e-3, so the per-array bound for them is 5e-3.
DIFF_KEYS = ("JmS", "H")
TOL_DIFF_FP32 = 5e-3
TOL_DIFF_OPERAND_FP32 = 2e-6


def r32(a):
    """Round an input to FP32 and back: the FP32 path's inputs, exactly."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _dev(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda:0")


def _case(nf=300, nb=3, nd_lo=20, nd_hi=40, n_core=8, seed=5, r_out=2.0, tau_hi=1e8):
    return W.spherical_batch(nb=nb, nd_lo=nd_lo, nd_hi=nd_hi, nf=nf, n_core=n_core, r_out=r_out,
                             tau_hi=tau_hi, B_slope=0.3, seed=seed)


@pytest.mark.parametrize("precision", [pprt.FP64, pprt.FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("lower", [pprt.BC_DIFFUSION, pprt.BC_GIVEN], ids=["diffusion", "given"])
@pytest.mark.parametrize("r_out", [2.0, 1.1], ids=["large", "small"])
def test_sph_formal_solution_parity(gpu_ctx, precision, lower, r_out):
    c = _case(r_out=r_out)
    rng = np.random.default_rng(11)
    rows, nf, nb = c.tau.shape[0], c.nf, c.nb
    Sg = rng.uniform(0.5, 1.5, size=(rows, nf))
    Itop = rng.uniform(0.0, 0.2, size=(nb, nf))
    Bb = rng.uniform(1.0, 1.5, size=(nb, nf))
    Bp = Bb * rng.uniform(0.8, 1.0, size=(nb, nf))
    dt = torch.float64 if precision == pprt.FP64 else torch.float32
    plan = pprt.SphPlan(gpu_ctx, c.nd, nf, c.r, c.n_core, precision=precision, lower_bc=lower,
                        outputs=OUTS)
    assert plan.rows == rows
    kw = dict(Itop=_dev(Itop, dt))
    if lower == pprt.BC_DIFFUSION:
        kw.update(Bbot=_dev(Bb, dt), Bbot_prev=_dev(Bp, dt))
    else:
        kw.update(Ibot=_dev(Bb, dt))
    print(f"  {c.name} precision={precision} lower={lower}", flush=True)
    out = plan.formal_solution(_dev(c.tau, torch.float64), _dev(c.q, dt), _dev(Sg, dt), **kw)
    torch.cuda.synchronize()
    got = {k: v.double().cpu().numpy() for k, v in out.items()}
    q = c.q
    if precision == pprt.FP32:      # the oracle sees exactly the inputs the FP32 path sees
        q, Sg, Itop, Bb, Bp = (r32(x) for x in (q, Sg, Itop, Bb, Bp))
    worst = {}
    for b in range(nb):
        s = c.rows(b)
        ref = spherical.formal_solution_sph(
            c.r[s], c.tau[s], q[s], Sg[s], c.n_core,
            lower="diffusion" if lower == pprt.BC_DIFFUSION else "given",
            Bbot=Bb[b], Bbot_prev=Bp[b], Itop=Itop[b])
        for name in ("J", "JmS", "lstar", "lstar_c", "H"):
            worst[name] = max(worst.get(name, 0.0), rel_err(got[name][s], ref[name]))
        scale = np.abs(ref["J"]).max()
        for name in DIFF_KEYS:
            e = float(np.max(np.abs(got[name][s] - ref[name])) / scale)
            worst[name + "_vs_J"] = max(worst.get(name + "_vs_J", 0.0), e)
    print("  " + ", ".join(f"{k} {v:.2e}" for k, v in worst.items()), flush=True)
    for name, e in worst.items():
        if precision == pprt.FP64:
            assert e < TOL[precision], name
        elif name.endswith("_vs_J"):
            assert e < TOL_DIFF_OPERAND_FP32, name
        else:
            assert e < (TOL_DIFF_FP32 if name in DIFF_KEYS else TOL[precision]), name


@pytest.mark.parametrize("precision", [pprt.FP64, pprt.FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("nb,n_core,lower", [(3, 8, pprt.BC_DIFFUSION), (19, 5, pprt.BC_DIFFUSION),
                                             (4, 3, pprt.BC_GIVEN)], ids=["3sph", "19sph", "given"])
def test_sph_group_sweep_parity(gpu_ctx, precision, nb, n_core, lower):
    """J - S and 1 - Lambda* only: the ray-group sweep.  Shell counts from 6
    (groups entirely within their last G shells) to 40, core-ray counts that
    are not multiples of the group size, a ragged frequency tile, and with 19
    spheres the XCD-grouped work list."""
    c = W.spherical_batch(nb=nb, nd_lo=6, nd_hi=40, nf=150, n_core=n_core, tau_hi=1e8,
                          B_slope=0.3, seed=13)
    rng = np.random.default_rng(17)
    rows, nf = c.tau.shape[0], c.nf
    Sg = rng.uniform(0.5, 1.5, size=(rows, nf))
    Itop = rng.uniform(0.0, 0.2, size=(nb, nf))
    Bb = rng.uniform(1.0, 1.5, size=(nb, nf))
    Bp = Bb * rng.uniform(0.8, 1.0, size=(nb, nf))
    dt = torch.float64 if precision == pprt.FP64 else torch.float32
    plan = pprt.SphPlan(gpu_ctx, c.nd, nf, c.r, c.n_core, precision=precision, lower_bc=lower,
                        outputs=pprt.OUT_JMS | pprt.OUT_LSTAR_C)
    kw = dict(Itop=_dev(Itop, dt))
    if lower == pprt.BC_DIFFUSION:
        kw.update(Bbot=_dev(Bb, dt), Bbot_prev=_dev(Bp, dt))
    else:
        kw.update(Ibot=_dev(Bb, dt))
    print(f"  {c.name} precision={precision} lower={lower}", flush=True)
    out = plan.formal_solution(_dev(c.tau, torch.float64), _dev(c.q, dt), _dev(Sg, dt), **kw)
    torch.cuda.synchronize()
    got = {k: v.double().cpu().numpy() for k, v in out.items()}
    q = c.q
    if precision == pprt.FP32:
        q, Sg, Itop, Bb, Bp = (r32(x) for x in (q, Sg, Itop, Bb, Bp))
    worst = {}
    for b in range(nb):
        s = c.rows(b)
        ref = spherical.formal_solution_sph(
            c.r[s], c.tau[s], q[s], Sg[s], c.n_core,
            lower="diffusion" if lower == pprt.BC_DIFFUSION else "given",
            Bbot=Bb[b], Bbot_prev=Bp[b], Itop=Itop[b])
        worst["lstar_c"] = max(worst.get("lstar_c", 0.0), rel_err(got["lstar_c"][s], ref["lstar_c"]))
        worst["JmS"] = max(worst.get("JmS", 0.0), rel_err(got["JmS"][s], ref["JmS"]))
        e = float(np.max(np.abs(got["JmS"][s] - ref["JmS"])) / np.abs(ref["J"]).max())
        worst["JmS_vs_J"] = max(worst.get("JmS_vs_J", 0.0), e)
    print("  " + ", ".join(f"{k} {v:.2e}" for k, v in worst.items()), flush=True)
    if precision == pprt.FP64:
        assert max(worst.values()) < TOL[precision]
    else:
        assert worst["lstar_c"] < TOL[precision]
        assert worst["JmS"] < TOL_DIFF_FP32
        assert worst["JmS_vs_J"] < TOL_DIFF_OPERAND_FP32


def test_sph_lstar_is_the_brute_force_diagonal(gpu_ctx):
    c = _case(nf=5, nb=1, nd_lo=9, nd_hi=9, n_core=4, seed=2)
    plan = pprt.SphPlan(gpu_ctx, c.nd, c.nf, c.r, c.n_core, precision=pprt.FP64,
                        lower_bc=pprt.BC_GIVEN, outputs=pprt.OUT_LSTAR | pprt.OUT_LSTAR_C)
    Sg = np.ones((c.tau.shape[0], c.nf))
    out = plan.formal_solution(_dev(c.tau, torch.float64), _dev(c.q, torch.float64),
                               _dev(Sg, torch.float64))
    torch.cuda.synchronize()
    L = spherical.lambda_matrix_sph(c.r, c.tau, c.q, c.n_core)
    diag = np.stack([np.diag(L[k]) for k in range(c.nf)], axis=1)
    assert rel_err(out["lstar"].cpu().numpy(), diag) < 1e-10
    assert rel_err(out["lstar_c"].cpu().numpy(), 1.0 - diag) < 1e-10


def _ali_inputs(c, dt):
    return dict(tau=_dev(c.tau, torch.float64), q=_dev(c.q, dt), eps=_dev(c.eps, torch.float64),
                B=_dev(c.B, torch.float64), wphi=_dev(c.wnu * c.phi, dt))


@pytest.mark.parametrize("precision", [pprt.FP64, pprt.FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("nb,nd_lo,nd_hi,nf", [(3, 16, 28, 41), (17, 6, 20, 70)], ids=["3sph", "17sph"])
def test_sph_ali_steps_parity(gpu_ctx, precision, nb, nd_lo, nd_hi, nf):
    c = W.spherical_batch(nb=nb, nd_lo=nd_lo, nd_hi=nd_hi, nf=nf, n_core=6, eps_lo=1e-4,
                          eps_hi=1e-1, tau_hi=1e6, B_slope=0.3, seed=9)
    dt = torch.float64 if precision == pprt.FP64 else torch.float32
    plan = pprt.SphPlan(gpu_ctx, c.nd, c.nf, c.r, c.n_core, precision=precision)
    a = _ali_inputs(c, dt)
    S = _dev(c.B, torch.float64)
    mx = torch.zeros(c.nb, dtype=torch.float64, device="cuda:0")
    nsteps = 6
    for _ in range(nsteps):
        plan.two_level_ali_step(a["tau"], a["q"], S, a["eps"], a["B"], a["wphi"], mx)
    torch.cuda.synchronize()
    got, got_mx = S.cpu().numpy(), mx.cpu().numpy()
    tol = 1e-10 if precision == pprt.FP64 else 2e-6
    for b in range(c.nb):
        s = c.rows(b)
        ref = spherical.two_level_ali_sph(c.r[s], c.tau[s], c.q[s], c.phi, c.wnu, float(c.eps[b]),
                                          c.B[s], c.n_core, tol=0.0, max_iter=nsteps)
        e = float(np.max(np.abs(got[s] / ref["S"] - 1)))
        em = abs(got_mx[b] / ref["max_rel"][-1] - 1)
        print(f"  b={b} nd={c.nd[b]} eps={c.eps[b]:.2e}: S {e:.2e}, max_rel {em:.2e}", flush=True)
        assert e < tol
        assert em < (1e-6 if precision == pprt.FP64 else 1e-2)


@pytest.mark.parametrize("precision", [pprt.FP64, pprt.FP32], ids=["fp64", "fp32"])
def test_sph_ali_step_whole_spheres_at_scale(gpu_ctx, precision):
    """A batch of 8192 small spheres at 16 frequency tiles already gives the
    two-level step its 131,072 waves: every sphere is one unit with one partial
    slot per tile (visible in the workspace size), the layout the chunked
    batches above never reach.  S after one step on a sample of the spheres
    (the smallest, the largest and 14 drawn at random) against the oracle."""
    c = W.spherical_batch(nb=8192, nd_lo=3, nd_hi=6, nf=1024, n_core=2, eps_lo=1e-4,
                          eps_hi=1e-1, tau_hi=1e4, B_slope=0.3, seed=12)
    dt = torch.float64 if precision == pprt.FP64 else torch.float32
    es = 8 if precision == pprt.FP64 else 4
    plan = pprt.SphPlan(gpu_ctx, c.nd, c.nf, c.r, c.n_core, precision=precision)
    rows = int(c.nd.sum())
    assert plan.workspace_bytes == (rows * 16 * 4 * es + 255) // 256 * 256
    a = _ali_inputs(c, dt)
    S = _dev(c.B, torch.float64)
    mx = torch.zeros(c.nb, dtype=torch.float64, device="cuda:0")
    plan.two_level_ali_step(a["tau"], a["q"], S, a["eps"], a["B"], a["wphi"], mx)
    torch.cuda.synchronize()
    got = S.cpu().numpy()
    rng = np.random.default_rng(3)
    sample = sorted({int(np.argmin(c.nd)), int(np.argmax(c.nd)),
                     *rng.choice(c.nb, size=14, replace=False).tolist()})
    tol = 1e-10 if precision == pprt.FP64 else 2e-6
    for b in sample:
        s = c.rows(b)
        ref = spherical.two_level_ali_sph(c.r[s], c.tau[s], c.q[s], c.phi, c.wnu, float(c.eps[b]),
                                          c.B[s], c.n_core, tol=0.0, max_iter=1)
        e = float(np.max(np.abs(got[s] / ref["S"] - 1)))
        print(f"  b={b} nd={c.nd[b]}: S {e:.2e}", flush=True)
        assert e < tol


def test_sph_ali_converges_to_the_oracle(gpu_ctx):
    c = W.spherical_batch(nb=2, nd_lo=14, nd_hi=20, nf=25, n_core=5, eps_lo=1e-2, eps_hi=1e-1,
                          tau_hi=1e4, B_slope=0.3, seed=4)
    plan = pprt.SphPlan(gpu_ctx, c.nd, c.nf, c.r, c.n_core, precision=pprt.FP64)
    a = _ali_inputs(c, torch.float64)
    S = _dev(c.B, torch.float64)
    mx = torch.zeros(c.nb, dtype=torch.float64, device="cuda:0")
    it = 0
    for it in range(1, 5001):
        plan.two_level_ali_step(a["tau"], a["q"], S, a["eps"], a["B"], a["wphi"], mx)
        if it % 25 == 0 and float(mx.max().item()) < 1e-12:
            break
    torch.cuda.synchronize()
    got = S.cpu().numpy()
    for b in range(c.nb):
        s = c.rows(b)
        ref = spherical.two_level_ali_sph(c.r[s], c.tau[s], c.q[s], c.phi, c.wnu, float(c.eps[b]),
                                          c.B[s], c.n_core, tol=1e-12, max_iter=5000)
        e = float(np.max(np.abs(got[s] / ref["S"] - 1)))
        print(f"  b={b}: gpu steps {it}, oracle {ref['iterations']}, S rel err {e:.2e}", flush=True)
        assert ref["converged"] and e < 1e-9


def test_sph_active_mask_leaves_atmospheres_untouched(gpu_ctx):
    c = W.spherical_batch(nb=3, nd_lo=12, nd_hi=16, nf=17, n_core=4, seed=6)
    plan = pprt.SphPlan(gpu_ctx, c.nd, c.nf, c.r, c.n_core, precision=pprt.FP64)
    a = _ali_inputs(c, torch.float64)
    S = _dev(c.B * 0.9, torch.float64)
    mx = torch.full((c.nb,), -1.0, dtype=torch.float64, device="cuda:0")
    active = torch.tensor([1, 0, 1], dtype=torch.int32, device="cuda:0")
    plan.two_level_ali_step(a["tau"], a["q"], S, a["eps"], a["B"], a["wphi"], mx, active=active)
    torch.cuda.synchronize()
    got, m = S.cpu().numpy(), mx.cpu().numpy()
    s1 = c.rows(1)
    assert np.array_equal(got[s1], c.B[s1] * 0.9)
    assert m[1] == -1.0 and m[0] > 0 and m[2] > 0
    assert not np.array_equal(got[c.rows(0)], c.B[c.rows(0)] * 0.9)


def test_sph_plan_argument_checks(gpu_ctx):
    c = _case(nf=8, nb=1, nd_lo=6, nd_hi=6)
    bad_r = c.r.copy()
    bad_r[2] = bad_r[1]                      # not strictly decreasing
    with pytest.raises(pprt.PprtError, match="E_INVALID_ARG"):
        pprt.SphPlan(gpu_ctx, c.nd, c.nf, bad_r, c.n_core)
    with pytest.raises(pprt.PprtError, match="E_SHAPE"):
        pprt.SphPlan(gpu_ctx, [1], c.nf, c.r[:1], c.n_core)
    with pytest.raises(pprt.PprtError, match="E_INVALID_ARG"):
        pprt.SphPlan(gpu_ctx, c.nd, c.nf, c.r, 0)
    with pytest.raises(pprt.PprtError, match="E_UNSUPPORTED"):
        pprt.SphPlan(gpu_ctx, c.nd, c.nf, c.r, c.n_core, outputs=pprt.OUT_IPLUS)
    plan = pprt.SphPlan(gpu_ctx, c.nd, c.nf, c.r, c.n_core, precision=pprt.FP64,
                        lower_bc=pprt.BC_DIFFUSION, outputs=pprt.OUT_J)
    Sg = _dev(np.ones((c.tau.shape[0], c.nf)), torch.float64)
    with pytest.raises(pprt.PprtError, match="E_INVALID_ARG"):   # diffusion needs Bbot
        plan.formal_solution(_dev(c.tau, torch.float64), _dev(c.q, torch.float64), Sg)
    big = W.spherical_batch(nb=1, nd_lo=1001, nd_hi=1001, nf=4, n_core=4, seed=1)
    with pytest.raises(pprt.PprtError, match="E_SHAPE"):          # more shells than the cap
        pprt.SphPlan(gpu_ctx, big.nd, big.nf, big.r, big.n_core)


def _edge_parity(ctx, c, outputs, precision=pprt.FP64):
    rng = np.random.default_rng(23)
    rows, nf, nb = c.tau.shape[0], c.nf, c.nb
    Sg = rng.uniform(0.5, 1.5, size=(rows, nf))
    Bb = rng.uniform(1.0, 1.5, size=(nb, nf))
    Bp = Bb * rng.uniform(0.8, 1.0, size=(nb, nf))
    dt = torch.float64 if precision == pprt.FP64 else torch.float32
    plan = pprt.SphPlan(ctx, c.nd, nf, c.r, c.n_core, precision=precision, outputs=outputs)
    out = plan.formal_solution(_dev(c.tau, torch.float64), _dev(c.q, dt), _dev(Sg, dt),
                               Bbot=_dev(Bb, dt), Bbot_prev=_dev(Bp, dt))
    torch.cuda.synchronize()
    worst = {}
    for b in range(nb):
        s = c.rows(b)
        ref = spherical.formal_solution_sph(c.r[s], c.tau[s], c.q[s], Sg[s], c.n_core,
                                            Bbot=Bb[b], Bbot_prev=Bp[b])
        for name, t in out.items():
            worst[name] = max(worst.get(name, 0.0), rel_err(t.double().cpu().numpy()[s], ref[name]))
    return worst


@pytest.mark.parametrize("outputs", [OUTS, pprt.OUT_JMS | pprt.OUT_LSTAR_C], ids=["all", "group"])
@pytest.mark.parametrize("shape", ["2shells_1core", "1freq", "40core", "400shells"])
def test_sph_edge_shapes(gpu_ctx, outputs, shape):
    """Degenerate and large shapes, FP64 against the oracle: two shells and a
    single core ray (one group, every shell in its last G); one frequency
    (63 idle lanes of the tile); 40 core rays (three groups hold core rays);
    400 shells (about 26 ray groups per sphere)."""
    kw = {"2shells_1core": dict(nb=2, nd_lo=2, nd_hi=2, nf=5, n_core=1),
          "1freq": dict(nb=3, nd_lo=10, nd_hi=30, nf=1, n_core=6),
          "40core": dict(nb=2, nd_lo=20, nd_hi=30, nf=7, n_core=40),
          "400shells": dict(nb=1, nd_lo=400, nd_hi=400, nf=3, n_core=8)}[shape]
    c = W.spherical_batch(tau_hi=1e8, B_slope=0.3, seed=31, **kw)
    worst = _edge_parity(gpu_ctx, c, outputs)
    print(f"  {shape}: " + ", ".join(f"{k} {v:.2e}" for k, v in worst.items()), flush=True)
    assert max(worst.values()) < 1e-10

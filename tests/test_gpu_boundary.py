"""GPU checks of the C-ABI calls around the hot path: the multilevel loop
(pprt_nlte_solve) against the oracle's loop, its failure returns
(E_NOT_CONVERGED, E_SINGULAR from the pattern pre-check, the SINGULAR device
bit with the old populations kept), model-atom tables rewritten in place,
the validation mode, and checkpoint/resume of the two-level ALI (bitwise)."""
import copy

import numpy as np
import pytest
import torch

from oracle import rates
from paper_0903_1949_amd import pprt
from paper_0903_1949_amd import workloads as W

pytestmark = pytest.mark.gpu


def _dev(a, dt=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda:0")


def _mplan(ctx, a):
    return pprt.Plan(ctx, a.nd, a.na, a.nf, precision=pprt.FP64, outputs=pprt.OUT_J | pprt.OUT_LSTAR)


@pytest.fixture(scope="module")
def small_atom():
    return W.multilevel_atom(nbound=3, ncont=2, nd=16, na=4, nline_pts=10, ncont_pts=6, seed=11)


def _count_slack(ref, tol):
    """0 when the oracle's last two changes sit clearly on either side of
    tol (10%), else 1: the populations of the two sides agree to ~1e-9
    relative, so a change that lands within rounding of tol may cross it one
    iteration earlier or later."""
    h = ref["max_rel"]
    k = ref["iterations"]
    clear = h[k - 1] < 0.9 * tol and (k < 2 or h[k - 2] > 1.1 * tol)
    return 0 if clear else 1


@pytest.mark.parametrize("tol", [1e-7, 1e-9])
def test_nlte_solve_matches_oracle_loop(gpu_ctx, small_atom, tol):
    a = small_atom
    plan = _mplan(gpu_ctx, a)
    da = pprt.DeviceAtom(a)
    pops = da.nstar.clone()
    iters = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    rep = plan.nlte_solve(da.tau, da, pops, tol=tol, max_iter=400, iters_per_sync=16, iters=iters)
    ref = rates.nlte_solve(a, plan.mu, plan.w, tol=tol, max_iter=400)
    e = float(np.max(np.abs(pops.cpu().numpy() / ref["pops"] - 1)))
    slack = _count_slack(ref, tol)
    print(f"  tol {tol:.0e}: gpu {rep['iterations']} iterations, oracle {ref['iterations']} "
          f"(last changes {ref['max_rel'][-2:]}, slack {slack}), rel err {e:.2e}", flush=True)
    assert rep["status"] == "OK" and rep["n_converged"] == 1
    assert int(iters.item()) == rep["iterations"]
    assert abs(rep["iterations"] - ref["iterations"]) <= slack
    assert e < 1e-8


def test_nlte_solve_batch_freezes_converged_atmospheres(gpu_ctx):
    a = W.multilevel_atom(nbound=3, ncont=2, nd=14, na=4, nline_pts=8, ncont_pts=6, seed=5, nb=3)
    # the recipe stacks identical atmospheres: scale the collision rates
    # (both ways, so detailed balance holds) so that each converges at its own pace
    a.Cul = a.Cul.copy(); a.Clu = a.Clu.copy()
    for b in range(a.nb):
        s = slice(int(a.off[b]), int(a.off[b + 1]))
        a.Cul[s] *= 10.0 ** (2 * b - 2); a.Clu[s] *= 10.0 ** (2 * b - 2)
    plan = _mplan(gpu_ctx, a)
    da = pprt.DeviceAtom(a)
    pops = da.nstar.clone()
    iters = torch.zeros(a.nb, dtype=torch.int32, device="cuda:0")
    plan.nlte_solve(da.tau, da, pops, tol=1e-7, max_iter=300, iters_per_sync=5, iters=iters)
    got = pops.cpu().numpy()
    off = a.off
    counts = []
    for b in range(a.nb):
        s = slice(int(off[b]), int(off[b + 1]))
        sub = copy.deepcopy(a)
        for k in ("tau", "T", "Gst", "Bnu", "kc", "sc", "nstar", "ntot", "Cul", "Clu"):
            setattr(sub, k, getattr(a, k)[s])
        sub.nd = a.nd[b:b + 1]
        ref = rates.nlte_solve(sub, plan.mu, plan.w, tol=1e-7, max_iter=300)
        e = float(np.max(np.abs(got[s] / ref["pops"] - 1)))
        print(f"  atmosphere {b}: gpu {int(iters[b])} oracle {ref['iterations']} rel err {e:.2e}", flush=True)
        counts.append(ref["iterations"])
        assert abs(int(iters[b]) - ref["iterations"]) <= _count_slack(ref, 1e-7)
        assert e < 1e-8
    assert len(set(counts)) > 1      # the atmospheres really stopped at different steps


def test_nlte_solve_not_converged(gpu_ctx, small_atom):
    plan = _mplan(gpu_ctx, small_atom)
    da = pprt.DeviceAtom(small_atom)
    pops = da.nstar.clone()
    rep = plan.nlte_solve(da.tau, da, pops, tol=1e-30, max_iter=2, iters_per_sync=1,
                          raise_not_converged=False)
    assert rep["status"] == "E_NOT_CONVERGED" and rep["iterations"] == 2 and rep["n_converged"] == 0


def _isolate(atom, j):
    a = copy.deepcopy(atom)
    a.sigma = a.sigma.copy(); a.Cul = a.Cul.copy(); a.Clu = a.Clu.copy()
    for t in range(a.nt):
        if int(a.lo[t]) == j or int(a.up[t]) == j:
            a.sigma[int(a.k0[t]):int(a.k1[t])] = 0.0
            a.Cul[:, t] = 0.0
            a.Clu[:, t] = 0.0
    return a


def test_nlte_solve_singular_pattern_refused_before_launch(gpu_ctx, small_atom):
    a = _isolate(small_atom, 1)
    plan = _mplan(gpu_ctx, a)
    da = pprt.DeviceAtom(a)
    pops = da.nstar.clone()
    before = pops.clone()
    with pytest.raises(pprt.PprtError, match="E_SINGULAR"):
        plan.nlte_solve(da.tau, da, pops, tol=1e-8, max_iter=5)
    assert torch.equal(pops, before)


def test_singular_rows_keep_old_populations(gpu_ctx, small_atom):
    """A level whose rates are all zero gives an exactly zero row (level
    j != 0): the device solve raises SINGULAR and leaves those rows'
    populations as they were instead of writing Inf/NaN."""
    a = _isolate(small_atom, 2)
    plan = _mplan(gpu_ctx, a)
    da = pprt.DeviceAtom(a)
    rows = a.tau.shape[0]
    rng = np.random.default_rng(4)
    J = rng.uniform(0.2, 2.0, size=(rows, a.nf)) * a.Bnu
    L = rng.uniform(0.0, 1.0, size=(rows, a.nf))
    ref = rates.preconditioned_rates(a, a.nstar, J, L)
    pops = _dev(a.nstar)
    gpu_ctx.sync()
    pn, _ = plan.rates_solve(da, pops, *[_dev(r) for r in ref])
    with pytest.raises(pprt.PprtError, match="E_SINGULAR"):
        gpu_ctx.sync()
    assert torch.equal(pn, pops)


def test_tables_rewritten_in_place_are_seen(gpu_ctx, small_atom):
    plan = _mplan(gpu_ctx, small_atom)
    da = pprt.DeviceAtom(small_atom)
    pops = da.nstar.clone()
    plan.nlte_opacity(da, pops)            # passes
    da.t["upper"][1] = small_atom.nl        # queued on the context stream, after the call above
    with pytest.raises(pprt.PprtError, match="E_INVALID_ARG"):
        plan.nlte_opacity(da, pops)
    da.t["upper"][1] = int(small_atom.up[1])
    plan.nlte_opacity(da, pops)
    gpu_ctx.sync()


def test_validation_mode(gpu_ctx):
    batch = W.two_level_batch(nb=3, nd_lo=10, nd_hi=20, na=4, nf=64, seed=2)
    plan = pprt.Plan(gpu_ctx, batch.nd, batch.na, batch.nf, precision=pprt.FP64,
                     outputs=pprt.OUT_JMS)
    db = pprt.upload_two_level(batch, pprt.FP64)
    Sg = _dev(np.repeat(batch.S_trial[:, None], batch.nf, 1))
    gpu_ctx.set_validation(True)
    try:
        plan.formal_solution(db.tau, db.q, Sg, Bbot=db.Bbot, Bbot_prev=db.Bbot_prev)
        tau = db.tau.clone()
        tau[int(batch.off[1]) + 3] = tau[int(batch.off[1]) + 2]
        with pytest.raises(pprt.PprtError, match="E_INVALID_ARG.*strictly increasing"):
            plan.formal_solution(tau, db.q, Sg, Bbot=db.Bbot, Bbot_prev=db.Bbot_prev)
        q = db.q.clone()
        q[5, 7] = float("nan")
        with pytest.raises(pprt.PprtError, match="E_NONFINITE"):
            plan.formal_solution(db.tau, q, Sg, Bbot=db.Bbot, Bbot_prev=db.Bbot_prev)
        q = db.q.clone()
        q[5, 7] = 0.0
        with pytest.raises(pprt.PprtError, match="E_INVALID_ARG"):
            plan.formal_solution(db.tau, q, Sg, Bbot=db.Bbot, Bbot_prev=db.Bbot_prev)
        S = db.S.clone()
        S[4] = float("inf")
        mx = torch.zeros(plan.nb, dtype=torch.float64, device="cuda:0")
        with pytest.raises(pprt.PprtError, match="E_NONFINITE"):
            plan.two_level_ali_step(db.tau, db.q, S, db.eps, db.B, db.wphi, mx)
    finally:
        gpu_ctx.set_validation(False)
    # off again: the non-monotone grid is not scanned (and nothing faults)
    plan.formal_solution(db.tau, db.q, Sg, Bbot=db.Bbot, Bbot_prev=db.Bbot_prev)
    gpu_ctx.sync()


@pytest.mark.parametrize("prec", [pprt.FP64, pprt.FP32])
@pytest.mark.parametrize("tri,ng", [(False, False), (True, True), (False, True)])
def test_ali_state_resume_is_bitwise(gpu_ctx, prec, tri, ng):
    batch = W.two_level_batch(nb=5, nd_lo=12, nd_hi=60, na=8, nf=128, seed=21)
    k = 7

    def fresh():
        plan = pprt.Plan(gpu_ctx, batch.nd, batch.na, batch.nf, precision=prec)
        plan.set_operator(pprt.LSTAR_TRI if tri else pprt.LSTAR_DIAG, ng)
        plan.two_level_reset()
        db = pprt.upload_two_level(batch, prec)
        db.S.copy_(db.B)
        return plan, db

    mx = torch.zeros(batch.nb, dtype=torch.float64, device="cuda:0")
    plan, db = fresh()
    for _ in range(2 * k):
        plan.two_level_ali_step(db.tau, db.q, db.S, db.eps, db.B, db.wphi, mx)
    S_ref = db.S.clone()

    plan, db = fresh()
    for _ in range(k):
        plan.two_level_ali_step(db.tau, db.q, db.S, db.eps, db.B, db.wphi, mx)
    image = plan.ali_state_export(db.S)
    del plan
    plan2, db2 = fresh()
    db2.S.fill_(-1.0)
    plan2.ali_state_import(image, db2.S)
    for _ in range(k):
        plan2.two_level_ali_step(db2.tau, db2.q, db2.S, db2.eps, db2.B, db2.wphi, mx)
    torch.cuda.synchronize()
    assert torch.equal(db2.S, S_ref)


def test_ali_loop_resume_is_bitwise(gpu_ctx):
    batch = W.two_level_batch(nb=6, nd_lo=12, nd_hi=60, na=8, nf=128, seed=22)

    def fresh():
        plan = pprt.Plan(gpu_ctx, batch.nd, batch.na, batch.nf, precision=pprt.FP32)
        plan.set_operator(pprt.LSTAR_TRI, True)
        db = pprt.upload_two_level(batch, pprt.FP32)
        db.S.copy_(db.B)
        return plan, db

    plan, db = fresh()
    rep = plan.two_level_ali(db.tau, db.q, db.S, db.eps, db.B, db.wphi, tol=1e-300, max_iter=24,
                             iters_per_sync=6, raise_not_converged=False)
    S_ref = db.S.clone()
    plan, db = fresh()
    plan.two_level_ali(db.tau, db.q, db.S, db.eps, db.B, db.wphi, tol=1e-300, max_iter=12,
                       iters_per_sync=6, raise_not_converged=False)
    image = plan.ali_state_export(db.S)
    plan2, db2 = fresh()
    plan2.ali_state_import(image, db2.S)
    rep2 = plan2.two_level_ali(db2.tau, db2.q, db2.S, db2.eps, db2.B, db2.wphi, tol=1e-300,
                               max_iter=24, iters_per_sync=6, raise_not_converged=False, resume=True)
    torch.cuda.synchronize()
    assert rep2["iterations"] == rep["iterations"] == 24
    assert torch.equal(db2.S, S_ref)


def test_ali_state_refuses_other_shapes(gpu_ctx):
    b1 = W.two_level_batch(nb=3, nd_lo=12, nd_hi=30, na=4, nf=64, seed=1)
    b2 = W.two_level_batch(nb=3, nd_lo=12, nd_hi=30, na=4, nf=64, seed=2)
    p1 = pprt.Plan(gpu_ctx, b1.nd, 4, 64, precision=pprt.FP64)
    d1 = pprt.upload_two_level(b1, pprt.FP64)
    image = p1.ali_state_export(d1.S)
    p2 = pprt.Plan(gpu_ctx, b2.nd, 4, 64, precision=pprt.FP64)
    d2 = pprt.upload_two_level(b2, pprt.FP64)
    with pytest.raises(pprt.PprtError, match="E_SHAPE"):
        p2.ali_state_import(image, d2.S)
    p3 = pprt.Plan(gpu_ctx, b1.nd, 4, 64, precision=pprt.FP32)
    with pytest.raises(pprt.PprtError, match="E_INVALID_ARG"):
        p3.ali_state_import(image, d1.S)
    with pytest.raises(pprt.PprtError, match="E_INVALID_ARG"):
        p1.ali_state_import(image[:100], d1.S)


@pytest.mark.parametrize("prec", [pprt.FP32, pprt.FP64])
def test_step_graph_replays_equal_eager_steps(gpu_ctx, prec):
    """pprt_two_level_graph_create / pprt_graph_launch: every replay, with
    eager work and a synchronisation between replays, equals the eager
    steps bit for bit (one-step and three-step graphs)."""
    batch = W.two_level_batch(nb=7, nd_lo=20, nd_hi=90, na=8, nf=200, seed=41)
    plan = pprt.Plan(gpu_ctx, batch.nd, batch.na, batch.nf, precision=prec)
    db = pprt.upload_two_level(batch, prec)
    ref = pprt.upload_two_level(batch, prec)
    mx = torch.zeros(batch.nb, dtype=torch.float64, device="cuda:0")
    mx_ref = torch.zeros_like(mx)
    g1 = plan.two_level_graph(db.tau, db.q, db.S, db.eps, db.B, db.wphi, mx, steps=1)
    g3 = plan.two_level_graph(db.tau, db.q, db.S, db.eps, db.B, db.wphi, mx, steps=3)
    for rep in range(3):
        g1.launch()
        plan.two_level_ali_step(ref.tau, ref.q, ref.S, ref.eps, ref.B, ref.wphi, mx_ref)
        torch.cuda.synchronize()
        assert torch.equal(db.S, ref.S) and torch.equal(mx, mx_ref), rep
        g3.launch()
        for _ in range(3):
            plan.two_level_ali_step(ref.tau, ref.q, ref.S, ref.eps, ref.B, ref.wphi, mx_ref)
        torch.cuda.synchronize()
        assert torch.equal(db.S, ref.S) and torch.equal(mx, mx_ref), rep
    g1.close(); g3.close()

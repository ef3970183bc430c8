"""GPU parity of the non-local (tri-diagonal) approximate operator and of Ng
acceleration with the oracle: the band from the sweep's closed forms against
the band of the brute-force Lambda matrix; one operator-splitting step; the
converged single slab with the same iteration counts; graph replay."""
import numpy as np
import pytest
import torch

from oracle import ali
from paper_0903_1949_amd import pprt
from paper_0903_1949_amd import workloads as W
from tests.conftest import rel_err, switch_slab
from tests.test_gpu_fs import _random_batch, r32

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,tol", [(pprt.FP64, 1e-10), (pprt.FP32, 1e-5)])
@pytest.mark.parametrize("na", [4, 8])
def test_band_matches_brute_force_lambda(gpu_ctx, prec, tol, na):
    nds, nf = [9, 16, 3, 2, 30], 37
    tau, q, S, Bb, Bp, _, _ = _random_batch(nds, nf, na, 17 + na, pprt.BC_DIFFUSION)
    plan = pprt.Plan(gpu_ctx, nds, na, nf, precision=prec,
                     outputs=pprt.OUT_LSTAR | pprt.OUT_LSTAR_SUB | pprt.OUT_LSTAR_SUP)
    dev = lambda a, d=plan.dtype: torch.as_tensor(np.ascontiguousarray(a), dtype=d, device="cuda:0")
    out = plan.formal_solution(dev(tau, torch.float64), dev(q), dev(S), Bbot=dev(Bb), Bbot_prev=dev(Bp))
    torch.cuda.synchronize()
    if prec == pprt.FP32:
        q = r32(q)
    off = np.concatenate([[0], np.cumsum(nds)])
    worst = {}
    for b in range(len(nds)):
        s = slice(off[b], off[b + 1])
        sub, diag, sup = ali.lambda_band(tau[s], q[s], plan.mu, plan.w)
        for name, ref in (("lstar_sub", sub), ("lstar", diag), ("lstar_sup", sup)):
            worst[name] = max(worst.get(name, 0.0), rel_err(out[name][s].double().cpu().numpy(), ref))
    print("  band errors", {k: f"{v:.2e}" for k, v in worst.items()}, flush=True)
    for k, e in worst.items():
        assert e < tol, (k, e)


def _small_batch(prec, nb=4, nf=64, na=4, seed=8):
    batch = W.two_level_batch(nb=nb, nd_lo=12, nd_hi=40, na=na, nf=nf, seed=seed)
    return batch, pprt.upload_two_level(batch, prec)


@pytest.mark.parametrize("prec,tol", [(pprt.FP64, 1e-10), (pprt.FP32, 1e-5)])
@pytest.mark.parametrize("ng", [False, True])
def test_nonlocal_steps_match_oracle(gpu_ctx, prec, tol, ng):
    """Four operator-splitting steps from S = B (with Ng the fourth state is
    the first extrapolation) against the oracle, atmosphere by atmosphere."""
    batch, db = _small_batch(prec)
    plan = pprt.Plan(gpu_ctx, batch.nd, batch.na, batch.nf, precision=prec)
    plan.set_operator(pprt.LSTAR_TRI, ng)
    plan.two_level_reset()
    db.S.copy_(db.B)
    mx = torch.zeros(plan.nb, dtype=torch.float64, device="cuda:0")
    for _ in range(4):
        plan.two_level_ali_step(db.tau, db.q, db.S, db.eps, db.B, db.wphi, mx)
    torch.cuda.synchronize()
    off = batch.off
    rnd = r32 if prec == pprt.FP32 else (lambda a: a)
    worst = 0.0
    for b in range(batch.nb):
        s = slice(off[b], off[b + 1])
        ref = ali.two_level_ali_nonlocal(batch.tau[s], rnd(batch.q[s]), batch.phi, rnd(batch.wnu),
                                         float(batch.eps[b]), batch.B[s], plan.mu, plan.w,
                                         tol=1e-300, max_iter=4, operator="tri", ng=ng)
        worst = max(worst, rel_err(db.S[s].cpu().numpy(), ref["S"]))
    print(f"  tri ng={ng} prec={prec}: S after 4 steps {worst:.2e}", flush=True)
    assert worst < tol


@pytest.mark.parametrize("prec,tol", [(pprt.FP64, 1e-10), (pprt.FP32, 2e-6)])
@pytest.mark.parametrize("na", [4, 8])
def test_tri_steps_across_the_thin_thick_switch(gpu_ctx, na, prec, tol):
    """The tri-diagonal sweep's alpha, gamma and e per angle switch from their
    series to the exponential at Delta = 1/4 (in FP32 decided once per layer
    when every angle agrees): two steps on a slab whose layers put Delta
    within 1e-9..1e-3 of 1/4 for every angle, against the oracle."""
    batch = switch_slab(na)
    db = pprt.upload_two_level(batch, prec)
    plan = pprt.Plan(gpu_ctx, batch.nd, na, batch.nf, precision=prec)
    plan.set_operator(pprt.LSTAR_TRI, False)
    plan.two_level_reset()
    db.S.copy_(db.B)
    mx = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    for _ in range(2):
        plan.two_level_ali_step(db.tau, db.q, db.S, db.eps, db.B, db.wphi, mx)
    torch.cuda.synchronize()
    # the device holds the profile weights w phi rounded to the plan precision
    wnu = batch.wnu
    if prec == pprt.FP32:
        wnu = (batch.wnu * batch.phi).astype(np.float32).astype(np.float64) / batch.phi
    ref = ali.two_level_ali_nonlocal(batch.tau, batch.q, batch.phi, wnu,
                                     float(batch.eps[0]), batch.B, plan.mu, plan.w,
                                     tol=1e-300, max_iter=2, operator="tri", ng=False)
    e = rel_err(db.S.cpu().numpy(), ref["S"])
    print(f"  tri na={na} prec={prec}: S after 2 steps {e:.2e}", flush=True)
    assert e < tol


@pytest.mark.parametrize("ng", [False, True])
def test_nonlocal_converges_like_oracle_fp64(gpu_ctx, ng):
    """The single slab (nd 64, na 4, nf 21, eps 1e-4, tol 1e-8) with the
    tri-diagonal operator: same S; without Ng the same iteration count.  With
    Ng at most one Ng cycle (4 iterations) apart: near convergence the 2 x 2
    normal equations of the extrapolation are nearly singular (the two
    difference vectors are almost parallel), so the summation order of their
    terms moves the extrapolated iterate at the 1e-8 level (here 1.8e-8 on the
    GPU against 1.6e-12 in the oracle after the first extrapolation), which
    can shift the step at which the change falls below 1e-8 by one cycle."""
    c = W.single_two_level()
    plan = pprt.Plan(gpu_ctx, c.nd, c.na, c.nf, precision=pprt.FP64)
    plan.set_operator(pprt.LSTAR_TRI, ng)
    db = pprt.upload_two_level(c, pprt.FP64)
    db.S.copy_(db.B)
    iters = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    rep = plan.two_level_ali(db.tau, db.q, db.S, db.eps, db.B, db.wphi, tol=1e-8,
                             max_iter=2000, iters_per_sync=10, iters=iters)
    ref = ali.two_level_ali_nonlocal(c.tau, c.q, c.phi, c.wnu, float(c.eps[0]), c.B, plan.mu, plan.w,
                                     tol=1e-8, operator="tri", ng=ng)
    e = rel_err(db.S.cpu().numpy(), ref["S"])
    print(f"  tri ng={ng}: gpu {rep} oracle iterations {ref['iterations']}, S err {e:.2e}", flush=True)
    assert rep["n_converged"] == 1
    if ng:
        assert abs(int(iters.item()) - ref["iterations"]) <= 4
    else:
        assert int(iters.item()) == ref["iterations"]
    assert e < 1e-10


def test_nonlocal_fp32_batch_converges(gpu_ctx):
    batch, db = _small_batch(pprt.FP32, nb=3, nf=128, na=8, seed=21)
    plan = pprt.Plan(gpu_ctx, batch.nd, batch.na, batch.nf, precision=pprt.FP32)
    plan.set_operator(pprt.LSTAR_TRI, True)
    db.S.copy_(db.B)
    iters = torch.zeros(plan.nb, dtype=torch.int32, device="cuda:0")
    rep = plan.two_level_ali(db.tau, db.q, db.S, db.eps, db.B, db.wphi, tol=1e-6,
                             max_iter=5000, iters_per_sync=20, iters=iters)
    assert rep["n_converged"] == plan.nb
    off = batch.off
    for b in range(batch.nb):
        s = slice(off[b], off[b + 1])
        ref = ali.two_level_ali_nonlocal(batch.tau[s], batch.q[s], batch.phi, batch.wnu,
                                         float(batch.eps[b]), batch.B[s], plan.mu, plan.w,
                                         tol=1e-6, operator="tri", ng=True)
        e = rel_err(db.S[s].cpu().numpy(), ref["S"])
        print(f"  b={b} eps={batch.eps[b]:.1e} it gpu={int(iters[b])} oracle={ref['iterations']} S {e:.2e}",
              flush=True)
        assert abs(int(iters[b]) - ref["iterations"]) <= 3
        assert e < 1e-5


def test_nonlocal_graph_replay_equals_eager(gpu_ctx):
    batch, db = _small_batch(pprt.FP64, nb=3, nf=64, seed=4)
    plan = pprt.Plan(gpu_ctx, batch.nd, batch.na, batch.nf, precision=pprt.FP64)
    plan.set_operator(pprt.LSTAR_TRI, True)
    res = {}
    for graph in (False, True):
        db.S.copy_(db.B)
        iters = torch.zeros(plan.nb, dtype=torch.int32, device="cuda:0")
        rep = plan.two_level_ali(db.tau, db.q, db.S, db.eps, db.B, db.wphi, tol=1e-10,
                                 max_iter=400, iters_per_sync=6, use_graph=graph, iters=iters)
        res[graph] = (db.S.clone(), iters.clone(), rep)
    assert torch.equal(res[True][0], res[False][0])
    assert torch.equal(res[True][1], res[False][1])


def test_ng_schedule_on_a_thick_small_eps_atmosphere(gpu_ctx):
    """The oracle's pin atmosphere for the Ng schedule (nd 151, eps 1.3e-6,
    nf 21, na 4), where Ng applied from the first iterates stalls: the FP64
    GPU iteration with the tri-diagonal operator and Ng converges to the
    oracle's fixed point within one Ng cycle of its iteration count."""
    b = W.two_level_batch(nb=4, nd_lo=150, nd_hi=230, na=4, nf=21, eps_lo=1e-6, eps_hi=1e-4, seed=5)
    a = b.atmosphere(2)
    plan = pprt.Plan(gpu_ctx, a.nd, a.na, a.nf, precision=pprt.FP64)
    plan.set_operator(pprt.LSTAR_TRI, True)
    db = pprt.upload_two_level(a, pprt.FP64)
    db.S.copy_(db.B)
    iters = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    rep = plan.two_level_ali(db.tau, db.q, db.S, db.eps, db.B, db.wphi, tol=1e-10,
                             max_iter=1000, iters_per_sync=10, iters=iters)
    ref = ali.two_level_ali_nonlocal(a.tau, a.q, a.phi, a.wnu, float(a.eps[0]), a.B, plan.mu, plan.w,
                                     tol=1e-10, operator="tri", ng=True, max_iter=1000)
    e = rel_err(db.S.cpu().numpy(), ref["S"])
    print(f"  gpu {rep}, oracle {ref['iterations']}, S err {e:.2e}", flush=True)
    assert rep["n_converged"] == 1 and ref["converged"]
    assert abs(int(iters.item()) - ref["iterations"]) <= 4
    assert e < 1e-9

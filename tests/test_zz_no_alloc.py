"""The allocation-free two-level step (pprt_two_level_ali_step_noalloc)
against the workspace step (pprt_two_level_ali_step) through the C ABI: the
same kernels on the same inputs, so S and the maximum relative change must
agree bit for bit; two calls in a row, the second on a smaller batch (the
static scratch keeps the first call's contents)."""
import numpy as np
import pytest
import torch

from paper_0903_1949_amd import pprt
from paper_0903_1949_amd import workloads as W

pytestmark = pytest.mark.gpu


def _step_pair(ctx, batch, prec, tri):
    plan = pprt.Plan(ctx, batch.nd, batch.na, batch.nf, precision=prec)
    if tri:
        plan.set_operator(pprt.LSTAR_TRI, False)
    db_ws = pprt.upload_two_level(batch, prec)
    db_na = pprt.upload_two_level(batch, prec)
    m_ws = torch.zeros(batch.nb, dtype=torch.float64, device="cuda:0")
    m_na = torch.full((batch.nb,), -1.0, dtype=torch.float64, device="cuda:0")
    plan.two_level_ali_step(db_ws.tau, db_ws.q, db_ws.S, db_ws.eps, db_ws.B, db_ws.wphi, m_ws)
    plan.two_level_ali_step_noalloc(db_na.tau, db_na.q, db_na.S, db_na.eps, db_na.B, db_na.wphi, m_na)
    torch.cuda.synchronize()
    return db_ws.S, db_na.S, m_ws, m_na, plan


@pytest.mark.parametrize("prec", [pprt.FP32, pprt.FP64])
@pytest.mark.parametrize("tri", [False, True])
def test_noalloc_step_equals_workspace_step(gpu_ctx, prec, tri):
    big = W.two_level_batch(nb=40, nd_lo=48, nd_hi=256, na=8, nf=512, seed=31)
    small = W.two_level_batch(nb=3, nd_lo=10, nd_hi=30, na=8, nf=100, seed=32)
    for batch in (big, small):
        print(f"[case] noalloc nb={batch.nb} nf={batch.nf} prec={prec} tri={tri}", flush=True)
        S_ws, S_na, m_ws, m_na, _ = _step_pair(gpu_ctx, batch, prec, tri)
        assert torch.equal(S_na, S_ws)
        assert torch.equal(m_na, m_ws)


def test_noalloc_refusals(gpu_ctx):
    batch = W.two_level_batch(nb=2, nd_lo=10, nd_hi=20, na=4, nf=64, seed=33)
    plan = pprt.Plan(gpu_ctx, batch.nd, batch.na, batch.nf, precision=pprt.FP64)
    plan.set_operator(pprt.LSTAR_DIAG, True)
    db = pprt.upload_two_level(batch, pprt.FP64)
    mx = torch.zeros(batch.nb, dtype=torch.float64, device="cuda:0")
    with pytest.raises(pprt.PprtError, match="E_UNSUPPORTED"):
        plan.two_level_ali_step_noalloc(db.tau, db.q, db.S, db.eps, db.B, db.wphi, mx)
    # a batch whose partials exceed the static scratch: refused before any
    # launch, so the (uninitialised) inputs are never read
    nd = np.full(600, 256, dtype=np.int32)
    plan = pprt.Plan(gpu_ctx, nd, 8, 1024, precision=pprt.FP64)
    assert plan.workspace_bytes > (64 << 20)
    rows, dev = int(nd.sum()), "cuda:0"
    e = lambda *shape: torch.empty(shape, dtype=torch.float64, device=dev)
    with pytest.raises(pprt.PprtError, match="E_WORKSPACE"):
        plan.two_level_ali_step_noalloc(e(rows), e(rows, 1024), e(rows), e(600), e(rows), e(1024), e(600))

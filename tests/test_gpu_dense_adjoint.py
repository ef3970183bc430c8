"""The hand-written adjoint of the emergent intensity with in-layer scattering
(pprt_formal_solution_scattering_vjp) against the FP64 oracle and against
properties that hold at any size.

* dL/dq, dL/dS^g and the lower-boundary derivatives against central
  differences of the oracle (its matrix-exponential + doubling route, one
  frequency column at a time) for a seeded loss L = sum g Iemerg.  The
  oracle's emergent intensity carries about 1e-11 of relative roughness
  (the discrete choices of its scaling-and-squaring), so the differences take
  a relative step of 1e-4 (truncation about 1e-8; measured agreement 6e-8 in
  a CPU prototype of the same adjoint); bar 1e-6.
* The emergent intensity is linear in S^g: <dL/dS^g, dS> must equal
  L(S^g + dS) - L(S^g) from the library's own forward to rounding, on a batch
  slice of realistic size.
* torch.autograd.gradcheck through the autograd binding."""
import numpy as np
import pytest
import torch

from oracle import dense
from paper_0903_1949_amd import autograd as AG
from paper_0903_1949_amd import pprt
from paper_0903_1949_amd import workloads as W
from tests.test_gpu_dense import _case

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def _oracle_col(c, b, off, k, mu, w, bc, q=None, S=None, Bb=None, Bp=None, Ib=None):
    """The oracle's emergent intensity of atmosphere b at frequency k."""
    s = slice(off[b], off[b + 1])
    qq = (c["q"][s, k] if q is None else q)[:, None]
    SS = (c["S"][s, k] if S is None else S)[:, None]
    kw = dict(lower="diffusion", Bbot=np.array([c["Bb"][b, k] if Bb is None else Bb]),
              Bbot_prev=np.array([c["Bp"][b, k] if Bp is None else Bp])) if bc == pprt.BC_DIFFUSION \
        else dict(lower="given", Ibot=(c["Ibot"][b, k] if Ib is None else Ib)[None, :])
    return dense.formal_solution_dense(c["tau"][s], qq, SS, mu, w, omega=c["om"][s, k][:, None],
                                       Itop=c["Itop"][b, k][None, :], **kw)["Iemerg"][0]


def _vjp(ctx, nds, na, nf, c, gI, bc):
    plan = pprt.Plan(ctx, nds, na, nf, precision=pprt.FP64, lower_bc=bc, outputs=pprt.OUT_IEMERG)
    g = plan.formal_solution_scattering_vjp(
        _dev(c["tau"]), _dev(c["q"]), _dev(c["S"]), _dev(c["om"]), _dev(gI), Bbot=_dev(c["Bb"]),
        Bbot_prev=_dev(c["Bp"]), Itop=_dev(c["Itop"]), Ibot=None if c["Ibot"] is None else _dev(c["Ibot"]))
    torch.cuda.synchronize()
    return plan, {k: v.cpu().numpy() for k, v in g.items() if not k.startswith("_")}


@pytest.mark.parametrize("nds,nf,na,bc", [
    ([6], 2, 1, pprt.BC_DIFFUSION), ([5, 4], 2, 2, pprt.BC_DIFFUSION), ([7, 3], 3, 4, pprt.BC_DIFFUSION),
    ([6, 5], 2, 8, pprt.BC_DIFFUSION), ([5], 2, 16, pprt.BC_DIFFUSION), ([6, 4], 2, 4, pprt.BC_GIVEN),
])
def test_scattering_vjp_against_oracle_differences(gpu_ctx, nds, nf, na, bc):
    seed = sum(nds) * 11 + nf + na + bc
    print(f"[case] scattering vjp nds={nds} nf={nf} na={na} bc={bc} seed={seed}", flush=True)
    c = _case(nds, nf, na, seed, bc=bc)
    rng = np.random.default_rng(seed)
    gI = rng.uniform(-1.0, 1.0, size=(len(nds), nf, na))
    plan, g = _vjp(gpu_ctx, nds, na, nf, c, gI, bc)
    mu, w = plan.mu, plan.w
    off = np.concatenate([[0], np.cumsum(nds)])
    fq, fS = np.zeros_like(g["dq"]), np.zeros_like(g["dSg"])
    fB, fBp = np.zeros((len(nds), nf)), np.zeros((len(nds), nf))
    fIb = np.zeros((len(nds), nf, na))
    for b in range(len(nds)):
        s = slice(off[b], off[b + 1])
        for k in range(nf):
            L = lambda **kw: float(gI[b, k] @ _oracle_col(c, b, off, k, mu, w, bc, **kw))
            q0, S0 = c["q"][s, k].copy(), c["S"][s, k].copy()
            for d in range(nds[b]):
                h = 1e-4 * q0[d]
                qp, qm = q0.copy(), q0.copy()
                qp[d] += h; qm[d] -= h
                fq[off[b] + d, k] = (L(q=qp) - L(q=qm)) / (2 * h)
                h = 1e-4 * max(abs(S0[d]), 1e-3)
                Sp, Sm = S0.copy(), S0.copy()
                Sp[d] += h; Sm[d] -= h
                fS[off[b] + d, k] = (L(S=Sp) - L(S=Sm)) / (2 * h)
            if bc == pprt.BC_DIFFUSION:
                Bb, Bp = c["Bb"][b, k], c["Bp"][b, k]
                fB[b, k] = (L(Bb=Bb + 1e-4 * Bb) - L(Bb=Bb - 1e-4 * Bb)) / (2e-4 * Bb)
                fBp[b, k] = (L(Bp=Bp + 1e-4 * Bp) - L(Bp=Bp - 1e-4 * Bp)) / (2e-4 * Bp)
            else:
                for i in range(na):
                    Ib = c["Ibot"][b, k].copy()
                    h = 1e-4 * abs(Ib[i])
                    Ip_, Im_ = Ib.copy(), Ib.copy()
                    Ip_[i] += h; Im_[i] -= h
                    fIb[b, k, i] = (L(Ib=Ip_) - L(Ib=Im_)) / (2 * h)

    def err(a, r, scale=None):
        return float(np.max(np.abs(a - r)) / (np.max(np.abs(r)) if scale is None else scale))

    # the boundary derivatives are on the footing of dL/dS^g at the bottom
    # node and vanish through a thick slab: they are held against the scale
    # of the source gradient (the differences' noise is about 5e-8 of L)
    sc = float(np.max(np.abs(fS)))
    errs = {"dq": err(g["dq"], fq), "dSg": err(g["dSg"], fS)}
    if bc == pprt.BC_DIFFUSION:
        errs["dBbot"] = err(g["dBbot"], fB, sc)
        errs["dBbot_prev"] = err(g["dBbot_prev"], fBp, sc)
    else:
        errs["dIbot"] = err(g["dIbot"], fIb, sc)
    print("  errors:", {k: f"{v:.1e}" for k, v in errs.items()}, flush=True)
    for k, e in errs.items():
        assert e < 1e-6, (k, e)


@pytest.mark.parametrize("bc", [pprt.BC_DIFFUSION, pprt.BC_GIVEN])
def test_scattering_vjp_boundary_derivatives_of_a_thin_slab(gpu_ctx, bc):
    """A slab of total optical depth 2 (albedo 0.5..0.9), where the lower
    boundary reaches the top: dL/dBbot, dL/dBbot_prev or dL/dIbot against
    the oracle's differences, relative to their own size."""
    nds, nf, na = [6], 2, 4
    print(f"[case] scattering vjp thin slab bc={bc}", flush=True)
    rng = np.random.default_rng(17 + bc)
    nd = nds[0]
    c = dict(tau=np.linspace(0.0, 2.0, nd) + 1e-6, q=rng.uniform(0.5, 1.5, size=(nd, nf)),
             S=rng.uniform(0.5, 1.5, size=(nd, nf)), om=rng.uniform(0.5, 0.9, size=(nd, nf)),
             Bb=rng.uniform(0.8, 1.2, size=(1, nf)), Bp=rng.uniform(0.6, 0.9, size=(1, nf)),
             Itop=rng.uniform(0.0, 0.3, size=(1, nf, na)),
             Ibot=rng.uniform(0.5, 1.5, size=(1, nf, na)) if bc == pprt.BC_GIVEN else None)
    gI = rng.uniform(-1.0, 1.0, size=(1, nf, na))
    plan, g = _vjp(gpu_ctx, nds, na, nf, c, gI, bc)
    off = np.array([0, nd])
    errs = {}
    for k in range(nf):
        L = lambda **kw: float(gI[0, k] @ _oracle_col(c, 0, off, k, plan.mu, plan.w, bc, **kw))
        if bc == pprt.BC_DIFFUSION:
            Bb, Bp = c["Bb"][0, k], c["Bp"][0, k]
            fB = (L(Bb=Bb * (1 + 1e-4)) - L(Bb=Bb * (1 - 1e-4))) / (2e-4 * Bb)
            fBp = (L(Bp=Bp * (1 + 1e-4)) - L(Bp=Bp * (1 - 1e-4))) / (2e-4 * Bp)
            errs[f"dBbot[{k}]"] = abs(g["dBbot"][0, k] - fB) / abs(fB)
            errs[f"dBbot_prev[{k}]"] = abs(g["dBbot_prev"][0, k] - fBp) / abs(fBp)
        else:
            fI = np.zeros(na)
            for i in range(na):
                Ib = c["Ibot"][0, k].copy()
                h = 1e-4 * Ib[i]
                Ip_, Im_ = Ib.copy(), Ib.copy()
                Ip_[i] += h; Im_[i] -= h
                fI[i] = (L(Ib=Ip_) - L(Ib=Im_)) / (2 * h)
            errs[f"dIbot[{k}]"] = float(np.max(np.abs(g["dIbot"][0, k] - fI)) / np.max(np.abs(fI)))
    print("  errors:", {k: f"{v:.1e}" for k, v in errs.items()}, flush=True)
    for k, e in errs.items():
        assert e < 1e-6, (k, e)


def test_scattering_vjp_source_derivative_is_exact_on_a_batch_slice(gpu_ctx):
    """Three atmospheres of the batch with the grey scattering continuum (nd
    60..120, 64 frequencies, 8 angles): the emergent intensity is linear in
    S^g, so <dL/dS^g, dS> equals the change of L under S^g + dS from the
    forward call to rounding; and the q-gradient matches a central difference
    of the forward call along a random direction."""
    full = W.two_level_batch(nb=3, nd_lo=60, nd_hi=120, nf=64, seed=33, cont_ratio=1e-3, eps_c=1e-4)
    Sg = full.pfrac * full.S_trial[:, None] + full.sg_const
    last = full.off[1:] - 1
    nds, nf, na = [int(x) for x in full.nd], full.nf, full.na
    print(f"[case] scattering vjp batch slice nds={nds} nf={nf} na={na}", flush=True)
    Bb = np.repeat(full.B[last][:, None], nf, 1)
    Bp = np.repeat(full.B[last - 1][:, None], nf, 1)
    rng = np.random.default_rng(7)
    gI = rng.uniform(-1.0, 1.0, size=(full.nb, nf, na))
    plan = pprt.Plan(gpu_ctx, nds, na, nf, precision=pprt.FP64, outputs=pprt.OUT_IEMERG)
    args = lambda q, S: (_dev(full.tau), _dev(q), _dev(S), _dev(full.omega))
    kw = dict(Bbot=_dev(Bb), Bbot_prev=_dev(Bp))
    g = plan.formal_solution_scattering_vjp(*args(full.q, Sg), _dev(gI), **kw)

    def L(q, S):
        out = plan.formal_solution_scattering(*args(q, S), **kw)
        return float((out["Iemerg"] * _dev(gI)).sum())

    dS = rng.uniform(-1.0, 1.0, size=Sg.shape) * 1e-3 * np.abs(Sg)
    lin = float((g["dSg"] * _dev(dS)).sum())
    dL = L(full.q, Sg + dS) - L(full.q, Sg)
    e_S = abs(lin - dL) / abs(dL)
    dqd = rng.uniform(-1.0, 1.0, size=full.q.shape) * full.q
    h = 1e-6
    lin_q = float((g["dq"] * _dev(dqd)).sum())
    fd_q = (L(full.q + h * dqd, Sg) - L(full.q - h * dqd, Sg)) / (2 * h)
    e_q = abs(lin_q - fd_q) / abs(fd_q)
    print(f"  source direction: {e_S:.1e}; opacity direction: {e_q:.1e}", flush=True)
    assert e_S < 1e-9
    assert e_q < 1e-6


def test_scattering_vjp_autograd_gradcheck(gpu_ctx):
    nds, nf, na = [5, 4], 2, 4
    c = _case(nds, nf, na, 3)
    plan = pprt.Plan(gpu_ctx, nds, na, nf, precision=pprt.FP64, outputs=pprt.OUT_IEMERG)
    q = _dev(c["q"]).requires_grad_(True)
    S = _dev(c["S"]).requires_grad_(True)
    Bb = _dev(c["Bb"]).requires_grad_(True)
    Bp = _dev(c["Bp"]).requires_grad_(True)
    fn = lambda q_, S_, Bb_, Bp_: AG.emergent_intensity_scattering(plan, _dev(c["tau"]), q_, S_, _dev(c["om"]),
                                                                   Bbot=Bb_, Bbot_prev=Bp_, Itop=_dev(c["Itop"]))
    assert torch.autograd.gradcheck(fn, (q, S, Bb, Bp), eps=1e-6, atol=1e-8, rtol=1e-5)


def test_scattering_vjp_refuses_unsupported_plans(gpu_ctx):
    z = torch.zeros((4, 2), dtype=torch.float32, device="cuda:0")
    plan = pprt.Plan(gpu_ctx, [4], 4, 2, precision=pprt.FP32, outputs=pprt.OUT_IEMERG)
    with pytest.raises(pprt.PprtError, match="E_UNSUPPORTED"):
        plan.formal_solution_scattering_vjp(_dev(np.logspace(-2, 1, 4)), z + 1, z, z,
                                            torch.zeros((1, 2, 4), dtype=torch.float32, device="cuda:0"),
                                            Bbot=z[:1], Bbot_prev=z[:1])
    z = torch.zeros((4, 2), dtype=torch.float64, device="cuda:0")
    plan = pprt.Plan(gpu_ctx, [4], 32, 2, precision=pprt.FP64, outputs=pprt.OUT_IEMERG)
    with pytest.raises(pprt.PprtError, match="E_UNSUPPORTED"):
        plan.formal_solution_scattering_vjp(_dev(np.logspace(-2, 1, 4)), z + 1, z, z,
                                            torch.zeros((1, 2, 32), dtype=torch.float64, device="cuda:0"),
                                            Bbot=z[:1], Bbot_prev=z[:1])

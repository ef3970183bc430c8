"""Oracle parity at the sizes the bench times, in the launch shapes it uses:
the headline step (512 two-level atmospheres, nd 48..256, na 8, nf 1024;
the batched sweep in its autotuned shape) in FP32 and FP64, the same batch
with a scattering continuum (the dense FP64 path, one launch over the whole
batch), and one multilevel iteration of the 6+1-level atom (15 lines, 5
continua, nd 128, na 8, nf 2000) stage by stage.  Sampled atmospheres are
checked against the oracle one by one; the multilevel populations against a
per-row bound from the componentwise (Skeel) condition of the scaled rate
system.  Every error is printed."""
import numpy as np
import pytest
import torch

from oracle import ali, dense, formal, rates
from paper_0903_1949_amd import pprt
from paper_0903_1949_amd import workloads as W
from tests.conftest import U64, rate_magnitudes, rel_err, skeel

pytestmark = pytest.mark.gpu

def r32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


@pytest.fixture(scope="module")
def c3a():
    return W.two_level_batch(seed=3)


def _pick(batch):
    """Eight atmospheres: the three smallest and three largest eps, the
    shortest and the longest."""
    o = np.argsort(batch.eps)
    idx = list(o[:3]) + list(o[-3:]) + [int(np.argmin(batch.nd)), int(np.argmax(batch.nd))]
    return sorted(set(int(i) for i in idx))


@pytest.mark.parametrize("prec", [pprt.FP32, pprt.FP64])
def test_c3a_step_full_batch(gpu_ctx, c3a, prec):
    batch = c3a
    print(f"[case] c3a full batch, one ALI step, prec={prec}", flush=True)
    plan = pprt.Plan(gpu_ctx, batch.nd, batch.na, batch.nf, precision=prec)
    db = pprt.upload_two_level(batch, prec)
    if prec == pprt.FP32:
        plan.autotune(db.tau, db.q, db.S, db.eps, db.B, db.wphi, force=True)
    S0 = batch.S_trial.copy()
    mx = torch.zeros(batch.nb, dtype=torch.float64, device="cuda:0")
    plan.two_level_ali_step(db.tau, db.q, db.S, db.eps, db.B, db.wphi, mx)
    torch.cuda.synchronize()
    S_gpu = db.S.cpu().numpy()
    mx_gpu = mx.cpu().numpy()
    off = batch.off
    # the oracle on exactly the inputs the kernel sees (FP32 q and weights)
    q = r32(batch.q) if prec == pprt.FP32 else batch.q
    wp = r32(batch.wnu * batch.phi) if prec == pprt.FP32 else batch.wnu * batch.phi
    worst = {"S": 0.0, "dS": 0.0, "max_rel": 0.0}
    for b in _pick(batch):
        s = slice(off[b], off[b + 1])
        out = formal.formal_solution(batch.tau[s], q[s], S0[s], plan.mu, plan.w, lower="diffusion",
                                     Bbot=np.full(batch.nf, batch.B[s][-1]),
                                     Bbot_prev=np.full(batch.nf, batch.B[s][-2]))
        jms = out["JmS"] @ wp
        olb = out["lstar_c"] @ wp
        S_ref, m_ref = ali.batch_two_level_update(batch.nd[b:b + 1], S0[s], batch.B[s],
                                                  batch.eps[b:b + 1], jms, olb)
        e = {"S": rel_err(S_gpu[s], S_ref), "dS": rel_err(S_gpu[s] - S0[s], S_ref - S0[s]),
             "max_rel": abs(mx_gpu[b] / m_ref[0] - 1)}
        print(f"  b={b} nd={batch.nd[b]} eps={batch.eps[b]:.1e}: " +
              " ".join(f"{k} {v:.2e}" for k, v in e.items()), flush=True)
        for k in worst:
            worst[k] = max(worst[k], e[k])
    print("  worst", {k: f"{v:.2e}" for k, v in worst.items()}, flush=True)
    if prec == pprt.FP32:
        assert worst["S"] < 1e-5
        assert worst["dS"] < 1e-4 and worst["max_rel"] < 1e-4
    else:
        assert worst["S"] < 1e-10 and worst["dS"] < 1e-10 and worst["max_rel"] < 1e-10


def test_c3b_step_full_batch(gpu_ctx):
    """The headline batch with the grey coherent continuum (r_c 1e-3,
    eps_c 1e-4): one continuum step of all 512 atmospheres through the dense
    FP64 path (about 100 GB of workspace), the two deepest atmospheres
    against the oracle's dense formal solution."""
    batch = W.two_level_batch(seed=3, cont_ratio=1e-3, eps_c=1e-4)
    print("[case] c3b full batch, one continuum step (FP64)", flush=True)
    plan = pprt.Plan(gpu_ctx, batch.nd, batch.na, batch.nf, precision=pprt.FP64)
    db = pprt.upload_two_level(batch, pprt.FP64)
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")
    pf, sc, om = d(batch.pfrac), d(batch.sg_const), d(batch.omega)
    S0 = batch.S_trial.copy()
    mx = torch.zeros(batch.nb, dtype=torch.float64, device="cuda:0")
    plan.two_level_ali_step_continuum(db.tau, db.q, db.S, db.eps, db.B, db.wphi, pf, sc, om,
                                      db.Bbot, db.Bbot_prev, mx)
    torch.cuda.synchronize()
    S_gpu = db.S.cpu().numpy()
    plan._cws = None
    del pf, sc, om
    torch.cuda.empty_cache()
    off = batch.off
    for b in [int(i) for i in np.argsort(-batch.nd, kind="stable")[:2]]:
        s = slice(off[b], off[b + 1])
        r = ali.two_level_ali(batch.tau[s], batch.q[s], batch.phi, batch.wnu, float(batch.eps[b]),
                              batch.B[s], plan.mu, plan.w, tol=1e-300, max_iter=1, S0=S0[s],
                              pfrac=batch.pfrac[s], sg_const=batch.sg_const[s],
                              fs=dense.formal_solution_dense, fs_kwargs={"omega": batch.omega[s]})
        e = rel_err(S_gpu[s], r["S"])
        e_d = rel_err(S_gpu[s] - S0[s], r["S"] - S0[s])
        print(f"  b={b} nd={batch.nd[b]} eps={batch.eps[b]:.1e}: S {e:.2e} dS {e_d:.2e}", flush=True)
        assert e < 1e-10 and e_d < 1e-10


@pytest.fixture(scope="module")
def c2():
    return W.multilevel_atom()


def test_c2_multilevel_iteration_full_config(gpu_ctx, c2):
    a = c2
    print(f"[case] c2 full configuration: {a.name}", flush=True)
    assert (a.nl, a.nt, int(a.nd[0]), a.na, a.nf) == (7, 20, 128, 8, 2000)
    plan = pprt.Plan(gpu_ctx, a.nd, a.na, a.nf, precision=pprt.FP64, outputs=pprt.OUT_J | pprt.OUT_LSTAR)
    da = pprt.DeviceAtom(a)
    d = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda:0")
    pops0 = a.nstar.copy()
    # stage 1: opacities
    q, om, Sg = plan.nlte_opacity(da, d(pops0))
    o_ref = rates.opacities(a, pops0)
    e_op = {k: rel_err(v.cpu().numpy(), o_ref[k]) for k, v in (("q", q), ("omega", om), ("Sg", Sg))}
    # stage 2: the dense formal solution on the oracle's opacities
    Bb = d(a.Bnu[-1][None, :]); Bp = d(a.Bnu[-2][None, :])
    fs = plan.formal_solution_scattering(da.tau, d(o_ref["q"]), d(o_ref["Sg"]), d(o_ref["omega"]),
                                         Bbot=Bb, Bbot_prev=Bp)
    torch.cuda.synchronize()
    fs_ref = dense.formal_solution_dense(a.tau, o_ref["q"], o_ref["Sg"], plan.mu, plan.w,
                                         omega=o_ref["omega"], lower="diffusion", Bbot=a.Bnu[-1],
                                         Bbot_prev=a.Bnu[-2])
    e_fs = {k: rel_err(fs[k].cpu().numpy(), fs_ref[k]) for k in ("J", "lstar")}
    del fs
    torch.cuda.empty_cache()
    # stage 3: rates from the oracle's J and Lambda*
    dR = plan.rates_assemble(da, d(pops0), d(fs_ref["J"]), d(fs_ref["lstar"]))
    r_ref = rates.preconditioned_rates(a, pops0, fs_ref["J"], fs_ref["lstar"])
    e_rt = [rel_err(g.cpu().numpy(), r) for g, r in zip(dR, r_ref)]
    # [dR] are sums of W sigma (J - Lambda* eta/kappa) over a window, whose
    # terms cancel where J is close to Lambda* S: their rounding is set by
    # the magnitude of the terms, sum W sigma (|J| + |Lambda* eta/kappa|)
    # (with G for [dR_ul], and sum W U (1 + p Lambda*) for [R*_ul])
    mag = rate_magnitudes(a, pops0, fs_ref["J"], fs_ref["lstar"])
    e_rt_mag = [float(np.max(np.abs(g.cpu().numpy() - r) / m)) for g, r, m in zip(dR, r_ref, mag)]
    # stage 4: the solve from the oracle's rates, bound per row by the condition
    pn, _ = plan.rates_solve(da, d(pops0), *[d(r) for r in r_ref])
    torch.cuda.synchronize()
    p_gpu = pn.cpu().numpy()
    rows = a.tau.shape[0]
    worst_ratio, worst_solve = 0.0, 0.0
    for r in range(rows):
        A, rhs = rates.rate_matrix(a, r, *r_ref)
        As = A * pops0[r][None, :]
        x_ref = np.linalg.solve(As, rhs)
        x = p_gpu[r] / pops0[r]
        err = np.abs(x - x_ref) / np.abs(x_ref)
        bound = 8.0 * a.nl * U64 * skeel(As, x_ref)
        worst_ratio = max(worst_ratio, float(np.max(err / bound)))
        worst_solve = max(worst_solve, float(np.max(err)))
    print(f"  opacity {e_op}", flush=True)
    print(f"  formal solution J {e_fs['J']:.2e} lstar {e_fs['lstar']:.2e}", flush=True)
    print(f"  rates (per array) {[f'{e:.2e}' for e in e_rt]}, relative to the magnitude of their "
          f"terms {[f'{e:.2e}' for e in e_rt_mag]}", flush=True)
    print(f"  solve: worst rel err {worst_solve:.2e}, worst err / (8 n u Skeel) {worst_ratio:.2e}",
          flush=True)
    assert max(e_op.values()) < 1e-13
    assert max(e_fs.values()) < 1e-10
    assert max(e_rt_mag) < 1e-13
    assert worst_ratio < 1.0
    # one whole iteration (nlte_step) against the oracle's iteration: the
    # rates differ by the formal-solution rounding (delta), so each row's
    # populations may differ by (delta + 8 n u) times its condition
    pops = d(pops0)
    mx = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    plan.nlte_step(da.tau, da, pops, mx)
    torch.cuda.synchronize()
    # the oracle's iteration from the same populations is the solve of the
    # rates above (opacities, dense formal solution, rates, solve)
    p_ref = rates.solve_populations(a, *r_ref, scale=pops0)
    m_ref = [float(np.max(np.abs(p_ref - pops0) / np.abs(p_ref)))]
    got = pops.cpu().numpy()
    # the GPU's rates differ from these by at most (e_fs + e_rt_mag) of the
    # magnitude of their terms: per row, relative to the rate-matrix entries
    # (collision rates included) that is delta_r
    eps_rate = max(e_fs.values()) + max(e_rt_mag)
    P_lu = r_ref[0] + a.Clu
    P_ul = r_ref[2] + r_ref[1] + a.Cul
    rel_lu = mag[0] / np.abs(P_lu)
    rel_ul = (mag[1] + mag[2]) / np.abs(P_ul)
    delta_row = eps_rate * np.maximum(rel_lu, rel_ul).max(axis=1)
    delta = float(delta_row.max())
    worst_step, worst_step_ratio = 0.0, 0.0
    for r in range(rows):
        A, rhs = rates.rate_matrix(a, r, *r_ref)
        As = A * pops0[r][None, :]
        x_ref = p_ref[r] / pops0[r]
        err = np.abs(got[r] / pops0[r] - x_ref) / np.abs(x_ref)
        bound = (delta_row[r] + 8.0 * a.nl * U64) * skeel(As, x_ref)
        worst_step = max(worst_step, float(np.max(err)))
        worst_step_ratio = max(worst_step_ratio, float(np.max(err / bound)))
    print(f"  step: populations worst rel err {worst_step:.2e}, err / bound {worst_step_ratio:.2e} "
          f"(delta {delta:.1e}); max_rel {float(mx.item()):.6e} vs {m_ref[0]:.6e}", flush=True)
    assert worst_step_ratio < 1.0
    assert abs(float(mx.item()) / m_ref[0] - 1) < 1e-6

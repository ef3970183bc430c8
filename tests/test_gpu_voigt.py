"""GPU Voigt profiles: the device Voigt function (Weideman's expansion)
against the Faddeeva function, and the multilevel path with depth-dependent
line profiles evaluated on the device (opacity assembly, rate assembly, one
full iteration, convergence) against the FP64 oracle."""
import numpy as np
import pytest
import torch
from scipy.special import wofz

from oracle import rates
from paper_0903_1949_amd import pprt
from paper_0903_1949_amd import workloads as W
from tests.conftest import population_error_ratio, rel_err

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


@pytest.mark.parametrize("a", [0.0, 1e-4, 1e-3, 1e-2, 1e-1, 1.0, 10.0])
def test_voigt_function(gpu_ctx, a):
    x = np.concatenate([np.linspace(-200.0, 200.0, 40001), np.geomspace(1e-6, 1e4, 2001)])
    H = gpu_ctx.voigt(_dev(np.full_like(x, a)), _dev(x))
    torch.cuda.synchronize()
    ref = np.real(wofz(x + 1j * a))
    got = H.cpu().numpy()
    e = rel_err(got, ref)
    pos = ref > 0
    e_rel = float(np.max(np.abs(got[pos] - ref[pos]) / ref[pos]))
    print(f"  a={a}: per-array {e:.2e}, pointwise relative {e_rel:.2e}", flush=True)
    assert e < 1e-10
    if a >= 1e-4:
        assert e_rel < 1e-9


@pytest.fixture(scope="module")
def atom():
    return W.multilevel_atom(nbound=4, ncont=3, nd=20, na=8, nline_pts=16, ncont_pts=10, seed=7,
                             nb=2, depth_profiles=True)


def _plan(ctx, a):
    return pprt.Plan(ctx, a.nd, a.na, a.nf, precision=pprt.FP64, outputs=pprt.OUT_J | pprt.OUT_LSTAR)


def test_depth_profile_opacity_parity(gpu_ctx, atom):
    plan = _plan(gpu_ctx, atom)
    da = pprt.DeviceAtom(atom)
    pops = atom.nstar * np.random.default_rng(0).uniform(0.5, 2.0, size=atom.nstar.shape)
    q, om, Sg = plan.nlte_opacity(da, _dev(pops))
    torch.cuda.synchronize()
    ref = rates.opacities(atom, pops)
    for name, got in (("q", q), ("omega", om), ("Sg", Sg)):
        e = rel_err(got.cpu().numpy(), ref[name])
        print(f"  {name}: {e:.2e}", flush=True)
        assert e < 1e-10, name


def test_depth_profile_rate_assembly_parity(gpu_ctx, atom):
    plan = _plan(gpu_ctx, atom)
    da = pprt.DeviceAtom(atom)
    rng = np.random.default_rng(1)
    rows = atom.tau.shape[0]
    pops = atom.nstar * rng.uniform(0.5, 2.0, size=atom.nstar.shape)
    J = rng.uniform(0.1, 2.0, size=(rows, atom.nf)) * atom.Bnu
    L = rng.uniform(0.0, 1.0, size=(rows, atom.nf))
    d = plan.rates_assemble(da, _dev(pops), _dev(J), _dev(L))
    torch.cuda.synchronize()
    ref = rates.preconditioned_rates(atom, pops, J, L)
    for got, r in zip(d, ref):
        assert rel_err(got.cpu().numpy(), r) < 1e-10


def test_depth_profile_iterations_and_convergence(gpu_ctx):
    a = W.multilevel_atom(nbound=3, ncont=2, nd=16, na=4, nline_pts=10, ncont_pts=6, seed=11,
                          depth_profiles=True)
    plan = _plan(gpu_ctx, a)
    da = pprt.DeviceAtom(a)
    pops = da.nstar.clone()
    mx = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    for it in range(2):
        p_start = pops.cpu().numpy()
        plan.nlte_step(da.tau, da, pops, mx)
        torch.cuda.synchronize()
        p_ref, _, aux = rates.nlte_iteration(a, p_start, plan.mu, plan.w)
        got = pops.cpu().numpy()
        e = np.max(np.abs(got / p_ref - 1))
        # bound from the componentwise condition of each row's system
        ratio, _, bw_ratio = population_error_ratio(a, p_start, (aux["dRlu"], aux["dRul"], aux["Rsul"]),
                                                    got, 1e-10, aux["J"], aux["lstar"])
        print(f"  iteration {it + 1}: populations rel err {e:.2e}, err / condition bound {ratio:.2e}, "
              f"backward error / bound {bw_ratio:.2e}", flush=True)
        assert ratio < 1.0 and bw_ratio < 1.0
    it = 2
    for it in range(3, 401):
        plan.nlte_step(da.tau, da, pops, mx)
        if it % 20 == 0 and float(mx.item()) < 1e-9:
            break
    torch.cuda.synchronize()
    ref = rates.nlte_solve(a, plan.mu, plan.w, tol=1e-9, max_iter=400)
    e = np.max(np.abs(pops.cpu().numpy() / ref["pops"] - 1))
    print(f"  gpu iterations {it}, oracle {ref['iterations']}, rel err {e:.2e}", flush=True)
    assert ref["converged"] and e < 1e-8


def test_depth_profile_tables_must_come_together(gpu_ctx, atom):
    plan = _plan(gpu_ctx, atom)
    da = pprt.DeviceAtom(atom)
    da.struct.dopp = None
    with pytest.raises(pprt.PprtError):
        plan.nlte_opacity(da, _dev(atom.nstar))

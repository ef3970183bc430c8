"""The large angle-coupled case on the GPU: a 20-level hydrogen-like atom
with 100 lines and 4 continua, 512 depths, 32 angles per hemisphere (64 x 64
block layer operators, on the matrix cores) and 16384 frequencies.

* The scattering formal solution over the whole frequency grid, compared
  with the oracle at 64 seeded frequencies (line cores and wings of
  strong and weak lines, continua), all depths and angles; the same on an
  FP32 plan at 16 frequencies against the oracle on FP32-rounded inputs.
* Rate assembly and the 20-level statistical-equilibrium solve at full size
  on seeded radiation fields, against the oracle.
* One full multilevel iteration of the same atom on a reduced grid (10
  depths, 3 points per line), against the oracle's iteration."""
import numpy as np
import pytest
import torch

from oracle import dense, rates
from paper_0903_1949_amd import pprt
from paper_0903_1949_amd import workloads as W
from tests.conftest import population_error_ratio, rate_magnitudes, rel_err, rel_err_terms

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


@pytest.fixture(scope="module")
def c5():
    return W.c5_atom()


def _sample_frequencies(atom, n=64, seed=5):
    """Seeded frequencies: for lines picked at random, the core point and a
    wing point; plus points of two continua."""
    rng = np.random.default_rng(seed)
    lines = np.flatnonzero(atom.kind == 0)
    conts = np.flatnonzero(atom.kind == 1)
    ks = []
    for t in rng.choice(lines, size=(n - 2) // 2, replace=False):
        k0, k1 = int(atom.k0[t]), int(atom.k1[t])
        ks += [(k0 + k1) // 2, int(rng.integers(k0, k0 + (k1 - k0) // 4))]
    for t in rng.choice(conts, size=2, replace=False):
        ks.append(int(rng.integers(atom.k0[t], atom.k1[t])))
    return np.array(sorted(ks))


def _release_device_memory():
    """Return cached device memory before a workspace of a good part of the
    card is allocated (an FP64 plan on the full grid needs 230 GB)."""
    import gc
    gc.collect()
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info()
    print(f"  device memory: {free / 1e9:.1f} GB free of {total / 1e9:.1f} GB", flush=True)


def test_c5_formal_solution_full_grid_sampled(gpu_ctx, c5):
    a = c5
    rows, nf, na = a.tau.shape[0], a.nf, a.na
    print(f"[case] C5 formal solution rows={rows} nf={nf} na={na}", flush=True)
    _release_device_memory()
    op = rates.opacities(a, a.nstar)          # the inputs of both sides
    ks = _sample_frequencies(a)
    plan = pprt.Plan(gpu_ctx, a.nd, na, nf, precision=pprt.FP64,
                     outputs=pprt.OUT_J | pprt.OUT_JMS | pprt.OUT_LSTAR | pprt.OUT_H | pprt.OUT_IEMERG)
    Bb, Bp = _dev(a.Bnu[-1:, :]), _dev(a.Bnu[-2:-1, :])
    out = plan.formal_solution_scattering(_dev(a.tau), _dev(op["q"]), _dev(op["Sg"]), _dev(op["omega"]),
                                          Bbot=Bb, Bbot_prev=Bp)
    torch.cuda.synchronize()
    got = {k: out[k].cpu().numpy() for k in ("J", "JmS", "lstar", "H", "Iemerg")}
    del out
    torch.cuda.empty_cache()
    ref = dense.formal_solution_dense(a.tau, op["q"][:, ks], op["Sg"][:, ks], plan.mu, plan.w,
                                      omega=op["omega"][:, ks], lower="diffusion", Bbot=a.Bnu[-1, ks],
                                      Bbot_prev=a.Bnu[-2, ks])
    errs = {k: rel_err(got[k][:, ks], ref[k]) for k in ("J", "lstar", "H")}
    errs["Iemerg"] = rel_err(got["Iemerg"][0, ks], ref["Iemerg"])
    # J - S against the magnitude of its terms: at the lower boundary it falls
    # to 6e-5 of S, and 511 layers of FP64 adding leave differences of order
    # 1e-13 of S on either side (8e-10 of J - S itself there)
    S = op["Sg"][:, ks]
    errs["JmS_vs_terms"] = rel_err_terms(got["JmS"][:, ks], ref["JmS"], np.abs(ref["J"]) + np.abs(S), scale=S)
    print(f"  frequencies {ks.tolist()}; errors:", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, e in errs.items():
        assert e < 1e-10, (k, e)
    assert np.isfinite(got["J"]).all() and np.isfinite(got["lstar"]).all()


def test_c5_formal_solution_fp32_plan_full_grid_sampled(gpu_ctx, c5):
    """The same formal solution on an FP32 plan (FP32 arrays and workspace,
    FP64 arithmetic at 32 angles) against the oracle on the FP32-rounded
    inputs at 16 sampled frequencies: the FP32 contract of the dense path
    (J 2e-6, Lambda* 1e-6 per array; J - S^g and H 2e-6 of their scale)."""
    a = c5
    rows, nf, na = a.tau.shape[0], a.nf, a.na
    print(f"[case] C5 formal solution, FP32 plan, rows={rows} nf={nf} na={na}", flush=True)
    _release_device_memory()
    op = rates.opacities(a, a.nstar)
    r32 = lambda x: np.asarray(x, np.float32).astype(np.float64)
    q, Sg, om = r32(op["q"]), r32(op["Sg"]), r32(op["omega"])
    Bb, Bp = r32(a.Bnu[-1:, :]), r32(a.Bnu[-2:-1, :])
    ks = _sample_frequencies(a, n=16, seed=6)
    plan = pprt.Plan(gpu_ctx, a.nd, na, nf, precision=pprt.FP32,
                     outputs=pprt.OUT_J | pprt.OUT_JMS | pprt.OUT_LSTAR | pprt.OUT_H)
    f32 = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32, device="cuda:0")
    out = plan.formal_solution_scattering(_dev(a.tau), f32(q), f32(Sg), f32(om), Bbot=f32(Bb), Bbot_prev=f32(Bp))
    torch.cuda.synchronize()
    kt = torch.as_tensor(ks, device="cuda:0")
    got = {k: out[k].index_select(1, kt).double().cpu().numpy() for k in ("J", "JmS", "lstar", "H")}
    del out
    torch.cuda.empty_cache()
    ref = dense.formal_solution_dense(a.tau, q[:, ks], Sg[:, ks], plan.mu, plan.w, omega=om[:, ks],
                                      lower="diffusion", Bbot=Bb[0, ks], Bbot_prev=Bp[0, ks])
    scale = lambda g, r: float(np.max(np.abs(g - r)) / np.max(np.abs(r)))
    errs = {"J": rel_err(got["J"], ref["J"]), "lstar": rel_err(got["lstar"], ref["lstar"]),
            "JmS": scale(got["JmS"], ref["JmS"]), "H": scale(got["H"], ref["H"])}
    print(f"  frequencies {ks.tolist()}; errors:", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    assert errs["J"] < 2e-6 and errs["lstar"] < 1e-6
    assert errs["JmS"] < 2e-6 and errs["H"] < 2e-6


def test_c5_rates_and_solve_full_size(gpu_ctx, c5):
    a = c5
    rows = a.tau.shape[0]
    print(f"[case] C5 rates and 20-level solve rows={rows} nf={a.nf} ntr={a.nt}", flush=True)
    plan = pprt.Plan(gpu_ctx, a.nd, a.na, a.nf, precision=pprt.FP64, outputs=pprt.OUT_J | pprt.OUT_LSTAR)
    da = pprt.DeviceAtom(a)
    rng = np.random.default_rng(21)
    # populations: a random multiple of LTE per depth.  Independent factors per
    # level would invert the closely spaced upper levels of this atom; the net
    # line opacity then nearly cancels the continuum (q down to 1e-6 of its
    # terms), and a comparison measures that cancellation, not the kernels
    pops = a.nstar * rng.uniform(0.5, 2.0, size=(rows, 1))
    J = rng.uniform(0.1, 2.0, size=(rows, a.nf)) * a.Bnu
    L = rng.uniform(0.0, 1.0, size=(rows, a.nf))
    d = plan.rates_assemble(da, _dev(pops), _dev(J), _dev(L))
    torch.cuda.synchronize()
    ref = rates.preconditioned_rates(a, pops, J, L)
    # each rate sums W sigma (J - Lambda* eta / kappa) over its window, and the
    # two terms can cancel: the error is held against the magnitude of the
    # summed terms (the device Voigt function is good to about 1e-12)
    mag = rate_magnitudes(a, pops, J, L)
    for name, got, r, m in zip(("dRlu", "dRul", "Rsul"), d, ref, mag):
        g = got.cpu().numpy()
        e_terms, e_arr = rel_err_terms(g, r, m), rel_err(g, r)
        print(f"  {name}: {e_terms:.2e} of its terms, {e_arr:.2e} per array", flush=True)
        assert e_terms < 1e-11, (name, e_terms)
    pn, mx = plan.rates_solve(da, _dev(pops), *[_dev(r) for r in ref])
    torch.cuda.synchronize()
    got = pn.cpu().numpy()
    ratio, worst, bw_ratio = population_error_ratio(a, pops, ref, got, 0.0, J, L)
    print(f"  populations: worst rel err {worst:.2e}, err / condition bound {ratio:.2e}, "
          f"backward error / bound {bw_ratio:.2e}", flush=True)
    assert ratio < 1.0 and bw_ratio < 1.0
    pref = rates.solve_populations(a, *ref, scale=pops)
    assert np.isclose(float(mx.cpu()[0]), float(np.max(np.abs(pref - pops) / np.abs(pref))), rtol=1e-8)


def test_c5_multilevel_iteration_reduced_grid(gpu_ctx):
    """The C5 atom (20 levels, 100 lines, 4 continua, Voigt lines, 32 angles)
    on 10 depths, 3 points per line and 4 per continuum: one iteration from
    LTE against the oracle's iteration from the same populations."""
    a = W.c5_atom(nd=10, nline_pts=3, ncont_pts=4)
    print(f"[case] C5 reduced iteration rows={a.tau.shape[0]} nf={a.nf} na={a.na}", flush=True)
    plan = pprt.Plan(gpu_ctx, a.nd, a.na, a.nf, precision=pprt.FP64, outputs=pprt.OUT_J | pprt.OUT_LSTAR)
    da = pprt.DeviceAtom(a)
    pops = da.nstar.clone()
    mx = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    p_start = pops.cpu().numpy()
    plan.nlte_step(da.tau, da, pops, mx)
    torch.cuda.synchronize()
    p_ref, m_ref, aux = rates.nlte_iteration(a, p_start, plan.mu, plan.w)
    got = pops.cpu().numpy()
    ratio, worst, bw_ratio = population_error_ratio(a, p_start, (aux["dRlu"], aux["dRul"], aux["Rsul"]),
                                                    got, 1e-10, aux["J"], aux["lstar"])
    print(f"  worst rel err {worst:.2e}, err / condition bound {ratio:.2e}, backward error / bound "
          f"{bw_ratio:.2e}", flush=True)
    assert ratio < 1.0 and bw_ratio < 1.0
    assert np.allclose(mx.cpu().numpy(), m_ref, rtol=1e-6)

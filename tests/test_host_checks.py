"""Host-side failure detection, without a device: the input scans of the
validation mode (tau monotone and finite, arrays finite), the model-atom
checks (index tables and the rate-matrix pattern) and the binding's
argument checks, which must refuse bad inputs before anything is launched.
The singular-pattern check is pinned against the oracle's own rate matrix."""
import copy

import numpy as np
import pytest
import torch

from oracle import rates
from paper_0903_1949_amd import pprt
from paper_0903_1949_amd import workloads as W


def test_check_tau_accepts_increasing_grids():
    nd = [5, 7]
    tau = np.concatenate([W.log_tau(5, 1e-4, 1e2), W.log_tau(7, 1e-3, 1e4)])
    assert pprt.check_tau(nd, tau) == ("OK", "")


@pytest.mark.parametrize("where", [1, 4, 6])
def test_check_tau_rejects_non_monotone(where):
    nd = [5, 7]
    tau = np.concatenate([W.log_tau(5, 1e-4, 1e2), W.log_tau(7, 1e-3, 1e4)])
    tau[where] = tau[where - 1]          # equal neighbours are not strictly increasing
    st, msg = pprt.check_tau(nd, tau)
    assert st == "E_INVALID_ARG" and "strictly increasing" in msg


def test_check_tau_decrease_across_atmospheres_is_fine():
    # each atmosphere starts afresh: the second may start below the first's end
    tau = np.array([1.0, 2.0, 3.0, 0.5, 0.7])
    assert pprt.check_tau([3, 2], tau)[0] == "OK"


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
def test_check_tau_rejects_non_finite(bad):
    tau = W.log_tau(6, 1e-4, 1e4)
    tau[3] = bad
    assert pprt.check_tau([6], tau)[0] == "E_NONFINITE"


def test_check_tau_rejects_single_node():
    assert pprt.check_tau([1], np.array([1.0]))[0] == "E_SHAPE"


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_check_finite(dtype):
    x = np.linspace(0, 1, 1000).astype(dtype)
    assert pprt.check_finite(x)[0] == "OK"
    x[777] = np.nan
    st, msg = pprt.check_finite(x)
    assert st == "E_NONFINITE" and "777" in msg


@pytest.fixture(scope="module")
def atom():
    return W.multilevel_atom(nbound=4, ncont=3, nd=12, na=4, nline_pts=8, ncont_pts=6, seed=7)


def test_atom_check_host_accepts_the_recipe_atom(atom):
    assert pprt.atom_check_host(atom) == ("OK", "")


def test_atom_check_host_rejects_bad_tables(atom):
    bad = copy.deepcopy(atom)
    bad.up = bad.up.copy()
    bad.up[2] = bad.nl          # level index out of range
    st, msg = pprt.atom_check_host(bad)
    assert st == "E_INVALID_ARG" and "transition 2" in msg
    bad = copy.deepcopy(atom)
    bad.k1 = bad.k1.copy()
    bad.k1[0] += 1              # window reaches into the next transition's first point
    assert pprt.atom_check_host(bad)[0] == "E_INVALID_ARG"


def _isolate_level(atom, j):
    """Zero every rate that could connect level j: collision rates both ways
    and the cross-section over the windows of its transitions."""
    a = copy.deepcopy(atom)
    a.sigma = a.sigma.copy()
    a.Cul = a.Cul.copy()
    a.Clu = a.Clu.copy()
    for t in range(a.nt):
        if int(a.lo[t]) == j or int(a.up[t]) == j:
            a.sigma[int(a.k0[t]):int(a.k1[t])] = 0.0
            a.Cul[:, t] = 0.0
            a.Clu[:, t] = 0.0
    return a


@pytest.mark.parametrize("j", [0, 2])
def test_isolated_level_is_singular_on_host_and_in_the_oracle(atom, j):
    a = _isolate_level(atom, j)
    st, msg = pprt.atom_check_host(a)
    assert st == "E_SINGULAR" and f"level {j}" in msg
    # the pin: the oracle's statistical-equilibrium matrix for these rates
    # (any radiation field) is rank-deficient at every depth
    rows = a.tau.shape[0]
    rng = np.random.default_rng(3)
    J = rng.uniform(0.2, 2.0, size=(rows, a.nf)) * a.Bnu
    L = rng.uniform(0.0, 1.0, size=(rows, a.nf))
    dRlu, dRul, Rsul = rates.preconditioned_rates(a, a.nstar, J, L)
    # (columns scaled by the populations, as both solvers do, and rows
    # equilibrated: the unknowns and the equations span many decades)
    def smallest_sv(A, s):
        As = A * s[None, :]
        As = As / np.maximum(np.abs(As).max(axis=1, keepdims=True), 1e-300)
        return np.linalg.svd(As, compute_uv=False)[-1]

    for r in (0, rows // 2, rows - 1):
        A, _ = rates.rate_matrix(a, r, dRlu, dRul, Rsul)
        assert smallest_sv(A, a.nstar[r]) < 1e-14
    # and an untouched atom is regular there (smallest value ~1e-8..1e-7)
    dRlu, dRul, Rsul = rates.preconditioned_rates(atom, atom.nstar, J, L)
    for r in (0, rows // 2, rows - 1):
        A, _ = rates.rate_matrix(atom, r, dRlu, dRul, Rsul)
        assert smallest_sv(A, atom.nstar[r]) > 1e-10


def test_one_zero_collision_rate_is_not_singular(atom):
    a = copy.deepcopy(atom)
    a.Cul = a.Cul.copy(); a.Clu = a.Clu.copy()
    a.Cul[:, 0] = 0.0; a.Clu[:, 0] = 0.0      # the line still carries radiative rates
    assert pprt.atom_check_host(a)[0] == "OK"


class _FakeAtom:
    def __init__(self, rows, nf, nlev, ntr):
        self.struct = pprt.Atom(nlev, ntr)
        self.rows, self.nf, self.nlev, self.ntr = rows, nf, nlev, ntr


def _fake_plan(rows=10, nf=6, na=4, nb=1):
    p = object.__new__(pprt.Plan)
    p.rows, p.nf, p.na, p.nd = rows, nf, na, np.array([rows], np.int32)
    p.precision, p.dtype = pprt.FP64, torch.float64
    p.h = None
    return p


def test_binding_refuses_host_tensors_in_multilevel_calls():
    # before the fix these calls handed host pointers to the kernels
    p = _fake_plan()
    a = _FakeAtom(10, 6, 5, 4)
    pops = torch.ones(10, 5, dtype=torch.float64)
    J = torch.ones(10, 6, dtype=torch.float64)
    R = torch.ones(10, 4, dtype=torch.float64)
    with pytest.raises(TypeError, match="CUDA"):
        p.nlte_opacity(a, pops)
    with pytest.raises(TypeError, match="CUDA"):
        p.rates_assemble(a, pops, J, J)
    with pytest.raises(TypeError, match="CUDA"):
        p.rates_solve(a, pops, R, R, R)
    with pytest.raises(TypeError, match="CUDA"):
        p.nlte_step(torch.ones(10, dtype=torch.float64), a, pops, torch.zeros(1, dtype=torch.float64))


def test_binding_refuses_an_atom_of_another_shape():
    p = _fake_plan()
    with pytest.raises(ValueError, match="rows"):
        p.nlte_opacity(_FakeAtom(11, 6, 5, 4), torch.ones(10, 5, dtype=torch.float64))
    with pytest.raises(TypeError, match="DeviceAtom"):
        p.rates_solve(object(), None, None, None, None)


def test_null_arguments_of_new_entry_points():
    lib = pprt.load_library()
    assert lib.pprt_nlte_solve(None, None, None, None, None, None, None, None) == 1
    assert lib.pprt_ali_state_bytes(None, None) == 1
    assert lib.pprt_ali_state_export(None, None, None, None, 0) == 1
    assert lib.pprt_ali_state_import(None, None, 0, None, None) == 1
    assert lib.pprt_set_validation(None, 1) == 1
    assert lib.pprt_atom_check_host(None, 1, 1, None, 0) == 1

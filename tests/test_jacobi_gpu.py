"""Jacobi preconditioning (Algorithm 1 step 5, Table 2's J-VI) on an MDP whose
self-loops make diag(J_pi) far from one, and a solve through an int64 row
pointer array.

* J-VI identity: Richardson with pc jacobi and one sweep per evaluation
  (-ksp_max_it 1) gives V_{k+1} = V_k + D^-1 (T V_k - V_k),
  D = diag(I - gamma P_pi), for k = 1, 2, 5 evaluations; compared with the
  oracle's J-VI step iterated from V_0 = 0.
* Parity of the full solve with every inner solver, preconditioned and not,
  against the oracle's exact policy iteration (1e-8 in V, policy outside the
  tie band); Jacobi cuts the Richardson sweeps on this MDP.
* An MDP borrowed from device arrays keeps its int64 row pointers; its solve
  reaches the same parity.
"""
import numpy as np
import pytest

from oracle import ipi_oracle as O
from paper_2507_22538_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _ipi():
    from paper_2507_22538_amd import ipi
    return ipi


@pytest.fixture(scope="module")
def lazy():
    d = W.lazy_random(3000, 4, 6, 0.99, seed=5, stay_lo=0.5, stay_hi=0.95)
    return d, O.policy_iteration(d)


def _solve(d, **kw):
    ipi = _ipi()
    dev = _dev()
    m = ipi.MDP.from_data(d)
    try:
        V, pi, info, st = m.solve(device=dev, **kw)
        torch.cuda.synchronize()
        return V.cpu().numpy(), pi.cpu().numpy(), info, st
    finally:
        m.close()


def _parity(d, ref, V, pi, rel=1e-8):
    scale = np.max(np.abs(ref.V))
    err = np.max(np.abs(V - ref.V)) / scale
    assert err <= rel, err
    tau = O.parity_tau(ref.V)
    assert not ((pi != ref.pi) & (ref.qgap >= tau)).any()
    return err


def test_lazy_mdp_diagonal_is_far_from_one(lazy):
    d, ref = lazy
    P, _ = O.policy_matrix(d, ref.pi)
    D = O.jacobi_diagonal(P, d.gamma)
    assert D.max() < 1 - 0.99 * 0.5 + 1e-12 and D.min() > 1 - 0.99 * 0.95 - 1e-12


@pytest.mark.parametrize("k", [1, 2, 5])
def test_jvi_identity(lazy, k):
    d, _ = lazy
    ipi = _ipi()
    V, pi, info, st = _solve(d, ksp_type="richardson", pc="jacobi", max_inner=1, max_outer=k, atol=0.0)
    assert st == ipi.IPI_E_NOT_CONVERGED and info["outer_iters"] == k and info["inner_iters"] == k
    Vo = np.zeros(d.S)
    for _ in range(k):
        Vo = O.jvi_step(d, Vo)
    np.testing.assert_allclose(V, Vo, rtol=0, atol=1e-13 * np.max(np.abs(Vo)))
    # differs from plain VI here (the check above is not VI's)
    Vvi = np.zeros(d.S)
    for _ in range(k):
        Vvi = O.vi_step(d, Vvi)
    assert np.max(np.abs(Vvi - Vo)) > 1e-3 * np.max(np.abs(Vo))


def test_jvi_identity_with_scale(lazy):
    d, _ = lazy
    V, _, info, _ = _solve(d, ksp_type="richardson", pc="jacobi", max_inner=1, max_outer=2, atol=0.0, omega=0.6)
    Vo = O.jvi_step(d, O.jvi_step(d, np.zeros(d.S), omega=0.6), omega=0.6)
    np.testing.assert_allclose(V, Vo, rtol=0, atol=1e-13 * np.max(np.abs(Vo)))


@pytest.mark.parametrize("inner", ["gmres", "richardson", "tfqmr", "bicgstab"])
@pytest.mark.parametrize("pc", ["none", "jacobi"])
def test_lazy_parity(lazy, inner, pc):
    d, ref = lazy
    V, pi, info, st = _solve(d, atol=1e-10, alpha=0.1, ksp_type=inner, pc=pc, max_inner=20000)
    assert st == 0 and info["final_rho"] <= 1e-10
    _parity(d, ref, V, pi)


def test_lazy_jacobi_cuts_richardson_sweeps(lazy):
    d, ref = lazy
    _, _, plain, _ = _solve(d, atol=1e-10, alpha=0.1, ksp_type="richardson", pc="none", max_inner=20000)
    _, _, jac, _ = _solve(d, atol=1e-10, alpha=0.1, ksp_type="richardson", pc="jacobi", max_inner=20000)
    # the Jacobi sweep contracts by at most gamma (1 - p) / (1 - gamma p) per
    # sweep (0.980 at the smallest stay probability p = 0.5) instead of gamma
    assert jac["inner_iters"] < 0.8 * plain["inner_iters"], (jac["inner_iters"], plain["inner_iters"])


@pytest.mark.parametrize("inner", ["gmres", "richardson"])
def test_solve_through_int64_row_pointers(inner):
    ipi = _ipi()
    dev = _dev()
    d = W.random_sparse(5000, 4, 3, 0.99, seed=23, k_hi=11)
    ref = O.policy_iteration(d)
    t = {k: torch.from_numpy(np.ascontiguousarray(getattr(d, k))).to(dev) for k in ("row_ptr", "col", "val", "g")}
    assert t["row_ptr"].dtype == torch.int64
    h = ipi.ipi_mdp_create_csr(d.S, d.A, d.nnz, t["row_ptr"], t["col"], t["val"], t["g"], d.gamma,
                               ipi.IPI_DEVICE_PTRS | ipi.IPI_BORROW)
    m = ipi.MDP(h, d.S, d.A)
    try:
        desc = m.describe()
        assert desc["row_ptr_bytes"] == 8 and not desc["uniform_k"]
        V, pi, info, st = m.solve(device=dev, atol=1e-10, alpha=0.1, ksp_type=inner, max_inner=20000)
        torch.cuda.synchronize()
    finally:
        m.close()
    assert st == 0
    _parity(d, ref, V.cpu().numpy(), pi.cpu().numpy())

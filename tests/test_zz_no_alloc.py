"""ipi_solve_noalloc (workspace in a fixed device array) against ipi_solve on
the same MDPs: identical V and pi bit for bit, the same iteration counts, and
V within 1e-8 of the oracle's exact policy iteration.  Two calls in a row,
the second on a smaller MDP (the array keeps the first call's contents), then
the other solvers, maximisation mode, a request that does not fit, and the
MDP's own workspace left as it was."""
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


def _both(d, flags=None, **kw):
    """(V, pi, info) of ipi_solve and of ipi_solve_noalloc on one MDP."""
    from paper_2507_22538_amd import ipi
    dev = _dev()
    m = ipi.MDP.from_data(d) if flags is None else ipi.MDP.from_data(d, flags=flags)
    try:
        out = []
        for fn in (ipi.ipi_solve, ipi.ipi_solve_noalloc):
            V = torch.full((d.S,), float("nan"), dtype=torch.float64, device=dev)
            pi = torch.full((d.S,), -1, dtype=torch.int32, device=dev)
            st, info = fn(m.handle, ipi.make_opts(**kw), V, pi)
            torch.cuda.synchronize()
            out.append((st, V.cpu().numpy(), pi.cpu().numpy(), info))
        return out
    finally:
        m.close()


def _check(d, ref, a, b, rel=1e-8, sign=1.0):
    (sa, Va, pa, ia), (sb, Vb, pb, ib) = a, b
    assert sa == sb == 0
    assert np.array_equal(Va, Vb) and np.array_equal(pa, pb)
    assert (ia["outer_iters"], ia["inner_iters"]) == (ib["outer_iters"], ib["inner_iters"])
    assert ia["final_rho"] == ib["final_rho"]
    err = np.max(np.abs(sign * Vb - ref.V)) / np.max(np.abs(ref.V))
    assert err <= rel, err
    assert not ((pb != ref.pi) & (ref.qgap >= O.parity_tau(ref.V))).any()


def test_split_values_and_stencil_products():
    """The pendulum (stencil form: the products read P_pi's row words from
    the array too) with its values held as float32 hi + lo, fp32_inner
    Jacobi-Richardson."""
    from paper_2507_22538_amd import ipi
    d = W.c3(32)
    a, b = _both(d, flags=ipi.IPI_VAL_SPLIT, atol=0.0, rtol_cert=1e-11, alpha=0.1, ksp_type="richardson",
                 pc="jacobi", max_inner=1000000, precision="fp32_inner")
    _check(d, O.policy_iteration(d), a, b)


def test_two_calls_second_smaller():
    big = W.random_sparse(4000, 4, 8, 0.99, seed=31)
    small = W.random_sparse(700, 3, 5, 0.95, seed=32)
    for d in (big, small):
        a, b = _both(d, atol=1e-10, alpha=0.1, ksp_type="gmres")
        _check(d, O.policy_iteration(d), a, b)


@pytest.mark.parametrize("inner", ["richardson", "tfqmr", "bicgstab"])
def test_other_inner_solvers(inner):
    d = W.c2(4096) if inner == "richardson" else W.random_sparse(2500, 5, 6, 0.99, seed=33, k_hi=9)
    a, b = _both(d, atol=1e-10, alpha=0.1, ksp_type=inner, max_inner=50000)
    _check(d, O.policy_iteration(d), a, b)


def test_fp32_mixed_and_jacobi():
    d = W.lazy_random(2000, 4, 6, 0.99, seed=34, stay_lo=0.5, stay_hi=0.95)
    a, b = _both(d, atol=1e-10, alpha=0.1, ksp_type="gmres", pc="jacobi", precision="fp32_mixed")
    _check(d, O.policy_iteration(d.fp32_rounded()), a, b)


def test_maxreward():
    d = W.random_sparse(1500, 4, 8, 0.99, seed=35)
    a, b = _both(d, atol=1e-10, alpha=0.1, ksp_type="gmres", mode="MAXREWARD")
    neg = W.MDPData(d.S, d.A, d.row_ptr, d.col, d.val, -d.g, d.gamma)
    # maximising the rewards g = minimising the costs -g; V is returned negated back
    _check(d, O.policy_iteration(neg), a, b, sign=-1.0)


def test_too_large_is_refused_and_own_workspace_kept():
    from paper_2507_22538_amd import ipi
    dev = _dev()
    # GMRES(30) on 300,000 states needs 31 basis vectors of 2.4 MB: past 64 MiB
    d = W.random_sparse(300_000, 2, 2, 0.9, seed=36)
    m = ipi.MDP.from_data(d)
    try:
        V = torch.empty(d.S, dtype=torch.float64, device=dev)
        pi = torch.empty(d.S, dtype=torch.int32, device=dev)
        with pytest.raises(ipi.IPIError) as e:
            ipi.ipi_solve_noalloc(m.handle, ipi.make_opts(ksp_type="gmres", restart=30), V, pi)
        assert e.value.status == ipi.IPI_E_TOO_LARGE and "bytes" in str(e.value)
        # Richardson needs no basis: fits, and leaves the MDP's workspace alone
        kw = dict(atol=1e-9, alpha=0.1, ksp_type="richardson", max_inner=100000)
        st0, i0 = ipi.ipi_solve(m.handle, ipi.make_opts(**kw), V, pi)
        V0, p0 = V.clone(), pi.clone()
        V1 = torch.empty_like(V)
        p1 = torch.empty_like(pi)
        st1, i1 = ipi.ipi_solve_noalloc(m.handle, ipi.make_opts(**kw), V1, p1)
        st2, i2 = ipi.ipi_solve(m.handle, ipi.make_opts(**kw), V, pi)
        torch.cuda.synchronize()
        assert st0 == st1 == st2 == 0
        assert torch.equal(V0, V1) and torch.equal(p0, p1) and torch.equal(V0, V) and torch.equal(p0, pi)
        assert m.describe()["device_bytes"] > 0
    finally:
        m.close()

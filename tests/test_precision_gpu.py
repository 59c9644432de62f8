"""Precision modes and float32-only storage.

* fp32_inner (the Bellman pass on FP64 values, the inner solve on a float32
  P_pi): V within 1e-8 of the oracle's V* of the FP64 MDP, with every inner
  solver; the inner solves move float32 bytes.
* The stated error bound of each result (ipi_solve_info.err_bound) holds
  against the FP64 oracle in every mode, and in fp32_mixed it comes from an
  FP64 Bellman pass on the returned V (fp64_rho equals the oracle's
  recomputed residual).
* IPI_VAL_FP32_ONLY keeps only float32 values: the row perturbation it
  records equals the one computed here from the FP64 input; fp32_mixed
  solves give the same bits as on an MDP holding both copies; the stated
  bound uses the recorded perturbation and still holds; FP64 work is refused.
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


def _row_perturbation(d):
    dv = np.abs(d.val - d.val.astype(np.float32).astype(np.float64))
    rid = np.repeat(np.arange(d.S * d.A), np.diff(d.row_ptr))
    return float(np.bincount(rid, weights=dv, minlength=d.S * d.A).max())


def _solve(m, d, **kw):
    dev = _dev()
    V, pi, info, st = m.solve(device=dev, **kw)
    torch.cuda.synchronize()
    return V.cpu().numpy(), pi.cpu().numpy(), info, st


@pytest.fixture(scope="module")
def rnd():
    d = W.random_sparse(3000, 5, 7, 0.995, seed=41, k_hi=10)
    return d, O.policy_iteration(d)


@pytest.mark.parametrize("inner", ["gmres", "richardson", "tfqmr", "bicgstab"])
def test_fp32_inner_reaches_fp64_vstar(rnd, inner):
    ipi = _ipi()
    d, ref = rnd
    m = ipi.MDP.from_data(d, flags=0)  # no float32 copy of P needed: P_pi is rounded when formed
    try:
        V, pi, info, st = _solve(m, d, atol=0.0, rtol_cert=1e-10, alpha=0.1, ksp_type=inner, max_inner=20000,
                                 precision="fp32_inner")
    finally:
        m.close()
    assert st == 0
    scale = np.max(np.abs(ref.V))
    err = np.max(np.abs(V - ref.V)) / scale
    assert err <= 1e-8, err
    assert not ((pi != ref.pi) & (ref.qgap >= O.parity_tau(ref.V))).any()
    assert info["fp64_rho"] == info["final_rho"]
    assert np.max(np.abs(V - ref.V)) <= info["err_bound"] * (1 + 1e-6) + 1e-13 * scale


def test_fp32_mixed_states_its_fp64_distance(rnd):
    ipi = _ipi()
    d, ref = rnd
    m = ipi.MDP.from_data(d, flags=ipi.IPI_VAL_FP32)
    try:
        V, pi, info, st = _solve(m, d, atol=0.0, rtol_cert=1e-10, alpha=0.1, precision="fp32_mixed")
        desc = m.describe()
    finally:
        m.close()
    assert st == 0
    # the extra FP64 pass: the oracle's own residual of V on the FP64 MDP
    cert = O.certificate(d, V)
    assert abs(info["fp64_rho"] - cert.rho) <= 1e-12 * np.max(np.abs(V))
    assert info["err_bound"] == info["fp64_rho"] / (1 - d.gamma)
    assert np.max(np.abs(V - ref.V)) <= info["err_bound"] * (1 + 1e-6)
    assert desc["has_fp64"] == 1 and desc["fp32_row_perturbation"] == pytest.approx(_row_perturbation(d), rel=1e-12)


@pytest.mark.parametrize("device_inputs", [False, True])
def test_fp32_only_storage(rnd, device_inputs):
    ipi = _ipi()
    dev = _dev()
    d, ref = rnd
    both = ipi.MDP.from_data(d, flags=ipi.IPI_VAL_FP32)
    if device_inputs:
        t = {k: torch.from_numpy(np.ascontiguousarray(getattr(d, k))).to(dev) for k in ("row_ptr", "col", "val", "g")}
        h = ipi.ipi_mdp_create_csr(d.S, d.A, d.nnz, t["row_ptr"], t["col"], t["val"], t["g"], d.gamma,
                                   ipi.IPI_DEVICE_PTRS | ipi.IPI_VAL_FP32_ONLY)
        only = ipi.MDP(h, d.S, d.A)
    else:
        only = ipi.MDP.from_data(d, flags=ipi.IPI_VAL_FP32_ONLY)
    try:
        db, do = both.describe(), only.describe()
        assert do["has_fp64"] == 0 and do["has_fp32"] == 1
        assert do["fp32_row_perturbation"] == pytest.approx(_row_perturbation(d), rel=1e-12)
        assert do["device_bytes"] <= db["device_bytes"] - 8 * d.nnz + 1024
        kw = dict(atol=0.0, rtol_cert=1e-10, alpha=0.1, precision="fp32_mixed")
        Vb, pib, ib, stb = _solve(both, d, **kw)
        Vo, pio, io, sto = _solve(only, d, **kw)
        assert stb == sto == 0
        assert np.array_equal(Vb, Vo) and np.array_equal(pib, pio)
        assert np.isnan(io["fp64_rho"])
        dp = do["fp32_row_perturbation"]
        want = (io["final_rho"] + d.gamma * dp * np.max(np.abs(Vo))) / (1 - d.gamma)
        assert io["err_bound"] == pytest.approx(want, rel=1e-12)
        assert io["err_bound"] >= ib["err_bound"] * (1 - 1e-9)
        assert np.max(np.abs(Vo - ref.V)) <= io["err_bound"]
        # FP64 work needs the FP64 values
        for prec in ("fp64", "fp32_inner"):
            with pytest.raises(ipi.IPIError) as e:
                _solve(only, d, precision=prec)
            assert e.value.status == ipi.IPI_E_INVALID_ARG
        with pytest.raises(ipi.IPIError):
            only.bellman(torch.zeros(d.S, dtype=torch.float64, device=dev), ipi.IPI_FP64)
        TV, pi32, _, rho = only.bellman(torch.from_numpy(Vo).to(dev), ipi.IPI_FP32_MIXED)
        torch.cuda.synchronize()
        br = O.bellman(d.fp32_rounded(), Vo)
        np.testing.assert_allclose(TV.cpu().numpy(), br.TV, rtol=0, atol=1e-12 * np.max(np.abs(Vo)))
    finally:
        both.close()
        only.close()


def test_fp32_only_in_batch(rnd):
    ipi = _ipi()
    dev = _dev()
    d, ref = rnd
    ds = [d, W.random_sparse(900, 4, 6, 0.97, seed=42)]
    mdps = [ipi.MDP.from_data(x, flags=ipi.IPI_VAL_FP32_ONLY) for x in ds]
    try:
        opts = [ipi.make_opts(atol=0.0, rtol_cert=1e-10, alpha=0.1, precision="fp32_mixed") for _ in ds]
        Vs = [torch.empty(x.S, dtype=torch.float64, device=dev) for x in ds]
        ps = [torch.empty(x.S, dtype=torch.int32, device=dev) for x in ds]
        sts, infos = ipi.ipi_solve_batch([m.handle for m in mdps], opts, Vs, ps)
        torch.cuda.synchronize()
        for x, V, st, info in zip(ds, Vs, sts, infos):
            assert st == 0 and np.isnan(info["fp64_rho"])
            r = O.policy_iteration(x)
            assert np.max(np.abs(V.cpu().numpy() - r.V)) <= info["err_bound"]
        with pytest.raises(ipi.IPIError):
            ipi.ipi_solve_batch([mdps[0].handle], [ipi.make_opts(precision="fp64")], Vs[:1], ps[:1])
    finally:
        for m in mdps:
            m.close()

"""Values held as float32 hi + lo (IPI_VAL_SPLIT) against the oracle.

* The create step splits P as the oracle's split rule does: the recorded row
  perturbations (of hi alone and of hi + lo) equal the oracle's, and the
  MDP holds 4 bytes a value less than one with FP64 values and a float32
  copy; host and device inputs give the same bits.
* A Bellman pass in FP64 arithmetic on split values is the FP64 pass on the
  MDP whose values are hi + lo: every launch form (CSR lanes, workgroup and
  wave tiles, band and stencil forms, every chunk width) within the rounding
  bound of the oracle on that MDP, and within gamma * dS * ||V|| of the pass
  on the FP64 values.
* fp32_inner solves on split values reach the FP64 oracle's V* within 1e-8
  and state a bound that holds; fp32_mixed solves give the same bits as on
  an MDP holding FP64 values and a float32 copy (they read hi alone), with
  their FP64 pass on hi + lo; fp64 solves and the combination with
  IPI_VAL_FP32_ONLY are refused.
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


def _effective(d):
    """The MDP whose values are hi + lo (the split rule of the oracle)."""
    return W.MDPData(d.S, d.A, d.row_ptr, d.col, O.split_effective(d.val), d.g, d.gamma, d.name + "-split")


def _pass_check(d, V, TV, pi, resid, rho):
    br = O.bellman(d, V)
    kmax = int(np.max(np.diff(d.row_ptr)))
    tol = 4 * (kmax + 2) * 2.0 ** -52 * (float(np.max(np.abs(d.g))) + d.gamma * float(np.max(np.abs(V))) + 1.0)
    np.testing.assert_allclose(TV, br.TV, rtol=0, atol=tol)
    gap = O.q_gap(br.Q, d.S, d.A)
    assert not ((pi != br.pi) & (gap > 2 * tol)).any()
    np.testing.assert_array_equal(resid, TV - V)
    assert rho == np.max(np.abs(TV - V))
    return tol


SHAPES = [
    ("random_ragged_S3000", lambda: W.random_sparse(3000, 5, 7, 0.995, seed=41, k_hi=10)),
    ("random_S3001_A5_k32", lambda: W.random_sparse(3001, 5, 32, 0.99, seed=31)),
    ("birth_death_4096_k24", lambda: W.c2(4096)),
    ("pendulum_40_k4", lambda: W.c3(40)),
]


@pytest.mark.parametrize("name,make", SHAPES, ids=[s[0] for s in SHAPES])
def test_split_bellman_is_the_pass_on_hi_plus_lo(name, make):
    ipi = _ipi()
    dev = _dev()
    d = make()
    de = _effective(d)
    V = np.random.default_rng(7).normal(size=d.S) * 5.0
    Vd = torch.from_numpy(V).to(dev)
    sp = ipi.MDP.from_data(d, flags=ipi.IPI_VAL_SPLIT)
    f64 = ipi.MDP.from_data(d, flags=0)
    try:
        desc = sp.describe()
        assert desc["has_split"] == 1 and desc["has_fp64"] == 0 and desc["has_fp32"] == 1
        dS = O.split_row_perturbation(d.S, d.A, d.row_ptr, d.val)
        assert desc["split_row_perturbation"] == pytest.approx(dS, rel=1e-12, abs=1e-300)
        uniform = desc["uniform_k"] == 1
        k = desc["k_max"]
        TV64, _, _, _ = f64.bellman(Vd, ipi.IPI_FP64)
        torch.cuda.synchronize()
        TV64 = TV64.cpu().numpy()
        ran = 0
        shapes = [(0, 0, 0)]
        if uniform:
            shapes += [(lanes, spt, chunk) for chunk in (4, 8, 16, 32) if k % chunk == 0
                       for lanes in (-1, -3, -2) for spt in (0, 5)]
        shapes += [(1, 0, 0), (4, 0, 0), (16, 3, 0)]
        for lanes, spt, chunk in shapes:
            sp.set_tuning(bellman_lanes=lanes, bellman_states_per_tile=spt, bellman_chunk=chunk)
            TV, pi, resid, rho = sp.bellman(Vd, ipi.IPI_FP64)
            torch.cuda.synchronize()
            TVh = TV.cpu().numpy()
            tol = _pass_check(de, V, TVh, pi.cpu().numpy(), resid.cpu().numpy(), float(rho.cpu()[0]))
            # against the pass on the FP64 values: the split's row perturbation
            assert np.max(np.abs(TVh - TV64)) <= d.gamma * desc["split_row_perturbation"] * np.max(np.abs(V)) + 2 * tol
            ran += 1
        assert ran >= 4
    finally:
        sp.close()
        f64.close()


def test_split_create_host_and_device_inputs():
    ipi = _ipi()
    dev = _dev()
    d = W.c2(4096)
    both = ipi.MDP.from_data(d, flags=ipi.IPI_VAL_FP32)
    host = ipi.MDP.from_data(d, flags=ipi.IPI_VAL_SPLIT)
    t = {k: torch.from_numpy(np.ascontiguousarray(getattr(d, k))).to(dev) for k in ("row_ptr", "col", "val", "g")}
    dv = ipi.MDP(ipi.ipi_mdp_create_csr(d.S, d.A, d.nnz, t["row_ptr"], t["col"], t["val"], t["g"], d.gamma,
                                        ipi.IPI_DEVICE_PTRS | ipi.IPI_VAL_SPLIT), d.S, d.A)
    bw = ipi.MDP(ipi.ipi_mdp_create_csr(d.S, d.A, d.nnz, t["row_ptr"], t["col"], t["val"], t["g"], d.gamma,
                                        ipi.IPI_DEVICE_PTRS | ipi.IPI_BORROW | ipi.IPI_VAL_SPLIT), d.S, d.A)
    try:
        db, dh = both.describe(), host.describe()
        # values: 8 bytes (hi + lo) instead of 12 (FP64 + float32)
        assert dh["device_bytes"] == db["device_bytes"] - 4 * d.nnz
        hi = d.val.astype(np.float32).astype(np.float64)
        rid = np.repeat(np.arange(d.S * d.A), np.diff(d.row_ptr))
        dp32 = float(np.bincount(rid, weights=np.abs(d.val - hi), minlength=d.S * d.A).max())
        assert dh["fp32_row_perturbation"] == pytest.approx(dp32, rel=1e-12)
        V = torch.from_numpy(np.random.default_rng(3).normal(size=d.S)).to(dev)
        outs = []
        for m in (host, dv, bw):
            desc = m.describe()
            assert desc["split_row_perturbation"] == dh["split_row_perturbation"]
            assert desc["fp32_row_perturbation"] == dh["fp32_row_perturbation"]
            TV, pi, _, _ = m.bellman(V, ipi.IPI_FP64)
            TV32, _, _, _ = m.bellman(V, ipi.IPI_FP32_MIXED)
            torch.cuda.synchronize()
            outs.append((TV.cpu(), pi.cpu(), TV32.cpu()))
        TVb, _, _, _ = both.bellman(V, ipi.IPI_FP32_MIXED)
        torch.cuda.synchronize()
        for o in outs[1:]:
            assert all(torch.equal(a, b) for a, b in zip(outs[0], o))
        # fp32_mixed passes read hi alone: the float32 copy's bits
        assert torch.equal(outs[0][2], TVb.cpu())
    finally:
        for m in (both, host, dv, bw):
            m.close()


@pytest.fixture(scope="module")
def rnd():
    d = W.random_sparse(3000, 5, 7, 0.995, seed=41, k_hi=10)
    return d, O.policy_iteration(d)


@pytest.mark.parametrize("inner", ["gmres", "richardson", "tfqmr"])
def test_split_fp32_inner_reaches_fp64_vstar(rnd, inner):
    ipi = _ipi()
    dev = _dev()
    d, ref = rnd
    m = ipi.MDP.from_data(d, flags=ipi.IPI_VAL_SPLIT)
    try:
        V, pi, info, st = m.solve(device=dev, atol=0.0, rtol_cert=1e-10, alpha=0.1, ksp_type=inner,
                                  max_inner=20000, precision="fp32_inner")
        torch.cuda.synchronize()
        V, pi = V.cpu().numpy(), pi.cpu().numpy()
        desc = m.describe()
    finally:
        m.close()
    assert st == 0
    scale = np.max(np.abs(ref.V))
    assert np.max(np.abs(V - ref.V)) / scale <= 1e-8
    assert not ((pi != ref.pi) & (ref.qgap >= O.parity_tau(ref.V))).any()
    # the bound: the residual on hi + lo plus the split's row perturbation
    want = (info["final_rho"] + d.gamma * desc["split_row_perturbation"] * np.max(np.abs(V))) / (1 - d.gamma)
    assert info["err_bound"] == pytest.approx(want, rel=1e-9)
    assert np.max(np.abs(V - ref.V)) <= info["err_bound"] * (1 + 1e-6) + 1e-13 * scale
    # the residual the solve stopped on is the oracle's residual on the MDP hi + lo
    cert = O.certificate(_effective(d), V)
    assert abs(info["final_rho"] - cert.rho) <= 1e-12 * scale


def test_split_fp32_mixed_and_refusals(rnd):
    ipi = _ipi()
    dev = _dev()
    d, ref = rnd
    both = ipi.MDP.from_data(d, flags=ipi.IPI_VAL_FP32)
    sp = ipi.MDP.from_data(d, flags=ipi.IPI_VAL_SPLIT)
    try:
        kw = dict(atol=0.0, rtol_cert=1e-10, alpha=0.1, precision="fp32_mixed")
        Vb, pib, ib, stb = both.solve(device=dev, **kw)
        Vs, pis, isp, sts = sp.solve(device=dev, **kw)
        torch.cuda.synchronize()
        assert stb == sts == 0
        assert torch.equal(Vb, Vs) and torch.equal(pib, pis)
        # its FP64 pass runs on hi + lo: the oracle's residual there
        Vh = Vs.cpu().numpy()
        cert = O.certificate(_effective(d), Vh)
        assert abs(isp["fp64_rho"] - cert.rho) <= 1e-12 * np.max(np.abs(Vh))
        dS = sp.describe()["split_row_perturbation"]
        want = (isp["fp64_rho"] + d.gamma * dS * np.max(np.abs(Vh))) / (1 - d.gamma)
        assert isp["err_bound"] == pytest.approx(want, rel=1e-9)
        assert np.max(np.abs(Vh - ref.V)) <= isp["err_bound"] * (1 + 1e-6)
        with pytest.raises(ipi.IPIError) as e:
            sp.solve(device=dev, precision="fp64")
        assert e.value.status == ipi.IPI_E_INVALID_ARG
        with pytest.raises(ipi.IPIError) as e:
            ipi.MDP.from_data(d, flags=ipi.IPI_VAL_SPLIT | ipi.IPI_VAL_FP32_ONLY)
        assert e.value.status == ipi.IPI_E_INVALID_ARG
    finally:
        both.close()
        sp.close()


def test_split_members_in_batch(rnd):
    """Batched fp32_mixed members on split values read hi alone: the same
    bits as members holding FP64 values and a float32 copy; their stated
    bound (from the float32 rounding, no FP64 pass in the batch) holds;
    fp32_inner members need FP64 values there."""
    ipi = _ipi()
    dev = _dev()
    d, ref = rnd
    ds = [d, W.random_sparse(900, 4, 6, 0.97, seed=42)]
    res = {}
    for flags in (ipi.IPI_VAL_SPLIT, ipi.IPI_VAL_FP32):
        mdps = [ipi.MDP.from_data(x, flags=flags) for x in ds]
        try:
            opts = [ipi.make_opts(atol=0.0, rtol_cert=1e-10, alpha=0.1, precision="fp32_mixed") for _ in ds]
            Vs = [torch.empty(x.S, dtype=torch.float64, device=dev) for x in ds]
            ps = [torch.empty(x.S, dtype=torch.int32, device=dev) for x in ds]
            sts, infos = ipi.ipi_solve_batch([m.handle for m in mdps], opts, Vs, ps)
            torch.cuda.synchronize()
            assert all(st == 0 for st in sts)
            res[flags] = [(V.cpu(), p.cpu(), info) for V, p, info in zip(Vs, ps, infos)]
            if flags == ipi.IPI_VAL_SPLIT:
                for x, V, info in zip(ds, Vs, infos):
                    assert np.isnan(info["fp64_rho"])
                    r = ref if x is d else O.policy_iteration(x)
                    assert np.max(np.abs(V.cpu().numpy() - r.V)) <= info["err_bound"]
                with pytest.raises(ipi.IPIError):
                    ipi.ipi_solve_batch([mdps[0].handle], [ipi.make_opts(precision="fp32_inner")], Vs[:1], ps[:1])
        finally:
            for m in mdps:
                m.close()
    for (Va, pa, _), (Vb, pb, _) in zip(res[ipi.IPI_VAL_SPLIT], res[ipi.IPI_VAL_FP32]):
        assert torch.equal(Va, Vb) and torch.equal(pa, pb)

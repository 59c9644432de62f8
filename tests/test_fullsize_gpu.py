"""Full-size checks at the benchmark shapes, in the launch configuration the
benchmark uses (default tuning: flat chunk streaming for these uniform-row
MDPs).

* Birth-death MDP, S = 2e6, A = 16, 768e6 nonzeros; pendulum 2048 x 2048,
  A = 11: the fused Bellman pass on sampled states, each recomputed one by one
  by the oracle (both precisions; the mixed mode against float32-rounded P).
* Birth-death full solves (FP64 and FP32-mixed): the oracle's FP64 Bellman
  pass over all states recomputes ||V - TV||_inf and certifies
  ||V - V*||_inf <= rho / (1 - gamma) <= 1e-9 ||V||_inf; pi must be greedy for V.
* Birth-death full solves compared element by element with the oracle's
  exact policy iteration at full size (banded LU evaluation): FP64 within
  1e-8 of V*, FP32-mixed within 1e-8 of the oracle on float32-rounded P,
  and its error against the FP64 original stated and bounded.
* Pendulum full solves (gamma = 0.9999, Richardson) in both precisions,
  certified by the oracle's Bellman pass: ||V - V*||_inf <= 1.05e-9 ||V||_inf
  and pi greedy for V.
* Pendulum: one Table 2 VI step at full size equals T(0) on sampled states.
"""
import sys

import numpy as np
import pytest

from oracle import ipi_oracle as O
from paper_2507_22538_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def c2():
    return W.c2()


@pytest.fixture(scope="module")
def c3():
    return W.c3(2048)


@pytest.fixture(scope="module")
def c2_oracle(c2):
    """The oracle's exact policy iteration on the full birth-death MDP (banded
    LU evaluation), on its FP64 values and on float32-rounded ones."""
    ref = O.policy_iteration(c2)
    ref32 = O.policy_iteration(c2.fp32_rounded())
    assert ref.tier == "banded" and ref32.tier == "banded"
    return ref, ref32


def _gpu_solve(d, precision, split=False, **kw):
    from paper_2507_22538_amd import ipi
    dev = _dev()
    m = ipi.MDP.from_data(d, flags=ipi.IPI_VAL_SPLIT if split else ipi.IPI_VAL_FP32)
    try:
        V, pi, info, st = m.solve(device=dev, precision=precision, **kw)
        torch.cuda.synchronize()
        return V.cpu().numpy(), pi.cpu().numpy(), info, st
    finally:
        m.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed", "fp32_inner", "fp32_inner_split"])
def test_c2_full_oracle_parity(c2, c2_oracle, precision):
    """fp32_inner_split: fp32_inner on the MDP holding its values as float32
    hi + lo (no FP64 values): the FP64 MDP's V* at the same bar."""
    from paper_2507_22538_amd import ipi
    ref, ref32 = c2_oracle
    split = precision == "fp32_inner_split"
    V, pi, info, st = _gpu_solve(c2, "fp32_inner" if split else precision, split=split, atol=0.0, rtol_cert=1e-9,
                                 alpha=0.1, ksp_type="richardson", max_inner=100000)
    assert st == ipi.IPI_OK
    target = ref32 if precision == "fp32_mixed" else ref
    scale = np.max(np.abs(target.V))
    err = np.max(np.abs(V - target.V)) / scale
    err64 = np.max(np.abs(V - ref.V)) / np.max(np.abs(ref.V))
    print(f"\nc2 {precision}: rel. error vs the oracle on its own P {err:.3e}, vs the FP64 oracle {err64:.3e}, "
          f"stated bound {info['err_bound'] / np.max(np.abs(ref.V)):.3e}", file=sys.stderr)
    assert err <= 1e-8, err
    # the library's stated bound on the distance to the FP64 MDP's V* holds
    assert np.max(np.abs(V - ref.V)) <= info["err_bound"] * (1 + 1e-6) + 1e-13 * np.max(np.abs(ref.V))
    tau = O.parity_tau(target.V)
    assert not ((pi != target.pi) & (target.qgap >= tau)).any()
    if precision == "fp32_mixed":
        # the float32 rounding of P moves V* by at most
        # gamma max_row ||dP_row||_1 ||V*||_inf / (1 - gamma)
        dP = np.abs(c2.val.astype(np.float32).astype(np.float64) - c2.val).reshape(-1, 24).sum(axis=1).max()
        bound = c2.gamma * dP / (1 - c2.gamma) + 2e-9
        assert err64 <= bound, (err64, bound)


@pytest.mark.parametrize("precision,pc", [("fp64", "none"), ("fp64", "jacobi"), ("fp32_mixed", "jacobi"),
                                          ("fp32_inner", "jacobi")])
def test_c3_full_solve_certificate(c3, precision, pc):
    """Richardson, plain and Jacobi-preconditioned (a third of the sweeps on
    this MDP: its low-velocity states keep much of their mass in their own
    cell, so diag(J_pi) is far from 1)."""
    from paper_2507_22538_amd import ipi
    V, pi, info, st = _gpu_solve(c3, precision, atol=0.0, rtol_cert=1e-9, alpha=0.1, ksp_type="richardson",
                                 pc=pc, max_inner=1000000)
    assert st == ipi.IPI_OK, info
    ref = c3.fp32_rounded() if precision == "fp32_mixed" else c3
    cert = O.certificate(ref, V, pi)
    print(f"\nc3 {precision} pc {pc}: {info['outer_iters']} outer, {info['inner_iters']} inner, certified error bound "
          f"{cert.bound / np.max(np.abs(V)):.3e} relative, {cert.uncertain} states in the tie band", file=sys.stderr)
    assert cert.bound <= 1.05e-9 * np.max(np.abs(V)), cert
    assert cert.greedy_ok


def _sample_states(S, n, seed):
    rng = np.random.default_rng(seed)
    pick = set(rng.choice(S, n, replace=False).tolist())
    pick.update([0, 1, 2, 11, 12, 13, S // 2, S - 3, S - 2, S - 1])
    return np.array(sorted(pick), dtype=np.int64)


def _bellman_sampled(d, precision, seed):
    from paper_2507_22538_amd import ipi
    dev = _dev()
    m = ipi.MDP.from_data(d, flags=ipi.IPI_VAL_FP32)
    try:
        rng = np.random.default_rng(seed)
        V = rng.random(d.S) * 100.0
        TV, pi, resid, rho = m.bellman(torch.from_numpy(V).to(dev), precision)
        torch.cuda.synchronize()
        TV, pi, resid, rho = TV.cpu().numpy(), pi.cpu().numpy(), resid.cpu().numpy(), float(rho.cpu()[0])
    finally:
        m.close()
    ref = d.fp32_rounded() if precision == 1 else d
    states = _sample_states(d.S, 1500, seed)
    TVo, pio, gap, _ = O.bellman_states(ref, V, states)
    kmax = int(np.max(np.diff(d.row_ptr[:1000])))
    tol = 4 * (kmax + 2) * 2.0 ** -52 * (np.max(np.abs(d.g)) + d.gamma * np.max(np.abs(V)) + 1)
    np.testing.assert_allclose(TV[states], TVo, rtol=0, atol=tol)
    bad = (pi[states] != pio) & (gap > 2 * tol)
    assert not bad.any()
    np.testing.assert_array_equal(resid, TV - V)
    assert rho == np.max(np.abs(TV - V))


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32mixed"])
def test_c2_bellman_sampled(c2, precision):
    _bellman_sampled(c2, precision, 1)


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32mixed"])
def test_c3_bellman_sampled(c3, precision):
    _bellman_sampled(c3, precision, 2)


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_c2_full_solve_certificate(c2, precision):
    from paper_2507_22538_amd import ipi
    dev = _dev()
    m = ipi.MDP.from_data(c2, flags=ipi.IPI_VAL_FP32)
    try:
        V, pi, info, st = m.solve(device=dev, atol=0.0, rtol_cert=1e-9, alpha=0.1, ksp_type="richardson",
                                  precision=precision, max_inner=100000)
        torch.cuda.synchronize()
        V, pi = V.cpu().numpy(), pi.cpu().numpy()
    finally:
        m.close()
    assert st == ipi.IPI_OK
    # the load policy at full size: an FP64 sweep (440 MB) exceeds the cache
    # budget and streams, an FP32 one (248 MB) is loaded through the caches;
    # the blocked sweeps always are (bit 1)
    assert info["ppi_cached"] == (2 if precision == "fp64" else 3)
    ref = c2.fp32_rounded() if precision == "fp32_mixed" else c2
    cert = O.certificate(ref, V, pi)
    assert cert.bound <= 1.05e-9 * np.max(np.abs(V)), cert
    assert cert.greedy_ok
    if precision == "fp32_mixed":
        # the FP64 original: same check with the rounding of P folded into the bound
        exact = O.certificate(c2, V)
        dP = np.abs(c2.val[:24 * 16 * 2000] - ref.val[:24 * 16 * 2000]).reshape(-1, 24).sum(axis=1).max()
        assert exact.bound <= 1.05e-9 * np.max(np.abs(V)) + c2.gamma * dP * np.max(np.abs(V)) / (1 - c2.gamma) * 2


def test_c3_vi_step_sampled(c3):
    from paper_2507_22538_amd import ipi
    dev = _dev()
    m = ipi.MDP.from_data(c3, flags=ipi.IPI_VAL_FP32)
    try:
        V, pi, info, st = m.solve(device=dev, max_outer=1, ksp_type="richardson", max_inner=1)
        torch.cuda.synchronize()
        V = V.cpu().numpy()
    finally:
        m.close()
    assert st == ipi.IPI_E_NOT_CONVERGED and info["outer_iters"] == 1
    states = _sample_states(c3.S, 1500, 3)
    TVo, _, _, _ = O.bellman_states(c3, np.zeros(c3.S), states)
    np.testing.assert_allclose(V[states], TVo, rtol=1e-15, atol=1e-12)

"""Parity of the full iPI solve (ipi_solve, Algorithm 1) with the CPU oracle.

Bar (per result): ||V_gpu - V*||_inf <= 1e-8 ||V*||_inf; pi_gpu equals the
oracle's greedy policy except at states whose Q-gap is below
tau = 1e-10 max(1, ||V*||_inf), and pi_gpu is near-optimal under the oracle's
Q* everywhere.  Table 2's special cases (VI, beta-VI, OPI(W)) are checked as
identities against the oracle's own DP steps.
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


def solve(d, v0=None, **kw):
    ipi = _ipi()
    dev = _dev()
    m = ipi.MDP.from_data(d)
    try:
        if v0 is not None:
            kw["v0"] = torch.from_numpy(np.ascontiguousarray(v0, np.float64)).to(dev)
        V, pi, info, st = m.solve(device=dev, **kw)
        torch.cuda.synchronize()
        return V.cpu().numpy(), pi.cpu().numpy(), info, st
    finally:
        m.close()


def assert_parity(d, V, pi, ref=None, rel=1e-8):
    ref = ref or O.policy_iteration(d)
    scale = np.max(np.abs(ref.V))
    err = np.max(np.abs(V - ref.V)) / max(scale, 1e-300)
    assert err <= rel, f"relative V error {err:.3e} > {rel}"
    tau = O.parity_tau(ref.V)
    mism = (pi != ref.pi) & (ref.qgap >= tau)
    assert not mism.any(), f"{mism.sum()} policy mismatches with Q-gap >= tau"
    Q = O.q_values(d.S, d.A, d.row_ptr, d.col, d.val, d.g, d.gamma, ref.V).reshape(d.S, d.A)
    assert np.all(Q[np.arange(d.S), pi] - Q.min(axis=1) <= tau)
    return err


@pytest.fixture(scope="module")
def c1_ref():
    return W.c1(), O.policy_iteration(W.c1())


@pytest.mark.parametrize("inner", ["gmres", "richardson", "bicgstab", "tfqmr"])
def test_c1_parity(c1_ref, inner):
    d, ref = c1_ref
    V, pi, info, st = solve(d, atol=1e-10, alpha=0.1, ksp_type=inner)
    assert st == 0 and info["converged"] == 1
    assert info["final_rho"] <= 1e-10
    assert_parity(d, V, pi, ref)
    assert info["outer_iters"] >= 1 and info["inner_iters"] >= info["outer_iters"]


@pytest.mark.parametrize("restart,reorth,pc", [(30, 1, "none"), (5, 1, "none"), (30, 2, "none"), (1, 1, "none"),
                                               (30, 1, "jacobi"), (64, 2, "jacobi")])
def test_c1_gmres_variants(c1_ref, restart, reorth, pc):
    d, ref = c1_ref
    V, pi, info, st = solve(d, atol=1e-10, alpha=0.1, restart=restart, reorth=reorth, pc=pc)
    assert st == 0
    assert_parity(d, V, pi, ref)


@pytest.mark.parametrize("inner", ["richardson", "bicgstab", "tfqmr"])
def test_c1_jacobi(c1_ref, inner):
    d, ref = c1_ref
    V, pi, info, st = solve(d, atol=1e-10, alpha=0.1, ksp_type=inner, pc="jacobi")
    assert st == 0
    assert_parity(d, V, pi, ref)


def test_bicgstab_safeguard_on_divergence():
    # BiCGStab diverges on this chain from V = 0; the correction then falls back
    # to one Richardson step, so one outer iteration equals one VI step
    d = W.c2(1024)
    Vg, _, info, _ = solve(d, max_outer=1, max_inner=3000, alpha=0.1, ksp_type="bicgstab")
    Vvi = O.vi_step(d, np.zeros(d.S))
    br = O.bellman(d, np.zeros(d.S))
    b = br.TV  # rhs T V_0 - V_0 of the first inner solve (V_0 = 0)
    assert np.all(np.isfinite(Vg))
    if not (info["inner_resid"] <= np.linalg.norm(b)):
        # safeguard fired: the correction is one Richardson step, V_1 = T V_0
        np.testing.assert_allclose(Vg, Vvi, rtol=0, atol=1e-12 * np.max(np.abs(Vvi)))
    else:
        # no fallback: V_1 - V_0 is BiCGStab's correction, whose true linear
        # residual b - J_pi delta (recomputed here) is the one reported
        P, _ = O.policy_matrix(d, br.pi)
        lin = b - (Vg - d.gamma * (P @ Vg))
        assert np.linalg.norm(lin) <= np.linalg.norm(b)
        assert abs(np.linalg.norm(lin) - info["inner_resid"]) <= 1e-7 * np.linalg.norm(b)


def test_bicgstab_residual_matches_recomputation():
    # the recursive residual equals the recomputed ||b - J_pi delta||_2 when the
    # iteration did not grow the residual; when it did (here after 2 iterations,
    # 114.9 > 16.3), the safeguard returns one Richardson step instead
    d = W.random_sparse(4000, 4, 8, 0.99, seed=11)
    br = O.bellman(d, np.zeros(d.S))
    P, _ = O.policy_matrix(d, br.pi)
    b = br.TV
    for steps in (1, 2, 4, 5):
        Vg, _, info, _ = solve(d, max_outer=1, max_inner=steps, alpha=1e-14, ksp_type="bicgstab")
        assert info["inner_iters"] == steps
        res = np.linalg.norm(b - (Vg - d.gamma * (P @ Vg)))
        if info["inner_resid"] <= np.linalg.norm(b):
            assert abs(info["inner_resid"] - res) <= 1e-9 * np.linalg.norm(b)
        else:
            np.testing.assert_allclose(Vg, b, rtol=0, atol=1e-14 * np.max(np.abs(b)))


def test_tfqmr_residual_within_bound():
    # TFQMR stops on the quasi-residual bound sqrt(k + 1) tau_k, which is an
    # upper bound of the true ||b - J_pi delta_k||_2: recompute the latter
    d = W.random_sparse(4000, 4, 8, 0.99, seed=11)
    br = O.bellman(d, np.zeros(d.S))
    P, _ = O.policy_matrix(d, br.pi)
    b = br.TV
    for steps in (1, 2, 3, 6, 11):
        Vg, _, info, _ = solve(d, max_outer=1, max_inner=steps, alpha=1e-14, ksp_type="tfqmr")
        assert info["inner_iters"] == steps
        # an unconverged end reports the recomputed true residual of its iterate
        # (and falls back to one Richardson step if that exceeds ||b||)
        assert info["inner_resid"] <= np.linalg.norm(b), "no fallback expected on this MDP"
        res = np.linalg.norm(b - (Vg - d.gamma * (P @ Vg)))
        assert abs(info["inner_resid"] - res) <= 1e-9 * np.linalg.norm(b)
    # a converged solve: the bound passed the forcing test, so the true residual did too
    target = 0.1 * np.max(np.abs(b))
    Vg, _, info, _ = solve(d, max_outer=1, max_inner=1000, alpha=0.1, ksp_type="tfqmr")
    res = np.linalg.norm(b - (Vg - d.gamma * (P @ Vg)))
    assert info["inner_resid"] < target and res <= info["inner_resid"] * (1 + 1e-12)


def test_tfqmr_safeguard_never_grows_residual():
    # on the birth-death chain at gamma = 0.999 TFQMR breaks down or stalls
    # from V = 0; the accepted correction then never has a larger residual
    # than the start (else it is one Richardson step)
    d = W.c2(1024)
    br = O.bellman(d, np.zeros(d.S))
    P, _ = O.policy_matrix(d, br.pi)
    b = br.TV
    for cap in (7, 300):
        Vg, _, info, _ = solve(d, max_outer=1, max_inner=cap, alpha=1e-3, ksp_type="tfqmr")
        assert np.all(np.isfinite(Vg))
        res = np.linalg.norm(b - (Vg - d.gamma * (P @ Vg)))
        if info["inner_resid"] <= np.linalg.norm(b):
            assert res <= np.linalg.norm(b) * (1 + 1e-12)
        else:
            np.testing.assert_allclose(Vg, b, rtol=0, atol=1e-14 * np.max(np.abs(b)))


_ORACLE_CACHE = {}


def _oracle(key, d):
    if key not in _ORACLE_CACHE:
        _ORACLE_CACHE[key] = O.policy_iteration(d)
    return _ORACLE_CACHE[key]


# Restarted GMRES stagnates and BiCGStab diverges on the strongly non-normal
# birth-death chain at gamma = 0.999 (the field of values of J_pi reaches
# Re < 0), where Richardson converges; GMRES(30) also stalls on the 64 x 64
# pendulum at gamma = 0.9999 but converges on the 32 x 32 one.
# Each case uses the inner solver that suits it, as the paper advises (Sec. III-A).
@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed", "fp32_inner"])
@pytest.mark.parametrize("name,make,inner", [
    ("birth_death_4096", lambda: W.c2(4096), "richardson"),
    ("pendulum_32", lambda: W.c3(32), "gmres"),
    ("pendulum_64", lambda: W.c3(64), "richardson"),
    ("random_S3000_A6_var4_12", lambda: W.random_sparse(3000, 6, 4, 0.95, seed=3, k_hi=12), "gmres"),
    ("maze_60x80", lambda: W.maze(60, 80), "tfqmr"),
    ("amdahl_S2000_A100_k150", lambda: W.amdahl(S=2000), "gmres"),
])
def test_reduced_configs(name, make, inner, precision):
    d = make()
    ref_d = d.fp32_rounded() if precision == "fp32_mixed" else d
    ref = _oracle((name, precision), ref_d)
    V, pi, info, st = solve(d, atol=0.0, rtol_cert=1e-9, alpha=0.1, precision=precision,
                            max_inner=3000 if inner == "richardson" else 5000, ksp_type=inner)
    assert st == 0, info
    # fp32_inner targets the FP64 MDP itself (float32 only in the inner solves)
    assert_parity(ref_d, V, pi, ref)
    exact = _oracle((name, "fp64"), d)
    # the stated bound on the distance to the FP64 MDP's V* holds (contraction
    # of T); in fp32_mixed it comes from an extra FP64 Bellman pass
    assert np.isfinite(info["err_bound"]) and info["err_bound"] == info["fp64_rho"] / (1 - d.gamma)
    assert np.max(np.abs(V - exact.V)) <= info["err_bound"] * (1 + 1e-6) + 1e-13 * np.max(np.abs(exact.V))
    if precision != "fp32_mixed":
        assert info["fp64_rho"] == info["final_rho"]
    if precision == "fp32_mixed":
        # against the FP64 original: bounded by gamma * max row |dP|_1 * ||V*|| / (1 - gamma)
        dP = np.abs(d.val - ref_d.val)
        rid = np.repeat(np.arange(d.S * d.A), np.diff(d.row_ptr))
        row_l1 = np.bincount(rid, weights=dP, minlength=d.S * d.A).max()
        bound = d.gamma * row_l1 * np.max(np.abs(exact.V)) / (1 - d.gamma) + 1e-8 * np.max(np.abs(exact.V))
        assert np.max(np.abs(V - exact.V)) <= bound


def test_single_action_is_linear_solve():
    d = W.random_sparse(2000, 1, 7, 0.98, seed=4)
    V, pi, info, st = solve(d, atol=1e-11, alpha=0.01)
    P, g = O.policy_matrix(d, np.zeros(d.S, dtype=np.int32))
    Vt = np.linalg.solve(np.eye(d.S) - d.gamma * P.toarray(), g)
    assert np.max(np.abs(V - Vt)) <= 1e-9 * np.max(np.abs(Vt))
    assert np.all(pi == 0)


def test_identity_transitions_happy_breakdown():
    # P_a = I: J_pi = (1 - gamma) I, GMRES is exact after one step
    S, A, gamma = 500, 3, 0.9
    P = np.zeros((S, A, S))
    for a in range(A):
        P[:, a, :] = np.eye(S)
    g = np.random.default_rng(5).random((S, A))
    d = W.from_dense(P, g, gamma)
    V, pi, info, st = solve(d, atol=1e-12, alpha=1e-6)
    np.testing.assert_allclose(V, g.min(axis=1) / (1 - gamma), rtol=1e-12)
    assert info["outer_iters"] == 1 and info["inner_iters"] == 1


def test_vi_identity():
    # Table 2 VI: Richardson, one sweep, scale 1 -> V_{k+1} = T V_k
    d = W.random_sparse(1500, 5, 6, 0.9, seed=6)
    for n in (1, 2, 5):
        Vg, _, info, st = solve(d, max_outer=n, ksp_type="richardson", max_inner=1)
        assert st == _ipi().IPI_E_NOT_CONVERGED and info["outer_iters"] == n
        Vr = np.zeros(d.S)
        for _ in range(n):
            Vr = O.vi_step(d, Vr)
        np.testing.assert_allclose(Vg, Vr, rtol=0, atol=1e-13 * max(1, np.max(np.abs(Vr))))


def test_beta_vi_identity():
    d = W.random_sparse(1500, 5, 6, 0.9, seed=7)
    v0 = np.random.default_rng(8).normal(size=d.S)
    Vg, _, _, _ = solve(d, v0=v0, max_outer=1, ksp_type="richardson", max_inner=1, omega=0.35)
    np.testing.assert_allclose(Vg, O.beta_vi_step(d, v0, 0.35), atol=1e-13)


@pytest.mark.parametrize("Wn", [1, 3, 10])
def test_opi_identity(Wn):
    d = W.random_sparse(1500, 5, 6, 0.9, seed=9)
    v0 = np.random.default_rng(10).normal(size=d.S)
    Vg, _, info, _ = solve(d, v0=v0, max_outer=1, ksp_type="richardson", max_inner=Wn, alpha=1e-15)
    assert info["inner_iters"] == Wn
    np.testing.assert_allclose(Vg, O.opi_step(d, v0, Wn), atol=1e-12)


def test_gmres_residual_estimate_matches_recomputation():
    # one outer iteration from V_0 = 0 with a few GMRES steps: the forcing test's
    # |g_{j+1}| must equal the recomputed ||b - J_pi delta||_2
    d = W.random_sparse(4000, 4, 8, 0.99, seed=11)
    for steps in (1, 3, 7):
        Vg, _, info, _ = solve(d, max_outer=1, max_inner=steps, alpha=1e-14)
        br = O.bellman(d, np.zeros(d.S))
        P, _ = O.policy_matrix(d, br.pi)
        b = br.TV  # T V_0 - V_0 with V_0 = 0
        delta = Vg
        res = np.linalg.norm(b - (delta - d.gamma * (P @ delta)))
        assert info["inner_iters"] == steps
        assert abs(info["inner_resid"] - res) <= 1e-10 * np.linalg.norm(b)


def test_cap_returns_not_converged_with_outputs(c1_ref):
    d, ref = c1_ref
    V, pi, info, st = solve(d, atol=1e-12, max_outer=1, alpha=0.5)
    assert st == _ipi().IPI_E_NOT_CONVERGED
    assert info["converged"] == 0 and info["outer_iters"] == 1
    assert np.all(np.isfinite(V)) and info["final_rho"] > 1e-12
    # pi is greedy for the returned V
    assert np.array_equal(pi, O.bellman(d, V).pi) or np.all(
        np.abs(O.bellman(d, V).Q.reshape(d.S, d.A)[np.arange(d.S), pi] - O.bellman(d, V).TV) < 1e-12)


def test_warm_start_from_solution(c1_ref):
    d, ref = c1_ref
    V, pi, info, st = solve(d, v0=ref.V, atol=1e-10)
    assert st == 0 and info["outer_iters"] == 0
    assert_parity(d, V, pi, ref)


def test_max_reward_mode():
    d = W.random_sparse(800, 4, 6, 0.97, seed=12)
    V, pi, info, st = solve(d, atol=1e-10, alpha=0.1, mode="MAXREWARD")
    neg = W.MDPData(d.S, d.A, d.row_ptr, d.col, d.val, -d.g, d.gamma)
    ref = O.policy_iteration(neg)
    assert_parity(neg, -V, pi, ref)


def test_solve_deterministic():
    d = W.random_sparse(30000, 6, 12, 0.99, seed=13)
    a = solve(d, atol=1e-9, alpha=0.1)
    b = solve(d, atol=1e-9, alpha=0.1)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert a[2]["inner_iters"] == b[2]["inner_iters"]


def test_brute_force_tiny_solves():
    ipi = _ipi()
    for seed in range(6):
        d = W.tiny_random(6, 3, seed, 0.9)
        Vstar, optimal = O.brute_force(d)
        V, pi, info, st = solve(d, atol=1e-12, alpha=0.01)
        assert st == ipi.IPI_OK
        np.testing.assert_allclose(V, Vstar, rtol=0, atol=1e-10 * max(1, np.max(np.abs(Vstar))))
        assert tuple(int(a) for a in pi) in set(optimal)


def test_invalid_options_rejected():
    ipi = _ipi()
    d = W.random_sparse(50, 2, 3, 0.9, seed=1)
    m = ipi.MDP.from_data(d, flags=0)
    try:
        with pytest.raises(ipi.IPIError):
            m.solve(precision="fp32_mixed")  # no float32 copy
    finally:
        m.close()


@pytest.mark.parametrize("name,make,kw", [
    ("c1_gmres", lambda: W.c1(), dict(atol=1e-10, alpha=0.1)),
    ("c1_gmres_cgs2_jacobi", lambda: W.c1(), dict(atol=1e-10, alpha=0.1, reorth=2, pc="jacobi", restart=7)),
    ("birth_death_4096_gmres_capped", lambda: W.c2(4096), dict(atol=1e-10, alpha=0.1, max_outer=3, restart=12)),
])
def test_graph_replay_equals_eager(name, make, kw):
    # Without profiling, GMRES cycles are captured once into a HIP graph and
    # replayed; with profiling they are launched one by one.  Every solve below
    # replays the cached graph many times, with eager launches (Bellman passes,
    # updates, a direct ipi_bellman call) between the replays: all results must
    # be bitwise equal to the eager run.
    ipi = _ipi()
    dev = _dev()
    d = make()
    m = ipi.MDP.from_data(d)
    try:
        eager = m.solve(device=dev, profile=1, **kw)
        torch.cuda.synchronize()
        runs = []
        for _ in range(3):
            runs.append(m.solve(device=dev, profile=0, **kw))
            torch.cuda.synchronize()
            m.bellman(torch.zeros(d.S, dtype=torch.float64, device=dev))
            torch.cuda.synchronize()
        for V, pi, info, st in runs:
            assert st == eager[3]
            assert torch.equal(V, eager[0]) and torch.equal(pi, eager[1])
            assert info["inner_iters"] == eager[2]["inner_iters"]
            assert info["outer_iters"] == eager[2]["outer_iters"]
    finally:
        m.close()


BLOCK_CASES = [
    ("birth_death_4096", lambda: W.c2(4096)),
    ("birth_death_1000", lambda: W.c2(1000)),      # one workgroup holds every state
    ("birth_death_20011", lambda: W.c2(20011)),    # a ragged last workgroup
]


@pytest.mark.parametrize("name,make", BLOCK_CASES, ids=[c[0] for c in BLOCK_CASES])
@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_richardson_blocked_sweeps_identical(name, make, precision):
    # temporally blocked sweeps compute every state exactly as one-sweep
    # launches do, and the stopping tests fall on the same sweeps
    dev = _dev()
    from paper_2507_22538_amd import ipi
    d = make()
    m = ipi.MDP.from_data(d, flags=ipi.IPI_VAL_FP32)
    try:
        assert m.describe()["band"] == 1
        runs = []
        for blk, prof in ((0, 0), (1, 0), (1, 2)):
            V, pi, info, st = m.solve(device=dev, atol=0.0, rtol_cert=1e-9, alpha=0.1, ksp_type="richardson",
                                      max_inner=100000, precision=precision, richardson_block=blk, profile=prof)
            torch.cuda.synchronize()
            assert st == ipi.IPI_OK
            runs.append((V.cpu().numpy(), pi.cpu().numpy(), info))
    finally:
        m.close()
    (V0, p0, i0), (V1, p1, i1), (V2, p2, i2) = runs
    assert i0["inner_iters"] > 300  # long enough for blocks of 8
    assert i1["inner_iters"] == i0["inner_iters"] and i1["outer_iters"] == i0["outer_iters"]
    np.testing.assert_array_equal(V1, V0)
    np.testing.assert_array_equal(p1, p0)
    np.testing.assert_array_equal(V2, V0)
    assert i2["product_calls"] > 0 and i2["product_ms"] > 0
    ref = d.fp32_rounded() if precision == "fp32_mixed" else d
    want = O.policy_iteration(ref)
    assert np.max(np.abs(V1 - want.V)) <= 1e-8 * np.max(np.abs(want.V))


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_richardson_blocked_persistent_many_blocks(precision):
    """More blocks than CUs (about 715 blocks of 840 states at 8 sweeps, 915 of
    656 at 16, a ragged last one): the persistent kernels (float32 rows:
    register prefetch; FP64 rows of 24: LDS prefetch) walk several blocks
    each and give the iterates of one block per workgroup and of one launch
    per sweep, bit for bit, with and without the Jacobi scaling."""
    dev = _dev()
    from paper_2507_22538_amd import ipi
    d = W.c2(600011)
    m = ipi.MDP.from_data(d, flags=ipi.IPI_VAL_FP32)
    try:
        for pc in ("none", "jacobi"):
            runs = []
            for blk, pf in ((0, 0), (1, 0), (1, -1)):
                m.set_tuning(blocked_prefetch=pf)
                V, pi, info, st = m.solve(device=dev, atol=0.0, rtol_cert=1e-9, alpha=0.1, ksp_type="richardson",
                                          max_inner=100000, precision=precision, richardson_block=blk, pc=pc)
                torch.cuda.synchronize()
                assert st == ipi.IPI_OK
                runs.append((V.cpu().numpy(), pi.cpu().numpy(), info))
            (V0, p0, i0), (V1, p1, i1), (V2, p2, i2) = runs
            assert i0["block_launches"] == 0 and i1["block_launches"] > 1000 and i2["block_launches"] > 1000
            # past sweep 1024 of an inner solve the tests fall every 16th sweep and
            # each launch runs 16 sweeps: fewer launches than with 4 and 8 only
            n_o = i1["outer_iters"]
            assert i1["block_launches"] < (i1["inner_iters"] - 1024 * n_o) / 8 + 156 * n_o - 10
            for V, p_, i in ((V1, p1, i1), (V2, p2, i2)):
                assert (i["inner_iters"], i["outer_iters"]) == (i0["inner_iters"], i0["outer_iters"])
                np.testing.assert_array_equal(V, V0)
                np.testing.assert_array_equal(p_, p0)
    finally:
        m.close()
    ref = d.fp32_rounded() if precision == "fp32_mixed" else d
    want = O.policy_iteration(ref)
    assert np.max(np.abs(V1 - want.V)) <= 1e-8 * np.max(np.abs(want.V))


def test_richardson_blocked_short_caps_and_other_mdps():
    # caps that cut the sweeps between two tests short, OPI(W) steps, and an
    # MDP without the band form: the option changes nothing but the launches
    dev = _dev()
    from paper_2507_22538_amd import ipi
    for d in (W.c2(4096), W.c3(24)):
        m = ipi.MDP.from_data(d, flags=ipi.IPI_VAL_FP32)
        try:
            for kw in (dict(max_outer=2, max_inner=37, alpha=1e-15), dict(max_outer=1, max_inner=300, alpha=1e-15),
                       dict(atol=0.0, rtol_cert=1e-9, alpha=0.1, max_inner=100000)):
                outs = []
                for blk in (0, 1):
                    V, pi, info, st = m.solve(device=dev, ksp_type="richardson", richardson_block=blk, **kw)
                    torch.cuda.synchronize()
                    outs.append((V.cpu().numpy(), info["inner_iters"], st))
                np.testing.assert_array_equal(outs[0][0], outs[1][0])
                assert outs[0][1:] == outs[1][1:]
        finally:
            m.close()


@pytest.mark.parametrize("extra", [dict(pc="jacobi"), dict(omega=0.8), dict(mode="MAXREWARD")],
                         ids=["jacobi", "omega0.8", "maxreward"])
def test_richardson_blocked_options(extra):
    # the blocked sweeps apply the Jacobi scaling and the Richardson scale
    # exactly as the one-sweep kernel does
    dev = _dev()
    from paper_2507_22538_amd import ipi
    d = W.c2(6007)
    m = ipi.MDP.from_data(d, flags=ipi.IPI_VAL_FP32)
    try:
        runs = []
        for blk in (0, 1):
            V, pi, info, st = m.solve(device=dev, atol=0.0, rtol_cert=1e-9, alpha=0.1, ksp_type="richardson",
                                      max_inner=100000, richardson_block=blk, **extra)
            torch.cuda.synchronize()
            assert st == ipi.IPI_OK
            runs.append((V.cpu().numpy(), pi.cpu().numpy(), info["inner_iters"]))
    finally:
        m.close()
    (V0, p0, n0), (V1, p1, n1) = runs
    assert n0 > 300 and n1 == n0
    np.testing.assert_array_equal(V1, V0)
    np.testing.assert_array_equal(p1, p0)


def _band_mdp(S, A, k, shift, seed=3):
    """Band rows of k consecutive columns starting at clip(s - k // 2 +
    shift(s, a), 0, S - k); seeded positive values normalised per row."""
    rng = np.random.default_rng(seed)
    R = S * A
    r = np.arange(R)
    s, a = r // A, r % A
    w = np.clip(s - k // 2 + shift(s, a), 0, S - k)
    col = (w[:, None] + np.arange(k)[None, :]).reshape(-1).astype(np.int32)
    val = rng.exponential(size=(R, k))
    val = (val / val.sum(axis=1, keepdims=True)).reshape(-1)
    row_ptr = np.arange(R + 1, dtype=np.int64) * k
    g = rng.random(R) + 0.1 * a
    return W.MDPData(S, A, row_ptr, col, val, g, 0.995, f"band_k{k}")


BAND_BLOCK_CASES = [(k, prec, sh) for k in (8, 16, 32) for prec in ("fp64", "fp32_mixed")
                    for sh in ("fixed", "varying")]


@pytest.mark.parametrize("k,precision,shift", BAND_BLOCK_CASES,
                         ids=[f"k{k}-{p}-{sh}" for k, p, sh in BAND_BLOCK_CASES])
def test_richardson_blocked_row_lengths(k, precision, shift):
    """Band rows of 8, 16 and 32 entries in both precisions run the blocked
    kernels' other instantiations (two states per thread for FP64 rows of 8
    and float32 rows of 8 and 16, register prefetch for 128-byte rows, one
    state per thread for FP64 rows of 32).  A first column at a fixed offset
    from the state gives adjacent windows; one that moves with the state
    parity and the action does not (each window read on its own).  Iterates
    and stopping sweeps equal one launch per sweep, bit for bit, with a
    ragged last block, and V* the oracle's."""
    dev = _dev()
    from paper_2507_22538_amd import ipi
    fn = (lambda s, a: np.zeros_like(s)) if shift == "fixed" else (lambda s, a: (s % 2) * (1 + a % 3) - 1)
    d = _band_mdp(20011, 4, k, fn)
    m = ipi.MDP.from_data(d, flags=ipi.IPI_VAL_FP32)
    try:
        assert m.describe()["band"] == 1
        runs = []
        for blk in (0, 1):
            V, pi, info, st = m.solve(device=dev, atol=0.0, rtol_cert=1e-9, alpha=0.1, ksp_type="richardson",
                                      max_inner=100000, precision=precision, richardson_block=blk)
            torch.cuda.synchronize()
            assert st == ipi.IPI_OK
            runs.append((V.cpu().numpy(), pi.cpu().numpy(), info))
    finally:
        m.close()
    (V0, p0, i0), (V1, p1, i1) = runs
    assert i0["inner_iters"] > 300 and i1["block_launches"] > 0
    assert (i1["inner_iters"], i1["outer_iters"]) == (i0["inner_iters"], i0["outer_iters"])
    np.testing.assert_array_equal(V1, V0)
    np.testing.assert_array_equal(p1, p0)
    ref = d.fp32_rounded() if precision == "fp32_mixed" else d
    want = O.policy_iteration(ref)
    assert np.max(np.abs(V1 - want.V)) <= 1e-8 * np.max(np.abs(want.V))

"""Pins for the oracle's certificate, its J-VI step and its C Bellman products.

* certificate (residual r(V) = V - TV of Sec. II and the contraction bound):
  at a hand-derived V* the residual vanishes; V* + c 1 has residual
  (1 - gamma)|c| and bound |c| (shift property of T, rows of P sum to one);
  the bound holds against brute-force V* for random V; a policy that is not
  greedy fails; a constructed set of Q-gaps around the tie band
  2 gamma rho / (1 - gamma) is counted exactly.
* J-VI (Table 2, Jacobi-preconditioned Richardson, one sweep): exact in one
  step when every action stays put (P_a = I: J_pi is diagonal); equal to VI
  on an MDP without self-loops; a two-state example derived by hand; V* is a
  fixed point.
* C Bellman products: bit-identical to the numpy definition.
* Planted mistakes in each of these must break a pin.
"""
import glob
import json
import os

import numpy as np
import pytest

from oracle import ipi_oracle as O
from paper_2507_22538_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden():
    out = []
    for path in sorted(glob.glob(os.path.join(GOLDEN, "*.json"))):
        case = json.load(open(path))
        d = W.from_dense(np.array(case["P"]), np.array(case["g"]), case["gamma"])
        out.append((os.path.basename(path), d, np.array(case["V_star"], dtype=np.float64),
                    np.array(case["pi_star"], dtype=np.int32)))
    return out


# ---------------------------------------------------------------------------
# certificate
# ---------------------------------------------------------------------------

def check_certificate_fixed_point_and_shift():
    for name, d, Vs, pis in _golden():
        scale = max(1.0, np.max(np.abs(Vs)))
        c0 = O.certificate(d, Vs, pis)
        assert c0.rho <= 1e-14 * scale, (name, c0)
        assert c0.greedy_ok, name
        for c in (-2.5, 0.75, 1e-3):
            cert = O.certificate(d, Vs + c)
            # T(V* + c 1) = T V* + gamma c 1 = V* + gamma c 1, so V - TV = (1 - gamma) c 1
            want = (1.0 - d.gamma) * abs(c)
            assert abs(cert.rho - want) <= 1e-13 * scale, (name, c, cert.rho, want)
            # the contraction bound is then exactly the distance |c| to V*
            assert abs(cert.bound - abs(c)) <= 1e-13 * scale / (1.0 - d.gamma), (name, c, cert.bound)


def check_certificate_bounds_true_error():
    rng = np.random.default_rng(41)
    for seed in range(6):
        d = W.tiny_random(5, 3, 200 + seed, gamma=float(rng.choice([0.5, 0.9, 0.99])))
        Vstar, _ = O.brute_force(d)
        for _ in range(4):
            V = Vstar + rng.normal(size=d.S) * 10.0 ** rng.uniform(-6, 1)
            cert = O.certificate(d, V)
            err = np.max(np.abs(V - Vstar))
            assert err <= cert.bound * (1 + 1e-12) + 1e-13, (seed, err, cert.bound)
            # and the bound is not vacuous: rho <= (1 + gamma) ||V - V*||
            assert cert.rho <= (1.0 + d.gamma) * err * (1 + 1e-12) + 1e-13


def _stay_put(gaps, gamma):
    """S states, A = 2, P_a = I: action 0 costs 0, action 1 costs gaps[s].
    V* = 0 and Q_V(s, a) = g(s, a) + gamma V(s), so the Q-gap is gaps[s] at any V."""
    S = len(gaps)
    P = np.zeros((S, 2, S))
    for a in range(2):
        P[:, a, :] = np.eye(S)
    g = np.stack([np.zeros(S), np.asarray(gaps, dtype=np.float64)], axis=1)
    return W.from_dense(P, g, gamma)


def check_certificate_greedy_and_uncertain():
    gamma, c = 0.9, 0.01
    gaps = [0.001, 0.01, 0.017, 0.019, 0.5, 1.0]
    d = _stay_put(gaps, gamma)
    V = np.full(d.S, c)                       # V* + c 1
    cert = O.certificate(d, V, np.zeros(d.S, dtype=np.int32))
    # rho = (1 - gamma) c = 1e-3; tie band 2 gamma rho / (1 - gamma) = 2 gamma c = 0.018
    assert abs(cert.rho - 1e-3) <= 1e-15
    assert cert.greedy_ok
    assert cert.uncertain == 3, cert        # gaps 0.001, 0.01, 0.017
    # a policy that takes the costlier action at one state is not greedy
    bad = np.zeros(d.S, dtype=np.int32)
    bad[4] = 1
    assert not O.certificate(d, V, bad).greedy_ok
    # ... unless its excess is inside the given tie tolerance
    assert O.certificate(d, V, bad, tie_tol=0.6).greedy_ok
    # golden cases: flipping the action of a state with a clear gap fails
    for name, dd, Vs, pis in _golden():
        if dd.A < 2:
            continue
        Q = O.q_values(dd.S, dd.A, dd.row_ptr, dd.col, dd.val, dd.g, dd.gamma, Vs).reshape(dd.S, dd.A)
        s = int(np.argmax(np.sort(Q, axis=1)[:, 1] - Q.min(axis=1)))
        other = pis.copy()
        other[s] = (pis[s] + 1) % dd.A
        assert O.certificate(dd, Vs, pis).greedy_ok, name
        assert not O.certificate(dd, Vs, other).greedy_ok, name


def test_certificate_fixed_point_and_shift():
    check_certificate_fixed_point_and_shift()


def test_certificate_bounds_true_error():
    check_certificate_bounds_true_error()


def test_certificate_greedy_and_uncertain():
    check_certificate_greedy_and_uncertain()


# ---------------------------------------------------------------------------
# J-VI
# ---------------------------------------------------------------------------

def check_jvi_stay_put_exact():
    rng = np.random.default_rng(5)
    S, A, gamma = 7, 3, 0.95
    P = np.zeros((S, A, S))
    for a in range(A):
        P[:, a, :] = np.eye(S)
    g = rng.random((S, A))
    d = W.from_dense(P, g, gamma)
    V0 = rng.normal(size=S) * 3
    # J_pi = (1 - gamma) I is its own diagonal: one J-VI step solves it
    np.testing.assert_allclose(O.jvi_step(d, V0), g.min(axis=1) / (1 - gamma), rtol=1e-13)


def check_jvi_no_self_loops_is_vi():
    d = W.random_sparse(300, 3, 5, 0.97, seed=12)
    rows = np.repeat(np.arange(d.S * d.A), np.diff(d.row_ptr))
    keep = d.col != rows // d.A
    assert (~keep).any()
    # drop the self-loops and renormalise: an MDP with P(s, s, a) = 0 everywhere
    val = d.val * keep
    sums = np.bincount(rows, weights=val, minlength=d.S * d.A)
    assert np.all(sums > 0)
    val = val / sums[rows]
    nd = W.MDPData(d.S, d.A, d.row_ptr, d.col, val, d.g, d.gamma)
    V = np.random.default_rng(3).random(d.S) * 10
    np.testing.assert_allclose(O.jvi_step(nd, V), O.vi_step(nd, V), rtol=1e-14)


def check_jvi_two_state_by_hand():
    # one action; P = [[1/2, 1/2], [1/4, 3/4]], g = (1, 2), gamma = 0.9:
    # D = (1 - 0.45, 1 - 0.675) = (11/20, 13/40)
    d = W.from_dense(np.array([[[0.5, 0.5]], [[0.25, 0.75]]]), np.array([[1.0], [2.0]]), 0.9)
    # from V = 0: V1 = g / D = (20/11, 80/13)
    np.testing.assert_allclose(O.jvi_step(d, np.zeros(2)), [20 / 11, 80 / 13], rtol=1e-15)
    # from V = 1: g - J V = g - (1 - gamma) = (0.9, 1.9); V1 = 1 + (18/11, 76/13)
    np.testing.assert_allclose(O.jvi_step(d, np.ones(2)), [29 / 11, 89 / 13], rtol=1e-15)
    # omega scales the correction
    np.testing.assert_allclose(O.jvi_step(d, np.ones(2), omega=0.5), [1 + 9 / 11, 1 + 38 / 13], rtol=1e-15)


def check_jvi_fixed_point():
    d = W.lazy_random(200, 3, 4, 0.95, seed=4)
    ref = O.policy_iteration(d)
    np.testing.assert_allclose(O.jvi_step(d, ref.V), ref.V, rtol=0, atol=1e-12 * np.max(np.abs(ref.V)))


def test_jvi_stay_put_exact():
    check_jvi_stay_put_exact()


def test_jvi_no_self_loops_is_vi():
    check_jvi_no_self_loops_is_vi()


def test_jvi_two_state_by_hand():
    check_jvi_two_state_by_hand()


def test_jvi_fixed_point():
    check_jvi_fixed_point()


def test_lazy_random_is_self_loop_heavy():
    d = W.lazy_random(400, 4, 6, 0.99, seed=2)
    O.validate(d.S, d.A, d.row_ptr, d.col, d.val, d.g, d.gamma)
    rows = np.repeat(np.arange(d.S * d.A), np.diff(d.row_ptr))
    diag = np.bincount(rows, weights=d.val * (d.col == rows // d.A), minlength=d.S * d.A)
    assert diag.min() >= 0.3 - 1e-12 and np.median(diag) > 0.5
    assert np.all(np.diff(d.col)[np.diff(rows) == 0] > 0)  # sorted, distinct columns


# ---------------------------------------------------------------------------
# C Bellman products
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("which", ["random_ragged", "birth_death", "pendulum", "lazy"])
def test_c_products_bitwise_equal_numpy(which):
    if O.c_library() is None:
        pytest.skip("oracle C library not built (run __graft_entry__.build())")
    d = {"random_ragged": lambda: W.random_sparse(3000, 5, 2, 0.95, seed=9, k_hi=17),
         "birth_death": lambda: W.birth_death(5000, 16, 0.999),
         "pendulum": lambda: W.pendulum(64, 11, 0.9999),
         "lazy": lambda: W.lazy_random(2000, 4, 6, 0.99, seed=1)}[which]()
    V = np.random.default_rng(11).normal(size=d.S) * 50
    ref = O.q_values(d.S, d.A, d.row_ptr, d.col, d.val, d.g, d.gamma, V)
    for threads in (1, 3, 0):
        got = O.q_values_chunked(d.S, d.A, d.row_ptr, d.col, d.val, d.g, d.gamma, V, threads=threads)
        assert np.array_equal(got, ref), which
    np.testing.assert_array_equal(
        O.q_values_numpy_chunked(d.S, d.A, d.row_ptr, d.col, d.val, d.g, d.gamma, V, chunk_states=77), ref)


# ---------------------------------------------------------------------------
# planted mistakes
# ---------------------------------------------------------------------------

def _cert_pins_pass():
    try:
        check_certificate_fixed_point_and_shift()
        check_certificate_bounds_true_error()
        check_certificate_greedy_and_uncertain()
        return True
    except AssertionError:
        return False


def _jvi_pins_pass():
    try:
        check_jvi_stay_put_exact()
        check_jvi_no_self_loops_is_vi()
        check_jvi_two_state_by_hand()
        return True
    except AssertionError:
        return False


@pytest.mark.parametrize("mistake", ["bound_1_plus_gamma", "bound_drop_gamma", "band_drop_gamma",
                                     "band_1_plus_gamma", "q_drop_gamma", "argmax_greedy", "rho_signed"])
def test_certificate_planted_mistakes(monkeypatch, mistake):
    assert _cert_pins_pass()
    real_q = O.q_values
    if mistake == "bound_1_plus_gamma":
        monkeypatch.setattr(O, "contraction_bound", lambda rho, gamma: rho / (1.0 + gamma))
    elif mistake == "bound_drop_gamma":
        monkeypatch.setattr(O, "contraction_bound", lambda rho, gamma: rho)
    elif mistake == "band_drop_gamma":
        monkeypatch.setattr(O, "tie_band", lambda rho, gamma: 2.0 * rho / (1.0 - gamma))
    elif mistake == "band_1_plus_gamma":
        monkeypatch.setattr(O, "tie_band", lambda rho, gamma: 2.0 * gamma * rho / (1.0 + gamma))
    elif mistake == "q_drop_gamma":
        monkeypatch.setattr(O, "q_values", lambda S, A, rp, c, v, g, gamma, V, rows=None:
                            real_q(S, A, rp, c, v, g, 1.0 - 1e-9, V, rows))
    elif mistake == "argmax_greedy":
        monkeypatch.setattr(O, "greedy", lambda Q, S, A: np.argmax(np.asarray(Q).reshape(S, A), 1).astype(np.int32))
    elif mistake == "rho_signed":
        real_b = O.bellman

        def signed(mdp, V, chunked=None):
            br = real_b(mdp, V)
            br.rho = float(np.max(br.r))      # max of V - TV instead of max |V - TV|
            return br
        monkeypatch.setattr(O, "bellman", signed)
    assert not _cert_pins_pass(), f"planted mistake {mistake} was not caught"


@pytest.mark.parametrize("mistake", ["diag_plus", "no_diag", "diag_of_P", "greedy_for_zero"])
def test_jvi_planted_mistakes(monkeypatch, mistake):
    assert _jvi_pins_pass()
    if mistake == "diag_plus":
        monkeypatch.setattr(O, "jacobi_diagonal", lambda P, gamma: 1.0 + gamma * P.diagonal())
    elif mistake == "no_diag":
        monkeypatch.setattr(O, "jacobi_diagonal", lambda P, gamma: np.ones(P.shape[0]))
    elif mistake == "diag_of_P":
        monkeypatch.setattr(O, "jacobi_diagonal", lambda P, gamma: np.maximum(P.diagonal(), 1e-3))
    elif mistake == "greedy_for_zero":
        real_b = O.bellman
        monkeypatch.setattr(O, "bellman", lambda mdp, V, chunked=None: real_b(mdp, np.zeros_like(V)))
    assert not _jvi_pins_pass(), f"planted mistake {mistake} was not caught"

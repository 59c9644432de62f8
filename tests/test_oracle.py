"""Pins for the CPU oracle: each check is fixed by the paper's definitions or by
mathematics, independently of the oracle's own code path.

* hand-derived fixtures (tests/golden/*.json, Sec. II equations);
* closed forms (S = 1, P_a = I, uniform rows, deterministic cycles, A = 1 via
  a Neumann series rather than an LU solve);
* brute force over every deterministic policy of tiny MDPs;
* invariants of T: fixed point, shift by constants, monotonicity, contraction;
* policy-iteration monotonicity and agreement between independent solve tiers;
* Table 2 identities of the Richardson special cases;
* planted mistakes: a wrong oracle must fail these pins.
"""
import glob
import json
import os

import numpy as np
import pytest

from oracle import ipi_oracle as O
from paper_2507_22538_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_cases():
    return sorted(glob.glob(os.path.join(GOLDEN, "*.json")))


@pytest.mark.parametrize("path", _golden_cases(), ids=os.path.basename)
def test_golden_hand_derived(path):
    case = json.load(open(path))
    d = W.from_dense(np.array(case["P"]), np.array(case["g"]), case["gamma"])
    O.validate(d.S, d.A, d.row_ptr, d.col, d.val, d.g, d.gamma)
    res = O.policy_iteration(d)
    np.testing.assert_allclose(res.V, case["V_star"], rtol=0, atol=1e-13)
    assert list(res.pi) == case["pi_star"]
    if "Q_star" in case:
        np.testing.assert_allclose(res.qgap, np.diff(np.sort(np.array(case["Q_star"]), axis=1)[:, :2]).ravel(),
                                   atol=1e-13)


# ---------------------------------------------------------------------------
# closed forms
# ---------------------------------------------------------------------------

def test_single_state():
    rng = np.random.default_rng(1)
    for A in (1, 2, 5):
        g = rng.random((1, A)) * 3 - 1
        d = W.from_dense(np.ones((1, A, 1)), g, 0.95)
        res = O.policy_iteration(d)
        assert res.V[0] == pytest.approx(g.min() / (1 - 0.95), rel=1e-14)
        assert res.pi[0] == int(np.argmin(g))


def test_identity_transitions():
    rng = np.random.default_rng(2)
    S, A, gamma = 7, 3, 0.9
    P = np.zeros((S, A, S))
    for a in range(A):
        P[:, a, :] = np.eye(S)
    g = rng.random((S, A))
    res = O.policy_iteration(W.from_dense(P, g, gamma))
    np.testing.assert_allclose(res.V, g.min(axis=1) / (1 - gamma), rtol=1e-13)
    assert np.array_equal(res.pi, np.argmin(g, axis=1))


def test_uniform_rows():
    rng = np.random.default_rng(3)
    S, A, gamma = 9, 4, 0.97
    P = np.full((S, A, S), 1.0 / S)
    g = rng.random((S, A))
    res = O.policy_iteration(W.from_dense(P, g, gamma))
    m = g.min(axis=1)
    np.testing.assert_allclose(res.V, m + gamma * m.mean() / (1 - gamma), rtol=1e-12)


@pytest.mark.parametrize("L", [1, 2, 5, 13])
def test_deterministic_cycle_equal_costs(L):
    gamma, c = 0.99, 2.5
    P = np.zeros((L, 1, L))
    for s in range(L):
        P[s, 0, (s + 1) % L] = 1.0
    res = O.policy_iteration(W.from_dense(P, np.full((L, 1), c), gamma))
    np.testing.assert_allclose(res.V, c / (1 - gamma), rtol=1e-13)


def test_single_action_neumann_series():
    """A = 1: V = sum_t gamma^t P^t g, summed until the tail is below 1e-16 relative."""
    d = W.random_sparse(300, 1, 6, 0.9, seed=5)
    res = O.policy_iteration(d)
    P, g = O.policy_matrix(d, np.zeros(d.S, dtype=np.int32))
    term = g.copy()
    total = np.zeros_like(g)
    for _ in range(2000):
        total += term
        term = d.gamma * (P @ term)
        if np.max(np.abs(term)) < 1e-17 * np.max(np.abs(total)):
            break
    np.testing.assert_allclose(res.V, total, rtol=1e-12)


# ---------------------------------------------------------------------------
# brute force
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(24))
def test_brute_force_tiny(seed):
    rng = np.random.default_rng(100 + seed)
    S = int(rng.integers(1, 9))
    A = int(rng.integers(1, 4))
    if A ** S > 7000:
        S = 6
    gamma = float(rng.choice([0.5, 0.9, 0.99]))
    d = W.tiny_random(S, A, seed, gamma)
    Vstar, optimal = O.brute_force(d)
    res = O.policy_iteration(d)
    scale = max(1.0, np.max(np.abs(Vstar)))
    np.testing.assert_allclose(res.V, Vstar, rtol=0, atol=1e-12 * scale)
    assert tuple(int(a) for a in res.pi) in set(optimal)


# ---------------------------------------------------------------------------
# invariants of T and of policy iteration
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def c1():
    return W.c1()


@pytest.fixture(scope="module")
def c1_solution(c1):
    return O.policy_iteration(c1, keep_history=True)


def test_fixed_point_and_consistency(c1, c1_solution):
    res = c1_solution
    br = O.bellman(c1, res.V)
    scale = max(1.0, np.max(np.abs(res.V)))
    assert br.rho <= 1e-12 * scale
    Vpi, _ = O.evaluate(c1, res.pi, "dense")
    np.testing.assert_allclose(Vpi, res.V, rtol=0, atol=1e-12 * scale)
    assert np.array_equal(br.pi, res.pi)


def test_policy_iteration_monotone(c1, c1_solution):
    vals = c1_solution.values
    assert len(vals) >= 2
    for a, b in zip(vals, vals[1:]):
        assert np.all(b <= a + 1e-12 * max(1.0, np.max(np.abs(a))))


def test_operator_properties(c1):
    rng = np.random.default_rng(7)
    U = rng.normal(size=c1.S) * 5
    V = rng.normal(size=c1.S) * 5
    TU = O.bellman(c1, U).TV
    TV = O.bellman(c1, V).TV
    # shift: T(V + c 1) = TV + gamma c 1 (rows of P sum to one)
    for c in (-3.0, 0.5, 11.0):
        np.testing.assert_allclose(O.bellman(c1, V + c).TV, TV + c1.gamma * c, atol=1e-12)
    # gamma-contraction in the sup norm
    assert np.max(np.abs(TU - TV)) <= c1.gamma * np.max(np.abs(U - V)) + 1e-12
    # monotone: U <= V  =>  TU <= TV
    Wv = np.minimum(U, V)
    assert np.all(O.bellman(c1, Wv).TV <= TV + 1e-12)


def test_sampled_bellman_matches_full(c1):
    rng = np.random.default_rng(8)
    V = rng.random(c1.S) * 10
    br = O.bellman(c1, V)
    states = np.sort(rng.choice(c1.S, 50, replace=False))
    TV, pi, gap, _ = O.bellman_states(c1, V, states)
    np.testing.assert_allclose(TV, br.TV[states], rtol=1e-14)
    assert np.array_equal(pi, br.pi[states])
    full = O.q_values_chunked(c1.S, c1.A, c1.row_ptr, c1.col, c1.val, c1.g, c1.gamma, V, chunk_states=97)
    np.testing.assert_allclose(full, br.Q, rtol=1e-15)


def test_tiers_agree():
    # banded chain: dense LU vs banded LU vs sparse LU
    d = W.c2(3000)
    pi = O.greedy(d.g, d.S, d.A)
    Vd, _ = O.evaluate(d, pi, "dense")
    for tier in ("banded", "splu"):
        V, used = O.evaluate(d, pi, tier)
        assert used == tier
        np.testing.assert_allclose(V, Vd, rtol=1e-11)
    # random sparse (well-conditioned Krylov spectrum): dense LU vs iterative tier
    d = W.random_sparse(2000, 3, 10, 0.99, seed=3)
    pi = O.greedy(d.g, d.S, d.A)
    Vd, _ = O.evaluate(d, pi, "dense")
    V, used = O.evaluate(d, pi, "gmres")
    np.testing.assert_allclose(V, Vd, rtol=1e-12)


def test_banded_auto_tier_large():
    d = W.c2(20_000)
    res = O.policy_iteration(d)
    assert res.tier == "banded"
    assert res.rho <= 1e-11 * np.max(np.abs(res.V))


# ---------------------------------------------------------------------------
# Table 2 identities (Richardson special cases) on hand-solvable MDPs
# ---------------------------------------------------------------------------

def test_vi_beta_opi_identities():
    rng = np.random.default_rng(9)
    S, A, gamma = 6, 3, 0.8
    P = np.zeros((S, A, S))
    for a in range(A):
        P[:, a, :] = np.eye(S)
    g = rng.random((S, A))
    d = W.from_dense(P, g, gamma)
    V0 = rng.random(S)
    m = g.min(axis=1)
    # with P_a = I: T V = min_a g + gamma V (greedy action is argmin g)
    np.testing.assert_allclose(O.vi_step(d, V0), m + gamma * V0, rtol=1e-15)
    np.testing.assert_allclose(O.beta_vi_step(d, V0, 0.3), V0 + 0.3 * (m + gamma * V0 - V0), rtol=1e-14)
    # OPI(W): T_pi^W V = m (1 - gamma^W)/(1 - gamma) + gamma^W V
    for Wn in (1, 2, 7):
        np.testing.assert_allclose(O.opi_step(d, V0, Wn),
                                   m * (1 - gamma ** Wn) / (1 - gamma) + gamma ** Wn * V0, rtol=1e-13)


# ---------------------------------------------------------------------------
# validation
# ---------------------------------------------------------------------------

def test_validation_rejects_malformed():
    d = W.random_sparse(20, 2, 3, 0.9, seed=1)
    args = dict(S=d.S, A=d.A, row_ptr=d.row_ptr, col=d.col, val=d.val, g=d.g, gamma=d.gamma)
    O.validate(**args)
    bad = []
    rp = d.row_ptr.copy(); rp[3], rp[4] = rp[4], rp[3]; bad.append(dict(args, row_ptr=rp))
    c = d.col.copy(); c[5] = d.S; bad.append(dict(args, col=c))
    v = d.val.copy(); v[0] = -v[0]; bad.append(dict(args, val=v))
    v = d.val.copy(); v[0] *= 1.5; bad.append(dict(args, val=v))
    gg = d.g.copy(); gg[2] = np.nan; bad.append(dict(args, g=gg))
    bad.append(dict(args, gamma=1.0))
    bad.append(dict(args, gamma=0.0))
    bad.append(dict(args, row_ptr=d.row_ptr[:-1]))
    for b in bad:
        with pytest.raises(O.OracleError):
            O.validate(**b)


# ---------------------------------------------------------------------------
# planted mistakes: a plausible bug in the oracle must break a pin
# ---------------------------------------------------------------------------

def _pins_pass():
    """A compact rerun of several pins; True iff all of them hold."""
    try:
        for path in _golden_cases():
            test_golden_hand_derived(path)
        test_identity_transitions()
        test_uniform_rows()
        for s in range(6):
            test_brute_force_tiny(s)
        test_single_action_neumann_series()
        return True
    except AssertionError:
        return False


@pytest.mark.parametrize("mistake", ["drop_gamma", "argmax", "transpose_action", "drop_cost", "wrong_sign_rhs"])
def test_planted_mistakes_are_caught(monkeypatch, mistake):
    assert _pins_pass()
    real_q = O.q_values
    real_eval = O.evaluate

    if mistake == "drop_gamma":
        monkeypatch.setattr(O, "q_values", lambda S, A, rp, c, v, g, gamma, V, rows=None:
                            real_q(S, A, rp, c, v, g, 1.0 - 1e-9, V, rows))
    elif mistake == "argmax":
        monkeypatch.setattr(O, "greedy", lambda Q, S, A: np.argmax(np.asarray(Q).reshape(S, A), 1).astype(np.int32))
    elif mistake == "transpose_action":
        # row index taken as a*S + s instead of s*A + a
        def bad_rows(S, A, pi):
            return np.asarray(pi, dtype=np.int64) * S + np.arange(S, dtype=np.int64)
        monkeypatch.setattr(O, "policy_rows", bad_rows)
    elif mistake == "drop_cost":
        monkeypatch.setattr(O, "q_values", lambda S, A, rp, c, v, g, gamma, V, rows=None:
                            real_q(S, A, rp, c, v, np.zeros_like(g), gamma, V, rows))
    elif mistake == "wrong_sign_rhs":
        def bad_eval(mdp, pi, tier="auto"):
            V, t = real_eval(mdp, pi, tier)
            return -V, t
        monkeypatch.setattr(O, "evaluate", bad_eval)
    try:
        ok = _pins_pass()
    except (IndexError, ValueError, O.OracleError):
        ok = False
    assert not ok, f"planted mistake {mistake} was not caught by the pins"

"""CPU FP64 oracle for inexact policy iteration (iPI) on discounted finite MDPs.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import or call this module.  It
shares no code with the GPU library (``paper_2507_22538_amd``): it receives
the same seeded input arrays and computes, plainly and slowly, what the GPU
path must reproduce.

Notation follows Sec. II of the paper:
  * MDP tuple {S, A, P, g, gamma}; P(s, s', a) row-stochastic for each
    (s, a); 0 < gamma < 1.
  * P is stored row-stacked (flattened-tensor equation, Sec. III-B.2): row
    s*A + a of the (S*A) x S matrix holds P(s, ., a).  0-based indices.
  * Bellman equation for a policy:   V_pi = g_pi + gamma P_pi V_pi.
  * Bellman optimality equation:     V* = min_pi { g_pi + gamma P_pi V* }.
  * Residuals: r(V) = V - T V and r_pi(V) = V - T_pi V.
  * Greedy policy: argmin over actions of g_pi + gamma P_pi V.

The oracle returns the plain definition of the answer: V* (the unique fixed
point of the contraction T) and a policy greedy for it, computed by exact
policy iteration (Table 2, row "PI") with a direct policy-evaluation solve.

Large MDPs (>= 2^20 nonzeros) take the Bellman products of orc_bellman.c,
plain C that sums each row in the same order as q_values and agrees with it
bit for bit (pinned in tests/test_oracle_certificate.py).

Readings of points the paper leaves open:
  * argmin ties break to the lowest action index;
  * the first policy is greedy for V = 0, i.e. argmin_a g(s, a);
  * during policy improvement the current action is kept unless another
    action is better by more than eps_sw = 1e-13 * max(1, ||V||_inf), so
    that policy iteration terminates;
  * Q-gap(s) = second-smallest minus smallest Q(s, .), +inf when A = 1.
"""
from __future__ import annotations

import ctypes
import itertools
import math
import os
from dataclasses import dataclass

import numpy as np
import scipy.linalg
import scipy.sparse
import scipy.sparse.linalg


class OracleError(ValueError):
    pass


# The same Bellman products in plain C with OpenMP (orc_bellman.c, built by
# __graft_entry__.build() into liborc.so beside this file).  It sums each row
# in the same order as q_values below and agrees with it bit for bit
# (tests/test_oracle.py); it only makes the full-size problems tractable.
_HERE = os.path.dirname(os.path.abspath(__file__))
_CLIB_PATH = os.path.join(_HERE, "liborc.so")
_clib = None


def c_library():
    """The oracle's C Bellman library, or None when it is not built."""
    global _clib
    if _clib is None and os.path.exists(_CLIB_PATH):
        lib = ctypes.CDLL(_CLIB_PATH)
        vp = ctypes.c_void_p
        lib.orc_q_values.restype = None
        lib.orc_q_values.argtypes = [ctypes.c_int64, vp, vp, vp, vp, ctypes.c_double, vp, vp, ctypes.c_int]
        lib.orc_threads.restype = ctypes.c_int
        lib.orc_threads.argtypes = []
        _clib = lib
    return _clib


def host_threads():
    """Threads the C Bellman products use (OpenMP's default on this host)."""
    lib = c_library()
    return int(lib.orc_threads()) if lib is not None else 1


# ---------------------------------------------------------------------------
# input validation (Sec. II: rows of P sum to one, gamma in (0,1))
# ---------------------------------------------------------------------------

def validate(S, A, row_ptr, col, val, g, gamma, row_sum_tol=None):
    """Raise OracleError unless {S, A, P, g, gamma} is a valid discounted MDP."""
    if S < 1 or A < 1:
        raise OracleError("S and A must be positive")
    if not (0.0 < gamma < 1.0):
        raise OracleError("gamma must lie in (0, 1)")
    R = S * A
    if len(row_ptr) != R + 1 or row_ptr[0] != 0:
        raise OracleError("row_ptr must have S*A+1 entries starting at 0")
    if np.any(np.diff(row_ptr) < 0):
        raise OracleError("row_ptr must be non-decreasing")
    nnz = int(row_ptr[-1])
    if len(col) != nnz or len(val) != nnz:
        raise OracleError("col/val length must equal row_ptr[-1]")
    if nnz and (col.min() < 0 or col.max() >= S):
        raise OracleError("column index out of range")
    if not np.all(np.isfinite(val)) or np.any(val < 0):
        raise OracleError("probabilities must be finite and non-negative")
    if len(g) != R or not np.all(np.isfinite(g)):
        raise OracleError("g must hold S*A finite costs")
    lens = np.diff(row_ptr)
    sums = row_sums(S, A, row_ptr, val)
    tol = row_sum_tol if row_sum_tol is not None else 1e-12 * np.maximum(1.0, lens)
    if np.any(np.abs(sums - 1.0) > tol):
        raise OracleError("every row of P must sum to one")


def row_sums(S, A, row_ptr, val):
    """Sum of P(s, ., a) for every row s*A + a, accumulated in column order."""
    R = S * A
    rows = np.repeat(np.arange(R), np.diff(row_ptr))
    return np.bincount(rows, weights=val, minlength=R)


# ---------------------------------------------------------------------------
# Bellman operator (Sec. II)
# ---------------------------------------------------------------------------

def q_values(S, A, row_ptr, col, val, g, gamma, V, rows=None):
    """Q(s, a) = g(s, a) + gamma * sum_{s'} P(s, s', a) V(s') for every row s*A + a.

    Each row is summed sequentially in column order (np.bincount accumulates
    in element order).  ``rows`` restricts the computation to a sorted subset
    of row indices (used for sampled checks at full size)."""
    V = np.asarray(V, dtype=np.float64)
    if rows is None:
        R = S * A
        rid = np.repeat(np.arange(R), np.diff(row_ptr))
        pv = np.bincount(rid, weights=val * V[col], minlength=R)
        return g + gamma * pv
    rows = np.asarray(rows, dtype=np.int64)
    out = np.empty(len(rows))
    for n, r in enumerate(rows):
        b, e = int(row_ptr[r]), int(row_ptr[r + 1])
        acc = 0.0
        for j in range(b, e):
            acc += float(val[j]) * float(V[col[j]])
        out[n] = g[r] + gamma * acc
    return out


def q_values_chunked(S, A, row_ptr, col, val, g, gamma, V, chunk_states=1 << 18, threads=0):
    """Same as q_values over all rows: in C (same summation order, OpenMP over
    rows) when the oracle's C library is built, else in numpy state chunks to
    bound host memory."""
    V = np.ascontiguousarray(V, dtype=np.float64)
    lib = c_library()
    if lib is not None:
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        c = np.ascontiguousarray(col, dtype=np.int32)
        v = np.ascontiguousarray(val, dtype=np.float64)
        gg = np.ascontiguousarray(g, dtype=np.float64)
        out = np.empty(S * A)
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        lib.orc_q_values(S * A, p(rp), p(c), p(v), p(gg), float(gamma), p(V), p(out), int(threads))
        return out
    return q_values_numpy_chunked(S, A, row_ptr, col, val, g, gamma, V, chunk_states)


def q_values_numpy_chunked(S, A, row_ptr, col, val, g, gamma, V, chunk_states=1 << 18):
    """q_values over all rows in numpy, one chunk of states at a time."""
    out = np.empty(S * A)
    for s0 in range(0, S, chunk_states):
        s1 = min(S, s0 + chunk_states)
        r0, r1 = s0 * A, s1 * A
        b, e = int(row_ptr[r0]), int(row_ptr[r1])
        lens = np.diff(row_ptr[r0:r1 + 1])
        rid = np.repeat(np.arange(r1 - r0), lens)
        pv = np.bincount(rid, weights=val[b:e] * V[col[b:e]], minlength=r1 - r0)
        out[r0:r1] = g[r0:r1] + gamma * pv
    return out


# MDPs with at least this many nonzeros take the C products (bit-identical to
# q_values); smaller ones, and every planted-mistake check, run q_values itself
C_MIN_NNZ = 1 << 20


def q_all(mdp, V):
    """Q(s, a) for every row of the MDP (q_values, or its C twin on large MDPs)."""
    if mdp.nnz >= C_MIN_NNZ:
        return q_values_chunked(mdp.S, mdp.A, mdp.row_ptr, mdp.col, mdp.val, mdp.g, mdp.gamma, V)
    return q_values(mdp.S, mdp.A, mdp.row_ptr, mdp.col, mdp.val, mdp.g, mdp.gamma, V)


def greedy(Q, S, A):
    """Lowest-index argmin over actions of Q reshaped to S x A (greedy-policy equation)."""
    return np.argmin(np.asarray(Q).reshape(S, A), axis=1).astype(np.int32)


def q_gap(Q, S, A):
    """Second-smallest minus smallest Q(s, .); +inf when A == 1."""
    Qm = np.asarray(Q).reshape(S, A)
    if A == 1:
        return np.full(S, np.inf)
    part = np.partition(Qm, 1, axis=1)
    return part[:, 1] - part[:, 0]


@dataclass
class BellmanResult:
    TV: np.ndarray      # (T V)(s) = min_a Q(s, a)
    pi: np.ndarray      # lowest-index greedy action
    r: np.ndarray       # r(V) = V - T V   (paper's sign)
    rho: float          # ||r(V)||_inf
    Q: np.ndarray


def bellman(mdp, V, chunked=None):
    """T V, the greedy policy and the residual r(V) = V - TV (Sec. II).
    ``chunked`` is accepted for older callers; large MDPs always take the C
    products (bit-identical)."""
    S, A = mdp.S, mdp.A
    Q = q_all(mdp, V)
    Qm = Q.reshape(S, A)
    pi = greedy(Q, S, A)
    TV = Qm[np.arange(S), pi]
    r = np.asarray(V, dtype=np.float64) - TV
    rho = float(np.max(np.abs(r))) if S else 0.0
    return BellmanResult(TV, pi, r, rho, Q)


def bellman_states(mdp, V, states):
    """T V, greedy action and Q-gap at a sorted list of states only (one by one)."""
    S, A = mdp.S, mdp.A
    states = np.asarray(states, dtype=np.int64)
    rows = (states[:, None] * A + np.arange(A)[None, :]).reshape(-1)
    Q = q_values(S, A, mdp.row_ptr, mdp.col, mdp.val, mdp.g, mdp.gamma, V, rows=rows).reshape(-1, A)
    pi = np.argmin(Q, axis=1).astype(np.int32)
    TV = Q[np.arange(len(states)), pi]
    gap = np.full(len(states), np.inf) if A == 1 else np.diff(np.sort(Q, axis=1)[:, :2], axis=1)[:, 0]
    return TV, pi, gap, Q


# ---------------------------------------------------------------------------
# policy operator and policy evaluation (Bellman equation for a policy)
# ---------------------------------------------------------------------------

def policy_rows(S, A, pi):
    return np.arange(S, dtype=np.int64) * A + np.asarray(pi, dtype=np.int64)


def policy_matrix(mdp, pi):
    """P_pi (scipy CSR, S x S) and g_pi: row s is row s*A + pi(s) of P."""
    S, A = mdp.S, mdp.A
    rows = policy_rows(S, A, pi)
    starts = mdp.row_ptr[rows]
    lens = mdp.row_ptr[rows + 1] - starts
    rp = np.zeros(S + 1, dtype=np.int64)
    np.cumsum(lens, out=rp[1:])
    # entry t of row s of P_pi is entry starts[s] + (t - rp[s]) of P
    idx = np.repeat(starts - rp[:-1], lens) + np.arange(int(rp[-1]), dtype=np.int64)
    P = scipy.sparse.csr_matrix((mdp.val[idx], mdp.col[idx], rp), shape=(S, S))
    return P, mdp.g[rows].copy()


def _bandwidths(P):
    coo = P.tocoo()
    if coo.nnz == 0:
        return 0, 0
    d = coo.col.astype(np.int64) - coo.row.astype(np.int64)
    return int(max(0, -d.min())), int(max(0, d.max()))


def evaluate(mdp, pi, tier="auto"):
    """Solve (I - gamma P_pi) V = g_pi directly.  Returns (V_pi, tier used).

    Tiers: "banded" (banded LU when the bandwidth is at most 256), "dense"
    (LU with partial pivoting, S <= 1024), "splu" (sparse LU, S <= 2e5),
    "gmres" (iterative
    FP64 GMRES to 1e-14 relative plus two refinement steps against the exact
    sparse matrix; labelled iterative)."""
    S = mdp.S
    P, gpi = policy_matrix(mdp, pi)
    J = scipy.sparse.identity(S, format="csr") - mdp.gamma * P
    if tier == "auto":
        lo, hi = _bandwidths(P)
        if lo + hi + 1 <= 256 and S > 64:
            tier = "banded"
        elif S <= 1024:
            tier = "dense"
        elif S <= 200_000:
            tier = "splu"
        else:
            tier = "gmres"
    if tier == "dense":
        V = np.linalg.solve(J.toarray(), gpi)
    elif tier == "banded":
        lo, hi = _bandwidths(J)
        ab = np.zeros((lo + hi + 1, S))
        coo = J.tocoo()
        coo.sum_duplicates()
        # ab[hi + i - j, j] = J[i, j] (one entry per (i, j) after summing duplicates)
        ab[hi + coo.row - coo.col, coo.col] = coo.data
        V = scipy.linalg.solve_banded((lo, hi), ab, gpi)
    elif tier == "splu":
        V = scipy.sparse.linalg.splu(J.tocsc()).solve(gpi)
    elif tier == "gmres":
        V = np.zeros(S)
        for _ in range(3):  # solve, then two refinement steps on the exact residual
            res = gpi - J @ V
            nb = np.linalg.norm(gpi)
            if np.linalg.norm(res) <= 1e-15 * nb:
                break
            d, info = scipy.sparse.linalg.gmres(J, res, rtol=1e-14, atol=0.0, restart=100,
                                                maxiter=10000)
            V = V + d
    else:
        raise OracleError(f"unknown tier {tier}")
    return V, tier


# ---------------------------------------------------------------------------
# exact policy iteration (Table 2, row "PI")
# ---------------------------------------------------------------------------

@dataclass
class PIResult:
    V: np.ndarray        # V* = V_{pi*}
    pi: np.ndarray       # lowest-index greedy policy for V*
    qgap: np.ndarray     # Q-gap at V*
    rho: float           # ||V* - T V*||_inf
    iters: int           # number of policy evaluations
    tier: str
    policies: list       # the policy sequence pi_0, pi_1, ...
    values: list         # the value sequence V_{pi_0}, V_{pi_1}, ...


def policy_iteration(mdp, tier="auto", max_iter=10_000, keep_history=False):
    """Exact policy iteration with a direct evaluation solve.

    pi_0 = argmin_a g(s, a) (greedy for V = 0).  Each step evaluates V_pi
    exactly, then improves: pi'(s) keeps pi(s) unless some action is better
    by more than eps_sw.  Stops when pi' == pi."""
    S, A = mdp.S, mdp.A
    pi = greedy(mdp.g, S, A)
    history_p, history_v = [], []
    used = None
    for it in range(1, max_iter + 1):
        V, used = evaluate(mdp, pi, tier)
        if keep_history:
            history_p.append(pi.copy())
            history_v.append(V.copy())
        Q = q_all(mdp, V).reshape(S, A)
        eps_sw = 1e-13 * max(1.0, float(np.max(np.abs(V))) if S else 1.0)
        best = np.argmin(Q, axis=1)
        q_cur = Q[np.arange(S), pi]
        switch = Q[np.arange(S), best] < q_cur - eps_sw
        new_pi = np.where(switch, best, pi).astype(np.int32)
        if np.array_equal(new_pi, pi):
            Qf = Q.reshape(-1)
            return PIResult(V, greedy(Qf, S, A), q_gap(Qf, S, A),
                            float(np.max(np.abs(V - Q.min(axis=1)))), it, used,
                            history_p, history_v)
        pi = new_pi
    raise OracleError("policy iteration did not terminate")


# ---------------------------------------------------------------------------
# brute force over all deterministic policies (tiny MDPs)
# ---------------------------------------------------------------------------

def brute_force(mdp, tol=1e-12):
    """V*(s) = min over all A^S deterministic policies of V_pi(s); also the set of
    optimal policies (those whose V_pi is within tol of V* everywhere)."""
    S, A = mdp.S, mdp.A
    if A ** S > 100_000:
        raise OracleError("brute force limited to A^S <= 1e5")
    allv = {}
    for pol in itertools.product(range(A), repeat=S):
        pi = np.array(pol, dtype=np.int32)
        V, _ = evaluate(mdp, pi, "dense")
        allv[pol] = V
    Vstar = np.min(np.stack(list(allv.values())), axis=0)
    scale = max(1.0, float(np.max(np.abs(Vstar))))
    optimal = [p for p, V in allv.items() if np.max(np.abs(V - Vstar)) <= tol * scale]
    return Vstar, optimal


# ---------------------------------------------------------------------------
# certificate (residual bound from the contraction property of T)
# ---------------------------------------------------------------------------

@dataclass
class Certificate:
    rho: float           # ||V - T V||_inf recomputed on the CPU
    bound: float         # ||V - V*||_inf <= rho / (1 - gamma)
    greedy_ok: bool      # the given policy attains min_a Q(s, a) within the tie band
    uncertain: int       # states whose Q-gap is below 2*gamma*rho/(1-gamma)


def contraction_bound(rho, gamma):
    """||V - V*||_inf <= ||V - T V||_inf / (1 - gamma).

    T is a gamma-contraction in the sup norm (Sec. II), so
    ||V - V*|| <= ||V - TV|| + ||TV - TV*|| <= rho + gamma ||V - V*||."""
    return rho / (1.0 - gamma)


def tie_band(rho, gamma):
    """Q-gap below which a state's greedy action for V may differ from the one for V*.

    |Q_V(s, a) - Q_V*(s, a)| <= gamma ||V - V*||_inf <= gamma rho / (1 - gamma)
    for every action, so the order of two actions can flip only when their
    gap is below twice that."""
    return 2.0 * gamma * rho / (1.0 - gamma)


def certificate(mdp, V, pi=None, tie_tol=None):
    """Check a candidate V (and policy) without knowing V*: the residual
    r(V) = V - TV of Sec. II, the contraction bound on ||V - V*||_inf, whether
    pi is greedy for V (within tie_tol, default 1e-12 max(1, ||V||_inf)), and
    how many states have a Q-gap inside the tie band."""
    br = bellman(mdp, V)
    bound = contraction_bound(br.rho, mdp.gamma)
    greedy_ok = True
    uncertain = 0
    if pi is not None:
        Qm = br.Q.reshape(mdp.S, mdp.A)
        qpi = Qm[np.arange(mdp.S), np.asarray(pi, dtype=np.int64)]
        tt = tie_tol if tie_tol is not None else 1e-12 * max(1.0, float(np.max(np.abs(V))))
        greedy_ok = bool(np.all(qpi - br.TV <= tt))
        gap = q_gap(br.Q, mdp.S, mdp.A)
        uncertain = int(np.sum(gap < tie_band(br.rho, mdp.gamma)))
    return Certificate(br.rho, bound, greedy_ok, uncertain)


# ---------------------------------------------------------------------------
# dynamic-programming special cases of iPI (Table 2) for identity checks
# ---------------------------------------------------------------------------

def vi_step(mdp, V):
    """Value iteration: V_{k+1} = T V_k (Richardson, one sweep, scale 1)."""
    return bellman(mdp, V).TV


def beta_vi_step(mdp, V, beta):
    """beta-VI: V_{k+1} = V_k + beta (T V_k - V_k) (Richardson, one sweep, scale beta)."""
    return np.asarray(V) + beta * (bellman(mdp, V).TV - np.asarray(V))


def opi_step(mdp, V, W):
    """OPI(W): V_{k+1} = T_pi^W V_k with pi greedy for V_k (Richardson, W sweeps)."""
    pi = bellman(mdp, V).pi
    P, gpi = policy_matrix(mdp, pi)
    x = np.asarray(V, dtype=np.float64).copy()
    for _ in range(W):
        x = gpi + mdp.gamma * (P @ x)
    return x


def jacobi_diagonal(P_pi, gamma):
    """D = diag(J_pi) = diag(I - gamma P_pi): D(s) = 1 - gamma P(s, s, pi(s))."""
    return 1.0 - gamma * P_pi.diagonal()


def jvi_step(mdp, V, omega=1.0):
    """J-VI (Table 2: Richardson with the Jacobi preconditioner, one sweep):
    from theta_0 = V_k with pi greedy for V_k (Algorithm 1 steps 2-5),
    V_{k+1} = V_k + omega D^-1 (g_pi - J_pi V_k), where J_pi = I - gamma P_pi
    and D = diag(J_pi)."""
    V = np.asarray(V, dtype=np.float64)
    pi = bellman(mdp, V).pi
    P, gpi = policy_matrix(mdp, pi)
    D = jacobi_diagonal(P, mdp.gamma)
    lin_resid = gpi - (V - mdp.gamma * (P @ V))
    return V + omega * lin_resid / D


def parity_tau(Vstar):
    """Scale-aware tie band tau = 1e-10 * max(1, ||V*||_inf)."""
    return 1e-10 * max(1.0, float(np.max(np.abs(Vstar))) if len(Vstar) else 1.0)


# ---------------------------------------------------------------------------
# Values held as two float32 parts (the hi + lo storage of the precision
# modes).  The paper's solver keeps every value in double precision; this
# is a storage form of the same P, so its oracle is the plain definition.
# ---------------------------------------------------------------------------

def split_values(val):
    """hi = float32(P), rounded to nearest; lo = float32(P - hi), where the
    difference P - hi is taken in float64 (exact: hi is the float32 nearest
    P, so the difference needs at most 29 significant bits)."""
    val = np.asarray(val, dtype=np.float64)
    hi = val.astype(np.float32)
    lo = (val - hi.astype(np.float64)).astype(np.float32)
    return hi, lo


def split_effective(val):
    """The value the split form stands for: hi + lo, both widened exactly
    to float64 and added once in float64."""
    hi, lo = split_values(val)
    return hi.astype(np.float64) + lo.astype(np.float64)


def split_row_perturbation(S, A, row_ptr, val):
    """max over rows of sum_j |P_rj - (hi_rj + lo_rj)|, every term in float64."""
    d = np.abs(np.asarray(val, dtype=np.float64) - split_effective(val))
    rows = np.repeat(np.arange(S * A), np.diff(np.asarray(row_ptr, dtype=np.int64)))
    return float(np.max(np.bincount(rows, weights=d, minlength=S * A))) if len(d) else 0.0

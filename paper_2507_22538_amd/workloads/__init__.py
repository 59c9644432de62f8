"""Seeded synthetic MDP inputs shared by the oracle tests, the GPU tests and bench.py.

This module produces inputs only (the row-stacked CSR tensor P of the
flattened-tensor equation in Sec. III-B.2, the stage-cost matrix g and the
discount gamma).  It contains none of the method's arithmetic.  Bulk arrays
come from ``gen.c`` (compiled to ``libipigen.so`` by ``__graft_entry__.build``);
small hand-built MDPs for closed-form checks are plain numpy here.

Every MDP is returned as a :class:`MDPData`.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBNAME = os.path.join(_HERE, "libipigen.so")
_lib = None

MASK64 = (1 << 64) - 1


@dataclass
class MDPData:
    """A discounted MDP {S, A, P, g, gamma} in row-stacked CSR form (row = s*A + a)."""

    S: int
    A: int
    row_ptr: np.ndarray  # int64[S*A+1]
    col: np.ndarray  # int32[nnz]
    val: np.ndarray  # float64[nnz]
    g: np.ndarray  # float64[S*A]
    gamma: float
    name: str = "mdp"
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def fp32_rounded(self) -> "MDPData":
        """Same MDP with P values rounded to float32 (the exact target of the mixed mode)."""
        return MDPData(self.S, self.A, self.row_ptr, self.col,
                       self.val.astype(np.float32).astype(np.float64), self.g,
                       self.gamma, self.name + "-f32P", dict(self.meta))


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBNAME):
            raise RuntimeError(f"{_LIBNAME} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(_LIBNAME)
        i64, i32, u64, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double
        vp = ctypes.c_void_p
        lib.ipigen_key.restype = u64
        lib.ipigen_key.argtypes = [u64, u64, u64, u64]
        lib.ipigen_random_rowptr.restype = i64
        lib.ipigen_random_rowptr.argtypes = [i64, i32, i32, i32, u64, u64, vp]
        lib.ipigen_random_fill.restype = None
        lib.ipigen_random_fill.argtypes = [i64, i32, u64, u64, vp, vp, vp, vp]
        lib.ipigen_birth_death.restype = None
        lib.ipigen_birth_death.argtypes = [i64, i32, u64, vp, vp, vp, vp]
        lib.ipigen_pendulum.restype = None
        lib.ipigen_pendulum.argtypes = [i64, i32, dbl, dbl, dbl, vp, vp, vp, vp]
        lib.ipigen_maze.restype = None
        lib.ipigen_maze.argtypes = [i64, i64, dbl, dbl, u64, vp, vp, vp, vp, vp]
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------------------
# counter-based hash (same definition as gen.c; used for per-MDP parameters)
# ---------------------------------------------------------------------------

def _sm64(z: int) -> int:
    z = (z + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def key(seed: int, mdp: int, row: int, j: int) -> int:
    return _sm64(_sm64(_sm64(_sm64(seed & MASK64) ^ (mdp & MASK64)) ^ (row & MASK64)) ^ (j & MASK64))


def u01(x: int) -> float:
    return (x >> 11) * (1.0 / 9007199254740992.0)


def uint_below(x: int, n: int) -> int:
    return (x * n) >> 64


# ---------------------------------------------------------------------------
# generators
# ---------------------------------------------------------------------------

def random_sparse(S: int, A: int, k: int, gamma: float, seed: int = 0, mdp: int = 0,
                  k_hi: int | None = None, name: str | None = None) -> MDPData:
    """Random sparse MDP: k distinct uniform columns per row (k uniform in
    [k, k_hi] per row when k_hi is given), Dirichlet(1) probabilities, g ~ U[0,1)."""
    k_lo = int(k)
    k_hi = int(k if k_hi is None else k_hi)
    if not (1 <= k_lo <= k_hi <= S):
        raise ValueError("need 1 <= k <= k_hi <= S")
    lib = _load()
    R = S * A
    row_ptr = np.empty(R + 1, dtype=np.int64)
    nnz = lib.ipigen_random_rowptr(S, A, k_lo, k_hi, seed, mdp, _p(row_ptr))
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    g = np.empty(R, dtype=np.float64)
    lib.ipigen_random_fill(S, A, seed, mdp, _p(row_ptr), _p(col), _p(val), _p(g))
    return MDPData(S, A, row_ptr, col, val, g, float(gamma),
                   name or f"random_S{S}_A{A}_k{k_lo}-{k_hi}_seed{seed}_mdp{mdp}",
                   {"k_lo": k_lo, "k_hi": k_hi, "seed": seed, "mdp": mdp})


def birth_death(S: int, A: int = 16, gamma: float = 0.999, seed: int = 0) -> MDPData:
    """Banded birth-death chain shaped like the SIS study: 24 nonzeros per row."""
    if S < 24:
        raise ValueError("birth_death needs S >= 24")
    lib = _load()
    R = S * A
    nnz = R * 24
    row_ptr = np.empty(R + 1, dtype=np.int64)
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    g = np.empty(R, dtype=np.float64)
    lib.ipigen_birth_death(S, A, seed, _p(row_ptr), _p(col), _p(val), _p(g))
    return MDPData(S, A, row_ptr, col, val, g, float(gamma), f"birth_death_S{S}_A{A}_seed{seed}",
                   {"k": 24, "seed": seed, "half_band": 23})


def pendulum(N: int, A: int = 11, gamma: float = 0.9999, fmin: float = -2.0, fmax: float = 2.0,
             Ts: float = 0.01) -> MDPData:
    """Discretised inverted pendulum on an N x N (angle, velocity) grid: 4 nonzeros per row."""
    if N < 2:
        raise ValueError("pendulum needs N >= 2")
    lib = _load()
    S = N * N
    R = S * A
    nnz = R * 4
    row_ptr = np.empty(R + 1, dtype=np.int64)
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    g = np.empty(R, dtype=np.float64)
    lib.ipigen_pendulum(N, A, fmin, fmax, Ts, _p(row_ptr), _p(col), _p(val), _p(g))
    return MDPData(S, A, row_ptr, col, val, g, float(gamma), f"pendulum_N{N}_A{A}",
                   {"N": N, "k": 4})


def maze(H: int, W: int, wall_frac: float = 0.2, wall_cost: float = 1e20, gamma: float = 0.99,
         seed: int = 0) -> MDPData:
    """Deterministic H x W grid world, A = 5 (stay, N, E, S, W), one nonzero per row."""
    lib = _load()
    S = H * W
    R = S * 5
    row_ptr = np.empty(R + 1, dtype=np.int64)
    col = np.empty(R, dtype=np.int32)
    val = np.empty(R, dtype=np.float64)
    g = np.empty(R, dtype=np.float64)
    wall = np.empty(S, dtype=np.uint8)
    lib.ipigen_maze(H, W, wall_frac, wall_cost, seed, _p(row_ptr), _p(col), _p(val), _p(g), _p(wall))
    return MDPData(S, 5, row_ptr, col, val, g, float(gamma), f"maze_{H}x{W}_seed{seed}",
                   {"H": H, "W": W, "wall": wall})


def lazy_random(S: int, A: int, k: int, gamma: float, seed: int = 0, stay_lo: float = 0.3,
                stay_hi: float = 0.9) -> MDPData:
    """Random sparse MDP with heavy self-loops: row s*A + a of random_sparse
    mixed with staying in s, P' = p e_s + (1 - p) P_row, p ~ U[stay_lo, stay_hi)
    per row (seeded numpy draws).  Columns stay sorted and distinct; a row
    whose columns already held s adds p to that entry."""
    import scipy.sparse
    base = random_sparse(S, A, k, gamma, seed=seed, mdp=77)
    R = S * A
    p = np.random.default_rng(seed + 7919).uniform(stay_lo, stay_hi, size=R)
    lens = np.diff(base.row_ptr)
    rows = np.repeat(np.arange(R, dtype=np.int64), lens)
    r_all = np.concatenate([rows, np.arange(R, dtype=np.int64)])
    c_all = np.concatenate([base.col.astype(np.int64), np.arange(R, dtype=np.int64) // A])
    v_all = np.concatenate([base.val * (1.0 - p[rows]), p])
    M = scipy.sparse.csr_matrix((v_all, (r_all, c_all)), shape=(R, S))
    M.sum_duplicates()
    M.sort_indices()
    return MDPData(S, A, M.indptr.astype(np.int64), M.indices.astype(np.int32), M.data.astype(np.float64),
                   base.g, float(gamma), f"lazy_random_S{S}_A{A}_k{k}_seed{seed}",
                   {"k": k, "seed": seed, "stay": (stay_lo, stay_hi)})


# ---------------------------------------------------------------------------
# the named workloads
# ---------------------------------------------------------------------------

def amdahl(S: int = 100_000, A: int = 100, k: int = 150, gamma: float = 0.69) -> MDPData:
    """The random MDP of the paper's parallel-efficiency study (Sec. IV-A):
    100,000 states, 100 actions, 150 reachable states per (s, a) (1.5e9
    nonzeros), uniform costs and probabilities, gamma = 0.69."""
    return random_sparse(S, A, k, gamma, seed=0, mdp=7, name=f"amdahl_S{S}_A{A}_k{k}")


def c1() -> MDPData:
    """Plain FP64 random sparse MDP: S=1000, A=4, k=8, gamma=0.99, seed 0."""
    d = random_sparse(1000, 4, 8, 0.99, seed=0, mdp=0, name="c1_random_S1000_A4_k8")
    d.meta.update(tol=1e-10, alpha=0.1)
    return d


def c2(S: int = 2_000_000, A: int = 16) -> MDPData:
    """Epidemic-shaped birth-death MDP: S=2e6, A=16, k=24 banded, gamma=0.999."""
    d = birth_death(S, A, 0.999, seed=0)
    d.name = f"c2_birth_death_S{S}_A{A}"
    return d


def c3(N: int = 2048) -> MDPData:
    """Discretised pendulum: N x N grid, A=11 torques in [-2,2], 4 nnz/row, gamma=0.9999."""
    d = pendulum(N, 11, 0.9999, -2.0, 2.0, 0.01)
    d.name = f"c3_pendulum_N{N}"
    return d


GAMMAS_C4 = (0.9, 0.99, 0.999)


def c4_params(i: int, seed: int = 0) -> dict:
    """Shape of batch member i: S log-uniform on [2e3, 2e5], A in {4..16}, k in {4..32}."""
    lo, hi = math.log(2e3), math.log(2e5)
    S = int(round(math.exp(lo + (hi - lo) * u01(key(seed, i, MASK64, 1)))))
    A = 4 + uint_below(key(seed, i, MASK64, 2), 13)
    k = 4 + uint_below(key(seed, i, MASK64, 3), 29)
    gamma = GAMMAS_C4[uint_below(key(seed, i, MASK64, 4), 3)]
    return {"S": S, "A": int(A), "k": int(k), "gamma": gamma, "mdp": i, "seed": seed}


def c4_member(i: int, seed: int = 0, scale: float = 1.0) -> MDPData:
    p = c4_params(i, seed)
    S = max(p["k"], int(p["S"] * scale))
    return random_sparse(S, p["A"], p["k"], p["gamma"], seed=seed, mdp=1000 + i,
                         name=f"c4_member{i}_S{S}_A{p['A']}_k{p['k']}")


def c5_params(i: int, seed: int = 0, s_max: float = 5e6) -> dict:
    """Serving request i: S log-uniform on [1e3, s_max], A in {4..32}, k in {8..32},
    1-gamma log-uniform on [1e-4, 5e-2]."""
    lo, hi = math.log(1e3), math.log(s_max)
    S = int(round(math.exp(lo + (hi - lo) * u01(key(seed, i, MASK64, 11)))))
    A = 4 + uint_below(key(seed, i, MASK64, 12), 29)
    k = 8 + uint_below(key(seed, i, MASK64, 13), 25)
    l1, l2 = math.log(1e-4), math.log(5e-2)
    one_m_gamma = math.exp(l1 + (l2 - l1) * u01(key(seed, i, MASK64, 14)))
    return {"S": S, "A": int(A), "k": int(k), "gamma": 1.0 - one_m_gamma, "mdp": i, "seed": seed}


def c5_request(i: int, seed: int = 0, s_max: float = 5e6) -> MDPData:
    p = c5_params(i, seed, s_max)
    S = max(p["k"], p["S"])
    return random_sparse(S, p["A"], p["k"], p["gamma"], seed=seed, mdp=500000 + i,
                         name=f"c5_req{i}_S{S}_A{p['A']}_k{p['k']}")


# ---------------------------------------------------------------------------
# small hand-built MDPs (closed-form cases)
# ---------------------------------------------------------------------------

def from_dense(P: np.ndarray, g: np.ndarray, gamma: float, name: str = "dense", keep_zeros=False) -> MDPData:
    """Build CSR from a dense tensor P[s, a, s'] and costs g[s, a]."""
    P = np.asarray(P, dtype=np.float64)
    S, A, S2 = P.shape
    assert S == S2
    flat = P.reshape(S * A, S)
    row_ptr = np.zeros(S * A + 1, dtype=np.int64)
    cols, vals = [], []
    for r in range(S * A):
        nzc = np.arange(S) if keep_zeros else np.nonzero(flat[r])[0]
        cols.append(nzc.astype(np.int32))
        vals.append(flat[r, nzc])
        row_ptr[r + 1] = row_ptr[r] + len(nzc)
    col = np.concatenate(cols) if cols else np.zeros(0, np.int32)
    val = np.concatenate(vals) if vals else np.zeros(0)
    return MDPData(S, A, row_ptr, col.astype(np.int32), val.astype(np.float64),
                   np.asarray(g, dtype=np.float64).reshape(S * A), float(gamma), name)


def tiny_random(S: int, A: int, seed: int, gamma: float = 0.9, density: float = 0.6) -> MDPData:
    """Small random MDP with random sparsity (each row keeps >= 1 entry), for brute force."""
    rng = np.random.default_rng(seed)
    P = rng.random((S, A, S)) * (rng.random((S, A, S)) < density)
    for s in range(S):
        for a in range(A):
            if P[s, a].sum() == 0:
                P[s, a, rng.integers(S)] = 1.0
    P /= P.sum(axis=2, keepdims=True)
    g = rng.random((S, A)) * 2.0 - 0.5
    return from_dense(P, g, gamma, f"tiny_S{S}_A{A}_seed{seed}")

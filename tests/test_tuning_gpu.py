"""Launch-shape knobs of the two streaming kernels against the CPU oracle.

* Bellman pass: every admissible flat chunk width and several tile sizes give
  the FP64 definition within the rounding bound (the chunking only changes
  the order of the k products of a row).
* P_pi products: workgroup tiles and wave tiles form the same sums in the
  same order, so OPI(W) steps (Table 2) agree bit for bit across schedules
  and tile sizes, and with the oracle's own OPI step within rounding.
* Autotuner: the chosen shape is admissible, is written to and read back from
  the cache file, and the solve with it stays at parity.
"""
import json

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


def _bellman_check(d, V, TV, pi, resid, rho, fp32):
    ref = d.fp32_rounded() if fp32 else d
    br = O.bellman(ref, V)
    kmax = int(np.max(np.diff(d.row_ptr)))
    tol = 4 * (kmax + 2) * 2.0 ** -52 * (float(np.max(np.abs(d.g))) + d.gamma * float(np.max(np.abs(V))) + 1.0)
    np.testing.assert_allclose(TV, br.TV, rtol=0, atol=tol)
    gap = O.q_gap(br.Q, d.S, d.A)
    assert not ((pi != br.pi) & (gap > 2 * tol)).any()
    np.testing.assert_array_equal(resid, TV - V)
    assert rho == np.max(np.abs(TV - V))


UNIFORM = [
    ("birth_death_4096_k24", lambda: W.c2(4096)),
    ("random_S3001_A5_k32", lambda: W.random_sparse(3001, 5, 32, 0.99, seed=31)),
    ("pendulum_40_k4", lambda: W.c3(40)),
]


@pytest.mark.parametrize("name,make", UNIFORM, ids=[u[0] for u in UNIFORM])
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32mixed"])
def test_bellman_chunk_widths(name, make, precision):
    ipi = _ipi()
    dev = _dev()
    d = make()
    k = int(d.row_ptr[1] - d.row_ptr[0])
    V = np.random.default_rng(7).normal(size=d.S) * 5.0
    m = ipi.MDP.from_data(d, flags=ipi.IPI_VAL_FP32)
    try:
        ran = 0
        for chunk in (2, 4, 8, 12, 16, 24, 32):
            if k % chunk or (precision == 1 and chunk % 4):
                continue
            outs = []
            # -3: wave tiles for 16-byte chunks (else workgroup tiles); -2: workgroup tiles
            for lanes in (-1, -3, -2):
                for spt in (0, 1, 5, 32):
                    m.set_tuning(bellman_lanes=lanes, bellman_states_per_tile=spt, bellman_chunk=chunk)
                    TV, pi, resid, rho = m.bellman(torch.from_numpy(V).to(dev), precision)
                    torch.cuda.synchronize()
                    _bellman_check(d, V, TV.cpu().numpy(), pi.cpu().numpy(), resid.cpu().numpy(),
                                   float(rho.cpu()[0]), precision == 1)
                    outs.append((TV.cpu(), pi.cpu(), float(rho.cpu()[0])))
                    ran += 1
            # every tile shape and both schedules form the same sums in the same order
            for o in outs[1:]:
                assert torch.equal(o[0], outs[0][0]) and torch.equal(o[1], outs[0][1]) and o[2] == outs[0][2]
        assert ran > 0
    finally:
        m.close()


@pytest.mark.parametrize("name,make", UNIFORM, ids=[u[0] for u in UNIFORM])
@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_product_schedules_identical(name, make, precision):
    ipi = _ipi()
    dev = _dev()
    d = make()
    k = int(d.row_ptr[1] - d.row_ptr[0])
    v0 = np.random.default_rng(11).normal(size=d.S)
    Wn = 4
    m = ipi.MDP.from_data(d, flags=ipi.IPI_VAL_FP32)
    outs = {}
    try:
        for chunk in (2, 4, 8):
            if k % chunk or (precision == "fp32_mixed" and chunk % 4):
                continue
            cpr = k // chunk
            shapes = [(1, 0), (1, 64), (1, 257)] + [(2, w) for w in (1, 7, 16, 64) if w * cpr <= 1024]
            for sched, spt in shapes:
                m.set_tuning(spmv_lanes=-1, spmv_chunk=chunk, spmv_schedule=sched, spmv_states_per_tile=spt)
                V, pi, info, st = m.solve(device=dev, v0=torch.from_numpy(v0).to(dev), max_outer=1,
                                          ksp_type="richardson", max_inner=Wn, alpha=1e-15, precision=precision)
                torch.cuda.synchronize()
                assert info["inner_iters"] == Wn
                outs[(chunk, sched, spt)] = V.cpu().numpy()
    finally:
        m.close()
    assert outs
    ref = d.fp32_rounded() if precision == "fp32_mixed" else d
    want = O.opi_step(ref, v0, Wn)
    by_chunk = {}
    for (chunk, sched, spt), V in outs.items():
        np.testing.assert_allclose(V, want, rtol=0, atol=1e-11 * max(1.0, np.max(np.abs(want))))
        first = by_chunk.setdefault(chunk, V)
        np.testing.assert_array_equal(V, first, err_msg=f"chunk {chunk} schedule {sched} spt {spt}")


def test_autotune_cache_roundtrip(tmp_path):
    ipi = _ipi()
    dev = _dev()
    d = W.c2(20000)
    ref = O.policy_iteration(d)
    cache = tmp_path / "tune.json"
    m = ipi.MDP.from_data(d, flags=ipi.IPI_VAL_FP32)
    try:
        ipi.ipi_autotune(m.handle, ipi.IPI_FP64, str(cache))
        torch.cuda.synchronize()
        t1 = ipi.ipi_get_tuning(m.handle)
        assert t1["bellman_lanes"] != 0 and t1["spmv_lanes"] != 0
        data = json.loads(cache.read_text())
        assert len(data) == 1 and len(next(iter(data.values()))) == 7
        V, pi, info, st = m.solve(device=dev, atol=0.0, rtol_cert=1e-12, alpha=0.1, ksp_type="richardson",
                                  max_inner=100000)
        torch.cuda.synchronize()
        assert st == ipi.IPI_OK
        err = np.max(np.abs(V.cpu().numpy() - ref.V)) / np.max(np.abs(ref.V))
        assert err <= 1e-8
    finally:
        m.close()
    # a second MDP of the same shape class takes the cached shape without
    # timing, and keeps the settings the cache does not hold
    shapes = ("bellman_lanes", "bellman_states_per_tile", "spmv_lanes", "spmv_states_per_tile", "bellman_chunk",
              "spmv_chunk", "spmv_schedule")
    m2 = ipi.MDP.from_data(W.c2(20000), flags=ipi.IPI_VAL_FP32)
    try:
        ipi.ipi_autotune(m2.handle, ipi.IPI_FP64, str(cache))
        assert ipi.ipi_get_tuning(m2.handle) == t1
        m2.set_tuning(ppi_cached=-1, spmv_workgroups=64)
        ipi.ipi_autotune(m2.handle, ipi.IPI_FP64, str(cache))
        t2 = ipi.ipi_get_tuning(m2.handle)
        assert (t2["ppi_cached"], t2["spmv_workgroups"]) == (-1, 64)
        assert all(t2[k] == t1[k] for k in shapes)
        # without the band form other kernels run: another shape class, tuned
        # once and added to the file, then taken from it
        m2.set_tuning(band_rows=-1, ppi_cached=-1, spmv_workgroups=64)
        ipi.ipi_autotune(m2.handle, ipi.IPI_FP64, str(cache))
        t3 = ipi.ipi_get_tuning(m2.handle)
        assert (t3["band_rows"], t3["ppi_cached"], t3["spmv_workgroups"]) == (-1, -1, 64)
        data = json.loads(cache.read_text())
        assert len(data) == 2 and sorted(k.split("|band")[1].split("|")[0] for k in data) == ["0", "1"]
        m2.set_tuning(band_rows=-1, ppi_cached=-1, spmv_workgroups=64)  # shapes back to automatic
        ipi.ipi_autotune(m2.handle, ipi.IPI_FP64, str(cache))
        assert ipi.ipi_get_tuning(m2.handle) == t3
        V, pi, info, st = m2.solve(device=dev, atol=0.0, rtol_cert=1e-12, alpha=0.1, ksp_type="richardson",
                                   max_inner=100000)
        torch.cuda.synchronize()
        assert st == ipi.IPI_OK
        assert np.max(np.abs(V.cpu().numpy() - ref.V)) / np.max(np.abs(ref.V)) <= 1e-8
    finally:
        m2.close()


def test_band_form_detection():
    ipi = _ipi()
    _dev()
    bd = W.c2(2048)  # 24 consecutive columns per row
    m = ipi.MDP.from_data(bd, flags=ipi.IPI_VAL_FP32)
    try:
        assert m.describe()["band"] == 1
    finally:
        m.close()
    # one row (state 1000, action 3) with a gap before its last column: no band form
    d = W.c2(2048)
    d.col = d.col.copy()
    lo = int(d.row_ptr[16 * 1000 + 3])
    assert d.col[lo + 23] + 1 < d.S
    d.col[lo + 23] += 1
    m = ipi.MDP.from_data(d, flags=ipi.IPI_VAL_FP32)
    try:
        assert m.describe()["band"] == 0
    finally:
        m.close()
    for other in (W.c3(32), W.c1()):
        m = ipi.MDP.from_data(other, flags=ipi.IPI_VAL_FP32)
        try:
            assert m.describe()["band"] == 0
        finally:
            m.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_band_form_bitwise_equal(precision):
    # the band form computes each chunk's columns instead of loading them: the
    # products and the Bellman pass form the same sums in the same order
    ipi = _ipi()
    dev = _dev()
    d = W.c2(4096)
    prec = 0 if precision == "fp64" else 1
    V0 = torch.from_numpy(np.random.default_rng(3).normal(size=d.S) * 10).to(dev)
    m = ipi.MDP.from_data(d, flags=ipi.IPI_VAL_FP32)
    try:
        # Bellman chunks of 16 bytes (wave tiles) and of 32 bytes (workgroup
        # tiles); the same chunk widths with and without the band form
        for bchunk in ((2, 4) if prec == 0 else (4, 8)):
            outs = []
            for band in (0, -1):
                m.set_tuning(band_rows=band, bellman_lanes=-1, bellman_chunk=bchunk,
                             spmv_chunk=2 if prec == 0 else 4)
                TV, pi, resid, rho = m.bellman(V0, prec)
                Vr, pr, ir, sr = m.solve(device=dev, v0=V0, max_outer=2, ksp_type="richardson", max_inner=6,
                                         alpha=1e-15, precision=precision)
                Vg, pg, ig, sg = m.solve(device=dev, atol=0.0, rtol_cert=1e-9, alpha=0.1, ksp_type="gmres",
                                         max_inner=400, max_outer=3, precision=precision)
                torch.cuda.synchronize()
                outs.append((TV.cpu(), pi.cpu(), Vr.cpu(), Vg.cpu(), ir["inner_iters"], ig["inner_iters"]))
            a, b = outs
            for x, y in zip(a[:4], b[:4]):
                assert torch.equal(x, y)
            assert a[4:] == b[4:]
    finally:
        m.close()


def _shifted_band(S, shift_of_action):
    """Birth-death rows moved to other consecutive column ranges: still a band
    form (every row's 24 columns consecutive), with first column - state
    spread as wide as the shifts."""
    d = W.c2(S)
    k = 24
    cols = d.col.reshape(-1, k).astype(np.int64)
    r = np.arange(S * d.A)
    w = cols[:, 0] + shift_of_action(r % d.A, r // d.A)
    w = np.clip(w, 0, S - k)
    d.col = (w[:, None] + np.arange(k)[None, :]).reshape(-1).astype(np.int32)
    d.name = d.name + "-shifted"
    return d


@pytest.mark.parametrize("case", ["wide", "bellman_only"])
@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_band_window_bounds(case, precision):
    # wide: first column - state spans thousands of states, so no tile's
    # window fits and both kernels read the columns; bellman_only: a spread
    # of 60 fits a Bellman wave tile (4 states) but not a 64-state product tile
    ipi = _ipi()
    dev = _dev()
    S = 4096
    if case == "wide":
        d = _shifted_band(S, lambda a, s: (a * 257) % 3000 - 1500)
    else:
        d = _shifted_band(S, lambda a, s: 60 * (a % 2))
    prec = 0 if precision == "fp64" else 1
    ref = d.fp32_rounded() if prec else d
    m = ipi.MDP.from_data(d, flags=ipi.IPI_VAL_FP32)
    try:
        assert m.describe()["band"] == 1
        V = np.random.default_rng(5).normal(size=S) * 10.0
        outs = []
        for band in (0, -1):
            m.set_tuning(band_rows=band)
            TV, pi, resid, rho = m.bellman(torch.from_numpy(V).to(dev), prec)
            Vs, ps, info, st = m.solve(device=dev, atol=0.0, rtol_cert=1e-10, alpha=0.1, ksp_type="richardson",
                                       max_inner=100000, precision=precision)
            torch.cuda.synchronize()
            assert st == ipi.IPI_OK
            _bellman_check(d, V, TV.cpu().numpy(), pi.cpu().numpy(), resid.cpu().numpy(), float(rho.cpu()[0]),
                           prec == 1)
            outs.append((TV.cpu(), Vs.cpu(), info["inner_iters"]))
        # with and without the band form: the same sums in the same order
        assert torch.equal(outs[0][0], outs[1][0])
        assert torch.equal(outs[0][1], outs[1][1]) and outs[0][2] == outs[1][2]
    finally:
        m.close()
    want = O.policy_iteration(ref)
    Vg = outs[0][1].numpy()
    assert np.max(np.abs(Vg - want.V)) <= 1e-8 * np.max(np.abs(want.V))


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32mixed"])
def test_bellman_single_entry_rows(precision):
    # a maze has one nonzero per row: the flat pass takes one value per chunk
    # (no row pointers) and must agree with the lane-group kernel bit for bit
    ipi = _ipi()
    dev = _dev()
    d = W.maze(60, 80)
    assert int(np.max(np.diff(d.row_ptr))) == 1
    V = torch.from_numpy(np.random.default_rng(9).normal(size=d.S) * 3.0).to(dev)
    m = ipi.MDP.from_data(d, flags=ipi.IPI_VAL_FP32)
    try:
        outs = []
        for lanes, spt in ((0, 0), (-1, 7), (1, 0), (2, 16)):
            m.set_tuning(bellman_lanes=lanes, bellman_states_per_tile=spt)
            TV, pi, resid, rho = m.bellman(V, precision)
            torch.cuda.synchronize()
            outs.append((TV.cpu(), pi.cpu(), float(rho.cpu()[0])))
        Vh = V.cpu().numpy()
        _bellman_check(d, Vh, outs[0][0].numpy(), outs[0][1].numpy(), outs[0][0].numpy() - Vh, outs[0][2],
                       precision == 1)
        for o in outs[1:]:
            assert torch.equal(o[0], outs[0][0]) and torch.equal(o[1], outs[0][1]) and o[2] == outs[0][2]
    finally:
        m.close()


@pytest.mark.parametrize("shift", [18, 19, 78, 79])
def test_band_window_limit(shift):
    # birth-death rows span first column - state in [-23, 0]; moving action
    # 1's rows by `shift` widens that to D = 23 + shift.  A 64-state product
    # tile's window has 63 + D + 24 entries (128 at shift 18, the LDS slice's
    # size; 129 at 19 falls back to column loads) and a 4-state FP64 Bellman
    # tile's 3 + D + 24 (128 at shift 78, 129 at 79); either way the results
    # equal those without the band form
    ipi = _ipi()
    dev = _dev()
    S = 4096
    d = _shifted_band(S, lambda a, s: np.where(a == 1, shift, 0))
    off = d.col.reshape(-1, 24).astype(np.int64)[:, 0] - np.arange(S * d.A) // d.A
    assert off.max() - off.min() == 23 + shift
    V0 = torch.from_numpy(np.random.default_rng(13).normal(size=S) * 4.0).to(dev)
    m = ipi.MDP.from_data(d, flags=ipi.IPI_VAL_FP32)
    try:
        assert m.describe()["band"] == 1
        outs = []
        for band in (0, -1):
            m.set_tuning(band_rows=band)
            TV, pi, resid, rho = m.bellman(V0, 0)
            Vr, pr, ir, sr = m.solve(device=dev, v0=V0, max_outer=2, ksp_type="richardson", max_inner=40,
                                     alpha=1e-15)
            torch.cuda.synchronize()
            outs.append((TV.cpu(), pi.cpu(), Vr.cpu()))
        for x, y in zip(*outs):
            assert torch.equal(x, y)
    finally:
        m.close()


@pytest.mark.parametrize("mdp", ["band", "columns"])
@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_cached_value_loads_identical(precision, mdp):
    # loading P_pi through the caches instead of streaming it changes where
    # the bytes come from, not the sums: every inner solver (and the blocked
    # sweeps) gives the same bits with the cached loads forced on, forced off
    # and chosen by size, in the band form and with loaded columns
    ipi = _ipi()
    dev = _dev()
    d = W.c2(20011) if mdp == "band" else W.random_sparse(3001, 5, 32, 0.99, seed=31)
    m = ipi.MDP.from_data(d, flags=ipi.IPI_VAL_FP32)
    try:
        assert m.describe()["band"] == (1 if mdp == "band" else 0)
        runs = [dict(ksp_type="richardson", max_inner=100000, rtol_cert=1e-9),
                dict(ksp_type="richardson", max_inner=100000, rtol_cert=1e-9, richardson_block=1),
                dict(ksp_type="richardson", max_inner=3000, pc="jacobi", rtol_cert=1e-9),
                dict(ksp_type="gmres", max_inner=400, max_outer=4),
                dict(ksp_type="tfqmr", max_inner=400, max_outer=4),
                dict(ksp_type="bicgstab", max_inner=400, max_outer=4)]
        outs = []
        for cached in (1, -1, 0):
            m.set_tuning(ppi_cached=cached)
            assert m.tuning()["ppi_cached"] == cached
            res = []
            for kw in runs:
                V, pi, info, st = m.solve(device=dev, atol=0.0, alpha=0.1, precision=precision, **kw)
                torch.cuda.synchronize()
                res.append((V.cpu(), pi.cpu(), info["inner_iters"], info["outer_iters"], st))
                # bit 0: one-sweep products (auto: this P_pi is far below the
                # cache budget), bit 1: blocked sweeps (band form only)
                assert info["ppi_cached"] == (0 if cached == -1 else (3 if mdp == "band" else 1))
            outs.append(res)
        for other in outs[1:]:
            for a, b in zip(outs[0], other):
                assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
                assert a[2:] == b[2:]
        with pytest.raises(Exception):
            m.set_tuning(ppi_cached=2)
    finally:
        m.close()


def _pattern_mdp(S, pattern_of_row, n_pat, k=4, A=2, seed=7):
    """Rows of k columns: first column c0(r) and offsets [0, 1 + p, 20 + 2 p,
    30 + 3 p] (p = pattern_of_row(r) < n_pat), so the stencil form holds
    n_pat patterns; values Dirichlet-like from a seeded generator."""
    rng = np.random.default_rng(seed)
    R = S * A
    r = np.arange(R)
    p = np.asarray(pattern_of_row(r), dtype=np.int64)
    assert p.max() < n_pat
    off = np.stack([np.zeros_like(p), 1 + p, 20 + 2 * p, 30 + 3 * p], axis=1)[:, :k]
    c0 = (r * 7919) % (S - 60)
    col = (c0[:, None] + off).reshape(-1).astype(np.int32)
    val = rng.exponential(size=(R, k))
    val = (val / val.sum(axis=1, keepdims=True)).reshape(-1)
    row_ptr = np.arange(R + 1, dtype=np.int64) * k
    g = rng.random(R)
    return W.MDPData(S, A, row_ptr, col, val, g, 0.99, f"patterns{n_pat}")


def test_stencil_form_detection():
    """The stencil form: every row's columns are its first column plus one of
    at most 8 offset patterns.  The pendulum's bilinear rows have two (c, c+1,
    c+N, c+N+1 and the rows wrapping around the angle); random rows have too
    many; band rows take the band form; 8 patterns are accepted and 9 are
    not, also when the last one first appears beyond the rows sampled on the
    host (4096).  The pendulum's patterns hold their columns in adjacent
    pairs (one 16-byte load of V per pair); the synthetic ones do not."""
    ipi = _ipi()
    _dev()
    cases = [(W.c3(32), 0, 2, 1), (W.c3(64), 0, 2, 1), (W.c1(), 0, 0, 0), (W.c2(2048), 1, 0, 0),
             (_pattern_mdp(3000, lambda r: r % 8, 8), 0, 8, 0),
             (_pattern_mdp(3000, lambda r: r % 9, 9), 0, 0, 0),
             # patterns 0..6 in the sampled rows, pattern 7 only at row 5001
             (_pattern_mdp(4000, lambda r: np.where(r == 5001, 7, r % 7), 8), 0, 8, 0),
             # a ninth pattern at row 7001 only
             (_pattern_mdp(4000, lambda r: np.where(r == 7001, 8, r % 8), 9), 0, 0, 0)]
    for d, band, pats, pairs in cases:
        m = ipi.MDP.from_data(d, flags=ipi.IPI_VAL_FP32)
        try:
            desc = m.describe()
            assert (desc["band"], desc["stencil_patterns"], desc["stencil_pairs"]) == (band, pats, pairs), d.name
        finally:
            m.close()


@pytest.mark.parametrize("make", [lambda: W.c3(64), lambda: _pattern_mdp(3000, lambda r: r % 8, 8),
                                  lambda: _pattern_mdp(3001, lambda r: r % 8, 8)],
                         ids=["pendulum_64", "patterns8_3000", "patterns8_3001"])
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32mixed"])
def test_stencil_form_bitwise_equal(make, precision):
    """The Bellman pass in the stencil form computes each chunk's columns from
    the row's word and its pattern: the same sums in the same order as with
    the columns loaded (tiles of 64 states, the last one ragged for 3000 and
    3001 states; automatic launch and workgroup tiles), and the oracle's
    values."""
    ipi = _ipi()
    dev = _dev()
    d = make()
    V = np.random.default_rng(11).normal(size=d.S) * 10.0
    m = ipi.MDP.from_data(d, flags=ipi.IPI_VAL_FP32)
    try:
        assert m.describe()["stencil_patterns"] > 0
        outs = []
        for form, lanes in ((0, -1), (0, -2), (-1, -2)):
            m.set_tuning(band_rows=form, bellman_lanes=lanes, bellman_states_per_tile=64)
            TV, pi, resid, rho = m.bellman(torch.from_numpy(V).to(dev), precision)
            torch.cuda.synchronize()
            _bellman_check(d, V, TV.cpu().numpy(), pi.cpu().numpy(), resid.cpu().numpy(), float(rho.cpu()[0]),
                           precision == 1)
            outs.append((TV.cpu(), pi.cpu(), resid.cpu()))
        for other in outs[1:]:
            for x, y in zip(outs[0], other):
                assert torch.equal(x, y)
    finally:
        m.close()


@pytest.mark.parametrize("make", [lambda: W.c3(64), lambda: _pattern_mdp(3000, lambda r: r % 8, 8),
                                  lambda: _pattern_mdp(3001, lambda r: r % 8, 8, A=3)],
                         ids=["pendulum_64", "patterns8_3000", "patterns8_3001_A3"])
@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
@pytest.mark.parametrize("inner", ["richardson", "gmres", "tfqmr", "bicgstab"])
def test_stencil_form_products_bitwise_equal(make, precision, inner):
    """The P_pi products in the stencil form (one word per row of P_pi, wave
    tiles) compute the same products in the same order as with the columns
    loaded: every inner solver gives the same bits with the form on and off
    (a few capped evaluations; Jacobi scaling with Richardson)."""
    ipi = _ipi()
    dev = _dev()
    d = make()
    m = ipi.MDP.from_data(d, flags=ipi.IPI_VAL_FP32)
    try:
        assert m.describe()["stencil_patterns"] > 0
        outs = []
        for form in (0, -1):
            m.set_tuning(band_rows=form)
            V, pi, info, st = m.solve(device=dev, atol=0.0, rtol_cert=1e-9, alpha=0.1, ksp_type=inner,
                                      pc="jacobi" if inner == "richardson" else "none", max_outer=4,
                                      max_inner=60, precision=precision)
            torch.cuda.synchronize()
            outs.append((V.cpu(), pi.cpu(), info["inner_iters"], info["final_rho"]))
        assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
        assert outs[0][2:] == outs[1][2:]
    finally:
        m.close()


def test_stencil_form_products_oracle_parity():
    """A converged solve of the pendulum (32 x 32, A = 11) with its products in
    the stencil form: V* within 1e-8 of the oracle's, the policy outside the
    tie band equal."""
    ipi = _ipi()
    dev = _dev()
    d = W.c3(32)
    ref = O.policy_iteration(d)
    m = ipi.MDP.from_data(d, flags=ipi.IPI_VAL_FP32)
    try:
        V, pi, info, st = m.solve(device=dev, atol=0.0, rtol_cert=1e-11, alpha=0.1, ksp_type="richardson",
                                  pc="jacobi", max_inner=1000000)
        torch.cuda.synchronize()
    finally:
        m.close()
    assert st == 0
    V, pi = V.cpu().numpy(), pi.cpu().numpy()
    scale = np.max(np.abs(ref.V))
    assert np.max(np.abs(V - ref.V)) / scale <= 1e-8
    assert not ((pi != ref.pi) & (ref.qgap >= O.parity_tau(ref.V))).any()

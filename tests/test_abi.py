"""CPU-side checks of the C ABI: the library loads, exports every declared
symbol, parses options, and rejects malformed MDPs from host memory before
any device call."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

from paper_2507_22538_amd import ipi
from paper_2507_22538_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s+\**(ipi_[a-z0-9_]+)\s*\(", text, re.M):
            names.add(m.group(1))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(ipi.LIB_PATH)
    names = _declared_functions()
    assert len(names) >= 14
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, f"undeclared exports missing: {missing}"


def test_version_and_last_error():
    assert "gfx950" in ipi.ipi_version()
    assert isinstance(ipi.ipi_last_error(), str)


def test_options_table1_names():
    o = ipi.ipi_opts_default()
    assert (o.max_outer, o.max_inner, o.atol, o.alpha, o.inner, o.pc) == (1000, 1000, 1e-8, 1e-4, 0, 0)
    ipi.ipi_opts_set(o, "-max_iter_pi", "7")
    ipi.ipi_opts_set(o, "max_iter_ksp", "3")
    ipi.ipi_opts_set(o, "-ksp_max_it", "5")
    ipi.ipi_opts_set(o, "-atol_pi", "1e-10")
    ipi.ipi_opts_set(o, "-alpha", "0.5")
    ipi.ipi_opts_set(o, "-ksp_type", "richardson")
    ipi.ipi_opts_set(o, "-ksp_richardson_scale", "0.7")
    ipi.ipi_opts_set(o, "-pc_type", "jacobi")
    ipi.ipi_opts_set(o, "-precision", "fp32_inner")
    assert o.precision == ipi.IPI_FP32_INNER
    ipi.ipi_opts_set(o, "-precision", "fp32_mixed")
    ipi.ipi_opts_set(o, "-mode", "MAXREWARD")
    assert (o.profile, o.richardson_block) == (0, 1)  # blocked sweeps wherever they apply
    ipi.ipi_opts_set(o, "-profile", "2")
    ipi.ipi_opts_set(o, "-ksp_richardson_block", "0")
    assert (o.max_outer, o.max_inner, o.atol, o.alpha, o.inner) == (7, 5, 1e-10, 0.5, 1)
    assert (o.richardson_scale, o.pc, o.precision, o.mode) == (0.7, 1, 1, 1)
    assert (o.profile, o.richardson_block) == (2, 0)
    for name, value in [("-alpha", "1.5"), ("-alpha", "0"), ("-max_iter_pi", "0"), ("-ksp_type", "sor"),
                        ("-pc_type", "svd"), ("-nonsense", "1"), ("-atol_pi", "abc"), ("-ksp_gmres_restart", "65"),
                        ("-profile", "3"), ("-ksp_richardson_block", "2")]:
        with pytest.raises(ipi.IPIError) as e:
            ipi.ipi_opts_set(o, name, value)
        assert e.value.status == ipi.IPI_E_INVALID_ARG


def _create(d, **over):
    a = dict(S=d.S, A=d.A, nnz=d.nnz, row_ptr=d.row_ptr, col=d.col, val=d.val, g=d.g, gamma=d.gamma)
    a.update(over)
    return ipi.ipi_mdp_create_csr(a["S"], a["A"], a["nnz"], a["row_ptr"], a["col"], a["val"], a["g"], a["gamma"],
                                  0, 0)


def test_host_validation_rejects_malformed():
    d = W.random_sparse(50, 3, 4, 0.9, seed=2)
    cases = []
    rp = d.row_ptr.copy(); rp[5], rp[6] = rp[6], rp[5]
    cases.append((dict(row_ptr=rp), ipi.IPI_E_INVALID_ARG))
    c = d.col.copy(); c[10] = d.S
    cases.append((dict(col=c), ipi.IPI_E_INVALID_ARG))
    c = d.col.copy(); c[1] = c[0]
    cases.append((dict(col=c), ipi.IPI_E_INVALID_ARG))
    v = d.val.copy(); v[3] = -0.1
    cases.append((dict(val=v), ipi.IPI_E_NOT_STOCHASTIC))
    v = d.val.copy(); v[3] += 1e-6
    cases.append((dict(val=v), ipi.IPI_E_NOT_STOCHASTIC))
    v = d.val.copy(); v[3] = np.inf
    cases.append((dict(val=v), ipi.IPI_E_NOT_STOCHASTIC))
    gg = d.g.copy(); gg[4] = np.nan
    cases.append((dict(g=gg), ipi.IPI_E_INVALID_ARG))
    cases.append((dict(gamma=1.0), ipi.IPI_E_INVALID_ARG))
    cases.append((dict(gamma=0.0), ipi.IPI_E_INVALID_ARG))
    cases.append((dict(gamma=float("nan")), ipi.IPI_E_INVALID_ARG))
    cases.append((dict(S=0), ipi.IPI_E_INVALID_ARG))
    cases.append((dict(A=0), ipi.IPI_E_INVALID_ARG))
    cases.append((dict(A=5000), ipi.IPI_E_INVALID_ARG))
    cases.append((dict(nnz=d.nnz - 1), ipi.IPI_E_INVALID_ARG))
    for over, status in cases:
        with pytest.raises(ipi.IPIError) as e:
            _create(d, **over)
        assert e.value.status == status, (over.keys(), e.value)
        assert ipi.ipi_last_error() != ""


def test_large_finite_costs_accepted_by_validation():
    # the maze uses 1e20 for walls (Sec. IV-D): valid input.  The library's
    # host validation runs before any device call, so on a host without a GPU
    # the call gets past it and fails only at the upload (IPI_E_DEVICE); with
    # a GPU it succeeds.  The same MDP with one cost set to inf is rejected by
    # the validation itself.
    d = W.maze(5, 5, seed=1)
    assert np.max(d.g) == 1e20
    try:
        h = _create(d)
    except ipi.IPIError as e:
        assert e.status == ipi.IPI_E_DEVICE, e
    else:
        ipi.ipi_mdp_destroy(h)
    gg = d.g.copy()
    gg[0] = np.inf
    with pytest.raises(ipi.IPIError) as e:
        _create(d, g=gg)
    assert e.value.status == ipi.IPI_E_INVALID_ARG


def test_footprint_formula():
    o = ipi.ipi_opts_default()
    f64 = ipi.ipi_footprint_bytes(2_000_000, 16, 768_000_000, 24, o)
    ipi.ipi_opts_set(o, "-precision", "fp32_mixed")
    mixed = ipi.ipi_footprint_bytes(2_000_000, 16, 768_000_000, 24, o)
    assert 9e9 < f64 < 14e9
    assert mixed > f64  # the mixed mode keeps the FP64 values plus a float32 copy
    assert ipi.ipi_footprint_bytes(0, 1, 1, 1, o) == -1

"""Pins of the scatter-angle-interpolation oracle (Sec. III-B): the SAI
adjoint is the transpose of the SAI forward; at a pair whose angle is a table
node, SAI equals the exact operator (the table holds the exact spectral part
and the geometric factor stays exact); refining the table converges to the
exact operator."""
import numpy as np
import pytest

from paper_1603_06400_amd import inputs


def small(oracle_mod, n=8, nq=12):
    g = inputs.standard_geometry(n, nq, ndet=n)
    f = inputs.phantom(g, 31, 2)
    g = g.with_(C=400.0 / oracle_mod.Oracle(g).forward(f).max())
    return g, f


@pytest.mark.parametrize("interp", [0, 1])
def test_sai_adjoint_identity(oracle_mod, interp):
    g, _ = small(oracle_mod)
    o = oracle_mod.Oracle(g)
    rng = np.random.Generator(np.random.PCG64(3))
    f = rng.uniform(0, 1, (g.nz, g.nx, g.nq))
    y = rng.uniform(0, 1, (g.ndy, g.ndx))
    tm = o.max_angle()
    lhs = np.sum(o.forward_sai(f, 100, tm, interp) * y)
    rhs = np.sum(f * o.adjoint_sai(y, 100, tm, interp))
    assert lhs == pytest.approx(rhs, rel=1e-12)


@pytest.mark.parametrize("interp", [0, 1])
def test_sai_is_exact_at_a_table_node(oracle_mod, interp):
    """Place node 37 of a 60-node table exactly at pair (j, i)'s angle; a lone
    voxel j then gives the exact g_i."""
    g, _ = small(oracle_mod)
    o = oracle_mod.Oracle(g)
    j, i = 13, 21
    pf = o.pair(j, i)
    th = 2.0 * np.arctan2(pf["sin_half"], pf["cos_half"])
    nt, node = 60, 37
    tm = th * (nt - 1) / node
    f = np.zeros((g.nz, g.nx, g.nq))
    f.reshape(-1, g.nq)[j] = np.linspace(0.3, 1.0, g.nq)
    ge = o.forward(f).reshape(-1)[i]
    gs = o.forward_sai(f, nt, tm, interp).reshape(-1)[i]
    assert ge != 0.0
    assert gs == pytest.approx(ge, rel=1e-12)


def test_sai_converges_to_the_exact_operator(oracle_mod):
    g, f = small(oracle_mod, 8, 16)
    o = oracle_mod.Oracle(g)
    tm = o.max_angle()
    ge = o.forward(f)
    y = o.forward(f)
    be = o.adjoint(y)
    errs_f, errs_b = [], []
    for nt in (32, 128, 512, 2048):
        errs_f.append(np.linalg.norm(o.forward_sai(f, nt, tm, 1) - ge) / np.linalg.norm(ge))
        errs_b.append(np.linalg.norm(o.adjoint_sai(y, nt, tm, 1) - be) / np.linalg.norm(be))
    assert all(a > b for a, b in zip(errs_f, errs_f[1:])), errs_f
    assert all(a > b for a, b in zip(errs_b, errs_b[1:])), errs_b
    assert errs_f[-1] < 2e-2 and errs_b[-1] < 2e-2
    # nearest-node interpolation converges too, more slowly
    e0 = np.linalg.norm(o.forward_sai(f, 2048, tm, 0) - ge) / np.linalg.norm(ge)
    assert e0 < 5e-2


def test_max_angle_bounds_every_pair(oracle_mod):
    g, _ = small(oracle_mod)
    o = oracle_mod.Oracle(g)
    tm = o.max_angle()
    rng = np.random.Generator(np.random.PCG64(9))
    for _ in range(50):
        j, i = int(rng.integers(g.nvox)), int(rng.integers(g.npix))
        p = o.pair(j, i)
        assert 2.0 * np.arctan2(p["sin_half"], p["cos_half"]) <= tm

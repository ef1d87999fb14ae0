"""Pins of the ordered-subsets oracle (Alg. 6 and the partition of Sec. VI):
the paper's printed partition example, partition invariants, P = 1 equal to
Alg. 5 through a different code path, and subset count conservation of the
unpenalised sub-step (an EM property on the subset's data)."""
import json
import os

import numpy as np
import pytest

from paper_1603_06400_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_partition_matches_the_printed_example(oracle_mod):
    ex = json.load(open(os.path.join(GOLDEN, "os_partition_example.json")))
    subs = oracle_mod.os_partition(ex["rows"], ex["columns"], ex["rho_z"], ex["rho_y"])
    assert len(subs) == ex["n_subsets"]
    owner = np.empty(ex["rows"] * ex["columns"], dtype=int)
    for p, pix in enumerate(subs):
        owner[pix] = p
    owner = owner.reshape(ex["rows"], ex["columns"])
    for row in range(ex["rows"]):                       # every row: these columns share a subset
        cols = [c - 1 for grp in ex["same_subset_columns"] for c in grp]
        assert len(set(owner[row, cols])) == 1
    for col in range(ex["columns"]):                    # every column: these rows share a subset
        rows = [r - 1 for grp in ex["same_subset_rows"] for r in grp]
        assert len(set(owner[rows, col])) == 1
    # and nothing else: 8 columns x 4 rows per subset
    assert all(len(p) == 8 * 4 for p in subs)


@pytest.mark.parametrize("ndy,ndx,rz,ry", [(32, 32, 8, 16), (128, 128, 8, 16), (12, 20, 3, 10), (8, 8, 1, 2)])
def test_partition_invariants(oracle_mod, ndy, ndx, rz, ry):
    subs = oracle_mod.os_partition(ndy, ndx, rz, ry)
    assert len(subs) == rz * (ry // 2)
    allpix = np.concatenate(subs)
    assert np.array_equal(np.sort(allpix), np.arange(ndy * ndx))      # disjoint cover
    assert len({len(p) for p in subs}) == 1                            # balanced
    for pix in subs:
        s = set(pix.tolist())
        for q in pix:
            r, c = divmod(int(q), ndx)
            assert (ndy - 1 - r) * ndx + c in s                         # up-down mirror
            assert r * ndx + (ndx - 1 - c) in s                         # left-right mirror
            assert r * ndx + (c + ry) % ndx in s or c + ry >= ndx       # translation step


def test_partition_rejects_unbalanced_steps(oracle_mod):
    with pytest.raises(ValueError):
        oracle_mod.os_partition(32, 32, 5, 16)
    with pytest.raises(ValueError):
        oracle_mod.os_partition(32, 32, 8, 12)


def tiny(oracle_mod, n=8, nq=6):
    """A small scan whose C puts the phantom's largest mean count at 400 (so
    that f is O(1) and beta = 1e-3 is a mild penalty, as in the workloads)."""
    g = inputs.standard_geometry(n, nq, ndet=n)
    f = inputs.phantom(g, 11, 2)
    g = g.with_(C=400.0 / oracle_mod.Oracle(g).forward(f).max())
    return g, f


def counts(o, f, seed):
    return inputs.poisson_counts(o.forward(f), seed)


def test_one_subset_is_alg5(oracle_mod):
    """P = 1: Alg. 6 reduces to Alg. 5 (forward at the subset's pixels and the
    back projection of a masked ratio against the full-image routines)."""
    g, f = tiny(oracle_mod)
    o = oracle_mod.Oracle(g)
    y = counts(o, f, 12)
    f0 = oracle_mod.uniform_start(y, o.sensitivity())
    fa, Ja = o.recon(y, None, f0, 3, 1e-3)
    fb, Jb = o.recon_os(y, None, f0, 3, 1e-3, [np.arange(g.npix)])
    np.testing.assert_allclose(fb, fa, rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(Jb, Ja, rtol=1e-12)


def test_subset_step_conserves_subset_counts(oracle_mod):
    """beta = 0: after the sub-step on subset p, sum_{i in p} (A f)_i equals
    sum_{i in p} y_i (the EM fixed total on the data the step used)."""
    g, f = tiny(oracle_mod)
    o = oracle_mod.Oracle(g)
    y = counts(o, f, 13)
    subs = oracle_mod.os_partition(g.ndy, g.ndx, 2, 4)
    f0 = oracle_mod.uniform_start(y, o.sensitivity())
    f1, _ = o.recon_os(y, None, f0, 1, 0.0, subs[:1])      # one sub-step on subset 0
    pix = subs[0]
    seen = o.forward_pixels(f0, pix) > 0
    assert np.all(seen)
    assert np.sum(o.forward_pixels(f1, pix)) == pytest.approx(np.sum(y.reshape(-1)[pix]), rel=1e-10)


def test_subsets_accelerate_the_first_sweep(oracle_mod):
    """One sweep over 8 subsets lowers J more than two Alg. 5 iterations."""
    g, f = tiny(oracle_mod, 16, 8)
    o = oracle_mod.Oracle(g)
    y = counts(o, f, 14)
    f0 = oracle_mod.uniform_start(y, o.sensitivity())
    _, Ja = o.recon(y, None, f0, 2, 1e-3)
    _, Jb = o.recon_os(y, None, f0, 1, 1e-3, oracle_mod.os_partition(g.ndy, g.ndx, 2, 8))
    assert Jb[0] == pytest.approx(Ja[0], rel=1e-14)
    assert Jb[1] < Ja[2] < Ja[0]

"""Batched form and launch shapes.

* Batched Alg. 5 over scans of uneven sizes (one merged launch per kernel
  variant, iteration captured in a HIP graph) reproduces the per-scan
  sequential reconstructions bitwise (same kernels and tile shapes).
* Any launch shape gives oracle parity; the autotuner's choice is valid.
"""
import numpy as np
import pytest
import torch

from paper_1603_06400_amd import autotune, csx, inputs

from .gpu_helpers import assert_parity, ragged_geometry, rel_l2, workload_data

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def mixed_scans():
    """Uneven scans: square slices of several sizes and q counts, plus an
    off-centre ragged one (no x-mirror)."""
    out = []
    for k, (n, nq) in enumerate([(16, 16), (24, 40), (32, 32), (20, 64), (48, 24)]):
        g = inputs.standard_geometry(n, nq, mask_seed=100 + k)
        f = inputs.phantom(g, 200 + k, 4)
        out.append((g, f))
    g = ragged_geometry(3, 12, 11, 14, 18, 30, 402.57)
    out.append((g, inputs.phantom(g, 300, 3)))
    return out


def counts_for(geo, f, seed):
    """Poisson counts with a mean from the GPU forward itself, scaled to 1e3
    (these inputs feed a GPU-vs-GPU comparison, not an oracle parity claim)."""
    g = host(geo.forward(dev(f)))
    return inputs.poisson_counts(1e3 * g / max(g.max(), 1e-30), seed)


def test_batch_equals_sequential():
    scans = mixed_scans()
    geos = [csx.Geometry(g) for g, _ in scans]
    ys = [dev(counts_for(geo, f, 7 + k)) for k, (geo, (_, f)) in enumerate(zip(geos, scans))]
    n_iter, beta = 4, 1e-3
    f_seq, J_seq = [], []
    for geo, y in zip(geos, ys):
        f = geo.new_image()
        J_seq.append(geo.recon(y, f, n_iter, beta))
        f_seq.append(f)
    geos2 = [csx.Geometry(g) for g, _ in scans]
    for a, b in zip(geos, geos2):
        lc = a.get_launch()
        b.set_launch(lc["fwd_splits"], lc["fwd_qw"], lc["adj_qw"])
    batch = csx.Batch(geos2)
    f_bat = [g.new_image() for g in geos2]
    J_bat = batch.recon(ys, f_bat, n_iter, beta)
    for k in range(len(scans)):
        assert torch.equal(f_seq[k], f_bat[k]), k
        np.testing.assert_array_equal(J_seq[k], J_bat[k])


def test_batch_per_scan_counts_equal_sequential():
    """Scans with their own iteration counts (including 0 and repeated counts)
    leave the merged launches when done; each equals its csx_recon run."""
    scans = mixed_scans()
    counts = [3, 0, 5, 3, 1, 6]
    geos = [csx.Geometry(g) for g, _ in scans]
    ys = [dev(counts_for(geo, f, 60 + k)) for k, (geo, (_, f)) in enumerate(zip(geos, scans))]
    f_seq, J_seq = [], []
    for geo, y, n in zip(geos, ys, counts):
        f = geo.new_image()
        J_seq.append(geo.recon(y, f, n, 1e-3))
        f_seq.append(f)
    geos2 = [csx.Geometry(g) for g, _ in scans]
    for a, b in zip(geos, geos2):
        lc = a.get_launch()
        b.set_launch(lc["fwd_splits"], lc["fwd_qw"], lc["adj_qw"])
    f_bat = [g.new_image() for g in geos2]
    J_bat = csx.Batch(geos2).recon(ys, f_bat, counts, 1e-3)
    assert J_bat.shape == (len(scans), max(counts) + 1)
    for k, n in enumerate(counts):
        assert torch.equal(f_seq[k], f_bat[k]), k
        np.testing.assert_array_equal(J_seq[k], J_bat[k, :n + 1])
        assert np.all(np.isnan(J_bat[k, n + 1:]))


def test_batch_resume_equals_continuous():
    scans = mixed_scans()[:4]
    geos = [csx.Geometry(g) for g, _ in scans]
    ys = [dev(counts_for(geo, f, 20 + k)) for k, (geo, (_, f)) in enumerate(zip(geos, scans))]
    batch = csx.Batch(geos)
    fa = [g.new_image() for g in geos]
    Ja = batch.recon(ys, fa, 6, 1e-3)
    fb = [g.new_image() for g in geos]
    Jb1 = batch.recon(ys, fb, 3, 1e-3)
    Jb2 = batch.recon(ys, fb, 3, 1e-3, init_uniform=False)
    for k in range(len(geos)):
        assert torch.equal(fa[k], fb[k])
        np.testing.assert_array_equal(Ja[k, :4], Jb1[k])
        np.testing.assert_array_equal(Ja[k, 3:], Jb2[k])
        assert np.all(np.diff(Ja[k]) <= 1e-7 * np.abs(Ja[k, 1:]))


def test_batch_scan_matches_oracle(oracle_mod):
    w, g, f, y = workload_data("slice32")
    others = mixed_scans()[:3]
    geos = [csx.Geometry(g)] + [csx.Geometry(gg) for gg, _ in others]
    ys = [dev(y)] + [dev(counts_for(geo, ff, 40 + k)) for k, (geo, (_, ff)) in enumerate(zip(geos[1:], others))]
    fs = [gg.new_image() for gg in geos]
    J = csx.Batch(geos).recon(ys, fs, 5, w.beta)
    o = oracle_mod.Oracle(g)
    f0 = oracle_mod.uniform_start(y, o.sensitivity())
    ref_f, ref_J = o.recon(y, None, f0, 5, w.beta)
    assert rel_l2(host(fs[0]), ref_f) <= 1e-4
    assert np.max(np.abs(J[0] - ref_J)) <= 1e-6 * abs(ref_J[0])


@pytest.mark.parametrize("shape", [(1, 64, 64, 1), (3, 32, 32, 3), (7, 16, 64, 16), (64, 64, 16, 1),
                                   (2, 32, 64, 64)])
def test_launch_shapes_keep_parity(oracle_mod, shape):
    """Every shape, with the direct operators (the interval form does not
    split) and with the adjoint's pixel classes in 1 to 64 tile ranges."""
    w, g, f, y = workload_data("slice32")
    o = oracle_mod.Oracle(g)
    geo = csx.Geometry(g)
    geo.set_interval_operators(False)
    geo.set_launch(*shape)
    assert geo.get_launch() == dict(zip(("fwd_splits", "fwd_qw", "adj_qw", "adj_splits"), shape))
    assert_parity(host(geo.forward(dev(f))), o.forward(f), what=f"forward {shape}")
    assert_parity(host(geo.backproject(dev(y))), o.adjoint(y), what=f"adjoint {shape}")


def test_launch_shape_validation():
    w, g, f, y = workload_data("slice32")
    geo = csx.Geometry(g)
    for bad in [(0, 64, 64), (65, 64, 64), (1, 48, 64), (1, 64, 8), (1, 64, 64, 65), (1, 64, 64, -1)]:
        with pytest.raises(csx.CsxError) as ei:
            geo.set_launch(*bad)
        assert ei.value.code == csx.CSX_EINVAL


def test_autotune_picks_a_valid_shape(oracle_mod, tmp_path):
    w, g, f, y = workload_data("slice32")
    geo = csx.Geometry(g)
    cache = {}
    c = autotune.tuned(geo, cache, reps=3)
    assert c["fwd_qw"] in autotune.QWS and c["adj_qw"] in autotune.QWS
    assert c["forward_ms"] > 0 and c["adjoint_ms"] > 0
    path = str(tmp_path / "tune.json")
    autotune.save_cache(cache, path)
    assert autotune.load_cache(path) == cache
    o = oracle_mod.Oracle(g)
    assert_parity(host(geo.forward(dev(f))), o.forward(f), what="forward tuned")


def test_batch64_shapes_in_a_merged_launch(oracle_mod):
    """Scans of the 64-scan batched workload at its largest shapes (128^2 x 64 q
    and 96^2 x 32 q, with a 48^2 x 64 q and a 64^2 x 32 q scan) in one merged
    batch: every scan bitwise equal to its own csx_recon run, and the two large
    scans within the float32 bar of the oracle's Alg. 5 after 2 iterations."""
    beta, n_iter = 1e-3, 2
    picks = inputs.batch_scans()[:4]      # 48^2 x 64, 128^2 x 64, 96^2 x 32, 64^2 x 32
    assert [(s.geom.nx, s.geom.nq) for s in picks] == [(48, 64), (128, 64), (96, 32), (64, 32)]
    geoms, ys = [], []
    for s in picks:
        f = inputs.phantom(s.geom, s.phantom_seed, s.n_rect)
        o1 = oracle_mod.Oracle(s.geom.with_(C=1.0))
        a1f = o1.forward(f)
        C = 1e4 / a1f.max()
        geoms.append(s.geom.with_(C=C))
        ys.append(inputs.poisson_counts(C * a1f, s.noise_seed))
        print(f"[batch64 scan {s.geom.nx}^2 x {s.geom.nq} q: counts ready]", flush=True)
    seq = [csx.Geometry(g) for g in geoms]
    f_seq, J_seq = [], []
    for geo, y in zip(seq, ys):
        f = geo.new_image()
        J_seq.append(geo.recon(dev(y), f, n_iter, beta))
        f_seq.append(f)
    bat = [csx.Geometry(g) for g in geoms]
    for a, b in zip(seq, bat):
        lc = a.get_launch()
        b.set_launch(lc["fwd_splits"], lc["fwd_qw"], lc["adj_qw"])
    f_bat = [g.new_image() for g in bat]
    J_bat = csx.Batch(bat).recon([dev(y) for y in ys], f_bat, n_iter, beta)
    for k in range(len(picks)):
        assert torch.equal(f_seq[k], f_bat[k]), k
        np.testing.assert_array_equal(J_seq[k], J_bat[k])
    for k in (1, 2):
        o = oracle_mod.Oracle(geoms[k])
        f0 = oracle_mod.uniform_start(ys[k], o.sensitivity())
        ref_f, ref_J = o.recon(ys[k], None, f0, n_iter, beta)
        e = assert_parity(host(f_bat[k]), ref_f, what=f"batched {geoms[k].nx}^2 scan, {n_iter} iterations")
        dJ = np.max(np.abs(J_bat[k] - ref_J) / ref_J)
        print(f"batched {geoms[k].nx}^2 x {geoms[k].nq} q: f rel-L2 {e:.3e}, max |dJ|/J {dJ:.3e}")
        assert dJ <= 1e-6


@pytest.mark.parametrize("direct_one", [False, True], ids=["all_interval", "one_direct"])
def test_batch_merged_elementwise_equals_sequential(direct_one):
    """Scans whose q counts are multiples of 4 take the merged elementwise
    launches (partial-image sums, ratios, updates, copy-backs of every
    interval-form scan in one launch each); with one scan on the direct
    operators beside them, that scan keeps its own launches.  Either way the
    batch reproduces the sequential runs bitwise, per-scan iteration counts
    included."""
    scans = [s for s in mixed_scans() if s[0].nq % 4 == 0]
    assert len(scans) >= 4
    geos = [csx.Geometry(g) for g, _ in scans]
    geos2 = [csx.Geometry(g) for g, _ in scans]
    if direct_one:
        geos[1].set_interval_operators(False)
        geos2[1].set_interval_operators(False)
    assert sum(g.interval_operators()["on"] for g in geos2) >= 3
    ys = [dev(counts_for(geo, f, 11 + k)) for k, (geo, (_, f)) in enumerate(zip(geos, scans))]
    counts = [3, 5, 0, 4, 2][:len(scans)]
    beta = 1e-3
    f_seq, J_seq = [], []
    for geo, y, n in zip(geos, ys, counts):
        f = geo.new_image()
        J_seq.append(geo.recon(y, f, n, beta))
        f_seq.append(f)
    for a, b in zip(geos, geos2):
        lc = a.get_launch()
        b.set_launch(lc["fwd_splits"], lc["fwd_qw"], lc["adj_qw"])
    batch = csx.Batch(geos2)
    f_bat = [g.new_image() for g in geos2]
    J_bat = batch.recon(ys, f_bat, counts, beta)
    for k in range(len(scans)):
        assert torch.equal(f_seq[k], f_bat[k]), k
        np.testing.assert_array_equal(J_seq[k], J_bat[k][:counts[k] + 1])

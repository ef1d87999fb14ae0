"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerance: rel-L2 <= 1e-5 for g, b and one reconstruction step (FP32 kernels
vs FP64 oracle), plus an element-wise cap of 1e-4 of the largest reference
magnitude.  Sizes span several tiles of every kernel and ragged tails; at the
full 128^2 x 64q slice every output of the forward and the adjoint is
compared, with one reconstruction step and three Alg. 5 iterations.
"""
import time

import numpy as np
import pytest
import torch

from paper_1603_06400_amd import csx, inputs

from .gpu_helpers import (assert_parity, near_edge_geometry, objective_tolerance, ragged_geometry, rel_l2,
                          workload_data)

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


RAGGED = [
    # (seed, nx, nz, ndx, ndy, nq, z_min): z_min chosen so every mask crossing
    # sits >= 2e-4 mm from a cell edge
    (1, 10, 7, 12, 10, 24, 402.57),     # one partial q chunk, ragged pixel-pair and voxel tails
    (2, 9, 5, 9, 6, 64, 404.77),        # odd nx and ndx, exactly one q chunk
    (3, 12, 11, 14, 18, 80, 402.57),    # two q chunks
    (4, 33, 3, 7, 2, 40, 402.57),       # a single detector row pair
    (5, 3, 70, 31, 22, 17, 401.9),      # tall slice, ragged everything
]

# centred voxel grids with even nx and ndx: the x -> -x mirror path
SYMMETRIC = [
    (11, 8, 5, 10, 6, 20, 404.77),      # two classes per wave instruction (nq <= 32)
    (12, 12, 9, 14, 12, 12, 402.57),    # four classes per wave instruction (nq <= 16)
    (13, 34, 7, 22, 8, 70, 403.93),     # two q chunks, voxel pairs beyond one batch
    (14, 6, 40, 6, 30, 64, 402.57),     # exactly one q chunk, tall slice
    (15, 16, 16, 16, 16, 8, 404.13),    # 8 q nodes
]


@pytest.mark.parametrize("case", RAGGED, ids=[f"r{c[0]}" for c in RAGGED])
def test_forward_adjoint_ragged(oracle_mod, case):
    print(f"[ragged {case}]", flush=True)
    g = ragged_geometry(*case)
    seed = case[0]
    o = oracle_mod.Oracle(g)
    assert o.margins()["mask_edge_mm"] > 1e-4   # no float32/float64 tie at a mask-cell edge
    geo = csx.Geometry(g)
    assert geo.info()["symmetric_lr"] == 0
    f = inputs.random_image(g, 100 + seed)
    y = inputs.random_detector(g, 200 + seed)
    assert_parity(host(geo.forward(dev(f))), o.forward(f), what="forward")
    assert_parity(host(geo.backproject(dev(y))), o.adjoint(y), what="adjoint")


@pytest.mark.parametrize("case", SYMMETRIC, ids=[f"s{c[0]}" for c in SYMMETRIC])
def test_forward_adjoint_mirror_path(oracle_mod, case):
    print(f"[symmetric {case}]", flush=True)
    g = ragged_geometry(*case, x=(-40.0, 40.0))
    o = oracle_mod.Oracle(g)
    assert o.margins()["mask_edge_mm"] > 1e-4
    geo = csx.Geometry(g)
    assert geo.info()["symmetric_lr"] == 1
    f = inputs.random_image(g, 300 + case[0])
    y = inputs.random_detector(g, 400 + case[0])
    assert_parity(host(geo.forward(dev(f))), o.forward(f), what="forward")
    assert_parity(host(geo.backproject(dev(y))), o.adjoint(y), what="adjoint")


@pytest.mark.parametrize("lr", [0, 1])
@pytest.mark.parametrize("delta", [1e-9, -1e-9])
@pytest.mark.parametrize("axis", ["x", "y"])
def test_mask_cell_near_tie(oracle_mod, axis, delta, lr):
    """A ray crossing the mask plane 1e-9 mm from the edge between an open and
    a closed cell (App. A): the library decides the cell in float64, as the
    oracle does, so the critical pixel sees the same cell.  A lone voxel's
    image and a lone pixel's back projection, then random data."""
    g, (ix, iz, a, b), T = near_edge_geometry(axis, delta, lr)
    print(f"[near tie {axis} {delta:+.0e} lr={lr}: critical cell open={T}]", flush=True)
    o = oracle_mod.Oracle(g)
    assert o.margins()["mask_edge_mm"] < 2e-9
    geo = csx.Geometry(g)
    assert geo.info()["symmetric_lr"] == lr
    f = np.zeros((g.nz, g.nx, g.nq))
    f[iz, ix, :] = 1.0
    ref = o.forward(f)
    got = host(geo.forward(dev(f)))
    assert (ref[b, a] != 0) == bool(T) and (got[b, a] != 0) == bool(T)
    assert_parity(got, ref, what="forward, lone voxel")
    y = np.zeros((g.ndy, g.ndx))
    y[b, a] = 1.0
    assert_parity(host(geo.backproject(dev(y))), o.adjoint(y), what="adjoint, lone pixel")
    fr = inputs.random_image(g, 70)
    yr = inputs.random_detector(g, 71)
    assert_parity(host(geo.forward(dev(fr))), o.forward(fr), what="forward")
    assert_parity(host(geo.backproject(dev(yr))), o.adjoint(yr), what="adjoint")


@pytest.mark.parametrize("lr", [True, False])
@pytest.mark.parametrize("mask_nx", [5, 32])
def test_nonuniform_q_and_mask_period(oracle_mod, lr, mask_nx):
    """q nodes off a uniform grid (spectrum bins from the q table) and mask
    periods other than 16."""
    rng = np.random.Generator(np.random.PCG64(600 + mask_nx))
    x = (-40.0, 40.0) if lr else (-37.3, 41.1)
    g = ragged_geometry(21, 10, 9, 12, 10, 40, 402.57, x=x, mask_nx=mask_nx)
    g = g.with_(q=np.sort(rng.uniform(0.5, 3.5, 40)))
    o = oracle_mod.Oracle(g)
    assert o.margins()["mask_edge_mm"] > 1e-5
    geo = csx.Geometry(g)
    assert geo.info()["symmetric_lr"] == int(lr)
    f = inputs.random_image(g, 31)
    y = inputs.random_detector(g, 32)
    assert_parity(host(geo.forward(dev(f))), o.forward(f), what="forward")
    assert_parity(host(geo.backproject(dev(y))), o.adjoint(y), what="adjoint")


@pytest.mark.parametrize("name", ["slice32"])
def test_workload_operators(oracle_mod, name):
    w, g, f, y = workload_data(name)
    o = oracle_mod.Oracle(g)
    geo = csx.Geometry(g)
    e1 = assert_parity(host(geo.forward(dev(f))), o.forward(f), what="forward phantom")
    e2 = assert_parity(host(geo.backproject(dev(y))), o.adjoint(y), what="adjoint counts")
    fr = inputs.random_image(g, 5)
    e3 = assert_parity(host(geo.forward(dev(fr))), o.forward(fr), what="forward random")
    print(f"{name}: fwd {e1:.2e} adj {e2:.2e} fwd-rand {e3:.2e}")


@pytest.fixture(scope="module")
def s128(oracle_mod):
    """The benchmark's 128^2 x 64 q slice with its stored counts, and a cache of
    the oracle's full-size results (each operator takes seconds on the host)."""
    w, g, f, y = workload_data("slice128")
    return dict(w=w, g=g, f=f, y=y, o=oracle_mod.Oracle(g), geo=csx.Geometry(g), cache={})


def oracle_cached(s, key, fn):
    if key not in s["cache"]:
        t0 = time.perf_counter()
        s["cache"][key] = fn()
        print(f"[oracle {key}: {time.perf_counter() - t0:.1f} s]", flush=True)
    return s["cache"][key]


def test_slice128_forward_every_pixel(s128):
    """Alg. 1 at the benchmark's size and launch shape: every one of the
    16384 detector pixels against the oracle."""
    g, f, o, geo = s128["g"], s128["f"], s128["o"], s128["geo"]
    ref = oracle_cached(s128, "forward f", lambda: o.forward(f))
    got = host(geo.forward(dev(f)))
    assert np.all(got >= 0)
    e = assert_parity(got, ref, what="slice128 forward (all pixels)")
    print(f"slice128 forward: rel-L2 {e:.3e}")


def test_slice128_adjoint_every_voxel(s128):
    """Alg. 3 at the benchmark's size: every voxel and q of A^T y."""
    g, y, o, geo = s128["g"], s128["y"], s128["o"], s128["geo"]
    ref = oracle_cached(s128, "adjoint y", lambda: o.adjoint(y))
    got = host(geo.backproject(dev(y)))
    assert np.all(got >= 0)
    e = assert_parity(got, ref, what="slice128 adjoint (all voxels)")
    print(f"slice128 adjoint: rel-L2 {e:.3e}")
    fr = inputs.random_image(g, 9)
    yr = inputs.random_detector(g, 10)
    lhs = float(np.sum(host(geo.forward(dev(fr))) * yr))
    rhs = float(np.sum(fr * host(geo.backproject(dev(yr)))))
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


def first_order_dJ(y, z, dz):
    w = np.where(z > 0, 1.0 - y / np.where(z > 0, z, 1.0), 0.0)
    return float(np.sum(w * dz))


def test_slice128_recon_step(oracle_mod, s128):
    """One Alg. 5 iteration (forward, ratio, adjoint, update, float64 J) at the
    benchmark's size from the uniform start."""
    w, g, y, o, geo = s128["w"], s128["g"], s128["y"], s128["o"], s128["geo"]
    b1 = oracle_cached(s128, "sensitivity", o.sensitivity)
    f0 = oracle_mod.uniform_start(y, b1)
    ref_f, ref_J = oracle_cached(s128, "step 1", lambda: o.recon_step(y, None, f0, w.beta, b1=b1))
    fd = dev(f0)
    J = torch.zeros(1, dtype=torch.float64, device="cuda")
    geo.recon_step(dev(y), fd, w.beta, J=J)
    e = assert_parity(host(fd), ref_f, what="slice128 recon_step f")
    z = oracle_cached(s128, "z0", lambda: o.forward(f0))
    dJ = J.item() - ref_J
    print(f"slice128 recon_step: f rel-L2 {e:.3e}, J {J.item():.10e} vs {ref_J:.10e} (dJ {dJ:.3e})")
    assert abs(dJ) <= objective_tolerance(y, z, 1e-5) + 1e-12 * abs(ref_J)
    # the float64 objective arithmetic is exact up to the float32 model mean it
    # is given: dJ equals the first-order effect of the measured z difference
    zg = host(geo.forward(dev(f0)))
    pred = first_order_dJ(y, z, zg - z)
    assert abs(dJ - pred) <= 1e-3 * abs(dJ) + 1e-9 * abs(ref_J)


def test_slice128_recon_three_iterations(oracle_mod, s128):
    """Three Alg. 5 iterations from the uniform start (the library's own
    sensitivity and start) against the oracle's, f and every J."""
    w, g, y, o, geo = s128["w"], s128["g"], s128["y"], s128["o"], s128["geo"]
    b1 = oracle_cached(s128, "sensitivity", o.sensitivity)
    f0 = oracle_mod.uniform_start(y, b1)
    f1, J0 = oracle_cached(s128, "step 1", lambda: o.recon_step(y, None, f0, w.beta, b1=b1))
    f, hist = f1, [J0]
    for t in range(2):
        f, J = oracle_cached(s128, f"step {t + 2}", lambda: o.recon_step(y, None, f, w.beta, b1=b1))
        hist.append(J)
    z3 = oracle_cached(s128, "z3", lambda: o.forward(f))
    hist.append(oracle_mod.objective_from_mean(y, z3, f, w.beta))
    fd = torch.empty((g.nz, g.nx, g.nq), dtype=torch.float32, device="cuda")
    Jg = geo.recon(dev(y), fd, 3, w.beta, init_uniform=True)
    e = assert_parity(host(fd), f, what="slice128 recon x3 f")
    ref_J = np.array(hist)
    print(f"slice128 recon x3: f rel-L2 {e:.3e}, J {Jg} vs {ref_J}, max |dJ| / J {np.max(np.abs(Jg - ref_J) / ref_J):.3e}")
    assert np.max(np.abs(Jg - ref_J)) <= objective_tolerance(y, z3, 1e-5) + 1e-12 * abs(ref_J[0])
    assert np.all(np.diff(Jg) <= 1e-7 * np.abs(Jg[1:]))


def test_adjoint_identity_fp32(oracle_mod):
    w, g, f, y = workload_data("slice32")
    geo = csx.Geometry(g)
    fr = inputs.random_image(g, 1)
    yr = inputs.random_detector(g, 2)
    lhs = float(np.sum(host(geo.forward(dev(fr))) * yr))
    rhs = float(np.sum(fr * host(geo.backproject(dev(yr)))))
    assert abs(lhs - rhs) <= 2e-6 * abs(lhs)


def test_deterministic_repeat():
    w, g, f, y = workload_data("slice32")
    geo = csx.Geometry(g)
    fd, yd = dev(f), dev(y)
    a1, a2 = host(geo.forward(fd)), host(geo.forward(fd))
    b1, b2 = host(geo.backproject(yd)), host(geo.backproject(yd))
    assert np.array_equal(a1, a2) and np.array_equal(b1, b2)


@pytest.mark.parametrize("beta", [1e-3, 0.0])
def test_recon_step_parity(oracle_mod, beta):
    w, g, f, y = workload_data("slice32")
    o = oracle_mod.Oracle(g)
    geo = csx.Geometry(g)
    f0 = oracle_mod.uniform_start(y, o.sensitivity())
    fd = dev(f0)
    J = torch.zeros(1, dtype=torch.float64, device="cuda")
    geo.recon_step(dev(y), fd, beta, J=J)
    ref_f, ref_J = o.recon_step(y, None, f0, beta)
    assert_parity(host(fd), ref_f, what="recon_step f")
    z = o.forward(f0)
    assert abs(J.item() - ref_J) <= objective_tolerance(y, z, 1e-5) + 1e-12 * abs(ref_J)
    # sharper: the float64 objective arithmetic is exact up to the float32 z it
    # is given -- J_gpu - J_oracle equals the first-order effect of the
    # measured z difference, sum (1 - y/z) dz
    zg = host(geo.forward(dev(f0)))
    dz = zg - z
    pred = float(np.sum(np.where(z > 0, 1.0 - y / np.where(z > 0, z, 1.0), 0.0) * dz))
    assert abs((J.item() - ref_J) - pred) <= 1e-3 * abs(J.item() - ref_J) + 1e-9 * abs(ref_J)


def test_recon_matches_oracle_iterations(oracle_mod):
    w, g, f, y = workload_data("slice32")
    o = oracle_mod.Oracle(g)
    geo = csx.Geometry(g)
    fd = torch.empty((g.nz, g.nx, g.nq), dtype=torch.float32, device="cuda")
    Jg = geo.recon(dev(y), fd, w.n_iter, w.beta, init_uniform=True)
    f0 = oracle_mod.uniform_start(y, o.sensitivity())
    ref_f, ref_J = o.recon(y, None, f0, w.n_iter, w.beta)
    e = rel_l2(host(fd), ref_f)
    assert e <= 1e-4, e
    # iterates may drift apart to 1e-4 over the run: bound J with that level
    z = o.forward(ref_f)
    assert np.max(np.abs(Jg - ref_J)) <= objective_tolerance(y, z, 1e-4) + 1e-12 * abs(ref_J[0])
    assert np.all(np.diff(Jg) <= 1e-7 * np.abs(Jg[1:]))


def test_recon_resume_equals_continuous():
    w, g, f, y = workload_data("slice32")
    geo = csx.Geometry(g)
    yd = dev(y)
    fa = torch.empty((g.nz, g.nx, g.nq), dtype=torch.float32, device="cuda")
    Ja = geo.recon(yd, fa, 6, w.beta)
    fb = torch.empty_like(fa)
    Jb1 = geo.recon(yd, fb, 3, w.beta)
    Jb2 = geo.recon(yd, fb, 3, w.beta, init_uniform=False)
    assert torch.equal(fa, fb)
    np.testing.assert_array_equal(Ja[:4], Jb1)
    np.testing.assert_array_equal(Ja[3:], Jb2)


def test_zero_mean_with_counts_is_an_error():
    g = ragged_geometry(7, 6, 6, 8, 8, 16, 402.11)
    g = g.with_(mask=np.zeros_like(g.mask))        # every pair blocked: A f = 0
    geo = csx.Geometry(g)
    fd = torch.ones((g.nz, g.nx, g.nq), dtype=torch.float32, device="cuda")
    y = torch.zeros(g.ndy, g.ndx, dtype=torch.float32, device="cuda")
    assert np.all(host(geo.forward(fd)) == 0)
    y[0, 0] = 3.0
    with pytest.raises(csx.CsxError) as ei:
        geo.recon(y, fd, 1, 1e-3, init_uniform=False)
    assert ei.value.code == csx.CSX_ENUMERIC
    y[0, 0] = -1.0
    with pytest.raises(csx.CsxError) as ei:
        geo.recon(y, fd, 1, 1e-3, init_uniform=False)
    assert ei.value.code == csx.CSX_EINVAL


def test_binding_rejects_wrong_buffers():
    w, g, f, y = workload_data("slice32")
    geo = csx.Geometry(g)
    with pytest.raises(ValueError):
        geo.forward(torch.zeros(10, device="cuda"))
    with pytest.raises(ValueError):
        geo.forward(torch.zeros(g.nz, g.nx, g.nq, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        geo.forward(torch.zeros(g.nz, g.nx, g.nq))


@pytest.mark.parametrize("name", ["slice128_open1", "slice128_open01"])
def test_sparse_masks(oracle_mod, name):
    """1 % and 0.1 % open masks: every pixel of the forward (most pixels see
    no open cell at 0.1 %), sampled voxels of the adjoint."""
    w, g, f, y = workload_data(name)
    o = oracle_mod.Oracle(g)
    geo = csx.Geometry(g)
    ref = o.forward(f)
    assert np.count_nonzero(ref) > 0
    gg = host(geo.forward(dev(f)))
    # same support (identical mask decisions): no GPU flux where the oracle
    # has none, none missing where the oracle has a visible amount (phantom
    # tails below float32's range are 0 in the library's float32 image)
    assert np.all(gg[ref == 0] == 0)
    assert np.all(gg[ref > 1e-6 * ref.max()] > 0)
    e = assert_parity(gg, ref, what=f"{name} forward (all pixels)")
    print(f"{name}: forward rel-L2 {e:.3e}, {np.count_nonzero(ref)} of {ref.size} pixels lit")
    rng = np.random.Generator(np.random.PCG64(78))
    vox = np.sort(rng.choice(g.nvox, 24, replace=False))
    yr = inputs.random_detector(g, 3)
    bb = host(geo.backproject(dev(yr))).reshape(g.nvox, g.nq)
    assert_parity(bb[vox], o.adjoint_voxels(yr, vox), what=f"{name} adjoint sampled")


def test_valu_peak_probe():
    """The FMA-chain probe the roofline quotes beside the published rate: at
    most the non-packed FP32 issue rate (256 CUs x 4 SIMDs x 16 lanes x
    2.4 GHz), and at least a third of it (a whole-chip launch)."""
    spec = 256 * 4 * 16 * 2.4e9
    v = csx.valu_peak()
    print(f"VALU FMA-chain rate {v / 1e12:.2f} T lane-ops/s ({v / spec:.3f} of {spec / 1e12:.2f})")
    assert spec / 3 < v <= 1.02 * spec


@pytest.mark.parametrize("lr", [True, False])
@pytest.mark.parametrize("case", ["high_e_lo", "q_near_zero"])
def test_uniform_q_spectrum_pads(oracle_mod, case, lr):
    """Uniform q grids at the ends of the padded spectrum table.  The uniform-grid
    operators read the table at the bin coordinate kappa q/dE + b0 without a
    clamp, from zero pads sized by the band test.  A high e_lo puts b0 far below
    0 (a long lower pad); q_min near 0 makes the implied upper pad exceed the
    table limit, and the clamped generic path runs instead."""
    x = (-40.0, 40.0) if lr else (-37.3, 41.1)
    g = ragged_geometry(41 + lr, 12, 10, 14, 12, 40, 402.57, x=x)
    if case == "high_e_lo":
        g = g.with_(e_lo=60.0, e_hi=160.0, phi=inputs.kramers_histogram(64, 60.0, 160.0))
    else:
        g = g.with_(q=np.linspace(0.02, 3.5, 40))
    o = oracle_mod.Oracle(g)
    assert o.margins()["mask_edge_mm"] > 1e-5
    geo = csx.Geometry(g)
    assert geo.info()["symmetric_lr"] == int(lr)
    f = inputs.random_image(g, 51)
    y = np.random.Generator(np.random.PCG64(52)).uniform(0.0, 1.0, (g.ndy, g.ndx))
    ref = o.forward(f)
    assert np.count_nonzero(ref) > ref.size // 4
    assert_parity(host(geo.forward(dev(f))), ref, what=f"forward {case}")
    assert_parity(host(geo.backproject(dev(y))), o.adjoint(y), what=f"adjoint {case}")

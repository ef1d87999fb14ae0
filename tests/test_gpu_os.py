"""Ordered subsets (Alg. 6) on the GPU against the FP64 oracle: the paper's
64-subset partition on the 32^2 workload, a ragged scan without the x-mirror,
one subset against the plain solver, and argument checks.

Tolerance: one sweep is P sub-steps, each as accurate as an Alg. 5 step
(rel-L2 <= 1e-5 per step); the errors of a few sweeps stay below 1e-4, the
bar of the 20-iteration Alg. 5 test, and J follows f to first order."""
import numpy as np
import pytest
import torch

from paper_1603_06400_amd import csx

from .gpu_helpers import ragged_geometry, rel_l2, workload_data

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def test_os_slice32_matches_oracle(oracle_mod):
    w, g, f, y = workload_data("slice32")
    o = oracle_mod.Oracle(g)
    subs = oracle_mod.os_partition(g.ndy, g.ndx, 8, 16)
    f0 = oracle_mod.uniform_start(y, o.sensitivity())
    ref_f, ref_J = o.recon_os(y, None, f0, 2, w.beta, subs)
    geo = csx.Geometry(g)
    fd = geo.new_image()
    J = geo.recon_os(dev(y), fd, 2, w.beta, 8, 16)
    assert rel_l2(host(fd), ref_f) <= 1e-4
    np.testing.assert_allclose(J, ref_J, rtol=1e-5)
    assert J[2] < J[1] < J[0]


def test_os_ragged_without_mirror(oracle_mod):
    g = ragged_geometry(3, 12, 11, 12, 8, 30, 402.57)
    o = oracle_mod.Oracle(g)
    assert o.margins()["mask_edge_mm"] > 1e-4
    f = np.random.Generator(np.random.PCG64(4)).uniform(0.0, 1.0, size=(g.nz, g.nx, g.nq))
    y = np.random.Generator(np.random.PCG64(5)).poisson(np.maximum(o.forward(f), 0.0)).astype(np.float64)
    geo = csx.Geometry(g)
    assert geo.info()["symmetric_lr"] == 0
    subs = oracle_mod.os_partition(g.ndy, g.ndx, 2, 4)
    f0 = oracle_mod.uniform_start(y, o.sensitivity())
    ref_f, ref_J = o.recon_os(y, None, f0, 2, 1e-3, subs)
    fd = geo.new_image()
    J = geo.recon_os(dev(y), fd, 2, 1e-3, 2, 4)
    assert rel_l2(host(fd), ref_f) <= 1e-4
    np.testing.assert_allclose(J, ref_J, rtol=1e-5)


@pytest.mark.parametrize("lr", [True, False])
def test_os_wide_q_grid_matches_oracle(oracle_mod, lr):
    """nq = 40 (64-wide default q chunks).  Subset adjoints over their short
    class lists run 32-wide chunks when they evaluate the pair factors and
    64-wide ones when they read the factor store in subset order (the
    default here).  The sweeps follow the oracle, repeat bit for bit, and
    forcing 32-wide chunks everywhere changes them only by float32 rounding
    (each q node's sum is the same, its lanes reduced in another order)."""
    x = (-40.0, 40.0) if lr else (-37.3, 41.1)
    g = ragged_geometry(7 + lr, 12, 10, 16, 8, 40, 402.57, x=x)
    o = oracle_mod.Oracle(g)
    assert o.margins()["mask_edge_mm"] > 1e-5
    f = np.random.Generator(np.random.PCG64(6)).uniform(0.0, 1.0, size=(g.nz, g.nx, g.nq))
    y = np.random.Generator(np.random.PCG64(7)).poisson(np.maximum(o.forward(f), 0.0)).astype(np.float64)
    geo = csx.Geometry(g)
    assert geo.info()["symmetric_lr"] == int(lr)
    assert geo.get_launch()["adj_qw"] == 64
    subs = oracle_mod.os_partition(g.ndy, g.ndx, 2, 4)
    f0 = oracle_mod.uniform_start(y, o.sensitivity())
    ref_f, ref_J = o.recon_os(y, None, f0, 2, 1e-3, subs)
    fd = geo.new_image()
    J = geo.recon_os(dev(y), fd, 2, 1e-3, 2, 4)
    assert rel_l2(host(fd), ref_f) <= 1e-4
    np.testing.assert_allclose(J, ref_J, rtol=1e-5)
    f1 = geo.new_image()
    J1 = geo.recon_os(dev(y), f1, 2, 1e-3, 2, 4)
    assert torch.equal(f1, fd) and np.array_equal(J1, J)
    # forcing 32-wide chunks for every adjoint
    lc = geo.get_launch()
    geo.set_launch(lc["fwd_splits"], lc["fwd_qw"], 32)
    f2 = geo.new_image()
    J2 = geo.recon_os(dev(y), f2, 2, 1e-3, 2, 4)
    assert rel_l2(host(f2), host(fd)) <= 1e-6
    np.testing.assert_allclose(J2, J, rtol=1e-9)


def test_one_subset_is_the_plain_solver():
    w, g, f, y = workload_data("slice32")
    geo = csx.Geometry(g)
    fa, fb = geo.new_image(), geo.new_image()
    Ja = geo.recon(dev(y), fa, 3, w.beta)
    Jb = geo.recon_os(dev(y), fb, 3, w.beta, 1, 2)
    assert rel_l2(host(fb), host(fa)) <= 1e-6
    np.testing.assert_allclose(Jb, Ja, rtol=1e-7)


def test_os_argument_errors():
    w, g, f, y = workload_data("slice32")
    geo = csx.Geometry(g)
    fd = geo.new_image()
    for rz, ry in [(3, 16), (8, 15), (8, 12), (0, 16)]:
        with pytest.raises(csx.CsxError) as ei:
            geo.recon_os(dev(y), fd, 1, w.beta, rz, ry)
        assert ei.value.code == csx.CSX_EINVAL


def test_os_after_a_launch_shape_change(oracle_mod):
    """The subset launches follow the handle's launch shape; a change after the
    partition was built (more forward partials) still gives the same sweep."""
    w, g, f, y = workload_data("slice32")
    geo = csx.Geometry(g)
    fa, fb = geo.new_image(), geo.new_image()
    Ja = geo.recon_os(dev(y), fa, 1, w.beta, 8, 16)
    lc = geo.get_launch()
    geo.set_launch(lc["fwd_splits"], 16, 16)
    Jb = geo.recon_os(dev(y), fb, 1, w.beta, 8, 16)
    assert rel_l2(host(fb), host(fa)) <= 1e-6
    np.testing.assert_allclose(Jb, Ja, rtol=1e-7)

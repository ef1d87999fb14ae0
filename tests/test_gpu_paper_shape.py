"""The paper's simulation shape (Sec. VII): 28 x 28 voxels x 79 q nodes and a
1536 x 2048 detector, with stand-ins for the measured spectrum and mask.

Its 1.5 million pixel classes per voxel group are beyond the interval form,
so the direct kernels run, the adjoint with its pixel classes split into tile
ranges (392 voxel groups alone would leave most of the device idle).  The
float64 oracle costs about a second per voxel here, so outputs are compared
on samples: 512 pixels of the forward, 4 voxels (every q node) of the
adjoint, each to the oracle bar.  A reconstruction step is checked by a
property that holds at any size: the surrogate update never raises J."""
import numpy as np
import pytest
import torch

from paper_1603_06400_amd import csx, inputs

from .gpu_helpers import assert_parity, rel_l2

pytestmark = pytest.mark.gpu


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


@pytest.fixture(scope="module")
def paper():
    g = inputs.paper_geometry()
    geo = csx.Geometry(g)
    return g, geo


def test_paper_shape_runs_the_split_direct_adjoint(paper):
    g, geo = paper
    assert not geo.interval_operators()["on"]
    lc = geo.get_launch()
    st = geo.factor_store()
    print(f"[paper shape: launch {lc}, factor store {st['bytes'] / 2**30:.1f} GiB in {st['build_ms']:.1f} ms]",
          flush=True)
    assert lc["adj_splits"] > 1
    # the uniform-q path with its factor store; the forward's q chunk narrowed
    # beside the 19.6 KB spectrum table; f is small, so no voxel split
    assert st["on"]
    assert lc["fwd_qw"] <= 32 and lc["fwd_splits"] == 1


def test_paper_shape_forward_sampled(oracle_mod, paper):
    g, geo = paper
    o = oracle_mod.Oracle(g)
    f = inputs.random_image(g, 31)
    got = host(geo.forward(torch.tensor(f, dtype=torch.float32, device="cuda"))).ravel()
    rng = np.random.Generator(np.random.PCG64(32))
    pix = rng.choice(g.npix, 512, replace=False)
    assert_parity(got[pix], o.forward_pixels(f, pix), what="paper-shape forward (512 pixels)")


def test_paper_shape_adjoint_sampled_and_split_invariant(oracle_mod, paper):
    g, geo = paper
    o = oracle_mod.Oracle(g)
    y = inputs.random_detector(g, 33)
    yd = torch.tensor(y, dtype=torch.float32, device="cuda")
    got = host(geo.backproject(yd)).reshape(g.nvox, g.nq)
    rng = np.random.Generator(np.random.PCG64(34))
    vox = rng.choice(g.nvox, 4, replace=False)
    assert_parity(got[vox], o.adjoint_voxels(y, vox), what="paper-shape adjoint (4 voxels)")
    # one tile range: the same sums in another order
    lc = geo.get_launch()
    geo.set_launch(lc["fwd_splits"], lc["fwd_qw"], lc["adj_qw"], 1)
    one = host(geo.backproject(yd)).reshape(g.nvox, g.nq)
    geo.set_launch(lc["fwd_splits"], lc["fwd_qw"], lc["adj_qw"], lc["adj_splits"])
    e = rel_l2(got, one)
    print(f"[paper shape: adjoint split {lc['adj_splits']} vs 1: rel-L2 {e:.2e}]", flush=True)
    assert e <= 1e-6


def test_paper_shape_step_lowers_the_objective(paper):
    g, geo = paper
    f_true = inputs.paper_phantom(g)
    ftd = torch.tensor(f_true, dtype=torch.float32, device="cuda")
    mean = host(geo.forward(ftd))
    C = 1e4 / mean.max()
    y = torch.tensor(inputs.poisson_counts(C * mean, 35), dtype=torch.float32, device="cuda")
    geo2 = csx.Geometry(g.with_(C=C))
    f = geo2.new_image()
    J = geo2.recon(y, f, 3, 1e-3, init_uniform=True)
    print(f"[paper shape: J over 3 iterations {J}]", flush=True)
    assert np.all(np.isfinite(J)) and np.all(np.diff(J) <= 1e-9 * abs(J[0]))

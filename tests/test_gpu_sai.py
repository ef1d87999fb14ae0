"""Scatter-angle interpolation (Sec. III-B) on the GPU against the FP64
oracle's SAI operators: forward and adjoint for both interpolation rules on
ragged, mirror-path and workload geometries (the full 128^2 x 64q slice in
the benchmark's launch configuration included), the adjoint identity,
bit-exact repeats, the table's angle range, the solver with interpolated
operators, and the argument checks.

Tolerance: rel-L2 <= 1e-5 as for the exact operators.  The nearest-node
rule decides angles close to a midpoint between two nodes in float64 on the
GPU too, so both sides take the same node there.
"""
import numpy as np
import pytest
import torch

from paper_1603_06400_amd import csx, inputs

from .gpu_helpers import assert_parity, ragged_geometry, rel_l2, workload_data

pytestmark = pytest.mark.gpu

INTERP = {0: "nearest", 1: "linear"}


def dev(a):
    return torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


CASES = [
    # (seed, nx, nz, ndx, ndy, nq, z_min, x range)
    (1, 10, 7, 12, 10, 24, 402.57, (-37.3, 41.1)),   # off-centre: no mirror path
    (5, 3, 23, 13, 8, 17, 401.9, (-37.3, 41.1)),     # odd sizes, ragged tiles
    (13, 34, 7, 22, 8, 70, 403.93, (-40.0, 40.0)),   # mirror path, voxel pairs beyond one batch
    (15, 16, 16, 16, 16, 8, 404.13, (-40.0, 40.0)),  # mirror path, 8 q nodes
]


@pytest.mark.parametrize("interp", [1, 0], ids=["linear", "nearest"])
@pytest.mark.parametrize("case", CASES, ids=[f"c{c[0]}" for c in CASES])
def test_sai_operators_match_oracle(oracle_mod, case, interp):
    print(f"[sai {case} {INTERP[interp]}]", flush=True)
    g = ragged_geometry(*case[:7], x=case[7])
    o = oracle_mod.Oracle(g)
    assert o.margins()["mask_edge_mm"] > 1e-4
    geo = csx.Geometry(g)
    assert geo.info()["symmetric_lr"] == int(case[7][0] == -case[7][1])
    tm = o.max_angle()
    nt = 250
    geo.sai_config(nt, INTERP[interp], tm)
    f = inputs.random_image(g, 500 + case[0])
    y = inputs.random_detector(g, 600 + case[0])
    assert_parity(host(geo.forward_sai(dev(f))), o.forward_sai(f, nt, tm, interp), what="forward_sai")
    assert_parity(host(geo.backproject_sai(dev(y))), o.adjoint_sai(y, nt, tm, interp), what="adjoint_sai")


@pytest.mark.parametrize("nt", [2, 64, 250, 1024, 2000, 2048])
def test_sai_table_sizes_slice32(oracle_mod, nt):
    """Linear interpolation at the extremes of the table size (2 nodes: one
    interval; 2048: the largest table, one wave per adjoint block), the
    paper's 250 and 2000, with the library's own angle range."""
    w, g, f, y = workload_data("slice32")
    o = oracle_mod.Oracle(g)
    geo = csx.Geometry(g)
    geo.sai_config(nt, "linear")
    tm = geo.sai_info()["theta_max"]
    assert_parity(host(geo.forward_sai(dev(f))), o.forward_sai(f, nt, tm, 1), what=f"forward_sai nt={nt}")
    assert_parity(host(geo.backproject_sai(dev(y))), o.adjoint_sai(y, nt, tm, 1), what=f"adjoint_sai nt={nt}")


@pytest.mark.parametrize("interp", ["linear", "nearest"])
@pytest.mark.parametrize("tm", [0.3, float(np.pi / 6)])
def test_sai_table_narrower_than_the_angles(oracle_mod, interp, tm):
    """An explicit theta_max: 0.3 rad, below the 32^2 slice's largest pair
    angle (0.334 rad), so that pairs beyond it take the last node on both
    sides, and the paper's pi/6, a table wider than the angles."""
    w, g, f, y = workload_data("slice32")
    o = oracle_mod.Oracle(g)
    assert (o.max_angle() > tm) == (tm < 0.33)
    geo = csx.Geometry(g)
    geo.sai_config(250, interp, tm)
    assert geo.sai_info()["theta_max"] == tm
    it = 1 if interp == "linear" else 0
    assert_parity(host(geo.forward_sai(dev(f))), o.forward_sai(f, 250, tm, it), what="forward_sai clamp")
    assert_parity(host(geo.backproject_sai(dev(y))), o.adjoint_sai(y, 250, tm, it), what="adjoint_sai clamp")


def test_sai_many_q_nodes(oracle_mod):
    """160 q nodes: the matrix-core products run a ragged K (W = f s^T) and a
    ragged N and K split (b = V s)."""
    g = ragged_geometry(31, 10, 9, 12, 10, 160, 402.57, x=(-40.0, 40.0))
    o = oracle_mod.Oracle(g)
    assert o.margins()["mask_edge_mm"] > 1e-4
    geo = csx.Geometry(g)
    tm = o.max_angle()
    geo.sai_config(97, "linear", tm)
    f = inputs.random_image(g, 51)
    y = inputs.random_detector(g, 52)
    assert_parity(host(geo.forward_sai(dev(f))), o.forward_sai(f, 97, tm, 1), what="forward_sai nq=160")
    assert_parity(host(geo.backproject_sai(dev(y))), o.adjoint_sai(y, 97, tm, 1), what="adjoint_sai nq=160")


def test_sai_theta_max_covers_every_pair(oracle_mod):
    for name in ["slice32", "slice128"]:
        w, g, f, y = workload_data(name)
        geo = csx.Geometry(g)
        geo.sai_config(100, "nearest")
        info = geo.sai_info()
        assert info["nt"] == 100 and info["interp"] == "nearest"
        ref = oracle_mod.Oracle(g).max_angle()
        assert ref <= info["theta_max"] <= ref * (1 + 3e-7), (name, ref, info["theta_max"])


def test_sai_slice128_full_parity(oracle_mod):
    """The full 128^2 x 64q slice in the launch configuration the benchmark
    times, every output against the oracle, and the adjoint identity."""
    w, g, f, y = workload_data("slice128")
    o = oracle_mod.Oracle(g)
    geo = csx.Geometry(g)
    geo.sai_config(250, "linear")
    tm = geo.sai_info()["theta_max"]
    gs = host(geo.forward_sai(dev(f)))
    assert_parity(gs, o.forward_sai(f, 250, tm, 1), what="forward_sai 128")
    bs = host(geo.backproject_sai(dev(y)))
    assert_parity(bs, o.adjoint_sai(y, 250, tm, 1), what="adjoint_sai 128")
    fr = inputs.random_image(g, 19)
    yr = inputs.random_detector(g, 20)
    lhs = float(np.sum(host(geo.forward_sai(dev(fr))) * yr))
    rhs = float(np.sum(fr * host(geo.backproject_sai(dev(yr)))))
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)
    # distance from the exact operators (an approximation, not a parity bar)
    ge, be = host(geo.forward(dev(f))), host(geo.backproject(dev(y)))
    print(f"SAI nt=250 linear vs exact: forward {rel_l2(gs, ge):.3e} adjoint {rel_l2(bs, be):.3e}")
    assert rel_l2(gs, ge) < 2e-2 and rel_l2(bs, be) < 2e-2


def test_sai_adjoint_scale_range(oracle_mod):
    """The adjoint's fixed-point histograms follow the data's magnitude: y
    scaled by 1e-20 and 1e20 gives b scaled alike, to the parity bar (near
    1e30 the float32 histogram V itself would overflow); a NaN in y gives NaN
    everywhere."""
    w, g, f, y = workload_data("slice32")
    o = oracle_mod.Oracle(g)
    geo = csx.Geometry(g)
    geo.sai_config(250, "linear")
    tm = geo.sai_info()["theta_max"]
    ref = o.adjoint_sai(y, 250, tm, 1)
    for k in (1e-20, 1e20):
        assert_parity(host(geo.backproject_sai(dev(y * k))) / k, ref, what=f"adjoint_sai y*{k:g}")
    # one large pixel among small ones: the small ones' share survives
    y2 = y.copy()
    y2.flat[77] = 1e6 * y.max()
    assert_parity(host(geo.backproject_sai(dev(y2))), o.adjoint_sai(y2, 250, tm, 1), what="adjoint_sai spike")
    yn = y.copy()
    yn.flat[5] = np.nan
    assert np.all(np.isnan(host(geo.backproject_sai(dev(yn)))))
    assert_parity(host(geo.backproject_sai(dev(y))), ref, what="adjoint_sai after NaN")


@pytest.mark.parametrize("interp", ["linear", "nearest"])
def test_sai_adjoint_identity_and_repeat(interp):
    w, g, f, y = workload_data("slice32")
    geo = csx.Geometry(g)
    geo.sai_config(250, interp)
    fr, yr = dev(inputs.random_image(g, 3)), dev(inputs.random_detector(g, 4))
    a1, a2 = host(geo.forward_sai(fr)), host(geo.forward_sai(fr))
    b1, b2 = host(geo.backproject_sai(yr)), host(geo.backproject_sai(yr))
    assert np.array_equal(a1, a2) and np.array_equal(b1, b2)
    lhs = float(np.sum(a1 * host(yr)))
    rhs = float(np.sum(host(fr) * b1))
    assert abs(lhs - rhs) <= 2e-6 * abs(lhs)


def test_sai_solver_matches_oracle(oracle_mod):
    """Alg. 5 with both operators interpolated: the oracle's update driven by
    its SAI forward and adjoint (sensitivity from the SAI adjoint too)."""
    w, g, f, y = workload_data("slice32")
    o = oracle_mod.Oracle(g)
    geo = csx.Geometry(g)
    geo.sai_config(250, "linear")
    tm = geo.sai_info()["theta_max"]
    geo.set_operator(forward_sai=True, adjoint_sai=True)
    fd = geo.new_image()
    n = 6
    J = geo.recon(dev(y), fd, n, w.beta)
    b1 = o.adjoint_sai(np.ones((g.ndy, g.ndx)), 250, tm, 1)
    fr = oracle_mod.uniform_start(y, b1)
    Jr = []
    for _ in range(n + 1):
        z = o.forward_sai(fr, 250, tm, 1)
        Jr.append(oracle_mod.objective_from_mean(y, z, fr, w.beta))
        if len(Jr) <= n:
            fr = oracle_mod.em_update(fr, b1, o.adjoint_sai(oracle_mod.poisson_ratio(y, z), 250, tm, 1), w.beta)
    assert rel_l2(host(fd), fr) <= 1e-4
    np.testing.assert_allclose(J, Jr, rtol=1e-6)
    assert np.all(np.diff(J) <= 1e-7 * np.abs(J[1:]))   # a consistent pair: monotone
    # back to the exact operators: the plain run again
    geo.set_operator()
    fe = geo.new_image()
    Je = geo.recon(dev(y), fe, 2, w.beta)
    ref_f, ref_J = o.recon(y, None, oracle_mod.uniform_start(y, o.sensitivity()), 2, w.beta)
    assert rel_l2(host(fe), ref_f) <= 1e-4
    np.testing.assert_allclose(Je, ref_J, rtol=1e-6)


@pytest.mark.parametrize("ops", [(True, False), (False, True)])
def test_sai_one_operator(oracle_mod, ops):
    """Table 1's single-operator rows: one step with only the forward or only
    the adjoint interpolated."""
    w, g, f, y = workload_data("slice32")
    o = oracle_mod.Oracle(g)
    geo = csx.Geometry(g)
    geo.sai_config(250, "nearest")
    tm = geo.sai_info()["theta_max"]
    geo.set_operator(*ops)
    f0 = np.asarray(f, dtype=np.float32).astype(np.float64) + 0.05
    fd = dev(f0)
    geo.recon_step(dev(y), fd, w.beta)
    fwd = (lambda v: o.forward_sai(v, 250, tm, 0)) if ops[0] else o.forward
    adj = (lambda v: o.adjoint_sai(v, 250, tm, 0)) if ops[1] else o.adjoint
    b1 = adj(np.ones((g.ndy, g.ndx)))
    ref = oracle_mod.em_update(f0, b1, adj(oracle_mod.poisson_ratio(y, fwd(f0))), w.beta)
    assert rel_l2(host(fd), ref) <= 1e-4


def test_sai_errors():
    w, g, f, y = workload_data("slice32")
    geo = csx.Geometry(g)
    fd, yd = dev(f), dev(y)
    for call in (lambda: geo.forward_sai(fd), lambda: geo.backproject_sai(yd), lambda: geo.sai_info(),
                 lambda: geo.set_operator(forward_sai=True)):
        with pytest.raises(csx.CsxError) as ei:
            call()
        assert ei.value.code == csx.CSX_EINVAL
    for nt, interp, tm in [(1, 1, 0.0), (csx.SAI_MAX_NODES + 1, 1, 0.0), (10, 2, 0.0), (10, 1, -0.1),
                           (10, 1, float("nan")), (10, 1, 4.0)]:
        with pytest.raises(csx.CsxError) as ei:
            csx._check(csx.lib().csx_sai_config(geo._h, nt, interp, tm))
        assert ei.value.code == csx.CSX_EINVAL
    geo.sai_config(64, "linear")
    with pytest.raises(csx.CsxError):
        csx._check(csx.lib().csx_set_operator(geo._h, 4))
    geo.set_operator(adjoint_sai=True)
    b = csx.Batch([geo])
    with pytest.raises(csx.CsxError) as ei:
        b.recon([yd], [geo.new_image()], 1, w.beta)
    assert ei.value.code == csx.CSX_EINVAL
    geo.set_operator()
    b.recon([yd], [geo.new_image()], 1, w.beta)


def test_sai_ordered_subsets_match_oracle(oracle_mod):
    """Alg. 6 (64 subsets) with both operators interpolated, as the paper runs
    its reconstructions: one sweep against the oracle's sub-steps driven by its
    SAI operators (subset forward, subset adjoint, subset sensitivities); then
    back to the exact operators, the exact sweep again."""
    w, g, f, y = workload_data("slice32")
    o = oracle_mod.Oracle(g)
    geo = csx.Geometry(g)
    geo.sai_config(250, "linear")
    tm = geo.sai_info()["theta_max"]
    geo.set_operator(forward_sai=True, adjoint_sai=True)
    fd = geo.new_image()
    J = geo.recon_os(dev(y), fd, 1, w.beta, 8, 16)
    subs = oracle_mod.os_partition(g.ndy, g.ndx, 8, 16)
    P = len(subs)
    fwd = lambda v: o.forward_sai(v, 250, tm, 1)
    adj = lambda v: o.adjoint_sai(v, 250, tm, 1)
    yf = y.reshape(-1)
    b1 = []
    for pix in subs:
        ind = np.zeros(g.npix)
        ind[pix] = 1.0
        b1.append(adj(ind.reshape(g.ndy, g.ndx)))
    fr = oracle_mod.uniform_start(y, adj(np.ones((g.ndy, g.ndx)))).reshape(g.nz, g.nx, g.nq)
    J0 = oracle_mod.objective_from_mean(y, fwd(fr), fr, w.beta)
    for p, pix in enumerate(subs):
        rho = np.zeros(g.npix)
        rho[pix] = oracle_mod.poisson_ratio(yf[pix], fwd(fr).reshape(-1)[pix])
        fr = oracle_mod.em_update(fr, b1[p], adj(rho.reshape(g.ndy, g.ndx)), w.beta / P)
    J1 = oracle_mod.objective_from_mean(y, fwd(fr), fr, w.beta)
    assert rel_l2(host(fd), fr) <= 1e-4
    np.testing.assert_allclose(J, [J0, J1], rtol=1e-5)
    # the exact operators again: the subset sensitivities are rebuilt
    geo.set_operator()
    fe = geo.new_image()
    Je = geo.recon_os(dev(y), fe, 1, w.beta, 8, 16)
    ref = csx.Geometry(g)
    fe2 = ref.new_image()
    Je2 = ref.recon_os(dev(y), fe2, 1, w.beta, 8, 16)
    assert torch.equal(fe, fe2)
    np.testing.assert_array_equal(Je, Je2)

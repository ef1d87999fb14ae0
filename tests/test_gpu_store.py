"""The factor store: the exact operators reading every class's pair factors
(kappa, A, mask values) from device records built once per geometry, against
the same operators evaluating them on the fly, and both against the FP64
oracle.

The records hold the values the on-the-fly kernels compute, by the same code
in the same translation unit, and the operators sum them in the same order:
the two paths give the same outputs bit for bit, and each is within the oracle
bar (rel-L2 <= 1e-5, element cap 1e-4).  The parity tests of the other modules
run with the store (csx_init_geometry builds it for every geometry of this
size that takes the uniform-q operators); this module keeps the on-the-fly
path under the same bar."""
import numpy as np
import pytest
import torch

from paper_1603_06400_amd import csx, inputs

from .gpu_helpers import assert_parity, ragged_geometry, rel_l2, workload_data
from .test_gpu_parity import RAGGED, SYMMETRIC

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def _both_paths(geo, f, y):
    # the class-record store serves the direct kernels (the interval form,
    # when built, takes precedence for the full operators)
    geo.set_interval_operators(False)
    assert geo.factor_store()["on"]
    fs, bs = host(geo.forward(dev(f))), host(geo.backproject(dev(y)))
    geo.set_factor_store(False)
    assert not geo.factor_store()["on"]
    fo, bo = host(geo.forward(dev(f))), host(geo.backproject(dev(y)))
    geo.set_factor_store(True)
    assert geo.factor_store()["on"]
    return fs, bs, fo, bo


CASES = [("ragged", c) for c in RAGGED[:3]] + [("symmetric", c) for c in SYMMETRIC]


@pytest.mark.parametrize("kind,case", CASES, ids=[f"{k[0]}{c[0]}" for k, c in CASES])
def test_store_and_on_the_fly_agree_and_match_oracle(oracle_mod, kind, case):
    print(f"[store {kind} {case}]", flush=True)
    g = ragged_geometry(*case) if kind == "ragged" else ragged_geometry(*case, x=(-40.0, 40.0))
    o = oracle_mod.Oracle(g)
    geo = csx.Geometry(g)
    if not geo.factor_store()["on"]:
        # a q grid whose padded spectrum table would exceed the LDS budget
        # (8 nodes: the pad reaches past 2048 entries) takes the generic
        # operators, which have no store
        with pytest.raises(csx.CsxError) as ei:
            geo.set_factor_store(True)
        assert ei.value.code == csx.CSX_EINVAL
        return
    f = inputs.random_image(g, 700 + case[0])
    y = inputs.random_detector(g, 800 + case[0])
    fs, bs, fo, bo = _both_paths(geo, f, y)
    ref_f, ref_b = o.forward(f), o.adjoint(y)
    for got, ref, what in [(fs, ref_f, "forward (store)"), (fo, ref_f, "forward (on the fly)"),
                           (bs, ref_b, "adjoint (store)"), (bo, ref_b, "adjoint (on the fly)")]:
        assert_parity(got, ref, what=what)
    assert np.array_equal(fs, fo), f"forward: store vs on the fly {rel_l2(fs, fo):.2e}"
    assert np.array_equal(bs, bo), f"adjoint: store vs on the fly {rel_l2(bs, bo):.2e}"


def test_store_slice128_operators_and_step(oracle_mod):
    """The benchmark workload: both paths give the same operators and the same
    reconstruction step, bit for bit (the step's parity with the oracle at
    this size is tested with the store in test_gpu_parity)."""
    w, g, ftrue, y = workload_data("slice128")
    geo = csx.Geometry(g)
    info = geo.factor_store()
    print(f"[slice128 store: {info['bytes'] / 2**30:.2f} GiB, built in {info['build_ms']:.1f} ms]", flush=True)
    # records: 16 B per (voxel group, class), 32 B per (pixel quad, voxel
    # group), and a 4-byte node range per 64-record tile
    n_groups, n_cls, n_quad = 128 * 64, 128 * 64, 64 * 64
    assert info["bytes"] == n_groups * n_cls * 16 + n_quad * n_groups * 32 + (n_groups * n_cls + n_quad * n_groups) // 16
    fs, bs, fo, bo = _both_paths(geo, ftrue, y)
    assert np.array_equal(fs, fo) and np.array_equal(bs, bo)
    f0 = np.full(ftrue.shape, 0.3)
    out = []
    geo.set_interval_operators(False)
    for on in (True, False):
        geo.set_factor_store(on)
        fd = dev(f0)
        J = torch.zeros(1, dtype=torch.float64, device="cuda")
        geo.recon_step(dev(y), fd, w.beta, J=J)
        out.append((host(fd), J.item()))
    assert np.array_equal(out[0][0], out[1][0]) and out[0][1] == out[1][1]


def test_store_needs_a_uniform_q_grid():
    g = ragged_geometry(1, 10, 7, 12, 10, 24, 402.57)
    q = g.q.copy()
    q[5] += 0.01                       # no longer uniform
    geo = csx.Geometry(g.with_(q=q))
    assert not geo.factor_store()["on"]
    with pytest.raises(csx.CsxError) as ei:
        geo.set_factor_store(True)
    assert ei.value.code == csx.CSX_EINVAL
    geo.set_factor_store(False)        # releasing nothing is fine

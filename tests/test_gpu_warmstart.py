"""Learned warm start on the GPU: every network kernel against the FP64 oracle
(oracle/cnn.py) on ragged shapes, a full training step's gradients, the
input / output maps, the judge and its fallback, and what the shipped network
gains over the plain start.

Tolerances.  A layer test hands both sides the same float32 inputs, so both
round the same binary16 operands; products of two binary16 values are exact
in float32, and a K-term float32 sum differs from the exact one by at most
gamma_K = K 2^-24 of the sum of |products| (K = 9 c_in for a convolution,
K = pixels for a weight gradient).  The bound is checked element by element
against that abs-sum.  Chained layers round float32 activations that differ
from the oracle's float64 ones, so a rare operand moves by one binary16 ulp
(2^-11 relative): the end-to-end checks use rel-L2 <= 4 * 2^-11.
"""
import os

import numpy as np
import pytest
import torch

from oracle import cnn
from paper_1603_06400_amd import csx, inputs, warmstart

from .gpu_helpers import rel_l2

pytestmark = pytest.mark.gpu

PAIRS = [(64, 32), (32, 32), (32, 64)]
U24 = 2.0 ** -24
E2E = 4 * 2.0 ** -11


def rnd(shape, seed, lo=-1.0, hi=1.0):
    return np.random.Generator(np.random.PCG64(seed)).uniform(lo, hi, size=shape).astype(np.float32)


def dev(a, dtype=torch.float32):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda").contiguous()


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def half_w(shape, seed, scale=0.2):
    w = (rnd(shape, seed) * scale).astype(np.float16)
    return w, dev(w, torch.float16)


def check_bound(got, ref, absref, K, what):
    bound = K * U24 * absref + 1e-30
    err = np.abs(got - ref)
    assert np.all(err <= bound), f"{what}: max err/bound {np.max(err / bound):.3g}"


@pytest.mark.parametrize("ci,co", PAIRS)
@pytest.mark.parametrize("relu,res", [(False, False), (True, False), (False, True)])
def test_conv_forward(ci, co, relu, res):
    nb, H, W = 2, 19, 37                     # ragged against the 8 x 16 tiles
    x = rnd((nb, H, W, ci), 1 + ci + co)
    w, w_d = half_w((9, ci, co), 2 + ci)
    b = rnd(co, 3)
    r = rnd((nb, H, W, co), 4) if res else None
    y = torch.empty((nb, H, W, co), device="cuda")
    csx.conv3x3_forward(dev(x), w_d, dev(b), y, relu, None if r is None else dev(r))
    ref = cnn.conv3x3(x, w.astype(np.float64), b, relu=relu, half=True, residual=r)
    absref = cnn.conv3x3(np.abs(x), np.abs(w.astype(np.float64)), np.abs(b), half=True,
                         residual=None if r is None else np.abs(r))
    check_bound(host(y), ref, absref, 9 * ci + 2, f"forward {ci}->{co}")


@pytest.mark.parametrize("ci,co", PAIRS)
@pytest.mark.parametrize("masked", [False, True])
def test_conv_backward_data(ci, co, masked):
    nb, H, W = 3, 13, 21
    dy = rnd((nb, H, W, co), 5 + co)
    w, w_d = half_w((9, ci, co), 6 + ci)
    mask = np.maximum(rnd((nb, H, W, ci), 7), 0.0) if masked else None
    dx = torch.empty((nb, H, W, ci), device="cuda")
    csx.conv3x3_backward_data(dev(dy), w_d, None if mask is None else dev(mask), dx)
    ref = cnn.conv3x3_backward_data(dy, w.astype(np.float64), mask, half=True)
    absref = cnn.conv3x3_backward_data(np.abs(dy), np.abs(w.astype(np.float64)), mask, half=True)
    check_bound(host(dx), ref, absref, 9 * co, f"backward data {ci}->{co}")
    if masked:
        assert np.all(host(dx)[mask <= 0] == 0.0)


@pytest.mark.parametrize("ci,co", PAIRS)
def test_conv_backward_weights(ci, co):
    nb, H, W = 3, 21, 35                     # 3 x 2 x 3 tiles of 16 x 16, ragged
    x = rnd((nb, H, W, ci), 8 + ci, 0.0, 2.0)
    dy = rnd((nb, H, W, co), 9 + co)
    dw = torch.empty((9, ci, co), device="cuda")
    db = torch.empty(co, device="cuda")
    ws = torch.empty(csx.cnn_workspace_bytes(nb, H, W), dtype=torch.uint8, device="cuda")
    csx.conv3x3_backward_weights(dev(x), dev(dy), dw, db, ws)
    ref_w, ref_b = cnn.conv3x3_backward_weights(x, dy, half=True)
    abs_w, abs_b = cnn.conv3x3_backward_weights(np.abs(x), np.abs(dy), half=True)
    K = nb * H * W
    check_bound(host(dw), ref_w, abs_w, K, f"weight grad {ci}->{co}")
    check_bound(host(db), ref_b, abs_b, K, f"bias grad {ci}->{co}")


def test_workspace_too_small_is_rejected():
    x = torch.zeros((1, 16, 16, 64), device="cuda")
    dy = torch.zeros((1, 16, 16, 32), device="cuda")
    dw = torch.empty((9, 64, 32), device="cuda")
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(csx.CsxError) as ei:
        csx.conv3x3_backward_weights(x, dy, dw, None, ws)
    assert ei.value.code == csx.CSX_EINVAL


def test_loss_head_and_adam():
    nb, n = 3, 5000
    o = rnd((nb, n), 11, -4.0, 4.0)
    t = rnd((nb, n), 12, -3.0, 3.0)
    d = torch.empty((nb, n), device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    ws = torch.empty(4096, dtype=torch.uint8, device="cuda")
    csx.warm_loss(dev(o), dev(t), d, loss, ws)
    L, dref = cnn.head(o, t, nb)
    assert abs(float(loss) - L) <= 1e-6 * L
    assert rel_l2(host(d), dref) <= 1e-6
    # Adam: three steps against the float64 recursion
    w = rnd(1000, 13)
    g = [rnd(1000, 14 + k) for k in range(3)]
    wd, md, vd = dev(w), torch.zeros(1000, device="cuda"), torch.zeros(1000, device="cuda")
    w16 = torch.empty(1000, dtype=torch.float16, device="cuda")
    wr, mr, vr = w.astype(np.float64), np.zeros(1000), np.zeros(1000)
    for k in range(3):
        csx.adam_step(wd, md, vd, dev(g[k]), w16, k + 1, 1e-2)
        wr, mr, vr = cnn.adam(wr, mr, vr, g[k], k + 1, 1e-2)
    np.testing.assert_allclose(host(wd), wr, rtol=0, atol=1e-6)
    np.testing.assert_array_equal(host(w16), cnn.f16(host(wd)))


def net_params(seed):
    p = inputs.cnn_init(seed)
    for lay in p:                            # binary16 weights on both sides
        lay["w"] = lay["w"].astype(np.float16).astype(np.float32)
        lay["b"] = lay["b"] + rnd(lay["b"].shape, seed + 5, -0.05, 0.05)
    return p


def test_training_step_gradients_match_oracle():
    nb, H, W = 2, 12, 20
    params = net_params(3)
    x = rnd((nb, H, W, 64), 21, -2.0, 2.0)
    t = rnd((nb, H, W, 64), 22, -1.5, 1.5)
    net = warmstart.WarmNet(params)
    tr = warmstart.Trainer(net, nb, H, W)
    tr.forward(dev(x))
    loss = float(tr.backward(dev(x), dev(t)))
    acts = cnn.forward([{"w": p["w"].astype(np.float64), "b": p["b"]} for p in params], x, half=True)
    L, grads = cnn.backward([{"w": p["w"].astype(np.float64), "b": p["b"]} for p in params], acts, t, half=True)
    assert rel_l2(host(tr.acts[-1]), acts[-1]) <= E2E
    assert abs(loss - L) <= E2E * L
    for k in range(4):
        assert rel_l2(host(net.gw[k]), grads[k]["w"]) <= E2E, f"dW layer {k}"
        assert rel_l2(host(net.gb[k]), grads[k]["b"]) <= E2E, f"db layer {k}"


def test_training_is_deterministic_and_reduces_the_loss():
    nb, H, W = 2, 16, 16
    x = rnd((4, H, W, 64), 31, 0.0, 2.0)
    t = 0.5 * x + 0.25                       # learnable: the FP64 recursion drops the loss
    X, T = dev(x), dev(t)
    runs = []
    for _ in range(2):
        net = warmstart.WarmNet.init(4)
        hist = warmstart.train(net, X, T, epochs=15, nb=nb, lr=3e-3, seed=2)
        runs.append((hist, [w.clone() for w in net.w32]))
    assert runs[0][0] == runs[1][0]
    for a, b in zip(runs[0][1], runs[1][1]):
        assert torch.equal(a, b)
    assert runs[0][0][-1] < 0.8 * runs[0][0][0]


def small_scan():
    g = inputs.standard_geometry(16, 64, ndet=16)
    f = inputs.phantom(g, 41, 3)
    return g, f


def test_warm_input_and_start_match_oracle(oracle_mod):
    g, f = small_scan()
    o = oracle_mod.Oracle(g)
    y = inputs.poisson_counts(o.forward(f) * (1e3 / o.forward(f).max()), 42)
    geo = csx.Geometry(g)
    yd = dev(y)
    d = 0.05
    x = geo.warm_input(yd, d)
    xref = cnn.features(cnn.warm_input(o, y), d)
    assert rel_l2(host(x), xref) <= 1e-5
    params = net_params(5)
    net = warmstart.WarmNet(params, d)
    f0 = geo.warm_start(yd, net.layers(), d)
    acts = cnn.forward([{"w": p["w"].astype(np.float64), "b": p["b"]} for p in params],
                       xref.reshape(1, g.nz, g.nx, g.nq), half=True)
    b1 = o.sensitivity()
    u = cnn.uniform_value(y, b1)
    ref = cnn.mass_normalise(cnn.warm_output(acts[-1][0], u, d), y, b1)
    assert rel_l2(host(f0), ref) <= E2E
    np.testing.assert_allclose(ref, cnn.warm_start(o, y, [{"w": p["w"].astype(np.float64), "b": p["b"]}
                                                          for p in params], d), rtol=1e-12)
    assert abs(float(np.sum(b1 * host(f0))) / float(np.sum(y)) - 1.0) <= 1e-5
    assert float(f0.min()) > 0.0
    # training target of an image
    fr = inputs.random_image(g, 43, 0.0, 5.0)
    t = geo.warm_target(yd, dev(fr), d)
    assert rel_l2(host(t), cnn.target(fr, u, d)) <= 1e-6
    with pytest.raises(csx.CsxError) as ei:
        geo.warm_input(yd, 0.0)
    assert ei.value.code == csx.CSX_EINVAL


def judge_case():
    w = inputs.workload("slice32")
    g = w.geom.with_(C=1e6)
    f = inputs.phantom(g, 51, 3)
    geo = csx.Geometry(g)
    y = warmstart.counts(geo, f, 52)
    return w, g, geo, y


def test_judge_accepts_a_better_start_and_rejects_a_worse_one():
    w, g, geo, y = judge_case()
    n_iter, k = 8, 2
    fp = geo.new_image()
    Jp = geo.recon(y, fp, n_iter, w.beta)
    # a start that is already the 8-iteration reconstruction is accepted
    good = fp.clone()
    f = geo.new_image()
    Jg, acc = geo.recon_warm(y, good, f, k, n_iter, w.beta)
    assert acc and Jg[0] == Jp[-1] and Jg[k] < Jp[k]
    # a start of random structure (EM keeps a start's multiplicative pattern;
    # a uniform start of any level gives the plain first iterate) is rejected:
    # the result is the plain run, bit for bit
    bad = dev(inputs.random_image(g, 53, 1e-3, 3.0)) * float(fp.mean())
    f2 = geo.new_image()
    Jb, acc2 = geo.recon_warm(y, bad, f2, k, n_iter, w.beta)
    assert not acc2
    np.testing.assert_array_equal(Jb, Jp)
    assert torch.equal(f2, fp)
    # k = 0 compares the starts themselves
    _, acc0 = geo.recon_warm(y, good, f, 0, n_iter, w.beta)
    assert acc0


def test_judge_argument_errors():
    w, g, geo, y = judge_case()
    f = geo.new_image().fill_(1.0)
    with pytest.raises(csx.CsxError) as ei:
        geo.recon_warm(y, f, geo.new_image(), 5, 3, w.beta)
    assert ei.value.code == csx.CSX_EINVAL
    with pytest.raises(csx.CsxError) as ei:
        geo.recon_warm(y, f, f, 1, 3, w.beta)
    assert ei.value.code == csx.CSX_EINVAL


@pytest.mark.skipif(not os.path.exists(warmstart.WEIGHTS), reason="no trained network shipped")
def test_shipped_network_reaches_the_plain_objective_sooner():
    """Held-out phantoms (seeds outside the training range): the judged warm
    start reaches J_plain(50) (1 + 1e-3) in fewer iterations than the plain
    start and is accepted by the judge."""
    w, g = warmstart.calibrated_geometry()
    geo = csx.Geometry(g)
    net = warmstart.WarmNet.load()
    rows = warmstart.evaluate(geo, net, inputs.warm_cases("eval", 3), w.n_iter, w.beta, k_judge=2)
    for r in rows:
        assert r["accepted"], r
        assert r["iters_warm"] is not None and r["iters_warm"] < r["iters_plain"], r

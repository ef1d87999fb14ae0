"""csx_forward_noalloc: the forward through the library's static scratch.

Called through the C ABI, its output must equal csx_forward's bit for bit (same
kernels, same partial images, same fixed-order sum), on two calls in a row
whose second input is smaller, and on a third call back at the larger size
(the scratch keeps the last call's contents, which no result may depend on).
A forward whose partial images exceed the scratch is refused before any launch,
and fits after fewer voxel splits.  The consecutive calls run the interval
form of the forward (its partial images, one per workgroup, in the scratch);
the refusal case runs the direct forward."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1603_06400_amd import csx, inputs  # noqa: E402

from .gpu_helpers import workload_data  # noqa: E402

pytestmark = pytest.mark.gpu


def _image(geo, seed):
    rng = np.random.default_rng(seed)
    return torch.tensor(rng.uniform(0.0, 1.0, geo.image_shape), dtype=torch.float32, device="cuda")


def test_noalloc_forward_equals_forward_on_consecutive_calls():
    assert torch.cuda.is_available()
    _, g128, f128, _ = workload_data("slice128")
    _, g32, f32, _ = workload_data("slice32")
    big, small = csx.Geometry(g128), csx.Geometry(g32)
    cases = [(big, torch.tensor(f128, dtype=torch.float32, device="cuda")),
             (small, torch.tensor(f32, dtype=torch.float32, device="cuda")),
             (big, _image(big, 3))]
    for k, (geo, f) in enumerate(cases):
        print(f"[noalloc call {k}: image {tuple(geo.image_shape)}, detector {geo.detector_shape}]", flush=True)
        ref = geo.forward(f)
        out = torch.full(geo.detector_shape, float("nan"), dtype=torch.float32, device="cuda")
        geo.forward_noalloc(f, out)
        torch.cuda.synchronize()
        a, b = ref.cpu().numpy(), out.cpu().numpy()
        assert np.all(np.isfinite(b))
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), f"call {k}: differs from csx_forward"
    big.close()
    small.close()


def test_noalloc_forward_refuses_partials_beyond_the_scratch():
    # 32 x 40 voxels (10 voxel tiles) against a 1024^2 detector, the forward
    # split 5 ways: 5 partial images of 2^20 pixels, more than the 2^22-float
    # scratch (the detector is too large for the interval form, so the direct
    # forward runs)
    g = inputs.standard_geometry(32, 16, ndet=1024).with_(nz=40)
    geo = csx.Geometry(g)
    assert not geo.interval_operators()["on"]
    lc = geo.get_launch()
    geo.set_launch(5, lc["fwd_qw"], lc["adj_qw"])
    parts = geo.get_launch()["fwd_splits"] * geo.npix
    assert parts > csx.SCRATCH_FLOATS, parts
    f = _image(geo, 5)
    out = torch.zeros(geo.detector_shape, dtype=torch.float32, device="cuda")
    with pytest.raises(csx.CsxError) as ei:
        geo.forward_noalloc(f, out)
    assert ei.value.code == csx.CSX_EINVAL
    lc = geo.get_launch()
    geo.set_launch(max(1, csx.SCRATCH_FLOATS // geo.npix), lc["fwd_qw"], lc["adj_qw"])
    ref = geo.forward(f)
    geo.forward_noalloc(f, out)
    torch.cuda.synchronize()
    assert np.array_equal(ref.cpu().numpy().view(np.uint32), out.cpu().numpy().view(np.uint32))
    geo.close()

"""The C ABI: the built library loads, exports every symbol include/csx.h
declares, and rejects bad descriptors before touching the GPU."""
import re

import numpy as np
import pytest

from paper_1603_06400_amd import csx, inputs

HEADER = __import__("os").path.join(__import__("os").path.dirname(__file__), "..", "include", "csx.h")


def declared_functions():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(csx_[a-z_0-9]+)\s*\(", txt)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(csx.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = csx.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def good():
    return inputs.standard_geometry(8, 6, ndet=10)


@pytest.mark.parametrize("mutate,code", [
    (lambda g: g.with_(ndy=9, mask=np.ones((9, 16), np.uint8)), csx.CSX_EGEOM),
    (lambda g: g.with_(z_max=750.0), csx.CSX_EGEOM),
    (lambda g: g.with_(z_min=-1.0), csx.CSX_EGEOM),
    (lambda g: g.with_(x_min=50.0), csx.CSX_EGEOM),
    (lambda g: g.with_(e_lo=200.0), csx.CSX_EGEOM),
    (lambda g: g.with_(det_pitch=0.0), csx.CSX_EGEOM),
    (lambda g: g.with_(q=np.array([0.5, -1.0, 2.0])), csx.CSX_EGEOM),
    (lambda g: g.with_(phi=np.array([1.0, np.nan])), csx.CSX_EGEOM),
    (lambda g: g.with_(mask=np.full((10, 16), 2, np.uint8)), csx.CSX_EGEOM),
    (lambda g: g.with_(C=-1.0), csx.CSX_EGEOM),
    (lambda g: g.with_(phi=np.ones(5000)), csx.CSX_EGEOM),
])
def test_validation_rejects(mutate, code):
    with pytest.raises(csx.CsxError) as ei:
        csx.validate(mutate(good()))
    assert ei.value.code == code


def test_validation_accepts_workloads():
    for name in ["slice32", "slice128", "slice128_open1", "slice128_open01"]:
        csx.validate(inputs.workload(name).geom)
        csx.validate(inputs.workload(name).geom, csx.TABLE_BF16)


def test_mask_limits():
    """The mask is held in LDS as one 32-bit word per row: period <= 32 cells,
    <= 4096 rows."""
    csx.validate(good().with_(mask=np.ones((10, 32), np.uint8)))
    for bad in (np.ones((10, 33), np.uint8), np.ones((4097, 16), np.uint8)):
        for td in (csx.TABLE_F32, csx.TABLE_BF16):
            with pytest.raises(csx.CsxError) as ei:
                csx.validate(good().with_(mask=bad), td)
            assert ei.value.code == csx.CSX_EGEOM

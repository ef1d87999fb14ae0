"""Python binding of libcsx.so (argument marshalling only).

Every computation runs in the HIP library; this module checks tensor shapes,
dtypes and devices, passes ``data_ptr()`` and the current HIP stream, and turns
status codes into exceptions.  PyTorch provides device memory and streams.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch

from .build import LIB

CSX_OK, CSX_EINVAL, CSX_EGEOM, CSX_EHIP, CSX_ENOMEM, CSX_ENUMERIC = 0, -1, -2, -3, -4, -5
TABLE_F32, TABLE_BF16 = 0, 1
PSI_QUADRATIC, PSI_HUBER = 0, 1
OP_FORWARD_SAI, OP_ADJOINT_SAI = 1, 2
SAI_MAX_NODES = 2048
SCRATCH_FLOATS = 1 << 22        # CSX_SCRATCH_FLOATS: static scratch of csx_forward_noalloc
_NAMES = {CSX_EINVAL: "EINVAL", CSX_EGEOM: "EGEOM", CSX_EHIP: "EHIP", CSX_ENOMEM: "ENOMEM",
          CSX_ENUMERIC: "ENUMERIC"}


class CsxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"csx {_NAMES.get(code, code)}: {msg}")
        self.code = code


class _Desc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("nz", ctypes.c_int),
        ("x_min", ctypes.c_double), ("x_max", ctypes.c_double),
        ("z_min", ctypes.c_double), ("z_max", ctypes.c_double),
        ("nq", ctypes.c_int), ("q", ctypes.POINTER(ctypes.c_double)),
        ("ndx", ctypes.c_int), ("ndy", ctypes.c_int),
        ("det_pitch", ctypes.c_double), ("det_z", ctypes.c_double),
        ("mask_z", ctypes.c_double), ("mask_pitch", ctypes.c_double),
        ("mask_nx", ctypes.c_int), ("mask_ny", ctypes.c_int),
        ("mask", ctypes.POINTER(ctypes.c_ubyte)),
        ("ne", ctypes.c_int), ("e_lo", ctypes.c_double), ("e_hi", ctypes.c_double),
        ("phi", ctypes.POINTER(ctypes.c_double)),
        ("C", ctypes.c_double), ("hc", ctypes.c_double),
        ("table_dtype", ctypes.c_int),
    ]


class _Launch(ctypes.Structure):
    _fields_ = [("fwd_splits", ctypes.c_int), ("fwd_qw", ctypes.c_int), ("adj_qw", ctypes.c_int),
                ("adj_splits", ctypes.c_int)]


class _Info(ctypes.Structure):
    _fields_ = [("nvox", ctypes.c_int), ("npix", ctypes.c_int), ("nq", ctypes.c_int),
                ("symmetric_lr", ctypes.c_int), ("table_dtype", ctypes.c_int),
                ("workspace_bytes", ctypes.c_int64)]


EXPORTS = ["csx_validate_desc", "csx_init_geometry", "csx_free_geometry", "csx_get_info",
           "csx_set_factor_store", "csx_get_factor_store", "csx_set_interval_operators",
           "csx_get_interval_operators",
           "csx_forward", "csx_forward_noalloc", "csx_backproject", "csx_recon_step", "csx_recon", "csx_recon_os", "csx_set_penalty",
           "csx_get_launch", "csx_set_launch", "csx_batch_create", "csx_batch_free",
           "csx_batch_recon", "csx_batch_recon_n", "csx_timing_enable", "csx_timing_read", "csx_last_error",
           "csx_cnn_workspace_bytes", "csx_conv3x3_forward", "csx_conv3x3_backward_data",
           "csx_conv3x3_backward_weights", "csx_warm_loss", "csx_adam_step", "csx_to_half",
           "csx_warm_input", "csx_warm_output", "csx_warm_target", "csx_warm_start", "csx_recon_warm",
           "csx_sai_config", "csx_sai_info", "csx_forward_sai", "csx_backproject_sai", "csx_set_operator",
           "csx_forward_energy", "csx_backproject_energy", "csx_recon_energy", "csx_valu_peak"]


class _WarmNet(ctypes.Structure):
    _fields_ = [("w", ctypes.c_void_p * 4), ("b", ctypes.c_void_p * 4)]

_lib = None


def lib():
    """Load libcsx.so; raises if the library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} is missing: run paper_1603_06400_amd.build.build() first")
        L = ctypes.CDLL(LIB)
        vp = ctypes.c_void_p
        dp = ctypes.POINTER(_Desc)
        L.csx_validate_desc.argtypes = [dp]
        L.csx_validate_desc.restype = ctypes.c_int
        L.csx_init_geometry.argtypes = [dp, ctypes.POINTER(vp)]
        L.csx_init_geometry.restype = ctypes.c_int
        L.csx_free_geometry.argtypes = [vp]
        L.csx_free_geometry.restype = None
        L.csx_get_info.argtypes = [vp, ctypes.POINTER(_Info)]
        L.csx_get_info.restype = ctypes.c_int
        L.csx_forward.argtypes = [vp, vp, vp, vp]
        L.csx_forward.restype = ctypes.c_int
        L.csx_set_factor_store.argtypes = [vp, ctypes.c_int]
        L.csx_set_factor_store.restype = ctypes.c_int
        L.csx_get_factor_store.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int64),
                                           ctypes.POINTER(ctypes.c_double)]
        L.csx_get_factor_store.restype = ctypes.c_int
        L.csx_set_interval_operators.argtypes = [vp, ctypes.c_int]
        L.csx_set_interval_operators.restype = ctypes.c_int
        L.csx_get_interval_operators.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int64),
                                                 ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]
        L.csx_get_interval_operators.restype = ctypes.c_int
        L.csx_forward_noalloc.argtypes = [vp, vp, vp, vp]
        L.csx_forward_noalloc.restype = ctypes.c_int
        L.csx_backproject.argtypes = [vp, vp, vp, vp]
        L.csx_backproject.restype = ctypes.c_int
        L.csx_recon_step.argtypes = [vp, vp, vp, vp, ctypes.c_double, vp, vp]
        L.csx_recon_step.restype = ctypes.c_int
        L.csx_recon.argtypes = [vp, vp, vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                ctypes.POINTER(ctypes.c_double), vp]
        L.csx_recon.restype = ctypes.c_int
        L.csx_recon_os.argtypes = [vp, vp, vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_double, ctypes.POINTER(ctypes.c_double), vp]
        L.csx_recon_os.restype = ctypes.c_int
        L.csx_set_penalty.argtypes = [vp, ctypes.c_int, ctypes.c_double]
        L.csx_set_penalty.restype = ctypes.c_int
        L.csx_sai_config.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_double]
        L.csx_sai_config.restype = ctypes.c_int
        L.csx_sai_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                   ctypes.POINTER(ctypes.c_double)]
        L.csx_sai_info.restype = ctypes.c_int
        L.csx_forward_sai.argtypes = [vp, vp, vp, vp]
        L.csx_forward_sai.restype = ctypes.c_int
        L.csx_backproject_sai.argtypes = [vp, vp, vp, vp]
        L.csx_backproject_sai.restype = ctypes.c_int
        L.csx_set_operator.argtypes = [vp, ctypes.c_int]
        L.csx_set_operator.restype = ctypes.c_int
        L.csx_forward_energy.argtypes = [vp, vp, vp, vp]
        L.csx_forward_energy.restype = ctypes.c_int
        L.csx_backproject_energy.argtypes = [vp, vp, vp, vp]
        L.csx_backproject_energy.restype = ctypes.c_int
        L.csx_recon_energy.argtypes = [vp, vp, vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                       ctypes.POINTER(ctypes.c_double), vp]
        L.csx_recon_energy.restype = ctypes.c_int
        L.csx_valu_peak.argtypes = [ctypes.POINTER(ctypes.c_double), vp]
        L.csx_valu_peak.restype = ctypes.c_int
        L.csx_get_launch.argtypes = [vp, ctypes.POINTER(_Launch)]
        L.csx_get_launch.restype = ctypes.c_int
        L.csx_set_launch.argtypes = [vp, ctypes.POINTER(_Launch)]
        L.csx_set_launch.restype = ctypes.c_int
        L.csx_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(vp)]
        L.csx_batch_create.restype = ctypes.c_int
        L.csx_batch_free.argtypes = [vp]
        L.csx_batch_free.restype = None
        L.csx_batch_recon.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                      ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                      ctypes.POINTER(ctypes.c_double), vp]
        L.csx_batch_recon.restype = ctypes.c_int
        L.csx_batch_recon_n.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                        ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_double,
                                        ctypes.POINTER(ctypes.c_double), ctypes.c_int, vp]
        L.csx_batch_recon_n.restype = ctypes.c_int
        L.csx_timing_enable.argtypes = [vp, ctypes.c_int]
        L.csx_timing_enable.restype = ctypes.c_int
        L.csx_timing_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]
        L.csx_timing_read.restype = ctypes.c_int
        i, d, sz = ctypes.c_int, ctypes.c_double, ctypes.c_size_t
        L.csx_cnn_workspace_bytes.argtypes = [i, i, i]
        L.csx_cnn_workspace_bytes.restype = sz
        L.csx_conv3x3_forward.argtypes = [vp, vp, vp, vp, vp, i, i, i, i, i, i, vp]
        L.csx_conv3x3_forward.restype = i
        L.csx_conv3x3_backward_data.argtypes = [vp, vp, vp, vp, i, i, i, i, i, vp]
        L.csx_conv3x3_backward_data.restype = i
        L.csx_conv3x3_backward_weights.argtypes = [vp, vp, vp, vp, i, i, i, i, i, vp, sz, vp]
        L.csx_conv3x3_backward_weights.restype = i
        L.csx_warm_loss.argtypes = [vp, vp, i, i, vp, vp, vp, sz, vp]
        L.csx_warm_loss.restype = i
        L.csx_adam_step.argtypes = [vp, vp, vp, vp, vp, i, d, d, d, d, i, vp]
        L.csx_adam_step.restype = i
        L.csx_to_half.argtypes = [vp, vp, i, vp]
        L.csx_to_half.restype = i
        L.csx_warm_input.argtypes = [vp, vp, ctypes.c_float, vp, vp]
        L.csx_warm_input.restype = i
        L.csx_warm_output.argtypes = [vp, vp, vp, ctypes.c_float, vp, vp]
        L.csx_warm_output.restype = i
        L.csx_warm_target.argtypes = [vp, vp, vp, ctypes.c_float, vp, vp]
        L.csx_warm_target.restype = i
        L.csx_warm_start.argtypes = [vp, vp, ctypes.POINTER(_WarmNet), ctypes.c_float, vp, vp]
        L.csx_warm_start.restype = i
        L.csx_recon_warm.argtypes = [vp, vp, vp, vp, vp, i, i, d, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(i), vp]
        L.csx_recon_warm.restype = i
        L.csx_last_error.argtypes = []
        L.csx_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(code: int):
    if code != CSX_OK:
        raise CsxError(code, lib().csx_last_error().decode())


def make_desc(geom, table_dtype: int = TABLE_F32):
    """ctypes descriptor for an ``inputs.ScanGeometry``; returns (desc, keepalive)."""
    q = np.ascontiguousarray(geom.q, dtype=np.float64)
    phi = np.ascontiguousarray(geom.phi, dtype=np.float64)
    mask = np.ascontiguousarray(geom.mask, dtype=np.uint8)
    d = _Desc()
    d.nx, d.nz = geom.nx, geom.nz
    d.x_min, d.x_max, d.z_min, d.z_max = geom.x_min, geom.x_max, geom.z_min, geom.z_max
    d.nq, d.q = q.shape[0], q.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.ndx, d.ndy, d.det_pitch, d.det_z = geom.ndx, geom.ndy, geom.det_pitch, geom.det_z
    d.mask_z, d.mask_pitch = geom.mask_z, geom.mask_pitch
    d.mask_ny, d.mask_nx = mask.shape
    d.mask = mask.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte))
    d.ne, d.e_lo, d.e_hi = phi.shape[0], geom.e_lo, geom.e_hi
    d.phi = phi.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.C, d.hc, d.table_dtype = geom.C, geom.hc, table_dtype
    return d, (q, phi, mask)


def validate(geom, table_dtype: int = TABLE_F32) -> None:
    d, keep = make_desc(geom, table_dtype)
    _check(lib().csx_validate_desc(ctypes.byref(d)))


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, numel: int, name: str) -> ctypes.c_void_p:
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous float32")
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


class Geometry:
    """A scan geometry resident on the current GPU (wraps a csx_geometry handle)."""

    def __init__(self, geom, table_dtype: int = TABLE_F32):
        self.geom = geom
        self.table_dtype = table_dtype
        self.nvox, self.npix, self.nq = geom.nx * geom.nz, geom.ndx * geom.ndy, int(len(geom.q))
        self.ne = int(len(geom.phi))
        self.image_shape = (geom.nz, geom.nx, self.nq)
        self.detector_shape = (geom.ndy, geom.ndx)
        d, keep = make_desc(geom, table_dtype)
        h = ctypes.c_void_p()
        _check(lib().csx_init_geometry(ctypes.byref(d), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().csx_free_geometry(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        out = _Info()
        _check(lib().csx_get_info(self._h, ctypes.byref(out)))
        return {k: getattr(out, k) for k, _ in _Info._fields_}

    def get_launch(self) -> dict:
        out = _Launch()
        _check(lib().csx_get_launch(self._h, ctypes.byref(out)))
        return {k: getattr(out, k) for k, _ in _Launch._fields_}

    def set_launch(self, fwd_splits: int, fwd_qw: int, adj_qw: int, adj_splits: int = 0) -> None:
        """adj_splits = 0: the default split of the direct adjoint's pixel classes."""
        lc = _Launch(int(fwd_splits), int(fwd_qw), int(adj_qw), int(adj_splits))
        _check(lib().csx_set_launch(self._h, ctypes.byref(lc)))

    def set_factor_store(self, on: bool) -> None:
        """Build (True) or release (False) the per-class pair-factor store."""
        _check(lib().csx_set_factor_store(self._h, int(bool(on))))

    def factor_store(self) -> dict:
        on, nb, ms = ctypes.c_int(), ctypes.c_int64(), ctypes.c_double()
        _check(lib().csx_get_factor_store(self._h, ctypes.byref(on), ctypes.byref(nb), ctypes.byref(ms)))
        return {"on": bool(on.value), "bytes": int(nb.value), "build_ms": float(ms.value)}

    def set_interval_operators(self, on: bool) -> None:
        """Build (True) or release (False) the interval form of the exact operators."""
        _check(lib().csx_set_interval_operators(self._h, int(bool(on))))

    def interval_operators(self) -> dict:
        on, nb, ms, nt = ctypes.c_int(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_int()
        _check(lib().csx_get_interval_operators(self._h, ctypes.byref(on), ctypes.byref(nb), ctypes.byref(ms),
                                                ctypes.byref(nt)))
        return {"on": bool(on.value), "bytes": int(nb.value), "build_ms": float(ms.value),
                "intervals": int(nt.value)}

    def timing_enable(self, on: bool = True) -> None:
        _check(lib().csx_timing_enable(self._h, int(bool(on))))

    def timing_read(self) -> dict:
        """Summed event times (ms) and launch counts of forward / adjoint kernels."""
        ms = (ctypes.c_double * 2)()
        n = (ctypes.c_int * 2)()
        _check(lib().csx_timing_read(self._h, ms, n))
        return {"forward_ms": ms[0], "forward_n": n[0], "adjoint_ms": ms[1], "adjoint_n": n[1]}

    def new_image(self) -> torch.Tensor:
        return torch.empty(self.image_shape, dtype=torch.float32, device="cuda")

    def new_detector(self) -> torch.Tensor:
        return torch.empty(self.detector_shape, dtype=torch.float32, device="cuda")

    def forward(self, f: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        out = self.new_detector() if out is None else out
        _check(lib().csx_forward(self._h, _dev(f, self.nvox * self.nq, "f"),
                                 _dev(out, self.npix, "g"), _stream()))
        return out

    def forward_noalloc(self, f: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        """csx_forward through the library's static scratch (no allocation);
        out must be given."""
        _check(lib().csx_forward_noalloc(self._h, _dev(f, self.nvox * self.nq, "f"),
                                         _dev(out, self.npix, "g"), _stream()))
        return out

    def backproject(self, y: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        out = self.new_image() if out is None else out
        _check(lib().csx_backproject(self._h, _dev(y, self.npix, "y"),
                                     _dev(out, self.nvox * self.nq, "b"), _stream()))
        return out

    def recon_step(self, y: torch.Tensor, f: torch.Tensor, beta: float,
                   r: Optional[torch.Tensor] = None, J: Optional[torch.Tensor] = None) -> None:
        """In-place Alg. 5 iteration on f; J (device float64 scalar) receives J(f^t)."""
        rp = ctypes.c_void_p(None) if r is None else _dev(r, self.npix, "r")
        if J is not None and (J.dtype != torch.float64 or J.device.type != "cuda" or J.numel() < 1):
            raise ValueError("J must be a CUDA float64 tensor")
        jp = ctypes.c_void_p(None) if J is None else ctypes.c_void_p(J.data_ptr())
        _check(lib().csx_recon_step(self._h, _dev(y, self.npix, "y"), rp,
                                    _dev(f, self.nvox * self.nq, "f"), float(beta), jp, _stream()))

    def recon(self, y: torch.Tensor, f: torch.Tensor, n_iter: int, beta: float,
              r: Optional[torch.Tensor] = None, init_uniform: bool = True) -> np.ndarray:
        """Alg. 5 for n_iter iterations in place on f; returns J(f^0..f^n) (float64)."""
        rp = ctypes.c_void_p(None) if r is None else _dev(r, self.npix, "r")
        hist = np.zeros(n_iter + 1, dtype=np.float64)
        _check(lib().csx_recon(self._h, _dev(y, self.npix, "y"), rp,
                               _dev(f, self.nvox * self.nq, "f"), int(bool(init_uniform)),
                               int(n_iter), float(beta),
                               hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream()))
        return hist


    def set_penalty(self, kind: str = "quadratic", delta: float = 0.0) -> None:
        """Penalty potential: "quadratic" (t^2/2) or "huber" with scale delta."""
        code = {"quadratic": PSI_QUADRATIC, "huber": PSI_HUBER}.get(kind)
        if code is None:
            raise ValueError(f"unknown potential {kind!r}")
        _check(lib().csx_set_penalty(self._h, code, float(delta)))

    def sai_config(self, nt: int, interp: str = "linear", theta_max: float = 0.0) -> None:
        """Scatter-angle interpolation table of nt angles on [0, theta_max]
        (0: the geometry's largest angle); interp "nearest" or "linear"."""
        code = {"nearest": 0, "linear": 1}.get(interp)
        if code is None:
            raise ValueError(f"unknown interpolation {interp!r}")
        _check(lib().csx_sai_config(self._h, int(nt), code, float(theta_max)))

    def sai_info(self) -> dict:
        nt, it, tm = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        _check(lib().csx_sai_info(self._h, ctypes.byref(nt), ctypes.byref(it), ctypes.byref(tm)))
        return {"nt": nt.value, "interp": ("nearest", "linear")[it.value], "theta_max": tm.value}

    def forward_sai(self, f: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        out = self.new_detector() if out is None else out
        _check(lib().csx_forward_sai(self._h, _dev(f, self.nvox * self.nq, "f"),
                                     _dev(out, self.npix, "g"), _stream()))
        return out

    def backproject_sai(self, y: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        out = self.new_image() if out is None else out
        _check(lib().csx_backproject_sai(self._h, _dev(y, self.npix, "y"),
                                         _dev(out, self.nvox * self.nq, "b"), _stream()))
        return out

    def forward_energy(self, f: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Energy-resolved detector image [ne][ndy][ndx] (App. A eq. energy_sensitive)."""
        out = torch.empty((self.ne,) + self.detector_shape, dtype=torch.float32, device="cuda") if out is None else out
        _check(lib().csx_forward_energy(self._h, _dev(f, self.nvox * self.nq, "f"),
                                        _dev(out, self.ne * self.npix, "gE"), _stream()))
        return out

    def backproject_energy(self, y: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Transpose of forward_energy; y of shape [ne][ndy][ndx]."""
        out = self.new_image() if out is None else out
        _check(lib().csx_backproject_energy(self._h, _dev(y, self.ne * self.npix, "yE"),
                                            _dev(out, self.nvox * self.nq, "b"), _stream()))
        return out

    def recon_energy(self, y: torch.Tensor, f: torch.Tensor, n_iter: int, beta: float,
                     r: Optional[torch.Tensor] = None, init_uniform: bool = True) -> np.ndarray:
        """Alg. 5 on energy-resolved counts y [ne][ndy][ndx], in place on f; returns J(f^0..f^n)."""
        rp = ctypes.c_void_p(None) if r is None else _dev(r, self.ne * self.npix, "rE")
        hist = np.zeros(n_iter + 1, dtype=np.float64)
        _check(lib().csx_recon_energy(self._h, _dev(y, self.ne * self.npix, "yE"), rp,
                                      _dev(f, self.nvox * self.nq, "f"), int(bool(init_uniform)), int(n_iter),
                                      float(beta), hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      _stream()))
        return hist

    def set_operator(self, forward_sai: bool = False, adjoint_sai: bool = False) -> None:
        """Operators of recon_step / recon / recon_warm: exact, or interpolated in angle."""
        ops = (OP_FORWARD_SAI if forward_sai else 0) | (OP_ADJOINT_SAI if adjoint_sai else 0)
        _check(lib().csx_set_operator(self._h, ops))

    def recon_os(self, y: torch.Tensor, f: torch.Tensor, n_iter: int, beta: float, rho_z: int = 8,
                 rho_y: int = 16, r: Optional[torch.Tensor] = None, init_uniform: bool = True) -> np.ndarray:
        """Alg. 6 (ordered subsets) for n_iter sweeps in place on f; returns J(f^0..f^n) (float64)."""
        rp = ctypes.c_void_p(None) if r is None else _dev(r, self.npix, "r")
        hist = np.zeros(n_iter + 1, dtype=np.float64)
        _check(lib().csx_recon_os(self._h, _dev(y, self.npix, "y"), rp, _dev(f, self.nvox * self.nq, "f"),
                                  int(bool(init_uniform)), int(n_iter), int(rho_z), int(rho_y), float(beta),
                                  hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream()))
        return hist

    # ---- learned warm start ----------------------------------------------------------
    def warm_input(self, y: torch.Tensor, delta: float, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Network input log(x + delta), x = A^T (y / (u A 1)) / b1, as an image [nz][nx][nq]."""
        out = self.new_image() if out is None else out
        _check(lib().csx_warm_input(self._h, _dev(y, self.npix, "y"), float(delta),
                                    _dev(out, self.nvox * self.nq, "x"), _stream()))
        return out

    def warm_output(self, y: torch.Tensor, o: torch.Tensor, delta: float,
                    out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """f0 = u max(exp(o) - delta, delta / 100)."""
        out = self.new_image() if out is None else out
        _check(lib().csx_warm_output(self._h, _dev(y, self.npix, "y"), _dev(o, self.nvox * self.nq, "o"),
                                     float(delta), _dev(out, self.nvox * self.nq, "f0"), _stream()))
        return out

    def warm_target(self, y: torch.Tensor, f: torch.Tensor, delta: float,
                    out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Training target log(f / u + delta)."""
        out = self.new_image() if out is None else out
        _check(lib().csx_warm_target(self._h, _dev(y, self.npix, "y"), _dev(f, self.nvox * self.nq, "f"),
                                     float(delta), _dev(out, self.nvox * self.nq, "t"), _stream()))
        return out

    def warm_start(self, y: torch.Tensor, net, delta: float, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Input map, the network (w16/b device tensors of 4 layers) and output map in one call."""
        out = self.new_image() if out is None else out
        wn = _WarmNet()
        for k in range(4):
            w16, b = net[k]
            if w16.dtype != torch.float16 or b.dtype != torch.float32 or not (w16.is_cuda and b.is_cuda):
                raise ValueError("layer weights must be CUDA float16 and biases CUDA float32")
            wn.w[k] = w16.data_ptr()
            wn.b[k] = b.data_ptr()
        _check(lib().csx_warm_start(self._h, _dev(y, self.npix, "y"), ctypes.byref(wn), float(delta),
                                    _dev(out, self.nvox * self.nq, "f0"), _stream()))
        return out

    def recon_warm(self, y: torch.Tensor, f_warm: torch.Tensor, f: torch.Tensor, k_judge: int, n_iter: int,
                   beta: float, r: Optional[torch.Tensor] = None):
        """The judge; returns (J history of the kept start, accepted)."""
        rp = ctypes.c_void_p(None) if r is None else _dev(r, self.npix, "r")
        hist = np.zeros(n_iter + 1, dtype=np.float64)
        acc = ctypes.c_int(0)
        _check(lib().csx_recon_warm(self._h, _dev(y, self.npix, "y"), rp,
                                    _dev(f_warm, self.nvox * self.nq, "f_warm"),
                                    _dev(f, self.nvox * self.nq, "f"), int(k_judge), int(n_iter), float(beta),
                                    hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(acc),
                                    _stream()))
        return hist, bool(acc.value)


def _img(t: torch.Tensor, dtype, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous CUDA {dtype} tensor")
    return ctypes.c_void_p(t.data_ptr())


def cnn_workspace_bytes(nb: int, h: int, w: int) -> int:
    return int(lib().csx_cnn_workspace_bytes(nb, h, w))


def conv3x3_forward(x: torch.Tensor, w16: torch.Tensor, bias: Optional[torch.Tensor], y: torch.Tensor,
                    relu: bool, residual: Optional[torch.Tensor] = None) -> torch.Tensor:
    """x [nb][h][w][cin] float32, w16 [9][cin][cout] float16 -> y [nb][h][w][cout]."""
    nb, h, w, ci = x.shape
    co = w16.shape[2]
    if tuple(w16.shape) != (9, ci, co) or tuple(y.shape) != (nb, h, w, co):
        raise ValueError("shape mismatch")
    if residual is not None and tuple(residual.shape) != tuple(y.shape):
        raise ValueError("residual shape mismatch")
    bp = ctypes.c_void_p(None) if bias is None else _img(bias, torch.float32, "bias")
    rp = ctypes.c_void_p(None) if residual is None else _img(residual, torch.float32, "residual")
    _check(lib().csx_conv3x3_forward(_img(x, torch.float32, "x"), _img(w16, torch.float16, "w"), bp, rp,
                                     _img(y, torch.float32, "y"), nb, h, w, ci, co, int(bool(relu)), _stream()))
    return y


def conv3x3_backward_data(dy: torch.Tensor, w16: torch.Tensor, mask: Optional[torch.Tensor],
                          dx: torch.Tensor) -> torch.Tensor:
    nb, h, w, co = dy.shape
    ci = w16.shape[1]
    if tuple(w16.shape) != (9, ci, co) or tuple(dx.shape) != (nb, h, w, ci):
        raise ValueError("shape mismatch")
    if mask is not None and tuple(mask.shape) != tuple(dx.shape):
        raise ValueError("mask shape mismatch")
    mp = ctypes.c_void_p(None) if mask is None else _img(mask, torch.float32, "mask")
    _check(lib().csx_conv3x3_backward_data(_img(dy, torch.float32, "dy"), _img(w16, torch.float16, "w"), mp,
                                           _img(dx, torch.float32, "dx"), nb, h, w, ci, co, _stream()))
    return dx


def conv3x3_backward_weights(x: torch.Tensor, dy: torch.Tensor, dw: torch.Tensor, dbias: Optional[torch.Tensor],
                             ws: torch.Tensor) -> None:
    nb, h, w, ci = x.shape
    co = dy.shape[3]
    if tuple(dy.shape) != (nb, h, w, co) or tuple(dw.shape) != (9, ci, co):
        raise ValueError("shape mismatch")
    bp = ctypes.c_void_p(None) if dbias is None else _img(dbias, torch.float32, "dbias")
    _check(lib().csx_conv3x3_backward_weights(_img(x, torch.float32, "x"), _img(dy, torch.float32, "dy"),
                                              _img(dw, torch.float32, "dw"), bp, nb, h, w, ci, co,
                                              _img(ws, torch.uint8, "ws"), ws.numel(), _stream()))


def warm_loss(o: torch.Tensor, t: torch.Tensor, d: torch.Tensor, loss: torch.Tensor, ws: torch.Tensor) -> None:
    nb = o.shape[0]
    if o.shape != t.shape or o.shape != d.shape or loss.dtype != torch.float64 or not loss.is_cuda:
        raise ValueError("shape / dtype mismatch")
    _check(lib().csx_warm_loss(_img(o, torch.float32, "o"), _img(t, torch.float32, "t"), nb, o.numel() // nb,
                               _img(d, torch.float32, "d"), ctypes.c_void_p(loss.data_ptr()),
                               _img(ws, torch.uint8, "ws"), ws.numel(), _stream()))


def adam_step(w: torch.Tensor, m: torch.Tensor, v: torch.Tensor, g: torch.Tensor, w16: Optional[torch.Tensor],
              step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> None:
    n = w.numel()
    for t, name in ((m, "m"), (v, "v"), (g, "g")):
        if t.numel() != n:
            raise ValueError(f"{name} size mismatch")
    hp = ctypes.c_void_p(None)
    if w16 is not None:
        if w16.numel() != n:
            raise ValueError("w16 size mismatch")
        hp = _img(w16, torch.float16, "w16")
    _check(lib().csx_adam_step(_img(w, torch.float32, "w"), _img(m, torch.float32, "m"),
                               _img(v, torch.float32, "v"), _img(g, torch.float32, "g"), hp, n, lr, beta1,
                               beta2, eps, int(step), _stream()))


def to_half(x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    if x.numel() != y.numel():
        raise ValueError("size mismatch")
    _check(lib().csx_to_half(_img(x, torch.float32, "x"), _img(y, torch.float16, "y"), x.numel(), _stream()))
    return y


def valu_peak() -> float:
    """Measured float32 FMA issue rate of the current GPU (lane-ops/s)."""
    v = ctypes.c_double()
    _check(lib().csx_valu_peak(ctypes.byref(v), _stream()))
    return v.value


class Batch:
    """Independent scans reconstructed together (the batched form)."""

    def __init__(self, geoms):
        self.geoms = list(geoms)
        arr = (ctypes.c_void_p * len(self.geoms))(*[g._h.value for g in self.geoms])
        h = ctypes.c_void_p()
        _check(lib().csx_batch_create(arr, len(self.geoms), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().csx_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def recon(self, ys, fs, n_iter, beta: float, rs=None, init_uniform: bool = True) -> np.ndarray:
        """Alg. 5 on every scan in place; returns J histories [n_scans][max(n_iter) + 1].
        n_iter is one count for all scans or a sequence of per-scan counts (then
        row k holds J(f^0..f^n_k) followed by NaN)."""
        n = len(self.geoms)
        if len(ys) != n or len(fs) != n or (rs is not None and len(rs) != n):
            raise ValueError("one y and one f per scan")
        yp = (ctypes.c_void_p * n)(*[_dev(y, g.npix, "y").value for y, g in zip(ys, self.geoms)])
        fp = (ctypes.c_void_p * n)(*[_dev(f, g.nvox * g.nq, "f").value for f, g in zip(fs, self.geoms)])
        rp = None
        if rs is not None:
            rp = (ctypes.c_void_p * n)(*[None if r is None else _dev(r, g.npix, "r").value
                                         for r, g in zip(rs, self.geoms)])
        if np.ndim(n_iter) == 0:
            hist = np.zeros((n, int(n_iter) + 1), dtype=np.float64)
            _check(lib().csx_batch_recon(self._h, yp, rp, fp, int(bool(init_uniform)), int(n_iter),
                                         float(beta), hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                         _stream()))
            return hist
        counts = [int(c) for c in n_iter]
        if len(counts) != n:
            raise ValueError("one iteration count per scan")
        stride = max(counts) + 1
        hist = np.full((n, stride), np.nan, dtype=np.float64)
        cp = (ctypes.c_int * n)(*counts)
        _check(lib().csx_batch_recon_n(self._h, yp, rp, fp, int(bool(init_uniform)), cp, float(beta),
                                       hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), stride,
                                       _stream()))
        return hist

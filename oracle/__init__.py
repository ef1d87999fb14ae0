"""FP64 CPU oracle for fan-beam coded-aperture coherent-scatter reconstruction.

TEST INFRASTRUCTURE.  Only tests/, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the GPU library (``paper_1603_06400_amd``) and neither imports the
other; both consume ``paper_1603_06400_amd.inputs`` (seeded inputs only).

Layers, each following the paper (Odinaka et al., arXiv:1603.06400):

* ``forward`` / ``adjoint`` / ``dense`` -- the system matrix of Sec. II eq. 2
  evaluated per triple in double precision by ``csx_oracle.c`` (Alg. 1 and
  Alg. 3 without any optimisation).
* ``objective`` -- J(f) = L(f) + beta R(f) of Sec. V (eqs. overall_objective,
  standard_EPR) with the quadratic potential psi(t) = t^2/2 or Huber's
  edge-preserving potential (``potential``).
* ``surrogate_coefficients`` / ``lemma_minimizer`` / ``recon_step`` /
  ``recon`` -- the separable-surrogate EM-type update of Sec. VI, Alg. 5 and
  App. B-C (eqs. grad_sep_obj, f_update, Lemma 1).
* ``os_partition`` / ``recon_os`` -- the ordered-subsets variant, Alg. 6,
  with the symmetry-preserving partition of Sec. VI.
* ``forward_sai`` / ``adjoint_sai`` -- scatter-angle interpolation (Sec.
  III-B, the precompute and interpolate lines of Alg. 2 / Alg. 4): W(r,
  theta) of eq. q_integral on a uniform angle table, interpolated per pair.
* ``forward_energy`` / ``adjoint_energy`` -- the energy-sensitive detector of
  App. A (eq. energy_sensitive): each triple's contribution is kept in the
  spectrum bin of its Bragg energy kappa q instead of being summed over E.

Parity status: every function here is pinned by tests in tests/test_oracle_*.py
(closed forms, brute force, invariants); the absolute normalisation C has no
numeric value in the paper and is an input.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np
from scipy.special import gammaln

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csx_oracle.c")
_LIBDIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_LIBDIR, "libcsx_oracle.so")


def build(force: bool = True) -> str:
    """Compile the C oracle (gcc, OpenMP, no fast-math, no FMA contraction)."""
    os.makedirs(_LIBDIR, exist_ok=True)
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        # CSX_ORACLE_LIB: another build of the same source (the sanitizer test's)
        path = os.environ.get("CSX_ORACLE_LIB")
        if not path:
            if not os.path.exists(_LIB):
                build(force=False)
            path = _LIB
        lib = ctypes.CDLL(path)
        P = ctypes.POINTER
        gp = P(_OrcGeom)
        dp = P(ctypes.c_double)
        ip = P(ctypes.c_int)
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_max_threads.restype = ctypes.c_int
        lib.orc_pair_factors.argtypes = [gp, ctypes.c_int, ctypes.c_int, dp]
        lib.orc_spectral_factor.argtypes = [gp, ctypes.c_int, ctypes.c_int, ctypes.c_double]
        lib.orc_spectral_factor.restype = ctypes.c_double
        lib.orc_forward.argtypes = [gp, dp, dp]
        lib.orc_forward_pixels.argtypes = [gp, dp, ip, ctypes.c_int, dp]
        lib.orc_adjoint.argtypes = [gp, dp, dp]
        lib.orc_adjoint_voxels.argtypes = [gp, dp, ip, ctypes.c_int, dp]
        lib.orc_dense.argtypes = [gp, dp]
        lib.orc_census.argtypes = [gp, dp]
        lib.orc_margins.argtypes = [gp, dp]
        lib.orc_forward_sai.argtypes = [gp, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, dp]
        lib.orc_adjoint_sai.argtypes = [gp, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, dp]
        lib.orc_max_angle.argtypes = [gp]
        lib.orc_max_angle.restype = ctypes.c_double
        lib.orc_forward_energy.argtypes = [gp, dp, dp]
        lib.orc_adjoint_energy.argtypes = [gp, dp, dp]
        _lib = lib
    return _lib


class _OrcGeom(ctypes.Structure):
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
    ]


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Oracle:
    """Binds one scan geometry (an ``inputs.ScanGeometry``) to the C oracle."""

    def __init__(self, geom, phi: Optional[np.ndarray] = None):
        self.geom = geom
        self._q = np.ascontiguousarray(geom.q, dtype=np.float64)
        self._phi = np.ascontiguousarray(geom.phi if phi is None else phi, dtype=np.float64)
        self._mask = np.ascontiguousarray(geom.mask, dtype=np.uint8)
        s = _OrcGeom()
        s.nx, s.nz = geom.nx, geom.nz
        s.x_min, s.x_max, s.z_min, s.z_max = geom.x_min, geom.x_max, geom.z_min, geom.z_max
        s.nq, s.q = self._q.shape[0], _dptr(self._q)
        s.ndx, s.ndy, s.det_pitch, s.det_z = geom.ndx, geom.ndy, geom.det_pitch, geom.det_z
        s.mask_z, s.mask_pitch = geom.mask_z, geom.mask_pitch
        s.mask_ny, s.mask_nx = self._mask.shape
        s.mask = self._mask.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte))
        s.ne, s.e_lo, s.e_hi, s.phi = self._phi.shape[0], geom.e_lo, geom.e_hi, _dptr(self._phi)
        s.C, s.hc = geom.C, geom.hc
        self._s = s
        self._lib = _load()

    # ---- system matrix -------------------------------------------------------------
    def pair(self, j: int, i: int) -> dict:
        out = np.zeros(9)
        self._lib.orc_pair_factors(ctypes.byref(self._s), int(j), int(i), _dptr(out))
        keys = ["Gso", "God", "T", "dtheta", "sin", "cos", "sin_half", "cos_half", "kappa"]
        return dict(zip(keys, out.tolist()))

    def spectral_factor(self, j: int, i: int, q: float) -> float:
        return float(self._lib.orc_spectral_factor(ctypes.byref(self._s), int(j), int(i), float(q)))

    def forward(self, f: np.ndarray) -> np.ndarray:
        g = self.geom
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(g.nz, g.nx, g.nq)
        out = np.zeros((g.ndy, g.ndx))
        self._lib.orc_forward(ctypes.byref(self._s), _dptr(f), _dptr(out))
        return out

    def forward_pixels(self, f: np.ndarray, pix: Sequence[int]) -> np.ndarray:
        g = self.geom
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(g.nz, g.nx, g.nq)
        pix = np.ascontiguousarray(pix, dtype=np.int32)
        out = np.zeros(pix.shape[0])
        self._lib.orc_forward_pixels(ctypes.byref(self._s), _dptr(f),
                                     pix.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                     int(pix.shape[0]), _dptr(out))
        return out

    def adjoint(self, y: np.ndarray) -> np.ndarray:
        g = self.geom
        y = np.ascontiguousarray(y, dtype=np.float64).reshape(g.ndy, g.ndx)
        out = np.zeros((g.nz, g.nx, g.nq))
        self._lib.orc_adjoint(ctypes.byref(self._s), _dptr(y), _dptr(out))
        return out

    def adjoint_voxels(self, y: np.ndarray, vox: Sequence[int]) -> np.ndarray:
        g = self.geom
        y = np.ascontiguousarray(y, dtype=np.float64).reshape(g.ndy, g.ndx)
        vox = np.ascontiguousarray(vox, dtype=np.int32)
        out = np.zeros((vox.shape[0], g.nq))
        self._lib.orc_adjoint_voxels(ctypes.byref(self._s), _dptr(y),
                                     vox.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                     int(vox.shape[0]), _dptr(out))
        return out

    def dense(self) -> np.ndarray:
        g = self.geom
        H = np.zeros((g.npix, g.nvox * g.nq))
        self._lib.orc_dense(ctypes.byref(self._s), _dptr(H))
        return H

    # ---- scatter-angle interpolation (Sec. III-B) --------------------------------
    def max_angle(self) -> float:
        """Largest scatter angle over all voxel-pixel pairs (rad)."""
        return float(self._lib.orc_max_angle(ctypes.byref(self._s)))

    def forward_sai(self, f: np.ndarray, nt: int, theta_max: float, interp: int = 1) -> np.ndarray:
        """g with W(r, theta) interpolated from nt uniform angles on [0, theta_max]
        (nearest node for interp = 0, linear for interp = 1); the geometric angle
        factor stays exact per pair."""
        g = self.geom
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(g.nz, g.nx, g.nq)
        out = np.zeros((g.ndy, g.ndx))
        self._lib.orc_forward_sai(ctypes.byref(self._s), int(nt), int(interp), float(theta_max), _dptr(f),
                                  _dptr(out))
        return out

    def adjoint_sai(self, y: np.ndarray, nt: int, theta_max: float, interp: int = 1) -> np.ndarray:
        """The transpose of forward_sai."""
        g = self.geom
        y = np.ascontiguousarray(y, dtype=np.float64).reshape(g.ndy, g.ndx)
        out = np.zeros((g.nz, g.nx, g.nq))
        self._lib.orc_adjoint_sai(ctypes.byref(self._s), int(nt), int(interp), float(theta_max), _dptr(y),
                                  _dptr(out))
        return out

    def forward_energy(self, f: np.ndarray) -> np.ndarray:
        """Energy-resolved detector (App. A eq. energy_sensitive): g_E[k][i]
        collects the triples whose Bragg energy kappa q falls in spectrum bin k;
        shape (ne, ndy, ndx)."""
        g = self.geom
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(g.nz, g.nx, g.nq)
        out = np.zeros((g.ne, g.ndy, g.ndx))
        self._lib.orc_forward_energy(ctypes.byref(self._s), _dptr(f), _dptr(out))
        return out

    def adjoint_energy(self, y: np.ndarray) -> np.ndarray:
        """The transpose of forward_energy; y of shape (ne, ndy, ndx)."""
        g = self.geom
        y = np.ascontiguousarray(y, dtype=np.float64).reshape(g.ne, g.ndy, g.ndx)
        out = np.zeros((g.nz, g.nx, g.nq))
        self._lib.orc_adjoint_energy(ctypes.byref(self._s), _dptr(y), _dptr(out))
        return out

    def census(self) -> dict:
        out = np.zeros(4)
        self._lib.orc_census(ctypes.byref(self._s), _dptr(out))
        return {"pairs": out[0], "open_pairs": out[1], "open_triples_in_band": out[2],
                "open_pairs_in_band": out[3]}

    def margins(self) -> dict:
        out = np.zeros(2)
        self._lib.orc_margins(ctypes.byref(self._s), _dptr(out))
        return {"mask_edge_mm": out[0], "bin_edge": out[1]}

    # ---- solver (Sec. V-VI, App. B-C) -------------------------------------------------
    def sensitivity(self) -> np.ndarray:
        """b^(1) = Back_project(1) (Alg. 5, precompute line)."""
        g = self.geom
        return self.adjoint(np.ones((g.ndy, g.ndx)))

    def recon_step(self, y, r, fhat, beta, b1=None, psi=None):
        """One iteration of Alg. 5 from fhat; returns (f_next, J(fhat))."""
        g = self.geom
        y = np.asarray(y, dtype=np.float64).reshape(g.ndy, g.ndx)
        r = np.zeros_like(y) if r is None else np.asarray(r, dtype=np.float64).reshape(y.shape)
        fhat = np.asarray(fhat, dtype=np.float64).reshape(g.nz, g.nx, g.nq)
        if b1 is None:
            b1 = self.sensitivity()
        z = self.forward(fhat) + r
        J = objective_from_mean(y, z, fhat, beta, psi)
        b2 = self.adjoint(poisson_ratio(y, z))
        return em_update(fhat, b1, b2, beta, psi), J

    def recon(self, y, r, f0, n_iter, beta, psi=None):
        """Alg. 5: n_iter iterations from f0; returns (f_T, [J(f^0), ..., J(f^T)])."""
        b1 = self.sensitivity()
        f = np.asarray(f0, dtype=np.float64).copy()
        hist = []
        for _ in range(n_iter):
            f, J = self.recon_step(y, r, f, beta, b1=b1, psi=psi)
            hist.append(J)
        g = self.geom
        rr = np.zeros((g.ndy, g.ndx)) if r is None else np.asarray(r, dtype=np.float64).reshape(g.ndy, g.ndx)
        hist.append(objective_from_mean(np.asarray(y, dtype=np.float64).reshape(g.ndy, g.ndx),
                                        self.forward(f) + rr, f, beta, psi))
        return f, np.array(hist)

    def recon_os(self, y, r, f0, n_iter, beta, subsets):
        """Alg. 6 (ordered subsets): n_iter outer iterations from f0, each a
        sweep over the pixel subsets in the given order.  Sub-step p uses the
        subset's data only: z_p = A_p f + r_p, b^(1)_p = A_p^T 1, b^(2)_p =
        A_p^T (y_p / z_p), and the update of eq. f_update with b^(1)_p,
        b^(2)_p and penalty weight beta / P (one penalty per sweep, like the
        data term).  Returns (f_T, [J(f^0), ..., J(f^T)]) with the full
        objective J."""
        g = self.geom
        y = np.asarray(y, dtype=np.float64).reshape(-1)
        rr = np.zeros(g.npix) if r is None else np.asarray(r, dtype=np.float64).reshape(-1)
        P = len(subsets)
        b1 = []
        for pix in subsets:
            ind = np.zeros(g.npix)
            ind[pix] = 1.0
            b1.append(self.adjoint(ind.reshape(g.ndy, g.ndx)))
        f = np.asarray(f0, dtype=np.float64).reshape(g.nz, g.nx, g.nq).copy()
        hist = [self.objective(y, r, f, beta)]
        for _ in range(n_iter):
            for p, pix in enumerate(subsets):
                z = self.forward_pixels(f, pix) + rr[pix]
                rho = np.zeros(g.npix)
                rho[pix] = poisson_ratio(y[pix], z)
                b2 = self.adjoint(rho.reshape(g.ndy, g.ndx))
                f = em_update(f, b1[p], b2, beta / P)
            hist.append(self.objective(y, r, f, beta))
        return f, np.array(hist)

    def objective(self, y, r, f, beta, psi=None) -> float:
        g = self.geom
        y = np.asarray(y, dtype=np.float64).reshape(g.ndy, g.ndx)
        r = np.zeros_like(y) if r is None else np.asarray(r, dtype=np.float64).reshape(y.shape)
        return objective_from_mean(y, self.forward(f) + r, f, beta, psi)


# ---- pieces of the objective and the update ----------------------------------------------

def uniform_start(y: np.ndarray, b1: np.ndarray) -> np.ndarray:
    """f^0 = sum(y) / sum(b^(1)) in every voxel and q (uniform initial image)."""
    return np.full(b1.shape, float(np.sum(y)) / float(np.sum(b1)))


def neighbour_diffs(f: np.ndarray):
    """Differences f_j - f_k over the 4 in-slice neighbours (+-x, +-z) at the same q,
    returned per direction with zeros where the neighbour does not exist, and the
    neighbour count |N_j| per voxel."""
    f = np.asarray(f, dtype=np.float64)
    nz, nx = f.shape[0], f.shape[1]
    d = np.zeros((4,) + f.shape)
    cnt = np.zeros((nz, nx))
    d[0, :, 1:] = f[:, 1:] - f[:, :-1]
    d[1, :, :-1] = f[:, :-1] - f[:, 1:]
    d[2, 1:] = f[1:] - f[:-1]
    d[3, :-1] = f[:-1] - f[1:]
    cnt[:, 1:] += 1
    cnt[:, :-1] += 1
    cnt[1:] += 1
    cnt[:-1] += 1
    return d, cnt


def neighbour_exists(f: np.ndarray) -> np.ndarray:
    """[4][nz][nx] masks of the neighbours used by neighbour_diffs."""
    nz, nx = np.asarray(f).shape[0], np.asarray(f).shape[1]
    e = np.zeros((4, nz, nx), dtype=bool)
    e[0, :, 1:] = True
    e[1, :, :-1] = True
    e[2, 1:] = True
    e[3, :-1] = True
    return e


def potential(psi):
    """(psi, psi', omega = psi'(t)/t) of a potential (Sec. V, App. B).
    psi None or ("quadratic",): t^2/2.  ("huber", delta): Huber's potential,
    t^2/2 for |t| <= delta and delta |t| - delta^2/2 beyond, so psi' = t or
    delta sign(t) and omega = 1 or delta/|t| (omega(0) = 1)."""
    if psi is None or psi[0] == "quadratic":
        return (lambda t: 0.5 * t * t, lambda t: t, lambda t: np.ones_like(t))
    if psi[0] == "huber":
        dl = float(psi[1])
        inner = lambda t: np.abs(t) <= dl
        return (lambda t: np.where(inner(t), 0.5 * t * t, dl * np.abs(t) - 0.5 * dl * dl),
                lambda t: np.where(inner(t), t, dl * np.sign(t)),
                lambda t: np.where(inner(t), 1.0, dl / np.where(inner(t), 1.0, np.abs(t))))
    raise ValueError(f"unknown potential {psi!r}")


def penalty(f: np.ndarray, psi=None) -> float:
    """R(f) = sum_j sum_{k in N_j} w_jk psi(f_j - f_k) with w = 1 (Sec. V eq.
    standard_EPR; every neighbour pair appears once from each side)."""
    d, _ = neighbour_diffs(f)
    e = neighbour_exists(f)
    p, _, _ = potential(psi)
    f = np.asarray(f)
    mask = e if f.ndim == 2 else e[..., None] * np.ones(f.shape[2:], dtype=bool)
    return float(np.sum(np.where(mask, p(d), 0.0)))


def poisson_ratio(y: np.ndarray, z: np.ndarray) -> np.ndarray:
    """y / z with 0/z = 0 (the data term's back-projected ratio, Alg. 5)."""
    out = np.zeros_like(z)
    nz = y > 0
    out[nz] = y[nz] / z[nz]
    return out


def data_fit(y: np.ndarray, z: np.ndarray) -> float:
    """L = sum_i (l_i + r_i) - y_i ln(l_i + r_i) + ln(y_i!) with z = l + r and 0 ln 0 = 0."""
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    if np.any((z <= 0) & (y > 0)):
        return float("inf")
    ylog = np.zeros_like(z)
    nz = y > 0
    ylog[nz] = y[nz] * np.log(z[nz])
    return float(np.sum(z - ylog + gammaln(y + 1.0)))


def objective_from_mean(y, z, f, beta, psi=None) -> float:
    """J(f) = L(f) + beta R(f) (Sec. V eq. overall_objective)."""
    return data_fit(y, z) + beta * penalty(f, psi)


def surrogate_coefficients(fhat, b1, b2, beta, psi=None):
    """b^(3)..b^(6) and chi^(1..3) of App. B with symmetric 4-neighbourhoods
    and w = 1: b3 = b4 = 2 sum_k omega(fhat_j - fhat_k), b5 = b6 = sum_k
    psi'(fhat_j - fhat_k)."""
    fhat = np.asarray(fhat, dtype=np.float64)
    d, cnt = neighbour_diffs(fhat)
    e = neighbour_exists(fhat)[..., None]
    _, dp, om = potential(psi)
    b3 = 2.0 * np.sum(np.where(e, om(d), 0.0), axis=0)   # 2 sum_k w omega
    b4 = b3.copy()                                        # same set for a symmetric N
    b5 = np.sum(np.where(e, dp(d), 0.0), axis=0)         # sum_k w psi'(fhat_j - fhat_k)
    b6 = b5.copy()
    chi1 = beta * (b3 + b4)
    chi2 = b1 + beta * (-fhat * (b3 + b4) + b5 + b6)
    chi3 = fhat * b2
    return chi1, chi2, chi3


def lemma_minimizer(a, b, c):
    """Minimiser of (1/2) a x^2 + b x - c ln x on [0, inf] (App. C, Lemma 1).

    a > 0: the positive root of a x^2 + b x - c = 0, written for b > 0 as
    2c / (b + sqrt(b^2 + 4ac)) (multiply the Lemma's form by its conjugate; no
    cancellation) and for b <= 0 as the Lemma's (-b + sqrt(b^2 + 4ac)) / (2a).
    a = 0, b > 0: c / b.  a = 0, b <= 0: +inf.
    """
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    a, b, c = np.broadcast_arrays(a, b, c)
    disc = np.sqrt(b * b + 4.0 * a * c)
    out = np.empty(a.shape)
    pos = b > 0
    out[pos] = 2.0 * c[pos] / (b[pos] + disc[pos])
    neg = ~pos
    with np.errstate(divide="ignore", invalid="ignore"):
        out[neg] = np.where(a[neg] > 0, (-b[neg] + disc[neg]) / (2.0 * a[neg]), np.inf)
    return out


def em_update(fhat, b1, b2, beta, psi=None):
    """f^{t+1} from eq. f_update (App. B) via Lemma 1.

    Lemma 1's unbounded case (chi1 = 0, chi2 <= 0) needs beta = 0 and a voxel
    that no pixel sees (b^(1)_j = 0); such a voxel keeps its previous value."""
    fhat = np.asarray(fhat, dtype=np.float64)
    chi1, chi2, chi3 = surrogate_coefficients(fhat, b1, b2, beta, psi)
    out = lemma_minimizer(chi1, chi2, chi3)
    stuck = (chi1 <= 0) & (chi2 <= 0)
    return np.where(stuck, fhat, out)


def os_partition(ndy: int, ndx: int, rho_z: int, rho_y: int):
    """The symmetry-preserving detector partition of Sec. VI (ordered subsets):
    a subset is one vertical class and one horizontal class.  Vertical class
    rz (0 <= rz < rho_z) holds rows rz, rz + rho_z, ... of one half of the
    detector (ndy / 2 rows) and their up-down mirrors ndy - 1 - row;
    horizontal class cy (0 <= cy < rho_y / 2) holds columns cy, cy + rho_y,
    ... and their left-right mirrors ndx - 1 - column.  Subset p = rz
    (rho_y / 2) + cy (the sweep order, which the paper leaves open); each is
    returned as sorted pixel indices row * ndx + column."""
    if ndy % 2 or (ndy // 2) % rho_z or ndx % rho_y or rho_y % 2:
        raise ValueError("need rho_z | ndy/2, rho_y | ndx and rho_y even")
    out = []
    for rz in range(rho_z):
        rows = list(range(rz, ndy // 2, rho_z))
        rows = sorted(set(rows + [ndy - 1 - r for r in rows]))
        for cy in range(rho_y // 2):
            cols = list(range(cy, ndx, rho_y))
            cols = sorted(set(cols + [ndx - 1 - c for c in cols]))
            out.append(np.array(sorted(r * ndx + c for r in rows for c in cols), dtype=np.int64))
    return out


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (round to nearest, ties to even) via float32, returned as
    float64: the table values the reduced-precision form is defined on."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


def set_threads(n: int) -> None:
    _load().orc_set_threads(int(n))


def max_threads() -> int:
    return int(_load().orc_max_threads())

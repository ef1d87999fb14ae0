"""Seeded synthetic inputs for fan-beam coded-aperture coherent-scatter scans.

This module builds the *inputs* of the reconstruction problem and nothing else:
the scan geometry, the q grid, the binned source spectrum, the binary
secondary-mask image, object phantoms and Poisson count sampling from a given
mean.  It holds none of the method's arithmetic (no forward model, adjoint,
objective or update), so both the FP64 oracle and the GPU path consume what it
makes without sharing any computation.

Frame (used everywhere in this repository): the source focal spot is the
origin, the fan plane is y = 0, depth runs along +z through the object, the
secondary mask and the detector are planes z = const.  A voxel is the point
(x, 0, z); a detector pixel centre is (x', y', det_z).  This is the paper's
frame (Sec. II) with its axes renamed: paper x (central ray) -> z, paper y
(in-plane transverse) -> x, paper z (out of plane) -> y.

q is in nm^-1 with q = E sin(theta/2) / hc (App. A, eq. bragg); hc is quoted in
the paper as 12.3984193 keV*Angstrom, i.e. 1.23984193 keV*nm.
"""
from __future__ import annotations

from dataclasses import dataclass, replace
from typing import List, Optional

import numpy as np

HC_KEV_NM = 1.23984193

# Shared scan layout of the synthetic workloads (mm, keV, nm^-1).
X_RANGE = (-40.0, 40.0)
Z_RANGE = (400.0, 600.0)
MASK_Z = 700.0
DET_Z = 800.0
PITCH = 1.0
MASK_PERIOD = 16
Q_RANGE = (0.5, 3.5)
E_RANGE = (20.0, 160.0)
PEAK_SIGMA = 0.05


@dataclass
class ScanGeometry:
    """Everything that defines the system matrix of one fan slice.

    Voxels are cell-centred on nx x nz cells covering [x_min,x_max] x
    [z_min,z_max]; f is laid out [nz][nx][nq] (q fastest).  Detector pixels
    are centred on the central ray: x'_a = (a - ndx/2 + 1/2) * det_pitch,
    y'_b = (b - ndy/2 + 1/2) * det_pitch; g is laid out [ndy][ndx].
    The mask image is [mask_ny][mask_nx] of 0/1; cell (c, r) covers
    x in [c, c+1) * mask_pitch (periodic in x with period mask_nx cells) and
    y in [r - mask_ny/2, r - mask_ny/2 + 1) * mask_pitch; rows outside the
    image are opaque.  The spectrum is a histogram of ne equal bins on
    [e_lo, e_hi); phi[k] is the flux of bin k.
    """

    nx: int
    nz: int
    x_min: float
    x_max: float
    z_min: float
    z_max: float
    q: np.ndarray
    ndx: int
    ndy: int
    det_pitch: float
    det_z: float
    mask_z: float
    mask_pitch: float
    mask: np.ndarray
    e_lo: float
    e_hi: float
    phi: np.ndarray
    C: float = 1.0
    hc: float = HC_KEV_NM

    @property
    def nq(self) -> int:
        return int(self.q.shape[0])

    @property
    def ne(self) -> int:
        return int(self.phi.shape[0])

    @property
    def mask_nx(self) -> int:
        return int(self.mask.shape[1])

    @property
    def mask_ny(self) -> int:
        return int(self.mask.shape[0])

    @property
    def nvox(self) -> int:
        return self.nx * self.nz

    @property
    def npix(self) -> int:
        return self.ndx * self.ndy

    def with_(self, **kw) -> "ScanGeometry":
        return replace(self, **kw)


def q_bin_centres(nq: int, lo: float = Q_RANGE[0], hi: float = Q_RANGE[1]) -> np.ndarray:
    """nq momentum-transfer nodes at the centres of equal bins on [lo, hi]."""
    dq = (hi - lo) / nq
    return lo + (np.arange(nq, dtype=np.float64) + 0.5) * dq


def kramers_histogram(ne: int, e_lo: float = E_RANGE[0], e_hi: float = E_RANGE[1],
                      kvp: float = 160.0) -> np.ndarray:
    """Kramers-law spectrum (kvp - E)/E sampled at the centres of ne equal bins."""
    de = (e_hi - e_lo) / ne
    ec = e_lo + (np.arange(ne, dtype=np.float64) + 0.5) * de
    return np.maximum(kvp - ec, 0.0) / ec


def make_mask(seed: int, rows: int, period: int = MASK_PERIOD,
              open_frac: float = 0.5) -> np.ndarray:
    """Binary mask image [rows][period] with max(1, round(frac*cells)) open cells
    placed by a seeded permutation."""
    cells = rows * period
    n_open = max(1, int(round(open_frac * cells)))
    rng = np.random.Generator(np.random.PCG64(seed))
    perm = rng.permutation(cells)
    m = np.zeros(cells, dtype=np.uint8)
    m[perm[:n_open]] = 1
    return m.reshape(rows, period)


def standard_geometry(n: int, nq: int, ne: Optional[int] = None, *, mask_seed: int = 7,
                      open_frac: float = 0.5, C: float = 1.0,
                      ndet: Optional[int] = None) -> ScanGeometry:
    """The synthetic scan layout: n x n voxels on x in [-40,40], z in [400,600] mm;
    mask at z=700 mm (1 mm cells, period 16, one row per detector row);
    ndet x ndet detector (default n) at z=800 mm with 1 mm pitch; nq q bins on
    [0.5, 3.5] nm^-1; ne (default nq) Kramers bins on [20, 160) keV."""
    ne = nq if ne is None else ne
    ndet = n if ndet is None else ndet
    return ScanGeometry(
        nx=n, nz=n, x_min=X_RANGE[0], x_max=X_RANGE[1], z_min=Z_RANGE[0], z_max=Z_RANGE[1],
        q=q_bin_centres(nq), ndx=ndet, ndy=ndet, det_pitch=PITCH, det_z=DET_Z,
        mask_z=MASK_Z, mask_pitch=PITCH,
        mask=make_mask(mask_seed, ndet, MASK_PERIOD, open_frac),
        e_lo=E_RANGE[0], e_hi=E_RANGE[1], phi=kramers_histogram(ne), C=C)


def phantom(geom: ScanGeometry, seed: int, n_rect: int = 3,
            sigma: float = PEAK_SIGMA) -> np.ndarray:
    """Object scatter density f [nz][nx][nq] (float64): n_rect axis-aligned
    rectangles in voxel-index space (each side >= 2 voxels, overlaps add), each
    carrying a form factor of 1-3 Gaussian peaks a*exp(-(q-mu)^2/(2 sigma^2))
    with mu ~ U[0.7, 3.3] nm^-1 and a ~ U[0.5, 1]; background 0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    f = np.zeros((geom.nz, geom.nx, geom.nq), dtype=np.float64)
    for _ in range(n_rect):
        i0 = int(rng.integers(0, max(1, geom.nx - 1)))
        i1 = int(rng.integers(min(i0 + 2, geom.nx), geom.nx + 1))
        k0 = int(rng.integers(0, max(1, geom.nz - 1)))
        k1 = int(rng.integers(min(k0 + 2, geom.nz), geom.nz + 1))
        npk = int(rng.integers(1, 4))
        mu = rng.uniform(0.7, 3.3, size=npk)
        amp = rng.uniform(0.5, 1.0, size=npk)
        prof = np.zeros(geom.nq)
        for a, m in zip(amp, mu):
            prof += a * np.exp(-(geom.q - m) ** 2 / (2.0 * sigma * sigma))
        f[k0:k1, i0:i1, :] += prof[None, None, :]
    return f


def random_image(geom: ScanGeometry, seed: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """Dense uniform random image [nz][nx][nq] (operator tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, size=(geom.nz, geom.nx, geom.nq))


def random_detector(geom: ScanGeometry, seed: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """Dense uniform random detector image [ndy][ndx] (operator tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, size=(geom.ndy, geom.ndx))


def poisson_counts(mean: np.ndarray, seed: int) -> np.ndarray:
    """Integer Poisson counts with the given mean (returned as float64).  A
    mean below zero counts as zero: a float32 forward of a nonnegative image
    can return -1e-15 of its maximum where the exact value is 0 (the interval
    form takes differences of prefix sums).  NaN still raises."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.poisson(np.maximum(np.asarray(mean, dtype=np.float64), 0.0)).astype(np.float64)


# ----------------------------------------------------------------------------
# Workload registry
# ----------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    geom: ScanGeometry
    phantom_seed: int
    noise_seed: int
    n_rect: int
    n_iter: int
    beta: float


def workload(name: str) -> Workload:
    """The synthetic workloads: 'slice32' (32^2 voxels x 32 q, 32^2 detector,
    20 iterations), 'slice128' (128^2 x 64 q, 128^2 detector, 50 iterations,
    beta 1e-3) and the open-fraction variants 'slice128_open1' (1 %) and
    'slice128_open01' (0.1 %)."""
    if name == "slice32":
        return Workload(name, standard_geometry(32, 32), 0, 1, 3, 20, 1e-3)
    if name == "slice128":
        return Workload(name, standard_geometry(128, 64), 0, 1, 3, 50, 1e-3)
    if name == "slice128_open1":
        return Workload(name, standard_geometry(128, 64, mask_seed=8, open_frac=0.01), 0, 1, 3, 50, 1e-3)
    if name == "slice128_open01":
        return Workload(name, standard_geometry(128, 64, mask_seed=9, open_frac=0.001), 0, 1, 3, 50, 1e-3)
    raise KeyError(name)


def paper_geometry(mask_seed: int = 17, open_frac: float = 0.5, ne: int = 64, C: float = 1.0) -> ScanGeometry:
    """The shape of the paper's simulation (Sec. VII) with stand-ins for what
    it measured: 28 x 28 voxels of 2.5 mm (x) by 3.04 mm (z), 70 mm across and
    85.12 mm deep, centred at z = 1035 mm; a 1536 x 2048 detector of 0.19 mm
    pixels at z = 1546.5 mm, the secondary mask 100 mm in front of it; 79 q
    nodes evenly spaced from 0.1 to 4.0 nm^-1 (0.01 to 0.4 A^-1, both ends
    included).  Stand-ins: a seeded random mask of 1 mm cells (period 16, 320
    rows, covering every ray) and a Kramers spectrum to 125 kVp in ne bins on
    [20, 125) keV."""
    return ScanGeometry(
        nx=28, nz=28, x_min=-35.0, x_max=35.0, z_min=1035.0 - 42.56, z_max=1035.0 + 42.56,
        q=np.linspace(0.1, 4.0, 79), ndx=1536, ndy=2048, det_pitch=0.19, det_z=1546.5,
        mask_z=1446.5, mask_pitch=1.0, mask=make_mask(mask_seed, 320, MASK_PERIOD, open_frac),
        e_lo=20.0, e_hi=125.0, phi=kramers_histogram(ne, 20.0, 125.0, kvp=125.0), C=C)


def paper_phantom(geom: ScanGeometry, sigma: float = PEAK_SIGMA) -> np.ndarray:
    """Two 4 x 4-voxel vials 20 mm apart across the fan, each holding a
    material with a Gaussian-peak form factor (peaks at 1.9 and 2.7 nm^-1 in
    one, 2.3 nm^-1 in the other); background 0."""
    f = np.zeros((geom.nz, geom.nx, geom.nq), dtype=np.float64)
    dx = (geom.x_max - geom.x_min) / geom.nx
    kz = geom.nz // 2 - 2
    for xc, peaks in ((-10.0, ((1.0, 1.9), (0.6, 2.7))), (10.0, ((0.8, 2.3),))):
        i0 = int(round((xc - geom.x_min) / dx)) - 2
        prof = np.zeros(geom.nq)
        for a, mu in peaks:
            prof += a * np.exp(-(geom.q - mu) ** 2 / (2.0 * sigma * sigma))
        f[kz:kz + 4, i0:i0 + 4, :] += prof[None, None, :]
    return f


@dataclass
class BatchScan:
    geom: ScanGeometry
    phantom_seed: int
    noise_seed: int
    n_rect: int


def batch_scans(n_scans: int = 64, seed0: int = 1000,
                sizes=(48, 64, 96, 128), nqs=(32, 64)) -> List[BatchScan]:
    """Uneven batch: scan i draws N ~ U(sizes), nq ~ U(nqs) and 3-6 rectangles
    from seed seed0+i; each scan has an N x N detector and N rows of mask."""
    out = []
    for i in range(n_scans):
        rng = np.random.Generator(np.random.PCG64(seed0 + i))
        n = int(rng.choice(sizes))
        nq = int(rng.choice(nqs))
        n_rect = int(rng.integers(3, 7))
        g = standard_geometry(n, nq, mask_seed=seed0 + i)
        out.append(BatchScan(g, seed0 + i, 50000 + seed0 + i, n_rect))
    return out


# ---- learned warm start: seeded network weights and phantom sets ------------------

WARM_CHANNELS = (64, 32, 32, 32, 64)


def cnn_init(seed: int, channels=WARM_CHANNELS, out_bias: float = 0.0) -> List[dict]:
    """Initial weights of the 3x3 network: per layer w [9][c_in][c_out] normal
    with std sqrt(2 / (9 c_in)) (He), the last layer's scaled by 0.1; biases
    zero except the last layer's (out_bias).  float32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    n = len(channels) - 1
    for k in range(n):
        ci, co = channels[k], channels[k + 1]
        std = np.sqrt(2.0 / (9.0 * ci)) * (0.1 if k == n - 1 else 1.0)
        w = rng.normal(0.0, std, size=(9, ci, co)).astype(np.float32)
        b = np.full(co, out_bias if k == n - 1 else 0.0, dtype=np.float32)
        out.append({"w": w, "b": b})
    return out


@dataclass
class WarmCase:
    phantom_seed: int
    noise_seed: int
    n_rect: int


def warm_cases(split: str, n: int) -> List[WarmCase]:
    """Phantoms of the learned warm start on the slice128 geometry: 'train'
    draws phantom seeds from 100000 up, 'eval' (held out) from 900000 up; each
    has 3 rectangles and its own noise seed."""
    base = {"train": 100000, "eval": 900000}[split]
    return [WarmCase(base + i, base + 500000 + i, 3) for i in range(n)]

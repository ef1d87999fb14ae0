"""Pins of the energy-sensitive detector model (App. A eq. energy_sensitive):
the oracle's energy-resolved forward against a dense sum of 50-digit textbook
matrix entries binned by their own Bragg energies; the sum over energy bins is
the energy-integrating forward; the adjoint is its transpose; data constant
over energy give the energy-integrating adjoint; and a lone on-axis voxel puts
each pixel's signal in the bin that Bragg's law names for the pixel's angle."""
import mpmath as mp
import numpy as np
import pytest

from paper_1603_06400_amd import inputs

from .test_oracle_factors import lone_voxel_geometry, mp_entry, tiny_geometry


def small(oracle_mod, seed=5):
    g = inputs.standard_geometry(8, 10, ndet=8)
    f = inputs.phantom(g, seed, 2)
    return g.with_(C=400.0 / oracle_mod.Oracle(g).forward(f).max()), f


def test_energy_forward_matches_textbook_dense(oracle_mod):
    """Every triple's H from textbook forms (acos angles, 1 - cos half angles,
    exact rational mask crossings) placed in the bin of its own 50-digit Bragg
    energy hc q / sin(theta/2)."""
    g = tiny_geometry(seed=11, ne=9)
    o = oracle_mod.Oracle(g)
    rng = np.random.Generator(np.random.PCG64(4))
    f = rng.uniform(0.2, 1.0, (g.nz, g.nx, g.nq))
    ref = np.zeros((g.ne, g.npix))
    de = (mp.mpf(g.e_hi) - mp.mpf(g.e_lo)) / g.ne
    for i in range(g.npix):
        for j in range(g.nvox):
            for m in range(g.nq):
                e = mp_entry(g, j, i, m)
                k = int(mp.floor((e["kappa"] * mp.mpf(g.q[m]) - mp.mpf(g.e_lo)) / de))
                if 0 <= k < g.ne:
                    ref[k, i] += float(e["H"]) * f.reshape(g.nvox, g.nq)[j, m]
                else:
                    assert e["H"] == 0
    got = o.forward_energy(f).reshape(g.ne, g.npix)
    assert np.count_nonzero(ref) > 10 and np.count_nonzero(np.sum(ref > 0, axis=0) > 1) > 0
    np.testing.assert_allclose(got, ref, rtol=1e-11, atol=1e-14 * np.abs(ref).max())


@pytest.mark.parametrize("seed", [5, 6])
def test_energy_bins_sum_to_the_integrating_forward(oracle_mod, seed):
    g, f = small(oracle_mod, seed)
    o = oracle_mod.Oracle(g)
    ge = o.forward_energy(f)
    assert ge.shape == (g.ne, g.ndy, g.ndx)
    np.testing.assert_allclose(ge.sum(axis=0), o.forward(f), rtol=1e-12, atol=0)
    # the signal is spread over many bins (not a bin shift of the integrating g)
    assert np.count_nonzero(ge.reshape(g.ne, -1).sum(axis=1)) > g.ne // 2


def test_energy_adjoint_identity(oracle_mod):
    g, _ = small(oracle_mod)
    o = oracle_mod.Oracle(g)
    rng = np.random.Generator(np.random.PCG64(12))
    f = rng.uniform(0, 1, (g.nz, g.nx, g.nq))
    y = rng.uniform(0, 1, (g.ne, g.ndy, g.ndx))
    lhs = np.sum(o.forward_energy(f) * y)
    rhs = np.sum(f * o.adjoint_energy(y))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_energy_constant_data_gives_the_integrating_adjoint(oracle_mod):
    g, _ = small(oracle_mod)
    o = oracle_mod.Oracle(g)
    y = np.random.Generator(np.random.PCG64(13)).uniform(0, 1, (g.ndy, g.ndx))
    np.testing.assert_allclose(o.adjoint_energy(np.broadcast_to(y, (g.ne,) + y.shape)), o.adjoint(y),
                               rtol=1e-12, atol=0)


def test_lone_voxel_energy_follows_bragg(oracle_mod):
    """A voxel on the central ray, all-open mask, one q node: pixel (a, b) at
    radius rho sees angle atan(rho / d), hence Bragg energy hc q / sin(theta/2),
    and all of its (energy-integrated) signal sits in that energy's bin."""
    g = lone_voxel_geometry(nq=3, ne=8, e_lo=20.0, e_hi=160.0, phi=np.linspace(1.0, 2.0, 8))
    o = oracle_mod.Oracle(g)
    d = g.det_z - 500.0
    de = (g.e_hi - g.e_lo) / g.ne
    for m in range(g.nq):
        f = np.zeros((1, 1, g.nq))
        f[0, 0, m] = 1.0
        ge, gi = o.forward_energy(f), o.forward(f)
        hit = set()
        for b in range(g.ndy):
            for a in range(g.ndx):
                rho = np.hypot((a - g.ndx / 2 + 0.5) * g.det_pitch, (b - g.ndy / 2 + 0.5) * g.det_pitch)
                E = g.hc * g.q[m] / np.sin(0.5 * np.arctan(rho / d))
                k = int(np.floor((E - g.e_lo) / de))
                col = ge[:, b, a]
                if 0 <= k < g.ne:
                    assert col[k] == pytest.approx(gi[b, a], rel=1e-13) and gi[b, a] > 0
                    assert np.count_nonzero(col) == 1
                    hit.add(k)
                else:
                    assert np.all(col == 0)
        assert len(hit) >= 2

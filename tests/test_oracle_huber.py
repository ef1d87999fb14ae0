"""Pins of the edge-preserving penalty (Sec. V eq. standard_EPR with Huber's
potential) and of its separable surrogate (App. B): the paper's pairwise
surrogate built term by term has the gradient that b^(3)..b^(6) give, it
majorises R and touches it at the expansion point; Huber with a scale above
every difference is the quadratic penalty; Alg. 5 stays monotone."""
import numpy as np
import pytest

from paper_1603_06400_amd import inputs


def pairwise_surrogate(oracle_mod, f, fhat, psi):
    """R~(f) of App. B written term by term: for every ordered neighbour pair
    (j, k), 0.5 [psi^(2 f_j - fh_j - fh_k) + psi^(2 f_k - fh_j - fh_k)] with
    psi^ the quadratic surrogate of psi at xh = fh_j - fh_k,
    psi^(x) = psi(xh) + psi'(xh)(x - xh) + omega(xh)(x - xh)^2 / 2."""
    p, dp, om = oracle_mod.potential(psi)
    nz, nx = f.shape[0], f.shape[1]
    tot = 0.0
    for iz in range(nz):
        for ix in range(nx):
            for dz, dx in ((0, -1), (0, 1), (-1, 0), (1, 0)):
                kz, kx = iz + dz, ix + dx
                if not (0 <= kz < nz and 0 <= kx < nx):
                    continue
                xh = fhat[iz, ix] - fhat[kz, kx]
                for x in (2 * f[iz, ix] - fhat[iz, ix] - fhat[kz, kx], 2 * f[kz, kx] - fhat[iz, ix] - fhat[kz, kx]):
                    tot += 0.5 * (p(xh) + dp(xh) * (x - xh) + 0.5 * om(xh) * (x - xh) ** 2)
    return float(np.sum(tot))


def rnd(shape, seed, lo, hi):
    return np.random.Generator(np.random.PCG64(seed)).uniform(lo, hi, size=shape)


@pytest.mark.parametrize("psi", [None, ("huber", 0.3), ("huber", 0.05)])
def test_separable_coefficients_are_the_pairwise_surrogate_gradient(oracle_mod, psi):
    fhat = rnd((4, 5, 2), 1, 0.0, 1.0)
    b1 = rnd(fhat.shape, 2, 0.5, 1.5)
    b2 = rnd(fhat.shape, 3, 0.5, 1.5)
    beta = 1.0
    chi1, chi2, chi3 = oracle_mod.surrogate_coefficients(fhat, b1, b2, beta, psi)
    # grad of b1 f - fh b2 ln f + beta R~(f) at f: b1 - fh b2 / f + beta dR~/df
    f = rnd(fhat.shape, 4, 0.2, 1.2)
    h = 1e-6
    for idx in [(0, 0, 0), (1, 2, 1), (3, 4, 0), (2, 1, 1)]:
        e = np.zeros_like(f)
        e[idx] = h
        dR = (pairwise_surrogate(oracle_mod, f + e, fhat, psi) - pairwise_surrogate(oracle_mod, f - e, fhat, psi)) / (2 * h)
        fd = b1[idx] - fhat[idx] * b2[idx] / f[idx] + beta * dR
        # eq. grad_sep_obj: chi1 f + chi2 - chi3 / f
        an = chi1[idx] * f[idx] + chi2[idx] - chi3[idx] / f[idx]
        assert an == pytest.approx(fd, rel=1e-6, abs=1e-8)


@pytest.mark.parametrize("delta", [0.02, 0.1, 0.4])
def test_surrogate_majorises_and_touches(oracle_mod, delta):
    psi = ("huber", delta)
    fhat = rnd((5, 4, 1), 5, 0.0, 1.0)
    assert pairwise_surrogate(oracle_mod, fhat, fhat, psi) == pytest.approx(oracle_mod.penalty(fhat, psi), rel=1e-13)
    for seed in range(6):
        f = rnd(fhat.shape, 10 + seed, 0.0, 1.0)
        assert pairwise_surrogate(oracle_mod, f, fhat, psi) >= oracle_mod.penalty(f, psi) - 1e-12


def test_huber_penalty_values(oracle_mod):
    """A 1 x 2 image with difference t: R = 2 psi(t) (the pair from each side)."""
    f = np.array([[0.0, 0.7]])
    assert oracle_mod.penalty(f, ("huber", 0.2)) == pytest.approx(2 * (0.2 * 0.7 - 0.02), rel=1e-15)
    assert oracle_mod.penalty(f, ("huber", 1.0)) == pytest.approx(2 * 0.245, rel=1e-15)
    assert oracle_mod.penalty(f, None) == pytest.approx(2 * 0.245, rel=1e-15)


def test_wide_huber_is_quadratic(oracle_mod):
    fhat = rnd((4, 5, 3), 6, 0.0, 1.0)
    b1 = rnd(fhat.shape, 7, 0.5, 1.5)
    b2 = rnd(fhat.shape, 8, 0.5, 1.5)
    a = oracle_mod.em_update(fhat, b1, b2, 0.3, None)
    b = oracle_mod.em_update(fhat, b1, b2, 0.3, ("huber", 2.0))
    np.testing.assert_array_equal(a, b)
    assert oracle_mod.penalty(fhat, ("huber", 2.0)) == oracle_mod.penalty(fhat, None)


def test_alg5_with_huber_is_monotone(oracle_mod):
    g = inputs.standard_geometry(8, 6, ndet=8)
    f = inputs.phantom(g, 21, 2)
    g = g.with_(C=400.0 / oracle_mod.Oracle(g).forward(f).max())
    o = oracle_mod.Oracle(g)
    y = inputs.poisson_counts(o.forward(f), 22)
    f0 = oracle_mod.uniform_start(y, o.sensitivity())
    _, J = o.recon(y, None, f0, 8, 0.05, ("huber", 0.05))
    assert np.all(np.diff(J) <= 1e-12 * np.abs(J[1:]))
    assert J[-1] < J[0]

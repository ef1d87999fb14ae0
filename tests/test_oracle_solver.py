"""Pins of the oracle's objective and separable-surrogate update (Sec. V-VI,
Alg. 5, App. B eqs. surrogate_data_fit / quadratic_surrogate_regularizer /
f_update, App. C Lemma 1).

The references are independent of the oracle's closed forms: brute-force 1D
minimisation for Lemma 1, the surrogate J-hat written out from its definition
on a dense H and minimised numerically coordinate by coordinate, textbook
MLEM for beta = 0 and its count conservation, scipy's Poisson log-pmf for the
data term, explicit neighbour loops for R, majorisation monotonicity, and an
L-BFGS-B solution of the penalised problem.
"""
import numpy as np
import pytest
from scipy import optimize, stats

from paper_1603_06400_amd import inputs

from .test_oracle_factors import tiny_geometry


def test_lemma1_cases_against_brute_force(oracle_mod):
    rng = np.random.Generator(np.random.PCG64(11))
    for _ in range(300):
        a = rng.uniform(0, 2) * (rng.uniform() > 0.2)
        b = rng.uniform(-3, 3)
        c = rng.uniform(0, 2) * (rng.uniform() > 0.1)
        x = float(oracle_mod.lemma_minimizer(a, b, c))
        if a == 0 and b <= 0:
            assert x == np.inf
            continue
        fun = lambda t: 0.5 * a * t * t + b * t - (c * np.log(t) if c > 0 else 0.0)
        hi = 10.0 * (abs(b) + c + 1.0) / max(a, 1e-3) + 10.0
        res = optimize.minimize_scalar(fun, bounds=(1e-14, hi), method="bounded",
                                       options={"xatol": 1e-12, "maxiter": 2000})
        assert fun(x) <= fun(res.x) + 1e-9 * (1 + abs(fun(res.x)))
        assert x == pytest.approx(res.x, rel=1e-5, abs=1e-7)
        if c > 0:  # stationarity a x + b - c / x = 0
            assert a * x + b - c / x == pytest.approx(0.0, abs=1e-12 * (abs(b) + c / x + a * x))
    # the printed special cases
    assert oracle_mod.lemma_minimizer(2.0, -3.0, 0.0) == pytest.approx(1.5)
    assert oracle_mod.lemma_minimizer(2.0, 3.0, 0.0) == 0.0
    assert oracle_mod.lemma_minimizer(0.0, 4.0, 2.0) == pytest.approx(0.5)


def test_data_fit_is_poisson_negative_log_likelihood(oracle_mod):
    rng = np.random.Generator(np.random.PCG64(12))
    z = rng.uniform(0.1, 30, size=200)
    y = rng.poisson(z).astype(float)
    ref = -float(np.sum(stats.poisson.logpmf(y, z)))
    assert oracle_mod.data_fit(y, z) == pytest.approx(ref, rel=1e-13)
    assert oracle_mod.data_fit(np.array([0.0, 3.0]), np.array([0.0, 1.0])) == pytest.approx(1.0 + np.log(6.0))
    assert oracle_mod.data_fit(np.array([2.0]), np.array([0.0])) == np.inf


def test_penalty_explicit_neighbour_loops(oracle_mod):
    rng = np.random.Generator(np.random.PCG64(13))
    f = rng.uniform(size=(4, 5, 3))
    ref = 0.0
    for k in range(4):
        for i in range(5):
            for dk, di in ((0, 1), (0, -1), (1, 0), (-1, 0)):
                kk, ii = k + dk, i + di
                if 0 <= kk < 4 and 0 <= ii < 5:
                    ref += 0.5 * np.sum((f[k, i] - f[kk, ii]) ** 2)
    assert oracle_mod.penalty(f) == pytest.approx(ref, rel=1e-14)


def surrogate_value(H, y, r, fhat, beta, f):
    """J-hat(f) of App. B written out from its definition (quadratic psi, w = 1)."""
    lhat = H @ fhat.ravel()
    zhat = lhat + r
    fh = fhat.ravel()
    ff = f.ravel()
    Lh = 0.0
    for i in range(H.shape[0]):
        for j in range(H.shape[1]):
            if H[i, j] == 0:
                continue
            term = H[i, j] * ff[j]
            if y[i] > 0:
                term -= y[i] * H[i, j] * fh[j] / zhat[i] * np.log(ff[j] / fh[j] * zhat[i])
            Lh += term
    nz, nx, nq = fhat.shape
    Rh = 0.0
    for k in range(nz):
        for i in range(nx):
            for dk, di in ((0, 1), (0, -1), (1, 0), (-1, 0)):
                kk, ii = k + dk, i + di
                if 0 <= kk < nz and 0 <= ii < nx:
                    a = 2 * f[k, i] - fhat[k, i] - fhat[kk, ii]
                    b = 2 * f[kk, ii] - fhat[k, i] - fhat[kk, ii]
                    Rh += np.sum(0.5 * (0.5 * a * a + 0.5 * b * b))
    return Lh + beta * Rh


@pytest.mark.parametrize("beta", [0.0, 0.05])
def test_update_minimises_the_written_out_surrogate(oracle_mod, beta):
    g = tiny_geometry(seed=4, nx=3, nz=2, ndx=4, ndy=4, nq=3)
    o = oracle_mod.Oracle(g)
    H = o.dense()
    ftrue = inputs.random_image(g, 30, 0.2, 1.0)
    y = inputs.poisson_counts(50.0 * (H @ ftrue.ravel()) / (H @ ftrue.ravel()).max(), 31)
    r = np.full(g.npix, 0.05)
    fhat = inputs.random_image(g, 32, 0.3, 1.5)
    fnew, _ = o.recon_step(y, r, fhat, beta)
    base = fnew.copy()
    seen = np.abs(H).sum(axis=0).reshape(fnew.shape) > 0
    checked = 0
    for idx in np.ndindex(fnew.shape):
        if beta == 0.0 and not seen[idx]:
            # J-hat does not depend on a voxel no pixel sees; the update keeps it
            assert fnew[idx] == fhat[idx]
            continue
        checked += 1
        def one(t):
            f = base.copy()
            f[idx] = t
            return surrogate_value(H, y, r, fhat, beta, f)
        x = fnew[idx]
        h = 1e-4 * max(x, 1e-6)
        # separable: J-hat along one coordinate is minimised at the update
        assert one(x) <= one(x + h) + 1e-13 and one(x) <= one(max(x - h, 1e-12)) + 1e-13
        res = optimize.minimize_scalar(one, bounds=(1e-10, 20 * (x + 1)), method="bounded",
                                       options={"xatol": 1e-11})
        assert x == pytest.approx(res.x, rel=1e-5, abs=1e-8)
    assert checked >= fnew.size // 2


def test_beta_zero_is_mlem_and_conserves_counts(oracle_mod):
    g = inputs.standard_geometry(10, 6, ndet=12)
    o = oracle_mod.Oracle(g)
    ftrue = inputs.phantom(g, 5)
    y = inputs.poisson_counts(1e3 * o.forward(ftrue) / o.forward(ftrue).max(), 6)
    b1 = o.sensitivity()
    f = oracle_mod.uniform_start(y, b1)
    for _ in range(3):
        z = o.forward(f)
        b2 = o.adjoint(oracle_mod.poisson_ratio(y, z))
        fnew = oracle_mod.em_update(f, b1, b2, 0.0)
        mlem = np.where(b1 > 0, f * b2 / np.where(b1 > 0, b1, 1.0), f)
        np.testing.assert_allclose(fnew, mlem, rtol=1e-13)
        seen = z > 0
        assert np.sum(o.forward(fnew)) == pytest.approx(np.sum(y[seen]), rel=1e-12)
        f = fnew


@pytest.mark.parametrize("beta", [0.0, 1e-3, 1e-1])
def test_objective_is_monotone_along_alg5(oracle_mod, beta):
    w = inputs.workload("slice32")
    g = w.geom.with_(C=1.0)
    o = oracle_mod.Oracle(g)
    ftrue = inputs.phantom(g, w.phantom_seed)
    l1 = o.forward(ftrue)
    g = g.with_(C=1e4 / l1.max())
    o = oracle_mod.Oracle(g)
    y = inputs.poisson_counts(o.forward(ftrue), w.noise_seed)
    f0 = oracle_mod.uniform_start(y, o.sensitivity())
    _, J = o.recon(y, None, f0, 8, beta)
    assert np.all(np.diff(J) <= 1e-12 * np.abs(J[1:]))
    assert J[-1] < J[0]


def test_noise_free_data_fit_approaches_its_floor(oracle_mod):
    g = inputs.standard_geometry(8, 6, ndet=10)
    o = oracle_mod.Oracle(g)
    ftrue = inputs.phantom(g, 9) + 0.1
    y = o.forward(ftrue)
    y = 100.0 * y / y.max()
    floor = float(np.sum(y - y * np.log(np.where(y > 0, y, 1)) + np.where(y > 0, 0, 0)))
    from scipy.special import gammaln
    floor += float(np.sum(gammaln(y + 1)))
    f0 = oracle_mod.uniform_start(y, o.sensitivity())
    _, J = o.recon(y, None, f0, 30, 0.0)
    assert np.all(J >= floor - 1e-9 * abs(floor))
    assert np.all(np.diff(J) <= 1e-12 * np.abs(J[1:]))
    assert (J[-1] - floor) < 0.2 * (J[0] - floor)


def test_converged_solution_matches_lbfgsb(oracle_mod):
    """Tiny strictly convex problem: Alg. 5 iterates approach the L-BFGS-B
    minimiser of J = L + beta R over f >= 0."""
    g = tiny_geometry(seed=6, nx=2, nz=2, ndx=6, ndy=6, nq=2, ne=3)
    o = oracle_mod.Oracle(g)
    H = o.dense()
    ftrue = inputs.random_image(g, 40, 0.3, 1.0)
    mean = H @ ftrue.ravel()
    y = inputs.poisson_counts(200.0 * mean / mean.max(), 41)
    H = H * (200.0 / mean.max())
    g2 = g.with_(C=g.C * 200.0 / mean.max())
    o = oracle_mod.Oracle(g2)
    beta = 5.0

    def J(v):
        z = H @ v
        return oracle_mod.data_fit(y, z) + beta * oracle_mod.penalty(v.reshape(ftrue.shape))

    def grad(v):
        z = H @ v
        gL = H.T @ (1 - oracle_mod.poisson_ratio(y, z))
        d, _ = oracle_mod.neighbour_diffs(v.reshape(ftrue.shape))
        gR = 2 * d.sum(axis=0)
        return gL + beta * gR.ravel()

    x0 = np.full(ftrue.size, 0.5)
    res = optimize.minimize(J, x0, jac=grad, method="L-BFGS-B", bounds=[(1e-12, None)] * x0.size,
                            options={"ftol": 1e-15, "gtol": 1e-12, "maxiter": 5000})
    f0 = oracle_mod.uniform_start(y, o.sensitivity())
    f, hist = o.recon(y.reshape(g.ndy, g.ndx), None, f0, 3000, beta)
    assert hist[-1] >= res.fun - 1e-8 * abs(res.fun)
    assert hist[-1] - res.fun < 1e-6 * abs(res.fun)
    np.testing.assert_allclose(f.ravel(), res.x, rtol=2e-2, atol=1e-3)

"""The seeded input generators (no method arithmetic): Poisson counts."""
import numpy as np
import pytest

from paper_1603_06400_amd import inputs


def test_poisson_counts_of_a_nonnegative_mean_are_numpys_draws():
    mean = np.random.Generator(np.random.PCG64(1)).uniform(0.0, 50.0, size=(16, 16))
    ref = np.random.Generator(np.random.PCG64(7)).poisson(mean).astype(np.float64)
    assert np.array_equal(inputs.poisson_counts(mean, 7), ref)


def test_poisson_counts_take_a_negative_rounding_residue_as_zero():
    mean = np.array([-2.1e-12, 0.0, 3.0, -1e-30])
    y = inputs.poisson_counts(mean, 3)
    assert y[0] == 0.0 and y[1] == 0.0 and y[3] == 0.0
    assert y[2] == np.random.Generator(np.random.PCG64(3)).poisson(np.array([0.0, 0.0, 3.0, 0.0]))[2]


def test_poisson_counts_reject_nan():
    with pytest.raises(ValueError):
        inputs.poisson_counts(np.array([1.0, np.nan]), 3)

"""The FP64 oracle against what the paper and mathematics fix (CPU only)."""
import numpy as np
import pytest

import oracle
from oracle_pins import pin_covariance, pin_eigh, pin_first, pin_fourier, pin_fresnel, pin_project
from paper_2004_00923_amd.synth import gen_stack


def test_pin_fresnel():
    assert pin_fresnel(oracle) == []


def test_pin_covariance_random():
    assert pin_covariance(oracle) == []


def test_pin_eigh_random():
    assert pin_eigh(oracle) == []


def test_pin_project_random():
    assert pin_project(oracle) == []


def test_pin_fourier():
    assert pin_fourier(oracle) == []


def test_pin_projection_first():
    assert pin_first(oracle) == []


@pytest.fixture(scope="module")
def small_stack():
    # the 32 x 128 x 128 synthetic stack of the small configuration
    return gen_stack(0, 32, 128, 128)


def test_pin_covariance_synthetic(small_stack):
    assert pin_covariance(oracle, small_stack) == []


def test_pin_eigh_synthetic(small_stack):
    assert pin_eigh(oracle, small_stack) == []


def test_pin_project_synthetic(small_stack):
    # kept range of the configuration: components 2..31 (descending order)
    assert pin_project(oracle, small_stack, 2, 31) == []


def test_paper_selector_mapping():
    # The paper keeps eigen-indices n1..n2 = 1..20 of 32, 1-based, counted in
    # increasing eigenvalue order; on the descending 0-based axis that is 12..31.
    nt, n1, n2 = 32, 1, 20
    asc = np.arange(nt)                 # ascending positions (0-based)
    kept_asc = asc[n1 - 1:n2]
    kept_desc = sorted(nt - 1 - kept_asc)
    assert kept_desc == list(range(12, 32))

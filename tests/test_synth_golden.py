"""Seeded input generator and the stored oracle values of the small configuration."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2004_00923_amd.synth import StackSource, batch_spec, gen_stack, radii, sha256

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_small_seed0.json")


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def small():
    return gen_stack(0, 32, 128, 128)


def test_generator_deterministic(small):
    assert np.array_equal(small, gen_stack(0, 32, 128, 128))
    assert not np.array_equal(small, gen_stack(1, 32, 128, 128))


def test_generator_stream_consistency():
    # frames drawn one at a time continue the same random stream as a stack
    src = StackSource(3, 64, 64)
    a = np.stack([src.next_frame() for _ in range(5)])
    assert np.array_equal(a, gen_stack(3, 5, 64, 64))


def test_generator_sha_pinned(small, golden):
    assert sha256(small) == golden["stack_sha256"]


def test_generator_range(small):
    # 12-bit scale, mean near 2048 (unit reference intensity), no clipping
    assert small.dtype == np.uint16
    assert 0 < small.min() and small.max() < 4095
    assert abs(small.mean() - 2048) < 20


def test_pca_image_reveals_flow(small):
    # Dropping the clutter components (the large-eigenvalue modes of the static
    # tissue and its global phase drift) leaves an image dominated by the flow
    # disk of the synthetic object: the contrast the method is built for.
    ny = nx = 128
    R, Rf = radii(ny, nx)
    assert (R, Rf) == (40.0, 12.0)
    r = oracle.pipeline_ref(small, 785e-9, 0.3, 20e-6, 3, 31)
    M = r["image"]
    yy, xx = np.mgrid[0:ny, 0:nx]
    flow = (yy - 64) ** 2 + (xx - 84) ** 2 <= (Rf - 2) ** 2
    disk = (yy - 64) ** 2 + (xx - 64) ** 2 <= (R - 3) ** 2
    rest = disk & ~((yy - 64) ** 2 + (xx - 84) ** 2 <= (Rf + 3) ** 2)
    assert M[flow].mean() > 4 * M[rest].mean()
    assert batch_spec(0) == (16, 512, 512) and batch_spec(2) == (64, 1024, 2048)


def test_golden_oracle_values(small, golden):
    r = oracle.pipeline_ref(small, 785e-9, 0.3, 20e-6, 2, 31)
    ev = np.array(golden["evals"])
    assert np.abs(r["evals"] - ev).max() <= 1e-12 * ev[0]
    assert abs(r["image"].sum() - golden["image_sum"]) <= 1e-11 * golden["image_sum"]
    for y, x, v in golden["image_samples"]:
        assert abs(r["image"][y, x] - v) <= 1e-9 * abs(v)
    for t, y, x, re, im in golden["holo_samples"]:
        assert abs(r["holo"][t, y, x] - complex(re, im)) <= 1e-9 * abs(complex(re, im))

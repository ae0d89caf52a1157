"""Parity on seeded random rings (tests/_rings.py): other circumferences,
harmonics, species and energies, above and below transition, synchrotron
tunes from 5e-4 to 5e-2, against the oracle for every scheme with the same
per-particle bounds and moment tolerance as the SPS-like ring
(tests/test_gpu_parity.py), on ragged bunch sizes."""
import numpy as np
import pytest

from tests._rings import matched_bunch, random_ring
from tests.test_gpu_parity import INTEGS, check_against_oracle, run_f64

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RING_SEEDS = list(range(12))


@pytest.fixture(scope="module")
def ltrk():
    import paper_1610_05801_amd as m
    m.ltrk_set_plan()
    yield m


@pytest.mark.parametrize("seed", RING_SEEDS)
def test_random_ring_against_oracle(ltrk, seed):
    ring = random_ring(seed)
    n = int(np.random.default_rng(9000 + seed).integers(1, 6000))
    z0, dp0 = matched_bunch(ring, n, seed)
    for integ in INTEGS:
        out = run_f64(ltrk, z0, dp0, 1000, integ, ring=ring)
        check_against_oracle(*out, z0, dp0, 1000, integ, ring=ring, label="ring %d" % seed)

"""Roofline probes on the GPU: every kind returns a finite positive rate, and the
streaming probes stay within the HBM peak (8 TB/s)."""
import math

import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind,nbytes", [(0, 0), (1, 0), (2, 0), (3, 1 << 28), (4, 0), (5, 0), (6, 1 << 28)])
def test_probe_rates(kind, nbytes):
    from paper_2204_13241_amd import api
    print("probe kind %d" % kind, flush=True)
    r = api.roofline_probe(kind, nbytes)
    assert math.isfinite(r) and r > 0
    if kind in (3, 6):
        assert r < 8.0e12

"""The allocation-free density-of-states entry point (cg_dos_noalloc, counts in the library's
file-scope device array) against cg_dos (counts in the arena) through the C ABI: equal counts
on two calls in a row, the second over fewer samples and fewer bins, so that the array keeps
the first call's larger contents where the second call's slots end."""
import numpy as np
import pytest

from tests.gpu_util import require_gpu, say
from workloads import Sample

pytestmark = pytest.mark.gpu


def _same(a, b):
    return all(np.array_equal(x, y) if isinstance(x, np.ndarray) else x == y for x, y in zip(a, b))


@pytest.mark.parametrize("precision", [0, 1])
def test_dos_noalloc_equals_dos(precision):
    cg = require_gpu()
    samples = [Sample(48, 1152, 1.0, 1.0, 6.0, 0.08, 0.008, 21, b) for b in range(3)]
    b = cg.Batch(samples, cg.make_opts(precision=precision, K_refresh=1024))
    b.run_hops(2500)
    calls = ((0, 3, -2.0, 2.0, 4096), (1, 1, -0.7, 0.9, 33))
    for first, count, lo, hi, nb in calls:
        ref = b.dos(first, count, lo, hi, nb)
        got = b.dos_noalloc(first, count, lo, hi, nb)
        assert _same(got, ref), (first, count, nb)
        n = 48 * 48 * count
        assert int(got[0].sum() + got[1].sum()) + got[2] + got[3] == n
    # the arena's call after the allocation-free one still gives the same counts
    assert _same(b.dos(0, 2, -1.0, 1.0, 100), b.dos_noalloc(0, 2, -1.0, 1.0, 100))
    with pytest.raises(cg.CgError):
        b.dos_noalloc(0, 1, -1.0, 1.0, 4097)
    b.close()
    say(f"cg_dos_noalloc equals cg_dos (precision {precision})")

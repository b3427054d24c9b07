"""gdc_philox_normals_noalloc, the entry point that allocates no device
memory (it stages through the library's fixed per-GPU array), against the
allocating gdc_philox_normals, through the C ABI: bit-identical normals on
two calls in a row (the second smaller, so values left in the staging array
by the first must not leak into it), at the staging limit, and a count above
the limit rejected with GDC_EINVAL.  A second handle on the same GPU shares
the array and gets the same normals."""
import sys

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def test_noalloc_normals_equal_the_allocating_entry_point():
    import paper_2106_00449_amd as g
    w = wl.small_case(n=8, L=8.0)
    s = g.Suspension(**wl.library_kwargs(w))
    t = g.Suspension(**wl.library_kwargs(w, seed=99))
    cases = [(12345, 3, 7, 1000, 50000), (2**40 + 5, 17, 2**33 + 1, 31, 777), (0, 0, 0, 0, 65536), (9, 1, 2, 5, 1)]
    for seed, c1, step, c0, count in cases:
        _say("noalloc normals", seed, c1, step, c0, count)
        ref = s.philox_normals(seed, c1, step, c0, count)
        got = s.philox_normals_noalloc(seed, c1, step, c0, count)
        assert got.shape == (count, 4) and np.array_equal(got, ref)
        other = t.philox_normals_noalloc(seed, c1, step, c0, count)
        assert np.array_equal(other, ref)
    _say("noalloc normals over the limit")
    with pytest.raises(g.GdcError) as e:
        s.philox_normals_noalloc(1, 0, 0, 0, 65537)
    assert e.value.code == g.GDC_EINVAL
    assert np.array_equal(s.philox_normals_noalloc(1, 0, 0, 0, 0), np.empty((0, 4)))
    s.close()
    t.close()

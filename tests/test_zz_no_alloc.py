"""kpx_philox_static, the allocation-free form of kpx_philox, against
kpx_philox itself: bit-identical words on two calls in a row, the second one
smaller (the static buffer keeps the first call's contents), plus the size
limit and the empty call."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kpx():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_02846_amd as K

    K.lib()
    torch.cuda.set_device(0)
    return K


def _records(rng, n):
    return rng.integers(0, 1 << 32, size=(n, 6), dtype=np.uint64).astype(np.uint32)


def test_static_philox_matches_the_allocating_call(kpx):
    rng = np.random.default_rng(2602)
    for n in (kpx.PHILOX_STATIC_MAX, 50_000, 1_000):
        ck = _records(rng, n)
        got = kpx.philox_static(ck)
        ref = kpx.philox(ck)
        assert got.shape == (n, 4)
        np.testing.assert_array_equal(got, ref, err_msg=f"{n} records")


def test_static_philox_limits(kpx):
    assert kpx.philox_static(np.zeros((0, 6), np.uint32)).shape == (0, 4)
    with pytest.raises(kpx.KPXError) as e:
        kpx.philox_static(np.zeros((kpx.PHILOX_STATIC_MAX + 1, 6), np.uint32))
    assert e.value.code == kpx.ERR_ARG
    # the buffer is still usable after a refused call
    ck = _records(np.random.default_rng(7), 33)
    np.testing.assert_array_equal(kpx.philox_static(ck), kpx.philox(ck))

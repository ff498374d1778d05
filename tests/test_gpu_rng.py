"""Device Philox4x32-10 against the reference generator and the published
known answers."""
import numpy as np
import pytest

from philox_ref import philox4
from test_oracle_rng import _kats

pytestmark = pytest.mark.gpu


def test_device_philox_known_answers_and_random():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_08195_amd import dsmc
    for ctr, key, exp in _kats():
        assert dsmc.philox([ctr], key)[0].tolist() == exp
    rng = np.random.default_rng(9)
    ctr = rng.integers(0, 2**32, size=(2000, 4), dtype=np.uint64).astype(np.uint32)
    key = [0x12345678, 0x9abcdef0]
    out = dsmc.philox(ctr, key)
    for i in range(0, 2000, 37):
        assert out[i].tolist() == philox4(ctr[i].tolist(), key)

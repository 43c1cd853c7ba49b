"""The host BF16 rounding used by the BF16-GEMM tests: round to nearest,
ties to even, against hand-worked bit patterns and torch's conversion."""

import numpy as np
import pytest

from bf16util import bf16_rne


def _f(bits):
    return np.array([bits], dtype=np.uint32).view(np.float32)


@pytest.mark.parametrize("bits,expect", [
    (0x3F800000, 0x3F800000),  # 1.0 exact
    (0x3F808000, 0x3F800000),  # halfway, even below: stays
    (0x3F818000, 0x3F820000),  # halfway, odd below: rounds up to even
    (0x3F807FFF, 0x3F800000),  # just below halfway
    (0x3F808001, 0x3F810000),  # just above halfway
    (0xBF818000, 0xBF820000),  # sign does not matter
    (0x7F7FFFFF, 0x7F800000),  # the largest float rounds to infinity
    (0x00008000, 0x00000000),  # subnormal halfway to zero, even
])
def test_bit_patterns(bits, expect):
    got = bf16_rne(_f(bits)).view(np.uint32)[0]
    assert got == expect, (hex(bits), hex(got), hex(expect))


def test_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.standard_normal(20000), rng.uniform(-1e30, 1e30, 2000),
                        rng.uniform(-1e-30, 1e-30, 2000)]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(bf16_rne(x).view(np.uint32), ref.view(np.uint32))

"""Host check of the window kernel's run-to-row arithmetic.

The molecule window kernel finds the row of output run j (VEC consecutive x
values) as floor(j / CW), CW = W / VEC runs per row, from the float estimate
(j + 1/2) * fl(1 / CW) corrected by one integer comparison on each side.
This replays that float32 arithmetic in numpy (IEEE round-to-nearest-even,
as the device evaluates it) over every run of planes the validation admits,
including the plane where the uncorrected estimate lands on the next row.
"""
import numpy as np
import pytest


def rows(j: np.ndarray, cw: int) -> np.ndarray:
    inv = np.float32(1.0) / np.float32(cw)
    yy = ((j.astype(np.float32) + np.float32(0.5)) * inv).astype(np.float32).astype(np.int64)
    yy = yy - (yy * cw > j)
    return yy + ((yy + 1) * cw <= j)


def test_uncorrected_estimate_misses_rows_of_this_plane():
    """The estimate alone is off by one for 187 runs of a 3296 x 1783 plane
    (one-element runs): the reason for the correction."""
    H, W = 3296, 1783
    j = np.arange(H * W, dtype=np.int64)
    inv = np.float32(1.0) / np.float32(W)
    est = ((j.astype(np.float32) + np.float32(0.5)) * inv).astype(np.float32).astype(np.int64)
    assert int(np.sum(est != j // W)) == 187
    assert np.array_equal(rows(j, W), j // W)


@pytest.mark.parametrize("H,W,vec", [(3296, 1783, 1), (32767, 32767, 1), (32767, 32764, 4),
                                     (20000, 16384, 8), (1, 1, 1), (7, 30000, 2)])
def test_corrected_row_exact(H, W, vec):
    cw = W // vec
    n = H * cw
    # every run of the plane when small, else its first and last million
    # runs and a million spread over it
    if n <= 3_000_000:
        j = np.arange(n, dtype=np.int64)
    else:
        rng = np.random.default_rng(H * 7 + W)
        j = np.concatenate([np.arange(1_000_000), np.arange(n - 1_000_000, n),
                            rng.integers(0, n, 1_000_000)]).astype(np.int64)
    assert np.array_equal(rows(j, cw), j // cw)


def test_corrected_row_exact_random_planes():
    rng = np.random.default_rng(5)
    for _ in range(200):
        W = int(rng.integers(1, 32768))
        vec = int(rng.choice([1, 2, 4, 8]))
        if W % vec:
            vec = 1
        cw = W // vec
        H = int(rng.integers(1, min(32767, (2**31 - 1) // W) + 1))
        n = H * cw
        j = np.unique(np.concatenate([rng.integers(0, n, 20000), np.arange(max(0, n - 5000), n),
                                      np.arange(min(n, 5000))])).astype(np.int64)
        assert np.array_equal(rows(j, cw), j // cw), (H, W, vec)

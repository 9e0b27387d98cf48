"""Host checks of the index arithmetic the PSD units of the loop kernels do in FP32 instead of
integer division (the kernels themselves run on the GPU only): the quotient e / kp from an
FP32 reciprocal, exact for every staged entry e < 8192 and padded order kp in {16, 32, 48,
64}; and the svec row -> (row, column) inverse from an FP32 square root with a correction
by one either way, exact for every row of every order up to 64 even when the square root is
off by a few units in the last place. Both are checked against plain integer arithmetic."""
import numpy as np
import pytest


def quot_kp(e, kp):
    rkp = np.float32(1.0) / np.float32(kp)
    return int((np.float32(e) + np.float32(0.5)) * rkp)


@pytest.mark.parametrize("kp", [16, 32, 48, 64])
def test_fp32_quotient_is_exact(kp):
    e = np.arange(8192, dtype=np.int64)
    rkp = np.float32(1.0) / np.float32(kp)
    q = ((e.astype(np.float32) + np.float32(0.5)) * rkp).astype(np.int64)
    assert np.array_equal(q, e // kp)
    assert quot_kp(kp * kp - 1, kp) == kp - 1


def svec_rc(i, k, ulps=0):
    b = 2 * k + 1
    r = np.sqrt(np.float32(b * b - 8 * i))
    for _ in range(abs(ulps)):
        r = np.nextafter(r, np.float32(np.inf if ulps > 0 else 0), dtype=np.float32)
    j = int((np.float32(b) - r) * np.float32(0.5))
    j = max(0, min(j, k - 1))
    if j * (b - j) // 2 > i:
        j -= 1
    elif (j + 1) * (b - j - 1) // 2 <= i:
        j += 1
    return j + (i - j * (b - j) // 2), j


@pytest.mark.parametrize("ulps", [0, -3, 3])
def test_svec_inverse_is_exact(ulps):
    for k in range(1, 65):
        i = 0
        for jj in range(k):          # svec order: column jj holds rows jj .. k-1
            for ii in range(jj, k):
                assert svec_rc(i, k, ulps) == (ii, jj), (k, i, ulps)
                i += 1

"""Host-side checks of two identities the LDS-staged gathers rely on (no GPU).

1. Exact small-integer division by one float product: for 0 <= a < 2^14 and
   1 <= b <= 4096, trunc(a * fl((1 + 2^-16) / b)) == a // b in IEEE single
   precision (round-to-nearest product, truncating conversion), so the
   staging loop needs no remainder correction.
2. Bank layout of the staged box: with the plane pitch pp = e2 p3 padded to
   pp = 16 (mod 64), four 16-lane groups reading contiguous runs at plane
   offsets 0, pp, 2 pp, 3 pp touch disjoint banks, both for 32 banks served
   per half wave and for 64 banks served per wave.
"""
import numpy as np
import pytest


def test_biased_reciprocal_division_is_exact():
    a = np.arange(0, 1 << 14, dtype=np.int64)
    af = a.astype(np.float32)
    one = np.float32(1.0) + np.float32(2.0 ** -16)
    for b in range(1, 4097):
        inv = np.float32(one / np.float32(b))
        q = np.trunc((af * inv).astype(np.float32)).astype(np.int64)
        assert np.array_equal(q, a // b), b
    # the bias is needed: the plain reciprocal fails somewhere in this range
    b = 41
    q = np.trunc((af * np.float32(np.float32(1.0) / np.float32(b))).astype(np.float32))
    assert not np.array_equal(q.astype(np.int64), a // b)


def plane_pitch(e2, p3):
    plane = e2 * p3
    return plane + ((16 - plane) & 63)


@pytest.mark.parametrize("e2", range(4, 40))
@pytest.mark.parametrize("p3", range(4, 68, 4))
def test_plane_pitch_gives_disjoint_banks(e2, p3):
    pp = plane_pitch(e2, p3)
    assert pp % 64 == 16 and pp >= e2 * p3 and pp - e2 * p3 < 64
    for start in range(0, 64):          # any row/column base of the wave
        addr = np.array([start + g * pp + l for g in range(4) for l in range(16)])
        # 64 banks, whole wave
        assert len(set(addr % 64)) == 64
        # 32 banks, each half wave
        for h in range(2):
            assert len(set(addr[32 * h:32 * h + 32] % 32)) == 32

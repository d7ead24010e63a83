"""Model of the per-pixel fixed-size sorter (Stage 3, "Sample blending": a
depth filter that is a fixed-size priority queue; one more slot detects bad
order) as the raster kernel runs it, checked on the CPU.

The kernel keeps K 32-bit order codes sorted ascending, pre-filled with
placeholder code 0 (smaller than any real code), and on every arrival emits
the smallest of queue + arrival.  A pixel is flagged when an emitted real
code is not strictly greater than the previous emitted code.  Claims:
  * unflagged  =>  the emitted real codes are all codes, sorted (exact);
  * flagged   <=>  the emitted sequence is not strictly increasing;
  * K >= fragment count and distinct codes => never flagged.
"""
import numpy as np
import pytest


def run_queue(codes, K):
    q = [0] * K
    last = 0
    flagged = False
    emitted = []

    def emit(pk):
        nonlocal last, flagged
        if (pk - 1) % (1 << 32) < last:
            flagged = True
        last = pk
        if pk != 0:
            emitted.append(pk)

    for x in codes:
        lt = [x < q[j] for j in range(K)]
        pk = x if lt[0] else q[0]
        nq = list(q)
        for j in range(K - 1):
            nq[j] = (q[j] if lt[j] else x) if lt[j + 1] else q[j + 1]
        nq[K - 1] = q[K - 1] if lt[K - 1] else x
        q = nq
        emit(pk)
    for j in range(K):
        emit(q[j])
    return emitted, flagged


def near_sorted(rng, n, disp, ties=False):
    base = np.sort(rng.choice(np.arange(0x80800000, 0x80900000), n, replace=False)).astype(np.int64)
    if ties and n > 2:
        k = int(rng.integers(1, n))
        base[k] = base[k - 1]
    noisy = np.arange(n) + rng.uniform(-disp, disp, n)
    return [int(c) for c in base[np.argsort(noisy, kind="stable")]]


@pytest.mark.parametrize("K", [1, 2, 3, 4, 8, 16])
def test_unflagged_pixels_are_exactly_sorted(K):
    rng = np.random.default_rng(K)
    seen_flag = seen_clean = 0
    for trial in range(400):
        n = int(rng.integers(0, 60))
        codes = near_sorted(rng, n, disp=float(rng.uniform(0, 6)))
        emitted, flagged = run_queue(codes, K)
        assert sorted(emitted) == sorted(codes)
        strictly = all(b > a for a, b in zip(emitted, emitted[1:]))
        assert flagged == (not strictly)
        if not flagged:
            assert emitted == sorted(codes)
            seen_clean += 1
        else:
            seen_flag += 1
    assert seen_clean > 0
    if K <= 4:
        assert seen_flag > 0


def test_deep_enough_queue_never_flags():
    rng = np.random.default_rng(9)
    for _ in range(200):
        n = int(rng.integers(1, 24))
        codes = [int(c) for c in rng.permutation(np.arange(0x80800000, 0x80800000 + n))]
        emitted, flagged = run_queue(codes, 32)
        assert not flagged and emitted == sorted(codes)


def test_equal_codes_always_flag():
    rng = np.random.default_rng(10)
    for _ in range(200):
        n = int(rng.integers(3, 30))
        codes = near_sorted(rng, n, disp=0.0, ties=True)
        _, flagged = run_queue(codes, 32)
        assert flagged

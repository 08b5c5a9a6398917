"""Pins for the oracle's RNG: Philox4x64-10 against NumPy's independent
implementation, the stream layout, and Lemire's bounded integers against
exact big-integer arithmetic (exact uniformity at every value boundary)."""
import numpy as np
import pytest

MASK = (1 << 64) - 1


def numpy_block(counter, key):
    """Philox4x64-10 block via numpy.random.Philox.  NumPy increments its
    256-bit counter before producing a block, so start one below."""
    c = 0
    for w, x in enumerate(counter):
        c |= int(x) << (64 * w)
    c = (c - 1) % (1 << 256)
    prev = np.array([(c >> (64 * w)) & MASK for w in range(4)], dtype=np.uint64)
    g = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=prev)
    return [int(v) for v in g.random_raw(4)]


CASES = [
    ((0, 0, 0, 0), (0, 0)),
    ((1, 0, 0, 0), (0, 0)),
    ((0, 0, 0, 0), (12345, 678)),
    ((5, 1, 2, 3), (12345, 678)),
    ((MASK, MASK, MASK, MASK), (MASK, MASK)),
    ((123456789, MASK, 0, 0), (250603071, 0)),
    ((1 << 20, 7, 1, 2), (250603071, 511)),
    ((0xDEADBEEF, 0, 15, 1), (0x0123456789ABCDEF, 0xFEDCBA9876543210)),
]


@pytest.mark.parametrize("ctr,key", CASES)
def test_philox_matches_numpy(orc, ctr, key):
    got = [int(v) for v in orc.philox4x64_10(ctr, key)]
    assert got == numpy_block(ctr, key)


def test_philox_random_counters(orc):
    rng = np.random.default_rng(7)
    for _ in range(200):
        ctr = [int(v) for v in rng.integers(0, 2**63, size=4, dtype=np.int64)]
        key = [int(v) for v in rng.integers(0, 2**63, size=2, dtype=np.int64)]
        assert [int(v) for v in orc.philox4x64_10(ctr, key)] == numpy_block(ctr, key)


def test_stream_layout(orc):
    seed, stream = 250603071, 3
    for i in (0, 1, 999, 2**20 + 5):
        for r in (0, 1, 2):
            for j in range(12):
                for k in (0, 1):
                    blk = numpy_block((i, r, j // 4, k), (seed, stream))
                    assert orc.word(seed, stream, i, r, j, k) == blk[j % 4]
        assert orc.sign_word(seed, stream, i) == numpy_block((i, MASK, 0, 0), (seed, stream))[0]


def lemire_reference(w, d):
    """Lemire (2019), written with Python integers."""
    prod = w * d
    low = prod & MASK
    t = ((1 << 64) - d) % d
    return None if low < t else prod >> 64


@pytest.mark.parametrize("d", [1, 2, 3, 5, 7, 400, 1000, 4000, 8192, 2**31 - 1])
def test_lemire_boundaries_exact(orc, d):
    """At every value boundary the C step agrees with big-integer arithmetic,
    and each value in [0,d) owns exactly floor(2^64/d) accepted words."""
    t = ((1 << 64) - d) % d
    values = range(d) if d <= 1000 else list(range(50)) + list(range(d - 50, d))
    per_value = (1 << 64) // d
    for v in values:
        lo = -((-(v << 64)) // d)           # ceil(v 2^64 / d): first word mapping to v
        hi = -((-((v + 1) << 64)) // d) - 1  # last word mapping to v
        hi = min(hi, MASK)
        # count of words in [lo, hi] whose low product half is >= t
        # low(w) = w*d - v*2^64 grows by d per word from low(lo)
        low_lo = lo * d - (v << 64)
        rejected = 0 if low_lo >= t else -((-(t - low_lo)) // d)
        assert (hi - lo + 1) - rejected == per_value
        for w in {lo, min(lo + 1, hi), hi, max(lo, hi - 1), min(hi, lo + rejected), max(lo, lo + rejected - 1)}:
            ref = lemire_reference(w, d)
            got = orc.lemire_step(w, d)
            assert got == ref, (d, v, w)
            if ref is not None:
                assert ref == v


def test_lemire_random_words(orc):
    rng = np.random.default_rng(11)
    for d in (3, 400, 4000, 8192, 65537, 2**31 - 1):
        for w in rng.integers(0, 2**63, size=500, dtype=np.int64):
            w = int(w) * 2 + int(rng.integers(0, 2))
            assert orc.lemire_step(w, d) == lemire_reference(w, d)
        for w in (0, 1, MASK, MASK - 1, 1 << 63):
            assert orc.lemire_step(w, d) == lemire_reference(w, d)


def test_bounded_follows_words(orc):
    seed, stream = 99, 0
    for i in range(50):
        for j in range(8):
            d = 7
            w = orc.word(seed, stream, i, 0, j, 0)
            v = lemire_reference(w, d)
            if v is not None:
                assert orc.bounded(seed, stream, i, 0, j, d) == v


def test_bounded_rejection_steps_to_next_word(orc):
    """d close to 2^63 makes rejection common: U must then take w(i,r,j,k+1)."""
    d = (1 << 63) + 12345
    seed, stream = 5, 6
    hit = 0
    for i in range(200):
        w0 = orc.word(seed, stream, i, 0, 0, 0)
        if lemire_reference(w0, d) is None:
            hit += 1
            k = 1
            while lemire_reference(orc.word(seed, stream, i, 0, 0, k), d) is None:
                k += 1
            assert orc.bounded(seed, stream, i, 0, 0, d) == lemire_reference(orc.word(seed, stream, i, 0, 0, k), d)
    assert hit > 20

"""Host Philox4x32-10 (synth.philox), the twin of the device input generator
fftu_fill_uniform: pinned to the generator's published known-answer vectors, and
the exact mapping of its words into [-1, 1)."""
import os

import numpy as np

from synth import philox

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox_kat.txt")


def kat_rows():
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        ctr, key, out = (part.split() for part in line.split("|"))
        yield [int(v, 16) for v in ctr], [int(v, 16) for v in key], [int(v, 16) for v in out]


def test_known_answer_vectors():
    rows = list(kat_rows())
    assert len(rows) == 3
    for ctr, key, want in rows:
        got = philox.philox4x32_10(*[np.array([c], dtype=np.uint64) for c in ctr], *key)
        assert [int(x[0]) for x in got] == want


def test_vectorised_equals_scalar_rounds():
    rng = np.random.default_rng(0)
    c = rng.integers(0, 2 ** 32, size=(4, 64), dtype=np.uint64)
    out = philox.philox4x32_10(*c, 7, 11)
    for i in range(0, 64, 13):
        one = philox.philox4x32_10(*[c[j, i:i + 1] for j in range(4)], 7, 11)
        assert all(int(a[0]) == int(b[i]) for a, b in zip(one, out))


def test_mapping_is_exact_and_in_range():
    for dt, bits in [(np.complex64, 23), (np.complex128, 52)]:
        x = philox.uniform_complex(50_000, 5, 3, dt)
        assert x.dtype == dt
        for part in (x.real, x.imag):
            p = part.astype(np.float64)
            assert p.min() >= -1.0 and p.max() < 1.0
            k = (p + 1.0) * 2.0 ** bits
            assert np.array_equal(k, np.floor(k))          # on the 2^-bits grid
            assert abs(p.mean()) < 0.02 and abs(p.var() - 1.0 / 3.0) < 0.02


def test_counter_base_shifts_the_stream_and_keys_differ():
    # element e of a stream with base B equals element B + e of the stream with base 0
    # (checked on a window that crosses 2^32, where the counter's high word changes)
    whole = philox.uniform_complex(300, 5, 9, np.complex128, counter_base=(1 << 32) - 100)
    head = philox.uniform_complex(100, 5, 9, np.complex128, counter_base=(1 << 32) - 100)
    tail = philox.uniform_complex(200, 5, 9, np.complex128, counter_base=1 << 32)
    assert np.array_equal(whole, np.concatenate([head, tail]))
    other = philox.uniform_complex(300, 5, 10, np.complex128, counter_base=(1 << 32) - 100)
    assert not np.any(other == whole)


def test_complex64_is_the_truncated_complex128_stream():
    """re of complex64 keeps the top 24 bits of x0; re of complex128 uses x0 then x1:
    so the complex64 value is the complex128 value truncated to the 2^-23 grid."""
    d = philox.uniform_complex(10_000, 5, 1, np.complex128)
    s = philox.uniform_complex(10_000, 5, 1, np.complex64)
    want = np.floor((d.real + 1.0) * 2.0 ** 23) * 2.0 ** -23 - 1.0
    assert np.array_equal(s.real.astype(np.float64), want)

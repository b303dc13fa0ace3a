"""Pins of the oracle's Delta-fix codec (section 2: Delta encoding stores the
first value and the differences of neighbouring values; the evaluation's
Delta-fix baseline runs it over fixed-length partitions).  Each partition
keeps its first value, and its first differences d_k as offsets from their
minimum at width bitlen(d_max - d_min).  CPU only."""
from __future__ import annotations

import numpy as np
import pytest

import oracle as R

HEADER, RECORD = 32, 32


def records(blob: np.ndarray):
    m = int(blob[24:32].view(np.uint64)[0])
    out = []
    for j in range(m):
        r = blob[HEADER + RECORD * j: HEADER + RECORD * (j + 1)]
        q = r[:24].view(np.uint64)
        dmin = int(q[1]) - (1 << 64 if r[25] == 0xFF else 0)
        out.append(dict(first=int(q[0]), dmin=dmin, word_off=int(q[2]), width=int(r[24])))
    return out


def closed_form(col, L: int):
    """Widths and total size from the definition, in Python integers."""
    v = [int(x) for x in col]
    widths, words = [], 0
    for a in range(0, len(v), L):
        part = v[a:a + L]
        d = [y - x for x, y in zip(part, part[1:])]
        w = (max(d) - min(d)).bit_length() if d else 0
        widths.append(w)
        words += ((len(part) - 1) * w + 63) // 64 if d else 0
    return widths, HEADER + RECORD * len(widths) + 8 * words


def test_figure_values_by_hand():
    """30 31 32 29 49 as one partition: differences 1 1 -3 20, d_min = -3,
    offsets 4 4 0 23, width bitlen(23) = 5.  Packed LSB first at bits 0, 5,
    10, 15: byte 0 = bit 2 + bit 7 = 132, byte 1 = bit 15 = 128, byte 2 =
    bits 16, 17, 19 = 11.  Size 32 + 32 + 8 = 72."""
    v = np.array([30, 31, 32, 29, 49], np.uint64)
    blob = R.delta_fix_encode(v, 5)
    assert len(blob) == 72 == R.delta_fix_bytes(v, 5)
    rec = records(blob)
    assert rec == [dict(first=30, dmin=-3, word_off=0, width=5)]
    assert list(blob[64:72]) == [132, 128, 11, 0, 0, 0, 0, 0]
    assert list(R.delta_fix_decode(blob)) == [30, 31, 32, 29, 49]


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
def test_closed_form_widths_and_size(seed, dtype):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 5000))
    L = int(rng.choice([1, 2, 3, 64, 100, 1000, 4096]))
    top = 2**32 - 1 if dtype == np.uint32 else 2**64 - 1
    kind = seed % 3
    if kind == 0:
        col = np.cumsum(rng.integers(0, 100, n, dtype=np.uint64)).astype(dtype)
    elif kind == 1:
        col = rng.integers(0, top, n, dtype=np.uint64, endpoint=True).astype(dtype)
    else:
        col = (np.arange(n, dtype=np.uint64) * np.uint64(7) % np.uint64(1000)).astype(dtype)
    blob = R.delta_fix_encode(col, L)
    widths, size = closed_form(col, L)
    assert len(blob) == size == R.delta_fix_bytes(col, L)
    assert [r["width"] for r in records(blob)] == widths
    assert np.array_equal(R.delta_fix_decode(blob), col)


def test_widest_differences_take_65_bits():
    """Values alternating 0 and 2^64 - 1: differences +-(2^64 - 1), range
    2^65 - 2, width 65."""
    col = np.array([0, 2**64 - 1] * 50, np.uint64)
    blob = R.delta_fix_encode(col, 100)
    assert records(blob)[0]["width"] == 65
    assert len(blob) == HEADER + RECORD + 8 * ((99 * 65 + 63) // 64)
    assert np.array_equal(R.delta_fix_decode(blob), col)


def test_progressions_store_no_offsets():
    """An arithmetic progression has one difference value: width 0, the
    blob is header and records only, and decoding rebuilds the line."""
    col = (np.uint64(5) + np.arange(10_000, dtype=np.uint64) * np.uint64(3)).astype(np.uint64)
    blob = R.delta_fix_encode(col, 1000)
    assert len(blob) == HEADER + RECORD * 10
    assert all(r["width"] == 0 and r["dmin"] == 3 for r in records(blob))
    assert np.array_equal(R.delta_fix_decode(blob), col)


@pytest.mark.parametrize("L", [2, 17, 1024])
def test_offsets_are_for_of_the_differences(ref, L):
    """Delta encoding is frame-of-reference coding of the first
    differences: for a non-decreasing column, each partition's offset words
    equal the words of the constant-model (FOR) blob of that partition's
    difference sequence, encoded as one partition by the codec's encoder."""
    rng = np.random.default_rng(L)
    col = np.cumsum(rng.integers(0, 5000, 20 * L + 3, dtype=np.uint64)).astype(np.uint64)
    blob = R.delta_fix_encode(col, L)
    recs = records(blob)
    m = len(recs)
    words = blob[HEADER + RECORD * m:]
    for j, r in enumerate(recs):
        part = col[j * L:(j + 1) * L]
        d = np.diff(part).astype(np.uint64)
        if len(d) == 0:
            continue
        for_blob = ref.encode(d, fixed_len=len(d), force_constant=True)
        hdr = for_blob[:64].view(np.uint64)
        woff, tw = int(hdr[6]), int(hdr[7])
        rec = ref.blob_record(for_blob, 0)
        assert rec["bits"] == r["width"] and rec["base"] == r["dmin"]
        span = words[8 * r["word_off"]: 8 * (r["word_off"] + tw)]
        assert np.array_equal(span, for_blob[woff: woff + 8 * tw])

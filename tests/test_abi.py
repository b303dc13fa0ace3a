"""CPU-side checks of the C ABI: the library builds, loads, exports every
symbol that include/leco.h declares, and its host-only calls (sizes, header
parsing, argument validation) behave as documented.  No kernel runs here."""
from __future__ import annotations

import os
import re

import numpy as np
import pytest

import paper_2306_15374_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols() -> list[str]:
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"\b(leco_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    L = P.lib()
    decl = declared_symbols()
    assert decl, "no declarations found"
    for name in decl:
        assert hasattr(L, name), name
    assert sorted(P.EXPORTS) == decl


def test_max_blob_bytes_bounds_the_oracle(ref):
    rng = np.random.default_rng(0)
    for dtype, npdt in ((P.LECO_U32, np.uint32), (P.LECO_U64, np.uint64)):
        for n in (0, 1, 1000, 4097):
            col = rng.integers(0, np.iinfo(npdt).max, size=n, dtype=npdt, endpoint=True)
            for L in (1, 7, 1024):
                part, _ = P.make_partitioning(fixed_len=L)
                bound = P.leco_max_blob_bytes(n, dtype, part)
                assert bound >= ref.blob_bytes(col, fixed_len=L)
                assert bound % 16 == 0


def test_max_blob_bytes_rejects_bad_partitionings():
    for starts in ([0, 5, 5, 10], [1, 10], [0, 9]):
        part, keep = P.make_partitioning(starts=starts)
        with pytest.raises(P.LecoError) as e:
            P.leco_max_blob_bytes(10, P.LECO_U64, part)
        assert e.value.status == P.LECO_EINVAL
    part, _ = P.make_partitioning(fixed_len=(1 << 20) + 1)
    with pytest.raises(P.LecoError):
        P.leco_max_blob_bytes(10, P.LECO_U64, part)
    part, _ = P.make_partitioning(fixed_len=8)
    with pytest.raises(P.LecoError):
        P.leco_max_blob_bytes(10, 5, part)


def test_blob_info_parses_oracle_header(ref):
    col = np.arange(5000, dtype=np.uint32) * np.uint32(3)
    blob = ref.encode(col, fixed_len=1000)
    assert P.leco_blob_info(blob.tobytes()) == (5000, 4, 5)
    bad = bytearray(blob.tobytes()[:64])
    bad[4] = 9
    with pytest.raises(P.LecoError) as e:
        P.leco_blob_info(bytes(bad))
    assert e.value.status == P.LECO_EFORMAT

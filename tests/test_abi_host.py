"""Host-only checks of the C-ABI library: it loads without a GPU, exports every
symbol include/perm.h declares, and its host-side logic (chunk plan, 0/1 range
bound, status strings) is right.  No kernel is launched here."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "perm.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(perm_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def b():
    from paper_1904_06229_amd import binding
    return binding


def test_library_exports_every_declared_symbol(b):
    names = header_functions()
    assert "perm_real" in names and "perm_batched" in names and "perm_partial" in names
    lib = ctypes.CDLL(b.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), f"libperm.so lacks {name}"
    assert set(names) == set(b.SIGNATURES), "binding signatures out of sync with perm.h"


def test_version_and_strerror(b):
    assert "gfx950" in b.perm_version()
    seen = set()
    for s in range(7):
        t = b.perm_strerror(s)
        assert t and t not in seen
        seen.add(t)


@pytest.mark.parametrize("n", [1, 2, 5, 20, 30, 40, 48, 64])
def test_plan_covers_range_exactly(b, n):
    T = 1 << (n - 1) if n < 64 else 1 << 63
    r = np.random.default_rng(n)
    cases = [(0, T, 0), (0, T, 3)]
    for _ in range(20):
        s = int(r.integers(0, T)) if T > 1 else 0
        c = int(r.integers(0, T - s + 1)) if T - s > 0 else 0
        cases.append((s, c, int(r.integers(0, 9))))
    for start, count, lc in cases:
        p = b.perm_plan(n, start, count, lc)
        L = 1 << p["log2_chunk"]
        if lc:
            assert p["log2_chunk"] == lc
        assert p["head_start"] == start
        assert p["head_count"] < L or p["body_chunks"] == 0
        body_start = start + p["head_count"]
        if p["body_chunks"]:
            assert p["body_first_chunk"] * L == body_start
        assert p["tail_start"] == body_start + p["body_chunks"] * L
        assert p["tail_start"] + p["tail_count"] == start + count
        assert p["tail_count"] < L
        assert p["body_tasks"] == 2 * ((p["body_chunks"] + 127) // 128)


def test_plan_auto_chunk_caps(b):
    assert b.perm_plan(30, 0, 1 << 29, 0, is_int01=True)["log2_chunk"] <= 10
    assert b.perm_plan(48, 0, 1 << 47, 0)["log2_chunk"] <= 12
    assert b.perm_plan(20, 0, 1 << 19, 0)["log2_chunk"] >= 0


def test_plan_rejects_bad_ranges(b):
    with pytest.raises(b.PermError):
        b.perm_plan(10, 500, 100)  # 500 + 100 > 2^9
    with pytest.raises(b.PermError):
        b.perm_plan(0, 0, 0)
    with pytest.raises(b.PermError):
        b.perm_plan(65, 0, 1)
    with pytest.raises(b.PermError):
        b.perm_plan(30, 0, 1 << 29, 11, is_int01=True)


def bregman_log2(deg):
    if any(d == 0 for d in deg):
        return 0.0
    return (len(deg) - 1) + sum(math.lgamma(d + 1) / math.log(2) / d for d in deg)


def test_int01_bound_matches_bregman(b):
    r = np.random.default_rng(1)
    for n in (5, 20, 30, 40):
        for _ in range(5):
            d = r.integers(1, n + 1, size=n)
            assert abs(b.perm_int01_bound(d) - bregman_log2(d)) < 1e-9
    assert b.perm_int01_bound([3, 0, 2]) == 0.0


def test_int01_bound_thresholds(b):
    # J_n: (n-1) + log2(n!) -- exact in 128 bits up to n = 28 (2^27 * 28! < 2^127)
    assert b.perm_int01_bound([28] * 28) < 127
    assert b.perm_int01_bound([29] * 29) >= 127
    assert math.log2(math.factorial(28)) + 27 < 127
    # the 30x30 Bernoulli(1/2) workload passes with margin
    from paper_1904_06229_amd import inputs
    B = inputs.bernoulli01(30, 20190413)
    assert b.perm_int01_bound(B.sum(axis=1)) < 120


def test_size_offset_arrays_checked(b):
    """Sizes and offsets reach the library as int32 / int64 arrays without a
    per-element copy; a value that does not fit raises instead of wrapping."""
    arr, ptr = b._host_ints(np.arange(5, dtype=np.int64), "int32")
    assert arr.dtype == np.int32 and list(arr) == [0, 1, 2, 3, 4] and ptr.value
    same = np.arange(3, dtype=np.int64)
    assert np.shares_memory(b._host_ints(same, "int64")[0], same)  # no copy
    for bad in ([2 ** 40], np.array([2 ** 33], dtype=np.int64), [-(2 ** 31) - 1]):
        with pytest.raises(ValueError):
            b._host_ints(bad, "int32")
    with pytest.raises(TypeError):
        b._host_ints([1.5], "int32")
    with pytest.raises(ValueError):
        b._host_ints([[1, 2]], "int64")


def test_struct_layouts_match_the_header(b, tmp_path):
    """The binding's ctypes structs have the C layout of perm.h (sizes and
    field offsets from a small C program built against the header)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"perm_opts": b.perm_opts, "perm_result": b.perm_result,
               "perm_plan_info": b.perm_plan_info}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "perm.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    for line in filter(None, out):
        name, field, value = line.split()
        cls = structs[name]
        want = ctypes.sizeof(cls) if field == "size" else getattr(cls, field).offset
        assert int(value) == want, line


def test_one_hip_runtime_whatever_the_import_order():
    """Importing the binding before torch must not load a second HIP runtime
    (torch ships its own libamdhip64; the library has to use that one)."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1904_06229_amd import binding\n"
            "import torch\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "print(len({l.split()[-1] for l in maps if 'libamdhip64' in l}))\n") % ROOT
    out = subprocess.run([sys.executable, "-c", code], check=True, capture_output=True,
                         text=True).stdout.strip().splitlines()[-1]
    assert out == "1"
